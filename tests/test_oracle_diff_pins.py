"""Pins of the differentiation oracle (oracle/diff.py): the functional F_U[g],
its gradient with respect to s_a(x) and the steepest-descent step of eq. (7),
checked against independent definitions (the C oracle's F and Delta, central
finite differences, scipy's expm)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import diff

LANDAU, COULOMB = 0, 1


def rand_alg(dims, sigma, seed):
    from paper_1412_1498_amd import synth
    return synth.random_algebra_field(dims, sigma, seed).numpy()


def test_exp_matches_scipy():
    s = rand_alg((2, 2, 2, 2), 0.7, 1)
    E = diff.gauge_fields(s)
    for x in range(4):
        H = np.einsum("a,aij->ij", s[0, 0, x // 2, x % 2], diff.LAMBDA) / 2
        np.testing.assert_allclose(E[0, 0, x // 2, x % 2], scipy.linalg.expm(1j * H), atol=1e-14)


@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_functional_is_F_of_the_transformed_field(oracle_lib, field_cache, gauge):
    dims = (4, 2, 4, 2)
    U = field_cache(dims, 0.5, 20)
    s = rand_alg(dims, 0.3, 21)
    assert abs(diff.functional(U, np.zeros_like(s), gauge) - oracle_lib.quality(U, dims, gauge)[0]) < 1e-15
    Ug = np.ascontiguousarray(diff.transform(U, diff.gauge_fields(s)))
    assert abs(diff.functional(U, s, gauge) - oracle_lib.quality(Ug, dims, gauge)[0]) < 1e-14


@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_gradient_at_zero_is_closed_form_delta(oracle_lib, field_cache, gauge):
    """dF/ds_a(x)|_{s=0} = delta_a(x) / (2 d N_c V), Delta = i sum delta_a lambda_a."""
    dims = (4, 4, 2, 2)
    U = field_cache(dims, 0.6, 22)
    V = int(np.prod(dims))
    nd = 3 if gauge == COULOMB else 4
    grad = diff.gradient(U, np.zeros(U.shape[:4] + (8,)), gauge).reshape(V, 8)
    Delta = oracle_lib.divergence_field(U, dims, gauge)
    delta = (np.einsum("aij,sji->sa", diff.LAMBDA, Delta) / 2j).real
    np.testing.assert_allclose(grad, delta / (2 * nd * 3 * V), atol=1e-16)


@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_gradient_matches_central_differences(field_cache, gauge):
    """Central differences (step 1e-6) of the local functional
    f_x(s) = Re Tr[g(x) K(x)] (the only part of F that depends on s(x))."""
    dims = (4, 2, 2, 4)
    U = field_cache(dims, 0.5, 23)
    s = rand_alg(dims, 0.1, 24)
    V = int(np.prod(dims))
    nd = 3 if gauge == COULOMB else 4
    grad = diff.gradient(U, s, gauge)
    g = diff.gauge_fields(s)
    K = diff.staple(U, g, gauge)
    h = 1e-6
    rng = np.random.default_rng(0)
    for _ in range(40):
        t, z, y, x = (rng.integers(n) for n in (dims[3], dims[2], dims[1], dims[0]))
        a = rng.integers(8)
        vals = []
        for sign in (+1, -1):
            sp = s[t, z, y, x].copy()
            sp[a] += sign * h
            gp = scipy.linalg.expm(1j * np.einsum("a,aij->ij", sp, diff.LAMBDA) / 2)
            vals.append(np.trace(gp @ K[t, z, y, x]).real)
        fd = (vals[0] - vals[1]) / (2 * h) / (nd * 3 * V)
        assert abs(fd - grad[t, z, y, x, a]) < 1e-8 * max(1e-3, abs(grad[t, z, y, x, a])) + 1e-12 / V


def test_sd_step_is_the_gradient_step(oracle_lib, field_cache):
    """Eq. (7)'s exponent equals (alpha/2) Delta(x); the step with
    s = alpha 2 d N_c V grad F (at s = 0) is the same transformation."""
    dims = (4, 4, 2, 2)
    U = field_cache(dims, 0.6, 25)
    V = int(np.prod(dims))
    X = diff.sd_direction(U)
    Delta = oracle_lib.divergence_field(U, dims, 0).reshape(X.shape)
    np.testing.assert_allclose(X, Delta, atol=1e-14)
    alpha = 0.08
    s = alpha * 2 * 4 * 3 * V * diff.gradient(U, np.zeros(U.shape[:4] + (8,)))
    np.testing.assert_allclose(diff.transform(U, diff.gauge_fields(s)), diff.sd_step(U, alpha), atol=1e-14)


def test_sd_steps_increase_F(oracle_lib, field_cache):
    dims = (4, 4, 4, 4)
    U = field_cache(dims, 0.4, 26)
    F = [oracle_lib.quality(U, dims, 0)[0]]
    for _ in range(30):
        U = np.ascontiguousarray(diff.sd_step(U, 0.08))
        F.append(oracle_lib.quality(U, dims, 0)[0])
    assert np.all(np.diff(F) > 0)
