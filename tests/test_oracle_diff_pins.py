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


def _textbook_gell_mann():
    """The eight Gell-Mann matrices written out, kept apart from the oracle's
    own table so that a slip in either shows up."""
    i = 1j
    r3 = 1 / np.sqrt(3)
    return np.array([
        [[0, 1, 0], [1, 0, 0], [0, 0, 0]],
        [[0, -i, 0], [i, 0, 0], [0, 0, 0]],
        [[1, 0, 0], [0, -1, 0], [0, 0, 0]],
        [[0, 0, 1], [0, 0, 0], [1, 0, 0]],
        [[0, 0, -i], [0, 0, 0], [i, 0, 0]],
        [[0, 0, 0], [0, 0, 1], [0, 1, 0]],
        [[0, 0, 0], [0, 0, -i], [0, i, 0]],
        [[r3, 0, 0], [0, r3, 0], [0, 0, -2 * r3]],
    ], dtype=np.complex128)


def _global_sum(oracle_lib, U, s, dims, gauge, lam):
    """d N_c V F_U[g] (eq. 1) for g(x) = expm(i sum_a s_a lambda_a / 2), built
    without oracle/diff.py: scipy's expm per site, the transformed links by
    plain products, and F from the C oracle."""
    nd = 3 if gauge == COULOMB else 4
    V = int(np.prod(dims))
    g = np.empty(s.shape[:4] + (3, 3), dtype=np.complex128)
    for idx in np.ndindex(*s.shape[:4]):
        g[idx] = scipy.linalg.expm(1j * np.tensordot(s[idx], lam, axes=1) / 2)
    Ut = np.empty_like(U)
    for mu in range(4):
        gfwd = np.roll(g, -1, axis=3 - mu)
        Ut[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(gfwd, -1, -2))
    return oracle_lib.quality(np.ascontiguousarray(Ut), dims, gauge)[0] * nd * 3 * V


@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_gradient_at_nonzero_s_matches_the_global_functional(oracle_lib, field_cache, gauge):
    """dF/ds_a(x) at s != 0 (sigma 0.3) for every (x, a) of a V = 32 lattice,
    against a fourth-order central difference (step 1e-3) of the whole
    functional F_U[g] of eq. (1) evaluated through the C oracle. The
    difference's truncation error is O(h^4) ~ 1e-13 and its rounding error
    ~1e-16 d N_c V / h ~ 1e-11 of an O(1) derivative of the unnormalised sum."""
    lam = _textbook_gell_mann()
    dims = (2, 4, 2, 2)
    U = field_cache(dims, 0.5, 27)
    s = rand_alg(dims, 0.3, 28)
    V = int(np.prod(dims))
    nd = 3 if gauge == COULOMB else 4
    grad = diff.gradient(U, s, gauge) * nd * 3 * V
    h = 1e-3
    worst = 0.0
    for idx in np.ndindex(*s.shape):
        vals = {}
        for k in (-2, -1, 1, 2):
            sp = s.copy()
            sp[idx] += k * h
            vals[k] = _global_sum(oracle_lib, U, sp, dims, gauge, lam)
        fd = (8 * (vals[1] - vals[-1]) - (vals[2] - vals[-2])) / (12 * h)
        worst = max(worst, abs(fd - grad[idx]) / max(1e-2, abs(grad[idx])))
    assert worst < 1e-8, worst
