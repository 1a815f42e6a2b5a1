"""Pins of the FP64 CPU oracle to what the paper and the mathematics fix.

None of these re-types an oracle formula: each checks the oracle against a
closed form, an invariant, a brute-force search, or a different definition of
the same quantity, chosen so that a plausible mistake (a dropped staple term,
a wrong conjugation or neighbour, a wrong normalisation of F or theta, a wrong
side for G on the backward links) fails at least one of them.

The paper prints no worked example with numbers, so there are no golden
values from it; the invariants below are the pins.
"""
import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

LANDAU, COULOMB = 0, 1
SUBGROUPS = [(0, 1), (0, 2), (1, 2)]


# --- helpers written from textbook definitions (not from the oracle) -----

def links(U):
    return U.reshape(-1, 4, 3, 3)


def dagger(m):
    return np.swapaxes(m, -1, -2).conj()


def shift(U, mu, step):
    """Field translated so that the result at x is U at x + step*mu."""
    return np.roll(U, -step, axis=3 - mu)


def plaquettes(U):
    """Re Tr of every plaquette U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+."""
    out = []
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a = U[..., mu, :, :]
            b = shift(U, mu, 1)[..., nu, :, :]
            c = dagger(shift(U, nu, 1)[..., mu, :, :])
            d = dagger(U[..., nu, :, :])
            out.append(np.trace(a @ b @ c @ d, axis1=-2, axis2=-1).real)
    return np.stack(out)


def unitarity_error(U):
    L = links(U)
    eye = np.eye(3)
    return (np.abs(L @ dagger(L) - eye).max(), np.abs(np.linalg.det(L) - 1).max())


def su2_matrix_textbook(x):
    """Unit 4-vectors -> SU(2) as [[alpha, beta], [-conj(beta), conj(alpha)]]."""
    alpha = x[..., 0] + 1j * x[..., 1]
    beta = x[..., 2] + 1j * x[..., 3]
    m = np.empty(x.shape[:-1] + (2, 2), dtype=np.complex128)
    m[..., 0, 0], m[..., 0, 1] = alpha, beta
    m[..., 1, 0], m[..., 1, 1] = -beta.conj(), alpha.conj()
    return m


def quat_to_matrix(q):
    """The oracle's quaternion convention, used only to read its output."""
    return np.array([[q[0] + 1j * q[3], q[2] + 1j * q[1]],
                     [-q[2] + 1j * q[1], q[0] - 1j * q[3]]])


def gell_mann_local():
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return lam


def site_coords(dims, s):
    nx, ny, nz, nt = dims
    return s % nx, (s // nx) % ny, (s // (nx * ny)) % nz, s // (nx * ny * nz)


def gauge_transform_site(U, dims, s, G):
    """Apply a gauge transformation that is G at site s and 1 elsewhere:
    U_mu(s) -> G U_mu(s), U_mu(s - mu) -> U_mu(s - mu) G^+."""
    x, y, z, t = site_coords(dims, s)
    W = U.copy()
    c = [x, y, z, t]
    for mu in range(4):
        W[t, z, y, x, mu] = G @ W[t, z, y, x, mu]
        b = list(c)
        b[mu] = (b[mu] - 1) % dims[mu]
        W[b[3], b[2], b[1], b[0], mu] = W[b[3], b[2], b[1], b[0], mu] @ dagger(G)
    return W


def embed(g2, a, b):
    G = np.eye(3, dtype=np.complex128)
    G[a, a], G[a, b], G[b, a], G[b, b] = g2[0, 0], g2[0, 1], g2[1, 0], g2[1, 1]
    return G


# --- SU(2) local solution, eq. (6), and its overrelaxed power -------------

def test_su2_solution_is_eq6(oracle_lib):
    """omega = 1 returns g = K^+ (det K^+)^(-1/2) for K in (R+) x SU(2)."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        b = rng.standard_normal(4) * rng.uniform(0.1, 10)
        k = quat_to_matrix(b)  # an SU(2) block times |b|
        kd = dagger(k)
        expected = kd / np.sqrt(np.linalg.det(kd))
        got = quat_to_matrix(oracle_lib.su2_solve(b, 1.0))
        np.testing.assert_allclose(got, expected, atol=1e-14)
        # and it maximises Re Tr[g k]: value 2 |b|
        assert abs(np.trace(got @ k).real - 2 * np.linalg.norm(b)) < 1e-12 * max(1, np.linalg.norm(b))


def _principal_power(g, w):
    """Principal power of a 2x2 unitary by eigendecomposition (log on (-pi, pi])."""
    ev, vec = np.linalg.eig(g)
    ang = np.angle(ev)
    return vec @ np.diag(np.exp(1j * w * ang)) @ np.linalg.inv(vec)


def test_su2_overrelaxation_power(oracle_lib):
    rng = np.random.default_rng(12)
    for _ in range(200):
        b = rng.standard_normal(4)
        g1 = quat_to_matrix(oracle_lib.su2_solve(b, 1.0))
        np.testing.assert_allclose(quat_to_matrix(oracle_lib.su2_solve(b, 0.0)), np.eye(2), atol=1e-15)
        np.testing.assert_allclose(quat_to_matrix(oracle_lib.su2_solve(b, 2.0)), g1 @ g1, atol=1e-14)
        h = quat_to_matrix(oracle_lib.su2_solve(b, 0.5))
        np.testing.assert_allclose(h @ h, g1, atol=1e-14)
        for w in (1.5, 1.7, 1.9):
            gw = quat_to_matrix(oracle_lib.su2_solve(b, w))
            np.testing.assert_allclose(gw, _principal_power(g1, w), atol=1e-12)
            # closed form of the local gain: f(g^w) = 2|b| cos((w - 1) phi)
            k = quat_to_matrix(b)
            phi = np.arctan2(np.linalg.norm(b[1:]), b[0])
            assert abs(np.trace(gw @ k).real - 2 * np.linalg.norm(b) * np.cos((w - 1) * phi)) < 1e-12


def test_su2_degenerate_cases(oracle_lib):
    np.testing.assert_array_equal(oracle_lib.su2_solve(np.zeros(4), 1.7), [1, 0, 0, 0])
    # b = (-1, 0, 0, 0): g = -1, over-rotated about the third axis
    q = oracle_lib.su2_solve(np.array([-2.0, 0, 0, 0]), 1.7)
    np.testing.assert_allclose(q, [np.cos(1.7 * np.pi), 0, 0, np.sin(1.7 * np.pi)], atol=1e-15)
    np.testing.assert_allclose(oracle_lib.su2_solve(np.array([3.0, 0, 0, 0]), 1.7), [1, 0, 0, 0], atol=1e-15)


# --- K(x) of eq. (5) pinned against F of eq. (1) ---------------------------

@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_staple_predicts_local_change_of_F(oracle_lib, field_cache, gauge):
    """F depends on g(x) only through Re Tr[g(x) K(x)] (eqs. 4-5): a gauge
    transformation at one site changes the unnormalised functional by exactly
    Re Tr[(G - 1) K]. Checked for random SU(3) G (not just subgroup ones)."""
    dims = (4, 2, 4, 2)
    U = field_cache(dims, 0.9, 3)
    V = int(np.prod(dims))
    nd = 3 if gauge == COULOMB else 4
    rng = np.random.default_rng(5)
    F0 = oracle_lib.quality(U, dims, gauge)[0]
    for s in rng.choice(V, 8, replace=False):
        K = oracle_lib.staple(U, dims, s, gauge)
        H = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        G = scipy.linalg.expm(1j * (H + dagger(H)) / 2)
        F1 = oracle_lib.quality(gauge_transform_site(U, dims, s, G), dims, gauge)[0]
        pred = np.trace((G - np.eye(3)) @ K).real / (nd * 3 * V)
        assert abs((F1 - F0) - pred) < 1e-14


# --- brute force over SU(2) ------------------------------------------------

def test_subgroup_step_is_the_su2_maximum_bruteforce(oracle_lib, field_cache):
    """On every site and subgroup of a 2^4 lattice, the oracle's omega = 1
    step reaches max over SU(2) of Re Tr[G K]: no Haar sample exceeds it and a
    polished maximum agrees with it."""
    dims = (2, 2, 2, 2)
    U = field_cache(dims, 1.2, 4)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((200_000, 4))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    samples = su2_matrix_textbook(x)
    for s in range(16):
        for sub, (a, b) in enumerate(SUBGROUPS):
            K = oracle_lib.staple(U, dims, s)
            W = U.copy()
            oracle_lib.subgroup_update(W, dims, s, sub, 1.0)
            t, z, y, xx = site_coords(dims, s)[::-1]
            G = W[t, z, y, xx, 0] @ dagger(U[t, z, y, xx, 0])
            f_oracle = np.trace(G @ K).real
            rest = sum(K[r, r].real for r in range(3) if r not in (a, b))
            k = K[np.ix_([a, b], [a, b])]
            f_samples = np.einsum("nij,ji->n", samples, k).real + rest
            best = f_samples.max()
            assert best <= f_oracle + 1e-12
            x0 = x[f_samples.argmax()]

            def negf(v):
                v = v / np.linalg.norm(v)
                return -(np.trace(su2_matrix_textbook(v) @ k).real + rest)
            res = scipy.optimize.minimize(negf, x0, method="Nelder-Mead",
                                          options=dict(xatol=1e-13, fatol=1e-15, maxiter=20000))
            assert abs(-res.fun - f_oracle) < 1e-9
            # and the step is a special unitary embedded in rows/cols (a, b)
            off = [r for r in range(3) if r not in (a, b)][0]
            assert abs(G[off, off] - 1) < 1e-14


# --- sweeps: monotonicity, unitarity, gauge invariance ----------------------

@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
@pytest.mark.parametrize("omega", [1.0, 1.5, 1.7, 1.9])
def test_F_non_decreasing_every_half_sweep(oracle_lib, field_cache, gauge, omega):
    dims = (4, 4, 4, 4)
    U = field_cache(dims, 0.7, 1)
    V = int(np.prod(dims))
    F_prev = oracle_lib.quality(U, dims, gauge)[0]
    for it in range(6):
        for p in (0, 1):
            oracle_lib.half_sweep(U, dims, p, omega, gauge)
            F = oracle_lib.quality(U, dims, gauge)[0]
            assert F >= F_prev - 1e-15
            assert F <= 1 + 1e-14
            F_prev = F


@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_sweeps_keep_unitarity_and_plaquettes(oracle_lib, field_cache, gauge):
    dims = (4, 4, 2, 6)
    U = field_cache(dims, 0.7, 2)
    P0 = plaquettes(U)
    for _ in range(5):
        oracle_lib.sweep(U, dims, 1.7, gauge)
        e_u, e_d = unitarity_error(U)
        assert e_u < 1e-13 and e_d < 1e-13
    np.testing.assert_allclose(plaquettes(U), P0, atol=1e-12)


def test_translation_covariance(oracle_lib, field_cache):
    """sweep(shift(U)) == shift(sweep(U)) for parity-preserving shifts."""
    dims = (4, 4, 4, 4)
    U = field_cache(dims, 0.5, 6)
    for shifts in [((0, 2),), ((0, 1), (1, 1)), ((2, 1), (3, -1))]:
        A = U.copy()
        oracle_lib.sweep(A, dims, 1.7)
        B = U.copy()
        for mu, st in shifts:
            B = shift(B, mu, st)
        B = np.ascontiguousarray(B)
        oracle_lib.sweep(B, dims, 1.7)
        for mu, st in shifts:
            A = shift(A, mu, st)
        np.testing.assert_array_equal(A, B)


def test_half_sweep_is_independent_of_site_order(oracle_lib, field_cache):
    """Same-parity sites share no link, so any visiting order gives the same
    bits (the race-freedom argument for a parallel half-sweep)."""
    dims = (4, 2, 4, 4)
    U = field_cache(dims, 0.8, 8)
    V = int(np.prod(dims))
    for p in (0, 1):
        A = U.copy()
        oracle_lib.half_sweep(A, dims, p, 1.7)
        order = np.random.default_rng(p).permutation(V)
        B = U.copy()
        oracle_lib.half_sweep_order(B, dims, p, 1.7, order)
        np.testing.assert_array_equal(A, B)


@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_sweeps_do_not_depend_on_the_thread_count(oracle_lib, field_cache, gauge):
    """The threaded half-sweep (the CPU baseline's timed form) gives bitwise
    the single-thread result, and both equal the sequential lexicographic
    visit of half_sweep_order."""
    import os
    dims = (6, 4, 4, 8)
    U = field_cache(dims, 0.7, 9)
    V = int(np.prod(dims))
    before = oracle_lib.set_threads(0)
    try:
        out = []
        for n in (1, max(2, os.cpu_count() or 2)):
            assert oracle_lib.set_threads(n) == n
            A = U.copy()
            for _ in range(3):
                oracle_lib.sweep(A, dims, 1.7, gauge)
            out.append(A)
        B = U.copy()
        for _ in range(3):
            for p in (0, 1):
                oracle_lib.half_sweep_order(B, dims, p, 1.7, np.arange(V), gauge)
        np.testing.assert_array_equal(out[0], out[1])
        np.testing.assert_array_equal(out[0], B)
    finally:
        oracle_lib.set_threads(before)


# --- F and theta, eqs. (1)-(3) ----------------------------------------------

@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_theta_is_the_squared_gradient_of_F(oracle_lib, field_cache, gauge):
    """With g(x) = exp(i s_a lambda_a / 2) at one site, central finite
    differences of F give dF/ds_a(x) = delta_a(x) / (2 d N_c V), where
    Delta = i sum_a delta_a lambda_a; summing squares gives
    theta = 8 d^2 N_c V sum (dF/ds)^2. Pins the literal Delta convention and
    the normalisations of F and theta at once."""
    dims = (2, 4, 2, 2)
    U = field_cache(dims, 0.8, 9)
    V = int(np.prod(dims))
    nd = 3 if gauge == COULOMB else 4
    lam = gell_mann_local()
    F0, theta = oracle_lib.quality(U, dims, gauge)
    Delta = oracle_lib.divergence_field(U, dims, gauge)
    h = 1e-5
    grad = np.zeros((V, 8))
    for s in range(V):
        for a in range(8):
            Gp = scipy.linalg.expm(1j * h * lam[a] / 2)
            Fp = oracle_lib.quality(gauge_transform_site(U, dims, s, Gp), dims, gauge)[0]
            Fm = oracle_lib.quality(gauge_transform_site(U, dims, s, dagger(Gp)), dims, gauge)[0]
            grad[s, a] = (Fp - Fm) / (2 * h)
    delta = np.einsum("aij,sji->sa", lam, Delta) / 2j
    assert np.abs(delta.imag).max() < 1e-13
    np.testing.assert_allclose(grad, delta.real / (2 * nd * 3 * V), atol=1e-10 / V)
    np.testing.assert_allclose(8 * nd**2 * 3 * V * (grad**2).sum(), theta, rtol=1e-8)
    # Delta is anti-hermitian and traceless
    assert np.abs(Delta + dagger(Delta)).max() < 1e-14
    assert np.abs(np.trace(Delta, axis1=1, axis2=2)).max() < 1e-14


def test_F_theta_invariant_under_global_rotation(oracle_lib, field_cache):
    dims = (4, 4, 2, 2)
    U = field_cache(dims, 0.6, 10)
    rng = np.random.default_rng(3)
    H = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    G = scipy.linalg.expm(1j * (H + dagger(H)) / 2)
    W = np.ascontiguousarray(G @ U @ dagger(G))
    for gauge in (LANDAU, COULOMB):
        F0, t0 = oracle_lib.quality(U, dims, gauge)
        F1, t1 = oracle_lib.quality(W, dims, gauge)
        assert abs(F0 - F1) < 1e-14 and abs(t0 - t1) < 1e-12 * max(1, t0)


def test_unit_field_values(oracle_lib):
    dims = (4, 2, 2, 2)
    U = np.zeros((2, 2, 2, 4, 4, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    for gauge in (LANDAU, COULOMB):
        F, th = oracle_lib.quality(U, dims, gauge)
        assert F == 1.0 and th == 0.0


# --- Alg. 1 end to end --------------------------------------------------------

@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_pure_gauge_is_fixed_to_unit_links(oracle_lib, field_cache, gauge):
    dims = (4, 4, 4, 4)
    U = field_cache(dims, 0.0, 0)
    r = oracle_lib.fix(U, dims, 1.7, 1e-12, 2000, gauge)
    assert r["converged"] and r["theta"] < 1e-12
    assert abs(r["F"] - 1) < 1e-12
    nd = 3 if gauge == COULOMB else 4
    L = links(U)[:, :nd]
    assert np.abs(L - np.eye(3)).max() < 1e-6  # |U - 1|^2 ~ (1 - F) scale


def test_landau_4x4_config_converges(oracle_lib, field_cache):
    """4^4, amp 0.3, seed 0, omega 1.7, theta < 1e-12 within 2000 sweeps."""
    dims = (4, 4, 4, 4)
    U = field_cache(dims, 0.3, 0)
    W = U.copy()
    Fs = [oracle_lib.quality(W, dims)[0]]
    for _ in range(300):
        oracle_lib.sweep(W, dims, 1.7)
        Fs.append(oracle_lib.quality(W, dims)[0])
    # monotone up to the rounding noise of the converged functional (~1e-15)
    assert np.all(np.diff(Fs) >= -1e-14)
    r = oracle_lib.fix(U, dims, 1.7, 1e-12, 2000)
    assert r["converged"] and 10 < r["iters"] < 2000
    assert r["theta"] < 1e-12


def test_resume_is_bitwise_equal(oracle_lib, field_cache):
    dims = (4, 4, 4, 4)
    U = field_cache(dims, 0.3, 0)
    A = U.copy()
    oracle_lib.fix(A, dims, 1.7, 0.0, 30, reunit_every=7)
    B = U.copy()
    oracle_lib.fix(B, dims, 1.7, 0.0, 12, reunit_every=7)
    oracle_lib.fix(B, dims, 1.7, 0.0, 18, reunit_every=7, start_sweep=12)
    np.testing.assert_array_equal(A, B)


# --- reunitarisation -----------------------------------------------------------

def test_reunit_matches_qr_orthonormalisation(oracle_lib, field_cache):
    """Rows 0, 1 equal a QR orthonormalisation (positive R diagonal) of the
    first two rows; the result is in SU(3) and an SU(3) input is unchanged."""
    U = field_cache((2, 2, 2, 2), 0.5, 12)
    rng = np.random.default_rng(1)
    L = links(U).reshape(-1, 3, 3)
    P = L + 1e-3 * (rng.standard_normal(L.shape) + 1j * rng.standard_normal(L.shape))
    R = np.ascontiguousarray(P)
    oracle_lib.reunit(R)
    for m, r in zip(P, R):
        q, rr = np.linalg.qr(m[:2].T)
        q = q * np.sign(np.diag(rr).real)  # positive real diagonal (rr diag is real here)
        ph = np.diag(rr) / np.abs(np.diag(rr))
        q = (q @ np.diag(ph.conj() / np.sign(np.diag(rr).real)))
        np.testing.assert_allclose(r[:2], q.T, atol=1e-13)
    e_u = np.abs(R @ dagger(R) - np.eye(3)).max()
    e_d = np.abs(np.linalg.det(R) - 1).max()
    assert e_u < 1e-14 and e_d < 1e-14
    S = np.ascontiguousarray(L.copy())
    oracle_lib.reunit(S)
    np.testing.assert_allclose(S, L, atol=1e-14)
