"""GPU parity of the differentiation line: F_U[g] for g = exp(i s_a lambda_a/2),
its hand-written backward kernel, the autograd.Function around them and the
steepest-descent cross-check, against the FP64 oracle (oracle/diff.py).

Tolerances: FP64 forward 1e-13 relative; FP64 gradient 1e-12 of its largest
entry (series vs eigendecomposition dexp differ at rounding level); FP32 runs
store U, s and g in float (relative rounding 6e-8 on O(10) terms per site),
so 2e-6 relative for F and 1e-4 of the largest gradient entry.
"""
import numpy as np
import pytest
import torch

from oracle import diff

pytestmark = pytest.mark.gpu

LANDAU, COULOMB = 0, 1


@pytest.fixture(scope="module")
def gf():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1412_1498_amd import gf as mod
    return mod


def rand_alg(dims, sigma, seed):
    from paper_1412_1498_amd import synth
    return synth.random_algebra_field(dims, sigma, seed).numpy()


def setup(gf, dims, gauge, prec, U, s):
    ctx = gf.Context(dims, gauge=gauge, prec=prec)
    Ug = ctx.pack(torch.from_numpy(np.ascontiguousarray(U)).to("cuda", dtype=ctx.cdtype))
    sg = ctx.pack_alg(torch.from_numpy(np.ascontiguousarray(s)).to("cuda", dtype=ctx.rdtype))
    return ctx, Ug, sg


def cast(U, s, prec):
    if prec == 1:
        return U.astype(np.complex64).astype(np.complex128), s.astype(np.float32).astype(np.float64)
    return U, s


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 8), (16, 16, 16, 16)])
def test_functional_and_gradient_match_oracle(gf, field_cache, prec, gauge, dims):
    U = field_cache(dims, 0.4, 30)
    s = rand_alg(dims, 0.1, 31)
    ctx, Ug, sg = setup(gf, dims, gauge, prec, U, s)
    Uo, so = cast(U, s, prec)
    F = ctx.functional(Ug, sg)
    Fo = diff.functional(Uo, so, gauge)
    assert abs(F - Fo) <= (1e-13 if prec == 0 else 2e-6) * abs(Fo)
    grad = ctx.unpack_alg(ctx.functional_grad(Ug, sg)).cpu().numpy().astype(np.float64)
    go = diff.gradient(Uo, so, gauge)
    scale = np.abs(go).max()
    assert np.abs(grad - go).max() <= (1e-12 if prec == 0 else 1e-4) * scale


@pytest.mark.parametrize("prec", [0, 1])
def test_gradient_at_zero_is_closed_form(gf, oracle_lib, field_cache, prec):
    dims = (8, 8, 8, 8)
    U = field_cache(dims, 0.4, 32)
    V = int(np.prod(dims))
    s = np.zeros(U.shape[:4] + (8,))
    ctx, Ug, sg = setup(gf, dims, LANDAU, prec, U, s)
    Uo, _ = cast(U, s, prec)
    grad = ctx.unpack_alg(ctx.functional_grad(Ug, sg)).cpu().numpy().astype(np.float64).reshape(V, 8)
    Delta = oracle_lib.divergence_field(np.ascontiguousarray(Uo), dims, LANDAU)
    delta = (np.einsum("aij,sji->sa", diff.LAMBDA, Delta) / 2j).real / (2 * 4 * 3 * V)
    assert np.abs(grad - delta).max() <= (1e-13 if prec == 0 else 1e-5) * np.abs(delta).max()
    # theta = 8 d^2 N_c V sum (dF/ds)^2
    _, theta = ctx.quality(Ug)
    assert abs(8 * 16 * 3 * V * (grad ** 2).sum() - theta) <= (1e-12 if prec == 0 else 1e-5) * theta


def test_gradient_central_differences_fp64(gf, field_cache):
    """Central differences (step 1e-6) of the GPU functional itself on a small
    lattice, against the backward kernel."""
    dims = (4, 4, 2, 2)
    U = field_cache(dims, 0.4, 33)
    s = rand_alg(dims, 0.1, 34)
    ctx, Ug, sg = setup(gf, dims, LANDAU, 0, U, s)
    grad = ctx.unpack_alg(ctx.functional_grad(Ug, sg)).cpu().numpy()
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(24):
        idx = tuple(int(rng.integers(n)) for n in (dims[3], dims[2], dims[1], dims[0], 8))
        vals = []
        for sign in (+1, -1):
            sp = s.copy()
            sp[idx] += sign * h
            spg = ctx.pack_alg(torch.from_numpy(sp).cuda())
            vals.append(ctx.functional(Ug, spg))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - grad[idx]) < 2e-6 * np.abs(grad).max()


@pytest.mark.parametrize("prec", [0, 1])
def test_autograd_function(gf, field_cache, prec):
    dims = (6, 4, 4, 2)
    U = field_cache(dims, 0.4, 35)
    s = rand_alg(dims, 0.1, 36)
    ctx, Ug, sg = setup(gf, dims, LANDAU, prec, U, s)
    sv = sg.clone().requires_grad_(True)
    F = gf.GaugeFunctional.apply(sv, Ug, ctx)
    (3.0 * F).backward()
    ref = ctx.functional_grad(Ug, sg, dF=3.0)
    assert torch.equal(sv.grad, ref)
    assert F.item() == ctx.functional(Ug, sg)


@pytest.mark.parametrize("prec", [0, 1])
def test_gauge_transform_matches_oracle(gf, field_cache, prec):
    dims = (4, 6, 2, 4)
    U = field_cache(dims, 0.4, 37)
    s = rand_alg(dims, 0.3, 38)
    ctx, Ug, sg = setup(gf, dims, LANDAU, prec, U, s)
    Uo, so = cast(U, s, prec)
    ctx.gauge_transform(Ug, sg)
    ref = diff.transform(Uo, diff.gauge_fields(so))
    err = np.abs(ctx.unpack(Ug).cpu().numpy() - ref).max()
    assert err < (1e-14 if prec == 0 else 2e-6)


def sd_run_gpu(ctx, Ug, sg0, steps, alpha):
    """Steepest descent driven by the forward/backward pair: s = alpha 2 d N_c V
    grad F at s = 0 (the backward kernel scaled by dF), then g = exp(S(s))."""
    V = ctx.volume()
    Fs = [ctx.quality(Ug)[0]]
    step = torch.empty_like(sg0)
    for _ in range(steps):
        ctx.functional_grad(Ug, sg0, dF=alpha * 2 * 4 * 3 * V, out=step)
        ctx.gauge_transform(Ug, step)
        Fs.append(ctx.quality(Ug)[0])
    return Fs


def test_sd_cross_check_trajectory_8x4(gf, field_cache):
    """200 steps, alpha = 0.08: the GPU forward/backward steepest descent
    follows the oracle's eq. (7) trajectory, F increasing."""
    dims = (8, 8, 8, 8)
    U = field_cache(dims, 0.4, 39)
    zero = np.zeros(U.shape[:4] + (8,))
    ctx, Ug, sg0 = setup(gf, dims, LANDAU, 0, U, zero)
    Fs = sd_run_gpu(ctx, Ug, sg0, 200, 0.08)
    Uo = U.copy()
    for _ in range(200):
        Uo = diff.sd_step(Uo, 0.08)
    assert np.all(np.diff(Fs) > -1e-15)
    assert np.abs(ctx.unpack(Ug).cpu().numpy() - Uo).max() < 1e-11
    assert Fs[-1] > Fs[0]


@pytest.mark.parametrize("dims", [(16, 16, 16, 16), (24, 24, 24, 24)])
@pytest.mark.parametrize("prec", [0, 1])
def test_sd_cross_check_large(gf, field_cache, dims, prec):
    """16^4 and 24^4, amp 0.4: 200 GPU steps with F non-decreasing; the first
    two steps agree with the oracle's eq. (7) step."""
    from paper_1412_1498_amd import synth
    U = synth.random_gauge_field(dims, 0.4, 0).numpy()
    zero = np.zeros(U.shape[:4] + (8,))
    ctx, Ug, sg0 = setup(gf, dims, LANDAU, prec, U, zero)
    Fs = sd_run_gpu(ctx, Ug, sg0, 2, 0.08)
    Uo, _ = cast(U, zero, prec)
    for _ in range(2):
        Uo = diff.sd_step(Uo, 0.08)
    assert np.abs(ctx.unpack(Ug).cpu().numpy() - Uo).max() < (1e-12 if prec == 0 else 2e-5)
    Fs += sd_run_gpu(ctx, Ug, sg0, 198, 0.08)[1:]
    assert np.all(np.diff(Fs) > (-1e-15 if prec == 0 else -2e-7))
    assert Fs[-1] > Fs[0]


def _expm_site(s_x):
    import scipy.linalg
    return scipy.linalg.expm(1j * np.tensordot(s_x, diff.LAMBDA, axes=1) / 2)


def _local_staple(U, s, site, gauge):
    """K(x) of eq. (5) at one site for g = expm(i s lambda / 2), from scipy's
    expm of the neighbours' s (independent of the oracle's eigh route):
    sum over mu in D of U_mu(x) g(x+mu)^+ + U_mu(x-mu)^+ g(x-mu)^+."""
    t, z, y, x = site
    n = U.shape[:4]
    K = np.zeros((3, 3), dtype=np.complex128)
    for mu in range(3 if gauge == COULOMB else 4):
        step = [0, 0, 0, 0]
        step[3 - mu] = 1
        fwd = tuple((c + d) % L for c, d, L in zip(site, step, n))
        bwd = tuple((c - d) % L for c, d, L in zip(site, step, n))
        K += U[t, z, y, x, mu] @ _expm_site(s[fwd]).conj().T
        K += U[bwd][mu].conj().T @ _expm_site(s[bwd]).conj().T
    return K


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dims", [(16, 16, 16, 16), (24, 24, 24, 24)])
def test_gradient_central_differences_256_pairs(gf, dims, prec):
    """Amp 0.4 (seed 0), s ~ N(0, 0.1) (seed 1): the backward kernel at 256
    random (x, a) pairs against central differences (step 1e-6, FP64) of the
    local functional f_x(s) = Re Tr[g(x) K(x)], the only part of eq. (1) that
    depends on s(x) (eqs. 4-5), divided by d N_c V. FP64: 1e-8 relative to
    max(|difference|, 5% of the largest entry) -- the quotient itself rounds
    by ~1e-16 |f_x| / h, about 1e-10 of the largest entry, which would swamp
    a plain relative bound on entries near zero. FP32: the kernel rounds U, s
    and g to float (6e-8 each on O(10) terms), measured 3e-8 of the largest
    entry, bound 2e-7."""
    from paper_1412_1498_amd import synth
    U = synth.random_gauge_field(dims, 0.4, 0).numpy()
    s = synth.random_algebra_field(dims, 0.1, 1).numpy()
    ctx, Ug, sg = setup(gf, dims, LANDAU, prec, U, s)
    Uo, so = cast(U, s, prec)
    grad = ctx.unpack_alg(ctx.functional_grad(Ug, sg)).cpu().numpy().astype(np.float64)
    V = int(np.prod(dims))
    scale = np.abs(grad).max()
    rng = np.random.default_rng(2)
    h = 1e-6
    worst = 0.0
    for _ in range(256):
        site = tuple(int(rng.integers(L)) for L in (dims[3], dims[2], dims[1], dims[0]))
        a = int(rng.integers(8))
        K = _local_staple(Uo, so, site, LANDAU)
        vals = []
        for sign in (+1, -1):
            sp = so[site].copy()
            sp[a] += sign * h
            vals.append(np.trace(_expm_site(sp) @ K).real)
        fd = (vals[0] - vals[1]) / (2 * h) / (4 * 3 * V)
        g = grad[site + (a,)]
        if prec == 0:
            worst = max(worst, abs(fd - g) / max(abs(fd), 0.05 * scale))
        else:
            worst = max(worst, abs(fd - g) / scale)
    print(f"{dims} prec {prec}: worst {worst:.2e}")
    assert worst < (1e-8 if prec == 0 else 2e-7)
