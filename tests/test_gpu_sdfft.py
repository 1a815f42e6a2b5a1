"""GPU parity of steepest descent with Fourier acceleration (Alg. 2) against
the FP64 oracle (oracle/sdfft.py), through the C ABI.

Tolerances: FP64 links after one step 1e-13 abs (the oracle transforms the
nine complex matrix elements with numpy's FFT, the GPU the eight real su(3)
components with its own two-level DFT passes: same linear map, different
rounding); FP32 5e-6 (a float spectrum between the passes and a float g).
The lattice extents include odd factors (6 = 3 2, 10 = 5 2, 12 = 4 3,
14 = 7 2) and the smallest, 2."""
import numpy as np
import pytest
import torch

from oracle import sdfft

pytestmark = pytest.mark.gpu

LANDAU, COULOMB = 0, 1


@pytest.fixture(scope="module")
def gf():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1412_1498_amd import gf as mod
    return mod


def setup(gf, dims, gauge, prec, U, **kw):
    ctx = gf.Context(dims, gauge=gauge, prec=prec, params=gf.default_params(prec, **kw))
    Ug = ctx.pack(torch.from_numpy(np.ascontiguousarray(U)).to("cuda", dtype=ctx.cdtype))
    return ctx, Ug


def host(ctx, Ug):
    return ctx.unpack(Ug).cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
@pytest.mark.parametrize("dims", [(4, 6, 2, 8), (8, 8, 8, 8), (6, 4, 4, 2), (10, 6, 12, 14), (2, 4, 2, 6)])
def test_sd_step_matches_oracle(gf, field_cache, prec, gauge, dims):
    U = field_cache(dims, 0.4, 70)
    ctx, Ug = setup(gf, dims, gauge, prec, U)
    Uo = U.astype(np.complex64).astype(np.complex128) if prec == 1 else U.copy()
    for _ in range(3):
        ctx.sd_step(Ug, 0.08)
        Uo = sdfft.sd_step(Uo, 0.08, gauge)
    assert np.abs(host(ctx, Ug) - Uo).max() < (1e-13 if prec == 0 else 5e-6)


def filter_gain(dims, gauge):
    """Largest factor p2max / p^2 the acceleration applies (at the lowest
    nonzero momentum of the longest transformed axis). Rounding differences
    between two transforms of Delta reach X multiplied by it, so a tolerance
    set on lattices of extent <= 14 (gain < 100) scales with gain / 100."""
    axes = dims[:3] if gauge == COULOMB else dims
    p2max = 12.0 if gauge == COULOMB else 16.0
    p2min = min(4 * np.sin(np.pi / L) ** 2 for L in axes)
    return p2max / p2min


@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
@pytest.mark.parametrize("dims", [(384, 2, 2, 2), (2, 1024, 2, 2), (2, 1018, 2, 2), (2, 2, 1022, 2), (2, 2, 2, 1000)])
def test_sd_step_long_axes(gf, field_cache, gauge, dims):
    """One long axis, FP64: tiles at their size limit (x: 384, one site row
    per workgroup; y: 1024 = 4^5, one pencil per workgroup), the direct-sum
    pass of large prime factors (1018 = 2 509, 1022 = 2 7 73) and radix 5
    (1000 = 4 2 5 5 5)."""
    U = field_cache(dims, 0.4, 72)
    ctx, Ug = setup(gf, dims, gauge, 0, U)
    ctx.sd_step(Ug, 0.08)
    Uo = sdfft.sd_step(U.copy(), 0.08, gauge)
    tol = 1e-13 * max(1.0, filter_gain(dims, gauge) / 100)
    assert np.abs(host(ctx, Ug) - Uo).max() < tol


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
@pytest.mark.parametrize("dims", [(46, 2, 2, 2), (2, 34, 2, 2), (2, 2, 26, 2), (2, 2, 2, 22)])
def test_sd_step_prime_factors(gf, field_cache, prec, gauge, dims):
    """Axes with a prime factor above 5 (46 = 2 23, 34 = 2 17, 26 = 2 13,
    22 = 2 11): the direct-sum pass, in both precisions."""
    U = field_cache(dims, 0.4, 73)
    ctx, Ug = setup(gf, dims, gauge, prec, U)
    Uo = U.astype(np.complex64).astype(np.complex128) if prec == 1 else U.copy()
    ctx.sd_step(Ug, 0.08)
    Uo = sdfft.sd_step(Uo, 0.08, gauge)
    tol = (1e-13 if prec == 0 else 5e-6) * max(1.0, filter_gain(dims, gauge) / 100)
    assert np.abs(host(ctx, Ug) - Uo).max() < tol


@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_sd_fix_matches_oracle(gf, oracle_lib, field_cache, gauge):
    dims = (8, 8, 8, 8)
    U = field_cache(dims, 0.3, 0)
    ctx, Ug = setup(gf, dims, gauge, 0, U)
    r = ctx.sd_fix(Ug, 0.08, 1e-12, 3000)
    Uo, ro = sdfft.sd_fix(U.copy(), dims, 0.08, 1e-12, 3000, gauge)
    assert r["converged"] and ro["converged"] and r["theta"] < 1e-12
    assert r["iters"] == ro["iters"], (r, ro)
    assert abs(r["F"] - ro["F"]) < 1e-13
    err = np.abs(host(ctx, Ug) - Uo).max()
    print(f"Alg. 2 gauge {gauge}: iters {r['iters']}, max|dU| {err:.2e}")
    assert err < 1e-12


@pytest.mark.parametrize("storage", [0, 1, 2])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
@pytest.mark.parametrize("check_every,max_iter", [(4, 7), (3, 3), (1, 2)])
def test_sd_fix_equals_repeated_steps(gf, field_cache, storage, prec, gauge, check_every, max_iter):
    """gf_sd_fix, with checks every check_every steps and a last period cut
    by max_iter, returns bitwise the field, F and theta of gf_sd_step
    repeated and a quality evaluation."""
    dims = (6, 4, 4, 8)
    U = field_cache(dims, 0.4, 74)
    c1, U1 = setup(gf, dims, gauge, prec, U, storage=storage, check_every=check_every)
    c2, U2 = setup(gf, dims, gauge, prec, U, storage=storage)
    r = c1.sd_fix(U1, 0.08, 0.0, max_iter)
    for _ in range(max_iter):
        c2.sd_step(U2, 0.08)
    F2, th2 = c2.quality(U2)
    assert r["iters"] == max_iter and not r["converged"]
    assert torch.equal(U1, U2)
    assert r["F"] == F2 and r["theta"] == th2


def test_sd_fft_fp32_reaches_1e7_and_tracks_or(gf, field_cache):
    """Alg. 2 in FP32 reaches theta < 1e-7 and lands on the same maximum as
    overrelaxation (Alg. 1) from the same start."""
    dims = (16, 16, 16, 16)
    U = field_cache(dims, 0.3, 71)
    ctx, Ug = setup(gf, dims, LANDAU, 1, U)
    r = ctx.sd_fix(Ug, 0.08, 1e-7, 5000)
    c2, U2 = setup(gf, dims, LANDAU, 1, U, check_every=10)
    r2 = c2.fix(U2, 1.7, 1e-7, 20000)
    assert r["converged"] and r2["converged"]
    assert r["iters"] < r2["iters"]
    assert abs(r["F"] - r2["F"]) < 1e-5


def test_sd_rejects_bad_alpha(gf, field_cache):
    dims = (4, 4, 4, 4)
    ctx, Ug = setup(gf, dims, LANDAU, 1, field_cache(dims, 0.3, 0))
    for a in (0.0, -0.1, float("nan")):
        with pytest.raises(gf.GFError) as e:
            ctx.sd_step(Ug, a)
        assert e.value.code == gf.EINVAL


@pytest.mark.parametrize("dims", [(386, 2, 2, 2), (2, 1026, 2, 2), (2, 2, 2, 1026)])
def test_sd_rejects_extents_beyond_the_transform_tile(gf, dims):
    """nx above 384 (a tile holds four complex pencils of each site row) or
    another extent above 1024 does not fit one transform tile: refused
    before any kernel runs."""
    ctx = gf.Context(dims, gauge=LANDAU, prec=1)
    U = ctx.empty_field()
    with pytest.raises(gf.GFError) as e:
        ctx.sd_step(U, 0.08)
    assert e.value.code == gf.EUNSUPPORTED
