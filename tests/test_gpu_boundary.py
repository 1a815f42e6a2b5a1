"""GPU checks of the boundary's bookkeeping entry points, through the C ABI:
the per-check JSON-lines log of the fix drivers (gf_params.log_path), the
per-time-slice F_t / theta_t diagnostic (gf_quality_slices) against the
definitions of eqs. (1)-(3) evaluated on the host from the oracle's Delta,
gf_batch_destroy, and the autotuner cache key.

Tolerances: F_t, theta_t 1e-13 relative (same double sums, another order);
the log's F and theta are printed with 17 significant digits, so they read
back bitwise."""
import json

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

LANDAU, COULOMB = 0, 1


@pytest.fixture(scope="module")
def gf():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1412_1498_amd import gf as mod
    return mod


def make_ctx(gf, dims, gauge, prec, **kw):
    return gf.Context(dims, gauge=gauge, prec=prec, params=gf.default_params(prec, **kw))


def to_gpu(ctx, U_np):
    return ctx.pack(torch.from_numpy(np.ascontiguousarray(U_np)).to("cuda", dtype=ctx.cdtype))


def read_log(path):
    with open(path) as fh:
        return [json.loads(line) for line in fh]


@pytest.mark.parametrize("prec", [0, 1])
def test_fix_log_records_every_check(gf, field_cache, tmp_path, prec):
    """check_every 3, max_iter 10: checks after sweeps 0, 3, 6, 9 and 10; the
    last line holds the returned F and theta; a second call is numbered 2."""
    dims = (4, 6, 2, 8)
    U = field_cache(dims, 0.5, 60)
    log = str(tmp_path / "fix.jsonl")
    ctx = make_ctx(gf, dims, LANDAU, prec, check_every=3, reunit_every=4, log_path=log)
    Ug = to_gpu(ctx, U)
    r = ctx.fix(Ug, 1.7, 0.0, 10)
    rows = read_log(log)
    assert [x["sweep"] for x in rows] == [0, 3, 6, 9, 10]
    assert all(x["driver"] == "alg1" and x["call"] == 1 and x["member"] == 0 for x in rows)
    assert rows[-1]["F"] == r["F"] and rows[-1]["theta"] == r["theta"]
    assert all(b["elapsed_s"] >= a["elapsed_s"] for a, b in zip(rows, rows[1:]))
    # the logged values are those of gf_quality at that point
    ctx2 = make_ctx(gf, dims, LANDAU, prec, reunit_every=4)
    U2 = to_gpu(ctx2, U)
    ctx2.sweeps(U2, 1.7, 3)
    F3, th3 = ctx2.quality(U2)
    assert (rows[1]["F"], rows[1]["theta"]) == (F3, th3)
    r2 = ctx.fix(Ug, 1.7, 1e30, 10)  # converged at once: one line, sweep 0
    rows = read_log(log)
    assert len(rows) == 6 and rows[-1]["call"] == 2 and rows[-1]["sweep"] == 0 and r2["iters"] == 0


def test_batch_fix_log_stops_per_member(gf, field_cache, tmp_path):
    """An ensemble whose members converge at different checks: each member
    is logged at every check until (and including) the one that retired it."""
    members = [((4, 4, 4, 4), LANDAU, 0.3, 61), ((6, 4, 4, 4), COULOMB, 0.5, 62), ((4, 4, 2, 6), LANDAU, 0.6, 63)]
    log = str(tmp_path / "batch.jsonl")
    ens = gf.Context(None, prec=0, params=gf.default_params(0, check_every=5, log_path=log),
                     ensemble=[(d, g) for d, g, _, _ in members])
    Us = []
    for d, g, amp, seed in members:
        c1 = make_ctx(gf, d, g, 0)
        Us.append(to_gpu(c1, field_cache(d, amp, seed)))
    r = ens.batch_fix(Us, 1.7, 1e-10, 2000)
    assert r["converged"]
    rows = read_log(log)
    for i in range(len(members)):
        mine = [x for x in rows if x["member"] == i]
        sweeps = [x["sweep"] for x in mine]
        assert sweeps == list(range(0, r["iters"][i] + 1, 5)), (i, sweeps[-3:], r["iters"][i])
        assert mine[-1]["theta"] == r["theta"][i] and mine[-1]["theta"] < 1e-10
        assert all(x["theta"] >= 1e-10 for x in mine[:-1])
    assert len(set(r["iters"])) > 1  # the members did stop at different checks
    ens.close()  # gf_batch_destroy


def test_sd_fix_log(gf, field_cache, tmp_path):
    dims = (4, 4, 4, 4)
    U = field_cache(dims, 0.3, 64)
    log = str(tmp_path / "sd.jsonl")
    ctx = make_ctx(gf, dims, LANDAU, 0, check_every=2, log_path=log)
    Ug = to_gpu(ctx, U)
    r = ctx.sd_fix(Ug, 0.08, 0.0, 5)
    rows = read_log(log)
    assert [x["step"] for x in rows] == [0, 2, 4, 5]
    assert all(x["driver"] == "alg2" for x in rows)
    assert rows[-1]["F"] == r["F"] and rows[-1]["theta"] == r["theta"]


def slice_reference(oracle_lib, U, dims, gauge):
    """F_t and theta_t from the definitions: per-site Re Tr of the
    functional's links and Tr Delta Delta^dagger with the oracle's Delta
    (eq. 3), summed over each time slice and normalised by its volume."""
    nx, ny, nz, nt = dims
    nd = 3 if gauge == COULOMB else 4
    Vt = nx * ny * nz
    tr = np.einsum("tzyxmii->tzyxm", U[..., :nd, :, :]).real.sum(axis=(1, 2, 3, 4))
    D = oracle_lib.divergence_field(np.ascontiguousarray(U), dims, gauge).reshape(nt, Vt, 3, 3)
    th = (np.abs(D) ** 2).sum(axis=(1, 2, 3))
    return tr / (nd * 3 * Vt), th / (3 * Vt)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
@pytest.mark.parametrize("dims", [(4, 6, 2, 8), (8, 8, 8, 4), (6, 10, 6, 6), (2, 2, 2, 2), (16, 16, 18, 4)])
def test_quality_slices_match_definition(gf, oracle_lib, field_cache, prec, gauge, dims):
    """Slices of 24, 256, 180, 4 and 2304 half sites per parity (tiles of 128:
    ragged, exact, ragged, one partial tile, several tiles)."""
    U = field_cache(dims, 0.6, 65)
    ctx = make_ctx(gf, dims, gauge, prec)
    Ug = to_gpu(ctx, U)
    ctx.sweeps(Ug, 1.7, 2)
    Uh = ctx.unpack(Ug).cpu().numpy().astype(np.complex128)
    Ft, tht = ctx.quality_slices(Ug)
    Fr, thr = slice_reference(oracle_lib, Uh, dims, gauge)
    np.testing.assert_allclose(Ft, Fr, rtol=1e-13, atol=0)
    np.testing.assert_allclose(tht, thr, rtol=1e-13, atol=0)
    F, th = ctx.quality(Ug)
    assert abs(np.mean(Ft) - F) <= 1e-13 * abs(F) and abs(np.mean(tht) - th) <= 1e-13 * th


def test_quality_slices_coulomb_fixed_slices(gf, field_cache):
    """After Coulomb gauge fixing to theta < 1e-10 every slice is fixed:
    theta_t < nt * 1e-10 on each and their mean is the global theta."""
    dims = (4, 4, 4, 6)
    U = field_cache(dims, 0.4, 66)
    ctx = make_ctx(gf, dims, COULOMB, 0)
    Ug = to_gpu(ctx, U)
    r = ctx.fix(Ug, 1.7, 1e-10, 3000)
    assert r["converged"]
    _, tht = ctx.quality_slices(Ug)
    assert max(tht) < dims[3] * 1e-10
    assert abs(np.mean(tht) - r["theta"]) <= 1e-12 * r["theta"]


def test_quality_slices_rejects_bad_arguments(gf, field_cache):
    dims = (4, 4, 4, 4)
    ctx = make_ctx(gf, dims, LANDAU, 0)
    Ug = to_gpu(ctx, field_cache(dims, 0.3, 67))
    import ctypes
    arr = (ctypes.c_double * 4)()
    assert gf.lib.gf_quality_slices(ctx._h, ctypes.c_void_p(Ug.data_ptr()), None, arr) == gf.EINVAL
    assert gf.lib.gf_quality_slices(ctx._h, None, arr, arr) == gf.EINVAL
    c4 = gf.Context(dims, prec=0, nc=4)
    U4 = c4.empty_field()
    assert gf.lib.gf_quality_slices(c4._h, ctypes.c_void_p(U4.data_ptr()), arr, arr) == gf.EUNSUPPORTED


def test_autotune_cache_keys_separate_colour_numbers(gf, tmp_path):
    """An SU(2) context and an SU(3) 8-real context (both four stored complex
    values per link) on the same lattice and precision get cache lines of
    their own, and the key names the library's sources."""
    from paper_1412_1498_amd import synth
    dims = (8, 8, 8, 8)
    cache = str(tmp_path / "tune.txt")
    c2 = gf.Context(dims, prec=1, nc=2)
    U2 = c2.pack(synth.random_sun_field(dims, 2, 0.5, 0, device="cuda").to(torch.complex64))
    c2.autotune([U2], 1.7, cache)
    c8 = gf.Context(dims, prec=1, params=gf.default_params(1, storage=gf.STORE_8))
    U8 = c8.pack(synth.random_gauge_field(dims, 0.5, 0, device="cuda").to(torch.complex64))
    c8.autotune([U8], 1.7, cache)
    lines = open(cache).read().splitlines()
    assert len(lines) == 2
    keys = [ln.split(" ")[0] for ln in lines]
    assert keys[0] != keys[1] and "|n2|" in keys[0] and "|n3|" in keys[1]
    assert all("|src" in k and "|srcunknown|" not in k for k in keys)
