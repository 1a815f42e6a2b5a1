"""gf_quality_noalloc (F and theta with no context and no allocation, for
callers that cannot allocate) through the C ABI, against gf_quality on the
same fields: the two share the reduction's tiles, order and normalisation, so
the results must be bitwise equal -- also where the context path takes the
tiles in another order (2-d column blocks) or walks them slice by slice
(double, Landau and Coulomb). Calls in a row, each later one on a smaller
lattice (the fixed scratch keeps the earlier call's partials), in both
precisions and all three storage forms, including the 48^4 FP32 field of the
benchmark; plus the size limit and argument errors."""
import ctypes

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


def noalloc(gf, U, dims, gauge, prec, storage, out):
    d = (ctypes.c_int * 4)(*dims)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return gf.lib.gf_quality_noalloc(ctypes.c_void_p(U.data_ptr()), d, gauge, prec, storage, st,
                                     ctypes.c_void_p(out.data_ptr()))


def field(gf, dims, gauge, prec, storage, amp, seed):
    from paper_1412_1498_amd import synth
    ctx = gf.Context(dims, gauge=gauge, prec=prec, params=gf.default_params(prec, storage=storage))
    U = ctx.pack(synth.random_gauge_field(dims, amp, seed, device="cuda").to(ctx.cdtype))
    ctx.sweeps(U, 1.7, 1)  # a field that is not the generator's output itself
    return ctx, U


@pytest.mark.parametrize("storage", [0, 1, 2])
@pytest.mark.parametrize("prec", [0, 1])
def test_two_calls_match_gf_quality(gf, prec, storage):
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    # (16, 16, 8, 14) Landau: in double the context path walks the 14 time
    # slices in runs of 5, 5 and 4, passing t links between lanes
    for dims, gauge, seed in (((16, 16, 16, 24), COULOMB, 1), ((16, 16, 8, 14), LANDAU, 3),
                              ((6, 4, 4, 2), LANDAU, 2)):
        ctx, U = field(gf, dims, gauge, prec, storage, 0.6, seed)
        assert noalloc(gf, U, dims, gauge, prec, storage, out) == gf.OK, gf.lib.gf_last_error(None)
        got = tuple(out.cpu().tolist())
        ref = ctx.quality(U)
        print(dims, prec, storage, got, ref)
        assert got == ref, (dims, got, ref)


def test_benchmark_field_then_small(gf):
    """The 48^4 FP32 field in the benchmark's configuration, then a 4^4 one."""
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    for dims, gauge in (((48, 48, 48, 48), LANDAU), ((4, 4, 4, 4), COULOMB)):
        ctx, U = field(gf, dims, gauge, 1, 0, 0.7, 0)
        assert noalloc(gf, U, dims, gauge, 1, 0, out) == gf.OK
        got = tuple(out.cpu().tolist())
        assert got == ctx.quality(U), dims
        del ctx, U
        torch.cuda.empty_cache()


def test_no_device_memory_is_taken(gf):
    dims = (8, 8, 8, 8)
    ctx, U = field(gf, dims, LANDAU, 0, 0, 0.5, 3)
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    assert noalloc(gf, U, dims, LANDAU, 0, 0, out) == gf.OK
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(5):
        assert noalloc(gf, U, dims, LANDAU, 0, 0, out) == gf.OK
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert tuple(out.cpu().tolist()) == ctx.quality(U)


def test_limits_and_bad_arguments(gf):
    U = torch.zeros(64, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    # 2^24 sites is the largest lattice (65536 tiles); one more time slice is refused
    assert noalloc(gf, U, (256, 256, 16, 18), LANDAU, 1, 0, out) == gf.EINVAL
    assert b"allocation-free limit" in gf.lib.gf_last_error(None)
    for dims in ((3, 4, 4, 4), (4, 4, 4, 0)):
        assert noalloc(gf, U, dims, LANDAU, 1, 0, out) == gf.EINVAL
    assert noalloc(gf, U, (4, 4, 4, 4), 2, 1, 0, out) == gf.EINVAL
    assert noalloc(gf, U, (4, 4, 4, 4), LANDAU, 2, 0, out) == gf.EINVAL
    assert noalloc(gf, U, (4, 4, 4, 4), LANDAU, 1, 3, out) == gf.EINVAL
    d = (ctypes.c_int * 4)(4, 4, 4, 4)
    assert gf.lib.gf_quality_noalloc(ctypes.c_void_p(U.data_ptr()), d, 0, 1, 0, None, None) == gf.EINVAL
    assert gf.lib.gf_quality_noalloc(None, d, 0, 1, 0, None, ctypes.c_void_p(out.data_ptr())) == gf.EINVAL
