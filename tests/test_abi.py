"""CPU-only checks of the C ABI library: it loads, exports every symbol the
header declares, validates arguments before touching a device, and its
host-callable pieces (index math, the SU(2) step and the trig it uses) agree
with independent definitions. No kernel is launched here."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def gf():
    from paper_1412_1498_amd import gf as mod
    return mod


def header_functions():
    txt = open(os.path.join(ROOT, "include", "gf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gf_\w+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(gf):
    names = header_functions()
    assert len(names) >= 25
    lib = ctypes.CDLL(gf.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_invalid_arguments_fail_before_device_use(gf):
    h = ctypes.c_void_p()
    p = gf.default_params(gf.F32)
    for dims in [(3, 4, 4, 4), (4, 4, 4, 0), (4, 4, 5, 4), (4, -2, 4, 4)]:
        rc = gf.lib.gf_create(ctypes.byref(h), gf._dims_arr(dims), 3, 0, gf.F32, None, ctypes.byref(p))
        assert rc == gf.EINVAL and not h.value
    # the largest lattice: 4V link indices must fit 31 bits
    for dims in [(256, 256, 256, 128), (2, 2, 2, 1 << 28)]:
        rc = gf.lib.gf_create(ctypes.byref(h), gf._dims_arr(dims), 3, 0, gf.F32, None, ctypes.byref(p))
        assert rc == gf.EINVAL and not h.value
    for nc in (1, 5, 8):
        assert gf.lib.gf_create(ctypes.byref(h), gf._dims_arr((4, 4, 4, 4)), nc, 0, gf.F32, None,
                                ctypes.byref(p)) == gf.EUNSUPPORTED
    # 12-real storage is SU(3) only; SU(4) links need two or more lanes per site
    p12 = gf.default_params(gf.F32, storage=gf.STORE_12)
    assert gf.lib.gf_create(ctypes.byref(h), gf._dims_arr((4, 4, 4, 4)), 4, 0, gf.F32, None,
                            ctypes.byref(p12)) == gf.EUNSUPPORTED
    p1 = gf.default_params(gf.F32, lanes_per_site=1)
    assert gf.lib.gf_create(ctypes.byref(h), gf._dims_arr((4, 4, 4, 4)), 4, 0, gf.F32, None,
                            ctypes.byref(p1)) == gf.EINVAL
    assert gf.lib.gf_create(ctypes.byref(h), gf._dims_arr((4, 4, 4, 4)), 3, 5, gf.F32, None,
                            ctypes.byref(p)) == gf.EINVAL
    assert gf.lib.gf_create(ctypes.byref(h), gf._dims_arr((4, 4, 4, 4)), 3, 0, 7, None,
                            ctypes.byref(p)) == gf.EINVAL
    bad = gf.default_params(gf.F32, lanes_per_site=3)
    assert gf.lib.gf_create(ctypes.byref(h), gf._dims_arr((4, 4, 4, 4)), 3, 0, gf.F32, None,
                            ctypes.byref(bad)) == gf.EINVAL
    bad = gf.default_params(gf.F32, block_threads=100)
    assert gf.lib.gf_create(ctypes.byref(h), gf._dims_arr((4, 4, 4, 4)), 3, 0, gf.F32, None,
                            ctypes.byref(bad)) == gf.EINVAL
    bad = gf.default_params(gf.F32, tile_order=2)
    assert gf.lib.gf_create(ctypes.byref(h), gf._dims_arr((4, 4, 4, 4)), 3, 0, gf.F32, None,
                            ctypes.byref(bad)) == gf.EINVAL
    # every entry point tolerates a NULL context
    assert gf.lib.gf_destroy(None) == gf.OK
    assert gf.lib.gf_sweep(None, None, 0, 1.7) == gf.EINVAL
    assert gf.lib.gf_quality(None, None, None, None) == gf.EINVAL


def canonical_halfindex(dims, x, y, z, t):
    nx, ny, nz, nt = dims
    return (x + nx * (y + ny * (z + nz * t))) // 2


def layout_offset(dims, mu, p, h, ne=9):
    """Element-0 offset of U_mu at site (p, h) in the documented blocked layout."""
    Vh = dims[0] * dims[1] * dims[2] * dims[3] // 2
    nb = (Vh + 63) // 64
    return (((p * nb + h // 64) * 4 + mu) * ne) * 64 + h % 64


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (4, 6, 2, 8), (6, 2, 4, 2), (8, 4, 6, 4),
                                  (10, 6, 4, 2)])
def test_half_sweep_touches_every_link_once(gf, dims):
    """The kernel's index math (the same inline function, run on the host):
    over the sites of one parity the eight links form a permutation of all
    4V links, and each is the link that the layout assigns to U_mu(x) or
    U_mu(x - mu)."""
    nx, ny, nz, nt = dims
    V = nx * ny * nz * nt
    all_links = {layout_offset(dims, mu, p, h) for mu in range(4) for p in (0, 1) for h in range(V // 2)}
    assert len(all_links) == 4 * V
    for p in (0, 1):
        seen = []
        sites = [(x, y, z, t) for t in range(nt) for z in range(nz) for y in range(ny) for x in range(nx)
                 if (x + y + z + t) % 2 == p]
        for (x, y, z, t) in sites:
            h = canonical_halfindex(dims, x, y, z, t)
            offs = gf.site_links(dims, p, h)
            c = [x, y, z, t]
            for mu in range(4):
                assert offs[mu] == layout_offset(dims, mu, p, h)
                b = list(c)
                b[mu] = (b[mu] - 1) % dims[mu]
                assert offs[4 + mu] == layout_offset(dims, mu, 1 - p, canonical_halfindex(dims, *b))
            seen += offs
        assert sorted(seen) == sorted(all_links)


def test_kernel_trig_matches_libm(gf):
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.uniform(0, 2 * math.pi, 20000),
                         [0.0, math.pi / 4, math.pi / 2, math.pi, 1.5 * math.pi, 2 * math.pi - 1e-12,
                          2 * math.pi]])
    err_s = err_c = 0.0
    for x in xs:
        s, c, _ = gf.host_trig(x, 1.0)
        err_s = max(err_s, abs(s - math.sin(x)))
        err_c = max(err_c, abs(c - math.cos(x)))
    assert err_s < 4e-16 and err_c < 4e-16
    err_a = 0.0
    for _ in range(20000):
        y, x = rng.standard_normal(2) * 10 ** rng.uniform(-3, 3, 2)
        a = gf.host_trig(x, y)[2]
        err_a = max(err_a, abs(a - math.atan2(y, x)) / max(1.0, abs(math.atan2(y, x))))
    for y, x in [(0, 1), (0, -1), (1, 0), (1, 1), (1, -1), (0, 0), (1e-300, 1), (1, 1e-300)]:
        assert abs(gf.host_trig(x, y)[2] - math.atan2(y, x)) < 4e-16
    assert err_a < 4e-16


def test_kernel_su2_step_matches_oracle(gf, oracle_lib):
    """The sweep kernels' SU(2) step (unnormalised, atan2/sincos form) equals
    the oracle's eq.-(6)-then-power form to rounding."""
    rng = np.random.default_rng(1)
    for _ in range(5000):
        b = rng.standard_normal(4) * 10 ** rng.uniform(-2, 2)
        w = rng.choice([1.0, 1.5, 1.7, 1.9, rng.uniform(0, 2)])
        np.testing.assert_allclose(gf.host_su2_step(b, w), oracle_lib.su2_solve(b, w), atol=2e-15)
    for b in ([0, 0, 0, 0], [-2.0, 0, 0, 0], [3.0, 0, 0, 0], [0, 1e-30, 0, 0], [-1, 0, 1e-300, 0]):
        np.testing.assert_allclose(gf.host_su2_step(b, 1.7), oracle_lib.su2_solve(np.array(b, float), 1.7),
                                   atol=1e-15)
