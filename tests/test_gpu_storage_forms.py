"""The differentiation calls and steepest descent with Fourier acceleration on
compressed links (12-real and 8-real storage), against the FP64 oracle given
the GPU's own field as unpacked (the links the kernels read).

Tolerances are those of the 18-real tests (tests/test_gpu_diff.py,
tests/test_gpu_sdfft.py); links written back in compressed form also carry
the format's rounding, bounded per link as in tests/test_gpu_link8.py
(8 u kappa; for 12-real kappa = 1, the rebuilt row)."""
import numpy as np
import pytest
import torch

from oracle import diff, sdfft

pytestmark = pytest.mark.gpu

LANDAU, COULOMB = 0, 1
U64, U32 = 2.0 ** -53, 2.0 ** -24


@pytest.fixture(scope="module")
def gf():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1412_1498_amd import gf as mod
    return mod


def setup(gf, dims, gauge, prec, storage, U):
    ctx = gf.Context(dims, gauge=gauge, prec=prec, params=gf.default_params(prec, storage=storage))
    Ug = ctx.pack(torch.from_numpy(np.ascontiguousarray(U)).to("cuda", dtype=ctx.cdtype))
    return ctx, Ug


def host(ctx, Ug):
    return ctx.unpack(Ug).cpu().numpy().astype(np.complex128)


def link_bound(ref, prec, storage, base):
    u = U32 if prec == 1 else U64
    if storage == 1:
        return base + 8 * u
    a = np.abs(ref)
    n2 = a[..., 0, 1] ** 2 + a[..., 0, 2] ** 2
    with np.errstate(divide="ignore"):
        kappa = 1 + 1 / a[..., 0, 0] + 1 / a[..., 2, 0] + 1 / np.sqrt(n2)
    return base + 8 * u * kappa


def check_links(got, ref, prec, storage, base):
    err = np.abs(got - ref).max(axis=(-1, -2))
    bound = link_bound(ref, prec, storage, base)
    assert (err <= bound).all(), (err[err > bound][:5], bound[err > bound][:5])


@pytest.mark.parametrize("storage", [1, 2])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_functional_and_gradient(gf, field_cache, storage, prec, gauge):
    from paper_1412_1498_amd import synth
    dims = (6, 4, 2, 8)
    U = field_cache(dims, 0.4, 30)
    s = synth.random_algebra_field(dims, 0.1, 31).numpy()
    ctx, Ug = setup(gf, dims, gauge, prec, storage, U)
    sg = ctx.pack_alg(torch.from_numpy(np.ascontiguousarray(s)).to("cuda", dtype=ctx.rdtype))
    Uo = host(ctx, Ug)
    so = s.astype(np.float32).astype(np.float64) if prec == 1 else s
    F = ctx.functional(Ug, sg)
    Fo = diff.functional(Uo, so, gauge)
    assert abs(F - Fo) <= (1e-13 if prec == 0 else 2e-6) * abs(Fo)
    grad = ctx.unpack_alg(ctx.functional_grad(Ug, sg)).cpu().numpy().astype(np.float64)
    go = diff.gradient(Uo, so, gauge)
    assert np.abs(grad - go).max() <= (1e-12 if prec == 0 else 1e-4) * np.abs(go).max()


@pytest.mark.parametrize("storage", [1, 2])
@pytest.mark.parametrize("prec", [0, 1])
def test_gauge_transform(gf, field_cache, storage, prec):
    from paper_1412_1498_amd import synth
    dims = (4, 4, 4, 4)
    U = field_cache(dims, 0.5, 32)
    s = synth.random_algebra_field(dims, 0.3, 33).numpy()
    ctx, Ug = setup(gf, dims, LANDAU, prec, storage, U)
    sg = ctx.pack_alg(torch.from_numpy(np.ascontiguousarray(s)).to("cuda", dtype=ctx.rdtype))
    Uo = host(ctx, Ug)
    so = s.astype(np.float32).astype(np.float64) if prec == 1 else s
    ctx.gauge_transform(Ug, sg)
    ref = diff.transform(Uo, diff.gauge_fields(so))
    check_links(host(ctx, Ug), ref, prec, storage, 1e-13 if prec == 0 else 5e-6)


@pytest.mark.parametrize("storage", [1, 2])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_sd_steps(gf, field_cache, storage, prec, gauge):
    dims = (4, 6, 2, 8)
    U = field_cache(dims, 0.4, 70)
    ctx, Ug = setup(gf, dims, gauge, prec, storage, U)
    for _ in range(3):
        cur = host(ctx, Ug)
        ctx.sd_step(Ug, 0.08)
        check_links(host(ctx, Ug), sdfft.sd_step(cur, 0.08, gauge), prec, storage,
                    1e-13 if prec == 0 else 5e-6)


def test_full_size_48_fp32_12real_sampled_sites(gf, oracle_lib):
    """48^4, amp 0.7, FP32 12-real links, the bench's default schedule: F and
    theta of the whole field (row 2 rebuilt) equal the oracle's (F 1e-11
    absolute, theta 1e-10 relative: the oracle's sequential sums); after one
    even half-sweep the eight links of 128 sampled even sites equal the
    oracle's single-site update of the same links, within the FP32 sweep
    tolerance plus the rebuilt row's rounding (8 u)."""
    from paper_1412_1498_amd import synth
    dims = (48, 48, 48, 48)
    U = synth.random_gauge_field(dims, 0.7, 0, device="cuda").to(torch.complex64)
    ctx = gf.Context(dims, gauge=LANDAU, prec=1, params=gf.default_params(1, storage=1))
    Ug = ctx.pack(U)
    del U
    Uo = host(ctx, Ug)
    F0, th0 = ctx.quality(Ug)
    Fo, tho = oracle_lib.quality(Uo, dims, LANDAU)
    assert abs(F0 - Fo) <= 1e-11 and abs(th0 - tho) <= 1e-10 * tho
    ctx.sweep(Ug, 0, 1.7)
    back = host(ctx, Ug).reshape(-1, 4, 3, 3)
    V = 48 ** 4
    par = oracle_lib.parity_of_sites(dims)
    rng = np.random.default_rng(0)
    sites = [int(s) for s in rng.choice(V, 400, replace=False) if par[s] == 0][:128]
    for s in sites:
        oracle_lib.site_update(Uo, dims, s, 1.7)
    O = Uo.reshape(-1, 4, 3, 3)
    got, ref = [], []
    for s in sites:
        x, y, z, t = s % 48, (s // 48) % 48, (s // 48 ** 2) % 48, s // 48 ** 3
        idx = [(s, mu) for mu in range(4)]
        for mu, (c, step) in enumerate(zip((x, y, z, t), (1, 48, 48 ** 2, 48 ** 3))):
            idx.append((s - step if c > 0 else s + 47 * step, mu))
        for i, mu in idx:
            got.append(back[i, mu])
            ref.append(O[i, mu])
    check_links(np.array(got), np.array(ref), 1, 1, 5e-6)
