"""GPU parity of the 8-real link storage (GF_STORE_8) against the FP64 oracle.

The kernels read a link by reconstructing it from U01, U02, U10 and two
phases, and write it by compressing it again; unpack reconstructs the same
way. So the oracle is given the GPU's unpacked field, and the GPU result is
compared with the oracle's on it with a per-link bound: the storage
precision's usual half-sweep tolerance plus 8 u kappa, kappa = 1 + 1/|U00| +
1/|U20| + 1/sqrt(|U01|^2 + |U02|^2) of the oracle's link (the format's
conditioning, pinned on the host in tests/test_link8.py)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

LANDAU, COULOMB = 0, 1
STORE_8 = 2
U64, U32 = 2.0 ** -53, 2.0 ** -24


@pytest.fixture(scope="module")
def gf():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1412_1498_amd import gf as mod
    return mod


def make_ctx(gf, dims, gauge, prec, **kw):
    return gf.Context(dims, gauge=gauge, prec=prec, params=gf.default_params(prec, storage=STORE_8, **kw))


def to_gpu(ctx, U):
    return ctx.pack(torch.from_numpy(np.ascontiguousarray(U)).to("cuda", dtype=ctx.cdtype))


def to_host(ctx, U):
    return ctx.unpack(U).cpu().numpy().astype(np.complex128)


def link_bound(ref, prec, base):
    """Per-link tolerance for links ref (..., 3, 3)."""
    u = U32 if prec == 1 else U64
    a = np.abs(ref)
    n2 = a[..., 0, 1] ** 2 + a[..., 0, 2] ** 2
    with np.errstate(divide="ignore"):
        kappa = 1 + 1 / a[..., 0, 0] + 1 / a[..., 2, 0] + 1 / np.sqrt(n2)
    return base + 8 * u * kappa


def check(got, ref, prec, base):
    err = np.abs(got - ref).max(axis=(-1, -2))
    bound = link_bound(ref, prec, base)
    bad = err > bound
    assert not bad.any(), (err[bad][:5], bound[bad][:5])


@pytest.mark.parametrize("prec", [0, 1])
def test_pack_unpack_is_the_host_format(gf, field_cache, prec):
    dims = (4, 6, 2, 8)
    U = field_cache(dims, 0.5, 1)
    ctx = make_ctx(gf, dims, LANDAU, prec)
    back = to_host(ctx, to_gpu(ctx, U))
    src = U.astype(np.complex64).astype(np.complex128) if prec == 1 else U
    check(back, src, prec, 0.0)
    # the host round trip runs the same code (the float GPU path takes the
    # hardware reciprocal and square root, about 1 ulp, where the host
    # rounds correctly), so the two agree to the format's own bound
    flat_b, flat_u = back.reshape(-1, 3, 3), U.reshape(-1, 3, 3)
    for i in range(0, flat_u.shape[0], 97):
        _, host = gf.host_link8(prec, flat_u[i])
        check(flat_b[i], host, prec, 0.0)
        if prec == 0:
            assert np.abs(flat_b[i] - host).max() <= 4 * U64


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
@pytest.mark.parametrize("lps", [1, 2, 4, 8])
def test_half_sweeps_match_oracle(gf, oracle_lib, field_cache, prec, gauge, lps):
    dims = (4, 6, 2, 8)
    U = field_cache(dims, 0.7, 4)
    ctx = make_ctx(gf, dims, gauge, prec, lanes_per_site=lps)
    Ug = to_gpu(ctx, U)
    base = 1e-13 if prec == 0 else 5e-6
    for p in (0, 1, 0, 1):
        cur = to_host(ctx, Ug)
        ctx.sweep(Ug, p, 1.7)
        oracle_lib.half_sweep(cur, dims, p, 1.7, gauge)
        check(to_host(ctx, Ug), cur, prec, base)


@pytest.mark.parametrize("prec", [0, 1])
def test_all_schedules_give_identical_bits(gf, field_cache, prec):
    dims = (8, 4, 6, 4)
    U = field_cache(dims, 0.6, 5)
    ref = None
    for lps in (1, 2, 4, 8):
        for block in (64, 128, 256):
            for nt, order in ((0, 0), (1, 1)):
                ctx = make_ctx(gf, dims, LANDAU, prec, lanes_per_site=lps, block_threads=block,
                               nontemporal=nt, tile_order=order, reunit_every=2)
                Ug = to_gpu(ctx, U)
                ctx.sweeps(Ug, 1.7, 3)
                if ref is None:
                    ref = Ug.clone()
                else:
                    assert torch.equal(Ug, ref), (lps, block, nt, order)


@pytest.mark.parametrize("prec", [0, 1])
def test_quality_matches_oracle(gf, oracle_lib, field_cache, prec):
    dims = (8, 6, 8, 8)
    U = field_cache(dims, 0.6, 6)
    for gauge in (LANDAU, COULOMB):
        ctx = make_ctx(gf, dims, gauge, prec)
        Ug = to_gpu(ctx, U)
        F, th = ctx.quality(Ug)
        Fo, tho = oracle_lib.quality(to_host(ctx, Ug), dims, gauge)
        assert abs(F - Fo) <= 1e-13 and abs(th - tho) <= 1e-13 * tho


def test_fp32_fix_reaches_target_and_tracks_fp64(gf, oracle_lib, field_cache):
    """Alg. 1 on 8-real FP32 links to theta < 1e-7 lands on the F of the
    FP64 oracle's run from the same field (full storage) within 1e-5."""
    dims = (8, 8, 8, 8)
    U = field_cache(dims, 0.5, 7)
    ctx = make_ctx(gf, dims, LANDAU, 1, check_every=10, reunit_every=10)
    r = ctx.fix(to_gpu(ctx, U), 1.7, 1e-7, 5000)
    ro = oracle_lib.fix(U.copy(), dims, 1.7, 1e-7, 5000, LANDAU, reunit_every=10, check_every=10)
    assert r["converged"] and ro["converged"]
    assert abs(r["F"] - ro["F"]) < 1e-5


def test_batch_fix_equals_single_fix(gf, field_cache):
    members = [((4, 4, 4, 4), LANDAU, 0.3, 10), ((6, 4, 4, 2), COULOMB, 0.4, 11), ((8, 8, 8, 8), LANDAU, 0.5, 12)]
    kw = dict(check_every=4, reunit_every=10, use_graph=1)
    ens = gf.Context(None, prec=1, params=gf.default_params(1, storage=STORE_8, **kw),
                     ensemble=[(d, g) for d, g, _, _ in members])
    Us = [to_gpu(make_ctx(gf, d, g, 1), field_cache(d, amp, seed)) for d, g, amp, seed in members]
    singles = [u.clone() for u in Us]
    rb = ens.batch_fix(Us, 1.7, 1e-7, 3000)
    assert rb["converged"]
    for i, (d, g, _, _) in enumerate(members):
        c1 = make_ctx(gf, d, g, 1, **kw)
        r1 = c1.fix(singles[i], 1.7, 1e-7, 3000)
        assert r1["iters"] == rb["iters"][i] and r1["theta"] == rb["theta"][i]
        assert torch.equal(singles[i], Us[i])


def test_full_size_48_fp32_sampled_sites(gf, oracle_lib):
    """48^4, amp 0.7, FP32 8-real links, default schedule: F and theta of the
    whole (reconstructed) field equal the oracle's (F 1e-11 absolute, theta
    1e-10 relative: the oracle's sequential sums); after one even half-sweep
    the eight links of 128 sampled even sites equal the oracle's single-site
    update of the same reconstructed links."""
    from paper_1412_1498_amd import synth
    dims = (48, 48, 48, 48)
    U = synth.random_gauge_field(dims, 0.7, 0, device="cuda").to(torch.complex64)
    ctx = make_ctx(gf, dims, LANDAU, 1)
    Ug = ctx.pack(U)
    del U
    Uo = to_host(ctx, Ug)
    F0, th0 = ctx.quality(Ug)
    Fo, tho = oracle_lib.quality(Uo, dims, LANDAU)
    assert abs(F0 - Fo) <= 1e-11 and abs(th0 - tho) <= 1e-10 * tho
    ctx.sweep(Ug, 0, 1.7)
    back = to_host(ctx, Ug).reshape(-1, 4, 3, 3)
    V = 48 ** 4
    par = oracle_lib.parity_of_sites(dims)
    rng = np.random.default_rng(0)
    sites = [int(s) for s in rng.choice(V, 400, replace=False) if par[s] == 0][:128]
    for s in sites:
        oracle_lib.site_update(Uo, dims, s, 1.7)
    O = Uo.reshape(-1, 4, 3, 3)
    for s in sites:
        x, y, z, t = s % 48, (s // 48) % 48, (s // 48 ** 2) % 48, s // 48 ** 3
        idx = [(s, mu) for mu in range(4)]
        for mu, (c, step) in enumerate(zip((x, y, z, t), (1, 48, 48 ** 2, 48 ** 3))):
            idx.append((s - step if c > 0 else s + 47 * step, mu))
        for i, mu in idx:
            check(back[i, mu], O[i, mu], 1, 5e-6)


@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
@pytest.mark.parametrize("amp", [0.3, 0.0])
def test_fp64_fix_to_1e12_matches_oracle(gf, oracle_lib, field_cache, gauge, amp):
    """Alg. 1 in FP64 on 8-real links to theta < 1e-12 (4^4, seed 0; amp 0.3
    as the small FP64 case, and amp 0, a pure gauge whose fixed links are
    the unit matrix, where the format's u/eps behaviour near 1 shows): the
    run converges and lands on the oracle's F and field, the oracle started
    from the GPU's reconstructed field."""
    dims = (4, 4, 4, 4)
    U = field_cache(dims, amp, 0)
    ctx = make_ctx(gf, dims, gauge, 0, reunit_every=20)
    Ug = to_gpu(ctx, U)
    Uo = to_host(ctx, Ug)
    r = ctx.fix(Ug, 1.7, 1e-12, 2000)
    ro = oracle_lib.fix(Uo, dims, 1.7, 1e-12, 2000, gauge, reunit_every=20)
    got = to_host(ctx, Ug)
    err = np.abs(got - Uo).max()
    print(f"amp {amp} gauge {gauge}: iters {r['iters']} (oracle {ro['iters']}), theta {r['theta']:.2e}, "
          f"|dF| {abs(r['F'] - ro['F']):.1e}, max|dU| {err:.1e}")
    assert r["converged"] and ro["converged"] and r["theta"] < 1e-12
    assert r["iters"] == ro["iters"]
    assert abs(r["F"] - ro["F"]) < 1e-12
    assert err < 1e-12  # measured 8e-14 .. 1.2e-13
    if amp == 0.0:
        assert abs(r["F"] - 1) < 1e-12


def degenerate_links(rng, n):
    """n SU(3) links with U01 = U02 = 0: diag(a) and a U(2) block of
    determinant conj(a) (a few exactly diagonal ones among them)."""
    out = np.zeros((n, 3, 3), dtype=np.complex128)
    for k in range(n):
        a = np.exp(1j * rng.uniform(-np.pi, np.pi))
        z = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        if k % 7 == 0:
            z[1] = 0
        z /= np.linalg.norm(z)
        out[k, 0, 0] = a
        out[k, 1:, 1:] = [[z[0], z[1]], [-np.conj(a * z[1]), np.conj(a * z[0])]]
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_links_without_off_diagonal_row0(gf, oracle_lib, prec):
    """Every link with U01 = U02 = 0 exactly: the field packs and unpacks to
    itself (U11 and the phase of U12 take the free slots), and half-sweeps
    from it follow the oracle."""
    dims = (4, 4, 2, 2)
    V = int(np.prod(dims))
    U = degenerate_links(np.random.default_rng(8), 4 * V).reshape(dims[3], dims[2], dims[1], dims[0], 4, 3, 3)
    ctx = make_ctx(gf, dims, LANDAU, prec)
    Ug = to_gpu(ctx, U)
    back = to_host(ctx, Ug)
    src = U.astype(np.complex64).astype(np.complex128) if prec == 1 else U
    u = U32 if prec == 1 else U64
    b = np.abs(src[..., 1, 2])
    with np.errstate(divide="ignore"):
        bound = 8 * u * (1 + np.where(b > 0, 1 / b, 0))
    assert (np.abs(back - src).max(axis=(-1, -2)) <= bound).all()
    assert (back[..., 0, 1] == 0).all() and (back[..., 1, 0] == 0).all()
    base = 1e-13 if prec == 0 else 5e-6
    for p in (0, 1):
        cur = to_host(ctx, Ug)
        ctx.sweep(Ug, p, 1.7)
        oracle_lib.half_sweep(cur, dims, p, 1.7)
        check(to_host(ctx, Ug), cur, prec, base)
