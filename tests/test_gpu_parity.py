"""GPU parity of the HIP path against the FP64 CPU oracle, called through the
C ABI. Inputs are seeded synthetic fields; both sides get the same values
(FP32 runs give the oracle the exact double promotion of the float field).

Tolerances (derived from the arithmetic, not tuned):
* FP64 links after a half-sweep: 1e-13 abs. Both sides do the same ~100
  double operations per link; libm vs the kernel's own trig differ by an ulp.
* FP32 links after a half-sweep: 5e-6 abs. The rotation is applied in float
  (G rounded to float, ~6 products per entry: a few 6e-8 roundings, times the
  3 subgroups).
* F, theta: 1e-13 relative (F32 fields are promoted exactly, so only the
  summation order differs).
"""
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
    t = torch.from_numpy(np.ascontiguousarray(U_np)).to("cuda", dtype=ctx.cdtype)
    return ctx.pack(t)


def to_host(ctx, U):
    return ctx.unpack(U).cpu().numpy().astype(np.complex128)


def oracle_input(U_np, prec):
    return U_np.astype(np.complex64).astype(np.complex128) if prec == 1 else U_np.copy()


# (8, 6, 8, 8): 12 quality tiles, not a multiple of the 8 XCDs the tiles are dealt to
DIMS = [(4, 4, 4, 4), (4, 6, 2, 8), (6, 4, 4, 2), (8, 8, 8, 8), (8, 6, 8, 8)]


def neighbour(dims, s, mu, sign):
    """Lexicographic index of x + sign * mu-hat (periodic)."""
    nx, ny, nz, nt = dims
    c = [s % nx, (s // nx) % ny, (s // (nx * ny)) % nz, s // (nx * ny * nz)]
    c[mu] = (c[mu] + sign) % dims[mu]
    return c[0] + nx * (c[1] + ny * (c[2] + nz * c[3]))


def oracle_full_sweep_at(oracle_lib, Uo, dims, odd_sites, omega, gauge):
    """The eight links of each given odd site after one full sweep, computed
    in place on Uo: an odd site's links are each changed by exactly one even
    neighbour in the even half-sweep, then by the site itself; even sites are
    independent of each other, so updating only the even neighbours of the
    sampled sites (each once, all before any odd update) gives exactly the
    even half-sweep's values on those links."""
    evens = []
    for s in odd_sites:
        for mu in range(4):
            for sign in (1, -1):
                e = neighbour(dims, s, mu, sign)
                if e not in evens:
                    evens.append(e)
    for e in evens:
        oracle_lib.site_update(Uo, dims, e, omega, gauge)
    for s in odd_sites:
        oracle_lib.site_update(Uo, dims, s, omega, gauge)


def site_links(U, dims, s):
    """(8, 3, 3): U_mu(x) for mu = 0..3, then U_mu(x - mu) for mu = 0..3."""
    V = int(np.prod(dims))
    B = U.reshape(V, 4, 3, 3)
    return np.stack([B[s, mu] for mu in range(4)] + [B[neighbour(dims, s, mu, -1), mu] for mu in range(4)])


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("storage", [0, 1])
def test_pack_roundtrip(gf, field_cache, prec, storage):
    dims = (4, 6, 2, 8)
    U = field_cache(dims, 0.5, 1)
    ctx = make_ctx(gf, dims, LANDAU, prec, storage=storage)
    back = to_host(ctx, to_gpu(ctx, U))
    src = oracle_input(U, prec)
    if storage == 0:
        np.testing.assert_array_equal(back, src)
    else:
        np.testing.assert_array_equal(back[..., :2, :], src[..., :2, :])
        np.testing.assert_allclose(back[..., 2, :], src[..., 2, :], atol=1e-14 if prec == 0 else 2e-6)


def test_internal_layout_positions(gf, field_cache):
    """Element (r, c) of U_mu at site (p, h) sits at
    (((p nb + h / 64) 4 + mu) ne + 3r + c) 64 + h % 64, h = (x + nx(y + ny(z + nz t)))/2."""
    dims = (4, 2, 6, 2)
    nx, ny, nz, nt = dims
    U = field_cache(dims, 0.5, 2)
    ctx = make_ctx(gf, dims, LANDAU, 0)
    I = to_gpu(ctx, U).cpu().numpy().reshape(-1, 2)
    nb = ctx.blocks()
    for t in range(nt):
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    p = (x + y + z + t) & 1
                    h = (x + nx * (y + ny * (z + nz * t))) // 2
                    for mu in range(4):
                        base = ((p * nb + h // 64) * 4 + mu) * 9 * 64 + h % 64
                        m = I[base + 64 * np.arange(9), 0] + 1j * I[base + 64 * np.arange(9), 1]
                        np.testing.assert_array_equal(m.reshape(3, 3), U[t, z, y, x, mu])


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
@pytest.mark.parametrize("dims", DIMS)
def test_quality_matches_oracle(gf, oracle_lib, field_cache, prec, gauge, dims):
    U = field_cache(dims, 0.7, 3)
    ctx = make_ctx(gf, dims, gauge, prec)
    F, th = ctx.quality(to_gpu(ctx, U))
    Fo, tho = oracle_lib.quality(oracle_input(U, prec), dims, gauge)
    assert abs(F - Fo) <= 1e-13 * abs(Fo)
    assert abs(th - tho) <= 1e-13 * abs(tho)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
@pytest.mark.parametrize("lps", [1, 2, 4, 8])
@pytest.mark.parametrize("dims", DIMS[:3])
def test_half_sweeps_match_oracle(gf, oracle_lib, field_cache, prec, gauge, lps, dims):
    U = field_cache(dims, 0.7, 4)
    ctx = make_ctx(gf, dims, gauge, prec, lanes_per_site=lps, block_threads=64)
    Ug = to_gpu(ctx, U)
    Uo = oracle_input(U, prec)
    tol = 1e-13 if prec == 0 else 5e-6
    for p in (0, 1, 0, 1):
        ctx.sweep(Ug, p, 1.7)
        oracle_lib.half_sweep(Uo, dims, p, 1.7, gauge)
        err = np.abs(to_host(ctx, Ug) - Uo).max()
        assert err < tol, (p, err)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("storage", [0, 1])
def test_all_schedules_give_identical_bits(gf, field_cache, prec, storage):
    dims = (8, 4, 6, 4)
    U = field_cache(dims, 0.6, 5)
    ref = None
    for lps in (1, 2, 4, 8):
        for block in (64, 128, 192, 256):
            for nt, order in ((0, 0), (1, 0), (1, 1), (0, 1)):
                ctx = make_ctx(gf, dims, LANDAU, prec, lanes_per_site=lps, block_threads=block,
                               nontemporal=nt, tile_order=order, storage=storage, reunit_every=2)
                Ug = to_gpu(ctx, U)
                ctx.sweeps(Ug, 1.7, 3)
                out = Ug.cpu()
                if ref is None:
                    ref = out
                else:
                    assert torch.equal(out, ref), (lps, block, nt, order)


@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_fix_matches_oracle_fp64(gf, oracle_lib, field_cache, gauge):
    """4^4, amp 0.3, seed 0, omega 1.7, theta < 1e-12 within 2000 sweeps."""
    dims = (4, 4, 4, 4)
    U = field_cache(dims, 0.3, 0)
    ctx = make_ctx(gf, dims, gauge, 0, reunit_every=20)
    Ug = to_gpu(ctx, U)
    r = ctx.fix(Ug, 1.7, 1e-12, 2000)
    Uo = U.copy()
    ro = oracle_lib.fix(Uo, dims, 1.7, 1e-12, 2000, gauge, reunit_every=20)
    assert r["converged"] and ro["converged"]
    assert r["theta"] < 1e-12
    # Same stopping sweep (the check/stop logic of Alg. 1), same F, theta and
    # the same gauge-fixed field.
    assert r["iters"] == ro["iters"], (r, ro)
    assert abs(r["F"] - ro["F"]) < 1e-13
    assert abs(r["theta"] - ro["theta"]) < 1e-3 * ro["theta"]
    err = np.abs(to_host(ctx, Ug) - Uo).max()
    print(f"gauge {gauge}: iters {r['iters']}, max|dU| {err:.2e}")
    assert err < 1e-12


@pytest.mark.parametrize("prec", [0, 1])
def test_fix_schedule_check_and_reunit(gf, oracle_lib, field_cache, prec):
    """check_every = 5, reunit_every = 7, a max_iter that is not a multiple of
    either: same sweeps, same final field as the oracle's Alg. 1."""
    dims = (4, 6, 2, 8)
    U = field_cache(dims, 0.5, 6)
    ctx = make_ctx(gf, dims, LANDAU, prec, check_every=5, reunit_every=7)
    Ug = to_gpu(ctx, U)
    r = ctx.fix(Ug, 1.7, 0.0, 23)
    Uo = oracle_input(U, prec)
    ro = oracle_lib.fix(Uo, dims, 1.7, 0.0, 23, reunit_every=7, check_every=5)
    assert r["iters"] == ro["iters"] == 23 and not r["converged"]
    assert abs(r["F"] - ro["F"]) < (1e-13 if prec == 0 else 1e-6)
    assert np.abs(to_host(ctx, Ug) - Uo).max() < (1e-12 if prec == 0 else 2e-5)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("storage", [0, 1])
def test_reunit_matches_oracle(gf, oracle_lib, field_cache, prec, storage):
    dims = (4, 4, 2, 2)
    rng = np.random.default_rng(3)
    U = field_cache(dims, 0.5, 7)
    P = U + 1e-3 * (rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape))
    ctx = make_ctx(gf, dims, LANDAU, prec, storage=storage)
    Ug = to_gpu(ctx, P)
    ctx.reunit(Ug)
    Po = oracle_input(P, prec)
    if storage == 1:  # the device never sees the stored third row
        Po = to_host(ctx, to_gpu(ctx, P))
    oracle_lib.reunit(Po)
    np.testing.assert_allclose(to_host(ctx, Ug), Po, atol=1e-14 if prec == 0 else 3e-7)


@pytest.mark.parametrize("use_graph", [0, 1])
def test_batch_fix_equals_single_fix(gf, field_cache, use_graph):
    members = [((4, 4, 4, 4), LANDAU, 0.3, 10), ((6, 4, 4, 2), COULOMB, 0.4, 11),
               ((8, 8, 8, 8), LANDAU, 0.5, 12), ((4, 6, 2, 8), LANDAU, 0.6, 13)]
    prec = 1
    kw = dict(check_every=4, reunit_every=10, use_graph=use_graph)
    ens = gf.Context(None, prec=prec, params=gf.default_params(prec, **kw),
                     ensemble=[(d, g) for d, g, _, _ in members])
    Us = []
    for d, g, amp, seed in members:
        c1 = make_ctx(gf, d, g, prec)
        Us.append(to_gpu(c1, field_cache(d, amp, seed)))
    singles = [u.clone() for u in Us]
    rb = ens.batch_fix(Us, 1.7, 1e-7, 3000)
    assert rb["converged"]
    for i, (d, g, _, _) in enumerate(members):
        c1 = make_ctx(gf, d, g, prec, **kw)
        r1 = c1.fix(singles[i], 1.7, 1e-7, 3000)
        assert r1["iters"] == rb["iters"][i]
        assert r1["F"] == rb["F"][i] and r1["theta"] == rb["theta"][i]
        assert torch.equal(singles[i], Us[i])


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
@pytest.mark.parametrize("diag", [(1, 1, 1), (-1, -1, 1), (1j, 1j, -1)])
def test_degenerate_constant_fields(gf, oracle_lib, prec, gauge, diag):
    """Constant diagonal links make every staple block degenerate in some
    subgroup: the unit field (b = 0 vector part, g = 1), diag(-1, -1, 1)
    (g = -1, over-rotated about the third axis) and diag(i, i, -1) (a zero
    SU(2) part, G = 1). One sweep on the GPU equals the oracle's."""
    dims = (4, 2, 2, 4)
    U = np.zeros((4, 2, 2, 4, 4, 3, 3), dtype=np.complex128)
    U[..., range(3), range(3)] = np.array(diag)
    ctx = make_ctx(gf, dims, gauge, prec)
    Ug = to_gpu(ctx, U)
    ctx.sweeps(Ug, 1.7, 1)
    ref = U.copy()
    oracle_lib.sweep(ref, dims, 1.7, gauge)
    got = to_host(ctx, Ug)
    assert np.abs(got - ref).max() < (1e-14 if prec == 0 else 1e-6)
    F, th = ctx.quality(Ug)
    Fo, tho = oracle_lib.quality(got, dims, gauge)  # the GPU's own field, promoted exactly
    assert abs(F - Fo) < 1e-13 and abs(th - tho) <= 1e-13 * max(tho, 1.0)


def test_graph_replay_follows_a_new_eps(gf, field_cache):
    """A context that replayed graphs for one threshold gives, for another
    threshold, exactly what a fresh context gives (the captured check period
    must not keep the first eps)."""
    d, amp, seed = (8, 8, 8, 8), 0.5, 12
    prec = 1
    kw = dict(check_every=5, reunit_every=5, use_graph=1)
    ctx = make_ctx(gf, d, LANDAU, prec, **kw)
    ctx.fix(to_gpu(ctx, field_cache(d, amp, seed)), 1.7, 1e-2, 3000)
    ctx.sweep_count = 0
    U = to_gpu(ctx, field_cache(d, amp, seed))
    r = ctx.fix(U, 1.7, 1e-8, 3000)
    fresh = make_ctx(gf, d, LANDAU, prec, **kw)
    V = to_gpu(fresh, field_cache(d, amp, seed))
    rf = fresh.fix(V, 1.7, 1e-8, 3000)
    assert r["converged"] and r["theta"] < 1e-8
    assert r["iters"] == rf["iters"] and torch.equal(U, V)


def test_fp32_reaches_target_and_tracks_fp64(gf, oracle_lib, field_cache):
    dims = (8, 8, 8, 8)
    U = field_cache(dims, 0.5, 14)
    c32 = make_ctx(gf, dims, LANDAU, 1, check_every=10, reunit_every=10)
    U32 = to_gpu(c32, U)
    r32 = c32.fix(U32, 1.7, 1e-7, 5000)
    Uo = U.copy()
    ro = oracle_lib.fix(Uo, dims, 1.7, 1e-7, 5000, reunit_every=20, check_every=10)
    assert r32["converged"] and r32["theta"] < 1e-7
    assert abs(r32["F"] - ro["F"]) < 1e-5


@pytest.mark.parametrize("prec", [0, 1])
def test_timing_counts_half_sweeps(gf, field_cache, prec):
    dims = (8, 8, 8, 8)
    ctx = make_ctx(gf, dims, LANDAU, prec, timing=1)
    Ug = to_gpu(ctx, field_cache(dims, 0.5, 15))
    ctx.sweeps(Ug, 1.7, 5)
    ms, n = ctx.timing()
    assert n == 10 and ms > 0


@pytest.mark.parametrize("prec", [1, 0])
def test_full_size_48_sampled_sites(gf, oracle_lib, prec):
    """48^4, amp 0.7, the default schedule (the bench's launch configuration),
    FP32 and FP64 links: F and theta of the whole field equal the oracle's;
    after one even half-sweep on the GPU every sampled even site's eight
    links equal the oracle's single-site update of the same (for FP32:
    double-promoted) links; F does not decrease; unitarity holds.

    F/theta tolerance 1e-10 relative: the oracle adds ~2e7 terms of one sign
    one after another (rounding error bound N u = 2e-9, random-walk size
    sqrt(N) u = 5e-13), the GPU in a fixed tree."""
    from paper_1412_1498_amd import synth
    dims = (48, 48, 48, 48)
    U64 = synth.random_gauge_field(dims, 0.7, 0, device="cuda")
    Uc = U64.to(torch.complex64) if prec == 1 else U64
    if prec == 1:
        del U64
    ctx = make_ctx(gf, dims, LANDAU, prec)
    Ug = ctx.pack(Uc)
    F0, th0 = ctx.quality(Ug)
    Uo = Uc.cpu().numpy().astype(np.complex128)
    del Uc
    Fo, tho = oracle_lib.quality(Uo, dims, LANDAU)
    assert abs(F0 - Fo) <= 1e-10 * abs(Fo) and abs(th0 - tho) <= 1e-10 * tho
    ctx.sweep(Ug, 0, 1.7)
    F1, _ = ctx.quality(Ug)
    assert F1 >= F0
    back = ctx.unpack(Ug).cpu().numpy().astype(np.complex128)
    rng = np.random.default_rng(0)
    V = 48 ** 4
    par = oracle_lib.parity_of_sites(dims)
    sites = [int(s) for s in rng.choice(V, 400, replace=False) if par[s] == 0][:128]
    for s in sites:
        oracle_lib.site_update(Uo, dims, s, 1.7)
    tol = 5e-6 if prec == 1 else 1e-13
    for s in sites:
        np.testing.assert_allclose(site_links(back, dims, s), site_links(Uo, dims, s), atol=tol)
    L = np.concatenate([site_links(back, dims, s) for s in sites])
    assert np.abs(L @ L.conj().transpose(0, 2, 1) - np.eye(3)).max() < (2e-6 if prec == 1 else 1e-13)


def test_full_size_ensemble_sampled_sites(gf, oracle_lib):
    """The uneven ensemble at full size (Coulomb 48^3 x 96 + 64 Landau
    lattices of sides 8..24, amp 0.6, FP32 links) in one context, as the
    ensemble bench runs it (graph replay): every member's F and theta equal
    the oracle's; after one batched sweep (Alg. 1 with max_iter 1) the eight
    links of sampled odd sites of the Coulomb member and of three Landau
    members equal the oracle's sweep at those sites.

    Link tolerance 2e-5: two half-sweeps applied in float (5e-6 each, see the
    module notes), the second on inputs that already carry the first's
    rounding. F/theta: 1e-10 relative (as at 48^4)."""
    from paper_1412_1498_amd import synth
    members = synth.ensemble_members(64, seed=0, amp=0.6)
    prec = 1
    ens = gf.Context(None, prec=prec, params=gf.default_params(prec, check_every=1, reunit_every=1000, use_graph=1),
                     ensemble=[(d, g) for d, g, _, _ in members])
    Us, host = [], []
    for i, (d, g, amp, seed) in enumerate(members):
        u = synth.random_gauge_field(d, amp, seed, device="cuda").to(torch.complex64)
        c1 = make_ctx(gf, d, g, prec)
        Us.append(c1.pack(u))
        host.append(u.cpu().numpy().astype(np.complex128))
        del u
    F, th = ens.batch_quality(Us)
    for i, (d, g, _, _) in enumerate(members):
        Fo, tho = oracle_lib.quality(host[i], d, g)
        assert abs(F[i] - Fo) <= 1e-10 * abs(Fo) and abs(th[i] - tho) <= 1e-10 * tho, i
    r = ens.batch_fix(Us, 1.7, 0.0, 1)
    assert r["iters"] == [1] * len(members)
    rng = np.random.default_rng(1)
    checked = [0] + [int(i) for i in rng.choice(np.arange(1, len(members)), 3, replace=False)]
    for i in checked:
        d, g, _, _ = members[i]
        V = int(np.prod(d))
        par = oracle_lib.parity_of_sites(d)
        sites = [int(s) for s in rng.choice(V, 200, replace=False) if par[s] == 1][:32]
        oracle_full_sweep_at(oracle_lib, host[i], d, sites, 1.7, g)
        c1 = make_ctx(gf, d, g, prec)
        back = c1.unpack(Us[i]).cpu().numpy().astype(np.complex128)
        for s in sites:
            np.testing.assert_allclose(site_links(back, d, s), site_links(host[i], d, s), atol=2e-5,
                                       err_msg=f"member {i} site {s}")


def test_autotune_keeps_bits_and_caches(gf, field_cache, tmp_path):
    """The autotuner picks a schedule, the result is bitwise that of the
    default schedule, and a cached choice is reused."""
    members = [((8, 8, 8, 8), LANDAU, 0.5, 40), ((6, 4, 4, 2), COULOMB, 0.5, 41)]
    prec = 1
    ens = gf.Context(None, prec=prec, params=gf.default_params(prec, reunit_every=3),
                     ensemble=[(d, g) for d, g, _, _ in members])
    Us = []
    for d, g, amp, seed in members:
        c1 = make_ctx(gf, d, g, prec)
        Us.append(to_gpu(c1, field_cache(d, amp, seed)))
    ref = [u.clone() for u in Us]
    cache = str(tmp_path / "tune.txt")
    s1 = ens.autotune(Us, 1.7, cache)
    assert s1["lanes_per_site"] in (1, 2, 4, 8) and s1["block_threads"] in (64, 128, 256)
    assert s1["tile_order"] in (0, 1)
    for u, r in zip(Us, ref):  # tuning ran on scratch copies
        assert torch.equal(u, r)
    rb = ens.batch_fix(Us, 1.7, 0.0, 7)
    for i, (d, g, _, _) in enumerate(members):
        c1 = make_ctx(gf, d, g, prec, reunit_every=3)
        c1.fix(ref[i], 1.7, 0.0, 7)
        assert torch.equal(ref[i], Us[i])
    ens2 = gf.Context(None, prec=prec, params=gf.default_params(prec), ensemble=[(d, g) for d, g, _, _ in members])
    assert ens2.autotune(Us, 1.7, cache) == s1
    assert open(cache).read().count("\n") == 1


def test_precision_line_32x4(gf, oracle_lib):
    """32^4, amp 0.5, seed 0: the FP64 GPU form reaches theta < 1e-12 and the
    FP32 form (reunitarised every 10 sweeps) theta < 1e-7; their F agree; the
    first FP64 sweeps follow the oracle."""
    from paper_1412_1498_amd import synth
    dims = (32, 32, 32, 32)
    U = synth.random_gauge_field(dims, 0.5, 0, device="cuda")
    c64 = make_ctx(gf, dims, LANDAU, 0, check_every=10)
    U64 = c64.pack(U)
    Uo = U.cpu().numpy()
    c64.sweeps(U64, 1.7, 2)
    for _ in range(2):
        oracle_lib.sweep(Uo, dims, 1.7)
    # Where a site's subgroup block is nearly degenerate (small |b|), rounding
    # differences in b are amplified ~1/|b| in g; over 10^6 sites a few such
    # sites show up, so the bound is on the distribution and on the maximum.
    err = np.abs(to_host(c64, U64) - Uo)
    print(f"32^4 FP64 two sweeps: median {np.median(err):.2e}, q99.9 {np.quantile(err, 0.999):.2e}, "
          f"max {err.max():.2e}")
    assert np.median(err) < 5e-15 and np.quantile(err, 0.999) < 5e-14 and err.max() < 1e-12
    c64.sweep_count = 0
    U64 = c64.pack(U)
    r64 = c64.fix(U64, 1.7, 1e-12, 20000)
    c32 = make_ctx(gf, dims, LANDAU, 1, check_every=10, reunit_every=10)
    U32 = c32.pack(U.to(torch.complex64))
    r32 = c32.fix(U32, 1.7, 1e-7, 20000)
    assert r64["converged"] and r64["theta"] < 1e-12
    assert r32["converged"] and r32["theta"] < 1e-7
    assert abs(r32["F"] - r64["F"]) < 1e-5
    L = c32.unpack(U32).reshape(-1, 3, 3)
    eye = torch.eye(3, dtype=L.dtype, device=L.device)
    assert (L @ L.conj().transpose(-1, -2) - eye).abs().max().item() < 5e-6


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 4, 2, 6), (8, 2, 2, 2)])
@pytest.mark.parametrize("gauge", [LANDAU, COULOMB])
def test_minimal_extents_match_oracle(gf, oracle_lib, field_cache, dims, gauge):
    """Extent 2 makes x - mu and x + mu the same site (two distinct links)."""
    U = field_cache(dims, 0.8, 50)
    ctx = make_ctx(gf, dims, gauge, 0)
    Ug = to_gpu(ctx, U)
    Uo = U.copy()
    for p in (0, 1, 0, 1):
        ctx.sweep(Ug, p, 1.7)
        oracle_lib.half_sweep(Uo, dims, p, 1.7, gauge)
    assert np.abs(to_host(ctx, Ug) - Uo).max() < 1e-13
    F, th = ctx.quality(Ug)
    Fo, tho = oracle_lib.quality(Uo, dims, gauge)
    assert abs(F - Fo) < 1e-13 and abs(th - tho) < 1e-12 * max(1.0, tho)


def test_converged_members_do_no_sweeps(gf, field_cache):
    """A member whose initial theta is already below eps reports 0 sweeps and
    an unchanged field, while the others are fixed."""
    members = [((4, 4, 4, 4), LANDAU), ((4, 4, 4, 4), LANDAU)]
    ens = gf.Context(None, prec=0, params=gf.default_params(0, check_every=2), ensemble=members)
    c1 = make_ctx(gf, (4, 4, 4, 4), LANDAU, 0)
    unit = np.zeros((4, 4, 4, 4, 4, 3, 3), dtype=np.complex128)
    unit[...] = np.eye(3)
    Us = [to_gpu(c1, unit), to_gpu(c1, field_cache((4, 4, 4, 4), 0.3, 0))]
    before = Us[0].clone()
    r = ens.batch_fix(Us, 1.7, 1e-12, 2000)
    assert r["converged"] and r["iters"][0] == 0 and r["iters"][1] > 0
    assert torch.equal(Us[0], before) and r["F"][0] == 1.0 and r["theta"][0] == 0.0


def test_non_finite_field_is_reported(gf, field_cache):
    dims = (4, 4, 4, 4)
    U = field_cache(dims, 0.3, 0)
    U[1, 2, 3, 0, 2, 1, 1] = np.nan
    ctx = make_ctx(gf, dims, LANDAU, 1)
    Ug = to_gpu(ctx, U)
    with pytest.raises(gf.GFError) as e:
        ctx.quality(Ug)
    assert e.value.code == gf.ENONFINITE
    with pytest.raises(gf.GFError) as e:
        ctx.fix(Ug, 1.7, 1e-7, 100)
    assert e.value.code == gf.ENONFINITE


def test_invalid_calls_are_rejected(gf, field_cache):
    dims = (4, 4, 4, 4)
    ctx = make_ctx(gf, dims, LANDAU, 1)
    Ug = to_gpu(ctx, field_cache(dims, 0.3, 0))
    for bad in (lambda: ctx.sweep(Ug, 2, 1.7), lambda: ctx.sweep(Ug, 0, 2.0), lambda: ctx.sweep(Ug, 0, 0.0),
                lambda: ctx.fix(Ug, 1.7, -1.0, 10), lambda: ctx.fix(Ug, 1.7, 1e-7, -1)):
        with pytest.raises(gf.GFError) as e:
            bad()
        assert e.value.code == gf.EINVAL
    with pytest.raises(ValueError):
        ctx.sweep(torch.zeros(10, device="cuda"), 0, 1.7)


@pytest.mark.parametrize("prec", [0, 1])
def test_resume_is_bitwise_equal(gf, field_cache, prec):
    """Checkpoint/resume: the state is the field plus the sweep counter (the
    reunitarisation phase); 12 + 18 sweeps with a restart in between equal
    30 sweeps in one go."""
    dims = (8, 4, 4, 6)
    U = field_cache(dims, 0.5, 51)
    ctx = make_ctx(gf, dims, LANDAU, prec, reunit_every=7)
    A = to_gpu(ctx, U)
    ctx.sweeps(A, 1.7, 30)
    B = to_gpu(ctx, U)
    c1 = make_ctx(gf, dims, LANDAU, prec, reunit_every=7)
    c1.sweeps(B, 1.7, 12)
    saved = B.cpu()
    c2 = make_ctx(gf, dims, LANDAU, prec, reunit_every=7, start_sweep=12)
    B2 = saved.cuda()
    c2.sweeps(B2, 1.7, 18)
    assert torch.equal(A, B2) and c2.sweep_count == 30
