#!/usr/bin/env python3
"""Throughput of checkerboard overrelaxation gauge fixing on one MI355X.

Workload: SU(3) Landau gauge, 48^4 lattice, FP32 links (FP64 staple sums,
SU(2) solve, reunitarisation and F/theta reductions), seeded synthetic field
U_mu(x) = h(x) exp(i 0.7 sum_a r_a lambda_a / 2) h(x+mu)^dagger, seed 0,
omega = 1.7.

One timed step = one check period of Alg. 1: 10 sweeps (even + odd
half-sweep each, reunitarisation fused into the 10th odd half-sweep) followed
by the F/theta reduction that gates convergence (host read-back included).
value = lattice sites x sweeps / wall time of the timed steps.

Also reported: the roofline of the dominant kernel (the half-sweep) from HIP
events recorded on the context's stream around every half-sweep launch in
the timed region; the plain FP64 GPU form on the same field; runs to
theta < 1e-7 in FP32 and FP64; and the FP64 CPU oracle timed on the host on
one full sweep of the same field.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ["sweep.hip", "su3_device.hpp", "gf_math.hpp", "gf_internal.hpp", "link8.hpp", "tile_order.hpp"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1412_1498_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(profile_name, khash):
    """HBM bytes per half-sweep launch from a committed rocprofv3 --pmc
    summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", profile_name)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_hash") != khash:
        return None
    try:
        return float(vals["hbm_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


def run_ensemble(args, gf, synth, torch, np):
    """Batching line: one Coulomb 48^3 x 96 lattice (amp 0.6, seed 0) and 64
    Landau lattices with volumes drawn uniformly from {8^4, 12^4, 16^4, 20^4,
    24^4} (seed 0; member i seed 1 + i, amp 0.6), FP32 links, omega 1.7, all
    fixed to theta < 1e-7 together (check every 10 sweeps, reunitarisation
    every 10, each check period one hipGraph replay, autotuned schedule).
    Compared with fixing the members one after another, in FP32 and FP64."""
    members = synth.ensemble_members(64, seed=0, amp=0.6)
    vols = [d[0] * d[1] * d[2] * d[3] for d, _, _, _ in members]
    eps, omega, max_iter = 1e-7, 1.7, 10000
    log(f"ensemble: {len(members)} members, {sum(vols)} sites; generating")
    fields = []
    for d, g, amp, seed in members:
        fields.append(synth.random_gauge_field(d, amp, seed, device="cuda"))
    torch.cuda.synchronize()

    def kw(prec, graph):
        return gf.default_params(prec, check_every=10, reunit_every=10, use_graph=graph)

    out = {"workload": "ensemble: Coulomb 48x48x48x96 + 64 Landau lattices in {8,12,16,20,24}^4, FP32 links, "
                       "amp 0.6, omega 1.7, theta < 1e-7",
           "members": len(members), "sites": sum(vols)}
    # batched, autotuned, graphs
    ens = gf.Context(None, prec=gf.F32, params=kw(gf.F32, 1), ensemble=[(d, g) for d, g, _, _ in members])
    singles = [gf.Context(d, gauge=g, prec=gf.F32, params=kw(gf.F32, 0)) for d, g, _, _ in members]
    Us = [c.pack(f.to(torch.complex64)) for c, f in zip(singles, fields)]
    log("autotuning the ensemble schedule")
    t0 = time.perf_counter()
    sched = ens.autotune(Us, omega)
    out["autotune_seconds"] = time.perf_counter() - t0
    out["schedule"] = sched
    Ub = [u.clone() for u in Us]
    torch.cuda.synchronize()
    log("batched fix")
    t0 = time.perf_counter()
    rb = ens.batch_fix(Ub, omega, eps, max_iter)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    sweeps = sum(it * v for it, v in zip(rb["iters"], vols))
    out["batched"] = dict(seconds=tb, all_converged=rb["converged"], site_sweeps=sweeps,
                          site_sweeps_per_s=sweeps / tb, iters_coulomb=rb["iters"][0],
                          iters_landau_min=min(rb["iters"][1:]), iters_landau_max=max(rb["iters"][1:]),
                          max_theta=max(rb["theta"]))
    # the same members one after another (FP32, default schedule, no graphs)
    log("sequential FP32 fixes")
    Us32 = [u.clone() for u in Us]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r32 = [c.fix(u, omega, eps, max_iter) for c, u in zip(singles, Us32)]
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t0
    same = all(torch.equal(a, b) for a, b in zip(Ub, Us32))  # every schedule gives the same bits
    out["sequential_fp32"] = dict(seconds=t32, iters_equal=[r["iters"] for r in r32] == rb["iters"],
                                  bitwise_equal_fields=same)
    del Us32
    log("sequential FP64 fixes")
    c64 = [gf.Context(d, gauge=g, prec=gf.F64, params=kw(gf.F64, 0)) for d, g, _, _ in members]
    t64 = 0.0
    F64 = []
    for c, f in zip(c64, fields):
        u = c.pack(f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = c.fix(u, omega, eps, max_iter)
        torch.cuda.synchronize()
        t64 += time.perf_counter() - t0
        F64.append(r["F"])
        del u
    out["sequential_fp64"] = dict(seconds=t64)
    out["batched_speedup_vs_sequential_fp32"] = t32 / tb
    out["batched_speedup_vs_sequential_fp64"] = t64 / tb
    out["batched_over_fp64"] = t64 / tb
    out["max_abs_F_fp32_batched_minus_fp64"] = max(abs(a - b) for a, b in zip(rb["F"], F64))
    return out


def run_sun(args, dims, gf, synth, torch):
    """SU(N) line (N = 2, 4; all N(N-1)/2 SU(2) subgroups per site): the
    half-sweep at the main lattice size in FP32 and FP64 (default schedule,
    amp 0.7, seed 0; 2 warm-up and 10 timed sweeps, HIP events per launch),
    and Alg. 1 to theta < 1e-7 at 24^4 in FP32 and FP64 (amp 0.5, seed 1,
    check and reunitarisation every 10 sweeps)."""
    V = dims[0] * dims[1] * dims[2] * dims[3]
    res = {}
    for n in (2, 4):
        log(f"SU({n}) half-sweeps at {'x'.join(map(str, dims))}")
        U64 = synth.random_sun_field(dims, n, 0.7, 0, device="cuda")
        for name, prec in (("fp32", gf.F32), ("fp64", gf.F64)):
            ctx = gf.Context(dims, prec=prec, nc=n, params=gf.default_params(prec, timing=1))
            U = ctx.pack(U64.to(ctx.cdtype))
            ctx.sweeps(U, args.omega, 2)
            ctx.timing()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.sweeps(U, args.omega, 10)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            ms, nl = ctx.timing()
            avg = ms / 1e3 / nl
            per_launch = 16 * n * n * (8 if prec == gf.F32 else 16) * (V // 2)
            res[f"su{n}_{name}"] = dict(site_sweeps_per_s=V * 10 / wall, avg_launch_us=avg * 1e6,
                                        algorithmic_bytes_per_launch=per_launch,
                                        achieved_gbs=per_launch / avg / 1e9,
                                        frac=per_launch / avg / 1e9 / PEAK_HBM_GBS, schedule=ctx.schedule())
            del U, ctx
        del U64
        torch.cuda.empty_cache()
        cd = (24, 24, 24, 24)
        Uc = synth.random_sun_field(cd, n, 0.5, 1, device="cuda")
        conv = {}
        for name, prec in (("fp32", gf.F32), ("fp64", gf.F64)):
            ctx = gf.Context(cd, prec=prec, nc=n, params=gf.default_params(prec, check_every=10, reunit_every=10))
            U = ctx.pack(Uc.to(ctx.cdtype))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ctx.fix(U, args.omega, 1e-7, 20000)
            torch.cuda.synchronize()
            conv[name] = dict(seconds=time.perf_counter() - t0, sweeps=r["iters"], converged=r["converged"],
                              F=r["F"], theta=r["theta"])
            del U, ctx
        conv["abs_F_fp32_minus_fp64"] = abs(conv["fp32"]["F"] - conv["fp64"]["F"])
        res[f"su{n}_24x4_to_theta_1e-7"] = conv
        del Uc
        torch.cuda.empty_cache()
    return res


def bw_reference(torch, nbytes, achieved_gbs):
    """HBM reference on the same GPU: torch's device copy (read one buffer,
    write another) and an in-place negation (read and write one buffer, the
    half-sweep's access kind), each over nbytes per buffer; 3 warm-up and 10
    timed launches, HIP events on torch's stream."""
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    res = {"buffer_bytes": n * 4}
    for name, op, moved in (("copy", lambda: b.copy_(a), 2 * n * 4), ("inplace_rmw", lambda: a.neg_(), 2 * n * 4)):
        for _ in range(3):
            op()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            op()
        e1.record()
        e1.synchronize()
        res[f"{name}_gbs"] = moved / (e0.elapsed_time(e1) / 10 * 1e-3) / 1e9
    res["halfsweep_over_copy"] = achieved_gbs / res["copy_gbs"]
    res["halfsweep_over_inplace_rmw"] = achieved_gbs / res["inplace_rmw_gbs"]
    del a, b
    torch.cuda.empty_cache()
    return res


def run_fixed_sweeps(gf, torch, U64, dims, params, nsweep=500):
    """Fixed sweep counts on the benchmark field: for omega 1.5, 1.7 and 1.9,
    nsweep FP32 sweeps with no theta checks (reunitarisation fused every 10),
    timed as one call after 10 untimed sweeps; FP64 at omega 1.7 beside it.
    theta after the sweeps is read afterwards, outside the timed region."""
    V = dims[0] * dims[1] * dims[2] * dims[3]
    res = {"workload": f"SU(3) Landau, {'x'.join(map(str, dims))}, amp 0.7, seed 0, {nsweep} sweeps, "
                       "reunitarisation every 10, no checks",
           "sweeps": nsweep}
    for name, prec, w in (("fp32_omega_1.5", gf.F32, 1.5), ("fp32_omega_1.7", gf.F32, 1.7),
                          ("fp32_omega_1.9", gf.F32, 1.9), ("fp64_omega_1.7", gf.F64, 1.7)):
        log(f"{nsweep} fixed sweeps, {name}")
        ctx = gf.Context(dims, gauge=gf.LANDAU, prec=prec, params=params(prec, 0))
        U = ctx.pack(U64 if prec == gf.F64 else U64.to(torch.complex64))
        ctx.sweeps(U, w, 10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.sweeps(U, w, nsweep)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        F, th = ctx.quality(U)
        res[name] = dict(seconds=sec, site_sweeps_per_s=V * nsweep / sec, F=F, theta_after=th)
        del U, ctx
        torch.cuda.empty_cache()
    return res


def run_slab_shape(gf, synth, torch, dims=(48, 48, 48, 12), nsweep=20):
    """The half-sweep at 48^3x12, the share of one GPU if the 48^3x96
    lattice were cut into eight slabs along t (the split is not built): the
    kernel-only half-sweep time (HIP events, FP32 and FP64 18-real), beside
    the size of the cut face's current-parity links that such a split would
    send each way per half-sweep, and that message's time over one xGMI link
    at its nominal 153 GB/s (an estimate, not a measurement)."""
    V = dims[0] * dims[1] * dims[2] * dims[3]
    face = dims[0] * dims[1] * dims[2] // 2
    res = {"workload": "SU(3) Landau, 48x48x48x12, amp 0.6, seed 0, omega 1.7", "lattice": list(dims)}
    U64 = synth.random_gauge_field(dims, 0.6, 0, device="cuda")
    for name, prec in (("fp32", gf.F32), ("fp64", gf.F64)):
        log(f"48^3x12 half-sweeps, {name}")
        ctx = gf.Context(dims, gauge=gf.LANDAU, prec=prec,
                         params=gf.default_params(prec, reunit_every=10, timing=1))
        U = ctx.pack(U64 if prec == gf.F64 else U64.to(torch.complex64))
        ctx.sweeps(U, 1.7, 4)
        ctx.timing()
        ctx.sweeps(U, 1.7, nsweep)
        ms, nl = ctx.timing()
        avg = ms / 1e3 / nl
        lb = 18 * (4 if prec == gf.F32 else 8)
        msg = face * lb
        res[name] = dict(avg_halfsweep_us=avg * 1e6, site_sweeps_per_s=V / (2 * avg),
                         achieved_gbs=16 * lb * (V // 2) / avg / 1e9,
                         face_message_bytes=msg, face_message_us_at_153_gbs=msg / 153e9 * 1e6)
        del U, ctx
        torch.cuda.empty_cache()
    del U64
    torch.cuda.empty_cache()
    return res


def run_diff(gf, synth, torch, sizes=(24, 48)):
    """Differentiation line: F_U[g] (gf_functional), its hand-written
    backward (gf_functional_grad) and the gauge transformation at L^4 for
    each L in sizes (amp 0.4, s_a ~ N(0, 0.1^2)), FP32 and FP64; 3 warm-up
    and 20 timed calls each, HIP events on the context's stream. Each call
    runs two kernels: g = exp(S(s)) into the g field, then the call's own.
    Algorithmic bytes per site (each datum once; r = bytes of a real): the
    exponential reads s (8r) and writes g (18r); the functional reads the
    four forward links (72r) and g (18r); the gradient reads all four links
    (72r), g (18r) and s (8r) and writes the gradient (8r); the
    transformation reads and writes the links (144r) and reads g (18r)."""
    res = {}
    for L in sizes:
        ddims = (L, L, L, L)
        Vd = L ** 4
        Ud = synth.random_gauge_field(ddims, 0.4, 0, device="cuda")
        sd = synth.random_algebra_field(ddims, 0.1, 1)
        out = {}
        for name, prec in (("fp32", gf.F32), ("fp64", gf.F64)):
            r = 4 if prec == gf.F32 else 8
            bytes_site = {"forward": (26 + 90) * r, "backward": (26 + 106) * r, "gauge_transform": (26 + 162) * r}
            ctx = gf.Context(ddims, gauge=gf.LANDAU, prec=prec)
            U = ctx.pack(Ud.to(ctx.cdtype))
            s = ctx.pack_alg(sd.to("cuda", dtype=ctx.rdtype))
            grad = ctx.functional_grad(U, s)
            calls = {"forward": lambda: ctx.functional(U, s),
                     "backward": lambda: ctx.functional_grad(U, s, 1.0, out=grad),
                     "gauge_transform": lambda: ctx.gauge_transform(U, s)}
            entry = {}
            for what, fn in calls.items():
                for _ in range(3):
                    fn()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(20):
                    fn()
                e1.record()
                e1.synchronize()
                sec = e0.elapsed_time(e1) / 20 / 1e3
                gbs = bytes_site[what] * Vd / sec / 1e9
                entry[what] = dict(ms=sec * 1e3, algorithmic_bytes_per_site=bytes_site[what], achieved_gbs=gbs,
                                   frac=gbs / PEAK_HBM_GBS)
            entry["sites_per_s_backward"] = Vd / (entry["backward"]["ms"] / 1e3)
            out[name] = entry
            del U, s, grad, ctx
        res[f"{L}x4"] = out
        del Ud
        torch.cuda.empty_cache()
    return res


def run_sd(args, dims, gf, synth, torch):
    """Fourier-accelerated steepest descent (Alg. 2, alpha 0.08, Landau) on the
    main lattice, FP32 and FP64 (amp 0.7, seed 0): the time of one step
    (2 warm-up and 20 timed gf_sd_step calls) and a run to theta < 1e-7 with a
    check every 10 steps."""
    res = {}
    U64 = synth.random_gauge_field(dims, args.amp, args.seed, device="cuda")
    for name, prec in (("fp32", gf.F32), ("fp64", gf.F64)):
        log(f"Alg. 2 steps at {'x'.join(map(str, dims))}, {name}")
        ctx = gf.Context(dims, prec=prec, params=gf.default_params(prec, check_every=10))
        U = ctx.pack(U64 if prec == gf.F64 else U64.to(torch.complex64))
        for _ in range(2):
            ctx.sd_step(U, 0.08)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            ctx.sd_step(U, 0.08)
        torch.cuda.synchronize()
        step_ms = (time.perf_counter() - t0) / 20 * 1e3
        U = ctx.pack(U64 if prec == gf.F64 else U64.to(torch.complex64), U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.sd_fix(U, 0.08, 1e-7, 5000)
        torch.cuda.synchronize()
        res[name] = {"step_ms": step_ms, "seconds_to_theta_1e-7": time.perf_counter() - t0, "steps": r["iters"],
                     "converged": r["converged"], "F": r["F"], "theta": r["theta"]}
        del U, ctx
        torch.cuda.empty_cache()
    return res


def run_precision_32(gf, synth, torch):
    """Precision line at 32^4 (Landau, amp 0.5, seed 0, omega 1.7, checks and
    reunitarisation every 10 sweeps): the plain FP64 GPU form to theta < 1e-12
    and to theta < 1e-7, and FP32 links (FP64 sums, solve, reunitarisation and
    F/theta) to theta < 1e-7; wall time of each gf_fix."""
    dims = (32, 32, 32, 32)
    U64 = synth.random_gauge_field(dims, 0.5, 0, device="cuda")
    res = {"workload": "SU(3) Landau, 32x32x32x32, amp 0.5, seed 0, omega 1.7, check and reunit every 10 sweeps"}
    for name, prec, eps in (("fp64_to_1e-12", gf.F64, 1e-12), ("fp64_to_1e-7", gf.F64, 1e-7),
                            ("fp32_to_1e-7", gf.F32, 1e-7)):
        log(f"32^4 {name}")
        ctx = gf.Context(dims, gauge=gf.LANDAU, prec=prec,
                         params=gf.default_params(prec, check_every=10, reunit_every=10))
        U = ctx.pack(U64 if prec == gf.F64 else U64.to(torch.complex64))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.fix(U, 1.7, eps, 20000)
        torch.cuda.synchronize()
        res[name] = dict(seconds=time.perf_counter() - t0, sweeps=r["iters"], converged=r["converged"],
                         F=r["F"], theta=r["theta"])
        del U, ctx
        torch.cuda.empty_cache()
    res["fp32_speedup_to_theta_1e-7"] = res["fp64_to_1e-7"]["seconds"] / res["fp32_to_1e-7"]["seconds"]
    res["abs_F_fp32_minus_fp64_1e-12"] = abs(res["fp32_to_1e-7"]["F"] - res["fp64_to_1e-12"]["F"])
    return res, U64


def run_cpu_baseline(gf, synth, torch, fields, main_name, gpu_value, gpu_fp64_time_16):
    """The FP64 C oracle on the host cores: site-sweeps/s over whole sweeps
    (even + odd half-sweep) of the benchmark's own fields, with one thread
    and with the threads of this process's CPU share (at most 16); and the
    time to theta < 1e-12 at 4^4 and 16^4 (amp 0.3, seed 0, omega 1.7,
    reunitarisation every 20 sweeps) next to the FP64 GPU time."""
    import oracle
    share = min(16, len(os.sched_getaffinity(0)))
    before = oracle.set_threads(0)
    runs = []
    plan = [(1, "32x32x32x32", 5), (share, "32x32x32x32", 5), (share, main_name, 5)]
    for threads, name, nsw in plan:
        Uh, dims = fields[name]
        A = Uh.copy()
        oracle.set_threads(threads)
        log(f"CPU oracle: {nsw} FP64 sweeps at {name} on {threads} thread(s)")
        t0 = time.perf_counter()
        for _ in range(nsw):
            oracle.sweep(A, dims, 1.7)
        dt = time.perf_counter() - t0
        V = dims[0] * dims[1] * dims[2] * dims[3]
        runs.append(dict(threads=threads, lattice=name, sweeps=nsw, seconds=dt, site_sweeps_per_s=V * nsw / dt))
        del A
    conv = {}
    oracle.set_threads(share)
    for L in (4, 16):
        dims = (L, L, L, L)
        Uh = synth.random_gauge_field(dims, 0.3, 0).numpy()
        log(f"CPU oracle: {L}^4 to theta < 1e-12 on {share} threads")
        t0 = time.perf_counter()
        ro = oracle.fix(Uh, dims, 1.7, 1e-12, 20000, reunit_every=20)
        conv[f"{L}x4"] = dict(threads=share, seconds=time.perf_counter() - t0, sweeps=ro["iters"],
                              converged=ro["converged"], theta=ro["theta"])
    conv["16x4"]["gpu_fp64_seconds"] = gpu_fp64_time_16
    oracle.set_threads(before)
    main = runs[2]
    return {
        "value": main["site_sweeps_per_s"],
        "unit": "site-sweeps/s",
        "cores": share,
        "kind": "oracle",
        "sample": f"5 FP64 sweeps (even + odd half-sweep) of the benchmark's {main_name} field by the C oracle "
                  f"on {share} threads ({main['seconds']:.1f} s); also 1 thread at 32^4 and runs to "
                  f"theta < 1e-12 at 4^4 and 16^4",
        "runs": runs,
        "to_theta_1e-12": conv,
        "gpu_over_cpu_threads": gpu_value / main["site_sweeps_per_s"],
        "gpu_over_cpu_1_thread": gpu_value / runs[0]["site_sweeps_per_s"],
    }


def gpu_fp64_time_16(gf, synth, torch):
    """FP64 GPU time to theta < 1e-12 at 16^4 (amp 0.3, seed 0, omega 1.7,
    reunitarisation every 20 sweeps, check every sweep), as the oracle runs it."""
    dims = (16, 16, 16, 16)
    ctx = gf.Context(dims, gauge=gf.LANDAU, prec=gf.F64, params=gf.default_params(gf.F64, reunit_every=20))
    U = ctx.pack(synth.random_gauge_field(dims, 0.3, 0, device="cuda"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.fix(U, 1.7, 1e-12, 20000)
    torch.cuda.synchronize()
    return dict(seconds=time.perf_counter() - t0, sweeps=r["iters"], converged=r["converged"])


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50, help="timed check periods")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dims", default="48,48,48,48")
    ap.add_argument("--amp", type=float, default=0.7)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--omega", type=float, default=1.7)
    ap.add_argument("--sweeps-per-step", type=int, default=10)
    ap.add_argument("--storage", type=int, choices=[18, 12, 8], default=18)
    ap.add_argument("--lps", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--nontemporal", type=int, default=-1)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-12real", action="store_true", help="skip the 12-real FP32 storage leg")
    ap.add_argument("--no-8real", action="store_true", help="skip the 8-real FP32 storage leg")
    ap.add_argument("--no-convergence", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-32", action="store_true",
                    help="skip the 32^4 FP64 / FP32 runs to theta < 1e-12 / 1e-7")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the ensemble leg (Coulomb 48^3x96 + 64 uneven Landau lattices)")
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiation timing leg")
    ap.add_argument("--no-fixed-sweeps", action="store_true",
                    help="skip the 500 fixed sweeps (no checks) at omega 1.5, 1.7, 1.9")
    ap.add_argument("--no-slab", action="store_true",
                    help="skip the half-sweep timing at 48^3x12 (one GPU's share of 48^3x96 split in eight)")
    ap.add_argument("--no-sun", action="store_true", help="skip the SU(2) / SU(4) leg")
    ap.add_argument("--no-bw-reference", action="store_true",
                    help="skip the device copy / in-place read-modify-write bandwidth reference")
    ap.add_argument("--workload", choices=["single", "ensemble", "sun", "sd", "diff"], default="single",
                    help="ensemble: Coulomb 48^3x96 plus 64 Landau lattices of uneven volume fixed together; "
                         "sun: only the SU(2) / SU(4) leg; sd: only steepest descent with Fourier acceleration; "
                         "diff: only the differentiation leg")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also launch one plain 1 GiB device copy (counter scale reference)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on exactly one GPU (no multi-GPU path); --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1412_1498_amd import gf, synth

    if args.workload == "ensemble":
        print(json.dumps(run_ensemble(args, gf, synth, torch, np)), flush=True)
        return

    dims = tuple(int(x) for x in args.dims.split(","))
    if args.workload == "sun":
        print(json.dumps({"workload": "SU(2) and SU(4) overrelaxation, Landau gauge",
                          "sun": run_sun(args, dims, gf, synth, torch)}), flush=True)
        return
    if args.workload == "diff":
        out = {"workload": "differentiation: F_U[g], its gradient and the gauge transformation, 24^4 and 48^4",
               "differentiation": run_diff(gf, synth, torch)}
        if args.copy_probe:
            a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
            torch.empty_like(a).copy_(a)
            torch.cuda.synchronize()
        print(json.dumps(out), flush=True)
        return
    if args.workload == "sd":
        out = {"workload": "steepest descent with Fourier acceleration (Alg. 2), Landau gauge, alpha 0.08",
               "sd": run_sd(args, dims, gf, synth, torch)}
        if args.copy_probe:
            a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
            torch.empty_like(a).copy_(a)
            torch.cuda.synchronize()
        print(json.dumps(out), flush=True)
        return
    V = dims[0] * dims[1] * dims[2] * dims[3]
    spp = args.sweeps_per_step
    storage = {12: gf.STORE_12, 8: gf.STORE_8}.get(args.storage, gf.STORE_18)
    log(f"generating {dims} amp {args.amp} seed {args.seed} (FP64, on the GPU)")
    t = time.perf_counter()
    U64 = synth.random_gauge_field(dims, args.amp, args.seed, device="cuda")
    torch.cuda.synchronize()
    log(f"generated in {time.perf_counter() - t:.1f} s")

    def params(prec, timing, store=None):
        return gf.default_params(prec, check_every=spp, reunit_every=10,
                                 storage=storage if store is None else store,
                                 lanes_per_site=args.lps, block_threads=args.block,
                                 nontemporal=args.nontemporal, timing=timing)

    def timed_run(prec, store=None):
        ctx = gf.Context(dims, gauge=gf.LANDAU, prec=prec, params=params(prec, 1, store))
        U = ctx.pack(U64 if prec == gf.F64 else U64.to(torch.complex64))
        F0, th0 = ctx.quality(U)
        for _ in range(args.warmup):
            ctx.sweeps(U, args.omega, spp)
            ctx.quality(U)
        ctx.timing()  # discard warm-up launches
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            ctx.sweeps(U, args.omega, spp)
            F, th = ctx.quality(U)
            if k % 10 == 9:
                log(f"{'fp64' if prec == gf.F64 else 'fp32'} step {k + 1}/{args.steps} F {F:.9f} theta {th:.3e}")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms, nl = ctx.timing()
        sched = ctx.schedule()
        del U, ctx
        torch.cuda.empty_cache()
        return dict(wall=wall, kernel_ms=ms, launches=nl, F=F, theta=th, F0=F0, theta0=th0, schedule=sched)


    def roofline(res, prec, reals=None):
        lb = (reals or args.storage) * (4 if prec == gf.F32 else 8)  # bytes of one stored link
        per_site = 16 * lb                                # 8 links read + 8 written per site update
        per_launch = per_site * (V // 2)
        avg = res["kernel_ms"] / 1e3 / res["launches"]
        ach = per_launch / avg / 1e9
        return dict(bytes_per_site_update=per_site, bytes_per_launch=per_launch,
                    avg_launch_s=avg, achieved_gbs=ach)

    log("timed FP32 run")
    r32 = timed_run(gf.F32)
    rf32 = roofline(r32, gf.F32)
    value = V * spp * args.steps / r32["wall"]
    khash = kernel_hash()
    traffic = measured_traffic(f"halfsweep_{'x'.join(map(str, dims))}_f32_{args.storage}real_pmc.txt", khash)

    out = {
        "metric": "site-sweeps/s (SU(3) OR, 48^4 FP32) + % HBM roofline vs FP64 at theta<1e-7",
        "value": value,
        "unit": "site-sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"SU(3) Landau overrelaxation gauge fixing, {'x'.join(map(str, dims))} lattice, "
                        f"FP32 links ({args.storage}-real storage), amp {args.amp}, seed {args.seed}, "
                        f"omega {args.omega}; step = {spp} sweeps + F/theta check, reunitarisation every 10 sweeps",
            "lattice": list(dims),
            "sweeps_per_step": spp,
            "schedule": r32["schedule"],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": rf32["achieved_gbs"],
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": rf32["achieved_gbs"] / PEAK_HBM_GBS,
            "traffic": traffic,
            "kernel": "k_half_sweep (one half-sweep: V/2 site updates)",
            "algorithmic_bytes_per_launch": rf32["bytes_per_launch"],
            "avg_launch_us": rf32["avg_launch_s"] * 1e6,
            "launches_timed": r32["launches"],
            "kernel_source_hash": khash,
        },
    }

    if args.storage == 18 and not args.no_12real:
        log("timed FP32 run, 12-real storage (rows 0, 1 stored, row 2 rebuilt)")
        r12 = timed_run(gf.F32, gf.STORE_12)
        rf12 = roofline(r12, gf.F32, 12)
        out["fp32_12real"] = {
            "value": V * spp * args.steps / r12["wall"],
            "unit": "site-sweeps/s",
            "achieved_gbs": rf12["achieved_gbs"],
            "frac": rf12["achieved_gbs"] / PEAK_HBM_GBS,
            "algorithmic_bytes_per_launch": rf12["bytes_per_launch"],
            "avg_launch_us": rf12["avg_launch_s"] * 1e6,
            "traffic": measured_traffic(f"halfsweep_{'x'.join(map(str, dims))}_f32_12real_pmc.txt", khash),
            "schedule": r12["schedule"],
        }

    if args.storage == 18 and not args.no_8real:
        log("timed FP32 run, 8-real storage (U01, U02, U10 and two phases stored)")
        r8 = timed_run(gf.F32, gf.STORE_8)
        rf8 = roofline(r8, gf.F32, 8)
        out["fp32_8real"] = {
            "value": V * spp * args.steps / r8["wall"],
            "unit": "site-sweeps/s",
            "achieved_gbs": rf8["achieved_gbs"],
            "frac": rf8["achieved_gbs"] / PEAK_HBM_GBS,
            "algorithmic_bytes_per_launch": rf8["bytes_per_launch"],
            "avg_launch_us": rf8["avg_launch_s"] * 1e6,
            "traffic": measured_traffic(f"halfsweep_{'x'.join(map(str, dims))}_f32_8real_pmc.txt", khash),
            "schedule": r8["schedule"],
            "F_after_timed_steps": r8["F"],
            "F_18real_after_timed_steps": r32["F"],
        }

    if not args.no_fp64:
        log("timed FP64 run (plain FP64 GPU form)")
        r64 = timed_run(gf.F64)
        rf64 = roofline(r64, gf.F64)
        out["fp64"] = {
            "value": V * spp * args.steps / r64["wall"],
            "unit": "site-sweeps/s",
            "achieved_gbs": rf64["achieved_gbs"],
            "frac": rf64["achieved_gbs"] / PEAK_HBM_GBS,
            "avg_launch_us": rf64["avg_launch_s"] * 1e6,
            "traffic": (measured_traffic(f"halfsweep_{'x'.join(map(str, dims))}_f64_{args.storage}real_pmc.txt", khash)
                        if args.storage == 18 else None),
            "schedule": r64["schedule"],
        }
        out["fp32_over_fp64_throughput"] = value / out["fp64"]["value"]
        if not args.no_8real and args.storage == 18:
            log("timed FP64 run, 8-real storage")
            r64_8 = timed_run(gf.F64, gf.STORE_8)
            rf64_8 = roofline(r64_8, gf.F64, 8)
            out["fp64_8real"] = {
                "value": V * spp * args.steps / r64_8["wall"],
                "unit": "site-sweeps/s",
                "achieved_gbs": rf64_8["achieved_gbs"],
                "frac": rf64_8["achieved_gbs"] / PEAK_HBM_GBS,
                "avg_launch_us": rf64_8["avg_launch_s"] * 1e6,
                "schedule": r64_8["schedule"],
            }

    if not args.no_convergence:
        conv = {}
        for name, prec in (("fp32", gf.F32), ("fp64", gf.F64)):
            log(f"{name} run to theta < 1e-7")
            ctx = gf.Context(dims, gauge=gf.LANDAU, prec=prec, params=params(prec, 0))
            U = ctx.pack(U64 if prec == gf.F64 else U64.to(torch.complex64))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ctx.fix(U, args.omega, 1e-7, 20000)
            torch.cuda.synchronize()
            conv[name] = dict(seconds=time.perf_counter() - t0, sweeps=r["iters"], converged=r["converged"],
                              F=r["F"], theta=r["theta"])
            del U, ctx
            torch.cuda.empty_cache()
        for w in (1.5, 1.9):
            log(f"fp32 run to theta < 1e-7 at omega {w}")
            ctx = gf.Context(dims, gauge=gf.LANDAU, prec=gf.F32, params=params(gf.F32, 0))
            U = ctx.pack(U64.to(torch.complex64))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ctx.fix(U, w, 1e-7, 20000)
            torch.cuda.synchronize()
            conv[f"fp32_omega_{w}"] = dict(seconds=time.perf_counter() - t0, sweeps=r["iters"],
                                           converged=r["converged"], F=r["F"], theta=r["theta"])
            del U, ctx
            torch.cuda.empty_cache()
        log("fp32 steepest descent with Fourier acceleration (alpha 0.08) to theta < 1e-7")
        ctx = gf.Context(dims, gauge=gf.LANDAU, prec=gf.F32, params=params(gf.F32, 0))
        U = ctx.pack(U64.to(torch.complex64))
        ctx.sd_step(U, 0.08)  # plans and scratch are made on the first call
        U = ctx.pack(U64.to(torch.complex64))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.sd_fix(U, 0.08, 1e-7, 5000)
        torch.cuda.synchronize()
        conv["fp32_sd_fourier"] = dict(seconds=time.perf_counter() - t0, steps=r["iters"],
                                       converged=r["converged"], F=r["F"], theta=r["theta"])
        del U, ctx
        torch.cuda.empty_cache()
        conv["fp32_speedup_to_theta_1e-7"] = conv["fp64"]["seconds"] / conv["fp32"]["seconds"]
        conv["abs_F_fp32_minus_fp64"] = abs(conv["fp32"]["F"] - conv["fp64"]["F"])
        conv["theta_convention"] = "literal eq. (3): A = M - M^+, minus trace/3, no 1/2 or 1/(2i)"
        out["convergence"] = conv

    if not args.no_fixed_sweeps:
        out["fixed_sweeps"] = run_fixed_sweeps(gf, torch, U64, dims, params)

    if not args.no_slab:
        out["slab_48x48x48x12"] = run_slab_shape(gf, synth, torch)

    if not args.no_diff:
        out["differentiation"] = run_diff(gf, synth, torch)

    if not args.no_sun:
        out["sun"] = run_sun(args, dims, gf, synth, torch)

    if not args.no_bw_reference:
        log("HBM reference: device copy and in-place read-modify-write of a field-sized buffer")
        out["bandwidth_reference"] = bw_reference(torch, rf32["bytes_per_launch"] // 2, rf32["achieved_gbs"])

    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * a.numel() * 4

    U32f = None
    if not args.no_precision_32:
        out["precision_32x4"], U32f = run_precision_32(gf, synth, torch)

    if not args.no_ensemble:
        ens = run_ensemble(args, gf, synth, torch, np)
        ens.pop("workload", None)
        out["ensemble"] = ens

    if not args.no_cpu_baseline:
        fields = {"x".join(map(str, dims)): (U64.cpu().numpy(), dims)}
        del U64
        if U32f is None:
            U32f = synth.random_gauge_field((32, 32, 32, 32), 0.5, 0, device="cuda")
        fields["32x32x32x32"] = (U32f.cpu().numpy(), (32, 32, 32, 32))
        del U32f
        torch.cuda.empty_cache()
        t16 = gpu_fp64_time_16(gf, synth, torch)
        out["cpu_baseline"] = run_cpu_baseline(gf, synth, torch, fields, "x".join(map(str, dims)), value, t16)
        out["gpu_over_cpu"] = out["cpu_baseline"]["gpu_over_cpu_threads"]

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
