// api.cpp -- the C ABI of libgf (declared in include/gf.h): contexts,
// argument validation, the Alg. 1 drivers for one lattice and for ensembles
// (with hipGraph replay of a check period), the schedule autotuner and
// kernel timing. All device work goes to the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "gf.h"
#include "gf_internal.hpp"
#include "fft.hpp"
#include "gf_math.hpp"
#include "link8.hpp"
#include "sun_internal.hpp"

using namespace gf;

// Hash of the library's sources, set by the build; keys autotuner cache
// entries so that a schedule measured on other kernels is not reused.
#ifndef GF_SOURCE_HASH
#define GF_SOURCE_HASH "unknown"
#endif

struct gf_ctx {
    int n = 0;
    int prec = 0;
    int nc = 3;                      // colours: 3, or 2 / 4 (SU(N) kernels)
    int nelem = 9;
    int device = 0;
    hipStream_t stream = nullptr;
    gf_params p{};
    std::vector<CfgDesc> desc;       // host copy of the member table
    CfgDesc *d_desc = nullptr;
    CfgDesc *h_stage = nullptr;      // pinned staging for table uploads
    hipEvent_t stage_evt = nullptr;  // last upload from h_stage
    int *d_tile_cfg = nullptr;
    int tile_cap = 0;
    int ntiles = 0;
    int *d_qtile_cfg = nullptr;
    int nqtiles = 0;
    SlabOrder qslab{0, 0, 0, 0, 0};  // quality tile order (single lattices only)
    bool qstream = false;            // F/theta by k_quality_tstream (single SU(3) lattices)
    double *d_partials = nullptr;
    double *d_result = nullptr;      // 2 per member
    int *d_active = nullptr;         // per member (batch driver)
    int *d_ones = nullptr;           // per member, all 1 (plain calls)
    int *d_iters = nullptr;
    double *h_result = nullptr;      // pinned: 2n results
    int *h_flags = nullptr;          // pinned: n active, n iters, n ones
    Schedule sched{};
    long long sweeps_done = 0;
    std::string err;
    // timing
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_busy, ev_free;
    // graphs of check periods, keyed by (sweeps, reunit pattern, bits of eps):
    // eps is a kernel argument of the captured final reduction
    std::map<std::tuple<int, unsigned long long, unsigned long long>, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
    hipStream_t cap_stream = nullptr;
    // differentiation scratch: g field (9 complex per site) and partials
    void *d_gfield = nullptr;
    double *d_fpart = nullptr;
    double *d_fout = nullptr;
    // Fourier-accelerated steepest descent: the half spectrum of the su(3)
    // components of Delta, and the tables of roots of unity for the x, y, z
    // and t lengths (FFT_MAX_N complex doubles each)
    void *d_spec = nullptr;
    void *d_roots = nullptr;
    // per-time-slice quality: partials and results
    double *d_slice_part = nullptr;
    double *d_slice_out = nullptr;
    // per-check JSON-lines log of the fix drivers (gf_params.log_path)
    std::string log_path;
    FILE *log = nullptr;
    long long log_calls = 0;
};

namespace {

int fail(gf_ctx *ctx, int code, const char *fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

#define HIPTRY(ctx, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(ctx, GF_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));         \
    } while (0)

#define CHECK(ctx, cond, code, ...)                                                              \
    do {                                                                                         \
        if (!(cond)) return fail(ctx, code, __VA_ARGS__);                                        \
    } while (0)

// ---- per-check log (gf_params.log_path) ----------------------------------
// One JSON object per line and per member at every F/theta evaluation of a
// fix driver: the driver ("alg1" overrelaxation, "alg2" Fourier-accelerated
// steepest descent), the driver call's number within the context, the
// member, its sweeps (steps) so far in this call, F, theta and the seconds
// since the call began. Appended to the file, flushed after every check.
using Clock = std::chrono::steady_clock;

void log_open(gf_ctx *ctx) {
    if (!ctx->log && !ctx->log_path.empty()) ctx->log = std::fopen(ctx->log_path.c_str(), "a");
}

void log_check(gf_ctx *ctx, bool sd, int member, long long iters, double F, double theta,
               Clock::time_point t0) {
    if (!ctx->log) return;
    const double el = std::chrono::duration<double>(Clock::now() - t0).count();
    std::fprintf(ctx->log,
                 "{\"driver\": \"%s\", \"call\": %lld, \"member\": %d, \"%s\": %lld, \"F\": %.17g, "
                 "\"theta\": %.17g, \"elapsed_s\": %.9f}\n",
                 sd ? "alg2" : "alg1", ctx->log_calls, member, sd ? "step" : "sweep", iters, F, theta, el);
}

void log_flush(gf_ctx *ctx) {
    if (ctx->log) std::fflush(ctx->log);
}

// Make the context's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

size_t csize(const gf_ctx *c) { return c->prec == GF_F64 ? 16 : 8; }

int check_dims(gf_ctx *ctx, const int *d) {
    CHECK(ctx, d != nullptr, GF_EINVAL, "dims is NULL");
    long long V = 1;
    for (int i = 0; i < 4; i++) {
        CHECK(ctx, d[i] >= 2 && d[i] % 2 == 0, GF_EINVAL,
              "dims[%d] = %d: every lattice dimension must be even and >= 2", i, d[i]);
        V *= d[i];
    }
    CHECK(ctx, 4 * V < (1LL << 31), GF_EINVAL, "lattice volume %lld too large (4V must fit 31 bits)", V);
    return GF_OK;
}

int check_field(gf_ctx *ctx, const void *U, const char *what) {
    CHECK(ctx, U != nullptr, GF_EINVAL, "%s is NULL", what);
    CHECK(ctx, (reinterpret_cast<uintptr_t>(U) & 15) == 0, GF_EINVAL,
          "%s must be at least 16-byte aligned", what);
    return GF_OK;
}

int check_omega(gf_ctx *ctx, double omega) {
    CHECK(ctx, std::isfinite(omega) && omega > 0.0 && omega < 2.0, GF_EINVAL,
          "omega = %g must lie in (0, 2)", omega);
    return GF_OK;
}

// Defaults from the schedule sweep at 48^4 on MI355X (blocked layout): one
// lane per site with non-temporal link traffic; 128-thread workgroups, 256
// for 12-real float storage. SU(4) links need LPS >= 2 (registers); the
// SU(N) sweep at 48^4 is fastest with LPS 2 for SU(4) and for double SU(2).
Schedule default_schedule(int prec, int nc, const gf_params &p) {
    Schedule s;
    s.lps = p.lanes_per_site > 0 ? p.lanes_per_site : ((nc == 4 || (nc == 2 && prec == GF_F64)) ? 2 : 1);
    s.block = p.block_threads > 0 ? p.block_threads
                                   : ((prec == GF_F32 && p.storage != GF_STORE_18) ? 256 : 128);
    s.nt = p.nontemporal >= 0 ? p.nontemporal : 1;
    s.order = p.tile_order >= 0 ? p.tile_order : 0;
    return s;
}

int check_schedule(gf_ctx *ctx, const Schedule &s, int nc) {
    CHECK(ctx, s.lps == 1 || s.lps == 2 || s.lps == 4 || s.lps == 8, GF_EINVAL,
          "lanes_per_site = %d must be 1, 2, 4 or 8", s.lps);
    CHECK(ctx, nc != 4 || s.lps >= 2, GF_EINVAL, "SU(4) links need lanes_per_site >= 2");
    CHECK(ctx, s.block >= 64 && s.block <= 256 && s.block % 64 == 0, GF_EINVAL,
          "block_threads = %d must be 64, 128, 192 or 256", s.block);
    CHECK(ctx, s.order == 0 || s.order == 1, GF_EINVAL, "tile_order = %d must be 0 or 1", s.order);
    return GF_OK;
}

void destroy_graphs(gf_ctx *ctx) {
    for (auto &kv : ctx->graphs) {
        (void)hipGraphExecDestroy(kv.second.second);
        (void)hipGraphDestroy(kv.second.first);
    }
    ctx->graphs.clear();
}

// Upload the member table (after the previous upload from the staging
// buffer has been consumed).
int upload_desc(gf_ctx *ctx) {
    HIPTRY(ctx, hipEventSynchronize(ctx->stage_evt));
    std::memcpy(ctx->h_stage, ctx->desc.data(), ctx->n * sizeof(CfgDesc));
    HIPTRY(ctx, hipMemcpyAsync(ctx->d_desc, ctx->h_stage, ctx->n * sizeof(CfgDesc),
                               hipMemcpyHostToDevice, ctx->stream));
    HIPTRY(ctx, hipEventRecord(ctx->stage_evt, ctx->stream));
    return GF_OK;
}

// (Re)build the sweep tile map for the current schedule.
int build_tiles(gf_ctx *ctx) {
    const int spt = ctx->sched.block / ctx->sched.lps;
    std::vector<int> map;
    for (int c = 0; c < ctx->n; c++) {
        ctx->desc[c].tile0 = (int)map.size();
        const int nt = (ctx->desc[c].g.Vh + spt - 1) / spt;
        map.insert(map.end(), nt, c);
    }
    if ((int)map.size() > ctx->tile_cap) {
        if (ctx->d_tile_cfg) HIPTRY(ctx, hipFree(ctx->d_tile_cfg));
        ctx->d_tile_cfg = nullptr;
        if (hipMalloc(&ctx->d_tile_cfg, map.size() * sizeof(int)) != hipSuccess)
            return fail(ctx, GF_ENOMEM, "cannot allocate the tile map (%zu tiles)", map.size());
        ctx->tile_cap = (int)map.size();
    }
    ctx->ntiles = (int)map.size();
    HIPTRY(ctx, hipStreamSynchronize(ctx->stream));  // no launch may still read the old map
    HIPTRY(ctx, hipMemcpy(ctx->d_tile_cfg, map.data(), map.size() * sizeof(int), hipMemcpyHostToDevice));
    destroy_graphs(ctx);
    return upload_desc(ctx);
}

// Point the member table at the given fields / omegas, uploading only on change.
int set_fields(gf_ctx *ctx, void *const *U, const double *omega) {
    bool changed = false;
    for (int c = 0; c < ctx->n; c++) {
        if (ctx->desc[c].U != U[c]) { ctx->desc[c].U = U[c]; changed = true; }
        const double w = omega ? omega[c] : ctx->desc[c].omega;
        if (ctx->desc[c].omega != w) { ctx->desc[c].omega = w; changed = true; }
    }
    if (changed) return upload_desc(ctx);
    return GF_OK;
}

int half_sweep(gf_ctx *ctx, int parity, int reunit, const int *d_active) {
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (ctx->p.timing) {
        if (ctx->ev_free.empty()) {
            HIPTRY(ctx, hipEventCreate(&ev.first));
            HIPTRY(ctx, hipEventCreate(&ev.second));
        } else {
            ev = ctx->ev_free.back();
            ctx->ev_free.pop_back();
        }
        HIPTRY(ctx, hipEventRecord(ev.first, ctx->stream));
    }
    if (ctx->nc == 3)
        HIPTRY(ctx, launch_half_sweep(ctx->prec, ctx->nelem, ctx->sched, ctx->d_desc, ctx->d_tile_cfg,
                                      d_active, ctx->ntiles, parity, reunit, ctx->stream));
    else
        HIPTRY(ctx, launch_sun_half_sweep(ctx->prec, ctx->nc, ctx->sched, ctx->d_desc, ctx->d_tile_cfg,
                                          d_active, ctx->ntiles, parity, reunit, ctx->stream));
    if (ctx->p.timing) {
        HIPTRY(ctx, hipEventRecord(ev.second, ctx->stream));
        ctx->ev_busy.push_back(ev);
    }
    return GF_OK;
}

bool reunit_due(const gf_ctx *ctx, long long sweep_index) {
    return ctx->p.reunit_every > 0 && sweep_index % ctx->p.reunit_every == 0;
}

// n full sweeps on `st` (the context stream, or a capture stream), with
// the reunitarisation schedule continuing from ctx->sweeps_done.
int full_sweeps(gf_ctx *ctx, int n, const int *d_active, hipStream_t st) {
    hipStream_t keep = ctx->stream;
    ctx->stream = st;
    int rc = GF_OK;
    for (int i = 0; i < n && rc == GF_OK; i++) {
        rc = half_sweep(ctx, 0, 0, d_active);
        if (rc == GF_OK) rc = half_sweep(ctx, 1, reunit_due(ctx, ctx->sweeps_done + 1) ? 1 : 0, d_active);
        if (rc == GF_OK) ctx->sweeps_done++;
    }
    ctx->stream = keep;
    return rc;
}

int quality_launch(gf_ctx *ctx, const int *d_active, int update, int swept, double eps, hipStream_t st) {
    if (ctx->qstream)
        HIPTRY(ctx, launch_quality_tstream(ctx->prec, ctx->nelem, ctx->desc[0].g, ctx->d_desc, d_active,
                                           ctx->d_partials, st));
    else if (ctx->nc == 3)
        HIPTRY(ctx, launch_quality(ctx->prec, ctx->nelem, ctx->d_desc, ctx->d_qtile_cfg, d_active,
                                   ctx->nqtiles, ctx->d_partials, ctx->qslab, st));
    else
        HIPTRY(ctx, launch_sun_quality(ctx->prec, ctx->nc, ctx->d_desc, ctx->d_qtile_cfg, d_active,
                                       ctx->nqtiles, ctx->d_partials, ctx->qslab, st));
    HIPTRY(ctx, launch_quality_final_nc(ctx->nc, ctx->d_desc, ctx->n, ctx->d_partials, ctx->d_result,
                                        update ? ctx->d_active : nullptr, ctx->d_iters, swept, eps,
                                        update, st));
    return GF_OK;
}

// Copy results (and, for the batch driver, the flags) to pinned memory and wait.
int read_back(gf_ctx *ctx, bool flags) {
    HIPTRY(ctx, hipMemcpyAsync(ctx->h_result, ctx->d_result, 2 * ctx->n * sizeof(double),
                               hipMemcpyDeviceToHost, ctx->stream));
    if (flags) {
        HIPTRY(ctx, hipMemcpyAsync(ctx->h_flags, ctx->d_active, ctx->n * sizeof(int),
                                   hipMemcpyDeviceToHost, ctx->stream));
        HIPTRY(ctx, hipMemcpyAsync(ctx->h_flags + ctx->n, ctx->d_iters, ctx->n * sizeof(int),
                                   hipMemcpyDeviceToHost, ctx->stream));
    }
    HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
    return GF_OK;
}

int create_impl(gf_ctx **out, int n, const int *dims, const int *gauge, int prec, void *stream,
                const gf_params *pp, int nc) {
    if (!out) return GF_EINVAL;
    *out = nullptr;
    gf_ctx tmp;  // for error messages during validation
    if (n < 1) return GF_EINVAL;
    if (prec != GF_F64 && prec != GF_F32) return GF_EINVAL;
    for (int c = 0; c < n; c++) {
        if (check_dims(&tmp, dims + 4 * c) != GF_OK) return GF_EINVAL;
        if (gauge[c] != GF_LANDAU && gauge[c] != GF_COULOMB) return GF_EINVAL;
    }
    gf_params p;
    gf_params_default(&p, prec);
    if (pp) p = *pp;
    if (p.check_every < 1) p.check_every = 1;
    if (p.reunit_every < 0) return GF_EINVAL;
    if (p.storage != GF_STORE_18 && p.storage != GF_STORE_12 && p.storage != GF_STORE_8) return GF_EINVAL;
    if (nc != 3 && p.storage != GF_STORE_18) return GF_EUNSUPPORTED;  // 12-/8-real are SU(3) only
    Schedule s = default_schedule(prec, nc, p);
    if (check_schedule(&tmp, s, nc) != GF_OK) return GF_EINVAL;

    gf_ctx *ctx = new gf_ctx();
    ctx->n = n;
    ctx->prec = prec;
    ctx->nc = nc;
    ctx->nelem = nc != 3 ? nc * nc : (p.storage == GF_STORE_12 ? 6 : p.storage == GF_STORE_8 ? 4 : 9);
    ctx->stream = (hipStream_t)stream;
    ctx->p = p;
    ctx->sched = s;
    ctx->sweeps_done = p.start_sweep;
    if (p.log_path) ctx->log_path = p.log_path;
    ctx->p.log_path = nullptr;  // the context keeps its own copy
    int rc = GF_OK;
    auto bail = [&](int code) { gf_destroy(ctx); return code; };
    if (hipGetDevice(&ctx->device) != hipSuccess) return bail(GF_EDEVICE);
    ctx->desc.resize(n);
    int nq = 0;
    for (int c = 0; c < n; c++) {
        CfgDesc &d = ctx->desc[c];
        std::memset(&d, 0, sizeof d);
        d.g = make_geom(dims + 4 * c, ctx->nelem);
        d.gauge = gauge[c];
        d.omega = 1.0;
        d.qtile0 = nq;
        d.nqtiles = (d.g.Vh + QTILE / 2 - 1) / (QTILE / 2);  // QTILE/2 half-indices, both parities
        nq += d.nqtiles;
    }
    ctx->nqtiles = nq;
    // an ensemble's tiles are several lattices end to end: plain order there
    if (n == 1) {
        const Geom &g0 = ctx->desc[0].g;
        const int nd = ctx->desc[0].gauge == GF_LANDAU ? 4 : 3;
        const long long tile_bytes = (long long)QTILE * nd * ctx->nelem * 2 * (prec == GF_F64 ? 8 : 4);
        ctx->qslab = pick_slab_order(g0.st, g0.sz, g0.hx, g0.nz, QTILE / 2, nq, tile_bytes);
    }
    // in double a single lattice's F/theta walks time slices (its tiles' t neighbours
    // missed L2 in any slab order); in float the slab order is as fast
    ctx->qstream = n == 1 && ctx->nc == 3 && prec == GF_F64 && quality_tstream_ok(ctx->desc[0].g);
    std::vector<int> qmap;
    for (int c = 0; c < n; c++) qmap.insert(qmap.end(), ctx->desc[c].nqtiles, c);
    if (hipMalloc(&ctx->d_desc, n * sizeof(CfgDesc)) != hipSuccess ||
        hipMalloc(&ctx->d_qtile_cfg, nq * sizeof(int)) != hipSuccess ||
        hipMalloc(&ctx->d_partials, 2 * (size_t)nq * sizeof(double)) != hipSuccess ||
        hipMalloc(&ctx->d_result, 2 * n * sizeof(double)) != hipSuccess ||
        hipMalloc(&ctx->d_active, n * sizeof(int)) != hipSuccess ||
        hipMalloc(&ctx->d_ones, n * sizeof(int)) != hipSuccess ||
        hipMalloc(&ctx->d_iters, n * sizeof(int)) != hipSuccess ||
        hipHostMalloc(&ctx->h_stage, n * sizeof(CfgDesc), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&ctx->h_result, 2 * n * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&ctx->h_flags, 3 * n * sizeof(int), hipHostMallocDefault) != hipSuccess)
        return bail(GF_ENOMEM);
    if (hipEventCreateWithFlags(&ctx->stage_evt, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(GF_EDEVICE);
    for (int c = 0; c < n; c++) ctx->h_flags[2 * n + c] = 1;
    if (hipMemcpy(ctx->d_ones, ctx->h_flags + 2 * n, n * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ctx->d_active, ctx->h_flags + 2 * n, n * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ctx->d_qtile_cfg, qmap.data(), nq * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        return bail(GF_EDEVICE);
    rc = build_tiles(ctx);
    if (rc != GF_OK) return bail(rc);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return bail(GF_EDEVICE);
    *out = ctx;
    return GF_OK;
}

int need_single(gf_ctx *ctx) {
    CHECK(ctx, ctx->n == 1, GF_EINVAL, "this entry point needs a single-lattice context (n = %d)", ctx->n);
    return GF_OK;
}

// The su(3)-algebra entry points (differentiation, Fourier-accelerated
// steepest descent) exist for N = 3 only.
int need_su3(gf_ctx *ctx) {
    CHECK(ctx, ctx->nc == 3, GF_EUNSUPPORTED, "this entry point is implemented for SU(3) only (nc = %d)", ctx->nc);
    return GF_OK;
}

}  // namespace

extern "C" {

void gf_params_default(gf_params *p, int prec) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->check_every = 1;
    p->reunit_every = prec == GF_F64 ? 20 : 10;
    p->start_sweep = 0;
    p->storage = GF_STORE_18;
    p->nontemporal = -1;
    p->tile_order = -1;
}

int gf_create(gf_ctx **out, const int dims[4], int nc, int gauge, int prec, void *stream,
              const gf_params *p) {
    if (!out) return GF_EINVAL;
    *out = nullptr;
    if (nc != 2 && nc != 3 && nc != 4) return GF_EUNSUPPORTED;
    return create_impl(out, 1, dims, &gauge, prec, stream, p, nc);
}

int gf_batch_create(gf_ctx **out, int n, const int *dims, const int *gauge, int prec, void *stream,
                    const gf_params *p) {
    if (!out) return GF_EINVAL;
    *out = nullptr;
    if (n < 1 || !dims || !gauge) return GF_EINVAL;
    return create_impl(out, n, dims, gauge, prec, stream, p, 3);
}

int gf_destroy(gf_ctx *ctx) {
    if (!ctx) return GF_OK;
    DeviceGuard dg(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    destroy_graphs(ctx);
    for (auto &e : ctx->ev_busy) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    for (auto &e : ctx->ev_free) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    if (ctx->stage_evt) (void)hipEventDestroy(ctx->stage_evt);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    (void)hipFree(ctx->d_desc);
    (void)hipFree(ctx->d_tile_cfg);
    (void)hipFree(ctx->d_qtile_cfg);
    (void)hipFree(ctx->d_partials);
    (void)hipFree(ctx->d_result);
    (void)hipFree(ctx->d_active);
    (void)hipFree(ctx->d_ones);
    (void)hipFree(ctx->d_iters);
    (void)hipFree(ctx->d_spec);
    (void)hipFree(ctx->d_roots);
    (void)hipFree(ctx->d_gfield);
    (void)hipFree(ctx->d_fpart);
    (void)hipFree(ctx->d_fout);
    if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
    if (ctx->h_result) (void)hipHostFree(ctx->h_result);
    if (ctx->h_flags) (void)hipHostFree(ctx->h_flags);
    (void)hipFree(ctx->d_slice_part);
    (void)hipFree(ctx->d_slice_out);
    if (ctx->log) std::fclose(ctx->log);
    delete ctx;
    return GF_OK;
}

int gf_batch_destroy(gf_ctx *ctx) { return gf_destroy(ctx); }

const char *gf_last_error(const gf_ctx *ctx) { return ctx ? ctx->err.c_str() : noalloc_last_error(); }

size_t gf_field_bytes(const gf_ctx *ctx, int member) {
    if (!ctx || member < 0 || member >= ctx->n) return 0;
    return (size_t)field_complex(ctx->desc[member].g) * csize(ctx);
}

int gf_pack(gf_ctx *ctx, const void *U_aos, void *U) {
    if (!ctx) return GF_EINVAL;
    int rc;
    if ((rc = need_single(ctx)) || (rc = check_field(ctx, U_aos, "U_aos")) || (rc = check_field(ctx, U, "U")))
        return rc;
    DeviceGuard dg(ctx->device);
    if (ctx->nc == 3)
        HIPTRY(ctx, launch_pack(ctx->prec, ctx->nelem, ctx->desc[0].g, U_aos, U, 0, ctx->stream));
    else
        HIPTRY(ctx, launch_sun_pack(ctx->prec, ctx->nc, ctx->desc[0].g, U_aos, U, 0, ctx->stream));
    return GF_OK;
}

int gf_unpack(gf_ctx *ctx, const void *U, void *U_aos) {
    if (!ctx) return GF_EINVAL;
    int rc;
    if ((rc = need_single(ctx)) || (rc = check_field(ctx, U_aos, "U_aos")) || (rc = check_field(ctx, U, "U")))
        return rc;
    DeviceGuard dg(ctx->device);
    if (ctx->nc == 3)
        HIPTRY(ctx, launch_pack(ctx->prec, ctx->nelem, ctx->desc[0].g, U_aos, const_cast<void *>(U), 1,
                                ctx->stream));
    else
        HIPTRY(ctx, launch_sun_pack(ctx->prec, ctx->nc, ctx->desc[0].g, U_aos, const_cast<void *>(U), 1,
                                    ctx->stream));
    return GF_OK;
}

int gf_sweep(gf_ctx *ctx, void *U, int parity, double omega) {
    if (!ctx) return GF_EINVAL;
    int rc;
    if ((rc = need_single(ctx)) || (rc = check_field(ctx, U, "U")) || (rc = check_omega(ctx, omega)))
        return rc;
    CHECK(ctx, parity == 0 || parity == 1, GF_EINVAL, "parity must be 0 or 1");
    DeviceGuard dg(ctx->device);
    if ((rc = set_fields(ctx, &U, &omega))) return rc;
    return half_sweep(ctx, parity, 0, ctx->d_ones);
}

int gf_sweeps(gf_ctx *ctx, void *U, double omega, int nsweeps) {
    if (!ctx) return GF_EINVAL;
    int rc;
    if ((rc = need_single(ctx)) || (rc = check_field(ctx, U, "U")) || (rc = check_omega(ctx, omega)))
        return rc;
    CHECK(ctx, nsweeps >= 0, GF_EINVAL, "nsweeps must be >= 0");
    DeviceGuard dg(ctx->device);
    if ((rc = set_fields(ctx, &U, &omega))) return rc;
    return full_sweeps(ctx, nsweeps, ctx->d_ones, ctx->stream);
}

int gf_reunit(gf_ctx *ctx, void *U) {
    if (!ctx) return GF_EINVAL;
    int rc;
    if ((rc = need_single(ctx)) || (rc = check_field(ctx, U, "U"))) return rc;
    DeviceGuard dg(ctx->device);
    if (ctx->nc == 3)
        HIPTRY(ctx, launch_reunit(ctx->prec, ctx->nelem, ctx->desc[0].g, U, ctx->stream));
    else
        HIPTRY(ctx, launch_sun_reunit(ctx->prec, ctx->nc, ctx->desc[0].g, U, ctx->stream));
    return GF_OK;
}

int gf_batch_quality(gf_ctx *ctx, void *const *U, double *F, double *theta) {
    if (!ctx) return GF_EINVAL;
    CHECK(ctx, U && F && theta, GF_EINVAL, "NULL argument");
    int rc;
    for (int c = 0; c < ctx->n; c++)
        if ((rc = check_field(ctx, U[c], "U[i]"))) return rc;
    DeviceGuard dg(ctx->device);
    if ((rc = set_fields(ctx, U, nullptr))) return rc;
    if ((rc = quality_launch(ctx, nullptr, 0, 0, 0.0, ctx->stream))) return rc;
    if ((rc = read_back(ctx, false))) return rc;
    int bad = 0;
    for (int c = 0; c < ctx->n; c++) {
        F[c] = ctx->h_result[2 * c];
        theta[c] = ctx->h_result[2 * c + 1];
        if (!std::isfinite(F[c]) || !std::isfinite(theta[c])) bad = 1;
    }
    if (bad) return fail(ctx, GF_ENONFINITE, "F or theta is not finite");
    return GF_OK;
}

int gf_quality(gf_ctx *ctx, const void *U, double *F, double *theta) {
    if (!ctx) return GF_EINVAL;
    int rc;
    if ((rc = need_single(ctx))) return rc;
    void *u = const_cast<void *>(U);
    return gf_batch_quality(ctx, &u, F, theta);
}

int gf_quality_slices(gf_ctx *ctx, const void *U, double *F_t, double *theta_t) {
    if (!ctx) return GF_EINVAL;
    int rc;
    if ((rc = need_single(ctx)) || (rc = need_su3(ctx)) || (rc = check_field(ctx, U, "U"))) return rc;
    CHECK(ctx, F_t && theta_t, GF_EINVAL, "NULL argument");
    DeviceGuard dg(ctx->device);
    const Geom &g = ctx->desc[0].g;
    if (!ctx->d_slice_part) {
        const size_t np = 2 * (size_t)g.nt * quality_slice_chunks(g);
        if (hipMalloc(&ctx->d_slice_part, np * sizeof(double)) != hipSuccess) {
            ctx->d_slice_part = nullptr;
            return fail(ctx, GF_ENOMEM, "cannot allocate the per-slice partials");
        }
    }
    if (!ctx->d_slice_out && hipMalloc(&ctx->d_slice_out, 2 * (size_t)g.nt * sizeof(double)) != hipSuccess) {
        ctx->d_slice_out = nullptr;
        return fail(ctx, GF_ENOMEM, "cannot allocate the per-slice results");
    }
    CfgDesc d = ctx->desc[0];
    d.U = const_cast<void *>(U);
    HIPTRY(ctx, launch_quality_slices(ctx->prec, ctx->nelem, d, ctx->d_slice_part, ctx->d_slice_out, ctx->stream));
    std::vector<double> h(2 * (size_t)g.nt);
    HIPTRY(ctx, hipMemcpyAsync(h.data(), ctx->d_slice_out, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
    bool bad = false;
    for (int t = 0; t < g.nt; t++) {
        F_t[t] = h[2 * t];
        theta_t[t] = h[2 * t + 1];
        if (!std::isfinite(F_t[t]) || !std::isfinite(theta_t[t])) bad = true;
    }
    if (bad) return fail(ctx, GF_ENONFINITE, "a slice's F or theta is not finite");
    return GF_OK;
}

int gf_fix(gf_ctx *ctx, void *U, double omega, double eps, int max_iter, int *iters, double *F,
           double *theta) {
    if (!ctx) return GF_EINVAL;
    int rc;
    if ((rc = need_single(ctx))) return rc;
    return gf_batch_fix(ctx, &U, &omega, eps, max_iter, iters, F, theta);
}

int gf_batch_fix(gf_ctx *ctx, void *const *U, const double *omega, double eps, int max_iter,
                 int *iters, double *F, double *theta) {
    if (!ctx) return GF_EINVAL;
    CHECK(ctx, U && omega && iters && F && theta, GF_EINVAL, "NULL argument");
    CHECK(ctx, std::isfinite(eps) && eps >= 0.0, GF_EINVAL, "eps must be finite and >= 0");
    CHECK(ctx, max_iter >= 0, GF_EINVAL, "max_iter must be >= 0");
    int rc;
    for (int c = 0; c < ctx->n; c++) {
        if ((rc = check_field(ctx, U[c], "U[i]")) || (rc = check_omega(ctx, omega[c]))) return rc;
    }
    DeviceGuard dg(ctx->device);
    if ((rc = set_fields(ctx, U, omega))) return rc;
    const int n = ctx->n;
    const Clock::time_point t0 = Clock::now();
    log_open(ctx);
    ctx->log_calls++;
    // every member starts active with zero sweeps
    for (int c = 0; c < n; c++) { ctx->h_flags[c] = 1; ctx->h_flags[n + c] = 0; }
    HIPTRY(ctx, hipMemcpyAsync(ctx->d_active, ctx->h_flags, n * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    HIPTRY(ctx, hipMemcpyAsync(ctx->d_iters, ctx->h_flags + n, n * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    if ((rc = quality_launch(ctx, ctx->d_active, 1, 0, eps, ctx->stream))) return rc;
    if ((rc = read_back(ctx, true))) return rc;
    // members active before a check (those whose result it refreshed)
    std::vector<int> was_active(n, 1);
    auto log_members = [&]() {
        if (!ctx->log) return;
        for (int c = 0; c < n; c++)
            if (was_active[c])
                log_check(ctx, false, c, ctx->h_flags[n + c], ctx->h_result[2 * c], ctx->h_result[2 * c + 1], t0);
        log_flush(ctx);
        for (int c = 0; c < n; c++) was_active[c] = ctx->h_flags[c];
    };
    log_members();
    const bool graphs = ctx->p.use_graph && !ctx->p.timing && ctx->p.check_every <= 64;
    int it = 0;
    auto any_active = [&]() {
        for (int c = 0; c < n; c++) if (ctx->h_flags[c]) return true;
        return false;
    };
    auto nonfinite = [&]() {
        for (int c = 0; c < n; c++)
            if (!std::isfinite(ctx->h_result[2 * c]) || !std::isfinite(ctx->h_result[2 * c + 1])) return true;
        return false;
    };
    while (it < max_iter && any_active() && !nonfinite()) {
        const int m = std::min(ctx->p.check_every, max_iter - it);
        if (graphs) {
            unsigned long long pattern = 0;
            for (int k = 1; k <= m; k++)
                if (reunit_due(ctx, ctx->sweeps_done + k)) pattern |= 1ULL << (k - 1);
            unsigned long long eps_bits;
            std::memcpy(&eps_bits, &eps, sizeof eps_bits);
            auto key = std::make_tuple(m, pattern, eps_bits);
            auto f = ctx->graphs.find(key);
            if (f == ctx->graphs.end()) {
                hipGraph_t g;
                hipGraphExec_t ge;
                const long long keep = ctx->sweeps_done;
                HIPTRY(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
                int r1 = full_sweeps(ctx, m, ctx->d_active, ctx->cap_stream);
                int r2 = r1 ? r1 : quality_launch(ctx, ctx->d_active, 1, m, eps, ctx->cap_stream);
                hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &g);
                ctx->sweeps_done = keep;
                if (r2) return r2;
                HIPTRY(ctx, ec);
                HIPTRY(ctx, hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
                f = ctx->graphs.emplace(key, std::make_pair(g, ge)).first;
            }
            HIPTRY(ctx, hipGraphLaunch(f->second.second, ctx->stream));
            ctx->sweeps_done += m;
        } else {
            if ((rc = full_sweeps(ctx, m, ctx->d_active, ctx->stream))) return rc;
            if ((rc = quality_launch(ctx, ctx->d_active, 1, m, eps, ctx->stream))) return rc;
        }
        it += m;
        if ((rc = read_back(ctx, true))) return rc;
        log_members();
    }
    bool all = true;
    for (int c = 0; c < n; c++) {
        F[c] = ctx->h_result[2 * c];
        theta[c] = ctx->h_result[2 * c + 1];
        iters[c] = ctx->h_flags[n + c];
        if (!(theta[c] < eps)) all = false;
    }
    if (nonfinite()) return fail(ctx, GF_ENONFINITE, "F or theta is not finite");
    return all ? GF_OK : GF_NOT_CONVERGED;
}

int gf_get_schedule(const gf_ctx *ctx, int *lps, int *block, int *nt, int *tile_order) {
    if (!ctx) return GF_EINVAL;
    if (lps) *lps = ctx->sched.lps;
    if (block) *block = ctx->sched.block;
    if (nt) *nt = ctx->sched.nt;
    if (tile_order) *tile_order = ctx->sched.order;
    return GF_OK;
}

int gf_timing(gf_ctx *ctx, double *ms, long long *launches) {
    if (!ctx) return GF_EINVAL;
    DeviceGuard dg(ctx->device);
    HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
    double tot = 0.0;
    for (auto &e : ctx->ev_busy) {
        float t = 0.f;
        HIPTRY(ctx, hipEventElapsedTime(&t, e.first, e.second));
        tot += t;
        ctx->ev_free.push_back(e);
    }
    if (ms) *ms = tot;
    if (launches) *launches = (long long)ctx->ev_busy.size();
    ctx->ev_busy.clear();
    return GF_OK;
}

int gf_set_sweep_count(gf_ctx *ctx, long long s) {
    if (!ctx) return GF_EINVAL;
    CHECK(ctx, s >= 0, GF_EINVAL, "sweep count must be >= 0");
    ctx->sweeps_done = s;
    return GF_OK;
}

long long gf_get_sweep_count(const gf_ctx *ctx) { return ctx ? ctx->sweeps_done : -1; }

// ---- autotuner ----------------------------------------------------------

int gf_autotune(gf_ctx *ctx, void *const *U, double omega, const char *cache_path) {
    if (!ctx) return GF_EINVAL;
    CHECK(ctx, U != nullptr, GF_EINVAL, "U is NULL");
    int rc;
    for (int c = 0; c < ctx->n; c++)
        if ((rc = check_field(ctx, U[c], "U[i]"))) return rc;
    if ((rc = check_omega(ctx, omega))) return rc;
    DeviceGuard dg(ctx->device);
    hipDeviceProp_t prop;
    HIPTRY(ctx, hipGetDeviceProperties(&prop, ctx->device));
    std::ostringstream key;
    key << prop.gcnArchName << "|cu" << prop.multiProcessorCount << "|src" << GF_SOURCE_HASH << "|n" << ctx->nc
        << "|p" << ctx->prec << "|e" << ctx->nelem;
    for (int c = 0; c < ctx->n; c++) {
        const Geom &g = ctx->desc[c].g;
        key << "|" << g.nx << "x" << g.ny << "x" << g.nz << "x" << g.nt << "g" << ctx->desc[c].gauge;
    }
    const std::string k = key.str();
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line, found;
        while (std::getline(in, line))
            if (line.compare(0, k.size() + 1, k + " ") == 0) found = line.substr(k.size() + 1);
        if (!found.empty()) {
            Schedule s{};
            std::istringstream is(found);
            if (is >> s.lps >> s.block >> s.nt >> s.order && check_schedule(ctx, s, ctx->nc) == GF_OK) {
                ctx->sched = s;
                return build_tiles(ctx);
            }
        }
    }
    // scratch copy of every member's field
    std::vector<size_t> bytes(ctx->n);
    size_t total = 0;
    for (int c = 0; c < ctx->n; c++) { bytes[c] = (gf_field_bytes(ctx, c) + 255) & ~size_t(255); total += bytes[c]; }
    char *scratch = nullptr;
    if (hipMalloc(&scratch, total) != hipSuccess) return fail(ctx, GF_ENOMEM, "autotune scratch (%zu bytes)", total);
    rc = GF_OK;
    auto ok = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && rc == GF_OK) rc = fail(ctx, GF_EDEVICE, "autotune: %s failed: %s", what, hipGetErrorString(e));
        return rc == GF_OK;
    };
    std::vector<void *> su(ctx->n);
    size_t o = 0;
    for (int c = 0; c < ctx->n; c++) {
        su[c] = scratch + o;
        ok(hipMemcpyAsync(su[c], U[c], gf_field_bytes(ctx, c), hipMemcpyDeviceToDevice, ctx->stream), "hipMemcpyAsync");
        o += bytes[c];
    }
    std::vector<double> om(ctx->n, omega);
    std::vector<void *> keepU(ctx->n);
    std::vector<double> keepW(ctx->n);
    for (int c = 0; c < ctx->n; c++) { keepU[c] = ctx->desc[c].U; keepW[c] = ctx->desc[c].omega; }
    const Schedule keep = ctx->sched;
    const int keep_timing = ctx->p.timing;
    ctx->p.timing = 0;
    if (rc == GF_OK) rc = set_fields(ctx, su.data(), om.data());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ok(hipEventCreate(&e0), "hipEventCreate");
    ok(hipEventCreate(&e1), "hipEventCreate");
    Schedule best = keep;
    float best_ms = 1e30f;
    const int lps_list[] = {1, 2, 4, 8};
    const int block_list[] = {64, 128, 256};
    for (int li = 0; li < 4 && rc == GF_OK; li++)
        for (int bi = 0; bi < 3 && rc == GF_OK; bi++)
            for (int nt = 0; nt < 2 && rc == GF_OK; nt++)
                // XCD-contiguous shares only for a single lattice: in an ensemble the
                // members that converge first leave their XCDs' shares empty while the
                // others still carry the large members' tiles (measured on the uneven
                // ensemble: tuned with every member active it won, then ran 11 % slower)
                for (int order = 0; order < (ctx->n == 1 ? 2 : 1) && rc == GF_OK; order++) {
                    Schedule s{lps_list[li], block_list[bi], nt, order};
                    if (ctx->nc == 4 && s.lps < 2) continue;       // registers
                    if (ctx->nc != 3 && nt != 1) continue;         // SU(N) links are always non-temporal
                    ctx->sched = s;
                    if ((rc = build_tiles(ctx))) break;
                    for (int w = 0; w < 2 && rc == GF_OK; w++) rc = half_sweep(ctx, w & 1, 0, ctx->d_ones);
                    ok(hipEventRecord(e0, ctx->stream), "hipEventRecord");
                    for (int w = 0; w < 6 && rc == GF_OK; w++) rc = half_sweep(ctx, w & 1, 0, ctx->d_ones);
                    ok(hipEventRecord(e1, ctx->stream), "hipEventRecord");
                    ok(hipEventSynchronize(e1), "hipEventSynchronize");
                    float ms = 0.f;
                    ok(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
                    if (rc == GF_OK && ms < best_ms) { best_ms = ms; best = s; }
                }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    ctx->p.timing = keep_timing;
    ok(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    (void)hipFree(scratch);
    for (int c = 0; c < ctx->n; c++) { ctx->desc[c].U = keepU[c]; ctx->desc[c].omega = keepW[c]; }
    ctx->sched = rc == GF_OK ? best : keep;
    const int rc2 = build_tiles(ctx);  // also re-uploads the restored member table
    if (rc) return rc;
    if (rc2) return rc2;
    if (cache_path) {
        std::ofstream outf(cache_path, std::ios::app);
        outf << k << " " << best.lps << " " << best.block << " " << best.nt << " " << best.order << " "
             << best_ms / 6.0f << "\n";
    }
    return GF_OK;
}

// ---- differentiation --------------------------------------------------------

namespace {

int ensure_diff_scratch(gf_ctx *ctx) {
    const Geom &g = ctx->desc[0].g;
    // each buffer on its own, so a call after a failed allocation retries it
    if (!ctx->d_gfield && hipMalloc(&ctx->d_gfield, (size_t)gfield_complex(g) * csize(ctx)) != hipSuccess) {
        ctx->d_gfield = nullptr;
        return fail(ctx, GF_ENOMEM, "cannot allocate the g field");
    }
    const int nb = (g.V + 255) / 256;
    if (!ctx->d_fpart && hipMalloc(&ctx->d_fpart, nb * sizeof(double)) != hipSuccess) {
        ctx->d_fpart = nullptr;
        return fail(ctx, GF_ENOMEM, "cannot allocate functional partials");
    }
    if (!ctx->d_fout && hipMalloc(&ctx->d_fout, sizeof(double)) != hipSuccess) {
        ctx->d_fout = nullptr;
        return fail(ctx, GF_ENOMEM, "cannot allocate the functional result");
    }
    return GF_OK;
}

int diff_prologue(gf_ctx *ctx, const void *U, const void *s) {
    int rc;
    if ((rc = need_single(ctx)) || (rc = need_su3(ctx)) || (rc = check_field(ctx, U, "U")) ||
        (rc = check_field(ctx, s, "s")))
        return rc;
    if ((rc = ensure_diff_scratch(ctx))) return rc;
    HIPTRY(ctx, launch_expS(ctx->prec, ctx->desc[0].g, s, ctx->d_gfield, ctx->stream));
    return GF_OK;
}

}  // namespace

int gf_pack_alg(gf_ctx *ctx, const void *s_aos, void *s) {
    if (!ctx) return GF_EINVAL;
    int rc;
    if ((rc = need_single(ctx)) || (rc = need_su3(ctx)) || (rc = check_field(ctx, s_aos, "s_aos")) ||
        (rc = check_field(ctx, s, "s")))
        return rc;
    DeviceGuard dg(ctx->device);
    HIPTRY(ctx, launch_pack_alg(ctx->prec, ctx->desc[0].g, s_aos, s, 0, ctx->stream));
    return GF_OK;
}

int gf_unpack_alg(gf_ctx *ctx, const void *s, void *s_aos) {
    if (!ctx) return GF_EINVAL;
    int rc;
    if ((rc = need_single(ctx)) || (rc = need_su3(ctx)) || (rc = check_field(ctx, s_aos, "s_aos")) ||
        (rc = check_field(ctx, s, "s")))
        return rc;
    DeviceGuard dg(ctx->device);
    HIPTRY(ctx, launch_pack_alg(ctx->prec, ctx->desc[0].g, s_aos, const_cast<void *>(s), 1, ctx->stream));
    return GF_OK;
}

int gf_functional(gf_ctx *ctx, const void *U, const void *s, double *F) {
    if (!ctx) return GF_EINVAL;
    CHECK(ctx, F != nullptr, GF_EINVAL, "F is NULL");
    DeviceGuard dg(ctx->device);
    int rc;
    if ((rc = diff_prologue(ctx, U, s))) return rc;
    const Geom &g = ctx->desc[0].g;
    const int nb = (g.V + 255) / 256;
    HIPTRY(ctx, launch_functional(ctx->prec, ctx->nelem, ctx->desc[0].gauge, g, U, ctx->d_gfield,
                                  ctx->d_fpart, ctx->stream));
    HIPTRY(ctx, launch_sum_partials(ctx->d_fpart, nb, ctx->d_fout, ctx->stream));
    HIPTRY(ctx, hipMemcpyAsync(ctx->h_result, ctx->d_fout, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
    const int nd = ctx->desc[0].gauge == GF_LANDAU ? 4 : 3;
    *F = ctx->h_result[0] / (nd * 3.0 * (double)g.V);
    if (!std::isfinite(*F)) return fail(ctx, GF_ENONFINITE, "F is not finite");
    return GF_OK;
}

int gf_functional_grad(gf_ctx *ctx, const void *U, const void *s, double dF, void *grad) {
    if (!ctx) return GF_EINVAL;
    CHECK(ctx, std::isfinite(dF), GF_EINVAL, "dF must be finite");
    int rc;
    if ((rc = check_field(ctx, grad, "grad"))) return rc;
    DeviceGuard dg(ctx->device);
    if ((rc = diff_prologue(ctx, U, s))) return rc;
    HIPTRY(ctx, launch_functional_grad(ctx->prec, ctx->nelem, ctx->desc[0].gauge, ctx->desc[0].g, U, s,
                                       ctx->d_gfield, dF, grad, ctx->stream));
    return GF_OK;
}

int gf_gauge_transform(gf_ctx *ctx, void *U, const void *s) {
    if (!ctx) return GF_EINVAL;
    DeviceGuard dg(ctx->device);
    int rc;
    if ((rc = diff_prologue(ctx, U, s))) return rc;
    HIPTRY(ctx, launch_gauge_transform(ctx->prec, ctx->nelem, ctx->desc[0].g, U, ctx->d_gfield, ctx->stream));
    return GF_OK;
}

// ---- steepest descent with Fourier acceleration (Alg. 2) ----------------------

namespace {

// Buffers of one step: the half spectrum spec[t][a][z][y][kx] (kx = 0..nx/2)
// of the eight su(3) components of Delta, and the root tables. Made once per
// context; a call after a failed allocation retries what is missing.
int sd_prepare(gf_ctx *ctx) {
    const Geom &g = ctx->desc[0].g;
    CHECK(ctx, g.nx <= FFT_MAX_NX && g.ny <= FFT_MAX_N && g.nz <= FFT_MAX_N && g.nt <= FFT_MAX_N,
          GF_EUNSUPPORTED, "Fourier acceleration supports nx up to %d and ny, nz, nt up to %d", FFT_MAX_NX,
          FFT_MAX_N);
    int rc;
    if ((rc = ensure_diff_scratch(ctx))) return rc;
    const size_t rs = ctx->prec == GF_F64 ? 8 : 4;
    const long long S = (long long)g.nz * g.ny * (g.nx / 2 + 1);
    if (!ctx->d_spec && hipMalloc(&ctx->d_spec, 8 * (size_t)g.nt * S * 2 * rs) != hipSuccess) {
        ctx->d_spec = nullptr;
        return fail(ctx, GF_ENOMEM, "cannot allocate the Fourier acceleration buffers");
    }
    if (!ctx->d_roots) {
        void *w = nullptr;
        if (hipMalloc(&w, 4 * (size_t)FFT_MAX_N * 16) != hipSuccess)
            return fail(ctx, GF_ENOMEM, "cannot allocate the Fourier acceleration buffers");
        const int len[4] = {g.nx, g.ny, g.nz, g.nt};
        for (int a = 0; a < 4; a++) {
            const hipError_t e = launch_fft_roots((char *)w + (size_t)a * FFT_MAX_N * 16, len[a], ctx->stream);
            if (e != hipSuccess) {
                (void)hipFree(w);
                return fail(ctx, GF_EDEVICE, "root tables: %s", hipGetErrorString(e));
            }
        }
        ctx->d_roots = w;
    }
    return GF_OK;
}

const void *sd_roots(const gf_ctx *ctx, int axis) {
    return (const char *)ctx->d_roots + (size_t)axis * FFT_MAX_N * 16;
}

// One step of Alg. 2: Delta -> F (x, y, z and, for Landau, t) -> times
// (alpha/2) p2max / p^2 / N -> F^-1 -> g = reunit(1 + X) -> U <- g U g^dagger.
// Delta is formed in the forward x pass and g in the inverse one; the filter
// sits in the last forward pass (t for Landau, z for Coulomb), between its
// forward and inverse transform.
int sd_step_impl(gf_ctx *ctx, void *U, double alpha) {
    const Geom &g = ctx->desc[0].g;
    const int gauge = ctx->desc[0].gauge;
    const bool landau = gauge == GF_LANDAU;
    const FftSite fx = make_fft_site(g);
    const FftAxis fy = make_fft_axis(g, 1, !landau);
    const FftAxis fz = make_fft_axis(g, 2, !landau);
    FftAxis flt = landau ? make_fft_axis(g, 3, false) : fz;
    const double nfft = landau ? (double)g.V : (double)g.nx * g.ny * g.nz;
    flt.scale = 0.5 * alpha / nfft;
    flt.p2max = landau ? 16.0 : 12.0;
    hipStream_t st = ctx->stream;
    const void *wx = sd_roots(ctx, 0), *wy = sd_roots(ctx, 1), *wz = sd_roots(ctx, 2), *wt = sd_roots(ctx, 3);
    HIPTRY(ctx, launch_sd_delta_fx(ctx->prec, ctx->nelem, gauge, g, fx, wx, U, ctx->d_spec, st));
    HIPTRY(ctx, launch_fft_axis(ctx->prec, fy, wy, ctx->d_spec, -1, 0, st));
    if (landau) HIPTRY(ctx, launch_fft_axis(ctx->prec, fz, wz, ctx->d_spec, -1, 0, st));
    HIPTRY(ctx, launch_fft_axis(ctx->prec, flt, landau ? wt : wz, ctx->d_spec, -1, 1, st));
    if (landau) HIPTRY(ctx, launch_fft_axis(ctx->prec, fz, wz, ctx->d_spec, 1, 0, st));
    HIPTRY(ctx, launch_fft_axis(ctx->prec, fy, wy, ctx->d_spec, 1, 0, st));
    HIPTRY(ctx, launch_sd_fx_gfield(ctx->prec, g, fx, wx, ctx->d_spec, ctx->d_gfield, st));
    HIPTRY(ctx, launch_gauge_transform(ctx->prec, ctx->nelem, g, U, ctx->d_gfield, st));
    return GF_OK;
}

int check_alpha(gf_ctx *ctx, double alpha) {
    CHECK(ctx, std::isfinite(alpha) && alpha > 0.0, GF_EINVAL, "alpha = %g must be finite and > 0", alpha);
    return GF_OK;
}

}  // namespace

int gf_sd_step(gf_ctx *ctx, void *U, double alpha) {
    if (!ctx) return GF_EINVAL;
    int rc;
    if ((rc = need_single(ctx)) || (rc = need_su3(ctx)) || (rc = check_field(ctx, U, "U")) ||
        (rc = check_alpha(ctx, alpha)))
        return rc;
    DeviceGuard dg(ctx->device);
    if ((rc = sd_prepare(ctx))) return rc;
    return sd_step_impl(ctx, U, alpha);
}

int gf_sd_fix(gf_ctx *ctx, void *U, double alpha, double eps, int max_iter, int *iters, double *F,
              double *theta) {
    if (!ctx) return GF_EINVAL;
    int rc;
    if ((rc = need_single(ctx)) || (rc = need_su3(ctx)) || (rc = check_field(ctx, U, "U")) ||
        (rc = check_alpha(ctx, alpha)))
        return rc;
    CHECK(ctx, iters && F && theta, GF_EINVAL, "NULL argument");
    CHECK(ctx, std::isfinite(eps) && eps >= 0.0, GF_EINVAL, "eps must be finite and >= 0");
    CHECK(ctx, max_iter >= 0, GF_EINVAL, "max_iter must be >= 0");
    DeviceGuard dg(ctx->device);
    if ((rc = sd_prepare(ctx))) return rc;
    const Clock::time_point t0 = Clock::now();
    log_open(ctx);
    ctx->log_calls++;
    *iters = 0;
    if ((rc = gf_quality(ctx, U, F, theta))) return rc;
    log_check(ctx, true, 0, 0, *F, *theta, t0);
    log_flush(ctx);
    int it = 0;
    while (it < max_iter && !(*theta < eps)) {
        const int m = std::min(ctx->p.check_every, max_iter - it);
        for (int k = 0; k < m; k++)
            if ((rc = sd_step_impl(ctx, U, alpha))) return rc;
        it += m;
        *iters = it;
        if ((rc = gf_quality(ctx, U, F, theta))) return rc;
        log_check(ctx, true, 0, it, *F, *theta, t0);
        log_flush(ctx);
    }
    return *theta < eps ? GF_OK : GF_NOT_CONVERGED;
}

// ---- host-only checks ------------------------------------------------------

void gf_host_su2_step(const double b[4], double omega, double r[4]) {
    if (b && r) gf_su2_overrelax(b, omega, r);
}

void gf_host_trig(double x, double y, double out[3]) {
    if (!out) return;
    gf_sincos(x, &out[0], &out[1]);
    out[2] = gf_atan2(y, x);
}

int gf_host_link8(int prec, const double in[18], double stored[8], double out[18]) {
    if (!in || !stored || !out || (prec != GF_F64 && prec != GF_F32)) return GF_EINVAL;
    if (prec == GF_F64) {
        double re[9], im[9], sre[4], sim[4];
        for (int e = 0; e < 9; e++) { re[e] = in[2 * e]; im[e] = in[2 * e + 1]; }
        link8_compress<double>(re, im, sre, sim);
        link8_reconstruct<double>(sre, sim, re, im);
        for (int e = 0; e < 4; e++) { stored[2 * e] = sre[e]; stored[2 * e + 1] = sim[e]; }
        for (int e = 0; e < 9; e++) { out[2 * e] = re[e]; out[2 * e + 1] = im[e]; }
    } else {
        float re[9], im[9], sre[4], sim[4];
        for (int e = 0; e < 9; e++) { re[e] = (float)in[2 * e]; im[e] = (float)in[2 * e + 1]; }
        link8_compress<float>(re, im, sre, sim);
        link8_reconstruct<float>(sre, sim, re, im);
        for (int e = 0; e < 4; e++) { stored[2 * e] = sre[e]; stored[2 * e + 1] = sim[e]; }
        for (int e = 0; e < 9; e++) { out[2 * e] = re[e]; out[2 * e + 1] = im[e]; }
    }
    return GF_OK;
}


int gf_site_links(const int dims[4], int parity, long long h, long long out[8]) {
    gf_ctx tmp;
    if (!out || check_dims(&tmp, dims) != GF_OK || (parity != 0 && parity != 1)) return GF_EINVAL;
    const Geom g = make_geom(dims, 9);
    if (h < 0 || h >= g.Vh) return GF_EINVAL;
    const SiteNbr nb = site_neighbours(g, parity, (int)h);
    for (int mu = 0; mu < 4; mu++) {
        out[mu] = link_off(g, mu, parity, (int)h);
        out[4 + mu] = link_off(g, mu, 1 - parity, nb.hb[mu]);
    }
    return GF_OK;
}

}  // extern "C"
