// quality.hip -- F (eq. 1) and theta (eqs. 2-3) of every ensemble member,
// reduced in double in a fixed order.
//
// Stage 1: one workgroup per tile of QTILE sites: the QTILE/2 half-indices
// h of the tile, both parities (each wave 32 half indices, even sites in its
// lower and odd sites in its upper 32 lanes). A
// site's backward links belong to the other parity at nearby h (x, y, z
// neighbours), so the tile's own forward reads bring most of them into
// cache; tiles are also handed out so that each XCD walks one contiguous
// range of h (its L2 then still holds the z neighbours). Each lane reads the
// eight links of its site, forms Delta(x) = A - (Tr A / 3) 1 with
// A = M - M^dagger, M = sum_nu [U_nu(x - nu) - U_nu(x)] and the site's Re Tr
// of its forward links, all in double (float links are promoted exactly).
// The workgroup sums its lanes with a fixed xor-butterfly and writes one
// partial pair.
// Stage 2: one workgroup (1024 lanes) per member sums that member's
// partials, strided per lane then by the same fixed butterfly, and
// normalises. Neither stage
// depends on the sweep schedule, so F and theta are bitwise reproducible.
#include "su3_device.hpp"
#include "sun_device.hpp"
#include "sun_internal.hpp"
#include "tile_order.hpp"

namespace gf {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = v + __shfl_xor(v, m);
    return v;
}

// Sum a pair over a workgroup of up to 1024 lanes (fixed order): result in
// lane 0.
__device__ __forceinline__ void block_sum2(double &a, double &b) {
    __shared__ double sa[16], sb[16];
    a = wave_sum(a);
    b = wave_sum(b);
    const int wid = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int nw = (blockDim.x + 63) / 64;
    if (lane == 0) { sa[wid] = a; sb[wid] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
        for (int w = 0; w < nw; w++) { ta += sa[w]; tb += sb[w]; }
        a = ta;
        b = tb;
    }
}

// Sums of Re Tr over the functional's forward links and of Tr Delta
// Delta^dagger at site (p, h), added to fsum / tsum (all in double). With TC
// (the slice-streaming kernel), tl carries the t links: on entry, when
// have_bt, the site's backward t link (taken instead of loading it); on exit,
// the site's forward t link.
template <typename R, int NE, bool TC = false>
__device__ __forceinline__ void site_quality(const Geom &g, const gchar *U, int gauge, int p, int h,
                                             double &fsum, double &tsum, bool have_bt = false,
                                             Mat<R> *tl = nullptr) {
    const int nd = gauge == 0 ? 4 : 3;
    const SiteNbr nb = site_neighbours(g, p, h);
    double mr[9], mi[9];
#pragma unroll
    for (int e = 0; e < 9; e++) { mr[e] = 0.0; mi[e] = 0.0; }
    for (int mu = 0; mu < nd; mu++) {
        Mat<R> f, b;
        load_link<R, NE, false>(f, U, link_off(g, mu, p, h));
        if constexpr (TC) {
            if (mu == 3 && have_bt) b = *tl;
            else load_link<R, NE, false>(b, U, link_off(g, mu, 1 - p, pick4(nb.hb, mu)));
            if (mu == 3) *tl = f;
        } else {
            load_link<R, NE, false>(b, U, link_off(g, mu, 1 - p, pick4(nb.hb, mu)));
        }
        fsum += (double)f.re[0] + (double)f.re[4] + (double)f.re[8];
#pragma unroll
        for (int e = 0; e < 9; e++) {
            mr[e] += (double)b.re[e] - (double)f.re[e];
            mi[e] += (double)b.im[e] - (double)f.im[e];
        }
    }
    // A = M - M^dagger: A_rc = M_rc - conj(M_cr)
    double ar[9], ai[9];
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int cc = 0; cc < 3; cc++) {
            ar[3 * r + cc] = mr[3 * r + cc] - mr[3 * cc + r];
            ai[3 * r + cc] = mi[3 * r + cc] + mi[3 * cc + r];
        }
    const double trr = (ar[0] + ar[4] + ar[8]) / 3.0;
    const double tri = (ai[0] + ai[4] + ai[8]) / 3.0;
#pragma unroll
    for (int r = 0; r < 3; r++) { ar[4 * r] -= trr; ai[4 * r] -= tri; }
#pragma unroll
    for (int e = 0; e < 9; e++) tsum += ar[e] * ar[e] + ai[e] * ai[e];
}

// Half offset within a tile and parity of lane `lane` of a tile: wave w
// takes half indices [32 w, 32 w + 32) of the tile, its lanes 0-31 the even
// and 32-63 the odd sites (so every 16 lanes read whole 128-byte lines, and
// the sites of lanes l and l ^ 32 are the even and odd site of one half
// index).
__device__ __forceinline__ int qlane_offset(int lane) { return (lane >> 6) * 32 + (lane & 31); }
__device__ __forceinline__ int qlane_parity(int lane) { return (lane >> 5) & 1; }

// Partial pair of quality tile `local` of member d (QTILE/2 half indices,
// both parities, lanes as qlane_offset / qlane_parity), summed over the
// workgroup: result in lane 0.
template <typename R, int NE>
__device__ __forceinline__ void quality_tile(const CfgDesc &d, int local, double &fsum, double &tsum) {
    constexpr int QH = QTILE / 2;
    const int p = qlane_parity(threadIdx.x);
    const int h = local * QH + qlane_offset(threadIdx.x);
    fsum = 0.0;
    tsum = 0.0;
    if (h < d.g.Vh) site_quality<R, NE>(d.g, as_global(d.U), d.gauge, p, h, fsum, tsum);
    block_sum2(fsum, tsum);
}

template <typename R, int NE>
__global__ void __launch_bounds__(QTILE)
k_quality(const CfgDesc *__restrict__ desc, const int *__restrict__ qtile_cfg,
          const int *__restrict__ active, double *__restrict__ partials, SlabOrder so) {
    const int tile = slab_tile(xcd_tile(blockIdx.x, gridDim.x), so);
    const int c = qtile_cfg[tile];
    if (active && !active[c]) return;
    const CfgDesc d = desc[c];
    double fsum, tsum;
    quality_tile<R, NE>(d, tile - d.qtile0, fsum, tsum);
    if (threadIdx.x == 0) {
        partials[2 * tile] = fsum;
        partials[2 * tile + 1] = tsum;
    }
}

// Slice-streaming form of k_quality for one lattice whose time slices split
// into whole tiles (st a multiple of QTILE/2, nchunk = st / (QTILE/2) tiles a
// slice). Workgroup b takes chunk `chunk` of the trun consecutive slices of
// run `run` and writes, slice by slice, the partial pair of tile
// t * nchunk + chunk: the same sites, lane mapping and sums as k_quality, so
// the partials are bitwise those of k_quality. The backward t link of a site
// is the forward t link of the opposite-parity site of the same half offset
// in the previous slice, which the partner lane (lane ^ 32) loaded there: it
// is passed across the lane pair instead of being loaded again (only the
// run's first slice loads it). The per-slice workgroup sum keeps the four
// waves of a workgroup on the same slice (without it they drift apart and
// re-read more of each other's x and y neighbours).
template <typename R, int NE>
__global__ void __launch_bounds__(QTILE)
k_quality_tstream(const CfgDesc *__restrict__ desc, const int *__restrict__ active, int nchunk, int trun,
                  double *__restrict__ partials) {
    constexpr int NW = QTILE / 64;
    __shared__ double sa[2][NW], sb[2][NW];
    if (active && !active[0]) return;
    const CfgDesc d = desc[0];
    const Geom &g = d.g;
    const gchar *U = as_global(d.U);
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int run = b / nchunk, chunk = b - run * nchunk;
    const int p = qlane_parity(threadIdx.x);
    const int o = chunk * (QTILE / 2) + qlane_offset(threadIdx.x);
    const int t0 = run * trun, nts = min(trun, g.nt - t0);
    const int wid = threadIdx.x / 64, lane = threadIdx.x % 64;
    Mat<R> tl;
    for (int i = 0; i < nts; i++) {
        const bool have_bt = d.gauge == 0 && i > 0;
        if (have_bt) {
#pragma unroll
            for (int e = 0; e < 9; e++) {
                tl.re[e] = __shfl_xor(tl.re[e], 32);
                tl.im[e] = __shfl_xor(tl.im[e], 32);
            }
        }
        double fsum = 0.0, tsum = 0.0;
        site_quality<R, NE, true>(g, U, d.gauge, p, (t0 + i) * g.st + o, fsum, tsum, have_bt, &tl);
        // block_sum2's order, into alternating buffers: the buffer written
        // here is next written two slices on, after another barrier
        const int buf = i & 1;
        fsum = wave_sum(fsum);
        tsum = wave_sum(tsum);
        if (lane == 0) { sa[buf][wid] = fsum; sb[buf][wid] = tsum; }
        __syncthreads();
        if (threadIdx.x == 0) {
            double ta = 0.0, tb = 0.0;
            for (int w = 0; w < NW; w++) { ta += sa[buf][w]; tb += sb[buf][w]; }
            const size_t tile = (size_t)(t0 + i) * nchunk + chunk;
            partials[2 * tile] = ta;
            partials[2 * tile + 1] = tb;
        }
    }
}

constexpr int QFINAL = 1024;

// Sum the nq partial pairs at pp over one workgroup of QFINAL lanes (strided
// per lane, then the fixed butterfly): result in lane 0.
__device__ __forceinline__ void sum_partials(const double *__restrict__ partials, int nq, double &fs,
                                             double &ts) {
    fs = 0.0;
    ts = 0.0;
    const double2 *pp = reinterpret_cast<const double2 *>(partials);
#pragma unroll 4
    for (int t = threadIdx.x; t < nq; t += QFINAL) {
        const double2 v = pp[t];
        fs += v.x;
        ts += v.y;
    }
    block_sum2(fs, ts);
}

// One workgroup per member. With update_active: members that were active
// get iters += swept, and are retired once theta < eps; retired members
// keep their previous result.
__global__ void __launch_bounds__(QFINAL)
k_quality_final(const CfgDesc *__restrict__ desc, const double *__restrict__ partials,
                double *__restrict__ result, int *__restrict__ active, int *__restrict__ iters,
                int swept, double eps, int update_active, double ncol) {
    const int c = blockIdx.x;
    if (update_active && !active[c]) return;
    const CfgDesc d = desc[c];
    double fs, ts;
    sum_partials(partials + 2 * (size_t)d.qtile0, d.nqtiles, fs, ts);
    if (threadIdx.x == 0) {
        const int nd = d.gauge == 0 ? 4 : 3;
        const double F = fs / (nd * ncol * (double)d.g.V);
        const double th = ts / (ncol * (double)d.g.V);
        result[2 * c] = F;
        result[2 * c + 1] = th;
        if (update_active) {
            iters[c] += swept;
            if (th < eps) active[c] = 0;
        }
    }
}

// Per time slice t (the Coulomb gauge's diagnostic, also defined for
// Landau): the same site sums over the nx ny nz sites of slice t, which are
// the half indices [t st, (t + 1) st) of both parities. Workgroup
// t * nchunk + chunk takes QTILE/2 of them (both parities) and writes one
// partial pair; then one workgroup per slice sums its nchunk pairs in the
// fixed order of the global reduction and normalises by the slice volume.
template <typename R, int NE>
__global__ void __launch_bounds__(QTILE)
k_quality_slices(const CfgDesc d, int nchunk, double *__restrict__ partials) {
    constexpr int QH = QTILE / 2;
    const int t = blockIdx.x / nchunk, chunk = blockIdx.x - t * nchunk;
    const int p = threadIdx.x >= QH;
    const int k = chunk * QH + (int)threadIdx.x - p * QH;
    double fsum = 0.0, tsum = 0.0;
    if (k < d.g.st) site_quality<R, NE>(d.g, as_global(d.U), d.gauge, p, t * d.g.st + k, fsum, tsum);
    block_sum2(fsum, tsum);
    if (threadIdx.x == 0) {
        partials[2 * (size_t)blockIdx.x] = fsum;
        partials[2 * (size_t)blockIdx.x + 1] = tsum;
    }
}

__global__ void __launch_bounds__(QFINAL)
k_quality_slices_final(const CfgDesc d, int nchunk, const double *__restrict__ partials,
                       double *__restrict__ out) {
    const int t = blockIdx.x;
    double fs, ts;
    sum_partials(partials + 2 * (size_t)t * nchunk, nchunk, fs, ts);
    if (threadIdx.x == 0) {
        const int nd = d.gauge == 0 ? 4 : 3;
        const double Vt = (double)d.g.nx * d.g.ny * d.g.nz;
        out[2 * t] = fs / (nd * 3.0 * Vt);
        out[2 * t + 1] = ts / (3.0 * Vt);
    }
}

template <typename R, int NE>
static hipError_t launch_qs(const CfgDesc &d, int nchunk, double *d_partials, double *d_out, hipStream_t st) {
    hipLaunchKernelGGL((k_quality_slices<R, NE>), dim3(d.g.nt * nchunk), dim3(QTILE), 0, st, d, nchunk,
                       d_partials);
    hipLaunchKernelGGL(k_quality_slices_final, dim3(d.g.nt), dim3(QFINAL), 0, st, d, nchunk, d_partials,
                       d_out);
    return hipGetLastError();
}

int quality_slice_chunks(const Geom &g) { return (g.st + QTILE / 2 - 1) / (QTILE / 2); }

hipError_t launch_quality_slices(int prec, int nelem, const CfgDesc &d, double *d_partials, double *d_out,
                                 hipStream_t st) {
    const int nchunk = quality_slice_chunks(d.g);
#define GF_QS(R)                                                                                  \
    (nelem == 9   ? launch_qs<R, 9>(d, nchunk, d_partials, d_out, st)                              \
     : nelem == 6 ? launch_qs<R, 6>(d, nchunk, d_partials, d_out, st)                              \
                  : launch_qs<R, 4>(d, nchunk, d_partials, d_out, st))
    const hipError_t e = prec == 0 ? GF_QS(double) : GF_QS(float);
#undef GF_QS
    return e;
}

// One member given by value (no member table, no tile map): the tiles,
// their order and the final reduction of k_quality / k_quality_final for a
// single lattice, so the results are bitwise those of the context path.
template <typename R, int NE>
__global__ void __launch_bounds__(QTILE)
k_quality_one(const CfgDesc d, double *__restrict__ partials, SlabOrder so) {
    const int tile = slab_tile(xcd_tile(blockIdx.x, gridDim.x), so);
    double fsum, tsum;
    quality_tile<R, NE>(d, tile, fsum, tsum);
    if (threadIdx.x == 0) {
        partials[2 * tile] = fsum;
        partials[2 * tile + 1] = tsum;
    }
}

__global__ void __launch_bounds__(QFINAL)
k_quality_one_final(const CfgDesc d, const double *__restrict__ partials, double *__restrict__ out) {
    double fs, ts;
    sum_partials(partials, d.nqtiles, fs, ts);
    if (threadIdx.x == 0) {
        const int nd = d.gauge == 0 ? 4 : 3;
        const double ncol = 3.0;
        out[0] = fs / (nd * ncol * (double)d.g.V);
        out[1] = ts / (ncol * (double)d.g.V);
    }
}

template <typename R, int NE>
static hipError_t launch_q1(const CfgDesc &d, double *d_partials, double *d_out, hipStream_t st) {
    const SlabOrder so = make_slab_order(d.g.st, QTILE / 2, d.nqtiles);
    hipLaunchKernelGGL((k_quality_one<R, NE>), dim3(d.nqtiles), dim3(QTILE), 0, st, d, d_partials, so);
    hipLaunchKernelGGL(k_quality_one_final, dim3(1), dim3(QFINAL), 0, st, d, d_partials, d_out);
    return hipGetLastError();
}

hipError_t launch_quality_one(int prec, int nelem, const CfgDesc &d, double *d_partials, double *d_out,
                              hipStream_t st) {
#define GF_Q1(R)                                                                                  \
    (nelem == 9   ? launch_q1<R, 9>(d, d_partials, d_out, st)                                      \
     : nelem == 6 ? launch_q1<R, 6>(d, d_partials, d_out, st)                                      \
                  : launch_q1<R, 4>(d, d_partials, d_out, st))
    const hipError_t e = prec == 0 ? GF_Q1(double) : GF_Q1(float);
#undef GF_Q1
    return e;
}

template <typename R, int NE>
static hipError_t launch_q(const CfgDesc *d_desc, const int *d_qtile_cfg, const int *d_active,
                           int nqtiles, double *d_partials, const SlabOrder &so, hipStream_t st) {
    if (nqtiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_quality<R, NE>), dim3(nqtiles), dim3(QTILE), 0, st, d_desc, d_qtile_cfg,
                       d_active, d_partials, so);
    return hipGetLastError();
}

hipError_t launch_quality(int prec, int nelem, const CfgDesc *d_desc, const int *d_qtile_cfg,
                          const int *d_active, int nqtiles, double *d_partials, const SlabOrder &so,
                          hipStream_t st) {
#define GF_Q3(R)                                                                                  \
    (nelem == 9   ? launch_q<R, 9>(d_desc, d_qtile_cfg, d_active, nqtiles, d_partials, so, st)       \
     : nelem == 6 ? launch_q<R, 6>(d_desc, d_qtile_cfg, d_active, nqtiles, d_partials, so, st)       \
                  : launch_q<R, 4>(d_desc, d_qtile_cfg, d_active, nqtiles, d_partials, so, st))
    const hipError_t e = prec == 0 ? GF_Q3(double) : GF_Q3(float);
#undef GF_Q3
    return e;
}

// Slices per run of k_quality_tstream (runs of 3 to 12 slices measured
// alike at 48^4; one round of resident workgroups, 24 to 48, was slower).
#ifndef GF_QSTREAM_T
#define GF_QSTREAM_T 6
#endif

// Whether k_quality_tstream can take lattice g (single lattices only).
bool quality_tstream_ok(const Geom &g) { return g.st % (QTILE / 2) == 0 && g.nt >= 2; }

template <typename R, int NE>
static hipError_t launch_qts(const Geom &g, const CfgDesc *d_desc, const int *d_active, double *d_partials,
                             hipStream_t st) {
    static_assert(GF_QSTREAM_T >= 1, "slices per run");
    const int nchunk = g.st / (QTILE / 2);
    const int runs0 = (g.nt + GF_QSTREAM_T - 1) / GF_QSTREAM_T;
    const int trun = (g.nt + runs0 - 1) / runs0;  // <= GF_QSTREAM_T slices, runs as even as they go
    const int runs = (g.nt + trun - 1) / trun;    // each holds >= 1 slice
    hipLaunchKernelGGL((k_quality_tstream<R, NE>), dim3(runs * nchunk), dim3(QTILE), 0, st, d_desc, d_active,
                       nchunk, trun, d_partials);
    return hipGetLastError();
}

hipError_t launch_quality_tstream(int prec, int nelem, const Geom &g, const CfgDesc *d_desc, const int *d_active,
                                  double *d_partials, hipStream_t st) {
    if (!quality_tstream_ok(g)) return hipErrorInvalidValue;
#define GF_QTS(R)                                                                                 \
    (nelem == 9   ? launch_qts<R, 9>(g, d_desc, d_active, d_partials, st)                          \
     : nelem == 6 ? launch_qts<R, 6>(g, d_desc, d_active, d_partials, st)                          \
                  : launch_qts<R, 4>(g, d_desc, d_active, d_partials, st))
    const hipError_t e = prec == 0 ? GF_QTS(double) : GF_QTS(float);
#undef GF_QTS
    return e;
}

hipError_t launch_quality_final(const CfgDesc *d_desc, int n, const double *d_partials,
                                double *d_result, int *d_active, int *d_iters, int swept,
                                double eps, int update_active, hipStream_t st) {
    return launch_quality_final_nc(3, d_desc, n, d_partials, d_result, d_active, d_iters, swept, eps,
                                   update_active, st);
}

hipError_t launch_quality_final_nc(int nc, const CfgDesc *d_desc, int n, const double *d_partials,
                                   double *d_result, int *d_active, int *d_iters, int swept, double eps,
                                   int update_active, hipStream_t st) {
    hipLaunchKernelGGL(k_quality_final, dim3(n), dim3(QFINAL), 0, st, d_desc, d_partials, d_result,
                       d_active, d_iters, swept, eps, update_active, (double)nc);
    return hipGetLastError();
}

// SU(N): the same tiles and reductions, N x N links, trace / N in Delta.
template <typename R, int N>
__global__ void __launch_bounds__(QTILE)
k_sun_quality(const CfgDesc *__restrict__ desc, const int *__restrict__ qtile_cfg,
              const int *__restrict__ active, double *__restrict__ partials, SlabOrder so) {
    const int tile = slab_tile(xcd_tile(blockIdx.x, gridDim.x), so);
    const int c = qtile_cfg[tile];
    if (active && !active[c]) return;
    const CfgDesc d = desc[c];
    const Geom &g = d.g;
    constexpr int QH = QTILE / 2;
    constexpr int E = N * N;
    const int p = threadIdx.x >= QH;
    const int h = (tile - d.qtile0) * QH + (int)threadIdx.x - p * QH;
    const int nd = d.gauge == 0 ? 4 : 3;
    double fsum = 0.0, tsum = 0.0;
    if (h < g.Vh) {
        const SiteNbr nb = site_neighbours(g, p, h);
        const gchar *U = as_global(d.U);
        double mr[E], mi[E];
#pragma unroll
        for (int e = 0; e < E; e++) { mr[e] = 0.0; mi[e] = 0.0; }
        for (int mu = 0; mu < nd; mu++) {
            MatN<R, N> f, b;
            load_link_n<R, N, false>(f, U, link_off(g, mu, p, h));
            load_link_n<R, N, false>(b, U, link_off(g, mu, 1 - p, pick4(nb.hb, mu)));
#pragma unroll
            for (int r = 0; r < N; r++) fsum += (double)f.re[(N + 1) * r];
#pragma unroll
            for (int e = 0; e < E; e++) {
                mr[e] += (double)b.re[e] - (double)f.re[e];
                mi[e] += (double)b.im[e] - (double)f.im[e];
            }
        }
        double ar[E], ai[E];
#pragma unroll
        for (int r = 0; r < N; r++)
#pragma unroll
            for (int cc = 0; cc < N; cc++) {
                ar[N * r + cc] = mr[N * r + cc] - mr[N * cc + r];
                ai[N * r + cc] = mi[N * r + cc] + mi[N * cc + r];
            }
        double trr = 0.0, tri = 0.0;
#pragma unroll
        for (int r = 0; r < N; r++) { trr += ar[(N + 1) * r]; tri += ai[(N + 1) * r]; }
        trr /= (double)N;
        tri /= (double)N;
#pragma unroll
        for (int r = 0; r < N; r++) { ar[(N + 1) * r] -= trr; ai[(N + 1) * r] -= tri; }
#pragma unroll
        for (int e = 0; e < E; e++) tsum += ar[e] * ar[e] + ai[e] * ai[e];
    }
    block_sum2(fsum, tsum);
    if (threadIdx.x == 0) {
        partials[2 * tile] = fsum;
        partials[2 * tile + 1] = tsum;
    }
}

hipError_t launch_sun_quality(int prec, int nc, const CfgDesc *d_desc, const int *d_qtile_cfg,
                              const int *d_active, int nqtiles, double *d_partials, const SlabOrder &so,
                              hipStream_t st) {
    if (nqtiles <= 0) return hipSuccess;
#define GF_Q(R, N)                                                                                 \
    hipLaunchKernelGGL((k_sun_quality<R, N>), dim3(nqtiles), dim3(QTILE), 0, st, d_desc, d_qtile_cfg, \
                       d_active, d_partials, so)
    if (nc == 2) { if (prec == 0) GF_Q(double, 2); else GF_Q(float, 2); }
    else if (nc == 4) { if (prec == 0) GF_Q(double, 4); else GF_Q(float, 4); }
    else return hipErrorInvalidValue;
#undef GF_Q
    return hipGetLastError();
}

}  // namespace gf
