// sweep.hip -- the overrelaxation half-sweep of Alg. 1 on gfx950.
//
// One launch updates every site of one parity of every active ensemble
// member. A site x owns the eight links that touch it: U_mu(x) (parity p
// array, "forward") and U_mu(x - mu) (parity 1 - p array, "backward");
// same-parity sites share none, so the sites are independent and each link
// is read and written exactly once per half-sweep.
//
// Per site: K(x) = sum_mu [U_mu(x) + U_mu(x - mu)^dagger] (eq. 5, the field
// already carrying every transformation so far) is built once, in double.
// Applying a subgroup element G to the site's links (U_mu(x) <- G U_mu(x),
// U_mu(x - mu) <- U_mu(x - mu) G^dagger) maps K to G K exactly, so the three
// subgroup steps of Alg. 1 -- solve eq. (6) on the (a, b) block, over-relax,
// rotate -- are carried out on K alone, in double, and the product
// G3 G2 G1 is applied to each of the eight links once at the end. The result
// is that of rotating the links after every subgroup, with two fewer
// roundings of each link.
//
// Schedules: LPS lanes cooperate on a site (LPS = 1, 2, 4, 8), each holding
// 8/LPS links. Link slots are ordered (fwd 0, bwd 0, fwd 1, bwd 1, ...,
// fwd 3, bwd 3); a lane owns consecutive slots and K is summed over slots in
// the fixed tree ((s0 + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7)), the
// upper levels by xor-shuffles between the site's lanes. Every lane then
// runs the (cheap, double) subgroup steps redundantly. The tree does not
// depend on LPS, so all schedules give bitwise identical links.
#include "su3_device.hpp"

namespace gf {

// 3x3 complex matrix in double.
struct DM {
    double re[9], im[9];
};

// The SU(2) solve with over-relaxation, kept out of line: inlined, its
// double-precision temporaries are scheduled across the link registers and
// raise the kernel's VGPR count by about half. Arguments and result travel
// in registers.
struct Q4 { double v[4]; };

__device__ __attribute__((noinline)) Q4 su2_step(Q4 b, double omega) {
    Q4 r;
    gf_su2_overrelax(b.v, omega, r.v);
    return r;
}

// Rows a, b of m <- g (rows a, b of m); g = [[g0 + i g3, g2 + i g1],
// [-g2 + i g1, g0 - i g3]] in double.
__device__ __forceinline__ void rot_rows_d(DM &m, int a, int b, const Q4 &g) {
    const double ar = g.v[0], ai = g.v[3], br = g.v[2], bi = g.v[1];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const double xr = m.re[3 * a + c], xi = m.im[3 * a + c];
        const double yr = m.re[3 * b + c], yi = m.im[3 * b + c];
        m.re[3 * a + c] = ar * xr - ai * xi + (br * yr - bi * yi);
        m.im[3 * a + c] = ar * xi + ai * xr + (br * yi + bi * yr);
        m.re[3 * b + c] = -br * xr - bi * xi + (ar * yr + ai * yi);
        m.im[3 * b + c] = -br * xi + bi * xr + (ar * yi - ai * yr);
    }
}

// o = g u (forward link) or o = u g^dagger (backward link), g in the link
// precision. The result goes to a separate matrix that is stored directly:
// copying it back into u would make the compiler keep a private array.
template <typename R>
__device__ __forceinline__ void apply_left(const Mat<R> &u, const Mat<R> &g, Mat<R> &o) {
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            R sr = g.re[3 * r] * u.re[c];
            R si = g.re[3 * r] * u.im[c];
            sr = fma(-g.im[3 * r], u.im[c], sr);
            si = fma(g.im[3 * r], u.re[c], si);
#pragma unroll
            for (int k = 1; k < 3; k++) {
                sr = fma(g.re[3 * r + k], u.re[3 * k + c], sr);
                sr = fma(-g.im[3 * r + k], u.im[3 * k + c], sr);
                si = fma(g.re[3 * r + k], u.im[3 * k + c], si);
                si = fma(g.im[3 * r + k], u.re[3 * k + c], si);
            }
            o.re[3 * r + c] = sr;
            o.im[3 * r + c] = si;
        }
}

// (u g^dagger)_rc = sum_k u_rk conj(g_ck)
template <typename R>
__device__ __forceinline__ void apply_right_dag(const Mat<R> &u, const Mat<R> &g, Mat<R> &o) {
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            R sr = u.re[3 * r] * g.re[3 * c];
            R si = u.im[3 * r] * g.re[3 * c];
            sr = fma(u.im[3 * r], g.im[3 * c], sr);
            si = fma(-u.re[3 * r], g.im[3 * c], si);
#pragma unroll
            for (int k = 1; k < 3; k++) {
                sr = fma(u.re[3 * r + k], g.re[3 * c + k], sr);
                sr = fma(u.im[3 * r + k], g.im[3 * c + k], sr);
                si = fma(u.im[3 * r + k], g.re[3 * c + k], si);
                si = fma(-u.re[3 * r + k], g.im[3 * c + k], si);
            }
            o.re[3 * r + c] = sr;
            o.im[3 * r + c] = si;
        }
}

template <typename R, int NE, int LPS, bool NT, bool RU>
__device__ __forceinline__ void or_site(const CfgDesc &d, int p, int h, int sub) {
    constexpr int L = 8 / LPS;  // links per lane
    const Geom &g = d.g;
    gchar *U = as_global(d.U);
    const SiteNbr nb = site_neighbours(g, p, h);
    const bool landau = d.gauge == 0;

    long long off[L];
    bool bwd[L], in[L];
#pragma unroll
    for (int k = 0; k < L; k++) {
        const int slot = sub * L + k;
        const int mu = slot >> 1;
        const bool b = (slot & 1) != 0;  // compile-time unless LPS == 8
        off[k] = b ? link_off(g, mu, 1 - p, pick4(nb.hb, mu)) : link_off(g, mu, p, h);
        bwd[k] = b;
        in[k] = landau || mu != 3;
    }

    Mat<R> w[L];
#pragma unroll
    for (int k = 0; k < L; k++) load_link<R, NE, NT>(w[k], U, off[k]);

    // K = sum over slots of U (forward) or U^dagger (backward), promoted to
    // double; per element, the lane's slots are summed in place in the fixed
    // tree, then the site's lanes combine by xor-shuffles.
    DM K;
#pragma unroll
    for (int r = 0; r < 3; r++) {
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const int e = 3 * r + c, et = 3 * c + r;
            double tr[L], ti[L];
#pragma unroll
            for (int k = 0; k < L; k++) {
                const double xr = bwd[k] ? (double)w[k].re[et] : (double)w[k].re[e];
                const double xi = bwd[k] ? -(double)w[k].im[et] : (double)w[k].im[e];
                tr[k] = in[k] ? xr : 0.0;
                ti[k] = in[k] ? xi : 0.0;
            }
#pragma unroll
            for (int step = 1; step < L; step *= 2)
#pragma unroll
                for (int k = 0; k < L; k += 2 * step) {
                    tr[k] = tr[k] + tr[k + step];
                    ti[k] = ti[k] + ti[k + step];
                }
#pragma unroll
            for (int m = 1; m < LPS; m <<= 1) {
                tr[0] = tr[0] + __shfl_xor(tr[0], m);
                ti[0] = ti[0] + __shfl_xor(ti[0], m);
            }
            K.re[e] = tr[0];
            K.im[e] = ti[0];
        }
    }

    // three subgroup steps on K: (0,1), (0,2), (1,2)
    Q4 gs[3];
#pragma unroll
    for (int sg = 0; sg < 3; sg++) {
        const int a = sg == 2 ? 1 : 0, b = sg == 0 ? 1 : 2;
        const int aa = 4 * a, bb = 4 * b, ab = 3 * a + b, ba = 3 * b + a;
        Q4 q;
        q.v[0] = 0.5 * (K.re[aa] + K.re[bb]);
        q.v[1] = 0.5 * (K.im[ab] + K.im[ba]);
        q.v[2] = 0.5 * (K.re[ab] - K.re[ba]);
        q.v[3] = 0.5 * (K.im[aa] - K.im[bb]);
        gs[sg] = su2_step(q, d.omega);
        if (sg < 2) rot_rows_d(K, a, b, gs[sg]);
    }

    // G = G3 G2 G1 (double), rounded to the link precision
    DM T;
#pragma unroll
    for (int e = 0; e < 9; e++) { T.re[e] = (e % 4 == 0) ? 1.0 : 0.0; T.im[e] = 0.0; }
    rot_rows_d(T, 0, 1, gs[0]);
    rot_rows_d(T, 0, 2, gs[1]);
    rot_rows_d(T, 1, 2, gs[2]);
    Mat<R> G;
#pragma unroll
    for (int e = 0; e < 9; e++) { G.re[e] = (R)T.re[e]; G.im[e] = (R)T.im[e]; }

#pragma unroll
    for (int k = 0; k < L; k++) {
        Mat<R> o;
        if (LPS == 8) {
            // the lane's one link is forward or backward at run time
            Mat<R> f, r;
            apply_left(w[k], G, f);
            apply_right_dag(w[k], G, r);
#pragma unroll
            for (int e = 0; e < 9; e++) {
                o.re[e] = bwd[k] ? r.re[e] : f.re[e];
                o.im[e] = bwd[k] ? r.im[e] : f.im[e];
            }
        } else if (bwd[k]) {
            apply_right_dag(w[k], G, o);
        } else {
            apply_left(w[k], G, o);
        }
        if constexpr (RU) reunitarise(o);
        store_link<R, NE, NT>(o, U, off[k]);
    }
}

// Waves per SIMD the compiler is asked to leave room for in the float
// 8-real sweep (decoding and encoding make its compute phase the longest of
// the storage forms); every other form fits one wave's registers.
#ifndef GF_SWEEP8_WAVES
#define GF_SWEEP8_WAVES 2
#endif

// One workgroup per tile of blockDim/LPS sites of one member. (A persistent
// grid-stride form was measured to double the register footprint, since
// loop-invariant state stays live across the tile loop, so every tile gets
// its own workgroup; the dispatcher balances the tiles over the CUs.)
template <typename R, int NE, int LPS, bool NT, bool RU>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((NE == 4 && sizeof(R) == 4) ? GF_SWEEP8_WAVES : 1)))
k_half_sweep(const CfgDesc *__restrict__ desc, const int *__restrict__ tile_cfg,
             const int *__restrict__ active, int parity, int order) {
    // the tile order is a schedule choice: every tile is independent
    const int tile = order ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int c = tile_cfg[tile];
    if (!active[c]) return;
    const CfgDesc d = desc[c];
    const int h = (tile - d.tile0) * (int)(blockDim.x / LPS) + (int)(threadIdx.x / LPS);
    if (h >= d.g.Vh) return;
    or_site<R, NE, LPS, NT, RU>(d, parity, h, threadIdx.x % LPS);
}

template <typename R, int NE, int LPS, bool NT>
static hipError_t launch_t(const Schedule &s, const CfgDesc *d_desc, const int *d_tile_cfg,
                           const int *d_active, int ntiles, int parity, int reunit, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (reunit)
        hipLaunchKernelGGL((k_half_sweep<R, NE, LPS, NT, true>), dim3(ntiles), dim3(s.block), 0, st,
                           d_desc, d_tile_cfg, d_active, parity, s.order);
    else
        hipLaunchKernelGGL((k_half_sweep<R, NE, LPS, NT, false>), dim3(ntiles), dim3(s.block), 0, st,
                           d_desc, d_tile_cfg, d_active, parity, s.order);
    return hipGetLastError();
}

template <typename R, int NE>
static hipError_t launch_lps(const Schedule &s, const CfgDesc *d_desc, const int *d_tile_cfg,
                             const int *d_active, int ntiles, int parity, int reunit, hipStream_t st) {
#define GF_CASE(L)                                                                                  \
    case L:                                                                                         \
        return s.nt ? launch_t<R, NE, L, true>(s, d_desc, d_tile_cfg, d_active, ntiles, parity,    \
                                               reunit, st)                                          \
                    : launch_t<R, NE, L, false>(s, d_desc, d_tile_cfg, d_active, ntiles, parity,   \
                                                reunit, st);
    switch (s.lps) {
        GF_CASE(1)
        GF_CASE(2)
        GF_CASE(4)
        GF_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef GF_CASE
}

hipError_t launch_half_sweep(int prec, int nelem, const Schedule &s, const CfgDesc *d_desc,
                             const int *d_tile_cfg, const int *d_active, int ntiles, int parity,
                             int reunit, hipStream_t st) {
#define GF_S3(R)                                                                                  \
    (nelem == 9   ? launch_lps<R, 9>(s, d_desc, d_tile_cfg, d_active, ntiles, parity, reunit, st)     \
     : nelem == 6 ? launch_lps<R, 6>(s, d_desc, d_tile_cfg, d_active, ntiles, parity, reunit, st)     \
                  : launch_lps<R, 4>(s, d_desc, d_tile_cfg, d_active, ntiles, parity, reunit, st))
    const hipError_t e = prec == 0 ? GF_S3(double) : GF_S3(float);
#undef GF_S3
    return e;
}

}  // namespace gf
