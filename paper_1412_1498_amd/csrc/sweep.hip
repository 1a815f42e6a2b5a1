// sweep.hip -- the overrelaxation half-sweep of Alg. 1 on gfx950.
//
// One launch updates every site of one parity of every active ensemble
// member. A site x owns the eight links that touch it: U_mu(x) (parity p
// array, "forward") and U_mu(x - mu) (parity 1 - p array, "backward");
// same-parity sites share none, so the sites are independent and each link
// is read and written exactly once per half-sweep.
//
// Register form: a forward link is held as W = U_mu(x), a backward one as
// W = U_mu(x - mu)^dagger. Then the staple of eq. (5) is K = sum W over the
// functional's directions, and the update U_mu(x) <- G U_mu(x),
// U_mu(x - mu) <- U_mu(x - mu) G^dagger is the same row rotation W <- G W
// for all eight links.
//
// Schedules: LPS lanes cooperate on one site (LPS = 1, 2, 4, 8), each lane
// holding 8/LPS links. A lane forms the quaternion part of its links' (a, b)
// blocks in double, sums them in the fixed tree
//     ((s0 + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7))
// (slots 0-3 forward mu = 0..3, 4-7 backward), finishing the upper levels
// with xor-shuffles between the site's lanes; every lane then solves the
// SU(2) problem redundantly and rotates its own links. The tree is the same
// for every LPS, so all schedules produce bitwise identical links. Links are
// rotated in the link precision with explicit fma; the solve, the power
// g^omega and reunitarisation run in double.
#include "su3_device.hpp"

namespace gf {

struct Q4 { double v[4]; };

// The SU(2) solve with over-relaxation, kept out of line: inlined, its
// double-precision temporaries are scheduled across the link registers and
// raise the kernel's VGPR count by about half. Arguments and result travel
// in registers.
__device__ __attribute__((noinline)) Q4 su2_step(Q4 b, double omega) {
    Q4 r;
    gf_su2_overrelax(b.v, omega, r.v);
    return r;
}

// Fixed-tree sum of the quaternion parts (times 2) of the (a, b) blocks of
// the lane's links LO .. LO+N-1; links outside the functional add 0.
template <int LO, int N, typename R, int L>
__device__ __forceinline__ Q4 tree_quat(const Mat<R> (&w)[L], const bool (&inK)[L], int a, int b) {
    Q4 r;
    if constexpr (N == 1) {
        double t[4];
        block_quat2(w[LO], a, b, t);
#pragma unroll
        for (int i = 0; i < 4; i++) r.v[i] = inK[LO] ? t[i] : 0.0;
    } else {
        const Q4 x = tree_quat<LO, N / 2>(w, inK, a, b);
        const Q4 y = tree_quat<LO + N / 2, N / 2>(w, inK, a, b);
#pragma unroll
        for (int i = 0; i < 4; i++) r.v[i] = x.v[i] + y.v[i];
    }
    return r;
}

template <typename R, int NE, int LPS, bool NT>
__device__ __forceinline__ void or_site(const CfgDesc &d, int p, int h, int sub, int reunit) {
    constexpr int L = 8 / LPS;  // links per lane
    const Geom &g = d.g;
    gchar *U = as_global(d.U);
    const SiteNbr nb = site_neighbours(g, p, h);
    const bool landau = d.gauge == 0;

    int off[L];
    bool fwd[L];
    bool inK[L];
#pragma unroll
    for (int k = 0; k < L; k++) {
        const int slot = sub * L + k;
        const int mu = slot & 3;
        const bool f = slot < 4;
        const int hh = f ? h : pick4(nb.hb, mu);
        off[k] = mu * g.V + (f ? p : 1 - p) * g.Vh + hh;
        fwd[k] = f;
        inK[k] = landau || mu != 3;
    }

    Mat<R> w[L];
#pragma unroll
    for (int k = 0; k < L; k++) {
        load_link<R, NE, NT>(w[k], U, g.es, off[k]);
        dagger_if(w[k], !fwd[k]);
    }

#pragma unroll
    for (int sg = 0; sg < 3; sg++) {
        const int a = sg == 2 ? 1 : 0, b = sg == 0 ? 1 : 2;  // (0,1), (0,2), (1,2)
        const Q4 tq = tree_quat<0, L>(w, inK, a, b);
        double q[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            double v = tq.v[i];
#pragma unroll
            for (int m = 1; m < LPS; m <<= 1) v = v + __shfl_xor(v, m);
            q[i] = 0.5 * v;
        }
        const Q4 r = su2_step(Q4{{q[0], q[1], q[2], q[3]}}, d.omega);
        const R gq[4] = {(R)r.v[0], (R)r.v[1], (R)r.v[2], (R)r.v[3]};
#pragma unroll
        for (int k = 0; k < L; k++) rotate_rows(w[k], a, b, gq);
    }

#pragma unroll
    for (int k = 0; k < L; k++) {
        dagger_if(w[k], !fwd[k]);
        if (reunit) reunitarise(w[k]);
        store_link<R, NE, NT>(w[k], U, g.es, off[k]);
    }
}

// One workgroup per tile of blockDim/LPS sites of one member. (A persistent
// grid-stride form was measured to double the register footprint, since
// loop-invariant state stays live across the tile loop, so every tile gets
// its own workgroup; the dispatcher balances the tiles over the CUs.)
template <typename R, int NE, int LPS, bool NT>
__global__ void __launch_bounds__(256)
k_half_sweep(const CfgDesc *__restrict__ desc, const int *__restrict__ tile_cfg,
             const int *__restrict__ active, int parity, int reunit) {
    const int tile = blockIdx.x;
    const int c = tile_cfg[tile];
    if (!active[c]) return;
    const CfgDesc d = desc[c];
    const int h = (tile - d.tile0) * (int)(blockDim.x / LPS) + (int)(threadIdx.x / LPS);
    if (h >= d.g.Vh) return;
    or_site<R, NE, LPS, NT>(d, parity, h, threadIdx.x % LPS, reunit);
}

template <typename R, int NE, int LPS, bool NT>
static hipError_t launch_t(const Schedule &s, const CfgDesc *d_desc, const int *d_tile_cfg,
                           const int *d_active, int ntiles, int parity, int reunit, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_half_sweep<R, NE, LPS, NT>), dim3(ntiles), dim3(s.block), 0, st, d_desc,
                       d_tile_cfg, d_active, parity, reunit);
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
    if (prec == 0) {
        return nelem == 9 ? launch_lps<double, 9>(s, d_desc, d_tile_cfg, d_active, ntiles, parity, reunit, st)
                          : launch_lps<double, 6>(s, d_desc, d_tile_cfg, d_active, ntiles, parity, reunit, st);
    }
    return nelem == 9 ? launch_lps<float, 9>(s, d_desc, d_tile_cfg, d_active, ntiles, parity, reunit, st)
                      : launch_lps<float, 6>(s, d_desc, d_tile_cfg, d_active, ntiles, parity, reunit, st);
}

}  // namespace gf
