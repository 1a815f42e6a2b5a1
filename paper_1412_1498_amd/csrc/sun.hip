// sun.hip -- Alg. 1 for SU(N) links, N = 2 and 4 (the paper's method for a
// general number of colours: the local maximisation visits all N(N-1)/2
// SU(2) subgroups (a, b), a < b, in lexicographic order).
//
// The half-sweep has the structure of the SU(3) kernel: a site owns its
// eight links; K(x) = sum_mu [U_mu(x) + U_mu(x - mu)^dagger] (eq. 5) is
// built once in double over the link slots (fwd 0, bwd 0, ..., fwd 3,
// bwd 3) in the fixed tree ((s0 + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7)),
// the upper levels by xor-shuffles between the LPS lanes of a site; every
// subgroup step (eq. 6 on the (a, b) block, exact principal power for the
// over-relaxation) acts on K (K <- G K) and on the running product T, and
// the eight links are rotated once by T (rounded to the link precision).
// All schedules give bitwise identical links. N = 4 needs LPS >= 2 (eight
// 4x4 links do not fit one lane's registers).
//
// Also here: pack/unpack between the canonical [site][mu][N][N] layout and
// the blocked layout, and standalone reunitarisation.
#include "sun_device.hpp"
#include "sun_internal.hpp"

namespace gf {

namespace {

struct Q4n { double v[4]; };

// Out of line, as in the SU(3) kernel, so the solve's double temporaries do
// not compete with the link registers.
__device__ __attribute__((noinline)) Q4n sun_su2_step(Q4n b, double omega) {
    Q4n r;
    gf_su2_overrelax(b.v, omega, r.v);
    return r;
}

// Rows a, b of m <- g (rows a, b of m), g = [[g0 + i g3, g2 + i g1],
// [-g2 + i g1, g0 - i g3]].
template <int N>
__device__ __forceinline__ void rot_rows_n(DMN<N> &m, int a, int b, const Q4n &g) {
    const double ar = g.v[0], ai = g.v[3], br = g.v[2], bi = g.v[1];
#pragma unroll
    for (int c = 0; c < N; c++) {
        const double xr = m.re[N * a + c], xi = m.im[N * a + c];
        const double yr = m.re[N * b + c], yi = m.im[N * b + c];
        m.re[N * a + c] = ar * xr - ai * xi + (br * yr - bi * yi);
        m.im[N * a + c] = ar * xi + ai * xr + (br * yi + bi * yr);
        m.re[N * b + c] = -br * xr - bi * xi + (ar * yr + ai * yi);
        m.im[N * b + c] = -br * xi + bi * xr + (ar * yi - ai * yr);
    }
}

// o = g u
template <typename R, int N>
__device__ __forceinline__ void apply_left_n(const MatN<R, N> &u, const MatN<R, N> &g, MatN<R, N> &o) {
#pragma unroll
    for (int r = 0; r < N; r++)
#pragma unroll
        for (int c = 0; c < N; c++) {
            R sr = g.re[N * r] * u.re[c];
            R si = g.re[N * r] * u.im[c];
            sr = fma(-g.im[N * r], u.im[c], sr);
            si = fma(g.im[N * r], u.re[c], si);
#pragma unroll
            for (int k = 1; k < N; k++) {
                sr = fma(g.re[N * r + k], u.re[N * k + c], sr);
                sr = fma(-g.im[N * r + k], u.im[N * k + c], sr);
                si = fma(g.re[N * r + k], u.im[N * k + c], si);
                si = fma(g.im[N * r + k], u.re[N * k + c], si);
            }
            o.re[N * r + c] = sr;
            o.im[N * r + c] = si;
        }
}

// o = u g^dagger: o_rc = sum_k u_rk conj(g_ck)
template <typename R, int N>
__device__ __forceinline__ void apply_right_dag_n(const MatN<R, N> &u, const MatN<R, N> &g, MatN<R, N> &o) {
#pragma unroll
    for (int r = 0; r < N; r++)
#pragma unroll
        for (int c = 0; c < N; c++) {
            R sr = u.re[N * r] * g.re[N * c];
            R si = u.im[N * r] * g.re[N * c];
            sr = fma(u.im[N * r], g.im[N * c], sr);
            si = fma(-u.re[N * r], g.im[N * c], si);
#pragma unroll
            for (int k = 1; k < N; k++) {
                sr = fma(u.re[N * r + k], g.re[N * c + k], sr);
                sr = fma(u.im[N * r + k], g.im[N * c + k], sr);
                si = fma(u.im[N * r + k], g.re[N * c + k], si);
                si = fma(-u.re[N * r + k], g.im[N * c + k], si);
            }
            o.re[N * r + c] = sr;
            o.im[N * r + c] = si;
        }
}

template <typename R, int N, int LPS, bool RU>
__device__ __forceinline__ void or_site_n(const CfgDesc &d, int p, int h, int sub) {
    constexpr int L = 8 / LPS;  // links per lane
    constexpr int E = N * N;
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
        const bool b = (slot & 1) != 0;
        off[k] = b ? link_off(g, mu, 1 - p, pick4(nb.hb, mu)) : link_off(g, mu, p, h);
        bwd[k] = b;
        in[k] = landau || mu != 3;
    }
    MatN<R, N> w[L];
#pragma unroll
    for (int k = 0; k < L; k++) load_link_n<R, N, true>(w[k], U, off[k]);

    DMN<N> K;
#pragma unroll
    for (int r = 0; r < N; r++) {
#pragma unroll
        for (int c = 0; c < N; c++) {
            const int e = N * r + c, et = N * c + r;
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

    DMN<N> T;
#pragma unroll
    for (int e = 0; e < E; e++) { T.re[e] = (e % (N + 1) == 0) ? 1.0 : 0.0; T.im[e] = 0.0; }
#pragma unroll
    for (int a = 0; a < N; a++)
#pragma unroll
        for (int b = a + 1; b < N; b++) {
            const int aa = N * a + a, bb = N * b + b, ab = N * a + b, ba = N * b + a;
            Q4n q;
            q.v[0] = 0.5 * (K.re[aa] + K.re[bb]);
            q.v[1] = 0.5 * (K.im[ab] + K.im[ba]);
            q.v[2] = 0.5 * (K.re[ab] - K.re[ba]);
            q.v[3] = 0.5 * (K.im[aa] - K.im[bb]);
            const Q4n gq = sun_su2_step(q, d.omega);
            rot_rows_n<N>(K, a, b, gq);
            rot_rows_n<N>(T, a, b, gq);
        }
    MatN<R, N> G;
#pragma unroll
    for (int e = 0; e < E; e++) { G.re[e] = (R)T.re[e]; G.im[e] = (R)T.im[e]; }

#pragma unroll
    for (int k = 0; k < L; k++) {
        MatN<R, N> o;
        if (LPS == 8) {
            MatN<R, N> f, r;
            apply_left_n(w[k], G, f);
            apply_right_dag_n(w[k], G, r);
#pragma unroll
            for (int e = 0; e < E; e++) {
                o.re[e] = bwd[k] ? r.re[e] : f.re[e];
                o.im[e] = bwd[k] ? r.im[e] : f.im[e];
            }
        } else if (bwd[k]) {
            apply_right_dag_n(w[k], G, o);
        } else {
            apply_left_n(w[k], G, o);
        }
        if constexpr (RU) reunitarise_n(o);
        store_link_n<R, N, true>(o, U, off[k]);
    }
}

template <typename R, int N, int LPS, bool RU>
__global__ void __launch_bounds__(256)
k_sun_half_sweep(const CfgDesc *__restrict__ desc, const int *__restrict__ tile_cfg,
                 const int *__restrict__ active, int parity, int order) {
    const int tile = order ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int c = tile_cfg[tile];
    if (!active[c]) return;
    const CfgDesc d = desc[c];
    const int h = (tile - d.tile0) * (int)(blockDim.x / LPS) + (int)(threadIdx.x / LPS);
    if (h >= d.g.Vh) return;
    or_site_n<R, N, LPS, RU>(d, parity, h, threadIdx.x % LPS);
}

template <typename R, int N, int LPS>
hipError_t launch_sun_t(const Schedule &s, const CfgDesc *d_desc, const int *d_tile_cfg,
                        const int *d_active, int ntiles, int parity, int reunit, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (reunit)
        hipLaunchKernelGGL((k_sun_half_sweep<R, N, LPS, true>), dim3(ntiles), dim3(s.block), 0, st,
                           d_desc, d_tile_cfg, d_active, parity, s.order);
    else
        hipLaunchKernelGGL((k_sun_half_sweep<R, N, LPS, false>), dim3(ntiles), dim3(s.block), 0, st,
                           d_desc, d_tile_cfg, d_active, parity, s.order);
    return hipGetLastError();
}

template <typename R, int N>
hipError_t launch_sun_lps(const Schedule &s, const CfgDesc *d_desc, const int *d_tile_cfg,
                          const int *d_active, int ntiles, int parity, int reunit, hipStream_t st) {
    switch (s.lps) {
        case 1:
            if constexpr (N == 2)
                return launch_sun_t<R, N, 1>(s, d_desc, d_tile_cfg, d_active, ntiles, parity, reunit, st);
            else
                return hipErrorInvalidValue;
        case 2: return launch_sun_t<R, N, 2>(s, d_desc, d_tile_cfg, d_active, ntiles, parity, reunit, st);
        case 4: return launch_sun_t<R, N, 4>(s, d_desc, d_tile_cfg, d_active, ntiles, parity, reunit, st);
        case 8: return launch_sun_t<R, N, 8>(s, d_desc, d_tile_cfg, d_active, ntiles, parity, reunit, st);
        default: return hipErrorInvalidValue;
    }
}

// Canonical AoS [site][mu][N][N] <-> blocked layout; one thread per link.
template <typename R, int N>
__global__ void __launch_bounds__(256) k_sun_pack(Geom g, const typename V2<R>::type *__restrict__ src,
                           typename V2<R>::type *__restrict__ dst, int to_aos) {
    const long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= 4LL * g.V) return;
    const int s = (int)(l >> 2), mu = (int)(l & 3);
    const int x = s % g.nx, y = (s / g.nx) % g.ny, z = (s / (g.nx * g.ny)) % g.nz, t = s / (g.nx * g.ny * g.nz);
    int p, h;
    site_to_ph(g, x, y, z, t, p, h);
    const long long o = link_off(g, mu, p, h);
#pragma unroll
    for (int e = 0; e < N * N; e++) {
        if (to_aos) dst[l * (N * N) + e] = src[o + (long long)e * BLK];
        else dst[o + (long long)e * BLK] = src[l * (N * N) + e];
    }
}

// Standalone reunitarisation of every link; one thread per link.
template <typename R, int N>
__global__ void __launch_bounds__(256) k_sun_reunit(Geom g, void *Uv) {
    const long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= 4LL * g.V) return;
    const int n = (int)(l >> 2), mu = (int)(l & 3);
    const int p = n >= g.Vh, h = n - p * g.Vh;
    gchar *U = as_global(Uv);
    const long long o = link_off(g, mu, p, h);
    MatN<R, N> m;
    load_link_n<R, N, false>(m, U, o);
    reunitarise_n(m);
    store_link_n<R, N, false>(m, U, o);
}

}  // namespace

hipError_t launch_sun_half_sweep(int prec, int nc, const Schedule &s, const CfgDesc *d_desc,
                                 const int *d_tile_cfg, const int *d_active, int ntiles, int parity,
                                 int reunit, hipStream_t st) {
    if (nc == 2)
        return prec == 0 ? launch_sun_lps<double, 2>(s, d_desc, d_tile_cfg, d_active, ntiles, parity, reunit, st)
                         : launch_sun_lps<float, 2>(s, d_desc, d_tile_cfg, d_active, ntiles, parity, reunit, st);
    if (nc == 4)
        return prec == 0 ? launch_sun_lps<double, 4>(s, d_desc, d_tile_cfg, d_active, ntiles, parity, reunit, st)
                         : launch_sun_lps<float, 4>(s, d_desc, d_tile_cfg, d_active, ntiles, parity, reunit, st);
    return hipErrorInvalidValue;
}

hipError_t launch_sun_pack(int prec, int nc, const Geom &g, const void *aos, void *U, int to_aos,
                           hipStream_t st) {
    const long long n = 4LL * g.V;
    const int B = 256;
    const dim3 grid((unsigned)((n + B - 1) / B));
#define GF_P(R, N)                                                                                 \
    hipLaunchKernelGGL((k_sun_pack<R, N>), grid, dim3(B), 0, st, g,                                \
                       (const V2<R>::type *)(to_aos ? U : aos), (V2<R>::type *)(to_aos ? aos : U), \
                       to_aos)
    if (nc == 2) { if (prec == 0) GF_P(double, 2); else GF_P(float, 2); }
    else if (nc == 4) { if (prec == 0) GF_P(double, 4); else GF_P(float, 4); }
    else return hipErrorInvalidValue;
#undef GF_P
    return hipGetLastError();
}

hipError_t launch_sun_reunit(int prec, int nc, const Geom &g, void *U, hipStream_t st) {
    const long long n = 4LL * g.V;
    const int B = 256;
    const dim3 grid((unsigned)((n + B - 1) / B));
    if (nc == 2) {
        if (prec == 0) hipLaunchKernelGGL((k_sun_reunit<double, 2>), grid, dim3(B), 0, st, g, U);
        else hipLaunchKernelGGL((k_sun_reunit<float, 2>), grid, dim3(B), 0, st, g, U);
    } else if (nc == 4) {
        if (prec == 0) hipLaunchKernelGGL((k_sun_reunit<double, 4>), grid, dim3(B), 0, st, g, U);
        else hipLaunchKernelGGL((k_sun_reunit<float, 4>), grid, dim3(B), 0, st, g, U);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gf
