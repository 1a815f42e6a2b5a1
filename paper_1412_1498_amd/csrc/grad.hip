// grad.hip -- F_U[g] of eq. (1) as a function of a gauge transformation
// g(x) = exp(S(x)), S = i sum_a s_a lambda_a / 2, its gradient with respect to
// s_a(x), and the application of g to the links.
//
// Gradient: F depends on g(x) through (1/(d N_c V)) Re Tr[g(x) K(x)] with
// K(x) = sum_mu [U_mu(x) g(x+mu)^dagger + U_mu(x-mu)^dagger g(x-mu)^dagger]
// (eq. 5). With dg/ds_a = e^S sum_k (-ad_S)^k (X_a) / (k+1)!, X_a = i lambda_a/2,
// and Tr[ad_S(A) B] = -Tr[A ad_S(B)], the gradient is
//     dF/ds_a(x) = (1/(d N_c V)) Re Tr[X_a Psi],  Psi = sum_k ad_S^k(K e^S)/(k+1)!,
// one series on a 3x3 matrix per site followed by eight traces. At s = 0 it
// reduces to Re Tr[X_a K(x)] / (d N_c V).
#include "dmat.hpp"
#include "su3_device.hpp"
#include "tile_order.hpp"

namespace gf {

// S = i sum_a s_a lambda_a / 2 (anti-hermitian, traceless).
__device__ __forceinline__ void algebra_matrix(const double s[8], DMat &S) {
    const double r3 = 0.57735026918962576451;  // 1/sqrt(3)
    // H = sum_a s_a lambda_a / 2 (hermitian), S = i H
    double hr[9], hi[9];
    hr[0] = 0.5 * (s[2] + r3 * s[7]);       hi[0] = 0.0;
    hr[4] = 0.5 * (-s[2] + r3 * s[7]);      hi[4] = 0.0;
    hr[8] = -r3 * s[7];                     hi[8] = 0.0;
    hr[1] = 0.5 * s[0];  hi[1] = -0.5 * s[1];
    hr[3] = 0.5 * s[0];  hi[3] = 0.5 * s[1];
    hr[2] = 0.5 * s[3];  hi[2] = -0.5 * s[4];
    hr[6] = 0.5 * s[3];  hi[6] = 0.5 * s[4];
    hr[5] = 0.5 * s[5];  hi[5] = -0.5 * s[6];
    hr[7] = 0.5 * s[5];  hi[7] = 0.5 * s[6];
#pragma unroll
    for (int e = 0; e < 9; e++) { S.re[e] = -hi[e]; S.im[e] = hr[e]; }
}

// exp(S) by scaling and squaring of a degree-DEG Taylor polynomial (scaled
// argument of Frobenius norm <= 1/2, so the truncation is below
// 2^-(DEG+1) / (DEG+1)!: ~1e-20 for DEG = 16, ~1e-11 for DEG = 10).
template <int DEG>
__device__ void dm_exp(const DMat &S, DMat &E) {
    double nrm2 = 0.0;
#pragma unroll
    for (int e = 0; e < 9; e++) nrm2 += S.re[e] * S.re[e] + S.im[e] * S.im[e];
    const double nrm = sqrt(nrm2);
    int k = 0;
    if (nrm > 0.5) k = (int)ceil(log2(nrm / 0.5));
    const double sc = ldexp(1.0, -k);
    DMat Y;
#pragma unroll
    for (int e = 0; e < 9; e++) { Y.re[e] = S.re[e] * sc; Y.im[e] = S.im[e] * sc; }
#pragma unroll
    for (int e = 0; e < 9; e++) { E.re[e] = (e % 4 == 0) ? 1.0 : 0.0; E.im[e] = 0.0; }
#pragma unroll
    for (int j = DEG; j >= 1; j--) {
        DMat T;
        dm_mul(Y, E, T);
        const double inv = 1.0 / j;  // a constant once unrolled
#pragma unroll
        for (int e = 0; e < 9; e++) {
            E.re[e] = ((e % 4 == 0) ? 1.0 : 0.0) + T.re[e] * inv;
            E.im[e] = T.im[e] * inv;
        }
    }
    for (int i = 0; i < k; i++) {
        DMat T;
        dm_mul(E, E, T);
        E = T;
    }
}

template <typename R>
__device__ __forceinline__ void load_s(const R *__restrict__ s, int V, int n, double out[8]) {
#pragma unroll
    for (int a = 0; a < 8; a++) out[a] = (double)s[(long long)a * V + n];
}

// g field (9 complex per site, layout [e][p][h]) from s.
template <typename R>
__global__ void __launch_bounds__(256) k_expS(Geom g, const R *__restrict__ s, typename V2<R>::type *__restrict__ gf) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.V) return;
    double sv[8];
    load_s(s, g.V, n, sv);
    DMat S, E;
    algebra_matrix(sv, S);
    // the g field is stored in R: degree 10 is exact to float rounding, 16 to double
    dm_exp<sizeof(R) == 4 ? 10 : 16>(S, E);
#pragma unroll
    for (int e = 0; e < 9; e++) {
        typename V2<R>::type v;
        v.x = (R)E.re[e];
        v.y = (R)E.im[e];
        gf[(long long)e * g.V + n] = v;
    }
}

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double sh[16];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = v + __shfl_xor(v, m);
    const int wid = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x + 63) / 64; w++) t += sh[w];
    return t;
}

// Per-workgroup partial sums of Re Tr[g(x) U_mu(x) g(x+mu)^dagger].
template <typename R, int NE, int ND>
__global__ void __launch_bounds__(256) k_functional(Geom g, const typename V2<R>::type *__restrict__ U,
                             const typename V2<R>::type *__restrict__ gf, double *__restrict__ part) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    double f = 0.0;
    if (n < g.V) {
        const int p = n >= g.Vh, h = n - p * g.Vh;
        const SiteNbr fw = site_fwd_neighbours(g, p, h);
        DMat gx;
        load_g<R>(gf, g.V, n, gx);
#pragma unroll
        for (int mu = 0; mu < ND; mu++) {
            DMat u, gu, gy;
            load_u<R, NE>(U, link_off(g, mu, p, h), u);
            load_g<R>(gf, g.V, (1 - p) * g.Vh + pick4(fw.hb, mu), gy);
            dm_mul(gx, u, gu);
#pragma unroll
            for (int e = 0; e < 9; e++) f += gu.re[e] * gy.re[e] + gu.im[e] * gy.im[e];
        }
    }
    const double t = block_sum(f);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(256) k_sum_partials(const double *__restrict__ part, int n, double *__restrict__ out) {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
    const double t = block_sum(v);
    if (threadIdx.x == 0) out[0] = t;
}

template <typename R, int NE, int ND>
__global__ void __launch_bounds__(256) k_functional_grad(Geom g, const typename V2<R>::type *__restrict__ U,
                                  const R *__restrict__ s, const typename V2<R>::type *__restrict__ gf,
                                  double scale, R *__restrict__ grad) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.V) return;
    const int p = n >= g.Vh, h = n - p * g.Vh;
    const SiteNbr fw = site_fwd_neighbours(g, p, h);
    const SiteNbr bw = site_neighbours(g, p, h);
    DMat K;
#pragma unroll
    for (int e = 0; e < 9; e++) { K.re[e] = 0.0; K.im[e] = 0.0; }
#pragma unroll
    for (int mu = 0; mu < ND; mu++) {
        DMat u, gy, t;
        // U_mu(x) g(x+mu)^dagger
        load_u<R, NE>(U, link_off(g, mu, p, h), u);
        load_g<R>(gf, g.V, (1 - p) * g.Vh + pick4(fw.hb, mu), gy);
        dm_mul_nd(u, gy, t);
#pragma unroll
        for (int e = 0; e < 9; e++) { K.re[e] += t.re[e]; K.im[e] += t.im[e]; }
        // U_mu(x-mu)^dagger g(x-mu)^dagger
        const int nb = (1 - p) * g.Vh + pick4(bw.hb, mu);
        load_u<R, NE>(U, link_off(g, mu, 1 - p, pick4(bw.hb, mu)), u);
        load_g<R>(gf, g.V, nb, gy);
        dm_mul_dd(u, gy, t);
#pragma unroll
        for (int e = 0; e < 9; e++) { K.re[e] += t.re[e]; K.im[e] += t.im[e]; }
    }
    double sv[8];
    load_s(s, g.V, n, sv);
    DMat S, gx, Y;
    algebra_matrix(sv, S);
    load_g<R>(gf, g.V, n, gx);
    dm_mul(K, gx, Y);  // K e^S
    // Psi = sum_k ad_S^k(Y) / (k+1)!
    DMat Psi = Y, T = Y;
    double ymax = 0.0;
#pragma unroll
    for (int e = 0; e < 9; e++) ymax = fmax(ymax, fabs(Y.re[e]) + fabs(Y.im[e]));
    double fact = 1.0;
    // the series stops once a term is below the output's rounding (float or double)
    const double tol = sizeof(R) == 4 ? 1e-10 : 1e-18;
    for (int k = 1; k <= 60; k++) {
        DMat A, B;
        dm_mul(S, T, A);
        dm_mul(T, S, B);
        double tmax = 0.0;
#pragma unroll
        for (int e = 0; e < 9; e++) {
            T.re[e] = A.re[e] - B.re[e];
            T.im[e] = A.im[e] - B.im[e];
            tmax = fmax(tmax, fabs(T.re[e]) + fabs(T.im[e]));
        }
        fact *= (k + 1);
        const double inv = 1.0 / fact;
#pragma unroll
        for (int e = 0; e < 9; e++) { Psi.re[e] += T.re[e] * inv; Psi.im[e] += T.im[e] * inv; }
        if (tmax * inv <= tol * ymax) break;
    }
    // Re Tr[(i lambda_a / 2) Psi] = -Im Tr[lambda_a Psi] / 2
    const double r3 = 0.57735026918962576451;
    double tr[8];
    tr[0] = Psi.im[3] + Psi.im[1];                        // Im(P10 + P01)
    tr[1] = -Psi.re[3] + Psi.re[1];                       // Im(-i P10 + i P01)
    tr[2] = Psi.im[0] - Psi.im[4];
    tr[3] = Psi.im[6] + Psi.im[2];
    tr[4] = -Psi.re[6] + Psi.re[2];
    tr[5] = Psi.im[7] + Psi.im[5];
    tr[6] = -Psi.re[7] + Psi.re[5];
    tr[7] = r3 * (Psi.im[0] + Psi.im[4] - 2.0 * Psi.im[8]);
    const double c = scale / (2.0 * ND * 3.0 * (double)g.V);
#pragma unroll
    for (int a = 0; a < 8; a++) grad[(long long)a * g.V + n] = (R)(-tr[a] * c);
}

// U_mu(x) <- g(x) U_mu(x) g(x+mu)^dagger for all four mu. A workgroup takes
// GT_TILE/2 half-indices in both parities, so the g(x+mu) it reads (the other
// parity, nearby h) were mostly brought into cache by its own g(x) reads;
// tiles are dealt XCD-contiguously.
constexpr int GT_TILE = 256;

template <typename R, int NE>
__global__ void __launch_bounds__(GT_TILE) k_gauge_transform(Geom g, typename V2<R>::type *__restrict__ U,
                                  const typename V2<R>::type *__restrict__ gf) {
    constexpr int QH = GT_TILE / 2;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int p = threadIdx.x >= QH;
    const int h = tile * QH + (int)threadIdx.x - p * QH;
    if (h >= g.Vh) return;
    const int n = p * g.Vh + h;
    const SiteNbr fw = site_fwd_neighbours(g, p, h);
    DMat gx;
    load_g<R>(gf, g.V, n, gx);
    for (int mu = 0; mu < 4; mu++) {
        DMat u, gy;
        load_u<R, NE, true>(U, link_off(g, mu, p, h), u);  // each link is read and written once: stream
        load_g<R>(gf, g.V, (1 - p) * g.Vh + pick4(fw.hb, mu), gy);
        Mat<R> m;
        gauge_rotate<R>(gx, u, gy, m);
        store_link<R, NE, true>(m, as_global((void *)U), link_off(g, mu, p, h));
    }
}

constexpr int GB = 256;

hipError_t launch_expS(int prec, const Geom &g, const void *s, void *gfield, hipStream_t st) {
    const dim3 grid((g.V + GB - 1) / GB);
    if (prec == 0)
        hipLaunchKernelGGL(k_expS<double>, grid, dim3(GB), 0, st, g, (const double *)s,
                           (V2<double>::type *)gfield);
    else
        hipLaunchKernelGGL(k_expS<float>, grid, dim3(GB), 0, st, g, (const float *)s,
                           (V2<float>::type *)gfield);
    return hipGetLastError();
}

hipError_t launch_functional(int prec, int nelem, int gauge, const Geom &g, const void *U,
                             const void *gfield, double *d_partials, hipStream_t st) {
    const dim3 grid((g.V + GB - 1) / GB);
#define GF_L(R, NE)                                                                               \
    do {                                                                                          \
        if (gauge == 0)                                                                           \
            hipLaunchKernelGGL((k_functional<R, NE, 4>), grid, dim3(GB), 0, st, g,                \
                               (const V2<R>::type *)U, (const V2<R>::type *)gfield, d_partials);   \
        else                                                                                      \
            hipLaunchKernelGGL((k_functional<R, NE, 3>), grid, dim3(GB), 0, st, g,                \
                               (const V2<R>::type *)U, (const V2<R>::type *)gfield, d_partials);   \
    } while (0)
    if (prec == 0) { if (nelem == 9) GF_L(double, 9); else if (nelem == 6) GF_L(double, 6); else GF_L(double, 4); }
    else { if (nelem == 9) GF_L(float, 9); else if (nelem == 6) GF_L(float, 6); else GF_L(float, 4); }
#undef GF_L
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double *d_partials, int n, double *d_out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, d_partials, n, d_out);
    return hipGetLastError();
}

hipError_t launch_functional_grad(int prec, int nelem, int gauge, const Geom &g, const void *U,
                                  const void *s, const void *gfield, double scale, void *grad,
                                  hipStream_t st) {
    const dim3 grid((g.V + GB - 1) / GB);
#define GF_L(R, NE)                                                                               \
    do {                                                                                          \
        if (gauge == 0)                                                                           \
            hipLaunchKernelGGL((k_functional_grad<R, NE, 4>), grid, dim3(GB), 0, st, g,           \
                               (const V2<R>::type *)U, (const R *)s, (const V2<R>::type *)gfield,  \
                               scale, (R *)grad);                                                 \
        else                                                                                      \
            hipLaunchKernelGGL((k_functional_grad<R, NE, 3>), grid, dim3(GB), 0, st, g,           \
                               (const V2<R>::type *)U, (const R *)s, (const V2<R>::type *)gfield,  \
                               scale, (R *)grad);                                                 \
    } while (0)
    if (prec == 0) { if (nelem == 9) GF_L(double, 9); else if (nelem == 6) GF_L(double, 6); else GF_L(double, 4); }
    else { if (nelem == 9) GF_L(float, 9); else if (nelem == 6) GF_L(float, 6); else GF_L(float, 4); }
#undef GF_L
    return hipGetLastError();
}

hipError_t launch_gauge_transform(int prec, int nelem, const Geom &g, void *U, const void *gfield,
                                  hipStream_t st) {
    const dim3 grid((g.Vh + GT_TILE / 2 - 1) / (GT_TILE / 2));
#define GF_L(R, NE)                                                                               \
    hipLaunchKernelGGL((k_gauge_transform<R, NE>), grid, dim3(GT_TILE), 0, st, g, (V2<R>::type *)U, \
                       (const V2<R>::type *)gfield)
    if (prec == 0) { if (nelem == 9) GF_L(double, 9); else if (nelem == 6) GF_L(double, 6); else GF_L(double, 4); }
    else { if (nelem == 9) GF_L(float, 9); else if (nelem == 6) GF_L(float, 6); else GF_L(float, 4); }
#undef GF_L
    return hipGetLastError();
}

}  // namespace gf
