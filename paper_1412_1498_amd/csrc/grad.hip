// grad.hip -- F_U[g] of eq. (1) as a function of a gauge transformation
// g(x) = exp(S(x)), S = i sum_a s_a lambda_a / 2, its gradient with respect to
// s_a(x), and the application of g to the links.
//
// Gradient: F depends on g(x) through (1/(d N_c V)) Re Tr[g(x) K(x)] with
// K(x) = sum_mu [U_mu(x) g(x+mu)^dagger + U_mu(x-mu)^dagger g(x-mu)^dagger]
// (eq. 5). With dg/ds_a = e^S sum_k (-ad_S)^k (X_a) / (k+1)!, X_a = i lambda_a/2,
// and Tr[ad_S(A) B] = -Tr[A ad_S(B)], the gradient is
//     dF/ds_a(x) = (1/(d N_c V)) Re Tr[X_a Psi],  Psi = sum_k ad_S^k(K e^S)/(k+1)!.
// ad_S maps hermitian to hermitian and anti-hermitian to anti-hermitian
// matrices and keeps traces at zero, and Re Tr[X_a H] = 0 for hermitian H,
// so only the eight su(3) components of K e^S matter: the series runs on
// those, with ad_S an 8 x 8 antisymmetric map built from the structure
// constants (54 multiply-adds a term instead of two 3x3 complex products).
// At s = 0 it reduces to Re Tr[X_a K(x)] / (d N_c V).
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

constexpr double inv_factorial(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; i++) f *= i;
    return 1.0 / f;
}

// c = a b for 3x3 complex matrices with elements of type T (float or
// double), each element an FMA chain (in double the same operations as
// dm_mul).
template <typename T>
__device__ __forceinline__ void cm_mul(const Mat<T> &a, const Mat<T> &b, Mat<T> &c) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            T r = a.re[3 * i] * b.re[j], m = a.re[3 * i] * b.im[j];
            r = fma(-a.im[3 * i], b.im[j], r);
            m = fma(a.im[3 * i], b.re[j], m);
#pragma unroll
            for (int k = 1; k < 3; k++) {
                r = fma(a.re[3 * i + k], b.re[3 * k + j], r);
                r = fma(-a.im[3 * i + k], b.im[3 * k + j], r);
                m = fma(a.re[3 * i + k], b.im[3 * k + j], m);
                m = fma(a.im[3 * i + k], b.re[3 * k + j], m);
            }
            c.re[3 * i + j] = r;
            c.im[3 * i + j] = m;
        }
}

// exp(S) in arithmetic of type T by scaling and squaring of the Taylor
// polynomial of degree B * NB - 1 (scaled argument Y of Frobenius norm
// <= 1/2, so the truncation is below 2^-(B NB) / (B NB)!: 5e-9 for degree 8,
// 2e-17 for degree 15), evaluated by the Paterson-Stockmeyer scheme: the
// powers Y^2 .. Y^B once, then Horner in Z = Y^B over coefficient blocks
// sum_j c_{B i + j} Y^j (j < B). Degree 8 takes 4 matrix products instead of
// 8, degree 15 takes 6 instead of 15.
template <typename T, int B, int NB>
__device__ void cm_exp(const Mat<T> &S, Mat<T> &E) {
    T nrm2 = T(0);
#pragma unroll
    for (int e = 0; e < 9; e++) nrm2 += S.re[e] * S.re[e] + S.im[e] * S.im[e];
    const T nrm = sqrt(nrm2);
    int k = 0;
    if (nrm > T(0.5)) k = (int)ceil(log2(nrm / T(0.5)));
    const T sc = ldexp(T(1), -k);
    Mat<T> pw[B + 1];  // pw[j] = Y^j, j = 1 .. B
#pragma unroll
    for (int e = 0; e < 9; e++) { pw[1].re[e] = S.re[e] * sc; pw[1].im[e] = S.im[e] * sc; }
#pragma unroll
    for (int j = 2; j <= B; j++) cm_mul(pw[j - 1], pw[1], pw[j]);
    // E = block NB - 1, then E <- E Z + block i for i = NB - 2 .. 0
#pragma unroll
    for (int i = NB - 1; i >= 0; i--) {
        Mat<T> Tm;
        if (i < NB - 1) cm_mul(E, pw[B], Tm);
#pragma unroll
        for (int e = 0; e < 9; e++) {
            T r = (e % 4 == 0) ? T(inv_factorial(B * i)) : T(0), m = T(0);
#pragma unroll
            for (int j = 1; j < B; j++) {
                r = fma(T(inv_factorial(B * i + j)), pw[j].re[e], r);
                m = fma(T(inv_factorial(B * i + j)), pw[j].im[e], m);
            }
            if (i < NB - 1) { r += Tm.re[e]; m += Tm.im[e]; }
            E.re[e] = r;
            E.im[e] = m;
        }
    }
    for (int i = 0; i < k; i++) {
        Mat<T> Tm;
        cm_mul(E, E, Tm);
        E = Tm;
    }
}

// s_a(x) of site (p, h) (layout alg_off).
template <typename R>
__device__ __forceinline__ void load_s(const R *__restrict__ s, const Geom &g, int p, int h, double out[8]) {
    const long long o = alg_off(g, p, h, 0);
#pragma unroll
    for (int a = 0; a < 8; a++) out[a] = (double)s[o + (long long)a * BLK];
}

// g field (9 complex per site, layout gfield_off) from s.
template <typename R>
__global__ void __launch_bounds__(256) k_expS(Geom g, const R *__restrict__ s, typename V2<R>::type *__restrict__ gf) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.V) return;
    const int p = n >= g.Vh, h = n - p * g.Vh;
    double sv[8];
    load_s(s, g, p, h, sv);
    DMat S;
    algebra_matrix(sv, S);
    // The g field is stored in R, and the exponential is evaluated in R:
    // degree 8 in float (truncation 5e-9, rounding a few units of float's,
    // as for the stored g itself; in float the kernel needs half the
    // registers and runs 136 -> 107 us at 48^4), degree 15 in double.
    Mat<R> Sr, E;
#pragma unroll
    for (int e = 0; e < 9; e++) { Sr.re[e] = (R)S.re[e]; Sr.im[e] = (R)S.im[e]; }
    if constexpr (sizeof(R) == 4) cm_exp<R, 3, 3>(Sr, E);
    else cm_exp<R, 4, 4>(Sr, E);
#pragma unroll
    for (int e = 0; e < 9; e++) {
        typename V2<R>::type v;
        v.x = E.re[e];
        v.y = E.im[e];
        gf[gfield_off(g, p, h, e)] = v;
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

// Sites of a workgroup: DT_TILE/2 consecutive half indices h in both parities
// (lanes [0, DT_TILE/2) even, the rest odd), tiles dealt XCD-contiguously.
// A site's neighbours x +- mu belong to the other parity at nearby h (x, y
// steps) or at h +- one z or t stride, so the workgroup's own reads bring
// most of the neighbours' links and g into the cache it shares with the
// tiles next to it, instead of each being fetched twice from HBM.
constexpr int DT_TILE = 256;

__device__ __forceinline__ bool tile_site(const Geom &g, const SlabOrder &so, int &p, int &h) {
    constexpr int QH = DT_TILE / 2;
    const int tile = slab_tile(xcd_tile(blockIdx.x, gridDim.x), so);
    p = threadIdx.x >= QH;
    h = tile * QH + (int)threadIdx.x - p * QH;
    return h < g.Vh;
}

// Per-workgroup partial sums of Re Tr[g(x) U_mu(x) g(x+mu)^dagger].
template <typename R, int NE, int ND>
__global__ void __launch_bounds__(DT_TILE) k_functional(Geom g, const typename V2<R>::type *__restrict__ U,
                             const typename V2<R>::type *__restrict__ gf, SlabOrder so, double *__restrict__ part) {
    int p, h;
    double f = 0.0;
    if (tile_site(g, so, p, h)) {
        const SiteNbr fw = site_fwd_neighbours(g, p, h);
        DMat gx;
        load_g<R>(gf, g, p, h, gx);
#pragma unroll
        for (int mu = 0; mu < ND; mu++) {
            DMat u, gu, gy;
            load_u<R, NE>(U, link_off(g, mu, p, h), u);
            load_g<R>(gf, g, 1 - p, pick4(fw.hb, mu), gy);
            dm_mul(gx, u, gu);
#pragma unroll
            for (int e = 0; e < 9; e++) f += gu.re[e] * gy.re[e] + gu.im[e] * gy.im[e];
        }
    }
    const double t = block_sum(f);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// One workgroup of 1024 lanes: strided sums per lane, then the fixed butterfly.
__global__ void __launch_bounds__(1024) k_sum_partials(const double *__restrict__ part, int n, double *__restrict__ out) {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
    const double t = block_sum(v);
    if (threadIdx.x == 0) out[0] = t;
}

// Components of the anti-hermitian traceless part of a 3x3 matrix Y in the
// basis X_a = i lambda_a / 2: out[a] = Im Tr[lambda_a Y] = -2 Re Tr[X_a Y]
// (the hermitian part and the trace give no real part to Re Tr[X_a Y]).
__device__ __forceinline__ void su3_components(const DMat &Y, double out[8]) {
    const double r3 = 0.57735026918962576451;
    out[0] = Y.im[3] + Y.im[1];            // Im(Y10 + Y01)
    out[1] = Y.re[1] - Y.re[3];            // Im(-i Y10 + i Y01)
    out[2] = Y.im[0] - Y.im[4];
    out[3] = Y.im[6] + Y.im[2];
    out[4] = Y.re[2] - Y.re[6];
    out[5] = Y.im[7] + Y.im[5];
    out[6] = Y.re[5] - Y.re[7];
    out[7] = r3 * (Y.im[0] + Y.im[4] - 2.0 * Y.im[8]);
}

// ad_S in components: with [X_a, X_b] = -sum_c f_abc X_c (f the structure
// constants of su(3), [lambda_a, lambda_b] = 2i f_abc lambda_c) and
// S = sum_a s_a X_a, ad_S(sum_b v_b X_b) = sum_c w_c X_c with
// w_c = -sum_{a,b} s_a f_abc v_b. Each totally antisymmetric triple
// (i, j, k; f) contributes w_i += f (s_k v_j - s_j v_k) and its cyclic
// images. Nonzero f (generators numbered from 1): f_123 = 1,
// f_147 = f_246 = f_257 = f_345 = 1/2, f_156 = f_367 = -1/2,
// f_458 = f_678 = sqrt(3)/2.
__device__ __forceinline__ void ad_triple(const double s[8], const double v[8], double w[8], int i, int j,
                                          int k, double f) {
    w[i] += f * (s[k] * v[j] - s[j] * v[k]);
    w[j] += f * (s[i] * v[k] - s[k] * v[i]);
    w[k] += f * (s[j] * v[i] - s[i] * v[j]);
}

__device__ __forceinline__ void ad_components(const double s[8], const double v[8], double w[8]) {
    const double h3 = 0.86602540378443864676;  // sqrt(3)/2
#pragma unroll
    for (int a = 0; a < 8; a++) w[a] = 0.0;
    ad_triple(s, v, w, 0, 1, 2, 1.0);
    ad_triple(s, v, w, 0, 3, 6, 0.5);
    ad_triple(s, v, w, 0, 4, 5, -0.5);
    ad_triple(s, v, w, 1, 3, 5, 0.5);
    ad_triple(s, v, w, 1, 4, 6, 0.5);
    ad_triple(s, v, w, 2, 3, 4, 0.5);
    ad_triple(s, v, w, 2, 5, 6, -0.5);
    ad_triple(s, v, w, 3, 4, 7, h3);
    ad_triple(s, v, w, 5, 6, 7, h3);
}

template <typename R, int NE, int ND>
__global__ void __launch_bounds__(DT_TILE) k_functional_grad(Geom g, const typename V2<R>::type *__restrict__ U,
                                  const R *__restrict__ s, const typename V2<R>::type *__restrict__ gf,
                                  double scale, SlabOrder so, R *__restrict__ grad) {
    int p, h;
    if (!tile_site(g, so, p, h)) return;
    const SiteNbr fw = site_fwd_neighbours(g, p, h);
    const SiteNbr bw = site_neighbours(g, p, h);
    // The site's own s and g first, then the staple from t and z down to x:
    // the t and z neighbours' links and g lie in other tiles, and the earlier
    // in a workgroup's life they are read, the fewer tiles have passed
    // through L2 since their own workgroups read them (the x and y
    // neighbours mostly lie in this tile).
    double sv[8];
    load_s(s, g, p, h, sv);
    DMat gx;
    load_g<R>(gf, g, p, h, gx);
    DMat K;
#pragma unroll
    for (int e = 0; e < 9; e++) { K.re[e] = 0.0; K.im[e] = 0.0; }
#pragma unroll
    for (int mu = ND - 1; mu >= 0; mu--) {
        DMat u, gy, t;
        // U_mu(x-mu)^dagger g(x-mu)^dagger
        load_u<R, NE>(U, link_off(g, mu, 1 - p, pick4(bw.hb, mu)), u);
        load_g<R>(gf, g, 1 - p, pick4(bw.hb, mu), gy);
        dm_mul_dd(u, gy, t);
#pragma unroll
        for (int e = 0; e < 9; e++) { K.re[e] += t.re[e]; K.im[e] += t.im[e]; }
        // U_mu(x) g(x+mu)^dagger
        load_u<R, NE>(U, link_off(g, mu, p, h), u);
        load_g<R>(gf, g, 1 - p, pick4(fw.hb, mu), gy);
        dm_mul_nd(u, gy, t);
#pragma unroll
        for (int e = 0; e < 9; e++) { K.re[e] += t.re[e]; K.im[e] += t.im[e]; }
    }
    DMat Y;
    dm_mul(K, gx, Y);  // K e^S
    // Only the anti-hermitian traceless part of Y reaches the traces, and
    // ad_S maps that part to itself, so the series runs on its components:
    // that part is sum_b alpha_b X_b with alpha_b = Im Tr[lambda_b Y]
    // (Tr X_a X_b = -delta_ab / 2), and the gradient is -psi_a / 2 times
    // 1 / (d N_c V) for psi = sum_k ad_S^k(alpha) / (k+1)!.
    double tr[8];
    su3_components(Y, tr);
    double term[8];
    double amax = 0.0;
#pragma unroll
    for (int a = 0; a < 8; a++) { term[a] = tr[a]; amax = fmax(amax, fabs(tr[a])); }
    // the series stops once a term is below the output's rounding (float or double)
    const double tol = sizeof(R) == 4 ? 1e-10 : 1e-18;
    for (int k = 1; k <= 60; k++) {
        double nxt[8];
        ad_components(sv, term, nxt);
        const double inv = 1.0 / (k + 1);
        double tmax = 0.0;
#pragma unroll
        for (int a = 0; a < 8; a++) {
            term[a] = nxt[a] * inv;
            tr[a] += term[a];
            tmax = fmax(tmax, fabs(term[a]));
        }
        if (tmax <= tol * amax) break;
    }
    const double c = scale / (2.0 * ND * 3.0 * (double)g.V);
    const long long o = alg_off(g, p, h, 0);
#pragma unroll
    for (int a = 0; a < 8; a++) grad[o + (long long)a * BLK] = (R)(-tr[a] * c);
}

// U_mu(x) <- g(x) U_mu(x) g(x+mu)^dagger for all four mu. A workgroup takes
// GT_TILE/2 half-indices in both parities, so the g(x+mu) it reads (the other
// parity, nearby h) were mostly brought into cache by its own g(x) reads;
// tiles are dealt XCD-contiguously.
constexpr int GT_TILE = 256;

template <typename R, int NE>
__global__ void __launch_bounds__(GT_TILE) k_gauge_transform(Geom g, typename V2<R>::type *__restrict__ U,
                                  const typename V2<R>::type *__restrict__ gf, SlabOrder so) {
    constexpr int QH = GT_TILE / 2;
    const int tile = slab_tile(xcd_tile(blockIdx.x, gridDim.x), so);
    const int p = threadIdx.x >= QH;
    const int h = tile * QH + (int)threadIdx.x - p * QH;
    if (h >= g.Vh) return;
    const SiteNbr fw = site_fwd_neighbours(g, p, h);
    DMat gx;
    load_g<R>(gf, g, p, h, gx);
    for (int mu = 0; mu < 4; mu++) {
        DMat u, gy;
        load_u<R, NE, true>(U, link_off(g, mu, p, h), u);  // each link is read and written once: stream
        load_g<R>(gf, g, 1 - p, pick4(fw.hb, mu), gy);
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
    const dim3 grid((g.Vh + DT_TILE / 2 - 1) / (DT_TILE / 2));
    const SlabOrder so = make_slab_order(g.st, DT_TILE / 2, (int)grid.x, 64);
#define GF_L(R, NE)                                                                               \
    do {                                                                                          \
        if (gauge == 0)                                                                           \
            hipLaunchKernelGGL((k_functional<R, NE, 4>), grid, dim3(DT_TILE), 0, st, g,           \
                               (const V2<R>::type *)U, (const V2<R>::type *)gfield, so, d_partials); \
        else                                                                                      \
            hipLaunchKernelGGL((k_functional<R, NE, 3>), grid, dim3(DT_TILE), 0, st, g,           \
                               (const V2<R>::type *)U, (const V2<R>::type *)gfield, so, d_partials); \
    } while (0)
    if (prec == 0) { if (nelem == 9) GF_L(double, 9); else if (nelem == 6) GF_L(double, 6); else GF_L(double, 4); }
    else { if (nelem == 9) GF_L(float, 9); else if (nelem == 6) GF_L(float, 6); else GF_L(float, 4); }
#undef GF_L
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double *d_partials, int n, double *d_out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, st, d_partials, n, d_out);
    return hipGetLastError();
}

hipError_t launch_functional_grad(int prec, int nelem, int gauge, const Geom &g, const void *U,
                                  const void *s, const void *gfield, double scale, void *grad,
                                  hipStream_t st) {
    const dim3 grid((g.Vh + DT_TILE / 2 - 1) / (DT_TILE / 2));
    const SlabOrder so = make_slab_order(g.st, DT_TILE / 2, (int)grid.x, 64);
#define GF_L(R, NE)                                                                               \
    do {                                                                                          \
        if (gauge == 0)                                                                           \
            hipLaunchKernelGGL((k_functional_grad<R, NE, 4>), grid, dim3(DT_TILE), 0, st, g,      \
                               (const V2<R>::type *)U, (const R *)s, (const V2<R>::type *)gfield,  \
                               scale, so, (R *)grad);                                             \
        else                                                                                      \
            hipLaunchKernelGGL((k_functional_grad<R, NE, 3>), grid, dim3(DT_TILE), 0, st, g,      \
                               (const V2<R>::type *)U, (const R *)s, (const V2<R>::type *)gfield,  \
                               scale, so, (R *)grad);                                             \
    } while (0)
    if (prec == 0) { if (nelem == 9) GF_L(double, 9); else if (nelem == 6) GF_L(double, 6); else GF_L(double, 4); }
    else { if (nelem == 9) GF_L(float, 9); else if (nelem == 6) GF_L(float, 6); else GF_L(float, 4); }
#undef GF_L
    return hipGetLastError();
}

hipError_t launch_gauge_transform(int prec, int nelem, const Geom &g, void *U, const void *gfield,
                                  hipStream_t st) {
    const dim3 grid((g.Vh + GT_TILE / 2 - 1) / (GT_TILE / 2));
    const SlabOrder so = make_slab_order(g.st, GT_TILE / 2, (int)grid.x, 64);
#define GF_L(R, NE)                                                                               \
    hipLaunchKernelGGL((k_gauge_transform<R, NE>), grid, dim3(GT_TILE), 0, st, g, (V2<R>::type *)U, \
                       (const V2<R>::type *)gfield, so)
    if (prec == 0) { if (nelem == 9) GF_L(double, 9); else if (nelem == 6) GF_L(double, 6); else GF_L(double, 4); }
    else { if (nelem == 9) GF_L(float, 9); else if (nelem == 6) GF_L(float, 6); else GF_L(float, 4); }
#undef GF_L
    return hipGetLastError();
}

}  // namespace gf
