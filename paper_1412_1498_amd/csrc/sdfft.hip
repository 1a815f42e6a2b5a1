// sdfft.hip -- kernels of steepest descent with Fourier acceleration
// (Alg. 2, eqs. 7-9): the divergence Delta(x) as 8 real su(3) components in
// lexicographic site order (the input of the transforms in fft.hip, which
// also apply the p^2_max / p^2 filter), and the first-order gauge
// transformation g(x) = reunit(1 + (alpha/2) F^-1[...] Delta) written as a g
// field for k_gauge_transform.
//
// Delta is anti-hermitian and traceless: Delta = i sum_a d_a lambda_a with
// d_a = Tr[lambda_a Delta] / (2i) real, so filtering the eight real d_a is
// the same linear map as filtering every matrix element.
#include "su3_device.hpp"
#include "tile_order.hpp"

namespace gf {

// Lexicographic index x + nx(y + ny(z + nz t)) of site (p, h): 2h + (x mod 2).
__device__ __forceinline__ int lex_of(const Geom &g, int p, int h) {
    const int q = h / g.hx;
    const int q2 = q / g.ny;
    const int j = q - q2 * g.ny;
    const int t = q2 / g.nz;
    const int k = q2 - t * g.nz;
    return 2 * h + ((p + j + k + t) & 1);
}

// d_a(x) = Tr[lambda_a Delta(x)] / (2i) for every site, Delta of eq. (3),
// stored [t][a][z][y][x].
// A workgroup takes SD_TILE/2 half-indices h in both parities (lanes below
// SD_TILE/2 even): a site's backward links are the other parity's links at
// nearby h, which the workgroup's own forward reads bring into cache, and
// the tile's lexicographic outputs 2h + (x mod 2) fill one contiguous range.
// Tiles are dealt XCD-contiguously (each XCD's L2 then holds the z
// neighbours).
constexpr int SD_TILE = 256;

template <typename R, int NE>
__global__ void __launch_bounds__(SD_TILE) k_sd_delta(Geom g, int nd, const typename V2<R>::type *__restrict__ Uv,
                           R *__restrict__ d) {
    constexpr int QH = SD_TILE / 2;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int p = threadIdx.x >= QH;
    const int h = tile * QH + (int)threadIdx.x - p * QH;
    if (h >= g.Vh) return;
    const SiteNbr nb = site_neighbours(g, p, h);
    const gchar *U = as_global((const void *)Uv);
    double mr[9], mi[9];
#pragma unroll
    for (int e = 0; e < 9; e++) { mr[e] = 0.0; mi[e] = 0.0; }
    for (int mu = 0; mu < nd; mu++) {
        Mat<R> f, b;
        load_link<R, NE, false>(f, U, link_off(g, mu, p, h));
        load_link<R, NE, false>(b, U, link_off(g, mu, 1 - p, pick4(nb.hb, mu)));
#pragma unroll
        for (int e = 0; e < 9; e++) {
            mr[e] += (double)b.re[e] - (double)f.re[e];
            mi[e] += (double)b.im[e] - (double)f.im[e];
        }
    }
    // A = M - M^dagger (anti-hermitian); its traceless part is Delta, whose
    // components need only Im of the diagonal and the off-diagonal entries.
    double ar[9], ai[9];
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            ar[3 * r + c] = mr[3 * r + c] - mr[3 * c + r];
            ai[3 * r + c] = mi[3 * r + c] + mi[3 * c + r];
        }
    const double r3 = 0.57735026918962576451;  // 1/sqrt(3)
    double o[8];
    // Tr[lambda_a A] / (2i) = Im(Tr[lambda_a A]) / 2 (the trace part drops out)
    o[0] = 0.5 * (ai[3] + ai[1]);
    o[1] = 0.5 * (ar[1] - ar[3]);
    o[2] = 0.5 * (ai[0] - ai[4]);
    o[3] = 0.5 * (ai[6] + ai[2]);
    o[4] = 0.5 * (ar[2] - ar[6]);
    o[5] = 0.5 * (ai[7] + ai[5]);
    o[6] = 0.5 * (ar[5] - ar[7]);
    o[7] = 0.5 * r3 * (ai[0] + ai[4] - 2.0 * ai[8]);
    const int lx = lex_of(g, p, h);
    // layout [t][a][z][y][x]: rows along x for the real transform
    const int V3 = g.V / g.nt;
    const int t = lx / V3, x3 = lx - t * V3;
#pragma unroll
    for (int a = 0; a < 8; a++) d[((long long)t * 8 + a) * V3 + x3] = (R)o[a];
}

// g(x) = reunit(1 + i sum_a d_a lambda_a) in double, stored as the g field
// [e][p][h] (9 complex per site) in the context precision.
// Tiled like k_sd_delta: the tile's lexicographic reads fill one range.
template <typename R>
__global__ void __launch_bounds__(SD_TILE) k_sd_gfield(Geom g, const R *__restrict__ d, typename V2<R>::type *__restrict__ gf) {
    constexpr int QH = SD_TILE / 2;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int p = threadIdx.x >= QH;
    const int h = tile * QH + (int)threadIdx.x - p * QH;
    if (h >= g.Vh) return;
    const int n = p * g.Vh + h;
    const int lx = lex_of(g, p, h);
    double s[8];
    const int V3 = g.V / g.nt;
    const int t = lx / V3, x3 = lx - t * V3;
#pragma unroll
    for (int a = 0; a < 8; a++) s[a] = (double)d[((long long)t * 8 + a) * V3 + x3];
    const double r3 = 0.57735026918962576451;
    // H = sum_a s_a lambda_a; 1 + i H
    double hr[9], hi[9];
    hr[0] = s[2] + r3 * s[7];  hi[0] = 0.0;
    hr[4] = -s[2] + r3 * s[7]; hi[4] = 0.0;
    hr[8] = -2.0 * r3 * s[7];  hi[8] = 0.0;
    hr[1] = s[0]; hi[1] = -s[1];
    hr[3] = s[0]; hi[3] = s[1];
    hr[2] = s[3]; hi[2] = -s[4];
    hr[6] = s[3]; hi[6] = s[4];
    hr[5] = s[5]; hi[5] = -s[6];
    hr[7] = s[5]; hi[7] = s[6];
    Mat<double> m;
#pragma unroll
    for (int e = 0; e < 9; e++) {
        m.re[e] = (e % 4 == 0 ? 1.0 : 0.0) - hi[e];
        m.im[e] = hr[e];
    }
    reunitarise(m);
#pragma unroll
    for (int e = 0; e < 9; e++) {
        typename V2<R>::type v;
        v.x = (R)m.re[e];
        v.y = (R)m.im[e];
        gf[(long long)e * g.V + n] = v;
    }
}

hipError_t launch_sd_delta(int prec, int nelem, int gauge, const Geom &g, const void *U, void *d,
                           hipStream_t st) {
    const int B = SD_TILE;
    const dim3 grid((g.Vh + B / 2 - 1) / (B / 2));
    const int nd = gauge == 0 ? 4 : 3;
#define GF_L(R, NE)                                                                              \
    hipLaunchKernelGGL((k_sd_delta<R, NE>), grid, dim3(B), 0, st, g, nd,                         \
                       (const V2<R>::type *)U, (R *)d)
    if (prec == 0) { if (nelem == 9) GF_L(double, 9); else if (nelem == 6) GF_L(double, 6); else GF_L(double, 4); }
    else { if (nelem == 9) GF_L(float, 9); else if (nelem == 6) GF_L(float, 6); else GF_L(float, 4); }
#undef GF_L
    return hipGetLastError();
}

hipError_t launch_sd_gfield(int prec, const Geom &g, const void *d, void *gfield, hipStream_t st) {
    const int B = SD_TILE;
    const dim3 grid((g.Vh + B / 2 - 1) / (B / 2));
    if (prec == 0)
        hipLaunchKernelGGL(k_sd_gfield<double>, grid, dim3(B), 0, st, g, (const double *)d,
                           (V2<double>::type *)gfield);
    else
        hipLaunchKernelGGL(k_sd_gfield<float>, grid, dim3(B), 0, st, g, (const float *)d,
                           (V2<float>::type *)gfield);
    return hipGetLastError();
}

}  // namespace gf
