// layout.hip -- conversion between the canonical [t][z][y][x][mu][r][c]
// link layout and the even/odd, element-major layout of the kernels
// (section "Implementation"), the same for algebra fields [t][z][y][x][a] <->
// [a][p][h], and standalone reunitarisation.
#include "su3_device.hpp"

namespace gf {

// One lane per (site, mu) link.
template <typename R, int NE>
__global__ void __launch_bounds__(256) k_pack(Geom g, const typename V2<R>::type *__restrict__ aos,
                       typename V2<R>::type *__restrict__ U, int unpack) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 4LL * g.V) return;
    const int s = (int)(idx >> 2), mu = (int)(idx & 3);
    const int x = s % g.nx;
    const int y = (s / g.nx) % g.ny;
    const int z = (s / (g.nx * g.ny)) % g.nz;
    const int t = s / (g.nx * g.ny * g.nz);
    int p, h;
    site_to_ph(g, x, y, z, t, p, h);
    const long long off = link_off(g, mu, p, h);
    const typename V2<R>::type *src = aos + idx * 9;
    typename V2<R>::type *dst = const_cast<typename V2<R>::type *>(aos) + idx * 9;
    if (!unpack) {
        Mat<R> m;
#pragma unroll
        for (int e = 0; e < 9; e++) {
            m.re[e] = src[e].x;
            m.im[e] = src[e].y;
        }
        store_link<R, NE, false>(m, as_global((void *)U), off);
    } else {
        Mat<R> m;
        load_link<R, NE, false>(m, as_global((const void *)U), off);
#pragma unroll
        for (int e = 0; e < 9; e++) {
            typename V2<R>::type v;
            v.x = m.re[e];
            v.y = m.im[e];
            dst[e] = v;
        }
    }
}

// One lane per (mu, site) link.
template <typename R, int NE>
__global__ void __launch_bounds__(256) k_reunit(Geom g, typename V2<R>::type *__restrict__ U) {
    const long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= 4LL * g.V) return;
    const int mu = (int)(l / g.V);
    const int n = (int)(l - (long long)mu * g.V);
    const int p = n >= g.Vh, h = n - p * g.Vh;
    const long long off = link_off(g, mu, p, h);
    Mat<R> m;
    load_link<R, NE, false>(m, as_global((const void *)U), off);
    reunitarise(m);
    store_link<R, NE, false>(m, as_global((void *)U), off);
}

// One lane per site: canonical s[site][a] <-> internal s[a][p][h].
template <typename R>
__global__ void __launch_bounds__(256) k_pack_alg(Geom g, const R *__restrict__ aos, R *__restrict__ s, int unpack) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.V) return;
    const int x = n % g.nx;
    const int y = (n / g.nx) % g.ny;
    const int z = (n / (g.nx * g.ny)) % g.nz;
    const int t = n / (g.nx * g.ny * g.nz);
    int p, h;
    site_to_ph(g, x, y, z, t, p, h);
    const long long off = alg_off(g, p, h, 0);
    R *a = const_cast<R *>(aos) + 8LL * n;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        if (!unpack) s[off + (long long)k * BLK] = a[k];
        else a[k] = s[off + (long long)k * BLK];
    }
}

hipError_t launch_pack(int prec, int nelem, const Geom &g, const void *aos, void *U, int unpack,
                       hipStream_t st) {
    const long long n = 4LL * g.V;
    const int B = 256;
    const dim3 grid((unsigned)((n + B - 1) / B));
#define GF_L(R, NE)                                                                              \
    hipLaunchKernelGGL((k_pack<R, NE>), grid, dim3(B), 0, st, g,                                 \
                       (const typename V2<R>::type *)aos, (typename V2<R>::type *)U, unpack)
    if (prec == 0) { if (nelem == 9) GF_L(double, 9); else if (nelem == 6) GF_L(double, 6); else GF_L(double, 4); }
    else { if (nelem == 9) GF_L(float, 9); else if (nelem == 6) GF_L(float, 6); else GF_L(float, 4); }
#undef GF_L
    return hipGetLastError();
}

hipError_t launch_reunit(int prec, int nelem, const Geom &g, void *U, hipStream_t st) {
    const long long n = 4LL * g.V;
    const int B = 256;
    const dim3 grid((unsigned)((n + B - 1) / B));
#define GF_L(R, NE) \
    hipLaunchKernelGGL((k_reunit<R, NE>), grid, dim3(B), 0, st, g, (typename V2<R>::type *)U)
    if (prec == 0) { if (nelem == 9) GF_L(double, 9); else if (nelem == 6) GF_L(double, 6); else GF_L(double, 4); }
    else { if (nelem == 9) GF_L(float, 9); else if (nelem == 6) GF_L(float, 6); else GF_L(float, 4); }
#undef GF_L
    return hipGetLastError();
}

hipError_t launch_pack_alg(int prec, const Geom &g, const void *aos, void *s, int unpack,
                           hipStream_t st) {
    const int B = 256;
    const dim3 grid((unsigned)((g.V + B - 1) / B));
    if (prec == 0)
        hipLaunchKernelGGL(k_pack_alg<double>, grid, dim3(B), 0, st, g, (const double *)aos,
                           (double *)s, unpack);
    else
        hipLaunchKernelGGL(k_pack_alg<float>, grid, dim3(B), 0, st, g, (const float *)aos,
                           (float *)s, unpack);
    return hipGetLastError();
}

}  // namespace gf
