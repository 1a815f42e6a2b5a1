// dmat.hpp -- 3x3 complex matrices in double for the kernels that apply a
// gauge transformation (grad.hip): products as FMA chains, loads of links and
// of the g field, and the rotation U -> g(x) U g(y)^dagger.
#pragma once

#include "su3_device.hpp"

namespace gf {

struct DMat {
    double re[9], im[9];
};

// 3x3 complex products in double, each element an FMA chain (4 per complex
// multiply-add).
__device__ __forceinline__ void dm_mul(const DMat &a, const DMat &b, DMat &c) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            double r = a.re[3 * i] * b.re[j], m = a.re[3 * i] * b.im[j];
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

// a * b^dagger
__device__ __forceinline__ void dm_mul_nd(const DMat &a, const DMat &b, DMat &c) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            double r = a.re[3 * i] * b.re[3 * j], m = a.im[3 * i] * b.re[3 * j];
            r = fma(a.im[3 * i], b.im[3 * j], r);
            m = fma(-a.re[3 * i], b.im[3 * j], m);
#pragma unroll
            for (int k = 1; k < 3; k++) {
                r = fma(a.re[3 * i + k], b.re[3 * j + k], r);
                r = fma(a.im[3 * i + k], b.im[3 * j + k], r);
                m = fma(a.im[3 * i + k], b.re[3 * j + k], m);
                m = fma(-a.re[3 * i + k], b.im[3 * j + k], m);
            }
            c.re[3 * i + j] = r;
            c.im[3 * i + j] = m;
        }
}

// a^dagger * b^dagger: element (i, j) = sum_k conj(a_ki) conj(b_jk)
__device__ __forceinline__ void dm_mul_dd(const DMat &a, const DMat &b, DMat &c) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            double r = a.re[i] * b.re[3 * j], m = -a.re[i] * b.im[3 * j];
            r = fma(-a.im[i], b.im[3 * j], r);
            m = fma(-a.im[i], b.re[3 * j], m);
#pragma unroll
            for (int k = 1; k < 3; k++) {
                r = fma(a.re[3 * k + i], b.re[3 * j + k], r);
                r = fma(-a.im[3 * k + i], b.im[3 * j + k], r);
                m = fma(-a.re[3 * k + i], b.im[3 * j + k], m);
                m = fma(-a.im[3 * k + i], b.re[3 * j + k], m);
            }
            c.re[3 * i + j] = r;
            c.im[3 * i + j] = m;
        }
}

// g(x) of site (p, h) from the g field (layout gfield_off).
template <typename R>
__device__ __forceinline__ void load_g(const typename V2<R>::type *__restrict__ gf, const Geom &g, int p, int h,
                                       DMat &m) {
    const long long o = gfield_off(g, p, h, 0);
#pragma unroll
    for (int e = 0; e < 9; e++) {
        typename V2<R>::type v = gf[o + (long long)e * BLK];
        m.re[e] = v.x;
        m.im[e] = v.y;
    }
}

template <typename R, int NE, bool NT = false>
__device__ __forceinline__ void load_u(const typename V2<R>::type *__restrict__ U, long long off, DMat &m) {
    Mat<R> t;
    load_link<R, NE, NT>(t, as_global((const void *)U), off);
#pragma unroll
    for (int e = 0; e < 9; e++) { m.re[e] = t.re[e]; m.im[e] = t.im[e]; }
}

// r = (gx u) gy^dagger in double, rounded to the link precision.
template <typename R>
__device__ __forceinline__ void gauge_rotate(const DMat &gx, const DMat &u, const DMat &gy, Mat<R> &m) {
    DMat t, r;
    dm_mul(gx, u, t);
    dm_mul_nd(t, gy, r);
#pragma unroll
    for (int e = 0; e < 9; e++) { m.re[e] = (R)r.re[e]; m.im[e] = (R)r.im[e]; }
}

}  // namespace gf
