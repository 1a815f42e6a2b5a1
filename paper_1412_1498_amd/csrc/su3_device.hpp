// su3_device.hpp -- register-level SU(3)/SU(2) arithmetic for the gfx950
// kernels of libgf: link loads/stores in the even/odd element-major layout,
// the SU(2) subgroup solve with exact over-relaxation, row rotations, and
// Gram-Schmidt reunitarisation.
#pragma once

#include <hip/hip_runtime.h>

#include "gf_internal.hpp"
#include "gf_math.hpp"
#include "link8.hpp"

namespace gf {

template <typename R> struct V2;
template <> struct V2<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct V2<double> { typedef double type __attribute__((ext_vector_type(2))); };

// Global-address-space views: a uniform (scalar) base pointer plus a 32-bit
// per-lane byte offset lets the compiler emit global_load/store with an SGPR
// base instead of 64-bit flat addresses per lane.
typedef __attribute__((address_space(1))) char gchar;

template <bool NT, typename T>
__device__ __forceinline__ T ld(const gchar *base, uint32_t byte_off) {
    const __attribute__((address_space(1))) T *p =
        reinterpret_cast<const __attribute__((address_space(1))) T *>(base + byte_off);
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool NT, typename T>
__device__ __forceinline__ void st(gchar *base, uint32_t byte_off, T v) {
    __attribute__((address_space(1))) T *p =
        reinterpret_cast<__attribute__((address_space(1))) T *>(base + byte_off);
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

__device__ __forceinline__ gchar *as_global(void *p) { return (gchar *)p; }
__device__ __forceinline__ const gchar *as_global(const void *p) { return (const gchar *)p; }

// A 3x3 complex matrix held in registers as separate real/imaginary parts,
// element (r, c) at index 3r + c.
template <typename R> struct Mat {
    R re[9], im[9];
};

// Rebuild row 2 of a special unitary matrix from rows 0 and 1:
// row2 = conj(row0 x row1).
template <typename R>
__device__ __forceinline__ void rebuild_row2(Mat<R> &m) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        // (row0 x row1)_c = r0[c1] r1[c2] - r0[c2] r1[c1]
        R xr = fma(m.re[c1], m.re[3 + c2], -m.im[c1] * m.im[3 + c2]);
        xr = fma(-m.re[c2], m.re[3 + c1], fma(m.im[c2], m.im[3 + c1], xr));
        R xi = fma(m.re[c1], m.im[3 + c2], m.im[c1] * m.re[3 + c2]);
        xi = fma(-m.re[c2], m.im[3 + c1], fma(-m.im[c2], m.re[3 + c1], xi));
        m.re[6 + c] = xr;
        m.im[6 + c] = -xi;
    }
}

// Link whose element 0 sits at complex offset `off` (see link_off); element
// e is BLK complex values further. NE = 9: full matrix; NE = 6: rows 0, 1;
// NE = 4: the 8-real form of link8.hpp.
template <typename R, int NE, bool NT>
__device__ __forceinline__ void load_link(Mat<R> &m, const gchar *base, long long off) {
    typedef typename V2<R>::type v2;
    const gchar *p = base + off * (long long)sizeof(v2);
    if constexpr (NE == 4) {
        R sre[4], sim[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            v2 v = ld<NT, v2>(p, (uint32_t)(e * BLK * sizeof(v2)));
            sre[e] = v.x;
            sim[e] = v.y;
        }
        link8_reconstruct<R>(sre, sim, m.re, m.im);
    } else {
#pragma unroll
        for (int e = 0; e < NE; e++) {
            v2 v = ld<NT, v2>(p, (uint32_t)(e * BLK * sizeof(v2)));
            m.re[e] = v.x;
            m.im[e] = v.y;
        }
        if constexpr (NE == 6) rebuild_row2(m);
    }
}

template <typename R, int NE, bool NT>
__device__ __forceinline__ void store_link(const Mat<R> &m, gchar *base, long long off) {
    typedef typename V2<R>::type v2;
    gchar *p = base + off * (long long)sizeof(v2);
    if constexpr (NE == 4) {
        R sre[4], sim[4];
        link8_compress<R>(m.re, m.im, sre, sim);
#pragma unroll
        for (int e = 0; e < 4; e++) {
            v2 v;
            v.x = sre[e];
            v.y = sim[e];
            st<NT, v2>(p, (uint32_t)(e * BLK * sizeof(v2)), v);
        }
    } else {
#pragma unroll
        for (int e = 0; e < NE; e++) {
            R x = m.re[e], y = m.im[e];
            // keep the pair as two register values: otherwise the compiler may
            // fetch re[e] together with its neighbour re[e + 1] as one 8-byte
            // load, which keeps m in memory (LDS) instead of registers
            asm("" : "+v"(x), "+v"(y));
            v2 v;
            v.x = x;
            v.y = y;
            st<NT, v2>(p, (uint32_t)(e * BLK * sizeof(v2)), v);
        }
    }
}

// m <- m^dagger when `flip` (a per-lane flag), else unchanged.
template <typename R>
__device__ __forceinline__ void dagger_if(Mat<R> &m, bool flip) {
#pragma unroll
    for (int r = 0; r < 3; r++) {
#pragma unroll
        for (int c = r; c < 3; c++) {
            const int a = 3 * r + c, b = 3 * c + r;
            R ar = m.re[a], ai = m.im[a], br = m.re[b], bi = m.im[b];
            m.re[a] = flip ? br : ar;
            m.im[a] = flip ? -bi : ai;
            m.re[b] = flip ? ar : br;
            m.im[b] = flip ? -ai : bi;
        }
    }
}

// Quaternion part of the (a, b) block of m, times 2:
//   t0 = Re(m_aa + m_bb), t1 = Im(m_ab + m_ba), t2 = Re(m_ab - m_ba), t3 = Im(m_aa - m_bb)
template <typename R>
__device__ __forceinline__ void block_quat2(const Mat<R> &m, int a, int b, double t[4]) {
    const int aa = 4 * a, bb = 4 * b, ab = 3 * a + b, ba = 3 * b + a;
    t[0] = (double)m.re[aa] + (double)m.re[bb];
    t[1] = (double)m.im[ab] + (double)m.im[ba];
    t[2] = (double)m.re[ab] - (double)m.re[ba];
    t[3] = (double)m.im[aa] - (double)m.im[bb];
}

// Rows a, b of m <- G (rows a, b of m), G = [[g0 + i g3, g2 + i g1],
// [-g2 + i g1, g0 - i g3]] given in the link precision.
template <typename R>
__device__ __forceinline__ void rotate_rows(Mat<R> &m, int a, int b, const R g[4]) {
    const R ar = g[0], ai = g[3];   // alpha
    const R br = g[2], bi = g[1];   // beta
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const R xr = m.re[3 * a + c], xi = m.im[3 * a + c];
        const R yr = m.re[3 * b + c], yi = m.im[3 * b + c];
        // row a: alpha x + beta y
        m.re[3 * a + c] = fma(ar, xr, fma(-ai, xi, fma(br, yr, -bi * yi)));
        m.im[3 * a + c] = fma(ar, xi, fma(ai, xr, fma(br, yi, bi * yr)));
        // row b: -conj(beta) x + conj(alpha) y
        m.re[3 * b + c] = fma(-br, xr, fma(-bi, xi, fma(ar, yr, ai * yi)));
        m.im[3 * b + c] = fma(-br, xi, fma(bi, xr, fma(ar, yi, -ai * yr)));
    }
}

// Gram-Schmidt reunitarisation in double: r0 /= |r0|; r1 -= (r0^+ r1) r0;
// r1 /= |r1|; r2 = conj(r0 x r1). Result rounded to the link precision.
template <typename R>
__device__ __forceinline__ void reunitarise(Mat<R> &m) {
    double r0r[3], r0i[3], r1r[3], r1i[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        r0r[c] = m.re[c]; r0i[c] = m.im[c];
        r1r[c] = m.re[3 + c]; r1i[c] = m.im[3 + c];
    }
    double n0 = sqrt(r0r[0] * r0r[0] + r0i[0] * r0i[0] + r0r[1] * r0r[1] + r0i[1] * r0i[1] +
                     r0r[2] * r0r[2] + r0i[2] * r0i[2]);
#pragma unroll
    for (int c = 0; c < 3; c++) { r0r[c] /= n0; r0i[c] /= n0; }
    double pr = 0.0, pi = 0.0;  // r0^+ r1
#pragma unroll
    for (int c = 0; c < 3; c++) {
        pr += r0r[c] * r1r[c] + r0i[c] * r1i[c];
        pi += r0r[c] * r1i[c] - r0i[c] * r1r[c];
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
        r1r[c] -= pr * r0r[c] - pi * r0i[c];
        r1i[c] -= pr * r0i[c] + pi * r0r[c];
    }
    double n1 = sqrt(r1r[0] * r1r[0] + r1i[0] * r1i[0] + r1r[1] * r1r[1] + r1i[1] * r1i[1] +
                     r1r[2] * r1r[2] + r1i[2] * r1i[2]);
#pragma unroll
    for (int c = 0; c < 3; c++) { r1r[c] /= n1; r1i[c] /= n1; }
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        double xr = r0r[c1] * r1r[c2] - r0i[c1] * r1i[c2] - (r0r[c2] * r1r[c1] - r0i[c2] * r1i[c1]);
        double xi = r0r[c1] * r1i[c2] + r0i[c1] * r1r[c2] - (r0r[c2] * r1i[c1] + r0i[c2] * r1r[c1]);
        m.re[6 + c] = (R)xr;
        m.im[6 + c] = (R)(-xi);
        m.re[c] = (R)r0r[c]; m.im[c] = (R)r0i[c];
        m.re[3 + c] = (R)r1r[c]; m.im[3 + c] = (R)r1i[c];
    }
}

// Binary-tree sum s[0..N) as ((s0 + s1) + (s2 + s3)) + ...
template <int N>
__device__ __forceinline__ double tree_sum(const double *s) {
    if constexpr (N == 1) return s[0];
    else return tree_sum<N / 2>(s) + tree_sum<N / 2>(s + N / 2);
}

__device__ __forceinline__ int pick4(const int v[4], int i) {
    return i == 0 ? v[0] : (i == 1 ? v[1] : (i == 2 ? v[2] : v[3]));
}

}  // namespace gf
