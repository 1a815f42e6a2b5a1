// sun_device.hpp -- register-level SU(N) helpers (N = 2, 4) for the general
// number of colours: N x N links in the blocked layout (N*N complex elements
// per link, element (r, c) at index N r + c), and reunitarisation.
#pragma once

#include "su3_device.hpp"

namespace gf {

template <typename R, int N> struct MatN {
    R re[N * N], im[N * N];
};

template <int N> struct DMN {
    double re[N * N], im[N * N];
};

template <typename R, int N, bool NT>
__device__ __forceinline__ void load_link_n(MatN<R, N> &m, const gchar *base, long long off) {
    typedef typename V2<R>::type v2;
    const gchar *p = base + off * (long long)sizeof(v2);
#pragma unroll
    for (int e = 0; e < N * N; e++) {
        v2 v = ld<NT, v2>(p, (uint32_t)(e * BLK * sizeof(v2)));
        m.re[e] = v.x;
        m.im[e] = v.y;
    }
}

template <typename R, int N, bool NT>
__device__ __forceinline__ void store_link_n(const MatN<R, N> &m, gchar *base, long long off) {
    typedef typename V2<R>::type v2;
    gchar *p = base + off * (long long)sizeof(v2);
#pragma unroll
    for (int e = 0; e < N * N; e++) {
        R x = m.re[e], y = m.im[e];
        asm("" : "+v"(x), "+v"(y));  // as in store_link: keeps m in registers
        v2 v;
        v.x = x;
        v.y = y;
        st<NT, v2>(p, (uint32_t)(e * BLK * sizeof(v2)), v);
    }
}

// Determinant of the 3x3 complex matrix formed by rows 0..2 of the double
// matrix (re, im) (row stride 4) at columns c0, c1, c2.
__device__ __forceinline__ void det3_cols(const double *re, const double *im, int c0, int c1, int c2,
                                          double &dr, double &di) {
    // minors of row 0 along the chosen columns
    auto mul = [](double ar, double ai, double br, double bi, double &xr, double &xi) {
        xr = ar * br - ai * bi;
        xi = ar * bi + ai * br;
    };
    double m0r, m0i, m1r, m1i, m2r, m2i, tr, ti;
    mul(re[4 + c1], im[4 + c1], re[8 + c2], im[8 + c2], m0r, m0i);
    mul(re[4 + c2], im[4 + c2], re[8 + c1], im[8 + c1], tr, ti);
    m0r -= tr; m0i -= ti;
    mul(re[4 + c0], im[4 + c0], re[8 + c2], im[8 + c2], m1r, m1i);
    mul(re[4 + c2], im[4 + c2], re[8 + c0], im[8 + c0], tr, ti);
    m1r -= tr; m1i -= ti;
    mul(re[4 + c0], im[4 + c0], re[8 + c1], im[8 + c1], m2r, m2i);
    mul(re[4 + c1], im[4 + c1], re[8 + c0], im[8 + c0], tr, ti);
    m2r -= tr; m2i -= ti;
    double ar, ai, br, bi, cr, ci;
    mul(re[c0], im[c0], m0r, m0i, ar, ai);
    mul(re[c1], im[c1], m1r, m1i, br, bi);
    mul(re[c2], im[c2], m2r, m2i, cr, ci);
    dr = ar - br + cr;
    di = ai - bi + ci;
}

// Reunitarise in double: Gram-Schmidt of rows 0..N-2, last row the complex
// conjugate of its cofactors (the unique unit row completing an SU(N)
// matrix, since U^dagger = adj U when det U = 1).
template <typename R, int N>
__device__ __forceinline__ void reunitarise_n(MatN<R, N> &m) {
    double re[N * N], im[N * N];
#pragma unroll
    for (int e = 0; e < N * N; e++) { re[e] = (double)m.re[e]; im[e] = (double)m.im[e]; }
#pragma unroll
    for (int r = 0; r < N - 1; r++) {
#pragma unroll
        for (int q = 0; q < r; q++) {
            double pr = 0.0, pi = 0.0;  // <row q, row r>
#pragma unroll
            for (int j = 0; j < N; j++) {
                pr += re[q * N + j] * re[r * N + j] + im[q * N + j] * im[r * N + j];
                pi += re[q * N + j] * im[r * N + j] - im[q * N + j] * re[r * N + j];
            }
#pragma unroll
            for (int j = 0; j < N; j++) {
                const double xr = re[q * N + j], xi = im[q * N + j];
                re[r * N + j] -= pr * xr - pi * xi;
                im[r * N + j] -= pr * xi + pi * xr;
            }
        }
        double nn = 0.0;
#pragma unroll
        for (int j = 0; j < N; j++) nn += re[r * N + j] * re[r * N + j] + im[r * N + j] * im[r * N + j];
        const double inv = 1.0 / sqrt(nn);
#pragma unroll
        for (int j = 0; j < N; j++) { re[r * N + j] *= inv; im[r * N + j] *= inv; }
    }
    if constexpr (N == 2) {
        // cofactors: C10 = -u01, C11 = u00
        re[2] = -re[1]; im[2] = im[1];
        re[3] = re[0];  im[3] = -im[0];
    } else {
        static_assert(N == 4, "SU(N) kernels are built for N = 2 and 4");
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int c0 = j == 0 ? 1 : 0, c1 = j <= 1 ? 2 : 1, c2 = j <= 2 ? 3 : 2;
            double dr, di;
            det3_cols(re, im, c0, c1, c2, dr, di);
            const double s = (j & 1) ? 1.0 : -1.0;  // (-1)^(3 + j)
            re[12 + j] = s * dr;
            im[12 + j] = -s * di;
        }
    }
#pragma unroll
    for (int e = 0; e < N * N; e++) { m.re[e] = (R)re[e]; m.im[e] = (R)im[e]; }
}

}  // namespace gf
