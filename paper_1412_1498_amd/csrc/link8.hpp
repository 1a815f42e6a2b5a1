// link8.hpp -- 8-real storage of SU(3) links (the paper's most compressed
// link format): a link is kept as U01, U02, U10 (three complex numbers) and
// the phases of U00 and U20 (coded as below). Usable on host and device,
// so host-side checks run the very code the kernels run.
//
// Reconstruction, from unitarity and det U = 1 (U^dagger = adj U, i.e. each
// element is the complex conjugate of its cofactor):
//   n2  = |U01|^2 + |U02|^2            (= 1 - |U00|^2, row 0 is a unit vector)
//   U00 = sqrt(1 - n2) e^{i phase00}
//   U20 = sqrt(n2 - |U10|^2) e^{i phase20}   (column 0 is a unit vector)
//   U11 = -(conj(U00) U01 U10 + conj(U02) conj(U20)) / n2
//   U12 =  (conj(U01) conj(U20) - conj(U00) U02 U10) / n2
//   U21 = -conj(U00 U12 - U02 U10)
//   U22 =  conj(U00 U11 - U01 U10)
// The divisor is formed as |U01|^2 + |U02|^2 rather than 1 - |U00|^2: near
// the unit matrix numerator and divisor are then products of small numbers,
// held to full relative precision. What remains near 1 is that the stored
// reals fix an exact SU(3) matrix, so a link that is SU(3) only to O(u) (u
// the unit roundoff of the storage precision) is moved to it: a link eps
// away from 1 moves by about u/eps. For float storage this stays at the
// float rounding of the link itself (measured below 3e-6 down to 1e-6 from
// 1); in double it is 2e-9 at 1e-6 from 1. Where |U00| or |U20| is tiny, the
// square roots lose digits: errors of about u/|U00|, u/|U20|.
//
// Row 0 without off-diagonal part (U01 = U02 = 0 exactly, n2 = 0; the unit
// matrix is one): then |U00| = 1, so U10 = U20 = 0, and the divisor above
// vanishes. The lower 2x2 block B is unitary with det B = conj(U00), i.e.
// B = [[a, b], [-conj(U00) conj(b), conj(U00) conj(a)]] with |a|^2 + |b|^2
// = 1. The U10 slot, free in this case, then holds a = U11, and the phase
// code of U20 is replaced by that of b = U12 (|b| = sqrt(1 - |a|^2)); the
// decoder recognises the case by n2 = 0 and the link is held exactly like
// any other.
//
// The phases are not stored as angles but as a rational code of the unit
// complex number w = z/|z| (no trigonometry either way): with
// t = Im w / (1 + |Re w|) in [-1, 1] (the tangent of half the angle
// between w and the real axis on its side), the stored value is t if
// Re w >= 0, else 2 - t (t >= 0) or -2 - t (t < 0). Decoding: the branch is
// |p| > 1, t = copysign(2 - |p|, p) there, and |Re w| = (1 - t^2)/(1 + t^2),
// Im w = 2t/(1 + t^2). z = 0 is stored as 4 and decodes to 0, so an element
// that is exactly zero comes back exactly zero whatever rounding its
// modulus, a square root of a difference, suffers.
#pragma once

#include <hip/hip_runtime.h>

namespace gf {

#define GF_HD __host__ __device__ __forceinline__

// Reciprocal and square root. In float on the GPU these are the hardware
// instructions (about 1 ulp) rather than the correctly rounded sequences:
// the format's own rounding (a few ulp) dominates, and the exact sequences
// made the float 8-real sweep instruction-bound. Double and host code use
// the correctly rounded operations.
template <typename R> GF_HD R link8_rcp(R x) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_rcpf(x);
#endif
    return R(1) / x;
}
template <typename R> GF_HD R link8_sqrt(R x) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_sqrtf(x);
#endif
    return sqrt(x);
}

template <typename R>
GF_HD R link8_phase_code(R re, R im) {
    const R m = link8_sqrt<R>(re * re + im * im);
    if (!(m > R(0))) return R(4);  // z = 0: a code outside [-2, 2] that decodes to 0
    const R t = im * link8_rcp<R>(m + fabs(re));
    return re >= R(0) ? t : (t >= R(0) ? R(2) - t : R(-2) - t);
}

// unit complex number (c, s) of a phase code; (0, 0) for the code of 0
template <typename R>
GF_HD void link8_phase_decode(R p, R *c, R *s) {
    const bool zero = fabs(p) > R(3);
    const bool neg = fabs(p) > R(1);
    const R t = neg ? copysign(R(2) - fabs(p), p) : p;
    const R d = link8_rcp<R>(R(1) + t * t);
    const R ac = (R(1) - t * t) * d;
    *s = zero ? R(0) : R(2) * t * d;
    *c = zero ? R(0) : (neg ? -ac : ac);
}

// The four stored complex values of a 3x3 link (re[9], im[9], element (r, c)
// at 3r + c): U01, U02, U10, (phase code of U00, phase code of U20).
// When U01 = U02 = 0, the third value is U11 and the second phase code is
// that of U12 instead (see above).
template <typename R>
GF_HD void link8_compress(const R *re, const R *im, R *sre, R *sim) {
    const bool deg = re[1] == R(0) && im[1] == R(0) && re[2] == R(0) && im[2] == R(0);
    sre[0] = re[1]; sim[0] = im[1];
    sre[1] = re[2]; sim[1] = im[2];
    sre[2] = deg ? re[4] : re[3]; sim[2] = deg ? im[4] : im[3];
    sre[3] = link8_phase_code<R>(re[0], im[0]);
    sim[3] = deg ? link8_phase_code<R>(re[5], im[5]) : link8_phase_code<R>(re[6], im[6]);
}

template <typename R>
GF_HD void link8_reconstruct(const R *sre, const R *sim, R *re, R *im) {
    const R a2r = sre[0], a2i = sim[0], a3r = sre[1], a3i = sim[1];
    const R n2 = a2r * a2r + a2i * a2i + (a3r * a3r + a3i * a3i);
    const bool deg = !(n2 > R(0));        // U01 = U02 = 0: the slot holds U11
    const R sl = sre[2] * sre[2] + sim[2] * sim[2];
    const R b1r = deg ? R(0) : sre[2], b1i = deg ? R(0) : sim[2];
    R s, c;
    link8_phase_decode<R>(sre[3], &c, &s);
    const R m1 = link8_sqrt<R>(fmax(R(1) - n2, R(0)));
    const R a1r = m1 * c, a1i = m1 * s;
    link8_phase_decode<R>(sim[3], &c, &s);
    // |U20| in general; |U12| = sqrt(1 - |U11|^2) in the n2 = 0 case
    const R m3 = link8_sqrt<R>(fmax(deg ? R(1) - sl : n2 - sl, R(0)));
    const R zr = m3 * c, zi = m3 * s;
    const R c1r = deg ? R(0) : zr, c1i = deg ? R(0) : zi;
    // conj(a1) a2 b1, conj(a1) a3 b1
    const R pr = a1r * a2r + a1i * a2i, pi = a1r * a2i - a1i * a2r;   // conj(a1) a2
    const R qr = a1r * a3r + a1i * a3i, qi = a1r * a3i - a1i * a3r;   // conj(a1) a3
    const R t1r = pr * b1r - pi * b1i, t1i = pr * b1i + pi * b1r;
    const R t2r = qr * b1r - qi * b1i, t2i = qr * b1i + qi * b1r;
    // conj(a3) conj(c1) = conj(a3 c1), conj(a2) conj(c1) = conj(a2 c1)
    const R u3r = a3r * c1r - a3i * c1i, u3i = -(a3r * c1i + a3i * c1r);
    const R u2r = a2r * c1r - a2i * c1i, u2i = -(a2r * c1i + a2i * c1r);
    R b2r, b2i, b3r, b3i;
    if (n2 > R(0)) {
        const R inv = link8_rcp<R>(n2);
        b2r = -(t1r + u3r) * inv; b2i = -(t1i + u3i) * inv;
        b3r = (u2r - t2r) * inv;  b3i = (u2i - t2i) * inv;
    } else {  // U01 = U02 = 0: U11 from the slot, U12 from its phase code and modulus
        b2r = sre[2]; b2i = sim[2];
        b3r = zr; b3i = zi;
    }
    // c2 = -conj(a1 b3 - a3 b1), c3 = conj(a1 b2 - a2 b1)
    const R x2r = a1r * b3r - a1i * b3i - (a3r * b1r - a3i * b1i);
    const R x2i = a1r * b3i + a1i * b3r - (a3r * b1i + a3i * b1r);
    const R x3r = a1r * b2r - a1i * b2i - (a2r * b1r - a2i * b1i);
    const R x3i = a1r * b2i + a1i * b2r - (a2r * b1i + a2i * b1r);
    re[0] = a1r; im[0] = a1i;
    re[1] = a2r; im[1] = a2i;
    re[2] = a3r; im[2] = a3i;
    re[3] = b1r; im[3] = b1i;
    re[4] = b2r; im[4] = b2i;
    re[5] = b3r; im[5] = b3i;
    re[6] = c1r; im[6] = c1i;
    re[7] = -x2r; im[7] = x2i;
    re[8] = x3r; im[8] = -x3i;
}

#undef GF_HD

}  // namespace gf
