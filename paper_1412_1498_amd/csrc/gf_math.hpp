// gf_math.hpp -- double-precision sine/cosine and arctangent for the bounded
// arguments of the SU(2) over-relaxation step, written to keep the register
// footprint of the sweep kernel small. Usable on host and device so the
// host-side checks exercise the very code the kernels run.
//
// sincos: argument in [0, 2 pi]. Quadrant reduction x = k pi/2 + r (k =
//   rint(2x/pi), r in [-pi/4, pi/4]) with pi/2 split into a double head and
//   a tail (Cody and Waite's method), each subtracted with one fused
//   multiply-add; then the Taylor series of sin r (to r^17) and cos r (to
//   r^18), whose first neglected terms are below 1e-19.
// atan2: octant reduction to t = min/max in [0, 1]; for t > tan(pi/8) the
//   identity atan t = pi/4 + atan((t - 1)/(t + 1)) brings the argument into
//   |u| <= tan(pi/8); there the alternating Taylor series of atan u is summed
//   to u^39 (first neglected term below 2^-53 |u|).
#pragma once

#include <hip/hip_runtime.h>

namespace gf {

#define GF_HD __host__ __device__ __forceinline__

constexpr double GF_PI = 3.141592653589793;         // pi rounded to double
constexpr double GF_PI_2 = 1.5707963267948966;      // pi/2 rounded to double
constexpr double GF_PI_2_TAIL = 6.123233995736766e-17;  // pi/2 - GF_PI_2
constexpr double GF_PI_4 = 0.7853981633974483;
constexpr double GF_2_PI = 0.6366197723675814;      // 2/pi
constexpr double GF_TAN_PI_8 = 0.41421356237309515; // sqrt(2) - 1

GF_HD void gf_sincos(double x, double *s, double *c) {
    const double k = rint(x * GF_2_PI);
    double r = fma(-k, GF_PI_2, x);
    r = fma(-k, GF_PI_2_TAIL, r);
    const double r2 = r * r;
    // sin r = r (1 - r^2/3! + r^4/5! - ... + r^16/17!)
    double ps = 1.0 / 355687428096000.0;        // 1/17!
    ps = fma(ps, r2, -1.0 / 1307674368000.0);   // 1/15!
    ps = fma(ps, r2, 1.0 / 6227020800.0);       // 1/13!
    ps = fma(ps, r2, -1.0 / 39916800.0);        // 1/11!
    ps = fma(ps, r2, 1.0 / 362880.0);           // 1/9!
    ps = fma(ps, r2, -1.0 / 5040.0);            // 1/7!
    ps = fma(ps, r2, 1.0 / 120.0);              // 1/5!
    ps = fma(ps, r2, -1.0 / 6.0);               // 1/3!
    const double sr = fma(ps * r2, r, r);
    // cos r = 1 - r^2/2! + r^4/4! - ... + r^18/18!
    double pc = 1.0 / 6402373705728000.0;       // 1/18!
    pc = fma(pc, r2, -1.0 / 20922789888000.0);  // 1/16!
    pc = fma(pc, r2, 1.0 / 87178291200.0);      // 1/14!
    pc = fma(pc, r2, -1.0 / 479001600.0);       // 1/12!
    pc = fma(pc, r2, 1.0 / 3628800.0);          // 1/10!
    pc = fma(pc, r2, -1.0 / 40320.0);           // 1/8!
    pc = fma(pc, r2, 1.0 / 720.0);              // 1/6!
    pc = fma(pc, r2, -1.0 / 24.0);              // 1/4!
    pc = fma(pc, r2, 0.5);
    const double cr = fma(-pc, r2, 1.0);
    const int q = ((int)k) & 3;
    const double sv = (q & 1) ? cr : sr;
    const double cv = (q & 1) ? sr : cr;
    *s = (q & 2) ? -sv : sv;
    *c = ((q + 1) & 2) ? -cv : cv;
}

// atan u for |u| <= tan(pi/8): u - u^3/3 + u^5/5 - ... - u^39/39.
GF_HD double gf_atan_small(double u) {
    const double u2 = u * u;
    double p = -1.0 / 39.0;
    p = fma(p, u2, 1.0 / 37.0);
    p = fma(p, u2, -1.0 / 35.0);
    p = fma(p, u2, 1.0 / 33.0);
    p = fma(p, u2, -1.0 / 31.0);
    p = fma(p, u2, 1.0 / 29.0);
    p = fma(p, u2, -1.0 / 27.0);
    p = fma(p, u2, 1.0 / 25.0);
    p = fma(p, u2, -1.0 / 23.0);
    p = fma(p, u2, 1.0 / 21.0);
    p = fma(p, u2, -1.0 / 19.0);
    p = fma(p, u2, 1.0 / 17.0);
    p = fma(p, u2, -1.0 / 15.0);
    p = fma(p, u2, 1.0 / 13.0);
    p = fma(p, u2, -1.0 / 11.0);
    p = fma(p, u2, 1.0 / 9.0);
    p = fma(p, u2, -1.0 / 7.0);
    p = fma(p, u2, 1.0 / 5.0);
    p = fma(p, u2, -1.0 / 3.0);
    return fma(p * u2, u, u);
}

// atan2(y, x) in (-pi, pi]; atan2(0, 0) = 0.
GF_HD double gf_atan2(double y, double x) {
    const double ax = fabs(x), ay = fabs(y);
    const double mx = fmax(ax, ay), mn = fmin(ax, ay);
    const double t = mx > 0.0 ? mn / mx : 0.0;
    const bool big = t > GF_TAN_PI_8;
    const double u = big ? (t - 1.0) / (t + 1.0) : t;
    double a = gf_atan_small(u) + (big ? GF_PI_4 : 0.0);
    a = ay > ax ? GF_PI_2 - a : a;
    a = x < 0.0 ? GF_PI - a : a;
    return y < 0.0 ? -a : a;
}

// Local SU(2) maximiser of Re Tr[g k] for a 2x2 block whose quaternion part
// is b = (b0, b1, b2, b3), i.e. eq. (6) g = q^dagger / |q|, raised to the
// exact principal power omega. With g = (cos phi, n sin phi),
// phi = atan2(|b_vec|, b0) in [0, pi], n = -b_vec / |b_vec|:
// g^omega = (cos(omega phi), n sin(omega phi)). A zero block gives g = 1;
// g = -1 (b_vec = 0, b0 < 0) turns about the third axis.
GF_HD void gf_su2_overrelax(const double b[4], double omega, double r[4]) {
    const double vn = sqrt(b[1] * b[1] + b[2] * b[2] + b[3] * b[3]);
    const double phi = gf_atan2(vn, b[0]);
    double s, c;
    gf_sincos(omega * phi, &s, &c);
    const bool deg = !(vn > 0.0);
    const double f = deg ? 0.0 : s / vn;
    r[0] = c;
    r[1] = -b[1] * f;
    r[2] = -b[2] * f;
    r[3] = deg ? s : -b[3] * f;
}

#undef GF_HD

}  // namespace gf
