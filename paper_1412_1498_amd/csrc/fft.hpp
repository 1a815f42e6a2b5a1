// fft.hpp -- the lattice Fourier transforms of Alg. 2 (fft.hip), as seen by
// the host code that plans and launches them.
#pragma once

#include "gf_internal.hpp"

namespace gf {

// Lattice Fourier transforms of Alg. 2 (fft.hip). Spectrum of the eight
// components spec[t][a][z][y][kx], kx = 0..nx/2. A workgroup transforms a tile
// of at most FFT_TILE_POINTS complex points in LDS (in place, in double, with
// the roots: <= 40 KB), so an axis may be at most FFT_MAX_N long (whose
// radices take at most FFT_MAX_PASSES passes).
constexpr int FFT_BLOCK = 256;
constexpr int FFT_TILE_POINTS = 1536;
constexpr int FFT_MAX_N = 1024;
// Along x a tile holds the eight components of whole site rows (four complex
// pencils per row), so nx is at most FFT_TILE_POINTS / 4.
constexpr int FFT_MAX_NX = FFT_TILE_POINTS / 4;

// Division by a small divisor d as a multiply-high: floor(n / d) =
// (n * ceil(2^32 / d)) >> 32 exactly for n, d < 2^16 (d = 1 kept apart).
struct FastDiv {
    unsigned d, m;
};

inline FastDiv make_fastdiv(unsigned d) {
    FastDiv f;
    f.d = d;
    f.m = d > 1 ? (unsigned)((0x100000000ULL + d - 1) / d) : 0u;
    return f;
}

__device__ __forceinline__ unsigned fdiv(unsigned n, const FastDiv &f) { return f.d == 1 ? n : __umulhi(n, f.m); }

constexpr int FFT_MAX_PASSES = 12;
struct FftPlan {     // radices of the Stockham passes, in order
    int nf;
    int fac[FFT_MAX_PASSES];
    FastDiv ns[FFT_MAX_PASSES];  // division by Ns = product of the earlier radices
};

struct FftSite {      // Delta and the real <-> half-complex transform along x, by site rows
    int n;            // nx
    FftPlan pl;
    int nkx;          // nx / 2 + 1
    int ys;           // site rows (lines along x) per workgroup: 4 ys complex pencils
    long long srows;  // nt * nz * ny
    FastDiv dn, dnkx, dnc;  // division by nx, nkx and 4 ys
};

struct FftAxis {     // complex, in place, along y, z or t
    int n;           // axis length
    FftPlan pl;
    int np, nkx, nchunk;  // kx per workgroup, kx count, kx chunks per row
    long long s_ax;  // spectrum stride along the axis
    int r[3];        // the other three of (t, a, z, y): extents ...
    long long s[3];  // ... and strides
    int Lx, Lax, L[3];    // lattice lengths entering p^2 (0: not a transformed direction)
    double scale, p2max;  // filter factor scale * p2max / p^2(k)
    FastDiv dnp;          // division by np
};

FftSite make_fft_site(const Geom &g);
FftAxis make_fft_axis(const Geom &g, int axis, bool coulomb);  // axis 1 = y, 2 = z, 3 = t
// W: a table of exp(2 pi i m / n), m < n, for the transform's length (launch_fft_roots fills it)
hipError_t launch_fft_roots(void *W, int n, hipStream_t st);
// Delta (eq. 3) of every site -> its components' x-transformed half spectrum
hipError_t launch_sd_delta_fx(int prec, int nelem, int gauge, const Geom &g, const FftSite &f, const void *W,
                              const void *U, void *spec, hipStream_t st);
// half spectrum -> inverse x transform -> g = reunit(1 + X) as the g field (gfield_off)
hipError_t launch_sd_fx_gfield(int prec, const Geom &g, const FftSite &f, const void *W, const void *spec,
                               void *gfield, hipStream_t st);
hipError_t launch_fft_axis(int prec, const FftAxis &f, const void *W, void *spec, int sign, int filter,
                           hipStream_t st);

}  // namespace gf
