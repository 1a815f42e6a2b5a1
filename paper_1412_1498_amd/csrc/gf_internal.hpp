// gf_internal.hpp -- lattice geometry, per-member descriptors and kernel
// launchers shared by the HIP translation units of libgf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tile_order.hpp"

namespace gf {

// Internal link layout. Sites are split by parity p = (x+y+z+t) mod 2 and
// indexed within a parity by h = (x + nx(y + ny(z + nz t))) / 2, as in the
// paper's implementation section; the sites of one parity are then grouped
// in blocks of BLK consecutive h, and each block stores, for mu = 0..3 and
// each stored matrix element e, the BLK complex values of that element
// contiguously:
//     complex index = (((p * nb + h / BLK) * 4 + mu) * ne + e) * BLK + h % BLK,
// with nb = ceil(V/2 / BLK) blocks per parity and ne = 9 (full matrix) or 6
// (rows 0 and 1). A wavefront's forward links are then one contiguous run of
// 4 * ne * BLK complex values, and its backward links a handful more, instead
// of 8 * ne separate arrays; HBM sustains much higher bandwidth on such runs.
constexpr int BLK_LOG2 = 6;
constexpr int BLK = 1 << BLK_LOG2;

struct Geom {
    int nx, ny, nz, nt;
    int hx;         // nx / 2
    int Vh;         // V / 2 (sites of one parity)
    int V;          // sites
    int sz;         // hx * ny       (half-index stride of one z step)
    int st;         // hx * ny * nz  (half-index stride of one t step)
    int nb;         // blocks of BLK sites per parity
    int ne;         // stored complex elements per link (9 or 6)
};

inline Geom make_geom(const int d[4], int ne) {
    Geom g;
    g.nx = d[0]; g.ny = d[1]; g.nz = d[2]; g.nt = d[3];
    g.hx = d[0] / 2;
    g.V = d[0] * d[1] * d[2] * d[3];
    g.Vh = g.V / 2;
    g.sz = g.hx * d[1];
    g.st = g.sz * d[2];
    g.nb = (g.Vh + BLK - 1) / BLK;
    g.ne = ne;
    return g;
}

// Complex offset of element 0 of U_mu at site (p, h); element e is BLK further.
__host__ __device__ inline long long link_off(const Geom &g, int mu, int p, int h) {
    return ((long long)((p * g.nb + (h >> BLK_LOG2)) * 4 + mu) * g.ne << BLK_LOG2) + (h & (BLK - 1));
}

// Complex values in one field (padding of the last block included).
inline long long field_complex(const Geom &g) { return 2LL * g.nb * 4 * g.ne * BLK; }

// The g field of a gauge transformation (9 complex elements per site, the
// library's own scratch) in the links' blocking: the sites of one parity in
// blocks of BLK consecutive h, each block holding element e of its BLK
// sites contiguously. (Nine arrays of V values instead would start at
// multiples of a large power of two, map to the same L2 sets and evict
// each other.)
__host__ __device__ inline long long gfield_off(const Geom &g, int p, int h, int e) {
    return ((long long)((p * g.nb + (h >> BLK_LOG2)) * 9 + e) << BLK_LOG2) + (h & (BLK - 1));
}
inline long long gfield_complex(const Geom &g) { return 2LL * g.nb * 9 * BLK; }

// An su(3) algebra field (8 reals per site: s_a(x), or a gradient) in the
// same blocking: component a of site (p, h).
__host__ __device__ inline long long alg_off(const Geom &g, int p, int h, int a) {
    return ((long long)((p * g.nb + (h >> BLK_LOG2)) * 8 + a) << BLK_LOG2) + (h & (BLK - 1));
}
inline long long alg_reals(const Geom &g) { return 2LL * g.nb * 8 * BLK; }

// Coordinates of site (p, h) and the half indices of its four backward
// neighbours x - mu (which have parity 1 - p).
struct SiteNbr {
    int hb[4];
};

__host__ __device__ inline SiteNbr site_neighbours(const Geom &g, int p, int h) {
    int q = h / g.hx;             // row index j + ny (k + nz t)
    int ih = h - q * g.hx;
    int q2 = q / g.ny;
    int j = q - q2 * g.ny;
    int t = q2 / g.nz;
    int k = q2 - t * g.nz;
    int b = (p + j + k + t) & 1;  // x = 2 ih + b
    SiteNbr n;
    n.hb[0] = (ih == 0 && b == 0) ? h + g.hx - 1 : h - 1 + b;
    n.hb[1] = (j == 0) ? h + (g.ny - 1) * g.hx : h - g.hx;
    n.hb[2] = (k == 0) ? h + (g.nz - 1) * g.sz : h - g.sz;
    n.hb[3] = (t == 0) ? h + (g.nt - 1) * g.st : h - g.st;
    return n;
}

// Half indices of the four forward neighbours x + mu (parity 1 - p).
__host__ __device__ inline SiteNbr site_fwd_neighbours(const Geom &g, int p, int h) {
    int q = h / g.hx;
    int ih = h - q * g.hx;
    int q2 = q / g.ny;
    int j = q - q2 * g.ny;
    int t = q2 / g.nz;
    int k = q2 - t * g.nz;
    int b = (p + j + k + t) & 1;
    SiteNbr n;
    n.hb[0] = (ih == g.hx - 1 && b == 1) ? h - g.hx + 1 : h + b;
    n.hb[1] = (j == g.ny - 1) ? h - (g.ny - 1) * g.hx : h + g.hx;
    n.hb[2] = (k == g.nz - 1) ? h - (g.nz - 1) * g.sz : h + g.sz;
    n.hb[3] = (t == g.nt - 1) ? h - (g.nt - 1) * g.st : h + g.st;
    return n;
}

// Half index and parity of the canonical site (x, y, z, t).
__host__ __device__ inline void site_to_ph(const Geom &g, int x, int y, int z, int t, int &p, int &h) {
    p = (x + y + z + t) & 1;
    h = (x + g.nx * (y + g.ny * (z + g.nz * t))) >> 1;
}

// One member of an ensemble as seen by the kernels.
struct CfgDesc {
    Geom g;
    void *U;         // device field in the internal layout
    double omega;    // over-relaxation parameter
    int gauge;       // 0 Landau, 1 Coulomb
    int tile0;       // first sweep tile of this member
    int qtile0;      // first quality tile of this member
    int nqtiles;     // quality tiles of this member
};

// Sites handled by one quality workgroup (fixed, so F and theta are
// bitwise independent of the sweep schedule).
constexpr int QTILE = 256;

struct Schedule {
    int lps;        // lanes per site: 1, 2, 4, 8
    int block;      // threads per workgroup
    int nt;         // non-temporal loads/stores
    int order;      // sweep tiles: 0 in dispatch order, 1 XCD-contiguous (xcd_tile)
};

// ---- launchers (defined in the .hip files) ----
hipError_t launch_half_sweep(int prec, int nelem, const Schedule &s, const CfgDesc *d_desc,
                             const int *d_tile_cfg, const int *d_active, int ntiles, int parity,
                             int reunit, hipStream_t st);
hipError_t launch_quality(int prec, int nelem, const CfgDesc *d_desc, const int *d_qtile_cfg,
                          const int *d_active, int nqtiles, double *d_partials, const SlabOrder &so,
                          hipStream_t st);
hipError_t launch_quality_final(const CfgDesc *d_desc, int n, const double *d_partials,
                                double *d_result, int *d_active, int *d_iters, int swept,
                                double eps, int update_active, hipStream_t st);
// Per-time-slice F_t and theta_t of one member into d_out[2 t], d_out[2 t + 1];
// d_partials holds 2 * nt * quality_slice_chunks(g) doubles.
int quality_slice_chunks(const Geom &g);
// k_quality for a single lattice whose time slices split into whole tiles,
// walking runs of slices (same partials as launch_quality)
bool quality_tstream_ok(const Geom &g);
hipError_t launch_quality_tstream(int prec, int nelem, const Geom &g, const CfgDesc *d_desc, const int *d_active,
                                  double *d_partials, hipStream_t st);
hipError_t launch_quality_slices(int prec, int nelem, const CfgDesc &d, double *d_partials, double *d_out,
                                 hipStream_t st);
// F and theta of one lattice given by value (d.qtile0 = 0, d.nqtiles tiles):
// d_partials holds 2 * d.nqtiles doubles, d_out receives {F, theta}.
hipError_t launch_quality_one(int prec, int nelem, const CfgDesc &d, double *d_partials, double *d_out,
                              hipStream_t st);
// Message of the last failed context-free call on this thread.
const char *noalloc_last_error();
hipError_t launch_pack(int prec, int nelem, const Geom &g, const void *aos, void *U, int unpack,
                       hipStream_t st);
hipError_t launch_reunit(int prec, int nelem, const Geom &g, void *U, hipStream_t st);
hipError_t launch_pack_alg(int prec, const Geom &g, const void *aos, void *s, int unpack,
                           hipStream_t st);
hipError_t launch_expS(int prec, const Geom &g, const void *s, void *gfield, hipStream_t st);
hipError_t launch_functional(int prec, int nelem, int gauge, const Geom &g, const void *U,
                             const void *gfield, double *d_partials, hipStream_t st);
hipError_t launch_functional_grad(int prec, int nelem, int gauge, const Geom &g, const void *U,
                                  const void *s, const void *gfield, double scale, void *grad,
                                  hipStream_t st);
hipError_t launch_gauge_transform(int prec, int nelem, const Geom &g, void *U, const void *gfield,
                                  hipStream_t st);
hipError_t launch_sum_partials(const double *d_partials, int n, double *d_out, hipStream_t st);

}  // namespace gf
