// tile_order.hpp -- order in which workgroups take tiles.
#pragma once

#include <hip/hip_runtime.h>

namespace gf {

// Workgroups are dispatched to the 8 XCDs round-robin by id. Map id b of n
// to a tile so that XCD k gets the k-th contiguous share of the tiles, in
// order (a bijection of [0, n) for any n).
__host__ __device__ __forceinline__ int xcd_tile(int b, int n) {
    constexpr int NX = 8;
    const int x = b % NX, i = b / NX;
    const int q = n / NX, r = n % NX;
    return x * q + min(x, r) + i;
}

// Slab order for the kernels whose sites read their neighbours' data
// (F/theta, the gauge transformation, the differentiation kernels). Their
// tiles are runs of consecutive half indices h; the neighbour one step in t
// is S = st / tile tiles further on (st the half sites of one time slice),
// one step in z about S / nz tiles, in x and y mostly the same tile. Walking
// the tiles in plain order, the t neighbour's data was fetched S tiles
// earlier -- for 48^4 some 30 MB of links before, far beyond the 4 MB L2 of
// an XCD -- and is fetched again. Viewing the first nrow * S tiles as rows
// of S (one time slice each, when S divides evenly) cut into column blocks
// of B tiles, the sequence below walks a column block down all rows before
// the next: the t neighbour is then B tiles back and the z neighbour (if
// S / nz < B) in the same row, both still in L2. Tiles past nrow * S keep
// their place. The XCDs take contiguous shares of the sequence, so the
// number of blocks is a multiple of 8 where it can be.
struct SlabOrder {
    int S;     // tiles per row (0: plain order)
    int nrow;  // rows
    int B;     // columns per block
    int P;     // 2-d blocks: tiles per z plane (0: blocks of B consecutive tiles)
    int w;     // 2-d blocks: tiles along the plane per block (B / w planes)
};

#ifndef GF_SLAB_BMAX
#define GF_SLAB_BMAX 32
#endif

inline SlabOrder make_slab_order(int st, int tile_h, int ntiles, int bmax = GF_SLAB_BMAX) {
    SlabOrder o{0, 0, 0, 0, 0};
    const int S = st / tile_h;
    if (S < 2 || ntiles / S < 2) return o;  // too small to matter
    const int BMAX = bmax;
    const int nblk = 8 * ((S + 8 * BMAX - 1) / (8 * BMAX));
    o.S = S;
    o.nrow = ntiles / S;
    o.B = (S + nblk - 1) / nblk;
    return o;
}

// 2-d column blocks: when a z plane of sz half indices is P whole tiles and
// a row is a whole time slice (nz planes), a block may instead be w tiles
// along the plane by d = B / w consecutive planes (w | P, d | nz): its z
// neighbours then stay inside the block for all but its first plane, at the
// price of the y neighbours of the first tile along the plane.
inline SlabOrder make_slab_order_2d(int st, int sz, int nz, int tile_h, int ntiles, int w, int d) {
    SlabOrder o{0, 0, 0, 0, 0};
    if (st % tile_h != 0 || sz % tile_h != 0 || ntiles % (st / tile_h) != 0) return o;
    const int P = sz / tile_h;
    if (w < 1 || d < 1 || P % w != 0 || nz % d != 0 || ntiles / (st / tile_h) < 2) return o;
    o.S = st / tile_h;
    o.nrow = ntiles / o.S;
    o.B = w * d;
    o.P = P;
    o.w = w;
    return o;
}

// Column blocks sized by bytes: a block's tiles of one row are to hold about
// GF_SLAB_BYTES of the kernel's data (tile_bytes per tile), so that the
// previous row's tiles -- the t neighbours -- are still in an XCD's 4 MB L2
// with room for the reads in flight. Among the 2-d blocks that fit, the one
// whose boundary cuts the fewest neighbour reads: a fraction hx / (w tile_h)
// of the sites lose their y neighbour (one row of the w tiles along the
// plane, none when the block spans the plane) and 1 / d their z neighbour
// (none when it spans all nz planes); ties go to the smaller block. Lattices
// whose planes are not whole tiles take 1-d blocks of the same size.
#ifndef GF_SLAB_BYTES
#define GF_SLAB_BYTES (3 << 19)
#endif

inline SlabOrder pick_slab_order(int st, int sz, int hx, int nz, int tile_h, int ntiles, long long tile_bytes) {
    const long long per = tile_bytes > 0 ? tile_bytes : 1;
    const int bmax = (int)(GF_SLAB_BYTES / per > 2 ? GF_SLAB_BYTES / per : 2);
    SlabOrder best{0, 0, 0, 0, 0};
    double best_cost = 0.0;
    if (tile_h > 0 && sz % tile_h == 0) {
        const int P = sz / tile_h;
        for (int w = 1; w <= P; w++) {
            if (P % w != 0) continue;
            for (int d = 1; d <= nz && w * d <= bmax; d++) {
                if (nz % d != 0) continue;
                const double cost = (w < P ? (double)hx / ((double)w * tile_h) : 0.0) + (d < nz ? 1.0 / d : 0.0);
                if (best.S && (cost > best_cost + 1e-12 || (cost > best_cost - 1e-12 && w * d >= best.B))) continue;
                const SlabOrder o = make_slab_order_2d(st, sz, nz, tile_h, ntiles, w, d);
                if (o.S) { best = o; best_cost = cost; }
            }
        }
    }
    return best.S ? best : make_slab_order(st, tile_h, ntiles, bmax);
}

// Tile of sequence position q (a bijection of [0, ntiles)).
__host__ __device__ __forceinline__ int slab_tile(int q, const SlabOrder &o) {
    if (o.S == 0) return q;
    const int m = o.nrow * o.S;
    if (q >= m) return q;
    const int full = o.nrow * o.B;
    const int cb = q / full;
    if (o.P) {
        const int rem = q - cb * full;
        const int r = rem / o.B, k = rem - r * o.B;
        const int nbc = o.P / o.w, d = o.B / o.w;
        const int bz = cb / nbc, bc = cb - bz * nbc;
        const int zz = k / o.w, cc = k - zz * o.w;
        return r * o.S + (bz * d + zz) * o.P + bc * o.w + cc;
    }
    const int w = min(o.B, o.S - cb * o.B);
    const int rem = q - cb * full;
    const int r = rem / w;
    return r * o.S + cb * o.B + (rem - r * w);
}

}  // namespace gf
