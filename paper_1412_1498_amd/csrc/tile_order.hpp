// tile_order.hpp -- order in which workgroups take tiles.
#pragma once

#include <hip/hip_runtime.h>

namespace gf {

// Workgroups are dispatched to the 8 XCDs round-robin by id. Map id b of n
// to a tile so that XCD k gets the k-th contiguous share of the tiles, in
// order (a bijection of [0, n) for any n).
__device__ __forceinline__ int xcd_tile(int b, int n) {
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
};

#ifndef GF_SLAB_BMAX
#define GF_SLAB_BMAX 32
#endif

inline SlabOrder make_slab_order(int st, int tile_h, int ntiles, int bmax = GF_SLAB_BMAX) {
    SlabOrder o{0, 0, 0};
    const int S = st / tile_h;
    if (S < 2 || ntiles / S < 2) return o;  // too small to matter
    const int BMAX = bmax;
    const int nblk = 8 * ((S + 8 * BMAX - 1) / (8 * BMAX));
    o.S = S;
    o.nrow = ntiles / S;
    o.B = (S + nblk - 1) / nblk;
    return o;
}

// Tile of sequence position q (a bijection of [0, ntiles)).
__device__ __forceinline__ int slab_tile(int q, const SlabOrder &o) {
    if (o.S == 0) return q;
    const int m = o.nrow * o.S;
    if (q >= m) return q;
    const int full = o.nrow * o.B;
    const int cb = q / full;
    const int w = min(o.B, o.S - cb * o.B);
    const int rem = q - cb * full;
    const int r = rem / w;
    return r * o.S + cb * o.B + (rem - r * w);
}

}  // namespace gf
