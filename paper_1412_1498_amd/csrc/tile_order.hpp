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

}  // namespace gf
