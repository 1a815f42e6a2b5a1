// Host check of the tile orders of tile_order.hpp: for each lattice and
// tile size on the command line, the order pick_slab_order chooses and
// whether q -> slab_tile(xcd_tile(q)) visits every tile exactly once (also
// for the plain 1-d column blocks of make_slab_order).
// Input lines: nx ny nz nt tile_h tile_bytes; output lines:
// S nrow B P w bijective_picked bijective_1d
#include <cstdio>
#include <vector>

#include "tile_order.hpp"

using namespace gf;

static int bijective(const SlabOrder &o, int n) {
    std::vector<int> seen(n, 0);
    for (int b = 0; b < n; b++) {
        const int t = slab_tile(xcd_tile(b, n), o);
        if (t < 0 || t >= n || seen[t]++) return 0;
    }
    return 1;
}

int main() {
    int nx, ny, nz, nt, th;
    long long bytes;
    while (std::scanf("%d %d %d %d %d %lld", &nx, &ny, &nz, &nt, &th, &bytes) == 6) {
        const int hx = nx / 2, sz = hx * ny, st = sz * nz;
        const long long vh = (long long)st * nt;
        const int n = (int)((vh + th - 1) / th);
        const SlabOrder o = pick_slab_order(st, sz, hx, nz, th, n, bytes);
        const SlabOrder o1 = make_slab_order(st, th, n);
        std::printf("%d %d %d %d %d %d %d\n", o.S, o.nrow, o.B, o.P, o.w, bijective(o, n), bijective(o1, n));
    }
    return 0;
}
