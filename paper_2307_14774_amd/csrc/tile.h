// Tile bookkeeping shared by the SPC5 kernels: one wavefront walks a tile of
// consecutive panels in sweeps of 64/r blocks (lane = one block row).
#pragma once

#include "wave.h"

#include <climits>

namespace spc5 {

constexpr int kSpmmTile = 1024;   // LDS row accumulators per wavefront (ppt*R*K)

struct TileCtx {
    int64_t p0;   // first panel of the tile
    int np;       // panels in the tile
    int pe;       // lane l < np: end block of panel p0+l, else INT_MAX
    int b0, b1;   // block range of the tile
};

__device__ __forceinline__ TileCtx tile_begin(int64_t tile, int ppt, int64_t npanels,
                                              const int32_t *__restrict__ blk_ptr) {
    TileCtx t;
    const int lane = lane_id();
    t.p0 = tile * ppt;
    t.np = (int)min((int64_t)ppt, npanels - t.p0);
    t.pe = lane < t.np ? blk_ptr[t.p0 + lane + 1] : INT_MAX;
    t.b0 = blk_ptr[t.p0];
    t.b1 = __shfl(t.pe, t.np - 1);
    return t;
}

// Index (within the tile) of the panel that holds block b: the number of
// tile panels that end at or before b.  Binary search over the lanes' `pe`.
__device__ __forceinline__ int tile_panel_of(int b, int pe) {
    int pid = 0;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        const int v = __shfl(pe, pid + s - 1);
        if (v <= b) pid += s;
    }
    return pid;
}

}  // namespace spc5
