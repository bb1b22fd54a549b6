// One tile of Y = A X over SPC5 beta(r,c) storage for K right-hand sides,
// shared by the single-matrix SpMM kernel and the batched persistent kernel.
#pragma once

#include "tile.h"

namespace spc5 {

// One tile (ppt consecutive panels) of Y = A X for a chunk of K right-hand
// sides; ytile: LDS, at least ppt*R*K entries.  Shared by the single-matrix
// kernel and the batched persistent kernel.
template <typename T, int R, int C, int K>
__device__ __forceinline__ void spmm_tile(
    int64_t tile, int ppt, int64_t npanels, int64_t nrows,
    const int32_t *__restrict__ blk_ptr, const int32_t *__restrict__ blk_col,
    const typename MaskOf<C>::type *__restrict__ masks, const T *__restrict__ val,
    const int32_t *__restrict__ panel_val, const T *__restrict__ X, T *__restrict__ Y, int ld,
    T *ytile)
{
    constexpr int BPS = kWave / R;
    constexpr int LANES = BPS * R;
    const int lane = lane_id();
    const TileCtx t = tile_begin(tile, ppt, npanels, blk_ptr);
    for (int q = lane; q < t.np * R * K; q += kWave) ytile[q] = T(0);
    __syncthreads();
    const int i = lane % R;
    const int bl = lane / R;
    int vbase = panel_val[t.p0];
    const int vsafe = vbase;      // a valid value index whenever the tile has blocks
    for (int bs = t.b0; bs < t.b1; bs += BPS) {
        const int b = bs + bl;
        const bool act = (lane < LANES) && (b < t.b1);
        const int bb = act ? b : t.b0;
        const unsigned m0 = (unsigned)masks[(int64_t)bb * R + i];
        const int c0 = blk_col[bb];
        const unsigned m = act ? m0 : 0u;
        const int col0 = c0;
        const int cnt = __popc(m);
        const int incl = wave_incl_scan(cnt);
        int j = vbase + incl - cnt;
        vbase += __shfl(incl, kWave - 1);
        const int pid = tile_panel_of(b, t.pe);
        T acc[K];
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = T(0);
        // branch-free: every lane issues the loads of every bit (a clear bit
        // reads a valid address and is dropped), so they are all in flight
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const bool on = (m >> k) & 1u;
            const T v = val[on ? j : vsafe];
            const T *xr = X + (int64_t)(col0 + (on ? k : 0)) * ld;
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const T r = fma(v, xr[q], acc[q]);
                acc[q] = on ? r : acc[q];
            }
            j += on ? 1 : 0;
        }
#pragma unroll
        for (int d = R; d < kWave; d <<= 1) {
            const int op = __shfl_up(pid, d);
            const bool take = lane >= d && op == pid;
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const T o = __shfl_up(acc[q], d);
                if (take) acc[q] += o;
            }
        }
        const int pn = __shfl_down(pid, R);
        const int bn = __shfl_down(b, R);
        const bool tail = act && (lane + R >= LANES || bn >= t.b1 || pn != pid);
        if (tail) {
#pragma unroll
            for (int q = 0; q < K; ++q) ytile[(pid * R + i) * K + q] += acc[q];
        }
    }
    __syncthreads();
    const int64_t row0 = t.p0 * R;
    const int nr = (int)min((int64_t)t.np * R, nrows - row0);
    for (int q = lane; q < nr * K; q += kWave) Y[(row0 + q / K) * ld + q % K] = ytile[q];
    __syncthreads();
}

}  // namespace spc5
