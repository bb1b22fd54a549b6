// Backward kernels of y = A(theta) x over SPC5 beta(r,c) storage:
//   xbar = A^T ybar  (masked scatter-transpose: each set bit k of row i of a
//                    block adds value * ybar[row] to xbar[anchor + k]);
//   vbar = d<ybar, y>/d theta, in packed order: vbar[v] = ybar[row(v)] * x[col(v)].
// Both walk the blocks exactly like the forward kernel (tile of panels per
// wavefront, lane = block row, popcount prefix for the packed value offset).
//
// The transpose scatters with hardware float atomics.  When r is a power of
// two the r lanes of one block (same anchor, same window of xbar) first sum
// their contributions column by column with cross-lane shuffles, so a block
// issues at most one atomic per column instead of one per nonzero.
#include "spc5_internal.h"
#include "stage.h"
#include "tile.h"

namespace spc5 {

template <typename T, int R, int C>
__global__ __launch_bounds__(kWave) void k_transpose(
    int64_t npanels, int64_t nrows, int ppt, int64_t ntiles,
    const int32_t *__restrict__ blk_ptr, const int32_t *__restrict__ blk_col,
    const typename MaskOf<C>::type *__restrict__ masks, const T *__restrict__ val,
    const int32_t *__restrict__ panel_val, const T *__restrict__ ybar, T *__restrict__ xbar)
{
    constexpr int BPS = kWave / R;
    constexpr int LANES = BPS * R;
    constexpr bool kGroup = R > 1 && (R & (R - 1)) == 0;
    const int lane = lane_id();
    const TileCtx t = tile_begin(xcd_remap(blockIdx.x, ntiles), ppt, npanels, blk_ptr);
    const int i = lane % R;
    const int bl = lane / R;
    int vbase = panel_val[t.p0];
    for (int bs = t.b0; bs < t.b1; bs += BPS) {
        const int b = bs + bl;
        const bool act = (lane < LANES) && (b < t.b1);
        const unsigned m = act ? (unsigned)masks[(int64_t)b * R + i] : 0u;
        const int col0 = act ? blk_col[b] : 0;
        const int cnt = __popc(m);
        const int incl = wave_incl_scan(cnt);
        int j = vbase + incl - cnt;
        vbase += __shfl(incl, kWave - 1);
        const int pid = tile_panel_of(b, t.pe);
        const T yv = m ? ybar[(t.p0 + pid) * R + i] : T(0);
        if constexpr (kGroup) {
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const bool has = (m >> k) & 1u;
                T contrib = has ? val[j] * yv : T(0);
                j += has ? 1 : 0;
                unsigned any = has ? 1u : 0u;
#pragma unroll
                for (int d = 1; d < R; d <<= 1) {
                    contrib += __shfl_xor(contrib, d);
                    any |= __shfl_xor(any, d);
                }
                if (any && i == (k % R)) atomicAdd(&xbar[col0 + k], contrib);
            }
        } else {
#pragma unroll
            for (int k = 0; k < C; ++k) {
                if ((m >> k) & 1u) {
                    atomicAdd(&xbar[col0 + k], val[j] * yv);
                    ++j;
                }
            }
        }
    }
}

template <typename T, int R, int C>
__global__ __launch_bounds__(kWave) void k_values_grad(
    int64_t npanels, int64_t nrows, int ppt, int64_t ntiles,
    const int32_t *__restrict__ blk_ptr, const int32_t *__restrict__ blk_col,
    const typename MaskOf<C>::type *__restrict__ masks, const int32_t *__restrict__ panel_val,
    const T *__restrict__ ybar, const T *__restrict__ x, T *__restrict__ vbar)
{
    constexpr int BPS = kWave / R;
    constexpr int LANES = BPS * R;
    const int lane = lane_id();
    const TileCtx t = tile_begin(xcd_remap(blockIdx.x, ntiles), ppt, npanels, blk_ptr);
    const int i = lane % R;
    const int bl = lane / R;
    int vbase = panel_val[t.p0];
    for (int bs = t.b0; bs < t.b1; bs += BPS) {
        const int b = bs + bl;
        const bool act = (lane < LANES) && (b < t.b1);
        const unsigned m = act ? (unsigned)masks[(int64_t)b * R + i] : 0u;
        const int col0 = act ? blk_col[b] : 0;
        const int cnt = __popc(m);
        const int incl = wave_incl_scan(cnt);
        int j = vbase + incl - cnt;
        vbase += __shfl(incl, kWave - 1);
        const int pid = tile_panel_of(b, t.pe);
        const T yv = m ? ybar[(t.p0 + pid) * R + i] : T(0);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            if ((m >> k) & 1u) {
                vbar[j] = yv * x[col0 + k];
                ++j;
            }
        }
    }
}

// The same scatter with hot-column pre-aggregation.  A workgroup of four
// wavefronts walks a contiguous range of tiles (one tile per wavefront at a
// time) and adds its contributions into an LDS table of kAggSlots columns
// (two probes, slot claimed by the first column that reaches it); a column
// that finds both probes taken goes straight to a global atomic.  At the end
// every occupied slot issues one global atomic.  A column shared by many rows
// (a popular node of a graph) then costs one global atomic per workgroup
// instead of one per row.
constexpr int kAggSlots = 2048;
constexpr int kAggGrid = 2048;

template <typename T>
__device__ __forceinline__ void agg_add(int *tag, T *acc, int col, T v, T *xbar) {
    const int s0 = (int)(((unsigned)col * 2654435761u) >> 21) & (kAggSlots - 1);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int sl = s0 ^ p;
        int t = tag[sl];
        if (t == -1) {
            const int old = atomicCAS(&tag[sl], -1, col);
            t = old == -1 ? col : old;
        }
        if (t == col) {
            atomicAdd(&acc[sl], v);
            return;
        }
    }
    atomicAdd(&xbar[col], v);
}

template <typename T, int R, int C>
__global__ __launch_bounds__(256) void k_transpose_agg(
    int64_t npanels, int ppt, int64_t ntiles, int64_t tpw,
    const int32_t *__restrict__ blk_ptr, const int32_t *__restrict__ blk_col,
    const typename MaskOf<C>::type *__restrict__ masks, const T *__restrict__ val,
    const int32_t *__restrict__ panel_val, const T *__restrict__ ybar, T *__restrict__ xbar)
{
    constexpr int BPS = kWave / R;
    constexpr int LANES = BPS * R;
    constexpr bool kGroup = R > 1 && (R & (R - 1)) == 0;
    __shared__ int s_tag[kAggSlots];
    __shared__ T s_acc[kAggSlots];
    const int th = threadIdx.x, lane = lane_id(), wv = th / kWave;
    for (int q = th; q < kAggSlots; q += 256) {
        s_tag[q] = -1;
        s_acc[q] = T(0);
    }
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * tpw;
    const int64_t t1 = min(t0 + tpw, ntiles);
    const int i = lane % R;
    const int bl = lane / R;
    for (int64_t tile = t0 + wv; tile < t1; tile += 256 / kWave) {
        const TileCtx t = tile_begin(tile, ppt, npanels, blk_ptr);
        int vbase = panel_val[t.p0];
        for (int bs = t.b0; bs < t.b1; bs += BPS) {
            const int b = bs + bl;
            const bool act = (lane < LANES) && (b < t.b1);
            const unsigned m = act ? (unsigned)masks[(int64_t)b * R + i] : 0u;
            const int col0 = act ? blk_col[b] : 0;
            const int cnt = __popc(m);
            const int incl = wave_incl_scan(cnt);
            int j = vbase + incl - cnt;
            vbase += __shfl(incl, kWave - 1);
            const int pid = tile_panel_of(b, t.pe);
            const T yv = m ? ybar[(t.p0 + pid) * R + i] : T(0);
            if constexpr (kGroup) {
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    const bool has = (m >> k) & 1u;
                    T contrib = has ? val[j] * yv : T(0);
                    j += has ? 1 : 0;
                    unsigned any = has ? 1u : 0u;
#pragma unroll
                    for (int d = 1; d < R; d <<= 1) {
                        contrib += __shfl_xor(contrib, d);
                        any |= __shfl_xor(any, d);
                    }
                    if (any && i == (k % R)) agg_add(s_tag, s_acc, col0 + k, contrib, xbar);
                }
            } else {
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    if ((m >> k) & 1u) {
                        agg_add(s_tag, s_acc, col0 + k, val[j] * yv, xbar);
                        ++j;
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int q = th; q < kAggSlots; q += 256)
        if (s_tag[q] >= 0) atomicAdd(&xbar[s_tag[q]], s_acc[q]);
}

template <typename T, int R, int C>
static hipError_t launch_tr(const spc5_matrix *A, const T *val, const T *ybar, T *xbar,
                            hipStream_t s) {
    hipError_t e = zero_fill(xbar, A->ncols, sizeof(T), s);
    if (e != hipSuccess) return e;
    const int64_t ntiles = (A->npanels + A->ppt - 1) / A->ppt;
    if (ntiles == 0) return hipSuccess;
    // aggregation pays where columns are shared by many rows; a banded
    // matrix's columns are short and go straight to global atomics
    if (A->hot_cols) {
        const int64_t tpw = (ntiles + kAggGrid - 1) / kAggGrid;
        const int64_t grid = (ntiles + tpw - 1) / tpw;
        hipLaunchKernelGGL((k_transpose_agg<T, R, C>), dim3((unsigned)grid), dim3(256), 0, s,
                           A->npanels, A->ppt, ntiles, tpw, A->blk_ptr, A->blk_col,
                           (const typename MaskOf<C>::type *)A->masks, val, A->panel_val, ybar,
                           xbar);
    } else {
        hipLaunchKernelGGL((k_transpose<T, R, C>), dim3((unsigned)ntiles), dim3(kWave), 0, s,
                           A->npanels, A->nrows, A->ppt, ntiles, A->blk_ptr, A->blk_col,
                           (const typename MaskOf<C>::type *)A->masks, val, A->panel_val, ybar,
                           xbar);
    }
    return hipGetLastError();
}

template <typename T, int R, int C>
static hipError_t launch_vg(const spc5_matrix *A, const T *ybar, const T *x, T *vbar,
                            hipStream_t s) {
    const int64_t ntiles = (A->npanels + A->ppt - 1) / A->ppt;
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL((k_values_grad<T, R, C>), dim3((unsigned)ntiles), dim3(kWave), 0, s,
                       A->npanels, A->nrows, A->ppt, ntiles, A->blk_ptr, A->blk_col,
                       (const typename MaskOf<C>::type *)A->masks, A->panel_val, ybar, x,
                       vbar);
    return hipGetLastError();
}

#define SPC5_SHAPE_SWITCH(CALL)                                                        \
    switch (A->r * 100 + (A->c <= 4 ? 4 : (A->c <= 8 ? 8 : 16))) {                    \
        SPC5_ROW(1, CALL) SPC5_ROW(2, CALL) SPC5_ROW(3, CALL) SPC5_ROW(4, CALL)        \
        SPC5_ROW(5, CALL) SPC5_ROW(6, CALL) SPC5_ROW(7, CALL) SPC5_ROW(8, CALL)        \
        default: return hipErrorInvalidValue;                                          \
    }
#define SPC5_ROW(RR, CALL) SPC5_CASE(RR, 4, CALL) SPC5_CASE(RR, 8, CALL) SPC5_CASE(RR, 16, CALL)

template <typename T>
static hipError_t tr_dispatch(const spc5_matrix *A, const void *val, const void *ybar,
                              void *xbar, hipStream_t s) {
#define SPC5_CASE(RR, CC, CALL) \
    case RR * 100 + CC: return launch_tr<T, RR, CC>(A, (const T *)val, (const T *)ybar, (T *)xbar, s);
    SPC5_SHAPE_SWITCH(0)
#undef SPC5_CASE
}

template <typename T>
static hipError_t vg_dispatch(const spc5_matrix *A, const void *ybar, const void *x,
                              void *vbar, hipStream_t s) {
#define SPC5_CASE(RR, CC, CALL) \
    case RR * 100 + CC: return launch_vg<T, RR, CC>(A, (const T *)ybar, (const T *)x, (T *)vbar, s);
    SPC5_SHAPE_SWITCH(0)
#undef SPC5_CASE
}

hipError_t launch_transpose(const spc5_matrix *A, const void *val, const void *ybar,
                            void *xbar, hipStream_t s) {
    return A->dtype == SPC5_F64 ? tr_dispatch<double>(A, val, ybar, xbar, s)
                                : tr_dispatch<float>(A, val, ybar, xbar, s);
}

// Values gradient for beta(1,c) (every block one row) over the staged tile
// schedule, one workgroup per tile.  The tile's row masks, anchors and panel
// bounds are read once; a scan of the block popcounts gives every block its
// first value slot; one thread per BPT consecutive blocks decodes the slots'
// columns and rows into LDS; then consecutive threads take consecutive slots,
// vbar[v] = ybar[row(v)] * x[col(v)], so the stores are contiguous and all
// gathers of a thread are in flight together.
template <typename T, int C>
__global__ __launch_bounds__(kWG) void k_values_grad_v(
    int64_t ntiles, const int32_t *__restrict__ tile_p, const int32_t *__restrict__ tile_b,
    const int32_t *__restrict__ tile_v, const int32_t *__restrict__ tile_f,
    const int32_t *__restrict__ blk_ptr, const int32_t *__restrict__ blk_col,
    const typename MaskOf<C>::type *__restrict__ masks, const T *__restrict__ ybar,
    const T *__restrict__ x, T *__restrict__ vbar)
{
    constexpr int BPT = 4;                                   // blocks per thread
    constexpr int VMAX = value_tile((int)sizeof(T));         // values per tile
    constexpr int NX = (VMAX + kWG - 1) / kWG;
    __shared__ int s_vcol[VMAX];
    __shared__ int s_vrow[VMAX];
    __shared__ int s_bp[kWG + 1];
    __shared__ int s_wsum[kWG / kWave];
    const int th = threadIdx.x, lane = lane_id(), wv = th / kWave;
    const int64_t t = xcd_chunks(blockIdx.x, ntiles, kXcdRun);
    const int f = tile_f[t];
    const int p0 = tile_p[t], p1 = f ? p0 + 1 : tile_p[t + 1];
    const int b0 = tile_b[t], nbt = tile_b[t + 1] - b0;
    const int v0 = tile_v[t], nv = tile_v[t + 1] - v0;
    const int np = p1 - p0;
    for (int i = th; i <= np; i += kWG) s_bp[i] = blk_ptr[p0 + i];
    unsigned m[BPT];
    int col[BPT];
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int tb = th * BPT + k;
        const bool ok = tb < nbt;
        m[k] = ok ? (unsigned)masks[b0 + tb] : 0u;
        col[k] = ok ? blk_col[b0 + tb] : 0;
        cnt += __popc(m[k]);
    }
    const int incl = wave_incl_scan(cnt);
    if (lane == kWave - 1) s_wsum[wv] = incl;
    __syncthreads();
    int off = incl - cnt;
#pragma unroll
    for (int w2 = 0; w2 < kWG / kWave; ++w2) off += w2 < wv ? s_wsum[w2] : 0;
    // row of my first block: the last panel starting at or before it
    int pl = 0;
    {
        const int b = b0 + th * BPT;
        int lo = 0, hi = np - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (s_bp[mid] <= b) lo = mid;
            else hi = mid - 1;
        }
        pl = lo;
    }
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int tb = th * BPT + k;
        if (tb >= nbt) break;
        while (pl + 1 < np && s_bp[pl + 1] <= b0 + tb) ++pl;
        unsigned mm = m[k];
        while (mm) {
            s_vcol[off] = col[k] + __ffs(mm) - 1;
            s_vrow[off] = p0 + pl;
            ++off;
            mm &= mm - 1u;
        }
    }
    __syncthreads();
    T yv[NX], xv[NX];
#pragma unroll
    for (int e = 0; e < NX; ++e) {
        const int q = th + e * kWG;
        const bool ok = q < nv;
        yv[e] = ok ? ybar[s_vrow[q]] : T(0);
        xv[e] = ok ? x[s_vcol[q]] : T(0);
    }
#pragma unroll
    for (int e = 0; e < NX; ++e) {
        const int q = th + e * kWG;
        if (q < nv) vbar[v0 + q] = yv[e] * xv[e];
    }
}

template <typename T, int C>
static hipError_t launch_vg_v(const spc5_matrix *A, const T *ybar, const T *x, T *vbar,
                              hipStream_t s) {
    hipLaunchKernelGGL((k_values_grad_v<T, C>), dim3((unsigned)A->ntiles_staged), dim3(kWG), 0,
                       s, A->ntiles_staged, A->tile_p, A->tile_b, A->tile_v, A->tile_f,
                       A->blk_ptr, A->blk_col, (const typename MaskOf<C>::type *)A->masks, ybar,
                       x, vbar);
    return hipGetLastError();
}

template <typename T>
static hipError_t vg_v_dispatch(const spc5_matrix *A, const void *ybar, const void *x,
                                void *vbar, hipStream_t s) {
    const T *yb = (const T *)ybar, *xx = (const T *)x;
    if (A->c <= 4) return launch_vg_v<T, 4>(A, yb, xx, (T *)vbar, s);
    if (A->c <= 8) return launch_vg_v<T, 8>(A, yb, xx, (T *)vbar, s);
    return launch_vg_v<T, 16>(A, yb, xx, (T *)vbar, s);
}

hipError_t launch_values_grad(const spc5_matrix *A, const void *ybar, const void *x,
                              void *vbar, hipStream_t s) {
    // beta(1,c) with a staged schedule: the value-mode kernel
    if (A->r == 1 && A->tile_p && A->ntiles_staged > 0)
        return A->dtype == SPC5_F64 ? vg_v_dispatch<double>(A, ybar, x, vbar, s)
                                    : vg_v_dispatch<float>(A, ybar, x, vbar, s);
    return A->dtype == SPC5_F64 ? vg_dispatch<double>(A, ybar, x, vbar, s)
                                : vg_dispatch<float>(A, ybar, x, vbar, s);
}

}  // namespace spc5
