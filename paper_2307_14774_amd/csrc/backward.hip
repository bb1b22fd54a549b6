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

template <typename T, int R, int C>
static hipError_t launch_tr(const spc5_matrix *A, const T *val, const T *ybar, T *xbar,
                            hipStream_t s) {
    hipError_t e = zero_fill(xbar, A->ncols, sizeof(T), s);
    if (e != hipSuccess) return e;
    const int64_t ntiles = (A->npanels + A->ppt - 1) / A->ppt;
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL((k_transpose<T, R, C>), dim3((unsigned)ntiles), dim3(kWave), 0, s,
                       A->npanels, A->nrows, A->ppt, ntiles, A->blk_ptr, A->blk_col,
                       (const typename MaskOf<C>::type *)A->masks, val, A->panel_val, ybar,
                       xbar);
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

hipError_t launch_values_grad(const spc5_matrix *A, const void *ybar, const void *x,
                              void *vbar, hipStream_t s) {
    return A->dtype == SPC5_F64 ? vg_dispatch<double>(A, ybar, x, vbar, s)
                                : vg_dispatch<float>(A, ybar, x, vbar, s);
}

}  // namespace spc5
