// Forward SPC5 product y = A x on gfx950 (Algorithm 1 of arXiv 2307.14774,
// re-mapped onto 64-lane wavefronts), and the plain CSR comparison kernel.
//
// Work decomposition.  One wavefront owns a tile of `ppt` consecutive panels
// (rows are grouped by r into panels, Section 2.4).  The tile's blocks are
// walked in sweeps of 64/r blocks; lane l of a sweep carries block row
// (block bs + l/r, row l%r), i.e. the mask at index b*r+i, so masks, anchors
// and packed values are read in storage order, coalesced.
//
// Mask expansion.  Algorithm 1 advances one running value index by the
// popcount of every mask it consumes.  Here every lane takes the popcount of
// its own row mask and a wavefront prefix sum gives each lane the offset of
// its first packed value; the tile's starting offset is the value offset of
// its first panel.  The lane then walks its c mask bits (unrolled,
// predicated): bit k multiplies the next packed value by x[anchor+k].
//
// Row reduction.  Partial sums of one row inside a sweep sit in lanes that
// are r apart; a segmented inclusive scan with stride r (segments = panels)
// leaves the sum in the last lane of each segment, which adds it to the
// tile's row accumulator in LDS.  At the end the tile writes its r*ppt rows
// of y once, coalesced (empty rows get 0: y is overwritten).  No atomics, so
// the result is bitwise reproducible run to run.
#include "spc5_internal.h"
#include "wave.h"

#include <climits>

namespace spc5 {

template <typename T, int R, int C, bool CSR>
__global__ __launch_bounds__(kWave) void k_spmv(
    int64_t npanels, int64_t nrows, int ppt, int64_t ntiles, int remap,
    const int32_t *__restrict__ blk_ptr, const int32_t *__restrict__ blk_col,
    const typename MaskOf<C>::type *__restrict__ masks, const T *__restrict__ val,
    const int32_t *__restrict__ panel_val, const T *__restrict__ x, T *__restrict__ y)
{
    constexpr int BPS = kWave / R;     // blocks per sweep
    constexpr int LANES = BPS * R;     // lanes that carry a block row
    __shared__ T ytile[kWave * R];

    const int lane = lane_id();
    const int64_t tile = remap ? xcd_remap(blockIdx.x, ntiles) : (int64_t)blockIdx.x;
    const int64_t p0 = tile * ppt;
    const int np = (int)min((int64_t)ppt, npanels - p0);
    // lane l < np holds the end block of panel p0+l
    const int pe = lane < np ? blk_ptr[p0 + lane + 1] : INT_MAX;
    const int b0 = blk_ptr[p0];
    const int b1 = __shfl(pe, np - 1);
    for (int t = lane; t < np * R; t += kWave) ytile[t] = T(0);
    __syncthreads();

    const int i = lane % R;
    const int bl = lane / R;
    int vbase = CSR ? 0 : panel_val[p0];
    for (int bs = b0; bs < b1; bs += BPS) {
        const int b = bs + bl;
        const bool act = (lane < LANES) && (b < b1);
        unsigned m;
        int col0, j;
        if (CSR) {
            m = act ? 1u : 0u;
            col0 = act ? blk_col[b] : 0;
            j = b;
        } else {
            m = act ? (unsigned)masks[(int64_t)b * R + i] : 0u;
            col0 = act ? blk_col[b] : 0;
            const int cnt = __popc(m);
            const int incl = wave_incl_scan(cnt);
            j = vbase + incl - cnt;
            vbase += __shfl(incl, kWave - 1);
        }
        // panel of block b within the tile: number of panels ending at or before b
        int pid = 0;
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) {
            const int v = __shfl(pe, pid + s - 1);
            if (v <= b) pid += s;
        }
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            if (m & (1u << k)) {
                acc = fma(val[j], x[col0 + k], acc);
                ++j;
            }
        }
        // segmented inclusive scan over the lanes of one (panel, row)
#pragma unroll
        for (int d = R; d < kWave; d <<= 1) {
            const T o = __shfl_up(acc, d);
            const int op = __shfl_up(pid, d);
            if (lane >= d && op == pid) acc += o;
        }
        const int pn = __shfl_down(pid, R);
        const int bn = __shfl_down(b, R);
        const bool tail = act && (lane + R >= LANES || bn >= b1 || pn != pid);
        if (tail) ytile[pid * R + i] += acc;
    }
    __syncthreads();
    const int64_t row0 = p0 * R;
    const int nr = (int)min((int64_t)np * R, nrows - row0);
    for (int t = lane; t < nr; t += kWave) y[row0 + t] = ytile[t];
}

static int g_remap = -1;
static int remap_enabled() {
    if (g_remap < 0) {
        const char *e = getenv("SPC5_XCD_REMAP");
        g_remap = (e && e[0] == '0') ? 0 : 1;
    }
    return g_remap;
}

template <typename T, int R, int C>
static hipError_t launch_t(const spc5_matrix *A, const T *val, const T *x, T *y,
                           hipStream_t s) {
    const int64_t ntiles = (A->npanels + A->ppt - 1) / A->ppt;
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL((k_spmv<T, R, C, false>), dim3((unsigned)ntiles), dim3(kWave), 0, s,
                       A->npanels, A->nrows, A->ppt, ntiles, remap_enabled(), A->blk_ptr,
                       A->blk_col, (const typename MaskOf<C>::type *)A->masks, val,
                       A->panel_val, x, y);
    return hipGetLastError();
}

template <typename T>
static hipError_t dispatch(const spc5_matrix *A, const void *val, const void *x, void *y,
                           hipStream_t s) {
    const T *v = (const T *)(val ? val : A->val);
    const int cm = A->c <= 4 ? 4 : (A->c <= 8 ? 8 : 16);
#define SPC5_CASE(RR, CC)                                                              \
    case RR * 100 + CC:                                                               \
        return launch_t<T, RR, CC>(A, v, (const T *)x, (T *)y, s);
#define SPC5_ROW(RR) SPC5_CASE(RR, 4) SPC5_CASE(RR, 8) SPC5_CASE(RR, 16)
    switch (A->r * 100 + cm) {
        SPC5_ROW(1) SPC5_ROW(2) SPC5_ROW(3) SPC5_ROW(4)
        SPC5_ROW(5) SPC5_ROW(6) SPC5_ROW(7) SPC5_ROW(8)
        default: return hipErrorInvalidValue;
    }
#undef SPC5_ROW
#undef SPC5_CASE
}

hipError_t launch_spmv(const spc5_matrix *A, const void *val, const void *x, void *y,
                       hipStream_t s) {
    return A->dtype == SPC5_F64 ? dispatch<double>(A, val, x, y, s)
                                : dispatch<float>(A, val, x, y, s);
}

template <typename T>
static hipError_t launch_csr_t(const spc5_csr *A, const void *x, void *y, hipStream_t s) {
    const int64_t ntiles = (A->nrows + A->rpt - 1) / A->rpt;
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL((k_spmv<T, 1, 1, true>), dim3((unsigned)ntiles), dim3(kWave), 0, s,
                       A->nrows, A->nrows, A->rpt, ntiles, remap_enabled(), A->rowptr,
                       A->colidx, (const uint8_t *)nullptr, (const T *)A->val,
                       (const int32_t *)nullptr, (const T *)x, (T *)y);
    return hipGetLastError();
}

hipError_t launch_csr_spmv(const spc5_csr *A, const void *x, void *y, hipStream_t s) {
    return A->dtype == SPC5_F64 ? launch_csr_t<double>(A, x, y, s)
                                : launch_csr_t<float>(A, x, y, s);
}

}  // namespace spc5
