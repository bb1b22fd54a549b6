// Y = A X with several right-hand sides over SPC5 beta(r,c) storage.
// Same walk as the forward kernel; every lane keeps K accumulators (one per
// right-hand side of the chunk) and reads the K contiguous entries of row
// anchor+k of X for each set mask bit, so the matrix is streamed once per
// chunk of K right-hand sides instead of once per vector.
#include "spc5_internal.h"
#include "spmm_tile.h"

namespace spc5 {

template <typename T, int R, int C, int K>
__global__ __launch_bounds__(kWave) void k_spmm(
    int64_t npanels, int64_t nrows, int ppt, int64_t ntiles,
    const int32_t *__restrict__ blk_ptr, const int32_t *__restrict__ blk_col,
    const typename MaskOf<C>::type *__restrict__ masks, const T *__restrict__ val,
    const int32_t *__restrict__ panel_val, const T *__restrict__ X, T *__restrict__ Y, int ld)
{
    __shared__ T ytile[kSpmmTile];
    spmm_tile<T, R, C, K>(xcd_remap(blockIdx.x, ntiles), ppt, npanels, nrows, blk_ptr, blk_col,
                          masks, val, panel_val, X, Y, ld, ytile);
}

template <typename T, int R, int C, int K>
static hipError_t launch_k(const spc5_matrix *A, const T *X, T *Y, int ld, hipStream_t s) {
    int ppt = A->ppt;
    const int cap = kSpmmTile / (R * K);
    if (ppt > cap) ppt = cap;
    if (ppt < 1) ppt = 1;
    const int64_t ntiles = (A->npanels + ppt - 1) / ppt;
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL((k_spmm<T, R, C, K>), dim3((unsigned)ntiles), dim3(kWave), 0, s,
                       A->npanels, A->nrows, ppt, ntiles, A->blk_ptr, A->blk_col,
                       (const typename MaskOf<C>::type *)A->masks, (const T *)A->val,
                       A->panel_val, X, Y, ld);
    return hipGetLastError();
}

template <typename T, int R, int C>
static hipError_t launch_rc(const spc5_matrix *A, int nrhs, const T *X, T *Y, hipStream_t s) {
    // split nrhs into chunks of 16, 8, 4, 2, 1 columns
    int t0 = 0;
    while (t0 < nrhs) {
        const int left = nrhs - t0;
        hipError_t e;
        int k;
        if (left >= 16) { k = 16; e = launch_k<T, R, C, 16>(A, X + t0, Y + t0, nrhs, s); }
        else if (left >= 8) { k = 8; e = launch_k<T, R, C, 8>(A, X + t0, Y + t0, nrhs, s); }
        else if (left >= 4) { k = 4; e = launch_k<T, R, C, 4>(A, X + t0, Y + t0, nrhs, s); }
        else if (left >= 2) { k = 2; e = launch_k<T, R, C, 2>(A, X + t0, Y + t0, nrhs, s); }
        else { k = 1; e = launch_k<T, R, C, 1>(A, X + t0, Y + t0, nrhs, s); }
        if (e != hipSuccess) return e;
        t0 += k;
    }
    return hipSuccess;
}

template <typename T>
static hipError_t spmm_dispatch(const spc5_matrix *A, int nrhs, const void *X, void *Y,
                                hipStream_t s) {
#define SPC5_CASE(RR, CC) \
    case RR * 100 + CC: return launch_rc<T, RR, CC>(A, nrhs, (const T *)X, (T *)Y, s);
#define SPC5_ROW(RR) SPC5_CASE(RR, 4) SPC5_CASE(RR, 8) SPC5_CASE(RR, 16)
    switch (A->r * 100 + (A->c <= 4 ? 4 : (A->c <= 8 ? 8 : 16))) {
        SPC5_ROW(1) SPC5_ROW(2) SPC5_ROW(3) SPC5_ROW(4)
        SPC5_ROW(5) SPC5_ROW(6) SPC5_ROW(7) SPC5_ROW(8)
        default: return hipErrorInvalidValue;
    }
#undef SPC5_ROW
#undef SPC5_CASE
}

hipError_t launch_spmm(const spc5_matrix *A, int nrhs, const void *X, void *Y,
                       hipStream_t s) {
    return A->dtype == SPC5_F64 ? spmm_dispatch<double>(A, nrhs, X, Y, s)
                                : spmm_dispatch<float>(A, nrhs, X, Y, s);
}

}  // namespace spc5

