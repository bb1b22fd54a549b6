// Y = A X with several right-hand sides over SPC5 beta(r,c) storage.
// Same walk as the forward kernel; every lane keeps K accumulators (one per
// right-hand side of the chunk) and reads the K contiguous entries of row
// anchor+k of X for each set mask bit, so the matrix is streamed once per
// chunk of K right-hand sides instead of once per vector.
#include "spc5_internal.h"
#include "tile.h"

namespace spc5 {

constexpr int kSpmmTile = 1024;   // LDS row accumulators per wavefront (ppt*R*K)

template <typename T, int R, int C, int K>
__global__ __launch_bounds__(kWave) void k_spmm(
    int64_t npanels, int64_t nrows, int ppt, int64_t ntiles,
    const int32_t *__restrict__ blk_ptr, const int32_t *__restrict__ blk_col,
    const typename MaskOf<C>::type *__restrict__ masks, const T *__restrict__ val,
    const int32_t *__restrict__ panel_val, const T *__restrict__ X, T *__restrict__ Y, int ld)
{
    constexpr int BPS = kWave / R;
    constexpr int LANES = BPS * R;
    __shared__ T ytile[kSpmmTile];
    const int lane = lane_id();
    const TileCtx t = tile_begin(xcd_remap(blockIdx.x, ntiles), ppt, npanels, blk_ptr);
    for (int q = lane; q < t.np * R * K; q += kWave) ytile[q] = T(0);
    __syncthreads();
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
        T acc[K];
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = T(0);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            if ((m >> k) & 1u) {
                const T v = val[j];
                const T *xr = X + (int64_t)(col0 + k) * ld;
#pragma unroll
                for (int q = 0; q < K; ++q) acc[q] = fma(v, xr[q], acc[q]);
                ++j;
            }
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

extern "C" {

int spc5_batch_create(int nmat, spc5_matrix *const *mats, spc5_batch **out) {
    (void)nmat; (void)mats;
    if (out) *out = nullptr;
    return spc5::fail(SPC5_EUNSUPPORTED, "batched launch not available yet");
}

void spc5_batch_free(spc5_batch *B) { (void)B; }

int spc5_batch_spmm(spc5_batch *B, int nrhs, const void *const *X, void *const *Y,
                    void *stream) {
    (void)B; (void)nrhs; (void)X; (void)Y; (void)stream;
    return spc5::fail(SPC5_EUNSUPPORTED, "batched launch not available yet");
}

}  // extern "C"
