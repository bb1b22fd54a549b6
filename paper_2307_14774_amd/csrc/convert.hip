// CSR -> SPC5 beta(r,c) conversion on the device (Section 2.4 of
// arXiv 2307.14774).
//
// Blocking rule: inside a panel of r rows, a block is anchored at the
// smallest column not yet covered among the panel's rows and takes, in every
// row, the nonzeros of columns [anchor, anchor+c).  Each panel is blocked
// independently by one thread (two passes: count, then fill after an
// exclusive scan of the per-panel counts gives every panel its first block);
// for r = 1 a row longer than kLongRow nonzeros is blocked by a whole
// wavefront instead (k_block_long_rows), with the same greedy rule.
// A panel's packed values occupy exactly the CSR value range of its rows, so
// the fill pass writes them at rowptr[first row of the panel] onward without
// any further scan.
#include "spc5_internal.h"
#include "wave.h"

#include <climits>
#include <vector>

namespace spc5 {

constexpr int kMaxR = 8;
constexpr int64_t kLongRow = 2048;

template <bool FILL, typename T, typename MT>
__global__ __launch_bounds__(256) void k_block_panels(
    int64_t nrows, int64_t npanels, int r, int c, const int64_t *__restrict__ rowptr,
    const int32_t *__restrict__ colidx, const T *__restrict__ vin,
    int64_t *__restrict__ count, const int64_t *__restrict__ bptr,
    int32_t *__restrict__ bcol, MT *__restrict__ masks, T *__restrict__ vout)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npanels) return;
    if (r == 1 && rowptr[p + 1] - rowptr[p] > kLongRow) return;    // k_block_long_rows
    const int64_t row0 = p * r;
    const int nr = (int)min((int64_t)r, nrows - row0);
    const int64_t kNone = INT64_MAX;
    int64_t cur[kMaxR], end[kMaxR], col[kMaxR];
#pragma unroll
    for (int i = 0; i < kMaxR; ++i) {
        cur[i] = i < nr ? rowptr[row0 + i] : 0;
        end[i] = i < nr ? rowptr[row0 + i + 1] : 0;
        col[i] = cur[i] < end[i] ? (int64_t)colidx[cur[i]] : kNone;
    }
    int64_t nb = 0;
    const int64_t first = FILL ? bptr[p] : 0;
    int64_t vo = FILL ? rowptr[row0] : 0;
    for (;;) {
        int64_t anchor = kNone;
#pragma unroll
        for (int i = 0; i < kMaxR; ++i) anchor = col[i] < anchor ? col[i] : anchor;
        if (anchor == kNone) break;
        const int64_t lim = anchor + c;
        if (FILL) bcol[first + nb] = (int32_t)anchor;
#pragma unroll
        for (int i = 0; i < kMaxR; ++i) {
            unsigned m = 0;
            while (col[i] < lim) {
                m |= 1u << (unsigned)(col[i] - anchor);
                if (FILL) vout[vo++] = vin[cur[i]];
                ++cur[i];
                col[i] = cur[i] < end[i] ? (int64_t)colidx[cur[i]] : kNone;
            }
            if (FILL && i < r) masks[(first + nb) * r + i] = (MT)m;
        }
        ++nb;
    }
    if (!FILL) count[p] = nb;
}

// beta(1,c) rows longer than kLongRow nonzeros, one wavefront each.  The
// lanes hold 64 consecutive columns at a time; the columns below the open
// block's end join it (their bits OR-reduced into its mask), and the first
// column at or past the end opens the next block -- the greedy rule of the
// thread walk, so the blocks are the same.  With r = 1 the packed values are
// the row's CSR values in order.
template <bool FILL, typename T, typename MT>
__global__ __launch_bounds__(256) void k_block_long_rows(
    int64_t nrows, int c, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
    const T *__restrict__ vin, int64_t *__restrict__ count, const int64_t *__restrict__ bptr,
    int32_t *__restrict__ bcol, MT *__restrict__ masks, T *__restrict__ vout)
{
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (row >= nrows) return;
    const int64_t b = rowptr[row], e = rowptr[row + 1];
    if (e - b <= kLongRow) return;    // uniform over the wavefront
    const int lane = lane_id();
    const int64_t first = FILL ? bptr[row] : 0;
    int64_t nb = 0, anchor = 0, lim = INT64_MIN;
    unsigned m = 0;
    bool open = false;
    // kLongGroup chunks of 64 columns are loaded together, so one memory
    // latency is paid per group rather than per chunk
    constexpr int kLongGroup = 8;
    for (int64_t gbase = b; gbase < e; gbase += kWave * kLongGroup) {
        int64_t xg[kLongGroup];
        T vg[kLongGroup];
#pragma unroll
        for (int q = 0; q < kLongGroup; ++q) {
            const int64_t k = gbase + q * kWave + lane;
            xg[q] = k < e ? (int64_t)colidx[k] : INT64_MAX;
            if (FILL) vg[q] = k < e ? vin[k] : T(0);
        }
#pragma unroll
        for (int q = 0; q < kLongGroup; ++q) {
            const int64_t k = gbase + q * kWave + lane;
            const bool valid = k < e;
            const int64_t x = xg[q];
            if (FILL && valid) vout[k] = vg[q];
            uint64_t pend = __ballot(valid);
            while (pend) {
                const uint64_t cov = __ballot(valid && x < lim) & pend;
                if (FILL) {
                    unsigned bit = ((cov >> lane) & 1ull) ? 1u << (unsigned)(x - anchor) : 0u;
                    for (int d = 1; d < kWave; d <<= 1) bit |= __shfl_xor(bit, d);
                    m |= bit;
                }
                pend &= ~cov;
                if (pend) {
                    if (open) {
                        if (FILL && lane == 0) {
                            bcol[first + nb] = (int32_t)anchor;
                            masks[first + nb] = (MT)m;
                        }
                        ++nb;
                    }
                    anchor = __shfl(x, __ffsll((unsigned long long)pend) - 1);
                    lim = anchor + c;
                    m = 0;
                    open = true;
                }
            }
        }
    }
    if (open) {
        if (FILL && lane == 0) {
            bcol[first + nb] = (int32_t)anchor;
            masks[first + nb] = (MT)m;
        }
        ++nb;
    }
    if (!FILL && lane == 0) count[row] = nb;
}

// Both walks over all panels (the long-row one only for r = 1).
template <bool FILL, typename T, typename MT>
static void launch_walk(const spc5_matrix *A, const int64_t *rowptr, const int32_t *colidx,
                        const T *vin, int64_t *count, const int64_t *bptr, int32_t *bcol,
                        MT *masks, T *vout, hipStream_t s) {
    const int64_t grid = (A->npanels + 255) / 256;
    if (grid == 0) return;
    hipLaunchKernelGGL((k_block_panels<FILL, T, MT>), dim3((unsigned)grid), dim3(256), 0, s,
                       A->nrows, A->npanels, A->r, A->c, rowptr, colidx, vin, count, bptr, bcol,
                       masks, vout);
    if (A->r == 1)
        hipLaunchKernelGGL((k_block_long_rows<FILL, T, MT>),
                           dim3((unsigned)((A->nrows * kWave + 255) / 256)), dim3(256), 0, s,
                           A->nrows, A->c, rowptr, colidx, vin, count, bptr, bcol, masks, vout);
}

// ---- exclusive scan of int64 counts: out[0..n] with out[n] = total ----------
constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanChunk = kScanThreads * kScanPer;

__device__ int64_t block_excl_scan(int64_t v, int64_t *sh, int64_t *total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const int64_t o = t >= d ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += o;
        __syncthreads();
    }
    const int64_t incl = sh[t];
    *total = sh[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int64_t *in, int64_t n,
                                                              int64_t *part) {
    __shared__ int64_t sh[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x * kScanPer;
    int64_t s = 0;
    for (int e = 0; e < kScanPer; ++e)
        if (base + e < n) s += in[base + e];
    int64_t tot;
    block_excl_scan(s, sh, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_parts(int64_t *part, int64_t nparts) {
    __shared__ int64_t sh[kScanThreads];
    int64_t carry = 0;
    for (int64_t base = 0; base < nparts; base += kScanThreads) {
        const int64_t idx = base + threadIdx.x;
        const int64_t v = idx < nparts ? part[idx] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(v, sh, &tot);
        if (idx < nparts) part[idx] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int64_t *in, int64_t n,
                                                             const int64_t *part,
                                                             int64_t *out) {
    __shared__ int64_t sh[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x * kScanPer;
    int64_t s = 0;
    for (int e = 0; e < kScanPer; ++e)
        if (base + e < n) s += in[base + e];
    int64_t tot;
    int64_t run = part[blockIdx.x] + block_excl_scan(s, sh, &tot);
    for (int e = 0; e < kScanPer; ++e) {
        if (base + e < n) {
            out[base + e] = run;
            run += in[base + e];
            if (base + e == n - 1) out[n] = run;
        }
    }
}

// blk_ptr (int32) and the value offset of every panel start.
__global__ void k_narrow(int64_t npanels, int64_t nrows, int r, const int64_t *bptr64,
                         const int64_t *rowptr, int32_t *bptr, int32_t *pval) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > npanels) return;
    bptr[p] = (int32_t)bptr64[p];
    const int64_t row = p * r < nrows ? p * r : nrows;
    pval[p] = (int32_t)rowptr[row];
}

// Every kColSample-th nonzero counted by column: a column with many entries
// (a popular node of a graph) reaches kHotSamples counts when it holds about
// kColSample*kHotSamples of them, and then raises the flag (once per column,
// so the flag itself sees no contention).
// The counters are at most kColBuckets, columns folded onto them by
// remainder: a fold can only add a false alarm (the aggregating transpose is
// then used where it was not needed, still correct), and with fewer than 2^31
// nonzeros no bucket of a uniform matrix comes near kHotSamples.
constexpr int64_t kColSample = 64;
constexpr int kHotSamples = 64;
constexpr int64_t kColBuckets = 1 << 20;

__global__ void k_col_sample(int64_t nnz, const int32_t *__restrict__ colidx, int nbuckets,
                             int *cnt, int *flag) {
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kColSample;
    if (k < nnz && atomicAdd(&cnt[colidx[k] % nbuckets], 1) + 1 == kHotSamples) *flag = 1;
}

__global__ void k_max(const int64_t *in, int64_t n, unsigned long long *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicMax(out, (unsigned long long)in[i]);
}

__global__ void k_zero(uint32_t *p, int64_t nwords, uint8_t *tail, int ntail) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nwords) p[i] = 0u;
    if (i < ntail) tail[i] = 0;
}

// 16 bytes per thread over a 16-byte aligned range.
__global__ void k_zero16(uint4 *p, int64_t n16) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

hipError_t zero_fill(void *p, int64_t n, int elem_bytes, hipStream_t s) {
    int64_t bytes = n * elem_bytes;
    if (bytes <= 0) return hipSuccess;
    if (((uintptr_t)p & 15) == 0 && bytes >= 4096) {
        // the 16-byte aligned bulk, then the rest word by word
        const int64_t n16 = bytes / 16;
        hipLaunchKernelGGL(k_zero16, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, s,
                           (uint4 *)p, n16);
        p = (uint8_t *)p + n16 * 16;
        bytes -= n16 * 16;
        if (bytes == 0) return hipGetLastError();
    }
    const int64_t nwords = bytes / 4;
    const int ntail = (int)(bytes - nwords * 4);
    const int64_t work = nwords > ntail ? nwords : ntail;
    const int64_t grid = (work + 255) / 256;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)grid), dim3(256), 0, s, (uint32_t *)p, nwords,
                       (uint8_t *)p + nwords * 4, ntail);
    return hipGetLastError();
}

hipError_t excl_scan_i64(const int64_t *in, int64_t n, int64_t *out, hipStream_t s,
                         int64_t **scratch) {
    hipError_t e;
    if (n == 0) return zero_fill(out, 1, 8, s);
    const int64_t nparts = (n + kScanChunk - 1) / kScanChunk;
    if ((e = hipMalloc((void **)scratch, (size_t)nparts * 8)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nparts), dim3(kScanThreads), 0, s, in, n,
                       *scratch);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kScanThreads), 0, s, *scratch, nparts);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nparts), dim3(kScanThreads), 0, s, in, n,
                       *scratch, out);
    return hipGetLastError();
}

template <typename T, typename MT>
static hipError_t launch_block(bool fill, spc5_matrix *A, const int64_t *rowptr,
                               const int32_t *colidx, const void *vin, int64_t *count,
                               const int64_t *bptr, hipStream_t s) {
    if (fill)
        launch_walk<true, T, MT>(A, rowptr, colidx, (const T *)vin, count, bptr, A->blk_col,
                                 (MT *)A->masks, (T *)A->val, s);
    else
        launch_walk<false, T, MT>(A, rowptr, colidx, (const T *)vin, count, bptr, nullptr,
                                  nullptr, nullptr, s);
    return hipGetLastError();
}

static hipError_t launch_block_any(bool fill, spc5_matrix *A, const int64_t *rowptr,
                                   const int32_t *colidx, const void *vin, int64_t *count,
                                   const int64_t *bptr, hipStream_t s) {
    if (A->dtype == SPC5_F64)
        return A->mask_bytes == 1
                   ? launch_block<double, uint8_t>(fill, A, rowptr, colidx, vin, count, bptr, s)
                   : launch_block<double, uint16_t>(fill, A, rowptr, colidx, vin, count, bptr,
                                                    s);
    return A->mask_bytes == 1
               ? launch_block<float, uint8_t>(fill, A, rowptr, colidx, vin, count, bptr, s)
               : launch_block<float, uint16_t>(fill, A, rowptr, colidx, vin, count, bptr, s);
}

int count_blocks_device(const int64_t *d_rowptr, const int32_t *d_colidx, int64_t nrows, int r,
                        int c, int64_t *nblocks) {
    spc5_matrix tmp;
    tmp.nrows = nrows;
    tmp.npanels = (nrows + r - 1) / r;
    tmp.r = r;
    tmp.c = c;
    tmp.mask_bytes = c <= 8 ? 1 : 2;
    hipStream_t s = nullptr;
    hipError_t e;
    int64_t *count = nullptr, *bptr64 = nullptr, *scratch = nullptr;
    const size_t np1 = (size_t)tmp.npanels + 1;
    int st = SPC5_OK;
    if ((e = hipMalloc((void **)&count, np1 * 8)) != hipSuccess ||
        (e = hipMalloc((void **)&bptr64, np1 * 8)) != hipSuccess ||
        (e = launch_block_any(false, &tmp, d_rowptr, d_colidx, nullptr, count, nullptr, s)) !=
            hipSuccess ||
        (e = excl_scan_i64(count, tmp.npanels, bptr64, s, &scratch)) != hipSuccess ||
        (e = hipMemcpy(nblocks, bptr64 + tmp.npanels, 8, hipMemcpyDeviceToHost)) != hipSuccess)
        st = hip_fail(e, "counting blocks");
    if (count) (void)hipFree(count);
    if (bptr64) (void)hipFree(bptr64);
    if (scratch) (void)hipFree(scratch);
    return st;
}

int convert_on_device(spc5_matrix *A, const int64_t *d_rowptr, const int32_t *d_colidx,
                      const void *d_values, const int32_t *d_payload,
                      int32_t *d_payload_out) {
    hipStream_t s = nullptr;
    hipError_t e;
    int64_t *count = nullptr, *bptr64 = nullptr, *scratch = nullptr;
    int status = SPC5_OK;
    const int vb = A->dtype == SPC5_F64 ? 8 : 4;
    auto cleanup = [&]() {
        if (count) (void)hipFree(count);
        if (bptr64) (void)hipFree(bptr64);
        if (scratch) (void)hipFree(scratch);
    };
    const size_t np1 = (size_t)A->npanels + 1;
    if ((e = hipMalloc((void **)&count, np1 * 8)) != hipSuccess ||
        (e = hipMalloc((void **)&bptr64, np1 * 8)) != hipSuccess) {
        cleanup();
        return hip_fail(e, "allocating conversion scratch");
    }
    if ((e = launch_block_any(false, A, d_rowptr, d_colidx, d_values, count, nullptr, s)) !=
            hipSuccess ||
        (e = excl_scan_i64(count, A->npanels, bptr64, s, &scratch)) != hipSuccess) {
        cleanup();
        return hip_fail(e, "counting blocks");
    }
    // longest panel (for the kernel choice): reuse the first partial slot
    unsigned long long *dmax = (unsigned long long *)scratch;
    if (A->npanels > 0) {
        if ((e = zero_fill(dmax, 1, 8, s)) != hipSuccess) { cleanup(); return hip_fail(e, "max"); }
        hipLaunchKernelGGL(k_max, dim3((unsigned)((A->npanels + 255) / 256)), dim3(256), 0, s,
                           count, A->npanels, dmax);
    }
    int64_t nblocks = 0;
    unsigned long long maxb = 0;
    if ((e = hipMemcpy(&nblocks, bptr64 + A->npanels, 8, hipMemcpyDeviceToHost)) !=
            hipSuccess ||
        (A->npanels > 0 &&
         (e = hipMemcpy(&maxb, dmax, 8, hipMemcpyDeviceToHost)) != hipSuccess)) {
        cleanup();
        return hip_fail(e, "reading the block count");
    }
    A->max_panel_blocks = (int64_t)maxb;
    // columns with thousands of entries: the atomic transpose aggregates them
    A->hot_cols = false;
    const int64_t nnz = A->nnz;
    if (nnz >= kColSample * kHotSamples && A->ncols > 0) {
        int *cnt = nullptr;
        int hot = 0;
        const int64_t ns = (nnz + kColSample - 1) / kColSample;
        const int nbk = (int)std::min<int64_t>(A->ncols, kColBuckets);
        if ((e = hipMalloc((void **)&cnt, (size_t)(nbk + 1) * 4)) != hipSuccess ||
            (e = zero_fill(cnt, nbk + 1, 4, s)) != hipSuccess) {
            if (cnt) (void)hipFree(cnt);
            cleanup();
            return hip_fail(e, "sampling column lengths");
        }
        hipLaunchKernelGGL(k_col_sample, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, s, nnz,
                           d_colidx, nbk, cnt, cnt + nbk);
        if ((e = hipGetLastError()) != hipSuccess ||
            (e = hipMemcpy(&hot, cnt + nbk, 4, hipMemcpyDeviceToHost)) != hipSuccess) {
            (void)hipFree(cnt);
            cleanup();
            return hip_fail(e, "sampling column lengths");
        }
        (void)hipFree(cnt);
        A->hot_cols = hot != 0;
    }
    if (nblocks >= ((int64_t)1 << 31)) {
        cleanup();
        return fail(SPC5_EUNSUPPORTED, "nblocks = %lld does not fit int32 device indices",
                    (long long)nblocks);
    }
    A->nblocks = nblocks;
    const size_t nb_alloc = (size_t)(nblocks > 0 ? nblocks : 1);
    const size_t nnz_alloc = (size_t)(A->nnz > 0 ? A->nnz : 1);
    // kPad trailing bytes: the staged kernel reads whole 16-byte vectors, so
    // the last vector of an array may extend past its last element
    if ((e = hipMalloc((void **)&A->blk_ptr, np1 * 4 + kPad)) != hipSuccess ||
        (e = hipMalloc((void **)&A->panel_val, np1 * 4 + kPad)) != hipSuccess ||
        (e = hipMalloc((void **)&A->blk_col, nb_alloc * 4 + kPad)) != hipSuccess ||
        (e = hipMalloc(&A->masks, nb_alloc * A->r * A->mask_bytes + kPad)) != hipSuccess ||
        (e = hipMalloc(&A->val, nnz_alloc * vb + kPad)) != hipSuccess) {
        cleanup();
        return hip_fail(e, "allocating SPC5 arrays");
    }
    if ((e = launch_block_any(true, A, d_rowptr, d_colidx, d_values, nullptr, bptr64, s)) !=
        hipSuccess) {
        cleanup();
        return hip_fail(e, "filling SPC5 arrays");
    }
    if (d_payload && d_payload_out && A->npanels > 0) {
        // the same walk once more with an int32 payload in place of the
        // values (anchors and masks are rewritten with identical contents)
        if (A->mask_bytes == 1)
            launch_walk<true, int32_t, uint8_t>(A, d_rowptr, d_colidx, d_payload, nullptr, bptr64,
                                                A->blk_col, (uint8_t *)A->masks, d_payload_out, s);
        else
            launch_walk<true, int32_t, uint16_t>(A, d_rowptr, d_colidx, d_payload, nullptr,
                                                 bptr64, A->blk_col, (uint16_t *)A->masks,
                                                 d_payload_out, s);
        if ((e = hipGetLastError()) != hipSuccess) {
            cleanup();
            return hip_fail(e, "placing the payload");
        }
    }
    hipLaunchKernelGGL(k_narrow, dim3((unsigned)((np1 + 255) / 256)), dim3(256), 0, s,
                       A->npanels, A->nrows, A->r, bptr64, d_rowptr, A->blk_ptr,
                       A->panel_val);
    if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
        status = hip_fail(e, "finishing the conversion");
    cleanup();
    return status;
}

}  // namespace spc5
