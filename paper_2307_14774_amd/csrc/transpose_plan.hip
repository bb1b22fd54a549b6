// Transposed-product plan: x_bar = A^T y_bar as a forward product over A^T.
//
// The masked scatter of the backward kernel adds every nonzero into x_bar
// with a float atomic; when many rows share a column (a popular node of a
// graph) those atomics serialise on one address.  The plan removes them: A^T
// is held in SPC5 beta(r,c) storage of its own (built once, on the device),
// and the transpose becomes the forward kernel run over A^T -- coalesced
// streams, the single x load per block, no atomics, bit-reproducible.
//
// Build (all on the device):
//  1. expand A's packed values into (row, column) pairs in packed order;
//  2. stable radix sort of the packed indices by column: inside one column
//     the packed order is the row order (a panel's block windows are
//     disjoint and increasing, and a block lists its rows in order), so the
//     result is A^T in CSR form with sorted column indices;
//  3. convert that CSR to beta(r,c) with the ordinary conversion, placing
//     A's values and, as an int32 payload, A's packed index of every entry:
//     the permutation perm (A^T's value q is A's value perm[q]);
//  4. split perm for caller-supplied values theta.  A single gather
//     theta[perm[q]] reads one scattered word per cache line (perm jumps
//     across all of A for every row of A^T).  Instead A^T's packed order is
//     cut into buckets of kPermBucket consecutive values, A's values are
//     scattered into staging slots grouped by bucket (slot order inside a
//     bucket: A's packed order), and each bucket is then gathered from its
//     own slots -- reads coalesced in the first pass, each bucket's window
//     small enough to stay in L2 in the second.
#include "spc5_internal.h"
#include "wave.h"

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include <algorithm>

namespace spc5 {

// Row and column of every packed value of A; one thread per panel walks its
// blocks in storage order.
template <typename MT>
__global__ void k_expand(int64_t npanels, int r, const int32_t *__restrict__ blk_ptr,
                         const int32_t *__restrict__ blk_col, const MT *__restrict__ masks,
                         const int32_t *__restrict__ panel_val, int32_t *__restrict__ row_of,
                         int32_t *__restrict__ col_of) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npanels) return;
    int v = panel_val[p];
    for (int b = blk_ptr[p]; b < blk_ptr[p + 1]; ++b) {
        const int c0 = blk_col[b];
        for (int i = 0; i < r; ++i) {
            unsigned m = masks[(int64_t)b * r + i];
            while (m) {
                const int k = __ffs(m) - 1;
                row_of[v] = (int32_t)(p * r + i);
                col_of[v] = c0 + k;
                ++v;
                m &= m - 1u;
            }
        }
    }
}

// rowptr of A^T from the sorted column keys: rowptr[c] = first index whose
// key is >= c.  Thread i covers the columns in (key[i-1], key[i]].
__global__ void k_rowptr_from_sorted(int64_t nnz, int64_t ncols, const int32_t *__restrict__ key,
                                     int64_t *__restrict__ rowptr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > nnz) return;
    const int64_t lo = i > 0 ? (int64_t)key[i - 1] : -1;
    const int64_t hi = i < nnz ? (int64_t)key[i] : ncols;
    for (int64_t c = lo + 1; c <= hi; ++c) rowptr[c] = i;
}

// colidx of A^T (A's rows) and its values, in the sorted order.
template <typename T>
__global__ void k_gather_csr(int64_t nnz, const int32_t *__restrict__ idx,
                             const int32_t *__restrict__ row_of, const T *__restrict__ val,
                             int32_t *__restrict__ colidx_t, T *__restrict__ val_t) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nnz) return;
    const int32_t k = idx[i];
    colidx_t[i] = row_of[k];
    val_t[i] = val[k];
}

// Values of A^T per bucket of the two-pass value move: the staging window of
// a bucket (512 KiB in FP32) stays in L2 while its outputs are gathered.
constexpr int64_t kPermBucket = 131072;

// key[perm[q]] = bucket of q: for every packed value of A, the bucket of its
// position in A^T.
__global__ void k_bucket_keys(int64_t nnz, const int32_t *__restrict__ perm,
                              int32_t *__restrict__ key) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnz) key[perm[q]] = (int32_t)(q / kPermBucket);
}

// slot[order[t]] = t: the staging slot of each value of A.
__global__ void k_invert(int64_t nnz, const int32_t *__restrict__ order,
                         int32_t *__restrict__ slot) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nnz) slot[order[t]] = (int32_t)t;
}

// perm[q] <- slot[perm[q]] (in place): the staging slot holding A^T's value q.
__global__ void k_compose(int64_t nnz, const int32_t *__restrict__ slot,
                          int32_t *__restrict__ perm) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnz) perm[q] = slot[perm[q]];
}

// Pass 1: stage[slot[i]] = in[i].  Each workgroup moves a contiguous chunk of
// kMoveChunk values of A, so its writes into one bucket's slots form one
// contiguous run (about kMoveChunk / number of buckets values) that a single
// L2 assembles into whole lines.
constexpr int64_t kMoveChunk = 16384;

template <typename T>
__global__ __launch_bounds__(256) void k_stage_scatter(int64_t n, const int32_t *__restrict__ slot,
                                                       const T *__restrict__ in,
                                                       T *__restrict__ stage) {
    const int64_t i0 = (int64_t)blockIdx.x * kMoveChunk;
    const int64_t i1 = min(i0 + kMoveChunk, n);
#pragma unroll 8
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) stage[slot[i]] = in[i];
}

// Pass 2: out[q] = stage[src[q]], src[q] inside q's bucket.  Workgroups reach
// the kXcds XCDs round robin; XCD x gathers buckets x, x + kXcds, ... and its
// kGatherPerXcd workgroups split each bucket, so an XCD's L2 holds one
// bucket's window at a time.
constexpr int kGatherPerXcd = 128;

template <typename T>
__global__ __launch_bounds__(256) void k_stage_gather(int64_t n, const int32_t *__restrict__ src,
                                                      const T *__restrict__ stage,
                                                      T *__restrict__ out) {
    constexpr int64_t share = kPermBucket / kGatherPerXcd;
    const int x = (int)(blockIdx.x % kXcds), j = (int)(blockIdx.x / kXcds);
    const int64_t nb = (n + kPermBucket - 1) / kPermBucket;
    for (int64_t b = x; b < nb; b += kXcds) {
        const int64_t q0 = b * kPermBucket + j * share;
        const int64_t q1 = min(q0 + share, n);
        for (int64_t q = q0 + threadIdx.x; q < q1; q += 256) out[q] = stage[src[q]];
    }
}

template <typename T>
static void launch_move(const spc5_matrix *A, const T *vals, hipStream_t s) {
    const int64_t n = A->nnz;
    hipLaunchKernelGGL(k_stage_scatter<T>, dim3((unsigned)((n + kMoveChunk - 1) / kMoveChunk)),
                       dim3(256), 0, s, n, A->tr_scatter, vals, (T *)A->tr_stage);
    hipLaunchKernelGGL(k_stage_gather<T>, dim3(kXcds * kGatherPerXcd), dim3(256), 0, s, n,
                       A->tr_gather, (const T *)A->tr_stage, (T *)A->tr_vals);
}

int build_transpose_plan(spc5_matrix *A, int r, int c) {
    if (A->tr) return SPC5_OK;
    hipStream_t s = nullptr;
    const int64_t nnz = A->nnz;
    const int vb = A->dtype == SPC5_F64 ? 8 : 4;
    int32_t *row_of = nullptr, *col_of = nullptr, *key_s = nullptr, *idx_s = nullptr;
    int32_t *colidx_t = nullptr;
    int64_t *rowptr_t = nullptr;
    void *val_t = nullptr, *tmp = nullptr;
    spc5_matrix *T = nullptr;
    int32_t *perm = nullptr, *scat = nullptr;
    void *gbuf = nullptr, *stage = nullptr;
    size_t tmp_bytes = 0;
    auto cleanup = [&]() {
        for (void *p : {(void *)row_of, (void *)col_of, (void *)key_s, (void *)idx_s,
                        (void *)colidx_t, (void *)rowptr_t, val_t, tmp})
            if (p) (void)hipFree(p);
    };
    auto fail_all = [&](int st) {
        cleanup();
        free_matrix(T);
        for (void *p : {(void *)perm, (void *)scat, gbuf, stage})
            if (p) (void)hipFree(p);
        return st;
    };
    const size_t nz = (size_t)std::max<int64_t>(nnz, 1);
    hipError_t e;
    if ((e = hipMalloc((void **)&row_of, nz * 4)) != hipSuccess ||
        (e = hipMalloc((void **)&col_of, nz * 4)) != hipSuccess ||
        (e = hipMalloc((void **)&key_s, nz * 4)) != hipSuccess ||
        (e = hipMalloc((void **)&idx_s, nz * 4)) != hipSuccess ||
        (e = hipMalloc((void **)&colidx_t, nz * 4)) != hipSuccess ||
        (e = hipMalloc((void **)&rowptr_t, (size_t)(A->ncols + 1) * 8)) != hipSuccess ||
        (e = hipMalloc(&val_t, nz * vb)) != hipSuccess)
        return fail_all(hip_fail(e, "allocating the transpose plan"));
    // 1. (row, column) of every packed value
    if (A->npanels > 0) {
        const unsigned grid = (unsigned)((A->npanels + 255) / 256);
        if (A->mask_bytes == 1)
            hipLaunchKernelGGL(k_expand<uint8_t>, dim3(grid), dim3(256), 0, s, A->npanels, A->r,
                               A->blk_ptr, A->blk_col, (const uint8_t *)A->masks, A->panel_val,
                               row_of, col_of);
        else
            hipLaunchKernelGGL(k_expand<uint16_t>, dim3(grid), dim3(256), 0, s, A->npanels,
                               A->r, A->blk_ptr, A->blk_col, (const uint16_t *)A->masks,
                               A->panel_val, row_of, col_of);
        if ((e = hipGetLastError()) != hipSuccess)
            return fail_all(hip_fail(e, "expanding the matrix"));
    }
    // 2. stable sort of the packed indices by column
    if (nnz > 0) {
        unsigned bits = 1;
        while (bits < 31 && ((int64_t)1 << bits) < A->ncols) ++bits;
        rocprim::counting_iterator<int32_t> iota(0);
        if ((e = rocprim::radix_sort_pairs(nullptr, tmp_bytes, col_of, key_s, iota, idx_s,
                                           (size_t)nnz, 0u, bits, s)) != hipSuccess ||
            (e = hipMalloc(&tmp, std::max<size_t>(tmp_bytes, 16))) != hipSuccess ||
            (e = rocprim::radix_sort_pairs(tmp, tmp_bytes, col_of, key_s, iota, idx_s,
                                           (size_t)nnz, 0u, bits, s)) != hipSuccess)
            return fail_all(hip_fail(e, "sorting by column"));
    }
    // 3. A^T in CSR form, then beta(r,c) with the permutation as payload
    hipLaunchKernelGGL(k_rowptr_from_sorted, dim3((unsigned)((nnz + 1 + 255) / 256)), dim3(256),
                       0, s, nnz, A->ncols, key_s, rowptr_t);
    if (nnz > 0) {
        const unsigned grid = (unsigned)((nnz + 255) / 256);
        if (A->dtype == SPC5_F64)
            hipLaunchKernelGGL(k_gather_csr<double>, dim3(grid), dim3(256), 0, s, nnz, idx_s,
                               row_of, (const double *)A->val, colidx_t, (double *)val_t);
        else
            hipLaunchKernelGGL(k_gather_csr<float>, dim3(grid), dim3(256), 0, s, nnz, idx_s,
                               row_of, (const float *)A->val, colidx_t, (float *)val_t);
    }
    if ((e = hipGetLastError()) != hipSuccess)
        return fail_all(hip_fail(e, "assembling the transposed CSR"));
    T = new (std::nothrow) spc5_matrix();
    if (!T) return fail_all(fail(SPC5_ENOMEM, "host allocation failed"));
    T->nrows = A->ncols;
    T->ncols = A->nrows;
    T->nnz = nnz;
    T->r = r;
    T->c = c;
    T->dtype = A->dtype;
    T->mask_bytes = c <= 8 ? 1 : 2;
    T->npanels = (T->nrows + r - 1) / r;
    T->device = A->device;
    if ((e = hipMalloc((void **)&perm, nz * 4 + kPad)) != hipSuccess ||
        (e = hipMalloc(&gbuf, nz * vb + kPad)) != hipSuccess)
        return fail_all(hip_fail(e, "allocating the transpose plan"));
    int st = convert_on_device(T, rowptr_t, colidx_t, val_t, idx_s, perm);
    if (st != SPC5_OK) return fail_all(st);
    if ((st = finish_matrix(T)) != SPC5_OK) return fail_all(st);
    // 4. staging slots: a stable sort of A's packed indices by the bucket of
    // their A^T position (row_of, col_of and key_s are free again)
    if ((e = hipMalloc((void **)&scat, nz * 4)) != hipSuccess ||
        (e = hipMalloc(&stage, nz * vb + kPad)) != hipSuccess)
        return fail_all(hip_fail(e, "allocating the transpose plan"));
    if (nnz > 0) {
        const unsigned grid = (unsigned)((nnz + 255) / 256);
        hipLaunchKernelGGL(k_bucket_keys, dim3(grid), dim3(256), 0, s, nnz, perm, row_of);
        const int64_t nb = (nnz + kPermBucket - 1) / kPermBucket;
        unsigned bits = 1;
        while (bits < 31 && ((int64_t)1 << bits) < nb) ++bits;
        size_t need = 0;
        rocprim::counting_iterator<int32_t> iota(0);
        if ((e = rocprim::radix_sort_pairs(nullptr, need, row_of, col_of, iota, key_s,
                                           (size_t)nnz, 0u, bits, s)) != hipSuccess)
            return fail_all(hip_fail(e, "sorting by bucket"));
        if (need > tmp_bytes) {
            if (tmp) (void)hipFree(tmp);
            tmp = nullptr;
            if ((e = hipMalloc(&tmp, need)) != hipSuccess)
                return fail_all(hip_fail(e, "allocating the transpose plan"));
            tmp_bytes = need;
        }
        if ((e = rocprim::radix_sort_pairs(tmp, need, row_of, col_of, iota, key_s, (size_t)nnz,
                                           0u, bits, s)) != hipSuccess)
            return fail_all(hip_fail(e, "sorting by bucket"));
        hipLaunchKernelGGL(k_invert, dim3(grid), dim3(256), 0, s, nnz, key_s, scat);
        hipLaunchKernelGGL(k_compose, dim3(grid), dim3(256), 0, s, nnz, scat, perm);
        if ((e = hipGetLastError()) != hipSuccess)
            return fail_all(hip_fail(e, "building the staging slots"));
    }
    cleanup();
    A->tr = T;
    A->tr_scatter = scat;
    A->tr_gather = perm;
    A->tr_stage = stage;
    A->tr_vals = gbuf;
    return SPC5_OK;
}

hipError_t launch_transpose_plan(const spc5_matrix *A, const void *vals, const void *ybar,
                                 void *xbar, hipStream_t s) {
    const spc5_matrix *T = A->tr;
    const void *tv = T->val;
    if (vals && A->nnz > 0) {
        // the caller's values (A's packed order) moved to A^T's packed order
        if (A->dtype == SPC5_F64) launch_move<double>(A, (const double *)vals, s);
        else launch_move<float>(A, (const float *)vals, s);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        tv = A->tr_vals;
    }
    return launch_spmv(T, tv, ybar, xbar, s);
}

}  // namespace spc5
