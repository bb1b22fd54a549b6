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
//     cut into buckets of W = 16384 values (one LDS window), A's values
//     get staging slots grouped by bucket (inside a bucket: A's packed
//     order), and two passes move them, each through LDS: pass 1 loads a
//     contiguous chunk of W values of A into LDS and writes them out in slot
//     order (one contiguous run per bucket); pass 2 loads one bucket's slots
//     into LDS and writes the bucket's values of A^T in order.  Every global
//     read and write is contiguous; the permutations happen in LDS, with
//     16-bit local indices.
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

// Values per LDS window of the two-pass value move (128 KiB in FP64, 64 KiB
// in FP32: two workgroups per compute unit), and threads per workgroup.
constexpr int kMoveValues = 16384;
constexpr int kMoveThreads = 1024;

// key[perm[q]] = bucket of q: for every packed value of A, the bucket of its
// position in A^T.
__global__ void k_bucket_keys(int64_t nnz, int64_t w, const int32_t *__restrict__ perm,
                              int32_t *__restrict__ key) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnz) key[perm[q]] = (int32_t)(q / w);
}

// slot[order[t]] = t: the staging slot of each value of A.
__global__ void k_invert(int64_t nnz, const int32_t *__restrict__ order,
                         int32_t *__restrict__ slot) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nnz) slot[order[t]] = (int32_t)t;
}

// src[q] = slot of A^T's value q, relative to its bucket's first slot.
__global__ void k_bucket_src(int64_t nnz, int64_t w, const int32_t *__restrict__ slot,
                             const int32_t *__restrict__ perm, uint16_t *__restrict__ src) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnz) src[q] = (uint16_t)(slot[perm[q]] - (q / w) * w);
}

// ckey[t] = chunk of A holding the value in slot t.
__global__ void k_chunk_keys(int64_t nnz, int64_t w, const int32_t *__restrict__ order,
                             int32_t *__restrict__ ckey) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nnz) ckey[t] = (int32_t)(order[t] / w);
}

// Pass 1 tables: position j of chunk c's slot-ordered list writes slot
// by_chunk[j], reading the chunk's local value order[by_chunk[j]] - c*w.
__global__ void k_chunk_lists(int64_t nnz, int64_t w, const int32_t *__restrict__ order,
                              const int32_t *__restrict__ by_chunk, uint16_t *__restrict__ lidx) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < nnz) lidx[j] = (uint16_t)(order[by_chunk[j]] - (j / w) * w);
}

// Pass 1: workgroup c loads values [c*W, c*W + m) of A into LDS, then writes
// stage[gpos[j]] = win[lidx[j]] over its slot-ordered list.  Each thread
// takes pairs of neighbouring entries, so the index tables load as one 64-bit
// (gpos) and one 32-bit (lidx) word per pair; a pair at the end of the
// tables reads into their 64 bytes of trailing padding, and its second entry
// is dropped.
template <typename T>
__global__ __launch_bounds__(kMoveThreads) void k_move_chunks(int64_t n,
                                                              const uint16_t *__restrict__ lidx,
                                                              const int32_t *__restrict__ gpos,
                                                              const T *__restrict__ in,
                                                              T *__restrict__ stage) {
    constexpr int W = kMoveValues;
    constexpr int P = W / (2 * kMoveThreads);
    __shared__ T win[W];
    const int64_t c0 = (int64_t)blockIdx.x * W;
    const int m = (int)min((int64_t)W, n - c0);
    const int th = threadIdx.x;
    uint64_t g[P];
    uint32_t l[P];
#pragma unroll
    for (int e = 0; e < P; ++e) {
        const int k = 2 * (th + e * kMoveThreads);
        g[e] = k < m ? *(const uint64_t *)(gpos + c0 + k) : 0;
        l[e] = k < m ? *(const uint32_t *)(lidx + c0 + k) : 0;
    }
#pragma unroll
    for (int e = 0; e < P; ++e) {
        const int k = 2 * (th + e * kMoveThreads);
        if (k < m) win[k] = in[c0 + k];
        if (k + 1 < m) win[k + 1] = in[c0 + k + 1];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < P; ++e) {
        const int k = 2 * (th + e * kMoveThreads);
        if (k < m) stage[(uint32_t)g[e]] = win[l[e] & 0xffffu];
        if (k + 1 < m) stage[(uint32_t)(g[e] >> 32)] = win[l[e] >> 16];
    }
}

// Pass 2: workgroup b loads bucket b's slots [b*W, b*W + m) into LDS, then
// writes out[b*W + q] = win[src[b*W + q]]; pairs as in pass 1.
template <typename T>
__global__ __launch_bounds__(kMoveThreads) void k_move_buckets(int64_t n,
                                                               const uint16_t *__restrict__ src,
                                                               const T *__restrict__ stage,
                                                               T *__restrict__ out) {
    constexpr int W = kMoveValues;
    constexpr int P = W / (2 * kMoveThreads);
    __shared__ T win[W];
    const int64_t q0 = (int64_t)blockIdx.x * W;
    const int m = (int)min((int64_t)W, n - q0);
    const int th = threadIdx.x;
    uint32_t l[P];
#pragma unroll
    for (int e = 0; e < P; ++e) {
        const int k = 2 * (th + e * kMoveThreads);
        l[e] = k < m ? *(const uint32_t *)(src + q0 + k) : 0;
    }
#pragma unroll
    for (int e = 0; e < P; ++e) {
        const int k = 2 * (th + e * kMoveThreads);
        if (k < m) win[k] = stage[q0 + k];
        if (k + 1 < m) win[k + 1] = stage[q0 + k + 1];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < P; ++e) {
        const int k = 2 * (th + e * kMoveThreads);
        if (k < m) out[q0 + k] = win[l[e] & 0xffffu];
        if (k + 1 < m) out[q0 + k + 1] = win[l[e] >> 16];
    }
}

template <typename T>
static void launch_move(const spc5_matrix *A, const T *vals, hipStream_t s, T *stage, T *out) {
    constexpr int64_t W = kMoveValues;
    const int64_t n = A->nnz;
    const unsigned grid = (unsigned)((n + W - 1) / W);
    hipLaunchKernelGGL(k_move_chunks<T>, dim3(grid), dim3(kMoveThreads), 0, s, n, A->tr_lidx,
                       A->tr_gpos, vals, stage);
    hipLaunchKernelGGL(k_move_buckets<T>, dim3(grid), dim3(kMoveThreads), 0, s, n, A->tr_src,
                       (const T *)stage, out);
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
    int32_t *perm = nullptr;
    uint16_t *lidx = nullptr, *src = nullptr;
    size_t tmp_bytes = 0;
    auto cleanup = [&]() {
        for (void *p : {(void *)row_of, (void *)col_of, (void *)key_s, (void *)idx_s,
                        (void *)colidx_t, (void *)rowptr_t, val_t, tmp})
            if (p) (void)hipFree(p);
    };
    auto fail_all = [&](int st) {
        cleanup();
        free_matrix(T);
        for (void *p : {(void *)perm, (void *)lidx, (void *)src})
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
    if ((e = hipMalloc((void **)&perm, nz * 4 + kPad)) != hipSuccess)
        return fail_all(hip_fail(e, "allocating the transpose plan"));
    int st = convert_on_device(T, rowptr_t, colidx_t, val_t, idx_s, perm);
    if (st != SPC5_OK) return fail_all(st);
    if ((st = finish_matrix(T)) != SPC5_OK) return fail_all(st);
    // 4. the value move's tables (row_of, col_of, key_s, idx_s and colidx_t
    // are free again).  Slots: a stable sort of A's packed indices by the
    // bucket of their A^T position; pass 1's lists: a stable sort of the
    // slots by the chunk of A they read.
    if ((e = hipMalloc((void **)&lidx, nz * 2 + kPad)) != hipSuccess ||
        (e = hipMalloc((void **)&src, nz * 2 + kPad)) != hipSuccess)
        return fail_all(hip_fail(e, "allocating the transpose plan"));
    if (nnz > 0) {
        const int64_t w = kMoveValues;
        const unsigned grid = (unsigned)((nnz + 255) / 256);
        const int64_t nb = (nnz + w - 1) / w;
        unsigned bits = 1;
        while (bits < 31 && ((int64_t)1 << bits) < nb) ++bits;
        rocprim::counting_iterator<int32_t> iota(0);
        auto sort = [&](int32_t *keys, int32_t *keys_out, int32_t *vals_out) -> hipError_t {
            size_t need = 0;
            hipError_t e2 = rocprim::radix_sort_pairs(nullptr, need, keys, keys_out, iota,
                                                      vals_out, (size_t)nnz, 0u, bits, s);
            if (e2 != hipSuccess) return e2;
            if (need > tmp_bytes) {
                if (tmp) (void)hipFree(tmp);
                tmp = nullptr;
                if ((e2 = hipMalloc(&tmp, need)) != hipSuccess) return e2;
                tmp_bytes = need;
            }
            return rocprim::radix_sort_pairs(tmp, need, keys, keys_out, iota, vals_out,
                                             (size_t)nnz, 0u, bits, s);
        };
        // order[t] (key_s): the value of A in slot t; slot (col_of) its inverse
        hipLaunchKernelGGL(k_bucket_keys, dim3(grid), dim3(256), 0, s, nnz, w, perm, row_of);
        if ((e = sort(row_of, col_of, key_s)) != hipSuccess)
            return fail_all(hip_fail(e, "sorting by bucket"));
        hipLaunchKernelGGL(k_invert, dim3(grid), dim3(256), 0, s, nnz, key_s, col_of);
        hipLaunchKernelGGL(k_bucket_src, dim3(grid), dim3(256), 0, s, nnz, w, col_of, perm, src);
        // pass 1 lists: slots sorted by chunk (stable, so ascending inside a
        // chunk); gpos (perm's memory) = the slots, lidx = local value index
        hipLaunchKernelGGL(k_chunk_keys, dim3(grid), dim3(256), 0, s, nnz, w, key_s, row_of);
        if ((e = sort(row_of, idx_s, perm)) != hipSuccess)
            return fail_all(hip_fail(e, "sorting by chunk"));
        hipLaunchKernelGGL(k_chunk_lists, dim3(grid), dim3(256), 0, s, nnz, w, key_s, perm, lidx);
        if ((e = hipGetLastError()) != hipSuccess)
            return fail_all(hip_fail(e, "building the value move"));
    }
    cleanup();
    A->tr = T;
    A->tr_lidx = lidx;
    A->tr_gpos = perm;
    A->tr_src = src;
    return SPC5_OK;
}

hipError_t launch_transpose_plan(const spc5_matrix *A, const void *vals, const void *ybar,
                                 void *xbar, hipStream_t s, const Scratch &sc) {
    const spc5_matrix *T = A->tr;
    const void *tv = T->val;
    if (vals && A->nnz > 0) {
        // the caller's values (A's packed order) moved to A^T's packed order
        if (!sc.stage || !sc.vals) return hipErrorInvalidValue;
        if (A->dtype == SPC5_F64)
            launch_move<double>(A, (const double *)vals, s, (double *)sc.stage,
                                (double *)sc.vals);
        else
            launch_move<float>(A, (const float *)vals, s, (float *)sc.stage, (float *)sc.vals);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        tv = sc.vals;
    }
    return launch_spmv(T, tv, ybar, xbar, s, sc.tr_partial);
}

}  // namespace spc5
