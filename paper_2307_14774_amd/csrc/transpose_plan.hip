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
//  4. tables for caller-supplied values theta (autograd).  Then the
//     transpose does not run the forward kernel over A^T at all: with
//     p_k = theta_k * ybar[row_k] (one product per nonzero, formed in A's
//     packed order, where ybar is read row after row), x_bar[j] is the sum
//     of the p's of A^T's row j, i.e. a segmented sum of p in A^T's CSR
//     order.  A single gather p[order[q]] would read one scattered word per
//     cache line, so A^T's CSR order is cut into buckets of 8192 positions
//     (one LDS window), A's values get staging slots grouped by bucket
//     (inside a bucket: A's packed order), and two passes run, each through
//     LDS: pass 1 loads a contiguous chunk of 16384 values of A, forms their
//     products and stores them contiguously in slot order (one run per
//     bucket the chunk reaches); pass 2 assembles one bucket's slots from
//     those runs, reads them in A^T's order through 16-bit local indices and
//     sums each row's run with a workgroup segmented scan.  A row inside one
//     bucket is stored there; a row cut by bucket edges leaves its
//     bucket-edge partial sums, added in bucket order by a fixup.  Apart
//     from the runs (a few dozen bytes each on a power-law graph, shared in
//     L2 by neighbouring buckets) every global access is contiguous; there
//     are no atomics, and the result is reproducible bit for bit.  (Chunks
//     are larger than buckets: longer runs; smaller windows, so more
//     workgroups resident per compute unit, in pass 2.)
#include "spc5_internal.h"
#include "wave.h"

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include <algorithm>
#include <vector>

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
constexpr int kChunkValues = 16384;   // pass 1: values of A per workgroup
constexpr int kChunkThreads = 1024;
constexpr int kBucketValues = 8192;   // pass 2: positions of A^T per workgroup
constexpr int kBucketThreads = 512;

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

// Inclusive maximum scan over the wavefront, the DPP steps of
// wave_incl_scan; lanes that a step shifts in from outside their row read 0,
// so the values must be non-negative.  Every lane must be active.
__device__ __forceinline__ int wave_incl_max(int v) {
    constexpr int kRowShr = 0x110, kBcast15 = 0x142, kBcast31 = 0x143;
    v = max(v, __builtin_amdgcn_update_dpp(0, v, kRowShr + 1, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, kRowShr + 2, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, kRowShr + 4, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, kRowShr + 8, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, kBcast15, 0xa, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, kBcast31, 0xc, 0xf, false));
    return v;
}

// Runs: slot t starts one when it is its bucket's first slot or holds a
// value of another chunk of A than slot t-1 (inside a bucket the slots
// follow A's packed order, so a chunk's values there are consecutive).
__global__ void k_run_flags(int64_t nnz, int64_t w, int64_t wc, const int32_t *__restrict__ order,
                            int32_t *__restrict__ flag) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nnz) flag[t] = (t % w == 0 || order[t] / wc != order[t - 1] / wc) ? 1 : 0;
}

// Run k = rnum[t] starting at slot t: its window slot u0 = t % w and its
// base, the position in pass 1's output (lpos: the output position of every
// slot) minus u0, so that window slot u of the run reads base + u; for a
// bucket's first slot also the bucket's first run.  Inside a bucket the
// bases never decrease: the runs follow the chunks in order, and a chunk's
// output ends no later than where the next one's starts.
__global__ void k_run_tables(int64_t nnz, int64_t w, const int32_t *__restrict__ flag,
                             const int32_t *__restrict__ rnum, const int32_t *__restrict__ lpos,
                             uint16_t *__restrict__ rslot, int32_t *__restrict__ rbase,
                             int32_t *__restrict__ rstart) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nnz || !flag[t]) return;
    const int k = rnum[t];
    const int u0 = (int)(t % w);
    rslot[k] = (uint16_t)u0;
    rbase[k] = lpos[t] - u0;
    if (u0 == 0) rstart[t / w] = k;
}

// Pass 1: workgroup c loads values [c*W, c*W + m) of A into LDS, each
// multiplied by ybar at its row, then writes position j of its list,
// out[c*W + j] = win[lidx[c*W + j]]: the chunk's products in slot order,
// bucket after bucket, stored contiguously (pass 2 gathers each bucket's
// runs).  The products are formed in pairs of consecutive values (4-byte
// loads of two 16-bit row offsets).  Rows come as 16-bit offsets from the
// chunk's base row (R16) or as full indices.
template <typename T, bool R16>
__global__ __launch_bounds__(kChunkThreads) void k_move_products(
    int64_t n, const uint16_t *__restrict__ lidx, const T *__restrict__ in,
    const void *__restrict__ arow, const int32_t *__restrict__ cbase, const T *__restrict__ ybar,
    T *__restrict__ stage) {
    constexpr int W = kChunkValues;
    constexpr int P = W / (2 * kChunkThreads);     // value pairs per thread
    constexpr int Q = W / kChunkThreads;           // list positions per thread
    __shared__ T win[W];
    const int64_t cb = blockIdx.x;
    const int64_t c0 = cb * W;
    const int m = (int)min((int64_t)W, n - c0);
    const int th = threadIdx.x;
    // the list's local indices: independent of the products, read first
    uint32_t l[Q];
#pragma unroll
    for (int e = 0; e < Q; ++e) {
        const int j = th + e * kChunkThreads;
        l[e] = j < m ? (uint32_t)lidx[c0 + j] : 0u;
    }
    if constexpr (R16) {
        const uint16_t *rr = (const uint16_t *)arow;
        const int rb = cbase[cb];
#pragma unroll
        for (int e = 0; e < P; ++e) {
            const int k = 2 * (th + e * kChunkThreads);
            const uint32_t rp = k < m ? *(const uint32_t *)(rr + c0 + k) : 0u;
            if (k < m) win[k] = in[c0 + k] * ybar[rb + (int)(rp & 0xffffu)];
            if (k + 1 < m) win[k + 1] = in[c0 + k + 1] * ybar[rb + (int)(rp >> 16)];
        }
    } else {
        const int32_t *rr = (const int32_t *)arow;
#pragma unroll
        for (int e = 0; e < P; ++e) {
            const int k = 2 * (th + e * kChunkThreads);
            if (k < m) win[k] = in[c0 + k] * ybar[rr[c0 + k]];
            if (k + 1 < m) win[k + 1] = in[c0 + k + 1] * ybar[rr[c0 + k + 1]];
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < Q; ++e) {
        const int j = th + e * kChunkThreads;
        if (j < m) stage[c0 + j] = win[l[e]];
    }
}

// Base row of every chunk of W packed values of A (the first row of its
// first value's panel) and a flag when some chunk spans 65536 rows or more.
__global__ void k_chunk_base(int64_t nnz, int64_t w, int r, const int32_t *__restrict__ row_of,
                             int32_t *__restrict__ cbase, int *__restrict__ wide) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c * w >= nnz) return;
    const int64_t last = min((c + 1) * w, nnz) - 1;
    const int32_t b = row_of[c * w] / r * r;
    const int32_t top = row_of[last] / r * r + r - 1;
    cbase[c] = b;
    if (top - b >= 65536) *wide = 1;
}

__global__ void k_rows16(int64_t nnz, int64_t w, const int32_t *__restrict__ row_of,
                         const int32_t *__restrict__ cbase, uint16_t *__restrict__ rows16) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) rows16[k] = (uint16_t)(row_of[k] - cbase[k / w]);
}

// Positions of a bucket per thread in pass 2 (consecutive).
constexpr int kSumPer = kBucketValues / kBucketThreads;
static_assert(kSumPer == 16, "two 16-byte loads of 16-bit indices per thread");

// Segmented-sum operator: (head seen, sum since the last head).
template <typename T>
struct SegSum {
    int f;
    T v;
};

template <typename T>
__device__ __forceinline__ SegSum<T> seg_join(SegSum<T> a, SegSum<T> b) {
    return {a.f | b.f, b.f ? b.v : a.v + b.v};
}

// Pass 2: workgroup b assembles bucket b's slots [b*W, b*W + m) in LDS from
// the runs of pass 1's output (a run: the values of one chunk of A inside
// the bucket, consecutive both there and in the chunk's output).  Thread t owns positions t*16 .. t*16+15 of the bucket in A^T's CSR order;
// position q's product is win[src[q]].  The heads (first positions of the
// nonempty rows of A^T) come from a bitmap over all positions, read straight
// from memory; a workgroup segmented scan carries each row's running sum,
// and the number of heads, across threads.  The sum of a row that starts
// and ends in the bucket goes to LDS, at its head's number inside the
// bucket, and all of them are stored to x_bar in one coalesced sweep at the
// end (rows from hrow, read up front).  The segment of a row that started in
// an earlier bucket goes to head[b], that of a row that starts here and goes
// on to tail[b] (k_edge_fixup adds them).  The workgroup first stores zeros
// to the rows it owns, [rlo[b], rlo[b+1]): those whose first position lies
// in the bucket (for the last bucket also the empty rows at the end), so
// empty rows need no fill of their own; a wait for those stores before the
// barrier that completes the window puts them ahead of the sums.
// FP32: four workgroups per compute unit (32 KiB of LDS each) need 8 waves
// per SIMD, i.e. at most 64 VGPRs.
template <typename T>
__global__ __launch_bounds__(kBucketThreads)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 4))) void k_bucket_sums(
    int64_t n, const uint16_t *__restrict__ src, const T *__restrict__ stage,
    const int32_t *__restrict__ rstart, const uint16_t *__restrict__ rslot,
    const int32_t *__restrict__ rbase, const uint32_t *__restrict__ hbits,
    const int32_t *__restrict__ hoff,
    const int32_t *__restrict__ hrow, const int32_t *__restrict__ rlo, T *__restrict__ head,
    T *__restrict__ tail, T *__restrict__ xbar) {
    constexpr int W = kBucketValues;
    constexpr int NWV = kBucketThreads / kWave;
    constexpr int kHr = sizeof(T) == 4 ? 1 : 2;          // head rows per thread read up front
    __shared__ T win[W];
    __shared__ int s_f[NWV], s_c[NWV], s_m[W / kBucketThreads * NWV];
    __shared__ T s_v[NWV];
    // runs of 16 consecutive buckets per XCD: neighbouring buckets read
    // adjacent runs of every chunk, so their cache lines are fetched into
    // one L2 once
    const int b = (int)xcd_chunks(blockIdx.x, gridDim.x, 16);
    const int64_t q0 = (int64_t)b * W;
    const int m = (int)min((int64_t)W, n - q0);
    const int th = threadIdx.x, lane = lane_id(), wv = th / kWave;
    const int t0 = th * kSumPer;
    const int h0 = hoff[b], h1 = hoff[b + 1];
    // the last head's row goes on past the bucket when the position after
    // the bucket exists and starts no row
    const int64_t qe = q0 + m;
    const bool has_tail =
        h1 > h0 && qe < n && !((hbits[qe >> 5] >> (unsigned)(qe & 31)) & 1u);
    const int nint = h1 - h0 - (has_tail ? 1 : 0);      // rows stored from LDS
    // zeros to the owned rows, first
    {
        const int rl0 = rlo[b], rl1 = rlo[b + 1];
        for (int j = rl0 + th; j < rl1; j += kBucketThreads) xbar[j] = T(0);
    }
    // this thread's 16 slot indices and its 17 head bits (bit 16: the next
    // thread's first position, or the next bucket's), read up front
    typedef unsigned v4 __attribute__((ext_vector_type(4)));
    v4 w0 = {0u, 0u, 0u, 0u}, w1 = {0u, 0u, 0u, 0u};
    if (t0 < m) {
        const v4 *sp = (const v4 *)(src + q0 + t0);
        w0 = sp[0];
        w1 = sp[1];
    }
    const int64_t pw = (q0 + t0) >> 5;                   // t0 & 31 is 0 or 16
    const uint32_t bw0 = hbits[pw];
    const uint32_t bw1 = (t0 & 31) ? hbits[pw + 1] : 0u;
    // The bucket's runs [rstart[b], rstart[b+1]) in slot order: run k starts
    // at window slot rslot[k], and slot u of it holds pass 1's output at
    // rbase[k] + u (the bases do not decrease along the bucket).  The slots
    // are taken in 16 rows of 512, slot u = row * 512 + thread.
    // 1. Each run's first slot is marked with its base plus one (the marks
    // sit in the window's memory, in the first 4 bytes of their slots, until
    // the products replace them).
    constexpr int NR = W / kBucketThreads;               // rows of slots
    constexpr int MS = (int)sizeof(T) / 4;               // ints per slot
    const int r0 = rstart[b], r1 = rstart[b + 1];
    int *wm = (int *)win;
#pragma unroll
    for (int k = 0; k < NR; ++k) wm[(th + k * kBucketThreads) * MS] = 0;
    __syncthreads();
    for (int k = r0 + th; k < r1; k += kBucketThreads) wm[(int)rslot[k] * MS] = rbase[k] + 1;
    __syncthreads();
    // 2. The base of every slot is the largest mark at or before it: a
    // wavefront maximum scan per row (kept in the slot), then one over the
    // 128 row segments' maxima (every wavefront scans them itself).
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        int *ws = wm + (th + k * kBucketThreads) * MS;
        const int a = wave_incl_max(*ws);
        *ws = a;
        if (lane == kWave - 1) s_m[k * NWV + wv] = a;
    }
    __syncthreads();
    constexpr int SPL = NR * NWV / kWave;                // row segments per lane
    static_assert(SPL == 1 || SPL == 2, "one or two row segments per lane");
    const int sa = s_m[SPL * lane], sb = SPL == 2 ? s_m[SPL * lane + 1] : 0;
    int ep = __shfl_up(wave_incl_max(max(sa, sb)), 1);
    ep = lane ? ep : 0;
    // largest mark before segment s = k * NWV + wv: on lane s / SPL
    const int pre = (SPL == 2 && (wv & 1)) ? max(ep, sa) : ep;
    // 3. The products from their runs, consecutive lanes on consecutive
    // slots; a slot's scan value is read, and the slot then overwritten, by
    // the thread that wrote it.  Slots past the bucket's end (last bucket)
    // read the last product instead: never used, no branch.
    const uint32_t lim = (uint32_t)min((int64_t)UINT32_MAX, n - 1);
#pragma unroll
    for (int h = 0; h < NR; h += 8) {
        T v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = h + i;
            const int before = __builtin_amdgcn_readlane(pre, (k * NWV + wv) / SPL);
            const int u = th + k * kBucketThreads;
            const int base = max(before, wm[u * MS]);
            v[i] = stage[min((uint32_t)(base - 1) + (uint32_t)u, lim)];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) win[th + (h + i) * kBucketThreads] = v[i];
    }
    // the zero stores complete before the barrier, so that the sums other
    // waves store to the same rows after it land later
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    // products of this thread's positions and their head bits
    T p[kSumPer];
    {
        const unsigned wd[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
        for (int i = 0; i < kSumPer; ++i) {
            const unsigned idx = (wd[i >> 1] >> (16 * (i & 1))) & 0xffffu;
            p[i] = t0 + i < m ? win[idx] : T(0);
        }
    }
    // positions at or past n carry no head bits (the bitmap is zero there)
    const unsigned hb = (t0 & 31) ? ((bw0 >> 16) | ((bw1 & 1u) << 16)) : (bw0 & 0x1ffffu);
    // thread aggregate: (head seen, open segment's sum), head count
    SegSum<T> agg = {0, T(0)};
#pragma unroll
    for (int i = 0; i < kSumPer; ++i) {
        const bool h = (hb >> i) & 1u;
        agg.v = h ? p[i] : agg.v + p[i];
        agg.f |= h ? 1 : 0;
    }
    const int cnt = __popc(hb & 0xffffu);
    // workgroup exclusive scans: segmented sums and head counts
    SegSum<T> inc = agg;
    int cinc = cnt;
    for (int d = 1; d < kWave; d <<= 1) {
        SegSum<T> o;
        o.f = __shfl_up(inc.f, d);
        o.v = __shfl_up(inc.v, d);
        const int oc = __shfl_up(cinc, d);
        if (lane >= d) {
            inc = seg_join(o, inc);
            cinc += oc;
        }
    }
    if (lane == kWave - 1) {
        s_f[wv] = inc.f;
        s_v[wv] = inc.v;
        s_c[wv] = cinc;
    }
    SegSum<T> exw;
    exw.f = __shfl_up(inc.f, 1);
    exw.v = __shfl_up(inc.v, 1);
    int cex = __shfl_up(cinc, 1);
    if (lane == 0) {
        exw = {0, T(0)};
        cex = 0;
    }
    // this barrier also ends every read of the window: from here on it
    // holds the rows' sums
    __syncthreads();
    // rows of up to kHr of the bucket's heads, read while the walk runs
    int hr[kHr];
#pragma unroll
    for (int i = 0; i < kHr; ++i) {
        const int u = th + i * kBucketThreads;
        hr[i] = u < nint ? hrow[h0 + u] : 0;
    }
    SegSum<T> carry = {0, T(0)};
    int heads_before = 0;
    for (int w2 = 0; w2 < wv; ++w2) {
        carry = seg_join(carry, SegSum<T>{s_f[w2], s_v[w2]});
        heads_before += s_c[w2];
    }
    carry = seg_join(carry, exw);
    heads_before += cex;
    // walk the positions; a segment ends at e when e+1 is a head or e is the
    // bucket's last position.  lh: the segment's head number in the bucket
    // (-1: the row started in an earlier bucket)
    T run = carry.v;
    int lh = heads_before - 1;
#pragma unroll
    for (int i = 0; i < kSumPer; ++i) {
        const int e = t0 + i;
        if (e < m) {
            if ((hb >> i) & 1u) {
                run = T(0);
                ++lh;
            }
            run += p[i];
            const bool last = e == m - 1;
            if (last || ((hb >> (i + 1)) & 1u)) {
                if (lh < 0)
                    head[b] = run;
                else if (last && has_tail)
                    tail[b] = run;
                else
                    win[lh] = run;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kHr; ++i) {
        const int u = th + i * kBucketThreads;
        if (u < nint) xbar[hr[i]] = win[u];
    }
    for (int u = th + kHr * kBucketThreads; u < nint; u += kBucketThreads)
        xbar[hrow[h0 + u]] = win[u];
}

// Rows of A^T cut by bucket edges: x_bar[j] = tail[bs] + head[bs+1] + ... +
// head[be], one wavefront per row, lanes striding the heads in bucket
// order, then a butterfly: a fixed order, so the result is reproducible.
template <typename T>
__global__ __launch_bounds__(256) void k_edge_fixup(int64_t nrows, const int32_t *__restrict__ rows,
                                                    const T *__restrict__ head,
                                                    const T *__restrict__ tail,
                                                    T *__restrict__ xbar) {
    const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (q >= nrows) return;    // uniform over the wavefront
    const int lane = lane_id();
    const int j = rows[3 * q], bs = rows[3 * q + 1], be = rows[3 * q + 2];
    T acc = T(0);
    for (int bb = bs + 1 + lane; bb <= be; bb += kWave) acc += head[bb];
    for (int d = 1; d < kWave; d <<= 1) acc += __shfl_xor(acc, d);
    if (lane == 0) xbar[j] = tail[bs] + acc;
}

template <typename T>
static hipError_t launch_theta_transpose(const spc5_matrix *A, const T *vals, const T *ybar,
                                         T *xbar, hipStream_t s, T *stage, T *edges) {
    const int64_t n = A->nnz;
    // no buckets: every row of A^T is empty
    if (n == 0) return zero_fill(xbar, A->ncols, (int)sizeof(T), s);
    const unsigned nch = (unsigned)((n + kChunkValues - 1) / kChunkValues);
    const unsigned nbk = (unsigned)A->tr_nbuckets;
    T *head = edges, *tail = edges + nbk;
    if (A->tr_cbase)
        hipLaunchKernelGGL((k_move_products<T, true>), dim3(nch), dim3(kChunkThreads), 0, s, n,
                           A->tr_lidx, vals, A->tr_arow, A->tr_cbase, ybar, stage);
    else
        hipLaunchKernelGGL((k_move_products<T, false>), dim3(nch), dim3(kChunkThreads), 0, s, n,
                           A->tr_lidx, vals, A->tr_arow, A->tr_cbase, ybar, stage);
    hipLaunchKernelGGL(k_bucket_sums<T>, dim3(nbk), dim3(kBucketThreads), 0, s, n, A->tr_src,
                       (const T *)stage, A->tr_rstart, A->tr_rslot, A->tr_rbase, A->tr_hbits,
                       A->tr_hoff, A->tr_hrow, A->tr_rlo, head,
                       tail, xbar);
    if (A->tr_nedge > 0) {
        const int64_t thr = A->tr_nedge * kWave;
        hipLaunchKernelGGL(k_edge_fixup<T>, dim3((unsigned)((thr + 255) / 256)), dim3(256), 0, s,
                           A->tr_nedge, A->tr_edge_rows, (const T *)head, (const T *)tail, xbar);
    }
    return hipGetLastError();
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
    int32_t *perm = nullptr, *hoff = nullptr, *hrow = nullptr, *rlo = nullptr;
    uint32_t *hbits = nullptr;
    int32_t *cbase = nullptr;
    void *arow = nullptr;
    int32_t *edge_rows = nullptr;
    uint16_t *lidx = nullptr, *src = nullptr, *rslot = nullptr;
    int32_t *rbase = nullptr, *rstart = nullptr;
    int64_t nruns = 0;
    size_t tmp_bytes = 0;
    auto cleanup = [&]() {
        for (void *p : {(void *)row_of, (void *)col_of, (void *)key_s, (void *)idx_s,
                        (void *)colidx_t, (void *)rowptr_t, val_t, tmp})
            if (p) (void)hipFree(p);
    };
    auto fail_all = [&](int st) {
        cleanup();
        free_matrix(T);
        for (void *p : {(void *)perm, (void *)lidx, (void *)src, arow, (void *)hoff,
                        (void *)hbits, (void *)hrow, (void *)rlo, (void *)edge_rows,
                        (void *)cbase, (void *)rslot, (void *)rbase, (void *)rstart})
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
    int st = convert_on_device(T, rowptr_t, colidx_t, val_t);
    if (st != SPC5_OK) return fail_all(st);
    if ((st = finish_matrix(T)) != SPC5_OK) return fail_all(st);
    // 4. the tables of the theta transpose (col_of, key_s and colidx_t are
    // free again; idx_s is A^T's CSR order).  Slots: a stable sort of A's
    // packed indices by the bucket of their A^T position; pass 1's lists: a
    // stable sort of the slots by the chunk of A they read.  A's row of
    // every packed value is kept for pass 1; for pass 2 the first position
    // and the row of every nonempty row of A^T, grouped by bucket, and the
    // rows cut by bucket edges.
    const int64_t W = kBucketValues, WC = kChunkValues;
    const int64_t nbk = (nnz + W - 1) / W, nch = (nnz + WC - 1) / WC;
    if ((e = hipMalloc((void **)&perm, nz * 4 + kPad)) != hipSuccess ||
        (e = hipMalloc((void **)&lidx, nz * 2 + kPad)) != hipSuccess ||
        (e = hipMalloc((void **)&src, nz * 2 + kPad)) != hipSuccess ||
        (e = hipMalloc((void **)&hoff, (size_t)(nbk + 1) * 4 + kPad)) != hipSuccess)
        return fail_all(hip_fail(e, "allocating the transpose plan"));
    // A's rows for pass 1: 16-bit offsets from each chunk's base row when
    // every chunk spans fewer than 65536 rows, else 32-bit rows
    if (nnz > 0) {
        int *wide = nullptr;
        int hw = 0;
        if ((e = hipMalloc((void **)&cbase, (size_t)nch * 4 + kPad)) != hipSuccess ||
            (e = hipMalloc((void **)&wide, 4)) != hipSuccess)
            return fail_all(hip_fail(e, "allocating the transpose plan"));
        if ((e = zero_fill(wide, 1, 4, s)) == hipSuccess) {
            hipLaunchKernelGGL(k_chunk_base, dim3((unsigned)((nch + 255) / 256)), dim3(256), 0, s,
                               nnz, WC, A->r, row_of, cbase, wide);
            e = hipMemcpy(&hw, wide, 4, hipMemcpyDeviceToHost);
        }
        (void)hipFree(wide);
        if (e != hipSuccess) return fail_all(hip_fail(e, "chunk rows"));
        if (!hw) {
            if ((e = hipMalloc(&arow, nz * 2 + kPad)) != hipSuccess)
                return fail_all(hip_fail(e, "allocating the transpose plan"));
            hipLaunchKernelGGL(k_rows16, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, nnz,
                               WC, row_of, cbase, (uint16_t *)arow);
        } else {
            (void)hipFree(cbase);
            cbase = nullptr;
            if ((e = hipMalloc(&arow, nz * 4 + kPad)) != hipSuccess ||
                (e = hipMemcpyAsync(arow, row_of, (size_t)nnz * 4, hipMemcpyDeviceToDevice, s)) !=
                    hipSuccess)
                return fail_all(hip_fail(e, "keeping the rows of A"));
        }
    }
    int64_t nedge = 0, nheads = 0;
    {
        std::vector<int64_t> rp((size_t)A->ncols + 1);
        if ((e = hipMemcpy(rp.data(), rowptr_t, rp.size() * 8, hipMemcpyDeviceToHost)) !=
            hipSuccess)
            return fail_all(hip_fail(e, "reading the rowptr of A^T"));
        // head bitmap over every position of every bucket (zero past nnz,
        // one spare word), rows of the heads grouped by bucket, the rows
        // each bucket owns (those starting in it; the trailing empty rows go
        // to the last bucket), and the rows cut by bucket edges
        const size_t nwords = (size_t)nbk * (W / 32) + 1;
        std::vector<uint32_t> hb(nwords, 0u);
        std::vector<int32_t> hr, ho((size_t)nbk + 1, 0), rl((size_t)nbk + 1, 0), er;
        for (int64_t jj = 0; jj < A->ncols; ++jj) {
            if (rp[jj + 1] == rp[jj]) continue;
            hb[(size_t)(rp[jj] >> 5)] |= 1u << (unsigned)(rp[jj] & 31);
            hr.push_back((int32_t)jj);
            ++ho[(size_t)(rp[jj] / W) + 1];
            const int64_t bs = rp[jj] / W, be = (rp[jj + 1] - 1) / W;
            if (bs != be) {
                er.push_back((int32_t)jj);
                er.push_back((int32_t)bs);
                er.push_back((int32_t)be);
            }
        }
        for (int64_t bk = 0; bk < nbk; ++bk) ho[bk + 1] += ho[bk];
        for (int64_t bk = 1; bk < nbk; ++bk)
            rl[bk] = (int32_t)(std::lower_bound(rp.begin(), rp.end(), bk * W) - rp.begin());
        rl[nbk] = (int32_t)A->ncols;
        nheads = (int64_t)hr.size();
        nedge = (int64_t)er.size() / 3;
        if ((e = hipMalloc((void **)&hbits, nwords * 4 + kPad)) != hipSuccess ||
            (e = hipMalloc((void **)&hrow, std::max<size_t>(hr.size(), 1) * 4 + kPad)) !=
                hipSuccess ||
            (e = hipMalloc((void **)&rlo, rl.size() * 4 + kPad)) != hipSuccess ||
            (e = hipMalloc((void **)&edge_rows, std::max<size_t>(er.size(), 3) * 4)) !=
                hipSuccess ||
            (e = hipMemcpy(hoff, ho.data(), ho.size() * 4, hipMemcpyHostToDevice)) !=
                hipSuccess ||
            (e = hipMemcpy(hbits, hb.data(), nwords * 4, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(rlo, rl.data(), rl.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
            (!hr.empty() &&
             (e = hipMemcpy(hrow, hr.data(), hr.size() * 4, hipMemcpyHostToDevice)) !=
                 hipSuccess) ||
            (!er.empty() &&
             (e = hipMemcpy(edge_rows, er.data(), er.size() * 4, hipMemcpyHostToDevice)) !=
                 hipSuccess))
            return fail_all(hip_fail(e, "uploading the bucket tables"));
    }
    if (nnz > 0) {
        const unsigned grid = (unsigned)((nnz + 255) / 256);
        unsigned bits = 1;
        while (bits < 31 && ((int64_t)1 << bits) < std::max(nbk, nch)) ++bits;
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
        hipLaunchKernelGGL(k_bucket_keys, dim3(grid), dim3(256), 0, s, nnz, W, idx_s, row_of);
        if ((e = sort(row_of, col_of, key_s)) != hipSuccess)
            return fail_all(hip_fail(e, "sorting by bucket"));
        hipLaunchKernelGGL(k_invert, dim3(grid), dim3(256), 0, s, nnz, key_s, col_of);
        hipLaunchKernelGGL(k_bucket_src, dim3(grid), dim3(256), 0, s, nnz, W, col_of, idx_s, src);
        // pass 1 lists: slots sorted by chunk (stable, so ascending inside a
        // chunk); perm = the slot of every list position (kept only until the
        // runs are found), lidx = local value index
        hipLaunchKernelGGL(k_chunk_keys, dim3(grid), dim3(256), 0, s, nnz, WC, key_s, row_of);
        if ((e = sort(row_of, idx_s, perm)) != hipSuccess)
            return fail_all(hip_fail(e, "sorting by chunk"));
        hipLaunchKernelGGL(k_chunk_lists, dim3(grid), dim3(256), 0, s, nnz, WC, key_s, perm, lidx);
        // runs for pass 2: flags (row_of), their numbers (idx_s), the output
        // position of every slot (col_of: the inverse of the lists)
        hipLaunchKernelGGL(k_run_flags, dim3(grid), dim3(256), 0, s, nnz, W, WC, key_s, row_of);
        hipLaunchKernelGGL(k_invert, dim3(grid), dim3(256), 0, s, nnz, perm, col_of);
        size_t need = 0;
        if ((e = rocprim::exclusive_scan(nullptr, need, row_of, idx_s, 0, (size_t)nnz,
                                         rocprim::plus<int32_t>(), s)) != hipSuccess)
            return fail_all(hip_fail(e, "numbering the runs"));
        if (need > tmp_bytes) {
            if (tmp) (void)hipFree(tmp);
            tmp = nullptr;
            if ((e = hipMalloc(&tmp, need)) != hipSuccess)
                return fail_all(hip_fail(e, "numbering the runs"));
            tmp_bytes = need;
        }
        if ((e = rocprim::exclusive_scan(tmp, need, row_of, idx_s, 0, (size_t)nnz,
                                         rocprim::plus<int32_t>(), s)) != hipSuccess)
            return fail_all(hip_fail(e, "numbering the runs"));
        int32_t tl[2] = {0, 0};
        if ((e = hipMemcpyAsync(&tl[0], idx_s + nnz - 1, 4, hipMemcpyDeviceToHost, s)) !=
                hipSuccess ||
            (e = hipMemcpyAsync(&tl[1], row_of + nnz - 1, 4, hipMemcpyDeviceToHost, s)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return fail_all(hip_fail(e, "counting the runs"));
        nruns = (int64_t)tl[0] + tl[1];
        const int32_t nr32 = (int32_t)nruns;
        if ((e = hipMalloc((void **)&rslot, (size_t)nruns * 2 + kPad)) != hipSuccess ||
            (e = hipMalloc((void **)&rbase, (size_t)nruns * 4 + kPad)) != hipSuccess ||
            (e = hipMalloc((void **)&rstart, (size_t)(nbk + 1) * 4 + kPad)) != hipSuccess ||
            (e = hipMemcpy(rstart + nbk, &nr32, 4, hipMemcpyHostToDevice)) != hipSuccess)
            return fail_all(hip_fail(e, "allocating the runs"));
        hipLaunchKernelGGL(k_run_tables, dim3(grid), dim3(256), 0, s, nnz, W, row_of, idx_s,
                           col_of, rslot, rbase, rstart);
        if ((e = hipGetLastError()) != hipSuccess)
            return fail_all(hip_fail(e, "building the value move"));
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess)
        return fail_all(hip_fail(e, "building the transpose plan"));
    cleanup();
    // the lists' slots served only to find the runs
    if (perm) (void)hipFree(perm);
    A->tr = T;
    A->tr_lidx = lidx;
    A->tr_rslot = rslot;
    A->tr_rbase = rbase;
    A->tr_rstart = rstart;
    A->tr_nruns = nruns;
    A->tr_src = src;
    A->tr_arow = arow;
    A->tr_cbase = cbase;
    A->tr_hoff = hoff;
    A->tr_hbits = hbits;
    A->tr_hrow = hrow;
    A->tr_rlo = rlo;
    A->tr_nheads = nheads;
    A->tr_edge_rows = edge_rows;
    A->tr_nedge = nedge;
    A->tr_nbuckets = nbk;
    return SPC5_OK;
}

hipError_t launch_transpose_plan(const spc5_matrix *A, const void *vals, const void *ybar,
                                 void *xbar, hipStream_t s, const Scratch &sc) {
    if (vals) {
        // caller values theta: products in A's order, segmented sums in A^T's
        if (A->nnz > 0 && (!sc.stage || !sc.edges)) return hipErrorInvalidValue;
        return A->dtype == SPC5_F64
                   ? launch_theta_transpose<double>(A, (const double *)vals,
                                                    (const double *)ybar, (double *)xbar, s,
                                                    (double *)sc.stage, (double *)sc.edges)
                   : launch_theta_transpose<float>(A, (const float *)vals, (const float *)ybar,
                                                   (float *)xbar, s, (float *)sc.stage,
                                                   (float *)sc.edges);
    }
    // the matrix's own values: the forward kernel over the stored A^T
    return launch_spmv(A->tr, A->tr->val, ybar, xbar, s, sc.tr_partial);
}

}  // namespace spc5
