// Forward SPC5 product y = A x on gfx950 (Algorithm 1 of arXiv 2307.14774,
// re-mapped onto 64-lane wavefronts), and the plain CSR comparison kernel.
//
// Two forward kernels share the storage:
//
// ROWS kernel (k_spmv_rows).  Lane = one row of a panel; the r lanes of a
// panel walk its blocks together.  For each block a lane reads the r row
// masks as one word (they are adjacent, index b*r+i), takes its own mask, the
// popcount of the lower rows' masks (its offset inside the block's packed
// values) and the popcount of the whole word (the block's value count, which
// advances the running value offset exactly as Algorithm 1 advances its
// value index).  Its row sum never leaves the lane: no shuffle, no LDS, one
// coalesced store of 64 rows at the end.  Blocks are unrolled by U so that
// the loads of U blocks are in flight together.
//
// SWEEP kernel (k_spmv).  One wavefront owns a tile of `ppt` consecutive panels
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
#include <type_traits>

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
        const int jsafe = j;
        const int bsafe = act ? b : b0;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const bool on = (m >> k) & 1u;
            const T r = fma(val[on ? j : (CSR ? bsafe : jsafe)], x[col0 + (on ? k : 0)], acc);
            acc = on ? r : acc;
            j += on ? 1 : 0;
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


// Row masks of block b for lane row i: own mask, popcount of rows < i, popcount
// of all r rows.  The r masks of a block are adjacent (index b*r+i), so when
// r*sizeof(mask) is 1, 2, 4 or 8 bytes they are read as one word.
template <int R, int C>
struct BlockMasks {
    using MT = typename MaskOf<C>::type;
    static constexpr int kBytes = R * (int)sizeof(MT);
    static constexpr int kBits = 8 * (int)sizeof(MT);
    static constexpr bool kWord = kBytes == 1 || kBytes == 2 || kBytes == 4 || kBytes == 8;
    using WT = typename std::conditional<kBytes <= 4, uint32_t, uint64_t>::type;

    __device__ __forceinline__ static void get(const MT *__restrict__ masks, int64_t b, int i,
                                               unsigned &m, int &pre, int &tot) {
        if constexpr (kWord) {
            WT w;
            if constexpr (kBytes == 1) w = *(const uint8_t *)(masks + b * R);
            else if constexpr (kBytes == 2) w = *(const uint16_t *)(masks + b * R);
            else if constexpr (kBytes == 4) w = *(const uint32_t *)(masks + b * R);
            else w = *(const uint64_t *)(masks + b * R);
            const int sh = i * kBits;
            m = (unsigned)(w >> sh) & ((1u << kBits) - 1u);
            if constexpr (sizeof(WT) == 8) {
                const WT low = sh ? (w & ((WT(1) << sh) - 1)) : WT(0);
                pre = __popcll(low);
                tot = __popcll(w);
            } else {
                const WT low = sh ? (w & ((WT(1) << sh) - 1)) : WT(0);
                pre = __popc(low);
                tot = __popc(w);
            }
        } else {
            pre = 0;
            tot = 0;
            m = 0;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const unsigned mr = masks[b * R + rr];
                const int pc = __popc(mr);
                pre += rr < i ? pc : 0;
                m = rr == i ? mr : m;
                tot += pc;
            }
        }
    }
};

template <typename T, int R, int C, int U>
__global__ __launch_bounds__(kWave) void k_spmv_rows(
    int64_t npanels, int64_t nrows, int64_t nwaves, int remap, int64_t nnz, int64_t ncols,
    const int32_t *__restrict__ blk_ptr, const int32_t *__restrict__ blk_col,
    const typename MaskOf<C>::type *__restrict__ masks, const T *__restrict__ val,
    const int32_t *__restrict__ panel_val, const T *__restrict__ x, T *__restrict__ y)
{
    constexpr int PPW = kWave / R;     // panels per wavefront
    const int lane = lane_id();
    const int64_t w = remap ? xcd_remap(blockIdx.x, nwaves) : (int64_t)blockIdx.x;
    const int64_t p = w * PPW + lane / R;
    const int i = lane % R;
    const bool live = lane < PPW * R && p < npanels;
    int b = 0, be = 0, vb = 0;
    if (live) {
        b = blk_ptr[p];
        be = blk_ptr[p + 1];
        vb = panel_val[p];
    }
    // value gathers through a buffer based at the wavefront's first value
    // (offsets stay small), x gathers through a buffer over x; a clear mask
    // bit passes an out-of-range offset, so the load moves no data
    const int64_t p_first = min(w * PPW, npanels);
    const int vwave = __builtin_amdgcn_readfirstlane(panel_val[p_first]);
    const Buf vbuf = make_buf(val + vwave, (nnz - vwave) * (int64_t)sizeof(T));
    const Buf xbuf = make_buf(x, ncols * (int64_t)sizeof(T));
    // one accumulator per unrolled block: U independent FMA chains
    T acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = T(0);
    for (; b < be; b += U) {
        // branch-free: absent blocks re-read block b and are masked out, so
        // all loads of the U blocks are issued together
        unsigned m[U];
        int pre[U], tot[U], col0[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = b + u < be;
            const int bb = ok ? b + u : b;
            BlockMasks<R, C>::get(masks, (int64_t)bb, i, m[u], pre[u], tot[u]);
            col0[u] = blk_col[bb];
            m[u] = ok ? m[u] : 0u;
            tot[u] = ok ? tot[u] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int j = vb + pre[u] - vwave;
            vb += tot[u];
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const bool on = (m[u] >> k) & 1u;
                const T v = buf_load<T>(vbuf, on ? (uint32_t)j * (uint32_t)sizeof(T) : kOOB);
                const T xv = buf_load<T>(
                    xbuf, on ? (uint32_t)(col0[u] + k) * (uint32_t)sizeof(T) : kOOB);
                const T r = fma(v, xv, acc[u]);
                acc[u] = on ? r : acc[u];
                j += on ? 1 : 0;
            }
        }
    }
    T sum = acc[0];
#pragma unroll
    for (int u = 1; u < U; ++u) sum += acc[u];
    const int64_t row = p * R + i;
    if (live && row < nrows) y[row] = sum;
}


// Plain CSR comparison kernel ("CSR-vector"): a group of G lanes per row
// strides over the row's nonzeros (coalesced values and column indices), then
// the group sums its partials with G-lane butterfly shuffles.  G is chosen
// from the mean row length.
template <typename T, int G>
__global__ __launch_bounds__(kWave) void k_csr_vector(
    int64_t nrows, int64_t nwaves, int remap, const int32_t *__restrict__ rowptr,
    const int32_t *__restrict__ colidx, const T *__restrict__ val, const T *__restrict__ x,
    T *__restrict__ y)
{
    constexpr int RPW = kWave / G;     // rows per wavefront
    const int lane = lane_id();
    const int64_t w = remap ? xcd_remap(blockIdx.x, nwaves) : (int64_t)blockIdx.x;
    const int64_t row = w * RPW + lane / G;
    const int g = lane % G;
    T acc = T(0);
    if (row < nrows) {
        const int e = rowptr[row + 1];
        for (int k = rowptr[row] + g; k < e; k += G) acc = fma(val[k], x[colidx[k]], acc);
    }
#pragma unroll
    for (int d = G / 2; d >= 1; d >>= 1) acc += __shfl_xor(acc, d);
    if (row < nrows && g == 0) y[row] = acc;
}

static int g_remap = -1;
int remap_enabled() {
    if (g_remap < 0) {
        const char *e = getenv("SPC5_XCD_REMAP");
        g_remap = (e && e[0] == '0') ? 0 : 1;
    }
    return g_remap;
}

template <typename T, int R, int C>
static hipError_t launch_t(const spc5_matrix *A, const T *val, const T *x, T *y,
                           hipStream_t s) {
    if (A->kernel == SPC5_KERNEL_ROWS) {
        constexpr int PPW = kWave / R;
        const int64_t nwaves = (A->npanels + PPW - 1) / PPW;
        if (nwaves == 0) return hipSuccess;
        hipLaunchKernelGGL((k_spmv_rows<T, R, C, 4>), dim3((unsigned)nwaves), dim3(kWave), 0, s,
                           A->npanels, A->nrows, nwaves, remap_enabled(), A->nnz, A->ncols,
                           A->blk_ptr,
                           A->blk_col, (const typename MaskOf<C>::type *)A->masks, val,
                           A->panel_val, x, y);
        return hipGetLastError();
    }
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
                       hipStream_t s, void *partial) {
    if (A->kernel == SPC5_KERNEL_STAGED)
        return launch_spmv_staged(A, val ? val : A->val, x, y, s, remap_enabled(), partial);
    return A->dtype == SPC5_F64 ? dispatch<double>(A, val, x, y, s)
                                : dispatch<float>(A, val, x, y, s);
}

template <typename T, int G>
static hipError_t launch_csr_vec(const spc5_csr *A, const void *x, void *y, hipStream_t s) {
    const int64_t nwaves = (A->nrows + kWave / G - 1) / (kWave / G);
    if (nwaves == 0) return hipSuccess;
    hipLaunchKernelGGL((k_csr_vector<T, G>), dim3((unsigned)nwaves), dim3(kWave), 0, s, A->nrows,
                       nwaves, remap_enabled(), A->rowptr, A->colidx, (const T *)A->val,
                       (const T *)x, (T *)y);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_csr_t(const spc5_csr *A, const void *x, void *y, hipStream_t s) {
    switch (A->group) {
        case 1: return launch_csr_vec<T, 1>(A, x, y, s);
        case 2: return launch_csr_vec<T, 2>(A, x, y, s);
        case 4: return launch_csr_vec<T, 4>(A, x, y, s);
        case 8: return launch_csr_vec<T, 8>(A, x, y, s);
        case 16: return launch_csr_vec<T, 16>(A, x, y, s);
        case 32: return launch_csr_vec<T, 32>(A, x, y, s);
        case 64: return launch_csr_vec<T, 64>(A, x, y, s);
        default: break;
    }
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
