// STAGED forward kernel: y = A x over SPC5 beta(r,c) storage, one 256-thread
// workgroup per tile of consecutive panels, the tile streamed through LDS.
//
// Why this shape.  On gfx950 a product over short rows is bound by the number
// of vector memory instructions (each costs the address unit about the same
// whatever its width) and by the latency of its dependent accesses.  So:
//
//  1. stage: the tile's packed values, row masks, anchors and panel bounds
//     are contiguous ranges; the workgroup copies them into LDS with 16-byte
//     vector loads (4 KiB per workgroup instruction), all issued before the
//     first store;
//  2. block value offsets: each block's value count is the popcount of its r
//     row masks; a workgroup prefix scan turns the counts into offsets -- the
//     parallel form of the running value index of Algorithm 1;
//  3. single x load per block: one thread per block gathers x[anchor + k] for
//     every column k that some row of the block uses (the union of its row
//     masks) into LDS.  This is the single-x-load scheme of Section 3.1: the
//     r rows of a block share one load of the x window, so x loads scale with
//     blocks, not with nonzeros;
//  4. rows: thread = (panel, sub-lane, row); it walks every S-th block of its
//     panel, takes its row mask and the popcount of the lower rows' masks
//     (its offset inside the block), and for every set bit k multiplies the
//     next packed value by the block's x entry k, both from LDS;
//  5. a butterfly over the S sub-lanes, one store per row.
//
// Tiles come from a schedule built at conversion (at most 256/r panels, VT
// values and BT blocks per tile).  A panel larger than a tile is cut into
// piece tiles spread over the grid (load balance for very long rows); their
// partial row sums are added in a fixed order by a small fixup kernel.  No
// atomics: results are reproducible bit for bit.  Workgroups reach the XCDs in
// runs of kXcdRun (xcd_chunks).
#include "spc5_internal.h"
#include "stage.h"
#include "wave.h"

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <type_traits>
#include <vector>

namespace spc5 {

// Tile capacities for a matrix (must match StreamCfg): values, blocks for
// value buffers of at most 12 KiB, and panels.
void staged_caps(const spc5_matrix *A, int *vt, int *bt, int *ppw) {
    const int sz = A->dtype == SPC5_F64 ? 8 : 4;
    const int cm = A->c <= 4 ? 4 : (A->c <= 8 ? 8 : 16);
    *vt = ((A->r == 1 ? value_tile(sz) * sz : 16384) - 16) / sz;
    *bt = A->r == 1 ? 4 * kWG : stream_bt(sz, cm, 3);
    *ppw = kWG / A->r;
}

// Value buffer (NVG 16-byte vectors per thread: 1..4) the staged kernel
// uses for tiles of at most maxv values.
static int stream_nvg(int64_t maxv, int sz) {
    const int64_t need = maxv * sz + 16;
    return need <= 4096 ? 1 : need <= 8192 ? 2 : need <= 12288 ? 3 : 4;
}

// Rows phase of one staged tile: thread = (panel pl, sub-lane, row i) with S
// sub-lanes per row (np*R*S <= 256 and S*R <= 64, so the butterfly stays in
// a wavefront).  Returns the row sum on every sub-lane; `lead` marks the
// sub-lane that stores it.  The blocks' x windows sit in LDS column-major,
// x of column k of block b at s_x[k*XS + b]: the sub-lanes of a row read
// consecutive blocks, so one read instruction hits consecutive words.
template <typename T, int R, int C, int U, bool SPARSE, int VAR, int XS>
__device__ __forceinline__ T tile_rows(int np, int b0, int b1, const int *sbp, const uint8_t *smb,
                                       const int *s_boff, const T *sval, const T *s_x,
                                       const T *s_zero, int &pl_out, int &i_out, bool &lead,
                                       const int *scol = nullptr, const Buf *xbuf = nullptr,
                                       T *s_red = nullptr) {
    const int th = threadIdx.x;
    int lgS = 0;
    if ((R & (R - 1)) == 0)
        while (np * R * (2 << lgS) <= kWG && R * (2 << lgS) <= kWave) ++lgS;
    const int S = 1 << lgS;
    const int lps = S * R;
    const int pl = th / lps, sub = (th / R) & (S - 1), i = th % R;
    const bool live = pl < np;
    // a piece tile holds only part of its panel's blocks: clamp.  Both
    // bounds are read on every thread (panel 0's on threads without a panel),
    // so the two reads go out together.
    const int plc = live ? pl : 0;
    const int sb0 = sbp[plc], sb1 = sbp[plc + 1];
    const int bs = live ? max(sb0, b0) - b0 : 0;
    const int be = live ? min(sb1, b1) - b0 : 0;
    // Masked-off (block, bit) pairs read a zero from s_zero for both
    // operands, so the FMA needs no select: 0*0 leaves the sum unchanged
    // and a non-finite x of another row's column is never touched.
    T acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = T(0);
    for (int b = bs + sub; b < be; b += U * S) {
        unsigned m[U];
        int j[U], tt[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = b + u * S < be;
            tt[u] = ok ? b + u * S : b;
            int pre, tot;
            lds_block_masks<R, C>(smb, tt[u], i, m[u], pre, tot);
            m[u] = ok ? m[u] : 0u;
            j[u] = s_boff[tt[u]] + pre;
        }
        if constexpr (SPARSE) {
            // low fill: the set bits two at a time (both pairs of LDS reads
            // in flight together), the wave running as many steps as its
            // fullest row-block has bit pairs; the products are added in
            // ascending bit order
            T a = acc[0];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                unsigned mm = m[u];
                int jj = j[u];
                const T *xb = s_x + tt[u];
                while (__ballot(mm != 0u)) {
                    const unsigned m1 = mm & (mm - 1u);
                    const bool on0 = mm != 0u, on1 = m1 != 0u;
                    const T *pv0 = on0 ? sval + jj : s_zero;
                    const T *px0 = on0 ? xb + (__ffs(mm) - 1) * XS : s_zero;
                    const T *pv1 = on1 ? sval + jj + 1 : s_zero;
                    const T *px1 = on1 ? xb + (__ffs(m1) - 1) * XS : s_zero;
                    const T v0 = *pv0, x0 = *px0, v1 = *pv1, x1 = *px1;
                    a = fma(v0, x0, a);
                    a = fma(v1, x1, a);
                    jj += 2;
                    mm = m1 & (m1 - 1u);
                }
            }
            acc[0] = a;
        } else {
            // high fill: every bit, branch-free; a bit's value index is the
            // row's first value plus the popcount of the lower bits
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c0u = (VAR & kVarPartialX) ? scol[tt[u]] : 0;
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    const bool on = (m[u] >> k) & 1u;
                    const int jk = k ? j[u] + __popc(m[u] & ((1u << k) - 1u)) : j[u];
                    const T *pv = on ? sval + jk : s_zero;
                    if constexpr (VAR & kVarPartialX) {
                        // partial x load: this row's own x entries, straight
                        // from memory (a clear bit moves no data)
                        const T xv = buf_load<T>(
                            *xbuf, on ? (uint32_t)(c0u + k) * (uint32_t)sizeof(T) : kOOB);
                        acc[u] = fma(*pv, xv, acc[u]);
                    } else {
                        const T *px = on ? s_x + k * XS + tt[u] : s_zero;
                        acc[u] = fma(*pv, *px, acc[u]);
                    }
                }
            }
        }
    }
    T accs = acc[0];
#pragma unroll
    for (int u = 1; u < U; ++u) accs += acc[u];
    if constexpr (VAR & kVarRowReduce) {
        // per-row reduction: the sub-lane partials go through LDS and the
        // row's lead thread adds them one after the other
        s_red[th] = accs;
        __syncthreads();
        if (live && sub == 0) {
            T r = T(0);
            for (int q = 0; q < S; ++q) r += s_red[pl * lps + q * R + i];
            accs = r;
        }
    } else {
        // multi-reduction: one butterfly step reduces every row of the tile
        // at once (sub-lanes of a row are R apart inside one wavefront)
        for (int d = R; d < lps; d <<= 1) accs += __shfl_xor(accs, d);
    }
    pl_out = pl;
    i_out = i;
    lead = live && sub == 0;
    return accs;
}

// Workgroups of k_spmv_stream that the LDS of a compute unit (160 KiB, in
// 512-byte allocation units) holds at once, at most 8.  The kernel asks the
// compiler for that many wavefronts per SIMD, so that registers do not cap
// residency below what LDS allows.
template <typename T, int R, int C, int NVG, int VAR>
constexpr int stream_residency() {
    using Cfg = StreamCfg<T, R, C, NVG>;
    constexpr int lds = 16 * (Cfg::VVEC + Cfg::MVEC + Cfg::CVEC + Cfg::PVEC) +
                        Cfg::BT * C * (int)sizeof(T) + 4 * Cfg::BT + 4 * (kWG / kWave) +
                        (int)sizeof(T) * ((VAR & kVarRowReduce) ? kWG + 1 : 2);
    constexpr int units = (lds + 511) / 512;
    constexpr int wg = (160 * 1024 / 512) / units;
    // FP32 with value buffers of at most 8 KiB only: elsewhere the register
    // budget this implies makes the compiler spill
    return sizeof(T) == 4 && NVG <= 2 && R != 3 ? (wg > 8 ? 8 : wg) : 1;
}

template <typename T, int R, int C, int NVG, bool SPARSE, int VAR>
__global__ __launch_bounds__(kWG)
__attribute__((amdgpu_waves_per_eu(stream_residency<T, R, C, NVG, VAR>()))) void k_spmv_stream(
    int64_t nrows, int64_t ncols, int64_t ntiles, int tiles_per_wg, int64_t nwg, int remap,
    const int32_t *__restrict__ tile_p, const int32_t *__restrict__ tile_b,
    const int32_t *__restrict__ tile_v, const int32_t *__restrict__ tile_f,
    const int32_t *__restrict__ blk_ptr,
    const int32_t *__restrict__ blk_col, const typename MaskOf<C>::type *__restrict__ masks,
    const T *__restrict__ val, const T *__restrict__ x, T *__restrict__ y,
    T *__restrict__ partial)
{
    using Cfg = StreamCfg<T, R, C, NVG>;
    constexpr int U = Cfg::U, BT = Cfg::BT;
    __shared__ v4u s_val[Cfg::VVEC];
    __shared__ v4u s_mask[Cfg::MVEC];
    __shared__ v4u s_col[Cfg::CVEC];
    __shared__ v4u s_bp[Cfg::PVEC];
    __shared__ T s_x[BT * C];
    __shared__ int s_boff[BT];
    __shared__ int s_wsum[kWG / kWave];
    __shared__ T s_zero[1];
    __shared__ T s_red[(VAR & kVarRowReduce) ? kWG : 1];

    const int th = threadIdx.x;
    const int lane = lane_id();
    const int wv = th / kWave;
    if (th == 0) s_zero[0] = T(0);   // published by the first tile's barrier
    const int64_t g = remap ? xcd_chunks(blockIdx.x, nwg, kXcdRun) : (int64_t)blockIdx.x;
    const int64_t t_begin = g * tiles_per_wg;
    const int64_t t_end = min(t_begin + tiles_per_wg, ntiles);
    const Buf xbuf = make_buf(x, ncols * (int64_t)sizeof(T));

    // a piece tile (part of a panel longer than a tile) covers that one panel
    int f0 = tile_f[t_begin];
    int p0 = tile_p[t_begin], p1 = f0 ? p0 + 1 : tile_p[t_begin + 1];
    int b0 = tile_b[t_begin], b1 = tile_b[t_begin + 1];
    int v0 = tile_v[t_begin], v1 = tile_v[t_begin + 1];
    // r in {2, 4, 8}: a block's row masks fill 2..16 bytes, loaded per block
    constexpr bool PB = R == 2 || R == 4 || R == 8;
    using Stage = std::conditional_t<PB, BlockStage<T, R, C, NVG>, TileStage<T, R, C, NVG>>;
    Stage st;
    st.issue(p0, p1, b0, b1, v0, v1, val, masks, blk_col, blk_ptr);

    for (int64_t t = t_begin; t < t_end; ++t) {
        // next tile's bounds (scalar loads, their own counter)
        const bool more = t + 1 < t_end;
        const int64_t tn = more ? t + 1 : t;
        const int g0 = tile_f[tn];
        const int q0 = tile_p[tn], q1 = g0 ? q0 + 1 : tile_p[tn + 1];
        const int c0 = tile_b[tn], c1 = tile_b[tn + 1];
        const int w0 = tile_v[tn], w1 = tile_v[tn + 1];
        const int np = p1 - p0;
        const int nbt = b1 - b0;
        const bool has = th < nbt;
        const int tb = has ? th : 0;

        // 1. land the staged tile, and 3. the single x load per block: one
        // thread per block gathers the whole window x[anchor .. anchor+C) in
        // 16-byte loads (the buffer range check is per dword, so a window
        // running past the last column reads zeros there, and blocks whose
        // rows use no column read nothing), then the next tile's staging
        // loads are issued, so both are in flight together and waiting for
        // the gathers does not wait for them (the scheduling barriers keep
        // the compiler from reordering the groups).  On the last tile the
        // current tile is re-requested (cache hits): keeping the issue
        // unconditional keeps the load counters exact on every path.
        unsigned un;
        int cnt, col0;
        T xw[C];
        auto gather = [&]() {
            un = has ? un : 0u;
            cnt = has ? cnt : 0;
            if constexpr (VAR & kVarPartialX) {
#pragma unroll
                for (int k = 0; k < C; ++k) xw[k] = T(0);   // rows load their own x
            } else if constexpr (VAR & kVarUnionX) {
                // merged predicate: only the pieces some row of the block uses
                load_window_union<T, C>(xbuf, un ? (uint32_t)col0 * (uint32_t)sizeof(T) : kOOB,
                                        un, xw);
            } else {
                load_window<T, C>(xbuf, un ? (uint32_t)col0 * (uint32_t)sizeof(T) : kOOB, xw);
            }
        };
        int skv, skm = 0, skc = 0, skp, incl;
        __syncthreads();
        if constexpr (PB) {
            // the block's masks and anchor are in this thread's registers:
            // the gather goes out before the tile is copied to LDS
            st.union_count(un, cnt);
            col0 = st.cw;
            gather();
            st.commit_block((uint8_t *)s_mask, (int *)s_col, has);
            st.rp.commit(s_bp, st.qp);
            st.rv.commit(s_val, st.qv);
            skv = st.qv.skew;
            skp = st.qp.skew;
            __builtin_amdgcn_sched_barrier(0);
            st.issue(q0, q1, c0, c1, w0, w1, val, masks, blk_col, blk_ptr);
            __builtin_amdgcn_sched_barrier(0);
            // 2. block value offsets: the wavefront scan of the block value
            // counts runs from registers too, so the wavefront totals share
            // the tile's barrier
            incl = wave_incl_scan(cnt);
            if (lane == kWave - 1) s_wsum[wv] = incl;
            __syncthreads();
        } else {
            st.rm.commit(s_mask, st.qm);
            st.rc.commit(s_col, st.qc);
            st.rp.commit(s_bp, st.qp);
            st.rv.commit(s_val, st.qv);
            skv = st.qv.skew;
            skm = st.qm.skew;
            skc = st.qc.skew;
            skp = st.qp.skew;
            __syncthreads();
            // the block's masks and anchor are read whether or not the thread
            // has a block (index 0 then, inside the buffers; the results are
            // dropped), so the reads go out together
            lds_block_union_count<R, C>((const uint8_t *)s_mask + skm, tb, un, cnt);
            col0 = ((const int *)((const uint8_t *)s_col + skc))[tb];
            gather();
            __builtin_amdgcn_sched_barrier(0);
            st.issue(q0, q1, c0, c1, w0, w1, val, masks, blk_col, blk_ptr);
            __builtin_amdgcn_sched_barrier(0);
        }
        const uint8_t *smb = (const uint8_t *)s_mask + skm;
        const int *scol = (const int *)((const uint8_t *)s_col + skc);
        const int *sbp = (const int *)((const uint8_t *)s_bp + skp);
        const T *sval = (const T *)((const uint8_t *)s_val + skv);

        if constexpr (!PB) {
            // 2. block value offsets (workgroup exclusive scan of block
            // popcounts): the wavefront totals need a barrier of their own
            incl = wave_incl_scan(cnt);
            if (lane == kWave - 1) s_wsum[wv] = incl;
            if (has) {
#pragma unroll
                for (int k = 0; k < C; ++k) s_x[k * BT + tb] = xw[k];
            }
            __syncthreads();
        }
        {
            int before = 0;
#pragma unroll
            for (int w2 = 0; w2 < kWG / kWave; ++w2) before += w2 < wv ? s_wsum[w2] : 0;
            if (has) {
                s_boff[tb] = before + incl - cnt;
                if constexpr (PB) {
#pragma unroll
                    for (int k = 0; k < C; ++k) s_x[k * BT + tb] = xw[k];
                }
            }
        }
        __syncthreads();

        // 4. rows and 5. butterfly, then one store per row
        int pl, i;
        bool lead;
        const T accs = tile_rows<T, R, C, U, SPARSE, VAR, BT>(np, b0, b1, sbp, smb, s_boff, sval,
                                                          s_x, s_zero, pl, i, lead, scol, &xbuf,
                                                          s_red);
        if (lead) {
            const int64_t row = (int64_t)(p0 + pl) * R + i;
            if (f0) partial[(f0 - 1) * R + i] = accs;    // piece slot: k_split_fixup
            else if (row < nrows) y[row] = accs;
        }
        f0 = g0; p0 = q0; p1 = q1; b0 = c0; b1 = c1; v0 = w0; v1 = w1;
    }
}

// ---------------------------------------------------------------- value mode

// Workgroups of k_spmv_vstream that the LDS of a compute unit holds at once
// (as for k_spmv_stream), requested from the compiler for FP32 only and at
// most 6: beyond that the register budget makes it spill.
template <typename T, int C, int NVG>
constexpr int vstream_residency() {
    using Cfg = StreamCfg<T, 1, C, NVG>;
    constexpr int vcap = Cfg::VVEC * 16 / (int)sizeof(T);
    constexpr int lds = 16 * (Cfg::VVEC + Cfg::MVEC + Cfg::CVEC + Cfg::PVEC) + 4 * vcap +
                        2 * (Cfg::BT + 2) + 4 * (kWG / kWave) + 4 * kWG + 4;
    constexpr int units = (lds + 511) / 512;
    constexpr int wg = (160 * 1024 / 512) / units;
    return sizeof(T) == 4 ? (wg > 6 ? 6 : wg) : 1;
}

// beta(1,c) in VALUE MODE: with one row per block there is no x window to
// share between rows, and at low fill most of a block's c columns are empty,
// so the x loads go per nonzero instead of per block column.  Per tile: the
// block popcount scan gives every block its first value; one thread per block
// decodes its values' columns (anchor + position of each set bit) into LDS;
// every thread then gathers x for a fixed number of value slots (unconditional
// buffer loads, out of range past the tile), multiplies in place, and the
// rows -- contiguous value ranges for r = 1 -- are summed by S sub-lanes and
// a butterfly.  The staging, prefetch and piece tiles are those of the
// staged kernel.
template <typename T, int C, int NVG>
__global__ __launch_bounds__(kWG)
__attribute__((amdgpu_waves_per_eu(vstream_residency<T, C, NVG>()))) void k_spmv_vstream(
    int64_t nrows, int64_t ncols, int64_t ntiles, int tiles_per_wg, int64_t nwg, int remap,
    const int32_t *__restrict__ tile_p, const int32_t *__restrict__ tile_b,
    const int32_t *__restrict__ tile_v, const int32_t *__restrict__ tile_f,
    const int32_t *__restrict__ blk_ptr,
    const int32_t *__restrict__ blk_col, const typename MaskOf<C>::type *__restrict__ masks,
    const T *__restrict__ val, const T *__restrict__ x, T *__restrict__ y,
    T *__restrict__ partial)
{
    using Cfg = StreamCfg<T, 1, C, NVG>;
    using MT = typename MaskOf<C>::type;
    constexpr int BT = Cfg::BT;
    constexpr int VCAP = Cfg::VVEC * 16 / (int)sizeof(T);    // value slots of a tile
    constexpr int NX = (VCAP + kWG - 1) / kWG;               // value slots per thread
    __shared__ v4u s_val[Cfg::VVEC];
    // block masks and anchors through LDS only for 16-bit masks
    constexpr bool kLdsMeta = sizeof(MT) != 1;
    __shared__ v4u s_mask[kLdsMeta ? Cfg::MVEC : 1];
    __shared__ v4u s_col[kLdsMeta ? Cfg::CVEC : 1];
    __shared__ v4u s_bp[Cfg::PVEC];
    __shared__ int s_vcol[VCAP];
    // first value of every block inside the tile (< VCAP, so 16 bits do)
    __shared__ uint16_t s_boff[BT + 2];
    static_assert(VCAP < 65536, "block value offsets kept in 16 bits");
    __shared__ int s_wsum[kWG / kWave];
    __shared__ int s_long[kWG];
    __shared__ int s_nlong;

    const int th = threadIdx.x;
    const int lane = lane_id();
    const int wv = th / kWave;
    const int64_t g = remap ? xcd_chunks(blockIdx.x, nwg, kXcdRun) : (int64_t)blockIdx.x;
    const int64_t t_begin = g * tiles_per_wg;
    const int64_t t_end = min(t_begin + tiles_per_wg, ntiles);
    const Buf xbuf = make_buf(x, ncols * (int64_t)sizeof(T));

    int f0 = tile_f[t_begin];
    int p0 = tile_p[t_begin], p1 = f0 ? p0 + 1 : tile_p[t_begin + 1];
    int b0 = tile_b[t_begin], b1 = tile_b[t_begin + 1];
    int v0 = tile_v[t_begin], v1 = tile_v[t_begin + 1];
    // byte masks (c <= 8): each thread loads its own blocks' masks and anchors
    constexpr bool PB = sizeof(MT) == 1;
    using Stage = std::conditional_t<PB, VBlockStage<T, C, NVG>, TileStage<T, 1, C, NVG>>;
    Stage st;
    st.issue(p0, p1, b0, b1, v0, v1, val, masks, blk_col, blk_ptr);

    for (int64_t t = t_begin; t < t_end; ++t) {
        const bool more = t + 1 < t_end;
        const int64_t tn = more ? t + 1 : t;
        const int g0 = tile_f[tn];
        const int q0 = tile_p[tn], q1 = g0 ? q0 + 1 : tile_p[tn + 1];
        const int c0 = tile_b[tn], c1 = tile_b[tn + 1];
        const int w0 = tile_v[tn], w1 = tile_v[tn + 1];
        const int np = p1 - p0;
        const int nbt = b1 - b0;
        const int nv = v1 - v0;

        // first value of every block (workgroup scan of popcounts); thread th
        // owns blocks BPT*th .. BPT*th+BPT-1
        constexpr int BPT = Cfg::BPT;
        unsigned m[BPT];
        int cnt[BPT], own = 0, incl, skv, skp;
        const int *scol = nullptr;
        if constexpr (PB) {
            // masks in registers: the scan needs no LDS and runs before the
            // tile's barrier
#pragma unroll
            for (int q = 0; q < BPT; ++q) {
                const int tb = BPT * th + q;
                m[q] = tb < nbt ? st.mask(q) : 0u;
                cnt[q] = __popc(m[q]);
                own += cnt[q];
            }
            incl = wave_incl_scan(own);
            __syncthreads();
            st.rp.commit(s_bp, st.qp);
            st.rv.commit(s_val, st.qv);
            if (th == 0) s_nlong = 0;
            if (lane == kWave - 1) s_wsum[wv] = incl;
            skv = st.qv.skew;
            skp = st.qp.skew;
            __syncthreads();
        } else {
            __syncthreads();
            st.rm.commit(s_mask, st.qm);
            st.rc.commit(s_col, st.qc);
            st.rp.commit(s_bp, st.qp);
            st.rv.commit(s_val, st.qv);
            if (th == 0) s_nlong = 0;
            skv = st.qv.skew;
            skp = st.qp.skew;
            const int skm = st.qm.skew, skc = st.qc.skew;
            __syncthreads();
            const MT *smk = (const MT *)((const uint8_t *)s_mask + skm);
            scol = (const int *)((const uint8_t *)s_col + skc);
#pragma unroll
            for (int q = 0; q < BPT; ++q) {
                const int tb = BPT * th + q;
                m[q] = tb < nbt ? (unsigned)smk[tb] : 0u;
                cnt[q] = __popc(m[q]);
                own += cnt[q];
            }
            incl = wave_incl_scan(own);
            if (lane == kWave - 1) s_wsum[wv] = incl;
            __syncthreads();
        }
        const int *sbp = (const int *)((const uint8_t *)s_bp + skp);
        T *sval = (T *)((uint8_t *)s_val + skv);
        int before = 0, total = 0;
#pragma unroll
        for (int w2 = 0; w2 < kWG / kWave; ++w2) {
            before += w2 < wv ? s_wsum[w2] : 0;
            total += s_wsum[w2];
        }
        int boff = before + incl - own;
        if (th == 0) s_boff[nbt] = (uint16_t)total;
        // column of every value: anchor + position of each set bit
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            const int tb = BPT * th + q;
            if (tb < nbt) {
                s_boff[tb] = (uint16_t)boff;
                int c0b;
                if constexpr (PB) c0b = (int)st.cl[q];
                else c0b = scol[tb];
                unsigned mm = m[q];
                int v = boff;
                while (mm) {
                    s_vcol[v++] = c0b + __ffs(mm) - 1;
                    mm &= mm - 1u;
                }
            }
            boff += cnt[q];
        }
        __syncthreads();

        // one x load per value slot, then the next tile's staging loads
        T xg[NX];
#pragma unroll
        for (int k = 0; k < NX; ++k) {
            const int v = th + kWG * k;
            xg[k] = buf_load<T>(xbuf, v < nv ? (uint32_t)s_vcol[v] * (uint32_t)sizeof(T) : kOOB);
        }
        __builtin_amdgcn_sched_barrier(0);
        st.issue(q0, q1, c0, c1, w0, w1, val, masks, blk_col, blk_ptr);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < NX; ++k) {
            const int v = th + kWG * k;
            if (v < nv) sval[v] = sval[v] * xg[k];
        }
        __syncthreads();

        // rows: contiguous sums of the products
        value_rows<T, 1>(
            np,
            [&](int pl, int &vs, int &ve) {
                vs = s_boff[max(sbp[pl], b0) - b0];
                ve = s_boff[min(sbp[pl + 1], b1) - b0];
            },
            [&](int v, T *acc) { acc[0] += sval[v]; },
            [&](int pl, const T *acc) {
                const int64_t row = (int64_t)(p0 + pl);
                if (f0) partial[f0 - 1] = acc[0];    // piece slot: k_split_fixup
                else if (row < nrows) y[row] = acc[0];
            },
            s_long, &s_nlong);
        f0 = g0; p0 = q0; p1 = q1; b0 = c0; b1 = c1; v0 = w0; v1 = w1;
    }
}

// ---------------------------------------------------------------- schedule

// Greedy tiles inside each group of kTileGroup*ppw consecutive panels: a
// panel starts a new tile when adding it would pass vt values, bt blocks or
// ppw panels.  A panel larger
// than a whole tile is cut into pieces of at most vt values and bt blocks,
// each a tile of its own flagged as a piece; the pieces' partial row sums
// are added in a fixed order by k_split_fixup, so the result stays
// reproducible.  One thread per group; pass 0 counts the tiles and the split
// panels of each group, pass 1 writes them.
// Tile groups are this many tile widths long: tiles never cross a group
// edge, so a group much longer than a tile leaves few short tiles at edges.
constexpr int kTileGroup = 8;

__global__ void k_tile_groups(int pass, int64_t npanels, int ppw, int vt, int bt,
                              const int32_t *bp, const int32_t *pv, const int64_t *vpre,
                              int64_t *count, const int64_t *first, int64_t *scount,
                              const int64_t *sfirst, int32_t *tp, int32_t *tb, int32_t *tv,
                              int32_t *tf, int32_t *sp, int32_t *st0, int32_t *st1,
                              int *maxvals) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t gw = (int64_t)kTileGroup * ppw;
    const int64_t ng = (npanels + gw - 1) / gw;
    if (g >= ng) return;
    const int64_t pa = g * gw, pz = min(pa + gw, npanels);
    int64_t n = 0, o = pass ? first[g] : 0;
    int64_t ns = 0, so = pass ? sfirst[g] : 0;
    int64_t start = -1;   // first panel of the open tile, -1: none open
    auto emit = [&](int64_t p, int b, int v, int flag) {
        if (pass) {
            tp[o + n] = (int32_t)p;
            tb[o + n] = b;
            tv[o + n] = v;
            tf[o + n] = flag;
        }
        ++n;
    };
    for (int64_t p = pa; p < pz; ++p) {
        if (pv[p + 1] - pv[p] > vt || bp[p + 1] - bp[p] > bt) {
            if (start >= 0) atomicMax(maxvals, pv[p] - pv[start]);
            start = -1;
            if (pass) {
                sp[so + ns] = (int32_t)p;
                st0[so + ns] = (int32_t)(o + n);
            }
            // pieces: from block pb, the longest run [pb, e) with at most bt
            // blocks and vt values (vpre: values before each block), found by
            // binary search -- the same cuts as a walk over the blocks
            const int be = bp[p + 1];
            int pb = bp[p];
            int64_t pvv = pv[p];
            emit(p, pb, (int)pvv, 1);
            for (;;) {
                int lo = pb + 1, hi = min(pb + bt, be);   // one block never exceeds vt
                while (lo < hi) {
                    const int mid = (lo + hi + 1) / 2;
                    if (vpre[mid] - pvv <= vt) lo = mid;
                    else hi = mid - 1;
                }
                atomicMax(maxvals, (int)(vpre[lo] - pvv));
                if (lo >= be) break;
                pb = lo;
                pvv = vpre[lo];
                emit(p, pb, (int)pvv, 1);
            }
            if (pass) st1[so + ns] = (int32_t)(o + n - 1);
            ++ns;
            continue;
        }
        const bool cut = start >= 0 && (pv[p + 1] - pv[start] > vt ||
                                        bp[p + 1] - bp[start] > bt || p - start >= ppw);
        if (start < 0 || cut) {
            if (start >= 0) atomicMax(maxvals, pv[p] - pv[start]);
            emit(p, bp[p], pv[p], 0);
            start = p;
        }
    }
    if (start >= 0) atomicMax(maxvals, pv[pz] - pv[start]);
    if (!pass) {
        count[g] = n;
        scount[g] = ns;
    }
}

__global__ void k_tile_sentinel(int64_t npanels, int64_t ntiles, const int32_t *bp,
                                const int32_t *pv, int32_t *tp, int32_t *tb, int32_t *tv,
                                int32_t *tf) {
    tp[ntiles] = (int32_t)npanels;
    tb[ntiles] = bp[npanels];
    tv[ntiles] = pv[npanels];
    tf[ntiles] = 0;
}

// Rows of a split panel: the partial sums of its pieces.  The pieces of
// split panel s are the consecutive tiles st0[s]..st1[s], whose piece slots
// (tile_f - 1) are consecutive too.  One wavefront per row (a hub row can
// have hundreds of pieces): lane l adds pieces l, l+64, ... in tile order,
// then a butterfly; the order is fixed, so the result is reproducible.
template <typename T>
__global__ __launch_bounds__(256) void k_split_fixup(int64_t nsplit, int r, int64_t nrows,
                                                     const int32_t *sp, const int32_t *st0,
                                                     const int32_t *st1, const int32_t *tile_f,
                                                     const T *partial, T *y) {
    const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (q >= nsplit * r) return;    // uniform over the wavefront
    const int lane = lane_id();
    const int64_t s = q / r;
    const int i = (int)(q % r);
    const int64_t row = (int64_t)sp[s] * r + i;
    if (row >= nrows) return;
    const int64_t t0 = st0[s], slot0 = (int64_t)tile_f[t0] - 1;
    T acc = T(0);
    for (int64_t t = t0 + lane; t <= st1[s]; t += kWave)
        acc += partial[(slot0 + t - t0) * r + i];
    for (int d = 1; d < kWave; d <<= 1) acc += __shfl_xor(acc, d);
    if (lane == 0) y[row] = acc;
}

static void launch_tile_groups(unsigned grid, int pass, const spc5_matrix *A, int ppw, int vt,
                               int bt, const int64_t *vpre, int64_t *count, const int64_t *first,
                               int64_t *scount, const int64_t *sfirst, int32_t *tp, int32_t *tb,
                               int32_t *tv, int32_t *tf, int32_t *sp, int32_t *st0, int32_t *st1,
                               int *maxvals) {
    hipLaunchKernelGGL(k_tile_groups, dim3(grid), dim3(256), 0, nullptr, pass, A->npanels, ppw,
                       vt, bt, A->blk_ptr, A->panel_val, vpre, count, first, scount, sfirst, tp,
                       tb, tv, tf, sp, st0, st1, maxvals);
}

// flag = 1 when some panel is longer than a tile (vt values or bt blocks).
__global__ void k_flag_long(int64_t npanels, const int32_t *bp, const int32_t *pv, int vt,
                            int bt, int *flag) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < npanels && (pv[p + 1] - pv[p] > vt || bp[p + 1] - bp[p] > bt)) *flag = 1;
}

// Values of every block (popcount of its r row masks).
template <typename MT>
__global__ void k_block_values(int64_t nblocks, int r, const MT *masks, int64_t *cnt) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblocks) return;
    int n = 0;
    for (int i = 0; i < r; ++i) n += __popc((unsigned)masks[b * r + i]);
    cnt[b] = n;
}

void free_staged_schedule(spc5_matrix *A) {
    for (int32_t **p : {&A->tile_p, &A->tile_b, &A->tile_v, &A->tile_f, &A->split_p,
                        &A->split_t0, &A->split_t1}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    A->ntiles_staged = 0;
    A->nsplit = 0;
    A->npieces = 0;
}

static int build_schedule_bt(spc5_matrix *A, int ppw_req, bool alone, int bt_cap,
                             int vt_cap = 0);
static int stream_occupancy(const spc5_matrix *A, int nvg);

// Tiles resident per compute unit over the launch: resident workgroups of
// the kernel the schedule selects, per tile of the schedule.  Tiles of one
// matrix carry the same bytes in total, so the larger this is, the more
// bytes are in flight.
static double schedule_score(const spc5_matrix *A) {
    if (A->ntiles_staged == 0) return 0.0;
    const int sz = A->dtype == SPC5_F64 ? 8 : 4;
    return (double)stream_occupancy(A, stream_nvg(A->max_tile_values, sz)) /
           (double)A->ntiles_staged;
}

// The staged schedule.  For r > 1 two tile sizes compete: values up to the
// 12 KiB buffer with the full block cap, and up to 16 KiB with the 16 KiB
// buffer's smaller block cap.  Larger tiles mean fewer tiles, but their
// kernel may hold fewer workgroups per compute unit; the schedule with more
// resident workgroups per tile is kept.
int build_staged_schedule(spc5_matrix *A, int ppw_req, bool alone) {
    int st = build_schedule_bt(A, ppw_req, alone, 0);
    if (st != SPC5_OK || A->r == 1) return st;
    const int sz = A->dtype == SPC5_F64 ? 8 : 4;
    const int cm = A->c <= 4 ? 4 : (A->c <= 8 ? 8 : 16);
    const int bt4 = stream_bt(sz, cm, 4);
    if (stream_nvg(A->max_tile_values, sz) < 4) return st;    // 12 KiB holds every tile
    // the 16 KiB buffer holds fewer blocks: rebuild with its cap, then
    // compare with tiles capped at 12 KiB of values
    if (bt4 < A->tile_bt && (st = build_schedule_bt(A, ppw_req, alone, bt4)) != SPC5_OK)
        return st;
    const double s4 = schedule_score(A);
    const int vt3 = (12288 - 16) / sz;
    if ((st = build_schedule_bt(A, ppw_req, alone, 0, vt3)) != SPC5_OK) return st;
    const double s3 = schedule_score(A);
    if (s4 > s3) st = build_schedule_bt(A, ppw_req, alone, bt4);
    return st;
}

int fit_schedule_to_variants(spc5_matrix *A, bool variant) {
    if (A->r == 1) return SPC5_OK;
    const int sz = A->dtype == SPC5_F64 ? 8 : 4;
    const int cm = A->c <= 4 ? 4 : (A->c <= 8 ? 8 : 16);
    const int bt4 = stream_bt(sz, cm, 4);
    if (variant) return A->tile_bt > bt4 ? build_schedule_bt(A, A->sppt, true, bt4) : SPC5_OK;
    int vt, bt, ppw;
    staged_caps(A, &vt, &bt, &ppw);
    return A->tile_bt < bt ? build_staged_schedule(A, A->sppt) : SPC5_OK;
}

static int build_schedule_bt(spc5_matrix *A, int ppw_req, bool alone, int bt_cap,
                             int vt_cap) {
    free_staged_schedule(A);
    A->staged_ok = true;
    int vt, bt, ppw;
    staged_caps(A, &vt, &bt, &ppw);
    if (bt_cap > 0) bt = std::min(bt, bt_cap);
    if (vt_cap > 0) vt = std::min(vt, vt_cap);
    if (ppw_req > 0) ppw = std::min(ppw, ppw_req);
    // small matrices launched alone: narrower tiles, so that there are about
    // 2048 of them to spread over the 256 compute units (a batch, which
    // spreads many matrices, keeps full tiles)
    if (alone) {
        bt = (int)std::min<int64_t>(bt, std::max<int64_t>(32, A->nblocks / 2048));
        vt = (int)std::min<int64_t>(vt, std::max<int64_t>(256, A->nnz / 2048));
    }
    A->sppt = ppw;
    A->tile_bt = bt;
    A->max_tile_values = 0;
    if (A->npanels == 0) return SPC5_OK;
    hipStream_t s = nullptr;
    hipError_t e;
    int64_t *count = nullptr, *first = nullptr, *scount = nullptr, *sfirst = nullptr;
    int64_t *scratch = nullptr, *scratch2 = nullptr, *bcnt = nullptr, *vpre = nullptr;
    int64_t *scratch3 = nullptr;
    int *maxv = nullptr;
    auto cleanup = [&]() {
        for (void *p : {(void *)count, (void *)first, (void *)scount, (void *)sfirst,
                        (void *)scratch, (void *)scratch2, (void *)maxv, (void *)bcnt,
                        (void *)vpre, (void *)scratch3})
            if (p) (void)hipFree(p);
    };
    auto bail = [&](hipError_t err, const char *what) {
        cleanup();
        free_staged_schedule(A);
        return hip_fail(err, what);
    };
    const int64_t np = A->npanels;
    const int64_t gw = (int64_t)kTileGroup * ppw;
    const int64_t ng = (np + gw - 1) / gw;
    const unsigned grid = (unsigned)((ng + 255) / 256);
    const bool m8 = A->mask_bytes == 1;
    if ((e = hipMalloc((void **)&count, (size_t)ng * 8)) != hipSuccess ||
        (e = hipMalloc((void **)&first, (size_t)(ng + 1) * 8)) != hipSuccess ||
        (e = hipMalloc((void **)&scount, (size_t)ng * 8)) != hipSuccess ||
        (e = hipMalloc((void **)&sfirst, (size_t)(ng + 1) * 8)) != hipSuccess ||
        (e = hipMalloc((void **)&maxv, 8)) != hipSuccess)
        return bail(e, "allocating the tile schedule");
    if ((e = zero_fill(maxv, 2, 4, s)) != hipSuccess) return bail(e, "clearing the schedule");
    // panels longer than a tile: values before every block, for the piece cuts
    hipLaunchKernelGGL(k_flag_long, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, np,
                       A->blk_ptr, A->panel_val, vt, bt, maxv + 1);
    int has_long = 0;
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpy(&has_long, maxv + 1, 4, hipMemcpyDeviceToHost)) != hipSuccess)
        return bail(e, "scanning panel lengths");
    if (has_long) {
        const int64_t nb = A->nblocks;
        if ((e = hipMalloc((void **)&bcnt, (size_t)std::max<int64_t>(nb, 1) * 8)) != hipSuccess ||
            (e = hipMalloc((void **)&vpre, (size_t)(nb + 1) * 8)) != hipSuccess)
            return bail(e, "allocating the tile schedule");
        const unsigned gb = (unsigned)((nb + 255) / 256);
        if (nb > 0) {
            if (m8)
                hipLaunchKernelGGL(k_block_values<uint8_t>, dim3(gb), dim3(256), 0, s, nb, A->r,
                                   (const uint8_t *)A->masks, bcnt);
            else
                hipLaunchKernelGGL(k_block_values<uint16_t>, dim3(gb), dim3(256), 0, s, nb,
                                   A->r, (const uint16_t *)A->masks, bcnt);
        }
        if ((e = hipGetLastError()) != hipSuccess ||
            (e = excl_scan_i64(bcnt, nb, vpre, s, &scratch3)) != hipSuccess)
            return bail(e, "counting block values");
    }
    launch_tile_groups(grid, 0, A, ppw, vt, bt, vpre, count, nullptr, scount, nullptr, nullptr,
                       nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, maxv);
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = excl_scan_i64(count, ng, first, s, &scratch)) != hipSuccess ||
        (e = excl_scan_i64(scount, ng, sfirst, s, &scratch2)) != hipSuccess)
        return bail(e, "counting tiles");
    int64_t ntiles = 0, nsplit = 0;
    if ((e = hipMemcpy(&ntiles, first + ng, 8, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(&nsplit, sfirst + ng, 8, hipMemcpyDeviceToHost)) != hipSuccess)
        return bail(e, "reading the tile count");
    if (ntiles >= ((int64_t)1 << 31)) {
        cleanup();
        free_staged_schedule(A);
        return fail(SPC5_EUNSUPPORTED, "too many tiles");
    }
    const size_t nt1 = (size_t)ntiles + 1, ns1 = (size_t)std::max<int64_t>(nsplit, 1);
    if ((e = hipMalloc((void **)&A->tile_p, nt1 * 4 + kPad)) != hipSuccess ||
        (e = hipMalloc((void **)&A->tile_b, nt1 * 4 + kPad)) != hipSuccess ||
        (e = hipMalloc((void **)&A->tile_v, nt1 * 4 + kPad)) != hipSuccess ||
        (e = hipMalloc((void **)&A->tile_f, nt1 * 4 + kPad)) != hipSuccess ||
        (e = hipMalloc((void **)&A->split_p, ns1 * 4)) != hipSuccess ||
        (e = hipMalloc((void **)&A->split_t0, ns1 * 4)) != hipSuccess ||
        (e = hipMalloc((void **)&A->split_t1, ns1 * 4)) != hipSuccess)
        return bail(e, "allocating the tile schedule");
    launch_tile_groups(grid, 1, A, ppw, vt, bt, vpre, nullptr, first, nullptr, sfirst, A->tile_p,
                       A->tile_b, A->tile_v, A->tile_f, A->split_p, A->split_t0, A->split_t1,
                       maxv);
    hipLaunchKernelGGL(k_tile_sentinel, dim3(1), dim3(1), 0, s, np, ntiles, A->blk_ptr,
                       A->panel_val, A->tile_p, A->tile_b, A->tile_v, A->tile_f);
    int hmax = 0;
    if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess ||
        (e = hipMemcpy(&hmax, maxv, 4, hipMemcpyDeviceToHost)) != hipSuccess)
        return bail(e, "filling the tile schedule");
    // piece slots: the pieces numbered in tile order, tile_f = slot + 1, so
    // that their partial row sums take npieces*r values rather than one row
    // set per tile
    int64_t npieces = 0;
    if (nsplit > 0) {
        std::vector<int32_t> tf(nt1);
        if ((e = hipMemcpy(tf.data(), A->tile_f, nt1 * 4, hipMemcpyDeviceToHost)) != hipSuccess)
            return bail(e, "numbering the piece tiles");
        for (size_t t = 0; t < (size_t)ntiles; ++t)
            if (tf[t]) tf[t] = (int32_t)++npieces;
        if ((e = hipMemcpy(A->tile_f, tf.data(), nt1 * 4, hipMemcpyHostToDevice)) != hipSuccess)
            return bail(e, "numbering the piece tiles");
    }
    A->max_tile_values = hmax;
    A->ntiles_staged = ntiles;
    A->nsplit = nsplit;
    A->npieces = npieces;
    cleanup();
    return SPC5_OK;
}

// ---------------------------------------------------------------- launch

template <typename T, int R, int C, int NVG, bool SPARSE, int VAR = 0>
static hipError_t launch_stream_g(const spc5_matrix *A, const T *val, const T *x, T *y,
                                  hipStream_t s, int remap, T *partial) {
    const int64_t nt = A->ntiles_staged;
    if (nt == 0) return hipSuccess;
    // consecutive tiles per workgroup, the next one always prefetched: 8 on
    // very large matrices (fewer workgroup start-ups), fewer on smaller ones
    // (enough workgroups to spread); SPC5_TILES_PER_WG overrides
    static int tpw_env = -2;
    if (tpw_env == -2) {
        const char *e = getenv("SPC5_TILES_PER_WG");
        tpw_env = e ? std::max(1, atoi(e)) : -1;
    }
    const int tpw = tpw_env > 0 ? tpw_env
                                : (nt >= 32768 ? 8 : nt >= 8192 ? 4 : nt >= 4096 ? 2 : 1);
    const int64_t nwg = (nt + tpw - 1) / tpw;
    if constexpr (R == 1)
        hipLaunchKernelGGL((k_spmv_vstream<T, C, NVG>), dim3((unsigned)nwg), dim3(kWG), 0, s,
                           A->nrows, A->ncols, nt, tpw, nwg, remap, A->tile_p, A->tile_b,
                           A->tile_v, A->tile_f, A->blk_ptr, A->blk_col,
                           (const typename MaskOf<C>::type *)A->masks, val, x, y, partial);
    else
        hipLaunchKernelGGL((k_spmv_stream<T, R, C, NVG, SPARSE, VAR>), dim3((unsigned)nwg), dim3(kWG),
                           0, s, A->nrows, A->ncols, nt, tpw, nwg, remap, A->tile_p, A->tile_b,
                           A->tile_v, A->tile_f, A->blk_ptr, A->blk_col,
                           (const typename MaskOf<C>::type *)A->masks, val, x, y, partial);
    if (A->nsplit > 0) {
        const int64_t n = A->nsplit * R * kWave;    // a wavefront per row
        hipLaunchKernelGGL(k_split_fixup<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           A->nsplit, R, A->nrows, A->split_p, A->split_t0, A->split_t1,
                           A->tile_f, (const T *)partial, y);
    }
    return hipGetLastError();
}

// The rows phase loops over set bits only when a row-block holds fewer than
// c/2 nonzeros on average.
static bool sparse_rows(const spc5_matrix *A) {
    static int mode = -2;
    if (mode == -2) {
        const char *e = getenv("SPC5_ROWS_MODE");
        mode = !e ? -1 : (e[0] == 's' ? 1 : (e[0] == 'd' ? 0 : -1));
    }
    if (mode >= 0) return mode == 1;
    return A->nblocks > 0 && 2.0 * (double)A->nnz < (double)A->nblocks * A->r * A->c;
}

template <typename T, int R, int C, int NVG>
static int occupancy_g(bool sparse) {
    int blocks = 0;
    const hipError_t e =
        sparse ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                     &blocks, k_spmv_stream<T, R, C, NVG, true, 0>, kWG, 0)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                     &blocks, k_spmv_stream<T, R, C, NVG, false, 0>, kWG, 0);
    return e == hipSuccess ? blocks : 0;
}

template <typename T, int R, int C>
static int occupancy_rc(bool sparse, int nvg) {
    switch (nvg) {
        case 1: return occupancy_g<T, R, C, 1>(sparse);
        case 2: return occupancy_g<T, R, C, 2>(sparse);
        case 3: return occupancy_g<T, R, C, 3>(sparse);
        default: return occupancy_g<T, R, C, 4>(sparse);
    }
}

template <typename T>
static int occupancy_t(const spc5_matrix *A, int nvg) {
    const bool sp = sparse_rows(A);
#define SPC5_CASE(RR, CC) \
    case RR * 100 + CC: return occupancy_rc<T, RR, CC>(sp, nvg);
#define SPC5_ROW(RR) SPC5_CASE(RR, 4) SPC5_CASE(RR, 8) SPC5_CASE(RR, 16)
    switch (A->r * 100 + (A->c <= 4 ? 4 : (A->c <= 8 ? 8 : 16))) {
        SPC5_ROW(2) SPC5_ROW(3) SPC5_ROW(4) SPC5_ROW(5) SPC5_ROW(6) SPC5_ROW(7) SPC5_ROW(8)
        default: return 0;
    }
#undef SPC5_ROW
#undef SPC5_CASE
}

// Workgroups of the r > 1 staged kernel with value buffer nvg that one
// compute unit holds (registers and LDS).
static int stream_occupancy(const spc5_matrix *A, int nvg) {
    return A->dtype == SPC5_F64 ? occupancy_t<double>(A, nvg) : occupancy_t<float>(A, nvg);
}

// LDS value buffer sized to the largest tile of the matrix: 4, 8, 12 or 16
// KiB (value-mode tiles at most value_tile() values).
template <typename T, int R, int C, bool SPARSE>
static hipError_t launch_stream_s(const spc5_matrix *A, const T *val, const T *x, T *y,
                                  hipStream_t s, int remap, T *partial) {
    const int nvg = stream_nvg(A->max_tile_values, (int)sizeof(T));
    if (nvg == 1)
        return launch_stream_g<T, R, C, 1, SPARSE>(A, val, x, y, s, remap, partial);
    if (nvg == 2)
        return launch_stream_g<T, R, C, 2, SPARSE>(A, val, x, y, s, remap, partial);
    // a 12 KiB buffer where the tiles fit: one more resident workgroup per
    // compute unit (FP64 beta(4,4) Laplacian: 6 instead of 5)
    if (nvg == 3)
        return launch_stream_g<T, R, C, 3, SPARSE>(A, val, x, y, s, remap, partial);
    // value-mode tiles stop at value_tile() values (8 or 12 KiB); the 16 KiB
    // buffer holds fewer blocks (the schedule was built for it)
    if constexpr (R == 1) return hipErrorInvalidValue;
    else {
        if (A->tile_bt > StreamCfg<T, R, C, 4>::BT) return hipErrorInvalidValue;
        return launch_stream_g<T, R, C, 4, SPARSE>(A, val, x, y, s, remap, partial);
    }
}

template <typename T, int R, int C>
static hipError_t launch_stream(const spc5_matrix *A, const T *val, const T *x, T *y,
                                hipStream_t s, int remap, T *partial) {
    // ablation variants: compiled for the paper's main shapes only
    constexpr bool kVarShape = (R == 2 || R == 4 || R == 8) && (C == 4 || C == 8);
    if (A->variant != 0) {
        if constexpr (kVarShape) {
            // the variants run the 16 KiB value buffer (spc5_set_variant
            // fitted the schedule to its block cap)
            if (A->tile_bt > StreamCfg<T, R, C, 4>::BT) return hipErrorInvalidValue;
            switch (A->variant) {
                case kVarPartialX:
                    return launch_stream_g<T, R, C, 4, false, kVarPartialX>(A, val, x, y, s,
                                                                           remap, partial);
                case kVarRowReduce:
                    return launch_stream_g<T, R, C, 4, false, kVarRowReduce>(A, val, x, y, s,
                                                                            remap, partial);
                case kVarUnionX:
                    return launch_stream_g<T, R, C, 4, false, kVarUnionX>(A, val, x, y, s,
                                                                          remap, partial);
                case kVarPartialX | kVarRowReduce:
                    return launch_stream_g<T, R, C, 4, false, kVarPartialX | kVarRowReduce>(
                        A, val, x, y, s, remap, partial);
                default:
                    return hipErrorInvalidValue;
            }
        }
        return hipErrorInvalidValue;
    }
    if constexpr (R == 1)
        return launch_stream_s<T, R, C, false>(A, val, x, y, s, remap, partial);
    else
        return sparse_rows(A)
                   ? launch_stream_s<T, R, C, true>(A, val, x, y, s, remap, partial)
                   : launch_stream_s<T, R, C, false>(A, val, x, y, s, remap, partial);
}

template <typename T>
static hipError_t staged_dispatch(const spc5_matrix *A, const void *val, const void *x, void *y,
                                  hipStream_t s, int remap, void *partial) {
#define SPC5_CASE(RR, CC)                                                                    \
    case RR * 100 + CC:                                                                     \
        return launch_stream<T, RR, CC>(A, (const T *)val, (const T *)x, (T *)y, s, remap, \
                                        (T *)partial);
#define SPC5_ROW(RR) SPC5_CASE(RR, 4) SPC5_CASE(RR, 8) SPC5_CASE(RR, 16)
    switch (A->r * 100 + (A->c <= 4 ? 4 : (A->c <= 8 ? 8 : 16))) {
        SPC5_ROW(1) SPC5_ROW(2) SPC5_ROW(3) SPC5_ROW(4)
        SPC5_ROW(5) SPC5_ROW(6) SPC5_ROW(7) SPC5_ROW(8)
        default: return hipErrorInvalidValue;
    }
#undef SPC5_ROW
#undef SPC5_CASE
}

hipError_t launch_spmv_staged(const spc5_matrix *A, const void *val, const void *x, void *y,
                              hipStream_t s, int remap, void *partial) {
    if (!A->staged_ok) return hipErrorInvalidValue;
    if (A->npieces > 0 && !partial) return hipErrorInvalidValue;
    return A->dtype == SPC5_F64 ? staged_dispatch<double>(A, val, x, y, s, remap, partial)
                                : staged_dispatch<float>(A, val, x, y, s, remap, partial);
}

}  // namespace spc5
