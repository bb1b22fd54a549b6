// Tile staging shared by the staged forward kernels and the batched
// kernel: tile capacities, LDS mask helpers, and the 16-byte register
// staging of a tile's contiguous ranges (values, row masks, anchors, panel
// bounds) through raw buffer descriptors.
#pragma once

#include "spc5_internal.h"
#include "wave.h"

namespace spc5 {

constexpr int kWG = 256;   // threads per workgroup (4 wavefronts)
constexpr int kXcdRun = 32; // consecutive workgroups kept on one XCD (xcd_chunks)

// Blocks per tile for r > 1: bounded by the x windows in LDS (8 KiB, c
// entries per block) and by one thread per block (256).  With the largest
// value buffer (NVG = 4, 16 KiB) the cap is 224 blocks: 1 KiB less of
// windows and per-block tables, which lets one more workgroup reside per
// compute unit (FP64 beta(4,4): 6 instead of 5).  sz: value bytes, cm: c
// rounded up to 4, 8 or 16.
constexpr int stream_bt(int sz, int cm, int nvg) {
    const int bt0 = 8192 / (cm * sz);
    const int cap = nvg >= 4 ? 224 : 256;
    return bt0 < cap ? bt0 : cap;
}

template <typename T, int R, int C, int NVG = 4>
struct StreamCfg {
    using MT = typename MaskOf<C>::type;
    static constexpr int MB = (int)sizeof(MT);
    // LDS bytes for the values of one tile: NVG 16-byte vectors per thread
    static constexpr int VBYTES = 4096 * NVG;
    // blocks per tile (stream_bt); beta(1,c) keeps no windows (value mode)
    // and gives each thread BPT blocks
    static constexpr int BPT = R == 1 ? 4 : 1;
    static constexpr int BT = R == 1 ? kWG * BPT : stream_bt((int)sizeof(T), C, NVG);
    static constexpr int PPW = kWG / R;                                // panels per tile
    static constexpr int VVEC = VBYTES / 16;
    static constexpr int MVEC = (BT * R * MB + 30) / 16;
    static constexpr int CVEC = (BT * 4 + 30) / 16;
    static constexpr int PVEC = ((PPW + 1) * 4 + 30) / 16;
    static constexpr int NV = VVEC / kWG;                              // vectors per thread
    static constexpr int NM = (MVEC + kWG - 1) / kWG;
    static constexpr int NC = (CVEC + kWG - 1) / kWG;
    static constexpr int NP = (PVEC + kWG - 1) / kWG;
    static constexpr int U = R * C <= 16 ? 4 : 2;                      // blocks per step
};

// Values per value-mode (beta(1,c)) tile for an element of sz bytes, 16 bytes
// of padding included: 8 KiB of LDS in FP32, 12 KiB in FP64.  Each value also
// keeps its decoded column in LDS; with block offsets in 16 bits these sizes
// leave room for 6 resident workgroups per compute unit in FP32 and 5 in
// FP64, which the per-nonzero gathers need.
constexpr int value_tile(int sz) { return sz == 8 ? 1536 : 2048; }

// Tile capacities for a matrix (must match StreamCfg).
void staged_caps(const spc5_matrix *A, int *vt, int *bt, int *ppw);

// Kernel variants for the paper's ablations (spc5_set_variant).
constexpr int kVarPartialX = 1;    // each row loads its own x (Section 3.1)
constexpr int kVarRowReduce = 2;   // per-row sums of the sub-lanes (Section 3.2)
constexpr int kVarUnionX = 4;      // window pieces the union of the row masks uses (3.1)

// C consecutive entries of x from byte offset off (kOOB: none) as 16-byte
// raw buffer loads; entries past the descriptor's range read as zero (the
// range check is per dword).
template <typename T, int C>
__device__ __forceinline__ void load_window(const Buf &xb, uint32_t off, T *out) {
    constexpr int NV = C * (int)sizeof(T) / 16;
    static_assert(NV >= 1, "window narrower than one 16-byte load");
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const v4u v = buf_load16(xb, off + 16u * q);
        if constexpr (sizeof(T) == 8) {
            typedef double v2d __attribute__((ext_vector_type(2)));
            const v2d f = __builtin_bit_cast(v2d, v);
            out[2 * q] = f.x;
            out[2 * q + 1] = f.y;
        } else {
            typedef float v4f __attribute__((ext_vector_type(4)));
            const v4f f = __builtin_bit_cast(v4f, v);
            out[4 * q] = f.x;
            out[4 * q + 1] = f.y;
            out[4 * q + 2] = f.z;
            out[4 * q + 3] = f.w;
        }
    }
}

// The same window, but only the 16-byte pieces that hold a column of `un`
// (the union of the block's row masks): a piece no row uses is not loaded
// and reads as zero.
template <typename T, int C>
__device__ __forceinline__ void load_window_union(const Buf &xb, uint32_t off, unsigned un,
                                                  T *out) {
    constexpr int NV = C * (int)sizeof(T) / 16;
    constexpr int PER = 16 / (int)sizeof(T);            // columns per piece
    static_assert(NV >= 1, "window narrower than one 16-byte load");
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const unsigned pm = ((1u << PER) - 1u) << (q * PER);
        const v4u v = buf_load16(xb, (un & pm) ? off + 16u * q : kOOB);
        if constexpr (sizeof(T) == 8) {
            typedef double v2d __attribute__((ext_vector_type(2)));
            const v2d f = __builtin_bit_cast(v2d, v);
            out[2 * q] = f.x;
            out[2 * q + 1] = f.y;
        } else {
            typedef float v4f __attribute__((ext_vector_type(4)));
            const v4f f = __builtin_bit_cast(v4f, v);
            out[4 * q] = f.x;
            out[4 * q + 1] = f.y;
            out[4 * q + 2] = f.z;
            out[4 * q + 3] = f.w;
        }
    }
}

// Row masks of block t in LDS (bytes of block t start at t*R*MB): the mask of
// row i, the popcount of the rows below i and of the whole block.
template <int R, int C>
__device__ __forceinline__ void lds_block_masks(const uint8_t *sm, int t, int i, unsigned &m,
                                                int &pre, int &tot) {
    using MT = typename MaskOf<C>::type;
    constexpr int MB = (int)sizeof(MT);
    constexpr int WB = R * MB;
    if constexpr (WB == 1 || WB == 2 || WB == 4 || WB == 8) {
        uint64_t w;
        if constexpr (WB == 1) w = sm[t];
        else if constexpr (WB == 2) w = *(const uint16_t *)(sm + 2 * t);
        else if constexpr (WB == 4) w = *(const uint32_t *)(sm + 4 * t);
        else w = *(const uint64_t *)(sm + 8 * t);
        const int sh = i * 8 * MB;
        m = (unsigned)(w >> sh) & ((1u << (8 * MB)) - 1u);
        pre = __popcll(sh ? (w & ((1ull << sh) - 1ull)) : 0ull);
        tot = __popcll(w);
    } else {
        m = 0;
        pre = 0;
        tot = 0;
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            unsigned mr;
            if constexpr (MB == 1) mr = sm[t * R + rr];
            else mr = ((const uint16_t *)sm)[t * R + rr];
            const int pc = __popc(mr);
            pre += rr < i ? pc : 0;
            m = rr == i ? mr : m;
            tot += pc;
        }
    }
}

// Union of the r row masks of block t (the columns the block touches) and
// the block's value count, from one LDS read where the r masks fill 1, 2, 4
// or 8 bytes.
template <int R, int C>
__device__ __forceinline__ void lds_block_union_count(const uint8_t *sm, int t, unsigned &u,
                                                      int &tot) {
    using MT = typename MaskOf<C>::type;
    constexpr int MB = (int)sizeof(MT);
    constexpr int WB = R * MB;
    u = 0;
    if constexpr (WB == 1 || WB == 2 || WB == 4 || WB == 8) {
        uint64_t w;
        if constexpr (WB == 1) w = sm[t];
        else if constexpr (WB == 2) w = *(const uint16_t *)(sm + 2 * t);
        else if constexpr (WB == 4) w = *(const uint32_t *)(sm + 4 * t);
        else w = *(const uint64_t *)(sm + 8 * t);
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
            u |= (unsigned)(w >> (rr * 8 * MB)) & ((1u << (8 * MB)) - 1u);
        tot = __popcll(w);
    } else {
        tot = 0;
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            unsigned mr;
            if constexpr (MB == 1) mr = sm[t * R + rr];
            else mr = ((const uint16_t *)sm)[t * R + rr];
            u |= mr;
            tot += __popc(mr);
        }
    }
}

// A contiguous byte range of global memory, as 16-byte vectors from an
// aligned base, addressed through a raw buffer descriptor whose record count
// is the range's length: vector indices past the range read zeros, so the
// staging loads need no clamping.
struct Range16 {
    Buf buf;
    int n;       // vectors
    int skew;    // bytes from the aligned base to the first wanted byte
};

__device__ __forceinline__ Range16 range16(const void *base, int64_t byte0, int64_t byte1) {
    const int64_t a0 = byte0 & ~(int64_t)15;
    Range16 r;
    r.n = byte1 > byte0 ? (int)((byte1 - a0 + 15) >> 4) : 0;
    r.skew = (int)(byte0 - a0);
    r.buf = make_buf((const char *)base + a0, (int64_t)r.n * 16);
    return r;
}

// Register stage of up to NVMAX vectors per thread and the matching LDS
// stores.
template <int NVMAX>
struct RegStage {
    v4u r[NVMAX];

    __device__ __forceinline__ void commit(v4u *dst, const Range16 &q) const {
        const int th = threadIdx.x;
#pragma unroll
        for (int g = 0; g < NVMAX; ++g) {
            const int v = th + kWG * g;
            if (v < q.n) dst[v] = r[g];
        }
    }
};

template <typename T, int R, int C, int NVG>
struct TileStage {
    using Cfg = StreamCfg<T, R, C, NVG>;
    Range16 qv, qm, qc, qp;
    RegStage<Cfg::NV> rv;
    RegStage<Cfg::NM> rm;
    RegStage<Cfg::NC> rc;
    RegStage<Cfg::NP> rp;

    // All NV + NM + NC + NP loads, unconditionally (vectors past a range read
    // zeros): a fixed count keeps the compiler's in-order load counters
    // exact, so waiting for later loads of the current tile never waits for
    // this prefetch.
    __device__ __forceinline__ void issue(int p0, int p1, int b0, int b1, int v0, int v1,
                                          const T *val, const void *masks, const int32_t *blk_col,
                                          const int32_t *blk_ptr) {
        qv = range16(val, (int64_t)v0 * (int64_t)sizeof(T), (int64_t)v1 * (int64_t)sizeof(T));
        qm = range16(masks, (int64_t)b0 * R * Cfg::MB, (int64_t)b1 * R * Cfg::MB);
        qc = range16(blk_col, (int64_t)b0 * 4, (int64_t)b1 * 4);
        qp = range16(blk_ptr, (int64_t)p0 * 4, (int64_t)(p1 + 1) * 4);
        fixed(rv, qv);
        fixed(rm, qm);
        fixed(rc, qc);
        fixed(rp, qp);
    }
    template <int N>
    __device__ __forceinline__ static void fixed(RegStage<N> &st, const Range16 &q) {
        const uint32_t th16 = (uint32_t)threadIdx.x * 16u;
#pragma unroll
        for (int g = 0; g < N; ++g) st.r[g] = buf_load16(q.buf, th16 + (uint32_t)(kWG * 16 * g));
    }
};

// Tile stage with the block metadata loaded per block, for r in {2, 4, 8}
// (the r row masks of a block fill 2, 4, 8 or 16 bytes): thread b loads the
// anchor and the row masks of the tile's block b straight into registers
// (zeros past the tile's blocks), so the block's x window can be requested
// as soon as the tile lands, before anything is copied to LDS.  Values and
// panel bounds are staged as 16-byte vectors, as in TileStage.
template <int WB> struct MaskWord;
template <> struct MaskWord<2> { using type = uint16_t; };
template <> struct MaskWord<4> { using type = uint32_t; };
template <> struct MaskWord<8> { using type = uint64_t; };
template <> struct MaskWord<16> { using type = v4u; };

template <int WB>
__device__ __forceinline__ typename MaskWord<WB>::type buf_load_word(const Buf &b, uint32_t off) {
    if constexpr (WB == 2)
        return (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(b.r, (int)off, 0, 0);
    else if constexpr (WB == 4)
        return __builtin_amdgcn_raw_buffer_load_b32(b.r, (int)off, 0, 0);
    else if constexpr (WB == 8)
        return __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(b.r, (int)off, 0, 0));
    else
        return buf_load16(b, off);
}

template <typename T, int R, int C, int NVG>
struct BlockStage {
    using Cfg = StreamCfg<T, R, C, NVG>;
    static constexpr int WB = R * Cfg::MB;
    using MW = typename MaskWord<WB>::type;
    static_assert(WB == 2 || WB == 4 || WB == 8 || WB == 16, "row masks of a block: 2..16 bytes");
    Range16 qv, qp;
    RegStage<Cfg::NV> rv;
    RegStage<Cfg::NP> rp;
    MW mw;        // this thread's block: its r row masks
    int cw;       // and its anchor

    // All loads unconditionally (past the tile's range they read zeros): a
    // fixed count keeps the compiler's in-order load counters exact.
    __device__ __forceinline__ void issue(int p0, int p1, int b0, int b1, int v0, int v1,
                                          const T *val, const void *masks, const int32_t *blk_col,
                                          const int32_t *blk_ptr) {
        qv = range16(val, (int64_t)v0 * (int64_t)sizeof(T), (int64_t)v1 * (int64_t)sizeof(T));
        qp = range16(blk_ptr, (int64_t)p0 * 4, (int64_t)(p1 + 1) * 4);
        const int nb = b1 - b0;
        const Buf mb = make_buf((const uint8_t *)masks + (int64_t)b0 * WB, (int64_t)nb * WB);
        const Buf cb = make_buf(blk_col + b0, (int64_t)nb * 4);
        const uint32_t th = threadIdx.x;
        TileStage<T, R, C, NVG>::fixed(rv, qv);
        TileStage<T, R, C, NVG>::fixed(rp, qp);
        mw = buf_load_word<WB>(mb, th * (uint32_t)WB);
        cw = (int)__builtin_amdgcn_raw_buffer_load_b32(cb.r, (int)(th * 4u), 0, 0);
    }

    // Union of the block's row masks (the columns it touches) and its value
    // count, from the registers.
    __device__ __forceinline__ void union_count(unsigned &u, int &tot) const {
        constexpr int FB = 8 * Cfg::MB;                 // bits per row mask
        constexpr unsigned FM = (1u << FB) - 1u;
        u = 0;
        if constexpr (WB <= 8) {
            const uint64_t w = (uint64_t)mw;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) u |= (unsigned)(w >> (rr * FB)) & FM;
            tot = __popcll(w);
        } else {
            tot = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const unsigned d = mw[q];
                u |= (d & 0xffffu) | (d >> 16);
                tot += __popc(d);
            }
        }
    }

    // The block's masks and anchor to LDS (masks of block b at b*WB bytes).
    __device__ __forceinline__ void commit_block(uint8_t *smask, int *scol, bool has) const {
        const int th = threadIdx.x;
        if (has) {
            *(MW *)(smask + th * WB) = mw;
            scol[th] = cw;
        }
    }
};

// Value-mode (r = 1, byte masks) tile stage with the block metadata in
// registers: thread t owns blocks 4t .. 4t+3 of the tile and loads their
// four byte masks (two aligned dwords, shifted into place: the tile's first
// block need not start a dword) and their four anchors (four dword loads) itself;
// values and panel bounds are staged as 16-byte vectors, as in TileStage.
template <typename T, int C, int NVG>
struct VBlockStage {
    using Cfg = StreamCfg<T, 1, C, NVG>;
    static_assert(sizeof(typename MaskOf<C>::type) == 1 && Cfg::BPT == 4, "byte masks, 4 blocks");
    Range16 qv, qp;
    RegStage<Cfg::NV> rv;
    RegStage<Cfg::NP> rp;
    unsigned m0, m1;   // the dwords holding this thread's four masks
    int sh;            // bytes from the first dword's start to the tile's first mask
    unsigned cl[4];    // the four anchors

    __device__ __forceinline__ void issue(int p0, int p1, int b0, int b1, int v0, int v1,
                                          const T *val, const void *masks, const int32_t *blk_col,
                                          const int32_t *blk_ptr) {
        qv = range16(val, (int64_t)v0 * (int64_t)sizeof(T), (int64_t)v1 * (int64_t)sizeof(T));
        qp = range16(blk_ptr, (int64_t)p0 * 4, (int64_t)(p1 + 1) * 4);
        const int64_t ma = (int64_t)b0 & ~(int64_t)3;
        sh = b0 & 3;
        // whole dwords (the range check is per dword): the last one may hold
        // masks of the next tile, which the caller drops
        const Buf mb = make_buf((const uint8_t *)masks + ma, ((int64_t)b1 - ma + 3) & ~(int64_t)3);
        const Buf cb = make_buf(blk_col + b0, (int64_t)(b1 - b0) * 4);
        const uint32_t th = threadIdx.x;
        TileStage<T, 1, C, NVG>::fixed(rv, qv);
        TileStage<T, 1, C, NVG>::fixed(rp, qp);
        m0 = __builtin_amdgcn_raw_buffer_load_b32(mb.r, (int)(th * 4u), 0, 0);
        m1 = __builtin_amdgcn_raw_buffer_load_b32(mb.r, (int)(th * 4u + 4u), 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            cl[q] = __builtin_amdgcn_raw_buffer_load_b32(cb.r, (int)(th * 16u + 4u * q), 0, 0);
    }

    // mask of the thread's block q (0..3)
    __device__ __forceinline__ unsigned mask(int q) const {
        const uint64_t w = ((uint64_t)m1 << 32) | m0;
        return (unsigned)(w >> (8 * (sh + q))) & 0xffu;
    }
};

// Row sums of a value-mode tile.  Rows are contiguous value ranges
// (range(row, vs, ve)).  Every row gets S sub-lanes (S the largest power of
// two with np*S <= 256, at most 64) that stride its values and meet in a
// butterfly; a row longer than S*kShortRow values is instead queued in LDS
// and summed by a whole wavefront, so one long row no longer holds up the
// tile.  Each row is summed in a fixed order: results are reproducible.
// term(v, acc) adds value slot v into acc[0..K); emit(row, acc) stores.
// *s_nlong must be zero at entry (the caller clears it between barriers).
constexpr int kShortRow = 32;

template <typename T, int K, typename Range, typename Term, typename Emit>
__device__ __forceinline__ void value_rows(int np, Range range, Term term, Emit emit,
                                           int *s_long, int *s_nlong) {
    const int th = threadIdx.x, lane = lane_id(), wv = th / kWave;
    int lgS = 0;
    while (np * (2 << lgS) <= kWG && (2 << lgS) <= kWave) ++lgS;
    const int S = 1 << lgS;
    const int pl = th >> lgS, sub = th & (S - 1);
    const bool live = pl < np;
    int vs = 0, ve = 0;
    if (live) range(pl, vs, ve);
    const bool lng = live && ve - vs > S * kShortRow;
    T acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = T(0);
    if (live && !lng)
        for (int v = vs + sub; v < ve; v += S) term(v, acc);
    if (lng && sub == 0) s_long[atomicAdd(s_nlong, 1)] = pl;
#pragma unroll
    for (int q = 0; q < K; ++q)
        for (int d = 1; d < S; d <<= 1) acc[q] += __shfl_xor(acc[q], d);
    if (live && !lng && sub == 0) emit(pl, acc);
    __syncthreads();
    const int nl = *s_nlong;
    for (int q0 = wv; q0 < nl; q0 += kWG / kWave) {
        const int row = s_long[q0];
        int rs, re;
        range(row, rs, re);
        T a[K];
#pragma unroll
        for (int q = 0; q < K; ++q) a[q] = T(0);
        for (int v = rs + lane; v < re; v += kWave) term(v, a);
#pragma unroll
        for (int q = 0; q < K; ++q)
            for (int d = 1; d < kWave; d <<= 1) a[q] += __shfl_xor(a[q], d);
        if (lane == 0) emit(row, a);
    }
}

// Bounds of staged tile t: piece flag, panel range [p0,p1), block range
// [b0,b1), value range [v0,v1).  A piece tile covers one panel.
struct TileBounds {
    int f, p0, p1, b0, b1, v0, v1;
};

__device__ __forceinline__ TileBounds tile_bounds(int64_t t, const int32_t *tp, const int32_t *tb,
                                                  const int32_t *tv, const int32_t *tf) {
    TileBounds b;
    b.f = tf[t];
    b.p0 = tp[t];
    b.p1 = b.f ? b.p0 + 1 : tp[t + 1];
    b.b0 = tb[t];
    b.b1 = tb[t + 1];
    b.v0 = tv[t];
    b.v1 = tv[t + 1];
    return b;
}

}  // namespace spc5
