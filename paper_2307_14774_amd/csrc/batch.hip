// Batched products Y_m = A_m X_m over many SPC5 matrices in ONE persistent
// launch, and the block-count planner used to choose beta(r,c) per matrix.
//
// Work items are (matrix, tile) pairs listed once per operand binding; a
// resident grid of single-wavefront workgroups pops items from a device
// counter until the list is exhausted (every wavefront reaches the exit), so
// small and large matrices share the GPU evenly.  The counter is cleared by a
// kernel, not a memset, and the run issues no copy and no allocation: it can
// be recorded in a HIP graph and replayed.
#include "spc5_internal.h"
#include "spmm_tile.h"
#include "stage.h"

#include <algorithm>
#include <vector>

struct spc5_batch {
    int nmat = 0;
    spc5_dtype dtype = SPC5_F64;
    int device = 0;
    std::vector<spc5_matrix *> mats;
    // bound operands
    int nrhs = 0, kchunk = 0;
    bool vmode = false;            // every matrix beta(1,c): value-mode tiles
    int nch = 0;                   // right-hand-side chunks per tile (value mode)
    int64_t nwork = 0;
    void *d_desc = nullptr;        // BatchDesc[nmat] or BatchDescV[nmat]
    int32_t *d_work = nullptr;     // matrix of each work item
    void *d_fix = nullptr;         // BatchFix[nfix]: rows of split panels
    int64_t nfix = 0;
    void *d_partial = nullptr;     // [nwork * kchunk] partial row sums of pieces
    unsigned *d_counter = nullptr;
    int grid = 0;
    // batch-private staged schedules with full-size tiles (value mode): the
    // schedule fields of these shallow copies only
    std::vector<spc5_matrix> sched;
};

namespace spc5 {

struct BatchDesc {
    const int32_t *blk_ptr;
    const int32_t *blk_col;
    const void *masks;
    const void *val;
    const int32_t *panel_val;
    const void *X;
    void *Y;
    int64_t npanels, nrows, tile0;
    int shape;   // r * 100 + (4, 8 or 16)
    int ppt;     // panels per tile for this chunk width
};

static bool batch_shape_ok(int shape) {
    switch (shape) {
        case 104: case 108: case 116: case 204: case 208: case 404: case 408: case 808:
            return true;
        default:
            return false;
    }
}

__global__ void k_reset(unsigned *c) { *c = 0u; }

template <typename T, int R, int C, int K>
__device__ __forceinline__ void batch_tile(const BatchDesc &d, int64_t tile, int t0, int ld,
                                           T *ytile) {
    spmm_tile<T, R, C, K>(tile, d.ppt, d.npanels, d.nrows, d.blk_ptr, d.blk_col,
                          (const typename MaskOf<C>::type *)d.masks, (const T *)d.val,
                          d.panel_val, (const T *)d.X + t0, (T *)d.Y + t0, ld, ytile);
}

template <typename T, int K>
__global__ __launch_bounds__(kWave) void k_batch(const BatchDesc *__restrict__ descs,
                                                 const int32_t *__restrict__ work,
                                                 int64_t nwork, unsigned *counter, int nrhs) {
    __shared__ T ytile[kSpmmTile];
    __shared__ unsigned s_w;
    for (;;) {
        if (lane_id() == 0) s_w = atomicAdd(counter, 1u);
        __syncthreads();
        const int64_t w = (int64_t)(unsigned)__builtin_amdgcn_readfirstlane((int)s_w);
        __syncthreads();
        if (w >= nwork) break;
        const BatchDesc d = descs[work[w]];
        const int64_t tile = w - d.tile0;
        for (int t0 = 0; t0 < nrhs; t0 += K) {
            switch (d.shape) {
                case 104: batch_tile<T, 1, 4, K>(d, tile, t0, nrhs, ytile); break;
                case 108: batch_tile<T, 1, 8, K>(d, tile, t0, nrhs, ytile); break;
                case 116: batch_tile<T, 1, 16, K>(d, tile, t0, nrhs, ytile); break;
                case 204: batch_tile<T, 2, 4, K>(d, tile, t0, nrhs, ytile); break;
                case 208: batch_tile<T, 2, 8, K>(d, tile, t0, nrhs, ytile); break;
                case 404: batch_tile<T, 4, 4, K>(d, tile, t0, nrhs, ytile); break;
                case 408: batch_tile<T, 4, 8, K>(d, tile, t0, nrhs, ytile); break;
                default: batch_tile<T, 8, 8, K>(d, tile, t0, nrhs, ytile); break;
            }
        }
    }
}

// ---------------------------------------------------------------- value mode

// A matrix of a value-mode batch: its staged tile schedule and operands.
struct BatchDescV {
    const int32_t *tile_p, *tile_b, *tile_v, *tile_f;
    const int32_t *blk_ptr, *blk_col;
    const void *masks, *val;
    const void *X;
    void *Y;
    int64_t nrows, ncols, w0;   // w0: first work item of the matrix
    int cclass;                 // c rounded up to 4, 8 or 16
    int pad;
};

// A split panel (a row longer than one tile) of a value-mode batch: the
// partial sums of its piece tiles t0..t1 are added in tile order.
struct BatchFix {
    int32_t mat, row, t0, t1;
};

// 16-byte value vectors per thread of a value-mode tile: value_tile() values,
// the cap of the batch-private schedules.
template <typename T>
constexpr int kBatchNVG = value_tile((int)sizeof(T)) * (int)sizeof(T) / 4096;

// Shared memory of one value-mode tile (sized for the widest mask type).
template <typename T>
struct VTileLds {
    using Cfg = StreamCfg<T, 1, 16, kBatchNVG<T>>;
    static constexpr int VCAP = Cfg::VVEC * 16 / (int)sizeof(T);
    static_assert(VCAP < 65536, "block value offsets kept in 16 bits");
    v4u val[Cfg::VVEC];
    v4u mask[Cfg::MVEC];
    v4u col[Cfg::CVEC];
    v4u bp[Cfg::PVEC];
    int vcol[VCAP];
    uint16_t boff[Cfg::BT + 2];    // first value of every block (< VCAP)
    int wsum[kWG / kWave];
    int longrow[kWG];
    int nlong;
};

// Staging registers of one value-mode tile whose masks are mb bytes wide
// (1 for c <= 8, 2 above); register counts are those of the widest case.
template <typename T>
struct BStage {
    using Cfg = StreamCfg<T, 1, 16, kBatchNVG<T>>;
    Range16 qv, qm, qc, qp;
    RegStage<Cfg::NV> rv;
    RegStage<Cfg::NM> rm;
    RegStage<Cfg::NC> rc;
    RegStage<Cfg::NP> rp;
    template <int N>
    __device__ __forceinline__ static void fixed(RegStage<N> &st, const Range16 &q) {
        const uint32_t th16 = (uint32_t)threadIdx.x * 16u;
#pragma unroll
        for (int g = 0; g < N; ++g) st.r[g] = buf_load16(q.buf, th16 + (uint32_t)(kWG * 16 * g));
    }
    __device__ __forceinline__ void issue(const BatchDescV &d, const TileBounds &b, int mb) {
        qv = range16(d.val, (int64_t)b.v0 * (int64_t)sizeof(T), (int64_t)b.v1 * (int64_t)sizeof(T));
        qm = range16(d.masks, (int64_t)b.b0 * mb, (int64_t)b.b1 * mb);
        qc = range16(d.blk_col, (int64_t)b.b0 * 4, (int64_t)b.b1 * 4);
        qp = range16(d.blk_ptr, (int64_t)b.p0 * 4, (int64_t)(b.p1 + 1) * 4);
        fixed(rv, qv);
        fixed(rm, qm);
        fixed(rc, qc);
        fixed(rp, qp);
    }
    __device__ __forceinline__ void commit(VTileLds<T> &L) const {
        rm.commit(L.mask, qm);
        rc.commit(L.col, qc);
        rp.commit(L.bp, qp);
        rv.commit(L.val, qv);
    }
};

// KC consecutive entries of row `row` of X (leading dimension ld).
template <typename T, int KC>
__device__ __forceinline__ void load_xrow(const Buf &xb, int64_t row, int ld, int t0, T *out) {
    const uint32_t off = (uint32_t)((row * ld + t0) * (int64_t)sizeof(T));
    if constexpr (KC == 1) {
        out[0] = buf_load<T>(xb, off);
    } else {
        constexpr int NV = KC * (int)sizeof(T) / 16;
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
}

// Row sums of a value-mode tile for K right-hand sides split over G lanes
// per row sub-lane (K/G each), for K up to 16: like value_rows, but the G
// lanes of a sub-lane walk the same values, each loading its K/G entries of
// the value's X row, so one wavefront load instruction covers whole X rows
// of several values instead of one entry group of many; the accumulators per
// lane stay at K/G.  Rows are summed in a fixed order (reproducible).
// term(v, g, acc) adds value slot v for lane group g into acc[0..K/G);
// emit(row, g, acc) stores.  *s_nlong must be zero at entry.
template <typename T, int KG, int G, typename Range, typename Term, typename Emit>
__device__ __forceinline__ void value_rows_g(int np, Range range, Term term, Emit emit,
                                             int *s_long, int *s_nlong) {
    const int th = threadIdx.x, lane = lane_id(), wv = th / kWave;
    int lgS = 0;
    while (np * (2 << lgS) * G <= kWG && (2 << lgS) * G <= kWave) ++lgS;
    const int S = 1 << lgS;
    // rows in rounds of kWG / (S*G): a tile may hold more rows than the
    // workgroup has lane groups
    const int per_round = kWG / (S * G);
    const int sub = (th / G) & (S - 1), g = th % G;
    for (int base = 0; base < np; base += per_round) {
        const int pl = base + th / (S * G);
        const bool live = pl < np;
        int vs = 0, ve = 0;
        if (live) range(pl, vs, ve);
        const bool lng = live && ve - vs > S * kShortRow;
        T acc[KG];
#pragma unroll
        for (int q = 0; q < KG; ++q) acc[q] = T(0);
        if (live && !lng)
            for (int v = vs + sub; v < ve; v += S) term(v, g, acc);
        if (lng && sub == 0 && g == 0) s_long[atomicAdd(s_nlong, 1)] = pl;
#pragma unroll
        for (int q = 0; q < KG; ++q)
            for (int d = G; d < S * G; d <<= 1) acc[q] += __shfl_xor(acc[q], d);
        if (live && !lng && sub == 0) emit(pl, g, acc);
    }
    __syncthreads();
    const int nl = *s_nlong;
    constexpr int WS = kWave / G;     // value strides of a wavefront
    for (int q0 = wv; q0 < nl; q0 += kWG / kWave) {
        const int row = s_long[q0];
        int rs, re;
        range(row, rs, re);
        const int ws = lane / G, wg = lane % G;
        T a[KG];
#pragma unroll
        for (int q = 0; q < KG; ++q) a[q] = T(0);
        for (int v = rs + ws; v < re; v += WS) term(v, wg, a);
#pragma unroll
        for (int q = 0; q < KG; ++q)
            for (int d = G; d < kWave; d <<= 1) a[q] += __shfl_xor(a[q], d);
        if (ws == 0) emit(row, wg, a);
    }
}

// The bounds are uniform; readfirstlane keeps them (and the staging ranges
// computed from them) in scalar registers.
__device__ __forceinline__ TileBounds item_bounds(const BatchDescV &d, int64_t tile) {
    TileBounds b = tile_bounds(tile, d.tile_p, d.tile_b, d.tile_v, d.tile_f);
    b.f = __builtin_amdgcn_readfirstlane(b.f);
    b.p0 = __builtin_amdgcn_readfirstlane(b.p0);
    b.p1 = __builtin_amdgcn_readfirstlane(b.p1);
    b.b0 = __builtin_amdgcn_readfirstlane(b.b0);
    b.b1 = __builtin_amdgcn_readfirstlane(b.b1);
    b.v0 = __builtin_amdgcn_readfirstlane(b.v0);
    b.v1 = __builtin_amdgcn_readfirstlane(b.v1);
    return b;
}

// Persistent value-mode batch.  Workgroups take chunks of kGrab consecutive
// (matrix, tile) items from a device counter until the list is exhausted;
// inside a chunk the next item is staged while the current one is computed,
// as in the single-matrix value-mode kernel.  Per item: block popcount scan,
// column decode, then for one right-hand side one x load per value slot (all
// in flight together) and in-place products summed per row; for several
// right-hand sides the tile stays in LDS (the matrix is streamed once) while
// each chunk of KC of them is summed, each value slot loading the chunk's KC
// entries of its X row together (for KC = 16 in FP64, one 128-byte line).  A
// butterfly over the S sub-lanes of a row, one store.
constexpr int kGrab = 4;

// FP32 tiles leave LDS for 6 resident workgroups per compute unit; the
// register budget is set to match (not for 16 right-hand sides at once, whose
// accumulators would then spill).
template <typename T, int KC>
__global__ __launch_bounds__(kWG)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && KC < 16 ? 6 : 1)))
void k_batch_v(const BatchDescV *__restrict__ descs, const int32_t *__restrict__ work,
               int64_t nwork, unsigned *counter, int nch, int ld, T *__restrict__ partial) {
    __shared__ VTileLds<T> L;
    __shared__ unsigned s_w;
    constexpr int VCAP = VTileLds<T>::VCAP;
    constexpr int NX = (VCAP + kWG - 1) / kWG;
    constexpr int BPT = StreamCfg<T, 1, 16, kBatchNVG<T>>::BPT;
    const int th = threadIdx.x;
    const int lane = lane_id();
    const int wv = th / kWave;
    for (;;) {
        if (th == 0) s_w = atomicAdd(counter, (unsigned)kGrab);
        __syncthreads();
        // uniform by construction; readfirstlane lets the compiler keep the
        // item's descriptor and pointers in scalar registers
        const int64_t wbase = (int64_t)(unsigned)__builtin_amdgcn_readfirstlane((int)s_w);
        __syncthreads();
        if (wbase >= nwork) break;
        const int64_t wend = min(wbase + kGrab, nwork);

        BatchDescV d = descs[work[wbase]];
        int64_t local = wbase - d.w0;
        TileBounds b = item_bounds(d, local);
        int mb = d.cclass > 8 ? 2 : 1;
        BStage<T> st;
        st.issue(d, b, mb);

        for (int64_t w = wbase; w < wend; ++w) {
            // the next item (the current one again past the chunk's end)
            const int64_t wn = w + 1 < wend ? w + 1 : w;
            const BatchDescV dn = descs[work[wn]];
            const int64_t localn = wn - dn.w0;
            const TileBounds bn = item_bounds(dn, localn);
            const int mbn = dn.cclass > 8 ? 2 : 1;

            __syncthreads();
            st.commit(L);
            if (th == 0) L.nlong = 0;
            __syncthreads();
            const uint8_t *smk = (const uint8_t *)L.mask + st.qm.skew;
            const int *scol = (const int *)((const uint8_t *)L.col + st.qc.skew);
            const int *sbp = (const int *)((const uint8_t *)L.bp + st.qp.skew);
            T *sval = (T *)((uint8_t *)L.val + st.qv.skew);
            const int np = b.p1 - b.p0, nbt = b.b1 - b.b0, nv = b.v1 - b.v0;

            // block value offsets and value columns
            unsigned m[BPT];
            int cnt[BPT], own = 0;
#pragma unroll
            for (int q = 0; q < BPT; ++q) {
                const int tb = BPT * th + q;
                m[q] = tb < nbt ? (mb == 1 ? (unsigned)smk[tb]
                                           : (unsigned)((const uint16_t *)smk)[tb])
                                : 0u;
                cnt[q] = __popc(m[q]);
                own += cnt[q];
            }
            const int incl = wave_incl_scan(own);
            if (lane == kWave - 1) L.wsum[wv] = incl;
            __syncthreads();
            int before = 0, total = 0;
#pragma unroll
            for (int w2 = 0; w2 < kWG / kWave; ++w2) {
                before += w2 < wv ? L.wsum[w2] : 0;
                total += L.wsum[w2];
            }
            int boff = before + incl - own;
            if (th == 0) L.boff[nbt] = (uint16_t)total;
#pragma unroll
            for (int q = 0; q < BPT; ++q) {
                const int tb = BPT * th + q;
                if (tb < nbt) {
                    L.boff[tb] = (uint16_t)boff;
                    const int c0b = scol[tb];
                    unsigned mm = m[q];
                    int v = boff;
                    while (mm) {
                        L.vcol[v++] = c0b + __ffs(mm) - 1;
                        mm &= mm - 1u;
                    }
                }
                boff += cnt[q];
            }
            __syncthreads();

            const Buf xb = make_buf(d.X, d.ncols * (int64_t)ld * (int64_t)sizeof(T));
            auto range = [&](int pl, int &vs, int &ve) {
                vs = L.boff[max(sbp[pl], b.b0) - b.b0];
                ve = L.boff[min(sbp[pl + 1], b.b1) - b.b0];
            };
            // one right-hand side: one x load per value slot (all in flight
            // together), then the next item's staging, then the products in
            // place and the row sums
            bool done = false;
            if constexpr (KC == 1) {
                if (nch == 1) {
                    T xg[NX];
#pragma unroll
                    for (int k = 0; k < NX; ++k) {
                        const int v = th + kWG * k;
                        xg[k] = buf_load<T>(xb, v < nv ? (uint32_t)L.vcol[v] * (uint32_t)sizeof(T)
                                                       : kOOB);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    st.issue(dn, bn, mbn);
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int k = 0; k < NX; ++k) {
                        const int v = th + kWG * k;
                        if (v < nv) sval[v] = sval[v] * xg[k];
                    }
                    __syncthreads();
                    value_rows<T, 1>(
                        np, range, [&](int v, T *acc) { acc[0] += sval[v]; },
                        [&](int pl, const T *acc) {
                            const int64_t row = (int64_t)(b.p0 + pl);
                            if (b.f) partial[w] = acc[0];    // summed by k_batch_fix
                            else if (row < d.nrows) ((T *)d.Y)[row] = acc[0];
                        },
                        L.longrow, &L.nlong);
                    done = true;
                }
            }
            if (!done) {
                // several right-hand sides: the tile stays in LDS while each
                // chunk of KC of them is summed, every value slot loading the
                // chunk's KC entries of its X row at once
                __builtin_amdgcn_sched_barrier(0);
                st.issue(dn, bn, mbn);
                __builtin_amdgcn_sched_barrier(0);
                for (int ch = 0; ch < nch; ++ch) {
                    const int t0 = ch * KC;
                    if (ch > 0) {
                        __syncthreads();    // every thread has read nlong
                        if (th == 0) L.nlong = 0;
                        __syncthreads();
                    }
                    // G lanes share a row sub-lane, KG right-hand sides each
                    constexpr int G = KC >= 16 ? 4 : 1, KG = KC / G;
                    value_rows_g<T, KG, G>(
                        np, range,
                        [&](int v, int g, T *acc) {
                            T xa[KG];
                            load_xrow<T, KG>(xb, L.vcol[v], ld, t0 + g * KG, xa);
                            const T a = sval[v];
#pragma unroll
                            for (int q = 0; q < KG; ++q) acc[q] = fma(a, xa[q], acc[q]);
                        },
                        [&](int pl, int g, const T *acc) {
                            const int64_t row = (int64_t)(b.p0 + pl);
                            const int c0 = t0 + g * KG;
#pragma unroll
                            for (int q = 0; q < KG; ++q) {
                                if (b.f) partial[w * ld + c0 + q] = acc[q];    // k_batch_fix
                                else if (row < d.nrows) ((T *)d.Y)[row * ld + c0 + q] = acc[q];
                            }
                        },
                        L.longrow, &L.nlong);
                }
            }
            d = dn;
            local = localn;
            b = bn;
            mb = mbn;
        }
    }
}

// Rows of split panels: partial sums of the pieces in tile order.
template <typename T, int KC>
__global__ void k_batch_fix(const BatchFix *__restrict__ fix, int64_t nfix,
                            const BatchDescV *__restrict__ descs, int nch, int ld,
                            const T *__restrict__ partial) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)nch * KC;
    if (g >= nfix * per) return;
    const BatchFix fx = fix[g / per];
    const int rhs = (int)(g % per);
    const int ch = rhs / KC, q = rhs % KC;
    const BatchDescV &d = descs[fx.mat];
    T acc = T(0);
    for (int64_t t = fx.t0; t <= fx.t1; ++t) acc += partial[(d.w0 + t) * ld + ch * KC + q];
    ((T *)d.Y)[(int64_t)fx.row * ld + rhs] = acc;
}

template <typename T, int K>
static int batch_grid() {
    int dev = 0, blocks = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<T, K>, kWave, 0) !=
            hipSuccess || blocks < 1)
        return 256 * 8;
    return blocks * prop.multiProcessorCount;
}

template <typename T, int KC>
static int batch_grid_v() {
    int dev = 0, blocks = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch_v<T, KC>, kWG, 0) !=
            hipSuccess || blocks < 1)
        return 256 * 4;
    return blocks * prop.multiProcessorCount;
}

template <typename T, int KC>
static void launch_batch_vk(const spc5_batch *B, hipStream_t s) {
    const BatchDescV *d = (const BatchDescV *)B->d_desc;
    hipLaunchKernelGGL((k_batch_v<T, KC>), dim3(B->grid), dim3(kWG), 0, s, d, B->d_work,
                       B->nwork, B->d_counter, B->nch, B->nrhs, (T *)B->d_partial);
    if (B->nfix > 0) {
        const int64_t n = B->nfix * B->nrhs;
        const unsigned g = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL((k_batch_fix<T, KC>), dim3(g), dim3(256), 0, s,
                           (const BatchFix *)B->d_fix, B->nfix, d, B->nch, B->nrhs,
                           (const T *)B->d_partial);
    }
}

template <typename T>
static hipError_t launch_batch_v(const spc5_batch *B, hipStream_t s) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, s, B->d_counter);
    if (B->kchunk == 16) launch_batch_vk<T, 16>(B, s);
    else if (B->kchunk == 4) launch_batch_vk<T, 4>(B, s);
    else launch_batch_vk<T, 1>(B, s);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_batch(const spc5_batch *B, hipStream_t s) {
    if (B->vmode) return launch_batch_v<T>(B, s);
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, s, B->d_counter);
    const BatchDesc *d = (const BatchDesc *)B->d_desc;
    switch (B->kchunk) {
        case 16:
            hipLaunchKernelGGL((k_batch<T, 16>), dim3(B->grid), dim3(kWave), 0, s, d, B->d_work,
                               B->nwork, B->d_counter, B->nrhs);
            break;
        case 4:
            hipLaunchKernelGGL((k_batch<T, 4>), dim3(B->grid), dim3(kWave), 0, s, d, B->d_work,
                               B->nwork, B->d_counter, B->nrhs);
            break;
        default:
            hipLaunchKernelGGL((k_batch<T, 1>), dim3(B->grid), dim3(kWave), 0, s, d, B->d_work,
                               B->nwork, B->d_counter, B->nrhs);
            break;
    }
    return hipGetLastError();
}

static void drop_operands(spc5_batch *B) {
    for (void *p : {B->d_desc, (void *)B->d_work, B->d_fix, B->d_partial})
        if (p) (void)hipFree(p);
    B->d_desc = nullptr;
    B->d_work = nullptr;
    B->d_fix = nullptr;
    B->d_partial = nullptr;
    B->nwork = 0;
    B->nfix = 0;
    B->nrhs = 0;
    B->vmode = false;
}

int count_blocks_device(const int64_t *d_rowptr, const int32_t *d_colidx, int64_t nrows, int r,
                        int c, int64_t *nblocks);

// Value-mode binding: every matrix is beta(1,c) with a staged schedule.
// Work items are (matrix, staged tile) pairs, each for all right-hand sides
// (chunks of KC = 16, 4 or 1 of them); the split panels of all matrices form
// the fixup list.
template <typename T>
static int bind_value_mode(spc5_batch *B, int nrhs, const void *const *X, void *const *Y) {
    const int KC = nrhs % 16 == 0 ? 16 : (nrhs % 4 == 0 ? 4 : 1);
    const int nch = nrhs / KC;
    std::vector<BatchDescV> desc(B->nmat);
    std::vector<int32_t> work;
    std::vector<BatchFix> fix;
    int64_t w0 = 0;
    hipError_t e;
    for (int m = 0; m < B->nmat; ++m) {
        const spc5_matrix *A = B->mats[m];
        const spc5_matrix *Sd = &B->sched[m];      // full-size tile schedule
        BatchDescV &d = desc[m];
        d.tile_p = Sd->tile_p;
        d.tile_b = Sd->tile_b;
        d.tile_v = Sd->tile_v;
        d.tile_f = Sd->tile_f;
        d.blk_ptr = A->blk_ptr;
        d.blk_col = A->blk_col;
        d.masks = A->masks;
        d.val = A->val;
        d.X = X[m];
        d.Y = Y[m];
        d.nrows = A->nrows;
        d.ncols = A->ncols;
        d.w0 = w0;
        d.cclass = A->c <= 4 ? 4 : (A->c <= 8 ? 8 : 16);
        d.pad = 0;
        const int64_t items = Sd->ntiles_staged;
        if (w0 + items >= ((int64_t)1 << 31)) return fail(SPC5_EUNSUPPORTED, "too many tiles");
        work.insert(work.end(), (size_t)items, (int32_t)m);
        if (Sd->nsplit > 0) {
            std::vector<int32_t> sp((size_t)Sd->nsplit), s0((size_t)Sd->nsplit),
                s1((size_t)Sd->nsplit);
            if ((e = hipMemcpy(sp.data(), Sd->split_p, sp.size() * 4, hipMemcpyDeviceToHost)) !=
                    hipSuccess ||
                (e = hipMemcpy(s0.data(), Sd->split_t0, s0.size() * 4, hipMemcpyDeviceToHost)) !=
                    hipSuccess ||
                (e = hipMemcpy(s1.data(), Sd->split_t1, s1.size() * 4, hipMemcpyDeviceToHost)) !=
                    hipSuccess)
                return hip_fail(e, "reading split panels");
            for (size_t q = 0; q < sp.size(); ++q) fix.push_back({m, sp[q], s0[q], s1[q]});
        }
        w0 += items;
    }
    drop_operands(B);
    const size_t nw = work.size();
    if ((e = hipMalloc(&B->d_desc, sizeof(BatchDescV) * desc.size())) != hipSuccess ||
        (e = hipMalloc((void **)&B->d_work, std::max<size_t>(4, nw * 4))) != hipSuccess ||
        (!fix.empty() &&
         ((e = hipMalloc(&B->d_fix, sizeof(BatchFix) * fix.size())) != hipSuccess ||
          (e = hipMalloc(&B->d_partial, nw * (size_t)nrhs * sizeof(T))) != hipSuccess)) ||
        (e = hipMemcpy(B->d_desc, desc.data(), sizeof(BatchDescV) * desc.size(),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (nw > 0 && (e = hipMemcpy(B->d_work, work.data(), nw * 4, hipMemcpyHostToDevice)) !=
                       hipSuccess) ||
        (!fix.empty() && (e = hipMemcpy(B->d_fix, fix.data(), sizeof(BatchFix) * fix.size(),
                                        hipMemcpyHostToDevice)) != hipSuccess)) {
        drop_operands(B);
        return hip_fail(e, "binding batch operands");
    }
    B->vmode = true;
    B->nrhs = nrhs;
    B->kchunk = KC;
    B->nch = nch;
    B->nwork = (int64_t)nw;
    B->nfix = (int64_t)fix.size();
    B->grid = KC == 16 ? batch_grid_v<T, 16>() : KC == 4 ? batch_grid_v<T, 4>()
                                                         : batch_grid_v<T, 1>();
    B->grid = (int)std::max<int64_t>(1, std::min<int64_t>(B->grid, B->nwork));
    return SPC5_OK;
}

}  // namespace spc5

using namespace spc5;

extern "C" {

int spc5_batch_create(int nmat, spc5_matrix *const *mats, spc5_batch **out) {
    if (!out) return fail(SPC5_EINVAL, "out is NULL");
    *out = nullptr;
    if (nmat < 1 || !mats) return fail(SPC5_EINVAL, "need at least one matrix");
    for (int m = 0; m < nmat; ++m) {
        if (!mats[m]) return fail(SPC5_EINVAL, "matrix %d is NULL", m);
        if (mats[m]->dtype != mats[0]->dtype) return fail(SPC5_EINVAL, "mixed dtypes");
        const int shape = mats[m]->r * 100 + (mats[m]->c <= 4 ? 4 : (mats[m]->c <= 8 ? 8 : 16));
        if (!batch_shape_ok(shape))
            return fail(SPC5_EUNSUPPORTED, "matrix %d: beta(%d,%d) is not a batched shape", m,
                        mats[m]->r, mats[m]->c);
    }
    spc5_batch *B = new (std::nothrow) spc5_batch();
    if (!B) return fail(SPC5_ENOMEM, "host allocation failed");
    B->nmat = nmat;
    B->dtype = mats[0]->dtype;
    B->mats.assign(mats, mats + nmat);
    hipError_t e = hipGetDevice(&B->device);
    if (e == hipSuccess) e = hipMalloc((void **)&B->d_counter, 256);
    if (e != hipSuccess) {
        delete B;
        return hip_fail(e, "creating the batch");
    }
    // beta(1,c) batches run value-mode tiles from their own full-size
    // schedules (a matrix's own schedule is sized for a launch of its own)
    bool r1 = true;
    for (int m = 0; m < nmat; ++m) r1 = r1 && mats[m]->r == 1;
    if (r1) {
        B->sched.resize(nmat);
        for (int m = 0; m < nmat; ++m) {
            spc5_matrix &S = B->sched[m];
            const spc5_matrix *A = mats[m];
            S.nrows = A->nrows; S.ncols = A->ncols; S.nnz = A->nnz;
            S.nblocks = A->nblocks; S.npanels = A->npanels;
            S.r = A->r; S.c = A->c; S.dtype = A->dtype; S.mask_bytes = A->mask_bytes;
            S.device = A->device;
            S.blk_ptr = A->blk_ptr; S.masks = A->masks; S.panel_val = A->panel_val;
            const int st = build_staged_schedule(&S, A->batch_ppt, false);
            S.blk_ptr = nullptr; S.masks = nullptr; S.panel_val = nullptr;
            if (st != SPC5_OK) {
                spc5_batch_free(B);
                return st;
            }
            const int sz = A->dtype == SPC5_F64 ? 8 : 4;
            if ((int64_t)S.max_tile_values * sz + 16 > (int64_t)value_tile(sz) * sz) {
                spc5_batch_free(B);
                return fail(SPC5_EUNSUPPORTED, "batch tile exceeds its LDS value buffer");
            }
        }
    }
    *out = B;
    return SPC5_OK;
}

void spc5_batch_free(spc5_batch *B) {
    if (!B) return;
    drop_operands(B);
    for (spc5_matrix &S : B->sched) free_staged_schedule(&S);
    if (B->d_counter) (void)hipFree(B->d_counter);
    delete B;
}

int spc5_set_batch_schedule(spc5_matrix *A, int panels_per_tile) {
    if (!A) return fail(SPC5_EINVAL, "A is NULL");
    if (panels_per_tile < 0 || panels_per_tile > 256)
        return fail(SPC5_EINVAL, "panels_per_tile must be in 0..256");
    A->batch_ppt = panels_per_tile;
    return SPC5_OK;
}

int spc5_batch_set_operands(spc5_batch *B, int nrhs, const void *const *X, void *const *Y) {
    if (!B || !X || !Y) return fail(SPC5_EINVAL, "NULL argument");
    if (nrhs < 1 || nrhs > 64) return fail(SPC5_EINVAL, "nrhs must be in 1..64");
    // value mode when every matrix is beta(1,c) with a staged schedule and
    // every X is addressable by a 2 GiB buffer range
    bool vm = true;
    const int64_t vb = B->dtype == SPC5_F64 ? 8 : 4;
    for (int m = 0; m < B->nmat; ++m) {
        const spc5_matrix *A = B->mats[m];
        if ((!X[m] && A->ncols > 0) || (!Y[m] && A->nrows > 0))
            return fail(SPC5_EINVAL, "NULL operand for matrix %d", m);
        if (A->r != 1 || B->sched.empty() || A->ncols * nrhs * vb > kMaxBufBytes) vm = false;
    }
    if (vm)
        return B->dtype == SPC5_F64 ? bind_value_mode<double>(B, nrhs, X, Y)
                                    : bind_value_mode<float>(B, nrhs, X, Y);
    const int K = nrhs % 16 == 0 ? 16 : (nrhs % 4 == 0 ? 4 : 1);
    std::vector<BatchDesc> desc(B->nmat);
    std::vector<int32_t> work;
    int64_t tile0 = 0;
    for (int m = 0; m < B->nmat; ++m) {
        const spc5_matrix *A = B->mats[m];
        if ((!X[m] && A->ncols > 0) || (!Y[m] && A->nrows > 0))
            return fail(SPC5_EINVAL, "NULL operand for matrix %d", m);
        BatchDesc &d = desc[m];
        d.blk_ptr = A->blk_ptr;
        d.blk_col = A->blk_col;
        d.masks = A->masks;
        d.val = A->val;
        d.panel_val = A->panel_val;
        d.X = X[m];
        d.Y = Y[m];
        d.npanels = A->npanels;
        d.nrows = A->nrows;
        d.shape = A->r * 100 + (A->c <= 4 ? 4 : (A->c <= 8 ? 8 : 16));
        // a wavefront tile holds at most 64 panels (one lane per panel end)
        const int want = A->batch_ppt ? std::min(A->batch_ppt, 64) : A->ppt;
        d.ppt = std::max(1, std::min(want, kSpmmTile / (A->r * K)));
        d.tile0 = tile0;
        const int64_t nt = (A->npanels + d.ppt - 1) / d.ppt;
        if (tile0 + nt >= ((int64_t)1 << 31)) return fail(SPC5_EUNSUPPORTED, "too many tiles");
        work.insert(work.end(), (size_t)nt, (int32_t)m);
        tile0 += nt;
    }
    drop_operands(B);
    hipError_t e;
    if ((e = hipMalloc(&B->d_desc, sizeof(BatchDesc) * desc.size())) != hipSuccess ||
        (e = hipMalloc((void **)&B->d_work, std::max<size_t>(4, work.size() * 4))) != hipSuccess ||
        (e = hipMemcpy(B->d_desc, desc.data(), sizeof(BatchDesc) * desc.size(),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (!work.empty() && (e = hipMemcpy(B->d_work, work.data(), work.size() * 4,
                                         hipMemcpyHostToDevice)) != hipSuccess)) {
        drop_operands(B);
        return hip_fail(e, "binding batch operands");
    }
    B->nrhs = nrhs;
    B->kchunk = K;
    B->nwork = (int64_t)work.size();
    if (B->dtype == SPC5_F64)
        B->grid = K == 16 ? batch_grid<double, 16>() : K == 4 ? batch_grid<double, 4>()
                                                               : batch_grid<double, 1>();
    else
        B->grid = K == 16 ? batch_grid<float, 16>() : K == 4 ? batch_grid<float, 4>()
                                                              : batch_grid<float, 1>();
    B->grid = (int)std::max<int64_t>(1, std::min<int64_t>(B->grid, B->nwork));
    return SPC5_OK;
}

int spc5_batch_run(const spc5_batch *B, void *stream) {
    if (!B) return fail(SPC5_EINVAL, "B is NULL");
    if (!B->nrhs) return fail(SPC5_EINVAL, "no operands bound");
    if (B->nwork == 0) return SPC5_OK;
    hipError_t e = B->dtype == SPC5_F64 ? launch_batch<double>(B, (hipStream_t)stream)
                                        : launch_batch<float>(B, (hipStream_t)stream);
    return e == hipSuccess ? SPC5_OK : hip_fail(e, "spc5_batch_run launch");
}

int spc5_batch_spmm(spc5_batch *B, int nrhs, const void *const *X, void *const *Y,
                    void *stream) {
    int st = spc5_batch_set_operands(B, nrhs, X, Y);
    return st ? st : spc5_batch_run(B, stream);
}

int spc5_plan(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *colidx,
              int ncand, const int *r, const int *c, int64_t *nblocks) {
    if (nrows < 0 || ncols < 0 || !rowptr || ncand < 1 || !r || !c || !nblocks)
        return fail(SPC5_EINVAL, "bad argument");
    for (int q = 0; q < ncand; ++q)
        if (r[q] < 1 || r[q] > 8 || c[q] < 1 || c[q] > 16)
            return fail(SPC5_EUNSUPPORTED, "candidate %d out of range", q);
    int64_t nnz = 0;
    // the values are not needed: pass a dummy non-NULL pointer to the checks
    int st0 = validate_csr(nrows, ncols, rowptr, colidx, rowptr, &nnz);
    if (st0 != SPC5_OK) return st0;
    int64_t *d_rowptr = nullptr;
    int32_t *d_colidx = nullptr;
    hipError_t e;
    int st = SPC5_OK;
    if ((e = hipMalloc((void **)&d_rowptr, (size_t)(nrows + 1) * 8)) != hipSuccess ||
        (e = hipMalloc((void **)&d_colidx, std::max<size_t>(4, (size_t)nnz * 4))) != hipSuccess ||
        (e = hipMemcpy(d_rowptr, rowptr, (size_t)(nrows + 1) * 8, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (nnz > 0 && (e = hipMemcpy(d_colidx, colidx, (size_t)nnz * 4, hipMemcpyHostToDevice)) !=
                        hipSuccess)) {
        st = hip_fail(e, "uploading CSR for planning");
    }
    for (int q = 0; st == SPC5_OK && q < ncand; ++q)
        st = count_blocks_device(d_rowptr, d_colidx, nrows, r[q], c[q], &nblocks[q]);
    if (d_rowptr) (void)hipFree(d_rowptr);
    if (d_colidx) (void)hipFree(d_colidx);
    return st;
}

}  // extern "C"
