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

#include <algorithm>
#include <vector>

struct spc5_batch {
    int nmat = 0;
    spc5_dtype dtype = SPC5_F64;
    int device = 0;
    std::vector<spc5_matrix *> mats;
    // bound operands
    int nrhs = 0, kchunk = 0;
    int64_t nwork = 0;
    void *d_desc = nullptr;        // BatchDesc[nmat]
    int32_t *d_work = nullptr;     // matrix of each work item
    unsigned *d_counter = nullptr;
    int grid = 0;
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
        const int64_t w = s_w;
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

template <typename T>
static hipError_t launch_batch(const spc5_batch *B, hipStream_t s) {
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
    if (B->d_desc) (void)hipFree(B->d_desc);
    if (B->d_work) (void)hipFree(B->d_work);
    B->d_desc = nullptr;
    B->d_work = nullptr;
    B->nwork = 0;
    B->nrhs = 0;
}

int count_blocks_device(const int64_t *d_rowptr, const int32_t *d_colidx, int64_t nrows, int r,
                        int c, int64_t *nblocks);

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
    *out = B;
    return SPC5_OK;
}

void spc5_batch_free(spc5_batch *B) {
    if (!B) return;
    drop_operands(B);
    if (B->d_counter) (void)hipFree(B->d_counter);
    delete B;
}

int spc5_batch_set_operands(spc5_batch *B, int nrhs, const void *const *X, void *const *Y) {
    if (!B || !X || !Y) return fail(SPC5_EINVAL, "NULL argument");
    if (nrhs < 1 || nrhs > 64) return fail(SPC5_EINVAL, "nrhs must be in 1..64");
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
        d.ppt = std::max(1, std::min(A->ppt, kSpmmTile / (A->r * K)));
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
