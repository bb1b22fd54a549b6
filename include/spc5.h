/*
 * spc5.h -- C ABI of the MI355X (gfx950) SPC5 sparse matrix/vector library.
 *
 * Method: Regnault & Bramas, "SPC5: an efficient SpMV framework vectorized
 * using ARM SVE and x86 AVX-512", arXiv 2307.14774.
 *
 * The problem statement is the one of Algorithm 1 (input: x and a matrix in
 * the beta(r,c) block format; output: y = A x), with the matrix handed over
 * in CSR (Section 2.3) and converted to SPC5 beta(r,c) (Section 2.4).
 *
 * beta(r,c) storage, as held on the device by a spc5_matrix:
 *   rows are grouped in panels of r consecutive rows, npanels = ceil(nrows/r);
 *   blk_ptr[npanels+1]  int32  block range of each panel        (block_rowptr)
 *   blk_col[nblocks]    int32  anchor column of each block      (block_colidx)
 *   masks[nblocks*r]    uint8 for c <= 8, uint16 for c > 8;
 *                              mask of row i of block b at b*r+i (block_masks)
 *   values[nnz]         packed nonzeros, block by block, row 0..r-1 inside a
 *                       block, ascending column inside a row   (values)
 * Bit k (least significant = 0) of a row mask marks column anchor+k
 * (Fig. 3 caption).  A block is anchored at the smallest column not yet
 * covered among its panel's rows and spans [anchor, anchor+c) (Section 2.4).
 * This layout is exported bit for bit by spc5_export().
 *
 * Conventions for every call:
 *  - Integer-returning calls return SPC5_OK (0) or a negative spc5_status;
 *    spc5_last_error() then holds a message for the calling thread.
 *  - No call throws; no call keeps a pointer to caller memory after it
 *    returns.
 *  - "device" pointers are HIP device allocations (e.g. torch tensors'
 *    data_ptr()) of the matrix's value type: double for SPC5_F64, float for
 *    SPC5_F32.  "host" pointers are ordinary CPU memory.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Compute calls are asynchronous on that stream; argument checks are
 *    synchronous.
 *  - A matrix handle is immutable after creation except for its schedule
 *    (spc5_set_schedule) and its transpose plan (spc5_prepare_transpose).
 *    Compute calls on one handle may overlap on several streams.  Products
 *    that need scratch memory (the partial row sums of panels cut into
 *    pieces, spc5_info.split_panels > 0; the value move of a transpose with
 *    caller values through a plan) take it from a set the handle keeps per
 *    stream, allocated on the stream's first such call and held until
 *    spc5_free: calls on one stream are ordered, and calls on different
 *    streams never share scratch.  A HIP graph captured on a stream keeps
 *    using that stream's set.  The caller must not free a handle while work
 *    that uses it is pending.
 *  - Calls must be made with the HIP device that was current at creation.
 */
#ifndef SPC5_H
#define SPC5_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spc5_matrix spc5_matrix;   /* opaque SPC5 beta(r,c) matrix */
typedef struct spc5_csr spc5_csr;         /* opaque CSR matrix (comparison kernel) */
typedef struct spc5_batch spc5_batch;     /* opaque batch of SPC5 matrices */

typedef enum { SPC5_F64 = 0, SPC5_F32 = 1 } spc5_dtype;

typedef enum {
    SPC5_OK = 0,
    SPC5_EINVAL = -1,       /* NULL pointer, negative size, bad enum value     */
    SPC5_EBADCSR = -2,      /* malformed CSR (see csr_to_spc5)                 */
    SPC5_ENOMEM = -3,       /* device or host allocation failed                */
    SPC5_EDEVICE = -4,      /* HIP runtime or launch error                     */
    SPC5_EUNSUPPORTED = -5  /* shape or size outside what the library handles  */
} spc5_status;

typedef struct {
    int64_t nrows, ncols, nnz;
    int64_t nblocks, npanels;
    int32_t r, c;
    int32_t dtype;            /* spc5_dtype */
    int32_t mask_bytes;       /* 1 (c <= 8) or 2 (c > 8) */
    int32_t panels_per_tile;  /* sweep kernel: panels handled by one wavefront */
    int32_t kernel;           /* spc5_kernel in use for the forward product */
    int64_t ntiles;           /* wavefronts of one forward launch */
    int64_t max_panel_blocks; /* longest panel, in blocks */
    double fill;              /* nnz / (nblocks * r * c), Table 1's block filling */
    int64_t spmv_bytes;       /* algorithmic bytes moved by one y = A x:
                                 values + anchors + masks + blk_ptr + x + y */
    int64_t device_bytes;     /* device memory held by the handle */
    /* transposed-product plan (spc5_prepare_transpose); all 0 without one */
    int transpose_r, transpose_c; /* beta(r,c) of the stored A^T */
    int transpose_kernel;     /* forward kernel run over A^T (spc5_kernel) */
    int variant;              /* staged-kernel variant flags (spc5_set_variant) */
    int64_t transpose_bytes;  /* algorithmic bytes of one x_bar = A^T y_bar
                                 through the plan (without the value gather) */
    int64_t split_panels;     /* panels longer than one staged tile, cut into
                                 pieces on several workgroups (0: none) */
} spc5_info;

/* ---------------------------------------------------------------- creation */

/* Convert a CSR matrix to SPC5 beta(r,c) on the device (Section 2.4).
 *  nrows, ncols >= 0, ncols <= 2^31-1;
 *  rowptr  host int64[nrows+1], rowptr[0] == 0, non-decreasing;
 *  colidx  host int32[nnz], nnz = rowptr[nrows], strictly increasing inside
 *          each row and in [0, ncols);
 *  values  host, nnz entries of double (SPC5_F64) or float (SPC5_F32);
 *          explicit zeros and non-finite values are kept as entries;
 *  1 <= r <= 8, 1 <= c <= 16.
 * The inputs are copied; the caller keeps them.  On success *out owns device
 * memory released by spc5_free; on failure *out is NULL.
 * Errors: SPC5_EINVAL (NULL out/array, negative size, bad dtype),
 * SPC5_EBADCSR (rowptr[0] != 0, decreasing rowptr, column out of range,
 * unsorted or duplicate column in a row), SPC5_EUNSUPPORTED (r or c out of
 * range, nnz or nblocks >= 2^31, ncols >= 2^31), SPC5_ENOMEM, SPC5_EDEVICE.
 * Synchronous: returns after the device arrays are complete. */
int csr_to_spc5(int64_t nrows, int64_t ncols, const int64_t *rowptr,
                const int32_t *colidx, const void *values, spc5_dtype dtype,
                int r, int c, spc5_matrix **out);

/* Release a matrix (NULL is ignored). */
void spc5_free(spc5_matrix *A);

/* Shape, sizes and schedule of a matrix.  out: host. */
int spc5_get_info(const spc5_matrix *A, spc5_info *out);

/* Copy the beta(r,c) arrays back to host memory, in the layout described at
 * the top of this file (blk_ptr widened to int64 for the caller).  Any output
 * pointer may be NULL to skip it.  Sizes: blk_ptr int64[npanels+1],
 * blk_col int32[nblocks], masks uint8/uint16[nblocks*r] (mask_bytes each),
 * values[nnz] of the matrix dtype.  Synchronous. */
int spc5_export(const spc5_matrix *A, int64_t *blk_ptr, int32_t *blk_col,
                void *masks, void *values);

/* The inverse conversion back to CSR (Section 2.4's format read the other
 * way): for each panel, block, row of the block and set mask bit in
 * ascending order, the entry (panel*r + row, anchor + bit, next packed
 * value).  Inside one row the blocks' windows are disjoint and increasing,
 * so each row comes out with its columns sorted; for a matrix made by
 * csr_to_spc5 the result is the input CSR, bit for bit.  Host outputs:
 * rowptr int64[nrows+1], colidx int32[nnz], values[nnz] of the matrix dtype;
 * colidx or values may be NULL to skip them.  Synchronous.
 * Errors: SPC5_EINVAL (NULL A or rowptr), SPC5_ENOMEM, SPC5_EDEVICE. */
int spc5_to_csr(const spc5_matrix *A, int64_t *rowptr, int32_t *colidx, void *values);

/* Forward-kernel choice.
 *  SPC5_KERNEL_STAGED: a 256-thread workgroup walks 1-8 consecutive tiles of
 *                     a schedule built at conversion (tiles capped by values
 *                     and blocks; a panel longer than a tile is cut into
 *                     pieces summed by a small fixup); each tile's packed
 *                     values, masks and anchors are pulled into LDS with
 *                     16-byte loads while the next tile's are in flight, a
 *                     workgroup scan gives every block its value offset;
 *                     r > 1: one thread per block gathers its x window
 *                     (Section 3.1's single load), rows are summed by
 *                     sub-lanes and a butterfly; r = 1: one x load per
 *                     nonzero from the decoded columns.  The default
 *                     whenever x fits a 2 GiB buffer.
 *  SPC5_KERNEL_ROWS:  one lane per panel row; the lane walks the blocks of
 *                     its panel (r lanes share a panel), no cross-lane
 *                     reduction.  Best for short and regular panels.
 *  SPC5_KERNEL_SWEEP: one wavefront per tile of consecutive panels, one lane
 *                     per block row, segmented wavefront reduction.  Handles
 *                     panels of any length evenly.
 *  SPC5_KERNEL_AUTO:  STAGED when x fits a 2 GiB buffer, SWEEP otherwise. */
typedef enum {
    SPC5_KERNEL_AUTO = 0, SPC5_KERNEL_ROWS = 1, SPC5_KERNEL_SWEEP = 2, SPC5_KERNEL_STAGED = 3
} spc5_kernel;

/* Schedule of the forward product: kernel choice and, for the sweep and
 * staged kernels, a cap on the consecutive panels of one tile (1..64; the
 * staged kernel also stops at 256/r; 0 = default: the mean panel length for
 * the sweep kernel, the value and block caps alone for the staged kernel).
 * Not safe to call while compute calls on A are in flight.
 * Errors: SPC5_EINVAL (NULL A, unknown kernel, cap out of range),
 * SPC5_EUNSUPPORTED (staged or rows kernel with x above 2 GiB). */
int spc5_set_schedule(spc5_matrix *A, int kernel, int panels_per_tile);

/* Process-wide tuning overrides, read from the environment once, at the first
 * product that needs them (for measurements; only SPC5_ROWS_MODE can change
 * the last bits of y, through another order of summation):
 *   SPC5_TILES_PER_WG=n  staged kernels: n consecutive tiles per workgroup
 *                        (default: 8 on matrices of at least 32768 tiles,
 *                        fewer on smaller ones);
 *   SPC5_ROWS_MODE=s|d   staged kernel, r > 1: the set-bit (s) or the
 *                        branch-free (d) rows loop (default: set-bit when a
 *                        block row averages fewer than c/2 nonzeros);
 *   SPC5_XCD_REMAP=0     workgroups in launch order instead of runs of 32
 *                        consecutive ones per XCD. */

/* Kernel variants of the staged forward product that reproduce the paper's
 * ablations (Table "res:perf:comp"); 0 restores the default.  Flags:
 *  SPC5_VARIANT_PARTIAL_X   "partial x load" (Section 3.1): every row loads
 *      its own x entries from memory, instead of the default single x load
 *      per block shared by the block's r rows;
 *  SPC5_VARIANT_ROW_REDUCE  per-row reduction (Section 3.2): the partial
 *      sums of a row are added one after the other through LDS, instead of
 *      the default multi-reduction (one cross-lane butterfly reducing every
 *      row of the tile together).
 *  SPC5_VARIANT_UNION_X     x load by the merged row predicates (Section
 *      3.1's third option): the single x load per block reads only the
 *      16-byte pieces of the window that hold a column some row of the block
 *      uses, instead of the whole window; not combined with the others.
 * Results stay within the accuracy of the default (summation order only).
 * Errors: SPC5_EINVAL (NULL A, unknown flags), SPC5_EUNSUPPORTED (the matrix
 * does not use the staged kernel, or r not in {2,4,8}, or c > 8). */
#define SPC5_VARIANT_PARTIAL_X 1
#define SPC5_VARIANT_ROW_REDUCE 2
#define SPC5_VARIANT_UNION_X 4
int spc5_set_variant(spc5_matrix *A, int flags);

/* ---------------------------------------------------------------- compute */

/* y[0..nrows) = A x[0..ncols) (Algorithm 1, with y overwritten: rows without
 * entries get 0).  x, y: device, matrix dtype, must not overlap.
 * Errors: SPC5_EINVAL (NULL A, or NULL x/y while the matrix is non-empty),
 * SPC5_EDEVICE. */
int spc5_spmv(const spc5_matrix *A, const void *x, void *y, void *stream);

/* y = A x like spc5_spmv, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): this call never allocates or frees.  The partial row sums of
 * panels cut into pieces (spc5_info.split_panels > 0) go to a fixed device
 * array of the library, SPC5_NOALLOC_SCRATCH_BYTES bytes, of which each GPU
 * holds its own copy until the process ends.  Every call on one GPU shares
 * that GPU's array, whatever the handle: calls that overlap in time on one
 * GPU (several streams, or several host threads) race when their matrices
 * have pieces.  Each call writes the partial sums it reads, so nothing
 * carries over between calls.  Matrices without pieces use no scratch.
 * Errors: as spc5_spmv, plus SPC5_EUNSUPPORTED when the pieces need more
 * than SPC5_NOALLOC_SCRATCH_BYTES (npieces * r * value bytes) or the device
 * index is 64 or more. */
#define SPC5_NOALLOC_SCRATCH_BYTES (1 << 20)
int spc5_spmv_noalloc(const spc5_matrix *A, const void *x, void *y, void *stream);

/* Same product with the packed values taken from `values` (device,
 * nnz entries, the packed order of spc5_export) instead of the matrix's own:
 * y = A(theta) x, used by the differentiable path. */
int spc5_spmv_values(const spc5_matrix *A, const void *values, const void *x,
                     void *y, void *stream);

/* xbar[0..ncols) = A^T ybar[0..nrows), the transposed product (the backward
 * of y = A x; the paper defines only the forward product, Algorithm 1).
 * xbar is overwritten.  values: device packed values (A's packed order), or
 * NULL for the matrix's own.  Device pointers.
 * Without a plan: masked scatter from A's blocks (each set mask bit adds
 * value * ybar[row] to xbar[anchor+k] with a float atomic; xbar is zeroed on
 * the stream first); the accumulation order varies between runs.  When some
 * column holds thousands of entries (sampled at conversion) the
 * contributions are first summed per workgroup in LDS, so a popular column
 * takes one atomic per workgroup rather than one per row.
 * With a plan (spc5_prepare_transpose) there are no atomics and the result
 * is reproducible bit for bit.  The matrix's own values: the forward kernel
 * over the stored A^T.  Caller values: each product value * ybar[row] is
 * formed in A's packed order and the products are summed in A^T's CSR order,
 * in two passes through the calling stream's scratch (nnz values plus two
 * per 8192 nonzeros): each chunk of A stores its products contiguously,
 * grouped by position in A^T; then each group gathers its runs from the
 * chunks, reads them in A^T's order and forms segmented row sums (rows cut
 * by a group edge are completed by a small fixup in group order). */
int spc5_spmv_transpose(const spc5_matrix *A, const void *ybar, void *xbar,
                        void *stream);
int spc5_spmv_transpose_values(const spc5_matrix *A, const void *values,
                               const void *ybar, void *xbar, void *stream);

/* Build the transposed-product plan of A: A^T converted on the device to
 * SPC5 beta(r,c) storage (r = c = 0: A's own shape), for transposes with the
 * matrix's own values, plus the tables of transposes with caller values:
 * A's row of every packed value, the index arrays that move products from
 * A's packed order to A^T's CSR order, and A^T's row pointer.  Costs about
 * the device memory of A once more, plus 12 bytes per nonzero and 4 per
 * column; held until spc5_free.  Each stream that calls a transpose with
 * caller values adds one value array of scratch.  Synchronous.
 * Calling it again with the same shape is a no-op.
 * Errors: SPC5_EINVAL (NULL A, a plan with another shape exists),
 * SPC5_EUNSUPPORTED (r or c out of range, A^T's block count >= 2^31),
 * SPC5_ENOMEM, SPC5_EDEVICE. */
int spc5_prepare_transpose(spc5_matrix *A, int r, int c);

/* Gradient of <ybar, A(theta) x> with respect to the packed values theta:
 * vbar[v] = ybar[row(v)] * x[col(v)], in packed order (nnz entries).
 * Device pointers. */
int spc5_values_grad(const spc5_matrix *A, const void *ybar, const void *x,
                     void *vbar, void *stream);

/* Y = A X for nrhs right-hand sides: X device [ncols][nrhs] row-major,
 * Y device [nrows][nrhs] row-major (overwritten).  1 <= nrhs <= 64. */
int spc5_spmm(const spc5_matrix *A, int nrhs, const void *X, void *Y, void *stream);

/* ---------------------------------------------------------------- batches */

/* Group matrices of one dtype so that Y_m = A_m X_m for every m runs as ONE
 * persistent launch: workgroups take (matrix, tile) work items from a device
 * queue until it is empty, so matrices of very different sizes share the GPU
 * evenly.  Shapes must come from the batched kernel's set: beta(1,4),
 * beta(1,8), beta(1,16), beta(2,4), beta(2,8), beta(4,4), beta(4,8),
 * beta(8,8) (else SPC5_EUNSUPPORTED).  The batch keeps pointers to the
 * handles, which must outlive it, and owns its own device tables.
 * Synchronous. */
int spc5_batch_create(int nmat, spc5_matrix *const *mats, spc5_batch **out);
void spc5_batch_free(spc5_batch *B);

/* Per-matrix schedule of the batches built afterwards (the paper notes that
 * the best kernel settings depend on the matrix, Section 2.2): the cap, in
 * panels, of one work item's tile.  Value-mode batches (every matrix
 * beta(1,c)) cut the matrix's batch schedule into tiles of at most this many
 * panels (besides the value and block caps); the work-queue kernel uses it as
 * the SpMM tile width (at most 64 panels there).  0 (the default) restores the built-in choice: as many
 * panels as a tile holds, or the matrix's sweep tile width.  1..256.  Takes
 * effect at spc5_batch_create.  Errors: SPC5_EINVAL (NULL A, cap out of
 * range). */
int spc5_set_batch_schedule(spc5_matrix *A, int panels_per_tile);

/* Bind the operands: X[m], Y[m] are host arrays of nmat device pointers,
 * laid out as in spc5_spmm, with the same nrhs (1..64) for every matrix.  The
 * pointer table and the work list are uploaded here (synchronous), so that
 * spc5_batch_run itself issues only kernels. */
int spc5_batch_set_operands(spc5_batch *B, int nrhs, const void *const *X,
                            void *const *Y);

/* Y_m = A_m X_m for all m with the bound operands: one queue-reset kernel
 * and one persistent launch on `stream`, no allocation and no host-device
 * copy, so the call can be recorded in a HIP graph and replayed. */
int spc5_batch_run(const spc5_batch *B, void *stream);

/* spc5_batch_set_operands followed by spc5_batch_run. */
int spc5_batch_spmm(spc5_batch *B, int nrhs, const void *const *X,
                    void *const *Y, void *stream);

/* Cost model input for choosing beta(r,c): for each candidate q, the number of
 * blocks of the CSR matrix in beta(r[q], c[q]) (counted on the device; the
 * matrix is not converted).  Arguments as in csr_to_spc5 (values are not
 * needed); nblocks: host int64[ncand].  Synchronous. */
int spc5_plan(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *colidx,
              int ncand, const int *r, const int *c, int64_t *nblocks);

/* ---------------------------------------------------------------- CSR */

/* Plain CSR matrix on the device, the comparison kernel (Section 2.3's CSR;
 * the paper's scalar CSR baseline).  Same argument rules as csr_to_spc5. */
int spc5_csr_create(int64_t nrows, int64_t ncols, const int64_t *rowptr,
                    const int32_t *colidx, const void *values, spc5_dtype dtype,
                    spc5_csr **out);
void spc5_csr_free(spc5_csr *A);
/* y = A x with the plain CSR storage; device pointers. */
int spc5_csr_spmv(const spc5_csr *A, const void *x, void *y, void *stream);
/* Algorithmic bytes of one CSR product (values + colidx + rowptr + x + y). */
int64_t spc5_csr_bytes(const spc5_csr *A);

/* ---------------------------------------------------------------- misc */

/* Message describing the last failure on the calling thread ("" if none). */
const char *spc5_last_error(void);

/* Library version string. */
const char *spc5_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPC5_H */
