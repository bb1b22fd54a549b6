// Internal declarations shared by the HIP translation units of libspc5.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "spc5.h"

namespace spc5 {
struct ScratchPool;
}

struct spc5_matrix {
    int64_t nrows = 0, ncols = 0, nnz = 0, nblocks = 0, npanels = 0;
    int r = 1, c = 1;
    spc5_dtype dtype = SPC5_F64;
    int mask_bytes = 1;
    int ppt = 1;           // panels per wavefront tile (sweep kernel)
    int sppt = 1;          // panels per wavefront tile (staged kernel)
    int batch_ppt = 0;     // tile cap in panels for batches (spc5_set_batch_schedule; 0: default)
    bool hot_cols = false; // some column holds thousands of entries (sampled at conversion)
    int kernel = SPC5_KERNEL_ROWS;   // forward kernel in use (never AUTO)
    int64_t max_panel_blocks = 0;
    int device = 0;
    int32_t *blk_ptr = nullptr;    // [npanels+1]
    int32_t *blk_col = nullptr;    // [nblocks]
    void *masks = nullptr;         // [nblocks*r], uint8 or uint16
    void *val = nullptr;           // [nnz]
    int32_t *panel_val = nullptr;  // [npanels+1], value offset of each panel
    // staged-kernel tile schedule: first panel / block / value of each tile
    int32_t *tile_p = nullptr, *tile_b = nullptr, *tile_v = nullptr;   // [ntiles_staged+1]
    int32_t *tile_f = nullptr;     // [ntiles_staged+1], piece slot + 1 of a piece tile, else 0
    int64_t ntiles_staged = 0;
    int max_tile_values = 0;       // largest tile, in values
    int tile_bt = 0;               // block cap the schedule was built with
    bool staged_ok = false;        // the staged schedule exists
    int variant = 0;               // staged-kernel ablation variant (spc5_set_variant)
    // panels longer than a tile: panel, first and last piece tile
    int32_t *split_p = nullptr, *split_t0 = nullptr, *split_t1 = nullptr;   // [nsplit]
    int64_t nsplit = 0;
    int64_t npieces = 0;           // piece tiles (their partial row sums: npieces*r values)
    // transposed-product plan (spc5_prepare_transpose): A^T in beta(r,c) and
    // the tables of the two LDS passes that move caller values from A's
    // packed order to A^T's (see transpose_plan.hip)
    spc5_matrix *tr = nullptr;
    uint16_t *tr_lidx = nullptr;   // [nnz] pass 1: chunk-local value to write
    uint16_t *tr_src = nullptr;    // [nnz] pass 2: bucket-local slot read
    // runs (the values of one chunk of A inside one bucket of A^T, in slot
    // order): window slot where each starts, its position in pass 1's output
    // minus that slot, each bucket's first run
    uint16_t *tr_rslot = nullptr;  // [nruns]
    int32_t *tr_rbase = nullptr;  // [nruns]
    int32_t *tr_rstart = nullptr;  // [nbuckets+1]
    int64_t tr_nruns = 0;
    void *tr_arow = nullptr;       // [nnz] A's row of every packed value (pass 1): uint16
                                   // offsets from tr_cbase[chunk], or int32 when it is NULL
    int32_t *tr_cbase = nullptr;   // [nbuckets] base row of every chunk of A
    int32_t *tr_hoff = nullptr;    // [nbuckets+1] first nonempty A^T row of each bucket
    uint32_t *tr_hbits = nullptr;  // [nbuckets*W/32+1] bit q: position q starts a row of A^T
    int32_t *tr_hrow = nullptr;    // [nheads] row index of each nonempty A^T row
    int32_t *tr_rlo = nullptr;     // [nbuckets+1] first row owned by each bucket
    int64_t tr_nheads = 0;
    int32_t *tr_edge_rows = nullptr;   // [3*nedge] (row, first bucket, last bucket)
    int64_t tr_nedge = 0, tr_nbuckets = 0;
    // per-stream scratch of the products (see Scratch)
    spc5::ScratchPool *pool = nullptr;
};

struct spc5_csr {
    int64_t nrows = 0, ncols = 0, nnz = 0;
    spc5_dtype dtype = SPC5_F64;
    int rpt = 1;                   // rows per wavefront tile (segmented kernel)
    int group = 0;                 // lanes per row of the CSR-vector kernel (0: segmented)
    int device = 0;
    int32_t *rowptr = nullptr;     // [nrows+1]
    int32_t *colidx = nullptr;     // [nnz]
    void *val = nullptr;           // [nnz]
};

namespace spc5 {

// Trailing padding (bytes) of every device array of a matrix.
constexpr size_t kPad = 64;

// Record a failure for spc5_last_error() and return `status`.
int fail(int status, const char *fmt, ...);
// Map a HIP error to SPC5_EDEVICE / SPC5_ENOMEM with a message.
int hip_fail(hipError_t e, const char *what);

// Default wavefront tile width (in panels) for a mean number of block rows
// per panel.
int default_ppt(double blockrows_per_panel);
// Host-side CSR checks (rowptr monotone from 0, columns sorted, unique and in
// range, nnz < 2^31); *nnz_out receives rowptr[nrows].
int validate_csr(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *colidx,
                 const void *values, int64_t *nnz_out);
// Forward kernel picked from the panel statistics of A.
int auto_kernel(const spc5_matrix *A);

// Scratch memory of one product call: the partial row sums of the piece
// tiles of A (npieces*r values) and of A^T's plan, and for a transpose with
// caller values the staging of the products (nnz values) and the
// bucket-edge partial sums (2 per bucket).  A call
// writes all of it before reading it, so nothing needs clearing.  The normal
// entry points take it from a pool of the handle with one set per stream
// (calls on one stream are ordered, calls on different streams do not
// share); the allocation-free entry point takes a fixed device array.
struct Scratch {
    void *partial = nullptr;
    void *tr_partial = nullptr;
    void *stage = nullptr;
    void *edges = nullptr;
};
constexpr int kNeedPartial = 1, kNeedTrPartial = 2, kNeedTheta = 4;
// Scratch of A for stream s with the parts `need` asks for, allocated on the
// stream's first call that needs them.
int pool_scratch(const spc5_matrix *A, hipStream_t s, int need, Scratch *out);
void free_pool(spc5_matrix *A);

// Forward product; `val` overrides the matrix's packed values when non-null;
// `partial` receives the piece tiles' row sums (A->npieces*r values, unused
// when A has no piece tiles).
hipError_t launch_spmv(const spc5_matrix *A, const void *val, const void *x, void *y,
                       hipStream_t s, void *partial);
hipError_t launch_spmv_staged(const spc5_matrix *A, const void *val, const void *x, void *y,
                              hipStream_t s, int remap, void *partial);
// (Re)build the staged kernel's tile schedule with at most ppw panels per tile
// (0: as many as one workgroup has rows for), for a launch of the matrix
// alone (small matrices: narrower tiles) or for the persistent batch kernel
// (alone = false: full-size tiles).
int build_staged_schedule(spc5_matrix *A, int ppw, bool alone = true);
void free_staged_schedule(spc5_matrix *A);
// Staged schedule for the ablation variants (which run the 16 KiB value
// buffer and its block cap) when `variant`, else back to the default one.
int fit_schedule_to_variants(spc5_matrix *A, bool variant);
hipError_t excl_scan_i64(const int64_t *in, int64_t n, int64_t *out, hipStream_t s,
                         int64_t **scratch);
int remap_enabled();
hipError_t launch_csr_spmv(const spc5_csr *A, const void *x, void *y, hipStream_t s);
hipError_t launch_spmm(const spc5_matrix *A, int nrhs, const void *X, void *Y,
                       hipStream_t s);
hipError_t launch_transpose(const spc5_matrix *A, const void *val, const void *ybar,
                            void *xbar, hipStream_t s);
hipError_t launch_values_grad(const spc5_matrix *A, const void *ybar, const void *x,
                              void *vbar, hipStream_t s);

// CSR -> SPC5 conversion on the device (d_* are device CSR arrays).  When
// d_payload is given, d_payload_out[nnz] receives it in packed order (the
// same placement as the values).
int convert_on_device(spc5_matrix *A, const int64_t *d_rowptr, const int32_t *d_colidx,
                      const void *d_values, const int32_t *d_payload = nullptr,
                      int32_t *d_payload_out = nullptr);
// Release every device array of A (and of its transposed plan) and A itself.
void free_matrix(spc5_matrix *A);
// Default schedule and kernel choice of a freshly converted matrix.
int finish_matrix(spc5_matrix *A);
// Transposed-product plan of A (see spc5_prepare_transpose).
int build_transpose_plan(spc5_matrix *A, int r, int c);
// x_out = A^T y_in through the plan; vals overrides A's values (packed order).
// Caller values: sc.stage and sc.edges; the matrix's own: sc.tr_partial.
hipError_t launch_transpose_plan(const spc5_matrix *A, const void *vals, const void *ybar,
                                 void *xbar, hipStream_t s, const Scratch &sc);

// Fill `n` elements of a device array with zero using a kernel (safe to
// record in a graph).
hipError_t zero_fill(void *p, int64_t n, int elem_bytes, hipStream_t s);

}  // namespace spc5
