/*
 * SPC5 oracle: plain, slow, obviously correct CPU reference for the SPC5
 * sparse matrix/vector product and its companions.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP library) never calls it, shares no code with it, and must fail loudly
 * rather than fall back to it.
 *
 * Everything is FP64.  Every sum is strictly sequential; only the
 * host-baseline form of O1 spreads whole rows over threads.  Build with
 * -ffp-contract=off so that no multiply-add is fused: each product is
 * rounded, then added.
 *
 * Paper: Regnault & Bramas, "SPC5: an efficient SpMV framework vectorized
 * using ARM SVE and x86 AVX-512" (arXiv 2307.14774).
 *
 * Storage conventions (the readings this oracle takes; the paper fixes the
 * first four, the rest are the stated readings where it is silent):
 *  - CSR input: rowptr[nrows+1] (int64), colidx[nnz] (int32, strictly
 *    increasing inside a row), values[nnz]  (Section 2.3, CSR paragraph).
 *  - SPC5 beta(r,c): rows grouped in panels of r consecutive rows
 *    (Section 2.4, multi-row extension).  block_rowptr[npanels+1] gives the
 *    block range of each panel, block_colidx[b] the anchor column of block b,
 *    block_masks[b*r+i] the c-bit mask of row i of block b, and the packed
 *    values hold only the nonzeros (Algorithm 1 indexing; Section 2.4).
 *  - Mask bit k (least significant bit = 0) marks column anchor+k
 *    (Fig. 3 caption: the lowest bit maps to the first vector element).
 *  - Packed value order: block after block; inside a block row 0..r-1; inside
 *    a row ascending k (the order in which the scalar loop of Algorithm 1
 *    consumes its running value index).
 *  - A block is anchored at the smallest column not yet covered among the
 *    panel's rows and spans [anchor, anchor+c) (Section 2.4: a block starts at
 *    a nonzero and takes the following nonzeros up to c-1 columns further).
 *  - npanels = ceil(nrows / r); rows past nrows in the last panel are empty.
 *  - y = A x overwrites y (empty rows give 0).
 *  Masks are always written as uint16 here (c <= 16).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* O1. Plain CSR SpMV, the definition y_i = sum_j A_ij x_j (Section 2.3, CSR;
 * the paper's scalar "CSR" baseline).  Each row sums from +0.0 in ascending
 * storage order. */
void oracle_csr_spmv(int64_t nrows, const int64_t *rowptr, const int32_t *colidx,
                     const double *values, const double *x, double *y)
{
    for (int64_t i = 0; i < nrows; ++i) {
        double s = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            double p = values[k] * x[colidx[k]];
            s = s + p;
        }
        y[i] = s;
    }
}

/* O1 on several CPU threads, for the host baseline only: the rows are cut
 * into nthreads contiguous ranges of equal row count, one per thread (the
 * paper's parallel runs split the rows "naively" among the threads, Section
 * 4.3).  Every row is still summed by one thread from +0.0 in ascending
 * storage order, so y is bitwise equal to O1. */
void oracle_csr_spmv_par(int64_t nrows, const int64_t *rowptr, const int32_t *colidx,
                         const double *values, const double *x, double *y, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        int t = 0, nt = 1;
#ifdef _OPENMP
        t = omp_get_thread_num();
        nt = omp_get_num_threads();
#endif
        int64_t lo = nrows * t / nt, hi = nrows * (t + 1) / nt;
        for (int64_t i = lo; i < hi; ++i) {
            double s = 0.0;
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                double q = values[k] * x[colidx[k]];
                s = s + q;
            }
            y[i] = s;
        }
    }
}

/* O1 with k right-hand sides: Y = A X, X is ncols x nrhs row-major, Y is
 * nrows x nrhs row-major.  Column t of Y is exactly O1 applied to column t of
 * X (same summation order). */
void oracle_csr_spmm(int64_t nrows, const int64_t *rowptr, const int32_t *colidx,
                     const double *values, int64_t nrhs, const double *X, double *Y)
{
    for (int64_t i = 0; i < nrows; ++i) {
        for (int64_t t = 0; t < nrhs; ++t) {
            double s = 0.0;
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                double p = values[k] * X[(int64_t)colidx[k] * nrhs + t];
                s = s + p;
            }
            Y[i * nrhs + t] = s;
        }
    }
}

/* O2. Transposed product xbar = A^T ybar, the definition
 * xbar_j = sum_i A_ij ybar_i, accumulated in row-major storage order. */
void oracle_csr_spmv_t(int64_t nrows, int64_t ncols, const int64_t *rowptr,
                       const int32_t *colidx, const double *values,
                       const double *ybar, double *xbar)
{
    for (int64_t j = 0; j < ncols; ++j) xbar[j] = 0.0;
    for (int64_t i = 0; i < nrows; ++i) {
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            double p = values[k] * ybar[i];
            xbar[colidx[k]] = xbar[colidx[k]] + p;
        }
    }
}

/* Greedy blocking of one panel (Section 2.4).  Rows [row0, row0+nr) with
 * nr <= 8.  When blk_col is NULL only the number of blocks is returned;
 * otherwise the anchors, masks (index blk*r + i) and packed values are
 * written starting at block index first_blk and value index first_val. */
static int64_t oracle_block_panel(int64_t row0, int nr, int r, int c,
                                  const int64_t *rowptr, const int32_t *colidx,
                                  const double *values, int64_t first_blk,
                                  int64_t first_val, int32_t *blk_col,
                                  uint16_t *masks, double *packed)
{
    int64_t cur[8], end[8];
    for (int i = 0; i < nr; ++i) {
        cur[i] = rowptr[row0 + i];
        end[i] = rowptr[row0 + i + 1];
    }
    int64_t nblk = 0, v = first_val;
    for (;;) {
        /* anchor: smallest column not yet covered among the panel's rows */
        int64_t anchor = -1;
        for (int i = 0; i < nr; ++i)
            if (cur[i] < end[i] && (anchor < 0 || colidx[cur[i]] < anchor))
                anchor = colidx[cur[i]];
        if (anchor < 0) break;
        if (blk_col) blk_col[first_blk + nblk] = (int32_t)anchor;
        for (int i = 0; i < r; ++i) {
            uint32_t m = 0;
            if (i < nr) {
                while (cur[i] < end[i] && (int64_t)colidx[cur[i]] < anchor + c) {
                    m |= 1u << (colidx[cur[i]] - anchor);
                    if (packed) packed[v] = values[cur[i]];
                    ++v;
                    ++cur[i];
                }
            }
            if (masks) masks[(first_blk + nblk) * r + i] = (uint16_t)m;
        }
        ++nblk;
    }
    return nblk;
}

/* O3a. Number of beta(r,c) blocks per panel (blk_count may be NULL); returns
 * the total. */
int64_t oracle_spc5_count(int64_t nrows, const int64_t *rowptr, const int32_t *colidx,
                          int r, int c, int64_t *blk_count)
{
    int64_t npanels = (nrows + r - 1) / r, total = 0;
    for (int64_t p = 0; p < npanels; ++p) {
        int64_t row0 = p * r;
        int nr = (int)((nrows - row0) < r ? (nrows - row0) : r);
        int64_t n = oracle_block_panel(row0, nr, r, c, rowptr, colidx, NULL, 0, 0,
                                       NULL, NULL, NULL);
        if (blk_count) blk_count[p] = n;
        total += n;
    }
    return total;
}

/* O3b. CSR -> SPC5 beta(r,c).  blk_ptr[npanels+1], blk_col[nblocks],
 * masks[nblocks*r], packed[nnz] must be sized by the caller (use O3a). */
void oracle_csr_to_spc5(int64_t nrows, const int64_t *rowptr, const int32_t *colidx,
                        const double *values, int r, int c, int64_t *blk_ptr,
                        int32_t *blk_col, uint16_t *masks, double *packed)
{
    int64_t npanels = (nrows + r - 1) / r, nb = 0;
    blk_ptr[0] = 0;
    for (int64_t p = 0; p < npanels; ++p) {
        int64_t row0 = p * r;
        int nr = (int)((nrows - row0) < r ? (nrows - row0) : r);
        nb += oracle_block_panel(row0, nr, r, c, rowptr, colidx, values, nb,
                                 rowptr[row0], blk_col, masks, packed);
        blk_ptr[p + 1] = nb;
    }
}

/* O4. SPC5 -> CSR (Fig. 2 caption: a column index is the block anchor plus
 * the bit position).  Row counts are gathered first, then entries placed.
 * rowptr[nrows+1], colidx[nnz], values[nnz] are outputs. */
void oracle_spc5_to_csr(int64_t nrows, int r, int c, const int64_t *blk_ptr,
                        const int32_t *blk_col, const uint16_t *masks,
                        const double *packed, int64_t *rowptr, int32_t *colidx,
                        double *values)
{
    int64_t npanels = (nrows + r - 1) / r;
    for (int64_t i = 0; i <= nrows; ++i) rowptr[i] = 0;
    for (int64_t p = 0; p < npanels; ++p)
        for (int64_t b = blk_ptr[p]; b < blk_ptr[p + 1]; ++b)
            for (int i = 0; i < r; ++i) {
                int64_t row = p * r + i;
                uint32_t m = masks[b * r + i];
                for (int k = 0; k < c; ++k)
                    if ((m >> k) & 1u) rowptr[row + 1] += 1;
            }
    for (int64_t i = 0; i < nrows; ++i) rowptr[i + 1] += rowptr[i];
    int64_t *fill = (int64_t *)malloc((size_t)(nrows > 0 ? nrows : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < nrows; ++i) fill[i] = rowptr[i];
    int64_t v = 0;
    for (int64_t p = 0; p < npanels; ++p)
        for (int64_t b = blk_ptr[p]; b < blk_ptr[p + 1]; ++b)
            for (int i = 0; i < r; ++i) {
                int64_t row = p * r + i;
                uint32_t m = masks[b * r + i];
                for (int k = 0; k < c; ++k)
                    if ((m >> k) & 1u) {
                        colidx[fill[row]] = blk_col[b] + k;
                        values[fill[row]] = packed[v++];
                        fill[row] += 1;
                    }
            }
    free(fill);
}

/* O5. The SPC5 product read straight from the format's definition
 * (Section 2.4, Fig. 2 caption): the beta(r,c) arrays describe the matrix
 * whose row p*r+i holds, for every block b of panel p and every set bit k of
 * the mask of row i, the entry (anchor(b)+k, next packed value).  So the
 * product is O4 (decode to CSR) followed by O1 (the CSR definition).  Each
 * row is still summed from +0.0 in ascending column order, which makes the
 * result bitwise equal to O1 on the original CSR.  y is overwritten. */
void oracle_spc5_spmv(int64_t nrows, int r, int c, const int64_t *blk_ptr,
                      const int32_t *blk_col, const uint16_t *masks,
                      const double *packed, const double *x, double *y)
{
    int64_t npanels = (nrows + r - 1) / r, nnz = 0;
    for (int64_t q = 0; q < blk_ptr[npanels] * r; ++q)
        for (int k = 0; k < c; ++k)
            if ((masks[q] >> k) & 1u) nnz += 1;
    int64_t *rowptr = (int64_t *)malloc((size_t)(nrows + 1) * sizeof(int64_t));
    int32_t *colidx = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    double *values = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    oracle_spc5_to_csr(nrows, r, c, blk_ptr, blk_col, masks, packed, rowptr, colidx, values);
    oracle_csr_spmv(nrows, rowptr, colidx, values, x, y);
    free(values);
    free(colidx);
    free(rowptr);
}

/* O6. Gradient of L = <ybar, A(theta) x> with respect to the packed values:
 * vbar[v] = ybar[row(v)] * x[col(v)], written in packed order. */
void oracle_spc5_values_grad(int64_t nrows, int r, int c, const int64_t *blk_ptr,
                             const int32_t *blk_col, const uint16_t *masks,
                             const double *ybar, const double *x, double *vbar)
{
    int64_t npanels = (nrows + r - 1) / r, v = 0;
    for (int64_t p = 0; p < npanels; ++p)
        for (int64_t b = blk_ptr[p]; b < blk_ptr[p + 1]; ++b)
            for (int i = 0; i < r; ++i) {
                uint32_t m = masks[b * r + i];
                for (int k = 0; k < c; ++k)
                    if ((m >> k) & 1u) {
                        vbar[v] = ybar[p * r + i] * x[blk_col[b] + k];
                        v += 1;
                    }
            }
}
