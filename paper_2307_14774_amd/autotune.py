"""Per-matrix choice of the beta(r,c) shape and of the panels-per-wavefront
schedule.

Shape: the product is bound by memory traffic, and the paper observes that
the SPC5 kernels' performance follows the block filling (Section 4.3), so the
model ranks the candidate shapes by the algorithmic bytes of one product,
    bytes(r,c) = vb*nnz + 4*nblocks + r*ceil(c/8)*nblocks + 4*(npanels+1)
                 + vb*(ncols + nrows)*k,
with nblocks counted on the device for every candidate (spc5_plan).
Schedule: measured -- for a single matrix's SpMM, the tile width (panels per
wavefront) is timed around the model's default and the fastest kept; for a
batch, each matrix's batch tile cap (spc5_set_batch_schedule) is timed on a
batch of that matrix alone with the batch's number of right-hand sides, and
the fastest candidate kept.
"""
from __future__ import annotations

import numpy as np

from . import spc5

# the shapes the batched persistent kernel is compiled for
CANDIDATES = [(1, 8), (2, 4), (4, 4), (2, 8), (4, 8), (8, 8), (1, 16), (1, 4)]


def model_bytes(nnz: int, nrows: int, ncols: int, r: int, c: int, nblocks: int, vb: int,
                nrhs: int = 1) -> int:
    npanels = (nrows + r - 1) // r
    mask_bytes = 1 if c <= 8 else 2
    return (vb * nnz + 4 * nblocks + r * mask_bytes * nblocks + 4 * (npanels + 1)
            + vb * (ncols + nrows) * nrhs)


def choose_shape(A, dtype: str = "float64", candidates=CANDIDATES, nrhs: int = 1):
    """A: workloads.Csr.  Returns ((r, c), {shape: model bytes})."""
    vb = 8 if dtype == "float64" else 4
    counts = spc5.plan(A.rowptr, A.colidx, A.ncols, candidates)
    table = {rc: model_bytes(A.nnz, A.nrows, A.ncols, rc[0], rc[1], nb, vb, nrhs)
             for rc, nb in zip(candidates, counts)}
    best = min(table, key=lambda rc: (table[rc], -rc[0]))
    return best, table


def tune_schedule(M: "spc5.Spc5Matrix", nrhs: int, repeats: int = 5) -> int:
    """Time the SpMM tile width around the default and keep the fastest;
    returns the chosen panels per tile."""
    import torch
    inf = M.info
    dev = torch.device("cuda")
    X = torch.zeros((inf.ncols, nrhs), dtype=M.torch_dtype, device=dev)
    Y = torch.empty((inf.nrows, nrhs), dtype=M.torch_dtype, device=dev)
    kernel = M.kernel
    staged_ppt = inf.panels_per_tile if kernel == "staged" else 0
    M.set_schedule("sweep")
    base = max(1, M.info.panels_per_tile)
    best, best_t = base, None
    for ppt in sorted({max(1, base // 2), base, min(64, base * 2)}):
        M.set_schedule("sweep", ppt)
        M.spmm(X, Y)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(repeats):
            M.spmm(X, Y)
        b.record()
        torch.cuda.synchronize()
        t = a.elapsed_time(b)
        if best_t is None or t < best_t:
            best, best_t = ppt, t
    # the sweep tile width is what SpMM and batches use; the staged forward
    # kernel keeps its own schedule
    M.set_schedule("sweep", best)
    if kernel != "sweep":
        M.set_schedule(kernel, staged_ppt if kernel == "staged" else best)
    return best


BATCH_PPT = (0, 128, 64, 32)    # 0: as many panels as a tile holds


def tune_batch_schedule(M: "spc5.Spc5Matrix", nrhs: int, candidates=BATCH_PPT,
                        repeats: int = 5) -> int:
    """Time a batch of M alone, with nrhs right-hand sides, for every
    candidate tile cap; keep the fastest on M (spc5_set_batch_schedule) and
    return it."""
    import torch
    inf = M.info
    dev = torch.device("cuda")
    X = torch.zeros((inf.ncols, nrhs), dtype=M.torch_dtype, device=dev)
    Y = torch.empty((inf.nrows, nrhs), dtype=M.torch_dtype, device=dev)
    best, best_t = 0, None
    for ppt in candidates:
        M.set_batch_schedule(ppt)
        B = spc5.Spc5Batch([M])
        B.set_operands([X], [Y])
        B.run()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(repeats):
            B.run()
        b.record()
        torch.cuda.synchronize()
        t = a.elapsed_time(b)
        B.free()
        if best_t is None or t < best_t:
            best, best_t = ppt, t
    M.set_batch_schedule(best)
    return best


def tune_batch(mats, nrhs: int, candidates=BATCH_PPT) -> list:
    """tune_batch_schedule for every matrix of a batch (before
    spc5_batch_create); returns the chosen caps."""
    return [tune_batch_schedule(M, nrhs, candidates) for M in mats]


def autotune(A, dtype: str = "float64", nrhs: int = 1, measure: bool = False):
    """Convert A with the model's best shape; optionally tune the schedule.
    Returns (Spc5Matrix, info dict)."""
    (r, c), table = choose_shape(A, dtype, nrhs=nrhs)
    M = spc5.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, r, c, dtype)
    ppt = M.info.panels_per_tile
    if measure:
        ppt = tune_schedule(M, nrhs)
    return M, {"shape": (r, c), "model_bytes": table, "panels_per_tile": ppt}
