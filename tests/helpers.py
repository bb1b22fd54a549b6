"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare with the CPU oracle on the same seeded inputs."""
import sys

import numpy as np

import oracle


def say(msg: str):
    """Name the case before a GPU step (flushed, so it survives a crash)."""
    print(msg, flush=True)
    sys.stdout.flush()


def row_error_bound_ok(y, A, x, dtype_eps: float, slack: float = 1.0):
    """Per-row forward error bound |y_i - exact_i| <= gamma_n sum_j |a_ij x_j|
    (holds for any summation order, with or without fused multiply-add),
    with exact_i taken from the FP64 oracle (whose own error is smaller)."""
    yref = oracle.csr_spmv(A.rowptr, A.colidx, A.values, x)
    absum = oracle.csr_spmv(A.rowptr, A.colidx, np.abs(A.values), np.abs(x))
    n = np.diff(A.rowptr).astype(np.float64)
    gamma = (n + 1) * dtype_eps / (1 - (n + 1) * dtype_eps)
    # the oracle's own error uses the FP64 unit roundoff
    g64 = n * 2.0 ** -53 / (1 - n * 2.0 ** -53)
    bound = slack * (gamma + g64) * absum
    err = np.abs(np.asarray(y, dtype=np.float64) - yref)
    bad = np.nonzero(err > bound)[0]
    return bad


def masks_u16(masks: np.ndarray) -> np.ndarray:
    return masks.astype(np.uint16)


def fem_block_count(n: int, r: int, c: int) -> int:
    """Closed-form beta(r,c) block count of the 3D 27-point, 3-dof FEM matrix
    on n^3 nodes (rows 3m+d, node m = (z*n+y)*n+x), for r dividing 3n so that
    no panel straddles two x-lines.  A row couples to the x-runs of up to 9
    (dz,dy) node lines; the (3n-2)^2 (line, band) pairs are alike.  Along one
    band, the panel of rows [pr, pr+r) covers nodes xmin..xmax (x = row // 3),
    so its rows' runs join into the contiguous columns of nodes
    max(xmin-1,0)..min(xmax+1,n-1), 3 per node, which the greedy anchor
    covers with ceil(len / c) windows.  Bands sit 3n columns apart, so for
    n >= 6 no window reaches the next band."""
    assert (3 * n) % r == 0 and n >= 6
    per_line = 0
    for p in range(3 * n // r):
        xmin, xmax = (p * r) // 3, (p * r + r - 1) // 3
        ln = 3 * (min(xmax + 1, n - 1) - max(xmin - 1, 0) + 1)
        per_line += -(-ln // c)
    return (3 * n - 2) ** 2 * per_line
