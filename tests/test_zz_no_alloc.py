"""The allocation-free forward product (spc5_spmv_noalloc) against the
ordinary one (spc5_spmv), through the C ABI: piece-tile partial sums in the
library's fixed device array instead of per-stream scratch.  Two calls in a
row, the second on a smaller matrix, each equal to spc5_spmv bit for bit
(same kernels, same summation order) and to the FP64 oracle within the
relative L2 gate."""
import numpy as np
import pytest

import oracle
from helpers import say
from paper_2307_14774_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def hub_matrix(n, m, hubs, lo, hi, seed):
    """Short rows plus a few hub rows of lo..hi nonzeros (half a dense run,
    half scattered), so that staged tiles cut their panels into pieces."""
    rng = np.random.default_rng(seed)
    counts, cols_all = [], []
    for i in range(n):
        if i in hubs:
            k = int(rng.integers(lo, hi))
            cols = np.unique(np.concatenate([np.arange(50, 50 + k // 2),
                                             rng.choice(m, k // 2, replace=False)]))
        else:
            cols = np.unique(rng.choice(m, int(rng.integers(0, 12)), replace=False))
        counts.append(len(cols))
        cols_all.append(cols)
    colidx = np.concatenate(cols_all).astype(np.int32)
    vals = rng.uniform(-1, 1, colidx.shape[0])
    x = rng.uniform(-1, 1, m)
    return W._finish(n, m, np.array(counts), colidx, vals, x, "hubs")


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("rc", [(1, 8), (4, 4)], ids=lambda t: "b%d_%d" % t)
def test_noalloc_matches_spmv_two_calls(rc, dtype, dev):
    from paper_2307_14774_amd import spc5 as S
    tdt = torch.float64 if dtype == "float64" else torch.float32
    gate = 1e-14 if dtype == "float64" else 1e-6
    big = hub_matrix(3000, 40000, (0, 9, 700, 2998, 2999), 4000, 12000, seed=61)
    small = hub_matrix(500, 9000, (3, 200), 2000, 5000, seed=62)
    for A in (big, small):          # the second call has the smaller input
        say(f"noalloc beta{rc} {dtype} rows={A.nrows} nnz={A.nnz}")
        M = S.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, *rc, dtype)
        assert M.kernel == "staged" and M.info.split_panels > 0
        x = torch.from_numpy(A.x).to(dev, tdt)
        y_ref = M.spmv(x)
        y = torch.full((A.nrows,), float("nan"), dtype=tdt, device=dev)
        M.spmv_noalloc(x, y)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref)
        if dtype == "float64":
            ref = oracle.csr_spmv(A.rowptr, A.colidx, A.values, A.x)
        else:
            ref = oracle.csr_spmv(A.rowptr, A.colidx,
                                  A.values.astype(np.float32).astype(np.float64),
                                  A.x.astype(np.float32).astype(np.float64))
        assert oracle.rel_l2(y.double().cpu().numpy(), ref) <= gate
        M.free()


def test_noalloc_without_pieces_and_empty(dev):
    """A matrix without pieces (no scratch used) and an empty one."""
    from paper_2307_14774_amd import spc5 as S
    A = W.laplacian_2d(40, seed=63)
    M = S.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, 4, 4)
    assert M.info.split_panels == 0
    x = torch.from_numpy(A.x).to(dev)
    y = torch.empty(A.nrows, dtype=torch.float64, device=dev)
    M.spmv_noalloc(x, y)
    assert torch.equal(y, M.spmv(x))
    E = S.Spc5Matrix.from_csr(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0), 0,
                              1, 8)
    E.spmv_noalloc(torch.empty(0, dtype=torch.float64, device=dev),
                   torch.empty(0, dtype=torch.float64, device=dev))
    torch.cuda.synchronize()


def test_noalloc_rejects_scratch_above_limit(dev):
    """Partial sums above the fixed array's size are refused with an error
    (nothing is launched)."""
    from paper_2307_14774_amd import spc5 as S
    rng = np.random.default_rng(64)
    n, m, k = 1024, 1 << 20, 6000
    cols = np.sort(np.stack([rng.choice(m, k, replace=False) for _ in range(n)]), axis=1)
    rowptr = np.arange(n + 1, dtype=np.int64) * k
    vals = rng.uniform(-1, 1, n * k)
    M = S.Spc5Matrix.from_csr(rowptr, cols.reshape(-1).astype(np.int32), vals, m, 8, 8)
    lib = S.lib()
    say(f"noalloc limit: split panels {M.info.split_panels}")
    assert M.kernel == "staged" and M.info.split_panels > 0
    x = torch.zeros(m, dtype=torch.float64, device=dev)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    with pytest.raises(S.Spc5Error) as e:
        M.spmv_noalloc(x, y)
    assert e.value.status == -5 and "fixed" in str(e.value)
    # the ordinary entry point takes per-stream scratch and runs
    M.spmv(x, y)
    torch.cuda.synchronize()
    assert torch.count_nonzero(y).item() == 0
