"""GPU parity at full benchmark sizes, in the launch configuration bench.py
times (default schedule): the whole y is compared with the CPU oracle, which
runs the plain CSR definition in FP64 in well under a few seconds."""
import numpy as np
import pytest

import oracle
from helpers import row_error_bound_ok, say
from paper_2307_14774_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


_cache = {}


def workload(name):
    if name not in _cache:
        _cache.clear()
        _cache[name] = {"random10k": lambda: W.random_uniform(10_000, 10, seed=0),
                        "laplacian2048": lambda: W.laplacian_2d(2048, seed=0),
                        "fem96": lambda: W.fem_3d(96, seed=0)}[name]()
    return _cache[name]


def check(A, r, c, dev, dtype="float64"):
    from paper_2307_14774_amd import spc5 as S
    tdt = torch.float64 if dtype == "float64" else torch.float32
    M = S.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, r, c, dtype)
    x = torch.from_numpy(A.x).to(dev, tdt)
    y = M.spmv(x)
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    yref = oracle.csr_spmv(A.rowptr, A.colidx, A.values, A.x)
    err = oracle.rel_l2(y, yref)
    M.free()
    return y, yref, err


@pytest.mark.parametrize("name", ["random10k", "laplacian2048"])
@pytest.mark.parametrize("rc", [(1, 8), (2, 4), (4, 4)], ids=lambda t: "b%d_%d" % t)
def test_full_size_f64(name, rc, dev):
    A = workload(name)
    say(f"full {name} beta{rc} f64")
    y, yref, err = check(A, *rc, dev)
    assert err <= 1e-14, err
    assert row_error_bound_ok(y, A, A.x, 2.0 ** -53).size == 0


def test_full_size_laplacian_conversion(dev):
    from paper_2307_14774_amd import spc5 as S
    A = workload("laplacian2048")
    for r, c in [(1, 8), (2, 4), (4, 4)]:
        say(f"full laplacian conversion beta({r},{c})")
        M = S.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, r, c)
        bp, bc, mk, va = M.export()
        O = oracle.csr_to_spc5(A.rowptr, A.colidx, A.values, A.ncols, r, c)
        assert np.array_equal(bp, O.blk_ptr) and np.array_equal(bc, O.blk_col)
        assert np.array_equal(mk.astype(np.uint16), O.masks)
        assert np.array_equal(va, O.values)
        N = 2048
        assert M.info.nblocks == {(1, 8): 3 * N * N - 2 * N, (2, 4): 3 * N * N // 2 - N,
                                  (4, 4): N * N - N // 2}[(r, c)]
        M.free()


def test_full_size_laplacian_f32(dev):
    A = workload("laplacian2048")
    say("full laplacian beta(4,4) f32")
    _, _, err = check(A, 4, 4, dev, "float32")
    assert err <= 1e-6, err


def test_full_size_laplacian_csr(dev):
    from paper_2307_14774_amd import spc5 as S
    A = workload("laplacian2048")
    say("full laplacian csr f64")
    M = S.CsrMatrix(A.rowptr, A.colidx, A.values, A.ncols)
    y = M.spmv(torch.from_numpy(A.x).to(dev)).cpu().numpy()
    assert oracle.rel_l2(y, oracle.csr_spmv(A.rowptr, A.colidx, A.values, A.x)) <= 1e-14


@pytest.mark.slow
@pytest.mark.parametrize("rc,dtype,tol", [((4, 4), "float64", 1e-14), ((1, 8), "float64", 1e-14),
                                          ((4, 4), "float32", 1e-6)],
                         ids=["b4_4-f64", "b1_8-f64", "b4_4-f32"])
def test_full_size_fem(rc, dtype, tol, dev):
    A = workload("fem96")
    say(f"full fem96 beta{rc} {dtype}")
    _, _, err = check(A, *rc, dev, dtype)
    assert err <= tol, err


def test_full_size_fem_conversion(dev):
    """FEM 96^3 x 3 (210.5 M nonzeros) converted on the device: bit-exact
    against the oracle's greedy conversion and equal to the closed-form
    block counts (beta(1,8) 46,623,720; beta(2,4) 35,172,280; beta(4,4)
    17,667,936)."""
    from helpers import fem_block_count
    from paper_2307_14774_amd import spc5 as S
    A = workload("fem96")
    closed = {(1, 8): 46_623_720, (2, 4): 35_172_280, (4, 4): 17_667_936}
    for (r, c), nb in closed.items():
        say(f"full fem96 conversion beta({r},{c})")
        assert fem_block_count(96, r, c) == nb
        M = S.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, r, c)
        assert M.info.nblocks == nb
        bp, bc, mk, va = M.export()
        M.free()
        O = oracle.csr_to_spc5(A.rowptr, A.colidx, A.values, A.ncols, r, c)
        assert O.nblocks == nb
        assert np.array_equal(bp, O.blk_ptr) and np.array_equal(bc, O.blk_col)
        assert np.array_equal(mk.astype(np.uint16), O.masks)
        assert np.array_equal(va.view(np.uint64), O.values.view(np.uint64))
        del bp, bc, mk, va, O


_batch_cache = {}


def batch_workload():
    """The 256 uneven matrices of the batched workload (rows log-uniform in
    1k..200k, Zipf(1.5) row lengths capped at 512, 30% of nonzeros in runs)."""
    if "mats" not in _batch_cache:
        _batch_cache["mats"] = W.batch_of_runs(256, seed=0)
    return _batch_cache["mats"]


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_full_size_batch_256(dtype, dev):
    """The batched workload at its stated size in the configuration the
    benchmark times: all 256 matrices, shapes from the autotuner, one
    persistent launch per k in {1, 4, 16}; every matrix's Y against the FP64
    oracle (CSR SpMM), relative L2 <= 1e-14 (FP64) / 1e-6 (FP32, against the
    oracle on the FP32-rounded data)."""
    from concurrent.futures import ThreadPoolExecutor

    from paper_2307_14774_amd import autotune
    from paper_2307_14774_amd import spc5 as S
    mats = batch_workload()
    tdt = torch.float64 if dtype == "float64" else torch.float32
    say(f"full batch 256 {dtype}: converting")
    Ms = []
    for A in mats:
        (r, c), _ = autotune.choose_shape(A, dtype)
        Ms.append(S.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, r, c, dtype))
    B = S.Spc5Batch(Ms)
    if dtype == "float64":
        vals = [A.values for A in mats]
    else:
        vals = [A.values.astype(np.float32).astype(np.float64) for A in mats]
    for k in (1, 4, 16):
        say(f"full batch 256 {dtype} k={k}")
        rng = np.random.default_rng(1000 + k)
        Xh = [rng.uniform(-1, 1, (A.ncols, k)) for A in mats]
        if dtype == "float32":
            Xh = [X.astype(np.float32).astype(np.float64) for X in Xh]
        Ys = B.spmm([torch.tensor(X, dtype=tdt, device=dev) for X in Xh])
        torch.cuda.synchronize()
        Yh = [Y.cpu().double().numpy() for Y in Ys]
        del Ys

        def err(m):
            A = mats[m]
            return oracle.rel_l2(Yh[m], oracle.csr_spmm(A.rowptr, A.colidx, vals[m], Xh[m]))
        with ThreadPoolExecutor(8) as ex:
            errs = list(ex.map(err, range(len(mats))))
        worst = int(np.argmax(errs))
        say(f"  worst rel L2 {errs[worst]:.3e} (matrix {worst})")
        assert errs[worst] <= (1e-14 if dtype == "float64" else 1e-6), (worst, errs[worst])
    B.free()
    for M in Ms:
        M.free()


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_full_size_graph_theta_transpose(dtype, dev):
    """The caller-values transpose on the 2^20-row Zipf graph at full size
    (16.8 M nonzeros: 1024 chunks of A, about a thousand runs per bucket of
    A^T, the popular columns' rows of A^T across many buckets), with small
    integer theta and ybar: every partial sum stays below 2^24, so FP32 is
    exact too; compared bit for bit with the oracle, twice in a row into an
    x_bar first filled with NaN."""
    from paper_2307_14774_amd import spc5 as S
    say(f"full Zipf graph theta transpose {dtype}")
    G = W.zipf_graph(1 << 20, seed=0)
    tdt = torch.float64 if dtype == "float64" else torch.float32
    M = S.Spc5Matrix.from_csr(G.rowptr, G.colidx, G.values, G.ncols, 1, 8, dtype)
    M.prepare_transpose(1, 8)
    rng = np.random.default_rng(81)
    for rep in range(2):
        # beta(1,8): the packed order is the CSR order
        theta = rng.integers(-3, 4, M.info.nnz).astype(np.float64)
        wv = rng.integers(-4, 5, G.nrows).astype(np.float64)
        xb = torch.full((G.ncols,), float("nan"), dtype=tdt, device=dev)
        M.transpose(torch.from_numpy(wv).to(dev, tdt), xb,
                    values=torch.from_numpy(theta).to(dev, tdt))
        got = xb.cpu().double().numpy()
        ref = oracle.csr_spmv_t(G.rowptr, G.colidx, theta, wv, G.ncols)
        assert np.array_equal(got, ref), (rep, int(np.sum(got != ref)))
    M.free()
