"""Batched products Y_m = A_m X_m over many uneven SPC5 matrices in one
persistent launch, the block-count planner and the shape autotuner.

Every matrix of a batch is checked against the FP64 oracle (CSR SpMM) on the
same seeded inputs; the planner's block counts against the oracle's greedy
conversion count (bit-exact); a HIP-graph capture of a batched run is replayed
several times with eager work in between and each replay compared with the
eager run (bit-exact: same kernel, same inputs, no atomics on the outputs).
"""
import numpy as np
import pytest

import oracle
from helpers import say
from paper_2307_14774_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BATCH_SHAPES = [(1, 8), (2, 4), (4, 4), (2, 8), (4, 8), (8, 8), (1, 16), (1, 4), (1, 3),
                (2, 5), (4, 7), (1, 12)]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def spc5():
    from paper_2307_14774_amd import spc5 as S
    return S


def small_batch():
    """Uneven sizes (log-uniform 40..3000 rows), power-law row lengths with
    runs, plus a matrix with empty rows and a 0-row matrix."""
    mats = W.batch_of_runs(nmat=22, seed=3, rows_lo=40, rows_hi=3000)
    mats.append(W.random_sparse(97, 61, 0.05, seed=4))
    mats.append(W.random_sparse(0, 5, 0.5, seed=5))
    return mats


BATCH = small_batch()


def build(S, mats, dtype):
    out = []
    for m, A in enumerate(mats):
        r, c = BATCH_SHAPES[m % len(BATCH_SHAPES)]
        out.append(S.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, r, c, dtype))
    return out


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("k", [1, 3, 4, 16, 20, 64])
def test_batch_parity(dtype, k, dev):
    S = spc5()
    say(f"batch parity {len(BATCH)} matrices {dtype} k={k}")
    mats = build(S, BATCH, dtype)
    B = S.Spc5Batch(mats)
    tdt = torch.float64 if dtype == "float64" else torch.float32
    rng = np.random.default_rng(100 + k)
    Xh = [rng.uniform(-1, 1, (A.ncols, k)) for A in BATCH]
    Xs = [torch.tensor(X, dtype=tdt, device=dev) for X in Xh]
    Ys = B.spmm(Xs)
    torch.cuda.synchronize()
    for m, A in enumerate(BATCH):
        Y = Ys[m].cpu().double().numpy()
        if dtype == "float64":
            ref = oracle.csr_spmm(A.rowptr, A.colidx, A.values, Xh[m])
            assert oracle.rel_l2(Y, ref) <= 1e-14, (m, A.name)
        else:
            v32 = A.values.astype(np.float32).astype(np.float64)
            x32 = Xh[m].astype(np.float32).astype(np.float64)
            ref = oracle.csr_spmm(A.rowptr, A.colidx, v32, x32)
            assert oracle.rel_l2(Y, ref) <= 1e-6, (m, A.name)
    B.free()


R1_SHAPES = [(1, 8), (1, 16), (1, 4), (1, 3), (1, 12), (1, 5)]


def r1_batch():
    """beta(1,c) batch (value-mode tiles): the uneven matrices plus one with
    hub rows of thousands of nonzeros (panels split over several tiles)."""
    from test_gpu_parity import long_panel_matrix
    return BATCH[:14] + [long_panel_matrix(29)]


R1 = r1_batch()


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("k", [1, 3, 4, 16, 20, 64])
def test_batch_value_mode_parity(dtype, k, dev):
    S = spc5()
    say(f"value-mode batch {len(R1)} matrices {dtype} k={k}")
    mats = [S.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols,
                                  *R1_SHAPES[m % len(R1_SHAPES)], dtype) for m, A in enumerate(R1)]
    assert mats[-1].info.split_panels > 0
    B = S.Spc5Batch(mats)
    tdt = torch.float64 if dtype == "float64" else torch.float32
    rng = np.random.default_rng(200 + k)
    Xh = [rng.uniform(-1, 1, (A.ncols, k)) for A in R1]
    Ys = B.spmm([torch.tensor(X, dtype=tdt, device=dev) for X in Xh])
    torch.cuda.synchronize()
    for m, A in enumerate(R1):
        Y = Ys[m].cpu().double().numpy()
        if dtype == "float64":
            ref = oracle.csr_spmm(A.rowptr, A.colidx, A.values, Xh[m])
            assert oracle.rel_l2(Y, ref) <= 1e-14, (m, A.name)
        else:
            ref = oracle.csr_spmm(A.rowptr, A.colidx, A.values.astype(np.float32).astype(np.float64),
                                  Xh[m].astype(np.float32).astype(np.float64))
            assert oracle.rel_l2(Y, ref) <= 1e-6, (m, A.name)


def test_batch_value_mode_graph_replay(dev):
    S = spc5()
    say("value-mode batch graph replays")
    mats = [S.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols,
                                  *R1_SHAPES[m % len(R1_SHAPES)]) for m, A in enumerate(R1)]
    B = S.Spc5Batch(mats)
    k = 4
    rng = np.random.default_rng(13)
    Xs = [torch.tensor(rng.uniform(-1, 1, (A.ncols, k)), device=dev) for A in R1]
    Ys = [torch.zeros((A.nrows, k), dtype=torch.float64, device=dev) for A in R1]
    B.set_operands(Xs, Ys)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        B.run(side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        B.run(torch.cuda.current_stream())
    torch.cuda.synchronize()
    for rep in range(3):
        for X in Xs:
            X.copy_(torch.tensor(rng.uniform(-1, 1, tuple(X.shape)), device=dev))
        for Y in Ys:
            Y.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [Y.clone() for Y in Ys]
        for Y in Ys:
            Y.fill_(float("nan"))
        B.run()
        torch.cuda.synchronize()
        for m, A in enumerate(R1):
            assert torch.equal(got[m], Ys[m]), (rep, m)
            ref = oracle.csr_spmm(A.rowptr, A.colidx, A.values, Xs[m].cpu().numpy())
            assert oracle.rel_l2(got[m].cpu().numpy(), ref) <= 1e-14, (rep, m)


def test_batch_rebind_smaller(dev):
    """A second binding with fewer right-hand sides and other vectors."""
    S = spc5()
    say("batch rebind 16 -> 3")
    mats = build(S, BATCH[:8], "float64")
    B = S.Spc5Batch(mats)
    rng = np.random.default_rng(7)
    for k in (16, 3):
        Xh = [rng.uniform(-1, 1, (A.ncols, k)) for A in BATCH[:8]]
        Ys = B.spmm([torch.tensor(X, device=dev) for X in Xh])
        for m, A in enumerate(BATCH[:8]):
            ref = oracle.csr_spmm(A.rowptr, A.colidx, A.values, Xh[m])
            assert oracle.rel_l2(Ys[m].cpu().numpy(), ref) <= 1e-14


def test_batch_graph_replay(dev):
    S = spc5()
    say("batch hip graph capture + replays")
    mats = build(S, BATCH, "float64")
    B = S.Spc5Batch(mats)
    k = 4
    rng = np.random.default_rng(11)
    Xs = [torch.tensor(rng.uniform(-1, 1, (A.ncols, k)), device=dev) for A in BATCH]
    Ys = [torch.zeros((A.nrows, k), dtype=torch.float64, device=dev) for A in BATCH]
    B.set_operands(Xs, Ys)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        B.run(side)            # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        B.run(torch.cuda.current_stream())
    torch.cuda.synchronize()
    for rep in range(4):
        # new inputs written eagerly between replays
        for X in Xs:
            X.copy_(torch.tensor(rng.uniform(-1, 1, tuple(X.shape)), device=dev))
        for Y in Ys:
            Y.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [Y.clone() for Y in Ys]
        for Y in Ys:
            Y.fill_(float("nan"))
        B.run()
        torch.cuda.synchronize()
        for m, A in enumerate(BATCH):
            assert torch.equal(got[m], Ys[m]), (rep, m)
            ref = oracle.csr_spmm(A.rowptr, A.colidx, A.values, Xs[m].cpu().numpy())
            assert oracle.rel_l2(got[m].cpu().numpy(), ref) <= 1e-14, (rep, m)


def test_batch_rejects_bad_input(dev):
    S = spc5()
    A = BATCH[0]
    say("batch error paths")
    M3 = S.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, 3, 4)
    with pytest.raises(S.Spc5Error) as ei:
        S.Spc5Batch([M3])
    assert ei.value.status == -5
    M64 = S.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, 2, 4)
    M32 = S.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, 2, 4, "float32")
    with pytest.raises(S.Spc5Error) as ei:
        S.Spc5Batch([M64, M32])
    assert ei.value.status == -1
    B = S.Spc5Batch([M64])
    with pytest.raises(S.Spc5Error) as ei:
        B.run()
    assert ei.value.status == -1
    X = torch.zeros((A.ncols, 65), dtype=torch.float64, device=dev)
    Y = torch.zeros((A.nrows, 65), dtype=torch.float64, device=dev)
    with pytest.raises(S.Spc5Error):
        B.set_operands([X], [Y])


@pytest.mark.parametrize("m", [0, 5, 22, 23])
def test_plan_counts_match_oracle(m, dev):
    S = spc5()
    A = BATCH[m]
    cands = [(1, 8), (2, 4), (4, 4), (3, 5), (8, 16), (1, 1), (7, 13)]
    say(f"plan {A.name}")
    got = S.plan(A.rowptr, A.colidx, A.ncols, cands)
    want = [oracle.spc5_count(A.rowptr, A.colidx, r, c) for r, c in cands]
    assert got == want


def test_autotune_shape_and_schedule(dev):
    from paper_2307_14774_amd import autotune
    A = W.laplacian_2d(64)
    say("autotune laplacian 64^2")
    (r, c), table = autotune.choose_shape(A)
    assert table[(r, c)] == min(table.values())
    # model bytes from the oracle's counts, independently
    for (rr, cc), b in table.items():
        nb = oracle.spc5_count(A.rowptr, A.colidx, rr, cc)
        assert b == autotune.model_bytes(A.nnz, A.nrows, A.ncols, rr, cc, nb, 8)
    M, info = autotune.autotune(A, measure=True, nrhs=4)
    assert info["shape"] == (r, c)
    assert M.info.panels_per_tile >= 1
    y = M.spmv(torch.tensor(A.x, device=dev)).cpu().numpy()
    ref = oracle.csr_spmv(A.rowptr, A.colidx, A.values, A.x)
    assert oracle.rel_l2(y, ref) <= 1e-14


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("k", [1, 4, 16])
def test_batch_per_matrix_schedules(dtype, k, dev):
    """Per-matrix batch tile caps (spc5_set_batch_schedule, as the autotuner
    sets them), on the value-mode batch (hub rows split into pieces) and on
    the work-queue batch: every matrix against the FP64 oracle; the tuner
    keeps one of its candidates per matrix."""
    from paper_2307_14774_amd import autotune
    S = spc5()
    tdt = torch.float64 if dtype == "float64" else torch.float32
    gate = 1e-14 if dtype == "float64" else 1e-6
    rng = np.random.default_rng(300 + k)
    for label, mats_h, shapes in (("value mode", R1, R1_SHAPES), ("work queue", BATCH, BATCH_SHAPES)):
        say(f"per-matrix batch schedules {label} {dtype} k={k}")
        mats = [S.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols,
                                      *shapes[m % len(shapes)], dtype) for m, A in enumerate(mats_h)]
        caps = [(0, 128, 64, 32, 8, 1)[m % 6] for m in range(len(mats))]
        for M, cp in zip(mats, caps):
            M.set_batch_schedule(cp)
        Xh = [rng.uniform(-1, 1, (A.ncols, k)) for A in mats_h]
        B = S.Spc5Batch(mats)
        Ys = B.spmm([torch.tensor(X, dtype=tdt, device=dev) for X in Xh])
        torch.cuda.synchronize()
        for m, A in enumerate(mats_h):
            v = A.values if dtype == "float64" else A.values.astype(np.float32).astype(np.float64)
            X = Xh[m] if dtype == "float64" else Xh[m].astype(np.float32).astype(np.float64)
            ref = oracle.csr_spmm(A.rowptr, A.colidx, v, X)
            assert oracle.rel_l2(Ys[m].cpu().double().numpy(), ref) <= gate, (label, m, caps[m])
        B.free()
        if label == "value mode":
            chosen = autotune.tune_batch(mats[:4], k)
            assert all(c in autotune.BATCH_PPT for c in chosen)
    with pytest.raises(S.Spc5Error):
        mats[0].set_batch_schedule(257)
