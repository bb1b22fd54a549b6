"""Differentiable path: y = A(theta) x through torch.autograd, backward in HIP.

Pins: (1) a dense float64 reference gradient on tiny matrices (torch dense
autograd on the CPU), (2) central finite differences with h = 1e-3 on the
1,048,576-row Zipf-column graph in FP32, evaluated with the FP64 oracle on the
FP32 data promoted to FP64.  The loss L = <w, A(theta) x> is bilinear, so the
central difference carries no truncation error, only rounding.
"""
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


def packed_coords(O):
    """(row, col) of every packed value, from the oracle's inverse expansion."""
    P = oracle.Spc5(**{**O.__dict__, "values": np.arange(O.nnz, dtype=np.float64)})
    rp, ci, idx = oracle.spc5_to_csr(P)
    rows = np.repeat(np.arange(O.nrows), np.diff(rp))
    order = idx.astype(np.int64)
    r = np.empty(O.nnz, np.int64)
    c = np.empty(O.nnz, np.int64)
    r[order] = rows
    c[order] = ci
    return r, c


@pytest.mark.parametrize("plan", [False, True], ids=["scatter", "plan"])
@pytest.mark.parametrize("rc", [(1, 8), (2, 4), (4, 4), (3, 5)], ids=str)
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_autograd_vs_dense_reference(rc, dtype, plan, dev):
    from paper_2307_14774_amd import spc5
    from paper_2307_14774_amd.autograd import spc5_matvec
    r, c = rc
    A = W.random_sparse(37, 29, 0.2, seed=31)
    say(f"autograd dense ref beta{rc} {dtype} plan={plan}")
    M = spc5.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, r, c, dtype)
    if plan:
        M.prepare_transpose()
    O = oracle.csr_to_spc5(A.rowptr, A.colidx, A.values, A.ncols, r, c)
    tdt = torch.float64 if dtype == "float64" else torch.float32
    rng = np.random.default_rng(5)
    theta0 = rng.uniform(-1, 1, O.nnz)
    w = rng.standard_normal(A.nrows)
    theta = torch.tensor(theta0, dtype=tdt, device=dev, requires_grad=True)
    x = torch.tensor(A.x, dtype=tdt, device=dev, requires_grad=True)
    y = spc5_matvec(M, theta, x)
    L = (y * torch.tensor(w, dtype=tdt, device=dev)).sum()
    L.backward()
    # dense reference in float64 on the CPU
    pr, pc = packed_coords(O)
    th = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    xr = torch.tensor(A.x, dtype=torch.float64, requires_grad=True)
    D = torch.zeros(A.nrows, A.ncols, dtype=torch.float64).index_put(
        (torch.from_numpy(pr), torch.from_numpy(pc)), th)
    Lr = (torch.tensor(w) * (D @ xr)).sum()
    Lr.backward()
    tol = 1e-12 if dtype == "float64" else 1e-5
    np.testing.assert_allclose(y.detach().cpu().double().numpy(), (D @ xr).detach().numpy(),
                               rtol=tol, atol=tol)
    np.testing.assert_allclose(theta.grad.cpu().double().numpy(), th.grad.numpy(), rtol=tol,
                               atol=tol)
    np.testing.assert_allclose(x.grad.cpu().double().numpy(), xr.grad.numpy(), rtol=tol * 10,
                               atol=tol * 10)


@pytest.mark.slow
@pytest.mark.parametrize("rc,plan", [((1, 8), True), ((2, 4), False)], ids=str)
def test_autograd_finite_differences_graph(rc, plan, dev):
    from paper_2307_14774_amd import spc5
    from paper_2307_14774_amd.autograd import spc5_matvec
    r, c = rc
    say(f"autograd FD on the 2^20 Zipf graph beta{rc} plan={plan}")
    G = W.zipf_graph(1 << 20, seed=0)
    M = spc5.Spc5Matrix.from_csr(G.rowptr, G.colidx, G.values, G.ncols, r, c, "float32")
    if plan:
        M.prepare_transpose()
    O = oracle.csr_to_spc5(G.rowptr, G.colidx, G.values, G.ncols, r, c)
    rng = np.random.default_rng(0)
    theta32 = rng.uniform(-1, 1, O.nnz).astype(np.float32)
    x32 = G.x.astype(np.float32)
    w = np.random.default_rng(0).standard_normal(G.nrows)
    theta = torch.tensor(theta32, device=dev, requires_grad=True)
    x = torch.tensor(x32, device=dev, requires_grad=True)
    y = spc5_matvec(M, theta, x)
    (y * torch.tensor(w, dtype=torch.float32, device=dev)).sum().backward()
    gth = theta.grad.cpu().double().numpy()
    gx = x.grad.cpu().double().numpy()
    # central differences of the full loss with the FP64 oracle (CSR form of
    # the same matrix: theta moved from packed to CSR order) on the FP32 data
    h = 1e-3
    pr, pc = packed_coords(O)
    # position of each packed value inside its CSR row (columns ascend)
    order = np.lexsort((pc, pr))
    pos = np.empty(O.nnz, np.int64)
    pos[order] = np.arange(O.nnz)
    th_csr = np.empty(O.nnz)
    th_csr[pos] = theta32.astype(np.float64)
    x64 = x32.astype(np.float64)

    def loss(th, xx):
        return float(w @ oracle.csr_spmv(G.rowptr, G.colidx, th, xx))

    for k in rng.choice(O.nnz, 64, replace=False):
        q = pos[k]
        keep = th_csr[q]
        th_csr[q] = keep + h
        lp = loss(th_csr, x64)
        th_csr[q] = keep - h
        lm = loss(th_csr, x64)
        th_csr[q] = keep
        fd = (lp - lm) / (2 * h)
        assert abs(gth[k] - fd) <= 1e-5 * max(1.0, abs(fd)), (k, gth[k], fd)
    for j in np.concatenate([[0, 1, 2], rng.choice(G.ncols, 61, replace=False)]):
        keep = x64[j]
        x64[j] = keep + h
        lp = loss(th_csr, x64)
        x64[j] = keep - h
        lm = loss(th_csr, x64)
        x64[j] = keep
        fd = (lp - lm) / (2 * h)
        assert abs(gx[j] - fd) <= 1e-3 * max(1.0, abs(fd)), (j, gx[j], fd)
