#!/usr/bin/env python3
"""SPC5 SpMV benchmark on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload laplacian|fem|random]

A step is one forward product y = A x over the SPC5 beta(r,c) storage (all
hot-path steps: panel scheduling, metadata stream, mask expansion, value
stream, x gather, FMA, row reduction and y store) of one seeded synthetic
matrix already resident in HBM.  The default workload is the largest one
that fits one GPU: the 3D vector-FEM-like matrix on 96^3 nodes x 3 dof
(2,654,208 rows, 210.5 M nonzeros) in FP64 with beta(4,4).  One JSON line
is printed: GFLOP/s (2 flops per stored nonzero), the roofline of the
forward kernel (algorithmic bytes / mean launch time against 8 TB/s), the
other kernels and formats and the plain CSR kernel on the same matrix, FP32,
the 2048^2 Laplacian (warm and with the Infinity Cache flushed), the
differentiated product (forward + backward) on the 2^20 Zipf graph, the
batched SpMM over 256 uneven matrices, the paper's ablations, and the CPU
oracle timed on this host as a baseline (one thread and all cores).  Launch times are means over back-to-back launches
between one HIP event pair on the launching stream (gaps between launches
included); the cold-cache run alone puts an event pair around every launch,
so that the flush between launches stays outside the events.

Profiling helpers (host only, no GPU):
    python bench.py --traffic-from FETCH.csv WRITE.csv
reads two rocprofv3 --pmc counter files (FETCH_SIZE, then WRITE_SIZE) of a
`--calibration-copy` run and writes the HBM traffic per launch of the forward
kernel, scaled by what the same counters read for a plain copy of known size.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SpMV GFLOP/s + achieved HBM GB/s (% peak), SPC5 vs CSR, fwd+bwd, FP64/FP32"
PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ["paper_2307_14774_amd/csrc/staged.hip", "paper_2307_14774_amd/csrc/stage.h",
                  "paper_2307_14774_amd/csrc/spmv.hip", "paper_2307_14774_amd/csrc/wave.h",
                  "paper_2307_14774_amd/csrc/tile.h"]
FWD_KERNEL = "k_spmv_stream"
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic_spc5_fwd.json")
COPY_ELEMS = 1 << 27          # calibration copy: 1 GiB read + 1 GiB written (float64)


def kernel_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


WORKLOADS = {   # name -> (tag, beta(r,c) of the timed product)
    "laplacian": ("laplacian2d_2048", (4, 4)),
    "fem": ("fem3d_96x3", (4, 4)),
    "random": ("random10k", (1, 8)),
    "zipf": ("zipf_graph_2^20", (1, 8)),
}


def make_workload(name, dtype="float64"):
    from paper_2307_14774_amd import workloads as W
    if name not in WORKLOADS:
        raise SystemExit(f"unknown workload {name}")
    tag, rc = WORKLOADS[name]
    A = {"laplacian": lambda: W.laplacian_2d(2048, seed=0),
         "fem": lambda: W.fem_3d(96, seed=0),
         "random": lambda: W.random_uniform(10_000, 10, seed=0),
         "zipf": lambda: W.zipf_graph(1 << 20, seed=0)}[name]()
    return A, rc, tag + (" fp64" if dtype == "float64" else " fp32")


def time_launches(fn, steps, warmup, flush=None):
    """Run fn() `warmup` times, then `steps` times with a HIP event pair around
    every launch on the current stream.  Returns (wall seconds of the timed
    region, list of per-launch ms)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        if flush is not None:
            flush()
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return t1 - t0, [a.elapsed_time(b) for a, b in ev]


def time_region(fn, steps, warmup):
    """Run fn() `warmup` times, then `steps` times back to back between one
    HIP event pair on the current stream (the stream the kernels run on).
    Returns (wall seconds of the timed region, mean ms per launch): the
    launches' own durations plus the gaps between consecutive launches."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return t1 - t0, a.elapsed_time(b) / steps


def traffic_from_profiles(workload_tag):
    """HBM bytes per launch of the forward kernel from the committed counter
    summary, or None when it is missing, for another workload, or was taken
    on kernel sources that have changed since."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    try:
        with open(TRAFFIC_JSON) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha") != kernel_sha() or d.get("workload") != workload_tag:
        return None
    return d.get("bytes_per_launch")


def _counter_means(path, counter):
    """Mean Counter_Value per dispatch, keyed by kernel name, of one rocprofv3
    counter-collection CSV (values of one dispatch are summed first)."""
    import csv
    per_dispatch = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] != counter:
                continue
            key = (row["Dispatch_Id"], row["Kernel_Name"])
            per_dispatch[key] = per_dispatch.get(key, 0.0) + float(row["Counter_Value"])
    sums = {}
    for (_, name), v in per_dispatch.items():
        n, t = sums.get(name, (0, 0.0))
        sums[name] = (n + 1, t + v)
    return {name: (t / n, n) for name, (n, t) in sums.items()}


def traffic_write(fetch_csv, write_csv, workload, dtype="float64"):
    """Scale the forward kernel's FETCH_SIZE and WRITE_SIZE (KiB per dispatch)
    by what the same counters read for the calibration copy (COPY_ELEMS
    float64 read and written once) and store bytes per launch."""
    tag, rc = WORKLOADS[workload]
    tag = tag + (" fp64" if dtype == "float64" else " fp32") + f" beta({rc[0]},{rc[1]})"
    fetch = _counter_means(fetch_csv, "FETCH_SIZE")
    write = _counter_means(write_csv, "WRITE_SIZE")

    def pick(table, needle):
        hits = [(k, v) for k, v in table.items() if needle in k]
        if len(hits) != 1:
            raise SystemExit(f"expected one kernel matching {needle!r}, found "
                             f"{[k[:80] for k, _ in hits]}")
        return hits[0]

    copy_bytes = COPY_ELEMS * 8
    kc, (fc, _) = pick(fetch, "neg_kernel")
    _, (wc, _) = pick(write, "neg_kernel")
    fetch_factor = copy_bytes / (fc * 1024.0)
    write_factor = copy_bytes / (wc * 1024.0)
    kf, (fk, nf) = pick(fetch, FWD_KERNEL)
    _, (wk, nw) = pick(write, FWD_KERNEL)
    fetch_b = fk * 1024.0 * fetch_factor
    write_b = wk * 1024.0 * write_factor
    out = {"kernel": kf, "kernel_sha": kernel_sha(), "workload": tag,
           "fetch_kib_per_dispatch": round(fk, 3), "write_kib_per_dispatch": round(wk, 3),
           "dispatches": [nf, nw], "calibration_kernel": kc,
           "calibration_bytes_each_way": copy_bytes,
           "fetch_factor": round(fetch_factor, 4), "write_factor": round(write_factor, 4),
           "fetch_bytes": int(fetch_b), "write_bytes": int(write_b),
           "bytes_per_launch": int(fetch_b + write_b)}
    os.makedirs(os.path.dirname(TRAFFIC_JSON), exist_ok=True)
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def host_identity():
    """CPU model name and the number of cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores, os.cpu_count() or 1


def cpu_baseline(A, passes=5):
    """The oracle as it stands, O1 (the CSR definition, FP64, built -O3
    -ffp-contract=off), timed on this host: one thread, and all the cores
    this process may use with the rows cut into equal contiguous ranges, one
    per thread (the paper's naive static split, Section 4.3).  Each leg runs
    `passes` full passes over the whole matrix after one untimed pass; the
    median pass is reported."""
    import numpy as np

    import oracle
    model, cores, nproc = host_identity()

    def leg(fn):
        fn()
        ts = []
        for _ in range(passes):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), ts

    t1, ts1 = leg(lambda: oracle.csr_spmv(A.rowptr, A.colidx, A.values, A.x))
    tn, tsn = leg(lambda: oracle.csr_spmv_par(A.rowptr, A.colidx, A.values, A.x, cores))
    gf = lambda t: round(2.0 * A.nnz / t / 1e9, 4)
    return {"value": gf(tn), "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"median of {passes} full passes of O1 (CSR definition, FP64) over the "
                      f"whole matrix on {cores} threads, rows split evenly; one thread: "
                      f"median of {passes} passes",
            "single_thread": {"value": gf(t1), "median_pass_s": round(t1, 4),
                              "passes_s": [round(t, 4) for t in ts1]},
            "all_cores": {"value": gf(tn), "threads": cores, "median_pass_s": round(tn, 4),
                          "passes_s": [round(t, 4) for t in tsn]},
            "host": {"cpu_model": model, "nproc": nproc, "cores_available": cores}}


def fem_extras(dev):
    """3D 3-dof 27-point FEM-like matrix (96^3 nodes, 210.5 M nonzeros): FP64
    and FP32 beta(4,4) and beta(1,8), plain CSR FP64; FP32 error against the
    FP64 oracle on the original FP64 data (used when the timed workload is
    another matrix)."""
    import torch

    import oracle
    from paper_2307_14774_amd import spc5
    from paper_2307_14774_amd import workloads as W
    log("generating the FEM workload")
    A = W.fem_3d(96, seed=0)
    yref = oracle.csr_spmv(A.rowptr, A.colidx, A.values, A.x)
    res = {"nrows": A.nrows, "nnz": A.nnz}
    for dt, tdt in (("float64", torch.float64), ("float32", torch.float32)):
        x = torch.from_numpy(A.x).to(dev, tdt)
        y = torch.empty(A.nrows, dtype=tdt, device=dev)
        shapes = [(4, 4), (1, 8), (2, 4)] if dt == "float64" else [(4, 4), (4, 8), (1, 16)]
        for rc in shapes:
            log(f"FEM {dt} beta{rc}")
            M = spc5.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, *rc, dt)
            avg = time_region(lambda: M.spmv(x, y), 30, 5)[1] * 1e-3
            nb = M.info.spmv_bytes
            res[f"{dt} beta({rc[0]},{rc[1]})"] = {
                "gflops": round(2.0 * A.nnz / avg / 1e9, 1), "launch_us": round(avg * 1e6, 1),
                "gbs": round(nb / avg / 1e9, 1), "frac_hbm": round(nb / avg / 1e9 / PEAK_HBM_GBS, 4),
                "rel_l2_vs_fp64_oracle": oracle.rel_l2(y.cpu().numpy(), yref),
                "kernel": M.kernel, "fill": round(M.info.fill, 4)}
            M.free()
    log("FEM plain CSR fp64")
    C = spc5.CsrMatrix(A.rowptr, A.colidx, A.values, A.ncols)
    x = torch.from_numpy(A.x).to(dev)
    y = torch.empty(A.nrows, dtype=torch.float64, device=dev)
    avg = time_region(lambda: C.spmv(x, y), 30, 5)[1] * 1e-3
    res["float64 csr"] = {"gflops": round(2.0 * A.nnz / avg / 1e9, 1),
                          "launch_us": round(avg * 1e6, 1),
                          "gbs": round(C.spmv_bytes / avg / 1e9, 1),
                          "frac_hbm": round(C.spmv_bytes / avg / 1e9 / PEAK_HBM_GBS, 4),
                          "rel_l2_vs_fp64_oracle": oracle.rel_l2(y.cpu().numpy(), yref)}
    C.free()
    return res


def laplacian_extras(dev, A):
    """The 2D 5-point Laplacian on a 2048^2 grid (20.96 M nonzeros, 272.6 MB
    in FP64 beta(4,4), about the size of the 256 MB Infinity Cache): FP64
    beta(4,4) warm (back-to-back launches) and flushed (a 1 GiB buffer read
    between launches, outside the timed events), FP32 beta(4,4), and the
    plain CSR kernel FP64."""
    import torch

    import oracle
    from paper_2307_14774_amd import spc5
    yref = oracle.csr_spmv(A.rowptr, A.colidx, A.values, A.x)
    res = {"nrows": A.nrows, "nnz": A.nnz}
    x = torch.from_numpy(A.x).to(dev)
    y = torch.empty(A.nrows, dtype=torch.float64, device=dev)

    def entry(avg_s, nb, yy):
        return {"gflops": round(2.0 * A.nnz / avg_s / 1e9, 1), "launch_us": round(avg_s * 1e6, 2),
                "gbs": round(nb / avg_s / 1e9, 1), "frac_hbm": round(nb / avg_s / 1e9 / PEAK_HBM_GBS, 4),
                "rel_l2_vs_fp64_oracle": oracle.rel_l2(yy.cpu().double().numpy(), yref)}
    log("Laplacian fp64 beta(4,4)")
    M = spc5.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, 4, 4)
    nb = M.info.spmv_bytes
    res["float64 beta(4,4)"] = entry(time_region(lambda: M.spmv(x, y), 200, 100)[1] * 1e-3, nb, y)
    scratch = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    sink = torch.empty((), dtype=torch.float64, device=dev)
    _, ms = time_launches(lambda: M.spmv(x, y), 30, 3,
                          flush=lambda: torch.sum(scratch, dim=0, out=sink))
    res["float64 beta(4,4) flushed"] = entry(float(sum(ms) / len(ms)) * 1e-3, nb, y)
    del scratch, sink
    M.free()
    log("Laplacian fp32 beta(4,4)")
    M = spc5.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, 4, 4, "float32")
    x32, y32 = x.float(), torch.empty(A.nrows, dtype=torch.float32, device=dev)
    res["float32 beta(4,4)"] = entry(time_region(lambda: M.spmv(x32, y32), 200, 100)[1] * 1e-3,
                                     M.info.spmv_bytes, y32)
    M.free()
    log("Laplacian plain CSR fp64")
    C = spc5.CsrMatrix(A.rowptr, A.colidx, A.values, A.ncols)
    res["float64 csr"] = entry(time_region(lambda: C.spmv(x, y), 100, 20)[1] * 1e-3,
                               C.spmv_bytes, y)
    C.free()
    res["speedup_vs_csr"] = round(res["float64 csr"]["launch_us"]
                                  / res["float64 beta(4,4)"]["launch_us"], 3)
    log("Laplacian rocSPARSE CSR fp64")
    rs = rocsparse_csr(dev, A, yref)
    if rs is not None:
        res["float64 csr rocsparse"] = rs
        res["speedup_vs_rocsparse_csr"] = round(rs["launch_us"]
                                                / res["float64 beta(4,4)"]["launch_us"], 3)
    return res


def rocsparse_csr(dev, A, yref, steps=100, warmup=20):
    """The vendor library's CSR product (rocSPARSE csrmv with its analysis
    step, FP64) on the same matrix: a run-only yardstick for the plain CSR
    format next to this library's own CSR kernel.  Returns None when the
    library cannot be loaded."""
    import ctypes

    import numpy as np
    import torch

    import oracle
    lib = None
    for name in ("librocsparse.so", "/opt/rocm/lib/librocsparse.so"):
        try:
            lib = ctypes.CDLL(name)
            break
        except OSError:
            continue
    if lib is None:
        return None
    P = ctypes.c_void_p

    def ok(st, what):
        if st != 0:
            raise RuntimeError(f"rocsparse {what}: status {st}")
    h, descr, info = P(), P(), P()
    ok(lib.rocsparse_create_handle(ctypes.byref(h)), "create_handle")
    ok(lib.rocsparse_set_stream(h, P(torch.cuda.current_stream().cuda_stream)), "set_stream")
    ok(lib.rocsparse_create_mat_descr(ctypes.byref(descr)), "create_mat_descr")
    ok(lib.rocsparse_create_mat_info(ctypes.byref(info)), "create_mat_info")
    m, n, nnz = A.nrows, A.ncols, A.nnz
    rp = torch.from_numpy(A.rowptr.astype(np.int32)).to(dev)
    ci = torch.from_numpy(A.colidx).to(dev)
    va = torch.from_numpy(A.values).to(dev)
    x = torch.from_numpy(A.x).to(dev)
    y = torch.empty(m, dtype=torch.float64, device=dev)
    ptr = lambda t: P(t.data_ptr())
    op_none = 111
    lib.rocsparse_dcsrmv_analysis.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int, P, P, P, P, P]
    lib.rocsparse_dcsrmv.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     P, P, P, P, P, P, P, P, P]
    ok(lib.rocsparse_dcsrmv_analysis(h, op_none, m, n, nnz, descr, ptr(va), ptr(rp), ptr(ci),
                                     info), "dcsrmv_analysis")
    alpha, beta = ctypes.c_double(1.0), ctypes.c_double(0.0)
    ap_, bp_ = ctypes.cast(ctypes.byref(alpha), P), ctypes.cast(ctypes.byref(beta), P)
    args = (h, op_none, m, n, nnz, ap_, descr, ptr(va), ptr(rp), ptr(ci), info, ptr(x), bp_,
            ptr(y))
    ok(lib.rocsparse_dcsrmv(*args), "dcsrmv")
    avg = time_region(lambda: lib.rocsparse_dcsrmv(*args), steps, warmup)[1] * 1e-3
    nb = 8 * nnz + 4 * nnz + 4 * (m + 1) + 8 * n + 8 * m
    res = {"kernel": "rocsparse_dcsrmv (adaptive, after csrmv_analysis)",
           "launch_us": round(avg * 1e6, 2), "gflops": round(2.0 * nnz / avg / 1e9, 1),
           "gbs": round(nb / avg / 1e9, 1), "frac_hbm": round(nb / avg / 1e9 / PEAK_HBM_GBS, 4),
           "rel_l2_vs_fp64_oracle": oracle.rel_l2(y.cpu().numpy(), yref)}
    lib.rocsparse_destroy_mat_info(info)
    lib.rocsparse_destroy_mat_descr(descr)
    lib.rocsparse_destroy_handle(h)
    return res


def backward_extras(dev):
    """Differentiated product y = A(theta) x in FP32 on the 2^20-row graph with
    Zipf(1.2) column popularity (16.8 M nonzeros): forward, transpose
    scatter xbar = A^T ybar and packed values gradient, each timed per launch,
    plus one autograd forward+backward; compared with plain FP64 CSR SpMV
    on the same matrix.  Parity: transpose against the FP64 oracle on the
    FP32 data (rel L2), values gradient bit-exact against the oracle's exact
    products rounded to FP32."""
    import numpy as np
    import torch

    import oracle
    from paper_2307_14774_amd import autotune, spc5
    from paper_2307_14774_amd import workloads as W
    from paper_2307_14774_amd.autograd import spc5_matvec
    log("generating the Zipf graph")
    G = W.zipf_graph(1 << 20, seed=0)
    (r, c), _ = autotune.choose_shape(G, "float32")
    log(f"graph beta({r},{c}) fp32")
    M = spc5.Spc5Matrix.from_csr(G.rowptr, G.colidx, G.values, G.ncols, r, c, "float32")
    nb = M.info.spmv_bytes
    rng = np.random.default_rng(0)
    theta_h = rng.uniform(-1, 1, G.nnz).astype(np.float32)
    x_h = G.x.astype(np.float32)
    w_h = rng.standard_normal(G.nrows).astype(np.float32)
    theta = torch.from_numpy(theta_h).to(dev)
    x = torch.from_numpy(x_h).to(dev)
    ybar = torch.from_numpy(w_h).to(dev)
    y = torch.empty(G.nrows, dtype=torch.float32, device=dev)
    xbar = torch.empty(G.ncols, dtype=torch.float32, device=dev)
    vbar = torch.empty(G.nnz, dtype=torch.float32, device=dev)
    res = {"nrows": G.nrows, "nnz": G.nnz, "beta": [r, c], "fill": round(M.info.fill, 4),
           "dtype": "f32"}
    def timed(fn, n=30):
        us = time_region(fn, n, 5)[1] * 1e3
        return {"launch_us": round(us, 2), "gbs": round(nb / us / 1e3, 1),
                "frac_hbm": round(nb / us / 1e3 / PEAK_HBM_GBS, 4)}
    res["forward"] = timed(lambda: M.spmv_values(theta, x, y))
    res["values_grad"] = timed(lambda: M.values_grad(ybar, x, vbar))
    # masked scatter with atomics (no plan): serialises on popular columns
    res["transpose_scatter"] = timed(lambda: M.transpose(ybar, xbar, values=theta), 5)
    t0 = time.perf_counter()
    M.prepare_transpose()
    res["transpose_plan_build_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    res["transpose_plan"] = {"beta": [M.info.transpose_r, M.info.transpose_c],
                             "kernel": {1: "rows", 2: "sweep", 3: "staged"}.get(
                                 M.info.transpose_kernel)}
    # through the plan: caller theta gathered to A^T order, then the forward
    # kernel over A^T (both launches inside the timed region)
    res["transpose"] = timed(lambda: M.transpose(ybar, xbar, values=theta))
    res["transpose_own_values"] = timed(lambda: M.transpose(ybar, xbar))
    res["fwd_bwd_us"] = round(sum(res[k]["launch_us"]
                                  for k in ("forward", "transpose", "values_grad")), 2)
    # one full autograd step, wall clock
    th = theta.clone().requires_grad_(True)
    xx = x.clone().requires_grad_(True)

    def step():
        th.grad = None
        xx.grad = None
        (spc5_matvec(M, th, xx) * ybar).sum().backward()
    res["autograd_step_us"] = round(time_region(step, 10, 3)[1] * 1e3, 1)
    # parity
    O = oracle.csr_to_spc5(G.rowptr, G.colidx, theta_h.astype(np.float64), G.ncols, r, c)
    M.transpose(ybar, xbar, values=theta)
    M.values_grad(ybar, x, vbar)
    # theta is in packed order: go back to CSR order for the CSR oracle
    rp, ci, vals = oracle.spc5_to_csr(O)
    xt_ref = oracle.csr_spmv_t(rp, ci, vals, w_h.astype(np.float64), G.ncols)
    res["transpose_rel_l2_vs_fp64_oracle"] = oracle.rel_l2(xbar.cpu().numpy(), xt_ref)
    vg_ref = oracle.spc5_values_grad(O, w_h.astype(np.float64), x_h.astype(np.float64))
    res["values_grad_bit_exact"] = bool(np.array_equal(vbar.cpu().numpy(),
                                                       vg_ref.astype(np.float32)))
    # plain FP64 CSR SpMV on the same matrix
    C = spc5.CsrMatrix(G.rowptr, G.colidx, G.values, G.ncols)
    x64 = torch.from_numpy(G.x).to(dev)
    y64 = torch.empty(G.nrows, dtype=torch.float64, device=dev)
    us_csr = time_region(lambda: C.spmv(x64, y64), 30, 5)[1] * 1e3
    res["csr_fp64_forward_us"] = round(us_csr, 2)
    res["speedup_fwd_vs_csr_fp64"] = round(res["csr_fp64_forward_us"]
                                           / res["forward"]["launch_us"], 3)
    res["fwd_bwd_vs_3x_csr_fp64"] = round(3 * res["csr_fp64_forward_us"] / res["fwd_bwd_us"], 3)
    C.free()
    M.free()
    return res


def batch_extras(dev, nmat=256, ks=(1, 4, 16), dtypes=("float64", "float32")):
    """Batched workload: `nmat` uneven matrices (log-uniform 1k..200k rows,
    Zipf(1.5) row lengths capped at 512, 30% of nonzeros in runs), beta(r,c)
    per matrix from the byte-model autotuner and each matrix's batch tile cap
    measured by it, k right-hand sides, all in one persistent launch; against
    plain FP64 single SpMVs (CSR kernel and SPC5 FP64 at the same shapes), one
    launch per matrix and vector.  Every matrix's Y is checked against the
    FP64 oracle."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import oracle
    from paper_2307_14774_amd import autotune, spc5
    from paper_2307_14774_amd import workloads as W
    log(f"generating {nmat} batch matrices")
    mats = W.batch_of_runs(nmat, seed=0)
    nnz = sum(A.nnz for A in mats)
    res = {"nmat": nmat, "nnz": nnz, "rows": sum(A.nrows for A in mats)}
    # plain FP64 single SpMVs: one CSR launch per matrix and vector
    log("batch: plain FP64 CSR launches")
    csrs = [spc5.CsrMatrix(A.rowptr, A.colidx, A.values, A.ncols) for A in mats]
    xs = [torch.from_numpy(A.x).to(dev) for A in mats]
    ys = [torch.empty(A.nrows, dtype=torch.float64, device=dev) for A in mats]

    def plain_csr():
        for C, x, y in zip(csrs, xs, ys):
            C.spmv(x, y)
    plain_csr_us = time_region(plain_csr, 5, 2)[1] * 1e3
    res["plain_fp64_csr_us_per_vector"] = round(plain_csr_us, 1)
    for C in csrs:
        C.free()
    del csrs
    for dt, tdt in (("float64", torch.float64), ("float32", torch.float32)):
        if dt not in dtypes:
            continue
        log(f"batch: autotune + convert {dt}")
        Ms, shapes = [], {}
        for A in mats:
            (r, c), _ = autotune.choose_shape(A, dt)
            shapes[f"{r},{c}"] = shapes.get(f"{r},{c}", 0) + 1
            Ms.append(spc5.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, r, c, dt))
        res[f"{dt} shapes"] = shapes
        if dt == "float64":
            log("batch: plain FP64 SPC5 launches")
            def plain_spc5():
                for M, x, y in zip(Ms, xs, ys):
                    M.spmv(x, y)
            us_plain = time_region(plain_spc5, 5, 2)[1] * 1e3
            res["plain_fp64_spc5_us_per_vector"] = round(us_plain, 1)
        B = spc5.Spc5Batch(Ms)
        vb = 8 if dt == "float64" else 4
        vals = [A.values if dt == "float64" else A.values.astype(np.float32).astype(np.float64)
                for A in mats]
        for k in ks:
            log(f"batch: {dt} k={k}")
            rng = np.random.default_rng(k)
            Xh = [rng.uniform(-1, 1, (A.ncols, k)) for A in mats]
            if dt == "float32":
                Xh = [X.astype(np.float32).astype(np.float64) for X in Xh]
            Xs = [torch.from_numpy(X).to(dev, tdt) for X in Xh]
            Ys = [torch.empty((A.nrows, k), dtype=tdt, device=dev) for A in mats]
            B.set_operands(Xs, Ys)
            us_default = time_region(B.run, 10, 3)[1] * 1e3
            # per-matrix schedule from the autotuner: each matrix's batch tile
            # cap timed on a batch of it alone with k right-hand sides
            log(f"batch: {dt} k={k} tuning the per-matrix schedule")
            t0 = time.perf_counter()
            caps = autotune.tune_batch(Ms, k)
            tune_s = time.perf_counter() - t0
            Bt = spc5.Spc5Batch(Ms)
            Bt.set_operands(Xs, Ys)
            us_tuned = time_region(Bt.run, 10, 3)[1] * 1e3
            for M in Ms:
                M.set_batch_schedule(0)
            use_tuned = us_tuned < us_default
            us = min(us_tuned, us_default)
            (Bt if use_tuned else B).run()
            torch.cuda.synchronize()
            Bt.free()
            # matrix streamed once per launch + k vectors in and out
            byts = sum(M.info.spmv_bytes - vb * (A.ncols + A.nrows) + k * vb * (A.ncols + A.nrows)
                       for M, A in zip(Ms, mats))
            Yh = [Y.cpu().double().numpy() for Y in Ys]

            def err(i):
                A = mats[i]
                return oracle.rel_l2(Yh[i], oracle.csr_spmm(A.rowptr, A.colidx, vals[i], Xh[i]))
            with ThreadPoolExecutor(8) as ex:
                errs = list(ex.map(err, range(nmat)))
            plain = k * plain_csr_us
            hist = {}
            for cp in caps:
                hist[str(cp)] = hist.get(str(cp), 0) + 1
            res[f"{dt} k={k}"] = {
                "launch_us": round(us, 1), "gflops": round(2.0 * nnz * k / us / 1e3, 1),
                "gbs": round(byts / us / 1e3, 1), "frac_hbm": round(byts / us / 1e3 / PEAK_HBM_GBS, 4),
                "default_schedule_us": round(us_default, 1), "tuned_schedule_us": round(us_tuned, 1),
                "schedule": "tuned" if use_tuned else "default",
                "tuned_tile_caps": hist, "tuning_s": round(tune_s, 2),
                "speedup_vs_plain_fp64_csr": round(plain / us, 2),
                "speedup_vs_plain_fp64_spc5": (round(k * res["plain_fp64_spc5_us_per_vector"] / us, 2)
                                               if "plain_fp64_spc5_us_per_vector" in res else None),
                "max_rel_l2_all_matrices": max(errs)}
            del Xs, Ys, Yh
        B.free()
        for M in Ms:
            M.free()
    return res


def ablation_extras(dev, A_lap):
    """The paper's ablations on this GPU.

    (a) x load and row reduction (Sections 3.1, 3.2; the paper's comparison
        table): the staged kernel with its single x load per block and the
        cross-lane multi-reduction, against the partial x load (each row its
        own x entries) and the per-row reduction, on the Laplacian 2048^2 and
        a 48^3 x 3 FEM matrix, FP64;
    (b) cost model (Section 4.3: a constant cost per block): forward times of
        five matrices x six shapes fitted by least squares to
        t = a*nblocks + b*nnz + c, with the GB/s and the nonzeros per block of
        every point."""
    import numpy as np
    import torch

    from paper_2307_14774_amd import spc5
    from paper_2307_14774_amd import workloads as W
    res = {}
    log("ablation: generating matrices")
    mats = {"laplacian2d_2048": A_lap, "fem3d_48x3": W.fem_3d(48, seed=1),
            "zipf_graph_2^18": W.zipf_graph(1 << 18, seed=2),
            "dense_2048": W.dense(2048, seed=3), "random10k": W.random_uniform(10_000, 10, seed=0)}

    def one(M, x, y, n=20):
        return time_region(lambda: M.spmv(x, y), n, 3)[1] * 1e3

    table = {}
    for name in ("laplacian2d_2048", "fem3d_48x3"):
        A = mats[name]
        x = torch.from_numpy(A.x).to(dev)
        y = torch.empty(A.nrows, dtype=torch.float64, device=dev)
        for rc in [(2, 4), (4, 4), (4, 8), (8, 8)]:
            log(f"ablation: variants {name} beta{rc}")
            M = spc5.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, *rc)
            row = {}
            for tag, v in (("single_x+multi_reduce", (False, False, False)),
                           ("partial_x", (True, False, False)),
                           ("per_row_reduce", (False, True, False)),
                           ("partial_x+per_row_reduce", (True, True, False)),
                           ("union_x+multi_reduce", (False, False, True))):
                M.set_variant(*v)
                us = one(M, x, y)
                row[tag] = {"launch_us": round(us, 2),
                            "gbs": round(M.info.spmv_bytes / us / 1e3, 1)}
            base = row["single_x+multi_reduce"]["launch_us"]
            for tag in row:
                row[tag]["speedup_of_default"] = round(row[tag]["launch_us"] / base, 3)
            table[f"{name} beta({rc[0]},{rc[1]})"] = row
            M.free()
    res["x_load_and_reduction"] = table

    pts = []
    for name, A in mats.items():
        x = torch.from_numpy(A.x).to(dev)
        y = torch.empty(A.nrows, dtype=torch.float64, device=dev)
        for rc in [(1, 8), (1, 16), (2, 4), (4, 4), (4, 8), (8, 8)]:
            log(f"ablation: model {name} beta{rc}")
            M = spc5.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, *rc)
            us = one(M, x, y)
            inf = M.info
            pts.append({"matrix": name, "beta": list(rc), "nblocks": inf.nblocks, "nnz": inf.nnz,
                        "nnz_per_block": round(inf.nnz / max(inf.nblocks, 1), 3),
                        "fill": round(inf.fill, 4), "launch_us": round(us, 2),
                        "gbs": round(inf.spmv_bytes / us / 1e3, 1),
                        "gflops": round(2.0 * inf.nnz / us / 1e3, 1)})
            M.free()
    X = np.array([[p["nblocks"], p["nnz"], 1.0] for p in pts], dtype=np.float64)
    t = np.array([p["launch_us"] for p in pts], dtype=np.float64)
    coef, *_ = np.linalg.lstsq(X, t, rcond=None)
    pred = X @ coef
    r2 = 1.0 - float(((t - pred) ** 2).sum() / ((t - t.mean()) ** 2).sum())
    res["cost_model"] = {"fit": "t_us = a*nblocks + b*nnz + c",
                         "a_ps_per_block": round(coef[0] * 1e6, 3),
                         "b_ps_per_nnz": round(coef[1] * 1e6, 3),
                         "c_us": round(coef[2], 2), "r2": round(r2, 4), "points": pts}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="fem", help="fem, laplacian, random or zipf")
    ap.add_argument("--dtype", default="float64",
                    help="value type of the timed product (float64; float32 for profiling)")
    ap.add_argument("--batch-ks", default="1,4,16", help="right-hand sides of the batch legs")
    ap.add_argument("--batch-dtypes", default="float64,float32")
    ap.add_argument("--no-extras", action="store_true", help="only the primary format")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-passes", type=int, default=5)
    ap.add_argument("--skip", default="", help="comma list of extras to skip: "
                    "kernels,formats,csr,flushed,other,backward,batch,ablation")
    ap.add_argument("--batch-mats", type=int, default=256)
    ap.add_argument("--calibration-copy", action="store_true",
                    help="before timing, negate a 1 GiB float64 buffer 3 times (a plain "
                         "copy of known size for counter calibration)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="host only: write the forward kernel's HBM traffic from two "
                         "rocprofv3 --pmc counter files and exit")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_write(args.traffic_from[0], args.traffic_from[1], args.workload, args.dtype)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: this library has no multi-GPU path, so "
                                   "--gpus must be 1"}))
        raise SystemExit(2)
    skip = set(filter(None, args.skip.split(",")))

    import numpy as np
    import torch

    import oracle
    from paper_2307_14774_amd import spc5

    dev = torch.device("cuda:0")
    log(f"generating workload {args.workload}")
    A, rc, tag = make_workload(args.workload, args.dtype)
    tdt = torch.float64 if args.dtype == "float64" else torch.float32
    x = torch.from_numpy(A.x).to(dev, tdt)
    yref = oracle.csr_spmv(A.rowptr, A.colidx, A.values, A.x)
    flops = 2.0 * A.nnz
    gate = 1e-14 if args.dtype == "float64" else 1e-6

    def measure(M, steps, warmup, nbytes, flush=None):
        """Mean launch time from one event pair around `steps` back-to-back
        launches; with a cache flush between launches, from an event pair
        around every launch (the flush stays outside the events)."""
        y = torch.empty(A.nrows, dtype=tdt, device=dev)
        if flush is None:
            wall, avg = time_region(lambda: M.spmv(x, y), steps, warmup)
            # per-launch event pairs on a few more launches: the fastest launch
            _, ms = time_launches(lambda: M.spmv(x, y), min(steps, 20), 0)
        else:
            wall, ms = time_launches(lambda: M.spmv(x, y), steps, warmup, flush)
            avg = float(np.mean(ms))
        err = oracle.rel_l2(y.cpu().double().numpy(), yref)
        return {"gflops": round(flops / (avg * 1e-3) / 1e9, 2),
                "launch_us": round(avg * 1e3, 2), "min_launch_us": round(min(ms) * 1e3, 2),
                "gbs": round(nbytes / (avg * 1e-3) / 1e9, 1),
                "frac_hbm": round(nbytes / (avg * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                "bytes": int(nbytes), "rel_l2": err}, wall, avg

    if args.calibration_copy:
        src = torch.ones(COPY_ELEMS, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    log(f"converting to beta{rc}")
    M = spc5.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, *rc, args.dtype)
    nbytes = M.info.spmv_bytes
    log(f"timing {args.steps} steps after {args.warmup} warmup")
    prim, wall, avg_ms = measure(M, args.steps, args.warmup, nbytes)
    if not prim["rel_l2"] <= gate:
        raise SystemExit(f"parity failure: rel L2 {prim['rel_l2']}")
    avg_s = avg_ms * 1e-3
    achieved = nbytes / avg_s / 1e9
    out = {
        "metric": METRIC,
        "value": round(flops * args.steps / wall / 1e9, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.dtype == "float64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{tag} beta({rc[0]},{rc[1]})", "nrows": A.nrows,
                   "ncols": A.ncols, "nnz": A.nnz, "r": rc[0], "c": rc[1],
                   "nblocks": M.info.nblocks, "panels_per_tile": M.info.panels_per_tile},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic_from_profiles(tag + f" beta({rc[0]},{rc[1]})"),
                     "kernel": f"{FWD_KERNEL} (forward, kernel choice: {M.kernel})",
                     "algorithmic_bytes_per_launch": int(nbytes),
                     "avg_launch_us": round(avg_s * 1e6, 2)},
        "parity_rel_l2": prim["rel_l2"],
    }
    extras = set() if args.no_extras else {"kernels", "formats", "csr", "flushed", "other",
                                           "backward", "batch", "ablation"} - skip
    if args.dtype != "float64" and extras & {"kernels", "formats", "csr", "flushed"}:
        raise SystemExit("a float32 timed product is for profiling: skip kernels, formats, csr "
                         "and flushed")
    if "kernels" in extras:
        prim["kernel"] = M.kernel
        kern = {M.kernel: prim}
        for other in ("staged", "sweep", "rows"):
            if other == M.kernel:
                continue
            log(f"timing the {other} kernel on beta{rc}")
            try:
                M.set_schedule(other)
            except spc5.Spc5Error as e:
                kern[other] = {"unsupported": str(e)}
                continue
            kern[other] = measure(M, 50, 5, nbytes)[0]
        M.set_schedule("auto")
        out["kernels"] = kern
    if "formats" in extras:
        formats = {f"beta({rc[0]},{rc[1]})": prim}
        for (r, c) in [(1, 8), (2, 4), (4, 4), (8, 8), (1, 16), (2, 8), (4, 8)]:
            if (r, c) == rc:
                continue
            log(f"timing beta({r},{c})")
            M2 = spc5.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, r, c)
            formats[f"beta({r},{c})"] = measure(M2, 100, 30, M2.info.spmv_bytes)[0]
            formats[f"beta({r},{c})"]["fill"] = round(M2.info.fill, 4)
            formats[f"beta({r},{c})"]["kernel"] = M2.kernel
            M2.free()
        # FP32 storage and accumulation (error against the FP64 oracle on the
        # original FP64 data): the timed shape and the paper's FP32
        # beta(r,VS) shapes (VS = 16)
        x32 = x.float()
        y32 = torch.empty(A.nrows, dtype=torch.float32, device=dev)
        for (r, c) in [rc, (4, 8), (1, 16), (2, 16), (4, 16), (8, 16)]:
            log(f"timing float32 beta({r},{c})")
            M3 = spc5.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, r, c, "float32")
            us32 = time_region(lambda: M3.spmv(x32, y32), 100, 30)[1] * 1e3
            formats[f"float32 beta({r},{c})"] = {
                "gflops": round(flops / us32 / 1e3, 2), "launch_us": round(us32, 2),
                "gbs": round(M3.info.spmv_bytes / us32 / 1e3, 1),
                "frac_hbm": round(M3.info.spmv_bytes / us32 / 1e3 / PEAK_HBM_GBS, 4),
                "bytes": int(M3.info.spmv_bytes), "fill": round(M3.info.fill, 4),
                "kernel": M3.kernel,
                "rel_l2_vs_fp64_oracle": oracle.rel_l2(y32.cpu().numpy(), yref),
                "speedup_vs_fp64_timed_shape": round(prim["launch_us"] / us32, 3)}
            M3.free()
        out["formats"] = formats
    if "csr" in extras:
        log("timing plain CSR")
        C = spc5.CsrMatrix(A.rowptr, A.colidx, A.values, A.ncols)
        out["csr"] = measure(C, 50, 5, C.spmv_bytes)[0]
        C.free()
        out["speedup_vs_csr"] = round(out["csr"]["launch_us"] / prim["launch_us"], 3)
        log("timing rocSPARSE CSR")
        rs = rocsparse_csr(dev, A, yref)
        if rs is not None:
            out["csr_rocsparse"] = rs
            out["speedup_vs_rocsparse_csr"] = round(rs["launch_us"] / prim["launch_us"], 3)
    if "flushed" in extras and args.workload == "laplacian":
        # cold-cache figure: a 1 GiB buffer is read between launches (outside
        # the timed events), so the matrix cannot stay in the 256 MB Infinity
        # Cache; reading (not writing) leaves clean lines behind, so the timed
        # launch does not pay for writing the flush buffer back
        scratch = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        sink = torch.empty((), dtype=torch.float64, device=dev)
        out["flushed"] = measure(M, 30, 3, nbytes,
                                 flush=lambda: torch.sum(scratch, dim=0, out=sink))[0]
        del scratch, sink
    M.free()
    A_lap = None
    if "other" in extras:
        if args.workload == "laplacian":
            out["fem"] = fem_extras(dev)
        else:
            from paper_2307_14774_amd import workloads as W
            log("generating the Laplacian workload")
            A_lap = W.laplacian_2d(2048, seed=0)
            out["laplacian"] = laplacian_extras(dev, A_lap)
    if "backward" in extras:
        out["backward"] = backward_extras(dev)
    if "batch" in extras:
        out["batch"] = batch_extras(dev, args.batch_mats,
                                    tuple(int(k) for k in args.batch_ks.split(",")),
                                    tuple(args.batch_dtypes.split(",")))
    if "ablation" in extras:
        if A_lap is None:
            from paper_2307_14774_amd import workloads as W
            A_lap = A if args.workload == "laplacian" else W.laplacian_2d(2048, seed=0)
        out["ablation"] = ablation_extras(dev, A_lap)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(A, args.cpu_passes)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
