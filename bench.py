#!/usr/bin/env python3
"""SPC5 SpMV benchmark on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload laplacian|fem|random]

A step is one forward product y = A x over the SPC5 beta(r,c) storage (all
hot-path steps: panel scheduling, metadata stream, mask expansion, value
stream, x gather, FMA, row reduction and y store) of one seeded synthetic
matrix already resident in HBM.  The default workload is the 5-point
Laplacian on a 2048 x 2048 grid in FP64 with beta(4,4).  One JSON line is
printed: GFLOP/s (2 flops per stored nonzero), the roofline of the forward
kernel (algorithmic bytes / measured launch time against 8 TB/s), the other
formats and the plain CSR kernel on the same GPU, and the CPU oracle timed on
this host as a baseline.
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
KERNEL_SOURCES = ["paper_2307_14774_amd/csrc/spmv.hip", "paper_2307_14774_amd/csrc/wave.h",
                  "paper_2307_14774_amd/csrc/tile.h"]


def kernel_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name):
    from paper_2307_14774_amd import workloads as W
    if name == "laplacian":
        return W.laplacian_2d(2048, seed=0), (4, 4), "laplacian2d_2048 fp64"
    if name == "fem":
        return W.fem_3d(96, seed=0), (4, 4), "fem3d_96x3 fp64"
    if name == "random":
        return W.random_uniform(10_000, 10, seed=0), (1, 8), "random10k fp64"
    raise SystemExit(f"unknown workload {name}")


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


def traffic_from_profiles(workload_tag):
    p = os.path.join(ROOT, "profiles", "traffic_spc5_fwd.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("kernel_sha") != kernel_sha() or d.get("workload") != workload_tag:
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(A, rc, budget_s=10.0):
    """The oracle as it stands (scalar Algorithm 1 over its own beta(r,c)
    conversion, FP64, one thread), on as many full passes as fit the budget."""
    import oracle
    S = oracle.csr_to_spc5(A.rowptr, A.colidx, A.values, A.ncols, *rc)
    t0 = time.perf_counter()
    n = 0
    while True:
        oracle.spc5_spmv(S, A.x)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": round(2.0 * A.nnz * n / dt / 1e9, 4), "unit": "GFLOP/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n} full passes of the scalar Algorithm 1 oracle over the whole matrix "
                      f"(beta{rc}, FP64, single thread, {dt:.1f} s)"}


def fem_extras(dev):
    """3D 3-dof 27-point FEM-like matrix (96^3 nodes, 210.5 M nonzeros): FP64
    and FP32 beta(4,4) and beta(1,8), plain CSR FP64; FP32 error against the
    FP64 oracle on the original FP64 data."""
    import numpy as np
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
            _, ms = time_launches(lambda: M.spmv(x, y), 30, 5)
            avg = float(np.mean(ms)) * 1e-3
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
    _, ms = time_launches(lambda: C.spmv(x, y), 30, 5)
    avg = float(np.mean(ms)) * 1e-3
    res["float64 csr"] = {"gflops": round(2.0 * A.nnz / avg / 1e9, 1),
                          "launch_us": round(avg * 1e6, 1),
                          "gbs": round(C.spmv_bytes / avg / 1e9, 1),
                          "frac_hbm": round(C.spmv_bytes / avg / 1e9 / PEAK_HBM_GBS, 4),
                          "rel_l2_vs_fp64_oracle": oracle.rel_l2(y.cpu().numpy(), yref)}
    C.free()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="laplacian")
    ap.add_argument("--no-extras", action="store_true", help="only the primary format")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        raise SystemExit(2)

    import numpy as np
    import torch

    import oracle
    from paper_2307_14774_amd import spc5

    dev = torch.device("cuda:0")
    log(f"generating workload {args.workload}")
    A, rc, tag = make_workload(args.workload)
    x = torch.from_numpy(A.x).to(dev)
    yref = oracle.csr_spmv(A.rowptr, A.colidx, A.values, A.x)
    flops = 2.0 * A.nnz

    def measure(M, steps, warmup, nbytes, flush=None):
        y = torch.empty(A.nrows, dtype=torch.float64, device=dev)
        wall, ms = time_launches(lambda: M.spmv(x, y), steps, warmup, flush)
        err = oracle.rel_l2(y.cpu().numpy(), yref)
        avg = float(np.mean(ms))
        return {"gflops": round(flops / (avg * 1e-3) / 1e9, 2),
                "launch_us": round(avg * 1e3, 2), "min_launch_us": round(min(ms) * 1e3, 2),
                "gbs": round(nbytes / (avg * 1e-3) / 1e9, 1),
                "frac_hbm": round(nbytes / (avg * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                "bytes": int(nbytes), "rel_l2": err}, wall, ms

    log(f"converting to beta{rc}")
    M = spc5.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, *rc)
    nbytes = M.info.spmv_bytes
    log(f"timing {args.steps} steps after {args.warmup} warmup")
    prim, wall, ms = measure(M, args.steps, args.warmup, nbytes)
    if not prim["rel_l2"] <= 1e-14:
        raise SystemExit(f"parity failure: rel L2 {prim['rel_l2']}")
    avg_s = float(np.mean(ms)) * 1e-3
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{tag} beta({rc[0]},{rc[1]})", "nrows": A.nrows,
                   "ncols": A.ncols, "nnz": A.nnz, "r": rc[0], "c": rc[1],
                   "nblocks": M.info.nblocks, "panels_per_tile": M.info.panels_per_tile},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic_from_profiles(tag + f" beta({rc[0]},{rc[1]})"),
                     "kernel": "k_spmv (spc5 forward)",
                     "algorithmic_bytes_per_launch": int(nbytes),
                     "avg_launch_us": round(avg_s * 1e6, 2)},
        "parity_rel_l2": prim["rel_l2"],
    }
    if not args.no_extras:
        other = "sweep" if M.kernel == "rows" else "rows"
        log(f"timing the {other} kernel on beta{rc}")
        M.set_schedule(other)
        alt = measure(M, 50, 5, nbytes)[0]
        M.set_schedule("auto")
        out["kernels"] = {M.kernel: prim, other: alt}
        prim["kernel"] = M.kernel
        formats = {f"beta({rc[0]},{rc[1]})": prim}
        for (r, c) in [(1, 8), (2, 4), (4, 4), (8, 8), (1, 16), (2, 8), (4, 8)]:
            if (r, c) == rc:
                continue
            log(f"timing beta({r},{c})")
            M2 = spc5.Spc5Matrix.from_csr(A.rowptr, A.colidx, A.values, A.ncols, r, c)
            formats[f"beta({r},{c})"] = measure(M2, 50, 5, M2.info.spmv_bytes)[0]
            formats[f"beta({r},{c})"]["fill"] = round(M2.info.fill, 4)
            formats[f"beta({r},{c})"]["kernel"] = M2.kernel
            M2.free()
        log("timing plain CSR")
        C = spc5.CsrMatrix(A.rowptr, A.colidx, A.values, A.ncols)
        formats["csr"] = measure(C, 50, 5, C.spmv_bytes)[0]
        C.free()
        # cold-cache figure: a 1 GiB buffer is rewritten between launches
        # (outside the timed events), so the matrix cannot stay in the 256 MB
        # Infinity Cache
        scratch = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        flushed = measure(M, 30, 3, nbytes, flush=lambda: scratch.fill_(1.0))[0]
        del scratch
        out["formats"] = formats
        out["flushed"] = flushed

        out["speedup_vs_csr"] = round(formats["csr"]["launch_us"] / prim["launch_us"], 3)
    if not args.no_extras and args.workload == "laplacian":
        out["fem"] = fem_extras(dev)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(A, rc, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
