#!/usr/bin/env python3
"""Benchmark of the CRS / JDS SpMV hot path on one MI355X.

Default run (the headline line): the power-law workload (n = 2,000,000 rows,
row lengths ~ L^-1.6929 on [1, 2000], mean 15 entries, half band / half uniform
columns, N(0,1) values, x ~ U[-1, 1]).  One step = the six products
  CRS, JDS, blocked JDS  x  {FP64 values, FP32 values with FP64 vectors}
on that matrix, inputs resident in HBM.  Prints ONE JSON line with GFLOP/s
(2 flops per stored entry), the per-kernel split, the roofline of the
dominant kernel (algorithmic bytes / its average launch time, against 8 TB/s)
and the serial CPU oracle timed on the host as a reported baseline.

--suite adds one JSON line per other workload (Laplacian, symmetric diagonals
in FP64/FP32/BF16, multi-vector, many matrices, Chebyshev backward).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--suite", action="store_true", help="also measure the other workloads")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", default="", help="comma list of kernels for profiling runs")
    ap.add_argument("--probe", choices=["copy", "triad"], default=None,
                    help="run only the bandwidth probe on 1 GiB arrays (counter calibration)")
    return ap.parse_args()


def run_probe(kind):
    import torch
    import paper_0910_4836_amd as sp
    dev = torch.device("cuda", 0)
    n = 1 << 27
    a = torch.empty(n, dtype=torch.float64, device=dev)
    b = torch.ones(n, dtype=torch.float64, device=dev)
    c = torch.ones(n, dtype=torch.float64, device=dev)
    for _ in range(10):
        if kind == "copy":
            sp.spmv_stream_copy(a, b)
        else:
            sp.spmv_stream_triad(a, b, c, 0.5)
    torch.cuda.synchronize()
    print(json.dumps({"probe": kind, "elements": n, "launches": 10,
                      "bytes_per_launch": (16 if kind == "copy" else 24) * n}))


# --------------------------------------------------------------------------- byte models


def bytes_crs(nnz, n_rows, n_cols, sv, sx, k=1, beta=False):
    return nnz * (sv + 4) + 4 * (n_rows + 1) + k * sx * n_cols + k * sx * n_rows * (2 if beta else 1)


def bytes_jds(nnz, n, n_cols, ndiag, sv, sx, k=1):
    return nnz * (sv + 4) + 4 * (ndiag + 1) + 4 * n + k * sx * (n_cols + n)


def bytes_blocked(nnz, n, n_cols, n_slices, sv, sx):
    return nnz * (sv + 4) + 12 * n_slices + 4 * n + sx * (n_cols + n)


# --------------------------------------------------------------------------- timing


class Timer:
    """HIP events (torch.cuda.Event) on the stream the kernels are launched on."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = {}

    def run(self, name, fn):
        t = self.torch
        a = t.cuda.Event(enable_timing=True)
        b = t.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        self.pairs.setdefault(name, []).append((a, b))

    def avg_ms(self, name):
        return float(np.mean([a.elapsed_time(b) for a, b in self.pairs[name]]))


def time_loop(torch, kernels, steps, warmup):
    """kernels: list of (name, fn).  Returns (ms_per_step, {name: avg ms})."""
    for _ in range(warmup):
        for _, fn in kernels:
            fn()
    torch.cuda.synchronize()
    timer = Timer(torch)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        for name, fn in kernels:
            timer.run(name, fn)
    end.record()
    torch.cuda.synchronize()
    total = start.elapsed_time(end)
    return total / steps, {name: timer.avg_ms(name) for name, _ in kernels}


def kernel_source_sha():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_0910_4836_amd", "csrc"))):
        h.update(open(os.path.join(ROOT, "paper_0910_4836_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None
    when they are missing or were taken on different kernel sources."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    ent = rec.get("entries", {}).get(f"{workload}:{kernel}")
    if not ent or ent.get("source_sha") != kernel_source_sha():
        return None
    return ent.get("bytes_per_launch")


# --------------------------------------------------------------------------- workloads


def load_powerlaw(torch, sp, dev):
    import synth
    t0 = time.time()
    r, c, v, n, _ = synth.powerlaw()
    x = synth.uniform_vector(n, synth.rng_for(2, 1))
    gen_s = time.time() - t0
    rd = torch.from_numpy(r).to(dev)
    cd = torch.from_numpy(c).to(dev)
    vd = torch.from_numpy(v).to(dev)
    torch.cuda.synchronize()
    setup = {}

    def timed(name, fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        setup[name] = round((time.perf_counter() - t) * 1e3, 2)
        return out

    A = timed("csr_from_coo_ms", lambda: sp.csr_from_coo(n, n, rd, cd, vd))
    del rd, cd, vd
    timed("crs_plan_ms", lambda: sp.spmv_crs_plan(A))
    J = timed("jds_from_csr_ms", lambda: sp.jds_from_csr(A))
    B = timed("jds_blocked_from_jds_ms", lambda: sp.jds_blocked_from_jds(J, 64))
    A32 = A.with_values(sp.spmv_convert_values(A.val, torch.float32))
    J32 = J.with_values(sp.spmv_convert_values(J.jd_val, torch.float32))
    B32 = B.with_values(sp.spmv_convert_values(B.bl_val, torch.float32))
    xd = torch.from_numpy(x).to(dev)
    host = (r, c, v, n, x)
    return dict(A=A, J=J, B=B, A32=A32, J32=J32, B32=B32, x=xd, n=n, nnz=A.nnz, setup=setup, gen_s=gen_s,
                host=host)


def powerlaw_kernels(sp, W, torch):
    n, nnz = W["n"], W["nnz"]
    y = torch.empty(n, dtype=torch.float64, device=W["x"].device)
    x = W["x"]
    J, B = W["J"], W["B"]
    ks = [
        ("crs_f64", lambda: sp.spmv_crs(W["A"], x, y)),
        ("jds_f64", lambda: sp.spmv_jds(J, x, y)),
        ("blocked_f64", lambda: sp.spmv_jds_blocked(B, x, y)),
        ("crs_f32val", lambda: sp.spmv_crs(W["A32"], x, y)),
        ("jds_f32val", lambda: sp.spmv_jds(W["J32"], x, y)),
        ("blocked_f32val", lambda: sp.spmv_jds_blocked(W["B32"], x, y)),
    ]
    bmin = {
        "crs_f64": bytes_crs(nnz, n, n, 8, 8),
        "jds_f64": bytes_jds(nnz, n, n, J.ndiag, 8, 8),
        "blocked_f64": bytes_blocked(nnz, n, n, B.n_slices, 8, 8),
        "crs_f32val": bytes_crs(nnz, n, n, 4, 8),
        "jds_f32val": bytes_jds(nnz, n, n, J.ndiag, 4, 8),
        "blocked_f32val": bytes_blocked(nnz, n, n, B.n_slices, 4, 8),
    }
    return ks, bmin


def cpu_baseline(W, budget_s=20.0):
    """The serial oracle (plain C, one core) on the same step, repeated for about
    budget_s seconds of CPU time; returns GFLOP/s."""
    import oracle
    r, c, v, n, x = W["host"]
    A = oracle.csr_from_coo(n, n, r, c, v)
    J = oracle.jds_from_csr(A)
    Bk = oracle.blocked_from_jds(J, 64)
    vq = oracle.round_f32(A.val).astype(np.float64)
    Aq = oracle.CSR(n, n, A.row_ptr, A.col, vq)
    Jq = oracle.JDS(J.n, J.perm, J.iperm, J.jd_ptr, J.jd_col, oracle.round_f32(J.jd_val).astype(np.float64), False)
    Bq = oracle.Blocked(Bk.n, Bk.perm, Bk.C, Bk.slice_ptr, Bk.slice_nd, Bk.bl_col,
                        oracle.round_f32(Bk.bl_val).astype(np.float64), False)
    step = [lambda: oracle.spmv_crs(A, x), lambda: oracle.spmv_jds(J, x), lambda: oracle.spmv_blocked(Bk, x),
            lambda: oracle.spmv_crs(Aq, x), lambda: oracle.spmv_jds(Jq, x), lambda: oracle.spmv_blocked(Bq, x)]
    reps = 0
    t0 = time.process_time()
    w0 = time.perf_counter()
    while True:
        for f in step:
            f()
        reps += 1
        if time.process_time() - t0 >= budget_s or reps >= 50:
            break
    cpu_s = time.process_time() - t0
    wall = time.perf_counter() - w0
    flops = 6 * 2.0 * A.nnz * reps
    return {"value": round(flops / wall / 1e9, 4), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} full steps (6 products each) of the n=2,000,000 power-law matrix, "
                      f"{cpu_s:.1f} s CPU, serial FP64 C oracle (-O2, no FMA), one thread",
            "host_cpu": platform.processor() or platform.machine(), "host_logical_cpus": os.cpu_count()}


def roofline_for(name, bytes_per_launch, ms, workload):
    achieved = bytes_per_launch / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(name, workload),
            "algorithmic_bytes_per_launch": int(bytes_per_launch), "avg_launch_ms": round(ms, 5)}


def attainable_bw(torch, sp, dev):
    n = 1 << 27                                  # 1 GiB per array
    a = torch.empty(n, dtype=torch.float64, device=dev)
    b = torch.ones(n, dtype=torch.float64, device=dev)
    c = torch.ones(n, dtype=torch.float64, device=dev)
    out = {}
    for name, fn, nbytes in (("triad", lambda: sp.spmv_stream_triad(a, b, c, 0.5), 24 * n),
                             ("copy", lambda: sp.spmv_stream_copy(a, b), 16 * n)):
        ms, _ = time_loop(torch, [(name, fn)], 20, 3)
        out[name + "_GBs"] = round(nbytes / (ms * 1e-3) / 1e9, 1)
    del a, b, c
    return out


# --------------------------------------------------------------------------- suite


def suite_lines(torch, sp, dev, W, steps, warmup):
    import synth
    lines = []
    x = W["x"]
    n = W["n"]
    # multi-vector forms on the power-law matrix
    for k in (8, 32):
        for dt, sv in ((torch.float64, 8), (torch.float32, 4)):
            A = W["A"] if dt == torch.float64 else W["A32"]
            X = sp.colmajor(n, k, dt, dev)
            X.copy_(torch.rand(n, k, dtype=dt, device=dev) * 2 - 1)
            Y = sp.colmajor(n, k, dt, dev)
            ms, per = time_loop(torch, [("spmm_crs", lambda: sp.spmm_crs(A, X, Y))], max(5, steps // 10), 2)
            bm = bytes_crs(W["nnz"], n, n, sv, sv, k)
            lines.append({"workload": f"powerlaw x {k} vectors (column-major)", "kernel": f"spmm_crs_{str(dt)[6:]}",
                          "gflops": round(2 * W["nnz"] * k / (ms * 1e-3) / 1e9, 1),
                          "roofline": roofline_for("spmm_crs", bm, per["spmm_crs"], "spmm")})
    return lines


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU row partition is "
              "a design in DESIGN.md, not a measured path", file=sys.stderr)
        sys.exit(2)
    if args.probe:
        run_probe(args.probe)
        return
    import torch
    import paper_0910_4836_amd as sp
    sp.load_library()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    W = load_powerlaw(torch, sp, dev)
    ks, bmin = powerlaw_kernels(sp, W, torch)
    if args.only:
        keep = set(args.only.split(","))
        ks = [k for k in ks if k[0] in keep]
    ms_step, per = time_loop(torch, ks, args.steps, args.warmup)
    flops_step = 2.0 * W["nnz"] * len(ks)
    value = flops_step / (ms_step * 1e-3) / 1e9
    dom = max(per, key=per.get)
    kernels = {}
    for name, _ in ks:
        kernels[name] = {"avg_ms": round(per[name], 5),
                         "gflops": round(2.0 * W["nnz"] / (per[name] * 1e-3) / 1e9, 1),
                         "algorithmic_GBs": round(bmin[name] / (per[name] * 1e-3) / 1e9, 1),
                         "frac_of_8TBs": round(bmin[name] / (per[name] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    out = {
        "metric": "SpMV GFLOP/s + % of HBM code-balance roofline, CRS vs JDS, FP64 vs mixed",
        "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"power-law n={W['n']} nnz={W['nnz']} (mean 15/row, max 2000; CRS, JDS, "
                               f"blocked JDS C=64; FP64 values and FP32 values with FP64 vectors)",
                   "n": W["n"], "nnz": W["nnz"], "ndiag": W["J"].ndiag, "products_per_step": len(ks)},
        "kernels": kernels,
        "roofline": roofline_for(dom, bmin[dom], per[dom], "powerlaw"),
        "setup_ms": W["setup"],
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(W)
    else:
        out["cpu_baseline"] = None
    out["attainable_hbm"] = attainable_bw(torch, sp, dev)
    print(json.dumps(out), flush=True)
    if args.suite:
        for line in suite_lines(torch, sp, dev, W, args.steps, args.warmup):
            print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
