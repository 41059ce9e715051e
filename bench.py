#!/usr/bin/env python3
"""Benchmark of the CRS / JDS SpMV hot path on one MI355X.

Default run (the headline line): the power-law workload (n = 2,000,000 rows,
row lengths ~ L^-1.6929 on [1, 2000], mean 15 entries, half band / half uniform
columns, N(0,1) values, x ~ U[-1, 1]).  One step = the three FP64 products
CRS, JDS and blocked JDS on that matrix, inputs resident in HBM; the JDS
unroll / split threshold and the blocked slice height / rows per wavefront /
unroll come from the library's autotuner, run on the device during setup.
Prints ONE JSON line with GFLOP/s (2 flops per stored entry), the per-kernel
times, the roofline of the dominant kernel (algorithmic bytes / its average
launch time, against 8 TB/s) and the serial CPU oracle timed on the host as a
reported baseline.  Beside the step (not in it) the same line reports the
FP32-value products, the column-split forms of all three and the row-split
forms of the two JDS products.

--suite adds one JSON line per other workload (Laplacian, symmetric diagonals
in FP64/FP32/BF16, multi-vector, many matrices, Chebyshev backward).
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import platform
import sys
import tempfile
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
    ap.add_argument("--suite-lines", default="", help="comma list: run only these suite lines")
    ap.add_argument("--no-graph", action="store_true",
                    help="time the step from the eager loop instead of HIP graph replays (profiler runs)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", default="", help="comma list of kernels for profiling runs")
    ap.add_argument("--probe", choices=["copy", "triad", "strides"], default=None,
                    help="copy / triad: only the bandwidth probe on 1 GiB arrays (counter calibration); "
                         "strides: the access-pattern microbenchmarks of the inner loop")
    ap.add_argument("--no-c3", action="store_true",
                    help="leave out the mixed-precision block on the symmetric-diagonals matrix")
    ap.add_argument("--no-hamiltonian", action="store_true",
                    help="leave out the DIA-hybrid block on the Hamiltonian-shaped matrix")
    ap.add_argument("--workload", choices=["powerlaw", "symdiag", "hamiltonian"], default="powerlaw",
                    help="symdiag / hamiltonian: time only that matrix's products named by --only (profiling runs)")
    ap.add_argument("--tune-cache", default="",
                    help="autotuner cache file (default: a fresh one, i.e. tune on this device now); "
                         "profiling runs share one so they time the same kernels")
    return ap.parse_args()


def run_probe(kind):
    import torch
    import paper_0910_4836_amd as sp
    dev = torch.device("cuda", 0)
    if kind == "strides":
        print(json.dumps(run_strides(torch, sp, dev)))
        return
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


STRIDE_SWEEP = (1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 256, 512, 530, 1024, 2048, 4096, 8192)
WRAP_SWEEP = (128, 512, 2048, 4096, 8192, 16384, 32768, 65536, 131072, 262144)
GAUSS_MEANS = (1, 2, 4, 8, 16, 32, 64, 128)
GAUSS_SDS = (0, 1, 2, 4, 8, 16, 32, 64, 128, 256)


def run_strides(torch, sp, dev, reps=5):
    """The basic operations of the inner loop (Section 4.1, Table 1) on this
    GPU: s += B(j) (ADD) or s += A(i)*B(j) (SCP) over i < n with j = i (PD),
    k*i (CS), ind(i) = k*i (IS), ind(i) with geometric strides of mean k (IR,
    the keep-with-probability-1/k rule) or Gaussian strides of given mean
    and standard deviation (the stride plane, backward jumps included).

    B is 2^31 doubles (16 GiB: every int32 index fits) and every launch is
    timed cold, right after a 512 MiB streaming copy, so nothing starts in
    the L2s or the 256 MB MALL, as the paper sizes its arrays beyond every
    cache.  Rates are updates per second; "cu_cycles" is the chip's CU-cycles
    per update (256 CUs at 2.4 GHz), the analogue of the paper's cycles per
    update.  A and B hold ones, so every launch must sum to exactly n."""
    import synth
    NB = 1 << 31
    NMAX = 1 << 25
    b = torch.ones(NB, dtype=torch.float64, device=dev)
    a = torch.ones(NMAX, dtype=torch.float64, device=dev)
    part = torch.zeros(1 << 16, dtype=torch.float64, device=dev)
    fa = torch.empty(1 << 26, dtype=torch.float64, device=dev)
    fb = torch.zeros(1 << 26, dtype=torch.float64, device=dev)
    cycles = 256 * 2.4e9
    rng = synth.rng_for(6, 1)

    def cold(fn, n):
        fn()
        pairs = []
        for r in range(reps):
            if r == reps - 1:
                part.zero_()
            sp.spmv_stream_copy(fa, fb)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            pairs.append((e0, e1))
        torch.cuda.synchronize()
        got = part.sum().item()
        if got != n:
            raise RuntimeError(f"stride probe summed {got}, expected {n}")
        return float(np.median([e0.elapsed_time(e1) for e0, e1 in pairs]))

    def lines(j):
        """Distinct 128-byte lines of B per update, counted over the 64
        consecutive updates that one wavefront load instruction issues
        (first 2^20 updates)."""
        j = np.asarray(j[: (min(len(j), 1 << 20) // 64) * 64], dtype=np.int64).reshape(-1, 64) // 16
        j = np.sort(j, axis=1)
        return float((1 + (np.diff(j, axis=1) != 0).sum(axis=1)).mean() / 64)

    def entry(name, n, ms, lpu, **kw):
        rate = n / (ms * 1e-3)
        e = {"case": name, "n": n, "us": round(ms * 1e3, 2), "Gupdates_s": round(rate / 1e9, 2),
             "cu_cycles": round(cycles / rate, 1), "lines_per_update": round(lpu, 4)}
        e.update(kw)
        print(json.dumps(e), file=sys.stderr, flush=True)
        return e

    def indirect(kind, k, n, sd=0.0):
        ind = synth.index_stream(kind, n, k, rng, sd)
        ind = ind[ind < NB]
        return torch.from_numpy(ind.astype(np.int32)).to(dev), len(ind), int(ind.max()), lines(ind)

    out = {"probe": "strides", "B_elements": NB, "reps": reps, "timing": "cold, median", "ops": [],
           "sweep": [], "wrap": [], "gauss": []}
    # launch and event overhead: one update
    out["launch_us"] = round(cold(lambda: sp.spmv_stride_probe(1, b, part), 1) * 1e3, 2)
    # Table 1's eight operations at the strides of the paper's Fig. 2
    for k in (1, 8, 530):
        n = min(NMAX, (NB - 1) // k + 1)
        for scp in (False, True):
            op = "SCP" if scp else "ADD"
            aa = a if scp else None
            lk = lines(np.arange(1 << 20) * k)
            ms = cold(lambda: sp.spmv_stride_probe(n, b, part, a=aa, k=k), n)
            out["ops"].append(entry(("PD" if k == 1 else "CS") + op, n, ms, lk, k=k))
            ind = (torch.arange(n, device=dev, dtype=torch.int64) * k).to(torch.int32)
            ms = cold(lambda: sp.spmv_stride_probe(n, b, part, a=aa, ind=ind, ind_max=k * (n - 1)), n)
            out["ops"].append(entry("IS" + op, n, ms, lk, k=k))
            ir, m, mx, li = indirect("IR", k, min(NMAX, int((NB - 1) / (k * 1.1)) + 1))
            ms = cold(lambda: sp.spmv_stride_probe(m, b, part, a=aa, ind=ir, ind_max=mx), m)
            out["ops"].append(entry("IR" + op, m, ms, li, k=k))
            del ind, ir
    # SCP against the stride: constant (CS, IS) and random (IR)
    for k in STRIDE_SWEEP:
        n = min(NMAX, (NB - 1) // k + 1)
        lk = lines(np.arange(1 << 20) * k)
        ms = cold(lambda: sp.spmv_stride_probe(n, b, part, a=a, k=k), n)
        out["sweep"].append(entry("CSSCP", n, ms, lk, k=k))
        ind = (torch.arange(n, device=dev, dtype=torch.int64) * k).to(torch.int32)
        ms = cold(lambda: sp.spmv_stride_probe(n, b, part, a=a, ind=ind, ind_max=k * (n - 1)), n)
        out["sweep"].append(entry("ISSCP", n, ms, lk, k=k))
        ir, m, mx, li = indirect("IR", k, min(NMAX, int((NB - 1) / (k * 1.1)) + 1))
        ms = cold(lambda: sp.spmv_stride_probe(m, b, part, a=a, ind=ir, ind_max=mx), m)
        out["sweep"].append(entry("IRSCP", m, ms, li, k=k))
        del ind, ir
    # ISSCP at strides up to 2 MiB with 2^24 updates each: the stream wraps
    # around B, each pass shifted by one 128-byte line, so no line is read
    # twice and every pass walks all 16 GiB again (the address translation
    # footprint of the stride, not of a short launch)
    for k in WRAP_SWEEP:
        n = 1 << 24
        t = torch.arange(n, device=dev, dtype=torch.int64) * k
        span = NB - 16 * (int(t[-1].item()) // NB + 2)
        ind = (t % span + 16 * (t // span)).to(torch.int32)
        mx = int(ind.max().item())
        del t
        ms = cold(lambda: sp.spmv_stride_probe(n, b, part, a=a, ind=ind, ind_max=mx), n)
        out["wrap"].append(entry("ISSCP_wrap", n, ms, 1.0, k=k))
        del ind
    # IRSCP with Gaussian strides: mean and standard deviation set independently
    for mean in GAUSS_MEANS:
        for sd in GAUSS_SDS:
            n = min(NMAX // 2, int((NB - 1) / (mean * 1.2)))
            g, m, mx, lg = indirect("GAUSS", mean, n, float(sd))
            ms = cold(lambda: sp.spmv_stride_probe(m, b, part, a=a, ind=g, ind_max=mx), m)
            out["gauss"].append(entry("IRSCP_gauss", m, ms, lg, mean=mean, sd=sd))
            del g
    del a, b, fa, fb, part
    return out


# --------------------------------------------------------------------------- byte models


def bytes_crs(nnz, n_rows, n_cols, sv, sx, k=1, beta=False):
    return nnz * (sv + 4) + 4 * (n_rows + 1) + k * sx * n_cols + k * sx * n_rows * (2 if beta else 1)


def bytes_jds(nnz, n, n_cols, ndiag, sv, sx, k=1):
    return nnz * (sv + 4) + 4 * (ndiag + 1) + 4 * n + k * sx * (n_cols + n)


def bytes_blocked(nnz, n, n_cols, n_slices, sv, sx, k=1):
    return nnz * (sv + 4) + 12 * n_slices + 4 * n + k * sx * (n_cols + n)


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

    def median_ms(self, name):
        return float(np.median([a.elapsed_time(b) for a, b in self.pairs[name]]))


def time_loop(torch, kernels, steps, warmup, medians=None):
    """kernels: list of (name, fn).  Returns (ms_per_step, {name: avg ms});
    `medians`, if given, receives {name: median ms}.

    Python's cyclic garbage collector is paused over the timed steps: one of
    its passes can hold the launching thread for tens of milliseconds, which
    would show up as idle GPU time inside whichever kernel's event pair it
    hits."""
    for _ in range(warmup):
        for _, fn in kernels:
            fn()
    torch.cuda.synchronize()
    timer = Timer(torch)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    gc.collect()
    gc.disable()
    try:
        torch.cuda.synchronize()
        start.record()
        for _ in range(steps):
            for name, fn in kernels:
                timer.run(name, fn)
        end.record()
        torch.cuda.synchronize()
    finally:
        gc.enable()
    total = start.elapsed_time(end)
    if medians is not None:
        medians.update({name: timer.median_ms(name) for name, _ in kernels})
    return total / steps, {name: timer.avg_ms(name) for name, _ in kernels}


def graph_step_ms(torch, sp, kernels, steps, warmup):
    """ms per step for `steps` replays of one HIP graph that holds one call of
    each kernel (after `warmup` replays), between two synchronised events."""
    g = sp.Graph()
    with g.capture():
        for _, fn in kernels:
            fn()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    gc.collect()
    gc.disable()
    try:
        e0.record()
        for _ in range(steps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
    finally:
        gc.enable()
    return e0.elapsed_time(e1) / steps


def cold_times(torch, sp, dev, kernels, reps=20):
    """Each product timed alone right after a streaming copy of 512 MiB into
    another 512 MiB buffer (twice the 256 MB MALL, far beyond the L2s), so it
    starts with none of its arrays in cache; median over `reps` launches."""
    n = 1 << 26
    a = torch.empty(n, dtype=torch.float64, device=dev)
    b = torch.zeros(n, dtype=torch.float64, device=dev)
    out = {}
    gc.collect()
    gc.disable()
    try:
        for name, fn in kernels:
            fn()
            pairs = []
            for _ in range(reps):
                sp.spmv_stream_copy(a, b)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                pairs.append((e0, e1))
            torch.cuda.synchronize()
            out[name] = float(np.median([e0.elapsed_time(e1) for e0, e1 in pairs]))
    finally:
        gc.enable()
    del a, b
    return out


KERNEL_SOURCES = {"crs": ("common.hpp", "crs.hip"), "jds": ("common.hpp", "jds.hip"),
                  "blocked": ("common.hpp", "jds.hip"), "dia": ("common.hpp", "dia.hip")}


def kernel_sources(kernel):
    """Sources a product's kernels are compiled from (the split forms add the
    combine kernel in util.hip; the probes live in util.hip)."""
    if kernel.startswith("gather_"):
        return ("common.hpp", "util.hip")
    fam = kernel.split("_")[0]
    files = KERNEL_SOURCES[fam]
    return files + ("util.hip",) if "_split" in kernel else files


def kernel_source_sha(files):
    h = hashlib.sha256()
    for f in sorted(files):
        h.update(f.encode())
        h.update(open(os.path.join(ROOT, "paper_0910_4836_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """L2-fill bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated on the
    copy probe) from the committed rocprofv3 counter runs, or None when they
    are missing or were taken on different kernel sources."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    ent = rec.get("entries", {}).get(f"{workload}:{kernel}")
    if not ent or ent.get("source_sha") != kernel_source_sha(kernel_sources(kernel)):
        return None
    return ent.get("bytes_per_launch")


# --------------------------------------------------------------------------- workloads


def load_powerlaw(torch, sp, dev, tune_cache=""):
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
    xd = torch.from_numpy(x).to(dev)
    # launch parameters from the library's autotuner, timed on this device
    # (fresh cache, so nothing is carried over from another machine)
    from paper_0910_4836_amd import autotune
    tuner = autotune.Autotuner(cache_path=tune_cache or os.path.join(tempfile.mkdtemp(), "autotune.json"))
    crs_bn = timed("autotune_crs_ms", lambda: autotune.tune_crs(tuner, A, xd, J.ndiag))
    jds_u, jds_mi, jds_w = timed("autotune_jds_ms", lambda: tuner.tune_jds(J, xd))
    bC, bR, bU, bW = timed("autotune_blocked_ms", lambda: tuner.tune_blocked(J, xd))
    B = timed("jds_blocked_from_jds_ms", lambda: sp.jds_blocked_from_jds(J, bC))
    # class plan or XCD-local tile plan, whichever the autotuner times faster
    jds_tiled = timed("autotune_jds_launch_ms", lambda: tuner.tune_jds_launch(J, xd, jds_u, jds_mi, jds_w))
    blk_tiled = timed("autotune_blocked_launch_ms", lambda: tuner.tune_blocked_launch(B, xd, bR, bU, bW))
    A32 = A.with_values(sp.spmv_convert_values(A.val, torch.float32))
    J32 = J.with_values(sp.spmv_convert_values(J.jd_val, torch.float32))
    B32 = B.with_values(sp.spmv_convert_values(B.bl_val, torch.float32))
    S = timed("split_columns_ms", lambda: sp.Split(A))
    timed("split_jds_parts_ms", lambda: S.jds_parts())
    timed("split_blocked_parts_ms", lambda: S.blocked_parts(64))
    RS = timed("split_rows_ms", lambda: sp.RowSplit(A))
    timed("row_split_jds_parts_ms", lambda: RS.jds_parts())
    timed("row_split_blocked_parts_ms", lambda: RS.blocked_parts(bC))
    wS, wC, wU, wW = timed("autotune_windowed_ms", lambda: tuner.tune_windowed(A, xd, J.ndiag))
    BW = timed("jds_blocked_windowed_from_csr_ms", lambda: sp.jds_blocked_windowed_from_csr(A, wC, wS))
    timed("windowed_tile_plan_ms", lambda: sp.spmv_jds_blocked_tiles(BW, 32, 0, wW))
    host = (r, c, v, n, x)
    tune = {"crs_block_nnz": crs_bn, "crs_staged": A.staged, "jds_unroll": jds_u, "jds_max_iters": jds_mi, "jds_wg_waves": jds_w,
            "jds_tiled": jds_tiled, "blocked_C": bC, "blocked_rows_per_wave": bR, "blocked_unroll": bU,
            "blocked_wg_waves": bW, "blocked_tiled": blk_tiled, "windowed_sigma": wS, "windowed_C": wC,
            "windowed_unroll": wU, "windowed_wg_waves": wW}
    return dict(A=A, J=J, B=B, A32=A32, J32=J32, B32=B32, S=S, RS=RS, BW=BW, x=xd, n=n, nnz=A.nnz, setup=setup,
                gen_s=gen_s, host=host, tune=tune)


def jds_launch(sp, T, x, y):
    """The JDS product with the tuned launch shape and plan (class plan, or
    the XCD-local tile plan when the autotuner timed it faster)."""
    ju, jm, jw = T["jds_unroll"], T["jds_max_iters"], T["jds_wg_waves"]
    if T.get("jds_tiled"):
        return lambda J: lambda: sp.spmv_jds_tiled(J, x, y, unroll=ju, max_iters=jm, wg_waves=jw)
    return lambda J: lambda: sp.spmv_jds(J, x, y, unroll=ju, max_iters=jm, wg_waves=jw)


def blocked_launch(sp, T, x, y):
    """The blocked-JDS product with the tuned launch shape and plan."""
    bR, bU, bW = T["blocked_rows_per_wave"], T["blocked_unroll"], T["blocked_wg_waves"]
    if T.get("blocked_tiled"):
        return lambda B: lambda: sp.spmv_jds_blocked_tiled(B, x, y, unroll=bU, rows_per_wave=bR, wg_waves=bW)
    return lambda B: lambda: sp.spmv_jds_blocked(B, x, y, rows_per_wave=bR, unroll=bU, wg_waves=bW)


def powerlaw_kernels(sp, W, torch):
    n, nnz = W["n"], W["nnz"]
    y = torch.empty(n, dtype=torch.float64, device=W["x"].device)
    x = W["x"]
    J, B = W["J"], W["B"]
    T = W["tune"]
    ju, jm, jw = T["jds_unroll"], T["jds_max_iters"], T["jds_wg_waves"]
    bR, bU, bW = T["blocked_rows_per_wave"], T["blocked_unroll"], T["blocked_wg_waves"]
    jl, bl = jds_launch(sp, T, x, y), blocked_launch(sp, T, x, y)
    ks = [
        ("crs_f64", lambda: sp.spmv_crs(W["A"], x, y)),
        ("jds_f64", jl(J)),
        ("blocked_f64", bl(B)),
        ("crs_f32val", lambda: sp.spmv_crs(W["A32"], x, y)),
        ("jds_f32val", jl(W["J32"])),
        ("blocked_f32val", bl(W["B32"])),
    ]
    S = W["S"]
    S32 = W.setdefault("S32", S.with_values(sp.spmv_convert_values(S.val, torch.float32)))
    ks += [
        ("crs_split_f64", lambda: sp.spmv_crs_split(S, x, y)),
        ("jds_split_f64", lambda: sp.spmv_jds_split(S, x, y)),
        ("blocked_split_f64", lambda: sp.spmv_jds_blocked_split(S, x, y)),
        ("crs_split_f32val", lambda: sp.spmv_crs_split(S32, x, y)),
        ("jds_split_f32val", lambda: sp.spmv_jds_split(S32, x, y)),
        ("blocked_split_f32val", lambda: sp.spmv_jds_blocked_split(S32, x, y)),
    ]
    RS, bC = W["RS"], T["blocked_C"]
    RS32 = W.setdefault("RS32", RS.with_values(torch.float32))
    ks += [
        ("jds_rowsplit_f64", lambda: sp.spmv_jds_row_split(RS, x, y, unroll=ju, max_iters=jm, wg_waves=jw)),
        ("blocked_rowsplit_f64", lambda: sp.spmv_jds_blocked_row_split(RS, x, y, C_=bC, rows_per_wave=bR,
                                                                         unroll=bU, wg_waves=bW)),
        ("jds_rowsplit_f32val", lambda: sp.spmv_jds_row_split(RS32, x, y, unroll=ju, max_iters=jm, wg_waves=jw)),
        ("blocked_rowsplit_f32val", lambda: sp.spmv_jds_blocked_row_split(RS32, x, y, C_=bC, rows_per_wave=bR,
                                                                            unroll=bU, wg_waves=bW)),
    ]
    BW = W["BW"]
    wU, wW = T["windowed_unroll"], T["windowed_wg_waves"]
    ks += [("blocked_windowed_f64", lambda: sp.spmv_jds_blocked_tiled(BW, x, y, unroll=wU, max_iters=32,
                                                                       wg_waves=wW))]
    bmin = {
        "blocked_windowed_f64": bytes_blocked(nnz, n, n, BW.n_slices, 8, 8),
        "crs_f64": bytes_crs(nnz, n, n, 8, 8),
        "jds_f64": bytes_jds(nnz, n, n, J.ndiag, 8, 8),
        "blocked_f64": bytes_blocked(nnz, n, n, B.n_slices, 8, 8),
        "crs_f32val": bytes_crs(nnz, n, n, 4, 8),
        "jds_f32val": bytes_jds(nnz, n, n, J.ndiag, 4, 8),
        "blocked_f32val": bytes_blocked(nnz, n, n, B.n_slices, 4, 8),
    }
    # the column- and row-split forms move the same algorithmic bytes as the unsplit ones
    for k in [k for k in bmin if "windowed" not in k]:
        base, tag = k.split("_", 1)
        bmin[f"{base}_split_{tag}"] = bmin[k]
        bmin[f"{base}_rowsplit_{tag}"] = bmin[k]
    return ks, bmin


def bytes_dia(D, s_v, s_x):
    """Stored diagonals read over their spans (zeros inside a span included),
    the remainder as CRS (or its padded window-sorted slices, 12 bytes of slice
    header each and one byte of slot row per row), x and y once."""
    span = sum(max(0, min(D.n_rows, D.n_cols - int(o)) - max(0, -int(o))) for o in D.offsets)
    if D.rem_slices is not None and D.rem.nnz:
        R = D.rem_slices
        rem = len(R.bl_col) * (s_v + 4) + 12 * len(R.slice_nd) + len(R.slot_row)
    else:
        rem = D.rem.nnz * (s_v + 4) + (4 * (D.n_rows + 1) if D.rem.nnz else 0)
    return span * s_v + rem + s_x * (D.n_cols + D.n_rows)


def host_cpu_model():
    """The host CPU's model name from /proc/cpuinfo (platform's name otherwise)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(W, budget_s=20.0, W3=None, HH=None):
    """The serial oracle (plain C, one core) on the same step, repeated for about
    budget_s seconds of CPU time; returns GFLOP/s.  The calling thread (the
    one that runs the oracle through ctypes) is pinned to one core for the
    duration, as the paper pins its threads; the GPU work is done by then.
    With W3 (the symmetric-diagonals workload) and HH (what the
    Hamiltonian-shaped block kept), the sampled rows of their products are
    also checked against the oracle, after the timing."""
    import oracle
    r, c, v, n, x = W["host"]
    A = oracle.csr_from_coo(n, n, r, c, v)
    J = oracle.jds_from_csr(A)
    Bk = oracle.blocked_from_jds(J, W["tune"]["blocked_C"])
    step = [lambda: oracle.spmv_crs(A, x), lambda: oracle.spmv_jds(J, x), lambda: oracle.spmv_blocked(Bk, x)]
    old_aff = None
    core = None
    if hasattr(os, "sched_getaffinity"):
        old_aff = os.sched_getaffinity(0)
        core = min(old_aff)
        os.sched_setaffinity(0, {core})
    try:
        reps = 0
        t0 = time.process_time()
        w0 = time.perf_counter()
        while True:
            for f in step:
                f()
            reps += 1
            if time.process_time() - t0 >= budget_s:
                break
        cpu_s = time.process_time() - t0
        wall = time.perf_counter() - w0
    finally:
        if old_aff is not None:
            os.sched_setaffinity(0, old_aff)
    flops = len(step) * 2.0 * A.nnz * reps
    out = {"value": round(flops / wall / 1e9, 4), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
           "sample": f"{reps} full steps (CRS, JDS, blocked JDS products in FP64) of the n=2,000,000 "
                     f"power-law matrix, "
                     f"{cpu_s:.1f} s CPU, serial FP64 C oracle (-O2, no FMA), one thread",
           "pinned_core": core, "host_cpu": host_cpu_model(), "host_logical_cpus": os.cpu_count()}
    if W3 is not None and "samples" in W3:
        out["symdiag_sampled_rows_max_rel_err_vs_oracle"] = c3_oracle_check(W3)
    if HH:
        out["hamiltonian_sampled_rows_max_rel_err_vs_oracle"] = sampled_oracle_check(HH["host"], HH["x"], HH["rows"],
                                                                                     HH["samples"])
    return out


def roofline_for(name, bytes_per_launch, ms, workload):
    achieved = bytes_per_launch / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(name, workload),
            "traffic_kind": "L2-fill bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-probe calibrated): "
                            "what the L2s exchange with the MALL and HBM, not HBM bytes alone",
            "algorithmic_bytes_per_launch": int(bytes_per_launch), "avg_launch_ms": round(ms, 5)}


def attainable_bw(torch, sp, dev):
    n = 1 << 27                                  # 1 GiB per array
    a = torch.empty(n, dtype=torch.float64, device=dev)
    b = torch.ones(n, dtype=torch.float64, device=dev)
    c = torch.ones(n, dtype=torch.float64, device=dev)
    part = torch.empty(1 << 16, dtype=torch.float64, device=dev)
    out = {}
    for name, fn, nbytes in (("triad", lambda: sp.spmv_stream_triad(a, b, c, 0.5), 24 * n),
                             ("copy", lambda: sp.spmv_stream_copy(a, b), 16 * n),
                             ("read", lambda: sp.spmv_stream_read(b, part), 8 * n),
                             ("torch_copy", lambda: a.copy_(b), 16 * n)):
        ms, _ = time_loop(torch, [(name, fn)], 20, 3)
        out[name + "_GBs"] = round(nbytes / (ms * 1e-3) / 1e9, 1)
    del a, b, c
    return out


def gather_rates(torch, sp, dev, n_idx=1 << 24):
    """Random 8-byte gathers per second (spmv_gather_probe) for x vectors that
    fit one XCD's L2, the 256 MB MALL, or only HBM."""
    g = torch.Generator(device=dev)
    g.manual_seed(20091026)
    part = torch.empty(1 << 16, dtype=torch.float64, device=dev)
    out = {}
    for label, nx in (("x_2MB_L2", 1 << 18), ("x_16MB_MALL", 1 << 21), ("x_512MB_HBM", 1 << 26)):
        x = torch.ones(nx, dtype=torch.float64, device=dev)
        idx = torch.randint(0, nx, (n_idx,), generator=g, device=dev, dtype=torch.int32)
        ms, _ = time_loop(torch, [(label, lambda: sp.spmv_gather_probe(idx, x, part))], 20, 3)
        out[label + "_Ggathers_s"] = round(n_idx / (ms * 1e-3) / 1e9, 1)
        # the line fills behind those gathers (rocprofv3 FETCH_SIZE of the probe), as a rate
        fill = measured_traffic("gather_" + label, "probe")
        if fill:
            out[label + "_fill_GBs"] = round(fill / (ms * 1e-3) / 1e9, 1)
        del x, idx
    return out


# --------------------------------------------------------------------------- suite


def _kernel_entry(name, nnz_flops, bmin, ms):
    gbs = bmin / (ms * 1e-3) / 1e9
    return {"avg_us": round(ms * 1e3, 2), "gflops": round(nnz_flops / (ms * 1e-3) / 1e9, 1),
            "algorithmic_GBs": round(gbs, 1), "frac_of_8TBs": round(gbs / HBM_PEAK_GBS, 4)}


def _rel_err_gpu(torch, sp, A64, x, y, y_ref):
    """max_i |y_i - y_ref_i| / sum_j |a_ij||x_j|, the scale from the library's own FP64 kernel."""
    Aabs = A64.with_values(A64.val.abs())
    D = sp.spmv_crs(Aabs, x.abs().to(torch.float64))
    d = (y.to(torch.float64) - y_ref).abs()
    nz = D > 0
    return float((d[nz] / D[nz]).max()) if bool(nz.any()) else 0.0


def suite_laplacian(torch, sp, dev, steps):
    import synth
    r, c, v, n, _ = synth.laplacian3d(20)
    A = sp.csr_from_coo(n, n, torch.from_numpy(r).to(dev), torch.from_numpy(c).to(dev), torch.from_numpy(v).to(dev))
    J = sp.jds_from_csr(A)
    B = sp.jds_blocked_from_jds(J, 64)
    x = torch.from_numpy(synth.uniform_vector(n, synth.rng_for(1, 1))).to(dev)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    ks = [("crs", lambda: sp.spmv_crs(A, x, y)), ("jds", lambda: sp.spmv_jds(J, x, y)),
          ("blocked", lambda: sp.spmv_jds_blocked(B, x, y))]
    _, per = time_loop(torch, ks, steps, 10)
    g = sp.Graph()
    with g.capture():
        for _ in range(100):
            sp.spmv_crs(A, x, y)
    ms_g, _ = time_loop(torch, [("graph", g.replay)], 20, 3)
    return {"workload": "7-point Laplacian 20^3 (n=8000, nnz=53600), FP64", "note": "L2-resident: latency and "
            "launch bound, no HBM roofline", "kernels": {k: {"avg_us": round(per[k] * 1e3, 2),
                                                             "gflops": round(2 * A.nnz / (per[k] * 1e-3) / 1e9, 1)}
                                                         for k, _ in ks},
            "crs_in_hip_graph_us_per_product": round(ms_g * 1e3 / 100, 2)}


def load_symdiag(torch, sp, dev, tune_cache=""):
    """The symmetric-diagonals workload (n = 6,000,000: the diagonal and 12
    mirrored secondary diagonals, N(0,1) values) in every storage the
    library has, with launch parameters from the autotuner on this device.
    The host triplets are kept for the oracle check of the CPU leg."""
    import synth
    from paper_0910_4836_amd import autotune
    r, c, v, n, _ = synth.sym_diagonals()
    A = sp.csr_from_coo(n, n, torch.from_numpy(r).to(dev), torch.from_numpy(c).to(dev), torch.from_numpy(v).to(dev))
    J = sp.jds_from_csr(A)
    x = torch.from_numpy(synth.uniform_vector(n, synth.rng_for(3, 1))).to(dev)
    tuner = autotune.Autotuner(cache_path=tune_cache or os.path.join(tempfile.mkdtemp(), "autotune.json"))
    crs_bn = autotune.tune_crs(tuner, A, x, J.ndiag)
    ju, jm, jw = tuner.tune_jds(J, x)
    bC, bR, bU, bW = tuner.tune_blocked(J, x)
    B = sp.jds_blocked_from_jds(J, bC)
    jds_tiled = tuner.tune_jds_launch(J, x, ju, jm, jw)
    blk_tiled = tuner.tune_blocked_launch(B, x, bR, bU, bW)
    setup = {}
    t0 = time.perf_counter()
    Dd = sp.dia_from_csr(A)
    torch.cuda.synchronize()
    setup["dia_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    t0 = time.perf_counter()
    Ds = sp.dia_from_csr(A, symmetric=True)
    torch.cuda.synchronize()
    setup["dia_sym_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    t0 = time.perf_counter()
    S = sp.csr_upper_from_csr(A)
    torch.cuda.synchronize()
    setup["crs_sym_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    sym_bn = autotune.tune_crs_sym(tuner, S, x, J.ndiag // 2 + 1)
    tune = {"crs_block_nnz": crs_bn, "crs_staged": A.staged, "jds_unroll": ju, "jds_max_iters": jm, "jds_wg_waves": jw,
            "jds_tiled": jds_tiled, "blocked_C": bC, "blocked_rows_per_wave": bR, "blocked_unroll": bU,
            "blocked_wg_waves": bW, "blocked_tiled": blk_tiled, "crs_sym_block_nnz": sym_bn,
            "crs_sym_staged": S.upper.staged}
    return dict(A=A, J=J, B=B, D=Dd, Ds=Ds, S=S, x=x, n=n, nnz=A.nnz, tune=tune, setup=setup, host=(r, c, v, n))


def symdiag_kernels(torch, sp, W3, vdt, y):
    """(name, fn, algorithmic bytes) of the six products with values in vdt
    and FP64 vectors (the one-triangle CRS counted over its stored entries,
    x and y once, like CRS)."""
    A, J, B, Dd, Ds, x, n, nnz = (W3[k] for k in ("A", "J", "B", "D", "Ds", "x", "n", "nnz"))
    T = W3["tune"]
    ju, jm, jw = T["jds_unroll"], T["jds_max_iters"], T["jds_wg_waves"]
    bR, bU, bW = T["blocked_rows_per_wave"], T["blocked_unroll"], T["blocked_wg_waves"]
    sv, tag = {torch.float64: (8, "f64"), torch.float32: (4, "f32val"), torch.bfloat16: (2, "bf16val")}[vdt]
    conv = (lambda t: t) if vdt == torch.float64 else (lambda t: sp.spmv_convert_values(t, vdt))
    Aq = A.with_values(conv(A.val))
    Jq = J.with_values(conv(J.jd_val))
    Bq = B.with_values(conv(B.bl_val))
    Dq = sp.DIA(Dd.n_rows, Dd.n_cols, Dd.offsets, conv(Dd.dia_val), Dd.rem)
    Dsq = sp.DIA(Ds.n_rows, Ds.n_cols, Ds.offsets, conv(Ds.dia_val), Ds.rem, True)
    Sq = W3["S"].with_values(conv(W3["S"].upper.val))
    return [(f"crs_{tag}", lambda: sp.spmv_crs(Aq, x, y), bytes_crs(nnz, n, n, sv, 8)),
            (f"jds_{tag}", jds_launch(sp, T, x, y)(Jq), bytes_jds(nnz, n, n, J.ndiag, sv, 8)),
            (f"blocked_{tag}", blocked_launch(sp, T, x, y)(Bq), bytes_blocked(nnz, n, n, B.n_slices, sv, 8)),
            (f"dia_{tag}", lambda: sp.spmv_dia(Dq, x, y), bytes_dia(Dd, sv, 8)),
            (f"dia_sym_{tag}", lambda: sp.spmv_dia(Dsq, x, y), bytes_dia(Ds, sv, 8)),
            (f"crs_sym_{tag}", lambda: sp.spmv_crs_sym(Sq, x, y), bytes_crs(Sq.nnz, n, n, sv, 8))]


def mixed_precision_c3(torch, sp, dev, W3, steps, n_sample=4000):
    """FP64 against reduced-precision value storage (FP32, BF16; FP64
    vectors) on the symmetric-diagonals matrix, in CRS, JDS, blocked JDS,
    DIA, symmetric DIA and one-triangle CRS: time, GFLOP/s, algorithmic bytes, fraction of
    8 TB/s, speed-up over the same format in FP64, the error against the
    FP64 product (the library's FP64 CRS, all rows, scaled by
    D_i = sum_j |a_ij||x_j|) and the committed counter runs' L2-fill bytes
    per launch (null when the kernel sources changed since).  Each product's output on a seeded sample of
    rows is kept for the oracle check of the CPU leg."""
    n, nnz, x = W3["n"], W3["nnz"], W3["x"]
    y = torch.empty(n, dtype=torch.float64, device=dev)
    y_ref = sp.spmv_crs(W3["A"], x)
    Aabs = W3["A"].with_values(W3["A"].val.abs())
    D = sp.spmv_crs(Aabs, x.abs())
    nz = D > 0
    rows = np.sort(np.random.default_rng(20091029).choice(n, n_sample, replace=False))
    rows_d = torch.from_numpy(rows).to(dev)
    out = {"workload": f"symmetric diagonals n={n} nnz={nnz} (diagonal + 12 mirrored secondary diagonals), "
                       f"values in FP64 / FP32 / BF16, x and y FP64", "autotuned": W3["tune"],
           "dia_diagonals": W3["D"].ndia, "dia_sym_diagonals": W3["Ds"].ndia, "crs_sym_stored": W3["S"].nnz,
           "setup_ms": W3["setup"],
           "kernels": {}}
    samples = {}
    fp64_ms = {}
    for vdt in (torch.float64, torch.float32, torch.bfloat16):
        ks = symdiag_kernels(torch, sp, W3, vdt, y)
        _, per = time_loop(torch, [(k, f) for k, f, _ in ks], max(10, steps // 4), 3)
        for name, fn, bmin in ks:
            ms = per[name]
            fam = name.rsplit("_", 1)[0]
            if vdt == torch.float64:
                fp64_ms[fam] = ms
            gbs = bmin / (ms * 1e-3) / 1e9
            fn()
            err = float(((y - y_ref).abs()[nz] / D[nz]).max())
            samples[name] = y[rows_d].cpu().numpy()
            out["kernels"][name] = {"avg_ms": round(ms, 5), "gflops": round(2.0 * nnz / (ms * 1e-3) / 1e9, 1),
                                    "algorithmic_bytes": int(bmin), "algorithmic_GBs": round(gbs, 1),
                                    "frac_of_8TBs": round(gbs / HBM_PEAK_GBS, 4),
                                    "speedup_vs_fp64": round(fp64_ms[fam] / ms, 3),
                                    "max_rel_err_vs_fp64_product": err,
                                    "l2_fill_bytes": measured_traffic(name, "symdiag")}
        del ks
    W3["samples"] = (rows, samples)
    return out


def sampled_oracle_check(host, x, rows, samples):
    """Sampled rows of products against the serial FP64 oracle (unrounded
    values): max_i |y_i - y_oracle_i| / D_i over the rows, per product.  Only
    the triplets of those rows go through the oracle's COO -> CRS."""
    import oracle
    r, c, v, n = host
    keep = np.zeros(n, dtype=bool)
    keep[rows] = True
    sel = keep[r]
    R = oracle.csr_from_coo(n, n, r[sel], c[sel], v[sel])
    x = x.cpu().numpy()
    want = oracle.spmv_crs(R, x)[rows]
    D = oracle.row_absdot(R, x)[rows]
    return {name: float(oracle.rel_err(got, want, D).max()) for name, got in samples.items()}


def c3_oracle_check(W3):
    """The sampled rows of every product of the mixed-precision block against
    the serial FP64 oracle."""
    rows, samples = W3["samples"]
    return sampled_oracle_check(W3["host"], W3["x"], rows, samples)


def suite_symdiag(torch, sp, dev, steps):
    """The symmetric-diagonals products (as in the default line) plus the
    SOJDS ordering of the blocked storage."""
    W3 = load_symdiag(torch, sp, dev)
    out = mixed_precision_c3(torch, sp, dev, W3, steps)
    n, nnz, x, J = W3["n"], W3["nnz"], W3["x"], W3["J"]
    T = W3["tune"]
    bC, bR, bU, bW = T["blocked_C"], T["blocked_rows_per_wave"], T["blocked_unroll"], T["blocked_wg_waves"]
    y = torch.empty(n, dtype=torch.float64, device=dev)
    y_ref = sp.spmv_crs(W3["A"], x)
    # SOJDS (paper Section 2): the same slices with every row's entries
    # re-assigned to diagonal slots for near-unit x strides across rows
    t0 = time.perf_counter()
    Bs = sp.jds_blocked_from_jds(J, bC, sojds=True)
    torch.cuda.synchronize()
    out["sojds_build_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    ks = [("blocked_sojds_f64", lambda: sp.spmv_jds_blocked(Bs, x, y, rows_per_wave=bR, unroll=bU, wg_waves=bW))]
    _, per = time_loop(torch, ks, max(10, steps // 4), 3)
    out["kernels"]["blocked_sojds_f64"] = _kernel_entry("blocked_sojds_f64", 2.0 * nnz,
                                                        bytes_blocked(nnz, n, n, Bs.n_slices, 8, 8),
                                                        per["blocked_sojds_f64"])
    ks[0][1]()
    out["kernels"]["blocked_sojds_f64"]["max_rel_err_vs_fp64_product"] = _rel_err_gpu(torch, sp, W3["A"], x, y, y_ref)
    del Bs
    W3.pop("samples", None)
    return out


def load_hamiltonian(torch, sp, dev, tune_cache=""):
    """A symmetric matrix shaped like the paper's Hamiltonian (the diagonal,
    six mirrored pairs of 70%-filled outer diagonals, 2-3 scattered entries
    per row and triangle inside a band of 500) in CRS, JDS, blocked JDS and
    the DIA hybrid with its remainder in CRS, in window-sorted slices, and
    over one triangle of the diagonals; launch shapes autotuned."""
    import synth
    from paper_0910_4836_amd import autotune
    r, c, v, n, _ = synth.heavy_diagonals_band()
    nnz = len(r)
    x = torch.from_numpy(synth.uniform_vector(n, synth.rng_for(6, 1))).to(dev)
    A = sp.csr_from_coo(n, n, torch.from_numpy(r).to(dev), torch.from_numpy(c).to(dev), torch.from_numpy(v).to(dev))
    J = sp.jds_from_csr(A)
    tuner = autotune.Autotuner(cache_path=tune_cache or os.path.join(tempfile.mkdtemp(), "autotune.json"))
    autotune.tune_crs(tuner, A, x, J.ndiag)
    ju, jm, jw = tuner.tune_jds(J, x)
    bC, bR, bU, bW = tuner.tune_blocked(J, x)
    B = sp.jds_blocked_from_jds(J, bC)
    T = {"crs_staged": A.staged, "jds_unroll": ju, "jds_max_iters": jm, "jds_wg_waves": jw,
         "jds_tiled": tuner.tune_jds_launch(J, x, ju, jm, jw),
         "blocked_C": bC, "blocked_rows_per_wave": bR, "blocked_unroll": bU, "blocked_wg_waves": bW,
         "blocked_tiled": tuner.tune_blocked_launch(B, x, bR, bU, bW)}
    return {"n": n, "nnz": nnz, "x": x, "A": A, "J": J, "B": B, "D": sp.dia_from_csr(A),
            "Ds": sp.dia_from_csr(A, sliced=True), "Dy": sp.dia_from_csr(A, symmetric=True, sliced=True),
            "tune": T, "host": (r, c, v, n)}


def hamiltonian_kernels(sp, H, y):
    """(name, launch, algorithmic bytes) of the Hamiltonian-shaped products."""
    A, J, B, D, Ds, Dy, x = H["A"], H["J"], H["B"], H["D"], H["Ds"], H["Dy"], H["x"]
    n, nnz = H["n"], H["nnz"]
    return [("crs", lambda: sp.spmv_crs(A, x, y), bytes_crs(nnz, n, n, 8, 8)),
            ("jds", jds_launch(sp, H["tune"], x, y)(J), bytes_jds(nnz, n, n, J.ndiag, 8, 8)),
            ("blocked", blocked_launch(sp, H["tune"], x, y)(B), bytes_blocked(nnz, n, n, B.n_slices, 8, 8)),
            ("dia_crs_remainder", lambda: sp.spmv_dia(D, x, y), bytes_dia(D, 8, 8)),
            ("dia_sliced_remainder", lambda: sp.spmv_dia(Ds, x, y), bytes_dia(Ds, 8, 8)),
            ("dia_sym_sliced_remainder", lambda: sp.spmv_dia(Dy, x, y), bytes_dia(Dy, 8, 8))]


def suite_hamiltonian(torch, sp, dev, steps, keep=None, n_sample=4000, sweep=False, tune_cache=""):
    """The Hamiltonian-shaped products: time, rate, and agreement with the
    library's FP64 CRS product.  With `keep` (a dict), each product's output
    on a seeded sample of rows and the host triplets are left there for the
    oracle check of the CPU leg.  With `sweep`, blocked JDS in slice order
    (RBJDS) and in SOJDS order over slice heights 64..4096 (the paper's
    block-size dependence, Fig. 7), same launch parameters."""
    H = load_hamiltonian(torch, sp, dev, tune_cache)
    n, nnz, A, D, Ds, Dy = H["n"], H["nnz"], H["A"], H["D"], H["Ds"], H["Dy"]
    y = torch.empty(n, dtype=torch.float64, device=dev)
    ks = hamiltonian_kernels(sp, H, y)
    _, per = time_loop(torch, [(k, f) for k, f, _ in ks], max(20, steps // 4), 5)
    out = {"workload": f"Hamiltonian-shaped symmetric matrix n={n} nnz={nnz} (diagonal, 6 mirrored pairs of "
                       "70%-filled outer diagonals, band of 500), FP64", "autotuned": H["tune"],
           "dia": {"stored_diagonals": int(D.ndia), "remainder_nnz": int(D.rem.nnz),
                   "remainder_padded_slots": int(Ds.rem_slices.bl_col.numel()),
                   "sym_stored_diagonals": int(Dy.ndia), "sym_remainder_nnz": int(Dy.rem.nnz)},
           "kernels": {}}
    y_ref = sp.spmv_crs(A, H["x"])
    rows = np.sort(np.random.default_rng(20091030).choice(n, n_sample, replace=False))
    rows_d = torch.from_numpy(rows).to(dev)
    samples = {}
    for k, fn, bmin in ks:
        out["kernels"][k] = _kernel_entry(k, 2.0 * nnz, bmin, per[k])
        fn()
        samples[k] = y[rows_d].cpu().numpy()
        out["kernels"][k]["max_rel_err_vs_fp64_crs"] = _rel_err_gpu(torch, sp, A, H["x"], y, y_ref)
        out["kernels"][k]["l2_fill_bytes"] = measured_traffic(k, "hamiltonian")
    if keep is not None:
        keep.update(host=H["host"], x=H["x"], rows=rows, samples=samples)
    if sweep:
        T = H["tune"]
        bR, bU, bW = T["blocked_rows_per_wave"], T["blocked_unroll"], T["blocked_wg_waves"]
        J, x = H["J"], H["x"]
        del H["B"], H["D"], H["Ds"], H["Dy"]
        torch.cuda.empty_cache()
        out["block_size_sweep_us"] = {}
        for C_ in (64, 128, 256, 512, 1024, 4096):
            for so in (False, True):
                Bc = sp.jds_blocked_from_jds(J, C_, sojds=so)
                name = f"{'sojds' if so else 'rbjds'}_{C_}"
                _, pc = time_loop(torch, [(name, lambda: sp.spmv_jds_blocked(Bc, x, y, rows_per_wave=bR, unroll=bU,
                                                                             wg_waves=bW))], 20, 3)
                out["block_size_sweep_us"][name] = round(pc[name] * 1e3, 1)
                del Bc
    return out


def suite_spmm(torch, sp, dev, W, steps):
    n, nnz = W["n"], W["nnz"]
    out = {"workload": f"power-law n={n} nnz={nnz} times k vectors (column-major X, Y)", "kernels": {}}
    # the multi-vector CRS kernel gets its own tuned plan (entries per block)
    from paper_0910_4836_amd import autotune
    tuner = autotune.Autotuner(cache_path=os.path.join(tempfile.mkdtemp(), "autotune.json"))
    out["autotuned_block_nnz"] = {}
    # blocked JDS over the windowed row order (C = 64), two window sizes: a
    # window's X rows at k = 32 (FP64: 2 or 8 MB) against one XCD's 4 MB L2
    wins = {sig: sp.jds_blocked_windowed_from_csr(W["A"], 64, sig) for sig in (8192, 32768)}
    out["windowed_sigma_ms"] = {}
    for k in (8, 32):
        for dt, sv, tag in ((torch.float64, 8, "f64"), (torch.float32, 4, "f32")):
            A = autotune.tune_spmm_crs(tuner, W["A"] if dt == torch.float64 else W["A32"], k, dt, W["J"].ndiag)
            out["autotuned_block_nnz"][f"{tag}_k{k}"] = A.block_nnz
            J = W["J"] if dt == torch.float64 else W["J32"]
            X = sp.colmajor(n, k, dt, dev)
            X.copy_(torch.rand(n, k, dtype=dt, device=dev) * 2 - 1)
            Y = sp.colmajor(n, k, dt, dev)
            ws = sp.spmm_workspace(n, k, dt, dev)
            wq = {sig: (B if dt == torch.float64 else B.with_values(sp.spmv_convert_values(B.bl_val, dt)))
                  for sig, B in wins.items()}
            _, pw = time_loop(torch, [(str(sig), (lambda B: lambda: sp.spmm_jds_blocked(B, X, Y, ws=ws))(B))
                                      for sig, B in wq.items()], max(5, steps // 20), 2)
            sig = int(min(pw, key=pw.get))
            out["windowed_sigma_ms"][f"{tag}_k{k}"] = {s_: round(ms, 4) for s_, ms in pw.items()}
            Bw = wq[sig]
            ks = [(f"spmm_crs_{tag}_k{k}", lambda: sp.spmm_crs(A, X, Y, ws=ws)),
                  (f"spmm_jds_{tag}_k{k}", lambda: sp.spmm_jds(J, X, Y, ws=ws)),
                  (f"spmm_windowed_{tag}_k{k}", lambda: sp.spmm_jds_blocked(Bw, X, Y, ws=ws))]
            _, per = time_loop(torch, ks, max(5, steps // 20), 2)
            out["kernels"][ks[0][0]] = _kernel_entry(ks[0][0], 2.0 * nnz * k, bytes_crs(nnz, n, n, sv, sv, k),
                                                     per[ks[0][0]])
            out["kernels"][ks[1][0]] = _kernel_entry(ks[1][0], 2.0 * nnz * k,
                                                     bytes_jds(nnz, n, n, J.ndiag, sv, sv, k), per[ks[1][0]])
            out["kernels"][ks[2][0]] = _kernel_entry(ks[2][0], 2.0 * nnz * k,
                                                     bytes_blocked(nnz, n, n, Bw.n_slices, sv, sv, k), per[ks[2][0]])
            out["kernels"][ks[2][0]]["sigma"] = sig
            del X, Y, ws, wq
    del wins
    return out


def suite_batched(torch, sp, dev, steps, count=512):
    import synth
    from paper_0910_4836_amd import autotune
    jds, xs = [], []
    nnz = 0
    rows = 0
    for r, c, v, n, x in synth.many_matrices(count=count):
        A = sp.csr_from_coo(n, n, torch.from_numpy(r).to(dev), torch.from_numpy(c).to(dev),
                            torch.from_numpy(v).to(dev))
        jds.append(sp.jds_from_csr(A))
        xs.append(torch.from_numpy(x).to(dev))
        nnz += A.nnz
        rows += n
        del A
    # slice height, rows per wavefront and unroll from the library's autotuner, on this device
    tuner = autotune.Autotuner(cache_path=os.path.join(tempfile.mkdtemp(), "autotune.json"))
    bC, bR, bU = tuner.tune_batched(jds)
    mats = [sp.jds_blocked_from_jds(J, bC) for J in jds]
    del jds
    Bt = sp.Batched(mats, rows_per_wave=bR or 64, unroll=bU)
    x = torch.cat(xs)
    y = torch.empty(Bt.total_rows, dtype=torch.float32, device=dev)
    g = sp.Graph()
    with g.capture():
        Bt(x, y)
    ms_graph, _ = time_loop(torch, [("batched_graph", g.replay)], max(5, steps // 10), 2)
    ms_eager, _ = time_loop(torch, [("batched", lambda: Bt(x, y))], max(5, steps // 10), 2)
    ys = [torch.empty(m.n, dtype=torch.float32, device=dev) for m in mats]

    def loop():
        for m, xm, ym in zip(mats, xs, ys):
            sp.spmv_jds_blocked(m, xm, ym)
    ms_loop, _ = time_loop(torch, [("per_matrix", loop)], 3, 1)
    bm = nnz * 8 + sum(12 * m.n_slices for m in mats) + 4 * rows + 4 * 2 * rows
    e = _kernel_entry("batched", 2.0 * nnz, bm, ms_graph)
    return {"workload": f"{count} matrices, n log-uniform [1e3, 2e5], 5-40 entries/row, FP32; sum n={rows}, "
                        f"sum nnz={nnz}", "persistent_graph": e,
            "persistent_eager_us": round(ms_eager * 1e3, 1), "one_launch_per_matrix_us": round(ms_loop * 1e3, 1),
            "tiles": Bt.n_tiles, "rows_per_wave": Bt.rows_per_wave, "autotuned": {"C": bC, "R": bR, "U": bU}}


def suite_chebyshev(torch, sp, dev, steps):
    import synth
    from paper_0910_4836_amd import autograd as AG
    r, c, v, n, _ = synth.banded_uniform()
    A = sp.csr_from_coo(n, n, torch.from_numpy(r).to(dev), torch.from_numpy(c).to(dev), torch.from_numpy(v).to(dev))
    del r, c, v
    nnz = A.nnz
    op = AG.SpMVOperator(A)
    vals = op.J.jd_val.clone()
    x = torch.from_numpy(synth.uniform_vector(n, synth.rng_for(5, 1), np.float32)).to(dev)
    # the operator's JDS launch parameters from the library's autotuner, on this device
    from paper_0910_4836_amd import autotune
    tuner = autotune.Autotuner(cache_path=os.path.join(tempfile.mkdtemp(), "autotune.json"))
    op.unroll, op.max_iters, op.wg_waves = tuner.tune_jds(op.J, x)
    g = torch.ones(n, dtype=torch.float32, device=dev)
    y = torch.empty(n, dtype=torch.float32, device=dev)
    dv = torch.empty(nnz, dtype=torch.float32, device=dev)
    ks = [("forward_spmv", lambda: op.matvec(vals, x, y)), ("transposed_spmv", lambda: op.rmatvec(vals, g, y)),
          ("grad_vals", lambda: op.grad_vals(g, x, dv))]
    _, per = time_loop(torch, ks, max(10, steps // 4), 3)
    bm = {"forward_spmv": bytes_jds(nnz, n, n, op.J.ndiag, 4, 4), "transposed_spmv": bytes_crs(nnz, n, n, 4, 4),
          "grad_vals": nnz * (4 + 4 + 4) + 4 * n + 4 * (op.J.ndiag + 1) + 8 * n}
    kern = {k: _kernel_entry(k, 2.0 * nnz, bm[k], per[k]) for k, _ in ks}

    def fwd_bwd():
        vv = vals.detach().requires_grad_(True)
        xx = x.detach().requires_grad_(True)
        AG.chebyshev_loss(op, vv, xx, 20, 5).backward()
    ms_fb, _ = time_loop(torch, [("cheb", fwd_bwd)], 5, 1)
    return {"workload": f"banded+uniform n={n} nnz={nnz} FP32, 20-step Chebyshev, checkpoint every 5", "kernels": kern,
            "autotuned_jds": {"unroll": op.unroll, "max_iters": op.max_iters, "wg_waves": op.wg_waves},
            "loss_and_gradient_ms": round(ms_fb, 3),
            "spmv_equivalents_per_gradient": "20 forward + 15 recomputed + 20 transposed products + 20 value gradients"}


def suite_orderings(torch, sp, dev, W, steps):
    """Blocked JDS of the power-law matrix in the slice order (RBJDS) and with
    the SOJDS re-assignment, same tuned launch parameters."""
    n, nnz = W["n"], W["nnz"]
    T = W["tune"]
    bC, bR, bU, bW = T["blocked_C"], T["blocked_rows_per_wave"], T["blocked_unroll"], T["blocked_wg_waves"]
    t0 = time.perf_counter()
    Bs = sp.jds_blocked_from_jds(W["J"], bC, sojds=True)
    torch.cuda.synchronize()
    build_ms = round((time.perf_counter() - t0) * 1e3, 1)
    x = W["x"]
    y = torch.empty(n, dtype=torch.float64, device=dev)
    ks = [("rbjds_f64", lambda: sp.spmv_jds_blocked(W["B"], x, y, rows_per_wave=bR, unroll=bU, wg_waves=bW)),
          ("sojds_f64", lambda: sp.spmv_jds_blocked(Bs, x, y, rows_per_wave=bR, unroll=bU, wg_waves=bW))]
    _, per = time_loop(torch, ks, max(10, steps // 4), 3)
    out = {"workload": f"power-law n={n} nnz={nnz}: blocked JDS (C={bC}) in slice order vs SOJDS order, FP64",
           "kernels": {name: _kernel_entry(name, 2.0 * nnz, bytes_blocked(nnz, n, n, Bs.n_slices, 8, 8), per[name])
                       for name, _ in ks},
           "sojds_build_ms": build_ms}
    del Bs
    return out


def _lines_per_wave(cols, chunk, line_elems):
    """Distinct x lines (of line_elems elements) per 64-lane gather, for entries
    grouped into wavefront gathers by `chunk`; padding (col < 0) left out."""
    ok = cols >= 0
    cols, chunk = cols[ok].astype(np.int64), chunk[ok].astype(np.int64)
    lines = cols // line_elems
    m = int(lines.max(initial=0)) + 1
    _, per_chunk = np.unique(np.unique(chunk * m + lines) // m, return_counts=True)
    return {"mean": round(float(per_chunk.mean()), 2), "median": float(np.median(per_chunk)),
            "frac_ge_32": round(float((per_chunk >= 32).mean()), 3)}


def suite_gather_model(torch, sp, W):
    """Host model of the x accesses (the GPU analogue of the paper's stride
    analysis, Section 4.2): how many distinct 128-byte lines of x one 64-lane
    gather instruction touches in each format's access order, from the
    library's own arrays.  CRS: 64 consecutive entries of the stream; JDS: 64
    consecutive permuted rows of one diagonal; blocked: 64 rows of one slice
    diagonal."""
    n, nnz = W["n"], W["nnz"]
    le = 128 // 8
    A, J, B = W["A"], W["J"], W["B"]
    col = A.col_idx.cpu().numpy()
    out = {"workload": f"power-law n={n} nnz={nnz}: distinct 128-byte x lines per 64-lane gather (FP64 x)",
           "lines_per_wave": {"crs": _lines_per_wave(col, np.arange(len(col)) // 64, le)}}
    jc = J.jd_col.cpu().numpy()
    idx = np.arange(len(jc), dtype=np.int64)
    d = np.searchsorted(J.h_jd_ptr, idx, side="right") - 1
    r = idx - J.h_jd_ptr[d]
    out["lines_per_wave"]["jds"] = _lines_per_wave(jc, d * (n // 64 + 1) + r // 64, le)
    del jc, idx, d, r
    bc = B.bl_col.cpu().numpy()
    out["lines_per_wave"][f"blocked_C{B.C}"] = _lines_per_wave(bc, np.arange(len(bc)) // 64, le)
    del bc
    # every line a miss: bytes of x fetched per stored entry, against the measured HBM-side bytes
    out["x_bytes_per_entry_if_every_line_misses"] = {k: round(v["mean"] * 128 / 64, 1)
                                                     for k, v in out["lines_per_wave"].items()}
    meas = {}
    for name in ("crs_f64", "jds_f64", "blocked_f64"):
        t = measured_traffic(name, "powerlaw")
        if t:
            meas[name] = round(t / nnz, 1)
    out["measured_hbm_bytes_per_entry"] = meas
    return out


STRIDE_EDGES = (8, 64, 512, 4096, 32768, 262144, 2097152, 16777216)


def _stride_dist(cols, sx=8):
    """Jumps in x between consecutive accesses of one serial traversal of the
    stored entries (padding, col < 0, left out), in bytes: the fraction of
    backward jumps, of forward jumps below 64 bytes, and the cumulative
    fractions below each edge for forward and backward jumps (each a share
    of all jumps)."""
    c = cols[cols >= 0].astype(np.int64)
    d = np.diff(c) * sx
    m = max(len(d), 1)
    fwd, bwd = d[d >= 0], -d[d < 0]
    return {"jumps": int(len(d)), "backward_frac": round(len(bwd) / m, 4),
            "forward_below_64B_frac": round(float((fwd < 64).sum()) / m, 4),
            "forward_cdf": {str(e): round(float((fwd < e).sum()) / m, 4) for e in STRIDE_EDGES},
            "backward_cdf": {str(e): round(float((bwd < e).sum()) / m, 4) for e in STRIDE_EDGES}}


def _row_order_cols(A, perm):
    """Columns in the order a row-by-row traversal of the permuted rows reads
    them (RBJDS with one-row blocks)."""
    rp = A.row_ptr.cpu().numpy().astype(np.int64)
    col = A.col_idx.cpu().numpy()
    lens = rp[perm + 1] - rp[perm]
    starts = np.repeat(rp[perm], lens)
    offs = np.arange(int(lens.sum()), dtype=np.int64) - np.repeat(np.cumsum(lens) - lens, lens)
    return col[starts + offs]


def suite_stride_dist(torch, sp, dev, W):
    """The paper's stride distributions (Fig. 6a, Section 4.2) on the library's
    own arrays: CRS, RBJDS with one-row blocks, blocked JDS (RBJDS) with 64-
    and 1024-row slices, SOJDS with 1024-row slices, and JDS, for the
    power-law matrix, a symmetric-diagonals matrix and a Hamiltonian-shaped
    one (partly filled outer diagonals and a band, the paper's matrix's
    structure).  A serial traversal is what the paper's CPU kernels do; a
    wavefront reads 64 of these entries at once (the gather model)."""
    import synth
    out = {"unit": "fractions of all jumps; x is FP64, edges in bytes", "matrices": {}}

    def schemes(A, J):
        perm = J.perm.cpu().numpy().astype(np.int64)
        res = {"crs": _stride_dist(A.col_idx.cpu().numpy()),
               "rbjds_1": _stride_dist(_row_order_cols(A, perm))}
        for C_, so in ((64, False), (1024, False), (1024, True)):
            B = sp.jds_blocked_from_jds(J, C_, sojds=so)
            res[("sojds_" if so else "rbjds_") + str(C_)] = _stride_dist(B.bl_col.cpu().numpy())
            del B
        res["jds"] = _stride_dist(J.jd_col.cpu().numpy())
        return res

    out["matrices"][f"power-law n={W['n']} nnz={W['nnz']}"] = schemes(W["A"], W["J"])
    r, c, v, n, _ = synth.sym_diagonals(n=1_000_000, ndiag=12)
    A = sp.csr_from_coo(n, n, torch.from_numpy(r).to(dev), torch.from_numpy(c).to(dev), torch.from_numpy(v).to(dev))
    J = sp.jds_from_csr(A)
    out["matrices"][f"symmetric diagonals n={n} nnz={len(r)}"] = schemes(A, J)
    del A, J
    r, c, v, n, _ = synth.heavy_diagonals_band(n=1_000_000)
    A = sp.csr_from_coo(n, n, torch.from_numpy(r).to(dev), torch.from_numpy(c).to(dev), torch.from_numpy(v).to(dev))
    J = sp.jds_from_csr(A)
    out["matrices"][f"Hamiltonian-shaped n={n} nnz={len(r)}"] = schemes(A, J)
    del A, J
    return out


def suite_shard(torch, sp, dev, W, steps, G=8, g=3):
    """One GPU's share of the row-partitioned product over G GPUs, at its real
    shape: rows [g*n/G, (g+1)*n/G) of the power-law matrix, split into the
    local block (the columns this GPU owns, read from its own slice of x) and
    the remote block (every other column, read from the all-gathered x):
    y = A_loc x_loc, then y += A_rem x (beta = 1), in CRS and in JDS.  The x
    exchange itself is not run (one GPU); its link time is the estimate of a
    16 MB all-gather over 7 xGMI links."""
    r, c, v, n, _ = W["host"]
    r0, r1 = g * n // G, (g + 1) * n // G
    m = r1 - r0
    a, b = np.searchsorted(r, [r0, r1])
    rr = (r[a:b] - r0).astype(np.int32)
    cc, vv = c[a:b], v[a:b]
    loc = (cc >= r0) & (cc < r1)

    def to(arr):
        return torch.from_numpy(np.ascontiguousarray(arr)).to(dev)
    AL = sp.csr_from_coo(m, m, to(rr[loc]), to((cc[loc] - r0).astype(np.int32)), to(vv[loc]))
    AR = sp.csr_from_coo(m, n, to(rr[~loc]), to(cc[~loc]), to(vv[~loc]))
    sp.spmv_crs_plan(AL)
    sp.spmv_crs_plan(AR)
    JL, JR = sp.jds_from_csr(AL), sp.jds_from_csr(AR)
    T = W["tune"]
    ju, jm, jw = T["jds_unroll"], T["jds_max_iters"], T["jds_wg_waves"]
    x = W["x"]
    xl = x[r0:r1]
    y = torch.empty(m, dtype=torch.float64, device=dev)
    pairs = {
        "crs": [("crs_local", lambda: sp.spmv_crs(AL, xl, y)),
                ("crs_remote", lambda: sp.spmv_crs(AR, x, y, beta=1.0))],
        "jds": [("jds_local", lambda: sp.spmv_jds(JL, xl, y, unroll=ju, max_iters=jm, wg_waves=jw)),
                ("jds_remote", lambda: sp.spmv_jds(JR, x, y, beta=1.0, unroll=ju, max_iters=jm, wg_waves=jw))]}
    # the shard's y against the same rows of the whole-matrix product
    A = W["A"]
    y_full = sp.spmv_crs(A, x)[r0:r1]
    D = sp.spmv_crs(A.with_values(A.val.abs()), x.abs())[r0:r1]
    nnz_shard = int(b - a)
    out = {"workload": f"power-law n={n}: rows {r0}..{r1} (GPU {g} of {G}), local block {int(loc.sum())} entries, "
                       f"remote block {int((~loc).sum())} entries, FP64",
           "nnz_shard": nnz_shard, "kernels": {}, "shard_product": {}}
    for fam, ks in pairs.items():
        for _, fn in ks:
            fn()
        err = float(((y - y_full).abs() / D.clamp_min(1e-300)).max())
        if err > 1e-12:
            raise RuntimeError(f"shard {fam} product differs from the whole-matrix rows: {err}")
        _, per = time_loop(torch, ks, max(20, steps), 5)
        ms = graph_step_ms(torch, sp, ks, max(20, steps), 5)
        for name, _ in ks:
            out["kernels"][name] = {"avg_us": round(per[name] * 1e3, 2)}
        out["shard_product"][fam] = {"us": round(ms * 1e3, 2),
                                     "gflops": round(2.0 * nnz_shard / (ms * 1e-3) / 1e9, 1),
                                     "max_rel_err_vs_whole": err}
    out["x_allgather_estimate_us"] = round((n - m) * 8 / (7 * 153e9) * 1e6, 1)
    del AL, AR, JL, JR
    return out


def suite_lines(torch, sp, dev, W, steps, warmup, only=""):
    lines = []
    keep = set(x for x in only.split(",") if x)
    for name, fn in (("laplacian", lambda: suite_laplacian(torch, sp, dev, steps)),
                     ("orderings", lambda: suite_orderings(torch, sp, dev, W, steps)),
                     ("gather-model", lambda: suite_gather_model(torch, sp, W)),
                     ("stride-distribution", lambda: suite_stride_dist(torch, sp, dev, W)),
                     ("one-shard-of-8", lambda: suite_shard(torch, sp, dev, W, steps)),
                     ("multi-vector", lambda: suite_spmm(torch, sp, dev, W, steps)),
                     ("symmetric-diagonals", lambda: suite_symdiag(torch, sp, dev, steps)),
                     ("hamiltonian-shaped", lambda: suite_hamiltonian(torch, sp, dev, steps, sweep=True)),
                     ("chebyshev", lambda: suite_chebyshev(torch, sp, dev, steps)),
                     ("many-matrices", lambda: suite_batched(torch, sp, dev, steps))):
        if keep and name not in keep:
            continue
        print(f"# suite: {name}", file=sys.stderr, flush=True)
        rec = fn()
        print(json.dumps(rec), flush=True)
        torch.cuda.empty_cache()
        lines.append(rec)
    return lines


def run_symdiag_only(torch, sp, dev, args):
    """Profiling runs of the symmetric-diagonals products: the kernels named
    by --only (all fifteen if none), eager loop, one JSON line."""
    W3 = load_symdiag(torch, sp, dev, args.tune_cache)
    y = torch.empty(W3["n"], dtype=torch.float64, device=dev)
    keep = set(args.only.split(",")) if args.only else None
    out = {"workload": "symdiag", "autotuned": W3["tune"], "kernels": {}, "algorithmic_bytes": {}}
    for vdt in (torch.float64, torch.float32, torch.bfloat16):
        kb = [(k, f, b) for k, f, b in symdiag_kernels(torch, sp, W3, vdt, y) if keep is None or k in keep]
        if not kb:
            continue
        _, per = time_loop(torch, [(k, f) for k, f, _ in kb], args.steps, args.warmup)
        out["kernels"].update({k: round(ms, 5) for k, ms in per.items()})
        out["algorithmic_bytes"].update({k: int(b) for k, _, b in kb})
    print(json.dumps(out), flush=True)


def run_hamiltonian_only(torch, sp, dev, args):
    """Profiling runs of the Hamiltonian-shaped products: the kernels named by
    --only (all six if none), eager loop, one JSON line."""
    H = load_hamiltonian(torch, sp, dev, args.tune_cache)
    y = torch.empty(H["n"], dtype=torch.float64, device=dev)
    keep = set(args.only.split(",")) if args.only else None
    kb = [(k, f, b) for k, f, b in hamiltonian_kernels(sp, H, y) if keep is None or k in keep]
    _, per = time_loop(torch, [(k, f) for k, f, _ in kb], args.steps, args.warmup)
    print(json.dumps({"workload": "hamiltonian", "n": H["n"], "nnz": H["nnz"],
                      "autotuned": H["tune"],
                      "kernels": {k: round(ms, 5) for k, ms in per.items()},
                      "algorithmic_bytes": {k: int(b) for k, _, b in kb}}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); a row partition over several GPUs is "
              "a design, not a built or measured path", file=sys.stderr)
        sys.exit(2)
    if args.probe:
        run_probe(args.probe)
        return
    import torch
    import paper_0910_4836_amd as sp
    sp.load_library()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.workload == "symdiag":
        run_symdiag_only(torch, sp, dev, args)
        return
    if args.workload == "hamiltonian":
        run_hamiltonian_only(torch, sp, dev, args)
        return
    W = load_powerlaw(torch, sp, dev, args.tune_cache)
    print("# power-law workload built", file=sys.stderr, flush=True)
    all_ks, bmin = powerlaw_kernels(sp, W, torch)
    # the step: the three FP64 products of the power-law workload
    plain = [k for k in all_ks if "split" not in k[0] and "windowed" not in k[0]]
    windowed = [k for k in all_ks if "windowed" in k[0]]
    ks = [k for k in plain if k[0].endswith("_f64")]
    mixed = [k for k in plain if not k[0].endswith("_f64")]
    split = [k for k in all_ks if "_split" in k[0]]
    rsplit = [k for k in all_ks if "_rowsplit" in k[0]]
    if args.only:
        keep = set(args.only.split(","))
        ks = [k for k in all_ks if k[0] in keep]
        mixed = []
        split = []
        rsplit = []
        windowed = []
    med = {}
    ms_eager, per = time_loop(torch, ks, args.steps, args.warmup, med)
    # the step itself runs as one HIP graph of its products (no launch gaps
    # between them); the per-kernel times above come from the eager loop,
    # with events between the products
    ms_step = ms_eager if args.no_graph else graph_step_ms(torch, sp, ks, args.steps, args.warmup)
    flops_step = 2.0 * W["nnz"] * len(ks)
    value = flops_step / (ms_step * 1e-3) / 1e9
    dom = max(per, key=per.get)

    def entry(name, ms):
        return {"avg_ms": round(ms, 5), "gflops": round(2.0 * W["nnz"] / (ms * 1e-3) / 1e9, 1),
                "algorithmic_GBs": round(bmin[name] / (ms * 1e-3) / 1e9, 1),
                "frac_of_8TBs": round(bmin[name] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    kernels = {name: dict(entry(name, per[name]), median_ms=round(med[name], 5)) for name, _ in ks}
    out = {
        "metric": "SpMV GFLOP/s + % of HBM code-balance roofline, CRS vs JDS, FP64 vs mixed",
        "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5), "ms_per_step_eager": round(ms_eager, 5),
        "step_timing": ("eager loop with HIP events between the products" if args.no_graph else
                        "K replays of one HIP graph holding the step's products; per-kernel times from an eager "
                        "loop with HIP events between the products"), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"power-law n={W['n']} nnz={W['nnz']} (mean 15/row, max 2000): CRS, JDS and "
                               f"blocked JDS (C={W['tune']['blocked_C']}) products in FP64",
                   "n": W["n"], "nnz": W["nnz"], "ndiag": W["J"].ndiag, "products_per_step": len(ks),
                   "autotuned": W["tune"]},
        "kernels": kernels,
        "roofline": roofline_for(dom, bmin[dom], per[dom], "powerlaw"),
        "setup_ms": W["setup"],
    }
    if mixed:
        _, per_m = time_loop(torch, mixed, max(10, args.steps // 2), 3)
        out["mixed_precision"] = {name: dict(entry(name, per_m[name]),
                                             speedup_vs_fp64=round(per[name.replace("_f32val", "_f64")] /
                                                                   per_m[name], 3))
                                  for name, _ in mixed}
    if split:
        _, per_s = time_loop(torch, split, max(10, args.steps // 2), 3)
        unsplit = dict(per, **(per_m if mixed else {}))
        out["column_split"] = {name: dict(entry(name, per_s[name]),
                                          speedup_vs_unsplit=round(unsplit[name.replace("_split", "")] / per_s[name],
                                                                   3))
                               for name, _ in split}
    if rsplit:
        _, per_r = time_loop(torch, rsplit, max(10, args.steps // 2), 3)
        unsplit = dict(per, **(per_m if mixed else {}))
        out["row_split"] = {name: dict(entry(name, per_r[name]),
                                       speedup_vs_unsplit=round(unsplit[name.replace("_rowsplit", "")] / per_r[name],
                                                                3))
                            for name, _ in rsplit}
    if windowed:
        _, per_w = time_loop(torch, windowed, max(10, args.steps // 2), 3)
        out["windowed"] = {name: dict(entry(name, per_w[name]),
                                      speedup_vs_blocked=round(per["blocked_f64"] / per_w[name], 3))
                           for name, _ in windowed}
        out["windowed"]["note"] = ("blocked JDS with rows sorted by length inside windows of "
                                   f"{W['tune']['windowed_sigma']} rows (slices C={W['tune']['windowed_C']}), "
                                   "launched from a tile plan that gives each XCD an eighth of the slices in order")
    W3 = None
    if not args.only and not args.no_c3:
        print("# mixed-precision block: symmetric-diagonals matrix", file=sys.stderr, flush=True)
        W3 = load_symdiag(torch, sp, dev, args.tune_cache)
        out["mixed_precision_c3"] = mixed_precision_c3(torch, sp, dev, W3, args.steps)
        for k in ("A", "J", "B", "D", "Ds"):
            W3.pop(k)
        torch.cuda.empty_cache()
    HH = {}
    if not args.only and not args.no_hamiltonian:
        print("# DIA hybrid block: Hamiltonian-shaped matrix", file=sys.stderr, flush=True)
        out["dia_hybrid_hamiltonian"] = suite_hamiltonian(torch, sp, dev, args.steps, keep=HH,
                                                           tune_cache=args.tune_cache)
        torch.cuda.empty_cache()
    if not args.no_cpu:
        print("# CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(W, W3=W3, HH=HH)
    else:
        out["cpu_baseline"] = None
    del W3, HH
    # the step's products from cold caches (MALL and L2 flushed before each launch)
    cold = cold_times(torch, sp, dev, ks)
    out["cold"] = {name: {"median_ms": round(ms, 5), "gflops": round(2.0 * W["nnz"] / (ms * 1e-3) / 1e9, 1),
                          "slowdown_vs_warm_median": round(ms / med[name], 3)} for name, ms in cold.items()}
    out["attainable_hbm"] = attainable_bw(torch, sp, dev)
    # every stored entry gathers one x element: the products are bound by the
    # random-gather rate of the level that holds x (16 MB here: the MALL for
    # the unsplit forms; one XCD's L2 holds each 2 MB slice of the split forms)
    rates = gather_rates(torch, sp, dev)
    nnz = W["nnz"]

    def gather_entry(name, ms):
        e = {"achieved_Ggathers_s": round(nnz / (ms * 1e-3) / 1e9, 1),
             "frac_of_mall_rate": round(nnz / (ms * 1e-3) / 1e9 / rates["x_16MB_MALL_Ggathers_s"], 3),
             "frac_of_l2_rate": round(nnz / (ms * 1e-3) / 1e9 / rates["x_2MB_L2_Ggathers_s"], 3)}
        # HBM-side (L2 fill) traffic per second against what the MALL gather probe draws
        t = measured_traffic(name, "powerlaw")
        probe_fill = rates.get("x_16MB_MALL_fill_GBs")
        if t and probe_fill:
            e["fill_GBs"] = round(t / (ms * 1e-3) / 1e9, 1)
            e["frac_of_mall_probe_fill"] = round(e["fill_GBs"] / probe_fill, 3)
        return e
    out["gather_bound"] = {
        "gathers_per_launch": nnz, "probe": rates,
        "kernels": {name: gather_entry(name, ms)
                    for name, ms in dict(per, **(per_s if split else {}), **(per_r if rsplit else {}),
                                         **(per_w if windowed else {})).items()
                    if name.endswith("_f64")}}
    print(json.dumps(out), flush=True)
    if args.suite:
        suite_lines(torch, sp, dev, W, args.steps, args.warmup, args.suite_lines)


if __name__ == "__main__":
    main()
