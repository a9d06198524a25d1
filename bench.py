"""Benchmark: LPs/s of the batched simplex on one MI355X.

Default workload: 100,000 independent LPs of 50 constraints x 50 variables
(A ~ U[1,10], b ~ U[100,1000], c ~ U[1,10], seed 1001), solved in FP64 with the
inputs already resident in HBM.  One step = one lp_batch_solve_ex over the
whole batch.  Prints one JSON line (rank 0) with the throughput, the roofline
of the dominant kernel and the CPU oracle timed on the host as a baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 0..4]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X figures: 256 CUs at 2.4 GHz; HBM3E 8 TB/s; LDS 128 B/clk per CU.
N_CU, CLOCK_HZ = 256, 2.4e9
PEAK_HBM = 8.0e12
PEAK_LDS = N_CU * 128 * CLOCK_HZ  # 78.6 TB/s

METRIC = "LPs/sec at batch 1e5 (50x50 FP64, warm-start vs plain); % LDS/HBM roofline"


def workload(cfg):
    from paper_1802_08557_amd import workloads as W
    if cfg == 0:
        return W.config0()
    if cfg == 1:
        return W.config1()
    if cfg == 2:
        return W.config2()
    if cfg == 3:
        return W.config3()[1]
    if cfg == 4:
        return W.config4()
    raise SystemExit(f"unknown config {cfg}")


def algorithmic_bytes(batch, stats, tsize):
    """Per-launch algorithmic bytes.
    LDS/tableau: s*(m+1)*(N+1) to build the condensed tableau plus, per pivot,
    one read and one write of it, 2*s*(m+1)*(N+1) (N = n non-basic columns for
    all-<= rows).  HBM: the inputs A, b, c, sense read once and x, obj, status,
    stats written once."""
    m = batch.m.astype(np.float64)
    n = batch.n.astype(np.float64)
    pivots = stats[:, 0].astype(np.float64) + stats[:, 1]
    cells = (m + 1) * (n + 1)
    tab = float(np.sum(tsize * cells * (1.0 + 2.0 * pivots)))
    hbm = float(np.sum(8 * (m * n + m + n) + m + 8 * n + 8 + 4 + 4 * 8))
    return tab, hbm, float(pivots.mean())


def cpu_baseline(batch, max_lps=100_000):
    import oracle
    k = min(batch.num_lps, max_lps)
    sample = batch.subset(np.arange(k)) if k < batch.num_lps else batch
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    oracle._load()
    t0 = time.perf_counter()
    res = oracle.solve(sample.A, sample.b, sample.c, sample.sense, sample.m, sample.n,
                       threads=threads)
    dt = time.perf_counter() - t0
    return res, dict(value=k / dt, unit="LPs/s", cores=int(threads), kind="oracle",
                     sample=f"first {k} LPs of the benchmarked batch, FP64 full-tableau oracle, "
                            f"{threads} threads, {dt:.2f} s wall")


KERNEL_SOURCES = ("paper_1802_08557_amd/csrc/wave_kernels.hip",
                  "paper_1802_08557_amd/csrc/simplex_kernels.hip",
                  "paper_1802_08557_amd/csrc/device_common.h",
                  "paper_1802_08557_amd/csrc/internal.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary (profiles/traffic.json), scaled
    by the factors the same counters read for a copy of known size; None when
    the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != kernel_source_hash():
        return None
    ent = rec.get("kernels", {}).get(f"{kernel}@{workload}")
    if not ent:
        return None
    return ent["fetch_bytes"] + ent["write_bytes"]


def copy_calibration(gib):
    """An elementwise copy kernel of a known size (dst = src * 1), for
    calibrating FETCH_SIZE and WRITE_SIZE under rocprofv3: each launch reads and
    writes gib GiB."""
    import torch
    n = int(gib * (1 << 30)) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_bytes=n * 8, repeats=3)), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32c"],
                    help="fp64: FP64 tableau; fp32c: FP32 tableau + FP64 certificate / re-solve")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="only run a device copy of this many GiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration > 0:
        return copy_calibration(args.copy_calibration)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(LPs are independent, so several GPUs would each run their own share).",
              file=sys.stderr)
        return 2

    import torch
    from paper_1802_08557_amd import lpbatch
    from paper_1802_08557_amd.lpbatch import DeviceBatch

    batch = workload(args.config)
    db = DeviceBatch.from_host(batch)
    ctx = lpbatch.Context(0)
    stream = torch.cuda.current_stream()
    N = batch.num_lps
    prec = lpbatch.PREC_FP64 if args.precision == "fp64" else lpbatch.PREC_FP32_CERT64
    out = ctx.solve(db, stats=True, stream=stream, precision=prec)  # allocates outputs once
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        ctx.solve(db, stats=True, stream=stream, out=out, precision=prec)
    torch.cuda.synchronize()

    ctx.kernel_times()  # forget warm-up timings
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record(stream)
    for _ in range(args.steps):
        ctx.solve(db, stats=True, stream=stream, out=out, time_kernels=True, precision=prec)
    stop.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(stop)
    ms_per_step = total_ms / args.steps

    per_kernel = {}
    for nm, v in ctx.kernel_times():
        per_kernel.setdefault(nm, []).append(v)
    per_kernel = {nm: float(np.mean(v)) for nm, v in per_kernel.items()}
    dom = max(per_kernel, key=per_kernel.get)
    stats = out.stats.cpu().numpy()
    status = out.status.cpu().numpy()
    obj = out.obj.cpu().numpy()
    tab_bytes, hbm_bytes, mean_piv = algorithmic_bytes(batch, stats, 8 if args.precision == "fp64" else 4)
    dom_s = per_kernel[dom] * 1e-3
    lds_resident = bool(np.all(stats[:, 6] == 1))
    if lds_resident:
        roof = dict(bound="lds", achieved=tab_bytes / dom_s / 1e9, peak=PEAK_LDS / 1e9, unit="GB/s",
                    frac=tab_bytes / dom_s / PEAK_LDS, traffic=None)
    else:
        roof = dict(bound="hbm", achieved=(tab_bytes + hbm_bytes) / dom_s / 1e9,
                    peak=PEAK_HBM / 1e9, unit="GB/s",
                    frac=(tab_bytes + hbm_bytes) / dom_s / PEAK_HBM, traffic=None)
    roof["traffic"] = measured_traffic(dom, batch.name)
    roof.update(kernel=dom, kernel_ms=per_kernel[dom], hbm_bytes_alg=hbm_bytes,
                hbm_frac=hbm_bytes / dom_s / PEAK_HBM, tableau_bytes_alg=tab_bytes,
                mean_pivots=mean_piv)

    rec = dict(metric=METRIC, value=N / (ms_per_step * 1e-3), unit="LPs/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=ms_per_step,
               higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f64" if args.precision == "fp64" else "f32+f64",
               data="synthetic",
               config=dict(workload=batch.name, num_lps=N, m=int(batch.m.max()),
                           n=int(batch.n.max()), precision=args.precision,
                           seed=batch.meta.get("seed"), placement="lds" if lds_resident else "hbm"),
               roofline=roof, kernels_ms=per_kernel, wall_s=t_wall)
    if not args.no_cpu:
        ref, cb = cpu_baseline(batch)
        rec["cpu_baseline"] = cb
        k = ref.status.shape[0]
        opt = ref.status == 0
        rel = np.abs(obj[:k][opt] - ref.obj[opt]) / np.maximum(1.0, np.abs(ref.obj[opt]))
        rec["parity"] = dict(compared=int(k), status_match=int(np.sum(status[:k] == ref.status)),
                             max_rel_obj_err=float(rel.max()) if rel.size else 0.0)
    if args.precision == "fp32c":
        rec["certificate"] = dict(certified=int(np.sum((stats[:, 5] & 3) == 3) + np.sum((stats[:, 5] & 4) != 0)),
                                  resolved_fp64=int(np.sum(stats[:, 3] == 1)))
    print(json.dumps(rec), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
