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

# MI355X published figures: 256 CUs at 2.4 GHz; HBM3E 8 TB/s.  LDS: 128 B/clk
# per CU is the CDNA3-class figure (78.6 TB/s), reported for reference; the
# denominator of the LDS roofline is the rate measured on the device itself
# for the pivot sweep's access mix (lp_measure_peaks: 16-byte reads each
# followed by a 16-byte write), used whenever the measurement ran.
N_CU, CLOCK_HZ = 256, 2.4e9
PEAK_HBM = 8.0e12
LDS_NOMINAL = N_CU * 128 * CLOCK_HZ  # 78.6 TB/s

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


def surplus_columns(batch):
    """Per LP, the rows that are >= after sign normalisation (rows with b < 0
    are negated, flipping <= and >=): each adds a surplus column."""
    neg = batch.b < 0
    ge = ((batch.sense == 1) & ~neg) | ((batch.sense == 0) & neg)
    roff = batch.offsets()[1]
    return np.add.reduceat(ge.astype(np.int64), roff[:-1]) if batch.num_lps else np.zeros(0, np.int64)


def algorithmic_bytes(batch, stats, tsize):
    """Per-launch algorithmic bytes, split by where each LP's tableau lived
    (stats column 6).  N = n + surplus columns non-basic columns.
      * one wavefront per LP (placement 1): the m x N constraint block lives in
        LDS (the objective row and the right-hand sides stay in registers):
        s*m*N written by the build, then read and written once per pivot;
      * workgroup kernel, tableau in LDS (3) or in a device-memory slot (2): the
        whole (m+1) x (N+1) condensed tableau, built once, read and written once
        per pivot -- LDS traffic for 3, HBM traffic for 2.
    HBM also carries the inputs A, b, c, sense read once and x, obj, status,
    stats written once.  Returns (lds_bytes, hbm_bytes, io_bytes, mean pivots)."""
    m = batch.m.astype(np.float64)
    n = batch.n.astype(np.float64)
    N = n + surplus_columns(batch)
    pivots = stats[:, 0].astype(np.float64) + stats[:, 1]
    place = stats[:, 6]
    cells = np.where(place == 1, m * N, (m + 1) * (N + 1))
    tab = tsize * cells * (1.0 + 2.0 * pivots)
    in_hbm = place == 2
    io = float(np.sum(8 * (m * n + m + n) + m + 8 * n + 8 + 4 + 4 * 8))
    return float(tab[~in_hbm].sum()), float(tab[in_hbm].sum()) + io, io, float(pivots.mean())


def roofline(per_kernel, dom, lds_bytes, hbm_bytes, peaks, workload_name):
    """Roofline of the dominant solve kernel: the busier memory tier for the
    algorithmic bytes, T = max(LDS bytes / LDS peak, HBM bytes / HBM peak),
    against the kernel's measured time per solve.

    The algorithmic LDS bytes of a pivot are one read and one write of the
    tableau (plus one write to build it), so the LDS peak is the rate the
    device itself reaches on that mix: 16-byte reads each followed by a
    16-byte write (lp_measure_peaks' read+write stream).  Reads alone run at
    about 2.5x the rate of writes alone on gfx950, so the read-only rate
    overstates what a half-write stream can reach; frac is also given
    against it and against the nominal 128 B/clk/CU.  The HBM peak is the
    published 8 TB/s (a device copy reaches hbm_copy).  traffic: measured
    HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated), null when
    the kernel sources changed since the counters were taken; lds_traffic:
    the same from the LDS bandwidth counters."""
    lds_mix = peaks.get("lds_read_write", 0.0)
    lds_peak = lds_mix if lds_mix > 0 else LDS_NOMINAL
    lds_read = peaks.get("lds_read", 0.0)
    dom_s = per_kernel[dom] * 1e-3
    if lds_bytes / lds_peak >= hbm_bytes / PEAK_HBM:
        roof = dict(bound="lds", achieved=lds_bytes / dom_s / 1e9, peak=lds_peak / 1e9, unit="GB/s",
                    frac=lds_bytes / dom_s / lds_peak)
    else:
        roof = dict(bound="hbm", achieved=hbm_bytes / dom_s / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s",
                    frac=hbm_bytes / dom_s / PEAK_HBM)
    tr = measured_traffic(dom, workload_name)
    roof["traffic"] = tr["hbm"] if tr else None
    roof.update(kernel=dom, kernel_ms=per_kernel[dom], lds_bytes_alg=lds_bytes, hbm_bytes_alg=hbm_bytes,
                lds_peak_basis="measured 16-byte read+write" if lds_mix > 0 else "nominal 128 B/clk/CU",
                lds_frac=lds_bytes / dom_s / lds_peak,
                lds_frac_vs_read_peak=lds_bytes / dom_s / lds_read if lds_read > 0 else None,
                lds_frac_vs_nominal=lds_bytes / dom_s / LDS_NOMINAL,
                hbm_frac=hbm_bytes / dom_s / PEAK_HBM,
                lds_traffic=tr["lds"] if tr else None)
    if tr and tr["hbm"]:
        # Measured bytes over the same time: below the algorithmic figure when
        # pivots share sweeps (one pass of the tableau for two or three pivots).
        roof.update(traffic_gb_per_s=tr["hbm"] / dom_s / 1e9, traffic_frac=tr["hbm"] / dom_s / PEAK_HBM)
    return roof


def cpu_baseline(batch, max_lps=100_000, one_thread_lps=100_000, min_s=5.0, max_reps=50):
    """The oracle (plain C, FP64 full tableau, built with -march=native for
    this host) on the first max_lps LPs of the benchmarked batch with one
    thread per host core, solved repeatedly until min_s seconds have passed
    (at most max_reps times; the median solve time is reported), and once on
    the first one_thread_lps LPs with one thread."""
    import oracle
    k = min(batch.num_lps, max_lps)
    sample = batch.subset(np.arange(k)) if k < batch.num_lps else batch
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    oracle.build(force=True, native=True)
    oracle._load(native=True)
    times, res = [], None
    start = time.perf_counter()
    while len(times) < max_reps and (not times or time.perf_counter() - start < min_s):
        t0 = time.perf_counter()
        res = oracle.solve(sample.A, sample.b, sample.c, sample.sense, sample.m, sample.n,
                           threads=threads, native=True)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    k1 = min(batch.num_lps, one_thread_lps)
    s1 = batch.subset(np.arange(k1)) if k1 < batch.num_lps else batch
    t1 = time.perf_counter()
    oracle.solve(s1.A, s1.b, s1.c, s1.sense, s1.m, s1.n, threads=1, native=True)
    dt1 = time.perf_counter() - t1
    cpu = ""
    try:
        cpu = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return res, dict(value=k / dt, unit="LPs/s", cores=int(threads), kind="oracle",
                     sample=f"first {k} LPs of the benchmarked batch, FP64 full-tableau oracle "
                            f"(gcc -O3 -march=native), {threads} threads, median of {len(times)} solves "
                            f"({dt:.3f} s each, {sum(times):.1f} s in all)",
                     one_thread=dict(value=k1 / dt1, unit="LPs/s", sample=f"first {k1} LPs, one solve, {dt1:.2f} s"),
                     cpu_model=cpu)


KERNEL_SOURCES = ("paper_1802_08557_amd/csrc/wave_kernels.hip",
                  "paper_1802_08557_amd/csrc/simplex_kernels.hip",
                  "paper_1802_08557_amd/csrc/certify_kernels.hip",
                  "paper_1802_08557_amd/csrc/certify_dense.hip",
                  "paper_1802_08557_amd/csrc/device_common.h",
                  "paper_1802_08557_amd/csrc/internal.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """Bytes per launch of `kernel` on `workload` from the committed rocprofv3
    counter summary (profiles/traffic.json): HBM from FETCH_SIZE + WRITE_SIZE
    and LDS from SQ_INSTS_LDS_LOAD_BANDWIDTH + SQ_INSTS_LDS_STORE_BANDWIDTH,
    each scaled by what the same counters read for kernels that move a known
    number of bytes (a device copy; the LDS peak kernels).  None when the
    kernel sources changed since the counters were taken; a missing figure is
    None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != kernel_source_hash():
        return None
    ent = rec.get("kernels", {}).get(f"{kernel}@{workload}")
    if not ent:
        return None
    hbm = ent["fetch_bytes"] + ent["write_bytes"] if "fetch_bytes" in ent and "write_bytes" in ent else None
    lds = ent["lds_load_bytes"] + ent["lds_store_bytes"] if "lds_load_bytes" in ent else None
    return dict(hbm=hbm, lds=lds)


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


def support_labels(P, dirs, chunk=20_000):
    """Oracle-solved tight-constraint labels of the split-form support LPs."""
    import oracle
    from oracle import mlp
    from paper_1802_08557_amd import workloads as W
    A1, b1 = W.split_form(P)
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    Y = np.empty((dirs.shape[0], A1.shape[0]), np.uint8)
    for lo in range(0, dirs.shape[0], chunk):
        bt = W.support_batch(P, dirs[lo:lo + chunk])
        r = oracle.solve(bt.A, bt.b, bt.c, bt.sense, bt.m, bt.n, threads=threads)
        Y[lo:lo + chunk] = mlp.tight_mask(A1, b1, r.x.reshape(-1, A1.shape[1]))
    return Y


def warm_start_block(args):
    """Support-function batch (1e5 directions over one 120 x 40 polytope):
    plain FP64, plain FP32 + certificate, and the network-screened FP32 +
    certificate solve with a trained and with an untrained network.  Every
    mode is checked against the oracle on a sample; times are per 1e5 LPs."""
    import torch
    import oracle
    from paper_1802_08557_amd import lpbatch, warmstart
    from paper_1802_08557_amd import workloads as W
    t0 = time.perf_counter()
    P = W.polytope(1003)
    A1, b1 = W.split_form(P)
    s1 = np.zeros(A1.shape[0], np.int8)
    dirs = W.directions(args.warm_lps, 1103)
    c = np.concatenate([dirs, -dirs], axis=1)
    train_dirs = W.directions(args.warm_train, 1203)
    Y = support_labels(P, train_dirs)
    label_s = time.perf_counter() - t0
    db = lpbatch.DeviceBatch.shared_from_host(A1, b1, s1, c)
    d_eval = torch.from_numpy(dirs.astype(np.float32)).cuda()
    d_train = torch.from_numpy(train_dirs.astype(np.float32)).cuda()
    y_train = torch.from_numpy(Y).cuda()
    ctx = lpbatch.Context(0)
    t1 = time.perf_counter()
    ctx.mlp_init(7)
    losses = warmstart.train(ctx, d_train, y_train, epochs=args.warm_epochs, seed=11)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    cold = lpbatch.Context(0)
    cold.mlp_init(7)
    stream = torch.cuda.current_stream()
    N = c.shape[0]

    def timed(fn, steps):
        out = fn(None)
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            fn(out)
        torch.cuda.synchronize()
        for cx in (ctx, cold):
            cx.kernel_times()
        st, sp = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        st.record(stream)
        for _ in range(steps):
            fn(out, timing=True)
        sp.record(stream)
        torch.cuda.synchronize()
        per_kernel = {}
        for cx in (ctx, cold):
            for nm, v in cx.kernel_times():
                per_kernel.setdefault(nm, []).append(v)
        return out, st.elapsed_time(sp) / steps, {k: float(np.sum(v)) / steps for k, v in per_kernel.items()}

    K = args.warm_k
    modes = {
        "plain_fp64": lambda out, timing=False: ctx.solve(db, stats=True, out=out, stream=stream,
                                                            time_kernels=timing),
        "plain_fp32_cert": lambda out, timing=False: ctx.solve(db, stats=True, out=out, stream=stream,
                                                                 precision=lpbatch.PREC_FP32_CERT64,
                                                                 time_kernels=timing),
        "warm_fp32_cert": lambda out, timing=False: warmstart.warm_solve(
            ctx, db, d_eval, K, stats=True, out=out, stream=stream, time_kernels=timing),
        "untrained_fp32_cert": lambda out, timing=False: warmstart.warm_solve(
            cold, db, d_eval, K, stats=True, out=out, stream=stream, time_kernels=timing),
    }
    # Oracle on a sample of the evaluation directions (all modes are compared with it).
    ns = min(N, args.warm_sample)
    bt = W.support_batch(P, dirs[:ns])
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    ref = oracle.solve(bt.A, bt.b, bt.c, bt.sense, bt.m, bt.n, threads=threads)
    res = {}
    for name, fn in modes.items():
        out, ms, kern = timed(fn, args.warm_steps)
        stn = out.status.cpu().numpy()
        obj = out.obj.cpu().numpy()
        stats = out.stats.cpu().numpy()
        opt = ref.status == 0
        rel = np.abs(obj[:ns][opt] - ref.obj[opt]) / np.maximum(1.0, np.abs(ref.obj[opt]))
        res[name] = dict(lps_per_s=N / (ms * 1e-3), ms_per_step=ms, kernels_ms=kern,
                         resolved_fp64=int(np.sum(stats[:, 3] >= 1)),
                         status_match=int(np.sum(stn[:ns] == ref.status)), compared=int(ns),
                         max_rel_obj_err=float(rel.max()) if rel.size else 0.0)
    if args.warm_k_sweep:
        sweep = {}
        for kk in [int(v) for v in args.warm_k_sweep.split(",") if v]:
            fn = lambda out, timing=False, kk=kk: warmstart.warm_solve(
                ctx, db, d_eval, kk, stats=True, out=out, stream=stream, time_kernels=timing)
            out, ms, _ = timed(fn, args.warm_steps)
            stats = out.stats.cpu().numpy()
            sweep[str(kk)] = dict(ms_per_step=ms, resolved_fp64=int(np.sum(stats[:, 3] >= 1)))
        res["warm_fp32_cert"]["screen_size_sweep"] = sweep
    # The network's share of the warm step: inference + top-k alone.
    warmstart.screen(ctx, d_eval, K)
    torch.cuda.synchronize()
    st, sp = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    st.record(stream)
    for _ in range(args.warm_steps):
        warmstart.screen(ctx, d_eval, K)
    sp.record(stream)
    torch.cuda.synchronize()
    res["warm_fp32_cert"]["mlp_infer_topk_ms"] = st.elapsed_time(sp) / args.warm_steps
    base = res["plain_fp64"]["lps_per_s"]
    for name in res:
        res[name]["speedup_vs_plain_fp64"] = res[name]["lps_per_s"] / base
    ctx.close()
    cold.close()
    return dict(workload=f"support_120x40_x{N}", screened_rows=K, train_lps=int(args.warm_train),
                epochs=int(args.warm_epochs), label_s=label_s, train_s=train_s,
                final_loss=losses[-1] if losses else None, modes=res)


def host_pipeline_block(batch, ctx, reps=3):
    """The benchmarked batch from host memory through lp_batch_solve_host
    (chunked upload / solve / download on three streams): end-to-end LPs/s
    including PCIe, for pinned and pageable host buffers and for one chunk (no
    overlap), next to the host->device copy rate of the same bytes.  Never the
    headline value: the device-resident solve is."""
    import torch
    N = batch.num_lps
    pin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
    hA, hb, hc, hs = pin(batch.A), pin(batch.b), pin(batch.c), pin(batch.sense)
    outs = (torch.empty(N, dtype=torch.int32).pin_memory(),
            torch.empty(int(batch.n.sum()), dtype=torch.float64).pin_memory(),
            torch.empty(N, dtype=torch.float64).pin_memory())

    def timed(fn):
        fn()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        return (time.perf_counter() - t0) / reps

    res = {}
    t = timed(lambda: ctx.solve_host(hA, hb, hc, hs, batch.m, batch.n, out=outs))
    res["pinned"] = dict(ms=t * 1e3, lps_per_s=N / t)
    t = timed(lambda: ctx.solve_host(hA, hb, hc, hs, batch.m, batch.n, out=outs, chunk_lps=N))
    res["pinned_one_chunk"] = dict(ms=t * 1e3, lps_per_s=N / t)
    pg = (np.empty(N, np.int32), np.empty(int(batch.n.sum())), np.empty(N))
    t = timed(lambda: ctx.solve_host(batch.A, batch.b, batch.c, batch.sense, batch.m, batch.n, out=pg))
    res["pageable"] = dict(ms=t * 1e3, lps_per_s=N / t)
    st_ok = bool(np.array_equal(outs[0].numpy(), pg[0]) and np.array_equal(outs[2].numpy(), pg[2]))
    d = torch.empty(hA.numel(), dtype=torch.float64, device="cuda")
    t = timed(lambda: (d.copy_(hA.view(-1), non_blocking=True), torch.cuda.synchronize()))
    in_bytes = hA.numel() * 8 + hb.numel() * 8 + hc.numel() * 8 + hs.numel()
    res["h2d_copy_of_A"] = dict(ms=t * 1e3, gb_per_s=hA.numel() * 8 / t / 1e9)
    res.update(input_bytes=int(in_bytes), pinned_equals_pageable=st_ok,
               note="host buffers -> device -> host, PCIe included; not the headline value")
    return res


def pricing_block(ctx, db, reps=5):
    """Optional steepest-edge pricing on the benchmark batch, FP64: ms per
    solve, LPs/s and pivots per LP, beside the same for Dantzig's rule (the
    paper's, and the headline value's)."""
    import torch
    from paper_1802_08557_amd.lpbatch import PRICE_DANTZIG, PRICE_STEEPEST_EDGE
    res = {}
    for name, pr in (("dantzig", PRICE_DANTZIG), ("steepest_edge", PRICE_STEEPEST_EDGE)):
        sol = ctx.solve(db, pricing=pr, stats=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            sol = ctx.solve(db, pricing=pr, stats=True)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        st = sol.stats.cpu().numpy()
        res[name] = dict(ms=t * 1e3, lps_per_s=db.num_lps / t,
                         pivots_per_lp=float((st[:, 0].astype(np.int64) + st[:, 1]).mean()))
    res["note"] = "optional pricing rule (default Dantzig); parity is checked in the tests"
    return res


def scaling_block(ctx, passes=4, reps=3, spread=3.0):
    """Optional scaling on a badly scaled copy of the benchmark batch (every
    row and column of every LP times 10^U[-spread, spread]; same optima): the
    solve with and without lp_options.scaling, in FP64 and FP32 + certificate.
    Per case: ms per solve (scale kernel included), pivots per LP, FP64
    re-solves; and the scale kernel's rate against HBM (algorithmic bytes:
    read A, b, c, write A', b', c' and the exponents)."""
    import torch
    from paper_1802_08557_amd import workloads as W
    from paper_1802_08557_amd.lpbatch import DeviceBatch, PREC_FP32_CERT64, PREC_FP64
    base = W.config1()
    bt = W.rescaled(base, seed=7, spread=spread)
    db = DeviceBatch.from_host(bt)
    N = bt.num_lps
    m, n = int(bt.m[0]), int(bt.n[0])
    res = dict(workload=f"rescaled_{m}x{n}_x{N}", spread=spread, passes=passes)
    for pname, prec in (("fp64", PREC_FP64), ("fp32c", PREC_FP32_CERT64)):
        for sc in (0, passes):
            sol = ctx.solve(db, precision=prec, scaling=sc, stats=True)
            torch.cuda.synchronize()
            ctx.kernel_times()
            t0 = time.perf_counter()
            for _ in range(reps):
                sol = ctx.solve(db, precision=prec, scaling=sc, stats=True, time_kernels=True)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / reps
            kt = {}
            for name, ms in ctx.kernel_times():
                kt[name] = kt.get(name, 0.0) + ms / reps
            st = sol.stats.cpu().numpy()
            key = f"{pname}_{'scaled' if sc else 'unscaled'}"
            res[key] = dict(ms=t * 1e3, lps_per_s=N / t,
                            pivots_per_lp=float((st[:, 0].astype(np.int64) + st[:, 1]).mean()),
                            fp64_resolves=int((st[:, 3] >= 1).sum()),
                            kernels_ms={k: round(v, 4) for k, v in kt.items()})
            if sc and "scale_fp64" in kt:
                nbytes = N * (16 * m * n + 20 * (m + n))
                res["scale_kernel"] = dict(ms=kt["scale_fp64"], algorithmic_bytes=nbytes,
                                           gb_per_s=nbytes / (kt["scale_fp64"] * 1e-3) / 1e9,
                                           frac_of_hbm=nbytes / (kt["scale_fp64"] * 1e-3) / 8e12)
    res["note"] = "optional preconditioning (default off); accuracy is checked in the tests, not here"
    return res


def timed_solves(ctx, db, reps, warmup=1, **kw):
    """reps solves of db timed with events on torch's current stream after
    `warmup` untimed ones; per-kernel times from the library's own events over
    the same solves.  Returns (ms per solve, {kernel: ms per solve},
    {kernel: launches per solve}, last Solution)."""
    import torch
    stream = torch.cuda.current_stream()
    out = ctx.solve(db, stats=True, stream=stream, **kw)
    kw.pop("autotune", None)
    for _ in range(warmup):
        ctx.solve(db, stats=True, stream=stream, out=out, **kw)
    torch.cuda.synchronize()
    ctx.kernel_times()
    st, sp = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    st.record(stream)
    for _ in range(reps):
        ctx.solve(db, stats=True, stream=stream, out=out, time_kernels=True, **kw)
    sp.record(stream)
    torch.cuda.synchronize()
    per, cnt = {}, {}
    for nm, v in ctx.kernel_times():
        per[nm] = per.get(nm, 0.0) + v / reps
        cnt[nm] = cnt.get(nm, 0) + 1
    return st.elapsed_time(sp) / reps, per, {k: v // reps for k, v in cnt.items()}, out


def leg_record(batch, ms, per, launches, out, peaks, prec_name):
    """One timed configuration: LPs/s, kernel times, the dominant solve
    kernel's roofline and the certificate's outcome."""
    stats = out.stats.cpu().numpy()
    solve_kernels = {k: v for k, v in per.items() if k.startswith("simplex_") and "resolve" not in k}
    dom = max(solve_kernels, key=solve_kernels.get)
    lds_b, hbm_b, io_b, piv = algorithmic_bytes(batch, stats, 4 if prec_name == "fp32c" else 8)
    roof = roofline(per, dom, lds_b, hbm_b, peaks, batch.name)
    roof.update(launches_per_solve=launches[dom], mean_pivots=piv,
                placement_counts={str(p): int(np.sum(stats[:, 6] == p)) for p in (1, 2, 3)})
    rec = dict(precision=prec_name, ms=ms, lps_per_s=batch.num_lps / (ms * 1e-3),
               kernels_ms={k: round(v, 4) for k, v in per.items()},
               launches={k: v for k, v in launches.items()}, roofline=roof)
    if prec_name == "fp32c":
        rec.update(certified=certified_count(stats),
                   fp64_resolves=int(np.sum(stats[:, 3] >= 1)),
                   resolved_from_fp32_basis=int(np.sum(stats[:, 3] == 2)))
    return rec


def certified_count(stats):
    """LPs whose FP32 result the FP64 certificate accepted: optimal (primal and
    dual feasible), unbounded (ray) or infeasible (Phase I certificate)."""
    cert = stats[:, 5]
    return int(np.sum((cert & 3) == 3) + np.sum((cert & 4) != 0) + np.sum((cert & 16) != 0))


def precision_block(ctx, db, batch, peaks, fp64_ms, reps=10):
    """The benchmark batch on the FP32 tableau with the FP64 certificate of
    every final basis (and the FP64 re-solve of those it rejects), beside the
    FP64 solve of the headline: time, kernel split and the speed ratio."""
    from paper_1802_08557_amd.lpbatch import PREC_FP32_CERT64
    ms, per, launches, out = timed_solves(ctx, db, reps, warmup=2, precision=PREC_FP32_CERT64)
    rec = leg_record(batch, ms, per, launches, out, peaks, "fp32c")
    rec.update(workload=batch.name, fp64_ms=fp64_ms, speed_vs_fp64=fp64_ms / ms)
    return rec


def config_block(ctx, cfg, peaks, reps=3, autotune=False):
    """Another configuration (500 x 500 tableaux streamed from device memory, or
    the uneven 10..300 batch in autotuned size bins), FP64 and FP32 +
    certificate: time per solve, LPs/s and the dominant solve kernel's roofline.
    Parity at these sizes is checked LP by LP in the tests."""
    from paper_1802_08557_amd.lpbatch import DeviceBatch, PREC_FP32_CERT64, PREC_FP64
    batch = workload(cfg)
    db = DeviceBatch.from_host(batch)
    res = dict(workload=batch.name, num_lps=batch.num_lps)
    for name, prec in (("fp64", PREC_FP64), ("fp32c", PREC_FP32_CERT64)):
        ms, per, launches, out = timed_solves(ctx, db, reps, warmup=1, precision=prec, autotune=autotune)
        res[name] = leg_record(batch, ms, per, launches, out, peaks, name)
    res["fp32c_speed_vs_fp64"] = res["fp64"]["ms"] / res["fp32c"]["ms"]
    if autotune:
        res["tuning"] = [dict(bin=b, fp32=f, threads=t, hbm=h) for b, f, t, h in ctx.tuning()]
    del db
    return res


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
    ap.add_argument("--no-warm", action="store_true", help="skip the warm-start comparison")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the size-binned launches on the first (untimed) solve")
    ap.add_argument("--graph", action="store_true",
                    help="capture one solve in a HIP graph and time its replays")
    ap.add_argument("--warm-only", action="store_true", help="print only the warm-start comparison")
    ap.add_argument("--warm-lps", type=int, default=100_000)
    ap.add_argument("--warm-train", type=int, default=200_000)
    ap.add_argument("--warm-epochs", type=int, default=40)
    ap.add_argument("--warm-k", type=int, default=48, help="rows each screened LP keeps")
    ap.add_argument("--warm-k-sweep", default="", help="also time these screen sizes, e.g. 48,52,60")
    ap.add_argument("--warm-steps", type=int, default=10)
    ap.add_argument("--warm-sample", type=int, default=20_000)
    ap.add_argument("--no-host", action="store_true", help="skip the host-resident pipeline leg")
    ap.add_argument("--no-scaling", action="store_true", help="skip the scaling comparison")
    ap.add_argument("--no-pricing", action="store_true", help="skip the steepest-edge comparison")
    ap.add_argument("--scaling-only", action="store_true", help="print only the scaling comparison")
    ap.add_argument("--peaks", action="store_true",
                    help="print only the measured LDS / HBM bandwidths (lp_measure_peaks)")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the peak measurement (the LDS roofline then uses the nominal figure)")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the FP32 + certificate, uneven 10..300 and 500 x 500 legs")
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
    if args.warm_only:
        print(json.dumps(warm_start_block(args)), flush=True)
        return 0
    if args.scaling_only:
        ctx = lpbatch.Context(0)
        print(json.dumps(scaling_block(ctx)), flush=True)
        ctx.close()
        return 0

    if args.peaks:
        ctx = lpbatch.Context(0)
        pk = ctx.measure_peaks()
        pk.update({f"{k}_bytes_per_clk_per_cu": pk[k] / pk["num_cu"] / pk["clock_hz"]
                   for k in ("lds_read", "lds_write", "lds_read_write", "lds_broadcast") if pk["clock_hz"] > 0})
        print(json.dumps(pk), flush=True)
        ctx.close()
        return 0

    batch = workload(args.config)
    db = DeviceBatch.from_host(batch)
    ctx = lpbatch.Context(0)
    stream = torch.cuda.current_stream()
    peaks = {} if args.no_peaks else ctx.measure_peaks()
    N = batch.num_lps
    prec = lpbatch.PREC_FP64 if args.precision == "fp64" else lpbatch.PREC_FP32_CERT64
    # allocates outputs once (and tunes the size bins when asked)
    out = ctx.solve(db, stats=True, stream=stream, precision=prec, autotune=args.autotune)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        ctx.solve(db, stats=True, stream=stream, out=out, precision=prec)
    torch.cuda.synchronize()

    graph = None
    if args.graph:
        # One solve captured on a side stream; its kernels' counters reset
        # themselves, so every replay is a full solve.
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            ctx.solve(db, stats=True, out=out, precision=prec)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            ctx.solve(db, stats=True, out=out, precision=prec)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()

    ctx.kernel_times()  # forget warm-up timings
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record(stream)
    for _ in range(args.steps):
        if graph is not None:
            graph.replay()
        else:
            ctx.solve(db, stats=True, stream=stream, out=out, time_kernels=True, precision=prec)
    stop.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(stop)
    ms_per_step = total_ms / args.steps
    if graph is not None:
        # Per-kernel times from one timed eager solve after the replays.
        ctx.solve(db, stats=True, stream=stream, out=out, time_kernels=True, precision=prec)
        torch.cuda.synchronize()

    # Per-kernel time per solve: the sum over a solve's launches (a batch of
    # mixed sizes launches the workgroup kernel once per size bin), averaged
    # over the timed solves.
    timed_solves = 1 if graph is not None else args.steps
    per_kernel, launches = {}, {}
    for nm, v in ctx.kernel_times():
        per_kernel[nm] = per_kernel.get(nm, 0.0) + v
        launches[nm] = launches.get(nm, 0) + 1
    per_kernel = {nm: float(v / timed_solves) for nm, v in per_kernel.items()}
    launches = {nm: c // timed_solves for nm, c in launches.items()}
    dom = max(per_kernel, key=per_kernel.get)
    stats = out.stats.cpu().numpy()
    status = out.status.cpu().numpy()
    obj = out.obj.cpu().numpy()
    lds_bytes, hbm_bytes, io_bytes, mean_piv = algorithmic_bytes(
        batch, stats, 8 if args.precision == "fp64" else 4)
    roof = roofline(per_kernel, dom, lds_bytes, hbm_bytes, peaks, batch.name)
    roof.update(launches_per_solve=launches[dom], io_bytes_alg=io_bytes, mean_pivots=mean_piv,
                placement_counts={str(p): int(np.sum(stats[:, 6] == p)) for p in (1, 2, 3)})
    lds_resident = bool(np.all(stats[:, 6] != 2))

    rec = dict(metric=METRIC, value=N / (ms_per_step * 1e-3), unit="LPs/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=ms_per_step,
               higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f64" if args.precision == "fp64" else "f32+f64",
               data="synthetic",
               config=dict(workload=batch.name, num_lps=N, m=int(batch.m.max()),
                           n=int(batch.n.max()), precision=args.precision,
                           seed=batch.meta.get("seed"), placement="lds" if lds_resident else "hbm"),
               roofline=roof, kernels_ms=per_kernel, wall_s=t_wall,
               launch="hip_graph_replay" if graph is not None else "eager",
               peaks=peaks or None)
    if args.autotune:
        rec["tuning"] = [dict(bin=b, fp32=f, threads=t, hbm=h) for b, f, t, h in ctx.tuning()]
    if not args.no_cpu:
        ref, cb = cpu_baseline(batch)
        rec["cpu_baseline"] = cb
        k = ref.status.shape[0]
        opt = ref.status == 0
        rel = np.abs(obj[:k][opt] - ref.obj[opt]) / np.maximum(1.0, np.abs(ref.obj[opt]))
        rec["parity"] = dict(compared=int(k), status_match=int(np.sum(status[:k] == ref.status)),
                             max_rel_obj_err=float(rel.max()) if rel.size else 0.0)
    if not args.no_host and not args.graph:
        try:
            rec["host_pipeline"] = host_pipeline_block(batch, ctx)
        except Exception as e:  # the main measurement stands on its own
            rec["host_pipeline"] = dict(error=f"{type(e).__name__}: {e}")
    if not args.no_pricing and not args.graph and args.precision == "fp64":
        try:
            rec["pricing"] = pricing_block(ctx, db)
        except Exception as e:  # the main measurement stands on its own
            rec["pricing"] = dict(error=f"{type(e).__name__}: {e}")
    if not args.no_scaling and not args.graph and args.config == 1:
        try:
            rec["lp_scaling"] = scaling_block(ctx)
        except Exception as e:  # the main measurement stands on its own
            rec["lp_scaling"] = dict(error=f"{type(e).__name__}: {e}")
    if not args.no_warm and args.config == 1:
        try:
            rec["warm_start"] = warm_start_block(args)
        except Exception as e:  # the main measurement stands on its own
            rec["warm_start"] = dict(error=f"{type(e).__name__}: {e}")
    if not args.no_legs and not args.graph and args.config == 1 and args.precision == "fp64":
        for key, fn in (("fp32_certified", lambda: precision_block(ctx, db, batch, peaks, ms_per_step)),
                        ("large_500x500", lambda: config_block(ctx, 4, peaks)),
                        ("uneven_10_300", lambda: config_block(ctx, 2, peaks, autotune=True))):
            try:
                rec[key] = fn()
            except Exception as e:  # the main measurement stands on its own
                rec[key] = dict(error=f"{type(e).__name__}: {e}")
    if args.precision == "fp32c":
        rec["certificate"] = dict(certified=certified_count(stats),
                                  resolved_fp64=int(np.sum(stats[:, 3] >= 1)))
    print(json.dumps(rec), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
