"""GPU parity: the HIP simplex (through the C ABI) against the CPU oracle.

Status must match exactly; the objective within 1e-9 relative (FP64 path); an
optimal x must be primal feasible with c^T x equal to the objective.  Inputs
are the seeded workloads at reduced and full sizes plus edge cases."""
import numpy as np
import pytest

import oracle
from helpers import assert_parity, oracle_solve
from paper_1802_08557_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1802_08557_amd import lpbatch
    c = lpbatch.Context(0)
    yield c
    c.close()


def run(ctx, batch, **kw):
    import torch
    from paper_1802_08557_amd.lpbatch import DeviceBatch
    print(f"[gpu] solve {batch.name} N={batch.num_lps} {kw}", flush=True)
    db = DeviceBatch.from_host(batch)
    sol = ctx.solve(db, stats=True, **kw)
    torch.cuda.synchronize()
    return (sol.status.cpu().numpy(), sol.obj.cpu().numpy(), sol.x.cpu().numpy(),
            sol.stats.cpu().numpy())


def check(ctx, batch, **kw):
    st, obj, x, stats = run(ctx, batch, **kw)
    ref = oracle_solve(batch)
    assert_parity(batch, st, obj, x, ref)
    return st, obj, x, stats, ref


def test_uniform_5x5_full(ctx):
    st, obj, x, stats, ref = check(ctx, W.config0())
    assert np.all(st == 0)


def test_uniform_50x50_reduced(ctx):
    st, obj, x, stats, ref = check(ctx, W.config1(4000))
    assert np.all(stats[:, 6] == 1)  # every LP solved by the one-wavefront kernel
    # Same pricing and ratio rules as the oracle: the pivot counts agree
    # except where rounding separates a near-tie.
    same = np.mean(stats[:, 1] == ref.stats[:, 1])
    assert same > 0.99, same


def test_uniform_50x50_full_size(ctx):
    """The benchmarked workload at full size: every LP compared."""
    check(ctx, W.config1())


def test_two_phase(ctx):
    bt = W.phase1_batch(3000, 20, 15, seed=31)
    st, obj, x, stats, ref = check(ctx, bt)
    assert (stats[:, 0] > 0).sum() > 1000
    assert {0} <= set(np.unique(st))


def test_uneven_gaussian_subset(ctx):
    bt = W.uneven_batch(300, seed=1002)
    st, obj, x, stats, ref = check(ctx, bt)
    assert set(np.unique(st)) >= {0, 1, 2}
    assert np.all(st[bt.meta["infeasible"]] == oracle.INFEASIBLE)
    assert np.all(st[bt.meta["unbounded"]] == oracle.UNBOUNDED)
    # The workgroup launch takes the CU's LDS share: some tableaux live in LDS
    # (placement 3), the largest in device-memory slots (placement 2).
    assert np.any(stats[:, 6] == 3) and np.any(stats[:, 6] == 2)


def test_uniform_500x500_hbm(ctx):
    bt = W.config4(12)
    st, obj, x, stats, ref = check(ctx, bt)
    assert np.all(stats[:, 6] == 2)  # tableau streamed from HBM


def test_support_function_batch(ctx):
    P, bt = W.config3(3000)
    st, obj, x, stats, ref = check(ctx, bt)
    assert np.all(st == 0)
    assert np.all(stats[:, 6] == 1)


RAGGED = [1, 2, 63, 64, 65, 127, 128, 129, 200]


def test_ragged_sizes_and_tails(ctx):
    rng = np.random.default_rng(41)
    parts = []
    for m in RAGGED:
        for n in RAGGED:
            if m * n > 40000:
                continue
            parts.append(W.uniform_batch(3, m, n, seed=int(rng.integers(1 << 30))))
            parts.append(W.phase1_batch(2, m, n, seed=int(rng.integers(1 << 30))))
    bt = W.Batch(np.concatenate([p.A for p in parts]), np.concatenate([p.b for p in parts]),
                 np.concatenate([p.c for p in parts]), np.concatenate([p.sense for p in parts]),
                 np.concatenate([p.m for p in parts]), np.concatenate([p.n for p in parts]),
                 "ragged")
    check(ctx, bt)


def test_edge_cases(ctx):
    import torch
    from paper_1802_08557_amd.lpbatch import DeviceBatch
    # Empty batch: nothing to do, returns OK.
    empty = W.Batch(np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0, np.int8),
                    np.zeros(0, np.int32), np.zeros(0, np.int32), "empty")
    sol = ctx.solve(DeviceBatch.from_host(empty))
    assert sol.status.numel() == 0
    # Hand examples, the cycling example, Klee-Minty, invalid input, 1x1 LPs.
    lps = [
        (np.array([[1.0, 1], [1, 3], [1, 0]]), [4, 6, 3.5], [2, 3], [0, 0, 0]),
        (np.array([[1.0, 1], [1, 1], [0, 1]]), [2, 4, 3], [1, 2], [1, 0, 0]),
        (np.array([[1.0, -1], [-1, 1]]), [1, 2], [1, 1], [0, 0]),
        (np.array([[1.0, 1]]), [-1], [1, 0], [0]),
        (np.array([[0.5, -5.5, -2.5, 9.0], [0.5, -1.5, -0.5, 1.0], [1.0, 0, 0, 0]]), [0, 0, 1],
         [10, -57, -9, -24], [0, 0, 0]),
        (np.array([[2.0]]), [3], [1], [0]),
        (np.array([[2.0]]), [3], [-1], [0]),
        (np.array([[1.0]]), [-3], [1], [2]),
        (np.array([[1.0, 1], [1, 1]]), [2, 2], [1, 1], [2, 2]),   # redundant equality
        (np.array([[1.0, np.nan]]), [1], [1, 1], [0]),            # invalid input
        (np.array([[1.0, 1]]), [1], [1, 1], [5]),                 # bad sense
    ]
    for n in range(2, 8):
        A = np.zeros((n, n)); b = np.zeros(n); c = np.zeros(n)
        for i in range(n):
            A[i, :i] = [2.0 * 10.0 ** (i - j) for j in range(i)]
            A[i, i] = 1.0; b[i] = 100.0 ** i
        c[:] = [10.0 ** (n - 1 - j) for j in range(n)]
        lps.append((A, b, c, [0] * n))
    bt = W.Batch(np.concatenate([np.asarray(a, float).ravel() for a, *_ in lps]),
                 np.concatenate([np.asarray(b, float) for _, b, *_ in lps]),
                 np.concatenate([np.asarray(c, float) for _, _, c, _ in lps]),
                 np.concatenate([np.asarray(s, np.int8) for *_, s in lps]),
                 np.array([np.asarray(a).shape[0] for a, *_ in lps], np.int32),
                 np.array([np.asarray(a).shape[1] for a, *_ in lps], np.int32), "edge")
    st, obj, x, stats = run(ctx, bt)
    ref = oracle_solve(bt)
    assert_parity(bt, st, obj, x, ref)
    assert list(st[:4]) == [0, 0, 2, 1]
    assert st[9] == oracle.INVALID_INPUT and st[10] == oracle.INVALID_INPUT
    assert obj[4] == pytest.approx(1.0, abs=1e-12)
    km = stats[11:, 1]
    assert list(km) == [2 ** n - 1 for n in range(2, 8)]
    # Pure Dantzig cycles on the degenerate example: the cap is hit.
    st2, *_ = run(ctx, bt.subset([4]), k_deg=-1)
    assert st2[0] == oracle.ITERATION_LIMIT
    st3, *_ = run(ctx, bt.subset([16]), max_iters=1)
    assert st3[0] == oracle.ITERATION_LIMIT


@pytest.mark.parametrize("pricing", [0, 1])
def test_placement_and_block_size_are_bitwise_identical(ctx, pricing):
    """Every kernel variant (one wavefront per LP, workgroups of 64..512
    threads, tableau in LDS or HBM) computes the same element updates in the
    same order, and under steepest-edge pricing the same column weights:
    bitwise-identical results expose races and missing barriers."""
    bt = W.Batch(*[np.concatenate(v) for v in zip(
        *[(p.A, p.b, p.c, p.sense, p.m, p.n) for p in
          (W.config1(300), W.phase1_batch(200, 30, 40, seed=5), W.uneven_batch(60, seed=9, lo=10, hi=120))])],
        name="mixed")
    runs = [((0, 0), run(ctx, bt, pricing=pricing))]  # automatic: one wavefront per small LP
    for placement in (1, 2):
        for nt in (64, 128, 256, 512):
            runs.append(((placement, nt), run(ctx, bt, placement=placement, block_threads=nt, pricing=pricing)))
    assert np.any(runs[0][1][3][:, 6] == 1)
    (k0, (st0, obj0, x0, s0)) = runs[0]
    for k, (st, obj, x, s) in runs[1:]:
        assert np.array_equal(st, st0), k
        assert np.array_equal(obj.view(np.int64), obj0.view(np.int64)), k
        assert np.array_equal(x.view(np.int64), x0.view(np.int64)), k
        assert np.array_equal(s[:, :3], s0[:, :3]), k


def test_synchronous_entry_point():
    import torch
    from paper_1802_08557_amd import lpbatch
    bt = W.config0(500)
    sol = lpbatch.batch_solve(lpbatch.DeviceBatch.from_host(bt))
    ref = oracle_solve(bt)
    assert_parity(bt, sol.status.cpu().numpy(), sol.obj.cpu().numpy(), sol.x.cpu().numpy(), ref)


# ---------------------------------------------------------------- FP32 tableau + FP64 certificate

FP32 = dict(precision=1)


def check_fp32(ctx, batch, rtol=1e-9):
    """Single-precision pivots, then the FP64 certificate / re-solve: results
    carry FP64 accuracy (the bar for this path is 1e-4 relative; it is held to
    1e-9 here)."""
    st, obj, x, stats = run(ctx, batch, **FP32)
    ref = oracle_solve(batch)
    assert_parity(batch, st, obj, x, ref, rtol=rtol)
    return st, obj, x, stats, ref


def test_fp32_certified_uniform_50x50(ctx):
    st, obj, x, stats, ref = check_fp32(ctx, W.config1(5000))
    assert np.all(stats[(stats[:, 3] == 0), 6] == 1)  # FP32 solves ran one wavefront per LP
    cert = stats[:, 5]
    assert np.mean((cert & 3) == 3) > 0.95  # most bases certified without a re-solve


def test_fp32_certified_two_phase_and_uneven(ctx):
    check_fp32(ctx, W.phase1_batch(1500, 20, 15, seed=32))
    bt = W.uneven_batch(200, seed=1002)
    st, obj, x, stats, ref = check_fp32(ctx, bt)
    assert np.any((stats[:, 5] & 4) != 0)   # unbounded rays certified in FP64
    # Infeasible results proven by the FP64 Phase I certificate, not re-solved.
    inf = np.asarray(bt.meta["infeasible"])
    assert np.all((stats[inf, 5] & 16) != 0)
    assert np.all(stats[inf, 3] == 0)
    assert np.all(st[(stats[:, 5] & 16) != 0] == oracle.INFEASIBLE)
    # Rows all <= with b >= 0: x = 0 is feasible, so the FP64 ray alone
    # certifies an unbounded result.
    unb = np.asarray(bt.meta["unbounded"])
    assert np.all((stats[unb, 5] & 4) != 0)


def test_fp32_certified_support_and_large(ctx):
    P, bt = W.config3(2000)
    st, obj, x, stats, ref = check_fp32(ctx, bt)
    assert np.all(stats[(stats[:, 3] == 0), 6] == 1)
    check_fp32(ctx, W.config4(8))


def test_fp32_edge_cases(ctx):
    lps = [
        (np.array([[1.0, 1], [1, 3], [1, 0]]), [4, 6, 3.5], [2, 3], [0, 0, 0]),
        (np.array([[1.0, 1], [1, 1], [0, 1]]), [2, 4, 3], [1, 2], [1, 0, 0]),
        (np.array([[1.0, -1], [-1, 1]]), [1, 2], [1, 1], [0, 0]),
        (np.array([[1.0, 1]]), [-1], [1, 0], [0]),
        (np.array([[0.5, -5.5, -2.5, 9.0], [0.5, -1.5, -0.5, 1.0], [1.0, 0, 0, 0]]), [0, 0, 1],
         [10, -57, -9, -24], [0, 0, 0]),
        (np.array([[1.0, 1], [1, 1]]), [2, 2], [1, 1], [2, 2]),
        (np.array([[1.0, np.nan]]), [1], [1, 1], [0]),
        (np.array([[3.0, 1.0]]), [6], [-1.0, -2.0], [0]),   # optimum at the origin (no basic structural)
    ]
    bt = W.Batch(np.concatenate([np.asarray(a, float).ravel() for a, *_ in lps]),
                 np.concatenate([np.asarray(b, float) for _, b, *_ in lps]),
                 np.concatenate([np.asarray(c, float) for _, _, c, _ in lps]),
                 np.concatenate([np.asarray(s, np.int8) for *_, s in lps]),
                 np.array([np.asarray(a).shape[0] for a, *_ in lps], np.int32),
                 np.array([np.asarray(a).shape[1] for a, *_ in lps], np.int32), "edge32")
    st, obj, x, stats, ref = check_fp32(ctx, bt)
    assert st[6] == oracle.INVALID_INPUT
