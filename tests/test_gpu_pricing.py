"""GPU: optional steepest-edge pricing (lp_options.pricing), in the wavefront
and the workgroup kernels.  Results must match the oracle run with the same
rule (status exact, objective 1e-9; x feasible with c^T x = z*), and the
textbook Klee-Minty cube must take one pivot instead of 2^n - 1."""
import numpy as np
import pytest

import oracle
from helpers import assert_parity, oracle_solve
from paper_1802_08557_amd import workloads as W

pytestmark = pytest.mark.gpu

SE = 1


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1802_08557_amd import lpbatch
    c = lpbatch.Context(0)
    yield c
    c.close()


def solve(ctx, bt, **kw):
    import torch
    from paper_1802_08557_amd.lpbatch import DeviceBatch
    print(f"[gpu] solve {bt.name} N={bt.num_lps} {kw}", flush=True)
    sol = ctx.solve(DeviceBatch.from_host(bt), stats=True, **kw)
    torch.cuda.synchronize()
    return (sol.status.cpu().numpy(), sol.x.cpu().numpy(), sol.obj.cpu().numpy(), sol.stats.cpu().numpy())


BATCHES = {
    "uniform": lambda: W.uniform_batch(2000, 50, 50, seed=71),
    "phase1": lambda: W.phase1_batch(400, 30, 30, seed=72),
    # 4..90 rows and columns: LPs of more than 64 columns go to the workgroup kernel.
    "uneven": lambda: W.uneven_batch(300, seed=73, lo=4, hi=90),
}


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name", list(BATCHES))
def test_steepest_edge_matches_the_oracle(ctx, name, prec):
    bt = BATCHES[name]()
    st, x, obj, _ = solve(ctx, bt, precision=prec, pricing=SE)
    assert_parity(bt, st, obj, x, oracle_solve(bt, pricing=SE))


@pytest.mark.parametrize("threads", [64, 256])
def test_steepest_edge_in_the_workgroup_kernel(ctx, threads):
    bt = W.phase1_batch(200, 40, 40, seed=74)
    st, x, obj, s = solve(ctx, bt, pricing=SE, block_threads=threads)
    assert (s[:, 6] != 1).all()  # no LP ran in the wavefront kernel
    assert_parity(bt, st, obj, x, oracle_solve(bt, pricing=SE))


def _klee_minty(n):
    A = np.zeros((n, n)); b = np.zeros(n); c = np.zeros(n)
    for i in range(n):
        for j in range(i):
            A[i, j] = 2.0 * 10.0 ** (i - j)
        A[i, i] = 1.0
        b[i] = 100.0 ** i
    for j in range(n):
        c[j] = 10.0 ** (n - 1 - j)
    return A, b, c


@pytest.mark.parametrize("threads", [0, 128])
def test_klee_minty_in_one_pivot(ctx, threads):
    parts = [_klee_minty(n) for n in range(2, 9)]
    bt = W.Batch(np.concatenate([p[0].ravel() for p in parts]), np.concatenate([p[1] for p in parts]),
                 np.concatenate([p[2] for p in parts]), np.zeros(sum(len(p[1]) for p in parts), np.int8),
                 np.array([len(p[1]) for p in parts], np.int32), np.array([len(p[2]) for p in parts], np.int32),
                 "klee_minty_2_8")
    st, x, obj, s = solve(ctx, bt, pricing=SE, block_threads=threads)
    assert (st == oracle.OPTIMAL).all()
    np.testing.assert_allclose(obj, [100.0 ** (n - 1) for n in range(2, 9)], rtol=1e-12)
    assert (s[:, 0] == 0).all() and (s[:, 1] == 1).all()
    st0, _, _, s0 = solve(ctx, bt, block_threads=threads)
    assert list(s0[:, 1]) == [2 ** n - 1 for n in range(2, 9)]


def test_pivot_counts_and_argument_errors(ctx):
    from paper_1802_08557_amd import lpbatch
    bt = W.uniform_batch(2000, 50, 50, seed=75)
    _, _, obj0, s0 = solve(ctx, bt)
    _, _, obj1, s1 = solve(ctx, bt, pricing=SE)
    np.testing.assert_allclose(obj1, obj0, rtol=1e-9)
    p0, p1 = s0[:, :2].sum(1).mean(), s1[:, :2].sum(1).mean()
    ref = oracle_solve(bt, pricing=SE)
    print(f"pivots per LP: Dantzig {p0:.2f}, steepest edge {p1:.2f} (oracle {ref.stats[:, :2].sum(1).mean():.2f})")
    with pytest.raises(lpbatch.LPBatchError) as ei:
        solve(ctx, bt, pricing=2)
    assert ei.value.code == lpbatch.LP_ERR_ARG


def test_steepest_edge_in_screened_and_host_solves(ctx):
    # Screened support-function solves (random 30-row relaxations, FP32, then
    # the FP64 certificate, repair and re-solve, all with the same rule) and
    # the host pipeline: every result equals the oracle's on the full LP.
    import torch
    from paper_1802_08557_amd.lpbatch import DeviceBatch
    N = 800
    P = W.polytope()
    A1, b1 = W.split_form(P)
    dirs = W.directions(N, seed=76)
    c = np.concatenate([dirs, -dirs], axis=1)
    m1, n1 = A1.shape
    bt = W.Batch(np.tile(A1.reshape(-1), N), np.tile(b1, N), c.reshape(-1), np.zeros(N * m1, np.int8),
                 np.full(N, m1, np.int32), np.full(N, n1, np.int32), "support_se")
    ref = oracle_solve(bt, pricing=SE)
    rng = np.random.default_rng(77)
    sub = np.stack([rng.permutation(m1)[:30] for _ in range(N)]).astype(np.int32)
    db = DeviceBatch.shared_from_host(A1, b1, np.zeros(m1, np.int8), c)
    print("[gpu] screened solve with steepest edge", flush=True)
    sol = ctx.solve(db, stats=True, precision=1, pricing=SE, row_subset=torch.from_numpy(sub).cuda())
    torch.cuda.synchronize()
    st, obj, x = sol.status.cpu().numpy(), sol.obj.cpu().numpy(), sol.x.cpu().numpy()
    assert_parity(bt, st, obj, x, ref)
    assert (sol.stats.cpu().numpy()[:, 3] > 0).any()  # some relaxations missed a tight row
    ub = W.uneven_batch(100, seed=78, lo=3, hi=40)
    print("[gpu] host solve with steepest edge", flush=True)
    hst, hx, hobj = ctx.solve_host(ub.A, ub.b, ub.c, ub.sense, ub.m, ub.n, chunk_lps=30, pricing=SE)
    assert_parity(ub, hst, hobj, hx, oracle_solve(ub, pricing=SE))
