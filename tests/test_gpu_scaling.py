"""GPU: power-of-two geometric-mean scaling (lp_batch_scale, lp_options.scaling).

The exponents are integer work and the scaled data are exact multiples, so the
GPU output must equal the scaling oracle bit for bit.  A solve with scaling
must match the oracle's scaled solve (status exact, objective 1e-9) on badly
scaled batches, in both precisions and through the host pipeline."""
import numpy as np
import pytest

import oracle
from helpers import assert_parity, oracle_solve
from oracle.scaling import scale_batch, solve_scaled
from paper_1802_08557_amd import workloads as W

pytestmark = pytest.mark.gpu

PASSES = 4


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1802_08557_amd import lpbatch
    c = lpbatch.Context(0)
    yield c
    c.close()


def gpu_scale(ctx, bt, passes, shared=False):
    import torch
    from paper_1802_08557_amd.lpbatch import DeviceBatch
    print(f"[gpu] scale {bt.name} N={bt.num_lps} passes={passes}", flush=True)
    db = DeviceBatch.from_host(bt)
    out = ctx.scale(db, passes)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def split(flat, sizes):
    return np.split(flat, np.cumsum(sizes)[:-1])


@pytest.mark.parametrize("passes", [0, 1, PASSES])
def test_factors_and_scaled_data_are_bit_exact(ctx, passes):
    # Ragged shapes on both sides of the LDS staging limit (8192 entries):
    # 3 x 3 up to 140 x 140; zeros and a column of zeros included.
    bt = W.rescaled(W.uneven_batch(60, seed=51, lo=3, hi=140), seed=52, spread=4.0)
    aoff, roff, coff = bt.offsets()
    bt.A[aoff[1]:aoff[2]][::3] = 0.0
    A2, b2, c2, rexp, cexp = gpu_scale(ctx, bt, passes)
    ref = scale_batch(bt, passes)
    r_gpu = split(rexp, bt.m)
    s_gpu = split(cexp, bt.n)
    for k, (r, s, As, bs, cs) in enumerate(ref):
        np.testing.assert_array_equal(r_gpu[k], r, err_msg=f"row exponents, LP {k}")
        np.testing.assert_array_equal(s_gpu[k], s, err_msg=f"column exponents, LP {k}")
        np.testing.assert_array_equal(A2[aoff[k]:aoff[k + 1]], As.ravel(), err_msg=f"A', LP {k}")
        np.testing.assert_array_equal(b2[roff[k]:roff[k + 1]], bs)
        np.testing.assert_array_equal(c2[coff[k]:coff[k + 1]], cs)
    assert (bt.m.astype(np.int64) * bt.n > 8192).any() and (bt.m.astype(np.int64) * bt.n <= 8192).any()


def test_uniform_and_shared_batches(ctx):
    import torch
    from paper_1802_08557_amd.lpbatch import DeviceBatch
    bt = W.rescaled(W.uniform_batch(500, 50, 50, seed=53), seed=54)
    A2, b2, c2, rexp, cexp = gpu_scale(ctx, bt, PASSES)
    ref = scale_batch(bt, PASSES)
    np.testing.assert_array_equal(A2, np.concatenate([p[2].ravel() for p in ref]))
    np.testing.assert_array_equal(rexp, np.concatenate([p[0] for p in ref]))
    np.testing.assert_array_equal(cexp, np.concatenate([p[1] for p in ref]))
    # Shared constraints: one A, the column factors applied to every c.
    P = W.polytope()
    sb = W.support_batch(P, W.directions(300, seed=55))
    A, b, _, sense = sb.lp(0)
    db = DeviceBatch.shared_from_host(A, b, sense, sb.c.reshape(sb.num_lps, -1))
    print("[gpu] scale shared", flush=True)
    A2, b2, c2, rexp, cexp = (t.cpu().numpy() for t in ctx.scale(db, PASSES))
    torch.cuda.synchronize()
    r, s, As, bs, _ = scale_batch(sb.subset([0]), PASSES)[0]
    np.testing.assert_array_equal(rexp, r)
    np.testing.assert_array_equal(cexp, s)
    np.testing.assert_array_equal(A2, As.ravel())
    np.testing.assert_array_equal(b2, bs)
    np.testing.assert_array_equal(c2.reshape(sb.num_lps, -1), np.ldexp(sb.c.reshape(sb.num_lps, -1), s.astype(np.int32)))


def solve(ctx, bt, **kw):
    import torch
    from paper_1802_08557_amd.lpbatch import DeviceBatch
    print(f"[gpu] solve {bt.name} N={bt.num_lps} {kw}", flush=True)
    sol = ctx.solve(DeviceBatch.from_host(bt), stats=True, **kw)
    torch.cuda.synchronize()
    return (sol.status.cpu().numpy(), sol.x.cpu().numpy(), sol.obj.cpu().numpy(), sol.stats.cpu().numpy())


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("base", ["phase1", "uneven", "uniform"])
def test_scaled_solve_matches_the_oracle(ctx, base, prec):
    bt = {"phase1": lambda: W.phase1_batch(400, 30, 30, seed=56),
          "uneven": lambda: W.uneven_batch(300, seed=57, lo=4, hi=90),
          "uniform": lambda: W.uniform_batch(1000, 50, 50, seed=58)}[base]()
    bt = W.rescaled(bt, seed=59, spread=3.0)
    st, x, obj, _ = solve(ctx, bt, precision=prec, scaling=PASSES)
    ref = solve_scaled(bt, PASSES, threads=8)
    assert_parity(bt, st, obj, x, ref)


def test_scaling_repairs_statuses_of_a_badly_scaled_batch(ctx):
    # Phase I on rows scaled by up to 10^3 either way: the unscaled FP64 solve
    # misjudges some LPs' feasibility (its thresholds are relative to the
    # largest right-hand side); the scaled solve agrees with the LPs as first
    # drawn on every status.
    base = W.phase1_batch(400, 30, 30, seed=60)
    bt = W.rescaled(base, seed=61, spread=3.0)
    truth = oracle_solve(base)
    st_plain = solve(ctx, bt)[0]
    st_scaled = solve(ctx, bt, scaling=PASSES)[0]
    assert (st_scaled == truth.status).sum() >= (st_plain == truth.status).sum()
    assert (st_scaled == truth.status).mean() >= 0.99


def test_scaling_restores_fp64_accuracy(ctx):
    # 50 x 50 LPs with rows and columns scaled by up to 10^3 either way.  Their
    # optimal values are those of the LPs as first drawn (row factors keep the
    # feasible set, column factors only substitute variables), which the
    # oracle solves reliably.  The thresholds of the unscaled simplex
    # (reduced costs against the largest |c_j|, feasibility against the
    # largest |b_i|) ignore columns and rows that were scaled down, so an
    # unscaled solve -- the oracle's as much as the GPU's -- can stop short by
    # up to ~1e-4; with scaling every LP meets the FP64 bar of 1e-9 in both
    # precisions.
    base = W.uniform_batch(2000, 50, 50, seed=62)
    bt = W.rescaled(base, seed=63, spread=3.0)
    truth = oracle_solve(base)
    off = lambda obj: int((np.abs(obj - truth.obj) > 1e-9 * np.maximum(1, np.abs(truth.obj))).sum())
    st0, x0, obj0, s0 = solve(ctx, bt, precision=1)
    assert_parity(bt, st0, obj0, x0, truth, rtol=1e-4, xtol=1e-4)
    counts = {"oracle unscaled": off(oracle_solve(bt).obj), "fp32 unscaled": off(obj0)}
    for prec in (0, 1):
        st1, x1, obj1, s1 = solve(ctx, bt, precision=prec, scaling=PASSES)
        assert_parity(bt, st1, obj1, x1, truth)
        counts[f"{'fp32' if prec else 'fp64'} scaled"] = off(obj1)
    print("LPs beyond 1e-9 of the optimum:", counts)


def test_host_pipeline_with_scaling(ctx):
    bt = W.rescaled(W.uneven_batch(120, seed=64, lo=3, hi=50), seed=65)
    print("[gpu] host solve with scaling", flush=True)
    st, x, obj = ctx.solve_host(bt.A, bt.b, bt.c, bt.sense, bt.m, bt.n, chunk_lps=25, scaling=PASSES)
    dst, dx, dobj, _ = solve(ctx, bt, scaling=PASSES)
    np.testing.assert_array_equal(st, dst)
    np.testing.assert_array_equal(obj, dobj)
    np.testing.assert_array_equal(x, dx)
    assert_parity(bt, st, obj, x, solve_scaled(bt, PASSES))


def test_argument_errors(ctx):
    from paper_1802_08557_amd import lpbatch
    bt = W.uniform_batch(4, 3, 3, seed=66)
    for bad in (-1, 65):
        with pytest.raises(lpbatch.LPBatchError) as ei:
            solve(ctx, bt, scaling=bad)
        assert ei.value.code == lpbatch.LP_ERR_ARG
        with pytest.raises(lpbatch.LPBatchError) as ei:
            gpu_scale(ctx, bt, bad)
        assert ei.value.code == lpbatch.LP_ERR_ARG


def test_shared_and_screened_solves_with_scaling(ctx):
    # Shared constraints: one scaled A, every c scaled by the same column
    # factors, x mapped back per LP; with and without a screened first pass.
    import torch
    from paper_1802_08557_amd.lpbatch import DeviceBatch
    N = 600
    P = W.polytope()
    A1, b1 = W.split_form(P)
    rng = np.random.default_rng(67)
    rf = 10.0 ** rng.uniform(-3, 3, size=A1.shape[0])
    A1, b1 = A1 * rf[:, None], b1 * rf  # badly scaled rows, same polytope
    dirs = W.directions(N, seed=68)
    c = np.concatenate([dirs, -dirs], axis=1)
    m1, n1 = A1.shape
    bt = W.Batch(np.tile(A1.reshape(-1), N), np.tile(b1, N), c.reshape(-1), np.zeros(N * m1, np.int8),
                 np.full(N, m1, np.int32), np.full(N, n1, np.int32), "support_rescaled_rows")
    ref = solve_scaled(bt, PASSES, threads=8)
    db = DeviceBatch.shared_from_host(A1, b1, np.zeros(m1, np.int8), c)
    sub = torch.from_numpy(np.stack([rng.permutation(m1)[:48] for _ in range(N)]).astype(np.int32)).cuda()
    for kw in (dict(precision=0), dict(precision=1, row_subset=sub)):
        print(f"[gpu] shared solve with scaling {list(kw)}", flush=True)
        sol = ctx.solve(db, stats=True, scaling=PASSES, **kw)
        torch.cuda.synchronize()
        assert_parity(bt, sol.status.cpu().numpy(), sol.obj.cpu().numpy(), sol.x.cpu().numpy(), ref)
