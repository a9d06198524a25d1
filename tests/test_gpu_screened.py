"""GPU parity of shared-constraint and screened solves (lp_options.shared,
row_subset) against the CPU oracle on the full LPs.

A screened solve first solves each LP on a subset of its rows (a relaxation),
then certifies the basis in FP64 against every row and re-solves the LPs whose
basis fails.  Whatever the subsets, every result must equal the oracle's on
the full LP; good subsets must pass the certificate without a re-solve."""
import numpy as np
import pytest

import oracle
from helpers import assert_parity, oracle_solve
from oracle import mlp
from paper_1802_08557_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1802_08557_amd import lpbatch
    ctx = lpbatch.Context(0)
    yield torch, lpbatch, ctx
    ctx.close()


def _support(N, seed, facets=80, box=True):
    P = W.polytope(1003, facets=facets)
    dirs = W.directions(N, seed)
    A1, b1 = W.split_form(P)
    if not box:
        A1, b1 = A1[:facets], b1[:facets]
    c = np.concatenate([dirs, -dirs], axis=1)
    bt = W.Batch(np.tile(A1.reshape(-1), N), np.tile(b1, N), c.reshape(-1),
                 np.zeros(N * A1.shape[0], np.int8), np.full(N, A1.shape[0], np.int32),
                 np.full(N, A1.shape[1], np.int32), f"support_{A1.shape[0]}x{A1.shape[1]}_x{N}")
    return A1, b1, np.zeros(A1.shape[0], np.int8), c, bt


def _solve(env, A1, b1, s1, c, subset=None, **kw):
    torch, lpbatch, ctx = env
    db = lpbatch.DeviceBatch.shared_from_host(A1, b1, s1, c)
    rs = None if subset is None else torch.from_numpy(np.ascontiguousarray(subset, np.int32)).cuda()
    print(f"[gpu] shared solve N={c.shape[0]} m={A1.shape[0]} subset="
          f"{None if subset is None else subset.shape[1]} {kw}", flush=True)
    sol = ctx.solve(db, stats=True, row_subset=rs, **kw)
    torch.cuda.synchronize()
    return (sol.status.cpu().numpy(), sol.obj.cpu().numpy(), sol.x.cpu().numpy(),
            sol.stats.cpu().numpy())


def test_shared_equals_replicated(env):
    torch, lpbatch, ctx = env
    A1, b1, s1, c, bt = _support(1500, 501)
    st, obj, x, stats = _solve(env, A1, b1, s1, c)
    db = lpbatch.DeviceBatch.from_host(bt)
    sol = ctx.solve(db, stats=True)
    torch.cuda.synchronize()
    # Same kernel, same data, same arithmetic: bitwise equal results.
    np.testing.assert_array_equal(st, sol.status.cpu().numpy())
    np.testing.assert_array_equal(obj, sol.obj.cpu().numpy())
    np.testing.assert_array_equal(x, sol.x.cpu().numpy())
    assert_parity(bt, st, obj, x, oracle_solve(bt))


@pytest.mark.parametrize("precision", [0, 1])
def test_screened_with_tight_rows_passes_certificate(env, precision):
    A1, b1, s1, c, bt = _support(1500, 502)
    ref = oracle_solve(bt)
    tight = mlp.tight_mask(A1, b1, ref.x.reshape(-1, 40))
    rng = np.random.default_rng(5)
    K = 40
    sub = np.empty((bt.num_lps, K), np.int32)
    for k in range(bt.num_lps):
        t = np.where(tight[k])[0]
        rest = rng.permutation(np.setdiff1d(np.arange(120), t))[:K - t.size]
        sub[k] = rng.permutation(np.concatenate([t, rest]))
    st, obj, x, stats = _solve(env, A1, b1, s1, c, sub, precision=precision)
    assert_parity(bt, st, obj, x, ref)
    assert np.all(stats[:, 3] == 0), "a relaxation containing every tight row needs no re-solve"
    assert np.all((stats[:, 5] & 3) == 3)


@pytest.mark.parametrize("K", [20, 30, 60])
def test_screened_random_rows_falls_back(env, K):
    A1, b1, s1, c, bt = _support(1200, 503 + K)
    ref = oracle_solve(bt)
    rng = np.random.default_rng(K)
    sub = np.stack([rng.permutation(120)[:K] for _ in range(bt.num_lps)]).astype(np.int32)
    st, obj, x, stats = _solve(env, A1, b1, s1, c, sub, precision=1)
    assert_parity(bt, st, obj, x, ref)
    assert stats[:, 3].sum() > 0  # random rows miss the tight set
    # Every certified LP's relaxation optimum is feasible for the full LP.
    ok = stats[:, 3] == 0
    assert np.all((stats[ok, 5] & 3) == 3)


def test_screened_identity_subset_equals_full(env):
    A1, b1, s1, c, bt = _support(800, 504)
    st0, obj0, x0, _ = _solve(env, A1, b1, s1, c, precision=1)
    sub = np.tile(np.arange(120, dtype=np.int32), (bt.num_lps, 1))
    st, obj, x, stats = _solve(env, A1, b1, s1, c, sub, precision=1)
    np.testing.assert_array_equal(st, st0)
    np.testing.assert_array_equal(obj, obj0)
    assert_parity(bt, st, obj, x, oracle_solve(bt))


def test_screened_unbounded_family(env):
    # 35 facets and no box in R^20: about nine directions in ten are unbounded.
    # Screened relaxations are unbounded more often still; the ray certificate
    # against every row decides, and the re-solve settles the rest.
    A1, b1, s1, c, bt = _support(1000, 505, facets=35, box=False)
    ref = oracle_solve(bt)
    frac = float(np.mean(ref.status == oracle.UNBOUNDED))
    assert 0.5 < frac < 0.99, frac
    rng = np.random.default_rng(6)
    sub = np.stack([rng.permutation(35)[:30] for _ in range(bt.num_lps)]).astype(np.int32)
    st, obj, x, stats = _solve(env, A1, b1, s1, c, sub, precision=1)
    assert_parity(bt, st, obj, x, ref)
    # Some unbounded LPs are settled by the relaxation's ray alone.
    assert np.any((st == oracle.UNBOUNDED) & (stats[:, 3] == 0) & ((stats[:, 5] & 4) != 0))


def test_screened_mixed_senses(env):
    # Shared constraints with >= and = rows (Phase I in every LP).
    rng = np.random.default_rng(7)
    m, n, N = 30, 25, 800
    A1 = rng.uniform(1, 10, (m, n))
    x0 = rng.uniform(0, 1, n)
    s1 = np.zeros(m, np.int8)
    s1[:6] = W.GE
    s1[6:9] = W.EQ
    b1 = A1 @ x0 + np.where(s1 == W.LE, rng.uniform(1, 20, m), np.where(s1 == W.GE, -rng.uniform(1, 5, m), 0.0))
    c = rng.uniform(-1, 10, (N, n))
    bt = W.Batch(np.tile(A1.reshape(-1), N), np.tile(b1, N), c.reshape(-1), np.tile(s1, N),
                 np.full(N, m, np.int32), np.full(N, n, np.int32), "shared_mixed")
    ref = oracle_solve(bt)
    assert np.all(ref.status == oracle.OPTIMAL)
    sub = np.stack([np.sort(rng.permutation(m)[:22]) for _ in range(N)]).astype(np.int32)
    for prec in (0, 1):
        st, obj, x, stats = _solve(env, A1, b1, s1, c, sub, precision=prec)
        assert_parity(bt, st, obj, x, ref)
    st, obj, x, stats = _solve(env, A1, b1, s1, c)
    assert_parity(bt, st, obj, x, ref)


def test_screened_bad_indices_resolved(env):
    A1, b1, s1, c, bt = _support(300, 506)
    ref = oracle_solve(bt)
    rng = np.random.default_rng(8)
    sub = np.stack([rng.permutation(120)[:40] for _ in range(bt.num_lps)]).astype(np.int32)
    sub[::7, 3] = -1
    sub[1::7, 5] = 120
    st, obj, x, stats = _solve(env, A1, b1, s1, c, sub, precision=1)
    assert_parity(bt, st, obj, x, ref)
    assert np.all(stats[::7, 3] == 1) and np.all(stats[1::7, 3] == 1)


def test_shared_argument_errors(env):
    torch, lpbatch, ctx = env
    A1, b1, s1, c, bt = _support(10, 507)
    db = lpbatch.DeviceBatch.shared_from_host(A1, b1, s1, c)
    with pytest.raises(lpbatch.LPBatchError):
        ctx.solve(db, row_subset=torch.zeros((10, 121), dtype=torch.int32, device="cuda"))
    db2 = lpbatch.DeviceBatch.from_host(bt)
    with pytest.raises(lpbatch.LPBatchError):  # row_subset without shared
        ctx.solve(db2, row_subset=torch.zeros((10, 5), dtype=torch.int32, device="cuda"))
    db.m = db.m.copy()
    db.m[3] = 119
    with pytest.raises(lpbatch.LPBatchError):  # shared needs equal sizes
        ctx.solve(db)


def test_screened_repair_from_relaxation_basis(env):
    # Subsets that hold every tight row but one: the relaxation's optimum
    # violates the missing row, the certificate rejects it, and the FP64
    # re-solve starts from the relaxation's basis (its structurals pivoted in,
    # then dual simplex pivots) instead of the slack basis, and still matches
    # the oracle.  The box rows (80..119) keep every relaxation bounded.
    A1, b1, s1, c, bt = _support(1500, 505)
    ref = oracle_solve(bt)
    tight = mlp.tight_mask(A1, b1, ref.x.reshape(-1, 40))
    rng = np.random.default_rng(6)
    K = 64
    sub = np.empty((bt.num_lps, K), np.int32)
    for k in range(bt.num_lps):
        tk = np.where(tight[k])[0]
        t = rng.permutation(tk)[1:]  # drop one tight row
        box = np.setdiff1d(np.arange(80, 120), tk)
        rest = rng.permutation(np.setdiff1d(np.arange(80), tk))[:K - t.size - box.size]
        sub[k] = rng.permutation(np.concatenate([t, box, rest]))
    st, obj, x, stats = _solve(env, A1, b1, s1, c, sub, precision=1)
    assert_parity(bt, st, obj, x, ref)
    fb = stats[:, 3] >= 1
    assert fb.sum() > 100, fb.sum()
    # Most are repaired from the relaxation's basis rather than re-solved from
    # the slack basis (a relaxation optimum that violates more than 16 rows
    # goes to the slack-basis solve).
    assert np.mean(stats[fb, 3] == 2) > 0.3, np.bincount(stats[fb, 3])


def test_full_size_support_batch_warm_and_plain(env):
    # The benchmarked configuration at its full size (1e5 directions over the
    # 120 x 40 polytope), in the launch configuration bench.py times: plain
    # FP64, FP32 + certificate, and the network-screened solve (network
    # trained briefly here); a sample of 4,000 LPs is checked against the
    # oracle one by one, and every LP's status must agree across the modes.
    torch, lpbatch, ctx = env
    from paper_1802_08557_amd import warmstart
    P = W.polytope(1003)
    A1, b1 = W.split_form(P)
    s1 = np.zeros(A1.shape[0], np.int8)
    dirs = W.directions(100_000, 1103)
    c = np.concatenate([dirs, -dirs], axis=1)
    db = lpbatch.DeviceBatch.shared_from_host(A1, b1, s1, c)
    tr = W.directions(40_000, 1203)
    bt_tr = W.support_batch(P, tr)
    r_tr = oracle.solve(bt_tr.A, bt_tr.b, bt_tr.c, bt_tr.sense, bt_tr.m, bt_tr.n, threads=8)
    Y = mlp.tight_mask(A1, b1, r_tr.x.reshape(-1, 40))
    net = lpbatch.Context(0)
    net.mlp_init(7)
    print("[gpu] train 8 epochs on 40k directions", flush=True)
    warmstart.train(net, torch.from_numpy(tr.astype(np.float32)).cuda(), torch.from_numpy(Y).cuda(),
                    epochs=8, seed=11)
    top = warmstart.screen(net, torch.from_numpy(dirs.astype(np.float32)).cuda(), 48)
    results = {}
    for name, kw in [("plain", {}), ("fp32c", dict(precision=1)), ("warm", dict(precision=1, row_subset=top))]:
        print(f"[gpu] full-size support batch: {name}", flush=True)
        sol = ctx.solve(db, stats=True, **kw)
        torch.cuda.synchronize()
        results[name] = (sol.status.cpu().numpy(), sol.obj.cpu().numpy(), sol.x.cpu().numpy())
    net.close()
    idx = np.random.default_rng(7).choice(100_000, 4000, replace=False)
    sample = W.support_batch(P, dirs[idx])
    ref = oracle_solve(sample)
    for name, (st, obj, x) in results.items():
        xs = x.reshape(-1, 40)[idx].reshape(-1)
        assert_parity(sample, st[idx], obj[idx], xs, ref)
        np.testing.assert_array_equal(st, results["plain"][0])
