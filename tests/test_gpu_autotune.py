"""Workgroup-kernel launches and the autotuner: results stay equal to the
oracle's whatever launch the tuner picks, and the table persists in the
context."""
import numpy as np
import pytest

from helpers import assert_parity, oracle_solve
from paper_1802_08557_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1802_08557_amd import lpbatch
    ctx = lpbatch.Context(0)
    yield torch, lpbatch, ctx
    ctx.close()


def _solve(env, bt, **kw):
    torch, lpbatch, ctx = env
    print(f"[gpu] {bt.name} N={bt.num_lps} {kw}", flush=True)
    db = lpbatch.DeviceBatch.from_host(bt)
    sol = ctx.solve(db, stats=True, **kw)
    torch.cuda.synchronize()
    return sol.status.cpu().numpy(), sol.obj.cpu().numpy(), sol.x.cpu().numpy(), sol.stats.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1])
def test_uneven_batch_autotuned(env, precision):
    torch, lpbatch, ctx = env
    bt = W.uneven_batch(500, seed=77, lo=10, hi=200)
    ref = oracle_solve(bt)
    st, obj, x, stats = _solve(env, bt, precision=precision, autotune=True)
    assert_parity(bt, st, obj, x, ref)
    table = ctx.tuning()
    fp32 = 1 if precision else 0
    mine = [e for e in table if e[1] == fp32]
    assert [e[0] for e in mine] == [4], table  # the one launch of the mixed batch was tuned
    for b, f, nt, hbm in table:
        assert 0 <= b <= 4 and nt in (64, 128, 256, 512) and hbm in (0, 1)
    # The tuned launches, without the flag.
    st2, obj2, x2, _ = _solve(env, bt, precision=precision)
    assert_parity(bt, st2, obj2, x2, ref)


def test_uniform_block_batch_autotuned(env):
    torch, lpbatch, ctx = env
    bt = W.uniform_batch(300, 150, 120, seed=78)
    ref = oracle_solve(bt)
    st, obj, x, stats = _solve(env, bt, autotune=True)
    assert_parity(bt, st, obj, x, ref)
    assert any(e[0] == 2 and e[1] == 0 for e in ctx.tuning())  # (151 x 121 cells: bin 2)
    st2, obj2, x2, _ = _solve(env, bt)
    np.testing.assert_array_equal(st2, st)
    assert_parity(bt, st2, obj2, x2, ref)
