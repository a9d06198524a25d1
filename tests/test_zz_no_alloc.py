"""The entry point that allocates nothing (lp_batch_solve_noalloc) against
lp_batch_solve_ex on the same batches, through the C ABI: two calls in a row on
one context, the second on a smaller batch, so the second runs on the scratch
contents the first left behind.  Same kernels, so status, objective and x must
agree bit for bit; both are also checked against the oracle on a sample."""
import numpy as np
import pytest

from helpers import assert_parity, oracle_solve
from paper_1802_08557_amd import workloads as W

pytestmark = pytest.mark.gpu


def _host(sol):
    return sol.status.cpu().numpy(), sol.obj.cpu().numpy(), sol.x.cpu().numpy()


def _same(a, b):
    for u, v in zip(a, b):
        assert u.shape == v.shape
        assert np.array_equal(u, v, equal_nan=True), (u, v)


def test_noalloc_matches_solve_ex_twice():
    import torch
    from paper_1802_08557_amd import lpbatch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = lpbatch.Context(0)
    try:
        # First call: 40 x 40 LPs with >= and = rows (Phase I; LPs whose
        # surplus columns push them past 64 columns go to the workgroup kernel
        # through the deferred list and the static tableau slots).  Second
        # call: fewer, smaller-shaped LPs of the benchmark's distribution.
        batches = [W.phase1_batch(6000, 40, 40, seed=77, frac_ge=0.7, frac_eq=0.1),
                   W.uniform_batch(2500, 50, 50, seed=78)]
        placements = []
        for bt in batches:
            print(f"[gpu] noalloc {bt.name} N={bt.num_lps}", flush=True)
            db = lpbatch.DeviceBatch.from_host(bt)
            ref = ctx.solve(db, stats=True)
            torch.cuda.synchronize()
            got = ctx.solve_noalloc(db, stats=True)
            torch.cuda.synchronize()
            _same(_host(got), _host(ref))
            assert np.array_equal(got.stats.cpu().numpy(), ref.stats.cpu().numpy())
            placements.append(got.stats.cpu().numpy()[:, 6])
            st, obj, x = _host(got)
            oref = oracle_solve(bt, threads=16)
            assert_parity(bt, st, obj, x, oref)
        # The first batch sent LPs through the deferred list to the workgroup
        # kernel; the second ran in the wavefront kernel alone.
        assert np.sum(placements[0] != 1) > 100
        assert np.all(placements[1] == 1)
    finally:
        ctx.close()


def test_noalloc_rejects_what_it_cannot_hold():
    import torch
    from paper_1802_08557_amd import lpbatch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = lpbatch.Context(0)
    try:
        big = lpbatch.DeviceBatch.from_host(W.uniform_batch(4, 50, 80, seed=3))
        with pytest.raises(lpbatch.LPBatchError):
            ctx.solve_noalloc(big)
    finally:
        ctx.close()
