"""Repeat solves captured in a HIP graph (through torch.cuda.CUDAGraph) give
the eager results on every replay.  Uniform and shared batches plan without
any host synchronisation, and a batch of mixed sizes reuses the plan an
uncaptured solve of the same shapes left on the device, so one solve call
(several kernels, counters that reset themselves) is capturable once its
buffers exist."""
import numpy as np
import pytest

from paper_1802_08557_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1802_08557_amd import lpbatch
    ctx = lpbatch.Context(0)
    yield torch, lpbatch, ctx
    ctx.close()


def _graph_replays(torch, fn, out, replays=4):
    """Capture fn(out) once, replay it `replays` times with eager work and a
    synchronisation between replays; returns the outputs after each replay."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn(out)  # warm-up on the capture stream: every buffer exists before capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn(out)
    torch.cuda.synchronize()
    got = []
    for r in range(replays):
        for t in (out.status, out.obj, out.x):
            t.fill_(-7)  # eager work between replays; the replay must overwrite it
        g.replay()
        torch.cuda.synchronize()
        got.append((out.status.cpu().numpy().copy(), out.obj.cpu().numpy().copy(), out.x.cpu().numpy().copy()))
    return got


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_uniform(env, precision):
    torch, lpbatch, ctx = env
    bt = W.config1(3000)
    db = lpbatch.DeviceBatch.from_host(bt)
    ref = ctx.solve(db, stats=True, precision=precision)
    torch.cuda.synchronize()
    want = (ref.status.cpu().numpy(), ref.obj.cpu().numpy(), ref.x.cpu().numpy())
    out = ctx.solve(db, stats=True, precision=precision)
    torch.cuda.synchronize()
    fn = lambda o: ctx.solve(db, stats=True, precision=precision, out=o)
    for st, obj, x in _graph_replays(torch, fn, out):
        np.testing.assert_array_equal(st, want[0])
        np.testing.assert_array_equal(obj, want[1])
        np.testing.assert_array_equal(x, want[2])


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_mixed_sizes(env, precision):
    torch, lpbatch, ctx = env
    bt = W.uneven_batch(600, seed=88, lo=10, hi=160)
    db = lpbatch.DeviceBatch.from_host(bt)
    ref = ctx.solve(db, stats=True, precision=precision)
    torch.cuda.synchronize()
    want = (ref.status.cpu().numpy(), ref.obj.cpu().numpy(), ref.x.cpu().numpy())
    st = ref.stats.cpu().numpy()
    assert np.any(st[:, 6] == 1) and np.any(st[:, 6] >= 2)  # both kernels in the graph
    out = ctx.solve(db, stats=True, precision=precision)
    torch.cuda.synchronize()
    fn = lambda o: ctx.solve(db, stats=True, precision=precision, out=o)
    for st, obj, x in _graph_replays(torch, fn, out):
        np.testing.assert_array_equal(st, want[0])
        np.testing.assert_array_equal(obj, want[1])
        np.testing.assert_array_equal(x, want[2])


def test_graph_replay_screened(env):
    torch, lpbatch, ctx = env
    P = W.polytope(1003)
    A1, b1 = W.split_form(P)
    dirs = W.directions(2000, 901)
    c = np.concatenate([dirs, -dirs], axis=1)
    db = lpbatch.DeviceBatch.shared_from_host(A1, b1, np.zeros(120, np.int8), c)
    rng = np.random.default_rng(1)
    sub = torch.from_numpy(np.stack([rng.permutation(120)[:60] for _ in range(2000)]).astype(np.int32)).cuda()
    ref = ctx.solve(db, stats=True, precision=1, row_subset=sub)
    torch.cuda.synchronize()
    want = (ref.status.cpu().numpy(), ref.obj.cpu().numpy(), ref.x.cpu().numpy())
    assert ref.stats.cpu().numpy()[:, 3].sum() > 0  # the re-solve pass is part of the graph
    out = ctx.solve(db, stats=True, precision=1, row_subset=sub)
    torch.cuda.synchronize()
    fn = lambda o: ctx.solve(db, stats=True, precision=1, row_subset=sub, out=o)
    for st, obj, x in _graph_replays(torch, fn, out):
        np.testing.assert_array_equal(st, want[0])
        np.testing.assert_array_equal(obj, want[1])
        np.testing.assert_array_equal(x, want[2])
