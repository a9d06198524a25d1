"""GPU parity of the closed-form box LP (Eq. (7)) against the oracle's
hyperbox_max: the maximiser bit for bit, the value within the rounding bound
of an n-term sum."""
import numpy as np
import pytest

from oracle import hyperbox_max
from paper_1802_08557_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1802_08557_amd import lpbatch
    ctx = lpbatch.Context(0)
    yield torch, ctx
    ctx.close()


def _check(val, x, lo, hi, l):
    want, h = hyperbox_max(lo, hi, l)
    np.testing.assert_array_equal(x, np.broadcast_to(h, x.shape))
    n = l.shape[-1]
    bound = 2 * n * np.finfo(np.float64).eps * np.sum(np.abs(l * h), axis=-1)
    assert np.all(np.abs(val - want) <= bound)


@pytest.mark.parametrize("N,n", [(1, 1), (1000, 20), (777, 3), (300, 513)])
def test_per_direction_boxes(env, N, n):
    torch, ctx = env
    lo, hi, l = W.hyperbox_batch(N, n, seed=N + n)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    val, x = ctx.hyperbox_support(t(lo), t(hi), t(l), want_x=True)
    torch.cuda.synchronize()
    _check(val.cpu().numpy(), x.cpu().numpy(), lo, hi, l)


def test_shared_box_support_directions(env):
    torch, ctx = env
    # The support-function use: one box, many directions (some entries exactly 0).
    rng = np.random.default_rng(3)
    n = 20
    lo = -rng.uniform(1, 10, n)
    hi = rng.uniform(1, 10, n)
    l = W.directions(100_000, 1103)
    l[::5, 3] = 0.0
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    val, x = ctx.hyperbox_support(t(lo), t(hi), t(l), want_x=True)
    val2, none = ctx.hyperbox_support(t(lo), t(hi), t(l))
    torch.cuda.synchronize()
    assert none is None
    _check(val.cpu().numpy(), x.cpu().numpy(), lo[None, :], hi[None, :], l)
    np.testing.assert_array_equal(val.cpu().numpy(), val2.cpu().numpy())


def test_empty_and_errors(env):
    torch, ctx = env
    from paper_1802_08557_amd import lpbatch
    z = torch.zeros((0, 4), dtype=torch.float64, device="cuda")
    b = torch.zeros(4, dtype=torch.float64, device="cuda")
    val, _ = ctx.hyperbox_support(b, b, z)
    assert val.numel() == 0
    with pytest.raises(ValueError):
        ctx.hyperbox_support(b, b, torch.zeros((3, 4), dtype=torch.float32, device="cuda"))
