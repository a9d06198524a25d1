"""GPU parity of the warm-start network kernels (lp_mlp_*) against the FP64
reference oracle/mlp.py, which applies the same BF16 roundings."""
import os

import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_ctx():
    import torch
    from paper_1802_08557_amd import lpbatch
    ctx = lpbatch.Context(0)
    yield torch, lpbatch, ctx
    ctx.close()


def _params(seed):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in mlp.SHAPES:
        if len(shape) == 2:
            p[name] = rng.uniform(-1, 1, shape) * np.sqrt(6.0 / shape[1])
        else:
            p[name] = rng.uniform(-0.2, 0.2, shape)
    return mlp.flatten(p).astype(np.float32).astype(np.float64)


def _dirs(seed, B):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((B, mlp.D_IN))
    return (g / np.linalg.norm(g, axis=1, keepdims=True)).astype(np.float32)


def _labels(seed, B):
    rng = np.random.default_rng(seed)
    return (rng.uniform(size=(B, mlp.D_OUT)) < 20 / 120).astype(np.uint8)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("B", [1, 37, 1000])
def test_forward_scores_match_oracle(torch_ctx, B):
    torch, lpbatch, ctx = torch_ctx
    flat = _params(1)
    ctx.mlp_set_params(_dev(torch, flat.astype(np.float32)))
    d = _dirs(2 + B, B)
    S, _ = ctx.mlp_infer(_dev(torch, d))
    S = S.cpu().numpy().astype(np.float64)
    ref = mlp.forward(mlp.unflatten(flat), d.astype(np.float64))["S"]
    # FP32 accumulation against FP64, plus a rare BF16 rounding of a hidden
    # activation that lands on the other side of a rounding boundary.
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(S - ref).max() <= 2e-3 * scale
    assert np.linalg.norm(S - ref) <= 1e-4 * np.linalg.norm(ref)


def test_topk_exact_on_device_scores(torch_ctx):
    torch, lpbatch, ctx = torch_ctx
    p = mlp.unflatten(_params(3))
    # Two identical output rows give exactly tied scores: the lower index wins.
    p["W3"][7] = p["W3"][5]
    p["b3"][7] = p["b3"][5]
    flat = mlp.flatten(p).astype(np.float32)
    ctx.mlp_set_params(_dev(torch, flat))
    d = _dirs(4, 513)
    for k in (1, 20, 48, 64, 65, 120):
        S, T = ctx.mlp_infer(_dev(torch, d), k=k)
        S = S.cpu().numpy()
        np.testing.assert_array_equal(S[:, 5], S[:, 7])
        np.testing.assert_array_equal(T.cpu().numpy(), mlp.topk(S, k))
        # The top-k alone (no scores written) is the same.
        _, T2 = ctx.mlp_infer(_dev(torch, d), k=k, scores=False)
        np.testing.assert_array_equal(T2.cpu().numpy(), T.cpu().numpy())


def test_gradients_match_oracle(torch_ctx):
    torch, lpbatch, ctx = torch_ctx
    flat = _params(5)
    ctx.mlp_set_params(_dev(torch, flat.astype(np.float32)))
    B = 300
    d = _dirs(6, B)
    Y = _labels(7, B)
    g, L = ctx.mlp_grads(_dev(torch, d), _dev(torch, Y))
    g = g.cpu().numpy().astype(np.float64)
    L_ref, g_ref = mlp.loss_and_grads(flat, d.astype(np.float64), Y)
    assert float(L.cpu()[0]) == pytest.approx(L_ref, rel=1e-5)
    o = 0
    for name, shape in mlp.SHAPES:
        k = int(np.prod(shape))
        a, r = g[o:o + k], g_ref[o:o + k]
        assert np.linalg.norm(a - r) <= 2e-3 * np.linalg.norm(r), name
        assert np.abs(a - r).max() <= 1e-2 * np.abs(r).max(), name
        o += k
    # Deterministic: the same call gives the same bits.
    g2, L2 = ctx.mlp_grads(_dev(torch, d), _dev(torch, Y))
    np.testing.assert_array_equal(g2.cpu().numpy(), g.astype(np.float32))
    assert float(L2.cpu()[0]) == float(L.cpu()[0])


def test_adamw_step_matches_oracle(torch_ctx):
    torch, lpbatch, ctx = torch_ctx
    flat = _params(8)
    ctx.mlp_set_params(_dev(torch, flat.astype(np.float32)))
    B = 128
    d, Y = _dirs(9, B), _labels(10, B)
    dd, YY = _dev(torch, d), _dev(torch, Y)
    w = flat.copy()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for t in range(1, 4):
        g, _ = ctx.mlp_grads(dd, YY)  # the gradient the step below uses
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        ctx.mlp_train_step(dd, YY, lr=1e-3, weight_decay=0.05, loss=loss)
        w, m, v = mlp.adamw(w, g.cpu().numpy().astype(np.float64), m, v, t, lr=1e-3, weight_decay=0.05)
        got = ctx.mlp_get_params().cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(got, w, rtol=0, atol=1e-6 * max(1.0, np.abs(w).max()))
        w = got  # continue from the device's FP32 values


def test_training_lowers_loss_and_save_load(torch_ctx, tmp_path):
    torch, lpbatch, ctx = torch_ctx
    import oracle
    from paper_1802_08557_amd import workloads as W
    P = W.polytope(1003)
    A1, b1 = W.split_form(P)
    dirs = W.directions(2048, 4242)
    bt = W.support_batch(P, dirs)
    r = oracle.solve(bt.A, bt.b, bt.c, bt.sense, bt.m, bt.n, threads=8)
    Y = mlp.tight_mask(A1, b1, r.x.reshape(-1, 40))
    dd = _dev(torch, dirs.astype(np.float32))
    YY = _dev(torch, Y)
    ctx.mlp_init(1234)
    first = torch.zeros(1, dtype=torch.float32, device="cuda")
    ctx.mlp_train_step(dd[:256], YY[:256], lr=2e-3, loss=first)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    for step in range(300):
        lo = (step * 256) % 2048
        ctx.mlp_train_step(dd[lo:lo + 256], YY[lo:lo + 256], lr=2e-3, weight_decay=1e-4, loss=loss)
    _, L_end = ctx.mlp_grads(dd, YY)
    assert float(L_end.cpu()[0]) < 0.6 * float(first.cpu()[0])
    path = os.path.join(str(tmp_path), "net.bin")
    ctx.mlp_save(path)
    S1, T1 = ctx.mlp_infer(dd, k=20)
    ctx2 = lpbatch.Context(0)
    try:
        ctx2.mlp_load(path)
        S2, T2 = ctx2.mlp_infer(dd, k=20)
        np.testing.assert_array_equal(S1.cpu().numpy(), S2.cpu().numpy())
        np.testing.assert_array_equal(T1.cpu().numpy(), T2.cpu().numpy())
    finally:
        ctx2.close()


def test_mlp_argument_errors(torch_ctx):
    torch, lpbatch, ctx = torch_ctx
    fresh = lpbatch.Context(0)
    try:
        d = _dev(torch, _dirs(11, 4))
        with pytest.raises(lpbatch.LPBatchError):
            fresh.mlp_infer(d, k=5)  # no parameters yet
        fresh.mlp_init(1)
        with pytest.raises(lpbatch.LPBatchError):
            fresh.mlp_infer(d, k=121)
    finally:
        fresh.close()
