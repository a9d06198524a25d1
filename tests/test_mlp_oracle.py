"""Pins of the FP64 warm-start network reference (oracle/mlp.py) against
independent implementations: torch's bfloat16 conversion, torch autograd,
torch's AdamW, central finite differences and the closed forms of the loss."""
import numpy as np
import pytest
import torch

from oracle import mlp


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in mlp.SHAPES:
        fan_in = shape[1] if len(shape) == 2 else 256
        p[name] = rng.uniform(-1, 1, shape) * scale * np.sqrt(6.0 / fan_in) if len(shape) == 2 \
            else rng.uniform(-0.1, 0.1, shape)
    return p


def _data(seed, B):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((B, mlp.D_IN))
    l = g / np.linalg.norm(g, axis=1, keepdims=True)
    Y = (rng.uniform(size=(B, mlp.D_OUT)) < 20 / 120).astype(np.uint8)
    return l, Y


def test_num_params():
    assert mlp.NUM_PARAMS == 102_008


def test_bf16_matches_torch_rounding():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 65504.0]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), ref)
    # Ties go to even: 1 + 2^-8 sits halfway between 1 and 1 + 2^-7.
    assert mlp.bf16(1.0 + 2 ** -8) == 1.0
    assert mlp.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6


def test_forward_matches_torch_without_rounding():
    p = _params(1)
    l, _ = _data(2, 64)
    S = mlp.forward(p, l, rounding=False)["S"]
    net = torch.nn.Sequential(torch.nn.Linear(20, 256), torch.nn.ReLU(), torch.nn.Linear(256, 256),
                              torch.nn.ReLU(), torch.nn.Linear(256, 120)).double()
    with torch.no_grad():
        for i, (w, b) in enumerate((("W1", "b1"), ("W2", "b2"), ("W3", "b3"))):
            net[2 * i].weight.copy_(torch.tensor(p[w]))
            net[2 * i].bias.copy_(torch.tensor(p[b]))
        ref = net(torch.tensor(l)).numpy()
    np.testing.assert_allclose(S, ref, rtol=1e-12, atol=1e-12)


def test_forward_rounding_error_is_bf16_sized():
    p = _params(3)
    l, _ = _data(4, 256)
    S_r = mlp.forward(p, l, rounding=True)["S"]
    S_x = mlp.forward(p, l, rounding=False)["S"]
    # A few bf16 roundings (relative 2^-9 each) per layer: well below 5 %.
    err = np.abs(S_r - S_x).max() / np.abs(S_x).max()
    assert 1e-5 < err < 5e-2


def test_loss_closed_forms_and_torch():
    S = np.zeros((3, 120))
    assert mlp.loss(S, np.ones((3, 120))) == pytest.approx(np.log(2.0), rel=1e-15)
    assert mlp.loss(np.full((1, 120), 40.0), np.ones((1, 120))) < 1e-17
    assert mlp.loss(np.full((1, 120), -40.0), np.ones((1, 120))) == pytest.approx(40.0, rel=1e-12)
    rng = np.random.default_rng(5)
    S = rng.standard_normal((17, 120)) * 5
    Y = (rng.uniform(size=(17, 120)) < 0.3).astype(np.float64)
    ref = torch.nn.functional.binary_cross_entropy_with_logits(torch.tensor(S), torch.tensor(Y)).item()
    assert mlp.loss(S, Y) == pytest.approx(ref, rel=1e-13)


def test_backward_matches_torch_autograd_without_rounding():
    p = _params(6)
    l, Y = _data(7, 32)
    L, g = mlp.loss_and_grads(mlp.flatten(p), l, Y, rounding=False)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}
    X = torch.tensor(l)
    h = torch.relu(X @ tp["W1"].T + tp["b1"])
    h = torch.relu(h @ tp["W2"].T + tp["b2"])
    S = h @ tp["W3"].T + tp["b3"]
    Lt = torch.nn.functional.binary_cross_entropy_with_logits(S, torch.tensor(Y, dtype=torch.float64))
    Lt.backward()
    assert L == pytest.approx(Lt.item(), rel=1e-13)
    ref = np.concatenate([tp[name].grad.numpy().reshape(-1) for name, _ in mlp.SHAPES])
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-15)


def test_backward_matches_finite_differences():
    p = _params(8)
    l, Y = _data(9, 8)
    flat = mlp.flatten(p)
    _, g = mlp.loss_and_grads(flat, l, Y, rounding=False)
    rng = np.random.default_rng(10)
    # A sample of coordinates from every parameter block.
    idx, o = [], 0
    for _, shape in mlp.SHAPES:
        k = int(np.prod(shape))
        idx.extend(o + rng.choice(k, size=8, replace=False))
        o += k
    h = 1e-6
    for i in idx:
        fp = flat.copy(); fp[i] += h
        fm = flat.copy(); fm[i] -= h
        fd = (mlp.loss_and_grads(fp, l, Y, False)[0] - mlp.loss_and_grads(fm, l, Y, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-4, abs(g[i])) + 1e-10, (i, fd, g[i])


def test_backward_with_rounding_stays_close():
    # The mixed-precision gradient differs from the exact one only by bf16
    # roundings of the operands.
    p = _params(11)
    l, Y = _data(12, 64)
    _, g_r = mlp.loss_and_grads(mlp.flatten(p), l, Y, rounding=True)
    _, g_x = mlp.loss_and_grads(mlp.flatten(p), l, Y, rounding=False)
    assert np.linalg.norm(g_r - g_x) / np.linalg.norm(g_x) < 5e-2


def test_adamw_matches_torch():
    p = _params(13)
    flat = mlp.flatten(p)
    rng = np.random.default_rng(14)
    tp = [torch.tensor(p[name], requires_grad=True) for name, _ in mlp.SHAPES]
    opt = torch.optim.AdamW([{"params": [tp[0], tp[2], tp[4]], "weight_decay": 0.01},
                             {"params": [tp[1], tp[3], tp[5]], "weight_decay": 0.0}],
                            lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(flat)
    v = np.zeros_like(flat)
    for t in range(1, 4):
        g = rng.standard_normal(flat.size) * 1e-3
        flat, m, v = mlp.adamw(flat, g, m, v, t, lr=3e-3, weight_decay=0.01)
        o = 0
        for i, (_, shape) in enumerate(mlp.SHAPES):
            k = int(np.prod(shape))
            tp[i].grad = torch.tensor(g[o:o + k].reshape(shape))
            o += k
        opt.step()
    ref = np.concatenate([x.detach().numpy().reshape(-1) for x in tp])
    np.testing.assert_allclose(flat, ref, rtol=1e-12, atol=1e-15)


def test_topk_ties_and_order():
    S = np.array([[1.0, 3.0, 3.0, 2.0, 3.0, -1.0]])
    np.testing.assert_array_equal(mlp.topk(S, 4), [[1, 2, 4, 3]])
    rng = np.random.default_rng(15)
    S = rng.integers(0, 5, (50, 120)).astype(np.float64)  # many ties
    for row, got in zip(S, mlp.topk(S, 20)):
        want = sorted(range(120), key=lambda i: (-row[i], i))[:20]
        assert list(got) == want


def test_tight_mask_on_support_lps():
    import oracle
    from paper_1802_08557_amd import workloads as W
    P = W.polytope(1003)
    A1, b1 = W.split_form(P)
    dirs = W.directions(200, 77)
    bt = W.support_batch(P, dirs)
    r = oracle.solve(bt.A, bt.b, bt.c, bt.sense, bt.m, bt.n, threads=4)
    assert np.all(r.status == oracle.OPTIMAL)
    tight = mlp.tight_mask(A1, b1, r.x.reshape(200, 40))
    # A vertex of the 20-dimensional polytope: 20 tight constraints, and the
    # tight rows' slacks are exactly the non-basic ones of the optimal basis.
    assert np.all(tight.sum(axis=1) == 20)
    basis = r.basis.reshape(200, 120)
    for k in range(200):
        basic_slack = set(int(v) - 40 for v in basis[k] if 40 <= v < 160)
        assert set(np.where(tight[k] == 0)[0]) == basic_slack
