"""FP64 reference of the warm-start scoring network -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg
may use this module; the GPU library shares no code with it.

The network serves the support-function workload of the paper's "Motivating
Application" section: many LPs max l^T x over one fixed polytope, one per
direction l.  It maps l (20 values) to one score per constraint of the
split-form LP (120 constraints: 80 facets, 20 upper and 20 lower box rows);
a high score marks a constraint expected to be tight at the optimum.  The
architecture is 20 -> 256 -> 256 -> 120 with ReLU, BF16 weights and BF16
activations as matrix-product operands, FP32 accumulation (the paper has no
learned component; this is the precision recipe the GPU kernels implement).

Every product and sum here is FP64.  q(.) rounds to bfloat16 at exactly the
points where the kernels feed a matrix product, so the two agree up to
accumulation order:

  forward   X  = q(l)
            Z1 = X q(W1)^T + b1,   H1 = q(relu(Z1))
            Z2 = H1 q(W2)^T + b2,  H2 = q(relu(Z2))
            S  = H2 q(W3)^T + b3                               [B, 120] scores
  loss      L = mean over the B x 120 entries of softplus(S) - Y S
            (binary cross-entropy with logits; Y = 1 for a tight constraint)
  backward  dS  = (sigmoid(S) - Y) / (120 B)
            dW3 = q(dS)^T H2,        db3 = sum_b dS
            dZ2 = (q(dS) q(W3)) * [Z2 > 0]
            dW2 = q(dZ2)^T H1,       db2 = sum_b dZ2
            dZ1 = (q(dZ2) q(W2)) * [Z1 > 0]
            dW1 = q(dZ1)^T X,        db1 = sum_b dZ1
  AdamW     decoupled weight decay (Loshchilov & Hutter) on the FP32 master
            weights; biases are not decayed:
              t += 1; m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2
              w -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps) + lr * wd * w

With ``rounding=False`` q is the identity, the loss is a smooth function of
the weights almost everywhere, and the backward pass is checked against
central finite differences of it.

q rounds an FP64 value first to FP32 (the kernels hold FP32 values) and then
to the nearest bfloat16, ties to even.

Parameters travel as one flat float32 vector in the order
W1 [256, 20], b1 [256], W2 [256, 256], b2 [256], W3 [120, 256], b3 [120]
(102,008 values; weights row-major, output index first).
"""
from __future__ import annotations

import numpy as np

D_IN, D_H, D_OUT = 20, 256, 120
SHAPES = (("W1", (D_H, D_IN)), ("b1", (D_H,)), ("W2", (D_H, D_H)), ("b2", (D_H,)),
          ("W3", (D_OUT, D_H)), ("b3", (D_OUT,)))
NUM_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
WEIGHTS = ("W1", "W2", "W3")


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (via FP32, nearest, ties to even); returns FP64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unflatten(flat) -> dict:
    flat = np.asarray(flat, dtype=np.float64).reshape(-1)
    if flat.size != NUM_PARAMS:
        raise ValueError(f"expected {NUM_PARAMS} parameters, got {flat.size}")
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = flat[o:o + k].reshape(shape).copy()
        o += k
    return out


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def forward(p: dict, l, rounding: bool = True) -> dict:
    """Scores S [B, 120] and the intermediate values the backward pass uses."""
    q = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    X = q(np.asarray(l, dtype=np.float64))
    Z1 = X @ q(p["W1"]).T + p["b1"]
    H1 = q(np.maximum(Z1, 0.0))
    Z2 = H1 @ q(p["W2"]).T + p["b2"]
    H2 = q(np.maximum(Z2, 0.0))
    S = H2 @ q(p["W3"]).T + p["b3"]
    return dict(X=X, Z1=Z1, H1=H1, Z2=Z2, H2=H2, S=S)


def loss(S, Y) -> float:
    """Mean binary cross-entropy with logits over all B x 120 entries."""
    S = np.asarray(S, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    sp = np.maximum(S, 0.0) + np.log1p(np.exp(-np.abs(S)))  # softplus(S)
    return float(np.mean(sp - Y * S))


def backward(p: dict, f: dict, Y, rounding: bool = True) -> dict:
    """Gradients of ``loss`` with respect to every parameter."""
    q = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    S = f["S"]
    B = S.shape[0]
    Y = np.asarray(Y, dtype=np.float64)
    dS = (1.0 / (1.0 + np.exp(-S)) - Y) / (D_OUT * B)
    g = {}
    dSq = q(dS)
    g["W3"] = dSq.T @ f["H2"]
    g["b3"] = dS.sum(axis=0)
    dZ2 = (dSq @ q(p["W3"])) * (f["Z2"] > 0.0)
    dZ2q = q(dZ2)
    g["W2"] = dZ2q.T @ f["H1"]
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2q @ q(p["W2"])) * (f["Z1"] > 0.0)
    dZ1q = q(dZ1)
    g["W1"] = dZ1q.T @ f["X"]
    g["b1"] = dZ1.sum(axis=0)
    return g


def loss_and_grads(flat, l, Y, rounding: bool = True):
    p = unflatten(flat)
    f = forward(p, l, rounding)
    return loss(f["S"], Y), flatten(backward(p, f, Y, rounding))


def adamw(flat, grad, m, v, t, lr, weight_decay, beta1=0.9, beta2=0.999, eps=1e-8):
    """One AdamW step (t = number of the step, starting at 1).  Returns the new
    (params, m, v); weight decay applies to W1, W2, W3 only."""
    w = np.asarray(flat, dtype=np.float64).copy()
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    decay = np.zeros_like(w)
    o = 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        if name in WEIGHTS:
            decay[o:o + k] = 1.0
        o += k
    w = w - lr * mhat / (np.sqrt(vhat) + eps) - lr * weight_decay * decay * w
    return w, m, v


def topk(S, k: int) -> np.ndarray:
    """Indices of the k highest scores per row, highest first; equal scores go
    to the lower index first."""
    S = np.asarray(S)
    order = np.argsort(-S, axis=1, kind="stable")
    return order[:, :k].astype(np.int32)


def tight_mask(A, b, x, tol: float = 1e-9) -> np.ndarray:
    """Training label of an optimum: row i of A x <= b is tight (1) when its
    slack b_i - a_i x is at most tol * (1 + |b_i|).  A [m, n], b [m] shared by
    the batch, x [B, n] optimal points; returns uint8 [B, m]."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).reshape(-1, A.shape[1])
    slack = b[None, :] - x @ A.T
    return (slack <= tol * (1.0 + np.abs(b))[None, :]).astype(np.uint8)
