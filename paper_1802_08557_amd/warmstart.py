"""Learned warm start for batches of LPs over one shared constraint set.

The support-function workload of the paper's "Motivating Application" section
asks max l^T x over one fixed polytope for very many directions l.  The
scoring network (lp_mlp_* in include/lpbatch.h) maps l to one score per
constraint; the k highest-scored constraints of each LP form its screened row
set.  ``warm_solve`` then runs the library's screened solve: each LP is solved
on its screened rows only, its basis is certified in FP64 against every row,
and the LPs whose basis fails are re-solved on all rows in FP64 -- so the
network can only change the speed of a solve, never its result.

Training labels (which constraints are tight at the optimum) come from an
exact solver run by the caller; ``train`` only drives the library's training
kernels over them.  Everything here is orchestration: the network's forward
and backward passes, the optimiser, the top-k and the solves run in the HIP
library.
"""
from __future__ import annotations

import math

import numpy as np

from . import lpbatch


def train(ctx: "lpbatch.Context", dirs, tight, *, epochs: int = 40, batch: int = 512,
          lr: float = 2e-3, lr_final: float = 1e-4, weight_decay: float = 1e-4,
          seed: int = 0, stream=None):
    """Minibatch AdamW training of the context's network.

    dirs: float32 [N, 20] and tight: uint8 [N, 120] device tensors.  Each epoch
    visits the rows in a fresh seeded order; the learning rate follows a cosine
    from ``lr`` to ``lr_final`` over all steps.  Returns the mean loss of each
    epoch (one host synchronisation per epoch)."""
    import torch
    N = int(dirs.shape[0])
    if N < 1 or tight.shape[0] != N:
        raise ValueError("dirs and tight must have the same number of rows")
    rng = np.random.default_rng(seed)
    steps_per_epoch = (N + batch - 1) // batch
    total = epochs * steps_per_epoch
    losses = []
    dev = dirs.device
    step = 0
    loss_buf = torch.zeros(steps_per_epoch, dtype=torch.float32, device=dev)
    for _ in range(epochs):
        perm = torch.from_numpy(rng.permutation(N).astype(np.int64)).to(dev)
        xs = dirs.index_select(0, perm)
        ys = tight.index_select(0, perm)
        for s in range(steps_per_epoch):
            lo, hi = s * batch, min(N, (s + 1) * batch)
            frac = step / max(1, total - 1)
            lr_t = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * frac))
            ctx.mlp_train_step(xs[lo:hi], ys[lo:hi], lr=lr_t, weight_decay=weight_decay,
                               loss=loss_buf[s:s + 1], stream=stream)
            step += 1
        losses.append(float(loss_buf.mean().cpu()))
    return losses


def screen(ctx: "lpbatch.Context", dirs, k: int, stream=None):
    """The k highest-scored constraints of every direction: int32 [N, k]."""
    _, top = ctx.mlp_infer(dirs, k=k, scores=False, stream=stream)
    return top


def warm_solve(ctx: "lpbatch.Context", batch: "lpbatch.DeviceBatch", dirs, k: int, *,
               precision=lpbatch.PREC_FP32_CERT64, **solve_kw):
    """Screened solve of a shared batch whose LP i maximises along dirs[i]."""
    if not batch.shared:
        raise ValueError("warm_solve needs a shared-constraint batch")
    top = screen(ctx, dirs, k, stream=solve_kw.get("stream"))
    return ctx.solve(batch, precision=precision, row_subset=top, **solve_kw)
