"""Shared test helpers: parity of GPU results against the CPU oracle."""
import numpy as np

import oracle


def oracle_solve(batch, threads=8, **kw):
    return oracle.solve(batch.A, batch.b, batch.c, batch.sense, batch.m, batch.n,
                        threads=threads, **kw)


def primal_residual(batch, x, k):
    """Largest violation of A x {<=,>=,=} b and x >= 0 for LP k, relative to 1 + |b|."""
    A, b, c, s = batch.lp(k)
    xs = x[batch.offsets()[2][k]:batch.offsets()[2][k + 1]]
    r = A @ xs - b
    viol = np.where(s == 0, np.maximum(r, 0), np.where(s == 1, np.maximum(-r, 0), np.abs(r)))
    scale = 1.0 + np.abs(b).max() + np.abs(A).max() * np.abs(xs).max()
    return max(float(viol.max()), float(np.maximum(-xs, 0).max())) / scale


def assert_parity(batch, status, obj, x, ref, idx=None, rtol=1e-9, xtol=1e-9):
    """Status equal; objective within rtol * max(1, |z|); every optimal x primal
    feasible with c^T x = obj (so x is optimal given the oracle's z*)."""
    status = np.asarray(status)
    obj = np.asarray(obj)
    x = np.asarray(x)
    idx = range(batch.num_lps) if idx is None else idx
    coff = batch.offsets()[2]
    bad = []
    for k in idx:
        if status[k] != ref.status[k]:
            bad.append((k, "status", int(status[k]), int(ref.status[k])))
            continue
        if ref.status[k] == oracle.OPTIMAL:
            z = ref.obj[k]
            if not abs(obj[k] - z) <= rtol * max(1.0, abs(z)):
                bad.append((k, "obj", float(obj[k]), float(z)))
                continue
            A, b, c, s = batch.lp(k)
            xs = x[coff[k]:coff[k + 1]]
            if primal_residual(batch, x, k) > xtol:
                bad.append((k, "primal", primal_residual(batch, x, k)))
            if not abs(float(c @ xs) - obj[k]) <= rtol * max(1.0, abs(z)) * 10:
                bad.append((k, "c^T x", float(c @ xs), float(obj[k])))
        elif ref.status[k] == oracle.UNBOUNDED:
            if not (obj[k] == np.inf):
                bad.append((k, "unbounded obj", float(obj[k])))
        else:
            if not np.isnan(obj[k]):
                bad.append((k, "nan obj", float(obj[k])))
    assert not bad, f"{len(bad)} mismatches, first: {bad[:5]}"
