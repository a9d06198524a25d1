"""Shared test helpers: parity of GPU results against the CPU oracle."""
import numpy as np

import oracle


def oracle_solve(batch, threads=8, **kw):
    return oracle.solve(batch.A, batch.b, batch.c, batch.sense, batch.m, batch.n,
                        threads=threads, **kw)


def _violation(A, b, s, xs):
    """Largest violation of A x {<=,>=,=} b and x >= 0, relative to the LP's scale."""
    r = A @ xs - b
    viol = np.where(s == 0, np.maximum(r, 0), np.where(s == 1, np.maximum(-r, 0), np.abs(r)))
    scale = 1.0 + np.abs(b).max() + np.abs(A).max() * np.abs(xs).max()
    return max(float(viol.max()), float(np.maximum(-xs, 0).max())) / scale


def primal_residual(batch, x, k):
    """Largest violation of A x {<=,>=,=} b and x >= 0 for LP k, relative to 1 + |b|."""
    A, b, c, s = batch.lp(k)
    coff = batch.offsets()[2]
    return _violation(A, b, s, x[coff[k]:coff[k + 1]])


def _uniform_checks(batch, x, idx):
    """Primal residuals and c^T x of the LPs idx of a batch with one shape,
    vectorised: (residual [len(idx)], c^T x [len(idx)])."""
    N, m, n = batch.num_lps, int(batch.m[0]), int(batch.n[0])
    A = batch.A.reshape(N, m, n)[idx]
    b = batch.b.reshape(N, m)[idx]
    c = batch.c.reshape(N, n)[idx]
    s = batch.sense.reshape(N, m)[idx]
    xs = x.reshape(N, n)[idx]
    r = np.einsum("kij,kj->ki", A, xs) - b
    viol = np.where(s == 0, np.maximum(r, 0), np.where(s == 1, np.maximum(-r, 0), np.abs(r)))
    scale = 1.0 + np.abs(b).max(axis=1) + np.abs(A).max(axis=(1, 2)) * np.abs(xs).max(axis=1)
    res = np.maximum(viol.max(axis=1), np.maximum(-xs, 0).max(axis=1)) / scale
    return res, np.einsum("kj,kj->k", c, xs)


def assert_parity(batch, status, obj, x, ref, idx=None, rtol=1e-9, xtol=1e-9):
    """Status equal; objective within rtol * max(1, |z|); every optimal x primal
    feasible with c^T x = obj (so x is optimal given the oracle's z*)."""
    status = np.asarray(status)
    obj = np.asarray(obj)
    x = np.asarray(x)
    idx = np.arange(batch.num_lps) if idx is None else np.asarray(idx, np.int64)
    aoff, roff, coff = batch.offsets()
    bad = []
    st_bad = idx[status[idx] != ref.status[idx]]
    bad += [(int(k), "status", int(status[k]), int(ref.status[k])) for k in st_bad[:5]]
    nbad_status = len(st_bad)
    ok = idx[status[idx] == ref.status[idx]]
    opt = ok[ref.status[ok] == oracle.OPTIMAL]
    z = ref.obj[opt]
    tol = rtol * np.maximum(1.0, np.abs(z))
    obj_bad = opt[~(np.abs(obj[opt] - z) <= tol)]
    bad += [(int(k), "obj", float(obj[k]), float(ref.obj[k])) for k in obj_bad[:5]]
    opt = opt[np.abs(obj[opt] - z) <= tol]
    uniform = batch.num_lps > 0 and np.all(batch.m == batch.m[0]) and np.all(batch.n == batch.n[0])
    if uniform and opt.size:
        res, ctx = _uniform_checks(batch, x, opt)
    else:
        res = np.empty(opt.size)
        ctx = np.empty(opt.size)
        for t, k in enumerate(opt):
            m, n = int(batch.m[k]), int(batch.n[k])
            A = batch.A[aoff[k]:aoff[k + 1]].reshape(m, n)
            xs = x[coff[k]:coff[k + 1]]
            res[t] = _violation(A, batch.b[roff[k]:roff[k + 1]], batch.sense[roff[k]:roff[k + 1]], xs)
            ctx[t] = float(batch.c[coff[k]:coff[k + 1]] @ xs)
    prim_bad = opt[~(res <= xtol)]
    bad += [(int(k), "primal", float(r)) for k, r in zip(prim_bad[:5], res[~(res <= xtol)][:5])]
    ctol = rtol * np.maximum(1.0, np.abs(ref.obj[opt])) * 10
    cx_bad = opt[~(np.abs(ctx - obj[opt]) <= ctol)]
    bad += [(int(k), "c^T x", float(v), float(obj[k]))
            for k, v in zip(cx_bad[:5], ctx[~(np.abs(ctx - obj[opt]) <= ctol)][:5])]
    unb = ok[ref.status[ok] == oracle.UNBOUNDED]
    unb_bad = unb[~(obj[unb] == np.inf)]
    bad += [(int(k), "unbounded obj", float(obj[k])) for k in unb_bad[:5]]
    other = ok[(ref.status[ok] != oracle.OPTIMAL) & (ref.status[ok] != oracle.UNBOUNDED)]
    nan_bad = other[~np.isnan(obj[other])]
    bad += [(int(k), "nan obj", float(obj[k])) for k in nan_bad[:5]]
    nbad = nbad_status + len(obj_bad) + len(prim_bad) + len(cx_bad) + len(unb_bad) + len(nan_bad)
    assert nbad == 0, f"{nbad} mismatches, first: {bad[:5]}"
