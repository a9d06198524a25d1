"""Geometric-mean scaling with power-of-two factors -- TEST INFRASTRUCTURE.

The paper solves every LP as given (Sec. 4 builds the tableau straight from A,
b and c; no scaling step is part of its method).  This module is the plain
definition of the optional preconditioning the GPU library offers on top, used
only to check it.

Definition (one LP, A of m x n):
  * E_ij = floor(log2 |a_ij|) for every finite non-zero a_ij (the binary
    exponent, read with frexp); zero and non-finite entries take no part;
  * row exponents r_i and column exponents s_j start at 0; each pass sets, for
    every row with a participating entry,
        hi = max_j (E_ij + s_j),  lo = min_j (E_ij + s_j),
        r_i = -floor((hi + lo + 1) / 2)
    (the power of two nearest the geometric mean of the row's largest and
    smallest magnitude, on exponents), then the same for every column with the
    new r_i; rows and columns without participating entries keep 0;
  * every exponent is clamped to [-EXP_CAP, EXP_CAP] when it is set;
  * the scaled LP is a'_ij = a_ij 2^(r_i + s_j), b'_i = b_i 2^r_i,
    c'_j = c_j 2^s_j (same senses); its solution maps back by x_j = x'_j 2^s_j
    and the objective is unchanged.
Multiplying by a power of two is exact, so the scaled LP has exactly the
original's feasible set (up to the map of x) and objective values.
"""
from __future__ import annotations

import numpy as np

EXP_CAP = 128


def _exponents(A):
    """E_ij as int64 and the mask of participating entries."""
    A = np.asarray(A, np.float64)
    ok = np.isfinite(A) & (A != 0)
    _, e = np.frexp(np.where(ok, A, 1.0))
    return e.astype(np.int64) - 1, ok


def _midpoint_exponent(v, ok, axis):
    """-floor((max + min + 1) / 2) over the participating entries along `axis`,
    0 where there are none, clamped to the cap."""
    big = np.int64(1 << 40)
    hi = np.where(ok, v, -big).max(axis=axis)
    lo = np.where(ok, v, big).min(axis=axis)
    out = -np.floor_divide(hi + lo + 1, 2)
    out = np.where(ok.any(axis=axis), out, 0)
    return np.clip(out, -EXP_CAP, EXP_CAP)


def scale_exponents(A, passes: int):
    """Row and column exponents (int64 arrays of m and n) of one LP after
    `passes` row-then-column passes."""
    E, ok = _exponents(A)
    m, n = E.shape
    r = np.zeros(m, np.int64)
    s = np.zeros(n, np.int64)
    for _ in range(passes):
        r = _midpoint_exponent(E + s[None, :], ok, axis=1)
        s = _midpoint_exponent(E + r[:, None], ok, axis=0)
    return r, s


def apply_scaling(A, b, c, r, s):
    """The scaled LP (A', b', c') for exponents r, s."""
    A = np.asarray(A, np.float64)
    return (np.ldexp(A, (r[:, None] + s[None, :]).astype(np.int32)),
            np.ldexp(np.asarray(b, np.float64), r.astype(np.int32)),
            np.ldexp(np.asarray(c, np.float64), s.astype(np.int32)))


def unscale_x(xs, s):
    return np.ldexp(np.asarray(xs, np.float64), s.astype(np.int32))


def scale_batch(batch, passes: int, idx=None):
    """Exponents and scaled data of LPs `idx` (default all) of a Batch.
    Returns a list of (r, s, A', b', c')."""
    idx = range(batch.num_lps) if idx is None else idx
    out = []
    for k in idx:
        A, b, c, _ = batch.lp(k)
        r, s = scale_exponents(A, passes)
        out.append((r, s) + apply_scaling(A, b, c, r, s))
    return out


def solve_scaled(batch, passes: int, **kw):
    """The oracle's answer for a solve with scaling: every LP scaled as above,
    solved by the plain two-phase simplex (``oracle.solve``), x mapped back.
    Status and objective refer to the LP as given."""
    from . import solve
    parts = scale_batch(batch, passes)
    A = np.concatenate([p[2].ravel() for p in parts])
    b = np.concatenate([p[3] for p in parts])
    c = np.concatenate([p[4] for p in parts])
    res = solve(A, b, c, batch.sense, batch.m, batch.n, **kw)
    coff = np.concatenate([[0], np.cumsum(batch.n.astype(np.int64))])
    res.x = np.concatenate([unscale_x(res.x[coff[k]:coff[k + 1]], parts[k][1])
                            for k in range(batch.num_lps)])
    return res
