"""Independent checks of the oracle -- TEST INFRASTRUCTURE.

``brute_force``  decides status and optimum of a tiny LP by enumerating the
                 vertices of its feasible region (no simplex involved).
``certificate``  checks an optimal basis by the KKT conditions and strong
                 duality, solving B x_B = b and B^T y = c_B with LAPACK.

LP: maximise c^T x subject to a_i^T x (<=, >=, =) b_i and x >= 0 (paper Sec. 4,
Eq. (1)-(3), widened to three senses).  The region is pointed (x >= 0), so a
feasible LP has a vertex, and it is unbounded exactly when some recession
direction d (d >= 0, A_le d <= 0, A_ge d >= 0, A_eq d = 0) has c^T d > 0.
"""
from __future__ import annotations

import itertools

import numpy as np

LE, GE, EQ = 0, 1, 2
OPTIMAL, INFEASIBLE, UNBOUNDED = 0, 1, 2


def _rows(A, b, sense):
    """Constraints as G x <= g plus equalities E x = e, and x >= 0 as -x <= 0."""
    m, n = A.shape
    G, g, E, e = [], [], [], []
    for i in range(m):
        if sense[i] == LE:
            G.append(A[i]); g.append(b[i])
        elif sense[i] == GE:
            G.append(-A[i]); g.append(-b[i])
        else:
            E.append(A[i]); e.append(b[i])
    for j in range(n):
        r = np.zeros(n); r[j] = -1.0
        G.append(r); g.append(0.0)
    G = np.array(G).reshape(-1, n)
    E = np.array(E).reshape(-1, n)
    return G, np.array(g), E, np.array(e)


def _independent_rows(E):
    """Indices of a maximal linearly independent subset of E's rows (greedy)."""
    keep = []
    for i in range(E.shape[0]):
        if np.linalg.matrix_rank(E[keep + [i]], tol=1e-10) == len(keep) + 1:
            keep.append(i)
    return keep


def _vertices(G, g, E, e, n, tol):
    """All points where n linearly independent constraints are tight (a maximal
    independent subset of the equalities among them) and every constraint,
    every equality included, holds within tol."""
    pts = []
    ind = _independent_rows(E) if E.shape[0] else []
    Ei, ei = E[ind], e[ind]
    ne = len(ind)
    k = n - ne
    if k < 0:
        return pts
    for sub in itertools.combinations(range(G.shape[0]), k):
        M = np.vstack([Ei, G[list(sub)]]) if ne else G[list(sub)]
        r = np.concatenate([ei, g[list(sub)]]) if ne else g[list(sub)]
        if abs(np.linalg.det(M)) < 1e-12 * max(1.0, np.abs(M).max()) ** n:
            continue
        try:
            v = np.linalg.solve(M, r)
        except np.linalg.LinAlgError:
            continue
        scale = 1.0 + np.abs(v).max()
        if np.all(G @ v <= g + tol * scale * (1 + np.abs(g))) and \
                (E.shape[0] == 0 or np.all(np.abs(E @ v - e) <= tol * scale * (1 + np.abs(e)))):
            pts.append(v)
    return pts


def brute_force(A, b, c, sense=None, tol=1e-9):
    """Return (status, z*) of a tiny LP by vertex enumeration.

    The optimum of a feasible bounded LP is attained at a vertex; an infeasible
    LP has no vertex; an unbounded one has a recession direction d >= 0 with
    sum(d) = 1 and c^T d > 0, found the same way on the recession polytope."""
    A = np.asarray(A, float)
    m, n = A.shape
    b = np.asarray(b, float)
    c = np.asarray(c, float)
    sense = np.zeros(m, int) if sense is None else np.asarray(sense, int)
    G, g, E, e = _rows(A, b, sense)
    verts = _vertices(G, g, E, e, n, tol)
    if not verts:
        return INFEASIBLE, float("nan")
    # Recession polytope: G d <= 0, E d = 0, sum(d) = 1.
    E2 = np.vstack([E, np.ones((1, n))]) if E.shape[0] else np.ones((1, n))
    e2 = np.concatenate([np.zeros(E.shape[0]), [1.0]])
    rays = _vertices(G, np.zeros_like(g), E2, e2, n, tol)
    if rays and max(float(c @ d) for d in rays) > tol * (1.0 + np.abs(c).max()):
        return UNBOUNDED, float("inf")
    return OPTIMAL, max(float(c @ v) for v in verts)


def certificate(A, b, c, sense, basis, x, tol=1e-7):
    """Check that ``basis`` (Bland indices per row: j < n structural, n+i the
    slack/surplus of row i, n+m+i the artificial of row i, -1 a dropped row) is
    an optimal basis and ``x`` its vertex.  Returns a dict of the residuals and
    ``ok``; all quantities are recomputed from A, b, c in float64.

    Checks: B x_B = b (the vertex), x >= 0 and A x {<=,>=,=} b (primal
    feasibility), y = B^-T c_B with every reduced cost c_j - y^T a_j <= 0 over
    structurals and logicals (dual feasibility), and c^T x = b^T y (strong
    duality)."""
    A = np.asarray(A, float)
    m, n = A.shape
    b = np.asarray(b, float).copy()
    c = np.asarray(c, float)
    sense = np.asarray(sense, int).copy()
    sgn = np.where(b < 0, -1.0, 1.0)
    flip = (b < 0) & (sense != EQ)
    sense[flip] = np.where(sense[flip] == LE, GE, LE)
    An = A * sgn[:, None]
    bn = b * sgn
    # Full column set of the normalised slack form, indexed by Bland index.
    cols = {}
    for j in range(n):
        cols[j] = An[:, j]
    for i in range(m):
        if sense[i] != EQ:
            v = np.zeros(m); v[i] = 1.0 if sense[i] == LE else -1.0
            cols[n + i] = v
        if sense[i] != LE:
            v = np.zeros(m); v[i] = 1.0
            cols[n + m + i] = v
    alive = [i for i in range(m) if basis[i] >= 0]
    Bidx = [int(basis[i]) for i in alive]
    B = np.stack([cols[k][alive] for k in Bidx], axis=1)
    cB = np.array([c[k] if k < n else 0.0 for k in Bidx])
    xB = np.linalg.solve(B, bn[alive])
    y_alive = np.linalg.solve(B.T, cB)
    y = np.zeros(m); y[alive] = y_alive
    xfull = np.zeros(n)
    for k, v in zip(Bidx, xB):
        if k < n:
            xfull[k] = v
    # Artificials left basic (redundant rows) must sit at zero.
    art_res = max([abs(v) for k, v in zip(Bidx, xB) if k >= n + m] + [0.0])
    bscale = 1.0 + np.abs(b).max()
    cscale = 1.0 + np.abs(c).max()
    r = An @ xfull - bn
    viol = np.where(sense == LE, np.maximum(r, 0), np.where(sense == GE, np.maximum(-r, 0), np.abs(r)))
    primal = max(float(viol.max()), float(np.maximum(-xB, 0).max()), art_res)
    dual = 0.0
    for k, col in cols.items():
        if k >= n + m:
            continue
        ck = c[k] if k < n else 0.0
        dual = max(dual, ck - float(y @ col))
    gap = abs(float(c @ xfull) - float(bn @ y))
    xdiff = float(np.abs(xfull - np.asarray(x, float)).max()) if x is not None else 0.0
    zscale = 1.0 + abs(float(c @ xfull))
    ok = (primal <= tol * bscale * (1 + np.abs(xfull).max()) and dual <= tol * cscale
          and gap <= tol * zscale and xdiff <= tol * (1 + np.abs(xfull).max()))
    return dict(ok=bool(ok), primal=primal, dual=dual, gap=gap, xdiff=xdiff, x=xfull, y=y)


def phase1_certificate(A, b, sense, basis, tol=1e-9):
    """Check that ``basis`` (Bland indices as in ``certificate``) is an optimal
    basis of the Phase I problem -- max -(sum of artificials) over the
    normalised slack form with one artificial per >= and = row (the paper's
    Sec. 4 start) -- whose optimum is negative, i.e. that it proves the LP
    infeasible.  Everything is recomputed from A and b in float64.

    x_B = B^-1 b must be >= 0 (Phase I primal feasibility), y = B^-T c_B with
    c = -1 on artificials and 0 elsewhere must leave the reduced cost
    c_k - y^T a_k <= 0 of every structural and slack / surplus column, and
    w* = c_B^T x_B = b^T y must lie below -tol (1 + |b|_inf).  Then -y is a
    Farkas certificate: -y^T a_j <= 0 for every column of the LP itself and
    -y^T b > 0, so no x >= 0 satisfies the constraints.  Artificial columns
    are not checked: they are not part of the LP, and the method never
    prices an artificial again once it has left the basis.  Returns a dict
    with ``ok``, ``w``, ``primal`` (largest negative x_B), ``dual`` (largest
    reduced cost) and ``y``."""
    A = np.asarray(A, float)
    m, n = A.shape
    b = np.asarray(b, float).copy()
    sense = np.asarray(sense, int).copy()
    sgn = np.where(b < 0, -1.0, 1.0)
    flip = (b < 0) & (sense != EQ)
    sense[flip] = np.where(sense[flip] == LE, GE, LE)
    An = A * sgn[:, None]
    bn = b * sgn
    cols, cost = {}, {}
    for j in range(n):
        cols[j], cost[j] = An[:, j], 0.0
    for i in range(m):
        if sense[i] != EQ:
            v = np.zeros(m); v[i] = 1.0 if sense[i] == LE else -1.0
            cols[n + i], cost[n + i] = v, 0.0
        if sense[i] != LE:
            v = np.zeros(m); v[i] = 1.0
            cols[n + m + i], cost[n + m + i] = v, -1.0
    Bidx = [int(k) for k in basis]
    if len(Bidx) != m or any(k not in cols for k in Bidx) or len(set(Bidx)) != m:
        return dict(ok=False, w=float("nan"), primal=float("inf"), dual=float("inf"), y=None)
    B = np.stack([cols[k] for k in Bidx], axis=1)
    cB = np.array([cost[k] for k in Bidx])
    xB = np.linalg.solve(B, bn)
    y = np.linalg.solve(B.T, cB)
    w = float(cB @ xB)
    primal = float(max(0.0, -xB.min()))
    basic = set(Bidx)
    dual = max([cost[k] - float(y @ col) for k, col in cols.items() if k not in basic and k < n + m] + [0.0])
    scale = 1.0 + np.abs(b).max()
    ok = primal <= tol * scale and dual <= tol * max(1.0, np.abs(An).sum(axis=0).max()) and w < -tol * scale
    return dict(ok=bool(ok), w=w, primal=primal, dual=dual, y=y)
