"""Seeded synthetic LP batches.

This module only draws random numbers and lays them out; it holds none of the
solver's arithmetic.  Both the GPU path and the CPU oracle are fed from it.

Layout of a batch (``Batch``): LPs stored back to back --
  A      float64 [sum_k m_k * n_k]   row-major m_k x n_k block of LP k
  b      float64 [sum_k m_k]
  c      float64 [sum_k n_k]         (maximise c^T x)
  sense  int8    [sum_k m_k]         0: <=, 1: >=, 2: =
  m, n   int32   [N]

Workloads (the paper's evaluation uses random dense LPs with A, b, c drawn
uniformly, Sec. 6, "dimension d" = d constraints x d variables; its Netlib and
reachability experiments need data that is not available, and these seeded
batches stand in for them):
  uniform_batch   A ~ U[1,10], b ~ U[100,1000], c ~ U[1,10], all <=: the origin
                  is feasible and every x_j is bounded, so every LP is OPTIMAL.
                  5x5 x 1e3 (seed 1000), 50x50 x 1e5 (seed 1001),
                  500x500 x 1e3 (seed 1004).
  uneven_batch    m, n ~ U{10..300}, A ~ N(0,1), 30 % of the rows >= with
                  b ~ U[-50,-1], the rest <= with b ~ U[1,100], c ~ U[-1,10];
                  5 % made infeasible (row x1 + x2 <= -1 appended) and a
                  disjoint 5 % made unbounded (a zero column with c_j > 0).
  support_batch   a fixed polytope {x in R^20 : G x <= h, -10 <= x <= 10}
                  (G rows ~ N(0,I) normalised, h ~ 1 + U[0,1]) queried in
                  directions l uniform on the unit sphere; x = x+ - x- splits
                  the free variable so every LP is in the x >= 0 form.
  phase1_batch    test-only: feasible LPs whose >= rows have a positive rhs,
                  so Phase I is needed and succeeds.
  rescaled        test-only: any batch with rows and columns multiplied by
                  random powers of ten (badly scaled, same optima).
Batch-sized draws use numpy's PCG64 in chunks of 10,000 LPs, each chunk from
``SeedSequence(seed).spawn(ceil(N / 1e4))``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CHUNK = 10_000
LE, GE, EQ = 0, 1, 2


@dataclass
class Batch:
    A: np.ndarray
    b: np.ndarray
    c: np.ndarray
    sense: np.ndarray
    m: np.ndarray
    n: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def num_lps(self) -> int:
        return int(self.m.shape[0])

    def offsets(self):
        m = self.m.astype(np.int64)
        n = self.n.astype(np.int64)
        aoff = np.concatenate([[0], np.cumsum(m * n)])
        roff = np.concatenate([[0], np.cumsum(m)])
        coff = np.concatenate([[0], np.cumsum(n)])
        return aoff, roff, coff

    def lp(self, k: int):
        """(A [m,n], b, c, sense) of LP k, as views."""
        aoff, roff, coff = self.offsets()
        m, n = int(self.m[k]), int(self.n[k])
        return (self.A[aoff[k]:aoff[k + 1]].reshape(m, n), self.b[roff[k]:roff[k + 1]],
                self.c[coff[k]:coff[k + 1]], self.sense[roff[k]:roff[k + 1]])

    def subset(self, idx) -> "Batch":
        idx = np.asarray(idx, dtype=np.int64)
        parts = [self.lp(int(k)) for k in idx]
        return Batch(np.concatenate([p[0].ravel() for p in parts]) if parts else np.zeros(0),
                     np.concatenate([p[1] for p in parts]) if parts else np.zeros(0),
                     np.concatenate([p[2] for p in parts]) if parts else np.zeros(0),
                     np.concatenate([p[3] for p in parts]).astype(np.int8) if parts else np.zeros(0, np.int8),
                     self.m[idx].copy(), self.n[idx].copy(), self.name + "[subset]", dict(self.meta))


def _chunks(N, seed):
    nchunk = max(1, -(-N // CHUNK))
    for ci, ss in enumerate(np.random.SeedSequence(seed).spawn(nchunk)):
        lo = ci * CHUNK
        yield lo, min(N, lo + CHUNK), np.random.default_rng(ss)


def uniform_batch(N: int, m: int, n: int, seed: int, name: str = "") -> Batch:
    """A ~ U[1,10], b ~ U[100,1000], c ~ U[1,10], all rows <=."""
    A = np.empty((N, m, n), np.float64)
    b = np.empty((N, m), np.float64)
    c = np.empty((N, n), np.float64)
    for lo, hi, rng in _chunks(N, seed):
        k = hi - lo
        A[lo:hi] = rng.uniform(1.0, 10.0, size=(k, m, n))
        b[lo:hi] = rng.uniform(100.0, 1000.0, size=(k, m))
        c[lo:hi] = rng.uniform(1.0, 10.0, size=(k, n))
    return Batch(A.reshape(-1), b.reshape(-1), c.reshape(-1), np.zeros(N * m, np.int8),
                 np.full(N, m, np.int32), np.full(N, n, np.int32),
                 name or f"uniform_{m}x{n}_x{N}", dict(seed=seed))


def config0(N: int = 1000, seed: int = 1000) -> Batch:
    return uniform_batch(N, 5, 5, seed, "uniform_5x5")


def config1(N: int = 100_000, seed: int = 1001) -> Batch:
    return uniform_batch(N, 50, 50, seed, "uniform_50x50")


def config4(N: int = 1000, seed: int = 1004) -> Batch:
    return uniform_batch(N, 500, 500, seed, "uniform_500x500")


def uneven_batch(N: int = 10_000, seed: int = 1002, lo: int = 10, hi: int = 300,
                 frac_infeasible: float = 0.05, frac_unbounded: float = 0.05) -> Batch:
    """m, n ~ U{lo..hi}; A ~ N(0,1); round(0.3 m) rows (by permutation) are >=
    with b ~ U[-50,-1], the rest <= with b ~ U[1,100]; c ~ U[-1,10].  Then a
    permutation of the LPs picks the infeasible injections (row x1 + x2 <= -1
    appended) and a disjoint set of unbounded injections (column j zeroed,
    c_j ~ U[1,10])."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    lps = []
    for _ in range(N):
        m = int(rng.integers(lo, hi + 1))
        n = int(rng.integers(lo, hi + 1))
        A = rng.standard_normal((m, n))
        perm = rng.permutation(m)
        ge = np.zeros(m, bool)
        ge[perm[:int(round(0.3 * m))]] = True
        b = np.where(ge, rng.uniform(-50.0, -1.0, m), rng.uniform(1.0, 100.0, m))
        c = rng.uniform(-1.0, 10.0, n)
        sense = np.where(ge, GE, LE).astype(np.int8)
        lps.append([A, b, c, sense])
    order = rng.permutation(N)
    n_inf = int(round(frac_infeasible * N))
    n_unb = int(round(frac_unbounded * N))
    inf_set = order[:n_inf]
    unb_set = order[n_inf:n_inf + n_unb]
    for k in inf_set:
        A, b, c, sense = lps[k]
        row = np.zeros(A.shape[1]); row[0] = 1.0; row[1] = 1.0
        lps[k] = [np.vstack([A, row]), np.append(b, -1.0), c, np.append(sense, LE).astype(np.int8)]
    for k in unb_set:
        A, b, c, sense = lps[k]
        j = int(rng.integers(0, A.shape[1]))
        A = A.copy(); A[:, j] = 0.0
        c = c.copy(); c[j] = rng.uniform(1.0, 10.0)
        lps[k] = [A, b, c, sense]
    return Batch(np.concatenate([p[0].ravel() for p in lps]),
                 np.concatenate([p[1] for p in lps]),
                 np.concatenate([p[2] for p in lps]),
                 np.concatenate([p[3] for p in lps]).astype(np.int8),
                 np.array([p[0].shape[0] for p in lps], np.int32),
                 np.array([p[0].shape[1] for p in lps], np.int32),
                 f"uneven_{lo}-{hi}_x{N}",
                 dict(seed=seed, infeasible=np.sort(inf_set), unbounded=np.sort(unb_set)))


def config2(N: int = 10_000, seed: int = 1002) -> Batch:
    return uneven_batch(N, seed)


def phase1_batch(N: int, m: int, n: int, seed: int, frac_ge: float = 0.3, frac_eq: float = 0.1) -> Batch:
    """Test-only two-phase stress set: A ~ U[1,10]; a fraction of rows are >=
    with b ~ U[1,50] and a fraction are = with b ~ U[100,1000]; the rest <= with
    b ~ U[100,1000]; c ~ U[-1,10]."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(1.0, 10.0, size=(N, m, n))
    u = rng.uniform(size=(N, m))
    sense = np.where(u < frac_ge, GE, np.where(u < frac_ge + frac_eq, EQ, LE)).astype(np.int8)
    b = np.where(sense == GE, rng.uniform(1.0, 50.0, (N, m)), rng.uniform(100.0, 1000.0, (N, m)))
    c = rng.uniform(-1.0, 10.0, size=(N, n))
    return Batch(A.reshape(-1), b.reshape(-1), c.reshape(-1), sense.reshape(-1),
                 np.full(N, m, np.int32), np.full(N, n, np.int32), f"phase1_{m}x{n}_x{N}",
                 dict(seed=seed))


def rescaled(batch: Batch, seed: int, spread: float = 3.0) -> Batch:
    """Test-only badly scaled copy of a batch: every row of every LP (its A row
    and b_i) times 10^u and every column (its A column and c_j) times 10^v,
    u, v ~ U[-spread, spread] drawn per row and per column.  Row factors keep
    the feasible set, column factors substitute x_j -> x_j / 10^v: the LPs keep
    their status and optimal value."""
    rng = np.random.default_rng(seed)
    aoff, roff, coff = batch.offsets()
    A, b, c = batch.A.copy(), batch.b.copy(), batch.c.copy()
    for k in range(batch.num_lps):
        m, n = int(batch.m[k]), int(batch.n[k])
        rf = 10.0 ** rng.uniform(-spread, spread, size=m)
        cf = 10.0 ** rng.uniform(-spread, spread, size=n)
        A[aoff[k]:aoff[k + 1]] = (A[aoff[k]:aoff[k + 1]].reshape(m, n) * rf[:, None] * cf[None, :]).ravel()
        b[roff[k]:roff[k + 1]] *= rf
        c[coff[k]:coff[k + 1]] *= cf
    return Batch(A, b, c, batch.sense.copy(), batch.m.copy(), batch.n.copy(),
                 batch.name + f"_rescaled{spread:g}", dict(batch.meta, rescale_seed=seed))


# ---- support-function batches over a fixed polytope ------------------------

@dataclass
class Polytope:
    G: np.ndarray   # [80, 20]
    h: np.ndarray   # [80]
    box: float      # |x_i| <= box

    @property
    def dim(self) -> int:
        return self.G.shape[1]


def polytope(seed: int = 1003, facets: int = 80, dim: int = 20, box: float = 10.0) -> Polytope:
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((facets, dim))
    G /= np.linalg.norm(G, axis=1, keepdims=True)
    h = 1.0 + rng.uniform(0.0, 1.0, facets)
    return Polytope(G, h, box)


def directions(N: int, seed: int, dim: int = 20) -> np.ndarray:
    """N directions uniform on the unit sphere (normalised Gaussians), float64 [N, dim]."""
    out = np.empty((N, dim), np.float64)
    for lo, hi, rng in _chunks(N, seed):
        g = rng.standard_normal((hi - lo, dim))
        out[lo:hi] = g / np.linalg.norm(g, axis=1, keepdims=True)
    return out


def split_form(P: Polytope):
    """Constraint block of max l^T x over P with x = x+ - x-, x+, x- >= 0:
    rows [G, -G] <= h (facets, ids 0..79), [I, -I] <= box (ids 80..99),
    [-I, I] <= box (ids 100..119).  Returns (A [120, 40], b [120])."""
    d = P.dim
    I = np.eye(d)
    A = np.vstack([np.hstack([P.G, -P.G]), np.hstack([I, -I]), np.hstack([-I, I])])
    b = np.concatenate([P.h, np.full(d, P.box), np.full(d, P.box)])
    return A, b


def support_batch(P: Polytope, dirs: np.ndarray) -> Batch:
    """One LP per direction: max [l; -l]^T [x+; x-] over the split form of P."""
    A1, b1 = split_form(P)
    N = dirs.shape[0]
    m, n = A1.shape
    A = np.tile(A1.reshape(-1), N)
    b = np.tile(b1, N)
    c = np.concatenate([dirs, -dirs], axis=1).reshape(-1)
    return Batch(A, b, c, np.zeros(N * m, np.int8), np.full(N, m, np.int32),
                 np.full(N, n, np.int32), f"support_{m}x{n}_x{N}", dict(shared_A=True))


def config3(N: int = 100_000, poly_seed: int = 1003, dir_seed: int = 1103):
    P = polytope(poly_seed)
    return P, support_batch(P, directions(N, dir_seed, P.dim))


def hyperbox_batch(N: int, n: int, seed: int):
    """Boxes [lo, hi] with lo ~ U[-10, 0], hi = lo + U[0.1, 10], and directions
    l ~ N(0, I) with about 5 % of the entries set to exactly 0."""
    rng = np.random.default_rng(seed)
    lo = rng.uniform(-10.0, 0.0, (N, n))
    hi = lo + rng.uniform(0.1, 10.0, (N, n))
    l = rng.standard_normal((N, n))
    l[rng.uniform(size=(N, n)) < 0.05] = 0.0
    return lo, hi, l
