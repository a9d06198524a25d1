"""CPU FP64 oracle for the batched dense-tableau simplex -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and shares
no code with it; the two meet only in the seeded input generators.

Contents
  * ``solve``      -- the plain C two-phase simplex (``simplex_oracle.c``) over a
                      batch, multithreaded over LPs (paper Sec. 4 / 4.1).
  * ``brute``      -- vertex enumeration for tiny LPs (an independent check).
  * ``certificate``-- KKT / strong-duality check of an optimal basis.
  * ``phase1_certificate`` -- the same for a Phase I basis that proves an LP
                      infeasible (Phase I optimum below zero; Farkas).
  * ``hyperbox``   -- the closed-form box LP of Eq. (7), Sec. 5.6.
  * ``scaling``    -- power-of-two geometric-mean scaling (not in the paper;
                      the reference for the optional preconditioning).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "simplex_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_NATIVE = os.path.join(_HERE, "liboracle_native.so")

OPTIMAL, INFEASIBLE, UNBOUNDED, ITERATION_LIMIT, NUMERICAL, INVALID_INPUT = range(6)
LE, GE, EQ = 0, 1, 2


def build(force: bool = True, native: bool = False) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` (portable x86-64, no
    fast-math, no FP contraction: each operation rounds once, as written).
    native=True builds ``liboracle_native.so`` with ``-march=native`` for the
    host it runs on (the CPU-baseline timing); without contraction or
    fast-math its results are the same bits."""
    lib = _LIB_NATIVE if native else _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O3"] + (["-march=native"] if native else []) +
            ["-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
             "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, lib)
    return lib


class _Params(ctypes.Structure):
    _fields_ = [("tol_piv", ctypes.c_double), ("tol_opt", ctypes.c_double),
                ("tol_feas", ctypes.c_double), ("k_deg", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("pricing", ctypes.c_int32)]


_libs = {}


def _load(native: bool = False):
    if native not in _libs:
        lib = ctypes.CDLL(build(force=False, native=native))
        lib.oracle_solve_batch.restype = ctypes.c_int
        lib.oracle_solve_batch.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 6 + [
            ctypes.POINTER(_Params), ctypes.c_int] + [ctypes.c_void_p] * 5
        _libs[native] = lib
    return _libs[native]


@dataclass
class Result:
    status: np.ndarray   # int32 [N]
    obj: np.ndarray      # float64 [N]
    x: np.ndarray        # float64 [sum n]
    basis: np.ndarray    # int32 [sum m]: Bland index of each row's basic variable, -1 dropped row
    stats: np.ndarray    # int32 [N, 3]: Phase I pivots, Phase II pivots, degenerate pivots


def _p(a, dt):
    a = np.ascontiguousarray(a, dtype=dt)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def solve(A, b, c, sense, m, n, *, tol_piv=1e-9, tol_opt=1e-9, tol_feas=1e-9,
          k_deg=50, max_iters=0, threads=1, pricing=0, native=False) -> Result:
    """Solve a batch of LPs (max c^T x, A x {<=,>=,=} b, x >= 0) stored back to
    back: A row-major per LP, b/sense per row, c per column, m/n per LP.
    pricing: 0 Dantzig (the paper's Step 1), 1 steepest edge.  native: the
    -march=native build (same results)."""
    lib = _load(native)
    m_, pm = _p(np.atleast_1d(m), np.int32)
    n_, pn = _p(np.atleast_1d(n), np.int32)
    N = m_.shape[0]
    A_, pA = _p(A, np.float64)
    b_, pb = _p(b, np.float64)
    c_, pc = _p(c, np.float64)
    s_, ps = _p(sense, np.int8)
    tot_a = int(np.sum(m_.astype(np.int64) * n_))
    if A_.size != tot_a or b_.size != int(m_.sum()) or c_.size != int(n_.sum()) or s_.size != b_.size:
        raise ValueError("batch arrays do not match m[] and n[]")
    status = np.empty(N, np.int32)
    obj = np.empty(N, np.float64)
    x = np.empty(int(n_.sum()), np.float64)
    basis = np.empty(int(m_.sum()), np.int32)
    stats = np.empty((N, 3), np.int32)
    prm = _Params(tol_piv, tol_opt, tol_feas, k_deg, max_iters, pricing)
    rc = lib.oracle_solve_batch(N, pA, pb, pc, ps, pm, pn, ctypes.byref(prm), int(threads),
                                status.ctypes.data_as(ctypes.c_void_p),
                                x.ctypes.data_as(ctypes.c_void_p),
                                obj.ctypes.data_as(ctypes.c_void_p),
                                basis.ctypes.data_as(ctypes.c_void_p),
                                stats.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise RuntimeError("oracle_solve_batch failed")
    return Result(status, obj, x, basis, stats)


def solve_traced(A, b, c, sense=None, *, tol_piv=1e-9, tol_opt=1e-9, tol_feas=1e-9,
                 k_deg=50, max_iters=0, max_snapshots=64, pricing=0):
    """Solve one LP and return (Result, snapshots [k, m+1, ncol+1]): the whole
    tableau after every pricing of an objective row and after every pivot."""
    lib = _load()
    A = np.ascontiguousarray(A, np.float64)
    m, n = A.shape
    b = np.ascontiguousarray(b, np.float64)
    c = np.ascontiguousarray(c, np.float64)
    sense = np.zeros(m, np.int8) if sense is None else np.ascontiguousarray(sense, np.int8)
    x = np.empty(n); obj = np.empty(1); basis = np.empty(m, np.int32); stats = np.empty(3, np.int32)
    ld_max = n + 2 * m + 1
    buf = np.zeros(max_snapshots * (m + 1) * ld_max)
    ncol = ctypes.c_int32(); nsnap = ctypes.c_int32()
    prm = _Params(tol_piv, tol_opt, tol_feas, k_deg, max_iters, pricing)
    v = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    lib.oracle_solve_traced.restype = ctypes.c_int
    st = lib.oracle_solve_traced(ctypes.c_int(m), ctypes.c_int(n), v(A), v(b), v(c), v(sense),
                                 ctypes.byref(prm), v(x), v(obj), v(basis), v(stats), v(buf),
                                 ctypes.c_int(max_snapshots), ctypes.byref(ncol), ctypes.byref(nsnap))
    ld = ncol.value + 1
    snaps = buf[:nsnap.value * (m + 1) * ld].reshape(nsnap.value, m + 1, ld)
    return Result(np.array([st], np.int32), obj, x, basis, stats.reshape(1, 3)), snaps


def solve_one(A, b, c, sense=None, **kw) -> Result:
    """Convenience wrapper for a single LP given as a 2-D A."""
    A = np.asarray(A, np.float64)
    m, n = A.shape
    if sense is None:
        sense = np.zeros(m, np.int8)
    return solve(A.ravel(), b, c, sense, [m], [n], **kw)


from .brute import brute_force, certificate, phase1_certificate  # noqa: E402
from .hyperbox import hyperbox_max  # noqa: E402
