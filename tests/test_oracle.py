"""Pins of the CPU oracle against facts that do not come from the oracle itself:
hand-worked tableaux, brute-force vertex enumeration, closed forms, textbook
pivot counts, KKT/strong duality, and HiGHS as a third opinion."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute_force, certificate, hyperbox_max
from paper_1802_08557_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _num(v):
    return float(Fraction(v)) if isinstance(v, str) else float(v)


# ---------------------------------------------------------------- hand-worked

@pytest.mark.parametrize("ex", json.load(open(GOLDEN))["examples"], ids=lambda e: e["name"])
def test_hand_worked_tableaux(ex):
    """Every tableau of a hand-worked run (paper Sec. 4.1 Steps 1-3, Sec. 4 two phases)."""
    r, snaps = oracle.solve_traced(np.array(ex["A"], float), ex["b"], ex["c"],
                                   np.array(ex["sense"], np.int8))
    assert r.status[0] == ex["status"]
    want = [np.array([[_num(v) for v in row] for row in t]) for t in ex["tableaux"]]
    assert len(snaps) == len(want)
    for got, w in zip(snaps, want):
        np.testing.assert_allclose(got, w, rtol=0, atol=1e-12)
    assert list(r.stats[0, :2]) == ex["pivots"]
    if ex["status"] == oracle.OPTIMAL:
        assert r.obj[0] == pytest.approx(ex["obj"], abs=1e-12)
        np.testing.assert_allclose(r.x, ex["x"], atol=1e-12)
        assert list(r.basis) == ex["basis"]
    elif ex["status"] == oracle.UNBOUNDED:
        assert r.obj[0] == math.inf and np.all(np.isnan(r.x))
    else:
        assert np.isnan(r.obj[0]) and np.all(np.isnan(r.x))


# ---------------------------------------------------------------- brute force

def _random_tiny(rng, kind):
    m = int(rng.integers(1, 6))
    n = int(rng.integers(1, 6))
    if kind == "int":   # small integers: plenty of degeneracy and ties
        A = rng.integers(-3, 4, (m, n)).astype(float)
        b = rng.integers(-3, 6, m).astype(float)
        c = rng.integers(-3, 4, n).astype(float)
    else:
        A = rng.standard_normal((m, n))
        b = rng.standard_normal(m) * 2 + 0.5
        c = rng.standard_normal(n)
    sense = rng.choice([0, 0, 0, 1, 2], m).astype(np.int8)
    return A, b, c, sense


@pytest.mark.parametrize("kind", ["int", "gauss"])
def test_brute_force_agreement(kind):
    """Status and optimum agree with vertex enumeration on 400 random tiny LPs
    of all three senses (covers OPTIMAL, INFEASIBLE and UNBOUNDED)."""
    rng = np.random.default_rng(7 if kind == "int" else 8)
    seen = set()
    for _ in range(400):
        A, b, c, sense = _random_tiny(rng, kind)
        st, z = brute_force(A, b, c, sense)
        r = oracle.solve_one(A, b, c, sense)
        seen.add(st)
        assert r.status[0] == st, (A, b, c, sense)
        if st == oracle.OPTIMAL:
            assert r.obj[0] == pytest.approx(z, rel=1e-9, abs=1e-9)
    assert seen == {0, 1, 2}


def test_brute_force_hypothesis():
    hyp = pytest.importorskip("hypothesis")
    from hypothesis import given, settings, strategies as st

    @settings(max_examples=150, deadline=None, derandomize=True)
    @given(st.integers(1, 4), st.integers(1, 4), st.data())
    def run(m, n, data):
        ints = st.integers(-4, 4)
        A = np.array(data.draw(st.lists(ints, min_size=m * n, max_size=m * n)), float).reshape(m, n)
        b = np.array(data.draw(st.lists(st.integers(-4, 8), min_size=m, max_size=m)), float)
        c = np.array(data.draw(st.lists(ints, min_size=n, max_size=n)), float)
        sense = np.array(data.draw(st.lists(st.sampled_from([0, 1, 2]), min_size=m, max_size=m)), np.int8)
        s, z = brute_force(A, b, c, sense)
        r = oracle.solve_one(A, b, c, sense)
        assert r.status[0] == s
        if s == 0:
            assert r.obj[0] == pytest.approx(z, rel=1e-9, abs=1e-9)
    run()


# ---------------------------------------------------------------- closed forms

def test_single_row_knapsack():
    """m = 1, a, b > 0: z* = b * max_j c_j / a_j."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        n = int(rng.integers(1, 30))
        a = rng.uniform(0.5, 5, n); c = rng.uniform(-1, 5, n); b = rng.uniform(1, 100)
        r = oracle.solve_one(a[None, :], [b], c)
        assert r.status[0] == 0
        assert r.obj[0] == pytest.approx(max(0.0, b * np.max(c / a)), rel=1e-12)


def test_diagonal():
    """Diagonal A with positive entries: z* = sum_i max(c_i, 0) b_i / a_ii."""
    rng = np.random.default_rng(4)
    for _ in range(20):
        n = int(rng.integers(1, 40))
        a = rng.uniform(0.5, 5, n); c = rng.uniform(-2, 5, n); b = rng.uniform(1, 100, n)
        r = oracle.solve_one(np.diag(a), b, c)
        assert r.obj[0] == pytest.approx(np.sum(np.maximum(c, 0) * b / a), rel=1e-12)


def test_hyperbox_eq7():
    """Box [lo, hi] (lo >= 0) written as rows x_i <= hi_i and x_i >= lo_i: the
    simplex (through Phase I) reaches Eq. (7)'s sum l_i h_i."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        n = int(rng.integers(1, 12))
        lo = rng.uniform(0, 5, n); hi = lo + rng.uniform(0.1, 5, n)
        l = rng.standard_normal(n); l[rng.uniform(size=n) < 0.2] = 0.0
        A = np.vstack([np.eye(n), np.eye(n)])
        b = np.concatenate([hi, lo])
        sense = np.array([0] * n + [1] * n, np.int8)
        r = oracle.solve_one(A, b, l, sense)
        want, _ = hyperbox_max(lo, hi, l)
        assert r.status[0] == 0
        assert r.obj[0] == pytest.approx(want, rel=1e-12, abs=1e-12)


def test_hyperbox_closed_form_direct():
    """Eq. (7) against brute force on the box's 2^n corners."""
    rng = np.random.default_rng(6)
    lo = rng.uniform(-3, 0, (30, 4)); hi = lo + rng.uniform(0.1, 3, (30, 4))
    l = rng.standard_normal((30, 4)); l[0, 1] = 0.0
    val, _ = hyperbox_max(lo, hi, l)
    import itertools
    for k in range(30):
        best = max(float(l[k] @ np.where(np.array(bits, bool), hi[k], lo[k]))
                   for bits in itertools.product([0, 1], repeat=4))
        assert val[k] == pytest.approx(best, rel=1e-14, abs=1e-14)


def _klee_minty(n):
    A = np.zeros((n, n)); b = np.zeros(n); c = np.zeros(n)
    for i in range(n):
        for j in range(i):
            A[i, j] = 2.0 * 10.0 ** (i - j)
        A[i, i] = 1.0
        b[i] = 100.0 ** i
    for j in range(n):
        c[j] = 10.0 ** (n - 1 - j)
    return A, b, c


@pytest.mark.parametrize("n", range(2, 8))
def test_klee_minty(n):
    """Klee-Minty cube: z* = 100^(n-1), and Dantzig's rule visits all 2^n
    vertices, i.e. 2^n - 1 pivots (textbook result that pins the pricing rule)."""
    A, b, c = _klee_minty(n)
    r = oracle.solve_one(A, b, c)
    assert r.status[0] == 0
    assert r.obj[0] == pytest.approx(100.0 ** (n - 1), rel=1e-12)
    assert r.stats[0, 1] == 2 ** n - 1


CYCLE = (np.array([[0.5, -5.5, -2.5, 9.0], [0.5, -1.5, -0.5, 1.0], [1.0, 0, 0, 0]]),
         np.array([0.0, 0.0, 1.0]), np.array([10.0, -57.0, -9.0, -24.0]))


def test_cycling_example_cycles_without_bland_switch():
    """The degenerate textbook example cycles under pure Dantzig pricing with
    smallest-index leaving ties; with the degenerate-streak switch to Bland's
    rule it reaches z* = 1 at x = (1, 0, 1, 0)."""
    A, b, c = CYCLE
    r = oracle.solve_one(A, b, c, k_deg=0)
    assert r.status[0] == oracle.ITERATION_LIMIT
    r = oracle.solve_one(A, b, c, k_deg=50)
    assert r.status[0] == 0
    assert r.obj[0] == pytest.approx(1.0, abs=1e-12)
    np.testing.assert_allclose(r.x, [1, 0, 1, 0], atol=1e-12)
    r = oracle.solve_one(A, b, c, k_deg=1)
    assert r.status[0] == 0 and r.obj[0] == pytest.approx(1.0, abs=1e-12)


def test_iteration_cap_and_invalid_input():
    A, b, c = _klee_minty(5)
    assert oracle.solve_one(A, b, c, max_iters=1).status[0] == oracle.ITERATION_LIMIT
    A2 = A.copy(); A2[1, 1] = np.nan
    r = oracle.solve_one(A2, b, c)
    assert r.status[0] == oracle.INVALID_INPUT and np.isnan(r.obj[0])
    r = oracle.solve_one(A, b, c, np.array([0, 3, 0, 0, 0], np.int8))
    assert r.status[0] == oracle.INVALID_INPUT


# ---------------------------------------------------------------- KKT / duality

def _check_certificates(batch, res, idx):
    aoff, roff, coff = batch.offsets()
    for k in idx:
        if res.status[k] != 0:
            continue
        A, b, c, s = batch.lp(k)
        cert = certificate(A, b, c, s, res.basis[roff[k]:roff[k + 1]], res.x[coff[k]:coff[k + 1]])
        assert cert["ok"], (k, cert)
        assert res.obj[k] == pytest.approx(float(c @ cert["x"]), rel=1e-9, abs=1e-9)


def test_duality_uniform():
    bt = W.uniform_batch(200, 12, 9, seed=11)
    res = oracle.solve(bt.A, bt.b, bt.c, bt.sense, bt.m, bt.n, threads=4)
    assert np.all(res.status == 0)
    _check_certificates(bt, res, range(200))


def test_duality_two_phase():
    bt = W.phase1_batch(200, 10, 8, seed=12)
    res = oracle.solve(bt.A, bt.b, bt.c, bt.sense, bt.m, bt.n, threads=4)
    assert (res.status == 0).sum() > 50 and (res.stats[:, 0] > 0).sum() > 50
    _check_certificates(bt, res, range(200))


def test_duality_uneven_gaussian():
    bt = W.uneven_batch(60, seed=13, lo=5, hi=40)
    res = oracle.solve(bt.A, bt.b, bt.c, bt.sense, bt.m, bt.n, threads=4)
    _check_certificates(bt, res, range(60))
    assert set(np.unique(res.status)) <= {0, 1, 2}


# ---------------------------------------------------------------- HiGHS third opinion

def _highs(A, b, c, sense):
    from scipy.optimize import linprog
    le = sense == 0; ge = sense == 1; eq = sense == 2
    Aub = np.vstack([A[le], -A[ge]]); bub = np.concatenate([b[le], -b[ge]])
    r = linprog(-c, A_ub=Aub if len(bub) else None, b_ub=bub if len(bub) else None,
                A_eq=A[eq] if eq.any() else None, b_eq=b[eq] if eq.any() else None,
                bounds=(0, None), method="highs")
    return {0: 0, 2: 1, 3: 2}.get(r.status, -1), (-r.fun if r.status == 0 else None)


@pytest.mark.parametrize("gen", ["c0", "c2small", "phase1", "c3"])
def test_highs_third_opinion(gen):
    if gen == "c0":
        bt = W.config0(100)
    elif gen == "c2small":
        bt = W.uneven_batch(40, seed=21, lo=10, hi=60)
    elif gen == "phase1":
        bt = W.phase1_batch(60, 15, 12, seed=22)
    else:
        P = W.polytope(1003)
        bt = W.support_batch(P, W.directions(30, 99))
    res = oracle.solve(bt.A, bt.b, bt.c, bt.sense, bt.m, bt.n, threads=4)
    for k in range(bt.num_lps):
        A, b, c, s = bt.lp(k)
        st, z = _highs(A, b, c, s)
        assert res.status[k] == st
        if st == 0:
            assert res.obj[k] == pytest.approx(z, rel=1e-7, abs=1e-7)


# ---------------------------------------------------------------- workload invariants

def test_workload_invariants():
    # uniform batches are always optimal (origin feasible, A > 0 bounds x)
    for bt in (W.config0(300), W.uniform_batch(50, 50, 50, 1001)):
        res = oracle.solve(bt.A, bt.b, bt.c, bt.sense, bt.m, bt.n, threads=4)
        assert np.all(res.status == 0)
    # uneven batch: injected infeasible / unbounded LPs have those statuses
    bt = W.uneven_batch(200, seed=1002, lo=10, hi=80)
    res = oracle.solve(bt.A, bt.b, bt.c, bt.sense, bt.m, bt.n, threads=4)
    assert np.all(res.status[bt.meta["infeasible"]] == oracle.INFEASIBLE)
    assert np.all(res.status[bt.meta["unbounded"]] == oracle.UNBOUNDED)
    # support batches: optimal with exactly 20 tight constraints (non-basic slacks)
    P = W.polytope(1003)
    bt = W.support_batch(P, W.directions(40, 5))
    res = oracle.solve(bt.A, bt.b, bt.c, bt.sense, bt.m, bt.n, threads=4)
    assert np.all(res.status == 0)
    for k in range(40):
        basis = res.basis[k * 120:(k + 1) * 120]
        slack_basic = np.sum(basis >= 40)
        assert 120 - slack_basic == 20


# ------------------------------------------------- steepest-edge pricing (optional)

def test_steepest_edge_enters_the_steepest_column():
    """max 3x1 + 2x2, 10x1 + x2 <= 10, x1 + x2 <= 4.  Dantzig enters x1 (d = 3 > 2),
    reaching z = 3; steepest edge scores d^2 / (1 + |column|^2): x1 9/102, x2 4/3,
    so x2 enters at row 2 (ratio 4 < 10) and z = 8.  Both end at (2/3, 10/3), z = 26/3."""
    A = np.array([[10.0, 1.0], [1.0, 1.0]])
    for pricing, z1 in ((0, 3.0), (1, 8.0)):
        r, snaps = oracle.solve_traced(A, [10.0, 4.0], [3.0, 2.0], pricing=pricing)
        assert r.status[0] == oracle.OPTIMAL
        assert abs(snaps[1][-1, -1]) == pytest.approx(z1, abs=1e-12)
        assert r.obj[0] == pytest.approx(26.0 / 3.0, abs=1e-12)
        np.testing.assert_allclose(r.x, [2.0 / 3.0, 10.0 / 3.0], atol=1e-12)


def test_steepest_edge_weight_counts_the_unit_term():
    """max x1 + 1.9x2, x1 + 2x2 <= 4.  With weights 1 + |column|^2 the scores are
    1/2 and 3.61/5, so x2 enters first and x1 second (2 pivots); a weight without
    the 1 would score 1 and 3.61/4 and finish in one pivot."""
    r = oracle.solve_one(np.array([[1.0, 2.0]]), [4.0], [1.0, 1.9], pricing=1)
    assert r.status[0] == oracle.OPTIMAL and r.obj[0] == pytest.approx(4.0, abs=1e-12)
    assert list(r.stats[0, :2]) == [0, 2]


@pytest.mark.parametrize("n", range(2, 9))
def test_steepest_edge_solves_klee_minty_in_one_pivot(n):
    """On the Klee-Minty cube above, column n has d = 1 and weight 2 (score 1/2),
    column j < n has d = 10^(n-j) and weight 2 + 4 sum_k 100^k, score < 1/4; x_n
    enters at row n with x_n = 100^(n-1), which is the optimum (every other
    reduced cost is then negative): one pivot instead of 2^n - 1."""
    A, b, c = _klee_minty(n)
    r = oracle.solve_one(A, b, c, pricing=1)
    assert r.status[0] == oracle.OPTIMAL
    assert r.obj[0] == pytest.approx(100.0 ** (n - 1), rel=1e-12)
    assert list(r.stats[0, :2]) == [0, 1]


@pytest.mark.parametrize("seed", range(4))
def test_steepest_edge_reaches_the_brute_force_optimum(seed):
    """Any pricing rule that only picks improving columns ends at the same
    status and optimum: vertex enumeration on random tiny LPs of all senses."""
    g = np.random.default_rng(7000 + seed)
    for _ in range(50):
        m, n = int(g.integers(1, 5)), int(g.integers(1, 5))
        A = np.round(g.normal(size=(m, n)), 2)
        b = np.round(g.uniform(-2, 6, size=m), 2)
        c = np.round(g.normal(size=n), 2)
        sense = g.integers(0, 3, size=m).astype(np.int8)
        st, z = brute_force(A, b, c, sense)
        r = oracle.solve_one(A, b, c, sense, pricing=1)
        assert r.status[0] == st
        if st == oracle.OPTIMAL:
            assert r.obj[0] == pytest.approx(z, rel=1e-9, abs=1e-9)


# ---------------------------------------------------------------- Phase I drive-out and redundant rows

def test_redundant_equality_row_is_dropped():
    # max x1 + x2  s.t.  x1 + x2 = 2,  2 x1 + 2 x2 = 4 (twice the first row),  x1 <= 1.5.
    # Both equalities get artificials; Phase I ends at w* = 0 with one artificial
    # still basic at zero in a row whose non-artificial entries are all zero
    # after the other equality's pivot: that row is redundant and is dropped
    # (basis -1).  The optimum is z = 2 (any split of x1 + x2 = 2 with x1 <= 1.5).
    A = np.array([[1.0, 1.0], [2.0, 2.0], [1.0, 0.0]])
    b = np.array([2.0, 4.0, 1.5])
    c = np.array([1.0, 1.0])
    s = np.array([oracle.EQ, oracle.EQ, oracle.LE], np.int8)
    r = oracle.solve_one(A, b, c, s)
    assert r.status[0] == oracle.OPTIMAL
    assert r.obj[0] == pytest.approx(2.0, abs=1e-12)
    assert np.sum(r.basis == -1) == 1
    n, m = 2, 3
    assert not np.any(r.basis >= n + m)  # no artificial left in the basis
    assert brute_force(A, b, c, s) == (oracle.OPTIMAL, pytest.approx(2.0, abs=1e-9))
    cert = certificate(A, b, c, s, r.basis, r.x)
    assert cert["ok"], cert


def test_artificial_at_zero_is_driven_out_not_dropped():
    # max x1 + 2 x2  s.t.  x1 - x2 = 0,  x1 + x2 <= 4.  Row 0 has b = 0: its
    # artificial is basic at zero from the start, Phase I is optimal at once,
    # and the drive-out pivots x1 (the smallest-index column with a non-zero
    # entry in that row) into it; nothing is dropped.  Optimum x = (2, 2), z = 6.
    A = np.array([[1.0, -1.0], [1.0, 1.0]])
    b = np.array([0.0, 4.0])
    c = np.array([1.0, 2.0])
    s = np.array([oracle.EQ, oracle.LE], np.int8)
    r = oracle.solve_one(A, b, c, s)
    assert r.status[0] == oracle.OPTIMAL
    assert r.obj[0] == pytest.approx(6.0, abs=1e-12)
    np.testing.assert_allclose(r.x, [2.0, 2.0], atol=1e-12)
    assert np.all(r.basis >= 0) and not np.any(r.basis >= 4)
    assert brute_force(A, b, c, s) == (oracle.OPTIMAL, pytest.approx(6.0, abs=1e-9))
