"""Pins of the oracle's KKT / strong-duality certificate (``oracle.certificate``).

The certificate is what the other oracle tests use to accept a basis as
optimal, so it must reject what is not: a feasible but non-optimal basis
(a reduced cost above zero), a primal-infeasible basis, and a vertex x that is
not the basis's.  Its duals are pinned by values worked out by hand."""
import numpy as np
import pytest

from oracle import certificate

# max 2 x1 + 3 x2  s.t.  x1 + x2 <= 4,  x1 + 3 x2 <= 6,  x1 <= 3.5,  x >= 0.
# Optimum x = (3, 1), z = 9; rows 0 and 1 tight; duals from
# y0 + y1 = 2 and y0 + 3 y1 = 3: y = (1.5, 0.5, 0).
A = np.array([[1.0, 1.0], [1.0, 3.0], [1.0, 0.0]])
b = np.array([4.0, 6.0, 3.5])
c = np.array([2.0, 3.0])
LE3 = np.zeros(3, np.int8)
N = 2  # Bland index n + i is the slack of row i


def test_optimal_basis_accepted_with_hand_worked_duals():
    cert = certificate(A, b, c, LE3, [0, 1, N + 2], [3.0, 1.0])
    assert cert["ok"]
    np.testing.assert_allclose(cert["x"], [3.0, 1.0], atol=1e-14)
    np.testing.assert_allclose(cert["y"], [1.5, 0.5, 0.0], atol=1e-14)
    assert cert["gap"] <= 1e-12
    # The order of the basic variables over the rows does not matter.
    assert certificate(A, b, c, LE3, [N + 2, 0, 1], [3.0, 1.0])["ok"]


def test_feasible_non_optimal_basis_rejected():
    # The slack basis: x = 0 is feasible, but both reduced costs are positive.
    cert = certificate(A, b, c, LE3, [N + 0, N + 1, N + 2], [0.0, 0.0])
    assert not cert["ok"]
    assert cert["primal"] == 0.0
    assert cert["dual"] == pytest.approx(3.0)
    # A vertex adjacent to the optimum: x = (3.5, 0.5) (rows 0 and 2 tight) is
    # feasible with z = 8.5 < 9; the slack of row 1 is basic, y = (3, 0, -1)
    # gives the slack of row 2 the reduced cost 0 - (-1) = 1 > 0.
    cert = certificate(A, b, c, LE3, [0, 1, N + 1], [3.5, 0.5])
    assert not cert["ok"]
    np.testing.assert_allclose(cert["y"], [3.0, 0.0, -1.0], atol=1e-14)
    assert cert["dual"] == pytest.approx(1.0)


def test_primal_infeasible_basis_rejected():
    # Rows 1 and 2 tight: x = (3.5, 5/6), and row 0's slack 4 - 3.5 - 5/6 < 0.
    cert = certificate(A, b, c, LE3, [0, 1, N + 0], [3.5, 5.0 / 6.0])
    assert not cert["ok"]
    assert cert["primal"] == pytest.approx(1.0 / 3.0)


def test_wrong_vertex_rejected():
    cert = certificate(A, b, c, LE3, [0, 1, N + 2], [3.0, 1.001])
    assert not cert["ok"]
    assert cert["xdiff"] == pytest.approx(1e-3)
    cert = certificate(A, b, c, LE3, [0, 1, N + 2], [1.0, 3.0])  # x1 and x2 swapped
    assert not cert["ok"]


def test_surplus_column_sign():
    # max -x1 - x2  s.t.  x1 + x2 >= 1: optimum z = -1 with x1 basic, y = -1.
    # The surplus column is -e_0, its reduced cost 0 - y * (-1) = -1 <= 0; with
    # a +e_0 column the same basis would look dual infeasible.
    A1 = np.array([[1.0, 1.0]])
    cert = certificate(A1, [1.0], [-1.0, -1.0], [1], [0], [1.0, 0.0])
    assert cert["ok"]
    np.testing.assert_allclose(cert["y"], [-1.0])
    # The surplus basic instead (x = 0) violates the row.
    cert = certificate(A1, [1.0], [-1.0, -1.0], [1], [2], [0.0, 0.0])
    assert not cert["ok"]
    assert cert["primal"] == pytest.approx(1.0)


def test_negative_rhs_row_is_normalised():
    # -x1 - x2 >= -4 is row 0 of the hand example written with b < 0; the
    # certificate normalises it to x1 + x2 <= 4 and accepts the same basis.
    A2 = A.copy()
    A2[0] *= -1.0
    b2 = b.copy()
    b2[0] = -4.0
    cert = certificate(A2, b2, c, np.array([1, 0, 0], np.int8), [0, 1, N + 2], [3.0, 1.0])
    assert cert["ok"]
    np.testing.assert_allclose(cert["y"], [1.5, 0.5, 0.0], atol=1e-14)


# ---------------------------------------------------------------- Phase I (infeasibility)

from oracle import phase1_certificate  # noqa: E402
import oracle  # noqa: E402

# x1 + x2 <= 4 and x1 + x2 >= 6.  By hand: Phase I starts with the slack of
# row 0 and the artificial of row 1 (index n + m + 1 = 5) basic; x1 enters
# (reduced cost 1, the smaller index of a tie), row 0 leaves (ratio 4 < 6), and
# then every reduced cost is <= 0 with a1 = 2: w* = -2.  Duals of the final
# basis {x1, a1}: y = (1, -1); -y = (-1, 1) is a Farkas certificate
# (-y^T A = (0, 0), -y^T b = 2 > 0).
A2 = np.array([[1.0, 1.0], [1.0, 1.0]])
b2 = np.array([4.0, 6.0])
s2 = np.array([0, 1], np.int8)


def test_phase1_hand_worked_basis_and_duals():
    r = oracle.solve_one(A2, b2, np.array([1.0, 1.0]), s2)
    assert r.status[0] == oracle.INFEASIBLE
    assert list(r.basis) == [0, 5]
    cert = phase1_certificate(A2, b2, s2, [0, 5])
    assert cert["ok"]
    assert cert["w"] == pytest.approx(-2.0)
    np.testing.assert_allclose(cert["y"], [1.0, -1.0], atol=1e-14)


def test_phase1_single_negative_row():
    # x1 + x2 <= -1 is -x1 - x2 >= 1 after normalisation: its artificial stays
    # basic (index n + m = 3) at 1, every reduced cost is -1: w* = -1, y = -1.
    A = np.array([[1.0, 1.0]])
    cert = phase1_certificate(A, [-1.0], [0], [3])
    assert cert["ok"] and cert["w"] == pytest.approx(-1.0)
    np.testing.assert_allclose(cert["y"], [-1.0])


def test_phase1_rejects_non_optimal_and_feasible():
    # The starting basis {s0, a1} of the hand example: x1's reduced cost is 1.
    cert = phase1_certificate(A2, b2, s2, [2, 5])
    assert not cert["ok"] and cert["dual"] == pytest.approx(1.0)
    # A feasible LP's optimal Phase I basis has w* = 0: no proof of infeasibility.
    A = np.array([[1.0, 1.0], [1.0, 1.0]])
    b = np.array([6.0, 4.0])
    s = np.array([0, 1], np.int8)  # x1 + x2 <= 6, x1 + x2 >= 4: feasible
    cert = phase1_certificate(A, b, s, [2, 0])  # slack of row 0 (index n + 0), x1 in row 1
    assert not cert["ok"] and cert["w"] == pytest.approx(0.0)
    # Not a basis of this LP (a repeated index).
    assert not phase1_certificate(A2, b2, s2, [0, 0])["ok"]


def test_phase1_oracle_bases_of_infeasible_lps_pass():
    # Brute force decides infeasibility of small random LPs of every sense;
    # the oracle's final Phase I basis of each infeasible one must prove it.
    rng = np.random.default_rng(5)
    seen = 0
    for _ in range(300):
        m, n = rng.integers(2, 5), rng.integers(2, 5)
        A = rng.integers(-4, 5, size=(m, n)).astype(float)
        b = rng.integers(-6, 7, size=m).astype(float)
        s = rng.integers(0, 3, size=m).astype(np.int8)
        st, _ = oracle.brute_force(A, b, np.ones(n), s)
        if st != oracle.INFEASIBLE:
            continue
        r = oracle.solve_one(A, b, np.ones(n), s)
        assert r.status[0] == oracle.INFEASIBLE
        assert phase1_certificate(A, b, s, r.basis)["ok"], (A, b, s, r.basis)
        seen += 1
    assert seen > 30


def test_phase1_oracle_bases_of_injected_infeasible_lps_pass():
    # The uneven workload's injected infeasible LPs (a row x1 + x2 <= -1
    # appended to Gaussian LPs with >= rows): every one is proven infeasible
    # by the oracle's final Phase I basis; a feasible LP's basis proves nothing.
    from paper_1802_08557_amd import workloads as W
    bt = W.uneven_batch(400, seed=31, lo=10, hi=40)
    ref = oracle.solve(bt.A, bt.b, bt.c, bt.sense, bt.m, bt.n, threads=4)
    aoff, roff, coff = bt.offsets()
    inf = [int(k) for k in bt.meta["infeasible"]]
    assert len(inf) >= 10
    for k in inf:
        A, b, c, s = bt.lp(k)
        assert ref.status[k] == oracle.INFEASIBLE
        assert phase1_certificate(A, b, s, ref.basis[roff[k]:roff[k + 1]])["ok"], k
    opt = [k for k in range(bt.num_lps) if ref.status[k] == oracle.OPTIMAL][:20]
    for k in opt:
        A, b, c, s = bt.lp(k)
        assert not phase1_certificate(A, b, s, ref.basis[roff[k]:roff[k + 1]])["ok"], k
