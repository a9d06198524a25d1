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
