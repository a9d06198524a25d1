"""Pins of the scaling oracle (geometric-mean scaling on binary exponents,
power-of-two factors) against facts that do not come from it: a hand-worked
case, the exact result on rank-one power-of-two matrices, the centring that the
last column pass leaves, and brute-force optima of tiny LPs before and after
scaling."""
import numpy as np
import pytest

import oracle
from oracle import brute_force
from oracle.scaling import (EXP_CAP, apply_scaling, scale_exponents,
                            unscale_x)


def test_hand_worked_two_by_two():
    # A = [[8, 0.5], [0, 32]]: exponents E = [[3, -1], [-, 5]].
    # Pass 1, rows (s = 0): row 0 hi 3, lo -1 -> r0 = -floor(3/2) = -1;
    #   row 1 hi = lo = 5 -> r1 = -floor(11/2) = -5.
    # Columns: col 0 {3-1} -> s0 = -floor(5/2) = -2; col 1 {-1-1, 5-5} = {-2, 0}
    #   -> s1 = -floor(-1/2) = 1.
    # Pass 2, rows: row 0 {3-2, -1+1} = {1, 0} -> r0 = -1; row 1 {5+1} -> r1 = -6.
    # Columns: col 0 {2} -> s0 = -2; col 1 {-2, -1} -> s1 = -floor(-2/2) = 1.
    # Scaled: 8*2^-3 = 1, 0.5*2^0 = 0.5, 32*2^-5 = 1.  Pass 3 changes nothing.
    A = np.array([[8.0, 0.5], [0.0, 32.0]])
    r1, s1 = scale_exponents(A, 1)
    assert list(r1) == [-1, -5] and list(s1) == [-2, 1]
    for p in (2, 3, 7):
        r, s = scale_exponents(A, p)
        assert list(r) == [-1, -6] and list(s) == [-2, 1]
    As, bs, cs = apply_scaling(A, [3.0, 5.0], [1.0, 1.0], r, s)
    np.testing.assert_array_equal(As, [[1.0, 0.5], [0.0, 1.0]])
    np.testing.assert_array_equal(bs, [1.5, 5.0 / 64])
    np.testing.assert_array_equal(cs, [0.25, 2.0])


@pytest.mark.parametrize("seed", range(5))
def test_rank_one_powers_of_two_become_unit(seed):
    # a_ij = +-2^(u_i + v_j): one pass makes every entry +-1 exactly (the row
    # pass leaves 2^(v_j - c) in every row, which the column pass cancels).
    g = np.random.default_rng(seed)
    m, n = g.integers(1, 9, size=2)
    u = g.integers(-30, 30, size=m)
    v = g.integers(-30, 30, size=n)
    sign = g.choice([-1.0, 1.0], size=(m, n))
    A = sign * np.ldexp(1.0, (u[:, None] + v[None, :]).astype(np.int32))
    for p in (1, 4):
        r, s = scale_exponents(A, p)
        As, _, _ = apply_scaling(A, np.zeros(m), np.zeros(n), r, s)
        np.testing.assert_array_equal(As, sign)


@pytest.mark.parametrize("seed", range(6))
def test_last_column_pass_centres_every_column(seed):
    # After the final column pass, the largest and smallest exponent of every
    # column with entries sum to -1 or 0 (floor((h + l + 1) / 2) taken off both).
    g = np.random.default_rng(100 + seed)
    m, n = 7, 9
    A = g.normal(size=(m, n)) * 10.0 ** g.uniform(-8, 8, size=(m, n))
    A[g.random((m, n)) < 0.2] = 0.0
    A[:, 0] = 0.0  # an empty column keeps exponent 0
    r, s = scale_exponents(A, 3)
    assert s[0] == 0
    As, _, _ = apply_scaling(A, np.zeros(m), np.zeros(n), r, s)
    for j in range(1, n):
        nz = As[:, j] != 0
        if not nz.any():
            continue
        e = np.frexp(As[nz, j])[1] - 1
        assert e.max() + e.min() in (-1, 0)


def test_zero_rows_nonfinite_entries_and_the_cap():
    A = np.array([[0.0, 0.0, 0.0], [np.inf, 4.0, np.nan], [1e-200, 1e-200, 0.0]])
    r, s = scale_exponents(A, 2)
    assert r[0] == 0                    # no entries: factor 1
    assert r[2] == EXP_CAP               # 2^664 wanted, clamped
    assert s[2] == 0                     # the NaN is not an entry
    As, _, _ = apply_scaling(A, np.zeros(3), np.zeros(3), r, s)
    assert np.isinf(As[1, 0]) and np.isnan(As[1, 2])  # still rejected later


@pytest.mark.parametrize("seed", range(40))
def test_scaled_lp_has_the_same_optimum(seed):
    # Brute-force vertex enumeration (no simplex involved) of the original LP
    # and of the scaled one: same status and optimum.  The oracle simplex on
    # the scaled LP, mapped back by x_j = x'_j 2^s_j, gives a point of the
    # original LP that is feasible and attains that optimum.
    g = np.random.default_rng(seed)
    m, n = int(g.integers(1, 4)), int(g.integers(1, 4))
    A = g.normal(size=(m, n)) * 10.0 ** g.uniform(-2, 2, size=(m, 1)) * 10.0 ** g.uniform(-2, 2, size=(1, n))
    b = g.uniform(-1, 5, size=m) * 10.0 ** g.uniform(-2, 2, size=m)
    c = g.normal(size=n) * 10.0 ** g.uniform(-2, 2, size=n)
    sense = g.integers(0, 3, size=m).astype(np.int8)
    if seed % 4 == 0:
        sense[:] = 0
        b = np.abs(b)
    st0, z0 = brute_force(A, b, c, sense)
    r, s = scale_exponents(A, 4)
    As, bs, cs = apply_scaling(A, b, c, r, s)
    st1, z1 = brute_force(As, bs, cs, sense)
    assert st0 == st1
    res = oracle.solve(As.ravel(), bs, cs, sense, np.array([m], np.int32), np.array([n], np.int32))
    assert res.status[0] == st0
    if st0 == oracle.OPTIMAL:
        assert z1 == pytest.approx(z0, rel=1e-9, abs=1e-12)
        x = unscale_x(res.x, s)
        assert float(c @ x) == pytest.approx(z0, rel=1e-9, abs=1e-12)
        assert x.min() >= -1e-12 * (1 + np.abs(x).max())
        ax = A @ x
        tol = 1e-9 * (1 + np.abs(b).max() + np.abs(A).max() * np.abs(x).max())
        assert np.all(np.where(sense == 0, ax - b, np.where(sense == 1, b - ax, np.abs(ax - b))) <= tol)
