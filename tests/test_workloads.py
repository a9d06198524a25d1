"""Seeded generators: reproducible, right shapes and distributions."""
import numpy as np

from paper_1802_08557_amd import workloads as W


def test_uniform_reproducible_and_ranges():
    a = W.uniform_batch(25_000, 5, 5, seed=1000)
    b = W.uniform_batch(25_000, 5, 5, seed=1000)
    assert np.array_equal(a.A, b.A) and np.array_equal(a.c, b.c)
    assert a.A.min() >= 1 and a.A.max() <= 10
    assert a.b.min() >= 100 and a.b.max() <= 1000
    assert a.c.min() >= 1 and a.c.max() <= 10
    assert a.A.shape == (25_000 * 25,) and np.all(a.sense == 0)
    assert abs(a.A.mean() - 5.5) < 0.02
    # chunks of 10,000 come from independent spawned streams
    assert not np.array_equal(a.A[:250], a.A[250_000:250_250])


def test_uneven_structure():
    bt = W.uneven_batch(300, seed=1002)
    assert bt.m.min() >= 10 and bt.m.max() <= 301 and bt.n.min() >= 10 and bt.n.max() <= 300
    inf, unb = bt.meta["infeasible"], bt.meta["unbounded"]
    assert len(inf) == 15 and len(unb) == 15 and not set(inf) & set(unb)
    for k in inf:
        A, b, c, s = bt.lp(k)
        assert b[-1] == -1 and A[-1, 0] == 1 and A[-1, 1] == 1 and s[-1] == 0
    for k in unb:
        A, b, c, s = bt.lp(k)
        zc = np.where(np.all(A == 0, axis=0))[0]
        assert len(zc) >= 1 and np.any(c[zc] >= 1)
    k = next(i for i in range(300) if i not in set(inf) | set(unb))
    A, b, c, s = bt.lp(k)
    assert (s == 1).sum() == int(round(0.3 * len(b)))
    assert np.all(b[s == 1] < 0) and np.all(b[s == 0] > 0)


def test_support_batch():
    P = W.polytope(1003)
    assert P.G.shape == (80, 20)
    np.testing.assert_allclose(np.linalg.norm(P.G, axis=1), 1.0)
    d = W.directions(1000, 1103)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0)
    bt = W.support_batch(P, d[:3])
    A, b, c, s = bt.lp(1)
    assert A.shape == (120, 40) and np.all(b > 0)
    np.testing.assert_allclose(c[:20], -c[20:])
