"""The split identity behind the streaming C_d kernels, checked on the CPU.

The paper-form C_d integrand (Sec. 5.1) is 2 / ((1 + q)(1 + s)) with q the sum of
the prefix products of the coordinates and s the sum of their suffix products.
The large-d kernels never walk a search point's m coordinates: they keep, for each
row of an index set, the running triple (P, q, s) over that row (P the product,
s the suffix-sum recurrence s <- y (1 + s)), take one step per node, and join the
right row's triple computed from zero:

    (P1, q1, s1) then (P2, q2, g2)  ->  (P1 P2, q1 + P1 q2, g2 + P2 s1).

A row's triple is itself built from sixteen parts joined in order.  These tests
restate that bookkeeping in plain Python and compare it with the oracle's
integrand, which forms every prefix and suffix product from its definition.
"""
import numpy as np
import pytest

from oracle import integrands


def walk(ys, state=(1.0, 0.0, 0.0)):
    P, q, s = state
    for y in ys:
        P = P * y
        q = q + P
        s = y * (1.0 + s)
    return P, q, s


def join(a, b):
    (P1, q1, s1), (P2, q2, g2) = a, b
    return P1 * P2, q1 + P1 * q2, g2 + P2 * s1


def parts_joined(ys, nparts):
    """A row's triple from nparts contiguous pieces walked from zero, joined in order."""
    bounds = np.linspace(0, len(ys), nparts + 1).astype(int)
    acc = (1.0, 0.0, 0.0)
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        acc = join(acc, walk(ys[lo:hi]))
    return acc


def joined_value(y, nl, nm, nparts=16):
    left = parts_joined(y[:nl], nparts)
    mid = walk(y[nl:nl + nm], left)
    right = parts_joined(y[nl + nm:], nparts)
    _, q, s = join(mid, right)
    return 2.0 / ((1.0 + q) * (1.0 + s))


@pytest.mark.parametrize("m", [3, 9, 40, 300])
@pytest.mark.parametrize("nm", [1, 2])
def test_joined_row_summaries_give_the_c_d_integrand(m, nm):
    rng = np.random.default_rng(1000 + m + nm)
    x = rng.uniform(0.02, 0.98, size=(24, m))
    want = integrands.f_values("ising_c", x)
    for p in range(x.shape[0]):
        nl = int(rng.integers(0, m - nm + 1))   # left row length; the right row takes the rest
        got = joined_value(x[p], nl, nm)
        assert got == pytest.approx(want[p], rel=1e-13, abs=0.0), (m, nm, nl)


def test_join_is_associative_and_the_walk_is_a_left_fold():
    rng = np.random.default_rng(7)
    y = rng.uniform(0.1, 0.99, size=37)
    a, b, c = walk(y[:11]), walk(y[11:20]), walk(y[20:])
    whole = walk(y)
    np.testing.assert_allclose(join(join(a, b), c), whole, rtol=1e-14)
    np.testing.assert_allclose(join(a, join(b, c)), whole, rtol=1e-14)
    # the identity triple changes nothing
    np.testing.assert_allclose(join((1.0, 0.0, 0.0), whole), whole, rtol=0)
    np.testing.assert_allclose(join(whole, (1.0, 0.0, 0.0)), whole, rtol=0)


def test_planted_mistake_in_the_join_is_caught():
    """Swapping which product scales the suffix recurrence breaks the identity."""
    rng = np.random.default_rng(11)
    x = rng.uniform(0.05, 0.95, size=(8, 12))
    want = integrands.f_values("ising_c", x)

    def bad_join(a, b):
        (P1, q1, s1), (P2, q2, g2) = a, b
        return P1 * P2, q1 + P1 * q2, g2 + P1 * s1   # wrong factor on s1

    errs = []
    for p in range(x.shape[0]):
        left = walk(x[p, :5])
        mid = walk(x[p, 5:6], left)
        _, q, s = bad_join(mid, walk(x[p, 6:]))
        errs.append(abs(2.0 / ((1.0 + q) * (1.0 + s)) - want[p]) / want[p])
    assert max(errs) > 1e-6
