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


# ---- the kernels' own arithmetic: partition of a row into sixteen parts, four-step
#      blocks inside a part, the tree join across the sixteen lanes, and the join
#      around one or two nodes at a search point, with every FMA rounded once
def fma(a, b, c):
    """a b + c rounded once (exact rational arithmetic, then one rounding to double)."""
    from fractions import Fraction
    return float(Fraction(a) * Fraction(b) + Fraction(c))


LANES = 16


def part_bounds(k0, k1):
    """[lo, hi) of each of the sixteen lanes that walk coordinates k0..k1-1 of a row."""
    chunk = ((k1 - k0 + LANES - 1) // LANES + 3) & ~3
    out = []
    for part in range(LANES):
        lo = min(k0 + part * chunk, k1)
        out.append((lo, min(lo + chunk, k1)))
    return out


def kernel_one(st, y):
    P, q, s = st
    P = P * y
    q = q + P
    s = fma(y, s, y)
    return P, q, s


def kernel_four(st, y0, y1, y2, y3):
    P, q, s = st
    p01 = y0 * y1
    p012 = p01 * y2
    p4 = p012 * y3
    q4 = (y0 + p01) + (p012 + p4)
    g4 = y0
    g4 = fma(y1, g4, y1)
    g4 = fma(y2, g4, y2)
    g4 = fma(y3, g4, y3)
    q = fma(P, q4, q)
    s = fma(p4, s, g4)
    P = P * p4
    return P, q, s


def kernel_span(row, lo, hi):
    st = (1.0, 0.0, 0.0)
    k = lo
    while k + 4 <= hi:
        st = kernel_four(st, *row[k:k + 4])
        k += 4
    while k < hi:
        st = kernel_one(st, row[k])
        k += 1
    return st


def kernel_row_summary(row, k0, k1):
    """The lane-0 result of the sixteen parts joined by the shuffle-down tree."""
    parts = [kernel_span(row, lo, hi) for lo, hi in part_bounds(k0, k1)]
    d = 1
    while d < LANES:
        new = list(parts)
        for part in range(LANES):
            if part & (2 * d - 1) == 0:
                P, q, s = parts[part]
                P2, q2, s2 = parts[part + d] if part + d < LANES else parts[part]
                new[part] = (P * P2, fma(P, q2, q), fma(P2, s, s2))
        parts = new
        d *= 2
    return parts[0]


def kernel_joined_value(left, nodes, right):
    """C_d at a point from its left row's summary, one or two nodes, and its right row's summary."""
    P, q, s = left
    for t in nodes:
        P, q, s = kernel_one((P, q, s), t)
    rP, rq, rs = right
    qq = fma(P, rq, q)
    sfx = fma(rP, s, rs)
    return 2.0 / ((1.0 + qq) * (1.0 + sfx))


@pytest.mark.parametrize("length", [0, 1, 3, 4, 5, 15, 16, 17, 33, 1022])
def test_kernel_partition_covers_each_row_once(length):
    for k0 in (0, 2, 7):
        bounds = part_bounds(k0, k0 + length)
        covered = [k for lo, hi in bounds for k in range(lo, hi)]
        assert covered == list(range(k0, k0 + length)), (k0, length, bounds)
        assert all(lo <= hi for lo, hi in bounds)


@pytest.mark.parametrize("length", [0, 1, 3, 4, 5, 15, 16, 17, 33, 1022])
@pytest.mark.parametrize("nm", [1, 2])
def test_kernel_summaries_and_join_give_the_c_d_integrand(length, nm):
    """Left and right rows of the given length around one or two nodes, as the kernels join them."""
    rng = np.random.default_rng(31 * length + nm)
    for trial in range(3):
        nl = length if trial != 1 else length // 2
        nr = length - nl if trial == 1 else length
        x = rng.uniform(0.02, 0.98, size=nl + nm + nr)
        want = integrands.f_values("ising_c", x.reshape(1, -1))[0]
        # the left row holds coordinates 0..nl-1; the right row is indexed by absolute coordinate
        left = kernel_row_summary(list(x), 0, nl)
        right = kernel_row_summary(list(x), nl + nm, nl + nm + nr)
        got = kernel_joined_value(left, list(x[nl:nl + nm]), right)
        assert got == pytest.approx(want, rel=1e-13, abs=0.0), (length, nm, nl, nr)


def test_planted_mistake_in_the_kernel_tree_join_is_caught():
    """Joining the tree's pairs in the wrong order (right part first) breaks the identity."""
    rng = np.random.default_rng(5)
    x = list(rng.uniform(0.05, 0.95, size=40))
    want = integrands.f_values("ising_c", np.array(x).reshape(1, -1))[0]
    parts = [kernel_span(x, lo, hi) for lo, hi in part_bounds(0, 39)]
    acc = (1.0, 0.0, 0.0)
    for p in reversed(parts):   # wrong: parts joined from the right end of the row
        P, q, s = acc
        P2, q2, s2 = p
        acc = (P * P2, fma(P, q2, q), fma(P2, s, s2))
    got = kernel_joined_value(acc, [x[39]], (1.0, 0.0, 0.0))
    assert abs(got - want) / want > 1e-6
