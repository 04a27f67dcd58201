"""Pins for the double-double oracle: arithmetic, nodes, integrand, quadrature, TT cross.

Every check compares with something computed another way: mpmath at 60
digits (arithmetic, solves, integrand, Legendre roots), the closed forms of
the Ising integrals (Bailey, Borwein & Crandall, cited by the paper for them),
brute-force tensor quadrature (T3 = T2), Thm. 1 on the evaluated fibres, and
the double oracle's decisions where the pivot errors are far above the double
rounding level.
"""
import mpmath as mp
import numpy as np
import pytest

from oracle import ttcross as tt64
from oracle.ddarith import DD, dd_solve
from oracle.gauss import gauss_legendre_01_dd
from oracle.integrands import f_values_dd
from oracle.quadrature import tensor_quadrature_dd
from oracle.ttcross_dd import TTCrossDD, solve_dd

U_DD = 2.0 ** -104


def closed(key):
    with mp.workdps(50):
        L3 = (mp.zeta(2, mp.mpf(1) / 3) - mp.zeta(2, mp.mpf(2) / 3)) / 9
        return {"c3": L3, "c4": 7 * mp.zeta(3) / 12, "d3": 8 + 4 * mp.pi ** 2 / 3 - 27 * L3,
                "d4": 4 * mp.pi ** 2 / 9 - mp.mpf(1) / 6 - 7 * mp.zeta(3) / 2}[key]


def mpval(hi, lo):
    return mp.mpf(float(hi)) + mp.mpf(float(lo))


def random_dd(rng, n, lo_exp=-3, hi_exp=3):
    mags = 10.0 ** rng.uniform(lo_exp, hi_exp, n)
    with mp.workdps(60):
        vals = [mp.mpf(float(s)) * mp.mpf(float(m)) * (1 + mp.mpf(float(u)) * mp.mpf(2) ** -60)
                for s, m, u in zip(rng.choice([-1.0, 1.0], n), mags, rng.uniform(0, 1, n))]
        return DD.from_mp(vals)


@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_dd_operations_against_mpmath(op):
    rng = np.random.default_rng(11)
    a, b = random_dd(rng, 400), random_dd(rng, 400)
    # near-cancelling pairs for the additive operations
    b.hi[:100], b.lo[:100] = -a.hi[:100] * (1 + 2.0 ** -40), -a.lo[:100]
    f = {"add": lambda x, y: x + y, "sub": lambda x, y: x - y,
         "mul": lambda x, y: x * y, "div": lambda x, y: x / y}[op]
    if op == "sub":
        b.hi[:100] = -b.hi[:100]
        b.lo[:100] = -b.lo[:100]
    c = f(a, b)
    with mp.workdps(60):
        am, bm, cm = a.to_mp(), b.to_mp(), c.to_mp()
        worst = max(abs(cm[i] - f(am[i], bm[i])) / abs(f(am[i], bm[i])) for i in range(400))
    assert worst <= 4 * U_DD, float(worst)
    # normalised: |lo| <= ulp(hi) / 2
    assert np.all(np.abs(c.lo) <= np.spacing(np.abs(c.hi)) / 2)


def test_dd_solve_against_mpmath():
    rng = np.random.default_rng(3)
    M = random_dd(rng, 144, -1, 1).reshape(12, 12)
    rhs = random_dd(rng, 36, -1, 1).reshape(12, 3)
    X = dd_solve(M, rhs)
    with mp.workdps(60):
        Mm = mp.matrix([[mpval(M.hi[i, j], M.lo[i, j]) for j in range(12)] for i in range(12)])
        for k in range(3):
            r = mp.matrix([mpval(rhs.hi[i, k], rhs.lo[i, k]) for i in range(12)])
            x = mp.lu_solve(Mm, r)
            cond = mp.mnorm(Mm, 1) * mp.mnorm(mp.inverse(Mm), 1)
            for i in range(12):
                assert abs(mpval(X.hi[i, k], X.lo[i, k]) - x[i]) <= 64 * U_DD * cond * mp.norm(x, mp.inf)


def test_gl_dd_moments_and_roots():
    n = 16
    t, w = gauss_legendre_01_dd(n)
    with mp.workdps(60):
        tm, wm = t.to_mp(), w.to_mp()
        assert abs(sum(wm) - 1) < 1e-31
        for k in range(2 * n):
            assert abs(sum(wi * ti ** k for ti, wi in zip(tm, wm)) - mp.mpf(1) / (k + 1)) < 1e-31, k
        for ti in tm:   # roots of P_n on [-1, 1] to the double-double rounding of the node
            x = 2 * ti - 1
            dp = n * (x * mp.legendre(n, x) - mp.legendre(n - 1, x)) / (x * x - 1)
            assert abs(mp.legendre(n, x) / dp) < 4 * U_DD


def mp_paper_form(family, xs):
    """The paper form (Sec. 5.1, eqs. c/d/e) at one point, in mpmath, written independently."""
    d = len(xs) + 1
    x = {l: xs[l - 2] for l in range(2, d + 1)}

    def pr(a, b):
        out = mp.mpf(1)
        for l in range(a, b + 1):
            out *= x[l]
        return out

    f = mp.mpf(2)
    if family in ("ising_c", "ising_d"):
        f /= (1 + sum(pr(2, k) for k in range(2, d + 1))) * (1 + sum(pr(k, d) for k in range(2, d + 1)))
    if family in ("ising_d", "ising_e"):
        for i in range(1, d):
            for j in range(i + 1, d + 1):
                p = pr(i + 1, j)
                f *= ((1 - p) / (1 + p)) ** 2
    return f


@pytest.mark.parametrize("family", ["ising_c", "ising_d", "ising_e"])
@pytest.mark.parametrize("m", [1, 3, 7, 11])
def test_dd_integrand_against_mpmath(family, m):
    rng = np.random.default_rng(100 + m)
    x = DD(rng.uniform(0, 1, (20, m)), rng.uniform(-1, 1, (20, m)) * 2.0 ** -60)
    v = f_values_dd(family, x)
    with mp.workdps(60):
        for p in range(20):
            xs = [mpval(x.hi[p, k], x.lo[p, k]) for k in range(m)]
            ref = mp_paper_form(family, xs)
            assert abs(mpval(v.hi[p], v.lo[p]) / ref - 1) < 1e-29, (family, m, p)


@pytest.mark.parametrize("key,family,m", [("c3", "ising_c", 2), ("d3", "ising_d", 2),
                                          ("c4", "ising_c", 3), ("d4", "ising_d", 3)])
def test_dd_brute_force_quadrature_closed_forms(key, family, m):
    hi, lo = tensor_quadrature_dd(family, m, 32)
    with mp.workdps(50):
        assert abs(mpval(hi, lo) / closed(key) - 1) < 1e-29


@pytest.mark.parametrize("family,d", [("ising_c", 4), ("ising_d", 4), ("ising_e", 4)])
def test_dd_ttcross_equals_brute_force(family, d):
    # n = 12 and rank cap 12 = n: the cross can reach the full grid's rank, so at
    # tol 1e-30 the TT quadrature must equal the brute-force sum (T3 = T2)
    tt = solve_dd(family, d, 12, 12, 1e-30, seed=d)
    hi, lo = tensor_quadrature_dd(family, d - 1, 12)
    with mp.workdps(50):
        assert abs(mpval(*tt.value_dd()) / mpval(hi, lo) - 1) < 1e-28


def test_dd_ttcross_closed_forms():
    for key, family in (("c4", "ising_c"), ("d4", "ising_d")):
        tt = solve_dd(family, 4, 32, 32, 1e-28, seed=4)
        with mp.workdps(50):
            assert abs(mpval(*tt.value_dd()) / closed(key) - 1) < 1e-27, key


def test_dd_interpolation_on_fibres():
    # Thm. 1: the cross interpolates B exactly on every fibre I_<=c-1 x [n] x I_>c
    tt = TTCrossDD("ising_d", 5, 10, 8, 1e-25, seed=3, max_sweeps=5)
    tt.run()
    for c in range(tt.m):
        pts = [l + (i,) + r for l in tt.left_set(c - 1) for i in range(tt.n) for r in tt.right_set(c)]
        want = tt.B(pts)
        got = tt.reconstruct_dd(pts)
        diff = (got - want)
        assert np.max(np.abs(diff.hi)) <= 1e-27 * np.max(np.abs(want.hi)), c


def test_dd_decisions_match_double_oracle_while_errors_are_large():
    # the decision logic is shared with the double oracle: while every pivot error
    # is far above the double rounding level, both take the same pivots
    kw = dict(family="ising_d", d=6, n=16, rank_cap=6, tol=1e-12, seed=6, max_sweeps=4)
    a = tt64.TTCross(**kw)
    b = TTCrossDD(**kw)
    assert a.start_index == b.start_index
    for _ in range(4):
        a.sweep()
        b.sweep()
    for sa, sb in zip(a.pivot_log, b.pivot_log):
        for ra, rb in zip(sa, sb):
            if ra.searched and abs(ra.err) > 1e-8 * a.scale[ra.bond]:
                assert (ra.row, ra.col, ra.accepted, ra.iters) == (rb.row, rb.col, rb.accepted, rb.iters)
                assert abs(ra.err - rb.err) <= 1e-13 * a.scale[ra.bond]
    assert abs(a.history[-1] / b.history[-1] - 1) < 1e-13
