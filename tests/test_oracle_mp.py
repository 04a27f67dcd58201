"""Pins of the 256-bit TT-cross oracle (oracle/ttcross_mp.py), the reference of the double-double path.

Every expected value comes from outside the oracle's cross: mpmath's own
Legendre function and exact moments for the rule; closed forms of the Ising
integrals (C_3 = L_{-3}(2), D_3 = 8 + 4 pi^2/3 - 27 L_{-3}(2), C_4 = 7 zeta(3)/12,
D_4 = 4 pi^2/9 - 1/6 - 7 zeta(3)/2, from Bailey, Borwein and Crandall, whom the
paper cites) reached by brute-force tensor quadrature at enough nodes; and the
cross against brute-force tensor quadrature of the same nodes (T3 = T2) at
n <= 6, where it recovers the whole tensor.  Planted mistakes in a copy of the
oracle must each break one of these pins.
"""
import importlib
import os
import shutil
import sys

import mpmath as mp
import pytest

from oracle import ttcross_mp as tm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PREC = 256


def closed_forms():
    with mp.workprec(PREC + 32):
        L3 = (mp.zeta(2, mp.mpf(1) / 3) - mp.zeta(2, mp.mpf(2) / 3)) / 9
        return {("ising_c", 3): L3, ("ising_d", 3): 8 + 4 * mp.pi ** 2 / 3 - 27 * L3,
                ("ising_c", 4): 7 * mp.zeta(3) / 12,
                ("ising_d", 4): 4 * mp.pi ** 2 / 9 - mp.mpf(1) / 6 - 7 * mp.zeta(3) / 2}


def rel(a, b):
    with mp.workprec(PREC + 32):
        return abs(a / b - 1)


@pytest.mark.parametrize("n", [1, 2, 7, 33, 64])
def test_gl_rule_256_bits(n):
    t, w = tm.gauss_legendre_01_mp(n)
    with mp.workprec(PREC):
        assert abs(mp.fsum(w) - 1) < mp.mpf(10) ** -74
        for k in range(2 * n):     # exact for degree <= 2n - 1
            assert abs(mp.fsum(wi * ti ** k for ti, wi in zip(t, w)) - mp.mpf(1) / (k + 1)) < mp.mpf(10) ** -73
        for ti in t:               # roots of P_n by mpmath's own Legendre function
            assert abs(mp.legendre(n, 2 * ti - 1)) < mp.mpf(10) ** -70 * n ** 2


@pytest.mark.parametrize("family,d,n,bound", [("ising_c", 3, 64, 1e-68), ("ising_d", 3, 64, 1e-68),
                                              ("ising_c", 4, 48, 1e-47), ("ising_d", 4, 48, 1e-47)])
def test_brute_force_quadrature_reaches_the_closed_forms(family, d, n, bound):
    q = tm.tensor_quadrature_mp(family, d, n)
    assert rel(q, closed_forms()[(family, d)]) < bound


@pytest.mark.parametrize("family,d,n", [("ising_d", 4, 5), ("ising_c", 4, 6), ("ising_e", 4, 6),
                                        ("ising_d", 6, 3), ("ising_e", 5, 3), ("ising_c", 6, 3)])
def test_cross_equals_brute_force_at_full_rank(family, d, n):
    """T3 = T2: where the cross reaches the full ranks min(n^(b+1), n^(m-b-1)) it holds the whole
    tensor (Thm. 2), so its quadrature is the rule's to the working precision."""
    tt = tm.solve(family, d, n, 64, 1e-40, seed=d)
    q = tm.tensor_quadrature_mp(family, d, n)
    m = d - 1
    assert tt.ranks() == [min(n ** (b + 1), n ** (m - b - 1)) for b in range(m - 1)]
    assert rel(tt.history[-1], q) < mp.mpf(10) ** -70, (tt.ranks(), mp.nstr(rel(tt.history[-1], q), 5))


def test_interpolation_on_the_fibres():
    """Thm. 1: the cross formula reproduces B on every fibre of its nested index sets."""
    tt = tm.TTCrossMP("ising_d", 6, 4, 8, 1e-30, seed=3, max_sweeps=4)
    for _ in range(4):
        tt.sweep()
    m, n = tt.m, tt.n
    with mp.workprec(PREC):
        lus = [tm.LU(tt.cross_matrix(b)) for b in range(m - 1)]
        for c in range(m):
            for l in tt.left_set(c - 1):
                for i in range(n):
                    for r in tt.right_set(c):
                        idx = l + (i,) + r
                        # eq. tt evaluated at idx: F_0(i_0) M_0^-1 F_1(i_1) ... F_{m-1}(i_{m-1})
                        v = [tt.B((idx[0],) + rr) for rr in tt.right[0]]
                        for k in range(1, m):
                            v = lus[k - 1].solve_transposed(v)
                            L, R = tt.left[k - 1], tt.right_set(k)
                            v = [mp.fsum(v[a] * tt.B(L[a] + (idx[k],) + rr) for a in range(len(L))) for rr in R]
                        assert abs(v[0] - tt.B(idx)) < mp.mpf(10) ** -60 * abs(tt.B(idx))


def test_matches_the_double_double_oracle_to_its_precision():
    """Same decisions and values as the double-double oracle to about 1e-28 on a small D_5."""
    from oracle.ttcross_dd import solve_dd
    dd = solve_dd("ising_d", 5, 6, 16, 1e-21, seed=5)
    mpo = tm.solve("ising_d", 5, 6, 16, 1e-21, seed=5)
    assert dd.ranks() == mpo.ranks() and dd.sweeps == mpo.sweeps
    for s, (a, b) in enumerate(zip(dd.pivot_log, mpo.pivot_log)):
        for x, y in zip(a, b):
            assert x.accepted == y.accepted, (s, x, y)
            if x.accepted:   # a rejected search's position is an argmax over rounding noise
                assert (x.row, x.col) == (y.row, y.col), (s, x, y)
    with mp.workprec(PREC):
        v = mp.mpf(dd.history[-1]) + mp.mpf(dd.history_lo[-1])
        assert rel(v, mpo.history[-1]) < 1e-27


# ----------------------------------------------------------- planted mistakes
def load_copy(tmp_path, name, old, new):
    pkg = tmp_path / name
    shutil.copytree(os.path.join(ROOT, "oracle"), pkg, ignore=shutil.ignore_patterns("__pycache__"))
    path = pkg / "ttcross_mp.py"
    src = path.read_text()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    path.write_text(src.replace(old, new))
    sys.path.insert(0, str(tmp_path))
    try:
        return importlib.import_module(f"{name}.ttcross_mp")
    finally:
        sys.path.remove(str(tmp_path))


def pin_closed_c3(o):
    return rel(o.tensor_quadrature_mp("ising_c", 3, 40), closed_forms()[("ising_c", 3)]) < 1e-45


def pin_closed_d3(o):
    return rel(o.tensor_quadrature_mp("ising_d", 3, 40), closed_forms()[("ising_d", 3)]) < 1e-45


def pin_t3_t2(o):
    tt = o.solve("ising_d", 6, 3, 64, 1e-40, seed=6)
    return rel(tt.history[-1], tm.tensor_quadrature_mp("ising_d", 6, 3)) < 1e-60


MUTATIONS = [
    ("node map", "t.append((x + 1) / 2)", "t.append((x + 1) / 3)", pin_closed_c3),
    ("weight square", "w.append(1 / ((1 - x * x) * dp * dp))", "w.append(1 / ((1 - x * x) * dp))", pin_closed_c3),
    ("pair square", "a_d *= ((1 - p) / (1 + p)) ** 2", "a_d *= ((1 - p) / (1 + p))", pin_closed_d3),
    ("suffix range", "prod_range(k, d) for k in range(2, d + 1)", "prod_range(k, d) for k in range(3, d + 1)",
     pin_closed_c3),
    ("transposed solve", "v = LU(self.cross_matrix(c - 1)).solve_transposed(v)",
     "v = LU(self.cross_matrix(c - 1)).solve(v)", pin_t3_t2),
    ("weight scale left in", "return v[0] * mp.ldexp(1, -self.wshift * m)", "return v[0]", pin_t3_t2),
    ("back substitution", "y[i] = (y[i] - mp.fsum(a[i][j] * y[j] for j in range(i + 1, n))) / a[i][i]",
     "y[i] = (y[i] - mp.fsum(a[i][j] * y[j] for j in range(i, n))) / a[i][i]", pin_t3_t2),
]


@pytest.mark.parametrize("k", range(len(MUTATIONS)))
def test_planted_mistake_breaks_a_pin(k, tmp_path):
    what, old, new, pin = MUTATIONS[k]
    assert pin(tm), f"pin fails on the unmutated oracle: {pin.__name__}"
    mutated = load_copy(tmp_path, f"oracle_mp_mut{k}", old, new)
    try:
        ok = pin(mutated)
    except (ZeroDivisionError, FloatingPointError, ValueError):
        ok = False
    assert not ok, f"planted mistake '{what}' passes {pin.__name__}"
