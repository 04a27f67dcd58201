"""Planted mistakes: each plausible slip in the oracle must break one of its pins.

A mutated copy of the oracle package is written to a temporary directory,
imported under another name, and checked with the same kind of pin the
regular tests use.  Every mutation must fail its pin, and the unmutated copy
must pass it (so the pin is not failing for an unrelated reason).
"""
import importlib
import os
import shutil
import sys

import mpmath as mp
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


def load_copy(tmp_path, name, file=None, old=None, new=None):
    pkg = tmp_path / name
    shutil.copytree(ORACLE, pkg, ignore=shutil.ignore_patterns("__pycache__"))
    if file is not None:
        path = pkg / file
        src = path.read_text()
        assert src.count(old) >= 1, f"mutation anchor not found in {file}: {old!r}"
        path.write_text(src.replace(old, new))
    sys.path.insert(0, str(tmp_path))
    try:
        return {m: importlib.import_module(f"{name}.{m}")
                for m in ("rng", "gauss", "integrands", "quadrature", "ttcross", "ddarith", "ttcross_dd",
                          "montecarlo")}
    finally:
        sys.path.remove(str(tmp_path))


def closed(key):
    with mp.workdps(30):
        L3 = (mp.zeta(2, mp.mpf(1) / 3) - mp.zeta(2, mp.mpf(2) / 3)) / 9
        return float({"c3": L3, "c4": 7 * mp.zeta(3) / 12,
                      "d4": 4 * mp.pi ** 2 / 9 - mp.mpf(1) / 6 - 7 * mp.zeta(3) / 2}[key])


# ---------------------------------------------------------------- pins
def pin_d2(o):
    t, w = o["gauss"].gauss_legendre_01(40)
    return abs(np.dot(w, o["integrands"].f_values("ising_d", t.reshape(-1, 1))) - 1 / 3) < 1e-15


def pin_c2(o):
    t, w = o["gauss"].gauss_legendre_01(40)
    return abs(np.dot(w, o["integrands"].f_values("ising_c", t.reshape(-1, 1))) - 1.0) < 1e-15


def pin_c3_brute(o):
    return abs(o["quadrature"].tensor_quadrature("ising_c", 2, 24) / closed("c3") - 1) < 1e-14


def pin_d4_tt(o):
    tt = o["ttcross"].solve("ising_d", 4, 24, 32, 1e-13, seed=4)
    return abs(tt.history[-1] / closed("d4") - 1) < 1e-12


def pin_rank2(o):
    r = np.random.default_rng(5)
    params = {"a": r.uniform(0.5, 4, 4).tolist(), "b": r.uniform(0.5, 4, 4).tolist()}
    try:
        tt = o["ttcross"].solve("sum2_exp_cos", 4, 6, 8, 1e-12, seed=9, params=params)
    except np.linalg.LinAlgError:
        return False
    q = o["quadrature"].tensor_quadrature("sum2_exp_cos", 4, 6, params)
    # at exact rank 2 every later search must see errors at the rounding level only
    late = [abs(rec.err) for sweep in tt.pivot_log[1:] for rec in sweep if rec.searched]
    return (max(tt.ranks()) == 2 and abs(tt.history[-1] - q) < 1e-13 * abs(q)
            and all(e < 1e-14 * abs(q) for e in late))


def pin_gl(o):
    t, w = o["gauss"].gauss_legendre_01(16)
    return abs(w.sum() - 1) < 1e-15 and all(abs(np.dot(w, t ** k) - 1 / (k + 1)) < 1e-15
                                            for k in range(32))


def pin_rng(o):
    return o["rng"].stream(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def pin_rook(o):
    # the matrix case (m = 2): check Alg. 2's result against the skeleton
    # formula eq. mat on the full matrix, over several sweeps
    tt = o["ttcross"].TTCross("ising_d", 3, 16, 12, 1e-15, seed=6, max_sweeps=6)
    full = np.array([[tt.B([(i, j)])[0] for j in range(16)] for i in range(16)])
    ok = True
    for _ in range(5):
        cores = [tt.core(c) for c in range(tt.m)]
        rec = tt.cross_step(0, tt.sweeps, cores)
        I = [l[0] for l in tt.left[0]]
        J = [r[0] for r in tt.right[0]]
        err = full - full[:, J] @ np.linalg.solve(full[np.ix_(I, J)], full[I, :])
        ok = ok and abs(err[rec.row, rec.col] - rec.err) < 1e-14 * np.abs(full).max()
        ok = ok and abs(err[rec.row, rec.col]) >= np.abs(err[rec.row, :]).max() * (1 - 1e-12)
        if rec.iters < o["ttcross"].T_ROOK:    # ended by the rook condition: column-dominant too
            ok = ok and abs(err[rec.row, rec.col]) >= np.abs(err[:, rec.col]).max() * (1 - 1e-12)
        tt.sweep()
        if tt.stop_reason:
            break
    return ok


def pin_dd_ops(o):
    DD = o["ddarith"].DD
    r = np.random.default_rng(2)
    a = DD(r.uniform(-2, 2, 200), r.uniform(-1, 1, 200) * 2.0 ** -56)
    b = DD(r.uniform(0.5, 2, 200), r.uniform(-1, 1, 200) * 2.0 ** -56)
    with mp.workdps(60):
        am = [mp.mpf(float(h)) + mp.mpf(float(l)) for h, l in zip(a.hi, a.lo)]
        bm = [mp.mpf(float(h)) + mp.mpf(float(l)) for h, l in zip(b.hi, b.lo)]
        for c, f in ((a + b, lambda x, y: x + y), (a * b, lambda x, y: x * y), (a / b, lambda x, y: x / y)):
            for i in range(200):
                ref = f(am[i], bm[i])
                if abs(mp.mpf(float(c.hi[i])) + mp.mpf(float(c.lo[i])) - ref) > 2.0 ** -102 * abs(ref):
                    return False
    return True


def pin_dd_integrand(o):
    from test_oracle_dd import mp_paper_form
    DD = o["ddarith"].DD
    r = np.random.default_rng(4)
    x = DD(r.uniform(0, 1, (10, 5)))
    v = o["integrands"].f_values_dd("ising_d", x)
    with mp.workdps(60):
        return all(abs((mp.mpf(float(v.hi[p])) + mp.mpf(float(v.lo[p])))
                       / mp_paper_form("ising_d", [mp.mpf(float(q)) for q in x.hi[p]]) - 1) < 1e-29
                   for p in range(10))


def pin_dd_quad(o):
    hi, lo = o["quadrature"].tensor_quadrature_dd("ising_d", 2, 32)
    with mp.workdps(50):
        L3 = (mp.zeta(2, mp.mpf(1) / 3) - mp.zeta(2, mp.mpf(2) / 3)) / 9
        return abs((mp.mpf(hi) + mp.mpf(lo)) / (8 + 4 * mp.pi ** 2 / 3 - 27 * L3) - 1) < 1e-29


def pin_dd_tt(o):
    tt = o["ttcross_dd"].solve_dd("ising_d", 4, 24, 24, 1e-28, seed=4)
    with mp.workdps(50):
        d4 = 4 * mp.pi ** 2 / 9 - mp.mpf(1) / 6 - 7 * mp.zeta(3) / 2
        return abs((mp.mpf(tt.history[-1]) + mp.mpf(tt.history_lo[-1])) / d4 - 1) < 1e-25


def pin_mc(o):
    mcm = o["montecarlo"]
    t, w = o["gauss"].gauss_legendre_01(64)
    fc = o["integrands"].f_values("ising_c", t.reshape(-1, 1))
    sd_c = float(np.sqrt(np.dot(w, fc * fc) - np.dot(w, fc) ** 2))
    mean, _ = mcm.error_estimate(mcm.estimators("ising_c", 2, 512, 16, mcm.RANDOM, seed=5))
    if not abs(mean - 1.0) < 5 * sd_c / np.sqrt(512 * 16):     # C_2 = 1
        return False
    f = o["integrands"].f_values("ising_d", t.reshape(-1, 1))
    sd = float(np.sqrt(np.dot(w, f * f) - np.dot(w, f) ** 2))
    _, eps2 = mcm.error_estimate(mcm.estimators("ising_d", 2, 400, 40, mcm.RANDOM, seed=11))
    x = mcm.lattice_points([1, 34], 89, mcm.shift(7, 0, 2))
    return 0.65 < eps2 / (sd / 20 / np.dot(w, f)) < 1.35 and bool(np.all(x < 1))


def pin_scaled_weights(o):
    tt = o["ttcross"]
    a = tt.TTCross("ising_d", 5, 10, 6, 1e-12, seed=3, max_sweeps=3)
    b = tt.TTCross("ising_d", 5, 10, 6, 1e-12, seed=3, max_sweeps=3, scale_weights=False)
    a.run()
    b.run()
    return a.history == b.history


def pin_scaled_chain(o):
    d, n = 300, 16
    a = np.random.default_rng(7).uniform(0.05, 0.3, d)
    tt = o["ttcross"].solve("prod_exp", d, n, 2, 1e-12, seed=1, max_sweeps=2,
                            params={"a": list(a), "b": [1.0] * d})
    t, w = o["gauss"].gauss_legendre_01(n)
    log_q = sum(np.log(np.dot(w, np.exp(-aj * t))) for aj in a)
    mant, e = tt.history_scaled[-1]
    if not 0.5 <= mant < 1.0:
        return False
    return bool(abs(np.log(mant) + e * np.log(2.0) - log_q) < 1e-10 * abs(log_q))


MUTATIONS = [
    # (file, original text, planted mistake, pin that must catch it)
    ("integrands.py", "a_d = a_d * ((1.0 - p) / (1.0 + p)) ** 2", "a_d = a_d * ((1.0 - p) / (1.0 + p))",
     pin_d2),                                                                # dropped square
    ("integrands.py", "s_right = s_right + prod_range(k, d)", "s_right = s_right + prod_range(2, k)",
     pin_c3_brute),                                                          # wrong index range
    ("integrands.py", "f = np.full(npts, 2.0)", "f = np.full(npts, 1.0)", pin_c2),   # lost prefactor
    ("integrands.py", "wt = np.prod(w[idx], axis=1)", "wt = np.prod(w[idx][:, :-1], axis=1)",
     pin_c3_brute),                                                          # dropped weight
    ("ttcross.py", "v = np.linalg.solve(M.T, v.T).T", "v = np.linalg.solve(M, v.T).T", pin_d4_tt),
    ("ttcross.py", "X = np.linalg.solve(M, Fb1[:, cols])", "X = np.linalg.solve(M.T, Fb1[:, cols])",
     pin_rank2),                                                             # transposed operand
    ("ttcross.py", "row = argmax_abs(a_col - approx(all_rows, [col] * nrows))",
     "row = argmax_abs(a_col)", pin_rook),                                   # dropped B~ term
    ("gauss.py", "w.append(1 / ((1 - x * x) * dp * dp))",
     "w.append(2 / ((1 - x * x) * dp * dp))", pin_gl),                       # interval map
    ("rng.py", "GAMMA = 0x9E3779B97F4A7C15", "GAMMA = 0x9E3779B97F4A7C13", pin_rng),
    ("rng.py", "z = ((z ^ (z >> 27)) * M2) & MASK", "z = ((z ^ (z >> 28)) * M2) & MASK", pin_rng),
    ("ttcross.py", "return mant, e + k - self.wshift * self.m", "return mant, e + k",
     pin_scaled_weights),                                                    # weight scale kept
    ("ttcross.py", "v = np.ldexp(v, -k)", "v = np.ldexp(v, k)", pin_scaled_chain),   # wrong-way rescale
    # double-double oracle
    ("ddarith.py", "e = e + (self.hi * y.lo + self.lo * y.hi)", "e = e + self.hi * y.lo", pin_dd_ops),
    ("ddarith.py", "SPLITTER = 134217729.0", "SPLITTER = 67108865.0", pin_dd_ops),
    ("ddarith.py", "        e = e + t\n", "        e = e\n", pin_dd_ops),    # dropped low-part sum
    ("ddarith.py", "X[k, :] = s / A[k, k]", "X[k, :] = s / A[k, k].hi", pin_dd_tt),
    ("integrands.py", "a_d = a_d * ((1.0 - p) / (1.0 + p)).square()", "a_d = a_d * ((1.0 - p) / (1.0 + p))",
     pin_dd_integrand),
    ("ttcross_dd.py", "v = dd_solve(M.T, v.T).T", "v = dd_solve(M, v.T).T", pin_dd_tt),
    ("ttcross_dd.py", "return dd_sum(Fb[np.asarray(rows), :] * X.T, axis=1)",
     "return DD(dd_sum(Fb[np.asarray(rows), :] * X.T, axis=1).hi)", pin_dd_tt),
    ("gauss.py", "return DD.from_mp(t), DD.from_mp(w)", "return DD.from_mp(t), DD([float(v) for v in w])",
     pin_dd_quad),
    # Monte Carlo / lattice oracle
    ("montecarlo.py", "    mean = sum(ests) / S", "    mean = sum(ests) / (S - 1)", pin_mc),
    ("montecarlo.py", "return mean, math.sqrt(var) / abs(mean)", "return mean, var / abs(mean)", pin_mc),
    ("montecarlo.py", "x[i - 1, k] = v - 1.0 if v >= 1.0 else v", "x[i - 1, k] = v", pin_mc),
]


@pytest.mark.parametrize("k", range(len(MUTATIONS)))
def test_planted_mistake_is_caught(tmp_path, k):
    file, old, new, pin = MUTATIONS[k]
    good = load_copy(tmp_path, f"oracle_ok_{k}")
    assert pin(good), "the pin must pass on the unmodified oracle"
    bad = load_copy(tmp_path, f"oracle_mut_{k}", file, old, new)
    try:
        caught = not pin(bad)
    except (FloatingPointError, np.linalg.LinAlgError, ValueError, ZeroDivisionError):
        caught = True
    assert caught, f"planted mistake in {file} not caught: {new}"
