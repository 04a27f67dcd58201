"""The start of jobs with more than 32 modes, and B carried as B 2^E (oracle side).

D_d falls near 10^(-0.7 d) (Sec. 5.5): from about d = 128 on a random grid
point's weighted value lies below the double range, so the start also takes the
n constant multi-indices as candidates, compares them in (mantissa, exponent)
form, and scales every B of the job by 2^E so that the start's B lies in
[1/2, 1).  Pinned here:
  * the logarithmic evaluation against the direct one wherever B is a normal
    double, and against a closed form on constant points far below the range;
  * the chosen start against a brute-force argmax over the same candidates;
  * the scaling's exactness: a run with E and one without take the same
    decisions, with every B and error differing by exactly 2^E, and the same
    integral;
  * planted mistakes (a dropped run multiplicity, a wrong sign of E).
"""
import math

import mpmath
import numpy as np
import pytest

from oracle import integrands
from oracle.gauss import gauss_legendre_01
from oracle.ttcross import TTCross


def closed_form_log2(family, m, x):
    """log2 f at the constant point (x, .., x) of m modes, from the run counts.

    A run of k consecutive coordinates has product x^k, and m + 1 - k runs have
    length k; B_d's prefix and suffix sums are both sum_{k=1..m} x^k.
    """
    with mpmath.workdps(60):
        x = mpmath.mpf(x)
        l = mpmath.mpf(1)    # log2 2
        if family in ("ising_d", "ising_e"):
            for k in range(1, m + 1):
                p = x ** k
                l += 2 * (m + 1 - k) * mpmath.log((1 - p) / (1 + p), 2)
        if family in ("ising_c", "ising_d"):
            q = mpmath.fsum(x ** k for k in range(1, m + 1))
            l -= 2 * mpmath.log(1 + q, 2)
        return float(l)


@pytest.mark.parametrize("family", ["ising_c", "ising_d", "ising_e"])
@pytest.mark.parametrize("m", [3, 17, 40, 90])
def test_log2_values_match_the_direct_evaluation(family, m):
    rng = np.random.default_rng(m)
    n = 33
    t, w = gauss_legendre_01(n)
    w = np.ldexp(w, 5)   # the folded weights of a job (times 2^s, s nearest log2 n)
    idx = np.vstack([rng.integers(0, n, size=(40, m)), np.repeat(np.arange(n)[:, None], m, axis=1)])
    direct = integrands.weighted_values(family, idx, t, w)
    ok = direct >= 2.0 ** -1000
    assert ok.sum() >= 12
    got = integrands.log2_weighted_values(family, idx[ok], t, w)
    want = np.log2(direct[ok])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * (m * m + np.abs(want)).max())


@pytest.mark.parametrize("family,m,n", [("ising_d", 255, 33), ("ising_d", 511, 65), ("ising_e", 300, 33),
                                        ("ising_c", 511, 33)])
def test_log2_values_on_constant_points_against_the_closed_form(family, m, n):
    t, _ = gauss_legendre_01(n)
    ones = np.ones(n)
    for j in (0, 3, 6, n // 2, n - 1):
        idx = np.full((1, m), j, dtype=np.int64)
        got = integrands.log2_weighted_values(family, idx, t, ones)[0]
        want = closed_form_log2(family, m, t[j])
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want)), (j, got, want)
    # far below the double range for the D family at these sizes
    if family == "ising_d":
        assert closed_form_log2(family, m, t[n // 2]) < -1100


def test_closed_form_catches_a_dropped_run_multiplicity():
    """Counting every run length once (instead of m + 1 - k times) is far off."""
    m, x = 60, 0.4
    good = closed_form_log2("ising_d", m, x)
    with mpmath.workdps(30):
        bad = 1 + sum(2 * mpmath.log((1 - x ** k) / (1 + x ** k), 2) for k in range(1, m + 1))
        bad -= 2 * mpmath.log(1 + sum(x ** k for k in range(1, m + 1)), 2)
    t = np.array([x])
    got = integrands.log2_weighted_values("ising_d", np.zeros((1, m), dtype=np.int64), t, np.ones(1))[0]
    assert abs(got - good) < 1e-10
    assert abs(float(bad) - good) > 1.0


def brute_start(tt, seed_idx):
    """argmax over the candidates of |B| from the direct evaluation (the largest is normal here)."""
    vals = integrands.weighted_values(tt.family, seed_idx, tt.t, tt.w)
    q = int(np.argmax(np.abs(vals)))
    assert abs(vals[q]) >= 2.0 ** -1022
    return q, vals


@pytest.mark.parametrize("family,d,n,seed", [("ising_d", 34, 5, 1), ("ising_c", 41, 8, 2),
                                             ("ising_e", 36, 6, 3)])
def test_start_is_the_largest_candidate_and_scales_it_into_half_one(family, d, n, seed):
    from oracle import rng
    tt = TTCross(family, d, n, 1, 1e-8, seed)
    m = tt.m
    nconst = n if family in ("ising_d", "ising_e") else 0   # C_d keeps the random candidates only
    cand = np.empty((1024 + nconst, m), dtype=np.int64)
    for q in range(1024):
        for k in range(m):
            cand[q, k] = rng.uniform_index(rng.value(seed, rng.start_counter(q, k)), n)
    cand[1024:] = np.arange(nconst)[:, None]
    q, vals = brute_start(tt, cand)
    assert tt.start_index == tuple(int(v) for v in cand[q])
    mant, e = math.frexp(abs(float(vals[q])))
    assert tt.escale == -e
    assert 0.5 <= tt.scale[0] < 1.0 and tt.scale[0] == mant
    assert tt.evals >= 1024 + nconst


def test_scaled_start_picks_a_constant_point_far_below_the_range():
    """D_129 with 33 nodes: most random candidates lie below the double range, the best constant point near 2^-101."""
    m = 128
    tt = TTCross("ising_d", m + 1, 33, 1, 1e-8, 129)
    j = tt.start_index[0]
    assert tt.start_index == (j,) * m
    t, w = tt.t, tt.w
    per_j = [closed_form_log2("ising_d", m, t[i]) + m * math.log2(w[i]) for i in range(33)]
    assert j == int(np.argmax(per_j))
    # the start's B = mantissa 2^-E with the mantissa in [1/2, 1)
    assert -tt.escale - 1 <= per_j[j] < -tt.escale and tt.escale > 80
    assert tt.history_scaled[0][0] != 0.0


@pytest.mark.parametrize("family,d,n,rank,seed", [("ising_d", 34, 5, 4, 5), ("ising_c", 36, 6, 5, 6)])
def test_scaling_by_two_to_the_e_changes_no_decision(family, d, n, rank, seed):
    a = TTCross(family, d, n, rank, 1e-9, seed, max_sweeps=6)
    b = TTCross(family, d, n, rank, 1e-9, seed, max_sweeps=6, value_scale=False)
    a.run()
    b.run()
    E = a.escale
    assert E != 0 and b.escale == 0
    assert a.start_index == b.start_index
    assert a.history == b.history
    assert len(a.pivot_log) == len(b.pivot_log)
    for la, lb in zip(a.pivot_log, b.pivot_log):
        for ra, rb in zip(la, lb):
            assert (ra.row, ra.col, ra.accepted, ra.iters) == (rb.row, rb.col, rb.accepted, rb.iters)
            assert ra.err == math.ldexp(rb.err, E) and ra.value == math.ldexp(rb.value, E)


def test_planted_wrong_sign_of_the_scale_is_caught():
    """Unscaling the integral by 2^+E instead of 2^-E moves it by 2^(2E)."""
    a = TTCross("ising_d", 34, 5, 3, 1e-9, 5, max_sweeps=2)
    a.run()
    mant, e = a.integral_scaled()
    b = TTCross("ising_d", 34, 5, 3, 1e-9, 5, max_sweeps=2, value_scale=False)
    b.run()
    assert math.ldexp(mant, e) == b.history[-1]
    wrong = math.ldexp(mant, e + 2 * a.escale)
    assert abs(wrong - b.history[-1]) > 1e3 * abs(b.history[-1])
