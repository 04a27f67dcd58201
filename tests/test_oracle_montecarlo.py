"""Pins for the Monte Carlo / shifted-lattice oracle (Sec. 4.2, eqs. mc, qmc, std)."""
import math

import numpy as np

from oracle import montecarlo as mc
from oracle import rng
from oracle.gauss import gauss_legendre_01
from oracle.integrands import exact_synthetic, f_values
from paper_1903_11554_amd.workloads import synthetic_params


def test_points_are_uniform_in_the_open_unit_cube():
    x = mc.random_points(3, 0, 4000, 3)
    assert np.all(x > 0) and np.all(x < 1)
    # first two moments of U(0,1): 1/2 and 1/3, within 5 standard errors
    assert np.all(np.abs(x.mean(axis=0) - 0.5) < 5 * math.sqrt(1 / 12 / 4000))
    assert np.all(np.abs((x ** 2).mean(axis=0) - 1 / 3) < 5 * math.sqrt(4 / 45 / 4000))
    # different estimators draw different points
    assert not np.array_equal(x, mc.random_points(3, 1, 4000, 3))


def sd_of_f(family, d, params=None):
    """Standard deviation of f over [0,1]^m by a tensor Gauss--Legendre rule (m <= 4)."""
    import itertools
    m = d - 1 if family.startswith("ising") else d
    t, w = gauss_legendre_01(24)
    idx = np.array(list(itertools.product(range(24), repeat=m)))
    f = f_values(family, t[idx], params)
    wt = np.prod(w[idx], axis=1)
    mean = np.dot(wt, f)
    return math.sqrt(np.dot(wt, f * f) - mean ** 2)


def test_monte_carlo_is_unbiased_against_exact_integrals():
    # the mean of S estimators of N points lies within 5 sd(f)/sqrt(N S) of the integral
    cases = [("ising_c", 2, None, 1.0), ("ising_d", 2, None, 1.0 / 3.0)]
    p = synthetic_params(4, 9)
    cases.append(("sum2_exp_cos", 4, p, exact_synthetic("sum2_exp_cos", p, 4)))
    N, S = 512, 16
    for family, d, params, exact in cases:
        ests = mc.estimators(family, d, N, S, mc.RANDOM, seed=5, params=params)
        mean, eps = mc.error_estimate(ests)
        assert abs(mean - exact) < 5 * sd_of_f(family, d, params) / math.sqrt(N * S), (family, mean, exact)


def test_error_estimate_matches_the_variance_of_f():
    # eq. std estimates sqrt(var f / N) / I; var f of D_2 from a 64-point GL rule
    t, w = gauss_legendre_01(64)
    f = f_values("ising_d", t.reshape(-1, 1))
    mean_f = np.dot(w, f)
    sd = math.sqrt(np.dot(w, f * f) - mean_f ** 2)
    N, S = 400, 40
    ests = mc.estimators("ising_d", 2, N, S, mc.RANDOM, seed=11)
    _, eps = mc.error_estimate(ests)
    predicted = sd / math.sqrt(N) / mean_f
    # the sample standard deviation of 40 estimators is within 35% of the truth
    # far beyond 5 standard errors (its relative standard error is 1/sqrt(2(S-1)) ~ 11%)
    assert 0.65 < eps / predicted < 1.35, (eps, predicted)


def test_lattice_rule_is_exact_on_the_trigonometric_polynomials_it_resolves():
    # a rank-1 lattice rule integrates exp(2 pi i h.x) exactly (to 0) unless h.q = 0 mod N,
    # whatever the shift: check the lattice points against that identity
    N, q = 89, [1, 34]            # Fibonacci lattice
    s = mc.shift(7, 0, 2)
    x = mc.lattice_points(q, N, s)
    for h in [(1, 0), (0, 1), (1, 1), (2, -3), (5, 7)]:
        dot = (h[0] * q[0] + h[1] * q[1]) % N
        val = np.mean(np.exp(2j * np.pi * (h[0] * x[:, 0] + h[1] * x[:, 1])))
        if dot != 0:
            assert abs(val) < 1e-12, (h, val)
    # (34, -1) . q = 34 - 34 = 0: resolved as 1 in modulus
    val = np.mean(np.exp(2j * np.pi * (34 * x[:, 0] - x[:, 1])))
    assert abs(abs(val) - 1) < 1e-12
    assert np.all(x >= 0) and np.all(x < 1)


def test_lattice_estimators_of_a_smooth_integrand():
    # shifted Fibonacci lattice on C_3 (two modes): unbiased, and far more accurate than MC
    N, q = 987, [1, 610]
    ests = mc.estimators("ising_c", 3, N, 8, mc.LATTICE, seed=3, gen=q)
    mean, eps = mc.error_estimate(ests)
    with __import__("mpmath").workdps(30):
        import mpmath as mp
        c3 = float((mp.zeta(2, mp.mpf(1) / 3) - mp.zeta(2, mp.mpf(2) / 3)) / 9)
    assert abs(mean / c3 - 1) < 5 * eps / math.sqrt(8) + 1e-12
    mc_ests = mc.estimators("ising_c", 3, N, 8, mc.RANDOM, seed=3)
    assert eps < mc.error_estimate(mc_ests)[1] / 5


def test_counters_do_not_collide_with_the_cross():
    assert rng.mc_counter(0, 0, 1, 0) > rng.sample_counter(1023, 31, 1 << 24)
    assert rng.mc_counter(4095, (1 << 31) - 1, 32, 31) < rng.shift_counter(0, 0)
    assert rng.shift_counter(4095, 63) < rng.start_counter(0, 0)
