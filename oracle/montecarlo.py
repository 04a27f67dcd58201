"""Equal-weight quadratures: Monte Carlo and randomly shifted lattice rules — oracle side.

Test infrastructure only.  Sec. 4.2 of the paper:

* Monte Carlo (eq. mc): I ~ (1/N) sum_{i=1..N} f(x_i), x_i uniform on [0,1]^m;
* lattice rule with a random shift (eq. qmc): x_i = frac(i q / N + s),
  i = 1..N, for a generating vector q of integers and a shift s uniform on
  [0,1]^m;
* both repeated S times (new points, or new shifts with the same q), with the
  error estimated as the empirical standard deviation of the S estimators
  relative to their mean (eq. std):
      eps = sqrt( sum_j (I_j - <I>)^2 / (S-1) ) / <I>,   <I> = (1/S) sum_j I_j.

Readings (the paper does not fix them): the random numbers are SplitMix64
draws keyed by (seed, estimator, point, coordinate) (oracle/rng.py), mapped to
the open interval (0, 1) so that integrands singular on the boundary (the
u-form) stay finite; the lattice point is formed as frac(((i q_k) mod N)/N +
s_k) with exact integer arithmetic for i q_k.  The paper's own generating
vectors are not available; the lattice rule takes a caller's vector.

The integrand is the unweighted f of oracle/integrands.py (the factor 2 of
eqs. c/d/e included).  Every estimator is a plain sum in point order.

Pinned by: unbiasedness against exact integrals (synthetic families, C_2 = 1,
D_2 = 1/3) within the statistical error, the error estimate against the
variance of f computed by Gauss--Legendre quadrature, and the exactness of a
rank-1 lattice rule for the trigonometric polynomials it integrates exactly
(tests/test_oracle_montecarlo.py).
"""

import math

import numpy as np

from . import rng
from .integrands import f_values, n_modes

RANDOM, LATTICE = 0, 1


def random_points(seed, j, n_points, m):
    """The N x m points of Monte Carlo estimator j."""
    x = np.empty((n_points, m))
    for i in range(n_points):
        for k in range(m):
            x[i, k] = rng.uniform_open01(rng.value(seed, rng.mc_counter(j, i, m, k)))
    return x


def shift(seed, j, m):
    """The random shift of lattice estimator j."""
    return np.array([rng.uniform_open01(rng.value(seed, rng.shift_counter(j, k))) for k in range(m)])


def lattice_points(gen, n_points, s):
    """x_i = frac(i q / N + s), i = 1..N (eq. qmc)."""
    m = len(gen)
    x = np.empty((n_points, m))
    for i in range(1, n_points + 1):
        for k in range(m):
            v = ((i * int(gen[k])) % n_points) / n_points + s[k]
            x[i - 1, k] = v - 1.0 if v >= 1.0 else v
    return x


def estimators(family, d, n_points, n_sets, kind, seed, gen=None, params=None):
    """The S estimators I_j (eq. mc on random points or on shifted lattice points)."""
    m = n_modes(family, d)
    out = []
    for j in range(n_sets):
        if kind == RANDOM:
            x = random_points(seed, j, n_points, m)
        else:
            x = lattice_points(gen, n_points, shift(seed, j, m))
        f = f_values(family, x, params)
        total = 0.0
        for v in f:            # plain sum in point order
            total += v
        out.append(total / n_points)
    return out


def error_estimate(ests):
    """(<I>, eps) of eq. std."""
    S = len(ests)
    mean = sum(ests) / S
    var = sum((e - mean) ** 2 for e in ests) / (S - 1)
    return mean, math.sqrt(var) / abs(mean)
