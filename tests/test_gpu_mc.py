"""Parity of the GPU Monte Carlo / shifted-lattice quadratures (Sec. 4.2) with the oracle.

Both sides draw the same points (the same counter-based generator, the same
lattice arithmetic), so the estimators differ only by the rounding of the
integrand and of the sums: each estimator within 1e-12 relative; the
relative error estimate (a standard deviation of estimators that differ
relatively by about that error) within 1e-8 relative.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from gpu_util import gpu_context
from oracle import montecarlo as omc
from paper_1903_11554_amd.ttcross import MC_LATTICE, MC_RANDOM, TTError
from paper_1903_11554_amd.workloads import Problem, synthetic_params

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("family,d", [("ising_c", 3), ("ising_d", 5), ("ising_e", 4),
                                      ("sum2_exp_cos", 6), ("ising_d_u", 3), ("ising_c", 2)])
def test_monte_carlo_matches_oracle(family, d):
    ctx = gpu_context()
    params = synthetic_params(d, 4) if family == "sum2_exp_cos" else None
    p = Problem(family, d, 16, 8, 1e-10, seed=21, params=params)
    N, S = 2048 + 37, 4
    print(f"mc {family} d={d}", flush=True)
    est, mean, err = ctx.mc_integrate(p, N, S, MC_RANDOM)
    ref = omc.estimators(family, d, N, S, omc.RANDOM, seed=21, params=params)
    rmean, rerr = omc.error_estimate(ref)
    np.testing.assert_allclose(est, ref, rtol=1e-12, atol=0)
    assert abs(mean / rmean - 1) < 1e-12
    assert abs(err / rerr - 1) < 1e-8


@pytest.mark.parametrize("family,d,N,gen", [("ising_c", 3, 987, [1, 610]),
                                            ("ising_d", 5, 1021, [1, 76, 671, 977])])
def test_lattice_matches_oracle(family, d, N, gen):
    ctx = gpu_context()
    p = Problem(family, d, 16, 8, 1e-10, seed=33)
    est, mean, err = ctx.mc_integrate(p, N, 6, MC_LATTICE, gen=gen)
    ref = omc.estimators(family, d, N, 6, omc.LATTICE, seed=33, gen=gen)
    rmean, rerr = omc.error_estimate(ref)
    np.testing.assert_allclose(est, ref, rtol=1e-12, atol=0)
    assert abs(mean / rmean - 1) < 1e-12
    assert abs(err / rerr - 1) < 1e-8


def test_large_monte_carlo_is_unbiased_for_c4():
    # 2^20 points x 8 estimators on C_4 = 7 zeta(3)/12: within 5 standard errors of the mean
    ctx = gpu_context()
    p = Problem("ising_c", 4, 16, 8, 1e-10, seed=4)
    est, mean, err = ctx.mc_integrate(p, 1 << 20, 8, MC_RANDOM)
    with mp.workdps(30):
        c4 = float(7 * mp.zeta(3) / 12)
    print(f"C_4 MC: mean {mean} rel err {err} vs {c4}", flush=True)
    assert abs(mean - c4) < 5 * err * abs(mean) / math.sqrt(8)
    assert 0 < err < 1e-3


def test_invalid_arguments():
    ctx = gpu_context()
    p = Problem("ising_d", 5, 16, 8, 1e-10)
    with pytest.raises(TTError):
        ctx.mc_integrate(p, 1024, 1, MC_RANDOM)            # one estimator: no error estimate
    with pytest.raises(TTError):
        ctx.mc_integrate(p, 1024, 4, MC_LATTICE)           # lattice without a generating vector
    with pytest.raises(TTError):
        ctx.mc_integrate(Problem("ising_d", 5, 16, 8, 1e-20, precision="dd"), 1024, 4, MC_RANDOM)
