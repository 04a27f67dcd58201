"""Pins for brute-force tensor quadrature (eq. quad_product) against closed forms.

Closed forms of the low-dimensional Ising integrals (Bailey, Borwein & Crandall,
"Integrals of the Ising class", 2006, cited by the paper as the source of the
integrals): C_3 = L_{-3}(2), C_4 = 7 zeta(3)/12, D_3 = 8 + 4 pi^2/3 - 27 L_{-3}(2),
D_4 = 4 pi^2/9 - 1/6 - 7 zeta(3)/2, where L_{-3}(2) = sum_k (3k+1)^-2 - (3k+2)^-2.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle.integrands import exact_synthetic
from oracle.quadrature import tensor_quadrature


def closed_forms():
    with mp.workdps(40):
        L3 = (mp.zeta(2, mp.mpf(1) / 3) - mp.zeta(2, mp.mpf(2) / 3)) / 9
        return {
            ("ising_c", 1): 2.0, ("ising_d", 1): 2.0,
            ("ising_c", 2): 1.0, ("ising_d", 2): 1.0 / 3.0,
            ("ising_c", 3): float(L3),
            ("ising_c", 4): float(7 * mp.zeta(3) / 12),
            ("ising_d", 3): float(8 + 4 * mp.pi ** 2 / 3 - 27 * L3),
            ("ising_d", 4): float(4 * mp.pi ** 2 / 9 - mp.mpf(1) / 6 - 7 * mp.zeta(3) / 2),
        }


def test_l3_series_definition():
    # L_{-3}(2) from its Dirichlet series, summed directly (slowly convergent: use mpmath nsum)
    with mp.workdps(30):
        direct = mp.nsum(lambda k: 1 / (3 * k + 1) ** 2 - 1 / (3 * k + 2) ** 2, [0, mp.inf])
    assert abs(float(direct) - closed_forms()[("ising_c", 3)]) < 1e-15


@pytest.mark.parametrize("key,n,tol", [
    (("ising_c", 1), 4, 0.0), (("ising_d", 1), 4, 0.0),
    (("ising_c", 2), 24, 1e-15), (("ising_d", 2), 24, 1e-15),
    (("ising_c", 3), 24, 1e-14), (("ising_d", 3), 32, 1e-14),
    (("ising_c", 4), 24, 1e-14), (("ising_d", 4), 32, 1e-13),
])
def test_brute_force_matches_closed_forms(key, n, tol):
    family, d = key
    got = tensor_quadrature(family, d - 1, n)
    want = closed_forms()[key]
    assert abs(got - want) <= tol * abs(want) + (0 if tol else 1e-300)


def test_brute_force_separable_product():
    params = {"a": [0.7, 1.9, 3.1], "b": [0.6, 2.2, 3.9]}
    for fam in ("prod_exp", "sum2_exp_cos"):
        got = tensor_quadrature(fam, 3, 20, params)
        assert abs(got - exact_synthetic(fam, params, 3)) < 2e-15


def test_u_form_converges_to_paper_form_slowly():
    # The u-form of C_3 integrates the same value, but its tensor GL rule converges
    # only algebraically (no closed-form target at finite n, only the trend).
    want = closed_forms()[("ising_c", 3)]
    e16 = abs(tensor_quadrature("ising_c_u", 3, 16) - want)
    e32 = abs(tensor_quadrature("ising_c_u", 3, 32) - want)
    assert e32 < e16 / 4 and e32 / want < 1e-3
