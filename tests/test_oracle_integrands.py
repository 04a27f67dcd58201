"""Pins for the oracle integrands: closed forms and adaptive quadrature.

None of these re-implements the integrand: every expected value is a closed
form of the integral or an independent adaptive quadrature (scipy) of it.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

from oracle.gauss import gauss_legendre_01
from oracle.integrands import (exact_synthetic, f_values, n_modes, weighted_values)


def gl_1d(family, n=48):
    t, w = gauss_legendre_01(n)
    return float(np.dot(w, f_values(family, t.reshape(-1, 1))))


def test_mode_counts():
    assert n_modes("ising_d", 10) == 9
    assert n_modes("ising_c_u", 3) == 3
    assert n_modes("sum2_exp_cos", 8) == 8


def test_d1_is_two():
    for fam in ("ising_c", "ising_d", "ising_e"):
        assert f_values(fam, np.zeros((3, 0))).tolist() == [2.0, 2.0, 2.0]


def test_c2_equals_one():
    # C_2 = 2 int_0^1 (1+x)^-2 dx = 1
    assert abs(gl_1d("ising_c") - 1.0) < 1e-15


def test_d2_equals_one_third():
    # D_2 = 2 int_0^1 (1-x)^2/(1+x)^4 dx = 1/3
    assert abs(gl_1d("ising_d") - 1.0 / 3.0) < 2e-16 * 4


def test_e2_closed_form():
    # E_2 = 2 int_0^1 ((1-x)/(1+x))^2 dx = 6 - 8 ln 2
    with mp.workdps(30):
        want = float(6 - 8 * mp.log(2))
    assert abs(gl_1d("ising_e") - want) < 2e-15 * want


def test_u_form_c1_equals_two():
    val, err = integrate.quad(lambda x: f_values("ising_c_u", np.array([[x]]))[0], 0, 1,
                              epsabs=0, epsrel=1e-13, limit=200)
    assert abs(val - 2.0) < 1e-11


@pytest.mark.parametrize("family,expect", [("ising_c_u", 1.0), ("ising_d_u", 1.0 / 3.0)])
def test_u_form_two_variables(family, expect):
    f = lambda y, x: f_values(family, np.array([[x, y]]))[0]
    val, err = integrate.dblquad(f, 0, 1, 0, 1, epsabs=0, epsrel=1e-11)
    assert abs(val - expect) < 1e-9


def test_paper_and_u_form_agree_pointwise_structure():
    # the D u-form vanishes where two variables coincide (a property of the formula)
    x = np.array([[0.3, 0.3, 0.7]])
    assert f_values("ising_d_u", x)[0] == 0.0


def test_synthetic_exact_1d():
    params = {"a": [1.7], "b": [2.9]}
    t, w = gauss_legendre_01(32)
    for fam in ("prod_exp", "sum2_exp_cos"):
        got = float(np.dot(w, f_values(fam, t.reshape(-1, 1), params)))
        assert abs(got - exact_synthetic(fam, params, 1)) < 1e-15


def test_weighted_values_fold_weights():
    t, w = gauss_legendre_01(6)
    idx = np.array([[0, 5, 2], [3, 3, 1]])
    got = weighted_values("ising_d", idx, t, w)
    want = np.prod(w[idx], axis=1) * f_values("ising_d", t[idx])
    np.testing.assert_array_equal(got, want)
