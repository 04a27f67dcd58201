"""Integrands and the weighted tensor B — oracle side (test infrastructure only).

Ising integrals, paper form (Sec. 5.1, eqs. c, d, e), integrated over
[0,1]^(d-1) in the variables x_2 .. x_d:

    C_d = 2 * int B_d,   D_d = 2 * int A_d B_d,   E_d = 2 * int A_d,
    A_d = prod_{1<=i<j<=d} ((1 - x_{i+1}...x_j) / (1 + x_{i+1}...x_j))^2,
    B_d = (1 + sum_{k=2}^d x_2...x_k)^(-1) * (1 + sum_{k=2}^d x_k...x_d)^(-1).

The factor 2 is part of the integrand here, so the tensor sums directly to the
integral.  With d = 1 there are no variables and every integrand equals 2.

u-form (the d-variable form on (0,inf)^d quoted with the workload definitions),
mapped to [0,1]^d by u = x/(1-x), du/u = dx/(x(1-x)):

    C_d = (4/d!) int [sum_j (u_j + 1/u_j)]^(-2) prod_j du_j/u_j,
    D_d = (4/d!) int prod_{i<j} ((u_i-u_j)/(u_i+u_j))^2 [sum_j (u_j + 1/u_j)]^(-2) prod_j du_j/u_j.

Synthetic families on [0,1]^d with parameters a_j, b_j:

    prod_exp:      prod_j exp(-a_j x_j)                        (TT rank 1)
    sum2_exp_cos:  prod_j exp(-a_j x_j) + prod_j cos(b_j x_j)  (TT rank 2)

Weights folded into the tensor (Sec. 4.1, last paragraph):
    B(i_1..i_m) = w_{i_1} ... w_{i_m} * f(t_{i_1}, ..., t_{i_m}).

Every formula below is written exactly as stated above (each pair product is
recomputed from its factors), with no reordering for speed.

Pinned by: closed forms C_2 = 1, D_2 = 1/3, E_2 = 6 - 8 ln 2 (1-D quadrature),
C_3 = L_{-3}(2), C_4 = 7 zeta(3)/12, D_3, D_4 (brute-force tensor quadrature),
the printed D_8 (Sec. 5.5 figure), u-form C_1 = 2, C_2 = 1, D_2 = 1/3 (adaptive
quadrature), and the exact integrals of the synthetic families.
"""

import math

import numpy as np

PAPER_FORM = ("ising_c", "ising_d", "ising_e")
U_FORM = ("ising_c_u", "ising_d_u")
SYNTHETIC = ("prod_exp", "sum2_exp_cos")
FAMILIES = PAPER_FORM + U_FORM + SYNTHETIC


def n_modes(family, d):
    """Number of tensor modes m for an integral of 'dimension' d."""
    if family in PAPER_FORM:
        return d - 1
    if family in U_FORM or family in SYNTHETIC:
        return d
    raise ValueError(family)


def _ising_paper(family, x):
    """x has shape (npts, d-1); column l-2 holds x_l, l = 2..d."""
    npts, m = x.shape
    d = m + 1

    def prod_range(a, b):  # x_a * ... * x_b  (a <= b, 2 <= a, b <= d)
        return np.prod(x[:, a - 2:b - 1], axis=1)

    f = np.full(npts, 2.0)
    if family in ("ising_c", "ising_d"):
        s_left = np.ones(npts)
        s_right = np.ones(npts)
        for k in range(2, d + 1):
            s_left = s_left + prod_range(2, k)
            s_right = s_right + prod_range(k, d)
        f = f / (s_left * s_right)
    if family in ("ising_d", "ising_e"):
        a_d = np.ones(npts)
        for i in range(1, d):
            for j in range(i + 1, d + 1):
                p = prod_range(i + 1, j)
                a_d = a_d * ((1.0 - p) / (1.0 + p)) ** 2
        f = f * a_d
    return f


def _ising_u(family, x):
    npts, d = x.shape
    u = x / (1.0 - x)
    s = np.zeros(npts)
    for j in range(d):
        s = s + (u[:, j] + 1.0 / u[:, j])
    jac = np.ones(npts)
    for j in range(d):
        jac = jac / (x[:, j] * (1.0 - x[:, j]))
    f = 4.0 / math.factorial(d) * s ** (-2) * jac
    if family == "ising_d_u":
        for i in range(d):
            for j in range(i + 1, d):
                f = f * ((u[:, i] - u[:, j]) / (u[:, i] + u[:, j])) ** 2
    return f


def _synthetic(family, x, params):
    npts, d = x.shape
    a = np.asarray(params["a"], dtype=np.float64)
    e = np.ones(npts)
    for j in range(d):
        e = e * np.exp(-a[j] * x[:, j])
    if family == "prod_exp":
        return e
    b = np.asarray(params["b"], dtype=np.float64)
    c = np.ones(npts)
    for j in range(d):
        c = c * np.cos(b[j] * x[:, j])
    return e + c


def f_values(family, x, params=None):
    """Unweighted integrand at points x (npts, m), prefactors included."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim != 2:
        raise ValueError("x must be 2-D (npts, m)")
    if family in PAPER_FORM:
        return _ising_paper(family, x)
    if family in U_FORM:
        return _ising_u(family, x)
    if family in SYNTHETIC:
        return _synthetic(family, x, params)
    raise ValueError(family)


def _ising_paper_dd(family, x):
    """The paper form in double-double; x is a DD array (npts, d-1).  Same formula as above."""
    from .ddarith import DD, dd_prod
    npts, m = x.shape
    d = m + 1

    def prod_range(a, b):
        return dd_prod(x[:, a - 2:b - 1], axis=1)

    f = DD(np.full(npts, 2.0))
    if family in ("ising_c", "ising_d"):
        s_left = DD(np.ones(npts))
        s_right = DD(np.ones(npts))
        for k in range(2, d + 1):
            s_left = s_left + prod_range(2, k)
            s_right = s_right + prod_range(k, d)
        f = f / (s_left * s_right)
    if family in ("ising_d", "ising_e"):
        a_d = DD(np.ones(npts))
        for i in range(1, d):
            for j in range(i + 1, d + 1):
                p = prod_range(i + 1, j)
                a_d = a_d * ((1.0 - p) / (1.0 + p)).square()
        f = f * a_d
    return f


def f_values_dd(family, x):
    """Unweighted integrand in double-double at points x (a DD array (npts, m)); paper form only."""
    if family not in PAPER_FORM:
        raise ValueError(f"no double-double path for {family}")
    if len(x.shape) != 2:
        raise ValueError("x must be 2-D (npts, m)")
    return _ising_paper_dd(family, x)


def weighted_values_dd(family, idx, t, w):
    """B in double-double at integer multi-indices idx (npts, m); t, w are DD node/weight tables."""
    from .ddarith import DD, dd_prod
    idx = np.asarray(idx, dtype=np.int64)
    if idx.ndim != 2:
        raise ValueError("idx must be 2-D (npts, m)")
    npts, m = idx.shape
    if m == 0:
        return f_values_dd(family, DD(np.zeros((npts, 0))))
    x = DD(t.hi[idx], t.lo[idx])
    wt = dd_prod(DD(w.hi[idx], w.lo[idx]), axis=1)
    return wt * f_values_dd(family, x)


def weighted_values(family, idx, t, w, params=None):
    """B at integer multi-indices idx (npts, m): prod_k w[idx_k] * f(t[idx])."""
    idx = np.asarray(idx, dtype=np.int64)
    if idx.ndim != 2:
        raise ValueError("idx must be 2-D (npts, m)")
    x = t[idx] if idx.shape[1] > 0 else np.zeros((idx.shape[0], 0))
    wt = np.prod(w[idx], axis=1) if idx.shape[1] > 0 else np.ones(idx.shape[0])
    return wt * f_values(family, x, params)


def log2_weighted_values(family, idx, t, w):
    """log2 of B at integer multi-indices idx (npts, m) for the paper-form integrands.

    The same formulas (eqs. c, d, e) taken through logarithms of their factors,
    so that values far below the double range (D_d near 10^(-0.7 d), Sec. 5.5)
    are represented:
        ln f = ln 2 + 2 sum_{runs} [ln(1 - p) - ln(1 + p)] - ln(1 + q) - ln(1 + s),
    each run product p = x_{i+1}..x_j recomputed from its factors (a product that
    underflows to 0 contributes ln 1 = 0, below the double rounding of the sum),
    plus the logarithms of the weights.  The absolute error of the result is
    about |log2 B| times the double rounding unit.
    """
    idx = np.asarray(idx, dtype=np.int64)
    if idx.ndim != 2:
        raise ValueError("idx must be 2-D (npts, m)")
    if family not in PAPER_FORM:
        raise ValueError(f"no log-scale path for {family}")
    npts, m = idx.shape
    d = m + 1
    x = t[idx] if m > 0 else np.zeros((npts, 0))

    def prod_range(a, b):  # x_a * ... * x_b  (a <= b, 2 <= a, b <= d)
        return np.prod(x[:, a - 2:b - 1], axis=1)

    lf = np.full(npts, math.log(2.0))
    if family in ("ising_c", "ising_d"):
        s_left = np.ones(npts)
        s_right = np.ones(npts)
        for k in range(2, d + 1):
            s_left = s_left + prod_range(2, k)
            s_right = s_right + prod_range(k, d)
        lf = lf - np.log(s_left) - np.log(s_right)
    if family in ("ising_d", "ising_e"):
        acc = np.zeros(npts)
        for i in range(1, d):
            for j in range(i + 1, d + 1):
                p = prod_range(i + 1, j)
                acc = acc + (np.log1p(-p) - np.log1p(p))
        lf = lf + 2.0 * acc
    lw = np.sum(np.log(w[idx]), axis=1) if m > 0 else np.zeros(npts)
    return (lf + lw) / math.log(2.0)


def exact_synthetic(family, params, d):
    """Exact integral over [0,1]^d of the synthetic families."""
    a = np.asarray(params["a"], dtype=np.float64)[:d]
    e = 1.0
    for j in range(d):
        e *= (1.0 - math.exp(-a[j])) / a[j]
    if family == "prod_exp":
        return e
    b = np.asarray(params["b"], dtype=np.float64)[:d]
    c = 1.0
    for j in range(d):
        c *= math.sin(b[j]) / b[j]
    return e + c
