"""Gauss--Legendre rule on [0,1] — oracle side (test infrastructure only).

Sec. 4.1 ("Tensor product quadratures") builds the tensor-product rule from a
one-dimensional Gauss--Legendre rule with nodes t_i in [0,1] and weights w_i;
Sec. 5.2 uses it for the Ising integrals.  The paper does not say how the
nodes are generated.  The oracle takes the textbook definition: the nodes on
[-1,1] are the roots of the Legendre polynomial P_n, found by Newton's method
in 40-digit mpmath arithmetic (P_n from the three-term recurrence), and the
weights are 2 / ((1 - x^2) P_n'(x)^2); both are mapped affinely to [0,1]
(t = (x+1)/2, w = w_x/2) and rounded once to float64.  Nodes are returned in
increasing order.

Pinned by: sum of weights = 1, exactness for monomials of degree <= 2n-1,
symmetry t_i + t_{n+1-i} = 1, and the nodes being roots of P_n evaluated in
mpmath at 40 digits with mpmath's own Legendre function
(tests/test_oracle_rng_gauss.py).
"""

import functools

import numpy as np


def _legendre_pair(n, x, mp):
    """P_n(x), P_{n-1}(x) by (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}."""
    p_prev, p = mp.mpf(1), x
    if n == 0:
        return p_prev, mp.mpf(0)
    for k in range(1, n):
        p_prev, p = p, ((2 * k + 1) * x * p - k * p_prev) / (k + 1)
    return p, p_prev


@functools.lru_cache(maxsize=64)
def _gl_mp(n):
    """Nodes and weights on [0,1] as 40-digit mpmath numbers, increasing nodes."""
    import mpmath as mp
    with mp.workdps(40):
        t, w = [], []
        for k in range(1, n + 1):
            x = mp.cos(mp.pi * (k - mp.mpf(1) / 4) / (n + mp.mpf(1) / 2))
            for _ in range(100):
                p, q = _legendre_pair(n, x, mp)
                dp = n * (x * p - q) / (x * x - 1)
                dx = p / dp
                x -= dx
                if abs(dx) < mp.mpf(10) ** -36:
                    break
            p, q = _legendre_pair(n, x, mp)
            dp = n * (x * p - q) / (x * x - 1)
            t.append((x + 1) / 2)
            w.append(1 / ((1 - x * x) * dp * dp))
    order = sorted(range(n), key=lambda i: t[i])
    return [t[i] for i in order], [w[i] for i in order]


@functools.lru_cache(maxsize=64)
def _gl_mp_rounded(n):
    t, w = _gl_mp(n)
    return np.array([float(v) for v in t]), np.array([float(v) for v in w])


def gauss_legendre_01(n):
    """Return (t, w): n Gauss--Legendre nodes and weights on [0,1], float64."""
    if n < 1:
        raise ValueError("n must be >= 1")
    t, w = _gl_mp_rounded(n)
    return t.copy(), w.copy()


def gauss_legendre_01_dd(n):
    """Return (t, w) as double-double arrays (the 40-digit values rounded to hi + lo)."""
    from .ddarith import DD
    if n < 1:
        raise ValueError("n must be >= 1")
    t, w = _gl_mp(n)
    return DD.from_mp(t), DD.from_mp(w)


def gauss_legendre_01_mp(n, dps=50):
    """High-precision nodes/weights on [0,1] via Newton on P_n in mpmath (pins only)."""
    import mpmath as mp
    with mp.workdps(dps):
        nodes, weights = [], []
        for k in range(1, n + 1):
            # classical initial guess for the k-th root of P_n on [-1,1]
            x = mp.cos(mp.pi * (k - mp.mpf(1) / 4) / (n + mp.mpf(1) / 2))
            for _ in range(100):
                p = mp.legendre(n, x)
                dp = n * (x * p - mp.legendre(n - 1, x)) / (x * x - 1)
                dx = p / dp
                x -= dx
                if abs(dx) < mp.mpf(10) ** (-dps + 5):
                    break
            dp = n * (x * mp.legendre(n, x) - mp.legendre(n - 1, x)) / (x * x - 1)
            wk = 2 / ((1 - x * x) * dp * dp)
            nodes.append((x + 1) / 2)
            weights.append(wk / 2)
        order = sorted(range(n), key=lambda i: nodes[i])
        return [nodes[i] for i in order], [weights[i] for i in order]
