"""Brute-force tensor-product quadrature — oracle side (test infrastructure only).

eq. quad_product (Sec. 4.1): the full sum over all n^m grid points of
w_{i_1} ... w_{i_m} f(t_{i_1}, ..., t_{i_m}).  This is the quantity the TT
quadrature approximates; it is affordable only for small m.

Pinned by: closed forms of low-dimensional Ising integrals and exact integrals
of separable functions (tests/test_oracle_quadrature.py).
"""

import itertools

import numpy as np

from .gauss import gauss_legendre_01
from .integrands import weighted_values


def tensor_quadrature(family, m, n, params=None, max_chunk=1 << 20):
    """Sum of B over the whole n^m grid in float64.

    The grid is enumerated in lexicographic order: the leading modes are looped
    over in Python, the trailing modes (at most ``max_chunk`` points) are
    evaluated as one numpy batch.
    """
    t, w = gauss_legendre_01(n)
    if m == 0:
        return float(weighted_values(family, np.zeros((1, 0), dtype=np.int64), t, w, params)[0])
    n_tail = 0
    while n_tail < m and n ** (n_tail + 1) <= max_chunk:
        n_tail += 1
    n_tail = max(n_tail, 1)
    n_lead = m - n_tail
    tail = np.array(list(itertools.product(range(n), repeat=n_tail)), dtype=np.int64)
    total = 0.0
    for lead in itertools.product(range(n), repeat=n_lead):
        idx = np.empty((tail.shape[0], m), dtype=np.int64)
        idx[:, :n_lead] = np.array(lead, dtype=np.int64)
        idx[:, n_lead:] = tail
        total += float(np.sum(weighted_values(family, idx, t, w, params)))
    return total


def tensor_quadrature_dd(family, m, n, max_chunk=1 << 16):
    """Sum of B over the whole n^m grid in double-double (paper-form integrands).

    Same enumeration as tensor_quadrature; every value and the running sum are
    double-double.  Returns (hi, lo).
    """
    from .ddarith import DD, dd_sum
    from .gauss import gauss_legendre_01_dd
    from .integrands import weighted_values_dd
    t, w = gauss_legendre_01_dd(n)
    if m == 0:
        return weighted_values_dd(family, np.zeros((1, 0), dtype=np.int64), t, w)[0].scalar()
    n_tail = 0
    while n_tail < m and n ** (n_tail + 1) <= max_chunk:
        n_tail += 1
    n_tail = max(n_tail, 1)
    n_lead = m - n_tail
    tail = np.array(list(itertools.product(range(n), repeat=n_tail)), dtype=np.int64)
    total = DD(0.0)
    for lead in itertools.product(range(n), repeat=n_lead):
        idx = np.empty((tail.shape[0], m), dtype=np.int64)
        idx[:, :n_lead] = np.array(lead, dtype=np.int64)
        idx[:, n_lead:] = tail
        total = total + dd_sum(weighted_values_dd(family, idx, t, w), axis=0)
    return total.scalar()
