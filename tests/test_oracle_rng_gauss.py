"""Pins for the oracle's SplitMix64 generator and Gauss--Legendre rule."""
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import rng
from oracle.gauss import gauss_legendre_01, gauss_legendre_01_mp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_stream():
    want = [int(line, 16) for line in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if line.startswith("0x")]
    assert rng.stream(0, 3) == want


def test_splitmix64_counter_form_matches_stream():
    seq = rng.stream(12345, 50)
    assert [rng.value(12345, c) for c in range(50)] == seq


def test_uniform_index_range_and_bias():
    n = 64
    draws = [rng.uniform_index(rng.value(7, c), n) for c in range(64 * 500)]
    assert min(draws) == 0 and max(draws) == n - 1
    counts = np.bincount(draws, minlength=n)
    assert counts.min() > 350 and counts.max() < 650   # 500 expected per bin


@pytest.mark.parametrize("n", [1, 2, 5, 16, 32, 64, 128])
def test_gl_weights_sum_and_symmetry(n):
    t, w = gauss_legendre_01(n)
    assert abs(w.sum() - 1.0) < 4e-16 * n
    assert np.all(np.diff(t) > 0) and t[0] > 0 and t[-1] < 1
    np.testing.assert_allclose(t + t[::-1], 1.0, rtol=0, atol=2e-16)
    np.testing.assert_allclose(w, w[::-1], rtol=1e-13, atol=0)


@pytest.mark.parametrize("n", [3, 8, 33, 64])
def test_gl_exact_for_monomials(n):
    t, w = gauss_legendre_01(n)
    for k in range(0, 2 * n):
        assert abs(np.dot(w, t ** k) - 1.0 / (k + 1)) < 1e-15
    # the first degree that is NOT integrated exactly
    assert abs(np.dot(w, t ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-300


@pytest.mark.parametrize("n", [5, 32])
def test_gl_nodes_are_legendre_roots(n):
    t, w = gauss_legendre_01(n)
    tm, wm = gauss_legendre_01_mp(n, dps=40)
    with mp.workdps(40):
        for k in range(n):
            assert abs(mp.legendre(n, 2 * tm[k] - 1)) < mp.mpf(10) ** -30
    np.testing.assert_allclose(t, [float(v) for v in tm], rtol=2e-16, atol=2e-16)
    np.testing.assert_allclose(w, [float(v) for v in wm], rtol=2e-16, atol=0)
    # numpy's own rule agrees to its documented accuracy
    x, wx = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(t, (x + 1) / 2, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, wx / 2, rtol=5e-13, atol=0)
