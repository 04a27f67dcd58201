"""Pins of the stored D_5..D_10 reference values (tests/golden/ising_d_n64_reference.txt).

The values are the oracle's TT cross at 64 nodes and tol 1e-13 (written by
tests/golden/make_ising_reference.py); the benchmark checks its results against
them.  They are pinned here by what lies outside the cross: brute-force tensor
quadrature (the rule converges exponentially for the paper form, so 20..32
nodes already give the 64-node value to ~1e-14) and the value the paper prints
for D_8 (Sec. 5.5).  D_9 and D_10 have no such check beyond the oracle's own
pins; their brute-force sums are beyond reach.
"""
import os

import pytest

from oracle.quadrature import tensor_quadrature

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def stored():
    out = {}
    for line in open(os.path.join(GOLDEN, "ising_d_n64_reference.txt")):
        if line.strip() and not line.startswith("#"):
            f = line.split()
            out[int(f[0])] = float(f[1])
    return out


def printed():
    out = {}
    for line in open(os.path.join(GOLDEN, "ising_printed.txt")):
        if line.strip() and not line.startswith("#"):
            d, v = line.split()
            out[int(d)] = float(v)
    return out


def test_reference_values_cover_d5_to_d10():
    assert sorted(stored()) == list(range(5, 11))


@pytest.mark.parametrize("d,n", [(5, 32), (6, 20)])
def test_reference_against_brute_force(d, n):
    q = tensor_quadrature("ising_d", d - 1, n)     # d - 1 modes in the paper form
    assert abs(stored()[d] / q - 1) < 1e-12, (d, stored()[d], q)


def test_reference_d8_against_the_printed_value():
    assert abs(stored()[8] / printed()[8] - 1) < 1e-12
