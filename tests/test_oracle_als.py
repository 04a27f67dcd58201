"""The ALS maxvol refresh (Sec. 3.3, Alg. 3; row swaps of Alg. 1, Sec. 2.4), oracle side.

Pins: Alg. 1's volume identity at every swap, the identity block and the final
dominance of C = A A(I,:)^-1, the exhaustive maximum-volume choice on small
matrices (rank 1 exactly; rank 2 within the dominance bound), nestedness and
unchanged ranks after a refresh, interpolation on every fibre of the refreshed
cross (Thm. 1), exact recovery on a rank-2 product (Thm. 2), and a planted
mistake (the swapped-out row taken from the wrong position).
"""
import itertools
import math

import numpy as np
import pytest

from oracle import als, ttcross
from oracle.quadrature import tensor_quadrature


def synth_params(d, seed):
    r = np.random.default_rng(seed)
    return {"a": r.uniform(0.5, 4.0, d).tolist(), "b": r.uniform(0.5, 4.0, d).tolist()}


@pytest.mark.parametrize("N,r,seed", [(20, 3, 1), (64, 5, 2), (200, 8, 3), (9, 9, 4)])
def test_maxvol_volume_identity_and_dominance(N, r, seed):
    A = np.random.default_rng(seed).standard_normal((N, r))
    rows, swaps, vols = als.maxvol(A)
    assert len(set(rows)) == r and len(vols) == swaps + 1
    # each swap multiplied the volume by |C(i*, j*)| > 1 + delta (replay the swaps)
    cur = als.gepp_rows(A)
    assert abs(np.linalg.det(A[cur, :])) == pytest.approx(vols[0], rel=1e-12)
    for k in range(swaps):
        C = np.linalg.solve(A[cur, :].T, A.T).T
        i, j = divmod(int(np.argmax(np.abs(C))), r)
        assert abs(C[i, j]) > 1 + als.DELTA
        cur[j] = i
        assert vols[k + 1] == pytest.approx(vols[k] * abs(C[i, j]), rel=1e-10)
    assert cur == rows
    C = np.linalg.solve(A[rows, :].T, A.T).T
    np.testing.assert_allclose(C[rows, :], np.eye(r), atol=1e-12)
    assert np.abs(C).max() <= 1 + als.DELTA + 1e-12


def test_maxvol_rank1_is_the_largest_entry():
    A = np.random.default_rng(7).standard_normal((50, 1))
    rows, _, _ = als.maxvol(A)
    assert rows == [int(np.argmax(np.abs(A[:, 0])))]


@pytest.mark.parametrize("seed", range(6))
def test_maxvol_rank2_against_exhaustive_search(seed):
    A = np.random.default_rng(100 + seed).standard_normal((12, 2))
    rows, _, vols = als.maxvol(A, delta=0.0, max_swaps=100)
    best = max(abs(np.linalg.det(A[list(p), :])) for p in itertools.combinations(range(12), 2))
    # a dominant (|C| <= 1) submatrix has at least 1/r^(r/2) of the largest volume
    assert vols[-1] >= best / 2.0 - 1e-12
    assert vols[-1] <= best + 1e-12


def test_planted_wrong_swap_position_breaks_the_volume_identity():
    A = np.random.default_rng(9).standard_normal((30, 4))
    rows = als.gepp_rows(A)
    C = np.linalg.solve(A[rows, :].T, A.T).T
    i, j = divmod(int(np.argmax(np.abs(C))), 4)
    assume = abs(C[i, j]) > 1 + als.DELTA
    if not assume:
        pytest.skip("GEPP start already dominant")
    wrong = list(rows)
    wrong[(j + 1) % 4] = i       # the swapped-out row taken from the wrong position
    v0 = abs(np.linalg.det(A[rows, :]))
    assert abs(abs(np.linalg.det(A[wrong, :])) - v0 * abs(C[i, j])) > 1e-6 * v0


def nested(tt):
    for b in range(1, tt.m - 1):
        for l in tt.left[b]:
            if l[:-1] not in tt.left[b - 1]:
                return False
    for b in range(0, tt.m - 2):
        for r in tt.right[b]:
            if r[1:] not in tt.right[b + 1]:
                return False
    return True


@pytest.mark.parametrize("family,d,n,rank", [("ising_d", 6, 10, 5), ("ising_c", 7, 12, 6), ("ising_e", 5, 9, 6)])
def test_refresh_keeps_ranks_nestedness_and_interpolation(family, d, n, rank):
    tt = ttcross.TTCross(family, d, n, rank, 1e-14, seed=3, max_sweeps=8)
    for _ in range(4):
        tt.sweep()
    assert tt.stop_reason is None
    ranks = tt.ranks()
    ev = tt.evals
    rec = als.refresh(tt)
    assert tt.ranks() == ranks and nested(tt)
    for b in range(tt.m - 1):
        assert len(set(tt.left[b])) == ranks[b] and len(set(tt.right[b])) == ranks[b]
    assert tt.evals > ev
    assert tt.history_scaled[-1] == rec["after"] and rec["before"] is not None
    for c in range(tt.m):   # Thm. 1 on the refreshed cross
        pts = [l + (i,) + r for l in tt.left_set(c - 1) for i in range(tt.n) for r in tt.right_set(c)]
        got, want = tt.reconstruct(pts), tt.B(pts)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-11 * np.abs(want).max())
    # the run continues from the refreshed sets
    tt.sweep()
    assert nested(tt) and tt.sweeps == 5


def test_refresh_on_an_exact_rank2_product_keeps_the_exact_integral():
    d, n = 5, 6
    params = synth_params(d, 5)
    tt = ttcross.TTCross("sum2_exp_cos", d, n, 2, 1e-14, seed=9, params=params, max_sweeps=6)
    for _ in range(3):
        tt.sweep()
    assert max(tt.ranks()) == 2
    als.refresh(tt)
    q_n = tensor_quadrature("sum2_exp_cos", d, n, params)
    assert abs(tt.history[-1] - q_n) < 1e-13 * abs(q_n)
    grid = np.array(list(itertools.product(range(n), repeat=d)))
    np.testing.assert_allclose(tt.reconstruct(grid), tt.B(grid), rtol=0, atol=1e-13 * np.abs(tt.B(grid)).max())


def test_refresh_leaves_a_stopped_integral_alone():
    tt = ttcross.solve("ising_d", 5, 8, 4, 1e-10, seed=2)
    left, right, ev = [list(x) for x in tt.left], [list(x) for x in tt.right], tt.evals
    assert als.refresh(tt) is None
    assert tt.left == left and tt.right == right and tt.evals == ev
