"""Pins for the TT-cross oracle (Alg. 2 inside Alg. 6, TT quadrature of Sec. 4.1).

Each expected value comes from outside the oracle's TT code: exact integrals,
closed forms, brute-force tensor quadrature, the paper's printed D_8, or the
theorems of Sec. 3 (interpolation on nested fibers, exact recovery at exact rank).
"""
import itertools
import math
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import ttcross
from oracle.integrands import exact_synthetic
from oracle.quadrature import tensor_quadrature

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def printed_d():
    vals = {}
    for line in open(os.path.join(GOLDEN, "ising_printed.txt")):
        if line.strip() and not line.startswith("#"):
            d, v = line.split()
            vals[int(d)] = float(v)
    return vals


def synth_params(d, seed):
    r = np.random.default_rng(seed)
    return {"a": r.uniform(0.5, 4.0, d).tolist(), "b": r.uniform(0.5, 4.0, d).tolist()}


@pytest.mark.parametrize("d", [1, 2, 3, 6])
def test_rank1_product_exact(d):
    params = synth_params(d, 11)
    tt = ttcross.solve("prod_exp", d, 16, 8, 1e-12, seed=3, params=params)
    assert tt.ranks() == [1] * (d - 1)          # nothing above tol after the start
    assert abs(tt.history[-1] / exact_synthetic("prod_exp", params, d) - 1) < 1e-14


@pytest.mark.parametrize("d", [2, 3, 5])
def test_rank2_exact_recovery(d):
    # Thm. 2: at exact TT rank the cross formula reproduces the whole tensor
    params = synth_params(d, 5)
    n = 6
    tt = ttcross.solve("sum2_exp_cos", d, n, 8, 1e-12, seed=9, params=params)
    assert max(tt.ranks()) == 2 and tt.stop_reason == "converged"
    grid = np.array(list(itertools.product(range(n), repeat=d)))
    np.testing.assert_allclose(tt.reconstruct(grid), tt.B(grid), rtol=0,
                               atol=1e-13 * np.abs(tt.B(grid)).max())
    exact = exact_synthetic("sum2_exp_cos", params, d)
    q_n = tensor_quadrature("sum2_exp_cos", d, n, params)
    assert abs(tt.history[-1] - q_n) < 1e-13 * abs(q_n)
    # after rank 2 is reached, every search sees only rounding-level errors
    # (pivot errors are entries of the tensor with scaled weights, 2^(s m) B)
    late = [abs(r.err) for sweep in tt.pivot_log[1:] for r in sweep if r.searched]
    assert all(e < 1e-14 * abs(q_n) * 2.0 ** (tt.wshift * tt.m) for e in late)
    # n = 6 is not enough for the exact integral: only the tensor sum is exact
    assert abs(q_n - exact) < 1e-3


def test_interpolation_on_fibers_and_nestedness():
    # Thm. 1 + eq. nest: the cross formula equals B on every evaluated fiber
    tt = ttcross.solve("ising_d", 6, 10, 6, 1e-14, seed=2, max_sweeps=5)
    m = tt.m
    for b in range(1, m - 1):
        for l in tt.left[b]:
            assert l[:-1] in tt.left[b - 1]
    for b in range(0, m - 2):
        for r in tt.right[b]:
            assert r[1:] in tt.right[b + 1]
    for c in range(m):
        pts = [l + (i,) + r for l in tt.left_set(c - 1) for i in range(tt.n)
               for r in tt.right_set(c)]
        got, want = tt.reconstruct(pts), tt.B(pts)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_entry_count_matches_compression_remark():
    # Remark "Compression": the cores hold sum r_{k-1} n r_k entries, the crosses sum r_k^2
    tt = ttcross.TTCross("ising_c", 6, 8, 5, 1e-14, seed=1, max_sweeps=4)
    tt.run()
    r = [1] + tt.ranks() + [1]
    entries = sum(r[k] * tt.n * r[k + 1] for k in range(tt.m))
    cores = [tt.core(c) for c in range(tt.m)]
    assert sum(c.size for c in cores) == entries
    distinct = {l + (i,) + rr for c in range(tt.m) for l in tt.left_set(c - 1)
                for i in range(tt.n) for rr in tt.right_set(c)}
    assert len(distinct) == entries - sum(x * x for x in tt.ranks())


@pytest.mark.parametrize("family,d,n", [("ising_d", 3, 24), ("ising_d", 4, 24),
                                        ("ising_c", 5, 16), ("ising_d", 5, 14)])
def test_tt_matches_brute_force(family, d, n):
    tt = ttcross.solve(family, d, n, 32, 1e-13, seed=4)
    q_n = tensor_quadrature(family, d - 1, n)
    assert abs(tt.history[-1] - q_n) < 2e-12 * abs(q_n)


def test_closed_forms_c3_c4():
    with mp.workdps(30):
        c3 = float((mp.zeta(2, mp.mpf(1) / 3) - mp.zeta(2, mp.mpf(2) / 3)) / 9)
        c4 = float(7 * mp.zeta(3) / 12)
    tt3 = ttcross.solve("ising_c", 3, 32, 8, 1e-10, seed=1)
    assert abs(tt3.history[-1] / c3 - 1) < 1e-10
    tt4 = ttcross.solve("ising_c", 4, 32, 16, 1e-12, seed=1)
    assert abs(tt4.history[-1] / c4 - 1) < 1e-13


def test_printed_d8():
    # D_8 printed in Sec. 5.5; 32 nodes are enough for ~1e-14 in the paper form
    tt = ttcross.solve("ising_d", 8, 32, 24, 1e-12, seed=8)
    assert abs(tt.history[-1] / printed_d()[8] - 1) < 1e-11


def test_rook_condition_on_matrix():
    # m = 2: one superblock, i.e. the matrix cross of Alg. 2 on an n x n matrix.
    tt = ttcross.TTCross("ising_d_u", 2, 12, 12, 1e-14, seed=6, max_sweeps=3)
    cores = [tt.core(c) for c in range(tt.m)]
    rec = tt.cross_step(0, tt.sweeps, cores)
    A = tt.core(0).reshape(12, -1)  # not the superblock: build the full matrix instead
    full = np.array([[tt.B([(i, j)])[0] for j in range(12)] for i in range(12)])
    L, R = tt.left[0], tt.right[0]
    I = [l[0] for l in L]
    J = [r[0] for r in R]
    approx = full[:, J] @ np.linalg.solve(full[np.ix_(I, J)], full[I, :])
    err = full - approx
    assert abs(err[rec.row, rec.col] - rec.err) < 1e-14 * np.abs(full).max()
    if rec.iters < ttcross.T_ROOK:     # loop ended by the rook condition eq. rook
        assert abs(err[rec.row, rec.col]) >= np.abs(err[rec.row, :]).max() * (1 - 1e-12)
        assert abs(err[rec.row, rec.col]) >= np.abs(err[:, rec.col]).max() * (1 - 1e-12)


def test_pivot_updates_volume():
    # Alg. 1: adding the pivot multiplies |det| of the cross by |err*| (Schur complement)
    tt = ttcross.TTCross("ising_d", 5, 10, 10, 1e-14, seed=3, max_sweeps=6)
    for _ in range(3):
        tt.sweep()
    cores = [tt.core(c) for c in range(tt.m)]
    for b in range(tt.m - 1):
        rec = tt.cross_step(b, tt.sweeps, cores)
        if not rec.accepted:
            continue
        M = tt.cross_matrix(b)
        newl, newr = rec._new
        Mp = tt.B([l + r for l in tt.left[b] + [newl] for r in tt.right[b] + [newr]])
        Mp = Mp.reshape(len(M) + 1, len(M) + 1)
        assert abs(np.linalg.det(Mp) - np.linalg.det(M) * rec.err) < 1e-10 * abs(np.linalg.det(Mp))


def test_deterministic_and_seed_dependent():
    a = ttcross.solve("ising_d", 5, 12, 8, 1e-12, seed=1)
    b = ttcross.solve("ising_d", 5, 12, 8, 1e-12, seed=1)
    c = ttcross.solve("ising_d", 5, 12, 8, 1e-12, seed=2)
    assert a.history == b.history and a.evals == b.evals
    assert [[(p.row, p.col) for p in s] for s in a.pivot_log] == \
           [[(p.row, p.col) for p in s] for s in b.pivot_log]
    assert a.start_index != c.start_index or a.pivot_log[0][0].row != c.pivot_log[0][0].row


def test_rank_cap_stop():
    tt = ttcross.solve("ising_d", 5, 16, 3, 1e-14, seed=1)
    assert tt.ranks() == [3, 3, 3] and tt.stop_reason == "rank_cap"


@pytest.mark.parametrize("d", [1, 2])
def test_degenerate_mode_counts(d):
    tt = ttcross.solve("ising_d", d, 20, 4, 1e-12, seed=1)
    assert tt.stop_reason == "converged"
    want = 2.0 if d == 1 else 1.0 / 3.0
    assert abs(tt.history[-1] - want) < 1e-15


def test_update_evaluations_exclude_the_reused_rook_fibres():
    """The core updates evaluate exactly the new core entries that no final rook step evaluated.

    Checked with explicit point sets: per core, the entries added by a sweep;
    the final row step of an accepted search at bond b covers the new row of
    core b+1 at its old columns, and its final column step (when taken at the
    final column) the new column of core b at its old rows.
    """
    tt = ttcross.TTCross("ising_d", 6, 10, 8, 1e-14, seed=3, max_sweeps=8)
    n = tt.n

    def core_points():
        return [{l + (i,) + r for l in tt.left_set(c - 1) for i in range(n) for r in tt.right_set(c)}
                for c in range(tt.m)]

    checked = 0
    for _ in range(6):
        if tt.stop_reason:
            break
        before = core_points()
        L = [list(tt.left_set(b - 1)) for b in range(tt.m - 1)]
        R = [list(tt.right_set(b + 1)) for b in range(tt.m - 1)]
        ev0 = tt.evals
        tt.sweep()
        recs = tt.pivot_log[-1]
        search = sum(min(r.n_rows + r.n_cols, ttcross.MAX_SAMPLES) + r.iters * (r.n_rows + r.n_cols)
                     for r in recs if r.searched)
        after = core_points()
        new = [after[c] - before[c] for c in range(tt.m)]
        reused = [set() for _ in range(tt.m)]
        for b, r in enumerate(recs):
            if not r.accepted:
                continue
            rR = len(R[b])
            al, i = divmod(r.row, n)
            j, be = divmod(r.col, rR)
            reused[b + 1] |= {L[b][al] + (i, jj) + rr for jj in range(n) for rr in R[b]}
            if r.col_fresh:
                reused[b] |= {ll + (ii, j) + R[b][be] for ll in L[b] for ii in range(n)}
        for c in range(tt.m):
            assert reused[c] <= new[c]
        assert tt.evals - ev0 - search == sum(len(new[c]) - len(reused[c]) for c in range(tt.m))
        checked += sum(len(x) for x in reused)
    assert checked > 0


@pytest.mark.parametrize("family,d,n,params", [
    ("ising_c", 6, 12, None), ("ising_d", 5, 10, None),
    ("sum2_exp_cos", 6, 8, {"a": [0.7, 1.9, 3.1, 0.9, 2.2, 1.4], "b": [1.3, 0.6, 2.4, 3.3, 1.1, 2.8]})])
def test_scaled_weights_give_the_unscaled_computation_bit_for_bit(family, d, n, params):
    # the weights carry an exact factor 2^s and the chain exact powers of two:
    # every decision and every value must be the unscaled one (values times 2^(s m))
    a = ttcross.TTCross(family, d, n, 8, 1e-12, seed=3, max_sweeps=4, params=params)
    b = ttcross.TTCross(family, d, n, 8, 1e-12, seed=3, max_sweeps=4, params=params, scale_weights=False)
    a.run()
    b.run()
    k = a.wshift * a.m
    assert a.wshift == round(math.log2(n)) and b.wshift == 0
    assert a.history == b.history and a.stop_reason == b.stop_reason and len(a.history) > 2
    for sa, sb in zip(a.pivot_log, b.pivot_log):
        for ra, rb in zip(sa, sb):
            assert (ra.row, ra.col, ra.accepted, ra.iters) == (rb.row, rb.col, rb.accepted, rb.iters)
            assert ra.err == math.ldexp(rb.err, k) and ra.value == math.ldexp(rb.value, k)


def test_rank1_product_of_300_modes_through_the_scaled_chain():
    # Thm. 2 (exact recovery at rank 1): the TT quadrature of a product function
    # is the product of its 1-D Gauss-Legendre sums.  Unscaled, the folded
    # weights' sum over the grid (16^300 times the integral, about 1e350) would
    # overflow; the scaled chain must still give the product to rounding.
    from oracle.gauss import gauss_legendre_01
    d, n = 300, 16
    a = np.random.default_rng(7).uniform(0.05, 0.3, d)
    tt = ttcross.solve("prod_exp", d, n, 2, 1e-12, seed=1, max_sweeps=2,
                       params={"a": list(a), "b": [1.0] * d})
    t, w = gauss_legendre_01(n)
    log_q = math.fsum(math.log(float(np.dot(w, np.exp(-aj * t)))) for aj in a)
    mant, e = tt.history_scaled[-1]
    assert 0.5 <= abs(mant) < 1.0 and max(tt.ranks()) == 1
    assert abs(math.log(mant) + e * math.log(2.0) - log_q) < 1e-12 * abs(log_q)
    assert tt.history[-1] == math.ldexp(mant, e)


# exp(alpha (x_1 + x_2)) with alpha = 355.1 on 64 Gauss-Legendre nodes overflows
# exactly when both coordinates sit at the largest node (2 t_63 alpha > log of
# the largest double); every point with at most one of them there is finite.
OVERFLOW_CASE = dict(family="prod_exp", d=2, n=64, rank_cap=4, tol=1e-10, seed=4,
                     params={"a": [-355.1, -355.1], "b": [1.0] * 2})


def test_overflow_in_a_sweep_is_a_numeric_error():
    """A non-finite B met by the search is an error, not a pivot (the start and cores are finite)."""
    from oracle.gauss import gauss_legendre_01
    c = OVERFLOW_CASE
    t, _ = gauss_legendre_01(c["n"])
    alpha = -c["params"]["a"][0]
    log_max = math.log(np.finfo(np.float64).max)
    assert 2 * alpha * t[-1] > log_max + 0.1 and alpha * (t[-1] + t[-2]) < log_max - 0.1
    tt = ttcross.TTCross(c["family"], c["d"], c["n"], c["rank_cap"], c["tol"], c["seed"],
                         params=c["params"])
    assert all(np.isfinite(tt.core(k)).all() for k in range(tt.m)) and math.isfinite(tt.history[0])
    with pytest.raises(FloatingPointError, match="non-finite"):
        tt.sweep()


def n64_reference():
    out = {}
    for line in open(os.path.join(GOLDEN, "ising_d_n64_reference.txt")):
        if line.strip() and not line.startswith("#"):
            f = line.split()
            out[int(f[0])] = float(f[1])
    return out


@pytest.mark.parametrize("d", [6, 7])
def test_strict_stop_rule(d):
    """The strict rule stops only on a sweep that accepts no pivot (or the caps).

    D_6 and D_7 with 64 nodes, rank <= 32, tol 1e-10: the default rule stops after
    two small relative changes while bonds still accept pivots, about 1e-10 from
    the integral; the strict run takes the same decisions up to there, continues
    until a sweep accepts nothing, and ends well within tol of the tol-1e-13
    reference of the same nodes.
    """
    loose = ttcross.TTCross("ising_d", d, 64, 32, 1e-10, d)
    loose.run()
    strict = ttcross.TTCross("ising_d", d, 64, 32, 1e-10, d, stop_rule="strict")
    strict.run()
    ref = n64_reference()[d]
    assert sum(r.accepted for r in loose.pivot_log[-1]) > 0          # stopped with pivots still accepted
    assert strict.sweeps > loose.sweeps
    assert strict.history[:loose.sweeps + 1] == loose.history
    for a, b in zip(loose.pivot_log, strict.pivot_log):
        assert [(r.row, r.col, r.accepted) for r in a] == [(r.row, r.col, r.accepted) for r in b]
    last = strict.pivot_log[-1]
    assert sum(r.accepted for r in last) == 0 and strict.stop_reason == "converged"
    assert abs(strict.history[-1] / ref - 1) < 2e-11
    with pytest.raises(ValueError):
        ttcross.TTCross("ising_d", d, 8, 4, 1e-10, d, stop_rule="sometimes")
