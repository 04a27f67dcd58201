"""ALS maxvol refresh of the index sets at fixed ranks — oracle side (test infrastructure only).

What is computed (Sec. 3.3, Alg. 3, with the row swaps of Alg. 1, Sec. 2.4)
-------------------------------------------------------------------------
One refresh of a TTCross object's nested index sets, ranks unchanged:

  left to right, b = 0 .. m-2: the r_{b-1} n x r_b matrix
        A = B(I_<=b-1^new x [n], I_>b),   rows (alpha, i) alpha-major,
    whose left factor was refreshed one step before; its r_b maxvol rows become
    the new I_<=b (each row (alpha, i) is the tuple I_<=b-1^new[alpha] + (i,),
    so the new sets are nested by construction);
  right to left, b = m-2 .. 0: the r_b x n r_{b+1} matrix
        A = B(I_<=b, [n] x I_>b+1^new),   columns (j, beta) j-major,
    with the left sets of the first pass; its r_b maxvol columns become the new
    I_>b ((j,) + I_>b+1^new[beta]).

After both passes the sets are nested again and the interpolation eq. tt on them
is a cross of the same ranks.  maxvol on an N x r matrix A (the transposed
matrix for columns) is, in this library's reading of "until the volume is large
enough" (Sec. 2.4):
  * start: r rows by Gaussian elimination with partial row pivoting; column k's
    pivot is the row of largest |residual| in column k, ties to the lowest row;
  * then Alg. 1 steps: C = A [A(I, :)]^-1 (so C(I, :) = identity), (i*, j*) the
    argmax of |C| over all entries (ties to the lowest i, then j); stop when
    |C(i*, j*)| <= 1 + delta, else replace the j*-th chosen row by i*; each step
    multiplies |det A(I, :)| by |C(i*, j*)|; at most max_swaps steps.
delta = 1e-2 and max_swaps = 4 r unless given.  C is recomputed from its
definition at every step (a dense solve), with no update formula.

A refresh evaluates every entry of every matrix A (counted in evals), and each
bond's scale (largest |B| it has evaluated) takes the largest |A| of the two
matrices that refresh its sets.  The integral on the new sets replaces the last
entry of the history (the pre-refresh value is kept in the refresh record), so
the next sweep's relative change is measured from the refreshed integral.

Pinned by: the volume identity of Alg. 1 at every step, the identity block
C(I, :) = I, maxvol's local optimality (no entry of the final C above 1 + delta),
exhaustive maximum-volume search on small matrices (rank 1: the largest entry;
rank 2: within the 1/r^(r/2) bound of a dominant submatrix), nestedness after
the refresh, exactness of the refreshed cross on exact low-rank tensors
(Thm. 2), and interpolation on every evaluated fibre (Thm. 1).
"""

import numpy as np

from .ttcross import scaled_ldexp

DELTA = 1e-2


def gepp_rows(A):
    """r row indices of the N x r matrix A chosen by Gaussian elimination with partial pivoting."""
    R = np.array(A, dtype=np.float64, copy=True)
    N, r = R.shape
    rows = []
    for k in range(r):
        col = np.abs(R[:, k])
        col[rows] = -1.0
        p = int(np.argmax(col))            # lowest index among equal maxima
        if not (col[p] > 0.0):
            raise np.linalg.LinAlgError("matrix of rank below r")
        rows.append(p)
        R = R - np.outer(R[:, k] / R[p, k], R[p, :])
    return rows


def maxvol(A, delta=DELTA, max_swaps=None):
    """(rows, swaps, volume log): r rows of the N x r matrix A by Alg. 1 steps from a GEPP start.

    volume log: |det A(I, :)| after the start and after every swap.
    """
    A = np.asarray(A, dtype=np.float64)
    N, r = A.shape
    if r == 0:
        return [], 0, []
    if max_swaps is None:
        max_swaps = 4 * r
    rows = gepp_rows(A)
    vols = [abs(np.linalg.det(A[rows, :]))]
    swaps = 0
    while swaps < max_swaps:
        C = np.linalg.solve(A[rows, :].T, A.T).T          # A [A(I,:)]^-1
        flat = int(np.argmax(np.abs(C)))                   # row-major: lowest i, then j
        i, j = divmod(flat, r)
        if not (abs(C[i, j]) > 1.0 + delta):
            break
        rows[j] = i
        swaps += 1
        vols.append(abs(np.linalg.det(A[rows, :])))
    return rows, swaps, vols


def refresh(tt, delta=DELTA, max_swaps=None):
    """One ALS maxvol refresh (left-to-right, then right-to-left) of tt's index sets; returns a record."""
    m, n = tt.m, tt.n
    if m < 2 or tt.stop_reason is not None:   # a stopped integral is left as it is
        return None
    before = tt.history_scaled[-1] if tt.history_scaled else None
    swaps_l, swaps_r = [], []
    scale_new = [0.0] * (m - 1)
    # left to right: I_<=b from B(I_<=b-1^new x [n], I_>b)
    new_left = [list(s) for s in tt.left]
    for b in range(m - 1):
        Lp = [()] if b == 0 else new_left[b - 1]
        R = tt.right[b]
        r = len(R)
        idx = [l + (i,) + rr for l in Lp for i in range(n) for rr in R]
        A = tt.B(idx).reshape(len(Lp) * n, r)
        tt.evals += A.size
        scale_new[b] = max(scale_new[b], float(np.max(np.abs(A))))
        rows, sw, _ = maxvol(A, delta, max_swaps)
        swaps_l.append(sw)
        new_left[b] = [Lp[q // n] + (q % n,) for q in rows]
    tt.left = new_left
    # right to left: I_>b from B(I_<=b, [n] x I_>b+1^new)
    new_right = [list(s) for s in tt.right]
    for b in range(m - 2, -1, -1):
        Rn = [()] if b == m - 2 else new_right[b + 1]
        L = tt.left[b]
        r = len(L)
        idx = [l + (j,) + rr for l in L for j in range(n) for rr in Rn]
        A = tt.B(idx).reshape(r, n * len(Rn))
        tt.evals += A.size
        scale_new[b] = max(scale_new[b], float(np.max(np.abs(A))))
        cols, sw, _ = maxvol(A.T, delta, max_swaps)
        swaps_r.append(sw)
        new_right[b] = [(q // len(Rn),) + Rn[q % len(Rn)] for q in cols]
    tt.right = new_right
    tt.scale = [max(a, s) for a, s in zip(tt.scale, scale_new)]
    # every core entry on the new sets is evaluated again by the next sweep's cores
    tt._core_sizes = [0] * m
    tt._count_new_core_entries()
    value = tt.integral_scaled()
    rec = {"after_sweep": tt.sweeps, "before": before, "after": value,
           "swaps_left": swaps_l, "swaps_right": swaps_r[::-1]}
    if tt.history_scaled:
        tt.history_scaled[-1] = value
        tt.history[-1] = scaled_ldexp(*value)
    if not hasattr(tt, "refreshes"):
        tt.refreshes = []
    tt.refreshes.append(rec)
    return rec
