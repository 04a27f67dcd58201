"""TT cross interpolation and TT quadrature in double-double — oracle side (test infrastructure only).

The same method as oracle/ttcross.py (Alg. 2 on every superblock with the
previous sweep's index sets, Alg. 6; the integral as the product of 2m-1
matrices of Sec. 4.1), with every value of the computation carried in
double-double arithmetic (oracle/ddarith.py): the nodes and weights, the
weighted tensor B, the approximation B~ and the error B - B~, the cross
matrices and their solves, and the quadrature.  This stands in for the
paper's quadruple- and multiple-precision runs (Sec. 5.2), which use the same
algorithm with a longer number type.

The decisions are taken on the leading (hi) part of double-double values:
argmax of |err| with ties to the lowest index, acceptance |err| > tol *
scale_b with scale_b the largest |B| seen by the bond (as a double), and the
stopping rule on the relative change of the integral, computed in
double-double and rounded to a double.  Everything else (the readings of the
start, the samples, the rook budget, the stopping rule) is that of the double
oracle.  Only the paper-form Ising integrands (eqs. c, d, e) have a
double-double evaluation.  The folded weights carry the double oracle's exact
factor 2^s (s the integer nearest log2 n), removed from the quadrature at the
end; no double-double size here leaves the double exponent range, so the
chain needs no rescaling.

As in the double oracle nothing is incremental: every sweep re-evaluates the
cores and cross matrices from the definition of B, and every approximate entry
is B(row, I_>b) solve(B(I_<=b, I_>b), B(I_<=b, col)) by Gaussian elimination
with partial pivoting.

Pinned by: tensor quadrature by brute force in double-double (T3 = T2), the
closed forms C_3, C_4, D_3, D_4 to the quadrature error of the node count,
interpolation on the evaluated fibres (Thm. 1), and agreement with the double
oracle's decisions where both resolve the same pivots
(tests/test_oracle_dd.py).
"""

import math

import numpy as np

from . import rng
from .ddarith import DD, dd_solve, dd_sum
from .gauss import gauss_legendre_01_dd
from .integrands import PAPER_FORM, weighted_values_dd
from .ttcross import PivotRecord, TTCross


class TTCrossDD(TTCross):
    """Alg. 6 over the weighted tensor B, every value in double-double."""

    def __init__(self, family, d, n, rank_cap, tol, seed, max_sweeps=0, **kw):
        if family not in PAPER_FORM:
            raise ValueError(f"no double-double path for {family}")
        self.history_lo = []
        super().__init__(family, d, n, rank_cap, tol, seed, max_sweeps=max_sweeps, **kw)

    # ----------------------------------------------------------------- tensor
    def _nodes(self, n):
        t, w = gauss_legendre_01_dd(n)
        return t, DD(np.ldexp(w.hi, self.wshift), np.ldexp(w.lo, self.wshift))   # exact scaling

    def _unscale(self, v):
        k = -self.wshift * self.m
        return DD(np.ldexp(v.hi, k), np.ldexp(v.lo, k))

    def B(self, idx):
        idx = np.asarray(idx, dtype=np.int64)
        idx = idx.reshape(-1, self.m) if self.m > 0 else idx.reshape(idx.shape[0], 0)
        return weighted_values_dd(self.family, idx, self.t, self.w)

    def _record(self, value):
        self.history.append(float(value.hi))
        self.history_lo.append(float(value.lo))

    def value_dd(self, k=-1):
        return self.history[k], self.history_lo[k]

    # ------------------------------------------------------------ the start
    def _start(self):
        m, n = self.m, self.n
        if m == 0:
            self._record(self.B(np.zeros((1, 0), dtype=np.int64))[0])
            self.stop_reason = "converged"
            return
        if m == 1:
            self.evals += n
            self._record(self._unscale(dd_sum(self.B(np.arange(n).reshape(n, 1)), axis=0)))
            self.stop_reason = "converged"
            return
        idx = np.empty((self.n_start, m), dtype=np.int64)
        for q in range(self.n_start):
            for k in range(m):
                idx[q, k] = rng.uniform_index(rng.value(self.seed, rng.start_counter(q, k)), n)
        vals = self.B(idx)
        self.evals += self.n_start
        if not np.isfinite(vals.hi).all():
            raise FloatingPointError("non-finite start sample")
        q = int(np.argmax(np.abs(vals.hi)))
        if vals.hi[q] == 0.0:
            raise FloatingPointError("all start samples are zero")
        i0 = tuple(int(v) for v in idx[q])
        self.start_index = i0
        for b in range(m - 1):
            self.left[b].append(i0[:b + 1])
            self.right[b].append(i0[b + 1:])
            self.scale[b] = abs(float(vals.hi[q]))
        self._count_new_core_entries()
        self._record(self.integral_dd())

    # ------------------------------------------------------------ quadrature
    def integral_dd(self):
        """Product of 2m-1 matrices (Sec. 4.1), weights folded into B, in double-double."""
        v = dd_sum(self.core(0), axis=1)                     # 1 x r_0
        for c in range(1, self.m):
            M = self.cross_matrix(c - 1)
            v = dd_solve(M.T, v.T).T                         # v [M]^-1
            S = dd_sum(self.core(c), axis=1)                 # r_{c-1} x r_c
            acc = DD(np.zeros((1, S.shape[1])))
            for a in range(S.shape[0]):
                acc = acc + v[:, a:a + 1] * S[a:a + 1, :]
            v = acc
        return self._unscale(v[0, 0])

    def integral(self):
        if self.m <= 1:
            return self.history[0]
        return float(self.integral_dd().hi)

    # ------------------------------------------------ Alg. 2 on superblock b
    def cross_step(self, b, sweep, cores):
        n = self.n
        L, R = self.left_set(b - 1), self.right_set(b + 1)
        rL, rR, r = len(L), len(R), len(self.left[b])
        rec = PivotRecord(b)
        if r >= self.rank_cap:
            return rec
        rec.searched = True
        Fb = cores[b].reshape(rL * n, r)
        Fb1 = cores[b + 1].reshape(r, n * rR)
        M = self.cross_matrix(b)
        nrows, ncols = rL * n, n * rR

        def point(row, col):
            alpha, i = divmod(row, n)
            j, beta = divmod(col, rR)
            return L[alpha] + (i, j) + R[beta]

        def exact(rows, cols):
            vals = self.B([point(p, q) for p, q in zip(rows, cols)])
            self.evals += len(rows)
            return vals

        def approx(rows, cols):
            # B(row, I_>b) [B(I_<=b, I_>b)]^-1 B(I_<=b, col), one solve per distinct column
            ucols, inv = np.unique(np.asarray(cols), return_inverse=True)
            X = dd_solve(M, Fb1[:, ucols])[:, inv]           # r x npts
            return dd_sum(Fb[np.asarray(rows), :] * X.T, axis=1)

        def argmax_abs(e):
            if not np.isfinite(e.hi).all():
                raise FloatingPointError(f"non-finite error in superblock {b}")
            return int(np.argmax(np.abs(e.hi)))

        seen = 0.0
        nsamp = min(nrows + ncols, self.max_samples)
        total = nrows * ncols
        draws = [rng.uniform_index(rng.value(self.seed, rng.sample_counter(sweep, b, j)), total)
                 for j in range(nsamp)]
        rows = [q // ncols for q in draws]
        cols = [q % ncols for q in draws]
        a = exact(rows, cols)
        seen = max(seen, float(np.max(np.abs(a.hi))))
        k = argmax_abs(a - approx(rows, cols))
        row, col = rows[k], cols[k]

        all_rows, all_cols = list(range(nrows)), list(range(ncols))
        for it in range(self.t_rook):
            a_col = exact(all_rows, [col] * nrows)
            seen = max(seen, float(np.max(np.abs(a_col.hi))))
            row = argmax_abs(a_col - approx(all_rows, [col] * nrows))
            a_row = exact([row] * ncols, all_cols)
            seen = max(seen, float(np.max(np.abs(a_row.hi))))
            e_row = a_row - approx([row] * ncols, all_cols)
            col_new = argmax_abs(e_row)
            rec.iters = it + 1
            done = col_new == col
            col = col_new
            if done:
                break
        rec.row, rec.col = row, col
        rec.col_fresh, rec.n_rows, rec.n_cols = done, nrows, ncols
        rec.err, rec.value = float(e_row.hi[col]), float(a_row.hi[col])
        rec.err_lo = float(e_row.lo[col])
        self.scale[b] = max(self.scale[b], seen)
        alpha, i = divmod(row, n)
        j, beta = divmod(col, rR)
        new_left, new_right = L[alpha] + (i,), (j,) + R[beta]
        rec.accepted = (abs(rec.err) > self.tol * self.scale[b]
                        and new_left not in self.left[b] and new_right not in self.right[b])
        rec._new = (new_left, new_right)
        return rec

    # ------------------------------------------------------- Alg. 6 sweep
    def sweep(self):
        if self.stop_reason is not None:
            return
        s = self.sweeps
        cores = [self.core(c) for c in range(self.m)]
        recs = [self.cross_step(b, s, cores) for b in range(self.m - 1)]
        nacc = 0
        for rec in recs:
            if rec.accepted:
                self.left[rec.bond].append(rec._new[0])
                self.right[rec.bond].append(rec._new[1])
                nacc += 1
            rec._new = None
        self.pivot_log.append(recs)
        self.sweeps += 1
        self._count_new_core_entries(recs)
        value = self.integral_dd()
        prev = DD(self.history[-1], self.history_lo[-1])
        rel = float(abs((value - prev) / value).hi) if value.hi != 0.0 else math.inf
        self._record(value)
        prev_rel = self.rel_changes[-1] if self.rel_changes else math.inf
        self.rel_changes.append(rel)
        if self.stop_rule == "rel2" and rel <= self.tol and prev_rel <= self.tol:
            self.stop_reason = "converged"
        elif nacc == 0:
            at_cap = all(len(self.left[b]) >= self.rank_cap for b in range(self.m - 1))
            self.stop_reason = "rank_cap" if at_cap else "converged"
        elif self.sweeps >= self.max_sweeps:
            self.stop_reason = "max_sweeps"

    # ----------------------------------------------------- checks / helpers
    def reconstruct_dd(self, idx):
        """TT cross formula eq. tt at multi-indices idx (npts, m), in double-double."""
        idx = np.asarray(idx, dtype=np.int64).reshape(-1, self.m)
        cores = [self.core(c) for c in range(self.m)]
        Ms = [self.cross_matrix(b) for b in range(self.m - 1)]
        hi, lo = np.empty(idx.shape[0]), np.empty(idx.shape[0])
        for p, ii in enumerate(idx):
            v = cores[0][:, ii[0], :]
            for c in range(1, self.m):
                v = dd_solve(Ms[c - 1].T, v.T).T
                G = cores[c][:, ii[c], :]
                acc = DD(np.zeros((1, G.shape[1])))
                for a in range(G.shape[0]):
                    acc = acc + v[:, a:a + 1] * G[a:a + 1, :]
                v = acc
            hi[p], lo[p] = float(v.hi[0, 0]), float(v.lo[0, 0])
        return DD(hi, lo)


def solve_dd(family, d, n, rank_cap, tol, seed, max_sweeps=0):
    """Run the double-double oracle to its stopping rule and return the TTCrossDD object."""
    tt = TTCrossDD(family, d, n, rank_cap, tol, seed, max_sweeps=max_sweeps)
    tt.run()
    return tt
