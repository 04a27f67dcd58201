"""TT cross interpolation and TT quadrature — oracle side (test infrastructure only).

What is computed
----------------
The weighted tensor B(i_1..i_m) = w_{i_1}..w_{i_m} f(t_{i_1},..,t_{i_m})
(Sec. 4.1) is interpolated in the TT cross form eq. tt (Sec. 3.2),

    B ~ B(i_1, I_>1) [B(I_<=1, I_>1)]^-1 B(I_<=1, i_2, I_>2) ... B(I_<=m-1, i_m),

with nested index sets (eq. nest), and the integral is the product of 2m-1
matrices of Sec. 4.1 (each core summed over its mode index, the cross matrices
inverted).  The index sets are grown by the dimension-parallel greedy cross of
Alg. 6 with one superblock per "process" (the paper's finest partitioning):
in a sweep every superblock b, seen as the (r_{b-1} n) x (n r_{b+1}) matrix
B(I_<=b-1 i_b, i_b+1 I_>b+1), is searched with the index sets of the PREVIOUS
sweep (Sec. 3.4: the sets of the neighbours are not expanded until the sweep
ends), by one step of Alg. 2 (random samples, then alternating column and row
pivoting until the rook condition eq. rook holds or the budget is spent).  The
new pivot of every accepted superblock is then appended to its two sets
(Alg. 5/6, set-expansion step), which keeps them nested.

This oracle deliberately does NOT update anything incrementally: every sweep
re-evaluates every core and cross matrix from the definition of B, and every
approximate entry is computed as B(row, I_>b) @ solve(B(I_<=b, I_>b), B(I_<=b, col))
with numpy's LU solve.

Scaled weights and a scaled quadrature (the paper does not say how its
1023-mode double-precision run keeps the folded weights in range): every
folded weight is multiplied by 2^s, s the integer nearest log2 n (the weights
sum to 1, so their mean becomes about 1), and the chain of Sec. 4.1 is brought
back after every factor to a vector whose largest entry lies in [1/2, 1),
counting the powers of two it removes.  The integral is the chain's value
times 2^(E - s m).  Both scalings are exact, so for every size that does not
leave the double range the decisions and the values are those of the unscaled
computation, bit for bit.

Readings of the paper where it is silent:
  * start: rank 1 at the largest |B| among 1024 SplitMix64 samples of the grid;
    above 32 modes, for D_d and E_d, the n constant multi-indices (every mode
    at node j) are candidates too, after the random ones, since a random
    point's B falls far below the double range for D_d from about d = 128 on
    (Sec. 5.5) while the constant points reach the largest entries (C_d and the
    synthetic families stay near 1).  Above 32 modes the candidates are
    compared by magnitude in (mantissa, exponent) form, and every B of the job
    is taken as B 2^E, E = -(the exponent of the chosen start's B), so that
    the start's B lies in [1/2, 1); the integral is unscaled by 2^-E.  The
    scaling is exact wherever the unscaled value is a normal double;
  * samples: |R| = min(r_{b-1} n + n r_{b+1}, 1024), uniform over the superblock,
    drawn from SplitMix64 keyed by (seed, sweep, bond, sample);
  * rook budget: at most 5 (column, row) pairs;
  * argmax ties go to the lowest index (rows (alpha, i) alpha-major, columns
    (j, beta) j-major, samples in draw order); a non-finite start sample or
    error (B infinite or NaN) is a numeric error;
  * acceptance: |err*| > tol * scale_b, where scale_b is the largest |B| the
    bond has evaluated so far, r_b < rank_cap, and neither half of the pivot is
    already in its set;
  * stopping ("rel2"): relative change of the integral <= tol on two
    consecutive sweeps, or a sweep that accepts no pivot, or max_sweeps;
    "strict" drops the first condition: only a sweep that accepts no pivot
    (every superblock error at most tol times its largest |B|), the rank cap on
    every bond, or max_sweeps end the run.

Pinned by: exact integrals of rank-1 and rank-2 synthetic functions (Thm. 2),
interpolation on every evaluated fiber (Thm. 1), brute-force tensor quadrature
for small m, closed forms C_3, C_4, D_3, D_4 and the printed D_8; the scaled
weights and chain by equality with the unscaled computation and by rank-1
products of 1100 factors far below the double range.
"""

import math

import numpy as np

from . import rng
from .gauss import gauss_legendre_01
from .integrands import PAPER_FORM, log2_weighted_values, n_modes, weighted_values

T_ROOK = 5
MAX_SAMPLES = 1024
N_START = 1024
SCALED_START_MODES = 32   # above this many modes: constant start candidates and the scale 2^E
DBL_MIN = 2.0 ** -1022


def weight_shift(n):
    """The integer nearest log2 n: floor(log2(n sqrt 2))."""
    return math.frexp(n * math.sqrt(2.0))[1] - 1


def scaled_ldexp(mant, e):
    """mant * 2^e as a double (0 below the range, +-inf above it)."""
    try:
        return math.ldexp(mant, e)
    except OverflowError:
        return math.copysign(math.inf, mant)


def renormalise(v, e):
    """Scale v by a power of two so that max |v| lies in [1/2, 1); returns (v, e + shift)."""
    mx = float(np.max(np.abs(v))) if v.size else 0.0
    if mx > 0.0 and math.isfinite(mx):
        k = math.frexp(mx)[1]
        v = np.ldexp(v, -k)
        e += k
    return v, e


def rel_change_scaled(cur, prev):
    """|I_s - I_{s-1}| / |I_s| for values given as (mantissa, exponent) pairs."""
    mc, ec = cur
    mp_, ep = prev
    if mc == 0.0:
        return math.inf
    return abs(mc - scaled_ldexp(mp_, ep - ec)) / abs(mc)


class PivotRecord:
    __slots__ = ("bond", "row", "col", "err", "err_lo", "value", "accepted", "iters", "searched", "_new",
                 "col_fresh", "n_rows", "n_cols")

    def __init__(self, bond, row=-1, col=-1, err=0.0, value=0.0, accepted=False, iters=0,
                 searched=False):
        self.bond, self.row, self.col = bond, row, col
        self.err, self.value = err, value
        self.err_lo = 0.0            # low part of err in the double-double oracle
        self.col_fresh = False       # the last column step was at the final column
        self.n_rows = self.n_cols = 0   # superblock size at the time of the search
        self.accepted, self.iters, self.searched = accepted, iters, searched
        self._new = None

    def __repr__(self):
        return (f"Pivot(b={self.bond}, row={self.row}, col={self.col}, err={self.err:.3e}, "
                f"acc={self.accepted}, it={self.iters})")


class TTCross:
    """Alg. 6 (one superblock per process) over the weighted tensor B."""

    def __init__(self, family, d, n, rank_cap, tol, seed, max_sweeps=0, params=None,
                 t_rook=T_ROOK, max_samples=MAX_SAMPLES, n_start=N_START, scale_weights=True,
                 value_scale=True, stop_rule="rel2"):
        self.family, self.d, self.n = family, d, n
        self.wshift = weight_shift(n) if scale_weights else 0
        self.rank_cap, self.tol, self.seed = rank_cap, tol, seed
        self.max_sweeps = max_sweeps if max_sweeps > 0 else 4 * rank_cap
        self.params = params
        self.t_rook, self.max_samples, self.n_start = t_rook, max_samples, n_start
        self.m = n_modes(family, d)
        self.t, self.w = self._nodes(n)
        nb = max(self.m - 1, 0)
        self.left = [[] for _ in range(nb)]    # left[b]:  I_<=b, tuples (i_0..i_b)
        self.right = [[] for _ in range(nb)]   # right[b]: I_>b,  tuples (i_b+1..i_m-1)
        self.scale = [0.0] * nb
        self.escale = 0         # E: every B of the job is taken times 2^E (above 32 modes)
        self.value_scale = value_scale   # False keeps E = 0 (the candidates stay the same)
        if stop_rule not in ("rel2", "strict"):
            raise ValueError(stop_rule)
        self.stop_rule = stop_rule
        self.sweeps = 0
        self.evals = 0
        self.history = []       # integral after the start and after every sweep
        self.history_scaled = []  # the same as (mantissa, exponent): value = mantissa * 2^exponent
        self.rel_changes = []
        self.pivot_log = []     # one list of PivotRecord per sweep
        self.stop_reason = None
        self._core_sizes = [0] * self.m
        self._start()

    # ----------------------------------------------------------------- tensor
    def _nodes(self, n):
        t, w = gauss_legendre_01(n)
        return t, np.ldexp(w, self.wshift)

    def B(self, idx):
        """B at the multi-indices idx, times 2^E."""
        idx = np.asarray(idx, dtype=np.int64)
        idx = idx.reshape(-1, self.m) if self.m > 0 else idx.reshape(idx.shape[0], 0)
        vals = weighted_values(self.family, idx, self.t, self.w, self.params)
        if self.escale == 0:
            return vals
        out = np.ldexp(vals, self.escale)
        low = np.abs(vals) < DBL_MIN   # zero or subnormal before scaling: take it through logarithms
        if low.any():
            if self.family not in PAPER_FORM:
                raise FloatingPointError("values below the double range outside the paper form")
            out[low] = np.exp2(log2_weighted_values(self.family, idx[low], self.t, self.w) + self.escale)
        return out

    def magnitudes(self, idx):
        """Unscaled |B| at idx as (mantissa in [1/2, 1), exponent) arrays; mantissa 0 for B = 0."""
        idx = np.asarray(idx, dtype=np.int64).reshape(-1, self.m)
        vals = weighted_values(self.family, idx, self.t, self.w, self.params)
        if not np.isfinite(vals).all():
            raise FloatingPointError("non-finite start sample")
        mant, ex = np.frexp(np.abs(vals))
        low = np.abs(vals) < DBL_MIN
        if low.any() and self.family in PAPER_FORM:
            l2 = log2_weighted_values(self.family, idx[low], self.t, self.w)
            e = np.floor(l2).astype(np.int64) + 1
            mant[low] = np.exp2(l2 - e)
            ex[low] = e
        return mant, ex.astype(np.int64)

    def left_set(self, b):
        return [()] if b < 0 else self.left[b]

    def right_set(self, b):
        return [()] if b >= self.m - 1 else self.right[b]

    def core(self, c):
        """F_c = B(I_<=c-1, i_c, I_>c) as an array (r_{c-1}, n, r_c)."""
        L, R = self.left_set(c - 1), self.right_set(c)
        idx = [l + (i,) + r for l in L for i in range(self.n) for r in R]
        return self.B(idx).reshape(len(L), self.n, len(R))

    def cross_matrix(self, b):
        """M_b = B(I_<=b, I_>b), r_b x r_b."""
        L, R = self.left[b], self.right[b]
        idx = [l + r for l in L for r in R]
        return self.B(idx).reshape(len(L), len(R))

    # ------------------------------------------------------------ the start
    def _start(self):
        m, n = self.m, self.n
        if m <= 1:
            self.evals += n if m == 1 else 0
            self._record(self.integral_scaled())
            self.stop_reason = "converged"
            return
        idx = np.empty((self.n_start, m), dtype=np.int64)
        for q in range(self.n_start):
            for k in range(m):
                idx[q, k] = rng.uniform_index(rng.value(self.seed, rng.start_counter(q, k)), n)
        if m > SCALED_START_MODES:
            if self.family in ("ising_d", "ising_e"):
                idx = np.vstack([idx, np.repeat(np.arange(n, dtype=np.int64)[:, None], m, axis=1)])
            mant, ex = self.magnitudes(idx)
            self.evals += len(idx)
            if not (mant > 0).any():
                raise FloatingPointError("all start samples are zero")
            etop = int(ex[mant > 0].max())
            keys = np.where(mant > 0, np.ldexp(mant, ex - etop), 0.0)
            q = int(np.argmax(keys))   # ties: the lowest candidate index
            self.escale = -etop if self.value_scale else 0
            start_value = math.ldexp(float(keys[q]), etop + self.escale)
        else:
            vals = self.B(idx)
            self.evals += self.n_start
            if not np.isfinite(vals).all():
                raise FloatingPointError("non-finite start sample")
            q = int(np.argmax(np.abs(vals)))
            if vals[q] == 0.0:
                raise FloatingPointError("all start samples are zero")
            start_value = abs(float(vals[q]))
        i0 = tuple(int(v) for v in idx[q])
        self.start_index = i0
        for b in range(m - 1):
            self.left[b].append(i0[:b + 1])
            self.right[b].append(i0[b + 1:])
            self.scale[b] = start_value
        self._count_new_core_entries()
        self._record(self.integral_scaled())

    def _record(self, scaled):
        self.history_scaled.append(scaled)
        self.history.append(scaled_ldexp(*scaled))

    def _count_new_core_entries(self, recs=()):
        """Count the entries the core updates evaluate after the sets grew.

        Reading: the last row step of an accepted search at bond b evaluated
        the new row of F_{b+1} at its old columns, and the last column step,
        when it was taken at the final column, the new column of F_b at its
        old rows (these are the same tensor entries); the updates reuse them,
        so only the remaining new entries are evaluated again.
        """
        reused = 0
        for rec in recs:
            if rec.accepted:
                reused += rec.n_cols + (rec.n_rows if rec.col_fresh else 0)
        for c in range(self.m):
            size = len(self.left_set(c - 1)) * self.n * len(self.right_set(c))
            self.evals += size - self._core_sizes[c]
            self._core_sizes[c] = size
        self.evals -= reused

    # ------------------------------------------------------------ quadrature
    def integral_scaled(self):
        """Product of 2m-1 matrices (Sec. 4.1) with weights folded into B, as (mantissa, exponent).

        The running vector is rescaled by a power of two after every factor;
        the exponent collects those powers and the weights' 2^(-s m).
        """
        if self.m == 0:
            v, e = np.array([[float(self.B(np.zeros((1, 0), dtype=np.int64))[0])]]), 0
        elif self.m == 1:
            v, e = np.array([[float(np.sum(self.B(np.arange(self.n).reshape(self.n, 1))))]]), 0
        else:
            v, e = renormalise(self.core(0).sum(axis=1), 0)          # 1 x r_0
            for c in range(1, self.m):
                M = self.cross_matrix(c - 1)                         # r_{c-1} x r_{c-1}
                v = np.linalg.solve(M.T, v.T).T                      # v [M]^-1
                v, e = renormalise(v @ self.core(c).sum(axis=1), e)  # r_{c-1} x r_c
        mant, k = math.frexp(float(v[0, 0]))
        return mant, e + k - self.wshift * self.m - self.escale

    def integral(self):
        return scaled_ldexp(*self.integral_scaled())

    # ------------------------------------------------ Alg. 2 on superblock b
    def cross_step(self, b, sweep, cores):
        n = self.n
        L, R = self.left_set(b - 1), self.right_set(b + 1)
        rL, rR, r = len(L), len(R), len(self.left[b])
        rec = PivotRecord(b)
        if r >= self.rank_cap:
            return rec
        rec.searched = True
        Fb = cores[b].reshape(rL * n, r)           # rows (alpha, i), alpha-major
        Fb1 = cores[b + 1].reshape(r, n * rR)      # columns (j, beta), j-major
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
            # B(row, I_>b) [B(I_<=b, I_>b)]^-1 B(I_<=b, col), for each (row, col) pair
            X = np.linalg.solve(M, Fb1[:, cols])
            return np.einsum("kr,rk->k", Fb[rows, :], X)

        def argmax_abs(e):
            if not np.isfinite(e).all():
                raise FloatingPointError(f"non-finite error in superblock {b}")
            return int(np.argmax(np.abs(e)))

        seen = 0.0
        # random samples (Alg. 2, first step)
        nsamp = min(nrows + ncols, self.max_samples)
        total = nrows * ncols
        draws = [rng.uniform_index(rng.value(self.seed, rng.sample_counter(sweep, b, j)), total)
                 for j in range(nsamp)]
        rows = [q // ncols for q in draws]
        cols = [q % ncols for q in draws]
        a = exact(rows, cols)
        seen = max(seen, float(np.max(np.abs(a))))
        k = argmax_abs(a - approx(rows, cols))
        row, col = rows[k], cols[k]

        # alternating column / row pivoting until the rook condition holds
        all_rows, all_cols = list(range(nrows)), list(range(ncols))
        for it in range(self.t_rook):
            a_col = exact(all_rows, [col] * nrows)
            seen = max(seen, float(np.max(np.abs(a_col))))
            row = argmax_abs(a_col - approx(all_rows, [col] * nrows))
            a_row = exact([row] * ncols, all_cols)
            seen = max(seen, float(np.max(np.abs(a_row))))
            e_row = a_row - approx([row] * ncols, all_cols)
            col_new = argmax_abs(e_row)
            rec.iters = it + 1
            done = col_new == col
            col = col_new
            if done:
                break
        rec.row, rec.col = row, col
        rec.col_fresh, rec.n_rows, rec.n_cols = done, nrows, ncols
        rec.err, rec.value = float(e_row[col]), float(a_row[col])
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
        for rec in recs:                       # expand the sets after the sweep
            if rec.accepted:
                self.left[rec.bond].append(rec._new[0])
                self.right[rec.bond].append(rec._new[1])
                nacc += 1
            rec._new = None
        self.pivot_log.append(recs)
        self.sweeps += 1
        self._count_new_core_entries(recs)
        value = self.integral_scaled()
        rel = rel_change_scaled(value, self.history_scaled[-1])
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

    def run(self):
        while self.stop_reason is None:
            self.sweep()
        return self.history[-1]

    # ----------------------------------------------------- checks / helpers
    def ranks(self):
        return [len(self.left[b]) for b in range(self.m - 1)]

    def reconstruct(self, idx):
        """TT cross formula eq. tt at multi-indices idx (npts, m)."""
        idx = np.asarray(idx, dtype=np.int64).reshape(-1, self.m)
        cores = [self.core(c) for c in range(self.m)]
        Ms = [self.cross_matrix(b) for b in range(self.m - 1)]
        out = np.empty(idx.shape[0])
        for p, ii in enumerate(idx):
            v = cores[0][:, ii[0], :]
            for c in range(1, self.m):
                v = np.linalg.solve(Ms[c - 1].T, v.T).T
                v = v @ cores[c][:, ii[c], :]
            out[p] = v[0, 0]
        return out


def solve(family, d, n, rank_cap, tol, seed, max_sweeps=0, params=None, stop_rule="rel2"):
    """Run the oracle to its stopping rule and return the TTCross object."""
    tt = TTCross(family, d, n, rank_cap, tol, seed, max_sweeps=max_sweeps, params=params, stop_rule=stop_rule)
    tt.run()
    return tt
