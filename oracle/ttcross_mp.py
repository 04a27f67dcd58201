"""TT cross interpolation and TT quadrature in 256-bit arithmetic — oracle side (test infrastructure only).

The same method as oracle/ttcross.py (Alg. 2 on every superblock against the
previous sweep's index sets, Alg. 6; the integral as the product of 2m-1
matrices of Sec. 4.1) with every value an mpmath number of a fixed binary
precision (256 bits, about 77 decimal digits, by default): the Gauss-Legendre
nodes and weights, the weighted tensor B, the approximation B~ and the error
B - B~, the cross matrices and their solves, and the quadrature.  It plays the
part of the paper's multiple-precision runs (Sec. 5.2: the same algorithm with
a longer number type) as the reference for the double-double library: at this
precision its rounding is some 45 digits below the double-double level, so a
double-double result that agrees with it to 1e-20 is accurate to 1e-20 in its
own right, not only consistent with another double-double computation.

Readings of the paper where it is silent are those of the double oracle: rank-1
start at the largest |B| among 1024 SplitMix64 grid samples, |R| =
min(r_{b-1} n + n r_{b+1}, 1024) samples per superblock keyed by (seed, sweep,
bond, sample), at most 5 rook (column, row) pairs, argmax of |err| with ties to
the lowest index, acceptance |err*| > tol * scale_b (scale_b the largest |B| the
bond has evaluated) with r_b below the cap and neither half of the pivot
already in its set, and the stopping rule on the relative change of the
integral (two consecutive sweeps at or below tol, or a sweep that accepts no
pivot, or max_sweeps).  The decisions compare the full-precision values; the
double-double library compares leading doubles, which decides the same way
except on ties closer than about 1e-16 relative.  Weights are folded into B
(Sec. 4.1) with the double oracle's exact factor 2^s (s the integer nearest
log2 n), removed from the integral at the end; in this arithmetic nothing
leaves the exponent range, so the chain is not rescaled.

Nothing is incremental: every sweep rebuilds the cores and cross matrices from
the definition of B (each distinct tensor entry is evaluated once and kept,
since B is a fixed function of the multi-index), and every approximate entry
is B(row, I_>b) M_b^-1 B(I_<=b, col) with M_b = B(I_<=b, I_>b) factorised by
Gaussian elimination with partial pivoting.  Only the paper-form Ising
integrands (eqs. c, d, e) are provided.

Pinned by (tests/test_oracle_mp.py): the 256-bit Gauss-Legendre rule against
mpmath's own Legendre function and exact moments; the integrands against the
closed forms C_3 = L_{-3}(2), C_4 = 7 zeta(3)/12, D_3, D_4 by brute-force
tensor quadrature at enough nodes for 1e-60; the cross against brute-force
tensor quadrature of the same nodes (T3 = T2) at n <= 6, where it recovers the
whole tensor; interpolation on every evaluated fibre (Thm. 1).
"""

import functools
import math

import mpmath as mp

from . import rng
from .integrands import PAPER_FORM, n_modes
from .ttcross import MAX_SAMPLES, N_START, T_ROOK, weight_shift

PREC = 256


# ------------------------------------------------------------ GL rule
def _legendre_pair(n, x):
    """P_n(x), P_{n-1}(x) by (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}."""
    p_prev, p = mp.mpf(1), x
    if n == 0:
        return p_prev, mp.mpf(0)
    for k in range(1, n):
        p_prev, p = p, ((2 * k + 1) * x * p - k * p_prev) / (k + 1)
    return p, p_prev


@functools.lru_cache(maxsize=64)
def gauss_legendre_01_mp(n, prec=PREC):
    """Nodes (increasing) and weights of the n-point rule on [0,1] at `prec` bits.

    The nodes are the roots of P_n on [-1,1] by Newton's method from the
    classical initial guess, carried 32 bits beyond `prec` and rounded once;
    the weights are 2 / ((1 - x^2) P_n'(x)^2); both mapped by t = (x+1)/2,
    w = w_x / 2.
    """
    with mp.workprec(prec + 32):
        t, w = [], []
        eps = mp.mpf(2) ** (-(prec + 24))
        for k in range(1, n + 1):
            x = mp.cos(mp.pi * (k - mp.mpf(1) / 4) / (n + mp.mpf(1) / 2))
            for _ in range(200):
                p, q = _legendre_pair(n, x)
                dp = n * (x * p - q) / (x * x - 1)
                dx = p / dp
                x -= dx
                if abs(dx) < eps:
                    break
            p, q = _legendre_pair(n, x)
            dp = n * (x * p - q) / (x * x - 1)
            t.append((x + 1) / 2)
            w.append(1 / ((1 - x * x) * dp * dp))
    with mp.workprec(prec):
        order = sorted(range(n), key=lambda i: t[i])
        return tuple(+t[i] for i in order), tuple(+w[i] for i in order)


# ----------------------------------------------------------- integrand
def ising_paper_mp(family, x):
    """The paper form (Sec. 5.1, eqs. c, d, e) at one point x = (x_2, .., x_d), factor 2 included.

    A_d = prod_{1<=i<j<=d} ((1 - x_{i+1}..x_j) / (1 + x_{i+1}..x_j))^2 and
    B_d = (1 + sum_{k=2}^d x_2..x_k)^-1 (1 + sum_{k=2}^d x_k..x_d)^-1, every run
    product recomputed from its factors.
    """
    d = len(x) + 1

    def prod_range(a, b):   # x_a .. x_b, 2 <= a <= b <= d
        p = mp.mpf(1)
        for k in range(a, b + 1):
            p *= x[k - 2]
        return p

    f = mp.mpf(2)
    if family in ("ising_c", "ising_d"):
        s_left = mp.mpf(1) + mp.fsum(prod_range(2, k) for k in range(2, d + 1))
        s_right = mp.mpf(1) + mp.fsum(prod_range(k, d) for k in range(2, d + 1))
        f = f / (s_left * s_right)
    if family in ("ising_d", "ising_e"):
        a_d = mp.mpf(1)
        for i in range(1, d):
            for j in range(i + 1, d + 1):
                p = prod_range(i + 1, j)
                a_d *= ((1 - p) / (1 + p)) ** 2
        f = f * a_d
    return f


# --------------------------------------------------- dense linear algebra
class LU:
    """P A = L U by Gaussian elimination with partial pivoting (textbook), for repeated solves."""

    def __init__(self, A):
        n = len(A)
        a = [list(row) for row in A]
        perm = list(range(n))
        for k in range(n):
            p = max(range(k, n), key=lambda i: abs(a[i][k]))
            if a[p][k] == 0:
                raise ZeroDivisionError("singular cross matrix")
            if p != k:
                a[k], a[p] = a[p], a[k]
                perm[k], perm[p] = perm[p], perm[k]
            for i in range(k + 1, n):
                f = a[i][k] / a[k][k]
                a[i][k] = f
                for j in range(k + 1, n):
                    a[i][j] -= f * a[k][j]
        self.a, self.perm, self.n = a, perm, n

    def solve(self, b):
        """x with A x = b."""
        a, n = self.a, self.n
        y = [b[self.perm[i]] for i in range(n)]
        for i in range(n):
            y[i] -= mp.fsum(a[i][j] * y[j] for j in range(i))
        for i in range(n - 1, -1, -1):
            y[i] = (y[i] - mp.fsum(a[i][j] * y[j] for j in range(i + 1, n))) / a[i][i]
        return y

    def solve_transposed(self, b):
        """x with A^T x = b (U^T z = b, L^T w = z, x = P^T w)."""
        a, n = self.a, self.n
        z = list(b)
        for i in range(n):
            z[i] = (z[i] - mp.fsum(a[j][i] * z[j] for j in range(i))) / a[i][i]
        for i in range(n - 1, -1, -1):
            z[i] -= mp.fsum(a[j][i] * z[j] for j in range(i + 1, n))
        x = [None] * n
        for i in range(n):
            x[self.perm[i]] = z[i]
        return x


def _dot(u, v):
    return mp.fsum(a * b for a, b in zip(u, v))


class Record:
    __slots__ = ("bond", "row", "col", "err", "value", "accepted", "iters", "col_fresh", "_new")

    def __init__(self, bond):
        self.bond, self.row, self.col = bond, -1, -1
        self.err = self.value = mp.mpf(0)
        self.accepted, self.iters, self.col_fresh, self._new = False, 0, False, None


class TTCrossMP:
    """Alg. 6 (one superblock per process) over the weighted tensor B, every value at `prec` bits."""

    def __init__(self, family, d, n, rank_cap, tol, seed, max_sweeps=0, prec=PREC, stop_rule="rel2"):
        if family not in PAPER_FORM:
            raise ValueError(f"no multiple-precision path for {family}")
        if stop_rule not in ("rel2", "strict"):
            raise ValueError(stop_rule)
        self.stop_rule = stop_rule
        self.family, self.d, self.n, self.prec = family, d, n, prec
        self.rank_cap, self.tol, self.seed = rank_cap, mp.mpf(tol), seed
        self.max_sweeps = max_sweeps if max_sweeps > 0 else 4 * rank_cap
        self.m = n_modes(family, d)
        self.wshift = weight_shift(n)
        with mp.workprec(prec):
            t, w = gauss_legendre_01_mp(n, prec)
            self.t = t
            self.w = tuple(mp.ldexp(v, self.wshift) for v in w)   # exact
        nb = max(self.m - 1, 0)
        self.left = [[] for _ in range(nb)]
        self.right = [[] for _ in range(nb)]
        self.scale = [mp.mpf(0)] * nb
        self.sweeps = 0
        self.history = []
        self.rel_changes = []
        self.pivot_log = []
        self.stop_reason = None
        self._memo = {}
        with mp.workprec(prec):
            self._start()

    # ----------------------------------------------------------------- tensor
    def B(self, idx):
        """Weighted tensor entry at one multi-index (a tuple of node indices)."""
        v = self._memo.get(idx)
        if v is None:
            with mp.workprec(self.prec):
                wt = mp.mpf(1)
                for i in idx:
                    wt *= self.w[i]
                v = wt * ising_paper_mp(self.family, [self.t[i] for i in idx])
            self._memo[idx] = v
        return v

    def left_set(self, b):
        return [()] if b < 0 else self.left[b]

    def right_set(self, b):
        return [()] if b >= self.m - 1 else self.right[b]

    def core(self, c):
        """F_c as rows (alpha, i), alpha-major, of r_c entries."""
        L, R = self.left_set(c - 1), self.right_set(c)
        return [[self.B(l + (i,) + r) for r in R] for l in L for i in range(self.n)]

    def cross_matrix(self, b):
        return [[self.B(l + r) for r in self.right[b]] for l in self.left[b]]

    # ------------------------------------------------------------ the start
    def _start(self):
        m, n = self.m, self.n
        if m <= 1:
            self.history.append(self.integral())
            self.stop_reason = "converged"
            return
        best, i0 = None, None
        for q in range(N_START):
            idx = tuple(rng.uniform_index(rng.value(self.seed, rng.start_counter(q, k)), n) for k in range(m))
            v = abs(self.B(idx))
            if best is None or v > best:
                best, i0 = v, idx
        if best == 0:
            raise FloatingPointError("all start samples are zero")
        self.start_index = i0
        for b in range(m - 1):
            self.left[b].append(i0[:b + 1])
            self.right[b].append(i0[b + 1:])
            self.scale[b] = best
        self.history.append(self.integral())

    # ------------------------------------------------------------ quadrature
    def integral(self):
        """Product of 2m-1 matrices (Sec. 4.1) with the weights folded into B."""
        with mp.workprec(self.prec):
            return self._integral()

    def _integral(self):
        n, m = self.n, self.m
        if m == 0:
            return self.B(())
        if m == 1:
            return mp.fsum(self.B((i,)) for i in range(n)) * mp.ldexp(1, -self.wshift)
        F0 = self.core(0)
        v = [mp.fsum(F0[i][k] for i in range(n)) for k in range(len(self.right[0]))]
        for c in range(1, m):
            v = LU(self.cross_matrix(c - 1)).solve_transposed(v)    # v M^-1
            Fc = self.core(c)
            rl, rr = len(self.left_set(c - 1)), len(self.right_set(c))
            v = [mp.fsum(v[a] * Fc[a * n + i][k] for a in range(rl) for i in range(n)) for k in range(rr)]
        return v[0] * mp.ldexp(1, -self.wshift * m)

    # ------------------------------------------------ Alg. 2 on superblock b
    def cross_step(self, b, sweep, cores):
        n = self.n
        L, R = self.left_set(b - 1), self.right_set(b + 1)
        rL, rR, r = len(L), len(R), len(self.left[b])
        rec = Record(b)
        if r >= self.rank_cap:
            return rec
        Fb = cores[b]                      # rows (alpha, i): r entries
        Fb1 = cores[b + 1]                 # rows (k, j): rR entries; column (j, beta)
        lu = LU(self.cross_matrix(b))
        nrows, ncols = rL * n, n * rR

        def point(row, col):
            alpha, i = divmod(row, n)
            j, beta = divmod(col, rR)
            return L[alpha] + (i, j) + R[beta]

        def f1col(col):                    # B(I_<=b, col)
            j, beta = divmod(col, rR)
            return [Fb1[k * n + j][beta] for k in range(r)]

        solved = {}

        def minv_col(col):                 # M_b^-1 B(I_<=b, col), once per column of this step
            x = solved.get(col)
            if x is None:
                x = solved[col] = lu.solve(f1col(col))
            return x

        def argmax_abs(vals):
            best, bi = None, -1
            for q, e in enumerate(vals):
                if not mp.isfinite(e):
                    raise FloatingPointError(f"non-finite error in superblock {b}")
                if best is None or abs(e) > best:
                    best, bi = abs(e), q
            return bi

        seen = mp.mpf(0)
        nsamp = min(nrows + ncols, MAX_SAMPLES)
        total = nrows * ncols
        draws = [rng.uniform_index(rng.value(self.seed, rng.sample_counter(sweep, b, j)), total)
                 for j in range(nsamp)]
        errs = []
        for q in draws:
            row, col = divmod(q, ncols)
            a = self.B(point(row, col))
            seen = max(seen, abs(a))
            errs.append(a - _dot(Fb[row], minv_col(col)))
        k = argmax_abs(errs)
        row, col = divmod(draws[k], ncols)
        done = False
        for it in range(T_ROOK):
            x = minv_col(col)                              # M^-1 B(I_<=b, col)
            a_col = [self.B(point(p, col)) for p in range(nrows)]
            seen = max([seen] + [abs(a) for a in a_col])
            row = argmax_abs([a_col[p] - _dot(Fb[p], x) for p in range(nrows)])
            y = lu.solve_transposed(Fb[row])               # B(row, I_>b) M^-1
            a_row = [self.B(point(row, q)) for q in range(ncols)]
            seen = max([seen] + [abs(a) for a in a_row])
            e_row = [a_row[q] - _dot(y, f1col(q)) for q in range(ncols)]
            col_new = argmax_abs(e_row)
            rec.iters = it + 1
            done = col_new == col
            col = col_new
            if done:
                break
        rec.row, rec.col, rec.col_fresh = row, col, done
        rec.err, rec.value = e_row[col], a_row[col]
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
        with mp.workprec(self.prec):
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
            value = self.integral()
            prev = self.history[-1]
            rel = abs(value - prev) / abs(value) if value != 0 else mp.inf
            self.history.append(value)
            prev_rel = self.rel_changes[-1] if self.rel_changes else mp.inf
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

    def ranks(self):
        return [len(self.left[b]) for b in range(self.m - 1)]


def solve(family, d, n, rank_cap, tol, seed, max_sweeps=0, prec=PREC):
    """Run the multiple-precision oracle to its stopping rule and return the TTCrossMP object."""
    tt = TTCrossMP(family, d, n, rank_cap, tol, seed, max_sweeps=max_sweeps, prec=prec)
    tt.run()
    return tt


def tensor_quadrature_mp(family, d, n, prec=PREC):
    """T2: the tensor-product Gauss-Legendre sum over all n^m nodes, at `prec` bits (brute force)."""
    import itertools
    m = n_modes(family, d)
    with mp.workprec(prec):
        t, w = gauss_legendre_01_mp(n, prec)
        total = []
        for idx in itertools.product(range(n), repeat=m):
            wt = mp.mpf(1)
            for i in idx:
                wt *= w[i]
            total.append(wt * ising_paper_mp(family, [t[i] for i in idx]))
        return mp.fsum(total)
