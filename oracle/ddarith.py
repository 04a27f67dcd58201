"""Double-double arithmetic on numpy arrays — oracle side (test infrastructure only).

The paper reaches 30 and more digits with quadruple and multiple precision
(Sec. 5.2); the double-double path of the library recovers about 32 digits with
pairs (hi, lo) of doubles whose exact sum is the value, |lo| <= ulp(hi)/2.
This module is the plain reference for that arithmetic, built only from the
textbook error-free transformations:

  * two_sum (Knuth): s = fl(a + b) and the exact error e, a + b = s + e;
  * quick_two_sum (Dekker): the same when |a| >= |b|;
  * split (Veltkamp, factor 2^27 + 1) and two_prod (Dekker): p = fl(a b) and
    the exact error, without a fused multiply-add;

and the usual double-double operations on top of them (the "accurate" addition
that adds the high and the low parts separately, multiplication with the two
cross terms, division by long division with three quotient digits).  Values
are numpy arrays of any shape (or scalars); no operation is fused or reordered
for speed.

Pinned by: every operation against mpmath at 60 digits on random operands,
including cancelling sums (tests/test_oracle_dd.py).
"""

import numpy as np

SPLITTER = 134217729.0     # 2^27 + 1


def two_sum(a, b):
    s = a + b
    bb = s - a
    e = (a - (s - bb)) + (b - bb)
    return s, e


def quick_two_sum(a, b):
    s = a + b
    e = b - (s - a)
    return s, e


def split(a):
    t = SPLITTER * a
    hi = t - (t - a)
    return hi, a - hi


def two_prod(a, b):
    p = a * b
    ah, al = split(a)
    bh, bl = split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


class DD:
    """An array of double-double numbers: value = hi + lo exactly."""

    __slots__ = ("hi", "lo")

    def __init__(self, hi, lo=None):
        self.hi = np.asarray(hi, dtype=np.float64)
        self.lo = np.zeros_like(self.hi) if lo is None else np.asarray(lo, dtype=np.float64)

    # ------------------------------------------------------------ conversions
    @staticmethod
    def from_mp(values, shape=None):
        """Round mpmath numbers to double-double (hi = nearest double, lo = nearest to the rest)."""
        import mpmath as mp
        vals = list(values)
        hi = np.array([float(v) for v in vals])
        lo = np.array([float(v - mp.mpf(h)) for v, h in zip(vals, hi)])
        if shape is not None:
            hi, lo = hi.reshape(shape), lo.reshape(shape)
        return DD(hi, lo)

    def to_mp(self):
        """The exact values hi + lo as a flat list of mpmath numbers."""
        import mpmath as mp
        return [mp.mpf(float(h)) + mp.mpf(float(l)) for h, l in zip(self.hi.ravel(), self.lo.ravel())]

    def scalar(self):
        return float(self.hi), float(self.lo)

    # ------------------------------------------------------------ array shape
    @property
    def shape(self):
        return self.hi.shape

    def __len__(self):
        return len(self.hi)

    def __getitem__(self, idx):
        return DD(self.hi[idx], self.lo[idx])

    def __setitem__(self, idx, v):
        v = as_dd(v)
        self.hi[idx] = v.hi
        self.lo[idx] = v.lo

    def reshape(self, *shape):
        return DD(self.hi.reshape(*shape), self.lo.reshape(*shape))

    @property
    def T(self):
        return DD(self.hi.T, self.lo.T)

    def copy(self):
        return DD(self.hi.copy(), self.lo.copy())

    # ------------------------------------------------------------ arithmetic
    def __neg__(self):
        return DD(-self.hi, -self.lo)

    def __add__(self, other):
        y = as_dd(other)
        s, e = two_sum(self.hi, y.hi)
        t, f = two_sum(self.lo, y.lo)
        e = e + t
        s, e = quick_two_sum(s, e)
        e = e + f
        s, e = quick_two_sum(s, e)
        return DD(s, e)

    __radd__ = __add__

    def __sub__(self, other):
        return self + (-as_dd(other))

    def __rsub__(self, other):
        return as_dd(other) + (-self)

    def __mul__(self, other):
        y = as_dd(other)
        p, e = two_prod(self.hi, y.hi)
        e = e + (self.hi * y.lo + self.lo * y.hi)
        p, e = quick_two_sum(p, e)
        return DD(p, e)

    __rmul__ = __mul__

    def __truediv__(self, other):
        y = as_dd(other)
        q1 = self.hi / y.hi
        r = self - y * q1
        q2 = r.hi / y.hi
        r = r - y * q2
        q3 = r.hi / y.hi
        q1, q2 = quick_two_sum(q1, q2)
        return DD(q1, q2) + q3

    def __rtruediv__(self, other):
        return as_dd(other) / self

    def __abs__(self):
        neg = self.hi < 0
        return DD(np.where(neg, -self.hi, self.hi), np.where(neg, -self.lo, self.lo))

    def square(self):
        return self * self


def as_dd(x):
    return x if isinstance(x, DD) else DD(x)


def zeros(shape):
    return DD(np.zeros(shape))


def ones(shape):
    return DD(np.ones(shape))


def dd_sum(x, axis):
    """Sum along one axis, accumulated left to right in double-double."""
    hi = np.moveaxis(x.hi, axis, 0)
    lo = np.moveaxis(x.lo, axis, 0)
    acc = DD(np.zeros(hi.shape[1:]))
    for k in range(hi.shape[0]):
        acc = acc + DD(hi[k], lo[k])
    return acc


def dd_prod(x, axis):
    """Product along one axis, left to right in double-double."""
    hi = np.moveaxis(x.hi, axis, 0)
    lo = np.moveaxis(x.lo, axis, 0)
    acc = DD(np.ones(hi.shape[1:]))
    for k in range(hi.shape[0]):
        acc = acc * DD(hi[k], lo[k])
    return acc


def dd_matmul(a, b):
    """(p x q) @ (q x s) in double-double, summing over the inner index in order."""
    p, q = a.shape
    q2, s = b.shape
    if q != q2:
        raise ValueError("inner dimensions differ")
    acc = zeros((p, s))
    for k in range(q):
        acc = acc + a[:, k:k + 1] * b[k:k + 1, :]
    return acc


def dd_solve(M, rhs):
    """Solve M X = rhs (M square) by Gaussian elimination with partial pivoting, in double-double."""
    A = M.copy()
    X = rhs.copy()
    vec = X.hi.ndim == 1
    if vec:
        X = X.reshape(-1, 1)
    r = A.shape[0]
    for k in range(r):
        piv = k + int(np.argmax(np.abs(A.hi[k:, k])))
        if A.hi[piv, k] == 0.0:
            raise np.linalg.LinAlgError("singular matrix")
        if piv != k:
            for arr in (A, X):
                for part in (arr.hi, arr.lo):
                    part[[k, piv]] = part[[piv, k]]
        f = A[k + 1:, k:k + 1] / A[k, k]               # multipliers of the rows below
        A[k + 1:, k:] = A[k + 1:, k:] - f * A[k:k + 1, k:]
        X[k + 1:, :] = X[k + 1:, :] - f * X[k:k + 1, :]
    for k in range(r - 1, -1, -1):                    # back substitution
        s = X[k, :]
        for j in range(k + 1, r):
            s = s - A[k, j] * X[j, :]
        X[k, :] = s / A[k, k]
    return X.reshape(-1) if vec else X
