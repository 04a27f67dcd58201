// Device-side building blocks for the gfx950 TT cross library:
//   * double-double error-free transforms (Dekker 1971; Knuth TAOCP vol. 2;
//     the accurate double-word sum/product of Joldes, Muller & Popescu 2017),
//   * the SplitMix64 counter-based generator (Steele, Lea & Flood 2014),
//   * the integrands of the Ising family (eqs. c, d, e of Sec. 5.1), their
//     u-form, and the synthetic product families, evaluated one point per lane
//     with the coordinates held in registers,
//   * the same integrands over coordinates produced one at a time, for any
//     number of modes (the streaming path of large integrals),
//   * workgroup argmax / max reductions for 64-wide wavefronts.
// All floating-point code is compiled with contraction off; every FMA below is
// written explicitly, so a point gets the same bits in every kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ttcross.h"

namespace ttx {

constexpr int kWave = 64;

// ------------------------------------------------------------ double-double
struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ __forceinline__ dd quick_two_sum(double a, double b) {
  double s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ dd two_prod(double a, double b) {
  double p = a * b;
  return {p, fma(a, b, -p)};
}
__device__ __forceinline__ dd dd_add(dd x, dd y) {
  dd s = two_sum(x.hi, y.hi);
  dd t = two_sum(x.lo, y.lo);
  double e = s.lo + t.hi;
  s = quick_two_sum(s.hi, e);
  e = s.lo + t.lo;
  return quick_two_sum(s.hi, e);
}
__device__ __forceinline__ dd dd_neg(dd x) { return {-x.hi, -x.lo}; }
__device__ __forceinline__ dd dd_sub(dd x, dd y) { return dd_add(x, dd_neg(y)); }
__device__ __forceinline__ dd dd_mul(dd x, dd y) {
  dd p = two_prod(x.hi, y.hi);
  double e = fma(x.hi, y.lo, fma(x.lo, y.hi, p.lo));
  return quick_two_sum(p.hi, e);
}
__device__ __forceinline__ dd dd_mul_d(dd x, double y) {
  dd p = two_prod(x.hi, y);
  double e = fma(x.lo, y, p.lo);
  return quick_two_sum(p.hi, e);
}
__device__ __forceinline__ dd dd_div(dd x, dd y) {
  double q1 = x.hi / y.hi;
  dd r = dd_sub(x, dd_mul_d(y, q1));
  double q2 = r.hi / y.hi;
  r = dd_sub(r, dd_mul_d(y, q2));
  double q3 = r.hi / y.hi;
  dd q = quick_two_sum(q1, q2);
  return dd_add(q, dd{q3, 0.0});
}
__device__ __forceinline__ dd dd_from(double a) { return {a, 0.0}; }

// ------------------------------------------------------------ quad-double
// A value is the unevaluated sum x0 + x1 + x2 + x3 of four doubles of
// decreasing magnitude, about 204 bits.  Every operation writes the exact
// result of its operands' components (their sum, or the exact partial products
// a_i b_j by two_prod) as a list of doubles and rounds that exact sum to four
// components (qd_round).  qd_round first turns the list into a nonoverlapping
// expansion of increasing magnitude by adding one double at a time with
// error-free sums (Grow-Expansion of Shewchuk, Adaptive Precision
// Floating-Point Arithmetic, 1997); the sum of a nonoverlapping expansion taken
// from its smallest component up is within two units in the last place of the
// exact sum, so four rounds of "take that sum as the next component and subtract
// it exactly" leave a remainder below 2^-204 of the value.  The operations are
// out-of-line calls: inlined, each would be thousands of instructions.
struct qd {
  double x0, x1, x2, x3;
};
constexpr int kQdMaxTerms = 27;   // a b + c: 20 two_prod parts, 3 plain products, 4 components of c

__device__ __noinline__ qd qd_round(const double* __restrict__ t, int n) {
  double e[kQdMaxTerms + 4];
  int len = 0;
  for (int i = 0; i < n; ++i) {
    double q = t[i];
    for (int j = 0; j < len; ++j) {
      const dd r = two_sum(q, e[j]);
      q = r.hi;
      e[j] = r.lo;
    }
    e[len++] = q;
  }
  double x[4];
  for (int k = 0; k < 4; ++k) {
    double s = 0.0;
    for (int j = 0; j < len; ++j) s += e[j];
    x[k] = s;
    double q = -s;
    for (int j = 0; j < len; ++j) {
      const dd r = two_sum(q, e[j]);
      q = r.hi;
      e[j] = r.lo;
    }
    e[len++] = q;
  }
  return {x[0], x[1], x[2], x[3]};
}
__device__ __forceinline__ qd qd_from(double a) { return {a, 0.0, 0.0, 0.0}; }
__device__ __forceinline__ qd qd_neg(qd a) { return {-a.x0, -a.x1, -a.x2, -a.x3}; }
__device__ __noinline__ qd qd_add(qd a, qd b) {
  const double t[8] = {a.x0, a.x1, a.x2, a.x3, b.x0, b.x1, b.x2, b.x3};
  return qd_round(t, 8);
}
// s a b + c (s = +1 or -1): the partial products a_i b_j with i + j <= 3 exactly
// (two_prod), those with i + j = 4 rounded once, the rest (below 2^-260 of a b) dropped
__device__ __noinline__ qd qd_fma(qd a, qd b, qd c, double s) {
  const double A[4] = {s * a.x0, s * a.x1, s * a.x2, s * a.x3};
  const double B[4] = {b.x0, b.x1, b.x2, b.x3};
  double t[kQdMaxTerms];
  int n = 0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; i + j <= 3; ++j) {
      const dd p = two_prod(A[i], B[j]);
      t[n++] = p.hi;
      t[n++] = p.lo;
    }
  t[n++] = A[1] * B[3];
  t[n++] = A[2] * B[2];
  t[n++] = A[3] * B[1];
  t[n++] = c.x0;
  t[n++] = c.x1;
  t[n++] = c.x2;
  t[n++] = c.x3;
  return qd_round(t, n);
}
__device__ __forceinline__ qd qd_mul(qd a, qd b) { return qd_fma(a, b, qd_from(0.0), 1.0); }
// c + s b for a double s (exact products of s with b's components)
__device__ __noinline__ qd qd_axpy_d(double s, qd b, qd c) {
  double t[12];
  const double B[4] = {b.x0, b.x1, b.x2, b.x3};
  for (int j = 0; j < 4; ++j) {
    const dd p = two_prod(s, B[j]);
    t[2 * j] = p.hi;
    t[2 * j + 1] = p.lo;
  }
  t[8] = c.x0;
  t[9] = c.x1;
  t[10] = c.x2;
  t[11] = c.x3;
  return qd_round(t, 12);
}
// a / b by long division: five quotient digits q_k = r_k / b_0, r_{k+1} = r_k - q_k b
__device__ __noinline__ qd qd_div(qd a, qd b) {
  double q[5];
  qd r = a;
  for (int k = 0; k < 5; ++k) {
    q[k] = r.x0 / b.x0;
    if (k < 4) r = qd_axpy_d(-q[k], b, r);
  }
  return qd_round(q, 5);
}

// ------------------------------------------------------- working number type
// The TT kernels are written once over the number type T of a job: double, or
// dd for the double-double path.  These overloads are the only arithmetic they
// apply to T values; for double each is the plain operation (n_mad is one FMA).
template <class T> struct is_dd_t { static constexpr bool value = false; };
template <> struct is_dd_t<dd> { static constexpr bool value = true; };
// the extended-precision types (double-double and quad-double)
template <class T> struct is_ext_t { static constexpr bool value = false; };
template <> struct is_ext_t<dd> { static constexpr bool value = true; };
template <> struct is_ext_t<qd> { static constexpr bool value = true; };

template <class T> __device__ __forceinline__ T num(double a);
template <> __device__ __forceinline__ double num<double>(double a) { return a; }
template <> __device__ __forceinline__ dd num<dd>(double a) { return {a, 0.0}; }
template <> __device__ __forceinline__ qd num<qd>(double a) { return qd_from(a); }

__device__ __forceinline__ double n_hi(double a) { return a; }
__device__ __forceinline__ double n_hi(dd a) { return a.hi; }
__device__ __forceinline__ double n_lo(double) { return 0.0; }
__device__ __forceinline__ double n_lo(dd a) { return a.lo; }
__device__ __forceinline__ double n_add(double a, double b) { return a + b; }
__device__ __forceinline__ dd n_add(dd a, dd b) { return dd_add(a, b); }
__device__ __forceinline__ double n_sub(double a, double b) { return a - b; }
__device__ __forceinline__ dd n_sub(dd a, dd b) { return dd_sub(a, b); }
__device__ __forceinline__ double n_mul(double a, double b) { return a * b; }
__device__ __forceinline__ dd n_mul(dd a, dd b) { return dd_mul(a, b); }
__device__ __forceinline__ double n_div(double a, double b) { return a / b; }
__device__ __forceinline__ dd n_div(dd a, dd b) { return dd_div(a, b); }
// a b + c and c - a b
__device__ __forceinline__ double n_mad(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ dd n_mad(dd a, dd b, dd c) { return dd_add(dd_mul(a, b), c); }
__device__ __forceinline__ double n_nmad(double a, double b, double c) { return fma(-a, b, c); }
__device__ __forceinline__ dd n_nmad(dd a, dd b, dd c) { return dd_sub(c, dd_mul(a, b)); }
// exact scaling by 2^e (both parts of a double-double)
__device__ __forceinline__ double n_ldexp(double a, int e) { return ldexp(a, e); }
__device__ __forceinline__ dd n_ldexp(dd a, int e) { return {ldexp(a.hi, e), ldexp(a.lo, e)}; }
__device__ __forceinline__ double n_shfl(double a, int lane) { return __shfl(a, lane, kWave); }
__device__ __forceinline__ dd n_shfl(dd a, int lane) {
  return {__shfl(a.hi, lane, kWave), __shfl(a.lo, lane, kWave)};
}
__device__ __forceinline__ double n_shfl_xor(double a, int off) { return __shfl_xor(a, off, kWave); }
__device__ __forceinline__ dd n_shfl_xor(dd a, int off) {
  return {__shfl_xor(a.hi, off, kWave), __shfl_xor(a.lo, off, kWave)};
}
// quad-double: the leading component is the hi part, the second the lo part
__device__ __forceinline__ double n_hi(qd a) { return a.x0; }
__device__ __forceinline__ double n_lo(qd a) { return a.x1; }
__device__ __forceinline__ qd n_add(qd a, qd b) { return qd_add(a, b); }
__device__ __forceinline__ qd n_sub(qd a, qd b) { return qd_add(a, qd_neg(b)); }
__device__ __forceinline__ qd n_mul(qd a, qd b) { return qd_mul(a, b); }
__device__ __forceinline__ qd n_div(qd a, qd b) { return qd_div(a, b); }
__device__ __forceinline__ qd n_mad(qd a, qd b, qd c) { return qd_fma(a, b, c, 1.0); }
__device__ __forceinline__ qd n_nmad(qd a, qd b, qd c) { return qd_fma(a, b, c, -1.0); }
__device__ __forceinline__ qd n_ldexp(qd a, int e) { return {ldexp(a.x0, e), ldexp(a.x1, e), ldexp(a.x2, e), ldexp(a.x3, e)}; }
__device__ __forceinline__ qd n_shfl(qd a, int lane) {
  return {__shfl(a.x0, lane, kWave), __shfl(a.x1, lane, kWave), __shfl(a.x2, lane, kWave), __shfl(a.x3, lane, kWave)};
}
__device__ __forceinline__ qd n_shfl_xor(qd a, int off) {
  return {__shfl_xor(a.x0, off, kWave), __shfl_xor(a.x1, off, kWave), __shfl_xor(a.x2, off, kWave),
          __shfl_xor(a.x3, off, kWave)};
}

// ---------------------------------------------------------------- SplitMix64
__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// (counter+1)-th output of the stream whose state starts at `seed`.
__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t counter) {
  return splitmix_mix(seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull);
}
// uniform integer in [0, n), n < 2^32, from the high 32 bits of a draw
__device__ __forceinline__ uint32_t uniform_below(uint64_t u, uint32_t n) {
  return (uint32_t)(((u >> 32) * (uint64_t)n) >> 32);
}
__device__ __forceinline__ uint64_t sample_counter(int sweep, int bond, int j) {
  return ((uint64_t)sweep << 40) + ((uint64_t)bond << 24) + (uint64_t)j;
}
__device__ __forceinline__ uint64_t start_counter(int q, int k) {
  return (1ull << 63) + ((uint64_t)q << 16) + (uint64_t)k;
}
// Monte Carlo point i of estimator j (m coordinates), and the lattice shifts
__device__ __forceinline__ uint64_t mc_counter(int j, int64_t i, int m, int k) {
  return (1ull << 62) + ((uint64_t)j << 40) + (uint64_t)i * (uint64_t)m + (uint64_t)k;
}
__device__ __forceinline__ uint64_t shift_counter(int j, int k) {
  return (1ull << 62) + (1ull << 61) + ((uint64_t)j << 6) + (uint64_t)k;
}
// a draw mapped to (0, 1): the top 53 bits, centred in their cell
__device__ __forceinline__ double uniform_open01(uint64_t u) {
  return ((double)(u >> 11) + 0.5) * 0x1.0p-53;
}

// ---------------------------------------------------------------- integrands
// y[0..m) holds the coordinates of one point (entries >= m are ignored).
// Returns the unweighted integrand f(y) including its constant prefactor.

// Paper form, y_k = x_{k+2} (k = 0..m-1).  Every run y_a..y_b (a <= b), i.e.
// every pair 1 <= i < j <= d with its product x_{i+1}..x_j, is visited once, in
// the order of its last index b: after step b, z[a] holds y_a..y_b for a <= b
// (the products are kept in place of the coordinates, so no extra registers).
//   A_d: pn = prod (1 - y_a..y_b), pd = prod (1 + y_a..y_b), A_d = (pn/pd)^2;
//   prefix sum q = sum_b y_0..y_b (the run starting at a = 0 after each step);
//   suffix sum s = sum_a y_a..y_{m-1} (all runs after the last step);
//   B_d = 1 / ((1 + q)(1 + s)).
// One uniform guard per b: modes beyond m are skipped in one branch each.
template <class T, int MAXM>
__device__ __forceinline__ T ising_paper(int family, int m, const T (&y)[MAXM]) {
  const T zero = num<T>(0.0), one = num<T>(1.0);
  T z[MAXM];
#pragma unroll
  for (int k = 0; k < MAXM; ++k) z[k] = (k < m) ? y[k] : zero;
  const bool need_a = family != TT_ISING_C;
  T pn = one, pd = one, q = zero;
#pragma unroll
  for (int b = 0; b < MAXM; ++b) {
    if (b < m) {
      const T yb = z[b];
#pragma unroll
      for (int a = 0; a < b; ++a) z[a] = n_mul(z[a], yb);   // z[a] = y_a..y_b
      q = n_add(q, z[0]);
      if (need_a) {
#pragma unroll
        for (int a = 0; a <= b; ++a) {
          pn = n_nmad(pn, z[a], pn);                          // pn * (1 - y_a..y_b)
          pd = n_mad(pd, z[a], pd);                           // pd * (1 + y_a..y_b)
        }
      }
    }
  }
  T nm = num<T>(2.0), den = one;
  if (family != TT_ISING_E) {
    T s = zero;
#pragma unroll
    for (int a = 0; a < MAXM; ++a) s = n_add(s, z[a]);      // zero beyond m
    den = n_mul(n_add(one, q), n_add(one, s));
  }
  if (need_a) {
    if (m <= 31) {               // pd^2 <= 2^(m(m+1)) stays finite
      nm = n_mul(n_mul(nm, pn), pn);
      den = n_mul(den, n_mul(pd, pd));
    } else {
      const T r = n_div(pn, pd);
      nm = n_mul(n_mul(nm, r), r);
    }
  }
  return n_div(nm, den);
}

// u-form, d = m variables x_j with u_j = x_j/(1-x_j):
//   f = 4/d! [sum_j (u_j + 1/u_j)]^-2 prod_j 1/(x_j(1-x_j)) [* prod_{i<j} ((u_i-u_j)/(u_i+u_j))^2]
// With h_j = x_j(1-x_j), g_j = x_j^2 + (1-x_j)^2: u_j + 1/u_j = g_j/h_j, so
// f = (4/d!) H / G^2 with H = prod h_j and G = sum_j g_j prod_{i != j} h_i;
// (u_i-u_j)/(u_i+u_j) = (x_i-x_j)/(x_i+x_j-2 x_i x_j).
template <int MAXM>
__device__ __forceinline__ double ising_u(int family, int m, const double (&y)[MAXM],
                                          double four_over_mfact) {
  double G = 0.0, H = 1.0;
#pragma unroll
  for (int k = 0; k < MAXM; ++k) {
    if (k < m) {
      double x = y[k], omx = 1.0 - x;
      double h = x * omx;
      double g = fma(x, x, omx * omx);
      G = fma(G, h, g * H);
      H = H * h;
    }
  }
  double f = four_over_mfact * H / (G * G);
  if (family == TT_ISING_D_U) {
    // prod ((x_i-x_j)/(x_i+x_j-2x_i x_j))^2 as a ratio of two products, brought
    // back to [1,2) by an exact power-of-two scaling after every row
    double pn = 1.0, pd = 1.0;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (i < m) {
#pragma unroll
        for (int j = i + 1; j < MAXM; ++j) {
          if (j < m) {
            const double dn = y[i] - y[j];
            const double dd_ = fma(-2.0 * y[i], y[j], y[i] + y[j]);
            pn = pn * (dn * dn);
            pd = pd * (dd_ * dd_);
          }
        }
        const int e = ilogb(pd);
        pn = ldexp(pn, -e);
        pd = ldexp(pd, -e);
      }
    }
    f = f * (pn / pd);
  }
  return f;
}

template <int MAXM>
__device__ __forceinline__ double synthetic(int family, int m, const double (&y)[MAXM],
                                            const double* __restrict__ a,
                                            const double* __restrict__ b) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < MAXM; ++k)
    if (k < m) s = fma(a[k], y[k], s);
  double e = exp(-s);
  if (family == TT_PROD_EXP) return e;
  double c = 1.0;
#pragma unroll
  for (int k = 0; k < MAXM; ++k)
    if (k < m) c = c * cos(b[k] * y[k]);
  return e + c;
}

struct FamilyArgs {
  int family, m;
  double four_over_mfact;    // u-form prefactor 4/m!
  const double* a;           // synthetic parameters (device)
  const double* b;
  int escale = 0;            // streaming integrands return f times 2^escale
};

template <int MAXM>
__device__ __forceinline__ double integrand(const FamilyArgs& fa, const double (&y)[MAXM]) {
  switch (fa.family) {
    case TT_ISING_C:
    case TT_ISING_D:
    case TT_ISING_E:
      return ising_paper<double, MAXM>(fa.family, fa.m, y);
    case TT_ISING_C_U:
    case TT_ISING_D_U:
      return ising_u<MAXM>(fa.family, fa.m, y, fa.four_over_mfact);
    default:
      return synthetic<MAXM>(fa.family, fa.m, y, fa.a, fa.b);
  }
}

// ------------------------------------------------------ streaming integrands
// Any number of modes: the coordinates come from an accessor y(k) (one load per
// use, from the index-set rows in memory) instead of registers.
//
// Paper form.  B_d in one forward pass: the prefix sum q = sum_b y_0..y_b and
// the suffix sum s = sum_a y_a..y_{m-1} by the recurrence s <- y_k (1 + s).
// A_d over the runs y_a..y_b by their first index a; a run is left as soon as
// its product p falls below 2^-54, since from there on p only decreases and
// pn (1 - p), pd (1 + p) round back to pn and pd (the FMA's exact product is
// below half an ulp), so stopping changes no bit.  pn and pd are each brought
// back near 1 by an exact power of two every 32 factors and after every run, and
// the difference x of the two exponents taken out is kept: the value is
// (2 (pn/pd)^2 / den) 2^(2x), returned as that mantissa with *ex = 2x.  Far
// below the double range (D_d near 10^(-0.7 d), Sec. 5.5) the mantissa stays
// exact; where nothing leaves the range the result equals the one-scale
// evaluation bit for bit, since every scaling is by a power of two.
__device__ __forceinline__ void pair_renorm(double& pn, double& pd, int& x) {
  const int en = ilogb(pn), ed = ilogb(pd);
  pn = ldexp(pn, -en);
  pd = ldexp(pd, -ed);
  x += en - ed;
}

template <class Y>
__device__ __forceinline__ double ising_paper_stream_me(int family, int m, const Y& y, int* ex) {
  double den = 1.0;
  if (family != TT_ISING_E) {
    double P = 1.0, q = 0.0, s = 0.0;
    for (int k = 0; k < m; ++k) {
      const double yk = y(k);
      P = P * yk;
      q = q + P;
      s = fma(yk, s, yk);
    }
    den = (1.0 + q) * (1.0 + s);
  }
  double nm = 2.0;
  int x = 0;
  if (family != TT_ISING_C) {
    double pn = 1.0, pd = 1.0;
    for (int a = 0; a < m; ++a) {
      double p = 1.0;
      for (int b = a; b < m; ++b) {
        p = p * y(b);
        if (p < 0x1.0p-54) break;
        pn = fma(-pn, p, pn);
        pd = fma(pd, p, pd);
        if (((b - a) & 31) == 31) pair_renorm(pn, pd, x);
      }
      pair_renorm(pn, pd, x);
    }
    const double r = pn / pd;
    nm = nm * r * r;
  }
  *ex = 2 * x;
  return nm / den;
}

template <class Y>
__device__ __forceinline__ double ising_paper_stream(int family, int m, const Y& y, int escale) {
  int ex;
  const double v = ising_paper_stream_me(family, m, y, &ex);
  return ldexp(v, ex + escale);
}

template <class Y>
__device__ __forceinline__ double synthetic_stream(int family, int m, const Y& y, const double* __restrict__ a,
                                                   const double* __restrict__ b) {
  double s = 0.0;
  for (int k = 0; k < m; ++k) s = fma(a[k], y(k), s);
  const double e = exp(-s);
  if (family == TT_PROD_EXP) return e;
  double c = 1.0;
  for (int k = 0; k < m; ++k) c = c * cos(b[k] * y(k));
  return e + c;
}

// The coordinates of a fibre point in the sweep kernels: the row of a left set
// (y_0..y_{nL-1}), one or two nodes, and the row of a right set (y_{nL+nM}..y_{m-1},
// indexed by the absolute coordinate).  Loops over the two rows are contiguous,
// so their loads issue several at a time instead of one per iteration.
struct Segs {
  const double* L;
  int nL;
  double mid0, mid1;
  int nM;          // 1 or 2 nodes
  const double* R;
  int m;
};

template <class F>
__device__ __forceinline__ void seg_each(const Segs& s, F&& f) {
#pragma unroll 4
  for (int k = 0; k < s.nL; ++k) f(k, s.L[k]);
  f(s.nL, s.mid0);
  if (s.nM > 1) f(s.nL + 1, s.mid1);
#pragma unroll 4
  for (int k = s.nL + s.nM; k < s.m; ++k) f(k, s.R[k]);
}

// Products of the runs y_a..y_b of A_d from a given a, in chunks of four factors:
// the exit test on p < 2^-54 is taken after each chunk, which changes no bit, since
// the factors after the first such p leave pn and pd unchanged (see above).
struct PairRun {
  double pn, pd, p;
  int x;   // pn / pd is the pair product times 2^-x (see ising_paper_stream_me)
  __device__ __forceinline__ void step(double y) {
    p = p * y;
    pn = fma(-pn, p, pn);
    pd = fma(pd, p, pd);
  }
  __device__ __forceinline__ bool done() const { return p < 0x1.0p-54; }
  __device__ __forceinline__ void renorm() { pair_renorm(pn, pd, x); }
  // factors ptr[k0..k1); returns true once the run is over
  __device__ __forceinline__ bool span(const double* __restrict__ ptr, int k0, int k1) {
    int k = k0;
    for (; k + 4 <= k1; k += 4) {
      const double y0 = ptr[k], y1 = ptr[k + 1], y2 = ptr[k + 2], y3 = ptr[k + 3];
      step(y0);
      step(y1);
      step(y2);
      step(y3);
      if (done()) return true;
      if (((k - k0) & 28) == 28) renorm();   // every 32 factors
    }
    for (; k < k1; ++k) {
      step(ptr[k]);
      if (done()) return true;
    }
    renorm();
    return false;
  }
};

// B_d's prefix sum q = sum_b y_0..y_b and suffix recurrence s <- y (1 + s) over a
// point, four coordinates at a time: a block of four is summarised on its own
// (its product p4, its prefix sum q4 and its recurrence value g4 from s = 0),
// then q <- q + P q4, s <- g4 + p4 s, P <- P p4.  The three running chains take
// one operation per block, so the blocks' own work overlaps.
struct PrefixSuffix {
  double P = 1.0, q = 0.0, s = 0.0;
  __device__ __forceinline__ void one(double y) {
    P = P * y;
    q = q + P;
    s = fma(y, s, y);
  }
  __device__ __forceinline__ void four(double y0, double y1, double y2, double y3) {
    const double p01 = y0 * y1, p012 = p01 * y2, p4 = p012 * y3;
    const double q4 = (y0 + p01) + (p012 + p4);
    double g4 = y0;
    g4 = fma(y1, g4, y1);
    g4 = fma(y2, g4, y2);
    g4 = fma(y3, g4, y3);
    q = fma(P, q4, q);
    s = fma(p4, s, g4);
    P = P * p4;
  }
  __device__ __forceinline__ void span(const double* __restrict__ ptr, int k0, int k1) {
    int k = k0;
    for (; k + 4 <= k1; k += 4) four(ptr[k], ptr[k + 1], ptr[k + 2], ptr[k + 3]);
    for (; k < k1; ++k) one(ptr[k]);
  }
};

__device__ __forceinline__ double ising_paper_seg(int family, const Segs& s, int escale) {
  const int m = s.m;
  double den = 1.0;
  if (family != TT_ISING_E) {
    PrefixSuffix ps;
    ps.span(s.L, 0, s.nL);
    ps.one(s.mid0);
    if (s.nM > 1) ps.one(s.mid1);
    ps.span(s.R, s.nL + s.nM, m);
    den = (1.0 + ps.q) * (1.0 + ps.s);
  }
  double nm = 2.0;
  int ex = 0;
  if (family != TT_ISING_C) {
    PairRun run{1.0, 1.0, 1.0, 0};
    const int mid = s.nL, right = s.nL + s.nM;
    for (int a = 0; a < m; ++a) {
      run.p = 1.0;
      bool over = false;
      if (a < mid) over = run.span(s.L, a, mid);
      if (!over && a <= mid) {
        run.step(s.mid0);
        over = run.done();
      }
      if (!over && s.nM > 1 && a <= mid + 1) {
        run.step(s.mid1);
        over = run.done();
      }
      if (!over) run.span(s.R, a > right ? a : right, m);
      run.renorm();
    }
    const double r = run.pn / run.pd;
    nm = nm * r * r;
    ex = 2 * run.x;
  }
  return ldexp(nm / den, ex + escale);
}

__device__ __forceinline__ double synthetic_seg(int family, const Segs& s, const double* __restrict__ a,
                                                const double* __restrict__ b) {
  double sum = 0.0;
  seg_each(s, [&](int k, double yk) { sum = fma(a[k], yk, sum); });
  const double e = exp(-sum);
  if (family == TT_PROD_EXP) return e;
  double c = 1.0;
  seg_each(s, [&](int k, double yk) { c = c * cos(b[k] * yk); });
  return e + c;
}

// ------------------------------------------ paper form from row summaries
// Points that share a left index-set row (coordinates y_0..y_{p-1}) and a right
// one (y_o..y_{m-1}, o = p + nM) around nM = 1 or 2 nodes: every run y_a..y_b of
// A_d lies inside the left row, inside the right row, or contains a node.  The
// runs inside a row, and B_d's sums over its coordinates, are the same for every
// point with that row, so they are formed once per row; a point multiplies only
// the runs through its nodes, (p + 1)(m - p) of them for one node instead of
// m(m + 1)/2.  The integral is unchanged; the rounding differs from the one-pass
// evaluation only in how each run's product is associated.
//
// A row summary: MAXM run products, then kSumScalars scalars:
//   run[k]  left row: y_k..y_{p-1} (k < p);  right row: y_o..y_k (o <= k < m)
//   an, ad  prod over the runs inside the row of (1 - run) and (1 + run)
//   q       left: sum_{b<p} y_0..y_b;   right: sum_{b>=o} y_o..y_b
//   P       product of the row's coordinates (1 for an empty row)
//   S       left: sum_{a<p} y_a..y_{p-1};   right: sum_{a>=o} y_a..y_{m-1}
//   W       product of the row's weights
constexpr int kSumScalars = 6;
enum { RS_AN = 0, RS_AD = 1, RS_Q = 2, RS_P = 3, RS_S = 4, RS_W = 5 };

// Summary of coordinates y[k0..k1) (y indexed by absolute coordinate) into out,
// as a left row (run[k] = suffix products) or a right row (run[k] = prefix
// products).  One thread per row.
template <class T, int MAXM>
__device__ __forceinline__ void summarise_row(int family, const T (&y)[MAXM], int k0, int k1, bool left, T w,
                                              T* __restrict__ out) {
  const T zero = num<T>(0.0), one = num<T>(1.0);
  const bool need_a = family != TT_ISING_C;
  T z[MAXM];
#pragma unroll
  for (int k = 0; k < MAXM; ++k) z[k] = (k >= k0 && k < k1) ? y[k] : zero;
  T an = one, ad = one, q = zero, pre = one;
#pragma unroll
  for (int b = 0; b < MAXM; ++b) {
    if (b >= k0 && b < k1) {
      const T yb = z[b];
#pragma unroll
      for (int a = 0; a < b; ++a)
        if (a >= k0) z[a] = n_mul(z[a], yb);            // z[a] = y_a..y_b
      pre = n_mul(pre, yb);                              // y_k0..y_b, as z[k0]
      q = n_add(q, pre);
      if (!left) out[b] = pre;
      if (need_a) {
#pragma unroll
        for (int a = 0; a <= b; ++a)
          if (a >= k0) {
            an = n_nmad(an, z[a], an);
            ad = n_mad(ad, z[a], ad);
          }
      }
    }
  }
  T S = zero;
#pragma unroll
  for (int a = 0; a < MAXM; ++a) {
    if (a >= k0 && a < k1) {
      S = n_add(S, z[a]);
      if (left) out[a] = z[a];                           // suffix product y_a..y_{p-1}
    }
  }
  out[MAXM + RS_AN] = an;
  out[MAXM + RS_AD] = ad;
  out[MAXM + RS_Q] = q;
  out[MAXM + RS_P] = pre;
  out[MAXM + RS_S] = S;
  out[MAXM + RS_W] = w;
}

// A left and a right row summary held in registers for the points that share
// them: the left row's suffix products y_a..y_{p-1} (a < p), the right row's
// prefix products y_o..y_{o+j} (j < nr = m - o), and the scalars of both.
template <class T, int MAXM>
struct RowPair {
  T lsuf[MAXM], rpre[MAXM];
  T an, ad, Lq, LP, LS, Rq, RP, Rs;
};

template <class T, int MAXM>
__device__ __forceinline__ void load_row_pair(RowPair<T, MAXM>& rp, const T* __restrict__ L,
                                              const T* __restrict__ R, int p, int o, int nr) {
#pragma unroll
  for (int a = 0; a < MAXM; ++a) rp.lsuf[a] = L[a < p ? a : 0];
#pragma unroll
  for (int j = 0; j < MAXM; ++j) rp.rpre[j] = R[o + (j < nr ? j : 0)];
  rp.an = n_mul(L[MAXM + RS_AN], R[MAXM + RS_AN]);
  rp.ad = n_mul(L[MAXM + RS_AD], R[MAXM + RS_AD]);
  rp.Lq = L[MAXM + RS_Q];
  rp.LP = L[MAXM + RS_P];
  rp.LS = L[MAXM + RS_S];
  rp.Rq = R[MAXM + RS_Q];
  rp.RP = R[MAXM + RS_P];
  rp.Rs = R[MAXM + RS_S];
}

// The paper-form integrand (factor 2 included) at a point joined from a row pair
// (left coordinates 0..p-1, right coordinates o..m-1, o = p + nM) and nM = 1 or
// 2 nodes t0, t1 at coordinates p, p+1.  Every run through a node is
// (y_a..y_{p-1}) t0 [t1] (y_o..y_b); the loops are unrolled over the mode bound
// with wave-uniform guards, so every product is read from registers.
template <class T, int MAXM>
__device__ __forceinline__ T ising_joined(int family, int m, int p, int nM, const RowPair<T, MAXM>& rp, T t0, T t1) {
  const T one = num<T>(1.0);
  const int nr = m - p - nM;
  T nm = num<T>(2.0), den = one;
  if (family != TT_ISING_E) {   // B_d: q and s joined around the nodes
    T q, sfx;
    if (nM == 2) {
      q = n_mad(n_mul(rp.LP, t0), n_mad(t1, n_add(one, rp.Rq), one), rp.Lq);
      sfx = n_mad(n_mul(t1, rp.RP), n_mad(t0, n_add(one, rp.LS), one), rp.Rs);
    } else {
      q = n_mad(n_mul(rp.LP, t0), n_add(one, rp.Rq), rp.Lq);
      sfx = n_mad(n_mul(t0, rp.RP), n_add(one, rp.LS), rp.Rs);
    }
    den = n_mul(n_add(one, q), n_add(one, sfx));
  }
  if (family != TT_ISING_C) {   // A_d: the runs inside the rows, then the runs through the nodes
    T pn = rp.an, pd = rp.ad;
#pragma unroll
    for (int a = 0; a < MAXM; ++a) {          // runs from coordinate a <= p through the first node
      if (a <= p) {
        T u = (a < p) ? n_mul(rp.lsuf[a], t0) : t0;
        pn = n_nmad(pn, u, pn);
        pd = n_mad(pd, u, pd);
        if (nM == 2) {
          u = n_mul(u, t1);
          pn = n_nmad(pn, u, pn);
          pd = n_mad(pd, u, pd);
        }
#pragma unroll
        for (int j = 0; j < MAXM; ++j) {
          if (j < nr) {
            const T v = n_mul(u, rp.rpre[j]);
            pn = n_nmad(pn, v, pn);
            pd = n_mad(pd, v, pd);
          }
        }
      }
    }
    if (nM == 2) {                            // runs from the second node
      pn = n_nmad(pn, t1, pn);
      pd = n_mad(pd, t1, pd);
#pragma unroll
      for (int j = 0; j < MAXM; ++j) {
        if (j < nr) {
          const T v = n_mul(t1, rp.rpre[j]);
          pn = n_nmad(pn, v, pn);
          pd = n_mad(pd, v, pd);
        }
      }
    }
    if (m <= 31) {                            // pd^2 <= 2^(m(m+1)) stays finite
      nm = n_mul(n_mul(nm, pn), pn);
      den = n_mul(den, n_mul(pd, pd));
    } else {
      const T r = n_div(pn, pd);
      nm = n_mul(n_mul(nm, r), r);
    }
  }
  return n_div(nm, den);
}

// Two points of one row pair at nodes ta and tb (one node each, nM = 1): the
// same operations as ising_joined for each, with the two points' products
// interleaved so that four independent chains are in flight.
template <class T, int MAXM>
__device__ __forceinline__ void ising_joined2(int family, int m, int p, const RowPair<T, MAXM>& rp, T ta, T tb,
                                              T& fa, T& fb) {
  const T one = num<T>(1.0);
  const int nr = m - p - 1;
  T nma = num<T>(2.0), nmb = num<T>(2.0), dena = one, denb = one;
  if (family != TT_ISING_E) {
    const T rq1 = n_add(one, rp.Rq), ls1 = n_add(one, rp.LS);
    const T qa = n_mad(n_mul(rp.LP, ta), rq1, rp.Lq), qb = n_mad(n_mul(rp.LP, tb), rq1, rp.Lq);
    const T sa = n_mad(n_mul(ta, rp.RP), ls1, rp.Rs), sb = n_mad(n_mul(tb, rp.RP), ls1, rp.Rs);
    dena = n_mul(n_add(one, qa), n_add(one, sa));
    denb = n_mul(n_add(one, qb), n_add(one, sb));
  }
  if (family != TT_ISING_C) {
    T pna = rp.an, pda = rp.ad, pnb = rp.an, pdb = rp.ad;
#pragma unroll
    for (int a = 0; a < MAXM; ++a) {
      if (a <= p) {
        const T ua = (a < p) ? n_mul(rp.lsuf[a], ta) : ta;
        const T ub = (a < p) ? n_mul(rp.lsuf[a], tb) : tb;
        pna = n_nmad(pna, ua, pna);
        pda = n_mad(pda, ua, pda);
        pnb = n_nmad(pnb, ub, pnb);
        pdb = n_mad(pdb, ub, pdb);
#pragma unroll
        for (int j = 0; j < MAXM; ++j) {
          if (j < nr) {
            const T va = n_mul(ua, rp.rpre[j]), vb = n_mul(ub, rp.rpre[j]);
            pna = n_nmad(pna, va, pna);
            pda = n_mad(pda, va, pda);
            pnb = n_nmad(pnb, vb, pnb);
            pdb = n_mad(pdb, vb, pdb);
          }
        }
      }
    }
    if (m <= 31) {
      nma = n_mul(n_mul(nma, pna), pna);
      dena = n_mul(dena, n_mul(pda, pda));
      nmb = n_mul(n_mul(nmb, pnb), pnb);
      denb = n_mul(denb, n_mul(pdb, pdb));
    } else {
      const T ra = n_div(pna, pda), rb = n_div(pnb, pdb);
      nma = n_mul(n_mul(nma, ra), ra);
      nmb = n_mul(n_mul(nmb, rb), rb);
    }
  }
  fa = n_div(nma, dena);
  fb = n_div(nmb, denb);
}

// ising_joined2 for a mode count M and a node position P known at compile time:
// every loop bound is a constant, so the runs through the node are straight-line
// code (the same operations in the same order as ising_joined2, hence the same
// bits).
template <class T, int M, int P>
__device__ __forceinline__ void ising_joined2_fixed(int family, const RowPair<T, M>& rp, T ta, T tb, T& fa, T& fb) {
  constexpr int NR = M - P - 1;
  const T one = num<T>(1.0);
  T nma = num<T>(2.0), nmb = num<T>(2.0), dena = one, denb = one;
  if (family != TT_ISING_E) {
    const T rq1 = n_add(one, rp.Rq), ls1 = n_add(one, rp.LS);
    const T qa = n_mad(n_mul(rp.LP, ta), rq1, rp.Lq), qb = n_mad(n_mul(rp.LP, tb), rq1, rp.Lq);
    const T sa = n_mad(n_mul(ta, rp.RP), ls1, rp.Rs), sb = n_mad(n_mul(tb, rp.RP), ls1, rp.Rs);
    dena = n_mul(n_add(one, qa), n_add(one, sa));
    denb = n_mul(n_add(one, qb), n_add(one, sb));
  }
  if (family != TT_ISING_C) {
    T pna = rp.an, pda = rp.ad, pnb = rp.an, pdb = rp.ad;
#pragma unroll
    for (int a = 0; a <= P; ++a) {
      const T ua = (a < P) ? n_mul(rp.lsuf[a], ta) : ta;
      const T ub = (a < P) ? n_mul(rp.lsuf[a], tb) : tb;
      pna = n_nmad(pna, ua, pna);
      pda = n_mad(pda, ua, pda);
      pnb = n_nmad(pnb, ub, pnb);
      pdb = n_mad(pdb, ub, pdb);
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        const T va = n_mul(ua, rp.rpre[j]), vb = n_mul(ub, rp.rpre[j]);
        pna = n_nmad(pna, va, pna);
        pda = n_mad(pda, va, pda);
        pnb = n_nmad(pnb, vb, pnb);
        pdb = n_mad(pdb, vb, pdb);
      }
    }
    if (M <= 31) {
      nma = n_mul(n_mul(nma, pna), pna);
      dena = n_mul(dena, n_mul(pda, pda));
      nmb = n_mul(n_mul(nmb, pnb), pnb);
      denb = n_mul(denb, n_mul(pdb, pdb));
    } else {
      const T ra = n_div(pna, pda), rb = n_div(pnb, pdb);
      nma = n_mul(n_mul(nma, ra), ra);
      nmb = n_mul(n_mul(nmb, rb), rb);
    }
  }
  fa = n_div(nma, dena);
  fb = n_div(nmb, denb);
}

// --------------------------------------------------------------- reductions
// argmax of |e| with ties to the lowest index; NaN never wins (comparisons are false).
struct ArgMax {
  double v;   // |e| (or -1 for "nothing")
  int idx;
};
__device__ __forceinline__ bool better(double v, int i, double bv, int bi) {
  return v > bv || (v == bv && i < bi);
}
__device__ __forceinline__ ArgMax wave_argmax(ArgMax a) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    double ov = __shfl_xor(a.v, off, kWave);
    int oi = __shfl_xor(a.idx, off, kWave);
    if (better(ov, oi, a.v, a.idx)) { a.v = ov; a.idx = oi; }
  }
  return a;
}
// Block-wide argmax; every thread receives the result.  scratch: >= 2*nwaves slots.
__device__ __forceinline__ ArgMax block_argmax(ArgMax a, double* sv, int* si) {
  a = wave_argmax(a);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  __syncthreads();
  if (lane == 0) { sv[wid] = a.v; si[wid] = a.idx; }
  __syncthreads();
  ArgMax r{-1.0, 0x7fffffff};
  for (int w = 0; w < nw; ++w)
    if (better(sv[w], si[w], r.v, r.idx)) { r.v = sv[w]; r.idx = si[w]; }
  __syncthreads();
  return r;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}
__device__ __forceinline__ double block_max(double v, double* sv) {
  v = wave_max(v);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  __syncthreads();
  if (lane == 0) sv[wid] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < nw; ++w) r = fmax(r, sv[w]);
  __syncthreads();
  return r;
}

}  // namespace ttx
