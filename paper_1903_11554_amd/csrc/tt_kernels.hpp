// HIP kernels of the TT cross library (gfx950, wave64).
//
// One sweep of Alg. 6 (dimension-parallel greedy cross, Sec. 3.4) over every
// integral of a job is one launch of k_sweep, one workgroup per superblock,
// running three phases that are handed over without any waiting (see k_sweep):
//   search    Alg. 2 on the (r_{b-1} n) x (n r_{b+1}) matrix
//             B(I_<=b-1 i_b, i_b+1 I_>b+1) with the previous sweep's sets:
//             random samples, then column / row steps until the rook condition
//             (eq. rook) holds; the approximation is B~ = C_b F_{b+1} with the
//             interpolation core C_b = F_b M_b^-1 (Alg. 1's matrix B);
//   update    per core c, run by the last of its two neighbouring superblocks:
//             appends the accepted pivots of bonds c-1 and c to I_<=c-1 and
//             I_>c (nestedness, eq. nest), evaluates the new fibre entries of
//             F_c = B(I_<=c-1, i_c, I_>c), and brings C_c up to date: new rows
//             are solved with the stored LU of the cross M_c = B(I_<=c, I_>c),
//             the new column enters by the exact rank-1 (Schur complement)
//             update of C_c, and the LU of M_c grows by one bordered row and
//             column; then sums the core over its mode index for the quadrature;
//   integral  per integral, run by the last core update: commits the ranks,
//             multiplies the 2m-1 matrices of the TT quadrature (Sec. 4.1) and
//             applies the stopping rule.
// Kernels are specialised by integrand class, so each carries one integrand,
// and templated on the number type T of the job (double, or dd for the
// double-double path): the arrays marked "T" below hold T values.
#pragma once

#include "tt_device.hpp"

namespace ttx {

struct PivRec {
  int32_t row, col, acc, iters;
  double err, val;
  int32_t col_fresh, pad;   // the last column step was at the final column
};
static_assert(sizeof(PivRec) == sizeof(tt_pivot), "PivRec must mirror tt_pivot");

// One record of a clustered search's exchange: a member's best |error| v at point
// idx with its error e and value a (argmax steps; e and a in the job's number
// type), or its largest |B| seen in v and its non-finite flag in idx (the closing
// step).  Each 64-bit word holds 32 bits of the record and, above them, the tag of
// the sweep and step it belongs to, and is written and read as one atomic: a
// reader that sees the tag in every word holds the whole record of that step,
// with no fence (a word is new or old as a whole).  Words: v (2), idx (1), then
// the doubles of e and of a (2 each): 7 for double, 11 for double-double, 19 for
// quad-double.
constexpr int kXWords = 3 + 4 * (int)(sizeof(qd) / sizeof(double));
struct XSlot {
  uint64_t w[kXWords + 1];
};
constexpr int kMaxGroup = 8;   // workgroups per superblock at most
template <class T>
struct XRec {                  // an exchange record unpacked
  double v;
  T e, a;
  int idx;
};

// The integral is value_mant * 2^vexp (with value_lo the low part of the
// mantissa for double-double jobs), 1/2 <= |value| < 1 or value = 0.
struct ProbState {
  int32_t sweeps, done, reason, err_flags;
  int32_t nacc, max_rank, vexp, recomputes;   // recomputes: interpolation cores rebuilt from F_c
  int32_t escale, pad0;                       // streaming path: every B is f W 2^escale
  unsigned long long evals;
  double value, rel, value_lo;
};

struct ProbDesc {
  int32_t family, m, n, R;
  int32_t max_sweeps, nbonds, wshift;   // weights w are the rule's times 2^wshift
  int32_t strict;                       // TT_STOP_STRICT: no stop on the relative change alone
  double tol, four_over_mfact;
  uint64_t seed;
  const double *t, *w;                   // T: nodes and weights
  const double *pa, *pb;                 // synthetic parameters
  int32_t *Lpar, *Lnode, *Rpar, *Rnode;  // [nbonds][R]
  double *Lx, *Rx;                       // T [nbonds][R][m]
  double *Lw, *Rw;                       // T [nbonds][R]
  double *F;                             // T cores, core c at F + Foff[c] (in T elements)
  int64_t *Foff;
  double *C;                             // T interpolation cores (transposed), bond b at C + Coff[b]
  int64_t *Coff;
  double *LU;                            // T [nbonds][R*R] LU of M_b in insertion order (no pivoting)
  double *S;                             // T [m][R*R] core sums over the mode index
  int32_t *rank;                         // [nbonds]
  PivRec *piv;                           // [nbonds] current sweep's pivots
  double *scale;                         // [nbonds] largest |B| seen per bond
  PivRec *log;                           // [max_sweeps][nbonds]
  double *hist;                          // T [max_sweeps+1] mantissas of the integral after each sweep
  int32_t *hexp;                         // [max_sweeps+1] their exponents
  int32_t *start;                        // [m] start multi-index
  int32_t *sync;                         // [m+1] per-sweep dataflow counters (cores ready, cores done)
  int32_t *rfl;                          // [m] 1: core c's interpolation core is recomputed every sweep
  int32_t *done_host;                    // pinned host flag mirrored when the integral stops (may be null)
  ProbState *st_host;                    // pinned host copy of the final state (may be null)
  long long *phase;                      // [max_sweeps][nbonds + m][kPhases] wall-clock marks, or null
  XSlot *xch;                            // [nbonds][2][kMaxGroup] exchange records of clustered searches
  ProbState *st;
};

// Phase marks of the sweep kernel's workgroups in one sweep (wall clock, written by
// thread 0), one row per superblock b, then one row per core c (row nbonds + c).
// Superblock rows: 0 start, 1 sets staged, 2 samples done, 3 rook pivoting done,
// 4 search done, 7 end.  Core rows: 0 start, 8 both neighbouring searches seen,
// 9 pivots appended and sets staged, 10 new entries evaluated, 11 new rows solved,
// 12 cross LU bordered, 13 rank-1 update done, 14 core summed, 5 update done,
// 6 quadrature done (the integral's last core), 7 end.
constexpr int kPhases = 16;
__device__ __forceinline__ void mark(const ProbDesc& p, int sweep, int row, int slot) {
  if (p.phase != nullptr && threadIdx.x == 0)
    p.phase[((size_t)sweep * (p.nbonds + p.m) + row) * kPhases + slot] = (long long)wall_clock64();
}
// Superblock rows also carry durations (ticks, summed over the search's steps):
// 8, 9, 10 the samples' point loop, block argmax and exchange; 11, 12, 13 the same
// over the rook steps; 14 the rook steps' set-up (the fixed fibre's B~ operand).
__device__ __forceinline__ void mark_value(const ProbDesc& p, int sweep, int row, int slot, long long v) {
  if (p.phase != nullptr && threadIdx.x == 0) p.phase[((size_t)sweep * (p.nbonds + p.m) + row) * kPhases + slot] = v;
}

// Mirror "this integral has stopped" into pinned host memory so the host can
// stop queueing sweeps (and read the result) without copying device state
// back: the final state first, then a system-scope fence, then the flag.
// Called by one thread, after every field of the state has its final value.
__device__ __forceinline__ void signal_done(const ProbDesc& p) {
  if (p.st_host) {
    const volatile ProbState* src = p.st;
    volatile ProbState* dst = p.st_host;
    dst->sweeps = src->sweeps;
    dst->done = src->done;
    dst->reason = src->reason;
    dst->err_flags = src->err_flags;
    dst->nacc = src->nacc;
    dst->max_rank = src->max_rank;
    dst->vexp = src->vexp;
    dst->recomputes = src->recomputes;
    dst->escale = src->escale;
    dst->evals = src->evals;
    dst->value = src->value;
    dst->rel = src->rel;
    dst->value_lo = src->value_lo;
    __threadfence_system();
  }
  if (p.done_host) {
    __hip_atomic_store(p.done_host, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __threadfence_system();
  }
}

constexpr int kBlock = 256;        // start, standalone evaluation
constexpr int kSweepBlock = 512;   // sweep and update kernels: 8 waves per workgroup
static_assert(kSweepBlock == 8 * kWave, "the core update assigns its phases to waves 0..7");
constexpr int kStart = 1024;       // rank-1 start samples
constexpr int kMaxSamples = 1024;
constexpr int kRook = 5;

// integrand classes a kernel can be specialised for
enum { FAM_PAPER = 0, FAM_UFORM = 1, FAM_SYNTH = 2, FAM_ANY = 3 };

template <class T, int FAM, int MAXM>
__device__ __forceinline__ T integrand_fam(const FamilyArgs& fa, const T (&y)[MAXM]) {
  if constexpr (is_ext_t<T>::value) {
    static_assert(FAM == FAM_PAPER, "the extended-precision paths cover the paper-form integrands");
    return ising_paper<T, MAXM>(fa.family, fa.m, y);
  } else if constexpr (FAM == FAM_PAPER) {
    return ising_paper<double, MAXM>(fa.family, fa.m, y);
  } else if constexpr (FAM == FAM_UFORM) {
    return ising_u<MAXM>(fa.family, fa.m, y, fa.four_over_mfact);
  } else if constexpr (FAM == FAM_SYNTH) {
    return synthetic<MAXM>(fa.family, fa.m, y, fa.a, fa.b);
  } else {
    return integrand<MAXM>(fa, y);
  }
}

// Streaming path (MAXM = 0, any number of modes, double precision): the
// paper-form and synthetic integrands over an accessor y(k), as f 2^escale.
// integrand_stream_me returns a mantissa and its exponent (f = v 2^ex) for the
// start, which fixes escale.
template <int FAM, class Y>
__device__ __forceinline__ double integrand_stream_me(const FamilyArgs& fa, const Y& y, int* ex) {
  static_assert(FAM == FAM_PAPER || FAM == FAM_SYNTH || FAM == FAM_ANY, "no streaming u-form");
  if constexpr (FAM == FAM_PAPER) {
    return ising_paper_stream_me(fa.family, fa.m, y, ex);
  } else if constexpr (FAM == FAM_SYNTH) {
    *ex = 0;
    return synthetic_stream(fa.family, fa.m, y, fa.a, fa.b);
  } else {
    if (fa.family == TT_ISING_C || fa.family == TT_ISING_D || fa.family == TT_ISING_E)
      return ising_paper_stream_me(fa.family, fa.m, y, ex);
    *ex = 0;
    return synthetic_stream(fa.family, fa.m, y, fa.a, fa.b);
  }
}

template <int FAM>
__device__ __forceinline__ double integrand_seg(const FamilyArgs& fa, const Segs& sg) {
  static_assert(FAM == FAM_PAPER || FAM == FAM_SYNTH || FAM == FAM_ANY, "no streaming u-form");
  if constexpr (FAM == FAM_PAPER) {
    return ising_paper_seg(fa.family, sg, fa.escale);
  } else if constexpr (FAM == FAM_SYNTH) {
    return ldexp(synthetic_seg(fa.family, sg, fa.a, fa.b), fa.escale);
  } else {
    if (fa.family == TT_ISING_C || fa.family == TT_ISING_D || fa.family == TT_ISING_E)
      return ising_paper_seg(fa.family, sg, fa.escale);
    return ldexp(synthetic_seg(fa.family, sg, fa.a, fa.b), fa.escale);
  }
}

// v = mant * 2^e with 1/2 <= |mant| < 1 (mant = v for 0 and non-finite v)
template <class T>
__device__ __forceinline__ T normalise(T v, int& e) {
  const double h = n_hi(v);
  e = 0;
  if (h == 0.0 || !isfinite(h)) return v;
  e = ilogb(h) + 1;
  return n_ldexp(v, -e);
}

// The arrays of a job hold T values; the descriptor carries them as double*.
template <class T> __device__ __forceinline__ T* tp(double* p) { return reinterpret_cast<T*>(p); }
template <class T> __device__ __forceinline__ const T* tp(const double* p) { return reinterpret_cast<const T*>(p); }

// the largest rank a job of number type T can have (quad-double jobs: TT_QD_MAX_RANK)
template <class T> constexpr int max_rank_of() { return sizeof(T) > 16 ? TT_QD_MAX_RANK : TT_MAX_RANK; }

__device__ __forceinline__ int rowcap(const ProbDesc& p, int c) { return c == 0 ? 1 : p.R; }
__device__ __forceinline__ int colcap(const ProbDesc& p, int c) { return c == p.m - 1 ? 1 : p.R; }

__device__ __forceinline__ FamilyArgs family_args(const ProbDesc& p) {
  return FamilyArgs{p.family, p.m, p.four_over_mfact, p.pa, p.pb, p.st->escale};
}

// ------------------------------------------------------------------ GL rule
// Nodes on [0,1] = (x+1)/2 for the roots x of P_n; weights 1/((1-x^2) P_n'(x)^2).
// Newton in double from the classical initial guess, then two Newton steps in
// double-double; the dd results are kept for the double-double path and
// rounded once to double for the double path.
__device__ inline void legendre_dd(int n, dd x, dd& pn, dd& pn1) {
  dd p0 = dd_from(1.0), p1 = x;
  if (n == 0) { pn = p0; pn1 = dd_from(0.0); return; }
  for (int k = 1; k < n; ++k) {
    dd a = dd_mul_d(dd_mul(x, p1), (double)(2 * k + 1));
    dd b = dd_mul_d(p0, (double)k);
    dd p2 = dd_div(dd_sub(a, b), dd_from((double)(k + 1)));
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pn1 = p0;
}

__device__ inline void gl_node(int n, int k, dd& t_out, dd& w_out) {
  // k-th root in decreasing order of x
  double x = cos(M_PI * ((double)k + 0.75) / ((double)n + 0.5));
  for (int it = 0; it < 100; ++it) {
    double p0 = 1.0, p1 = x;
    for (int j = 1; j < n; ++j) {
      double p2 = ((2 * j + 1) * x * p1 - j * p0) / (j + 1);
      p0 = p1;
      p1 = p2;
    }
    double dp = n * (x * p1 - p0) / (x * x - 1.0);
    double dx = p1 / dp;
    x -= dx;
    if (fabs(dx) < 1e-16) break;
  }
  dd X = dd_from(x), pn, pn1, dp;
  for (int it = 0; it < 2; ++it) {
    legendre_dd(n, X, pn, pn1);
    dd x2m1 = dd_sub(dd_mul(X, X), dd_from(1.0));
    dp = dd_div(dd_mul_d(dd_sub(dd_mul(X, pn), pn1), (double)n), x2m1);
    X = dd_sub(X, dd_div(pn, dp));
  }
  legendre_dd(n, X, pn, pn1);
  dd x2m1 = dd_sub(dd_mul(X, X), dd_from(1.0));
  dp = dd_div(dd_mul_d(dd_sub(dd_mul(X, pn), pn1), (double)n), x2m1);
  dd one_m_x2 = dd_neg(x2m1);
  dd wk = dd_div(dd_from(1.0), dd_mul(one_m_x2, dd_mul(dp, dp)));   // = w_x / 2
  t_out = dd_mul_d(dd_add(X, dd_from(1.0)), 0.5);
  w_out = wk;
}

// Quad-double nodes and weights: two Newton steps in quad-double from the
// double-double root (each step doubles the correct digits), then the weight
// 1/((1-x^2) P_n'(x)^2) in quad-double.
__device__ inline void legendre_qd(int n, qd x, qd& pn, qd& pn1) {
  qd p0 = qd_from(1.0), p1 = x;
  if (n == 0) { pn = p0; pn1 = qd_from(0.0); return; }
  for (int k = 1; k < n; ++k) {
    // P_{k+1} = ((2k+1) x P_k - k P_{k-1}) / (k+1)
    const qd a = qd_axpy_d((double)(2 * k + 1), qd_mul(x, p1), qd_from(0.0));
    const qd p2 = qd_div(qd_axpy_d(-(double)k, p0, a), qd_from((double)(k + 1)));
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pn1 = p0;
}

__device__ inline void gl_node_qd(int n, int k, qd& t_out, qd& w_out) {
  dd t2, w2;
  gl_node(n, k, t2, w2);
  // x = 2 t - 1 from the double-double node (exact)
  qd X = qd_add(qd{2.0 * t2.hi, 2.0 * t2.lo, 0.0, 0.0}, qd_from(-1.0));
  qd pn, pn1, dp, x2m1;
  for (int it = 0; it < 3; ++it) {
    legendre_qd(n, X, pn, pn1);
    x2m1 = qd_add(qd_mul(X, X), qd_from(-1.0));
    // P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1)
    dp = qd_div(qd_axpy_d((double)n, qd_add(qd_mul(X, pn), qd_neg(pn1)), qd_from(0.0)), x2m1);
    if (it < 2) X = qd_add(X, qd_neg(qd_div(pn, dp)));
  }
  w_out = qd_div(qd_from(1.0), qd_mul(qd_neg(x2m1), qd_mul(dp, dp)));   // = w_x / 2
  t_out = n_ldexp(qd_add(X, qd_from(1.0)), -1);
}

static __global__ void k_gl_qd(int n, qd* __restrict__ t4, qd* __restrict__ w4, int shift, qd* __restrict__ ws4) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    qd tk, wk;
    gl_node_qd(n, k, tk, wk);
    t4[n - 1 - k] = tk;   // increasing order
    w4[n - 1 - k] = wk;
    ws4[n - 1 - k] = n_ldexp(wk, shift);
  }
}

// ws, ws2: the weights times 2^shift (exact), the scale a job folds in
static __global__ void k_gl(int n, double* __restrict__ t, double* __restrict__ w, dd* __restrict__ t2,
                            dd* __restrict__ w2, int shift, double* __restrict__ ws, dd* __restrict__ ws2) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    dd tk, wk;
    gl_node(n, k, tk, wk);
    const double w1 = wk.hi + wk.lo;
    t[n - 1 - k] = tk.hi + tk.lo;   // increasing order
    w[n - 1 - k] = w1;
    t2[n - 1 - k] = tk;
    w2[n - 1 - k] = wk;
    ws[n - 1 - k] = ldexp(w1, shift);
    ws2[n - 1 - k] = n_ldexp(wk, shift);
  }
}


// ----------------------------------------------------- rank-1 start (m >= 0)
template <class T, int FAM, int MAXM>
__global__ __launch_bounds__(kBlock) void k_start(ProbDesc* __restrict__ P) {
  constexpr bool kStream = MAXM == 0;   // coordinates one at a time, any number of modes
  const ProbDesc p = P[blockIdx.x];
  const int m = p.m, n = p.n, tid = threadIdx.x;
  const FamilyArgs fa{p.family, p.m, p.four_over_mfact, p.pa, p.pb};   // unscaled: the start fixes the scale
  const T* __restrict__ tt = tp<T>(p.t);
  const T* __restrict__ ww = tp<T>(p.w);
  __shared__ double sv[kBlock / kWave + 1];
  __shared__ int si[kBlock / kWave + 1];
  __shared__ int s_i0[kStream ? TT_MAX_MODES : MAXM];
  __shared__ T s_buf[TT_MAX_NODES];
  __shared__ double s_cm[kStream ? kStart + TT_MAX_NODES : 1];   // streaming start candidates: mantissa
  __shared__ int s_ce[kStream ? kStart + TT_MAX_NODES : 1];      // and exponent
  ProbState* st = p.st;
  // clustered searches match exchange records by tag: none may survive from the
  // memory's earlier use
  constexpr int kSlotWords = (int)(sizeof(XSlot) / sizeof(uint64_t));
  for (int e = tid; e < p.nbonds * 2 * kMaxGroup * kSlotWords; e += blockDim.x)
    p.xch[e / kSlotWords].w[e % kSlotWords] = 0;

  if constexpr (!kStream) if (m <= 1) {   // no bond: the tensor is a vector (or a scalar for m = 0)
    T val = num<T>(0.0);
    if (m == 0) {
      T y[MAXM];
#pragma unroll
      for (int k = 0; k < MAXM; ++k) y[k] = num<T>(0.0);
      val = integrand_fam<T, FAM, MAXM>(fa, y);
    } else {
      for (int i = tid; i < n; i += blockDim.x) {
        T y[MAXM];
#pragma unroll
        for (int k = 0; k < MAXM; ++k) y[k] = num<T>(0.0);
        y[0] = tt[i];
        s_buf[i] = n_mul(ww[i], integrand_fam<T, FAM, MAXM>(fa, y));
      }
      __syncthreads();
      if (tid == 0)
        for (int i = 0; i < n; ++i) val = n_add(val, s_buf[i]);
    }
    if (tid == 0) {
      int e;
      const T mant = normalise(val, e);
      e -= p.wshift * m;
      tp<T>(p.hist)[0] = mant;
      p.hexp[0] = e;
      st->value = n_hi(mant);
      st->value_lo = n_lo(mant);
      st->vexp = e;
      st->rel = 0.0;
      st->sweeps = 0;
      st->done = 1;
      st->err_flags = isfinite(n_hi(val)) ? 0 : 1;
      st->recomputes = 0;
      st->escale = 0;
      st->reason = st->err_flags ? TT_STOP_ERROR : TT_STOP_CONVERGED;
      st->evals = (m == 1) ? (unsigned long long)n : 0ull;
      st->max_rank = 1;
      signal_done(p);
    }
    return;
  }

  ArgMax best{-1.0, 0x7fffffff};
  bool bad = false;
  int escale = 0;
  if constexpr (kStream) {
    // The streaming kernels: the candidates are the kStart random multi-indices
    // and, for D_d and E_d above 32 modes, the n constant ones (every mode at
    // node q - kStart).  A
    // random point's B falls far below the double range for D_d from about
    // d = 128 on, while the constant points reach the largest entries (C_d and
    // the synthetic families stay near 1 and keep the random candidates only).
    // Each candidate is formed as a mantissa and an exponent (the weight product
    // renormalised every 16 factors, the integrand by ising_paper_stream_me),
    // compared at the largest exponent, and escale = -(that exponent) brings the
    // chosen start's B into [1/2, 1).  Every later B of the job is f W 2^escale.
    const bool consts = (p.family == TT_ISING_D || p.family == TT_ISING_E) && m > TT_MAX_REG_MODES;
    const int ncand = kStart + (consts ? n : 0);
    constexpr int kOff = 1 << 24;   // exponents offset to positive keys; zero values get no key
    ArgMax emax{-1.0, 0x7fffffff};
    for (int q = tid; q < ncand; q += blockDim.x) {
      auto node = [&](int k) {
        return q < kStart ? (int)uniform_below(splitmix_at(p.seed, start_counter(q, k)), (uint32_t)n)
                          : q - kStart;
      };
      double Wm = 1.0;
      int We = 0;
      for (int k = 0; k < m; ++k) {
        Wm = Wm * n_hi(ww[node(k)]);
        if ((k & 15) == 15) {
          int e;
          Wm = frexp(Wm, &e);
          We += e;
        }
      }
      int fe;
      const double fv = integrand_stream_me<FAM>(fa, [&](int k) { return n_hi(tt[node(k)]); }, &fe);
      int e;
      const double mant = frexp(Wm * fv, &e);
      if (!isfinite(mant)) bad = true;
      s_cm[q] = mant;
      s_ce[q] = e + We + fe;
      if (mant != 0.0 && isfinite(mant) && better((double)(s_ce[q] + kOff), q, emax.v, emax.idx)) {
        emax.v = (double)(s_ce[q] + kOff);
        emax.idx = q;
      }
    }
    emax = block_argmax(emax, sv, si);   // its barriers also publish s_cm, s_ce
    const int etop = emax.v > 0.0 ? (int)emax.v - kOff : 0;
    escale = -etop;
    for (int q = tid; q < ncand; q += blockDim.x) {
      const double v = s_cm[q] != 0.0 && isfinite(s_cm[q]) ? ldexp(fabs(s_cm[q]), s_ce[q] - etop) : 0.0;
      if (better(v, q, best.v, best.idx)) { best.v = v; best.idx = q; }
    }
  } else {
    for (int q = tid; q < kStart; q += blockDim.x) {
      T y[MAXM];
      T W = num<T>(1.0);
#pragma unroll
      for (int k = 0; k < MAXM; ++k) {
        if (k < m) {
          int ik = (int)uniform_below(splitmix_at(p.seed, start_counter(q, k)), (uint32_t)n);
          y[k] = tt[ik];
          W = n_mul(W, ww[ik]);
        } else {
          y[k] = num<T>(0.0);
        }
      }
      const double v = n_hi(n_mul(W, integrand_fam<T, FAM, MAXM>(fa, y)));
      if (!isfinite(v)) bad = true;
      if (better(fabs(v), q, best.v, best.idx)) { best.v = fabs(v); best.idx = q; }
    }
  }
  best = block_argmax(best, sv, si);
  int any_bad = __syncthreads_or(bad);
  const int q = best.idx;
  for (int k = tid; k < m; k += blockDim.x)
    s_i0[k] = q < kStart ? (int)uniform_below(splitmix_at(p.seed, start_counter(q, k)), (uint32_t)n) : q - kStart;
  __syncthreads();
  if (any_bad || !(best.v > 0.0)) {
    if (tid == 0) {
      st->err_flags = any_bad ? 1 : 4;
      st->recomputes = 0;
      st->escale = 0;
      st->done = 1;
      st->reason = TT_STOP_ERROR;
      st->evals = kStart;
      st->sweeps = 0;
      st->max_rank = 0;
      st->value = 0.0;
      st->value_lo = 0.0;
      st->vexp = 0;
      st->rel = __builtin_huge_val();
      signal_done(p);
    }
    return;
  }
  const int nb = m - 1, R = p.R;
  T* __restrict__ Lx = tp<T>(p.Lx);
  T* __restrict__ Rx = tp<T>(p.Rx);
  T* __restrict__ Lw = tp<T>(p.Lw);
  T* __restrict__ Rw = tp<T>(p.Rw);
  // left sets I_<=b = {(i0_0..i0_b)}, right sets I_>b = {(i0_b+1..i0_m-1)}
  for (int e = tid; e < nb * m; e += blockDim.x) {
    int b = e / m, k = e % m;
    const T tk = tt[s_i0[k]];
    if (k <= b) Lx[((size_t)b * R) * m + k] = tk;
    else Rx[((size_t)b * R) * m + k] = tk;
  }
  if (tid == 0) {
    T lw = num<T>(1.0);
    for (int b = 0; b < nb; ++b) {
      lw = n_mul(lw, ww[s_i0[b]]);
      Lw[(size_t)b * R] = lw;
      p.Lpar[(size_t)b * R] = 0;
      p.Lnode[(size_t)b * R] = s_i0[b];
    }
    T rw = num<T>(1.0);
    for (int b = nb - 1; b >= 0; --b) {
      rw = n_mul(ww[s_i0[b + 1]], rw);
      Rw[(size_t)b * R] = rw;
      p.Rpar[(size_t)b * R] = 0;
      p.Rnode[(size_t)b * R] = s_i0[b + 1];
    }
    for (int b = 0; b < nb; ++b) {
      p.rank[b] = 1;
      p.scale[b] = best.v;
    }
    for (int k = 0; k < m; ++k) p.start[k] = s_i0[k];
    for (int k = 0; k <= m; ++k) p.sync[k] = 0;
    for (int k = 0; k < m; ++k) p.rfl[k] = 0;
    st->sweeps = 0;
    st->done = 0;
    st->reason = TT_RUNNING;
    st->err_flags = 0;
    st->recomputes = 0;
    st->escale = escale;
    st->evals = kStart + ((p.family == TT_ISING_D || p.family == TT_ISING_E) && m > TT_MAX_REG_MODES ? n : 0);
    st->max_rank = 1;
    st->rel = __builtin_huge_val();
  }
}

// ------------------------------------------------------------ search (Alg. 2)
template <class T, int MAXM>
struct SearchSmem {
  T Lx[max_rank_of<T>() * (MAXM + 1)];
  T Rx[max_rank_of<T>() * (MAXM + 1)];
  T Lw[max_rank_of<T>()], Rw[max_rank_of<T>()];
  T t[TT_MAX_NODES], w[TT_MAX_NODES];
  T vec[max_rank_of<T>()];
  // streaming C_d: B_d's running (P, q, s) over each left row and (P, q, g) over
  // each right row (g: the suffix recurrence started from zero)
  double sL[MAXM == 0 ? 3 * TT_MAX_RANK : 1], sR[MAXM == 0 ? 3 * TT_MAX_RANK : 1];
  double red_v[kSweepBlock / kWave + 1];
  int red_i[kSweepBlock / kWave + 1];
  T e_star, a_star;
  XRec<T> xres;   // a clustered search's combined record of the last exchange
  int xfail;
};

constexpr long long kWaitTicks = 1000000000LL;   // 10 s of the 100 MHz constant clock

// One step's combination across the G workgroups (members) of a superblock's
// search.  Thread 0 of each member posts its record as tagged words (XSlot); lanes
// 0..G-1 of wave 0 read the G records of this step until every word carries the
// step's tag.  argmax: the record of largest v, ties to the lowest idx (the
// block_argmax rule, so the result is the argmax over every member's points);
// otherwise v combines by max and idx by or.  publish: the member's earlier global
// writes are released before its record and acquired by the readers (the closing
// step, after which member 0 hands the results to the core updates).  Every thread
// receives the result through LDS; fail is set when a wait exceeded kWaitTicks.
// Records alternate between two rows by the step's parity: a member can only post
// step s + 2 after every member has posted step s + 1, hence after every member has
// read step s.  Called by the whole workgroup.
template <class T>
__device__ __forceinline__ XRec<T> group_exchange(XSlot* __restrict__ xs, const int g, const int G,
                                                  const uint32_t tag, const bool argmax, const bool publish,
                                                  const XRec<T> mine, XRec<T>& res, int& fail) {
  constexpr int W = (int)(sizeof(T) / sizeof(double)), NW = 3 + 4 * W;
  static_assert(NW <= kXWords, "an exchange record fits its slot");
  XSlot* row = xs + (tag & 1) * kMaxGroup;
  const uint64_t tg = (uint64_t)tag << 32;
  if (threadIdx.x == 0) {
    uint64_t* my = row[g].w;
    uint64_t words[NW];
    auto put = [&](int k, double x) {
      const uint64_t bits = (uint64_t)__double_as_longlong(x);
      words[k] = tg | (bits & 0xffffffffu);
      words[k + 1] = tg | (bits >> 32);
    };
    put(0, mine.v);
    words[2] = tg | (uint32_t)mine.idx;
    const double* ec = reinterpret_cast<const double*>(&mine.e);
    const double* ac = reinterpret_cast<const double*>(&mine.a);
#pragma unroll
    for (int c = 0; c < W; ++c) {
      put(3 + 2 * c, ec[c]);
      put(3 + 2 * W + 2 * c, ac[c]);
    }
    if (publish) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
#pragma unroll
    for (int k = 0; k < NW; ++k) __hip_atomic_store(&my[k], words[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (threadIdx.x < kWave) {
    const int h = threadIdx.x;
    int ok = 1;
    XRec<T> r{argmax ? -1.0 : 0.0, num<T>(0.0), num<T>(0.0), argmax ? 0x7fffffff : 0};
    double* rec = reinterpret_cast<double*>(&r.e);
    double* rac = reinterpret_cast<double*>(&r.a);
    if (h < G) {
      const uint64_t* src = row[h].w;
      uint64_t w[NW];
      const long long t0 = (long long)wall_clock64();
      for (;;) {
#pragma unroll
        for (int k = 0; k < NW; ++k) w[k] = __hip_atomic_load(&src[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bool all = true;
#pragma unroll
        for (int k = 0; k < NW; ++k) all = all && (w[k] >> 32) == tag;
        if (all) break;
        if ((long long)wall_clock64() - t0 > kWaitTicks) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (ok) {
        auto get = [&](int k) { return __longlong_as_double((long long)((w[k] & 0xffffffffu) | (w[k + 1] << 32))); };
        r.v = get(0);
        r.idx = (int)(uint32_t)w[2];
#pragma unroll
        for (int c = 0; c < W; ++c) {
          rec[c] = get(3 + 2 * c);
          rac[c] = get(3 + 2 * W + 2 * c);
        }
      }
    }
    if (publish) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#pragma unroll
    for (int off = 1; off < kMaxGroup; off <<= 1) {   // lanes 0..7 hold the records (or neutral ones)
      const double ov = __shfl_xor(r.v, off, kWave);
      const int oi = __shfl_xor(r.idx, off, kWave);
      double oe[W], oa[W];
#pragma unroll
      for (int c = 0; c < W; ++c) {
        oe[c] = __shfl_xor(rec[c], off, kWave);
        oa[c] = __shfl_xor(rac[c], off, kWave);
      }
      if (argmax) {
        if (better(ov, oi, r.v, r.idx)) {
          r.v = ov;
          r.idx = oi;
#pragma unroll
          for (int c = 0; c < W; ++c) {
            rec[c] = oe[c];
            rac[c] = oa[c];
          }
        }
      } else {
        r.v = fmax(r.v, ov);
        r.idx |= oi;
      }
    }
    const int all_ok = __all(ok);
    if (h == 0) {
      res = r;
      fail = !all_ok;
    }
  }
  __syncthreads();
  return res;
}

// C_d's value depends on the coordinates only through B_d's prefix sum and suffix
// recurrence, and both compose over a split of the coordinates: (P1, q1, s1) then
// (P2, q2, g2) give (P1 P2, q1 + P1 q2, g2 + P2 s1), g2 being the recurrence over
// the second part from zero.  row_summaries writes (P, q, s) over coordinates
// kL0..kL1-1 of the left rows Lrows[a] (a < nL) to dL[a], dL[TT_MAX_RANK + a],
// dL[2 TT_MAX_RANK + a], and the same from zero over kR0..kR1-1 of the right rows
// to dR.  Each row is walked by 16 lanes, a sixteenth each, the parts joined in
// order.  Called by the whole workgroup; a barrier must follow before dL, dR are
// read.
__device__ __forceinline__ void row_summaries(const double* __restrict__ Lrows, int nL, int kL0, int kL1,
                                              double* dL, const double* __restrict__ Rrows, int nR, int kR0,
                                              int kR1, double* dR, int m) {
  constexpr int kLpr = 16;   // lanes per row
  const int part = threadIdx.x % kLpr;
  for (int row = threadIdx.x / kLpr; row < nL + nR; row += blockDim.x / kLpr) {
    const bool left = row < nL;
    const int idx = left ? row : row - nL;
    const double* ptr = (left ? Lrows : Rrows) + (size_t)idx * m;
    const int k0 = left ? kL0 : kR0, k1 = left ? kL1 : kR1;
    const int chunk = ((k1 - k0 + kLpr - 1) / kLpr + 3) & ~3;
    const int lo = min(k0 + part * chunk, k1), hi = min(lo + chunk, k1);
    PrefixSuffix ps;
    ps.span(ptr, lo, hi);
#pragma unroll
    for (int d = 1; d < kLpr; d <<= 1) {   // join part + d onto part, in order
      const double P2 = __shfl_down(ps.P, d, kLpr), q2 = __shfl_down(ps.q, d, kLpr);
      const double s2 = __shfl_down(ps.s, d, kLpr);
      if ((part & (2 * d - 1)) == 0) {
        ps.q = fma(ps.P, q2, ps.q);
        ps.s = fma(P2, ps.s, s2);
        ps.P = ps.P * P2;
      }
    }
    if (part == 0) {
      double* dst = left ? dL : dR;
      dst[idx] = ps.P;
      dst[TT_MAX_RANK + idx] = ps.q;
      dst[2 * TT_MAX_RANK + idx] = ps.s;
    }
  }
}

// C_d at a point from its left row's summary, one or two nodes and its right
// row's summary (from zero): the value 2 / ((1 + q)(1 + s)) of B_d's sums, times
// 2^escale.
__device__ __forceinline__ double ising_c_joined(const double* sL, int al, double t0, double t1, int nM,
                                                 const double* sR, int be, int escale) {
  PrefixSuffix ps;
  ps.P = sL[al];
  ps.q = sL[TT_MAX_RANK + al];
  ps.s = sL[2 * TT_MAX_RANK + al];
  ps.one(t0);
  if (nM > 1) ps.one(t1);
  const double q = fma(ps.P, sR[TT_MAX_RANK + be], ps.q);
  const double sfx = fma(sR[be], ps.s, sR[2 * TT_MAX_RANK + be]);
  return ldexp(2.0 / ((1.0 + q) * (1.0 + sfx)), escale);
}

// One step of Alg. 2 on superblock b.  The random samples, every column step and
// every row step run through the same evaluation loop (one inlined integrand).
// Decisions (argmax, acceptance) are taken on the leading double of |error|.
//
// A search may be spread over G workgroups (members g = 0..G-1 of a cluster):
// member g evaluates the points q with q / blockDim = g mod G, and after each
// loop the members combine their block argmaxes (group_exchange), so every
// member takes the decisions one workgroup would take, on the same values.  A last
// exchange combines the largest |B| seen and the non-finite flags; member 0 then
// writes the pivot record.  Only member 0 returns true (it is to signal the cores).
template <class T, int FAM, int MAXM>
__device__ __forceinline__ bool search_bond(const ProbDesc& p, const int b, const int g, const int G,
                                            SearchSmem<T, MAXM>& sm) {
  constexpr int LD = MAXM + 1;
  constexpr bool kStream = MAXM == 0;   // coordinates read from the index-set rows in memory
  const int tid = threadIdx.x;
  ProbState* st = p.st;
  const int m = p.m, n = p.n, R = p.R, nb = p.nbonds;
  const int sweep = st->sweeps;
  const int rb = p.rank[b];
  const int rL = b > 0 ? p.rank[b - 1] : 1;
  const int rR = b < m - 2 ? p.rank[b + 1] : 1;
  if (rb >= R) {
    if (tid == 0 && g == 0) {
      PivRec rec{-1, -1, 0, 0, 0.0, 0.0, 0, 0};
      p.piv[b] = rec;
      p.log[(size_t)sweep * nb + b] = rec;
    }
    return g == 0;
  }
  XSlot* const xs = p.xch + (size_t)b * 2 * kMaxGroup;
  uint32_t xstep = 0;                                        // exchanges of this search so far
  const uint32_t xtag0 = (uint32_t)(sweep + 1) << 5;         // at most 2 + 2 kRook exchanges
  const FamilyArgs fa = family_args(p);
  const T* __restrict__ gLx = tp<T>(p.Lx);
  const T* __restrict__ gRx = tp<T>(p.Rx);
  const T* __restrict__ gLw = tp<T>(p.Lw);
  const T* __restrict__ gRw = tp<T>(p.Rw);
  const T* __restrict__ gt = tp<T>(p.t);
  const T* __restrict__ gw = tp<T>(p.w);
  if (g == 0) mark(p, sweep, b, 0);
  // stage index-set coordinates, node table and weights in LDS
  if constexpr (!kStream) {
    for (int e = tid; e < rL * b; e += blockDim.x) {
      const int a = e / b, k = e % b;
      sm.Lx[a * LD + k] = gLx[((size_t)(b - 1) * R + a) * m + k];
    }
    const int nright = m - b - 2;
    for (int e = tid; e < rR * nright; e += blockDim.x) {
      const int a = e / nright, k = b + 2 + e % nright;
      sm.Rx[a * LD + k] = gRx[((size_t)(b + 1) * R + a) * m + k];
    }
  }
  for (int a = tid; a < rL; a += blockDim.x) sm.Lw[a] = b > 0 ? gLw[(size_t)(b - 1) * R + a] : num<T>(1.0);
  for (int a = tid; a < rR; a += blockDim.x)
    sm.Rw[a] = (b + 1 <= m - 2) ? gRw[(size_t)(b + 1) * R + a] : num<T>(1.0);
  for (int i = tid; i < n; i += blockDim.x) { sm.t[i] = gt[i]; sm.w[i] = gw[i]; }
  if (tid == 0) { sm.e_star = num<T>(0.0); sm.a_star = num<T>(0.0); }
  // C_d: every row of the two index sets is summarised once, so a point of the
  // search costs two node steps and a join instead of a pass over m coordinates
  bool rowsum = false;
  if constexpr (kStream && (FAM == FAM_PAPER || FAM == FAM_ANY)) {
    rowsum = fa.family == TT_ISING_C;
    if (rowsum)
      row_summaries(gLx + (size_t)(b > 0 ? b - 1 : 0) * R * m, rL, 0, b > 0 ? b : 0, sm.sL,
                    gRx + (size_t)(b + 1 <= m - 2 ? b + 1 : 0) * R * m, rR, b + 2,
                    b + 1 <= m - 2 ? m : b + 2, sm.sR, m);
  }
  __syncthreads();
  if (g == 0) mark(p, sweep, b, 1);

  const int nrows = rL * n, ncols = n * rR;
  const T* __restrict__ F1 = tp<T>(p.F) + p.Foff[b + 1];
  const int cc1 = colcap(p, b + 1);
  // The column step at col = (j, beta) evaluates F_b(alpha, i, (j, beta)) for every old
  // row: the new column of F_b if this pivot is accepted; the row step at row = (alpha,
  // i) evaluates F_{b+1}((alpha, i), j, beta) for every old column: its new row.  Both
  // are written into the free slot (column r_b of F_b, row r_b of F_{b+1}) as they are
  // evaluated, so the core updates need not evaluate them again.
  T* Fb_new = tp<T>(p.F) + p.Foff[b] + rb;
  const int ccb = colcap(p, b);
  T* F1_new = tp<T>(p.F) + p.Foff[b + 1] + (size_t)rb * n * cc1;
  const T* __restrict__ Cb = tp<T>(p.C) + p.Coff[b];
  const size_t ldC = (size_t)rowcap(p, b) * n;
  const int nsamp = min(nrows + ncols, kMaxSamples);
  const uint32_t total = (uint32_t)nrows * (uint32_t)ncols;

  double seen = 0.0;
  bool bad = false, invalid = false;
  int mode = 0;            // 0: random samples, 1: column step, 2: row step
  int row = 0, col = 0, iters = 0;
  bool col_fresh = false;  // the last column step was taken at the final column
  const bool timed = p.phase != nullptr && g == 0 && tid == 0;   // profiled runs: step durations
  long long tq0 = 0, tq1 = 0, tq2 = 0, tq3 = 0, tq4 = 0, tq5 = 0, tq6 = 0;
  long long t0 = timed ? (long long)wall_clock64() : 0;
  for (;;) {
    if (mode == 1) {          // B~(:, col) = C_b F_{b+1}(:, col)
      const int j = col / rR, be = col - j * rR;
      if (tid < rb) sm.vec[tid] = F1[((size_t)tid * n + j) * cc1 + be];
    } else if (mode == 2) {   // B~(row, :) = C_b(row, :) F_{b+1}
      if (tid < rb) sm.vec[tid] = Cb[(size_t)tid * ldC + row];
    }
    __syncthreads();
    long long t1 = 0;
    if (timed) {
      t1 = (long long)wall_clock64();
      if (mode != 0) tq6 += t1 - t0;
    }
    const int count = mode == 0 ? nsamp : (mode == 1 ? nrows : ncols);
    ArgMax best{-1.0, 0x7fffffff};
    T my_e = num<T>(0.0), my_a = num<T>(0.0);
    for (int q = g * (int)blockDim.x + tid; q < count; q += G * (int)blockDim.x) {
      int pr, pc;
      if (mode == 0) {
        const uint32_t id = uniform_below(splitmix_at(p.seed, sample_counter(sweep, b, q)), total);
        pr = (int)(id / (uint32_t)ncols);
        pc = (int)(id % (uint32_t)ncols);
      } else if (mode == 1) {
        pr = q;
        pc = col;
      } else {
        pr = row;
        pc = q;
      }
      // B at (alpha, i, j, beta): coordinates of I_<=b-1[alpha], t_i, t_j, I_>b+1[beta]
      const int al = pr / n, i = pr - al * n;
      const int j = pc / rR, be = pc - j * rR;
      // weights multiplied in the order the core update uses for the same entry
      const T W = (mode == 1) ? n_mul(n_mul(sm.Lw[al], sm.w[i]), n_mul(sm.w[j], sm.Rw[be]))
                              : n_mul(n_mul(n_mul(sm.Lw[al], sm.w[i]), sm.w[j]), sm.Rw[be]);
      T a;
      if constexpr (kStream) {
        if (rowsum) {
          a = n_mul(W, ising_c_joined(sm.sL, al, sm.t[i], sm.t[j], 2, sm.sR, be, fa.escale));
        } else {
          const T* Lrow = gLx + ((size_t)(b > 0 ? b - 1 : 0) * R + al) * m;
          const T* Rrow = gRx + ((size_t)(b + 1 <= m - 2 ? b + 1 : 0) * R + be) * m;
          const Segs sg{Lrow, b, sm.t[i], sm.t[j], 2, Rrow, m};
          a = n_mul(W, integrand_seg<FAM>(fa, sg));
        }
      } else {
        T y[MAXM];
#pragma unroll
        for (int k = 0; k < MAXM; ++k) {
          T v = num<T>(0.0);
          if (k < m) {
            v = (k < b) ? sm.Lx[al * LD + k] : sm.Rx[be * LD + k];
            v = (k == b) ? sm.t[i] : v;
            v = (k == b + 1) ? sm.t[j] : v;
          }
          y[k] = v;
        }
        a = n_mul(W, integrand_fam<T, FAM, MAXM>(fa, y));
      }
      if (mode == 1) Fb_new[(size_t)pr * ccb] = a;
      else if (mode == 2) F1_new[(size_t)j * cc1 + be] = a;
      T s = num<T>(0.0);
      if (mode == 0) {
#pragma unroll 8
        for (int k = 0; k < rb; ++k) s = n_mad(Cb[(size_t)k * ldC + pr], F1[((size_t)k * n + j) * cc1 + be], s);
      } else if (mode == 1) {
#pragma unroll 8
        for (int k = 0; k < rb; ++k) s = n_mad(Cb[(size_t)k * ldC + pr], sm.vec[k], s);
      } else {
#pragma unroll 8
        for (int k = 0; k < rb; ++k) s = n_mad(sm.vec[k], F1[((size_t)k * n + j) * cc1 + be], s);
      }
      const T e = n_sub(a, s);
      const double ae = fabs(n_hi(e));
      bad |= !isfinite(n_hi(e));
      seen = fmax(seen, fabs(n_hi(a)));
      if (better(ae, q, best.v, best.idx)) { best.v = ae; best.idx = q; my_e = e; my_a = a; }
    }
    long long t2 = 0;
    if (timed) t2 = (long long)wall_clock64();
    best = block_argmax(best, sm.red_v, sm.red_i);
    if (timed) {
      const long long t3 = (long long)wall_clock64();
      if (mode == 0) {
        tq0 += t2 - t1;
        tq1 += t3 - t2;
      } else {
        tq3 += t2 - t1;
        tq4 += t3 - t2;
      }
      t0 = t3;
    }
    {
      if (G > 1) {   // the members' argmaxes combined (with the winner's error and value at a row step)
        if (mode == 2) {
          if (best.idx % (int)blockDim.x == tid) {
            sm.e_star = my_e;
            sm.a_star = my_a;
          }
          __syncthreads();
        }
        const XRec<T> mine{best.v, mode == 2 ? sm.e_star : num<T>(0.0), mode == 2 ? sm.a_star : num<T>(0.0),
                           best.idx};
        const XRec<T> r = group_exchange<T>(xs, g, G, xtag0 + xstep++, true, false, mine, sm.xres, sm.xfail);
        best.v = r.v;
        best.idx = r.idx;
        my_e = r.e;   // held by every thread: the owner test below is replaced
        my_a = r.a;
        if (timed) {
          const long long t4 = (long long)wall_clock64();
          if (mode == 0) tq2 += t4 - t0;
          else tq5 += t4 - t0;
          t0 = t4;
        }
        if (sm.xfail) {
          if (tid == 0) atomicOr(&st->err_flags, 16);
          invalid = true;
          break;
        }
      }
    }
    if (!(best.v >= 0.0)) { invalid = true; break; }   // every error non-finite
    if (mode == 0) {
      if (g == 0) mark(p, sweep, b, 2);
      const uint32_t id = uniform_below(splitmix_at(p.seed, sample_counter(sweep, b, best.idx)), total);
      row = (int)(id / (uint32_t)ncols);
      col = (int)(id % (uint32_t)ncols);
      mode = 1;
      continue;
    }
    if (mode == 1) {
      row = best.idx;
      mode = 2;
      continue;
    }
    if (G > 1 ? tid == 0 : best.idx % (int)blockDim.x == tid) {   // the thread that evaluated the winner
      sm.e_star = my_e;
      sm.a_star = my_a;
    }
    __syncthreads();
    ++iters;
    const bool same = (best.idx == col);   // rook condition: the row step kept the column
    col = best.idx;
    col_fresh = same;
    if (same || iters == kRook) break;
    mode = 1;
  }
  if (g == 0) {
    mark(p, sweep, b, 3);
    mark_value(p, sweep, b, 8, tq0);
    mark_value(p, sweep, b, 9, tq1);
    mark_value(p, sweep, b, 10, tq2);
    mark_value(p, sweep, b, 11, tq3);
    mark_value(p, sweep, b, 12, tq4);
    mark_value(p, sweep, b, 13, tq5);
    mark_value(p, sweep, b, 14, tq6);
  }
  seen = block_max(seen, sm.red_v);
  int any_bad = __syncthreads_or(bad);
  {
    if (G > 1) {   // every member's largest |B| and flags; also: every member's writes are done
      const XRec<T> r = group_exchange<T>(xs, g, G, xtag0 + xstep++, false, true,
                                          XRec<T>{seen, num<T>(0.0), num<T>(0.0), any_bad}, sm.xres, sm.xfail);
      seen = r.v;
      any_bad = r.idx;
      if (sm.xfail) {
        if (tid == 0) atomicOr(&st->err_flags, 16);
        invalid = true;
      }
    }
  }
  if (g != 0) return false;
  // is either half of the pivot already in its set? (one thread per set element)
  const int al_s = row / n, i_s = row - al_s * n;
  const int j_s = col / rR, be_s = col - j_s * rR;
  int mine = 0;
  if (tid < rb) {
    mine = (p.Lpar[(size_t)b * R + tid] == al_s && p.Lnode[(size_t)b * R + tid] == i_s) ||
           (p.Rnode[(size_t)b * R + tid] == j_s && p.Rpar[(size_t)b * R + tid] == be_s);
  }
  const int dup = __syncthreads_or(mine);
  if (tid == 0) {
    const double e_star = n_hi(sm.e_star), a_star = n_hi(sm.a_star);
    const double scale = fmax(p.scale[b], seen);
    p.scale[b] = scale;
    const int acc = (fabs(e_star) > p.tol * scale) && !dup && !any_bad && !invalid;
    PivRec rec{row, col, acc, iters, e_star, a_star, col_fresh ? 1 : 0, 0};
    p.piv[b] = rec;
    p.log[(size_t)sweep * nb + b] = rec;
    if (any_bad || invalid) atomicOr(&st->err_flags, 1);
    const int per_step = nrows + ncols;
    atomicAdd(&st->evals, (unsigned long long)(nsamp + iters * per_step));
  }
  return true;
}

// ------------------------------------------------------------ core update
template <class T, int MAXM, int RMAX>
struct UpdateSmem {
  union {
    struct {                       // fibre evaluation stage
      T Lx[max_rank_of<T>() * (MAXM + 1)];
      T Rx[max_rank_of<T>() * (MAXM + 1)];
      T Lw[max_rank_of<T>()], Rw[max_rank_of<T>()];
      T t[TT_MAX_NODES], w[TT_MAX_NODES];
      // streaming C_d: row summaries of I_<=c-1 and of the new rows of I_>c
      double sL[MAXM == 0 ? 3 * TT_MAX_RANK : 1], sR[MAXM == 0 ? 3 * TT_MAX_RANK : 1];
    };
    T A[RMAX * (RMAX + 1)];        // the stored LU of the cross, zero-padded to RMAX
  };
  T u[RMAX], cp[RMAX];
  int rowidx[RMAX];
  int perm[RMAX];                  // row permutation of the recomputation
  int zf;                          // the recomputation met a zero pivot
  double rv[kSweepBlock / kWave];  // per-wave largest |C_c| written this sweep
  T delta;
};

// |C_c| above which a core's interpolation core is recomputed (see update_core):
// an incremental step amplifies the rounding already in C_c by about |C_c|^2, so
// at 16 a double step adds at most ~256 eps (3e-14); the Ising crosses of the
// benchmark stay below 5, while C_d with few nodes reaches 1e10.  Double-double
// and quad-double values carry 2^-104 and 2^-204 rounding: at 1024 a step adds
// at most 5e-26 and 1e-55, below the tolerances those jobs are run at, and the
// rank-64 crosses of D_11 and D_12 with 128 nodes (|C_c| between 16 and 1024)
// keep their incremental updates.
template <class T> constexpr double dominance_of() { return sizeof(T) > sizeof(double) ? 1024.0 : 16.0; }

// running max of |x| for the dominance test; a non-finite x counts as infinite
__device__ __forceinline__ double cmax_of(double cmax, double x) {
  const double a = fabs(x);
  return (a <= cmax) ? cmax : (isfinite(a) ? a : __builtin_huge_val());
}

// Gaussian elimination with partial pivoting of the r x r matrix in sm.A (leading
// dimension RMAX + 1), in wave 0 alone with wave-level ordering only: P A = L U in
// place (L unit lower, its multipliers below the diagonal), the row permutation in
// sm.perm (filled by the caller with 0..RMAX-1), sm.zf = 1 if a column has no
// nonzero pivot.  Every thread of the workgroup calls it; a barrier follows.
template <int RMAX, class Smem>
__device__ __forceinline__ void lu_pivoted(const int r, Smem& sm) {
  using T = typename std::remove_reference<decltype(sm.A[0])>::type;
  constexpr int LA = RMAX + 1;
  const int tid = threadIdx.x;
  if (tid < kWave) {   // the elimination runs in wave 0 alone, with wave-level ordering only
    bool zero = false;
#pragma unroll 1
    for (int k = 0; k < r && !zero; ++k) {
      // pivot row among k..r-1 (r <= 64), ties to the lowest row, NaN never
      ArgMax a{-1.0, 0x7fffffff};
      const int i = k + tid;
      if (i < r) {
        a.v = fabs(n_hi(sm.A[i * LA + k]));
        a.idx = i;
      }
      a = wave_argmax(a);
      zero = !(a.v > 0.0);                   // a zero column: M_c is singular
      if (zero) break;
      const int pi = a.idx;
      if (pi != k) {
        if (tid < r) {
          const T tmp = sm.A[k * LA + tid];
          sm.A[k * LA + tid] = sm.A[pi * LA + tid];
          sm.A[pi * LA + tid] = tmp;
        }
        if (tid == 0) {
          const int t2 = sm.perm[k];
          sm.perm[k] = sm.perm[pi];
          sm.perm[pi] = t2;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int i2 = k + 1 + tid;           // multipliers of the rows below, stored in place (L)
      if (i2 < r) sm.A[i2 * LA + k] = n_div(sm.A[i2 * LA + k], sm.A[k * LA + k]);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int w = r - k - 1;
      for (int e = tid; e < w * w; e += kWave) {
        const int i3 = k + 1 + e / w, j = k + 1 + e % w;
        sm.A[i3 * LA + j] = n_nmad(sm.A[i3 * LA + k], sm.A[k * LA + j], sm.A[i3 * LA + j]);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (tid == 0) sm.zf = zero ? 1 : 0;
  }
  __syncthreads();
}

// x = U^-1 L^-1 P f for the rows row = tid, tid + blockDim.x, .. < N of the
// workgroup, with the factors of lu_pivoted: f(row, q) reads entry q of row f and
// xat(q, row) is unknown q of that row's solution (read and written in place).
template <int RMAX, class Smem, class FGet, class XAt>
__device__ __forceinline__ void solve_rows(const int r, const int N, Smem& sm, FGet&& fget, XAt&& xat) {
  using T = typename std::remove_reference<decltype(sm.A[0])>::type;
  constexpr int LA = RMAX + 1;
  const int tid = threadIdx.x;
  // Row solves in blocks of kB unknowns held in registers: the earlier (forward)
  // or later (backward) unknowns are read from the unknowns' storage once per block, not once per
  // unknown.  The guards on q0 + t < r depend only on the block: no divergence.
  constexpr int kB = 4;
#pragma unroll 1
  for (int row = tid; row < N; row += blockDim.x) {
#pragma unroll 1
    for (int q0 = 0; q0 < r; q0 += kB) {   // L y = P f (unit lower)
      T acc[kB];
#pragma unroll
      for (int t = 0; t < kB; ++t) acc[t] = (q0 + t < r) ? fget(row, sm.perm[q0 + t]) : num<T>(0.0);
#pragma unroll 1
      for (int pp = 0; pp < q0; ++pp) {
        const T y = xat(pp, row);
#pragma unroll
        for (int t = 0; t < kB; ++t)
          if (q0 + t < r) acc[t] = n_nmad(sm.A[(q0 + t) * LA + pp], y, acc[t]);
      }
#pragma unroll
      for (int t = 1; t < kB; ++t)
#pragma unroll
        for (int u = 0; u < t; ++u)
          if (q0 + t < r) acc[t] = n_nmad(sm.A[(q0 + t) * LA + q0 + u], acc[u], acc[t]);
#pragma unroll
      for (int t = 0; t < kB; ++t)
        if (q0 + t < r) xat(q0 + t, row) = acc[t];
    }
#pragma unroll 1
    for (int q0 = ((r - 1) / kB) * kB; q0 >= 0; q0 -= kB) {   // U x = y
      T acc[kB];
#pragma unroll
      for (int t = 0; t < kB; ++t) acc[t] = (q0 + t < r) ? xat(q0 + t, row) : num<T>(0.0);
#pragma unroll 1
      for (int pp = q0 + kB; pp < r; ++pp) {
        const T x = xat(pp, row);
#pragma unroll
        for (int t = 0; t < kB; ++t)
          if (q0 + t < r) acc[t] = n_nmad(sm.A[(q0 + t) * LA + pp], x, acc[t]);
      }
#pragma unroll
      for (int t = kB - 1; t >= 0; --t)
        if (q0 + t < r) {
#pragma unroll
          for (int u = t + 1; u < kB; ++u)
            if (q0 + u < r) acc[t] = n_nmad(sm.A[(q0 + t) * LA + q0 + u], acc[u], acc[t]);
          acc[t] = n_div(acc[t], sm.A[(q0 + t) * LA + q0 + t]);
        }
#pragma unroll
      for (int t = 0; t < kB; ++t)
        if (q0 + t < r) xat(q0 + t, row) = acc[t];
    }
  }
}

// C_c = F_c M_c^-1 from scratch (in the job's number type): M_c = F_c(I_<=c, :r), the
// old cross rows sm.rowidx[0..r0) and, when a pivot was accepted this sweep,
// prow.  With A = M_c^T, Gaussian elimination with partial pivoting gives
// P A = L U in LDS (lu_pivoted); every row f of F_c is then solved by the
// workgroup as A x = f^T, x = U^-1 L^-1 P f^T, in place in C_c (solve_rows: a
// solve, not a product with an inverse: its residual stays at the rounding level
// of the factors, so C_c(I_<=c, :) stays the identity to rounding even for a
// nearly singular cross).  Loops are kept rolled so the routine adds few
// registers to the sweep kernel.  Marks the core for later sweeps.
template <int RMAX, class T, class Smem>
__device__ __forceinline__ void refresh_core(const ProbDesc& p, const int c, const int r, const int N, const int prow,
                                             const int r0, const T* __restrict__ Fc, const int cc,
                                             T* __restrict__ Cc, const size_t ldC, Smem& sm) {
  constexpr int LA = RMAX + 1;
  const int tid = threadIdx.x;
  if (tid == 0) {
    p.rfl[c] = 1;
    atomicAdd(&p.st->recomputes, 1);
    if (prow >= 0) sm.rowidx[r0] = prow;
  }
  if (tid < RMAX) sm.perm[tid] = tid;
  __syncthreads();
  for (int e = tid; e < r * r; e += blockDim.x) {
    const int i = e / r, j = e % r;
    sm.A[i * LA + j] = Fc[(size_t)sm.rowidx[j] * cc + i];
  }
  __syncthreads();
  lu_pivoted<RMAX>(r, sm);
  if (tid == 0 && sm.zf) atomicOr(&p.st->err_flags, 2);
  solve_rows<RMAX>(r, N, sm, [&](int row, int q) { return Fc[(size_t)row * cc + q]; },
                   [&](int q, int row) -> T& { return Cc[(size_t)q * ldC + row]; });
  __syncthreads();
}

template <class T, int FAM, int MAXM, int RMAX>
__device__ __forceinline__ void update_core(const ProbDesc& p, const int c, const int init,
                                            UpdateSmem<T, MAXM, RMAX>& sm, const int mb = -1) {
  constexpr int LD = MAXM + 1;
  constexpr int LA = RMAX + 1;
  constexpr bool kStream = MAXM == 0;   // coordinates read from the index-set rows in memory
  // a row of C_c is kept in registers while it is updated when it is small
  // enough; otherwise it is worked on in place in memory
  constexpr bool kRowInRegs = sizeof(T) * RMAX <= 256;
  const int tid = threadIdx.x;
  ProbState* st = p.st;
  if (st->done) return;
  const int m = p.m, n = p.n, R = p.R;
  const FamilyArgs fa = family_args(p);
  T* __restrict__ gLx = tp<T>(p.Lx);
  T* __restrict__ gRx = tp<T>(p.Rx);
  T* __restrict__ gLw = tp<T>(p.Lw);
  T* __restrict__ gRw = tp<T>(p.Rw);
  const T* __restrict__ gt = tp<T>(p.t);
  const T* __restrict__ gw = tp<T>(p.w);
  const bool hasL = c >= 1, hasR = c <= m - 2;
  const int accL = (!init && hasL) ? p.piv[c - 1].acc : 0;
  const int accR = (!init && hasR) ? p.piv[c].acc : 0;
  const int rL_com = hasL ? p.rank[c - 1] : 1;
  const int rR_com = hasR ? p.rank[c] : 1;
  const int rL_old = init ? 0 : rL_com, rL_new = rL_com + accL;
  const int rR_old = init ? 0 : rR_com, rR_new = rR_com + accR;
  const int msw = init ? 0 : st->sweeps;

  // ---- append the accepted pivots (each set element is written by exactly one workgroup)
  int alL = 0, iL = 0;   // new element of I_<=c-1: (alpha*, i*) with alpha* in I_<=c-2
  if (accL) {
    const int row = p.piv[c - 1].row;
    alL = row / n;
    iL = row - alL * n;
  }
  int jR = 0, beR = 0;   // new element of I_>c: (j*, beta*) with beta* in I_>c+1
  if (accR) {
    const int rRR = (c + 1 <= m - 2) ? p.rank[c + 1] : 1;
    const int col = p.piv[c].col;
    jR = col / rRR;
    beR = col - jR * rRR;
  }
  // their weights, multiplied as the earlier elements' were
  const T wL = accL ? n_mul(c - 1 >= 1 ? gLw[(size_t)(c - 2) * R + alL] : num<T>(1.0), gw[iL]) : num<T>(0.0);
  const T wR = accR ? n_mul(gw[jR], (c + 1 <= m - 2) ? gRw[(size_t)(c + 1) * R + beR] : num<T>(1.0)) : num<T>(0.0);
  if (accL) {
    const int bl = c - 1;
    const size_t dst = (size_t)bl * R + rL_old;
    for (int k = tid; k < bl; k += blockDim.x) gLx[dst * m + k] = gLx[((size_t)(bl - 1) * R + alL) * m + k];
    if (tid == 0) {
      p.Lpar[dst] = alL;
      p.Lnode[dst] = iL;
      gLx[dst * m + bl] = gt[iL];
      gLw[dst] = wL;
    }
  }
  if (accR) {
    const size_t dst = (size_t)c * R + rR_old;
    for (int k = c + 2 + tid; k < m; k += blockDim.x)
      gRx[dst * m + k] = gRx[((size_t)(c + 1) * R + beR) * m + k];
    if (tid == 0) {
      p.Rnode[dst] = jR;
      p.Rpar[dst] = beR;
      gRx[dst * m + c + 1] = gt[jR];
      gRw[dst] = wR;
    }
  }
  // ---- stage I_<=c-1 and I_>c coordinates; a new element is staged from its parent
  //      row, so the staging does not wait for the appended rows (the streaming
  //      evaluation reads those after the barrier below)
  if constexpr (!kStream) {
    for (int e = tid; e < rL_new * c; e += blockDim.x) {
      const int a = e / c, k = e % c;
      T v;
      if (accL && a == rL_old)
        v = (k < c - 1) ? gLx[((size_t)(c - 2) * R + alL) * m + k] : gt[iL];
      else
        v = gLx[((size_t)(c - 1) * R + a) * m + k];
      sm.Lx[a * LD + k] = v;
    }
    const int nright = m - c - 1;
    for (int e = tid; e < rR_new * nright; e += blockDim.x) {
      const int a = e / nright, k = c + 1 + e % nright;
      T v;
      if (accR && a == rR_old)
        v = (k == c + 1) ? gt[jR] : gRx[((size_t)(c + 1) * R + beR) * m + k];
      else
        v = gRx[((size_t)c * R + a) * m + k];
      sm.Rx[a * LD + k] = v;
    }
  }
  for (int a = tid; a < rL_new; a += blockDim.x)
    sm.Lw[a] = !hasL ? num<T>(1.0) : (accL && a == rL_old) ? wL : gLw[(size_t)(c - 1) * R + a];
  for (int a = tid; a < rR_new; a += blockDim.x)
    sm.Rw[a] = !hasR ? num<T>(1.0) : (accR && a == rR_old) ? wR : gRw[(size_t)c * R + a];
  for (int i = tid; i < n; i += blockDim.x) { sm.t[i] = gt[i]; sm.w[i] = gw[i]; }
  __syncthreads();
  if (mb >= 0) mark(p, msw, mb, 9);

  // ---- evaluate the new entries of F_c = B(I_<=c-1, i_c, I_>c) that no search evaluated:
  //      the new row at the old columns came from bond c-1's last row step and the new
  //      column at the old rows from bond c's last column step (when taken at the final
  //      column); what remains is the corner (new row, new column), or the new column
  //      at every row.  At init every entry is new.
  T* __restrict__ Fc = tp<T>(p.F) + p.Foff[c];
  const int cc = colcap(p, c);
  const int nBc = rR_new - rR_old;
  const int nA = (rL_new - rL_old) * n * nBc;               // new rows x new columns
  const bool col_done = !init && accR && p.piv[c].col_fresh;
  const int nB = col_done ? 0 : rL_old * n * nBc;           // new column (old rows)
  bool rowsum = false;   // streaming C_d: the points joined from row summaries
  if constexpr (kStream && (FAM == FAM_PAPER || FAM == FAM_ANY)) {
    rowsum = fa.family == TT_ISING_C && nA + nB > 0;
    if (rowsum) {
      row_summaries(gLx + (size_t)(hasL ? c - 1 : 0) * R * m, rL_new, 0, hasL ? c : 0, sm.sL,
                    gRx + ((size_t)(hasR ? c : 0) * R + rR_old) * m, nBc, c + 1, hasR ? m : c + 1,
                    sm.sR + rR_old, m);
      __syncthreads();
    }
  }
  bool bad = false;
  for (int e = tid; e < nA + nB; e += blockDim.x) {
    int al, i, be;
    if (e < nA) {
      al = rL_old + e / (n * nBc);
      const int rem = e % (n * nBc);
      i = rem / nBc;
      be = rR_old + rem % nBc;
    } else {
      const int e2 = e - nA;
      al = e2 / (n * nBc);
      const int rem = e2 % (n * nBc);
      i = rem / nBc;
      be = rR_old + rem % nBc;
    }
    const T W = n_mul(n_mul(sm.Lw[al], sm.w[i]), sm.Rw[be]);
    T v;
    if constexpr (kStream) {
      if (rowsum) {
        v = n_mul(W, ising_c_joined(sm.sL, al, sm.t[i], 0.0, 1, sm.sR, be, fa.escale));
      } else {
        const T* Lrow = gLx + ((size_t)(c > 0 ? c - 1 : 0) * R + al) * m;
        const T* Rrow = gRx + ((size_t)(c <= m - 2 ? c : 0) * R + be) * m;
        const Segs sg{Lrow, c, sm.t[i], 0.0, 1, Rrow, m};
        v = n_mul(W, integrand_seg<FAM>(fa, sg));
      }
    } else {
      T y[MAXM];
#pragma unroll
      for (int k = 0; k < MAXM; ++k) {
        T yk = num<T>(0.0);
        if (k < m) {
          yk = (k < c) ? sm.Lx[al * LD + k] : sm.Rx[be * LD + k];
          yk = (k == c) ? sm.t[i] : yk;
        }
        y[k] = yk;
      }
      v = n_mul(W, integrand_fam<T, FAM, MAXM>(fa, y));
    }
    bad |= !isfinite(n_hi(v));
    Fc[((size_t)al * n + i) * cc + be] = v;
  }
  const int any_bad = __syncthreads_or(bad);
  if (mb >= 0) mark(p, msw, mb, 10);
  if (tid == 0) {
    atomicAdd(&st->evals, (unsigned long long)(nA + nB));
    if (any_bad) atomicOr(&st->err_flags, 1);
  }

  T* __restrict__ S = tp<T>(p.S) + (size_t)c * R * R;
  if (!hasR) {   // last core: S(alpha) = sum_i F(alpha, i)
    for (int al = tid; al < rL_new; al += blockDim.x) {
      T s = num<T>(0.0);
#pragma unroll 16
      for (int i = 0; i < n; ++i) s = n_add(s, Fc[(size_t)al * n + i]);
      S[(size_t)al * R] = s;
    }
    return;
  }

  // ---- interpolation core C_c = F_c M_c^-1, M_c = rows I_<=c of F_c (insertion order)
  const int r0 = rR_old;     // rank of bond c before this sweep
  const int r = rR_new;
  const int N = rL_new * n;
  if (r > RMAX) {            // the host picks RMAX >= any rank reachable this sweep
    if (tid == 0) atomicOr(&st->err_flags, 8);
    return;
  }
  T* __restrict__ LU = tp<T>(p.LU) + (size_t)c * R * R;
  T* __restrict__ Cc = tp<T>(p.C) + p.Coff[c];
  const size_t ldC = (size_t)rowcap(p, c) * n;
  __syncthreads();   // the evaluation stage's LDS is reused below
  double cmax = 0.0;   // largest |entry| of C_c written below
  bool sing = false;   // a zero pivot in the incremental steps
  if (init == 2) {   // every entry re-evaluated on refreshed sets: C_c from F_c with a pivoted solve
    if (tid < r) sm.rowidx[tid] = p.Lpar[(size_t)c * R + tid] * n + p.Lnode[(size_t)c * R + tid];
    __syncthreads();
    refresh_core<RMAX>(p, c, r, N, -1, r, Fc, cc, Cc, ldC, sm);
  } else if (init) {   // rank 1: M_c = (B(i0)), C_c = F_c / M_c
    const int row0 = p.Lpar[(size_t)c * R] * n + p.Lnode[(size_t)c * R];
    const T m00 = Fc[(size_t)row0 * cc];
    if (tid == 0) {
      LU[0] = m00;
      if (n_hi(m00) == 0.0) atomicOr(&st->err_flags, 2);
    }
    for (int row = tid; row < N; row += blockDim.x) Cc[row] = n_div(Fc[(size_t)row * cc], m00);
  } else {
    for (int e = tid; e < RMAX * RMAX; e += blockDim.x) {
      const int a = e / RMAX, q = e % RMAX;
      sm.A[a * LA + q] = (a < r0 && q < r0) ? LU[(size_t)a * R + q] : num<T>(0.0);
    }
    if (tid < r0) sm.rowidx[tid] = p.Lpar[(size_t)c * R + tid] * n + p.Lnode[(size_t)c * R + tid];
    __syncthreads();
    // (a) rows of the new element of I_<=c-1: solve x M_c = f with M_c = L U
    //     (x L) U = f: forward over columns for g = x L, then backward over rows for x.
    //     (a) and the bordering (c) below are independent (c reads only old rows of
    //     C_c); (a) runs on waves 0 and 4..7, (c) on waves 1..3, side by side.
    const int wv = tid / kWave, ln = tid % kWave;
    const int aslot = wv == 0 ? 0 : wv - 3;   // waves 0, 4, 5, 6, 7 -> slots 0..4
    if (accL && (wv == 0 || wv >= 4)) {
      for (int i = aslot * kWave + ln; i < n; i += 5 * kWave) {
        const int row = rL_old * n + i;
        if constexpr (kRowInRegs) {
          T x[RMAX];
#pragma unroll
          for (int q = 0; q < RMAX; ++q) x[q] = (q < r0) ? Fc[(size_t)row * cc + q] : num<T>(0.0);
#pragma unroll
          for (int q = 0; q < RMAX; ++q) {
            if (q < r0) {
              T s = x[q];
#pragma unroll
              for (int pp = 0; pp < q; ++pp) s = n_nmad(x[pp], sm.A[pp * LA + q], s);
              x[q] = n_div(s, sm.A[q * LA + q]);
            }
          }
#pragma unroll
          for (int a = RMAX - 1; a >= 0; --a) {
            if (a < r0) {
              T s = x[a];
#pragma unroll
              for (int bb = a + 1; bb < RMAX; ++bb) s = n_nmad(x[bb], sm.A[bb * LA + a], s);
              x[a] = s;
            }
          }
#pragma unroll
          for (int a = 0; a < RMAX; ++a)
            if (a < r0) {
              Cc[(size_t)a * ldC + row] = x[a];
              cmax = cmax_of(cmax, n_hi(x[a]));
            }
        } else {   // the same solves with the row of C_c as the working storage
          for (int q = 0; q < r0; ++q) {
            T s = Fc[(size_t)row * cc + q];
            for (int pp = 0; pp < q; ++pp) s = n_nmad(Cc[(size_t)pp * ldC + row], sm.A[pp * LA + q], s);
            Cc[(size_t)q * ldC + row] = n_div(s, sm.A[q * LA + q]);
          }
          for (int a = r0 - 1; a >= 0; --a) {
            T s = Cc[(size_t)a * ldC + row];
            for (int bb = a + 1; bb < r0; ++bb) s = n_nmad(Cc[(size_t)bb * ldC + row], sm.A[bb * LA + a], s);
            Cc[(size_t)a * ldC + row] = s;
            cmax = cmax_of(cmax, n_hi(s));
          }
        }
      }
    }
    if (mb >= 0) mark(p, msw, mb, 11);
    if (accR) {
      const int prow = p.piv[c].row;   // the row of F_c appended to I_<=c this sweep
      // (c) border the LU: w = L^-1 u, l = v U^-1 and the pivot delta, with u = F_c(I_<=c, r0)
      //     the new column at the old cross rows and v = F_c(prow, :r0).  The three are
      //     independent sequential chains, one wave each (waves 1, 2, 3; lane k holds
      //     entry k), run while the other waves solve the new rows (a).
      //
      // The pivot is the residual of the new cross row, delta = F_c(prow, r0) - C_c(prow, :) u
      // (equal to F_c(prow, r0) - l . w in exact arithmetic), computed with the very operations
      // the update below applies to row prow: the update then gives C_c(prow, :) = e_r0 exactly,
      // keeping the interpolation property at the new cross row.  With the Schur complement of
      // the bordered LU instead, the two roundings differ by about eps |C_c(prow,:)| |u|, which
      // a pivot near the rounding level of the cross turns into an O(1) error of that row.
      if (wv == 1) {
        T wa = (ln < r0) ? Fc[(size_t)sm.rowidx[ln] * cc + r0] : num<T>(0.0);
        if (ln < r0) sm.u[ln] = wa;
        for (int k2 = 0; k2 < r0; ++k2) {
          const T wk = n_shfl(wa, k2);
          if (ln > k2 && ln < r0) wa = n_nmad(sm.A[ln * LA + k2], wk, wa);
        }
        if (ln < r0) LU[(size_t)ln * R + r0] = wa;
      } else if (wv == 2) {
        T lq = (ln < r0) ? Fc[(size_t)prow * cc + ln] : num<T>(0.0);
        for (int k2 = 0; k2 < r0; ++k2) {
          const T lk = n_div(n_shfl(lq, k2), sm.A[k2 * LA + k2]);
          if (ln == k2) lq = lk;
          else if (ln > k2 && ln < r0) lq = n_nmad(lk, sm.A[k2 * LA + ln], lq);
        }
        if (ln < r0) LU[(size_t)r0 * R + ln] = lq;
      } else if (wv == 3) {
        const T uk = (ln < r0) ? Fc[(size_t)sm.rowidx[ln] * cc + r0] : num<T>(0.0);
        const T ck = (ln < r0) ? Cc[(size_t)ln * ldC + prow] : num<T>(0.0);   // C_c(prow, :) before the update
        if (ln < r0) sm.cp[ln] = ck;
        T e = Fc[(size_t)prow * cc + r0];
        for (int k = 0; k < r0; ++k) e = n_nmad(n_shfl(ck, k), n_shfl(uk, k), e);
        if (ln == 0) {
          LU[(size_t)r0 * R + r0] = e;
          sm.delta = e;
          // a zero pivot leaves C_c non-finite: the core is then recomputed (below)
        }
      }
      __syncthreads();
      if (mb >= 0) mark(p, msw, mb, 12);
      // (b) rank-1 update of every row: e = F_c(:, r0) - C_c u, C_c <- [C_c - (e/delta) c_piv, e/delta]
      const T delta = sm.delta;
      sing = n_hi(delta) == 0.0;
      for (int row = tid; row < N; row += blockDim.x) {
        if constexpr (kRowInRegs) {
          T x[RMAX];
#pragma unroll
          for (int k = 0; k < RMAX; ++k) x[k] = (k < r0) ? Cc[(size_t)k * ldC + row] : num<T>(0.0);
          T e = Fc[(size_t)row * cc + r0];
#pragma unroll
          for (int k = 0; k < RMAX; ++k)
            if (k < r0) e = n_nmad(x[k], sm.u[k], e);
          const T f = n_div(e, delta);
#pragma unroll
          for (int k = 0; k < RMAX; ++k)
            if (k < r0) {
              const T cn = n_nmad(f, sm.cp[k], x[k]);
              Cc[(size_t)k * ldC + row] = cn;
              cmax = cmax_of(cmax, n_hi(cn));
            }
          Cc[(size_t)r0 * ldC + row] = f;
          cmax = cmax_of(cmax, n_hi(f));
        } else {
          T e = Fc[(size_t)row * cc + r0];
          for (int k = 0; k < r0; ++k) e = n_nmad(Cc[(size_t)k * ldC + row], sm.u[k], e);
          const T f = n_div(e, delta);
          for (int k = 0; k < r0; ++k) {
            const T cn = n_nmad(f, sm.cp[k], Cc[(size_t)k * ldC + row]);
            Cc[(size_t)k * ldC + row] = cn;
            cmax = cmax_of(cmax, n_hi(cn));
          }
          Cc[(size_t)r0 * ldC + row] = f;
          cmax = cmax_of(cmax, n_hi(f));
        }
      }
    }
    if (mb >= 0) mark(p, msw, mb, 13);
    // the largest |C_c| written (infinite for a zero pivot): one value per wave,
    // combined after the barrier below
    const double cm = wave_max(sing ? __builtin_huge_val() : cmax);
    if ((tid & (kWave - 1)) == 0) sm.rv[tid / kWave] = cm;
  }
  __syncthreads();
  // ---- recomputation of C_c for crosses far from dominant.  The
  //      incremental steps above are exact algebra, but each carries the rounding
  //      already in C_c over with a factor of about |C_c|^2.  Alg. 6 takes each
  //      bond's pivot against the neighbours' previous sets, and on some
  //      integrands (C_d with few nodes) the crosses lose dominance, |C_c|
  //      reaching 1e4 within a few sweeps.  Once |C_c| exceeds dominance_of<T>() (or a
  //      pivot is zero) the core is recomputed from F_c with a pivoted LU of the
  //      cross in this and every later sweep, as the plain definition does
  //      (double and double-double jobs alike).
  if (!init) {
    double cm = 0.0;
    for (int w = 0; w < kSweepBlock / kWave; ++w) cm = fmax(cm, sm.rv[w]);
    if (p.rfl[c] || !(cm <= dominance_of<T>()))
      refresh_core<RMAX>(p, c, r, N, accR ? p.piv[c].row : -1, r0, Fc, cc, Cc, ldC, sm);
  }
  // ---- S_c(alpha, k) = sum_i C_c(alpha, i, k)
  for (int e = tid; e < rL_new * r; e += blockDim.x) {
    const int al = e / r, k = e % r;
    const T* __restrict__ src = Cc + (size_t)k * ldC + (size_t)al * n;
    T s = num<T>(0.0);
#pragma unroll 16
    for (int i = 0; i < n; ++i) s = n_add(s, src[i]);
    S[(size_t)al * R + k] = s;
  }
  if (mb >= 0) {
    __syncthreads();
    mark(p, msw, mb, 14);
  }
}

// ------------------------------------------- ALS maxvol refresh (Alg. 3, Alg. 1)
// One refresh of an integral's index sets at fixed ranks, by one workgroup,
// bonds in order.  Left to right, bond b: the r_{b-1} n x r_b matrix
// A = B(I_<=b-1 x [n], I_>b) on the left set of bond b-1 refreshed one step
// before; its maxvol rows (alpha, i) become I_<=b.  Right to left: the
// n r_{b+1} x r_b matrix B(I_<=b, [n] x I_>b+1)^T on the refreshed right set of
// bond b+1; its maxvol rows (j, beta) become I_>b.  maxvol (Sec. 2.4): r rows by
// Gaussian elimination with partial pivoting, then Alg. 1 steps on
// C = A A(I,:)^-1, recomputed from A after every swap, while the largest |C|
// exceeds 1 + kMaxvolDelta (at most 4 r swaps).  The matrices are kept column by
// column in the storage of the cores (A) and of the interpolation cores (the
// elimination copy, then C); the cores, interpolation cores and core sums are
// then rebuilt on the new sets (update_core, init 2), which recomputes every
// interpolation core from its core in later sweeps as well.
constexpr double kMaxvolDelta = 1e-2;

template <int MAXM>
struct AlsSmem {
  union {
    struct {
      double Lx[TT_MAX_RANK * (MAXM + 1)];
      double Rx[TT_MAX_RANK * (MAXM + 1)];
      double Lw[TT_MAX_RANK], Rw[TT_MAX_RANK];
    } ev;
    double A[TT_MAX_RANK * (TT_MAX_RANK + 1)];   // LU of A(I, :)^T
  };
  double t[TT_MAX_NODES], w[TT_MAX_NODES];
  double prow[TT_MAX_RANK];
  int rows[TT_MAX_RANK], perm[TT_MAX_RANK];
  double red_v[kSweepBlock / kWave + 1];
  int red_i[kSweepBlock / kWave + 1];
  int zf;
};

// The entries F_c(alpha, i, beta) = B(I_<=c-1[alpha], t_i, I_>c[beta]) of core c on
// the current sets (alpha < rl, beta < rr), each written to W[at(alpha, i, beta)];
// returns this thread's largest |B| and sets bad on a non-finite value.
template <int FAM, int MAXM, class At>
__device__ __forceinline__ double als_core_values(const ProbDesc& p, const FamilyArgs& fa, const int c,
                                                  const int rl, const int rr, double* __restrict__ W, At&& at,
                                                  AlsSmem<MAXM>& sm, bool& bad) {
  constexpr int LD = MAXM + 1;
  constexpr bool kStream = MAXM == 0;
  const int tid = threadIdx.x, m = p.m, n = p.n, R = p.R;
  const double* __restrict__ gLx = p.Lx;
  const double* __restrict__ gRx = p.Rx;
  const bool hasL = c >= 1, hasR = c <= m - 2;
  if constexpr (!kStream) {
    for (int e = tid; e < rl * c; e += blockDim.x) {
      const int a = e / c, k = e % c;
      sm.ev.Lx[a * LD + k] = gLx[((size_t)(c - 1) * R + a) * m + k];
    }
    const int nright = m - c - 1;
    for (int e = tid; e < rr * nright; e += blockDim.x) {
      const int a = e / nright, k = c + 1 + e % nright;
      sm.ev.Rx[a * LD + k] = gRx[((size_t)c * R + a) * m + k];
    }
  }
  for (int a = tid; a < rl; a += blockDim.x) sm.ev.Lw[a] = hasL ? p.Lw[(size_t)(c - 1) * R + a] : 1.0;
  for (int a = tid; a < rr; a += blockDim.x) sm.ev.Rw[a] = hasR ? p.Rw[(size_t)c * R + a] : 1.0;
  __syncthreads();
  double amax = 0.0;
  const int total = rl * n * rr;
  for (int e = tid; e < total; e += blockDim.x) {
    const int al = e / (n * rr), rem = e % (n * rr), i = rem / rr, be = rem % rr;
    const double Wt = (sm.ev.Lw[al] * sm.w[i]) * sm.ev.Rw[be];
    double v;
    if constexpr (kStream) {
      const double* Lrow = gLx + ((size_t)(hasL ? c - 1 : 0) * R + al) * m;
      const double* Rrow = gRx + ((size_t)(hasR ? c : 0) * R + be) * m;
      const Segs sg{Lrow, c, sm.t[i], 0.0, 1, Rrow, m};
      v = Wt * integrand_seg<FAM>(fa, sg);
    } else {
      double y[MAXM];
#pragma unroll
      for (int k = 0; k < MAXM; ++k) {
        double yk = 0.0;
        if (k < m) {
          yk = (k < c) ? sm.ev.Lx[al * LD + k] : sm.ev.Rx[be * LD + k];
          yk = (k == c) ? sm.t[i] : yk;
        }
        y[k] = yk;
      }
      v = Wt * integrand_fam<double, FAM, MAXM>(fa, y);
    }
    bad |= !isfinite(v);
    amax = fmax(amax, fabs(v));
    W[at(al, i, be)] = v;
  }
  __syncthreads();
  return amax;
}

// maxvol rows of the N x r matrix W (column q at W + q N) into sm.rows; V holds
// N r doubles of working storage.  Returns the number of swaps, or -1 if W has
// rank below r.
template <class Smem>
__device__ __forceinline__ int als_maxvol(const double* __restrict__ W, const int N, const int r,
                                          double* __restrict__ V, Smem& sm) {
  constexpr int LA = TT_MAX_RANK + 1;
  const int tid = threadIdx.x;
  for (int e = tid; e < N * r; e += blockDim.x) V[e] = W[e];
  __syncthreads();
  // start: Gaussian elimination with partial (row) pivoting, column by column
  for (int k = 0; k < r; ++k) {
    ArgMax a{-1.0, 0x7fffffff};
    for (int row = tid; row < N; row += blockDim.x) {
      const double v = fabs(V[(size_t)k * N + row]);
      if (better(v, row, a.v, a.idx)) { a.v = v; a.idx = row; }
    }
    a = block_argmax(a, sm.red_v, sm.red_i);
    if (!(a.v > 0.0)) return -1;
    const int pr = a.idx;
    if (tid == 0) sm.rows[k] = pr;
    for (int q = tid; q < r; q += blockDim.x) sm.prow[q] = V[(size_t)q * N + pr];
    __syncthreads();
    const double piv = sm.prow[k];
    for (int row = tid; row < N; row += blockDim.x) {
      const double f = V[(size_t)k * N + row] / piv;
      for (int q = k + 1; q < r; ++q) V[(size_t)q * N + row] = V[(size_t)q * N + row] - f * sm.prow[q];
    }
    __syncthreads();
  }
  // Alg. 1 steps: C = W W(I,:)^-1 (A = W(I,:)^T factored, each row solved), swap at max |C|
  int swaps = 0;
  for (;;) {
    if (tid < TT_MAX_RANK) sm.perm[tid] = tid;
    for (int e = tid; e < r * r; e += blockDim.x) {
      const int i = e / r, j = e % r;
      sm.A[i * LA + j] = W[(size_t)i * N + sm.rows[j]];
    }
    __syncthreads();
    lu_pivoted<TT_MAX_RANK>(r, sm);
    if (sm.zf) return -1;
    solve_rows<TT_MAX_RANK>(r, N, sm, [&](int row, int q) { return W[(size_t)q * N + row]; },
                            [&](int q, int row) -> double& { return V[(size_t)q * N + row]; });
    __syncthreads();
    ArgMax a{-1.0, 0x7fffffff};
    for (int row = tid; row < N; row += blockDim.x)
      for (int q = 0; q < r; ++q) {
        const double v = fabs(V[(size_t)q * N + row]);
        if (better(v, row * r + q, a.v, a.idx)) { a.v = v; a.idx = row * r + q; }
      }
    a = block_argmax(a, sm.red_v, sm.red_i);
    if (!(a.v > 1.0 + kMaxvolDelta) || swaps >= 4 * r) break;
    if (tid == 0) sm.rows[a.idx % r] = a.idx / r;
    ++swaps;
    __syncthreads();
  }
  return swaps;
}

template <int FAM, int MAXM>
__device__ __forceinline__ void als_refresh(const ProbDesc& p, AlsSmem<MAXM>& sm) {
  const int tid = threadIdx.x;
  ProbState* st = p.st;
  const int m = p.m, n = p.n, R = p.R;
  if (st->done || m < 2) return;
  const FamilyArgs fa = family_args(p);
  for (int i = tid; i < n; i += blockDim.x) { sm.t[i] = p.t[i]; sm.w[i] = p.w[i]; }
  __syncthreads();
  bool bad = false;
  int fail = 0;
  unsigned long long evals = 0;
  // left to right: I_<=b from core b on the refreshed I_<=b-1 and the current I_>b
  for (int b = 0; b < m - 1 && !fail; ++b) {
    const int rl = b > 0 ? p.rank[b - 1] : 1, r = p.rank[b], N = rl * n;
    double* W = p.F + p.Foff[b];
    double* V = p.C + p.Coff[b];
    const double amax = als_core_values<FAM, MAXM>(p, fa, b, rl, r, W,
        [&](int al, int i, int be) { return (size_t)be * N + (size_t)al * n + i; }, sm, bad);
    const double am = block_max(amax, sm.red_v);
    if (__syncthreads_or(bad)) { fail = 1; break; }
    if (als_maxvol(W, N, r, V, sm) < 0) { fail = 2; break; }
    double* gLx = p.Lx;
    for (int e = tid; e < r * (b + 1); e += blockDim.x) {   // row a: I_<=b-1[alpha] + (i)
      const int a = e / (b + 1), k = e % (b + 1), q = sm.rows[a], al = q / n, i = q % n;
      gLx[((size_t)b * R + a) * m + k] = (k < b) ? gLx[((size_t)(b - 1) * R + al) * m + k] : sm.t[i];
    }
    for (int a = tid; a < r; a += blockDim.x) {
      const int q = sm.rows[a], al = q / n, i = q % n;
      p.Lpar[(size_t)b * R + a] = al;
      p.Lnode[(size_t)b * R + a] = i;
      p.Lw[(size_t)b * R + a] = (b > 0 ? p.Lw[(size_t)(b - 1) * R + al] : 1.0) * sm.w[i];
    }
    if (tid == 0) p.scale[b] = fmax(p.scale[b], am);
    evals += (unsigned long long)N * r;
    __syncthreads();
  }
  // right to left: I_>b from core b+1 on the refreshed I_<=b and I_>b+1
  for (int b = m - 2; b >= 0 && !fail; --b) {
    const int r = p.rank[b], rn = b + 1 <= m - 2 ? p.rank[b + 1] : 1, N = n * rn;
    double* W = p.F + p.Foff[b + 1];
    double* V = p.C + (b + 1 <= m - 2 ? p.Coff[b + 1] : p.Coff[b]);
    const double amax = als_core_values<FAM, MAXM>(p, fa, b + 1, r, rn, W,
        [&](int al, int j, int be) { return (size_t)al * N + (size_t)j * rn + be; }, sm, bad);
    const double am = block_max(amax, sm.red_v);
    if (__syncthreads_or(bad)) { fail = 1; break; }
    if (als_maxvol(W, N, r, V, sm) < 0) { fail = 2; break; }
    double* gRx = p.Rx;
    const int w = m - b - 1;                                  // coordinates b+1 .. m-1
    for (int e = tid; e < r * w; e += blockDim.x) {           // row a: (j) + I_>b+1[beta]
      const int a = e / w, k = b + 1 + e % w, q = sm.rows[a], j = q / rn, be = q % rn;
      gRx[((size_t)b * R + a) * m + k] = (k == b + 1) ? sm.t[j] : gRx[((size_t)(b + 1) * R + be) * m + k];
    }
    for (int a = tid; a < r; a += blockDim.x) {
      const int q = sm.rows[a], j = q / rn, be = q % rn;
      p.Rnode[(size_t)b * R + a] = j;
      p.Rpar[(size_t)b * R + a] = be;
      p.Rw[(size_t)b * R + a] = sm.w[j] * (b + 1 <= m - 2 ? p.Rw[(size_t)(b + 1) * R + be] : 1.0);
    }
    if (tid == 0) p.scale[b] = fmax(p.scale[b], am);
    evals += (unsigned long long)N * r;
    __syncthreads();
  }
  if (tid == 0) {
    atomicAdd(&st->evals, evals);
    if (fail) {   // a numeric failure ends the integral (the sets may be half refreshed)
      atomicOr(&st->err_flags, fail == 1 ? 1 : 2);
      st->reason = TT_STOP_ERROR;
      st->done = 1;
      signal_done(p);
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------ k_integral
constexpr int kIntBlock = 512;
constexpr int kIntStageBytes = 49152;   // S staged in LDS at once

template <class T>
struct IntSmem {
  static constexpr int kMaxR = max_rank_of<T>();
  static constexpr int kStage = kIntStageBytes / (int)sizeof(T) > kMaxR * (kMaxR + 1)
                                     ? kIntStageBytes / (int)sizeof(T) : kMaxR * (kMaxR + 1);
  static constexpr int kIntBatch = 6;   // staging loads (of one double) in flight per thread
  T v[kWave], v2[kWave];
  T stage[kStage];
  int s_rank[TT_MAX_MODES];
  int s_off[TT_MAX_MODES + 1];
  int wsum[kSweepBlock / kWave];
  int cnt[2];   // accepted pivots, largest rank
};

// Column entries of a factor read at once in the quadrature chain: a rank-16 or
// rank-32 kernel reads 16 (one block covers rank 16), the others 8, which keeps
// their register count where the rest of the sweep puts it; 4 for double-double.
template <class T, int RMAX>
constexpr int chain_block_size() {
  return sizeof(T) != sizeof(double) ? 4 : (RMAX == 16 || RMAX == 32) ? 16 : 8;
}

template <class T, int CB>
__device__ __forceinline__ void integral_problem(const ProbDesc& p, const int init, IntSmem<T>& sm) {
  constexpr int kStage = IntSmem<T>::kStage;
  constexpr int kIntBatch = IntSmem<T>::kIntBatch;
  constexpr int kChainBlk = CB;
  static_assert(kWave % kChainBlk == 0, "a block of v never runs past entry kWave - 1");
  ProbState* st = p.st;
  if (st->done) return;
  T* __restrict__ hist = tp<T>(p.hist);
  const T* __restrict__ gS = tp<T>(p.S);
  // state needed by the stopping rule, loaded now so its latency overlaps the chain
  const int sw0 = st->sweeps;
  const T prev = hist[sw0];
  const int prev_exp = p.hexp[sw0];
  const double prev_rel = st->rel;
  T* v = sm.v;
  T* v2 = sm.v2;
  T* stage = sm.stage;
  int* s_rank = sm.s_rank;
  int* s_off = sm.s_off;
  const int m = p.m, R = p.R, nb = p.nbonds, tid = threadIdx.x;
  // commit the ranks: r_b += accepted_b
  if (tid == 0) {
    sm.cnt[0] = 0;
    sm.cnt[1] = 1;
  }
  __syncthreads();
  int acc = 0, below = 0, maxr = 1;
  for (int b = tid; b < nb; b += blockDim.x) {
    const int a = init ? 0 : p.piv[b].acc;
    const int r = p.rank[b] + a;
    p.rank[b] = r;
    s_rank[b] = r;
    acc += a;
    below |= r < R;
    maxr = max(maxr, r);
  }
  if (acc) atomicAdd(&sm.cnt[0], acc);
  if (maxr > 1) atomicMax(&sm.cnt[1], maxr);
  const int below_cap = __syncthreads_or(below);
  const int nacc = sm.cnt[0];
  maxr = sm.cnt[1];
  // In LDS a factor S_c (r_{c-1} x r_c, r_{m-1} = 1) is held column by column,
  // each column padded with zeros to a whole number of chain blocks plus one
  // entry: the odd stride puts the columns that neighbouring lanes read in
  // different LDS banks.  s_off[c] is the summed size of S_c' over 1 <= c' < c:
  // where each factor sits once the factors are laid out back to back
  auto pad = [](int r) { return (r + kChainBlk - 1) / kChainBlk * kChainBlk + 1; };
  {
    const int nf = m - 1, per = (nf + (int)blockDim.x - 1) / (int)blockDim.x, f0 = tid * per;
    const int f1 = min(f0 + per, nf), lane = tid & (kWave - 1), wid = tid / kWave;
    int loc = 0;
    for (int f = f0; f < f1; ++f) loc += pad(s_rank[f]) * (f + 1 <= m - 2 ? s_rank[f + 1] : 1);
    int x = loc;   // inclusive scan over the wave, then over the waves
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int y = __shfl_up(x, d, kWave);
      if (lane >= d) x += y;
    }
    if (lane == kWave - 1) sm.wsum[wid] = x;
    __syncthreads();
    int run = x - loc;
    for (int w = 0; w < wid; ++w) run += sm.wsum[w];
    for (int f = f0; f < f1; ++f) {
      run += pad(s_rank[f]) * (f + 1 <= m - 2 ? s_rank[f + 1] : 1);
      s_off[f + 2] = run;
    }
    if (tid == 0) s_off[1] = 0;
  }
  // v = S_0 (1 x r_0), then v <- v S_c for c = 1..m-1 (2m-1 matrices, inverses in C)
  if (tid < kWave) v[tid] = tid < s_rank[0] ? gS[tid] : num<T>(0.0);
  __syncthreads();
  int vexp = 0;   // v times 2^vexp is the chain's value (kept by wave 0)
  int c0 = 1;
  while (c0 < m) {
    // stage S_c0 .. S_c1-1, as many consecutive factors as fit (the stage holds
    // at least one S_c of the largest rank), as one flat range of doubles (a
    // double-double entry is two): each thread issues all its loads before the
    // first store, so a stage costs one memory latency, not one per core
    const int base = s_off[c0];
    int c1 = c0 + 1;
    for (int hi = m; c1 < hi;) {   // last c1 with s_off[c1] - base <= kStage
      const int mid = (c1 + hi + 1) >> 1;
      if (s_off[mid] - base <= kStage) c1 = mid;
      else hi = mid - 1;
    }
    {
      constexpr int W = (int)(sizeof(T) / sizeof(double));
      const double* __restrict__ gSw = reinterpret_cast<const double*>(gS);
      double* stw = reinterpret_cast<double*>(stage);
      const int total = (s_off[c1] - base) * W;
      for (int w0 = tid; w0 < total; w0 += kIntBatch * (int)blockDim.x) {
        double buf[kIntBatch];
#pragma unroll
        for (int u = 0; u < kIntBatch; ++u) {
          const int w = w0 + u * (int)blockDim.x;
          if (w < total) {
            const int e = w / W;
            int c = c0;   // the factor holding entry e: last s_off[c] - base <= e
            for (int hi = c1 - 1; c < hi;) {
              const int mid = (c + hi + 1) >> 1;
              if (s_off[mid] - base <= e) c = mid;
              else hi = mid - 1;
            }
            const int rl = s_rank[c - 1], ap = pad(rl), el = e - (s_off[c] - base);
            const int k = el / ap, a = el - k * ap;
            buf[u] = a < rl ? gSw[((size_t)c * R * R + (size_t)a * R + k) * W + (w - e * W)] : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < kIntBatch; ++u) {
          const int w = w0 + u * (int)blockDim.x;
          if (w < total) stw[w] = buf[u];
        }
      }
      __syncthreads();
    }
    // the chain itself runs in wave 0 alone: lane k owns column k of every staged
    // S_c (r <= 64) and v ping-pongs between two LDS vectors with wave-level
    // ordering only (all 64 entries written, zero above the rank).  A factor's
    // rank and place are read one factor ahead; a block of its column (contiguous,
    // zero-padded) and of v (a broadcast) are read at once, and v[a] S_c(a, k) is
    // summed in four interleaved partial sums (a = 0, 4, 8, .. in the first).
    // Lanes above the rank read the last column and are zeroed after.  Every 16
    // factors v is brought back near 1 by an exact power of two, so long chains
    // (up to a thousand modes) stay in the double range
    if (tid < kWave) {
      int rl = s_rank[c0 - 1];
      int rr = (c0 <= m - 2) ? s_rank[c0] : 1, off = 0;
      for (int c = c0; c < c1; ++c) {
        const int rrn = (c + 1 <= m - 2) ? s_rank[c + 1] : 1;
        const int offn = s_off[c + 1] - base;
        const T* colp = stage + off + min(tid, rr - 1) * pad(rl);
        T acc[4] = {num<T>(0.0), num<T>(0.0), num<T>(0.0), num<T>(0.0)};
        for (int a0 = 0; a0 < rl; a0 += kChainBlk) {
          T col[kChainBlk], vv[kChainBlk];
#pragma unroll
          for (int u = 0; u < kChainBlk; ++u) {
            col[u] = colp[a0 + u];
            vv[u] = v[a0 + u];
          }
#pragma unroll
          for (int u = 0; u < kChainBlk; ++u) acc[u & 3] = n_mad(vv[u], col[u], acc[u & 3]);
        }
        T s = n_add(n_add(acc[0], acc[1]), n_add(acc[2], acc[3]));
        if (tid >= rr) s = num<T>(0.0);
        if ((c & 15) == 0) {
          const double mag = wave_max(fabs(n_hi(s)));
          if (mag > 0.0 && isfinite(mag)) {
            const int e = ilogb(mag) + 1;
            s = n_ldexp(s, -e);
            vexp += e;
          }
        }
        v2[tid] = s;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        T* tmp = v;
        v = v2;
        v2 = tmp;
        rl = rr;
        rr = rrn;
        off = offn;
      }
    } else {
      for (int c = c0; c < c1; ++c) {   // the other waves track which buffer holds v
        T* tmp = v;
        v = v2;
        v2 = tmp;
      }
    }
    __syncthreads();
    c0 = c1;
  }
  if (tid != 0) return;
  // the integral as mantissa * 2^exponent; the folded weights carried 2^wshift per mode
  int e;
  const T value = normalise(v[0], e);
  const int vx = vexp + e - p.wshift * m - st->escale;
  st->max_rank = maxr;
  if (!isfinite(n_hi(value))) st->err_flags |= 1;
  if (init) {   // 1: after the start; 2: after a refresh of the sets (replaces the current entry)
    const int h = init == 2 ? sw0 : 0;
    hist[h] = value;
    p.hexp[h] = vx;
    st->value = n_hi(value);
    st->value_lo = n_lo(value);
    st->vexp = vx;
    return;
  }
  // relative change, the previous value brought to this one's exponent (exact scaling)
  const T prev_al = n_ldexp(prev, prev_exp - vx);
  const double rel = n_hi(value) != 0.0 ? fabs(n_hi(n_div(n_sub(value, prev_al), value))) : __builtin_huge_val();
  const int s = sw0 + 1;
  st->sweeps = s;
  hist[s] = value;
  p.hexp[s] = vx;
  st->value = n_hi(value);
  st->value_lo = n_lo(value);
  st->vexp = vx;
  st->rel = rel;
  st->nacc = nacc;
  int done = 0, reason = TT_RUNNING;
  if (!p.strict && rel <= p.tol && prev_rel <= p.tol) {
    done = 1;
    reason = TT_STOP_CONVERGED;
  } else if (nacc == 0) {
    done = 1;
    reason = below_cap ? TT_STOP_CONVERGED : TT_STOP_RANK_CAP;
  } else if (s >= p.max_sweeps) {
    done = 1;
    reason = TT_STOP_MAX_SWEEPS;
  }
  if (st->err_flags) {   // a numeric failure ends the integral whatever the rule said
    done = 1;
    reason = TT_STOP_ERROR;
  }
  if (done) {
    st->reason = reason;
    st->done = 1;
    signal_done(p);
  }
}

// ------------------------------------------------------------ kernels
template <class T, int FAM, int MAXM, int RMAX>
__global__ __launch_bounds__(kSweepBlock) void k_update(ProbDesc* __restrict__ P,
                                                        const int2* __restrict__ tasks, int init) {
  __shared__ UpdateSmem<T, MAXM, RMAX> sm;
  const int2 tk = tasks[blockIdx.x];
  update_core<T, FAM, MAXM, RMAX>(P[tk.x], tk.y, init, sm);
}

// The ALS refresh of every integral of the job (one workgroup each), followed in
// the same workgroup by the rebuild of its cores on the new sets.
template <int FAM, int MAXM>
union AlsKernelSmem {
  AlsSmem<MAXM> a;
  UpdateSmem<double, MAXM, TT_MAX_RANK> u;
};
template <int FAM, int MAXM>
__global__ __launch_bounds__(kSweepBlock) void k_als(ProbDesc* __restrict__ P) {
  __shared__ AlsKernelSmem<FAM, MAXM> sm;
  const ProbDesc& p = P[blockIdx.x];
  als_refresh<FAM, MAXM>(p, sm.a);
  for (int c = 0; c < p.m; ++c) {
    update_core<double, FAM, MAXM, TT_MAX_RANK>(p, c, 2, sm.u);
    __syncthreads();
  }
}

template <class T>
__global__ __launch_bounds__(kIntBlock) void k_integral(ProbDesc* __restrict__ P, int init) {
  __shared__ IntSmem<T> sm;
  integral_problem<T, chain_block_size<T, 8>()>(P[blockIdx.x], init, sm);
}

template <class T, int MAXM, int RMAX>
union SweepSmem {
  SearchSmem<T, MAXM> s;
  UpdateSmem<T, MAXM, RMAX> u;
  IntSmem<T> i;
};

// One sweep of Alg. 6 in one launch: G workgroups per superblock search it
// together (Alg. 2; G = 1 for the extended precisions), one workgroup per core
// updates the core once both neighbouring searches are done, and the last core
// of an integral to finish runs the quadrature and the stopping rule.  The kinds
// run side by side, so no search waits behind a core update.
//
// Tasks are taken in ticket order (an atomic counter), superblocks first, so a
// core's workgroup only ever waits for searches that workgroups already running
// hold.  The members of a superblock's search (consecutive tickets) wait for each
// other; the running workgroups always hold a prefix of the tickets, every
// cluster inside that prefix completes without waiting on later tickets, and its
// exit frees room for the rest of a cluster cut at the prefix's end.  So every
// wait ends whatever subset of workgroups is resident.  The hand-over from a
// search to its cores is a release fence plus an atomic increment by the search's
// member 0; the core's workgroup polls the counter and takes an acquire fence (an
// L2 invalidate) before it reads the searches' results.  A wait beyond kWaitTicks
// of the constant clock gives up (err_flags 16) and the integral stops with an
// error.  The last workgroup to finish puts the launch counters back to zero for
// the next launch.
//
// The paper-form streaming kernels of rank 8 and 16 (the large integrals, a
// thousand superblocks per launch) are compiled for four waves per SIMD (at most
// 128 VGPRs).  Measured on C_1024 before the row summaries, its sweeps took
// 13.7 ms instead of 15.8.

template <class T, int FAM, int MAXM, int RMAX>
__device__ __forceinline__ void sweep_search(const ProbDesc& p, const int b, const int g, const int G,
                                             SweepSmem<T, MAXM, RMAX>& sm) {
  if (p.st->done) return;
  const int sweep = p.st->sweeps;
  if (!search_bond<T, FAM, MAXM>(p, b, g, G, sm.s)) return;   // members other than 0 are done
  __syncthreads();
  mark(p, sweep, b, 4);
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    atomicAdd(&p.sync[b], 1);
    atomicAdd(&p.sync[b + 1], 1);
  }
  mark(p, sweep, b, 7);
}

template <class T, int FAM, int MAXM, int RMAX>
__device__ __forceinline__ void sweep_core(const ProbDesc& p, const int c, SweepSmem<T, MAXM, RMAX>& sm,
                                           int& s_flag) {
  const int tid = threadIdx.x, m = p.m;
  if (p.st->done || m < 2) return;
  const int sweep = p.st->sweeps, row = p.nbonds + c;
  mark(p, sweep, row, 0);
  if (tid == 0) {
    const int target = (c >= 1 ? 1 : 0) + (c <= m - 2 ? 1 : 0);
    const long long t0 = (long long)wall_clock64();
    int ok = 1;
    while (__hip_atomic_load(&p.sync[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if ((long long)wall_clock64() - t0 > kWaitTicks) {
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (!ok) atomicOr(&p.st->err_flags, 16);
    s_flag = ok;
  }
  __syncthreads();
  mark(p, sweep, row, 8);
  if (s_flag) update_core<T, FAM, MAXM, RMAX>(p, c, 0, sm.u, row);
  __syncthreads();
  mark(p, sweep, row, 5);
  if (tid == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    s_flag = (atomicAdd(&p.sync[m], 1) + 1 == m);
    if (s_flag) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (s_flag) {
    integral_problem<T, chain_block_size<T, RMAX>()>(p, 0, sm.i);
    __syncthreads();
    for (int k = tid; k <= m; k += blockDim.x) p.sync[k] = 0;   // every hand-over of this sweep is done
    mark(p, sweep, row, 6);
  }
  mark(p, sweep, row, 7);
}

// ctr: two launch counters (tickets taken, workgroups finished), zero at launch.
// group: workgroups per superblock search (1..kMaxGroup; 1 for double-double and
// quad-double jobs).  The grid is group * nbond + ncore workgroups; the members of
// one superblock take consecutive tickets.
template <class T, int FAM, int MAXM, int RMAX>
__global__ __launch_bounds__(kSweepBlock, FAM == 0 && MAXM == 0 && RMAX <= 16 ? 4 : 1) void k_sweep(
    ProbDesc* __restrict__ P, const int2* __restrict__ bond_tasks, int nbond, const int2* __restrict__ core_tasks,
    int32_t* __restrict__ ctr, int group) {
  __shared__ SweepSmem<T, MAXM, RMAX> sm;
  __shared__ int s_task, s_flag;
  if (threadIdx.x == 0) s_task = atomicAdd(&ctr[0], 1);
  __syncthreads();
  const int t = s_task;
  if (t < group * nbond) {
    const int2 tk = bond_tasks[t / group];
    sweep_search<T, FAM, MAXM, RMAX>(P[tk.x], tk.y, t % group, group, sm);
  } else {
    const int2 tk = core_tasks[t - group * nbond];
    sweep_core<T, FAM, MAXM, RMAX>(P[tk.x], tk.y, sm, s_flag);
  }
  if (threadIdx.x == 0 && atomicAdd(&ctr[1], 1) + 1 == (int)gridDim.x) {   // every ticket was taken
    __hip_atomic_store(&ctr[0], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ctr[1], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ------------------------------------------------------- standalone eval
template <class T, int FAM, int MAXM>
__global__ __launch_bounds__(kBlock) void k_eval_points(FamilyArgs fa, const T* __restrict__ t,
                                                        const T* __restrict__ w,
                                                        const int32_t* __restrict__ idx,
                                                        int64_t npts, T* __restrict__ out) {
  const int m = fa.m;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < npts;
       q += (int64_t)gridDim.x * blockDim.x) {
    T y[MAXM];
    T W = num<T>(1.0);
#pragma unroll
    for (int k = 0; k < MAXM; ++k) {
      y[k] = num<T>(0.0);
      if (k < m) {
        const int ik = idx[q * m + k];
        y[k] = t[ik];
        W = n_mul(W, w[ik]);
      }
    }
    out[q] = n_mul(W, integrand_fam<T, FAM, MAXM>(fa, y));
  }
}

// Fibre set I_left x [n] x I_right at mode `pos`: one point per lane, the index
// rows and node tables staged in LDS once per workgroup, output ordered
// (alpha, i, beta) with beta fastest.  The grid is bounded and strides over the
// points; each lane advances its (alpha, i, beta) by the fixed stride with
// carries instead of dividing.  EXACT = true compiles the kernel for exactly
// MAXM modes: every guard on the number of modes folds away, and the
// integrand is straight-line code (the same operations in the same order, so
// the same bits as the bucketed kernel).
template <class T, int FAM, int MAXM, bool EXACT = false>
__global__ __launch_bounds__(kBlock) void k_eval_fibers(FamilyArgs fa_in, int n, const T* __restrict__ t,
                                                        const T* __restrict__ w, int pos,
                                                        const int32_t* __restrict__ left, int rl,
                                                        const int32_t* __restrict__ right, int rr,
                                                        T* __restrict__ out) {
  constexpr int LD = MAXM + 1;
  FamilyArgs fa = fa_in;
  if constexpr (EXACT) fa.m = MAXM;
  __shared__ T sLx[TT_MAX_RANK * LD], sRx[TT_MAX_RANK * LD];
  __shared__ T sLw[TT_MAX_RANK], sRw[TT_MAX_RANK];
  __shared__ T st[TT_MAX_NODES], sw[TT_MAX_NODES];
  const int m = fa.m, tid = threadIdx.x, nr = m - pos - 1;
  for (int i = tid; i < n; i += blockDim.x) { st[i] = t[i]; sw[i] = w[i]; }
  __syncthreads();
  for (int a = tid; a < rl; a += blockDim.x) {
    T ww = num<T>(1.0);
    for (int k = 0; k < pos; ++k) {
      const int ik = left[a * pos + k];
      sLx[a * LD + k] = st[ik];
      ww = n_mul(ww, sw[ik]);
    }
    sLw[a] = ww;
  }
  for (int a = tid; a < rr; a += blockDim.x) {
    T ww = num<T>(1.0);
    for (int k = nr - 1; k >= 0; --k) {
      const int ik = right[a * nr + k];
      sRx[a * LD + pos + 1 + k] = st[ik];
      ww = n_mul(sw[ik], ww);
    }
    sRw[a] = ww;
  }
  __syncthreads();
  const uint32_t total = (uint32_t)rl * (uint32_t)n * (uint32_t)rr;
  const uint32_t stride = gridDim.x * blockDim.x;
  uint32_t q = blockIdx.x * blockDim.x + tid;
  if (q >= total) return;
  // position of q and the stride in (alpha, i, beta)
  int be = (int)(q % (uint32_t)rr), i = (int)((q / (uint32_t)rr) % (uint32_t)n), al = (int)(q / ((uint32_t)rr * n));
  const int dbe = (int)(stride % (uint32_t)rr), di = (int)((stride / (uint32_t)rr) % (uint32_t)n);
  const int dal = (int)(stride / ((uint32_t)rr * n));
  for (; q < total; q += stride) {
    T y[MAXM];
#pragma unroll
    for (int k = 0; k < MAXM; ++k) {
      T v = num<T>(0.0);
      if (k < m) {
        v = (k < pos) ? sLx[al * LD + k] : sRx[be * LD + k];
        v = (k == pos) ? st[i] : v;
      }
      y[k] = v;
    }
    const T W = n_mul(n_mul(sLw[al], sw[i]), sRw[be]);
    out[q] = n_mul(W, integrand_fam<T, FAM, MAXM>(fa, y));
    be += dbe;
    int ci = 0;
    if (be >= rr) { be -= rr; ci = 1; }
    i += di + ci;
    int ca = 0;
    if (i >= n) { i -= n; ca = 1; }
    al += dal + ca;
  }
}

constexpr int kFibreNodesPerLane = 4;
constexpr int kRowsMaxModes = 16;   // the row-summary fibre kernel serves exact mode counts up to 16

// The point loop of k_eval_fibers_rows: work item q = (alpha, node chunk, beta),
// beta fastest; the row pair is loaded once per item and the nodes of the chunk
// are taken two at a time.  With P >= 0 the node position is the compile-time P.
template <class T, int MAXM, int P>
__device__ __forceinline__ void fibre_rows_items(int family, int m, int n, int pos_rt, const int32_t* __restrict__ left,
                                                 int rl, const int32_t* __restrict__ right, int rr, T* sL, T* sR,
                                                 const T* st, const T* sw, T* __restrict__ out, uint32_t total,
                                                 uint32_t nchunk, uint32_t stride) {
  constexpr int RS = MAXM + kSumScalars;
  const int pos = P >= 0 ? P : pos_rt;   // a constant where the caller fixed it: every guard folds
  const int nr = m - pos - 1;
  const int tid = threadIdx.x;
  // the left rows of this workgroup's first stride of items (the right rows are all needed)
  const bool one_pass = stride >= total;   // every lane takes at most one item
  const uint32_t q_first = blockIdx.x * blockDim.x;
  const int al_lo = one_pass ? (int)(q_first / ((uint32_t)rr * nchunk)) : 0;
  const int al_hi = one_pass ? min(rl, (int)((min(q_first + blockDim.x, total) - 1) / ((uint32_t)rr * nchunk)) + 1) : rl;
  const int nl = q_first < total ? al_hi - al_lo : 0;
  for (int r = tid; r < nl + rr; r += blockDim.x) {   // one thread per row
    const bool isl = r < nl;
    const int a = isl ? al_lo + r : r - nl;
    T y[MAXM];
    T ww = num<T>(1.0);
#pragma unroll
    for (int k = 0; k < MAXM; ++k) y[k] = num<T>(0.0);
    if (isl) {
#pragma unroll
      for (int k = 0; k < MAXM; ++k)
        if (k < pos) {
          const int ik = left[a * pos + k];
          y[k] = st[ik];
          ww = n_mul(ww, sw[ik]);
        }
      summarise_row<T, MAXM>(family, y, 0, pos, true, ww, sL + a * RS);
    } else {
#pragma unroll
      for (int k = MAXM - 1; k >= 0; --k)            // weights multiplied from the right end
        if (k > pos && k < m) {
          const int ik = right[a * nr + (k - pos - 1)];
          y[k] = st[ik];
          ww = n_mul(sw[ik], ww);
        }
      summarise_row<T, MAXM>(family, y, pos + 1, m, false, ww, sR + a * RS);
    }
  }
  __syncthreads();
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride) {
    const int be = (int)(q % (uint32_t)rr);
    const uint32_t rest = q / (uint32_t)rr;
    const int c = (int)(rest % nchunk), al = (int)(rest / nchunk);
    const T* L = sL + al * RS;
    const T* R = sR + be * RS;
    RowPair<T, MAXM> rp;
    load_row_pair<T, MAXM>(rp, L, R, pos, pos + 1, nr);
    const T WL = L[MAXM + RS_W], WR = R[MAXM + RS_W];
    const int i0 = c * kFibreNodesPerLane;
#pragma unroll
    for (int k = 0; k < kFibreNodesPerLane; k += 2) {   // the node pairs of a lane unrolled: their chains interleave
      const int ia = i0 + k;
      if (ia >= n) break;
      const int ib = ia + 1 < n ? ia + 1 : ia;
      T fa, fb;
      if constexpr (P >= 0)
        ising_joined2_fixed<T, MAXM, P>(family, rp, st[ia], st[ib], fa, fb);
      else
        ising_joined2<T, MAXM>(family, m, pos, rp, st[ia], st[ib], fa, fb);
      out[((size_t)al * n + ia) * rr + be] = n_mul(n_mul(n_mul(WL, sw[ia]), WR), fa);
      if (ia + 1 < n) out[((size_t)al * n + ib) * rr + be] = n_mul(n_mul(n_mul(WL, sw[ib]), WR), fb);
    }
  }
}

// dispatch on the node position: compile-time P for exact mode counts up to 16
template <class T, int MAXM, bool EXACT, int P = 0>
__device__ __forceinline__ void fibre_rows_points(int family, int m, int n, int pos, const int32_t* left, int rl,
                                                  const int32_t* right, int rr, T* sL, T* sR, const T* st,
                                                  const T* sw, T* __restrict__ out, uint32_t total, uint32_t nchunk,
                                                  uint32_t stride) {
  if constexpr (EXACT && MAXM <= 16) {
    if constexpr (P < MAXM) {
      if (pos == P)
        fibre_rows_items<T, MAXM, P>(family, m, n, pos, left, rl, right, rr, sL, sR, st, sw, out, total, nchunk,
                                     stride);
      else
        fibre_rows_points<T, MAXM, EXACT, P + 1>(family, m, n, pos, left, rl, right, rr, sL, sR, st, sw, out,
                                                 total, nchunk, stride);
    }
  } else {
    fibre_rows_items<T, MAXM, -1>(family, m, n, pos, left, rl, right, rr, sL, sR, st, sw, out, total, nchunk,
                                  stride);
  }
}

// The fibre set I_left x [n] x I_right of the paper-form integrands (eqs. c, d,
// e) from row summaries: each left and right row is summarised once per
// workgroup into LDS (the runs inside it, B_d's sums over it, its weight), and
// a lane takes one (alpha, beta) pair and kFibreNodesPerLane consecutive nodes,
// joining the two summaries around each node (ising_joined).  Lanes are ordered
// (alpha, node chunk, beta), beta fastest, so the stores of one node are
// consecutive across lanes.  The grid is bounded and strides over the work
// items.  EXACT = true compiles for exactly MAXM modes.


template <class T, int MAXM, bool EXACT>
__global__ __launch_bounds__(kBlock) void k_eval_fibers_rows(FamilyArgs fa_in, int n, const T* __restrict__ t,
                                                             const T* __restrict__ w, int pos,
                                                             const int32_t* __restrict__ left, int rl,
                                                             const int32_t* __restrict__ right, int rr,
                                                             T* __restrict__ out) {
  constexpr int RS = MAXM + kSumScalars;
  __shared__ T sL[TT_MAX_RANK * RS], sR[TT_MAX_RANK * RS];
  __shared__ T st[TT_MAX_NODES], sw[TT_MAX_NODES];
  const int family = fa_in.family;
  const int m = EXACT ? MAXM : fa_in.m, tid = threadIdx.x;
  for (int i = tid; i < n; i += blockDim.x) { st[i] = t[i]; sw[i] = w[i]; }
  __syncthreads();
  const uint32_t nchunk = (uint32_t)(n + kFibreNodesPerLane - 1) / kFibreNodesPerLane;
  const uint32_t total = (uint32_t)rl * nchunk * (uint32_t)rr;
  const uint32_t stride = gridDim.x * blockDim.x;
  fibre_rows_points<T, MAXM, EXACT>(family, m, n, pos, left, rl, right, rr, sL, sR, st, sw, out, total, nchunk,
                                    stride);
}

// ------------------------------------------------- equal-weight quadrature
// Monte Carlo (eq. mc) and randomly shifted rank-1 lattice rules (eq. qmc),
// Sec. 4.2.  Estimator j = blockIdx.y sums f over its N points: random points
// (kind 0) drawn from the counter-based generator, or x_i = frac(i q / N + s_j)
// for i = 1..N (kind 1), with (i q_k) mod N in exact integer arithmetic.  Each
// workgroup writes one partial sum; k_mc_finish adds them in a fixed order.
// The generating vector (reduced mod N) and the synthetic parameters travel by
// value in the kernel arguments, so the only device buffer besides the output
// is the partial sums.
struct McParams {
  int64_t gen[TT_MAX_REG_MODES];                   // q_k mod N (lattice rules)
  double a[TT_MAX_REG_MODES], b[TT_MAX_REG_MODES];   // synthetic parameters
};

template <int FAM, int MAXM>
__global__ __launch_bounds__(kBlock) void k_mc(FamilyArgs fa, int kind, int64_t N, McParams mp, uint64_t seed,
                                               double* __restrict__ partial) {
  __shared__ double sshift[TT_MAX_REG_MODES];
  __shared__ double sa[TT_MAX_REG_MODES], sb[TT_MAX_REG_MODES];
  __shared__ double red[kBlock / kWave];
  const int j = blockIdx.y, m = fa.m, tid = threadIdx.x;
  if (tid < m) {
    sshift[tid] = uniform_open01(splitmix_at(seed, shift_counter(j, tid)));
    sa[tid] = mp.a[tid];
    sb[tid] = mp.b[tid];
  }
  fa.a = sa;
  fa.b = sb;
  __syncthreads();
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + tid; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    double y[MAXM];
#pragma unroll
    for (int k = 0; k < MAXM; ++k) {
      double v = 0.0;
      if (k < m) {
        if (kind == 0) {
          v = uniform_open01(splitmix_at(seed, mc_counter(j, i, m, k)));
        } else {
          const uint64_t r = ((uint64_t)(i + 1) * (uint64_t)mp.gen[k]) % (uint64_t)N;
          v = (double)r / (double)N + sshift[k];
          v = (v >= 1.0) ? v - 1.0 : v;
        }
      }
      y[k] = v;
    }
    acc += integrand_fam<double, FAM, MAXM>(fa, y);
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
  if ((tid & (kWave - 1)) == 0) red[tid / kWave] = acc;
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) sum += red[w];
    partial[(size_t)j * gridDim.x + blockIdx.x] = sum;
  }
}

// out[j] = (sum of the partial sums of estimator j) / N for j < S, then
// out[S] = their mean and out[S+1] = the relative standard deviation (eq. std).
static __global__ __launch_bounds__(kBlock) void k_mc_finish(const double* __restrict__ partial, int blocks, int S,
                                                             int64_t N, double* __restrict__ out) {
  for (int j = threadIdx.x; j < S; j += blockDim.x) {
    double sum = 0.0;
    for (int b = 0; b < blocks; ++b) sum += partial[(size_t)j * blocks + b];
    out[j] = sum / (double)N;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mean = 0.0;
    for (int j = 0; j < S; ++j) mean += out[j];
    mean = mean / S;
    double var = 0.0;
    for (int j = 0; j < S; ++j) var += (out[j] - mean) * (out[j] - mean);
    var = var / (S - 1);
    out[S] = mean;
    out[S + 1] = sqrt(var) / fabs(mean);
  }
}

}  // namespace ttx
