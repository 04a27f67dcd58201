// Host-side helpers shared by the job API (ttcross.hip) and the serving loop
// (tt_server.hip): the context, problem validation, the per-problem device
// layout, node tables and launch helpers.  Host code only validates, lays out
// and launches; it computes no part of the method.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "tt_kernels.hpp"
#include "tt_launch.hpp"

using namespace ttx;

#define TT_HIP(call)                                    \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) {                             \
      last_hip_error() = e_;                            \
      return TT_EDEVICE;                                \
    }                                                   \
  } while (0)

inline hipError_t& last_hip_error() {
  static thread_local hipError_t e = hipSuccess;
  return e;
}

// kernel kinds timed by the optional event profiler
enum { KK_SWEEP = 0, KK_UPDATE = 1, KK_INTEGRAL = 2, KK_START = 3, KK_GL = 4, KK_EVAL_POINTS = 5,
       KK_EVAL_FIBERS = 6, KK_MC = 7, KK_REFRESH = 8, KK_COUNT = 9 };

struct tt_ctx {
  int device = 0;
  bool profiling = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;   // kind, (start, stop)
  std::vector<hipEvent_t> pool;
  double kernel_ms[KK_COUNT] = {0};
  long long kernel_launches[KK_COUNT] = {0};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::mutex mu;
  struct GL {
    double *t, *w;     // nodes and weights rounded to double
    dd *t2, *w2;       // the same in double-double
    double* ws;        // weights times 2^weight_shift(n), the scale jobs fold in
    dd* ws2;
    qd *t4, *w4, *ws4;  // quad-double tables, made on the first quad-double job of this n
  };
  std::map<int, GL> gl;                            // n -> device tables
  double* params = nullptr;                        // device scratch for synthetic params
  size_t params_cap = 0;
  std::multimap<size_t, void*> arenas;             // freed job arenas kept for reuse
  std::multimap<size_t, void*> pinned;             // freed pinned host blocks kept for reuse
  size_t pinned_cached = 0;
  std::vector<hipEvent_t> ring_pool;               // timing-less events kept for reuse
  double* mc_buf = nullptr;                        // device scratch of tt_mc_integrate
  size_t mc_cap = 0;
  double* scratch = nullptr;                       // this device's static scratch (tt_mc_integrate_noalloc)
  size_t arena_bytes_cached = 0;
  // kernel variants chosen by tt_autotune, per (integrand class, double-double,
  // largest m, largest rank cap): (mode bucket, rank policy, rule ms, tuned ms,
  // search group; 0: the rule's)
  struct Tuned {
    int mbucket, rank_policy;
    double rule_ms, tuned_ms;
    int group;
  };
  std::map<std::array<int, 4>, Tuned> tune;
  std::string tune_path;                           // TTCROSS_TUNE_CACHE, or empty
  bool force_variant = false;                      // tt_autotune's candidate for the next job
  Tuned forced{0, 0, 0.0, 0.0, 0};
  int cus = 0;                                     // compute units of the device
  int search_group = 0;                            // workgroups per superblock search (0: the rule)
};

// Workgroups per superblock search of a job with nbond superblocks and ncore
// cores: as many as keep at most two workgroups per compute unit, capped per
// number type.  Each member adds a record to every exchange, so the split pays
// only where the points are costly: on the headline Ising job (double) 3
// measured fastest, on the double-double job of D_8..D_12 (128 nodes, rank 64)
// 6 (79.7 ms; 3: 99.4, 4: 89.2, 8: 82.9).  tt_autotune may choose another.
constexpr int kRuleGroup = 3;      // double
constexpr int kRuleGroupExt = 6;   // double-double and quad-double
inline int search_group_rule(int cus, int nbond, int ncore, int prec) {
  if (nbond <= 0) return 1;
  const int cap = prec == TT_FP64 ? kRuleGroup : kRuleGroupExt;
  const int g = (2 * cus - ncore) / nbond;
  return g < 1 ? 1 : g > cap ? cap : g;
}
// The rule's group for one sweep launch of a double job whose kernel is sized
// for rank bucket rbucket: the searches of small ranks read little, so the
// exchanges would cost more than the split saves (headline job, median of 15:
// 1 / 2 / 3 workgroups for buckets 8 / 16 / 32 took 2.38 ms, 3 for every bucket
// 2.47 ms).  Extended-precision launches keep the job's group.
inline int search_group_for_bucket(int group_rule, int rbucket, int prec) {
  if (prec != TT_FP64) return group_rule;
  const int g = rbucket <= 8 ? 1 : rbucket <= 16 ? 2 : kRuleGroup;
  return g < group_rule ? g : group_rule;
}

// Arenas of freed jobs are kept by the context (up to this many bytes) and
// handed to later jobs of the same or smaller size, so a stream of jobs does
// not call hipMalloc/hipFree every time.
constexpr size_t kArenaCacheBytes = size_t(4) << 30;

namespace ttx_host {

// Bracket one kernel launch with a pair of events on the context stream.
struct Timed {
  tt_ctx* c;
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  hipEvent_t take() {
    hipEvent_t e = nullptr;
    if (!c->pool.empty()) {
      e = c->pool.back();
      c->pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  Timed(tt_ctx* ctx, int k) : c(ctx), kind(k) {
    if (c->profiling) {
      a = take();
      b = take();
      if (a && b) (void)hipEventRecord(a, c->stream);
    }
  }
  ~Timed() {
    if (c->profiling && a && b) {
      (void)hipEventRecord(b, c->stream);
      c->pending.push_back({kind, {a, b}});
    }
  }
};

inline void drain_profile(tt_ctx* c) {
  if (c->pending.empty()) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto& pe : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pe.second.first, pe.second.second) == hipSuccess) {
      c->kernel_ms[pe.first] += ms;
      c->kernel_launches[pe.first] += 1;
    }
    c->pool.push_back(pe.second.first);
    c->pool.push_back(pe.second.second);
  }
  c->pending.clear();
}

inline int modes_of(const tt_problem& p) {
  switch (p.integrand) {
    case TT_ISING_C: case TT_ISING_D: case TT_ISING_E: return p.d - 1;
    case TT_ISING_C_U: case TT_ISING_D_U: case TT_PROD_EXP: case TT_SUM2_EXP_COS: return p.d;
    default: return -1;
  }
}

inline bool is_synthetic(int f) { return f == TT_PROD_EXP || f == TT_SUM2_EXP_COS; }

inline int fam_of(int f) {
  if (f == TT_ISING_C || f == TT_ISING_D || f == TT_ISING_E) return FAM_PAPER;
  if (f == TT_ISING_C_U || f == TT_ISING_D_U) return FAM_UFORM;
  return FAM_SYNTH;
}

inline tt_status validate(const tt_problem* p) {
  if (!p) return TT_EINVAL;
  const int m = modes_of(*p);
  if (m < 0 || p->d < 1 || m > TT_MAX_MODES) return TT_EINVAL;
  if (p->n_nodes < 1 || p->n_nodes > TT_MAX_NODES) return TT_EINVAL;
  if (p->rank_cap < 1 || p->rank_cap > TT_MAX_RANK) return TT_EINVAL;
  if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return TT_EINVAL;
  if (p->precision != TT_FP64 && p->precision != TT_DD && p->precision != TT_QD) return TT_EINVAL;
  if (p->precision != TT_FP64 && fam_of(p->integrand) != FAM_PAPER) return TT_EINVAL;
  // quad-double: the register kernels of up to TT_QD_MAX_MODES modes and rank TT_QD_MAX_RANK
  if (p->precision == TT_QD && (m > TT_QD_MAX_MODES || p->rank_cap > TT_QD_MAX_RANK)) return TT_EINVAL;
  // beyond the register bucket only the streaming kernels (double, paper form and synthetic)
  if (m > TT_MAX_REG_MODES && (p->precision != TT_FP64 || fam_of(p->integrand) == FAM_UFORM)) return TT_EINVAL;
  if (p->max_sweeps < 0 || p->max_sweeps > 1024) return TT_EINVAL;
  if ((p->stop_rule != TT_STOP_REL2 && p->stop_rule != TT_STOP_STRICT) || p->reserved != 0) return TT_EINVAL;
  if (is_synthetic(p->integrand) && !p->params) return TT_EINVAL;
  // the superblock size r n n r must fit a 32-bit sample index
  const double sb = (double)p->rank_cap * p->n_nodes * p->n_nodes * p->rank_cap;
  if (sb >= 4294967296.0) return TT_EINVAL;
  return TT_OK;
}

inline int max_sweeps_of(const tt_problem& p) { return p.max_sweeps > 0 ? p.max_sweeps : 4 * p.rank_cap; }

// byte layout of one problem inside a job arena
struct Layout {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = (off + 255) & ~size_t(255);
    off = o + bytes;
    return o;
  }
};

struct ProbOffsets {
  size_t Lpar, Lnode, Rpar, Rnode, Lx, Rx, Lw, Rw, F, C, LU, S, rank, piv, scale, log, hist, hexp, start, sync,
      rfl, phase, xch;
  std::vector<int64_t> foff, coff;
};

inline ProbOffsets layout_problem(const tt_problem& p, Layout& L) {
  ProbOffsets o;
  const int m = modes_of(p), n = p.n_nodes, R = p.rank_cap;
  const int nb = m > 1 ? m - 1 : 0;
  const int ms = max_sweeps_of(p);
  // D: bytes of one value of the job's number type; plain doubles use sizeof(double)
  const size_t D = p.precision == TT_QD ? sizeof(qd) : p.precision == TT_DD ? sizeof(dd) : sizeof(double),
               I = sizeof(int32_t);
  o.Lpar = L.take((size_t)nb * R * I);
  o.Lnode = L.take((size_t)nb * R * I);
  o.Rpar = L.take((size_t)nb * R * I);
  o.Rnode = L.take((size_t)nb * R * I);
  o.Lx = L.take((size_t)nb * R * m * D);
  o.Rx = L.take((size_t)nb * R * m * D);
  o.Lw = L.take((size_t)nb * R * D);
  o.Rw = L.take((size_t)nb * R * D);
  int64_t fsz = 0, csz = 0;
  for (int c = 0; c < m; ++c) {
    const int rc = c == 0 ? 1 : R, cc = c == m - 1 ? 1 : R;
    o.foff.push_back(fsz);
    fsz += (int64_t)rc * n * cc;
  }
  for (int b = 0; b < nb; ++b) {
    const int rc = b == 0 ? 1 : R;
    o.coff.push_back(csz);
    csz += (int64_t)R * rc * n;
  }
  o.F = L.take((size_t)fsz * D);
  o.C = L.take((size_t)csz * D);
  o.LU = L.take((size_t)(nb > 0 ? nb : 1) * R * R * D);
  o.S = L.take((size_t)(m > 0 ? m : 1) * R * R * D);
  o.rank = L.take((size_t)(nb > 0 ? nb : 1) * I);
  o.piv = L.take((size_t)(nb > 0 ? nb : 1) * sizeof(PivRec));
  o.scale = L.take((size_t)(nb > 0 ? nb : 1) * sizeof(double));
  o.log = L.take((size_t)ms * (nb > 0 ? nb : 1) * sizeof(PivRec));
  o.hist = L.take((size_t)(ms + 1) * D);
  o.hexp = L.take((size_t)(ms + 1) * I);
  o.start = L.take((size_t)(m > 0 ? m : 1) * I);
  o.sync = L.take((size_t)(m + 1) * I);
  o.rfl = L.take((size_t)(m > 0 ? m : 1) * I);
  o.phase = L.take((size_t)ms * (nb + m > 0 ? nb + m : 1) * kPhases * sizeof(long long));
  o.xch = L.take((size_t)(nb > 0 ? nb : 1) * 2 * kMaxGroup * sizeof(XSlot));
  return o;
}

inline int bucket_m(int m) { return m <= 8 ? 8 : m <= 16 ? 16 : 32; }
// Mode bucket of the sweep kernels of one integrand class and number type
// (must match the instantiations in tt_inst.hip); 0 is the streaming bucket
// for more modes than the register kernels hold.  prec: a tt_precision.
inline int bucket_m_for(int fam, int prec, int m) {
  if (m > TT_MAX_REG_MODES) return 0;
  if (prec == TT_QD) return 16;
  if (fam == FAM_PAPER && prec == TT_FP64) return m <= 4 ? 4 : m <= 8 ? 8 : m <= 10 ? 10 : m <= 12 ? 12 : m <= 16 ? 16 : m <= 24 ? 24 : 32;
  return bucket_m(m);
}
inline int bucket_r(int r) { return r <= 8 ? 8 : r <= 16 ? 16 : r <= 32 ? 32 : 64; }
// Every mode bucket instantiated for a class and number type (tt_inst.hip), the
// streaming bucket 0 last where it exists.
inline std::vector<int> mode_buckets(int fam, int prec) {
  std::vector<int> b;
  if (prec == TT_QD) return {16};
  if (fam == FAM_PAPER && prec == TT_FP64) b = {4, 8, 10, 12, 16, 24, 32};
  else b = {8, 16, 32};
  if (prec == TT_FP64 && fam != FAM_UFORM) b.push_back(0);
  return b;
}
inline std::array<int, 4> tune_key(int fam, int prec, int maxm, int maxR) { return {fam, prec, maxm, maxR}; }
// A mode bucket a job of this class, precision and largest m can launch.
inline bool variant_valid(int fam, int prec, int maxm, int mb) {
  if (mb == 0) return prec == TT_FP64 && fam != FAM_UFORM;
  if (maxm > TT_MAX_REG_MODES || mb < maxm) return false;
  for (int b : mode_buckets(fam, prec))
    if (b == mb) return true;
  return false;
}

inline double four_over_fact(int m) {
  double f = 1.0;
  for (int k = 2; k <= m; ++k) f *= k;
  return 4.0 / f;
}

// Power of two carried by the folded weights of a job: the integer nearest
// log2 n, so that the weights (which sum to 1) have a mean of about 1.
inline int weight_shift(int n) { return std::ilogb((double)n * 1.4142135623730951); }

inline void fill_info(const ProbState& s, tt_info* out) {
  out->sweeps = s.sweeps;
  out->max_rank = s.max_rank;
  out->reason = s.done ? s.reason : TT_RUNNING;
  out->err_flags = s.err_flags;
  out->evals = (int64_t)s.evals;
  out->value = std::ldexp(s.value, s.vexp);
  out->rel_change = s.rel;
  out->value_lo = std::ldexp(s.value_lo, s.vexp);
  out->value_mant = s.value;
  out->value_exp2 = s.vexp;
  out->recomputes = s.recomputes;
  out->value_scale = s.escale;
  out->reserved = 0;
}

// Node tables for n, generated on first use (defined in ttcross.hip).  With
// prec TT_DD or TT_QD the returned pointers are the double-double or
// quad-double tables (as double*);
// with scaled the weights are the rule's times 2^weight_shift(n) (exact).
tt_status gl_table(tt_ctx* ctx, int n, double** t, double** w, int prec = TT_FP64, bool scaled = false);

inline tt_status family_for(tt_ctx* ctx, const tt_problem* p, FamilyArgs* fa) {
  const int m = modes_of(*p);
  fa->family = p->integrand;
  fa->m = m;
  fa->four_over_mfact = four_over_fact(m);
  fa->a = fa->b = nullptr;
  if (is_synthetic(p->integrand)) {
    const size_t need = 2 * (size_t)m * sizeof(double);
    if (need > ctx->params_cap) {
      TT_HIP(hipStreamSynchronize(ctx->stream));
      if (ctx->params) TT_HIP(hipFree(ctx->params));
      ctx->params = nullptr;
      ctx->params_cap = 0;
      TT_HIP(hipMalloc(&ctx->params, need));
      ctx->params_cap = need;
    }
    // synchronous copy: earlier kernels may still read the old parameters
    TT_HIP(hipStreamSynchronize(ctx->stream));
    TT_HIP(hipMemcpy(ctx->params, p->params, need, hipMemcpyHostToDevice));
    fa->a = ctx->params;
    fa->b = ctx->params + m;
  }
  return TT_OK;
}

// Small per-problem tables (core and interpolation-core offsets, synthetic
// parameters) in the layout the descriptor points at.
struct ProbTables {
  size_t foff, coff, par;   // byte offsets inside the table region
};
inline ProbTables take_tables(const tt_problem& p, Layout& L) {
  const int m = modes_of(p);
  ProbTables t;
  t.foff = L.take(sizeof(int64_t) * std::max(m, 1));
  t.coff = L.take(sizeof(int64_t) * std::max(m - 1, 1));
  t.par = L.take(sizeof(double) * 2 * std::max(m, 1));
  return t;
}
// Host image of those tables (img points at the start of the table region).
inline void write_tables(const tt_problem& p, const ProbOffsets& o, const ProbTables& tb, char* img) {
  const int m = modes_of(p);
  if (!o.foff.empty()) std::memcpy(img + tb.foff, o.foff.data(), o.foff.size() * sizeof(int64_t));
  if (!o.coff.empty()) std::memcpy(img + tb.coff, o.coff.data(), o.coff.size() * sizeof(int64_t));
  if (is_synthetic(p.integrand)) {
    std::memcpy(img + tb.par, p.params, m * sizeof(double));
    std::memcpy(img + tb.par + std::max(m, 1) * sizeof(double), p.params + m, m * sizeof(double));
  }
}
// Descriptor of one problem: per-problem arrays at pb (layout o), tables at
// tbase (device address of the table region), node tables t, w.
inline ProbDesc make_desc(const tt_problem& p, const ProbOffsets& o, char* pb, char* tbase, const ProbTables& tb,
                          const double* t, const double* w, int32_t* done_host, ProbState* st,
                          ProbState* st_host, bool profiling) {
  ProbDesc d;
  std::memset(&d, 0, sizeof(d));
  d.family = p.integrand;
  d.m = modes_of(p);
  d.n = p.n_nodes;
  d.R = p.rank_cap;
  d.max_sweeps = max_sweeps_of(p);
  d.nbonds = d.m > 1 ? d.m - 1 : 0;
  d.wshift = weight_shift(p.n_nodes);
  d.strict = p.stop_rule == TT_STOP_STRICT;
  d.tol = p.tol;
  d.four_over_mfact = four_over_fact(d.m);
  d.seed = p.seed;
  d.t = t;
  d.w = w;
  d.pa = (double*)(tbase + tb.par);
  d.pb = d.pa + std::max(d.m, 1);
  d.Lpar = (int32_t*)(pb + o.Lpar);
  d.Lnode = (int32_t*)(pb + o.Lnode);
  d.Rpar = (int32_t*)(pb + o.Rpar);
  d.Rnode = (int32_t*)(pb + o.Rnode);
  d.Lx = (double*)(pb + o.Lx);
  d.Rx = (double*)(pb + o.Rx);
  d.Lw = (double*)(pb + o.Lw);
  d.Rw = (double*)(pb + o.Rw);
  d.F = (double*)(pb + o.F);
  d.Foff = (int64_t*)(tbase + tb.foff);
  d.C = (double*)(pb + o.C);
  d.LU = (double*)(pb + o.LU);
  d.Coff = (int64_t*)(tbase + tb.coff);
  d.S = (double*)(pb + o.S);
  d.rank = (int32_t*)(pb + o.rank);
  d.piv = (PivRec*)(pb + o.piv);
  d.scale = (double*)(pb + o.scale);
  d.log = (PivRec*)(pb + o.log);
  d.hist = (double*)(pb + o.hist);
  d.hexp = (int32_t*)(pb + o.hexp);
  d.start = (int32_t*)(pb + o.start);
  d.sync = (int32_t*)(pb + o.sync);
  d.rfl = (int32_t*)(pb + o.rfl);
  d.done_host = done_host;
  d.st_host = st_host;
  d.phase = profiling ? (long long*)(pb + o.phase) : nullptr;
  d.xch = (XSlot*)(pb + o.xch);
  d.st = st;
  return d;
}

}  // namespace ttx_host
