// Host side of the gfx950 TT cross library: the C ABI of include/ttcross.h.
// The host validates problems, lays out one device arena per job, and
// enqueues the kernels of tt_kernels.hpp; it never computes any part of the
// method itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "tt_host.hpp"

using namespace ttx;
using namespace ttx_host;

struct tt_job {
  tt_ctx* ctx = nullptr;
  int nprob = 0;
  std::vector<tt_problem> probs;
  std::vector<int> modes;
  std::vector<ProbDesc> hdesc;
  void* arena = nullptr;
  size_t bytes = 0;
  ProbDesc* ddesc = nullptr;
  int2* dbond = nullptr;
  int nbond = 0;
  int2* dcore = nullptr;
  int32_t* dctr = nullptr;   // the sweep kernel's launch counters (in the table region, zero at upload)
  int ncore = 0;
  int maxm = 0, maxR = 1;
  int fam = 3;            // integrand class the job's kernels are specialised for
  bool dd = false;        // double-double job
  bool qd = false;        // quad-double job
  int prec = TT_FP64;     // the job's tt_precision
  bool full_bucket = false;   // sweeps were enqueued for graph capture: size kernels for the rank caps
  int mbucket = 0;            // mode bucket of the job's kernels (the rule's, or a tuned one)
  int rank_policy = 0;        // 1: every sweep kernel sized for the rank caps (tuned)
  int group = 1;              // workgroups per superblock search (the rule's: its largest)
  bool group_ruled = false;   // the group is the rule's (not fixed by the context or tuned)
  std::vector<std::pair<double*, double*>> gl64;   // per integral: the double node tables
  int launched = 0;       // sweeps enqueued so far
  int max_sweeps_all = 0;
  ProbState* dstate = nullptr;
  char* pinned = nullptr;                  // pinned host block: done flags, then the table image
  size_t pinned_bytes = 0;
  int32_t* done_host = nullptr;            // pinned, one flag per integral, written by the kernels
  std::vector<hipEvent_t> ring;            // one event per queued sweep (tt_cross_run)
};

namespace ttx_host {
// Node tables for n, generated on first use.  With prec TT_DD or TT_QD the
// returned pointers are the double-double or quad-double tables (reinterpreted
// as double*); the quad-double ones are made on their first request.
tt_status gl_table(tt_ctx* ctx, int n, double** t, double** w, int prec, bool scaled) {
  auto it = ctx->gl.find(n);
  if (it == ctx->gl.end()) {
    tt_ctx::GL g{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // inserted first so that tt_ctx_destroy frees whatever was allocated
    it = ctx->gl.emplace(n, g).first;
    tt_ctx::GL& e = it->second;
    TT_HIP(hipMalloc(&e.t, n * sizeof(double)));
    TT_HIP(hipMalloc(&e.w, n * sizeof(double)));
    TT_HIP(hipMalloc(&e.t2, n * sizeof(dd)));
    TT_HIP(hipMalloc(&e.w2, n * sizeof(dd)));
    TT_HIP(hipMalloc(&e.ws, n * sizeof(double)));
    TT_HIP(hipMalloc(&e.ws2, n * sizeof(dd)));
    {
      Timed tm(ctx, KK_GL);
      hipLaunchKernelGGL(k_gl, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, n, e.t, e.w, e.t2, e.w2,
                         weight_shift(n), e.ws, e.ws2);
    }
    TT_HIP(hipGetLastError());
  }
  tt_ctx::GL& g = it->second;
  if (prec == TT_QD && !g.t4) {
    TT_HIP(hipMalloc(&g.t4, n * sizeof(qd)));
    TT_HIP(hipMalloc(&g.w4, n * sizeof(qd)));
    TT_HIP(hipMalloc(&g.ws4, n * sizeof(qd)));
    {
      Timed tm(ctx, KK_GL);
      hipLaunchKernelGGL(k_gl_qd, dim3((n + 63) / 64), dim3(64), 0, ctx->stream, n, g.t4, g.w4, weight_shift(n), g.ws4);
    }
    TT_HIP(hipGetLastError());
  }
  if (prec == TT_QD) {
    *t = reinterpret_cast<double*>(g.t4);
    *w = reinterpret_cast<double*>(scaled ? g.ws4 : g.w4);
  } else if (prec == TT_DD) {
    *t = reinterpret_cast<double*>(g.t2);
    *w = reinterpret_cast<double*>(scaled ? g.ws2 : g.w2);
  } else {
    *t = g.t;
    *w = scaled ? g.ws : g.w;
  }
  return TT_OK;
}

}  // namespace ttx_host

namespace {

// Pinned host blocks of freed jobs are kept (up to this many bytes) for later jobs.
constexpr size_t kPinnedCacheBytes = size_t(64) << 20;

tt_status pinned_take(tt_ctx* c, size_t bytes, char** out, size_t* got) {
  auto it = c->pinned.lower_bound(bytes);
  if (it != c->pinned.end() && it->first <= 2 * bytes + 4096) {
    *out = (char*)it->second;
    *got = it->first;
    c->pinned_cached -= it->first;
    c->pinned.erase(it);
    return TT_OK;
  }
  if (hipHostMalloc((void**)out, bytes, hipHostMallocDefault) != hipSuccess) return TT_ENOMEM;
  *got = bytes;
  return TT_OK;
}

void pinned_give(tt_ctx* c, char* p, size_t bytes) {
  if (!p) return;
  if (c->pinned_cached + bytes <= kPinnedCacheBytes) {
    c->pinned.emplace(bytes, p);
    c->pinned_cached += bytes;
  } else {
    (void)hipHostFree(p);
  }
}

void launch(tt_job* j, int what, int rb) {
  // the rule's group depends on the launch's rank bucket; a fixed or tuned one does not
  const int grp = j->group_ruled ? search_group_for_bucket(j->group, rb, j->prec) : j->group;
  LaunchArgs a{j->ddesc,   j->dbond,       j->nbond, j->dcore, j->ncore,
               j->nprob,   j->mbucket,     j->ctx->stream, j->dctr, grp};
  Timed tm(j->ctx, what == LAUNCH_SWEEP   ? KK_SWEEP
                   : what == LAUNCH_START ? KK_START
                   : what == LAUNCH_ALS   ? KK_REFRESH
                                          : KK_UPDATE);
  if (j->dd) {
    launch_paper_dd(a, what, rb);
    return;
  }
  if (j->qd) {
    launch_paper_qd(a, what, rb);
    return;
  }
  switch (j->fam) {
    case FAM_PAPER: launch_paper(a, what, rb); break;
    case FAM_UFORM: launch_uform(a, what, rb); break;
    case FAM_SYNTH: launch_synth(a, what, rb); break;
    default: launch_any(a, what, rb); break;
  }
}
void enqueue_update(tt_job* j, int, int) { launch(j, LAUNCH_INIT_UPDATE, 8); }
void enqueue_sweep(tt_job* j, int rb) { launch(j, LAUNCH_SWEEP, rb); }

tt_status enqueue_sweeps(tt_job* j, int n_sweeps) {
  for (int s = 0; s < n_sweeps; ++s) {
    if (j->launched >= j->max_sweeps_all) break;
    const bool caps = j->full_bucket || j->rank_policy == 1;
    if (j->nbond > 0) enqueue_sweep(j, bucket_r(caps ? j->maxR : std::min(j->maxR, j->launched + 2)));
    ++j->launched;
  }
  TT_HIP(hipGetLastError());
  return TT_OK;
}

// Fill the infos; TT_ENUMERIC if an integral stopped on a numeric error, else
// TT_CONVERGED once every integral has stopped.
tt_status sweep_status(const std::vector<ProbState>& st, int nprob, tt_info* info) {
  bool all = true, failed = false;
  for (int k = 0; k < nprob; ++k) {
    if (info) fill_info(st[k], &info[k]);
    all = all && st[k].done;
    failed = failed || (st[k].done && st[k].reason == TT_STOP_ERROR);
  }
  return failed ? TT_ENUMERIC : all ? TT_CONVERGED : TT_NOT_CONVERGED;
}

tt_status read_states(tt_job* j, std::vector<ProbState>& st) {
  st.resize(j->nprob);
  TT_HIP(hipMemcpyAsync(st.data(), j->dstate, sizeof(ProbState) * j->nprob, hipMemcpyDeviceToHost,
                        j->ctx->stream));
  TT_HIP(hipStreamSynchronize(j->ctx->stream));
  return TT_OK;
}


}  // namespace

namespace {
template <int MAXM>
void eval_points_m(tt_ctx* ctx, bool use_dd, dim3 grid, dim3 block, const FamilyArgs& fa, const double* t,
                   const double* w, const int32_t* d_idx, int64_t npts, double* d_out) {
  if (use_dd)
    hipLaunchKernelGGL((k_eval_points<dd, FAM_PAPER, MAXM>), grid, block, 0, ctx->stream, fa,
                       reinterpret_cast<const dd*>(t), reinterpret_cast<const dd*>(w), d_idx, npts,
                       reinterpret_cast<dd*>(d_out));
  else
    hipLaunchKernelGGL((k_eval_points<double, FAM_ANY, MAXM>), grid, block, 0, ctx->stream, fa, t, w, d_idx,
                       npts, d_out);
}

template <class T, int FAM, int MAXM, bool EXACT = false>
void eval_fibers_k(tt_ctx* ctx, dim3 grid, dim3 block, const FamilyArgs& fa, int n, const double* t,
                   const double* w, int pos, const int32_t* d_left, int r_left, const int32_t* d_right,
                   int r_right, double* d_out) {
  hipLaunchKernelGGL((k_eval_fibers<T, FAM, MAXM, EXACT>), grid, block, 0, ctx->stream, fa, n,
                     reinterpret_cast<const T*>(t), reinterpret_cast<const T*>(w), pos, d_left, r_left,
                     d_right, r_right, reinterpret_cast<T*>(d_out));
}

// The paper form from row summaries (k_eval_fibers_rows).
template <class T, int MAXM, bool EXACT>
void eval_fibers_rows(tt_ctx* ctx, dim3 grid, dim3 block, const FamilyArgs& fa, int n, const double* t,
                      const double* w, int pos, const int32_t* d_left, int r_left, const int32_t* d_right,
                      int r_right, double* d_out) {
  hipLaunchKernelGGL((k_eval_fibers_rows<T, MAXM, EXACT>), grid, block, 0, ctx->stream, fa, n,
                     reinterpret_cast<const T*>(t), reinterpret_cast<const T*>(w), pos, d_left, r_left, d_right,
                     r_right, reinterpret_cast<T*>(d_out));
}

// Paper form in double: one kernel per exact number of modes (1..TT_MAX_REG_MODES).
template <int M>
void eval_fibers_exact(tt_ctx* ctx, int m, dim3 grid, dim3 block, const FamilyArgs& fa, int n, const double* t,
                       const double* w, int pos, const int32_t* d_left, int r_left, const int32_t* d_right,
                       int r_right, double* d_out) {
  if constexpr (M <= TT_MAX_REG_MODES) {
    if (m == M) {
      if constexpr (M <= kRowsMaxModes)
        eval_fibers_rows<double, M, true>(ctx, grid, block, fa, n, t, w, pos, d_left, r_left, d_right, r_right,
                                          d_out);
      else
        eval_fibers_k<double, FAM_PAPER, M, true>(ctx, grid, block, fa, n, t, w, pos, d_left, r_left, d_right,
                                                  r_right, d_out);
    }
    else
      eval_fibers_exact<M + 1>(ctx, m, grid, block, fa, n, t, w, pos, d_left, r_left, d_right, r_right, d_out);
  }
}

template <class T, int FAM>
void eval_fibers_f(tt_ctx* ctx, int mb, dim3 grid, dim3 block, const FamilyArgs& fa, int n, const double* t,
                   const double* w, int pos, const int32_t* d_left, int r_left, const int32_t* d_right,
                   int r_right, double* d_out) {
  switch (mb) {
    case 8: eval_fibers_k<T, FAM, 8>(ctx, grid, block, fa, n, t, w, pos, d_left, r_left, d_right, r_right, d_out); break;
    case 16: eval_fibers_k<T, FAM, 16>(ctx, grid, block, fa, n, t, w, pos, d_left, r_left, d_right, r_right, d_out); break;
    default: eval_fibers_k<T, FAM, 32>(ctx, grid, block, fa, n, t, w, pos, d_left, r_left, d_right, r_right, d_out); break;
  }
}

// Validation and kernel arguments shared by the two Monte Carlo entry points:
// the integrand class's FamilyArgs (synthetic parameters are set in-kernel from
// the by-value McParams), the generating vector reduced mod N, and the number of
// workgroups per estimator.
tt_status mc_setup(tt_ctx* ctx, const tt_problem* p, int32_t kind, int64_t n_points, int32_t n_sets,
                   const int64_t* gen, FamilyArgs* fa, McParams* mp, int* blocks) {
  if (!ctx || validate(p) != TT_OK || p->precision != TT_FP64 || modes_of(*p) > TT_MAX_REG_MODES)
    return TT_EINVAL;
  if (kind != TT_MC_RANDOM && kind != TT_MC_LATTICE) return TT_EINVAL;
  if (n_points < 1 || n_points >= (int64_t(1) << 31) || n_sets < 2 || n_sets > 4096) return TT_EINVAL;
  if (kind == TT_MC_LATTICE && !gen) return TT_EINVAL;
  const int m = modes_of(*p);
  if (m < 1) return TT_EINVAL;
  fa->family = p->integrand;
  fa->m = m;
  fa->four_over_mfact = four_over_fact(m);
  fa->a = fa->b = nullptr;
  std::memset(mp, 0, sizeof(*mp));
  for (int k = 0; k < m; ++k) {
    if (kind == TT_MC_LATTICE) mp->gen[k] = ((gen[k] % n_points) + n_points) % n_points;
    if (is_synthetic(p->integrand)) {
      mp->a[k] = p->params[k];
      mp->b[k] = p->params[m + k];
    }
  }
  *blocks = (int)std::min<int64_t>((n_points + kBlock - 1) / kBlock, 256);
  return TT_OK;
}

// Enqueue the estimators (partial sums into `partial`, S x blocks) and the
// finish (estimates, mean and relative error into `out`, S + 2) on the stream.
void mc_launch(tt_ctx* ctx, const tt_problem* p, int kind, int64_t n_points, int n_sets, const FamilyArgs& fa,
               const McParams& mp, int blocks, double* partial, double* out) {
  const dim3 grid((unsigned)blocks, (unsigned)n_sets), block(kBlock);
  const int fam = fam_of(p->integrand), mb = bucket_m(fa.m);
#define TT_MC(F, M) \
  hipLaunchKernelGGL((k_mc<F, M>), grid, block, 0, ctx->stream, fa, kind, n_points, mp, p->seed, partial)
#define TT_MC_M(F)               \
  switch (mb) {                  \
    case 8: TT_MC(F, 8); break;   \
    case 16: TT_MC(F, 16); break; \
    default: TT_MC(F, 32); break; \
  }
  if (fam == FAM_PAPER) { TT_MC_M(FAM_PAPER) }
  else if (fam == FAM_UFORM) { TT_MC_M(FAM_UFORM) }
  else { TT_MC_M(FAM_SYNTH) }
#undef TT_MC_M
#undef TT_MC
  hipLaunchKernelGGL(k_mc_finish, dim3(1), block, 0, ctx->stream, partial, blocks, n_sets, n_points, out);
}

// Scratch of tt_mc_integrate_noalloc: the partial sums of one call in a static
// device array, so that the entry point allocates nothing.  Every GPU the
// library runs on holds its own copy until the process ends; host code must use
// the address hipGetSymbolAddress returns for the device (kept per device
// below, looked up by tt_ctx_create), never this name.
static __device__ __align__(256) double scratch[TT_MC_NOALLOC_MAX_PARTIALS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (which must be `device`).
tt_status scratch_address(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return TT_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      last_hip_error() = e;
      return TT_EDEVICE;
    }
    g_scratch_ptr[device] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return TT_OK;
}
}  // namespace

// ---------------------------------------------------------------- autotuning
// Cache file: one key per line, "class precision max_modes max_rank mode_bucket
// rank_policy rule_ms tuned_ms search_group" (a line without the last field reads
// as search group 0, the rule's); lines starting with '#' are comments.  Entries
// that name a variant the key cannot launch are ignored.
static void tune_load(tt_ctx* c) {
  FILE* f = std::fopen(c->tune_path.c_str(), "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    int fam, prec, maxm, maxR, mb, pol, grp = 0;
    double rule_ms, tuned_ms;
    const int got = std::sscanf(line, "%d %d %d %d %d %d %lf %lf %d", &fam, &prec, &maxm, &maxR, &mb, &pol, &rule_ms,
                                &tuned_ms, &grp);
    if (got != 8 && got != 9) continue;
    if (fam < FAM_PAPER || fam > FAM_ANY || prec < TT_FP64 || prec > TT_QD || (pol != 0 && pol != 1) ||
        !variant_valid(fam, prec, maxm, mb) || grp < 0 || grp > kMaxGroup)
      continue;
    c->tune[tune_key(fam, prec, maxm, maxR)] = tt_ctx::Tuned{mb, pol, rule_ms, tuned_ms, grp};
  }
  std::fclose(f);
}

static tt_status tune_save(tt_ctx* c) {
  if (c->tune_path.empty()) return TT_OK;
  const std::string tmp = c->tune_path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return TT_EDEVICE;
  std::fprintf(f,
               "# ttcross kernel variants: class precision max_modes max_rank mode_bucket rank_policy rule_ms tuned_ms "
               "search_group\n");
  for (const auto& e : c->tune)
    std::fprintf(f, "%d %d %d %d %d %d %.6f %.6f %d\n", e.first[0], e.first[1], e.first[2], e.first[3],
                 e.second.mbucket, e.second.rank_policy, e.second.rule_ms, e.second.tuned_ms, e.second.group);
  const bool ok = std::fclose(f) == 0;
  if (!ok || std::rename(tmp.c_str(), c->tune_path.c_str()) != 0) return TT_EDEVICE;
  return TT_OK;
}

extern "C" {

const char* tt_status_string(tt_status s) {
  switch (s) {
    case TT_OK: return "TT_OK";
    case TT_CONVERGED: return "TT_CONVERGED";
    case TT_NOT_CONVERGED: return "TT_NOT_CONVERGED";
    case TT_PENDING: return "TT_PENDING";
    case TT_EINVAL: return "TT_EINVAL: invalid argument";
    case TT_ENOMEM: return "TT_ENOMEM: out of device memory";
    case TT_EDEVICE: return "TT_EDEVICE: HIP runtime error";
    case TT_ENUMERIC: return "TT_ENUMERIC: non-finite or singular values";
  }
  return "unknown tt_status";
}

tt_status tt_ctx_create(int device, void* hip_stream, tt_ctx** out) {
  if (!out) return TT_EINVAL;
  int count = 0;
  TT_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return TT_EINVAL;
  TT_HIP(hipSetDevice(device));
  tt_ctx* c = new (std::nothrow) tt_ctx;
  if (!c) return TT_ENOMEM;
  c->device = device;
  if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
    delete c;
    return TT_EDEVICE;
  }
  if (scratch_address(device, &c->scratch) != TT_OK) {
    delete c;
    return TT_EDEVICE;
  }
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      delete c;
      return TT_EDEVICE;
    }
    c->own_stream = true;
  }
  if (const char* path = std::getenv("TTCROSS_TUNE_CACHE")) {
    c->tune_path = path;
    tune_load(c);
  }
  *out = c;
  return TT_OK;
}

void tt_ctx_destroy(tt_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  for (auto& kv : c->gl) {
    hipFree(kv.second.t);
    hipFree(kv.second.w);
    hipFree(kv.second.t2);
    hipFree(kv.second.w2);
    hipFree(kv.second.ws);
    hipFree(kv.second.ws2);
    if (kv.second.t4) hipFree(kv.second.t4);
    if (kv.second.w4) hipFree(kv.second.w4);
    if (kv.second.ws4) hipFree(kv.second.ws4);
  }
  if (c->params) hipFree(c->params);
  for (auto& kv : c->arenas) hipFree(kv.second);
  for (auto& kv : c->pinned) hipHostFree(kv.second);
  for (hipEvent_t e : c->ring_pool) hipEventDestroy(e);
  if (c->mc_buf) hipFree(c->mc_buf);
  for (auto& pe : c->pending) {
    hipEventDestroy(pe.second.first);
    hipEventDestroy(pe.second.second);
  }
  for (hipEvent_t e : c->pool) hipEventDestroy(e);
  if (c->own_stream) hipStreamDestroy(c->stream);
  delete c;
}

tt_status tt_ctx_profile(tt_ctx* c, int32_t enable) {
  if (!c) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(c->mu);
  drain_profile(c);
  c->profiling = enable != 0;
  for (int k = 0; k < KK_COUNT; ++k) {
    c->kernel_ms[k] = 0.0;
    c->kernel_launches[k] = 0;
  }
  return TT_OK;
}

tt_status tt_ctx_set_search_group(tt_ctx* c, int32_t group) {
  if (!c || group < 0 || group > kMaxGroup) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(c->mu);
  c->search_group = group;
  return TT_OK;
}

tt_status tt_ctx_kernel_time(tt_ctx* c, int32_t kind, int64_t* launches, double* total_ms) {
  if (!c || kind < 0 || kind >= KK_COUNT || !launches || !total_ms) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(c->mu);
  drain_profile(c);
  *launches = c->kernel_launches[kind];
  *total_ms = c->kernel_ms[kind];
  return TT_OK;
}

tt_status tt_autotune(tt_ctx* ctx, const tt_problem* problems, int32_t count, int32_t reps, tt_tune_result* out) {
  if (!ctx || !problems || count < 1 || reps < 1 || !out) return TT_EINVAL;
  int fam = FAM_ANY, maxm = 0, maxR = 1;
  for (int k = 0; k < count; ++k) {
    if (validate(&problems[k]) != TT_OK || problems[k].precision != problems[0].precision) return TT_EINVAL;
    const int fk = fam_of(problems[k].integrand);
    fam = (k == 0) ? fk : (fam == fk ? fk : FAM_ANY);
    maxm = std::max(maxm, modes_of(problems[k]));
    maxR = std::max(maxR, problems[k].rank_cap);
  }
  const int prec = problems[0].precision;
  const int rule_mb = bucket_m_for(fam, prec, maxm);
  // (mode bucket, rank policy, search group; 0: the rule's)
  std::vector<std::array<int, 3>> cands{{rule_mb, 0, 0}, {rule_mb, 1, 0}};
  for (int mb : mode_buckets(fam, prec))
    if (mb != rule_mb && variant_valid(fam, prec, maxm, mb)) {
      cands.push_back({mb, 0, 0});
      cands.push_back({mb, 1, 0});
    }
  if (ctx->search_group == 0)
    for (int g : {1, 2, 4, 6})   // the rule's variant with other search groups
      cands.push_back({rule_mb, 0, g});
  std::vector<tt_info> ref(count), got(count);
  auto same = [&](const std::vector<tt_info>& a, const std::vector<tt_info>& b) {
    for (int k = 0; k < count; ++k)
      if (a[k].value_mant != b[k].value_mant || a[k].value_exp2 != b[k].value_exp2 || a[k].value_lo != b[k].value_lo ||
          a[k].sweeps != b[k].sweeps || a[k].evals != b[k].evals || a[k].reason != b[k].reason)
        return false;
    return true;
  };
  double best_ms = 0.0, rule_ms = 0.0;
  int best = -1, matching = 0;
  for (size_t c = 0; c < cands.size(); ++c) {
    std::vector<double> ms;
    bool match = true;
    for (int r = 0; r < reps && match; ++r) {
      ctx->forced = tt_ctx::Tuned{cands[c][0], cands[c][1], 0.0, 0.0, cands[c][2]};
      ctx->force_variant = true;
      if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
        ctx->force_variant = false;
        return TT_EDEVICE;
      }
      const auto t0 = std::chrono::steady_clock::now();
      tt_job* j = nullptr;
      tt_status s = tt_cross_init(ctx, problems, count, &j);
      ctx->force_variant = false;
      if (s == TT_OK) s = tt_cross_run(j, got.data());
      const auto t1 = std::chrono::steady_clock::now();
      if (j) tt_cross_free(j);
      if (s < 0 && c == 0) return s;          // the rule's own run failed: that is the job's error
      if (s < 0) {
        match = false;
        break;
      }
      ms.push_back(std::chrono::duration<double, std::milli>(t1 - t0).count());
      if (c == 0 && r == 0) ref = got;
      else match = same(ref, got);
    }
    if (!match) continue;
    ++matching;
    std::sort(ms.begin(), ms.end());
    const double med = ms[ms.size() / 2];
    if (c == 0) rule_ms = med;
    if (best < 0 || med < best_ms) {
      best = (int)c;
      best_ms = med;
    }
  }
  ctx->tune[tune_key(fam, prec, maxm, maxR)] =
      tt_ctx::Tuned{cands[best][0], cands[best][1], rule_ms, best_ms, cands[best][2]};
  out->mode_bucket = cands[best][0];
  out->rank_policy = cands[best][1];
  out->rule_mode_bucket = rule_mb;
  out->candidates = (int32_t)cands.size();
  out->matching = matching;
  out->search_group = cands[best][2];
  out->rule_ms = rule_ms;
  out->tuned_ms = best_ms;
  return tune_save(ctx);
}

tt_status tt_ctx_synchronize(tt_ctx* c) {
  if (!c) return TT_EINVAL;
  TT_HIP(hipStreamSynchronize(c->stream));
  return TT_OK;
}

size_t tt_job_footprint(const tt_problem* p) {
  if (validate(p) != TT_OK) return 0;
  Layout L;
  layout_problem(*p, L);
  L.take(sizeof(ProbState));
  L.take(sizeof(ProbDesc));
  return L.off;
}

tt_status tt_cross_init(tt_ctx* ctx, const tt_problem* problems, int32_t count, tt_job** out) {
  if (!ctx || !problems || count < 1 || !out) return TT_EINVAL;
  for (int k = 0; k < count; ++k) {
    if (validate(&problems[k]) != TT_OK) return TT_EINVAL;
    if (problems[k].precision != problems[0].precision) return TT_EINVAL;
  }
  std::lock_guard<std::mutex> lock(ctx->mu);
  TT_HIP(hipSetDevice(ctx->device));
  tt_job* j = new (std::nothrow) tt_job;
  if (!j) return TT_ENOMEM;
  j->ctx = ctx;
  j->nprob = count;
  j->probs.assign(problems, problems + count);
  j->prec = problems[0].precision;
  j->dd = j->prec == TT_DD;
  j->qd = j->prec == TT_QD;
  // Gauss--Legendre tables are computed once per node count and shared by all jobs of the context
  std::vector<std::pair<double*, double*>> gl(count);
  j->gl64.resize(count);
  for (int k = 0; k < count; ++k) {
    tt_status s = gl_table(ctx, problems[k].n_nodes, &j->gl64[k].first, &j->gl64[k].second);
    if (s == TT_OK) s = gl_table(ctx, problems[k].n_nodes, &gl[k].first, &gl[k].second, j->prec, true);
    if (s != TT_OK) {
      delete j;
      return s;
    }
  }
  // ---- layout: a small table region (uploaded in one copy), then the bulk per-problem state
  std::vector<int2> bond_tasks, core_tasks;
  for (int k = 0; k < count; ++k) {
    const int m = modes_of(problems[k]);
    j->modes.push_back(m);
    j->maxm = std::max(j->maxm, m);
    j->maxR = std::max(j->maxR, problems[k].rank_cap);
    j->max_sweeps_all = std::max(j->max_sweeps_all, max_sweeps_of(problems[k]));
    const int fk = fam_of(problems[k].integrand);
    j->fam = (k == 0) ? fk : (j->fam == fk ? fk : FAM_ANY);
    if (m >= 2) {
      for (int b = 0; b < m - 1; ++b) bond_tasks.push_back(make_int2(k, b));
      for (int c = 0; c < m; ++c) core_tasks.push_back(make_int2(k, c));
    }
  }
  // kernel variant: the rule's, a tuned one recorded in the context, or tt_autotune's candidate
  j->mbucket = bucket_m_for(j->fam, j->prec, j->maxm);
  int tuned_group = 0;
  if (ctx->force_variant) {
    j->mbucket = ctx->forced.mbucket;
    j->rank_policy = ctx->forced.rank_policy;
    tuned_group = ctx->forced.group;
  } else {
    auto t = ctx->tune.find(tune_key(j->fam, j->prec, j->maxm, j->maxR));
    if (t != ctx->tune.end() && variant_valid(j->fam, j->prec, j->maxm, t->second.mbucket)) {
      j->mbucket = t->second.mbucket;
      j->rank_policy = t->second.rank_policy;
      tuned_group = t->second.group;
    }
  }
  Layout L;
  const size_t st_off = L.take(sizeof(ProbState) * count);
  const size_t desc_off = L.take(sizeof(ProbDesc) * count);
  const size_t bond_off = L.take(sizeof(int2) * (bond_tasks.size() + 1));
  const size_t core_off = L.take(sizeof(int2) * (core_tasks.size() + 1));
  const size_t ctr_off = L.take(2 * sizeof(int32_t));
  std::vector<ProbOffsets> offs;
  std::vector<ProbTables> tabs;
  for (int k = 0; k < count; ++k) {
    Layout pl;
    offs.push_back(layout_problem(problems[k], pl));
    tabs.push_back(take_tables(problems[k], L));
  }
  const size_t table_bytes = L.take(0);
  std::vector<size_t> bases;
  for (int k = 0; k < count; ++k) {
    Layout pl;
    layout_problem(problems[k], pl);
    bases.push_back(L.take(pl.off));
  }
  j->bytes = L.off;
  // ---- device arena: reuse a cached one of a suitable size, else allocate
  auto it = ctx->arenas.lower_bound(j->bytes);
  if (it != ctx->arenas.end() && it->first <= 2 * j->bytes + (size_t(1) << 20)) {
    j->arena = it->second;
    j->bytes = it->first;
    ctx->arena_bytes_cached -= it->first;
    ctx->arenas.erase(it);
  } else if (hipMalloc(&j->arena, j->bytes) != hipSuccess) {
    delete j;
    return TT_ENOMEM;
  }
  char* base = (char*)j->arena;
  auto fail = [&](tt_status s) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(j->arena);
    if (j->pinned) (void)hipHostFree(j->pinned);
    delete j;
    return s;
  };
  j->dstate = (ProbState*)(base + st_off);
  j->ddesc = (ProbDesc*)(base + desc_off);
  j->dbond = (int2*)(base + bond_off);
  j->dcore = (int2*)(base + core_off);
  j->dctr = (int32_t*)(base + ctr_off);
  j->nbond = (int)bond_tasks.size();
  j->ncore = (int)core_tasks.size();
  if (ctx->search_group > 0) j->group = ctx->search_group;   // tt_ctx_set_search_group
  else if (tuned_group > 0) j->group = tuned_group;
  else {
    j->group = search_group_rule(ctx->cus, j->nbond, j->ncore, j->prec);
    j->group_ruled = true;
  }
  // one pinned block (reused from the context when possible): done flags, then
  // the host image of the table region, the source of the asynchronous upload
  const size_t flags_bytes = (sizeof(int32_t) * count + 255) & ~size_t(255);
  if (pinned_take(ctx, flags_bytes + table_bytes, &j->pinned, &j->pinned_bytes) != TT_OK) return fail(TT_ENOMEM);
  j->done_host = (int32_t*)j->pinned;
  char* img = j->pinned + flags_bytes;
  std::memset(img, 0, table_bytes);
  for (int k = 0; k < count; ++k) j->done_host[k] = 0;
  for (int k = 0; k < count; ++k) {
    const tt_problem& p = problems[k];
    j->hdesc.push_back(make_desc(p, offs[k], base + bases[k], base, tabs[k], gl[k].first, gl[k].second,
                                 j->done_host + k, j->dstate + k, nullptr, ctx->profiling));
    write_tables(p, offs[k], tabs[k], img);
  }
  std::memcpy(img + desc_off, j->hdesc.data(), sizeof(ProbDesc) * count);
  if (!bond_tasks.empty()) std::memcpy(img + bond_off, bond_tasks.data(), sizeof(int2) * bond_tasks.size());
  if (!core_tasks.empty()) std::memcpy(img + core_off, core_tasks.data(), sizeof(int2) * core_tasks.size());
  // one table upload (the host image lives until the job is freed), then the kernels, all in stream order
  if (hipMemcpyAsync(base, img, table_bytes, hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
    return fail(TT_EDEVICE);
  launch(j, LAUNCH_START, 8);
  if (j->ncore > 0) {
    enqueue_update(j, 4, 1);
    Timed tm(ctx, KK_INTEGRAL);
    if (j->qd)
      hipLaunchKernelGGL(k_integral<qd>, dim3(count), dim3(kIntBlock), 0, ctx->stream, j->ddesc, 1);
    else if (j->dd)
      hipLaunchKernelGGL(k_integral<dd>, dim3(count), dim3(kIntBlock), 0, ctx->stream, j->ddesc, 1);
    else
      hipLaunchKernelGGL(k_integral<double>, dim3(count), dim3(kIntBlock), 0, ctx->stream, j->ddesc, 1);
  }
  if (hipGetLastError() != hipSuccess) return fail(TT_EDEVICE);
  std::vector<ProbState> st;
  if (read_states(j, st) != TT_OK) return fail(TT_EDEVICE);
  for (int k = 0; k < count; ++k) {
    if (st[k].err_flags & (1 | 4)) return fail(TT_ENUMERIC);
    if (st[k].done) j->done_host[k] = 1;
  }
  *out = j;
  return TT_OK;
}

tt_status tt_cross_sweep(tt_job* j, int32_t n_sweeps, tt_info* info) {
  if (!j || n_sweeps < 0) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(j->ctx->mu);
  TT_HIP(hipSetDevice(j->ctx->device));
  tt_status s = enqueue_sweeps(j, n_sweeps);
  if (s != TT_OK) return s;
  std::vector<ProbState> st;
  s = read_states(j, st);
  if (s != TT_OK) return s;
  return sweep_status(st, j->nprob, info);
}

tt_status tt_cross_refresh(tt_job* j, tt_info* info) {
  if (!j || j->prec != TT_FP64) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(j->ctx->mu);
  TT_HIP(hipSetDevice(j->ctx->device));
  if (j->nbond > 0) {
    launch(j, LAUNCH_ALS, 64);
    Timed tm(j->ctx, KK_INTEGRAL);
    hipLaunchKernelGGL(k_integral<double>, dim3(j->nprob), dim3(kIntBlock), 0, j->ctx->stream, j->ddesc, 2);
  }
  TT_HIP(hipGetLastError());
  std::vector<ProbState> st;
  tt_status s = read_states(j, st);
  if (s != TT_OK) return s;
  return sweep_status(st, j->nprob, info);
}

tt_status tt_cross_enqueue(tt_job* j, int32_t n_sweeps) {
  if (!j || n_sweeps < 0) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(j->ctx->mu);
  if (j->ctx->profiling) return TT_EINVAL;   // event pairs would be captured too
  TT_HIP(hipSetDevice(j->ctx->device));
  j->full_bucket = true;                      // from now on the host does not know the ranks
  if (j->nbond > 0)
    for (int s = 0; s < n_sweeps; ++s) enqueue_sweep(j, bucket_r(j->maxR));
  j->launched += n_sweeps;
  TT_HIP(hipGetLastError());
  return TT_OK;
}

// Sweeps are queued kQueued ahead of the last one known complete; after each
// completed sweep the host reads the pinned done flags that the kernels write,
// and stops queueing once every integral has stopped.  Sweeps still queued for
// stopped integrals return at once.
static const int kQueued = 2;

tt_status tt_cross_run(tt_job* j, tt_info* info) {
  if (!j) return TT_EINVAL;
  {
    std::lock_guard<std::mutex> lock(j->ctx->mu);
    TT_HIP(hipSetDevice(j->ctx->device));
    while ((int)j->ring.size() < kQueued) {
      hipEvent_t e;
      if (!j->ctx->ring_pool.empty()) {
        e = j->ctx->ring_pool.back();
        j->ctx->ring_pool.pop_back();
      } else {
        TT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      }
      j->ring.push_back(e);
    }
    auto all_done = [&]() {
      for (int k = 0; k < j->nprob; ++k)
        if (__atomic_load_n(&j->done_host[k], __ATOMIC_ACQUIRE) == 0) return false;
      return true;
    };
    int queued = 0;   // sweeps queued by this call
    while (j->launched < j->max_sweeps_all && !all_done()) {
      if (queued >= kQueued) {
        TT_HIP(hipEventSynchronize(j->ring[queued % kQueued]));
        if (all_done()) break;
      }
      tt_status s = enqueue_sweeps(j, 1);
      if (s != TT_OK) return s;
      TT_HIP(hipEventRecord(j->ring[queued % kQueued], j->ctx->stream));
      ++queued;
    }
  }
  std::vector<ProbState> st;
  {
    std::lock_guard<std::mutex> lock(j->ctx->mu);
    tt_status s = read_states(j, st);
    if (s != TT_OK) return s;
  }
  return sweep_status(st, j->nprob, info);
}

tt_status tt_batch_run(tt_ctx* ctx, const tt_problem* problems, int32_t count, tt_info* info) {
  if (!info) return TT_EINVAL;
  tt_job* j = nullptr;
  tt_status s = tt_cross_init(ctx, problems, count, &j);
  if (s != TT_OK) return s;
  s = tt_cross_run(j, info);
  tt_cross_free(j);
  return s;
}

tt_status tt_cross_integrate(tt_job* j, double* values, tt_info* info) {
  if (!j || !values) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(j->ctx->mu);
  TT_HIP(hipSetDevice(j->ctx->device));
  std::vector<ProbState> st;
  tt_status s = read_states(j, st);
  if (s != TT_OK) return s;
  for (int k = 0; k < j->nprob; ++k) {
    values[k] = std::ldexp(st[k].value, st[k].vexp);
    if (info) fill_info(st[k], &info[k]);
  }
  return TT_OK;
}

tt_status tt_job_pivot_log(tt_job* j, int32_t k, tt_pivot* log, int64_t capacity, int64_t* written) {
  if (!j || k < 0 || k >= j->nprob || !log || !written) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(j->ctx->mu);
  std::vector<ProbState> st;
  tt_status s = read_states(j, st);
  if (s != TT_OK) return s;
  const ProbDesc& d = j->hdesc[k];
  const int64_t nrec = (int64_t)st[k].sweeps * d.nbonds;
  if (nrec > capacity) return TT_EINVAL;
  if (nrec > 0) TT_HIP(hipMemcpy(log, d.log, nrec * sizeof(PivRec), hipMemcpyDeviceToHost));
  *written = nrec;
  return TT_OK;
}

tt_status tt_job_history(tt_job* j, int32_t k, double* values, double* values_lo, int32_t* exp2,
                         int64_t capacity, int64_t* written) {
  if (!j || k < 0 || k >= j->nprob || !values || !written) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(j->ctx->mu);
  std::vector<ProbState> st;
  tt_status s = read_states(j, st);
  if (s != TT_OK) return s;
  const int64_t nv = st[k].sweeps + 1;
  if (nv > capacity) return TT_EINVAL;
  // the device keeps mantissas and exponents
  std::vector<dd> h(nv);
  std::vector<int32_t> e(nv);
  if (j->qd) {
    std::vector<qd> h4(nv);
    TT_HIP(hipMemcpy(h4.data(), j->hdesc[k].hist, nv * sizeof(qd), hipMemcpyDeviceToHost));
    for (int64_t q = 0; q < nv; ++q) h[q] = dd{h4[q].x0, h4[q].x1};
  } else if (j->dd) {
    TT_HIP(hipMemcpy(h.data(), j->hdesc[k].hist, nv * sizeof(dd), hipMemcpyDeviceToHost));
  } else {
    std::vector<double> h1(nv);
    TT_HIP(hipMemcpy(h1.data(), j->hdesc[k].hist, nv * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t q = 0; q < nv; ++q) h[q] = dd{h1[q], 0.0};
  }
  TT_HIP(hipMemcpy(e.data(), j->hdesc[k].hexp, nv * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int64_t q = 0; q < nv; ++q) {
    const int x = exp2 ? 0 : e[q];
    values[q] = std::ldexp(h[q].hi, x);
    if (values_lo) values_lo[q] = std::ldexp(h[q].lo, x);
    if (exp2) exp2[q] = e[q];
  }
  *written = nv;
  return TT_OK;
}

tt_status tt_job_index_sets(tt_job* j, int32_t k, int32_t* ranks, int32_t* nodes, int64_t capacity,
                            int64_t* written) {
  if (!j || k < 0 || k >= j->nprob || !ranks || !nodes || !written) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(j->ctx->mu);
  TT_HIP(hipStreamSynchronize(j->ctx->stream));
  const ProbDesc& d = j->hdesc[k];
  const int m = d.m, R = d.R, nb = d.nbonds;
  *written = 0;
  if (nb == 0) return TT_OK;
  std::vector<int32_t> rk(nb), lp(nb * R), ln(nb * R), rp(nb * R), rn(nb * R);
  TT_HIP(hipMemcpy(rk.data(), d.rank, nb * sizeof(int32_t), hipMemcpyDeviceToHost));
  TT_HIP(hipMemcpy(lp.data(), d.Lpar, nb * R * sizeof(int32_t), hipMemcpyDeviceToHost));
  TT_HIP(hipMemcpy(ln.data(), d.Lnode, nb * R * sizeof(int32_t), hipMemcpyDeviceToHost));
  TT_HIP(hipMemcpy(rp.data(), d.Rpar, nb * R * sizeof(int32_t), hipMemcpyDeviceToHost));
  TT_HIP(hipMemcpy(rn.data(), d.Rnode, nb * R * sizeof(int32_t), hipMemcpyDeviceToHost));
  int64_t need = 0;
  for (int b = 0; b < nb; ++b) need += (int64_t)rk[b] * m;
  if (need > capacity) return TT_EINVAL;
  // expand (parent, node) chains into full multi-indices
  std::vector<std::vector<std::vector<int32_t>>> left(nb), right(nb);
  for (int b = 0; b < nb; ++b) {
    left[b].resize(rk[b]);
    for (int a = 0; a < rk[b]; ++a) {
      std::vector<int32_t> v;
      if (b > 0) v = left[b - 1][lp[b * R + a]];
      v.push_back(ln[b * R + a]);
      left[b][a] = v;
    }
  }
  for (int b = nb - 1; b >= 0; --b) {
    right[b].resize(rk[b]);
    for (int a = 0; a < rk[b]; ++a) {
      std::vector<int32_t> v{rn[b * R + a]};
      if (b < nb - 1) {
        const auto& tail = right[b + 1][rp[b * R + a]];
        v.insert(v.end(), tail.begin(), tail.end());
      }
      right[b][a] = v;
    }
  }
  int64_t pos = 0;
  for (int b = 0; b < nb; ++b) {
    ranks[b] = rk[b];
    for (int a = 0; a < rk[b]; ++a)
      for (int32_t x : left[b][a]) nodes[pos++] = x;
    for (int a = 0; a < rk[b]; ++a)
      for (int32_t x : right[b][a]) nodes[pos++] = x;
  }
  *written = pos;
  return TT_OK;
}

tt_status tt_job_phase_times(tt_job* j, int32_t k, int64_t* marks, int64_t capacity, int64_t* written,
                             double* clock_mhz) {
  if (!j || k < 0 || k >= j->nprob || !marks || !written || !clock_mhz) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(j->ctx->mu);
  std::vector<ProbState> st;
  tt_status s = read_states(j, st);
  if (s != TT_OK) return s;
  const ProbDesc& d = j->hdesc[k];
  *written = 0;
  int rate_khz = 0;
  TT_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, j->ctx->device));
  *clock_mhz = rate_khz / 1000.0;
  if (!d.phase) return TT_OK;
  const int64_t nrec = (int64_t)st[k].sweeps * (d.nbonds + d.m) * kPhases;
  if (nrec > capacity) return TT_EINVAL;
  if (nrec > 0) TT_HIP(hipMemcpy(marks, d.phase, nrec * sizeof(long long), hipMemcpyDeviceToHost));
  *written = nrec;
  return TT_OK;
}

tt_status tt_job_nodes(tt_job* j, int32_t k, double* t, double* w, double* t_lo, double* w_lo) {
  if (!j || k < 0 || k >= j->nprob || !t || !w) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(j->ctx->mu);
  TT_HIP(hipStreamSynchronize(j->ctx->stream));
  const ProbDesc& d = j->hdesc[k];
  TT_HIP(hipMemcpy(t, j->gl64[k].first, d.n * sizeof(double), hipMemcpyDeviceToHost));
  TT_HIP(hipMemcpy(w, j->gl64[k].second, d.n * sizeof(double), hipMemcpyDeviceToHost));
  if (t_lo || w_lo) {
    const tt_ctx::GL& g = j->ctx->gl.at(d.n);
    std::vector<dd> h(d.n);
    if (t_lo) {
      TT_HIP(hipMemcpy(h.data(), g.t2, d.n * sizeof(dd), hipMemcpyDeviceToHost));
      for (int i = 0; i < d.n; ++i) t_lo[i] = h[i].lo;
    }
    if (w_lo) {
      TT_HIP(hipMemcpy(h.data(), g.w2, d.n * sizeof(dd), hipMemcpyDeviceToHost));
      for (int i = 0; i < d.n; ++i) w_lo[i] = h[i].lo;
    }
  }
  return TT_OK;
}

tt_status tt_job_history_parts(tt_job* j, int32_t k, int32_t parts, double* values, int32_t* exp2,
                               int64_t capacity, int64_t* written) {
  if (!j || k < 0 || k >= j->nprob || parts < 1 || parts > 4 || !values || !exp2 || !written) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(j->ctx->mu);
  std::vector<ProbState> st;
  tt_status s = read_states(j, st);
  if (s != TT_OK) return s;
  const int64_t nv = st[k].sweeps + 1;
  if (nv > capacity) return TT_EINVAL;
  const int np = j->qd ? 4 : j->dd ? 2 : 1;   // components stored per value
  std::vector<double> h((size_t)nv * np);
  TT_HIP(hipMemcpy(h.data(), j->hdesc[k].hist, h.size() * sizeof(double), hipMemcpyDeviceToHost));
  TT_HIP(hipMemcpy(exp2, j->hdesc[k].hexp, nv * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int64_t q = 0; q < nv; ++q)
    for (int c = 0; c < parts; ++c) values[q * parts + c] = c < np ? h[(size_t)q * np + c] : 0.0;
  *written = nv;
  return TT_OK;
}

tt_status tt_job_nodes_parts(tt_job* j, int32_t k, int32_t parts, double* t, double* w) {
  if (!j || k < 0 || k >= j->nprob || parts < 1 || parts > 4 || !t || !w) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(j->ctx->mu);
  TT_HIP(hipStreamSynchronize(j->ctx->stream));
  const ProbDesc& d = j->hdesc[k];
  const tt_ctx::GL& g = j->ctx->gl.at(d.n);
  // the unscaled tables of the job's precision: 1, 2 or 4 components per value
  const int np = j->qd ? 4 : j->dd ? 2 : 1;
  const double* st = j->qd ? (const double*)g.t4 : j->dd ? (const double*)g.t2 : g.t;
  const double* sw = j->qd ? (const double*)g.w4 : j->dd ? (const double*)g.w2 : g.w;
  std::vector<double> ht((size_t)d.n * np), hw((size_t)d.n * np);
  TT_HIP(hipMemcpy(ht.data(), st, ht.size() * sizeof(double), hipMemcpyDeviceToHost));
  TT_HIP(hipMemcpy(hw.data(), sw, hw.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (int i = 0; i < d.n; ++i)
    for (int c = 0; c < parts; ++c) {
      t[i * parts + c] = c < np ? ht[(size_t)i * np + c] : 0.0;
      w[i * parts + c] = c < np ? hw[(size_t)i * np + c] : 0.0;
    }
  return TT_OK;
}

tt_status tt_job_core(tt_job* j, int32_t k, int32_t c, double* F, double* C, int64_t capacity, int32_t* rows,
                      int32_t* cols) {
  if (!j || k < 0 || k >= j->nprob || !F || !rows || !cols) return TT_EINVAL;
  const ProbDesc& d = j->hdesc[k];
  if (c < 0 || c >= d.m) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(j->ctx->mu);
  TT_HIP(hipStreamSynchronize(j->ctx->stream));
  const int m = d.m, n = d.n, R = d.R;
  int rl = 1, rr = 1;
  if (c >= 1) TT_HIP(hipMemcpy(&rl, d.rank + (c - 1), sizeof(int32_t), hipMemcpyDeviceToHost));
  if (c <= m - 2) TT_HIP(hipMemcpy(&rr, d.rank + c, sizeof(int32_t), hipMemcpyDeviceToHost));
  const int64_t nr = (int64_t)rl * n;
  if (nr * rr > capacity) return TT_EINVAL;
  const int rowcap = c == 0 ? 1 : R, colcap = c == m - 1 ? 1 : R;
  const size_t es = j->qd ? sizeof(qd) : j->dd ? sizeof(dd) : sizeof(double);
  // offsets of core c and interpolation core c inside the job's arrays (host copies of the tables)
  std::vector<int64_t> foff(m), coff(std::max(m - 1, 1));
  {
    Layout pl;
    const ProbOffsets o = layout_problem(j->probs[k], pl);
    for (int q = 0; q < m; ++q) foff[q] = o.foff[q];
    for (int q = 0; q < m - 1; ++q) coff[q] = o.coff[q];
  }
  std::vector<char> fbuf((size_t)rowcap * n * colcap * es);
  TT_HIP(hipMemcpy(fbuf.data(), (char*)d.F + foff[c] * es, fbuf.size(), hipMemcpyDeviceToHost));
  auto lead = [&](const char* base, size_t idx) {
    double v;
    std::memcpy(&v, base + idx * es, sizeof(double));   // the leading double of a dd or qd value comes first
    return v;
  };
  for (int64_t row = 0; row < nr; ++row)
    for (int q = 0; q < rr; ++q) F[row * rr + q] = lead(fbuf.data(), (size_t)row * colcap + q);
  if (C && c <= m - 2) {
    const size_t ldC = (size_t)rowcap * n;   // stored transposed: C[q][row]
    std::vector<char> cbuf((size_t)R * ldC * es);
    TT_HIP(hipMemcpy(cbuf.data(), (char*)d.C + coff[c] * es, cbuf.size(), hipMemcpyDeviceToHost));
    for (int64_t row = 0; row < nr; ++row)
      for (int q = 0; q < rr; ++q) C[row * rr + q] = lead(cbuf.data(), (size_t)q * ldC + row);
  }
  *rows = (int32_t)nr;
  *cols = rr;
  return TT_OK;
}

void tt_cross_free(tt_job* j) {
  if (!j) return;
  tt_ctx* c = j->ctx;
  std::lock_guard<std::mutex> lock(c->mu);
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  pinned_give(c, j->pinned, j->pinned_bytes);
  for (hipEvent_t e : j->ring) c->ring_pool.push_back(e);
  if (c->arena_bytes_cached + j->bytes <= kArenaCacheBytes) {
    c->arenas.emplace(j->bytes, j->arena);
    c->arena_bytes_cached += j->bytes;
  } else {
    (void)hipFree(j->arena);
  }
  delete j;
}


tt_status tt_eval_points(tt_ctx* ctx, const tt_problem* p, const int32_t* d_idx, int64_t npts,
                         double* d_out) {
  if (!ctx || validate(p) != TT_OK || npts < 0 || (npts > 0 && (!d_idx || !d_out))) return TT_EINVAL;
  if (modes_of(*p) > TT_MAX_REG_MODES) return TT_EINVAL;
  if (npts == 0) return TT_OK;
  std::lock_guard<std::mutex> lock(ctx->mu);
  TT_HIP(hipSetDevice(ctx->device));
  if (p->precision == TT_QD) return TT_EINVAL;
  const bool use_dd = p->precision == TT_DD;
  double *t, *w;
  tt_status s = gl_table(ctx, p->n_nodes, &t, &w, use_dd ? TT_DD : TT_FP64);
  if (s != TT_OK) return s;
  FamilyArgs fa;
  s = family_for(ctx, p, &fa);
  if (s != TT_OK) return s;
  const int64_t blocks64 = std::min<int64_t>((npts + kBlock - 1) / kBlock, 1 << 20);
  const dim3 grid((unsigned)blocks64), block(kBlock);
  Timed tm(ctx, KK_EVAL_POINTS);
  switch (bucket_m(fa.m)) {
    case 8: eval_points_m<8>(ctx, use_dd, grid, block, fa, t, w, d_idx, npts, d_out); break;
    case 16: eval_points_m<16>(ctx, use_dd, grid, block, fa, t, w, d_idx, npts, d_out); break;
    default: eval_points_m<32>(ctx, use_dd, grid, block, fa, t, w, d_idx, npts, d_out); break;
  }
  TT_HIP(hipGetLastError());
  return TT_OK;
}

tt_status tt_eval_fibers(tt_ctx* ctx, const tt_problem* p, int32_t pos, const int32_t* d_left,
                         int32_t r_left, const int32_t* d_right, int32_t r_right, double* d_out) {
  if (!ctx || validate(p) != TT_OK || modes_of(*p) > TT_MAX_REG_MODES) return TT_EINVAL;
  const int m = modes_of(*p);
  if (m < 1 || pos < 0 || pos >= m) return TT_EINVAL;
  if (r_left < 1 || r_left > TT_MAX_RANK || r_right < 1 || r_right > TT_MAX_RANK || !d_out) return TT_EINVAL;
  if ((pos > 0 && !d_left) || (pos < m - 1 && !d_right)) return TT_EINVAL;
  if ((pos == 0 && r_left != 1) || (pos == m - 1 && r_right != 1)) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  TT_HIP(hipSetDevice(ctx->device));
  if (p->precision == TT_QD) return TT_EINVAL;
  const bool use_dd = p->precision == TT_DD;
  double *t, *w;
  tt_status s = gl_table(ctx, p->n_nodes, &t, &w, use_dd ? TT_DD : TT_FP64);
  if (s != TT_OK) return s;
  FamilyArgs fa;
  s = family_for(ctx, p, &fa);
  if (s != TT_OK) return s;
  const int fam = fam_of(p->integrand);
  // work items: points, or for the row-summary kernel (alpha, node chunk, beta) triples
  const bool rows = fam == FAM_PAPER && !use_dd && m <= kRowsMaxModes;
  const int64_t chunks = rows ? (p->n_nodes + kFibreNodesPerLane - 1) / kFibreNodesPerLane : p->n_nodes;
  const int64_t total = (int64_t)r_left * chunks * r_right;   // < 2^31 by the rank and node limits
  const int64_t blocks64 = std::min<int64_t>((total + kBlock - 1) / kBlock, 1024);
  const dim3 grid((unsigned)blocks64), block(kBlock);
  const int n = p->n_nodes, mb = bucket_m(m);
  Timed tm(ctx, KK_EVAL_FIBERS);
  if (use_dd)
    eval_fibers_f<dd, FAM_PAPER>(ctx, mb, grid, block, fa, n, t, w, pos, d_left, r_left, d_right, r_right, d_out);
  else if (fam == FAM_PAPER)
    eval_fibers_exact<1>(ctx, m, grid, block, fa, n, t, w, pos, d_left, r_left, d_right, r_right, d_out);
  else if (fam == FAM_UFORM)
    eval_fibers_f<double, FAM_UFORM>(ctx, mb, grid, block, fa, n, t, w, pos, d_left, r_left, d_right, r_right,
                                     d_out);
  else
    eval_fibers_f<double, FAM_SYNTH>(ctx, mb, grid, block, fa, n, t, w, pos, d_left, r_left, d_right, r_right,
                                     d_out);
  TT_HIP(hipGetLastError());
  return TT_OK;
}

tt_status tt_mc_integrate(tt_ctx* ctx, const tt_problem* p, int32_t kind, int64_t n_points, int32_t n_sets,
                          const int64_t* gen, double* estimates, double* mean, double* rel_err) {
  FamilyArgs fa;
  McParams mp;
  int blocks = 0;
  tt_status s = mc_setup(ctx, p, kind, n_points, n_sets, gen, &fa, &mp, &blocks);
  if (s != TT_OK) return s;
  if (!estimates || !mean || !rel_err) return TT_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  TT_HIP(hipSetDevice(ctx->device));
  // partial sums [S x blocks], then the results [S + 2]
  const size_t need = sizeof(double) * ((size_t)n_sets * blocks + n_sets + 2);
  if (need > ctx->mc_cap) {
    TT_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->mc_buf) TT_HIP(hipFree(ctx->mc_buf));
    ctx->mc_buf = nullptr;
    ctx->mc_cap = 0;
    if (hipMalloc(&ctx->mc_buf, need) != hipSuccess) return TT_ENOMEM;
    ctx->mc_cap = need;
  }
  double* partial = ctx->mc_buf;
  double* out = partial + (size_t)n_sets * blocks;
  {
    Timed tm(ctx, KK_MC);
    mc_launch(ctx, p, kind, n_points, n_sets, fa, mp, blocks, partial, out);
  }
  TT_HIP(hipGetLastError());
  std::vector<double> h(n_sets + 2);
  TT_HIP(hipMemcpyAsync(h.data(), out, sizeof(double) * (n_sets + 2), hipMemcpyDeviceToHost, ctx->stream));
  TT_HIP(hipStreamSynchronize(ctx->stream));
  for (int j = 0; j < n_sets; ++j) estimates[j] = h[j];
  *mean = h[n_sets];
  *rel_err = h[n_sets + 1];
  return TT_OK;
}

tt_status tt_mc_integrate_noalloc(tt_ctx* ctx, const tt_problem* p, int32_t kind, int64_t n_points,
                                  int32_t n_sets, const int64_t* gen, double* d_out) {
  FamilyArgs fa;
  McParams mp;
  int blocks = 0;
  tt_status s = mc_setup(ctx, p, kind, n_points, n_sets, gen, &fa, &mp, &blocks);
  if (s != TT_OK) return s;
  if (!d_out || (int64_t)n_sets * blocks > TT_MC_NOALLOC_MAX_PARTIALS) return TT_EINVAL;
  if (!ctx->scratch) return TT_EDEVICE;   // the symbol lookup at tt_ctx_create failed
  std::lock_guard<std::mutex> lock(ctx->mu);
  TT_HIP(hipSetDevice(ctx->device));
  mc_launch(ctx, p, kind, n_points, n_sets, fa, mp, blocks, ctx->scratch, d_out);
  TT_HIP(hipGetLastError());
  return TT_OK;
}

}  // extern "C"
