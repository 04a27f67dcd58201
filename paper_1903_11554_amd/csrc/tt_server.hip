// Serving loop of the TT cross library (include/ttcross.h, tt_server_*):
// continuous batching of single-integral requests.  A worker thread owns the
// running set; each loop iteration retires the integrals whose pinned done flag
// is up, admits queued requests into the freed memory and slots, enqueues the
// start of the admitted ones and one sweep launch that advances every running
// integral (k_sweep is indexed by (integral, superblock) tasks, so integrals of
// any d, rank cap, tolerance or age share a launch).  All device work is on the
// context stream, so memory freed by a retired integral may be handed to a new
// one at once: its initialisation is ordered after every launch that could
// still read the old one.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "tt_host.hpp"

using namespace ttx;
using namespace ttx_host;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kMaxBonds = TT_MAX_REG_MODES - 1;
constexpr int kStages = 4;       // pinned upload buffers in rotation
constexpr int kInFlight = 3;     // sweep launches allowed ahead of the host

struct Request {
  uint64_t ticket;
  tt_problem prob;
  std::vector<double> params;
  size_t bytes;
  Clock::time_point t_submit;
};

struct Running {
  Request req;
  int slot;            // index of its pinned flag / state mirror
  size_t off;          // its sub-allocation in the arena
  int m, fam, launched;
  ProbDesc desc;
};

struct Result {
  tt_info info;
  double latency_s;
};

// First-fit allocator over the server arena (offsets, 256-byte granules).
struct SubAlloc {
  std::map<size_t, size_t> free_;   // offset -> size
  explicit SubAlloc(size_t total) { free_[0] = total; }
  bool take(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

// bytes of one request in the arena: its device state, small tables and arrays
size_t request_bytes(const tt_problem& p) {
  Layout L;
  L.take(sizeof(ProbState));
  take_tables(p, L);
  Layout pl;
  layout_problem(p, pl);
  L.take(pl.off);
  return L.off;
}

}  // namespace

struct tt_server {
  tt_ctx* ctx = nullptr;
  size_t max_bytes = 0;
  int max_active = 0;
  int search_group = 0;                  // the context's fixed search group when the server was created (0: rule)
  char* arena = nullptr;                 // device
  SubAlloc* alloc = nullptr;
  // device table: sweep descriptors and tasks, init descriptors and core tasks
  char* dtable = nullptr;
  size_t off_sdesc = 0, off_stask = 0, off_score = 0, off_idesc = 0, off_itask = 0, off_ctr = 0, table_bytes = 0;
  // pinned host memory
  int32_t* flags = nullptr;              // [max_active] done flags
  ProbState* mirror = nullptr;           // [max_active] final states
  char* stage[kStages] = {};
  size_t stage_bytes = 0;
  hipEvent_t stage_ev[kStages] = {};
  int stage_next = 0;
  std::vector<hipEvent_t> sweep_ev;
  int64_t sweep_count = 0;
  // state shared with the API threads
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request> queue;
  std::unordered_map<uint64_t, Result> results;
  uint64_t next_ticket = 1;
  bool stopping = false;
  tt_status fatal = TT_OK;
  tt_server_stats stats{};
  // worker-only state
  std::vector<Running> running;
  std::vector<int> free_slots;
  std::thread worker;
};

namespace {

double seconds_since(Clock::time_point t0) {
  return std::chrono::duration<double>(Clock::now() - t0).count();
}

// Wait for a pinned staging buffer whose previous upload has completed.
tt_status take_stage(tt_server* s, char** buf, int* idx) {
  const int k = s->stage_next;
  s->stage_next = (k + 1) % kStages;
  TT_HIP(hipEventSynchronize(s->stage_ev[k]));
  *buf = s->stage[k];
  *idx = k;
  return TT_OK;
}

// Admitted requests: lay out their arrays, upload their tables and
// descriptors, and enqueue the rank-1 start, first cores and first quadrature.
tt_status start_requests(tt_server* s, std::vector<Running>& fresh) {
  tt_ctx* ctx = s->ctx;
  char* stg;
  int si;
  tt_status st = take_stage(s, &stg, &si);
  if (st != TT_OK) return st;
  size_t used = 0;
  std::vector<ProbDesc> idesc;
  std::vector<int2> itask;
  int maxm = 0, fam = -1;
  for (size_t q = 0; q < fresh.size(); ++q) {
    Running& r = fresh[q];
    const tt_problem& p = r.req.prob;
    char* base = s->arena + r.off;
    Layout L;
    const size_t st_off = L.take(sizeof(ProbState));
    const ProbTables tb = take_tables(p, L);
    const size_t tables_end = L.take(0);
    Layout pl;
    const ProbOffsets o = layout_problem(p, pl);
    const size_t arrays = L.take(pl.off);
    double *t, *w;
    st = gl_table(ctx, p.n_nodes, &t, &w, false, true);
    if (st != TT_OK) return st;
    s->flags[r.slot] = 0;
    r.desc = make_desc(p, o, base + arrays, base, tb, t, w, s->flags + r.slot, (ProbState*)(base + st_off),
                       s->mirror + r.slot, false);
    // tables of this request: staged, then copied into its own sub-allocation
    char* img = stg + used;
    std::memset(img, 0, tables_end);
    write_tables(p, o, tb, img);
    TT_HIP(hipMemcpyAsync(base, img, tables_end, hipMemcpyHostToDevice, ctx->stream));
    used += (tables_end + 255) & ~size_t(255);
    idesc.push_back(r.desc);
    if (r.m >= 2)
      for (int c = 0; c < r.m; ++c) itask.push_back(make_int2((int)q, c));
    maxm = std::max(maxm, r.m);
    fam = (fam < 0) ? r.fam : (fam == r.fam ? fam : FAM_ANY);
  }
  char* dimg = stg + used;
  std::memcpy(dimg, idesc.data(), idesc.size() * sizeof(ProbDesc));
  TT_HIP(hipMemcpyAsync(s->dtable + s->off_idesc, dimg, idesc.size() * sizeof(ProbDesc), hipMemcpyHostToDevice,
                        ctx->stream));
  used += (idesc.size() * sizeof(ProbDesc) + 255) & ~size_t(255);
  if (!itask.empty()) {
    char* timg = stg + used;
    std::memcpy(timg, itask.data(), itask.size() * sizeof(int2));
    TT_HIP(hipMemcpyAsync(s->dtable + s->off_itask, timg, itask.size() * sizeof(int2), hipMemcpyHostToDevice,
                          ctx->stream));
  }
  TT_HIP(hipEventRecord(s->stage_ev[si], ctx->stream));
  LaunchArgs a{(ProbDesc*)(s->dtable + s->off_idesc), nullptr, 0, (const int2*)(s->dtable + s->off_itask),
               (int)itask.size(), (int)fresh.size(), bucket_m_for(fam, TT_FP64, maxm), ctx->stream, nullptr, 1};
  auto go = [&](int what) {
    switch (fam) {
      case FAM_PAPER: launch_paper(a, what, 8); break;
      case FAM_UFORM: launch_uform(a, what, 8); break;
      case FAM_SYNTH: launch_synth(a, what, 8); break;
      default: launch_any(a, what, 8); break;
    }
  };
  {
    Timed tm(ctx, KK_START);
    go(LAUNCH_START);
  }
  if (!itask.empty()) {
    {
      Timed tm(ctx, KK_UPDATE);
      go(LAUNCH_INIT_UPDATE);
    }
    Timed tm(ctx, KK_INTEGRAL);
    hipLaunchKernelGGL(k_integral<double>, dim3((unsigned)fresh.size()), dim3(kIntBlock), 0, ctx->stream,
                       (ProbDesc*)(s->dtable + s->off_idesc), 1);
  }
  TT_HIP(hipGetLastError());
  return TT_OK;
}

// Upload the running set's descriptors, superblock tasks and core tasks.
tt_status upload_running(tt_server* s, int* nbond, int* ncore) {
  char* stg;
  int si;
  tt_status st = take_stage(s, &stg, &si);
  if (st != TT_OK) return st;
  const size_t nd = s->running.size();
  ProbDesc* d = (ProbDesc*)stg;
  int2* tk = (int2*)(stg + ((nd * sizeof(ProbDesc) + 255) & ~size_t(255)));
  int nt = 0;
  for (size_t q = 0; q < nd; ++q) {
    d[q] = s->running[q].desc;
    for (int b = 0; b + 1 < s->running[q].m; ++b) tk[nt++] = make_int2((int)q, b);
  }
  int2* ck = tk + nt;   // core tasks of the integrals that have superblocks
  int nc = 0;
  for (size_t q = 0; q < nd; ++q)
    if (s->running[q].m >= 2)
      for (int c = 0; c < s->running[q].m; ++c) ck[nc++] = make_int2((int)q, c);
  if (nd) TT_HIP(hipMemcpyAsync(s->dtable + s->off_sdesc, d, nd * sizeof(ProbDesc), hipMemcpyHostToDevice,
                                s->ctx->stream));
  if (nt) TT_HIP(hipMemcpyAsync(s->dtable + s->off_stask, tk, nt * sizeof(int2), hipMemcpyHostToDevice,
                                s->ctx->stream));
  if (nc) TT_HIP(hipMemcpyAsync(s->dtable + s->off_score, ck, nc * sizeof(int2), hipMemcpyHostToDevice,
                                s->ctx->stream));
  TT_HIP(hipEventRecord(s->stage_ev[si], s->ctx->stream));
  *nbond = nt;
  *ncore = nc;
  return TT_OK;
}

void worker_main(tt_server* s) {
  tt_ctx* ctx = s->ctx;
  bool changed = true;
  int nbond = 0, ncore = 0;
  Clock::time_point busy_since{};
  bool busy = false;
  for (;;) {
    std::vector<Running> fresh;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      // retire: integrals whose kernels raised the done flag
      for (size_t q = 0; q < s->running.size();) {
        Running& r = s->running[q];
        if (__atomic_load_n(&s->flags[r.slot], __ATOMIC_ACQUIRE) != 0) {
          Result res;
          fill_info(s->mirror[r.slot], &res.info);
          res.info.reason = s->mirror[r.slot].reason;
          res.latency_s = seconds_since(r.req.t_submit);
          s->results[r.req.ticket] = res;
          s->alloc->give(r.off, r.req.bytes);
          s->free_slots.push_back(r.slot);
          s->running.erase(s->running.begin() + q);
          s->stats.completed += 1;
          changed = true;
        } else {
          ++q;
        }
      }
      if (changed) s->cv_done.notify_all();
      // admit in arrival order while memory and slots allow
      while (!s->queue.empty() && !s->free_slots.empty()) {
        size_t off;
        if (!s->alloc->take(s->queue.front().bytes, &off)) break;
        Running r;
        r.req = std::move(s->queue.front());
        s->queue.pop_front();
        r.req.prob.params = r.req.params.empty() ? nullptr : r.req.params.data();
        r.slot = s->free_slots.back();
        s->free_slots.pop_back();
        r.off = off;
        r.m = modes_of(r.req.prob);
        r.fam = fam_of(r.req.prob.integrand);
        r.launched = 0;
        fresh.push_back(std::move(r));
      }
      s->stats.queued = (int64_t)s->queue.size();
      if (s->running.empty() && fresh.empty()) {
        if (busy) {
          s->stats.busy_s += seconds_since(busy_since);
          busy = false;
        }
        if (s->stopping) break;
        s->cv_work.wait(lk, [&] { return s->stopping || !s->queue.empty(); });
        continue;
      }
    }
    if (!busy) {
      busy = true;
      busy_since = Clock::now();
    }
    tt_status st = TT_OK;
    {
      std::lock_guard<std::mutex> cl(ctx->mu);
      if (!fresh.empty()) {
        st = start_requests(s, fresh);
        for (Running& r : fresh) s->running.push_back(std::move(r));
        changed = true;
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.admissions += 1;
      }
      if (st == TT_OK && changed) {
        st = upload_running(s, &nbond, &ncore);
        changed = false;
      }
      if (st == TT_OK && nbond > 0) {
        int maxm = 0, fam = -1, rmax = 1;
        for (Running& r : s->running) {
          maxm = std::max(maxm, r.m);
          fam = (fam < 0) ? r.fam : (fam == r.fam ? fam : FAM_ANY);
          rmax = std::max(rmax, std::min(r.req.prob.rank_cap, r.launched + 2));
          r.launched += 1;
        }
        LaunchArgs a{(ProbDesc*)(s->dtable + s->off_sdesc), (const int2*)(s->dtable + s->off_stask), nbond,
                     (const int2*)(s->dtable + s->off_score), ncore, (int)s->running.size(),
                     bucket_m_for(fam, TT_FP64, maxm), ctx->stream, (int32_t*)(s->dtable + s->off_ctr),
                     s->search_group > 0 ? s->search_group
                                         : search_group_for_bucket(search_group_rule(ctx->cus, nbond, ncore, TT_FP64),
                                                                   bucket_r(rmax), TT_FP64)};
        {
          Timed tm(ctx, KK_SWEEP);
          switch (fam) {
            case FAM_PAPER: launch_paper(a, LAUNCH_SWEEP, bucket_r(rmax)); break;
            case FAM_UFORM: launch_uform(a, LAUNCH_SWEEP, bucket_r(rmax)); break;
            case FAM_SYNTH: launch_synth(a, LAUNCH_SWEEP, bucket_r(rmax)); break;
            default: launch_any(a, LAUNCH_SWEEP, bucket_r(rmax)); break;
          }
        }
        if (hipGetLastError() != hipSuccess) st = TT_EDEVICE;
        hipEvent_t ev = s->sweep_ev[s->sweep_count % kInFlight];
        if (st == TT_OK && hipEventRecord(ev, ctx->stream) != hipSuccess) st = TT_EDEVICE;
        s->sweep_count += 1;
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.sweep_launches += 1;
        s->stats.running = (int64_t)s->running.size();
        s->stats.max_running = std::max(s->stats.max_running, (int64_t)s->running.size());
      }
      if (st == TT_OK && nbond == 0) {
        // only integrals without bonds (m <= 1) are running: their start decides them
        if (hipStreamSynchronize(ctx->stream) != hipSuccess) st = TT_EDEVICE;
      }
    }
    if (st == TT_OK && s->sweep_count >= kInFlight) {
      // at most kInFlight sweeps ahead of the last one known complete
      if (hipEventSynchronize(s->sweep_ev[s->sweep_count % kInFlight]) != hipSuccess) st = TT_EDEVICE;
    }
    if (st != TT_OK) {
      std::lock_guard<std::mutex> lk(s->mu);
      s->fatal = st;
      s->stopping = true;
      s->cv_done.notify_all();
      break;
    }
  }
  std::lock_guard<std::mutex> cl(ctx->mu);
  (void)hipStreamSynchronize(ctx->stream);
}

}  // namespace

extern "C" {

tt_status tt_server_create(tt_ctx* ctx, size_t max_bytes, int32_t max_active, tt_server** out) {
  if (!ctx || !out || max_active < 1 || max_active > 4096 || max_bytes < 4096) return TT_EINVAL;
  tt_server* s = new (std::nothrow) tt_server;
  if (!s) return TT_ENOMEM;
  s->ctx = ctx;
  s->max_bytes = max_bytes;
  s->max_active = max_active;
  auto fail = [&](tt_status st) {
    if (s->arena) (void)hipFree(s->arena);
    if (s->dtable) (void)hipFree(s->dtable);
    if (s->flags) (void)hipHostFree(s->flags);
    if (s->mirror) (void)hipHostFree(s->mirror);
    for (int k = 0; k < kStages; ++k) {
      if (s->stage[k]) (void)hipHostFree(s->stage[k]);
      if (s->stage_ev[k]) (void)hipEventDestroy(s->stage_ev[k]);
    }
    for (hipEvent_t e : s->sweep_ev) (void)hipEventDestroy(e);
    delete s->alloc;
    delete s;
    return st;
  };
  {
    std::lock_guard<std::mutex> cl(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(TT_EDEVICE);
    s->search_group = ctx->search_group;
    if (hipMalloc(&s->arena, max_bytes) != hipSuccess) return fail(TT_ENOMEM);
    Layout L;
    s->off_sdesc = L.take(sizeof(ProbDesc) * max_active);
    s->off_stask = L.take(sizeof(int2) * max_active * kMaxBonds);
    s->off_score = L.take(sizeof(int2) * max_active * TT_MAX_REG_MODES);
    s->off_idesc = L.take(sizeof(ProbDesc) * max_active);
    s->off_itask = L.take(sizeof(int2) * max_active * TT_MAX_REG_MODES);
    s->off_ctr = L.take(2 * sizeof(int32_t));
    s->table_bytes = L.off;
    if (hipMalloc(&s->dtable, s->table_bytes) != hipSuccess) return fail(TT_ENOMEM);
    // the sweep kernel's launch counters start at zero (each launch leaves them so)
    if (hipMemset(s->dtable + s->off_ctr, 0, 2 * sizeof(int32_t)) != hipSuccess) return fail(TT_EDEVICE);
    if (hipHostMalloc((void**)&s->flags, sizeof(int32_t) * max_active, hipHostMallocDefault) != hipSuccess)
      return fail(TT_ENOMEM);
    if (hipHostMalloc((void**)&s->mirror, sizeof(ProbState) * max_active, hipHostMallocDefault) != hipSuccess)
      return fail(TT_ENOMEM);
    // one staging buffer holds a full table upload or one admission round
    s->stage_bytes = s->table_bytes + (size_t)max_active * 2048;
    for (int k = 0; k < kStages; ++k) {
      if (hipHostMalloc((void**)&s->stage[k], s->stage_bytes, hipHostMallocDefault) != hipSuccess)
        return fail(TT_ENOMEM);
      if (hipEventCreateWithFlags(&s->stage_ev[k], hipEventDisableTiming) != hipSuccess) return fail(TT_EDEVICE);
    }
    for (int k = 0; k < kInFlight; ++k) {
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail(TT_EDEVICE);
      s->sweep_ev.push_back(e);
    }
  }
  s->alloc = new (std::nothrow) SubAlloc(max_bytes);
  if (!s->alloc) return fail(TT_ENOMEM);
  for (int k = max_active - 1; k >= 0; --k) s->free_slots.push_back(k);
  try {
    s->worker = std::thread(worker_main, s);
  } catch (...) {
    return fail(TT_ENOMEM);
  }
  *out = s;
  return TT_OK;
}

tt_status tt_server_submit(tt_server* s, const tt_problem* p, uint64_t* ticket) {
  if (!s || !p || !ticket || validate(p) != TT_OK || p->precision != TT_FP64) return TT_EINVAL;
  if (modes_of(*p) > TT_MAX_REG_MODES) return TT_EINVAL;
  Request r;
  r.prob = *p;
  const int m = modes_of(*p);
  if (is_synthetic(p->integrand)) r.params.assign(p->params, p->params + 2 * m);
  r.prob.params = nullptr;
  r.bytes = request_bytes(*p);
  if (r.bytes > s->max_bytes) return TT_ENOMEM;
  r.t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) return s->fatal != TT_OK ? s->fatal : TT_EINVAL;
  r.ticket = s->next_ticket++;
  *ticket = r.ticket;
  s->queue.push_back(std::move(r));
  s->stats.submitted += 1;
  s->stats.queued = (int64_t)s->queue.size();
  s->cv_work.notify_one();
  return TT_OK;
}

static tt_status take_result(tt_server* s, uint64_t ticket, tt_info* info, double* latency_s, bool wait) {
  std::unique_lock<std::mutex> lk(s->mu);
  if (ticket == 0 || ticket >= s->next_ticket) return TT_EINVAL;
  for (;;) {
    auto it = s->results.find(ticket);
    if (it != s->results.end()) {
      if (info) *info = it->second.info;
      if (latency_s) *latency_s = it->second.latency_s;
      s->results.erase(it);
      return TT_OK;
    }
    if (s->fatal != TT_OK) return s->fatal;
    if (!wait) return TT_PENDING;
    s->cv_done.wait(lk);
  }
}

tt_status tt_server_poll(tt_server* s, uint64_t ticket, tt_info* info, double* latency_s) {
  if (!s) return TT_EINVAL;
  return take_result(s, ticket, info, latency_s, false);
}

tt_status tt_server_wait(tt_server* s, uint64_t ticket, tt_info* info, double* latency_s) {
  if (!s) return TT_EINVAL;
  return take_result(s, ticket, info, latency_s, true);
}

tt_status tt_server_get_stats(tt_server* s, tt_server_stats* out) {
  if (!s || !out) return TT_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  return TT_OK;
}

void tt_server_destroy(tt_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->queue.clear();
    s->stopping = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->ctx->device);
  (void)hipFree(s->arena);
  (void)hipFree(s->dtable);
  (void)hipHostFree(s->flags);
  (void)hipHostFree(s->mirror);
  for (int k = 0; k < kStages; ++k) {
    (void)hipHostFree(s->stage[k]);
    (void)hipEventDestroy(s->stage_ev[k]);
  }
  for (hipEvent_t e : s->sweep_ev) (void)hipEventDestroy(e);
  delete s->alloc;
  delete s;
}

}  // extern "C"
