// Serving runtime of libsknr: continuous batching of independent OT solves.
//
// Requests are deep-copied to host memory at submit and wait in a FIFO
// queue.  Worker lanes (one host thread, one HIP stream, one graph cache
// each) admit requests whenever device memory for the request (inputs +
// workspace, and its outputs) can be carved out of one pre-allocated pool:
// admission is by HBM footprint, first fit, in arrival order with bounded
// backfilling (a request that does not fit lets younger ones pass at most
// kMaxBackfill times before the queue waits for it).  Admitted requests run
// the same schedule as sknr_solve on their own stream, so the work of all
// running requests overlaps on the device; a request joins as soon as a
// lane and memory are free and leaves when its schedule ends, and its
// potentials stay in the pool until the caller collects them.  The kernels
// of a request do not depend on the other requests (fixed reduction orders,
// geometry from the request's own shape), so a result is the same alone
// and in the mix.
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "sknr_host.h"

namespace sknr_host {

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxBackfill = 16;
inline size_t al(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }
using Clock = std::chrono::steady_clock;

// First-fit allocator over one device allocation.
struct Pool {
  char* base = nullptr;
  size_t cap = 0, used = 0, peak = 0;
  std::map<size_t, size_t> free_;  // offset -> size, coalesced
  void init(size_t bytes) {
    bytes = bytes & ~(kAlign - 1);
    hipError_t e = hipMalloc((void**)&base, bytes);
    if (e != hipSuccess) throw Err{SKNR_ENOMEM, "serving pool allocation failed"};
    cap = bytes;
    free_.clear();
    free_[0] = bytes;
  }
  size_t alloc(size_t bytes) {
    bytes = al(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, rem = it->second - bytes;
      free_.erase(it);
      if (rem) free_[off + bytes] = rem;
      used += bytes;
      peak = std::max(peak, used);
      return off;
    }
    return SIZE_MAX;
  }
  void release(size_t off, size_t bytes) {
    bytes = al(std::max<size_t>(bytes, 1));
    used -= bytes;
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

enum ReqState { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2 };

struct Request {
  uint64_t id = 0;
  sknr_problem prob{};  // device pointers point into the pool once admitted
  Prepared P;
  sknr_opts opts{};
  std::vector<double> eps;
  std::vector<double> ha, hb;
  std::vector<float> hx, hy, hC;
  size_t in_bytes = 0, ws = 0, out_bytes = 0;
  size_t work_off = SIZE_MAX, out_off = SIZE_MAX;
  int state = RQ_QUEUED;
  bool claimed = false;  // a wait() is collecting it
  int status = SKNR_OK;
  std::string err;
  sknr_result res{};
  std::atomic<int> cancel{0};
  Clock::time_point t_submit, t_start, t_end;
};

}  // namespace

// --------------------------------------------------------------- batcher
// One host thread and one stream launch the iteration chunks of all lanes.
// Jobs that arrive within a short window (or until every running lane has
// submitted one) are grouped by their unit's kernel sequence; a group runs
// min(reps) repetitions of its unit, each kernel of the unit as ONE launch
// whose tile table covers every job of the group.  Each request's kernels
// read only its own arguments and device state (gating included), so the
// result of a request does not depend on the group it ran in.
struct Batcher {
  std::mutex mu;
  std::condition_variable cv_job, cv_launched;
  std::vector<BatchJob*> pending;
  bool stop = false;
  int expected = 1;   // lanes running a request (an upper bound on the jobs of a batch)
  int iterating = 0;  // lanes inside a stage's iteration loop
  hipStream_t stream = nullptr;
  std::thread th;
  // tile tables: a ring of pinned host / device buffer pairs, each reused
  // only after the copy and the launches that used it before have finished
  static constexpr int kRing = 4;
  char* d_tab[kRing] = {};
  char* h_tab[kRing] = {};
  size_t tab_cap[kRing] = {};
  hipEvent_t tab_ev[kRing] = {};
  bool tab_used[kRing] = {};
  int ring = 0;
  int64_t batches = 0, jobs = 0, launches = 0;
};

int batcher_run(Batcher* b, BatchJob* job) {
  std::unique_lock<std::mutex> lk(b->mu);
  b->pending.push_back(job);
  b->cv_job.notify_one();
  b->cv_launched.wait(lk, [&] { return job->launched; });
  return job->reps_done;
}

void batcher_iterating(Batcher* b, int delta) {
  {
    std::lock_guard<std::mutex> lk(b->mu);
    b->iterating += delta;
  }
  b->cv_job.notify_one();
}

namespace {

// a batch waits for every iterating lane's job, at most this long
constexpr auto kBatchWindow = std::chrono::microseconds(1500);

// launch one group of jobs with identical unit kernel sequences
hipError_t run_group(Batcher* b, std::vector<BatchJob*>& g) {
  const int B = (int)g.size();
  const int nrec = g[0]->nrec;
  int reps = g[0]->reps;
  for (BatchJob* j : g) reps = std::min(reps, j->reps);
  for (BatchJob* j : g) {
    hipError_t e = hipStreamWaitEvent(b->stream, j->ev_in, 0);
    if (e != hipSuccess) return e;
  }
  // tables per unit launch i: args[B] pointers, off[B + 1], gx[B]
  const size_t per = al((size_t)B * 8) + al((size_t)(B + 1) * 4) + al((size_t)B * 4);
  const size_t bytes = per * (size_t)nrec;
  const int k = b->ring;
  b->ring = (b->ring + 1) % Batcher::kRing;
  if (b->tab_used[k]) {
    hipError_t e = hipEventSynchronize(b->tab_ev[k]);
    if (e != hipSuccess) return e;
  }
  if (bytes > b->tab_cap[k]) {
    if (b->d_tab[k]) (void)hipFree(b->d_tab[k]);
    if (b->h_tab[k]) (void)hipHostFree(b->h_tab[k]);
    b->d_tab[k] = b->h_tab[k] = nullptr;
    b->tab_cap[k] = 0;
    const size_t cap = std::max<size_t>(bytes * 2, 1 << 16);
    hipError_t e = hipMalloc((void**)&b->d_tab[k], cap);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_tab[k], cap, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    b->tab_cap[k] = cap;
  }
  if (!b->tab_ev[k]) {
    hipError_t e = hipEventCreateWithFlags(&b->tab_ev[k], hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  std::memset(b->h_tab[k], 0, bytes);
  std::vector<int> total(nrec, 0);
  std::vector<unsigned> lds(nrec, 0);
  for (int i = 0; i < nrec; ++i) {
    char* base = b->h_tab[k] + per * i;
    const void** args = reinterpret_cast<const void**>(base);
    int* off = reinterpret_cast<int*>(base + al((size_t)B * 8));
    int* gx = reinterpret_cast<int*>(base + al((size_t)B * 8) + al((size_t)(B + 1) * 4));
    long long t = 0;
    for (int j = 0; j < B; ++j) {
      const BatchLaunch& L = g[j]->unit[i];
      args[j] = L.args_dev;
      off[j] = (int)t;
      gx[j] = L.gx;
      t += (long long)L.gx * L.gy;
      lds[i] = std::max(lds[i], L.lds);
    }
    if (t > (1ll << 30)) return hipErrorInvalidValue;
    off[B] = (int)t;
    total[i] = (int)t;
  }
  hipError_t e = hipMemcpyAsync(b->d_tab[k], b->h_tab[k], bytes, hipMemcpyHostToDevice, b->stream);
  if (e != hipSuccess) return e;
  for (int r = 0; r < reps; ++r) {
    for (int i = 0; i < nrec; ++i) {
      char* base = b->d_tab[k] + per * i;
      BatchTab T;
      T.args = reinterpret_cast<const void* const*>(base);
      T.off = reinterpret_cast<const int*>(base + al((size_t)B * 8));
      T.gx = reinterpret_cast<const int*>(base + al((size_t)B * 8) + al((size_t)(B + 1) * 4));
      T.nslot = B;
      void* kargs[] = {&T};
      const BatchLaunch& L0 = g[0]->unit[i];
      e = hipLaunchKernel(L0.bfunc, dim3(total[i]), dim3(L0.block), kargs, lds[i], b->stream);
      if (e != hipSuccess) return e;
      b->launches++;
    }
  }
  e = hipEventRecord(b->tab_ev[k], b->stream);
  if (e != hipSuccess) return e;
  b->tab_used[k] = true;
  for (BatchJob* j : g) {
    e = hipEventRecord(j->ev_done, b->stream);
    if (e != hipSuccess) return e;
    j->reps_done = reps;
  }
  return hipSuccess;
}

bool same_sequence(const BatchJob* a, const BatchJob* b) {
  if (a->nrec != b->nrec) return false;
  for (int i = 0; i < a->nrec; ++i)
    if (a->unit[i].bfunc != b->unit[i].bfunc || a->unit[i].block != b->unit[i].block) return false;
  return true;
}

void batcher_main(Batcher* b, int device) {
  (void)hipSetDevice(device);
  for (;;) {
    std::vector<BatchJob*> jobs;
    {
      std::unique_lock<std::mutex> lk(b->mu);
      b->cv_job.wait(lk, [&] { return b->stop || !b->pending.empty(); });
      if (b->pending.empty() && b->stop) return;
      b->cv_job.wait_for(lk, kBatchWindow, [&] {
        return b->stop || (int)b->pending.size() >= std::max(1, std::min(b->expected, b->iterating));
      });
      jobs.swap(b->pending);
    }
    std::vector<std::vector<BatchJob*>> groups;
    for (BatchJob* j : jobs) {
      bool placed = false;
      for (auto& g : groups)
        if (same_sequence(g[0], j)) {
          g.push_back(j);
          placed = true;
          break;
        }
      if (!placed) groups.push_back({j});
    }
    for (auto& g : groups) {
      const hipError_t e = run_group(b, g);
      if (e != hipSuccess)
        for (BatchJob* j : g) j->status = (int)e;
    }
    {
      std::lock_guard<std::mutex> lk(b->mu);
      b->batches++;
      b->jobs += (int64_t)jobs.size();
      for (BatchJob* j : jobs) j->launched = true;
    }
    b->cv_launched.notify_all();
  }
}

}  // namespace

struct Server {
  Ctx* ctx = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, Request*> reqs;
  Pool pool;
  std::vector<std::thread> workers;
  std::vector<Lane*> lanes;
  bool stop = false;
  uint64_t next_id = 1;
  int backfilled = 0;  // younger requests admitted past a blocked head
  int running = 0;
  int64_t completed = 0;
  std::mutex copy_mu;           // serialises the output copies of wait()
  hipStream_t copy_stream = nullptr;
  Batcher* batcher = nullptr;   // batched iteration chunks (null: lanes launch their own)

  // under mu: the next admissible request with its memory reserved, or null
  Request* pick_locked() {
    for (size_t i = 0; i < queue.size(); ++i) {
      if (i > 0 && backfilled >= kMaxBackfill) break;
      Request* r = queue[i];
      const size_t w = pool.alloc(r->in_bytes + r->ws);
      if (w == SIZE_MAX) continue;
      const size_t o = pool.alloc(r->out_bytes);
      if (o == SIZE_MAX) {
        pool.release(w, r->in_bytes + r->ws);
        continue;
      }
      r->work_off = w;
      r->out_off = o;
      queue.erase(queue.begin() + (long)i);
      backfilled = (i == 0) ? 0 : backfilled + 1;
      return r;
    }
    return nullptr;
  }
};

namespace {

// Upload the request's inputs into its block and run the schedule.
void run_request(Server* S, Lane* L, Request* r) {
  char* wb = S->pool.base + r->work_off;
  hipStream_t s = L->own;
  const size_t n0 = (size_t)r->P.n0, m0 = (size_t)r->P.m0;
  size_t off = 0;
  auto place = [&](size_t bytes) {
    char* p = wb + off;
    off += al(bytes);
    return p;
  };
  double* da = (double*)place(8 * n0);
  double* db = (double*)place(8 * m0);
  HIPCHK(hipMemcpyAsync(da, r->ha.data(), 8 * n0, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(db, r->hb.data(), 8 * m0, hipMemcpyHostToDevice, s));
  r->prob.a = da;
  r->prob.b = db;
  if (r->prob.kind == SKNR_COST_STORED) {
    float* dC = (float*)place(4 * n0 * m0);
    HIPCHK(hipMemcpyAsync(dC, r->hC.data(), 4 * n0 * m0, hipMemcpyHostToDevice, s));
    r->prob.C = dC;
    r->prob.ldc = (int64_t)m0;
  } else {
    const size_t d = (size_t)r->prob.d;
    float* dx = (float*)place(4 * n0 * d);
    float* dy = (float*)place(4 * m0 * d);
    HIPCHK(hipMemcpyAsync(dx, r->hx.data(), 4 * n0 * d, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dy, r->hy.data(), 4 * m0 * d, hipMemcpyHostToDevice, s));
    r->prob.x = dx;
    r->prob.y = dy;
  }
  if (off != r->in_bytes) throw Err{SKNR_EINTERNAL, "request input layout mismatch"};
  rebind(r->P, &r->prob);
  L->arena.base = wb + r->in_bytes;
  L->arena.cap = r->ws;
  L->arena.off = 0;
  L->arena_external = true;
  L->cancel = &r->cancel;
  double* f = (double*)(S->pool.base + r->out_off);
  double* g = (double*)((char*)f + al(8 * n0));
  r->status = solve_on_lane(L, &r->prob, r->P, &r->opts, f, g, &r->res);
}

void worker_main(Server* S, Lane* L) {
  (void)hipSetDevice(S->ctx->device);
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || (r = S->pick_locked()) != nullptr; });
      if (!r) return;
      r->state = RQ_RUNNING;
      r->t_start = Clock::now();
      S->running++;
      if (S->batcher) {
        std::lock_guard<std::mutex> bl(S->batcher->mu);
        S->batcher->expected = std::max(1, S->running);
      }
    }
    try {
      run_request(S, L, r);
    } catch (const Err& e) {
      r->status = e.code;
      r->err = e.msg;
    } catch (const std::exception& e) {
      r->status = SKNR_EINTERNAL;
      r->err = e.what();
    }
    // the block is reused by the next request: drain the stream first
    (void)hipStreamSynchronize(L->own);
    L->cancel = nullptr;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->pool.release(r->work_off, r->in_bytes + r->ws);
      r->work_off = SIZE_MAX;
      r->t_end = Clock::now();
      r->res.queue_seconds = std::chrono::duration<double>(r->t_start - r->t_submit).count();
      r->res.latency_seconds = std::chrono::duration<double>(r->t_end - r->t_submit).count();
      r->state = RQ_DONE;
      S->running--;
      S->completed++;
      if (S->batcher) {
        std::lock_guard<std::mutex> bl(S->batcher->mu);
        S->batcher->expected = std::max(1, S->running);
      }
    }
    if (S->batcher) S->batcher->cv_job.notify_one();
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
}

struct ServeConfig {
  int max_active = 0;
  uint64_t pool_bytes = 0;
  int batched = 0;
};
std::mutex g_cfg_mu;
std::unordered_map<Ctx*, ServeConfig> g_cfg;

Server* ensure_server(Ctx* c) {
  if (c->server) return c->server;
  ServeConfig cfg;
  {
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    auto it = g_cfg.find(c);
    if (it != g_cfg.end()) cfg = it->second;
  }
  int lanes = cfg.max_active;
  if (lanes <= 0) {
    const char* e = getenv("SKNR_SERVE_LANES");
    lanes = e ? atoi(e) : 8;
  }
  lanes = std::max(1, std::min(64, lanes));
  uint64_t pool = cfg.pool_bytes ? cfg.pool_bytes : std::min<uint64_t>(c->budget, 8ull << 30);
  pool = std::min<uint64_t>(pool, c->budget);
  Server* S = new Server();
  S->ctx = c;
  try {
    S->pool.init(pool);
    HIPCHK(hipStreamCreateWithFlags(&S->copy_stream, hipStreamNonBlocking));
    // Lanes launch eagerly: a graph capture in progress on any stream makes
    // the caller's own work on the legacy default stream fail, and callers
    // keep working while requests run (SKNR_SERVE_GRAPHS=1 re-enables it).
    const char* sg = getenv("SKNR_SERVE_GRAPHS");
    for (int i = 0; i < lanes; ++i) {
      Lane* L = new Lane();
      S->lanes.push_back(L);
      lane_init(L, c->device);
      L->use_graphs = L->use_graphs && sg && sg[0] == '1';
    }
  } catch (...) {
    for (Lane* L : S->lanes) {
      lane_release(L);
      delete L;
    }
    if (S->pool.base) (void)hipFree(S->pool.base);
    if (S->copy_stream) (void)hipStreamDestroy(S->copy_stream);
    delete S;
    throw;
  }
  if (cfg.batched) {
    Batcher* b = new Batcher();
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      throw Err{SKNR_EDEVICE, "batcher stream creation failed"};
    }
    b->th = std::thread(batcher_main, b, c->device);
    S->batcher = b;
    for (Lane* L : S->lanes) L->batcher = b;
  }
  for (Lane* L : S->lanes) S->workers.emplace_back(worker_main, S, L);
  c->server = S;
  return S;
}

Request* find_locked(Server* S, uint64_t ticket) {
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) throw Err{SKNR_EINVAL, "unknown ticket"};
  return it->second;
}

}  // namespace

void server_destroy(Ctx* c) {
  Server* S = c->server;
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    for (Request* r : S->queue) {
      r->state = RQ_DONE;
      r->status = SKNR_ECANCELED;
    }
    S->queue.clear();
    for (auto& kv : S->reqs) kv.second->cancel.store(1);
  }
  S->cv_work.notify_all();
  S->cv_done.notify_all();
  for (auto& t : S->workers) t.join();
  if (S->batcher) {
    Batcher* b = S->batcher;
    {
      std::lock_guard<std::mutex> lk(b->mu);
      b->stop = true;
    }
    b->cv_job.notify_all();
    b->th.join();
    (void)hipStreamSynchronize(b->stream);
    for (int k = 0; k < Batcher::kRing; ++k) {
      if (b->d_tab[k]) (void)hipFree(b->d_tab[k]);
      if (b->h_tab[k]) (void)hipHostFree(b->h_tab[k]);
      if (b->tab_ev[k]) (void)hipEventDestroy(b->tab_ev[k]);
    }
    (void)hipStreamDestroy(b->stream);
    delete b;
    S->batcher = nullptr;
  }
  for (Lane* L : S->lanes) {
    L->arena.base = nullptr;
    L->arena.cap = 0;
    lane_release(L);
    delete L;
  }
  for (auto& kv : S->reqs) delete kv.second;
  if (S->copy_stream) (void)hipStreamDestroy(S->copy_stream);
  if (S->pool.base) (void)hipFree(S->pool.base);
  delete S;
  c->server = nullptr;
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  g_cfg.erase(c);
}

}  // namespace sknr_host

using namespace sknr_host;

extern "C" {

int sknr_serve_config(void* ctx, int32_t max_active, uint64_t pool_bytes) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    if (c->server) throw Err{SKNR_EBUSY, "serving already started on this context"};
    REQUIRE(max_active >= 0 && max_active <= 64, "max_active must be in [0, 64]");
    REQUIRE(pool_bytes == 0 || pool_bytes >= (1u << 20), "pool_bytes must be 0 or >= 1 MiB");
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    ServeConfig& cf = g_cfg[c];
    cf.max_active = max_active;
    cf.pool_bytes = pool_bytes;
    return SKNR_OK;
  });
}

int sknr_serve_batching(void* ctx, int32_t batched) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    if (c->server) throw Err{SKNR_EBUSY, "serving already started on this context"};
    REQUIRE(batched == 0 || batched == 1, "batched must be 0 or 1");
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    g_cfg[c].batched = batched;
    return SKNR_OK;
  });
}

int sknr_submit(void* ctx, const sknr_problem* prob, const sknr_opts* opts, uint64_t* ticket) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    REQUIRE(prob && opts && ticket, "prob, opts and ticket are required");
    REQUIRE(!opts->f0 && !opts->g0 && !opts->V0, "serving requests take no f0 / g0 / V0");
    REQUIRE(opts->ell == 0 || opts->warm_mode != SKNR_WARM_USER, "serving requests take no WARM_USER basis");
    hipStream_t cs = as_stream(opts->stream);
    sknr_problem staged;
    prob = stage_problem(c, prob, cs, &staged);
    Prepared P = prepare(prob, cs, c->prep);
    check_opts(opts, P);
    Server* S = ensure_server(c);
    Request* r = new Request();
    try {
      r->prob = *prob;
      r->P = P;
      r->opts = *opts;
      r->eps.assign(opts->eps, opts->eps + opts->n_eps);
      r->opts.eps = r->eps.data();
      r->opts.stream = nullptr;
      const size_t n0 = (size_t)P.n0, m0 = (size_t)P.m0;
      r->ha.resize(n0);
      r->hb.resize(m0);
      HIPCHK(hipMemcpyAsync(r->ha.data(), prob->a, 8 * n0, hipMemcpyDeviceToHost, cs));
      HIPCHK(hipMemcpyAsync(r->hb.data(), prob->b, 8 * m0, hipMemcpyDeviceToHost, cs));
      r->in_bytes = al(8 * n0) + al(8 * m0);
      if (prob->kind == SKNR_COST_STORED) {
        r->hC.resize(n0 * m0);
        HIPCHK(hipMemcpy2DAsync(r->hC.data(), 4 * m0, prob->C, 4 * (size_t)prob->ldc, 4 * m0, n0,
                                hipMemcpyDeviceToHost, cs));
        r->in_bytes += al(4 * n0 * m0);
        // geometry of the dense, aligned pool copy
        r->P.ldc = (long long)m0;
        r->P.C = reinterpret_cast<const float*>(kAlign);
      } else {
        const size_t d = (size_t)prob->d;
        r->hx.resize(n0 * d);
        r->hy.resize(m0 * d);
        HIPCHK(hipMemcpyAsync(r->hx.data(), prob->x, 4 * n0 * d, hipMemcpyDeviceToHost, cs));
        HIPCHK(hipMemcpyAsync(r->hy.data(), prob->y, 4 * m0 * d, hipMemcpyDeviceToHost, cs));
        r->in_bytes += al(4 * n0 * d) + al(4 * m0 * d);
      }
      HIPCHK(hipStreamSynchronize(cs));
      r->ws = ws_bytes(r->P, ell_pad(opts->ell), nullptr);
      r->out_bytes = al(8 * n0) + al(8 * m0);
    } catch (...) {
      delete r;
      throw;
    }
    if (al(r->in_bytes + r->ws) + al(r->out_bytes) > S->pool.cap) {
      delete r;
      throw Err{SKNR_ENOMEM, "request larger than the serving pool"};
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      r->id = S->next_id++;
      r->t_submit = Clock::now();
      S->reqs[r->id] = r;
      S->queue.push_back(r);
    }
    S->cv_work.notify_one();
    *ticket = r->id;
    return SKNR_OK;
  });
}

int sknr_poll(void* ctx, uint64_t ticket, int32_t* done) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    REQUIRE(done, "done is NULL");
    REQUIRE(c->server, "no serving requests on this context");
    std::lock_guard<std::mutex> lk(c->server->mu);
    Request* r = find_locked(c->server, ticket);
    *done = r->state == RQ_DONE ? 1 : 0;
    return SKNR_OK;
  });
}

int sknr_wait(void* ctx, uint64_t ticket, double* f_out, double* g_out, sknr_result* res) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    Server* S = c->server;
    REQUIRE(S, "no serving requests on this context");
    Request* r;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      r = find_locked(S, ticket);
      REQUIRE(!r->claimed, "ticket already being collected");
      r->claimed = true;
      S->cv_done.wait(lk, [&] { return r->state == RQ_DONE; });
    }
    int status = r->status;
    std::string err = r->err;
    hipError_t ce = hipSuccess;
    if (status >= 0 && r->out_off != SIZE_MAX) {
      const size_t n0 = (size_t)r->P.n0, m0 = (size_t)r->P.m0;
      const double* f = (const double*)(S->pool.base + r->out_off);
      const double* g = (const double*)((const char*)f + al(8 * n0));
      std::lock_guard<std::mutex> lk(S->copy_mu);
      if (f_out) ce = hipMemcpyAsync(f_out, f, 8 * n0, hipMemcpyDeviceToDevice, S->copy_stream);
      if (ce == hipSuccess && g_out) ce = hipMemcpyAsync(g_out, g, 8 * m0, hipMemcpyDeviceToDevice, S->copy_stream);
      if (ce == hipSuccess) ce = hipStreamSynchronize(S->copy_stream);
      if (res) *res = r->res;
    } else if (res) {
      std::memset(res, 0, sizeof(*res));
      res->status = status;
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (r->out_off != SIZE_MAX) S->pool.release(r->out_off, r->out_bytes);
      S->reqs.erase(r->id);
    }
    delete r;
    S->cv_work.notify_all();  // its output memory is free
    if (ce != hipSuccess) throw Err{SKNR_EDEVICE, std::string("output copy: ") + hipGetErrorString(ce)};
    if (status < 0) throw Err{status, err.empty() ? std::string(sknr_status_str(status)) : err};
    return status;
  });
}

int sknr_cancel(void* ctx, uint64_t ticket) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    Server* S = c->server;
    REQUIRE(S, "no serving requests on this context");
    {
      std::lock_guard<std::mutex> lk(S->mu);
      Request* r = find_locked(S, ticket);
      if (r->state == RQ_QUEUED) {
        for (auto it = S->queue.begin(); it != S->queue.end(); ++it)
          if (*it == r) {
            S->queue.erase(it);
            break;
          }
        // nothing was reserved for it; release its output slot lazily in wait
        r->out_off = SIZE_MAX;
        r->state = RQ_DONE;
        r->status = SKNR_ECANCELED;
        r->err = "request cancelled";
      } else if (r->state == RQ_RUNNING) {
        r->cancel.store(1);
      }
    }
    S->cv_done.notify_all();
    return SKNR_OK;
  });
}

int sknr_serve_stats(void* ctx, sknr_serve_info* out) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    REQUIRE(out, "out is NULL");
    std::memset(out, 0, sizeof(*out));
    Server* S = c->server;
    if (!S) return SKNR_OK;
    std::lock_guard<std::mutex> lk(S->mu);
    out->lanes = (int32_t)S->lanes.size();
    out->queued = (int32_t)S->queue.size();
    out->running = S->running;
    out->completed = S->completed;
    out->pool_bytes = S->pool.cap;
    out->pool_used = S->pool.used;
    out->pool_peak = S->pool.peak;
    if (S->batcher) {
      std::lock_guard<std::mutex> bl(S->batcher->mu);
      out->batches = S->batcher->batches;
      out->batched_jobs = S->batcher->jobs;
      out->batched_launches = S->batcher->launches;
    }
    return SKNR_OK;
  });
}

}  // extern "C"
