// Host-side types shared by the engine (sknr_api.cpp) and the serving
// runtime (sknr_serve.cpp) of libsknr.  Internal; the public ABI is
// include/sknr.h.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sknr.h"
#include "sknr_internal.h"

namespace sknr_host {

using namespace sknr;

extern thread_local std::string g_last_error;


struct Err {
  int code;
  std::string msg;
};

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) throw Err{SKNR_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)
#define REQUIRE(cond, msg)                                   \
  do {                                                       \
    if (!(cond)) throw Err{SKNR_EINVAL, std::string(msg)};   \
  } while (0)

inline float2 split_df(double v) {
  float hi = (float)v;
  float lo = (float)(v - (double)hi);
  return make_float2(hi, lo);
}

// ------------------------------------------------------------------ arena
// One device allocation carved into aligned buffers; grown (reallocated)
// when a larger problem arrives.  Counters inside are zeroed at growth.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t off = 0;
  void reset() { off = 0; }
  void* take(size_t bytes) {
    size_t a = (off + 255) & ~size_t(255);
    if (a + bytes > cap) throw Err{SKNR_EINTERNAL, "arena overflow"};
    off = a + bytes;
    return base + a;
  }
};

// Per-kernel-kind timing with HIP events recorded on the launch stream
// around each sweep (enabled by sknr_profile).
struct ProfEntry {
  std::string name;
  long long launches = 0;
  double total_ms = 0;
  double units = 0;  // algorithmic elements (n_out * n_red) processed
};
struct Pending {
  int kind;
  hipEvent_t e0, e1;
  double units;
};
// A captured chunk of solver iterations.  Every pointer and constant baked
// into its kernel arguments is part of the key; eps-dependent values live
// in the device state, so one graph serves all stages of a schedule.
struct GraphKey {
  const void* ws;
  const void* C;
  const void* X;
  const void* Y;
  const void* wX;
  const void* wY;
  const void* xcost;  // transposed copy of a stored cost used by the sweeps (or null)
  long long ldc;
  int n, m, d, kind, ell, ellp, iters, ctrans;
  float cscale, cmax;
  void* stream;
  bool operator==(const GraphKey& o) const { return std::memcmp(this, &o, sizeof(GraphKey)) == 0; }
};
struct CachedGraph {
  GraphKey key;
  hipGraphExec_t exec;
};
// Batched execution of iteration chunks (serving): a lane records one unit
// (one SK-NR iteration, or two SK iterations) of its request's launches,
// uploads the argument blocks, and hands the batcher a job; the batcher
// runs the units of every job with the same kernel sequence as one launch
// per kernel over a tile table, `reps` times.
struct BatchLaunch {
  const void* bfunc;     // batched twin kernel
  const void* args_dev;  // the request's argument block (device)
  int gx, gy, block;
  unsigned lds;
};
struct BatchJob {
  const BatchLaunch* unit = nullptr;
  int nrec = 0;
  int reps = 0;            // repetitions of the unit requested
  hipEvent_t ev_in = nullptr;    // the request's stream up to the job
  hipEvent_t ev_done = nullptr;  // recorded by the batcher after the job's launches
  int reps_done = 0;       // set by the batcher
  bool launched = false;
  int status = 0;          // 0 or a HIP error
};
struct Batcher;
// Submit a job and block until the batcher has enqueued it together with
// the other requests' jobs; returns the repetitions run (>= 1).
int batcher_run(Batcher* b, BatchJob* job);
// A lane entering (+1) or leaving (-1) a stage's iteration loop: a batch
// waits (briefly) until every lane in an iteration loop has submitted, so
// the iterating requests fall into step and share their launches.
void batcher_iterating(Batcher* b, int delta);
constexpr int kMaxUnitLaunches = 64;

struct Lane {
  int device = 0;
  Batcher* batcher = nullptr;    // serving: batched iteration chunks
  LaunchRec* recbuf = nullptr;   // kMaxUnitLaunches records (host)
  BatchLaunch* units = nullptr;  // kMaxUnitLaunches (host)
  unsigned char* arg_pinned = nullptr;  // kMaxUnitLaunches * kMaxArgBytes (pinned)
  hipEvent_t ev_in = nullptr, ev_done = nullptr;
  Arena arena;                   // workspace (owned, or a block lent by the serving pool)
  bool arena_external = false;   // true: never reallocated or freed here
  // transposed copy of a large stored cost for the weighted sweeps along its
  // rows (owned lanes only; rebuilt by every call that uses it)
  float* xcost = nullptr;
  size_t xcost_cap = 0;
  hipStream_t own = nullptr;     // solver stream (default priority); graphs are captured on it
  bool use_graphs = true;
  const std::atomic<int>* cancel = nullptr;  // serving: abort flag polled between chunks
  std::vector<CachedGraph> graphs;
  void drop_graphs() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  }
  // workspace generation (make_ws counts up): a record of the arena's
  // contents is valid while its generation is current
  uint64_t ws_gen = 0;
  // the basis of the last sknr_solve (engine orientation, padded FP32 rows)
  struct Subspace {
    const float* V = nullptr;
    int n = 0, ellp = 0, ell = 0;
    bool transposed = false;
    uint64_t gen = 0;
  } sub;
  DevState* st_host = nullptr;  // pinned mirror of the state
  bool profile = false;
  std::vector<ProfEntry> prof;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> evpool;
  hipEvent_t get_event() {
    if (!evpool.empty()) {
      hipEvent_t e = evpool.back();
      evpool.pop_back();
      return e;
    }
    // timing only, between records on one stream: no system-scope fence
    // (it would add a write-back of L2 to every bracket)
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
      throw Err{SKNR_EDEVICE, "hipEventCreate failed"};
    return e;
  }
  int kind_of(const std::string& name) {
    for (size_t i = 0; i < prof.size(); ++i)
      if (prof[i].name == name) return (int)i;
    prof.push_back(ProfEntry{name});
    return (int)prof.size() - 1;
  }
  // after a stream synchronisation: fold completed event pairs
  void drain() {
    hipEvent_t last_e0 = nullptr;
    for (auto& p : pending) {
      hipEvent_t e0 = p.e0 ? p.e0 : last_e0;  // a ":main" entry starts at its sweep's start
      float ms = 0;
      if (e0 && hipEventElapsedTime(&ms, e0, p.e1) == hipSuccess) {
        prof[p.kind].launches += 1;
        prof[p.kind].total_ms += ms;
        prof[p.kind].units += p.units;
      }
      if (p.e0) last_e0 = p.e0;
    }
    for (auto& p : pending) {
      if (p.e0) evpool.push_back(p.e0);
      evpool.push_back(p.e1);
    }
    pending.clear();
  }
};

struct Prepared {
  // caller orientation
  int n0, m0;
  // engine orientation
  int n, m;
  bool transposed;
  int kind;
  const float* C;
  long long ldc;
  bool ctrans;  // engine element (i, j) is C[j*ldc + i]
  const float* X;  // points of side X (n x d)
  const float* Y;  // points of side Y (m x d)
  int d;
  float cscale;
  double cscale64;
  float cmax;
  // cross term of a SQEUCLID cost: 1 FP32 direct, 2 bf16, 3 bf16 hi/lo split,
  // 4 bf16 hi/mid/lo split
  int xmode = 0;
  int dpad = 0;          // bf16 rows: d rounded up to a multiple of 32
  std::vector<float> mu;  // centring point (bf16-rounded mean of all points)
  const double* wX;  // device FP64 weights
  const double* wY;
  // weight statistics (engine orientation): min, max, sum w log w
  double wminX = 1, wmaxX = 1, wminY = 1, wmaxY = 1;
  double entX = 0, entY = 0;
};

// A library context: the lane used by the synchronous entry points, the
// budget, and the serving runtime (created at the first submit).
struct Server;
struct Ctx {
  int device = 0;
  uint64_t budget = 0;
  void* prep = nullptr;  // kPrepBytes of device memory for prepare()
  // device copies of host-resident problem arrays (sknr_problem.on_host)
  char* stage = nullptr;
  size_t stage_cap = 0;
  Lane lane;
  Lane lane_na;  // sknr_solve_noalloc: workspace in the library's static device array, no graphs
  hipEvent_t order_ev = nullptr;  // orders the solver stream after the caller's stream
  Server* server = nullptr;
};

// lane set-up / tear-down (stream, pinned state mirror, graphs)
void lane_init(Lane* L, int device);
void lane_release(Lane* L);

int ell_pad(int ell);
void check_eps(double eps);
// dmax_dev: optional device float for the stored-cost bound (null: a
// stream-ordered allocation of 4 bytes)
// Validate a problem and gather what the solver needs about it; the input
// checks (weights positive, finite and summing to 1, finite points or cost)
// run on the device and come back in one read.  scratch: kPrepBytes of
// device memory (the context's block, or the static array's tail).
constexpr size_t kPrepBytes = 96 * 1024;
Prepared prepare(const sknr_problem* pr, hipStream_t s, void* scratch);
// A problem with host-resident arrays (on_host): copies them into the
// context's staging block on stream s and returns *tmp describing the
// device copies; any other problem is returned unchanged.
const sknr_problem* stage_problem(Ctx* c, const sknr_problem* pr, hipStream_t s, sknr_problem* tmp);
// point the device pointers of P at another copy of the same problem
void rebind(Prepared& P, const sknr_problem* pr);
size_t ws_bytes(const Prepared& P, int ellp, int* geo);
// validate solve options against the prepared problem
void check_opts(const sknr_opts* opts, const Prepared& P);
// Run a full solve (eps schedule) on a lane whose stream already follows
// any work the inputs depend on.  Outputs f_out, g_out (device, caller
// orientation) and res; returns OK or NOT_CONVERGED, throws Err on failure.
int solve_on_lane(Lane* L, const sknr_problem* prob, const Prepared& P, const sknr_opts* opts, double* f_out,
                  double* g_out, sknr_result* res);

void server_destroy(Ctx* c);

// sknr_noalloc.hip: the device address of the static workspace array on
// `device`, taken once per device with hipGetSymbolAddress (called by
// sknr_ctx_create with the device current), and its size in bytes
void noalloc_setup(int device);
char* noalloc_scratch(int device, size_t* bytes);

inline hipStream_t as_stream(void* p) { return reinterpret_cast<hipStream_t>(p); }

template <typename Fn>
int guarded(Fn fn) {
  try {
    return fn();
  } catch (const Err& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return SKNR_EINTERNAL;
  } catch (...) {
    g_last_error = "unknown error";
    return SKNR_EINTERNAL;
  }
}

inline Ctx* as_ctx(void* p) {
  if (!p) throw Err{SKNR_EINVAL, "context is NULL"};
  Ctx* c = reinterpret_cast<Ctx*>(p);
  HIPCHK(hipSetDevice(c->device));
  return c;
}

}  // namespace sknr_host
