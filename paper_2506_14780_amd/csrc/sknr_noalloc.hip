// Allocation-free full solve (sknr_solve_noalloc) for callers that cannot
// allocate device memory: code under graph capture, tight serving loops,
// harnesses that forbid hipMalloc.  The solver's workspace (potentials,
// split partials, the state block, the Newton and warm-start blocks) lives
// in `scratch`, a file-scope device array of kScratchBytes; each device the
// library runs on holds its own copy until the process ends.
//
// Host code never passes the array's name to a kernel or a copy: in host
// code the name is a host-side stand-in, not a device address.  The device
// address is taken once per device with hipGetSymbolAddress (noalloc_setup,
// called by sknr_ctx_create with that device current) and used from then
// on.  Every call on one device shares that device's array, which keeps
// the last call's contents: the solver resets its state block and loads
// its potentials before any kernel reads them, so nothing relies on zeros;
// calls that overlap on one device race (one at a time per device).
#include <mutex>

#include "sknr_host.h"

namespace sknr_host {

namespace {
constexpr size_t kScratchBytes = 64ull << 20;  // 64 MiB per device
constexpr size_t kTailBytes = kPrepBytes;      // tail: the scratch of prepare()
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
std::vector<char*> g_ptr;  // per device: the address of `scratch`, or null before set-up
}  // namespace

void noalloc_setup(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_ptr.size() <= device) g_ptr.resize(device + 1, nullptr);
  if (g_ptr[device]) return;
  int cur = -1;
  HIPCHK(hipGetDevice(&cur));
  if (cur != device) throw Err{SKNR_EINTERNAL, "noalloc_setup: device is not current"};
  void* p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Err{SKNR_EDEVICE, "hipGetSymbolAddress returned no address for the workspace array"};
  g_ptr[device] = static_cast<char*>(p);
}

char* noalloc_scratch(int device, size_t* bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (device < 0 || device >= (int)g_ptr.size() || !g_ptr[device])
    throw Err{SKNR_EINTERNAL, "allocation-free workspace not set up on this device"};
  if (bytes) *bytes = kScratchBytes;
  return g_ptr[device];
}

}  // namespace sknr_host

using namespace sknr_host;

extern "C" int sknr_solve_noalloc(void* ctx, const sknr_problem* prob, const sknr_opts* opts, double* f_out,
                                  double* g_out, sknr_result* res) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    REQUIRE(opts && res && f_out && g_out, "opts, res, f_out, g_out are required");
    REQUIRE(prob && !prob->on_host, "the allocation-free solve takes device-resident inputs only (on_host = 0)");
    size_t cap = 0;
    char* base = noalloc_scratch(c->device, &cap);
    Lane* L = &c->lane_na;
    hipStream_t cs = as_stream(opts->stream);
    hipStream_t s = L->own;
    HIPCHK(hipEventRecord(c->order_ev, cs));
    HIPCHK(hipStreamWaitEvent(s, c->order_ev, 0));
    // the scratch of prepare() goes to the array's last bytes, the
    // workspace below them
    Prepared P = prepare(prob, s, base + cap - kTailBytes);
    check_opts(opts, P);
    const size_t need = ws_bytes(P, ell_pad(opts->ell), nullptr);
    if (need > cap - kTailBytes)
      throw Err{SKNR_EINVAL, "workspace of " + std::to_string(need) + " bytes exceeds the " +
                                 std::to_string((cap - kTailBytes) >> 20) +
                                 " MiB limit of the allocation-free solve (use sknr_solve)"};
    L->arena.base = base;
    L->arena.cap = cap - kTailBytes;
    L->arena.off = 0;
    L->arena_external = true;
    L->use_graphs = false;  // graph instantiation may allocate
    return solve_on_lane(L, prob, P, opts, f_out, g_out, res);
  });
}
