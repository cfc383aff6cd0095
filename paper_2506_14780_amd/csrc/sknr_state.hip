// Device-side reset of the solver state block between stages, so that the
// host does not wait for the stream: the state is rebuilt from a template
// carrying the constants of the new eps (counters and flags zero), and with
// `keep` the slots describing the current potentials (max |U.hi| and the
// dots of F and G[0]) are carried over.
#include "sknr_internal.h"

namespace sknr {

__global__ void k_state_reset(DevState* st, DevState z, int keep) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (keep) {
    z.maxabs[MA_F] = st->maxabs[MA_F];
    z.maxabs[MA_G] = st->maxabs[MA_G];
    z.dots[DOT_F] = st->dots[DOT_F];
    z.dots[DOT_G] = st->dots[DOT_G];
  }
  *st = z;
}

hipError_t launch_state_reset(DevState* st, const DevState& z, bool keep, hipStream_t s) {
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, st, z, keep ? 1 : 0);
  return hipGetLastError();
}

}  // namespace sknr
