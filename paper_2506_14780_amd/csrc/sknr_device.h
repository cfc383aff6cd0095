// Device-side helpers shared by the sweep kernels of libsknr: double-float
// (hi, lo FP32) arithmetic, exp2/log2 builtins, gating, the fixed-order FP32
// squared distance, block reductions, the merge of online log-sum-exp states
// and the per-output epilogue of a c-transform sweep.
#pragma once
#include "sknr_internal.h"

#include <float.h>
#include <math.h>

namespace sknr {

#define SIG0 (-3.0e38f)
constexpr int TPB = 256;
constexpr int WAVES = TPB / 64;

// ------------------------------------------------------- double-float
__device__ __forceinline__ float2 two_sum(float a, float b) {
  float s = a + b;
  float bb = s - a;
  float e = (a - (s - bb)) + (b - bb);
  return make_float2(s, e);
}
__device__ __forceinline__ float2 fast_two_sum(float a, float b) {
  float s = a + b;
  float e = b - (s - a);
  return make_float2(s, e);
}
__device__ __forceinline__ float2 df_add(float2 a, float2 b) {
  float2 s = two_sum(a.x, b.x);
  float2 t = two_sum(a.y, b.y);
  s.y += t.x;
  s = fast_two_sum(s.x, s.y);
  s.y += t.y;
  return fast_two_sum(s.x, s.y);
}
__device__ __forceinline__ float2 df_add_f(float2 a, float b) {
  float2 s = two_sum(a.x, b);
  s.y += a.y;
  return fast_two_sum(s.x, s.y);
}
__device__ __forceinline__ float2 df_mul(float2 a, float2 b) {
  float p = a.x * b.x;
  float e = fmaf(a.x, b.x, -p);
  e = fmaf(a.x, b.y, e);
  e = fmaf(a.y, b.x, e);
  return fast_two_sum(p, e);
}
__device__ __forceinline__ float2 df_neg(float2 a) { return make_float2(-a.x, -a.y); }

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }

// Offset L of the streaming sweeps.  The reduce side enters as U + L (a
// normalised double-float (h, l), |U| <= maxabs) and the running max sig of
// a column is one of the values fl(h - C) with |C| <= cmax, so h lies in
// [L - maxabs, L + maxabs] and sig in [L - maxabs - cmax, L + maxabs].
// With L = 3 (cmax + maxabs), h / sig stays within [1/2, 2] (with a margin
// of cmax on both sides), so h - sig is exact (Sterbenz) and the exponent
// argument ((h - sig) - C + l) K is rounded only relative to its own size:
// it is formed as fma((h - sig) - C, K, l K) with l K staged per row.
__device__ __forceinline__ float sweep_offset(float cmax, float maxabs) { return 3.f * (cmax + maxabs); }


__device__ __forceinline__ float lg2(float x) { return __builtin_amdgcn_logf(x); }

// The flags are written by earlier kernels (visible at this kernel's
// start; no workgroup of a kernel writes them before every workgroup has
// read them): plain loads, issued together.
__device__ __forceinline__ bool gate_closed(const DevState* st, int gate) {
  if (!gate) return false;
  const int done = st->done, chol = st->chol_ok, acc = st->accept;
  if ((gate & G_NOT_DONE) && done) return true;
  if ((gate & G_CHOL_OK) && !chol) return true;
  if ((gate & G_ACCEPT) && !acc) return true;
  if ((gate & G_NOT_ACCEPT) && acc) return true;
  return false;
}

// squared distance in the fixed order k = 0..d-1 (the defined FP32 cost;
// symmetric in its arguments bit for bit since (p-q)^2 == (q-p)^2)
template <int D>
__device__ __forceinline__ float sqdist(const float* p, const float* q) {
  float t = p[0] - q[0];
  float acc = t * t;
#pragma unroll
  for (int k = 1; k < D; ++k) {
    t = p[k] - q[k];
    acc = fmaf(t, t, acc);
  }
  return acc;
}
__device__ __forceinline__ float sqdist_rt(const float* p, const float* q, int d) {
  float t = p[0] - q[0];
  float acc = t * t;
  for (int k = 1; k < d; ++k) {
    t = p[k] - q[k];
    acc = fmaf(t, t, acc);
  }
  return acc;
}

// ------------------------------------------------------ block reductions
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}
// deterministic block sum (fixed tree): result valid in thread 0
__device__ __forceinline__ double block_sum_d(double v, double* sbuf) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sbuf[w] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sbuf[i];
  }
  return r;
}
__device__ __forceinline__ float block_max_f(float v, float* sbuf) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sbuf[w] = v;
  __syncthreads();
  float r = 0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r = fmaxf(r, sbuf[i]);
  }
  return r;
}


// ----------------------------------------------------- LSE state merging
// (sig, S, Sc): the partial sum  sum exp2((t - sig)*K) = S + Sc.
__device__ __forceinline__ void lse_merge(float& sig, float& S, float& Sc, float sig2, float S2, float Sc2,
                                          float K, float& f1, float& f2) {
  float mx = fmaxf(sig, sig2);
  f1 = ex2((sig - mx) * K);
  f2 = ex2((sig2 - mx) * K);
  float p1 = S * f1, p2 = S2 * f2;
  float e1 = fmaf(S, f1, -p1), e2 = fmaf(S2, f2, -p2);
  float2 s = two_sum(p1, p2);
  Sc = fmaf(Sc, f1, fmaf(Sc2, f2, e1 + e2 + s.y));
  S = s.x;
  sig = mx;
}

// Finalise one output of a sweep from its merged (sig, S, Sc) and write the
// potential, the marginal-ratio term and the weighted average.
// Returns |mdiff| (error contribution), accumulates dot and max.
struct EpsConst {
  float K, inv_eps;
  float2 eps_df, eln2_df;
};
__device__ __forceinline__ EpsConst eps_const(const DevState* st) {
  EpsConst c;
  c.K = st->K;
  c.inv_eps = st->inv_eps;
  c.eps_df = st->eps_df;
  c.eln2_df = st->eln2_df;
  return c;
}

template <int ELL>
__device__ __forceinline__ void finalize_output(const SweepArgs& A, const EpsConst& E, int o, float L, float sig,
                                                float S, float Sc, const float* acc, double& err, double& dot,
                                                float& mx) {
  // log2(S + Sc) = k + log2(mant) + Sc/(S ln 2), S = mant * 2^k with mant
  // in [sqrt(1/2), sqrt(2)): a sum just above a power of two then gets a
  // small log of the mantissa (accurate relative to itself) instead of
  // log2(~0.5) ~ -1 whose last-bit error survives the cancellation with k
  int k;
  float mant = frexpf(S, &k);
  if (mant < 0.70710678f) {
    mant *= 2.f;
    k -= 1;
  }
  float lm = lg2(mant);
  float corr = (Sc / S) * 1.4426950408889634f;
  float2 l2 = fast_two_sum((float)k, lm);
  l2.y += corr;
  float2 t = df_mul(E.eln2_df, l2);
  float2 out = df_mul(E.eps_df, A.lw_out[o]);
  out = df_add_f(out, -sig);
  out = df_add_f(out, L);
  out = df_add(out, df_neg(t));
  if (ELL > 0 && A.wmode == W_CAND) {
    // candidate of the Newton step: T_c(f')_o = T_c(f)_o - eps log1p(w_o),
    // w_o = the softmax(f)-weighted average of expm1((f' - f)/eps); the
    // error slot collects sum_o w_out_o eps log1p(w_o) for Q(f') - Q(f)
    const double w = (double)acc[0] / ((double)S + (double)Sc);
    const double tt = ((double)E.eps_df.x + (double)E.eps_df.y) * log1p(w);
    const float th = (float)tt;
    out = df_add(out, make_float2(-th, -(float)(tt - (double)th)));
    err += A.w_out64[o] * tt;
  }
  A.Uout[o] = out;
  float ratio_m1 = 0.f;
  if (A.Uold) {
    float2 dlt = df_add(A.Uold[o], df_neg(out));
    ratio_m1 = expm1f((dlt.x + dlt.y) * E.inv_eps);
    float md = A.w_out[o] * ratio_m1;
    if (A.mdiff) A.mdiff[o] = md;
    err += fabs((double)md);
  }
  dot += A.w_out64[o] * ((double)out.x + (double)out.y);
  mx = fmaxf(mx, fabsf(out.x));
  if (ELL > 0 && A.wmode != W_CAND) {
    float inv = 1.f / (S + Sc);
    float scale = A.wmode == W_SCALE_WEIGHT ? A.w_out[o]
                  : A.wmode == W_SCALE_RATIO ? 1.f + ratio_m1
                  : A.wmode == W_SCALE_MASS  ? A.w_out[o] * (1.f + ratio_m1)
                                             : 1.f;
    scale *= inv;
#pragma unroll
    for (int l = 0; l < ELL; ++l) A.Wout[(size_t)o * ELL + l] = acc[l] * scale;
  }
}

// Per-block scalar partials of a sweep (error, dot, max) for the scalar
// finishing kernel.
// value of a double in lane k of the wave (k wave-uniform)
__device__ __forceinline__ double lane_read_d(double v, int k) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, k);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Store that is coherent across the device at once (agent scope; on
// gfx950 written through the XCD's L2), so that another workgroup can read
// it within the same kernel after an arrival count (arrive_count).
__device__ __forceinline__ void store_wt(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_wt(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Arrival count in *ctr: true in the workgroup that arrives last of
// `total` (a block-uniform result).  The data a workgroup hands on must
// have been written with store_wt: every thread waits for its stores to
// complete before the workgroup's arrival, and the last workgroup drops
// stale cached lines (acquire) before it reads them, so no cache
// write-back is needed.  The last workgroup resets the count, so it is
// zero again at the kernel's end.  Each of the `total` workgroups calls it
// once.  arrive_last counts a whole grid in st->tail_ctr (which a state
// reset also zeroes).
__device__ __forceinline__ bool arrive_count(unsigned* ctr, int total) {
  __shared__ int s_last;
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have completed
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int last = prev + 1u == (unsigned)total;
    if (last) __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = last;
  }
  __syncthreads();
  const bool last = s_last != 0;
  if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // drop stale lines
  return last;
}
__device__ __forceinline__ bool arrive_last(DevState* st, int nblk) { return arrive_count(&st->tail_ctr, nblk); }

// (read within the kernel by the finishing workgroup: coherent stores)
__device__ __forceinline__ void write_block_scalars(const SweepArgs& A, int bid, double err, double dot, float mx) {
  if (threadIdx.x == 0) {
    store_wt(A.blk_err + bid, err);
    store_wt(A.blk_dot + bid, dot);
    store_wt(A.blk_max + bid, mx);
  }
}

}  // namespace sknr
