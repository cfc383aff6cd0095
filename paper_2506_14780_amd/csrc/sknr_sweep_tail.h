// Completion of a split-K sweep: the split merge of 64 outputs and the
// finishing reduction of a sweep's block scalars.
#pragma once
#include "sknr_internal.h"
#include "sknr_device.h"

namespace sknr {

// The last workgroup of a sweep's output kernel (merge, or the row sweep of
// a stored cost) to finish: reduce the per-block scalars in block order and
// update the solver state (error, dots, max, convergence and acceptance
// decisions).  The arrival count makes the other workgroups' scalars
// visible to it.
__device__ __forceinline__ void sweep_finish_body(const SweepArgs& A) {
  if (gate_closed(A.st, A.gate)) return;
  __shared__ double sbd[32];  // up to 16 waves
  __shared__ float sbf[16];
  double e = 0, d = 0;
  float m = 0;
  for (int b = threadIdx.x; b < A.nblk; b += blockDim.x) {
    e += A.blk_err[b];
    d += A.blk_dot[b];
    m = fmaxf(m, A.blk_max[b]);
  }
  e = block_sum_d(e, sbd);
  d = block_sum_d(d, sbd + 16);
  m = block_max_f(m, sbf);
  // the Newton update's scalars from its block partials (same order as a
  // one-workgroup reduction of them)
  double dax = 0, ddx = 0;
  float mxa = 0.f;
  if (A.aux_blkdot) {
    __shared__ double sbd2[32];
    __shared__ float sbf2[16];
    for (int b = threadIdx.x; b < A.aux_nblk; b += blockDim.x) {
      dax += A.aux_blkdot[b];
      if (A.aux_blkddot) ddx += A.aux_blkddot[b];
      mxa = fmaxf(mxa, A.aux_blkmax[b]);
    }
    dax = block_sum_d(dax, sbd2);
    ddx = block_sum_d(ddx, sbd2 + 16);
    mxa = block_max_f(mxa, sbf2);
  }
  if (threadIdx.x == 0) {
    DevState* st = A.st;
    if (A.aux_blkdot) {
      st->dots[A.aux_dot_slot] = dax;
      st->maxabs[A.aux_ma_slot] = mxa;
    }
    if (A.Uold) {
      if (A.mdiff) st->err_aux = e; else st->err = e;
    }
    if (A.dot_slot >= 0) st->dots[A.dot_slot] = d;
    if (A.ma_out >= 0) st->maxabs[A.ma_out] = m;
    if (A.flags & F_COUNT) st->npass += 1;
    if (A.flags & F_CHECK) {
      if (st->npass == 1) st->err1 = e;
      if (st->armed && e < st->tol) {
        st->done = 1;
        if (A.flags & F_GSEL) st->gsel = A.gsel_val;
      }
      st->armed = 1;
    }
    if (A.flags & F_ACCEPT_DQ) {
      // Q(f') - Q(f) = <f' - f, a> - sum_o b_o eps log1p(w_o): both terms are
      // accurate relative to themselves, so the sign is reliable where the
      // difference of two FP32 c-transform sums is not.  A step so large
      // that some w_o rounds to -1 (or overflows) gives a non-finite gain:
      // rejected, the SK step is taken
      const double dq = ddx - e;
      int acc = (st->chol_ok && dq > 0 && dq < INFINITY) ? 1 : 0;
      st->accept = acc;
      st->newton_accepted += acc;
    }
  }
}


// Merge the split-K partials of a sweep: LPO = merge_lanes(ELL) lanes per
// output, each merging a contiguous range of the splits in order, then a
// fixed shuffle tree across the LPO lanes (xor 1, 2, ...: neighbours first,
// so split order is preserved and the result is deterministic), and
// finalise.  A workgroup of 64 * LPO threads covers 64 outputs.
template <int ELL>
__device__ __forceinline__ void sweep_merge_block(const SweepArgs& A, const int bx) {
  constexpr int NQ = 3 + (ELL > 0 ? ELL : 0);
  constexpr int EL = ELL > 0 ? ELL : 1;
  constexpr int LPO = merge_lanes(ELL);
  constexpr int OPB = 64;
  const EpsConst EC = eps_const(A.st);
  const float K = EC.K;
  const float L = sweep_offset_bound(A, A.st->maxabs[A.ma_in], A.st->eps);
  const int n_out = A.n_out;
  const int col = bx * OPB + (int)threadIdx.x / LPO, part = (int)threadIdx.x % LPO;
  const int colc = min(col, n_out - 1);
  const int ns = A.nsplit;
  const int per = (ns + LPO - 1) / LPO;
  const int s0 = part * per, s1 = min(ns, s0 + per);
  const float* pp = A.part + colc;
  const size_t stride = (size_t)n_out;
  float sg = SIG0, Ss = 0.f, Sx = 0.f;
  float ac[EL];
#pragma unroll
  for (int l = 0; l < EL; ++l) ac[l] = 0.f;
  constexpr int BATCH = ELL > 0 ? 4 : 16;
  for (int sp0 = s0; sp0 < s1; sp0 += BATCH) {
    float bs[BATCH], bS[BATCH], bC[BATCH];
    float ba[BATCH][EL];
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int sp = min(sp0 + q, ns - 1);
      const float* q2 = pp + (size_t)sp * NQ * stride;
      bs[q] = q2[0];
      bS[q] = q2[stride];
      bC[q] = q2[2 * stride];
#pragma unroll
      for (int l = 0; l < (ELL > 0 ? ELL : 0); ++l) ba[q][l] = q2[(3 + l) * stride];
    }
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      if (sp0 + q < s1) {
        float f1, f2;
        lse_merge(sg, Ss, Sx, bs[q], bS[q], bC[q], K, f1, f2);
#pragma unroll
        for (int l = 0; l < (ELL > 0 ? ELL : 0); ++l) ac[l] = ac[l] * f1 + ba[q][l] * f2;
      }
    }
  }
  // neighbouring lanes first: split order is preserved
#pragma unroll
  for (int off = 1; off < LPO; off <<= 1) {
    float sg2 = __shfl_xor(sg, off, 64), S2 = __shfl_xor(Ss, off, 64), C2 = __shfl_xor(Sx, off, 64);
    float a2[EL];
#pragma unroll
    for (int l = 0; l < (ELL > 0 ? ELL : 0); ++l) a2[l] = __shfl_xor(ac[l], off, 64);
    const bool lower = (part & off) == 0;
    float f1, f2;
    if (lower) {
      lse_merge(sg, Ss, Sx, sg2, S2, C2, K, f1, f2);
#pragma unroll
      for (int l = 0; l < (ELL > 0 ? ELL : 0); ++l) ac[l] = ac[l] * f1 + a2[l] * f2;
    } else {
      float t1 = sg2, t2 = S2, t3 = C2;
      lse_merge(t1, t2, t3, sg, Ss, Sx, K, f1, f2);
#pragma unroll
      for (int l = 0; l < (ELL > 0 ? ELL : 0); ++l) ac[l] = a2[l] * f1 + ac[l] * f2;
      sg = t1;
      Ss = t2;
      Sx = t3;
    }
  }
  double err = 0, dot = 0;
  float mxo = 0.f;
  if (col < n_out && part == 0) finalize_output<ELL>(A, EC, col, L, sg, Ss, Sx, ac, err, dot, mxo);
  __shared__ double sbd[32];  // up to 16 waves
  __shared__ float sbf[16];
  err = block_sum_d(err, sbd);
  dot = block_sum_d(dot, sbd + 16);
  mxo = block_max_f(mxo, sbf);
  write_block_scalars(A, bx, err, dot, mxo);
}
}  // namespace sknr
