// HIP kernels of libsknr for gfx950 (MI355X).
//
// The hot path is the c-transform sweep (paper Sec. 2, eq. foc_f / foc_g):
//   out_o = eps*log(w_o) - eps*log sum_r exp((U_r - C_ro)/eps),
// with hat potentials U = potential + eps*log(weight), so that the weights
// fold into the exponent.  A sweep reads (or builds) every cost element once
// and runs an online max-shifted log-sum-exp in FP32.  Precision (the FP32
// exponent (U_r - C_ro)/eps cancels O(|C|) terms down to O(eps)) is kept by:
//   * double-float potentials (hi, lo FP32 pairs);
//   * an argument formed without cancellation error: after offsetting U by
//     L = 3 (max|C| + max|U|) the difference of (U + L) and the running max
//     is exact (Sterbenz), and C is subtracted from that small difference
//     (streaming sweeps); TwoSum in the row sweep of a stored cost;
//   * compensated accumulation of the exponentials and of the split merges;
//   * log of the sum split into exponent + log2 of the mantissa.
// Everything else (cross-block merges, epilogues) works on O(n + m) data.
#include "sknr_internal.h"
#include "sknr_device.h"
#include "sknr_sweep_tail.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>

#include <type_traits>

namespace sknr {

thread_local Recorder* g_recorder = nullptr;

// ============================================================================
// Streaming sweep: each workgroup owns NC = 64*CPT outputs (lane-contiguous
// groups of CPT) and a contiguous range of the reduce side (split-K).  Its 4
// waves take interleaved reduce rows; per row the reduce-side data
// (offset potential, point) is a wave-uniform LDS broadcast.  For a stored
// cost the outputs are columns of the row-major C, so each wave reads
// 64*CPT*4 contiguous bytes per row.  Per-wave states merge through LDS and
// the workgroup writes its (sig, S, Sc, acc) partial; the merge kernel then
// combines the splits of each output in split order (deterministic).
// ============================================================================
template <int CPT, int ELL, int COST, int D, int R, bool SCALE>
__device__ __forceinline__ void sweep_stream_body(const SweepArgs& A, const int bx, const int by) {
  if (gate_closed(A.st, A.gate)) return;
  extern __shared__ float4 smem4[];
  char* smem = reinterpret_cast<char*>(smem4);
  constexpr int NC = 64 * CPT;
  constexpr int DD = (COST == 1) ? (D > 0 ? D : 1) : 1;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r0 = by * A.rows_per_split;
  const int nr = min(A.rows_per_split, A.n_red - r0);
  // points: dg coordinates in memory; d = the compile-time width D >= dg
  // (rows zero-padded in LDS and registers, which leaves the FP32 cost
  // unchanged: the padded terms are fma(0, 0, acc)), or dg when D == 0
  const int dg = A.d;
  const int d = (COST == 1 && D > 0) ? D : dg;
  const EpsConst EC = eps_const(A.st);
  const float K = EC.K;
  const float L = sweep_offset(A.cmax, A.st->maxabs[A.ma_in]);

  // sU[r] = (h, l K) of the offset potential U_r + L = h + l
  float2* sU = reinterpret_cast<float2*>(smem);
  float* sX = reinterpret_cast<float*>(smem + (size_t)A.rows_per_split * sizeof(float2));
  for (int t = threadIdx.x; t < nr; t += TPB) {
    float2 u = A.Uin[r0 + t];
    float2 s = two_sum(L, u.x);
    s.y += u.y;
    s = fast_two_sum(s.x, s.y);
    sU[t] = make_float2(s.x, s.y * K);
    if (COST == 1) {
      for (int k = 0; k < d; ++k) sX[t * d + k] = k < dg ? A.Pred[(size_t)(r0 + t) * dg + k] : 0.f;
    }
  }
  __syncthreads();

  const int colbase = bx * NC + lane * CPT;
  float q[CPT][DD];
  const float* crow0 = nullptr;
  int ccol[CPT];
  if (COST == 1) {
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      int col = min(colbase + c, A.n_out - 1);
      if (D > 0) {
#pragma unroll
        for (int k = 0; k < DD; ++k) q[c][k] = k < dg ? A.Pout[(size_t)col * dg + k] : 0.f;
      }
      ccol[c] = col;
    }
  } else {
#pragma unroll
    for (int c = 0; c < CPT; ++c) ccol[c] = min(colbase + c, A.n_out - 1);
    if (CPT == 4) ccol[0] = min(colbase, A.n_out - 4);  // vector path: n_out % 4 == 0
    crow0 = A.C + ccol[0];
  }

  float sig[CPT], S[CPT], Sc[CPT];
  float acc[CPT][ELL > 0 ? ELL : 1];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    sig[c] = SIG0;
    S[c] = 0.f;
    Sc[c] = 0.f;
#pragma unroll
    for (int l = 0; l < (ELL > 0 ? ELL : 1); ++l) acc[c][l] = 0.f;
  }

  // one chunk of R rows per wave (MASK: rows past nr present)
  auto chunk = [&](auto maskc, int rb) __attribute__((always_inline)) {
    constexpr bool MASK = decltype(maskc)::value;
    float s[R][CPT], cvr[R][CPT], ux[R], uk[R];
    bool okr[R];
    int rowl[R];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      int rl = rb + rr * WAVES;
      bool ok = MASK ? rl < nr : true;
      int rlc = ok ? rl : (nr - 1);
      rowl[rr] = rlc;
      okr[rr] = ok;
      float2 u = sU[rlc];
      ux[rr] = u.x;
      uk[rr] = u.y;
      float cv[CPT];
      if (COST == 0) {
        const float* crow = crow0 + (size_t)(r0 + rlc) * A.ldc;
        if (CPT == 4) {
          float4 v = *reinterpret_cast<const float4*>(crow);
          cv[0] = v.x; cv[1 % CPT] = v.y; cv[2 % CPT] = v.z; cv[3 % CPT] = v.w;
        } else {
#pragma unroll
          for (int c = 0; c < CPT; ++c) cv[c] = A.C[(size_t)(r0 + rlc) * A.ldc + ccol[c]];
        }
      } else {
        const float* xp = &sX[rlc * d];
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          float cc;
          if (D > 0) cc = sqdist<DD>(xp, q[c]);
          else cc = sqdist_rt(xp, A.Pout + (size_t)ccol[c] * d, d);
          cv[c] = SCALE ? cc * A.cscale : cc;
        }
      }
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        cvr[rr][c] = cv[c];
        s[rr][c] = ok ? u.x - cv[c] : SIG0;
      }
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      float mx = s[0][c];
#pragma unroll
      for (int rr = 1; rr < R; ++rr) mx = fmaxf(mx, s[rr][c]);
      if (mx > sig[c]) {
        float sc = ex2((sig[c] - mx) * K);
        S[c] *= sc;
        Sc[c] *= sc;
#pragma unroll
        for (int l = 0; l < (ELL > 0 ? ELL : 0); ++l) acc[c][l] *= sc;
        sig[c] = mx;
      }
      float p[R];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const float pv = ex2(fmaf((ux[rr] - sig[c]) - cvr[rr][c], K, uk[rr]));
        p[rr] = (!MASK || okr[rr]) ? pv : 0.f;
      }
      // pairwise sum of the chunk, then a compensated add
      float t[R];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) t[rr] = p[rr];
#pragma unroll
      for (int w = 1; w < R; w <<= 1) {
#pragma unroll
        for (int rr = 0; rr + w < R; rr += 2 * w) t[rr] += t[rr + w];
      }
      float2 ts = two_sum(S[c], t[0]);
      S[c] = ts.x;
      Sc[c] += ts.y;
      if (ELL > 0) {
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          const float* vr = A.Vred + (size_t)(r0 + rowl[rr]) * (ELL > 0 ? ELL : 1);
#pragma unroll
          for (int l = 0; l < (ELL > 0 ? ELL : 0); ++l) acc[c][l] = fmaf(p[rr], vr[l], acc[c][l]);
        }
      }
    }
  };
  // full chunks, then at most one chunk with rows past nr
  int rb = wave;
  for (; rb + (R - 1) * WAVES < nr; rb += WAVES * R) chunk(std::integral_constant<bool, false>{}, rb);
  if (rb < nr) chunk(std::integral_constant<bool, true>{}, rb);

  // ---- merge the 4 waves through LDS, in wave order (deterministic)
  __syncthreads();
  constexpr int ELLZ = ELL > 0 ? ELL : 0;
  constexpr int NQ = 3 + ELLZ;
  float* cmb = reinterpret_cast<float*>(smem);  // [NQ][NC]
  for (int w = 0; w < WAVES; ++w) {
    if (wave == w) {
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const int idx = lane * CPT + c;
        if (w > 0) {
          float sg = cmb[0 * NC + idx], Ss = cmb[1 * NC + idx], Sx = cmb[2 * NC + idx];
          float f1, f2;
          lse_merge(sg, Ss, Sx, sig[c], S[c], Sc[c], K, f1, f2);
#pragma unroll
          for (int l = 0; l < ELLZ; ++l) acc[c][l] = cmb[(3 + l) * NC + idx] * f1 + acc[c][l] * f2;
          sig[c] = sg;
          S[c] = Ss;
          Sc[c] = Sx;
        }
        cmb[0 * NC + idx] = sig[c];
        cmb[1 * NC + idx] = S[c];
        cmb[2 * NC + idx] = Sc[c];
#pragma unroll
        for (int l = 0; l < ELLZ; ++l) cmb[(3 + l) * NC + idx] = acc[c][l];
      }
    }
    __syncthreads();
  }
  const int n_out = A.n_out;
  for (int t = threadIdx.x; t < NC; t += TPB) {
    int col = bx * NC + t;
    if (col < n_out) {
      size_t base = (size_t)by * NQ * n_out + col;
#pragma unroll
      for (int q2 = 0; q2 < NQ; ++q2) store_wt(A.part + base + q2 * (size_t)n_out, cmb[q2 * NC + t]);
    }
  }
}

template <int CPT, int ELL, int COST, int D, int R, bool SCALE>
__global__ __launch_bounds__(TPB) void k_sweep_stream(SweepArgs A) {
  sweep_stream_body<CPT, ELL, COST, D, R, SCALE>(A, blockIdx.x, blockIdx.y);
}
template <int CPT, int ELL, int COST, int D, int R, bool SCALE>
__global__ __launch_bounds__(TPB) void k_sweep_stream_b(BatchTab T) {
  int bx, by;
  const int slot = batch_slot(T, blockIdx.x, &bx, &by);
  sweep_stream_body<CPT, ELL, COST, D, R, SCALE>(*static_cast<const SweepArgs*>(T.args[slot]), bx, by);
}

template <int ELL>
__device__ __forceinline__ void sweep_merge_body(const SweepArgs& A, const int bx) {
  if (gate_closed(A.st, A.gate)) return;
  sweep_merge_block<ELL>(A, bx);
  if (arrive_last(A.st, A.nblk)) sweep_finish_body(A);
}

template <int ELL>
__global__ __launch_bounds__(64 * merge_lanes(ELL)) void k_sweep_merge(SweepArgs A) {
  sweep_merge_body<ELL>(A, blockIdx.x);
}
template <int ELL>
__global__ __launch_bounds__(64 * merge_lanes(ELL)) void k_sweep_merge_b(BatchTab T) {
  int bx, by;
  const int slot = batch_slot(T, blockIdx.x, &bx, &by);
  sweep_merge_body<ELL>(*static_cast<const SweepArgs*>(T.args[slot]), bx);
}

// ============================================================================
// Row sweep of a stored cost: the outputs are rows of C (n_out = rows), the
// reduce side runs along each row.  A workgroup owns RPW rows; its threads
// stride over the row in float4 groups (coalesced), each thread keeps an
// online (sig, S, Sc) per row, then wave shuffles and LDS merge them.
// The subtraction U_r - C_ro uses TwoSum (no precondition).
// ============================================================================
template <int RPW, int ELL, bool VEC4>
__global__ __launch_bounds__(TPB) void k_sweep_rows(SweepArgs A) {
  if (gate_closed(A.st, A.gate)) return;
  const EpsConst EC = eps_const(A.st);
  const float K = EC.K;
  const int o0 = blockIdx.x * RPW;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int EL = ELL > 0 ? ELL : 1;
  float sig[RPW], S[RPW], Sc[RPW], acc[RPW][EL];
  const float* crow[RPW];
#pragma unroll
  for (int rr = 0; rr < RPW; ++rr) {
    sig[rr] = SIG0;
    S[rr] = 0.f;
    Sc[rr] = 0.f;
#pragma unroll
    for (int l = 0; l < EL; ++l) acc[rr][l] = 0.f;
    int o = min(o0 + rr, A.n_out - 1);
    crow[rr] = A.C + (size_t)o * A.ldc;
  }
  const int nr = A.n_red;
  if (VEC4) {
    const int ng = nr >> 2;
    const float4* U4 = reinterpret_cast<const float4*>(A.Uin);
    for (int g = threadIdx.x; g < ng; g += TPB) {
      float4 ua = U4[2 * g], ub = U4[2 * g + 1];  // (hi0, lo0, hi1, lo1), (hi2, lo2, hi3, lo3)
      float uh[4] = {ua.x, ua.z, ub.x, ub.z};
      float ul[4] = {ua.y, ua.w, ub.y, ub.w};
#pragma unroll
      for (int rr = 0; rr < RPW; ++rr) {
        float4 cv4 = *reinterpret_cast<const float4*>(crow[rr] + 4 * g);
        float cv[4] = {cv4.x, cv4.y, cv4.z, cv4.w};
        float s[4], e[4];
        float mx = SIG0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          float2 ts = two_sum(uh[k], -cv[k]);
          s[k] = ts.x;
          e[k] = ts.y + ul[k];
          mx = fmaxf(mx, s[k]);
        }
        if (mx > sig[rr]) {
          float sc = ex2((sig[rr] - mx) * K);
          S[rr] *= sc;
          Sc[rr] *= sc;
#pragma unroll
          for (int l = 0; l < (ELL > 0 ? ELL : 0); ++l) acc[rr][l] *= sc;
          sig[rr] = mx;
        }
        float p[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) p[k] = ex2(((s[k] - sig[rr]) + e[k]) * K);
        float2 ts = two_sum(S[rr], (p[0] + p[1]) + (p[2] + p[3]));
        S[rr] = ts.x;
        Sc[rr] += ts.y;
        if (ELL > 0) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const float* vr = A.Vred + (size_t)(4 * g + k) * EL;
#pragma unroll
            for (int l = 0; l < (ELL > 0 ? ELL : 0); ++l) acc[rr][l] = fmaf(p[k], vr[l], acc[rr][l]);
          }
        }
      }
    }
  } else {
    for (int j = threadIdx.x; j < nr; j += TPB) {
      float2 u = A.Uin[j];
#pragma unroll
      for (int rr = 0; rr < RPW; ++rr) {
        float cvv = crow[rr][j];
        float2 ts = two_sum(u.x, -cvv);
        float s = ts.x, e = ts.y + u.y;
        if (s > sig[rr]) {
          float sc = ex2((sig[rr] - s) * K);
          S[rr] *= sc;
          Sc[rr] *= sc;
#pragma unroll
          for (int l = 0; l < (ELL > 0 ? ELL : 0); ++l) acc[rr][l] *= sc;
          sig[rr] = s;
        }
        float p = ex2(((s - sig[rr]) + e) * K);
        float2 t2 = two_sum(S[rr], p);
        S[rr] = t2.x;
        Sc[rr] += t2.y;
        if (ELL > 0) {
          const float* vr = A.Vred + (size_t)j * EL;
#pragma unroll
          for (int l = 0; l < (ELL > 0 ? ELL : 0); ++l) acc[rr][l] = fmaf(p, vr[l], acc[rr][l]);
        }
      }
    }
  }
  // ---- wave merge (butterfly), then LDS merge across waves
#pragma unroll
  for (int rr = 0; rr < RPW; ++rr) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      float sg2 = __shfl_xor(sig[rr], off, 64);
      float S2 = __shfl_xor(S[rr], off, 64);
      float Sc2 = __shfl_xor(Sc[rr], off, 64);
      float f1, f2;
      float a2[EL];
#pragma unroll
      for (int l = 0; l < (ELL > 0 ? ELL : 0); ++l) a2[l] = __shfl_xor(acc[rr][l], off, 64);
      lse_merge(sig[rr], S[rr], Sc[rr], sg2, S2, Sc2, K, f1, f2);
#pragma unroll
      for (int l = 0; l < (ELL > 0 ? ELL : 0); ++l) acc[rr][l] = acc[rr][l] * f1 + a2[l] * f2;
    }
  }
  constexpr int NQ = 3 + (ELL > 0 ? ELL : 0);
  __shared__ float cmb[WAVES][RPW][NQ];
  if (lane == 0) {
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
      cmb[wave][rr][0] = sig[rr];
      cmb[wave][rr][1] = S[rr];
      cmb[wave][rr][2] = Sc[rr];
#pragma unroll
      for (int l = 0; l < (ELL > 0 ? ELL : 0); ++l) cmb[wave][rr][3 + l] = acc[rr][l];
    }
  }
  __syncthreads();
  double err = 0, dot = 0;
  float mxo = 0.f;
  if (threadIdx.x < RPW && o0 + (int)threadIdx.x < A.n_out) {
    const int rr = threadIdx.x;
    float sg = cmb[0][rr][0], Ss = cmb[0][rr][1], Sx = cmb[0][rr][2];
    float ac[EL];
#pragma unroll
    for (int l = 0; l < (ELL > 0 ? ELL : 0); ++l) ac[l] = cmb[0][rr][3 + l];
    for (int w = 1; w < WAVES; ++w) {
      float f1, f2;
      lse_merge(sg, Ss, Sx, cmb[w][rr][0], cmb[w][rr][1], cmb[w][rr][2], K, f1, f2);
#pragma unroll
      for (int l = 0; l < (ELL > 0 ? ELL : 0); ++l) ac[l] = ac[l] * f1 + cmb[w][rr][3 + l] * f2;
    }
    finalize_output<ELL>(A, EC, o0 + rr, 0.f, sg, Ss, Sx, ac, err, dot, mxo);
  }
  __shared__ double sbd[16];
  __shared__ float sbf[8];
  err = block_sum_d(err, sbd);
  dot = block_sum_d(dot, sbd + 8);
  mxo = block_max_f(mxo, sbf);
  write_block_scalars(A, blockIdx.x, err, dot, mxo);
  if (arrive_last(A.st, A.nblk)) sweep_finish_body(A);
}

// ----------------------------------------------------------- launch config
// LDS / register width of the points of a streaming sweep: d itself up to
// 8 (one kernel per d), else padded to 16, 32 or 64, else d (generic loop)
static int point_width(int d) {
  if (d <= 8) return d;
  if (d <= 16) return 16;
  if (d <= 32) return 32;
  if (d <= 64) return 64;
  return d;
}

static int rps_max(int cost_kind, int d) {
  if (cost_kind == 0) return 4096;                   // 8 B per row of LDS
  int per = 8 + 4 * point_width(d);
  int cap = (40 * 1024) / per;
  return cap < 16 ? 16 : cap;
}

// outputs per thread of the streaming sweep (shared by sizing and launch)
static int stream_cpt(int cost_kind, int ell, bool vec, int d) {
  if (cost_kind == 0) {
    if (ell > 16) return 2;
    return vec ? 4 : 1;
  }
  if (d > 8 && d <= 64) return 1;  // padded widths: the points of one output fill the registers
  return ell > 0 ? 2 : 4;
}

size_t sweep_part_floats(int n_out, int n_red, int ell, int cost_kind, int d, bool vec, int* nsplit, int* rps,
                         int* nblk, bool stream_kernel) {
  if (cost_kind >= 2) return mfma_part_floats(n_out, n_red, ell, cost_kind - 1, nsplit, rps, nblk);
  if (cost_kind == 1 && stream_kernel && sweep_pw_eligible(ell, d))
    return mfma_part_floats(n_out, n_red, ell, 0, nsplit, rps, nblk);
  if (!stream_kernel) {
    int rpw = ell > 0 ? 1 : 4;
    *nsplit = 1;
    *rps = n_red;
    *nblk = (n_out + rpw - 1) / rpw;
    return 0;
  }
  int cpt = stream_cpt(cost_kind, ell, vec, d);
  int nc = 64 * cpt;
  int ncb = (n_out + nc - 1) / nc;
  // split-K geometry: about `target` workgroups, at least `rmin` reduce
  // rows each (SKNR_SWEEP_TARGET_WG / SKNR_SWEEP_MIN_ROWS override)
  static const int env_target = getenv("SKNR_SWEEP_TARGET_WG") ? atoi(getenv("SKNR_SWEEP_TARGET_WG")) : 0;
  static const int env_rmin = getenv("SKNR_SWEEP_MIN_ROWS") ? atoi(getenv("SKNR_SWEEP_MIN_ROWS")) : 0;
  int target = env_target > 0 ? env_target : 2048;
  int ns = (target + ncb - 1) / ncb;
  int r = (n_red + ns - 1) / ns;
  int rmin = env_rmin > 0 ? env_rmin : (ell > 0 ? 128 : 64);
  if (r < rmin) r = rmin;
  int rmx = rps_max(cost_kind, d);
  if (r > rmx) r = rmx;
  if (r > n_red) r = n_red;
  ns = (n_red + r - 1) / r;
  *nsplit = ns;
  *rps = r;
  *nblk = merge_blocks(n_out, ell);
  (void)ncb;
  int ellp = ell <= 0 ? 0 : (ell <= 8 ? 8 : (ell <= 16 ? 16 : 32));
  return (size_t)ns * (3 + ellp) * n_out;
}

template <int CPT, int ELL, int COST, int D, int R>
static hipError_t go_stream(const SweepArgs& a, hipStream_t s, hipEvent_t mid) {
  constexpr int NC = 64 * CPT;
  int ncb = (a.n_out + NC - 1) / NC;
  dim3 grid(ncb, a.nsplit);
  size_t rows_bytes = (size_t)a.rows_per_split * (8 + (COST == 1 ? 4 * (D > 0 ? D : a.d) : 0));
  size_t cmb_bytes = (size_t)(3 + ELL) * NC * 4;
  size_t sm = rows_bytes > cmb_bytes ? rows_bytes : cmb_bytes;
  bool scale = (COST == 1) && a.cscale != 1.0f;
  if (g_recorder) {
    record_launch(scale ? (const void*)k_sweep_stream_b<CPT, ELL, COST, D, R, true>
                        : (const void*)k_sweep_stream_b<CPT, ELL, COST, D, R, false>,
                  a, grid, TPB, sm);
    record_launch((const void*)k_sweep_merge_b<ELL>, a, dim3(merge_blocks(a.n_out, ELL)), 64 * merge_lanes(ELL), 0);
    return hipSuccess;
  }
  if (scale)
    hipLaunchKernelGGL((k_sweep_stream<CPT, ELL, COST, D, R, true>), grid, dim3(TPB), sm, s, a);
  else
    hipLaunchKernelGGL((k_sweep_stream<CPT, ELL, COST, D, R, false>), grid, dim3(TPB), sm, s, a);
  if (mid) (void)hipEventRecord(mid, s);
  hipLaunchKernelGGL((k_sweep_merge<ELL>), dim3(merge_blocks(a.n_out, ELL)), dim3(64 * merge_lanes(ELL)), 0, s, a);
  return hipGetLastError();
}

template <int CPT, int ELL>
static hipError_t go_stream_points(const SweepArgs& a, hipStream_t s, hipEvent_t mid) {
  switch (a.d) {
    case 1: return go_stream<CPT, ELL, 1, 1, 4>(a, s, mid);
    case 2: return go_stream<CPT, ELL, 1, 2, 4>(a, s, mid);
    case 3: return go_stream<CPT, ELL, 1, 3, 4>(a, s, mid);
    case 4: return go_stream<CPT, ELL, 1, 4, 4>(a, s, mid);
    case 5: return go_stream<CPT, ELL, 1, 5, 2>(a, s, mid);
    case 6: return go_stream<CPT, ELL, 1, 6, 2>(a, s, mid);
    case 7: return go_stream<CPT, ELL, 1, 7, 2>(a, s, mid);
    case 8: return go_stream<CPT, ELL, 1, 8, 2>(a, s, mid);
    default:
      if (a.d <= 16) return go_stream<1, ELL, 1, 16, 2>(a, s, mid);
      if (a.d <= 32) return go_stream<1, ELL, 1, 32, 2>(a, s, mid);
      if (a.d <= 64) return go_stream<1, ELL, 1, 64, 2>(a, s, mid);
      return go_stream<CPT, ELL, 1, 0, 2>(a, s, mid);
  }
}

hipError_t launch_sweep_tail(const SweepArgs& a, hipStream_t s) {
  dim3 grid(merge_blocks(a.n_out, a.ell));
  if (g_recorder) {
    record_launch(a.ell == 0 ? (const void*)k_sweep_merge_b<0>
                  : a.ell <= 8 ? (const void*)k_sweep_merge_b<8>
                  : a.ell <= 16 ? (const void*)k_sweep_merge_b<16>
                                : (const void*)k_sweep_merge_b<32>,
                  a, grid, 64 * merge_lanes(a.ell), 0);
    return hipSuccess;
  }
  if (a.ell == 0) hipLaunchKernelGGL((k_sweep_merge<0>), grid, dim3(64 * merge_lanes(0)), 0, s, a);
  else if (a.ell <= 8) hipLaunchKernelGGL((k_sweep_merge<8>), grid, dim3(64 * merge_lanes(8)), 0, s, a);
  else if (a.ell <= 16) hipLaunchKernelGGL((k_sweep_merge<16>), grid, dim3(64 * merge_lanes(16)), 0, s, a);
  else hipLaunchKernelGGL((k_sweep_merge<32>), grid, dim3(64 * merge_lanes(32)), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sweep_stream(const SweepArgs& a, int cost_kind, bool vec, hipStream_t s, hipEvent_t mid) {
  if (cost_kind >= 2) return launch_sweep_mfma(a, cost_kind - 1, s, mid);
  if (cost_kind == 1 && sweep_pw_eligible(a.ell, a.d)) return launch_sweep_pw(a, s, mid);
  const int cpt = stream_cpt(cost_kind, a.ell, vec, a.d);
  if (cost_kind == 0) {
    if (a.ell == 0) return cpt == 4 ? go_stream<4, 0, 0, 1, 8>(a, s, mid) : go_stream<1, 0, 0, 1, 8>(a, s, mid);
    if (a.ell <= 8) return cpt == 4 ? go_stream<4, 8, 0, 1, 4>(a, s, mid) : go_stream<1, 8, 0, 1, 4>(a, s, mid);
    if (a.ell <= 16) return cpt == 4 ? go_stream<4, 16, 0, 1, 4>(a, s, mid) : go_stream<1, 16, 0, 1, 4>(a, s, mid);
    return go_stream<2, 32, 0, 1, 4>(a, s, mid);
  }
  if (a.ell == 0) return go_stream_points<4, 0>(a, s, mid);
  if (a.ell <= 8) return go_stream_points<2, 8>(a, s, mid);
  if (a.ell <= 16) return go_stream_points<2, 16>(a, s, mid);
  return go_stream_points<2, 32>(a, s, mid);
}

hipError_t launch_sweep_rows(const SweepArgs& a, hipStream_t s, hipEvent_t mid) {
  if (g_recorder) {  // stored-cost row sweeps have no batched twin
    g_recorder->unsupported = true;
    return hipSuccess;
  }
  bool vec = (a.n_red % 4 == 0) && (a.ldc % 4 == 0) && ((uintptr_t)a.C % 16 == 0) && ((uintptr_t)a.Uin % 16 == 0);
  if (a.ell == 0) {
    dim3 grid((a.n_out + 3) / 4);
    if (vec) hipLaunchKernelGGL((k_sweep_rows<4, 0, true>), grid, dim3(TPB), 0, s, a);
    else hipLaunchKernelGGL((k_sweep_rows<4, 0, false>), grid, dim3(TPB), 0, s, a);
  } else {
    dim3 grid(a.n_out);
    if (a.ell <= 8) {
      if (vec) hipLaunchKernelGGL((k_sweep_rows<1, 8, true>), grid, dim3(TPB), 0, s, a);
      else hipLaunchKernelGGL((k_sweep_rows<1, 8, false>), grid, dim3(TPB), 0, s, a);
    } else if (a.ell <= 16) {
      if (vec) hipLaunchKernelGGL((k_sweep_rows<1, 16, true>), grid, dim3(TPB), 0, s, a);
      else hipLaunchKernelGGL((k_sweep_rows<1, 16, false>), grid, dim3(TPB), 0, s, a);
    } else {
      if (vec) hipLaunchKernelGGL((k_sweep_rows<1, 32, true>), grid, dim3(TPB), 0, s, a);
      else hipLaunchKernelGGL((k_sweep_rows<1, 32, false>), grid, dim3(TPB), 0, s, a);
    }
  }
  if (mid) (void)hipEventRecord(mid, s);
  return hipGetLastError();
}

// ============================================================================
// Conversions, rebase, selection
// ============================================================================
// U = f + eps*log(w) as double-float; max |U.hi| into st->maxabs[ma] (atomic
// max on the bit pattern of a non-negative float is order independent);
// <U, w> partial sums into scratch[blockIdx.x].
__global__ void k_to_hat(const double* f, const double* logw, double eps, float2* U, int n, DevState* st, int ma,
                         const double* w, double* scratch) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double dot = 0;
  float mx = 0.f;
  if (i < n) {
    double v = (f ? f[i] : 0.0) + eps * logw[i];
    float hi = (float)v;
    float lo = (float)(v - (double)hi);
    U[i] = make_float2(hi, lo);
    mx = fabsf(hi);
    dot = w[i] * v;
  }
  __shared__ double sbd[16];
  __shared__ float sbf[8];
  dot = block_sum_d(dot, sbd);
  mx = block_max_f(mx, sbf);
  if (threadIdx.x == 0) {
    scratch[blockIdx.x] = dot;
    atomicMax(reinterpret_cast<unsigned*>(&st->maxabs[ma]), __float_as_uint(mx));
  }
}
__global__ void k_sum_blocks(const double* scratch, int nb, double* out) {
  __shared__ double sbd[16];
  double s = 0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += scratch[b];
  s = block_sum_d(s, sbd);
  if (threadIdx.x == 0) *out = s;
}

hipError_t launch_to_hat(const double* f, const double* logw, double eps, float2* U, int n, DevState* st, int ma,
                         const double* w, int dot_slot, double* scratch, hipStream_t s) {
  int nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_to_hat, dim3(nb), dim3(256), 0, s, f, logw, eps, U, n, st, ma, w, scratch);
  hipLaunchKernelGGL(k_sum_blocks, dim3(1), dim3(256), 0, s, scratch, nb,
                     dot_slot >= 0 ? &st->dots[dot_slot] : scratch + nb);
  return hipGetLastError();
}

__global__ void k_from_hat(const float2* U, const double* logw, double eps, double* f, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    float2 u = U[i];
    f[i] = ((double)u.x + (double)u.y) - eps * logw[i];
  }
}
hipError_t launch_from_hat(const float2* U, const double* logw, double eps, double* f, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_from_hat, dim3((n + 255) / 256), dim3(256), 0, s, U, logw, eps, f, n);
  return hipGetLastError();
}

// U += deps * lw (double-float), for a change of eps between stages; the
// max |U.hi| goes to st->maxabs[ma] by atomic max (slot zeroed beforehand).
__global__ void k_rebase(float2* U, const float2* lw, float2 deps, int n, DevState* st, int ma) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  float mx = 0.f;
  if (i < n) {
    float2 u = df_add(U[i], df_mul(deps, lw[i]));
    U[i] = u;
    mx = fabsf(u.x);
  }
  __shared__ float sbf[8];
  mx = block_max_f(mx, sbf);
  if (threadIdx.x == 0) atomicMax(reinterpret_cast<unsigned*>(&st->maxabs[ma]), __float_as_uint(mx));
}
hipError_t launch_rebase(float2* U, const float2* lw, float2 deps_df, int n, DevState* st, int ma, hipStream_t s) {
  hipLaunchKernelGGL(k_rebase, dim3((n + 255) / 256), dim3(256), 0, s, U, lw, deps_df, n, st, ma);
  return hipGetLastError();
}

__global__ void k_copy_slot(DevState* st, int dd, int sd, int dm, int sm) {
  if (threadIdx.x == 0) {
    if (dd >= 0) st->dots[dd] = st->dots[sd];
    if (dm >= 0) st->maxabs[dm] = st->maxabs[sm];
  }
}
hipError_t launch_copy_state_slot(DevState* st, int dst_dot, int src_dot, int dst_ma, int src_ma, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_slot, dim3(1), dim3(64), 0, s, st, dst_dot, src_dot, dst_ma, src_ma);
  return hipGetLastError();
}

// Newton acceptance selection: accepted -> (F, G) = (F', G'); rejected ->
// (F, G) = (F_sk, G~), i.e. the plain SK iterate.
__device__ __forceinline__ void select_body(const SelectArgs& q, const int bx) {
  const float2* Fp = q.Fp;
  const float2* Fsk = q.Fsk;
  float2* F = q.F;
  const int n = q.n;
  const float2* Gp = q.Gp;
  const float2* Gt = q.Gt;
  float2* G = q.G;
  const int m = q.m;
  DevState* st = q.st;
  if (gate_closed(st, q.gate)) return;
  const int acc = ((volatile DevState*)st)->accept;
  int i = bx * blockDim.x + threadIdx.x;
  if (i < n) F[i] = acc ? Fp[i] : Fsk[i];
  else if (i < n + m) G[i - n] = acc ? Gp[i - n] : Gt[i - n];
  if (bx == 0 && threadIdx.x == 0) {
    st->dots[DOT_F] = acc ? st->dots[DOT_FP] : st->dots[DOT_FSK];
    st->dots[DOT_G] = acc ? st->dots[DOT_GP] : st->dots[DOT_GT];
    st->maxabs[MA_F] = acc ? st->maxabs[MA_FP] : st->maxabs[MA_FSK];
    st->maxabs[MA_G] = acc ? st->maxabs[MA_GP] : st->maxabs[MA_GT];
  }
}
__global__ void k_select(SelectArgs q) { select_body(q, blockIdx.x); }
__global__ void k_select_b(BatchTab T) {
  int bx, by;
  const int slot = batch_slot(T, blockIdx.x, &bx, &by);
  select_body(*static_cast<const SelectArgs*>(T.args[slot]), bx);
}
hipError_t launch_select(const float2* Fp, const float2* Fsk, float2* F, int n, const float2* Gp, const float2* Gt,
                         float2* G, int m, DevState* st, int gate, hipStream_t s) {
  const SelectArgs q{Fp, Fsk, F, n, Gp, Gt, G, m, st, gate};
  const dim3 grid((n + m + 255) / 256);
  if (g_recorder) {
    record_launch((const void*)k_select_b, q, grid, 256, 0);
    return hipSuccess;
  }
  hipLaunchKernelGGL(k_select, grid, dim3(256), 0, s, q);
  return hipGetLastError();
}

// ============================================================================
// Projected Newton system (FP64), Algorithm 4.1:
//   G = V^T diag(r) V - W^T diag(b)^-1 W,  grad = V^T (a - r) = -V^T mdiff,
//   c = eps G^-1 grad,  Delta f = V c.
// r = a + mdiff is the row marginal of P~ = pi(f, f^{C,eps}).
// ============================================================================
template <int ELL>
__device__ __forceinline__ void nr_assemble_body(const NrAssembleArgs& q, const int bx) {
  const float* V = q.V;
  const float* mdiff = q.mdiff;
  const double* a = q.a;
  const int n = q.n;
  const float* W = q.W;
  const double* b = q.b;
  const int m = q.m;
  double* part = q.part;
  const int nrow_blk = q.nrow_blk, rows_per_blk = q.rows_per_blk;
  if (gate_closed(q.st, q.gate)) return;
  // G is symmetric: only the upper triangle (k <= l) is summed, TRI entries
  // in row-major order of the triangle
  constexpr int TRI = ELL * (ELL + 1) / 2;
  constexpr int PER = (TRI + 255) / 256;
  __shared__ __align__(16) float tile[64][ELL];
  __shared__ double wrow[64];
  __shared__ double mrow[64];
  double accv[PER];
  int ek[PER], el[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    accv[p] = 0;
    int e = threadIdx.x + 256 * p, k = 0;
    while (k < ELL - 1 && e >= ELL - k) {  // row k of the triangle holds ELL - k entries
      e -= ELL - k;
      ++k;
    }
    ek[p] = k;
    el[p] = k + e;
    if ((int)threadIdx.x + 256 * p >= TRI) ek[p] = el[p] = 0;  // no entry: in-bounds reads, unused
  }
  double gacc = 0;
  const bool rows = (int)bx < nrow_blk;
  const int blk = rows ? bx : bx - nrow_blk;
  const int beg = blk * rows_per_blk;
  const int cnt = rows ? n : m;
  const int end = min(beg + rows_per_blk, cnt);
  for (int t0 = beg; t0 < end; t0 += 64) {
    int nt = min(64, end - t0);
    __syncthreads();
    {
      // rows t0 .. t0+nt-1 are one contiguous block (16-byte aligned): all
      // of a thread's float4 loads in flight at once; rows past nt are zero
      constexpr int T4 = 64 * ELL / 4, U4 = (T4 + 255) / 256;
      const float4* s4 = reinterpret_cast<const float4*>((rows ? V : W) + (size_t)t0 * ELL);
      const int valid4 = nt * ELL / 4;
      float4 v[U4];
#pragma unroll
      for (int u = 0; u < U4; ++u) v[u] = s4[min((int)threadIdx.x + 256 * u, valid4 - 1)];
#pragma unroll
      for (int u = 0; u < U4; ++u) {
        const int i4 = threadIdx.x + 256 * u;
        if (i4 < T4) reinterpret_cast<float4*>(&tile[0][0])[i4] = i4 < valid4 ? v[u] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    if (threadIdx.x < 64) {
      int rr = threadIdx.x;
      double wv = 0;
      double md = 0;
      if (rr < nt && rows) md = (double)mdiff[t0 + rr];
      if (rr < nt) wv = rows ? (a[t0 + rr] + md) : -1.0 / b[t0 + rr];
      wrow[rr] = wv;
      mrow[rr] = md;
    }
    __syncthreads();
    // all 64 rows of the tile (rows past nt are zero and add exact zeros),
    // eight at a time: the LDS reads of eight rows go out before the sums
    const bool gpath = rows && (int)threadIdx.x < ELL;
    const int gcol = (int)threadIdx.x < ELL ? (int)threadIdx.x : 0;
    for (int r0 = 0; r0 < 64; r0 += 8) {
      double wv[8], mr[8];
      float ta[8][PER], tb[8][PER], tg[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        wv[u] = wrow[r0 + u];
        mr[u] = mrow[r0 + u];
        tg[u] = tile[r0 + u][gcol];
#pragma unroll
        for (int p = 0; p < PER; ++p) {
          ta[u][p] = tile[r0 + u][ek[p]];
          tb[u][p] = tile[r0 + u][el[p]];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
#pragma unroll
        for (int p = 0; p < PER; ++p)
          if ((int)threadIdx.x + 256 * p < TRI) accv[p] += wv[u] * (double)ta[u][p] * (double)tb[u][p];
        if (gpath) gacc -= (double)tg[u] * mr[u];
      }
    }
  }
  double* out = part + (size_t)bx * (TRI + ELL);
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int e = threadIdx.x + 256 * p;
    if (e < TRI) out[e] = accv[p];
  }
  if ((int)threadIdx.x < ELL) out[TRI + threadIdx.x] = gacc;
}

template <int ELL>
__global__ __launch_bounds__(256) void k_nr_assemble(NrAssembleArgs q) { nr_assemble_body<ELL>(q, blockIdx.x); }
template <int ELL>
__global__ __launch_bounds__(256) void k_nr_assemble_b(BatchTab T) {
  int bx, by;
  const int slot = batch_slot(T, blockIdx.x, &bx, &by);
  nr_assemble_body<ELL>(*static_cast<const NrAssembleArgs*>(T.args[slot]), bx);
}

// sum over nblk (<= 32) partial blocks of entry e, loads issued together
__device__ __forceinline__ double sum_partials(const double* part, int nblk, int stride, int e) {
  double v[32];
#pragma unroll
  for (int b = 0; b < 32; ++b) v[b] = b < nblk ? part[(size_t)b * stride + e] : 0.0;
  double s = 0;
#pragma unroll
  for (int b = 0; b < 32; ++b) s += v[b];
  return s;
}

// One workgroup: the l x l Newton system (Algorithm 4.1, NR update) from the
// block partials of k_nr_assemble.  The partials are summed per entry in
// block order (chunks of 32 blocks); G is symmetrised and modes beyond
// ell_real (zero columns of V) become identity rows.  So do basis columns
// without numerical mass, |G_ii| <= 1e-12 max_j G_jj (||v_i||_a below
// ~1e-6): the warm start leaves such columns where the spectrum of M lies
// below FP32 resolution (large eps).  Their coefficients are zero and the
// step is the Newton step on the span of the other columns; the modes they
// miss have rho_k^2 ~ 0, which SK already removes.  [G | grad] is then
// reduced by Gauss-Jordan elimination without pivoting in one wave (a row
// per lane): step k updates the entries (i, j), i != k, j > k, from column
// k and row k, which it does not write.  Its pivots are those of
// G = L D L^T, so the positive-definiteness test (every pivot > 1e-15 of
// the largest diagonal entry) is the one of a Cholesky factorisation.
//
// solver = NR_CG or NR_NEWTON_SCHULZ replaces the elimination by the GPU
// friendly alternatives the paper names for the NR step (Sec. 4,
// disadvantages of the algorithm): no pivoting, only products of G with
// vectors or matrices.
//   NR_CG: conjugate gradients on [G | grad] with the Jacobi (diagonal)
//     preconditioner, one wave, lane i owning row i; stops when
//     ||grad - G z|| <= rtol ||grad|| (in the scaled system) or after max_it
//     steps; a direction with p^T G^ p <= 1e-15 |p|^2 fails the
//     positive-definiteness test.
//   NR_NEWTON_SCHULZ: iterative inversion X <- X (2 I - G^ X) of the
//     Jacobi-scaled G^ = D^-1/2 G D^-1/2 (unit diagonal) from X0 = I /
//     ||G^||_inf, whose error squares every step for an SPD G^; stops when
//     ||I - G^ X||_F <= rtol or after max_it steps, and fails the test when
//     the residual has not fallen below 1e-6 by then.
// Both start with the same per-column checks (padding, massless columns,
// positive diagonal) as the elimination.
template <int ELL>
__device__ void nr_iterative(double (*A)[ELL + 2], int solver, int max_it, double rtol, double* z, int* ok_io,
                             int* iters_out) {
  constexpr int NA = ELL + 1;
  const int tid = threadIdx.x;
  __shared__ double X[ELL][ELL + 1], Y[ELL][ELL + 1], dsc[ELL];
  __shared__ double s_x0, s_res;
  // Jacobi scaling: d_i = 1/sqrt(A_ii) (a non-positive diagonal fails)
  if (tid < ELL) {
    const double dii = A[tid][tid];
    dsc[tid] = dii > 0 ? 1.0 / sqrt(dii) : 1.0;
    if (!(dii > 0)) atomicAnd(ok_io, 0);
  }
  __syncthreads();
  if (solver == NR_CG) {
    if (tid < 64) {
      const int i = tid < ELL ? tid : 0;
      const bool own = tid < ELL;
      // scaled system  G^ y = b^,  G^ = D A D,  b^ = D grad,  z = D y
      double x = 0, r = own ? dsc[i] * A[i][ELL] : 0.0, zz = r, p = zz;
      double rz = wave_sum(r * zz);
      const double bn = sqrt(wave_sum(r * r));
      int it = 0, good = 1;
      for (; it < max_it; ++it) {
        if (!(sqrt(wave_sum(r * r)) > rtol * bn)) break;
        double q = 0;
#pragma unroll
        for (int j = 0; j < ELL; ++j) q += (own ? dsc[i] * A[i][j] * dsc[j] : 0.0) * __shfl(p, j, 64);
        // G^ has a unit diagonal: a curvature below 1e-15 |p|^2 is the
        // elimination's pivot test (pivot > 1e-15 of the largest diagonal)
        const double pq = wave_sum(own ? p * q : 0.0);
        const double pp = wave_sum(p * p);
        if (!(pq > 1e-15 * pp)) {
          good = 0;
          break;
        }
        const double alpha = rz / pq;
        x += alpha * p;
        r -= alpha * q;
        zz = r;
        const double rz2 = wave_sum(r * zz);
        const double beta = rz2 / rz;
        rz = rz2;
        p = zz + beta * p;
      }
      if (own) z[i] = dsc[i] * x;
      if (tid == 0) {
        if (!good) atomicAnd(ok_io, 0);
        *iters_out = it;
      }
    }
    __syncthreads();
    return;
  }
  // Newton-Schulz: X0 = I / ||G^||_inf
  if (tid == 0) {
    double nrm = 0;
    for (int i = 0; i < ELL; ++i) {
      double rs = 0;
      for (int j = 0; j < ELL; ++j) rs += fabs(dsc[i] * A[i][j] * dsc[j]);
      nrm = fmax(nrm, rs);
    }
    s_x0 = nrm > 0 ? 1.0 / nrm : 1.0;
  }
  __syncthreads();
  const double x0 = s_x0;
  for (int e = tid; e < ELL * ELL; e += 256) {
    const int i = e / ELL, j = e - i * ELL;
    X[i][j] = i == j ? x0 : 0.0;
  }
  __syncthreads();
  double res = 1.0;
  int it = 0;
  for (; it < max_it; ++it) {
    // Y = G^ X
    for (int e = tid; e < ELL * ELL; e += 256) {
      const int i = e / ELL, j = e - i * ELL;
      double v = 0;
#pragma unroll 8
      for (int k = 0; k < ELL; ++k) v += dsc[i] * A[i][k] * dsc[k] * X[k][j];
      Y[i][j] = v;
    }
    __syncthreads();
    // residual ||I - Y||_F (all threads read the same sum: fixed order)
    if (tid == 0) {
      double acc = 0;
      for (int i = 0; i < ELL; ++i)
        for (int j = 0; j < ELL; ++j) {
          const double d = (i == j ? 1.0 : 0.0) - Y[i][j];
          acc += d * d;
        }
      s_res = sqrt(acc);
    }
    __syncthreads();
    res = s_res;
    if (!(res > rtol)) break;
    // X <- X (2 I - Y): entries (i, j) = 2 X_ij - sum_k X_ik Y_kj
    double nv[(ELL * ELL + 255) / 256];
#pragma unroll
    for (int q = 0; q < (ELL * ELL + 255) / 256; ++q) {
      const int e = tid + 256 * q;
      nv[q] = 0;
      if (e < ELL * ELL) {
        const int i = e / ELL, j = e - i * ELL;
        double v = 2.0 * X[i][j];
#pragma unroll 8
        for (int k = 0; k < ELL; ++k) v -= X[i][k] * Y[k][j];
        nv[q] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (ELL * ELL + 255) / 256; ++q) {
      const int e = tid + 256 * q;
      if (e < ELL * ELL) X[e / ELL][e % ELL] = nv[q];
    }
    __syncthreads();
  }
  if (tid < ELL) {
    double v = 0;
    for (int j = 0; j < ELL; ++j) v += X[tid][j] * dsc[j] * A[j][ELL];
    z[tid] = dsc[tid] * v;
  }
  if (tid == 0) {
    if (!(res <= 1e-6)) atomicAnd(ok_io, 0);
    *iters_out = it;
  }
  __syncthreads();
  (void)NA;
}

// The direct solver in one wave: lane i < ELL sums row i of [G | grad]
// from the partials (both triangles from the stored upper one) into
// registers, the per-column checks become a ballot mask, and Gauss-Jordan
// runs on the registers (the steps unrolled, so every index is a constant;
// step k reads the pivot row from lane k; row i's diagonal is final once
// step i has used it as the pivot).
template <int ELL>
__device__ __forceinline__ void nr_solve_direct(const NrSolveArgs& q, double eps) {
  constexpr int TRI = ELL * (ELL + 1) / 2, NA = ELL + 1, LEN = TRI + ELL;
  const int tid = threadIdx.x;
  if (tid >= 64) return;
  const int row = tid < ELL ? tid : ELL - 1;
  const int ell_real = q.ell_real;
  // entry (k, l), k <= l, of the upper triangle in row-major order
  auto tri = [](int k, int l) { return k * ELL - (k * (k - 1)) / 2 + (l - k); };
  double x[NA];
  {
    int idx[NA];
#pragma unroll
    for (int j = 0; j < ELL; ++j) idx[j] = j >= row ? tri(row, j) : tri(j, row);
    idx[ELL] = TRI + row;
#pragma unroll
    for (int j = 0; j < NA; ++j) x[j] = 0.0;
    // sums in block order, in chunks of 32 blocks
    for (int b0 = 0; b0 < q.nblk; b0 += 32) {
      const int nb = min(32, q.nblk - b0);
      double c[NA];
#pragma unroll
      for (int j = 0; j < NA; ++j) c[j] = 0.0;
      for (int b = 0; b < nb; ++b) {
        const double* pb = q.part + (size_t)(b0 + b) * LEN;
#pragma unroll
        for (int j = 0; j < NA; ++j) c[j] += pb[idx[j]];
      }
#pragma unroll
      for (int j = 0; j < NA; ++j) x[j] += c[j];
    }
  }
  double dgo = 0.0;  // this row's diagonal entry
#pragma unroll
  for (int j = 0; j < ELL; ++j)
    if (j == row) dgo = x[j];
  double dmax = tid < ell_real ? dgo : 0.0;
  for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
  if (q.Gout && tid < ell_real) {
#pragma unroll
    for (int j = 0; j < ELL; ++j)
      if (j < ell_real) q.Gout[tid * ell_real + j] = 0.5 * (x[j] + x[j]);
    q.gout[tid] = x[ELL];
  }
  // column i takes part unless it is padding or carries no mass (a NaN or
  // negative diagonal still fails the pivot test below)
  const bool act = row < ell_real && !(fabs(dgo) <= 1e-12 * dmax);
  const unsigned long long am = __ballot(tid < ELL && act);
#pragma unroll
  for (int j = 0; j < ELL; ++j) {
    const bool aj = (am >> j) & 1ull;
    x[j] = (act && aj) ? 0.5 * (x[j] + x[j]) : (j == row ? 1.0 : 0.0);
  }
  x[ELL] = act ? x[ELL] : 0.0;
  int ok = 1;
  double dg = 1.0;
#pragma unroll
  for (int k = 0; k < ELL; ++k) {
    double piv = lane_read_d(x[k], k);
    if (!(piv > 1e-300 && piv > 1e-15 * dmax)) {
      ok = 0;
      piv = 1.0;
    }
    if (row == k) dg = piv;
    // row i subtracts (A_ik / A_kk) times row k; row k keeps its entries
    // (a zero multiplier; a non-finite pivot row fails the test below)
    const double mk = row == k ? 0.0 : x[k] * (1.0 / piv);
#pragma unroll
    for (int j = k + 1; j < NA; ++j) x[j] = fma(-mk, lane_read_d(x[j], k), x[j]);
  }
  // the system is now diagonal: z_i = A[i][ELL] / A[i][i]
  const double c = eps * (x[ELL] / dg);
  const int bad = (tid < ELL) && !(fabs(c) < 1e30);
  ok = ok && !__any(bad);
  if (tid < ELL) {
    q.coef64[tid] = c;
    q.coef32[tid] = ok ? (float)c : 0.f;
  }
  if (tid == 0) {
    DevState* st = q.st;
    st->chol_ok = ok;
    st->accept = 0;
    st->newton_tried += 1;
    st->nr_iters = 0;
  }
}

template <int ELL>
__device__ __forceinline__ void nr_solve_body(const NrSolveArgs& q) {
  const double* part = q.part;
  const int nblk = q.nblk, ell_real = q.ell_real;
  float* coef32 = q.coef32;
  double* coef64 = q.coef64;
  double* Gout = q.Gout;
  double* gout = q.gout;
  DevState* st = q.st;
  const int solver = q.solver, max_it = q.max_it;
  const double rtol = q.rtol;
  if (gate_closed(st, q.gate)) return;
  constexpr int NE = ELL * ELL;
  constexpr int TRI = ELL * (ELL + 1) / 2;
  constexpr int NA = ELL + 1;  // augmented width
  const int tid = threadIdx.x;
  const double eps = st->eps;
  if (solver == NR_DIRECT) {
    nr_solve_direct<ELL>(q, eps);
    return;
  }
  __shared__ double R[NE + ELL];   // sums: G row-major (both triangles), then grad
  __shared__ double A[ELL][NA + 1];
  // the partials hold the upper triangle of G then grad: sum them (block
  // order) and mirror the triangle
  for (int e = tid; e < TRI + ELL; e += 256) {
    double v = 0;
    if (nblk == 1) v = part[e];  // summed beforehand
    else
      for (int b0 = 0; b0 < nblk; b0 += 32)
        v += sum_partials(part + (size_t)b0 * (TRI + ELL), min(32, nblk - b0), TRI + ELL, e);
    if (e >= TRI) {
      R[NE + (e - TRI)] = v;
    } else {
      int k = 0, r = e;
      while (k < ELL - 1 && r >= ELL - k) {
        r -= ELL - k;
        ++k;
      }
      R[k * ELL + k + r] = v;
      R[(k + r) * ELL + k] = v;
    }
  }
  __syncthreads();
  double dmax = 0;
  for (int j = 0; j < ell_real; ++j) dmax = fmax(dmax, R[j * ELL + j]);
  // column i takes part unless it is padding or carries no mass (a NaN or
  // negative diagonal still fails the pivot test below)
  auto active = [&](int i) { return i < ell_real && !(fabs(R[i * ELL + i]) <= 1e-12 * dmax); };
  for (int e = tid; e < ELL * NA; e += 256) {
    const int i = e / NA, j = e - i * NA;
    double v;
    if (j == ELL) v = active(i) ? R[NE + i] : 0.0;
    else if (!active(i) || !active(j)) v = (i == j) ? 1.0 : 0.0;
    else v = 0.5 * (R[i * ELL + j] + R[j * ELL + i]);
    A[i][j] = v;
  }
  if (Gout) {
    for (int e = tid; e < ell_real * ell_real; e += 256) {
      const int i = e / ell_real, j = e - i * ell_real;
      Gout[e] = 0.5 * (R[i * ELL + j] + R[j * ELL + i]);
    }
    for (int e = tid; e < ell_real; e += 256) gout[e] = R[NE + e];
  }
  __syncthreads();
  if (solver != NR_DIRECT) {
    __shared__ double zs[ELL];
    __shared__ int s_ok, s_its;
    if (tid == 0) {
      s_ok = 1;
      s_its = 0;
    }
    __syncthreads();
    nr_iterative<ELL>(A, solver, max_it, rtol, zs, &s_ok, &s_its);
    if (tid < 64) {
      const int i = tid < ELL ? tid : ELL - 1;
      const double c = eps * zs[i];
      const int bad = (tid < ELL) && !(fabs(c) < 1e30);
      const int ok = s_ok && !__any(bad);
      if (tid < ELL) {
        coef64[tid] = c;
        coef32[tid] = ok ? (float)c : 0.f;
      }
      if (tid == 0) {
        st->chol_ok = ok;
        st->accept = 0;
        st->newton_tried += 1;
        st->nr_iters = s_its;
      }
    }
    return;
  }
}

template <int ELL>
__global__ __launch_bounds__(256) void k_nr_solve(NrSolveArgs q) { nr_solve_body<ELL>(q); }
template <int ELL>
__global__ __launch_bounds__(256) void k_nr_solve_b(BatchTab T) {
  int bx, by;
  const int slot = batch_slot(T, blockIdx.x, &bx, &by);
  nr_solve_body<ELL>(*static_cast<const NrSolveArgs*>(T.args[slot]));
}

template <int ELL>
__device__ __forceinline__ void nr_apply_body(const NrApplyArgs& q, const int bx) {
  const float2* F = q.F;
  const float* V = q.V;
  const float* coef = q.coef;
  const double* a = q.a;
  float2* Fp = q.Fp;
  const int n = q.n;
  double* blk = q.blk;
  float* blkmax = q.blkmax;
  double* blkd = q.blkd;
  float* E1 = q.E1;
  DevState* st = q.st;
  if (gate_closed(st, q.gate)) return;
  __shared__ float c[ELL];
  if (threadIdx.x < ELL) c[threadIdx.x] = coef[threadIdx.x];
  __syncthreads();
  const float inv_eps = st->inv_eps;
  int i = bx * blockDim.x + threadIdx.x;
  double dot = 0, dd = 0;
  float mx = 0.f;
  if (i < n) {
    float dl = 0.f;
    const float* vr = V + (size_t)i * ELL;
#pragma unroll
    for (int l = 0; l < ELL; ++l) dl = fmaf(vr[l], c[l], dl);
    float2 u = df_add_f(F[i], dl);
    Fp[i] = u;
    dot = a[i] * ((double)u.x + (double)u.y);
    dd = a[i] * (double)dl;
    mx = fabsf(u.x);
    float4* e = reinterpret_cast<float4*>(E1 + (size_t)i * 8);
    e[0] = make_float4(expm1f(dl * inv_eps), 0.f, 0.f, 0.f);
    e[1] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __shared__ double sbd[16];
  __shared__ double sbd2[16];
  __shared__ float sbf[8];
  dot = block_sum_d(dot, sbd);
  dd = block_sum_d(dd, sbd2);
  mx = block_max_f(mx, sbf);
  if (threadIdx.x == 0) {
    blk[bx] = dot;
    blkd[bx] = dd;
    blkmax[bx] = mx;
  }
}

template <int ELL>
__global__ __launch_bounds__(256) void k_nr_apply(NrApplyArgs q) { nr_apply_body<ELL>(q, blockIdx.x); }
template <int ELL>
__global__ __launch_bounds__(256) void k_nr_apply_b(BatchTab T) {
  int bx, by;
  const int slot = batch_slot(T, blockIdx.x, &bx, &by);
  nr_apply_body<ELL>(*static_cast<const NrApplyArgs*>(T.args[slot]), bx);
}

template <int E>
static void nr_assemble_e(const float* V, const float* mdiff, const double* a, int n, const float* W, const double* b,
                          int m, double* part, int nrow_blk, int ncol_blk, int rpb, DevState* st, int gate,
                          hipStream_t s) {
  const NrAssembleArgs q{V, mdiff, a, n, W, b, m, part, nrow_blk, rpb, st, gate};
  const dim3 grid(nrow_blk + ncol_blk);
  if (g_recorder) record_launch((const void*)k_nr_assemble_b<E>, q, grid, 256, 0);
  else hipLaunchKernelGGL((k_nr_assemble<E>), grid, dim3(256), 0, s, q);
}
hipError_t launch_nr_assemble(int ell, const float* V, const float* mdiff, const double* a, int n, const float* W,
                              const double* b, int m, double* part, int nrow_blk, int ncol_blk, DevState* st, int gate,
                              hipStream_t s) {
  int rpb_r = (n + nrow_blk - 1) / nrow_blk;
  int rpb_c = (m + ncol_blk - 1) / ncol_blk;
  int rpb = rpb_r > rpb_c ? rpb_r : rpb_c;  // one block length for rows and columns
  if (((uintptr_t)V | (uintptr_t)W) & 15) return hipErrorInvalidValue;  // float4 row loads
  if (ell <= 8) nr_assemble_e<8>(V, mdiff, a, n, W, b, m, part, nrow_blk, ncol_blk, rpb, st, gate, s);
  else if (ell <= 16) nr_assemble_e<16>(V, mdiff, a, n, W, b, m, part, nrow_blk, ncol_blk, rpb, st, gate, s);
  else nr_assemble_e<32>(V, mdiff, a, n, W, b, m, part, nrow_blk, ncol_blk, rpb, st, gate, s);
  return hipGetLastError();
}
template <int E>
static void nr_solve_e(const double* part, int nblk, int ell, float* coef32, double* coef64, double* Gout,
                       double* gout, DevState* st, int gate, const NrSolver& sv, hipStream_t s) {
  const NrSolveArgs q{part, nblk, ell, coef32, coef64, Gout, gout, st, gate, sv.kind, sv.max_iter, sv.rtol};
  if (g_recorder) record_launch((const void*)k_nr_solve_b<E>, q, dim3(1), 256, 0);
  else hipLaunchKernelGGL((k_nr_solve<E>), dim3(1), dim3(256), 0, s, q);
}
hipError_t launch_nr_solve(int ell, const double* part, int nblk, float* coef32, double* coef64, double* Gout,
                           double* gout, DevState* st, int gate, hipStream_t s, const NrSolver& sv) {
  if (ell <= 8) nr_solve_e<8>(part, nblk, ell, coef32, coef64, Gout, gout, st, gate, sv, s);
  else if (ell <= 16) nr_solve_e<16>(part, nblk, ell, coef32, coef64, Gout, gout, st, gate, sv, s);
  else nr_solve_e<32>(part, nblk, ell, coef32, coef64, Gout, gout, st, gate, sv, s);
  return hipGetLastError();
}
template <int E>
static void nr_apply_e(const float2* F, const float* V, const float* coef, const double* a, float2* Fp, int n,
                       double* blk, float* blkmax, double* blkd, float* E1, DevState* st, int gate, hipStream_t s) {
  const NrApplyArgs q{F, V, coef, a, Fp, n, blk, blkmax, blkd, E1, st, gate};
  const dim3 grid((n + 255) / 256);
  if (g_recorder) record_launch((const void*)k_nr_apply_b<E>, q, grid, 256, 0);
  else hipLaunchKernelGGL((k_nr_apply<E>), grid, dim3(256), 0, s, q);
}
hipError_t launch_nr_apply(int ell, const float2* F, const float* V, const float* coef, const double* a, float2* Fp,
                           int n, double* blk, float* blkmax, double* blkd, float* E1, DevState* st, int gate,
                           hipStream_t s) {
  if (ell <= 8) nr_apply_e<8>(F, V, coef, a, Fp, n, blk, blkmax, blkd, E1, st, gate, s);
  else if (ell <= 16) nr_apply_e<16>(F, V, coef, a, Fp, n, blk, blkmax, blkd, E1, st, gate, s);
  else nr_apply_e<32>(F, V, coef, a, Fp, n, blk, blkmax, blkd, E1, st, gate, s);
  return hipGetLastError();
}

// ---------------------------------------------------- gradients of W_eps
__global__ void k_pack_cols(const float* P, int np, int d, int c0, int dc, int ellp, float* out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  for (int k = 0; k < ellp; ++k) out[(size_t)p * ellp + k] = k < dc ? P[(size_t)p * d + c0 + k] : 0.f;
}
hipError_t launch_pack_cols(const float* P, int np, int d, int c0, int dc, int ellp, float* out, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_cols, dim3((np + 255) / 256), dim3(256), 0, s, P, np, d, c0, dc, ellp, out);
  return hipGetLastError();
}

// grad[p, c0+k] = two_s ((w_p + mdiff_p) P[p, c0+k] - Wsum[p, k]): the
// output marginal is w_p + mdiff_p, Wsum the pi-weighted sum of the other
// side's coordinates
__global__ void k_grad_points(const float* P, int np, int d, int c0, int dc, const double* w, const float* mdiff,
                              const float* Wsum, int ellp, double two_s, double* grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const double mass = w[p] + (double)mdiff[p];
  for (int k = 0; k < dc; ++k)
    grad[(size_t)p * d + c0 + k] =
        two_s * (mass * (double)P[(size_t)p * d + c0 + k] - (double)Wsum[(size_t)p * ellp + k]);
}
hipError_t launch_grad_points(const float* P, int np, int d, int c0, int dc, const double* w, const float* mdiff,
                              const float* Wsum, int ellp, double two_s, double* grad, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_points, dim3((np + 255) / 256), dim3(256), 0, s, P, np, d, c0, dc, w, mdiff, Wsum,
                     ellp, two_s, grad);
  return hipGetLastError();
}

// gradw[p] = pot[p] - eps (w_p + mdiff_p) / w_p
__global__ void k_grad_weights(const double* pot, const double* w, const float* mdiff, int np, double eps,
                               double* grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  grad[p] = pot[p] - eps * (1.0 + (double)mdiff[p] / w[p]);
}
hipError_t launch_grad_weights(const double* pot, const double* w, const float* mdiff, int np, double eps,
                               double* grad, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_weights, dim3((np + 255) / 256), dim3(256), 0, s, pot, w, mdiff, np, eps, grad);
  return hipGetLastError();
}

// ============================================================================
// FP64 evaluation of (f, g): row / column sums of pi, <C,pi>, sum pi,
// sum pi*log(pi/(a b)).  Tiles of 64 rows x 256 columns; deterministic
// two-stage sums.
// ============================================================================
template <int COST, int D>
__global__ __launch_bounds__(256) void k_eval(SweepArgs G, const double* f, const double* g, const double* a,
                                              const double* b, double eps, double* rowpart, double* colpart,
                                              double* scal, int n, int m) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int i0 = blockIdx.y * 64;
  const int jc = min(j, m - 1);
  const double inv = 1.0 / eps;
  const double gj = g[jc], bj = b[jc];
  float q[D > 0 ? D : 1];
  if (COST == 1 && D > 0)
    for (int k = 0; k < D; ++k) q[k] = G.Pout[(size_t)jc * D + k];
  __shared__ double srow[WAVES][64];
  double cs = 0, cost = 0, mass = 0, ent = 0;
  for (int r = 0; r < 64; ++r) {
    int i = i0 + r;
    double p = 0, cij = 0;
    if (i < n && j < m) {
      if (COST == kEvalExact) {
        // the exact cost of the FP32 points, in FP64
        const float* xp = G.Pred + (size_t)i * G.d;
        const float* yp = G.Pout + (size_t)jc * G.d;
        double s2 = 0;
        for (int k = 0; k < G.d; ++k) {
          const double t = (double)xp[k] - (double)yp[k];
          s2 = fma(t, t, s2);
        }
        cij = s2 * G.cscale64;
      } else {
        float cf;
        if (COST == 0) cf = G.C[(size_t)i * G.ldc + j];
        else {
          const float* xp = G.Pred + (size_t)i * G.d;
          float cc = (D > 0) ? sqdist<D>(xp, q) : sqdist_rt(xp, G.Pout + (size_t)jc * G.d, G.d);
          cf = (G.cscale != 1.0f) ? cc * G.cscale : cc;
        }
        cij = (double)cf;
      }
      double t = (f[i] + gj - cij) * inv;
      p = a[i] * bj * exp(t);
      cs += p;
      cost += p * cij;
      mass += p;
      ent += p * t;
    }
    double rs = wave_sum(p);
    if (lane == 0) srow[wave][r] = rs;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    int i = i0 + threadIdx.x;
    if (i < n) rowpart[(size_t)blockIdx.x * n + i] = srow[0][threadIdx.x] + srow[1][threadIdx.x] +
                                                     srow[2][threadIdx.x] + srow[3][threadIdx.x];
  }
  if (j < m) colpart[(size_t)blockIdx.y * m + j] = cs;
  __shared__ double sbd[16];
  double c1 = block_sum_d(cost, sbd);
  double c2 = block_sum_d(mass, sbd);
  double c3 = block_sum_d(ent, sbd);
  if (threadIdx.x == 0) {
    size_t bid = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    scal[bid * 3 + 0] = c1;
    scal[bid * 3 + 1] = c2;
    scal[bid * 3 + 2] = c3;
  }
}

hipError_t launch_eval(const SweepArgs& geo, int cost_kind, const double* f, const double* g, const double* a,
                       const double* b, double eps, double* rowpart, double* colpart, double* scal, int n, int m,
                       int* nrb, int* ncb, hipStream_t s) {
  dim3 grid((m + 255) / 256, (n + 63) / 64);
  *ncb = grid.x;
  *nrb = grid.y;
  if (cost_kind == 0) {
    hipLaunchKernelGGL((k_eval<0, 1>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, rowpart, colpart, scal, n, m);
  } else if (cost_kind == kEvalExact) {
    hipLaunchKernelGGL((k_eval<kEvalExact, 0>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, rowpart, colpart, scal, n, m);
  } else {
    switch (geo.d) {
      case 1: hipLaunchKernelGGL((k_eval<1, 1>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, rowpart, colpart, scal, n, m); break;
      case 2: hipLaunchKernelGGL((k_eval<1, 2>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, rowpart, colpart, scal, n, m); break;
      case 3: hipLaunchKernelGGL((k_eval<1, 3>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, rowpart, colpart, scal, n, m); break;
      case 4: hipLaunchKernelGGL((k_eval<1, 4>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, rowpart, colpart, scal, n, m); break;
      case 5: hipLaunchKernelGGL((k_eval<1, 5>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, rowpart, colpart, scal, n, m); break;
      case 6: hipLaunchKernelGGL((k_eval<1, 6>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, rowpart, colpart, scal, n, m); break;
      case 7: hipLaunchKernelGGL((k_eval<1, 7>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, rowpart, colpart, scal, n, m); break;
      case 8: hipLaunchKernelGGL((k_eval<1, 8>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, rowpart, colpart, scal, n, m); break;
      default: hipLaunchKernelGGL((k_eval<1, 0>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, rowpart, colpart, scal, n, m); break;
    }
  }
  return hipGetLastError();
}

// first stage: per block of rows / columns, sum the tile partials of each
// row (column) in order and accumulate |sum - weight|; block results in blk
__global__ __launch_bounds__(256) void k_eval_marg(const double* rowpart, const double* colpart, const double* a,
                                                   const double* b, int n, int m, int nrb, int ncb, double* blk) {
  __shared__ double sbd[16];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0;
  if (i < n) {
    double s = 0;
    for (int cb = 0; cb < ncb; ++cb) s += rowpart[(size_t)cb * n + i];
    v = fabs(s - a[i]);
  } else if (i < n + m) {
    const int j = i - n;
    double s = 0;
    for (int rb = 0; rb < nrb; ++rb) s += colpart[(size_t)rb * m + j];
    v = fabs(s - b[j]);
  }
  v = block_sum_d(v, sbd);
  if (threadIdx.x == 0) blk[blockIdx.x] = v;
}

// out8 = {row_err, col_err, cost, mass, ent_sum, 0, 0, 0}; nrowblk blocks of
// blk hold row terms only when n is a multiple of 256 -- rows and columns
// are kept apart by the block boundary at n
__global__ __launch_bounds__(256) void k_eval_finish(const double* blk, int nb_rows, int nb_all, const double* scal,
                                                     int nscal, double* out8) {
  __shared__ double sbd[16];
  double re = 0, ce = 0, c1 = 0, c2 = 0, c3 = 0;
  for (int q = threadIdx.x; q < nb_all; q += blockDim.x) {
    if (q < nb_rows) re += blk[q];
    else ce += blk[q];
  }
  for (int q = threadIdx.x; q < nscal; q += blockDim.x) {
    c1 += scal[(size_t)q * 3 + 0];
    c2 += scal[(size_t)q * 3 + 1];
    c3 += scal[(size_t)q * 3 + 2];
  }
  re = block_sum_d(re, sbd);
  ce = block_sum_d(ce, sbd);
  c1 = block_sum_d(c1, sbd);
  c2 = block_sum_d(c2, sbd);
  c3 = block_sum_d(c3, sbd);
  if (threadIdx.x == 0) {
    out8[0] = re;
    out8[1] = ce;
    out8[2] = c1;
    out8[3] = c2;
    out8[4] = c3;
  }
}
hipError_t launch_eval_finish(const double* rowpart, const double* colpart, const double* scal, const double* a,
                              const double* b, int n, int m, int nrb, int ncb, double* out8, double* blk,
                              hipStream_t s) {
  // rows and columns in separate block ranges so that each block holds one kind
  const int nbr = (n + 255) / 256, nbc = (m + 255) / 256;
  hipLaunchKernelGGL(k_eval_marg, dim3(nbr), dim3(256), 0, s, rowpart, colpart, a, b, n, 0, nrb, ncb, blk);
  hipLaunchKernelGGL(k_eval_marg, dim3(nbc), dim3(256), 0, s, rowpart, colpart, a, b, 0, m, nrb, ncb, blk + nbr);
  hipLaunchKernelGGL(k_eval_finish, dim3(1), dim3(256), 0, s, blk, nbr, nbr + nbc, scal, nrb * ncb, out8);
  return hipGetLastError();
}

// coupling pi_ij = a_i b_j exp((f_i + g_j - C_ij)/eps) as FP32
template <int COST>
__global__ void k_coupling(SweepArgs G, const double* f, const double* g, const double* a, const double* b,
                           double eps, float* P, int n, int m) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int i = blockIdx.y;
  if (j >= m) return;
  float cf;
  if (COST == 0) cf = G.C[(size_t)i * G.ldc + j];
  else {
    float cc = sqdist_rt(G.Pred + (size_t)i * G.d, G.Pout + (size_t)j * G.d, G.d);
    cf = (G.cscale != 1.0f) ? cc * G.cscale : cc;
  }
  P[(size_t)i * m + j] = (float)(a[i] * b[j] * exp((f[i] + g[j] - (double)cf) / eps));
}
hipError_t launch_coupling(const SweepArgs& geo, int cost_kind, const double* f, const double* g, const double* a,
                           const double* b, double eps, float* P, int n, int m, hipStream_t s) {
  dim3 grid((m + 255) / 256, n);
  if (cost_kind == 0) hipLaunchKernelGGL((k_coupling<0>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, P, n, m);
  else hipLaunchKernelGGL((k_coupling<1>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, P, n, m);
  return hipGetLastError();
}

// ------------------------------------------------------ small utilities
__global__ void k_dot64(const double* x, const double* w, int n, double* out) {
  __shared__ double sbd[16];
  double s = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += x[i] * w[i];
  s = block_sum_d(s, sbd);
  if (threadIdx.x == 0) *out = s;
}
hipError_t launch_dot64(const double* x, const double* w, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_dot64, dim3(1), dim3(256), 0, s, x, w, n, out);
  return hipGetLastError();
}
// x += sign * 0.5 * (dots[1] - dots[0])  (gauge normalisation <f,a> = <g,b>)
__global__ void k_shift64(double* x, int n, const double* dots, double sign) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += sign * 0.5 * (dots[1] - dots[0]);
}
hipError_t launch_shift64(double* x, int n, const double* dots, double sign, hipStream_t s) {
  hipLaunchKernelGGL(k_shift64, dim3((n + 255) / 256), dim3(256), 0, s, x, n, dots, sign);
  return hipGetLastError();
}

// max |C_ij| as the bit pattern of a non-negative float (atomic max on the
// bits is order independent); a NaN or infinite entry gives +inf, which the
// host rejects
__global__ void k_cost_absmax(const float* C, long long ldc, int n, int m, unsigned* out) {
  __shared__ float sbf[8];
  float mx = 0.f;
  int i = blockIdx.x;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const float v = fabsf(C[(size_t)i * ldc + j]);
    mx = v <= FLT_MAX ? fmaxf(mx, v) : INFINITY;
  }
  mx = block_max_f(mx, sbf);
  if (threadIdx.x == 0) atomicMax(out, __float_as_uint(mx));
}
__global__ void k_zero_u32(unsigned* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0u;
}
hipError_t launch_cost_max(int cost_kind, const float* C, long long ldc, int n, int m, const float* x, const float* y,
                           int d, float* out2, hipStream_t s) {
  (void)x; (void)y; (void)d;
  if (cost_kind != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned*>(out2));
  hipLaunchKernelGGL(k_cost_absmax, dim3(n), dim3(256), 0, s, C, ldc, n, m, reinterpret_cast<unsigned*>(out2));
  return hipGetLastError();
}

// Transposed copy of a stored cost: X[j * rows + i] = C[i * ldc + j] for
// i < rows, j < cols, through 64 x 64 LDS tiles (coalesced reads of C's
// rows and of X's rows; the odd row pitch keeps the column reads of the
// tile free of bank conflicts).  The weighted sweeps whose outputs run
// along C's rows then take the streaming kernel on X.
__global__ __launch_bounds__(256) void k_transpose_cost(const float* __restrict__ C, long long ldc, int rows, int cols,
                                                        float* __restrict__ X) {
  __shared__ float t[64][65];
  const int j0 = blockIdx.x * 64, i0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int i = i0 + r, j = j0 + tx;
    t[r][tx] = (i < rows && j < cols) ? C[(size_t)i * ldc + j] : 0.f;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int j = j0 + r, i = i0 + tx;
    if (j < cols && i < rows) X[(size_t)j * rows + i] = t[tx][r];
  }
}
hipError_t launch_transpose_cost(const float* C, long long ldc, int rows, int cols, float* X, hipStream_t s) {
  if (rows <= 0 || cols <= 0 || ldc < cols) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_transpose_cost, dim3((cols + 63) / 64, (rows + 63) / 64), dim3(256), 0, s, C, ldc, rows, cols,
                     X);
  return hipGetLastError();
}

// Input statistics (prepare): block 0 covers the weights a (n), block 1
// the weights b (m); with points, block 2 + k coordinate k of x and block
// 2 + d + k coordinate k of y.  out[5 blk + 0 .. 4] = min, max, sum, the
// count of bad entries (weights: not positive or not finite; points: not
// finite) and, for weights, the entropy term sum v log v.  Each thread sums
// its entries in index order, then a fixed tree (deterministic).
__device__ __forceinline__ double block_reduce_d(double v, double* sbuf, int op) {  // op 0 sum, 1 min, 2 max
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(v, off, 64);
    v = op == 0 ? v + o : (op == 1 ? fmin(v, o) : fmax(v, o));
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sbuf[w] = v;
  __syncthreads();
  double r = sbuf[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = op == 0 ? r + sbuf[i] : (op == 1 ? fmin(r, sbuf[i]) : fmax(r, sbuf[i]));
  return r;
}
__global__ __launch_bounds__(256) void k_input_stats(const double* a, int n, const double* b, int m, const float* x,
                                                     const float* y, int d, double* out) {
  __shared__ double sb[4];
  const int blk = blockIdx.x;
  double mn = INFINITY, mx = -INFINITY, sm = 0, bad = 0, ent = 0;
  if (blk < 2) {
    const double* w = blk == 0 ? a : b;
    const int len = blk == 0 ? n : m;
    for (int i = threadIdx.x; i < len; i += blockDim.x) {
      const double v = w[i];
      if (!(v > 0) || !isfinite(v)) {
        bad += 1;
      } else {
        ent += v * log(v);
        mn = fmin(mn, v);
        mx = fmax(mx, v);
      }
      sm += v;
    }
  } else {
    const bool isy = blk - 2 >= d;
    const int k = isy ? blk - 2 - d : blk - 2;
    const float* pts = isy ? y : x;
    const int len = isy ? m : n;
    for (int i = threadIdx.x; i < len; i += blockDim.x) {
      const double v = pts[(size_t)i * d + k];
      if (!isfinite(v)) {
        bad += 1;
      } else {
        mn = fmin(mn, v);
        mx = fmax(mx, v);
      }
      sm += v;
    }
  }
  mn = block_reduce_d(mn, sb, 1);
  mx = block_reduce_d(mx, sb, 2);
  sm = block_reduce_d(sm, sb, 0);
  bad = block_reduce_d(bad, sb, 0);
  ent = block_reduce_d(ent, sb, 0);
  if (threadIdx.x == 0) {
    double* o = out + 5 * (size_t)blk;
    o[0] = mn;
    o[1] = mx;
    o[2] = sm;
    o[3] = bad;
    o[4] = ent;
  }
}
hipError_t launch_input_stats(const double* a, int n, const double* b, int m, const float* x, const float* y, int d,
                              double* out, hipStream_t s) {
  const int nb = 2 + (x ? 2 * d : 0);
  hipLaunchKernelGGL(k_input_stats, dim3(nb), dim3(256), 0, s, a, n, b, m, x, y, x ? d : 1, out);
  return hipGetLastError();
}

// weights -> FP32 copy, FP64 log and its double-float split
__global__ void k_weight_prep(const double* w, int n, float* w32, double* l64, float2* ldf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = w[i];
  const double l = log(v);
  w32[i] = (float)v;
  l64[i] = l;
  const float hi = (float)l;
  ldf[i] = make_float2(hi, (float)(l - (double)hi));
}
hipError_t launch_weight_prep(const double* w, int n, float* w32, double* l64, float2* ldf, hipStream_t s) {
  hipLaunchKernelGGL(k_weight_prep, dim3((n + 255) / 256), dim3(256), 0, s, w, n, w32, l64, ldf);
  return hipGetLastError();
}

__global__ void k_f32_to_f64(const float* s, double* d, long long cnt) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < cnt) d[i] = s[i];
}
__global__ void k_f64_to_f32(const double* s, float* d, long long cnt) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < cnt) d[i] = (float)s[i];
}
hipError_t launch_f32_to_f64(const float* src, double* dst, long long count, hipStream_t s) {
  hipLaunchKernelGGL(k_f32_to_f64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, src, dst, count);
  return hipGetLastError();
}
hipError_t launch_f64_to_f32(const double* src, float* dst, long long count, hipStream_t s) {
  hipLaunchKernelGGL(k_f64_to_f32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, src, dst, count);
  return hipGetLastError();
}

}  // namespace sknr
