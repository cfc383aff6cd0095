// Single-read SK iteration over a stored cost (Sec. 2, eq. SK_iterations).
//
// The two-pass iteration reads C twice: g = T_c(f) by columns, then
// f = T_r(g) by rows.  Here one pass reads each row of C once and does both
// halves that touch it.  A workgroup owns a contiguous block of rows (a
// split of the column reduction); each thread owns 4Q columns.
//
// Row half: f_r = T_r(g)_r (eq. foc_f) by the arithmetic of the streaming
// sweeps: the reduce side enters offset by L as a double-float (h, l) with
// l pre-scaled by K = log2(e)/eps, and the terms
// t_rj = exp((g^_j + L - C_rj - sigma_r)/eps) are formed as
// ex2(fma((h - sigma_r) - C, K, l K)), with h - sigma_r exact (both lie in
// [L/2, 2L]), so the exponent is rounded only relative to its own size.
// The shift needs no max pass.  g = T_c(f^prev) for the previous pass's row
// output f^prev, so every plan entry of (f^prev, g) is at most b_j, and the
// base shift L - f^prev_r + eps log a_r bounds the terms by b_j / a_r; their
// sum S_r (that plan's row marginal over a_r) is at least min_j b_j, since
// f^prev is itself a row transform (true from a stage's second pass on).
// Each pass also records log2 of the row's largest term (one max per
// element) and the next pass raises its base by it, so that the largest
// terms sit near 1 and their exponents are rounded as finely as under a
// max shift (with the base alone the exponents of a row's main terms lie
// several binades down, and the rounding of their arguments left a 1.6e-7
// floor on the L1 error).  A row with no recorded maximum (the first pass
// of a stage) or whose S_r falls outside [2^-24, 2^24] is redone with its
// own max as the shift.  The t_rj stay in the registers that held the
// costs.
//
// Column half: with f_r = eps log a_r - eps log sum_j exp((g_j - C_rj)/eps),
// the plan entry of the pair (f, g) is pi_rj = a_r t_rj / S_r (S_r the row
// sum relative to the same shift), and
//   sum_r exp((f_r - C_rj)/eps) = exp(-g_j/eps) M_j,   M_j = sum_r pi_rj,
// the column marginal of pi.  So the column half is one FP64 fma per
// element: the split's M_j += (a_r / S_r) t_rj.  The merge kernel sums the
// splits' M_j in split order and forms g'_j = g_j + eps log b_j - eps log M_j
// (eq. foc_g) through the finalisation of the streaming sweeps, which also
// tests the pair (f, g) for convergence (its L1 error is sum_j |M_j - b_j|).
// M_j <= sum_r a_r = 1; an FP32 term t_rj below 2^-126 adds at most
// 2^-126 a_r / S_r <= 2^-102 a_r to M_j, at most 2^-102 in all, so an M_j
// below 2^-76 is not resolved to FP32 accuracy (relative 2^-26).
// For such a column the merge recomputes T_c(f)_j exactly from the column
// of C and the f just written, by the online log-sum-exp of the streaming
// sweeps.  It is rare: g = T_c(f_prev) gives a plan of (f_prev, g) with
// column marginals b and row marginals r_i <= 1, and rescaling its rows to
// a gives M_j = sum_i pi_ij a_i / r_i >= b_j min_i a_i, so only weights
// whose products fall below 2^-76 take this path.
#include "sknr_internal.h"
#include "sknr_device.h"
#include "sknr_sweep_tail.h"

namespace sknr {

namespace {
constexpr int kMaxWaves = 16;
constexpr int kMaxCols = 16384;  // staged offset g^ + L_r: 8 bytes per column of LDS
}  // namespace

// FT threads, Q float4 groups of columns per thread: columns 4 (t + FT q) + k.
// FULL: m == 4 FT Q (no column past m, no masks).
template <int Q, int FT, bool FULL>
__global__ __launch_bounds__(FT) void k_sk_fused_stored(SweepArgs A) {
  constexpr int FW = FT / 64;
  if (gate_closed(A.st, A.gate)) return;
  extern __shared__ float4 fsm4[];
  float4* sG4 = fsm4;                                            // m/2 float4: (h, lK) pairs of g^ + L_r
  float* xs = reinterpret_cast<float*>(fsm4 + (A.n_out >> 1));    // [2][FW][2] wave (sum, max), [2][FW] max-shift path
  float2* sF = reinterpret_cast<float2*>(xs + 2 * kMaxWaves * 3);  // this split's row outputs
  float4* sW = reinterpret_cast<float4*>(sF + A.rows_per_split);   // per row: (log a as double-float, a as FP64)
  float* sP = reinterpret_cast<float*>(sW + A.rows_per_split);     // per row: the shift sigma_r
  float* sE = sP + A.rows_per_split;                                // per row: the shift above the base (log2), NaN: none yet
  float* sB = sE + A.rows_per_split;                                // per row: the base shift
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m = A.n_out;
  const EpsConst EC = eps_const(A.st);
  const float K = EC.K;
  const float Lr = sweep_offset(A.cmax, A.st->maxabs[MA_G]);
  const float2* G = A.Uold;
  for (int j2 = tid; j2 < (m >> 1); j2 += FT) {
    float4 u = reinterpret_cast<const float4*>(G)[j2];
    float2 s0 = two_sum(Lr, u.x);
    s0.y += u.y;
    s0 = fast_two_sum(s0.x, s0.y);
    float2 s1 = two_sum(Lr, u.z);
    s1.y += u.w;
    s1 = fast_two_sum(s1.x, s1.y);
    sG4[j2] = make_float4(s0.x, s0.y * K, s1.x, s1.y * K);
  }
  constexpr int NC = 4 * Q;
  double cM[NC];  // this split's column sums of the plan entries
#pragma unroll
  for (int k = 0; k < NC; ++k) cM[k] = 0.0;
  const int r0 = blockIdx.x * A.rows_per_split;
  const int nr = min(A.rows_per_split, A.n_red - r0);
  // shift of row r: the base L_r - f^prev_r + eps log a_r (f^prev the
  // previous pass's row output, so g = T_c(f^prev)) raised by the previous
  // pass's log2 of the row's largest term, so that the largest terms sit
  // near 1; kept in [L_r - max|g^| - cmax, L_r + max|g^|] (there every
  // h - sigma is exact).  A row with no recorded maximum (NaN: the first
  // pass of a stage) takes the max-shift path.
  const float mg = A.st->maxabs[MA_G];
  const float eln2 = (float)(A.st->eps * 0.6931471805599453);
  for (int t = tid; t < nr; t += FT) {
    const float2 lw = A.lw_red[r0 + t];
    const double w = A.w_red64[r0 + t];
    sW[t] = make_float4(lw.x, lw.y, __int_as_float(__double2loint(w)), __int_as_float(__double2hiint(w)));
    const float base = (Lr - A.Uin[r0 + t].x) + (float)A.st->eps * lw.x;
    const float e0 = A.rowmax[r0 + t];
    const bool known = e0 == e0;
    sB[t] = base;
    sE[t] = known ? 0.f : __int_as_float(0x7fc00000);
    sP[t] = fminf(fmaxf(base + (known ? e0 : 0.f) * eln2, Lr - mg - A.cmax), Lr + mg);
  }
  float cv[NC], cn[NC];
  auto load_row = [&](int rl, float* dst) __attribute__((always_inline)) {
    const float* crow = A.C + (size_t)(r0 + rl) * A.ldc;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      // clamped, not skipped: no branch around the load (groups past m are
      // masked where they are used)
      const int j0 = min(4 * (tid + FT * q), m - 4);
      const float4 v = *reinterpret_cast<const float4*>(crow + j0);
      dst[4 * q] = v.x;
      dst[4 * q + 1] = v.y;
      dst[4 * q + 2] = v.z;
      dst[4 * q + 3] = v.w;
    }
  };
  load_row(0, cv);
  __syncthreads();
  // one row: cur holds its costs; the next row's costs are loaded into nxt
  // first, so they are in flight during this row's work (the two buffers
  // alternate, no register copies, so the wait for cur counts only older
  // loads)
  auto row = [&](int rl, int par, float* cur, float* nxt) __attribute__((always_inline)) {
    // unconditional (the last row reloads itself), so that the wait for cur
    // can count exactly the Q younger loads
    load_row(min(rl + 1, nr - 1), nxt);
    // ---- row half: the terms t_rj = 2^((g^_j + L_r - C_rj - sigma_r) K) of
    // row r and their sum S_r (fixed butterfly: the same value in every wave)
    float sig = sP[rl];
    // read before this row's barrier: thread 0 rewrites sE[rl] after it
    // (every wave takes the same branch below)
    const bool known = sE[rl] == sE[rl];
    float tS = 0.f, tY = SIG0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int j2 = 2 * (tid + FT * q);
      if (FULL || 4 * (tid + FT * q) < m) {
        const float4 ga = sG4[j2];
        const float4 gb = sG4[j2 + 1];
        const float y0 = fmaf((ga.x - sig) - cur[4 * q], K, ga.y);
        const float y1 = fmaf((ga.z - sig) - cur[4 * q + 1], K, ga.w);
        const float y2 = fmaf((gb.x - sig) - cur[4 * q + 2], K, gb.y);
        const float y3 = fmaf((gb.z - sig) - cur[4 * q + 3], K, gb.w);
        tY = fmaxf(fmaxf(tY, fmaxf(y0, y1)), fmaxf(y2, y3));
        const float p0 = ex2(y0), p1 = ex2(y1), p2 = ex2(y2), p3 = ex2(y3);
        tS += (p0 + p1) + (p2 + p3);
        cur[4 * q] = p0;
        cur[4 * q + 1] = p1;
        cur[4 * q + 2] = p2;
        cur[4 * q + 3] = p3;
      }
    }
    const int src = lane & (FW - 1);
    float S = wave_sum(tS);
    const float Y = wave_max(tY);
    if (lane == 0) {
      xs[(par * FW + wave) * 2] = S;
      xs[(par * FW + wave) * 2 + 1] = Y;
    }
    // barrier on the LDS writes only: the prefetch of the next row stays in
    // flight (__syncthreads would also wait for every outstanding global load)
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    // states of the other parity are written only after the next barrier,
    // so one barrier per row suffices
    float rS = xs[(par * FW + src) * 2], rY = xs[(par * FW + src) * 2 + 1];
#pragma unroll
    for (int off = FW / 2; off > 0; off >>= 1) {
      rS += __shfl_xor(rS, off, 64);
      rY = fmaxf(rY, __shfl_xor(rY, off, 64));
    }
    // S_r = (row marginal of the plan of (f^prev, g)) / a_r >= min_j b_j and
    // every term <= b_j / a_r; outside [2^-24, 2^24] (extreme weights, or a
    // clamped shift) the row is redone with its own max as the shift (then
    // S_r >= 1)
    if (!known || !(rS >= 0x1p-24f && rS <= 0x1p24f) || (A.flags & F_EXACT_ALL)) {
      load_row(rl, cur);
      float tmax = SIG0;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int j2 = 2 * (tid + FT * q);
        if (FULL || 4 * (tid + FT * q) < m) {
          const float4 ga = sG4[j2];
          const float4 gb = sG4[j2 + 1];
          tmax = fmaxf(fmaxf(fmaxf(tmax, ga.x - cur[4 * q]), ga.z - cur[4 * q + 1]),
                       fmaxf(gb.x - cur[4 * q + 2], gb.z - cur[4 * q + 3]));
        }
      }
      float* xf = xs + 4 * FW;
      const float wm = wave_max(tmax);
      if (lane == 0) xf[wave] = wm;
      __syncthreads();
      sig = xf[src];
#pragma unroll
      for (int off = FW / 2; off > 0; off >>= 1) sig = fmaxf(sig, __shfl_xor(sig, off, 64));
      tS = 0.f;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int j2 = 2 * (tid + FT * q);
        if (FULL || 4 * (tid + FT * q) < m) {
          const float4 ga = sG4[j2];
          const float4 gb = sG4[j2 + 1];
          const float p0 = ex2(fmaf((ga.x - sig) - cur[4 * q], K, ga.y));
          const float p1 = ex2(fmaf((ga.z - sig) - cur[4 * q + 1], K, ga.w));
          const float p2 = ex2(fmaf((gb.x - sig) - cur[4 * q + 2], K, gb.y));
          const float p3 = ex2(fmaf((gb.z - sig) - cur[4 * q + 3], K, gb.w));
          tS += (p0 + p1) + (p2 + p3);
          cur[4 * q] = p0;
          cur[4 * q + 1] = p1;
          cur[4 * q + 2] = p2;
          cur[4 * q + 3] = p3;
        }
      }
      S = wave_sum(tS);
      if (lane == 0) xf[FW + wave] = S;
      __syncthreads();
      rS = xf[FW + src];
#pragma unroll
      for (int off = FW / 2; off > 0; off >>= 1) rS += __shfl_xor(rS, off, 64);
      // the largest term is now 2^(l K) ~ 1
      rY = 0.f;
    }
    // the next pass's shift above its base: this shift's, plus the largest
    // term's exponent (written after the loop)
    if (tid == 0) sE[rl] = (sig - sB[rl]) * K + rY;
    // f^_r = eps log a_r - eps log sum exp((g^ - C)/eps), as double-float:
    // eps lw_r - (sigma - L_r) - eps ln2 log2(S)
    int ke;
    float mant = frexpf(rS, &ke);
    if (mant < 0.70710678f) {
      mant *= 2.f;
      ke -= 1;
    }
    const float2 l2 = fast_two_sum((float)ke, lg2(mant));
    const float2 t = df_mul(EC.eln2_df, l2);
    const float4 wr = sW[rl];
    float2 out = df_mul(EC.eps_df, make_float2(wr.x, wr.y));
    out = df_add_f(out, -sig);
    out = df_add_f(out, Lr);
    out = df_add(out, df_neg(t));
    if (tid == 0) sF[rl] = out;  // written out after the loop: no store in the loop
    // ---- column half: pi_rj = (a_r / S_r) t_rj
    const double wt = __hiloint2double(__float_as_int(wr.w), __float_as_int(wr.z)) / (double)rS;
#pragma unroll
    for (int k = 0; k < NC; ++k) cM[k] = fma(wt, (double)cur[k], cM[k]);
  };
  int rl = 0;
  for (; rl + 1 < nr; rl += 2) {
    row(rl, 0, cv, cn);
    row(rl + 1, 1, cn, cv);
  }
  if (rl < nr) row(rl, 0, cv, cn);
  __syncthreads();
  for (int t = tid; t < nr; t += FT) {
    const_cast<float2*>(A.Uin)[r0 + t] = sF[t];
    A.rowmax[r0 + t] = sE[t];
  }
  // the split's <f^, a> and max |f^.hi| in row order
  double dotF = 0;
  float maxF = 0.f;
  if (tid == 0) {
    for (int t = 0; t < nr; ++t) {
      const float2 o = sF[t];
      const float4 wr = sW[t];
      dotF += __hiloint2double(__float_as_int(wr.w), __float_as_int(wr.z)) * ((double)o.x + (double)o.y);
      maxF = fmaxf(maxF, fabsf(o.x));
    }
  }
  // split partials M[split][m] (FP64) for the merge kernel
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int j0 = 4 * (tid + FT * q);
    if (j0 < m) {
      double2* base = reinterpret_cast<double2*>(reinterpret_cast<double*>(A.part) + (size_t)blockIdx.x * m + j0);
      base[0] = make_double2(cM[4 * q], cM[4 * q + 1]);
      base[1] = make_double2(cM[4 * q + 2], cM[4 * q + 3]);
    }
  }
  if (tid == 0) {
    const_cast<double*>(A.aux_blkdot)[blockIdx.x] = dotF;
    const_cast<float*>(A.aux_blkmax)[blockIdx.x] = maxF;
  }
}

// Merge of the single-read pass: M_j = the splits' column sums in split
// order (four lanes per column, each a contiguous range of splits, then a
// neighbour-first shuffle tree: deterministic), then the finalisation of a
// streaming column sweep with a fixed max.  With sigma_j = fl(L - g_j.hi)
// (exact: |g_j| <= L/3, Sterbenz) and d_j = (sigma_j - L) + g_j.hi its exact
// rounding error, exp((sigma_j - L)/eps) S_j = exp(-g_j/eps) M_j for
// S_j = M_j exp(-(d_j + g_j.lo)/eps) (in FP64), so the finalisation's
// eps log w_j - (sigma_j - L) - eps log S_j is g'_j = T_c(f)_j (eq. foc_g).
// A column with M_j below 2^-76 (or not finite) takes the exact path: its
// four lanes run the online (max, sum) over contiguous row ranges of f^ + L
// - C_rj (the streaming sweeps' arithmetic) and merge them in lane order.
__global__ __launch_bounds__(256) void k_fused_merge(SweepArgs A) {
  if (gate_closed(A.st, A.gate)) return;
  constexpr int LPO = 4, OPB = 64, BATCH = 16;
  const EpsConst EC = eps_const(A.st);
  const float K = EC.K;
  const int n_out = A.n_out, ns = A.nsplit;
  const int col = blockIdx.x * OPB + (int)threadIdx.x / LPO, part = (int)threadIdx.x % LPO;
  const int colc = min(col, n_out - 1);
  const int per = (ns + LPO - 1) / LPO;
  const int s0 = part * per, s1 = min(ns, s0 + per);
  const double* pp = reinterpret_cast<const double*>(A.part) + colc;
  double M = 0.0;
  for (int sp0 = s0; sp0 < s1; sp0 += BATCH) {
    double v[BATCH];
#pragma unroll
    for (int q = 0; q < BATCH; ++q) v[q] = pp[(size_t)min(sp0 + q, ns - 1) * n_out];
#pragma unroll
    for (int q = 0; q < BATCH; ++q)
      if (sp0 + q < s1) M += v[q];
  }
#pragma unroll
  for (int off = 1; off < LPO; off <<= 1) {
    const double o = __shfl_xor(M, off, 64);
    M = (part & off) == 0 ? M + o : o + M;
  }
  const float L = sweep_offset_bound(A, A.st->maxabs[A.ma_in], A.st->eps);
  // the same decision in the column's four lanes (same M)
  const bool exact = (A.flags & F_EXACT_ALL) || !(M >= 0x1p-76);
  float sg = SIG0, Ss = 0.f, Sx = 0.f;
  if (exact && col < n_out) {
    const int nr = A.n_red, per_r = (nr + LPO - 1) / LPO;
    const int r0 = part * per_r, r1 = min(nr, r0 + per_r);
    for (int r = r0; r < r1; ++r) {
      const float2 fu = A.Uin[r];
      float2 hh = two_sum(L, fu.x);
      hh.y += fu.y;
      hh = fast_two_sum(hh.x, hh.y);
      const float c = A.C[(size_t)r * A.ldc + col];
      const float v = hh.x - c;
      if (v > sg) {
        const float sc = ex2((sg - v) * K);
        Ss *= sc;
        Sx *= sc;
        sg = v;
      }
      const float2 t = two_sum(Ss, ex2(fmaf((hh.x - sg) - c, K, hh.y * K)));
      Ss = t.x;
      Sx += t.y;
    }
  }
  // lanes in order (every lane takes part in the shuffles)
#pragma unroll
  for (int off = 1; off < LPO; off <<= 1) {
    const float sg2 = __shfl_xor(sg, off, 64), S2 = __shfl_xor(Ss, off, 64), C2 = __shfl_xor(Sx, off, 64);
    float f1, f2;
    if ((part & off) == 0) {
      lse_merge(sg, Ss, Sx, sg2, S2, C2, K, f1, f2);
    } else {
      float t1 = sg2, t2 = S2, t3 = C2;
      lse_merge(t1, t2, t3, sg, Ss, Sx, K, f1, f2);
      sg = t1;
      Ss = t2;
      Sx = t3;
    }
  }
  double err = 0, dot = 0;
  float mxo = 0.f;
  if (col < n_out && part == 0) {
    if (exact) {
      finalize_output<0>(A, EC, col, L, sg, Ss, Sx, nullptr, err, dot, mxo);
    } else {
      const float2 go = A.Uold[col];
      const float sig = L - go.x;
      const float dl = (sig - L) + go.x;
      // the factor is within ~1e-3 of 1: in FP64 (an FP32 rounding of it
      // would put a 6e-8 relative error on every column's M_j, a floor under
      // the L1 error)
      const double Ms = M * exp(-((double)dl + (double)go.y) / A.st->eps);
      const float S = (float)Ms;
      finalize_output<0>(A, EC, col, L, sig, S, (float)(Ms - (double)S), nullptr, err, dot, mxo);
    }
  }
  __shared__ double sbd[8];
  __shared__ float sbf[4];
  err = block_sum_d(err, sbd);
  dot = block_sum_d(dot, sbd + 4);
  mxo = block_max_f(mxo, sbf);
  write_block_scalars(A, blockIdx.x, err, dot, mxo);
  if (arrive_last(A.st, A.nblk)) sweep_finish_body(A);
}

constexpr int kMaxRowsPerSplit = 1024;  // row outputs held in LDS until the end of the pass

bool fused_stored_ok(int n_red, int n_out, long long ldc, const float* C) {
  return n_out >= 4 && n_out <= kMaxCols && n_out % 4 == 0 && ldc % 4 == 0 && ((uintptr_t)C % 16) == 0 &&
         n_red >= 1 && n_red <= 256 * kMaxRowsPerSplit;
}

// rows per workgroup: one workgroup per CU-sized share of the rows, at
// least 16 rows each (the split partials cost 12 bytes per column per split)
int fused_stored_splits(int n_red, int n_out) {
  (void)n_out;
  int rps = (n_red + 255) / 256;
  if (rps < 16) rps = 16;
  return (n_red + rps - 1) / rps;
}

size_t fused_stored_lds(int n_out, int rows_per_split) {
  return (size_t)(n_out / 2) * sizeof(float4) + 2 * kMaxWaves * 3 * sizeof(float) +
         (size_t)rows_per_split * (sizeof(float2) + sizeof(float4) + 3 * sizeof(float));
}

template <int Q, int FT>
static hipError_t go_fused(const SweepArgs& a, hipStream_t s, hipEvent_t mid) {
  const size_t sm = fused_stored_lds(a.n_out, a.rows_per_split);
  // the unmasked form of the 128-register 16-column variant spills: masks there
  const bool full = a.n_out == 4 * FT * Q && FT == 1024 && Q <= 2;
  const void* fn = (const void*)k_sk_fused_stored<Q, FT, false>;
  if constexpr (FT == 1024) {
    if (full) fn = (const void*)k_sk_fused_stored<Q, FT, true>;
  }
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  if constexpr (FT == 1024) {
    if (full) hipLaunchKernelGGL((k_sk_fused_stored<Q, FT, true>), dim3(a.nsplit), dim3(FT), sm, s, a);
    else hipLaunchKernelGGL((k_sk_fused_stored<Q, FT, false>), dim3(a.nsplit), dim3(FT), sm, s, a);
  } else {
    hipLaunchKernelGGL((k_sk_fused_stored<Q, FT, false>), dim3(a.nsplit), dim3(FT), sm, s, a);
  }
  if (mid) (void)hipEventRecord(mid, s);
  hipLaunchKernelGGL(k_fused_merge, dim3((a.n_out + 63) / 64), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sk_fused_stored(const SweepArgs& a, hipStream_t s, hipEvent_t mid) {
  if (g_recorder) {  // no batched twin
    g_recorder->unsupported = true;
    return hipSuccess;
  }
  if (!fused_stored_ok(a.n_red, a.n_out, a.ldc, a.C) || a.ell != 0 || a.rows_per_split > kMaxRowsPerSplit)
    return hipErrorInvalidValue;
  if (a.rows_per_split * (long long)(a.nsplit - 1) >= a.n_red || a.rows_per_split * (long long)a.nsplit < a.n_red)
    return hipErrorInvalidValue;
  // 1024 threads (four waves per SIMD) with 4, 8 or 16 columns each
  if (a.n_out <= 4096) return go_fused<1, 1024>(a, s, mid);
  if (a.n_out <= 8192) return go_fused<2, 1024>(a, s, mid);
  return go_fused<4, 1024>(a, s, mid);
}

}  // namespace sknr
