// Single-read SK iteration over a stored cost (Sec. 2, eq. SK_iterations).
//
// The two-pass iteration reads C twice: g = T_c(f) by columns, then
// f = T_r(g) by rows.  Here one pass reads each row of C once and does both
// halves that touch it: the row's output f_i = T_r(g)_i (eq. foc_f), then,
// with that f_i, the row's terms of the column log-sum-exp of T_c(f)
// (eq. foc_g) for the next g.  A workgroup owns a contiguous block of rows
// (a split of the column reduction) and keeps the running (max, S, Sc) of
// its 4Q columns per thread in registers; the split partials then go
// through the merge and finish kernels of the streaming column sweep, which
// also test the pair (f, g_in) for convergence against g_out = T_c(f).
//
// Arithmetic of both halves is the one of the streaming sweeps: the reduce
// side enters offset by L as a double-float (h, l) with l pre-scaled by
// K = log2(e)/eps, the running max sigma is one of the values fl(h - C), so
// h - sigma is exact and the exponent fma((h - sigma) - C, K, l K) is
// rounded only relative to its own size.  The row half uses L_r from
// max|g^|; the column half cannot know max|f^| before its rows exist and
// uses the bound |f^_i| <= max|g^| + max|C| + eps (max|log a| + max|log b|)
// (a c-transform lies between the extremes of g_j - C_ij), which the merge
// kernel forms in the same order.
#include "sknr_internal.h"
#include "sknr_device.h"

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
  float* xs = reinterpret_cast<float*>(fsm4 + (A.n_out >> 1));    // [2][FW][2] wave states
  float2* sF = reinterpret_cast<float2*>(xs + 2 * kMaxWaves * 3);  // this split's row outputs
  float4* sW = reinterpret_cast<float4*>(sF + A.rows_per_split);   // per row: (log a as double-float, a as FP64)
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m = A.n_out;
  const EpsConst EC = eps_const(A.st);
  const float K = EC.K;
  const float Lr = sweep_offset(A.cmax, A.st->maxabs[MA_G]);
  const float Lc = sweep_offset_bound(A, A.st->maxabs[MA_G], A.st->eps);
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
  float csig[NC], cS[NC], cSc[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    csig[k] = SIG0;
    cS[k] = 0.f;
    cSc[k] = 0.f;
  }
  const int r0 = blockIdx.x * A.rows_per_split;
  const int nr = min(A.rows_per_split, A.n_red - r0);
  for (int t = tid; t < nr; t += FT) {
    const float2 lw = A.lw_red[r0 + t];
    const double w = A.w_red64[r0 + t];
    sW[t] = make_float4(lw.x, lw.y, __int_as_float(__double2loint(w)), __int_as_float(__double2hiint(w)));
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
    // ---- row half: (sigma, S) of this thread's terms of row r, g^ + L_r - C
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
    float tS = 0.f;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int j2 = 2 * (tid + FT * q);
      if (FULL || 4 * (tid + FT * q) < m) {
        float4 ga = sG4[j2];
        float4 gb = sG4[j2 + 1];
        const float p0 = ex2(fmaf((ga.x - tmax) - cur[4 * q], K, ga.y));
        const float p1 = ex2(fmaf((ga.z - tmax) - cur[4 * q + 1], K, ga.w));
        const float p2 = ex2(fmaf((gb.x - tmax) - cur[4 * q + 2], K, gb.y));
        const float p3 = ex2(fmaf((gb.z - tmax) - cur[4 * q + 3], K, gb.w));
        tS += (p0 + p1) + (p2 + p3);
      }
    }
    // wave state: the wave max, each lane's sum rescaled to it, then a
    // fixed butterfly sum (all lanes end with the same values)
    const float wmax = wave_max(tmax);
    float S = tS * ex2((tmax - wmax) * K);
    S = wave_sum(S);
    float* slot = xs + (par * FW + wave) * 2;
    if (lane == 0) {
      slot[0] = wmax;
      slot[1] = S;
    }
    // barrier on the LDS writes only: the prefetch of the next row stays in
    // flight (__syncthreads would also wait for every outstanding global load)
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    // every wave merges the FW wave states with the same FW-lane butterfly
    // (the same result in every wave); states of the other parity are
    // written only after the next barrier, so one barrier per row suffices
    const float* xp = xs + par * FW * 2;
    const int src = lane & (FW - 1);
    const float ws = xp[2 * src];
    float rs = ws;
#pragma unroll
    for (int off = FW / 2; off > 0; off >>= 1) rs = fmaxf(rs, __shfl_xor(rs, off, 64));
    float rS = xp[2 * src + 1] * ex2((ws - rs) * K);
#pragma unroll
    for (int off = FW / 2; off > 0; off >>= 1) rS += __shfl_xor(rS, off, 64);
    const float rSc = 0.f;
    // f^_r = eps log a_r - eps log sum exp((g^ - C)/eps), as double-float:
    // eps lw_r - (sigma - L_r) - eps ln2 log2(S + Sc)
    int ke;
    float mant = frexpf(rS, &ke);
    if (mant < 0.70710678f) {
      mant *= 2.f;
      ke -= 1;
    }
    float2 l2 = fast_two_sum((float)ke, lg2(mant));
    l2.y += (rSc / rS) * 1.4426950408889634f;
    const float2 t = df_mul(EC.eln2_df, l2);
    const float4 wr = sW[rl];
    float2 out = df_mul(EC.eps_df, make_float2(wr.x, wr.y));
    out = df_add_f(out, -rs);
    out = df_add_f(out, Lr);
    out = df_add(out, df_neg(t));
    if (tid == 0) sF[rl] = out;  // written out after the loop: no store in the loop
    // ---- column half: this row's terms f^_r + L_c - C_rj
    float2 hh = two_sum(Lc, out.x);
    hh.y += out.y;
    hh = fast_two_sum(hh.x, hh.y);
    const float hc = hh.x, lcK = hh.y * K;
    // a new column max is rare after the first rows: one test per row,
    // then the rescale pass only when some lane needs it
    bool up = false;
#pragma unroll
    for (int k = 0; k < NC; ++k) up |= hc - cur[k] > csig[k];
    if (__any(up)) {
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const float sv = hc - cur[k];
        const bool raise = sv > csig[k] && (FULL || 4 * (tid + FT * (k >> 2)) < m);
        const float sc = raise ? ex2((csig[k] - sv) * K) : 1.f;
        cS[k] *= sc;
        cSc[k] *= sc;
        csig[k] = raise ? sv : csig[k];
      }
    }
    // S >= 1 >= p here (the split's max term is in S, every p <= 1 up to
    // rounding), so Fast2Sum keeps the error term
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const float pk = ex2(fmaf((hc - csig[k]) - cur[k], K, lcK));
      const float p = (FULL || 4 * (tid + FT * (k >> 2)) < m) ? pk : 0.f;
      const float2 ts = fast_two_sum(cS[k], p);
      cS[k] = ts.x;
      cSc[k] += ts.y;
    }
  };
  int rl = 0;
  for (; rl + 1 < nr; rl += 2) {
    row(rl, 0, cv, cn);
    row(rl + 1, 1, cn, cv);
  }
  if (rl < nr) row(rl, 0, cv, cn);
  __syncthreads();
  for (int t = tid; t < nr; t += FT) const_cast<float2*>(A.Uin)[r0 + t] = sF[t];
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
  // split partials [split][3][m] for the merge kernel (float4 stores)
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int j0 = 4 * (tid + FT * q);
    if (j0 < m) {
      float* base = A.part + (size_t)blockIdx.x * 3 * m + j0;
      *reinterpret_cast<float4*>(base) = make_float4(csig[4 * q], csig[4 * q + 1], csig[4 * q + 2], csig[4 * q + 3]);
      *reinterpret_cast<float4*>(base + m) = make_float4(cS[4 * q], cS[4 * q + 1], cS[4 * q + 2], cS[4 * q + 3]);
      *reinterpret_cast<float4*>(base + 2 * (size_t)m) =
          make_float4(cSc[4 * q], cSc[4 * q + 1], cSc[4 * q + 2], cSc[4 * q + 3]);
    }
  }
  if (tid == 0) {
    const_cast<double*>(A.aux_blkdot)[blockIdx.x] = dotF;
    const_cast<float*>(A.aux_blkmax)[blockIdx.x] = maxF;
  }
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
         (size_t)rows_per_split * (sizeof(float2) + sizeof(float4));
}

template <int Q, int FT>
static hipError_t go_fused(const SweepArgs& a, hipStream_t s, hipEvent_t mid) {
  const size_t sm = fused_stored_lds(a.n_out, a.rows_per_split);
  // the unmasked form of the 256-register variant spills: masks there
  const bool full = a.n_out == 4 * FT * Q && FT == 1024;
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
  return launch_sweep_tail(a, s);
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
  // 1024 threads while the columns of a thread fit in 128 registers, then
  // 512 threads with twice the columns (256 registers)
  if (a.n_out <= 4096) return go_fused<1, 1024>(a, s, mid);
  if (a.n_out <= 8192) return go_fused<2, 1024>(a, s, mid);
  return go_fused<8, 512>(a, s, mid);
}

}  // namespace sknr
