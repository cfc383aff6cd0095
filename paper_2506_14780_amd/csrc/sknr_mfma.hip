// Matrix-core cost for squared-Euclidean problems with the cross term on
// bf16 MFMA (gfx950 v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
// The cost of a pair is built as
//     C~_ij = fma(-2 s, xy_ij, n_i + n_j),   n_i = fl32(s * ||x~_i||^2),
// where x~ are the centred points rounded to bf16 (BF16), to a hi + lo
// pair of bf16 (BF16X3) or to hi + mid + lo (BF16X6), s is the cost scale
// and xy_ij = x~_i . y~_j comes from matrix-core tiles.  BF16X3 keeps
// hi*hi + hi*lo + lo*hi; BF16X6 keeps hi*hi + hi*mid + mid*hi + hi*lo +
// lo*hi + mid*mid.  Each mirrored pair (a*b, b*a) runs as two chains in
// separate accumulators joined by an FP32 add (commutative), and every
// other chain is a single operand pair used in both orders, so C~ is the
// same matrix whichever side is the reduce side of a sweep: a matrix-core
// tile is symmetric under swapping its two operands, and so the row and
// column c-transforms see one and the same cost.
//
// The MFMA 16x16x32 lane layout (64 lanes, g = lane / 16, c = lane % 16):
//   operand A (16 x 32): lane supplies row c, k = 8g .. 8g+7
//   operand B (32 x 16): lane supplies column c, k = 8g .. 8g+7
//   result    (16 x 16): lane holds rows 4g .. 4g+3 of column c
// With A = reduce-side points and B = output-side points, a lane of the
// result owns one output column and four reduce rows of each tile, so the
// online log-sum-exp of the streaming sweep runs directly on MFMA results.
#include "sknr_device.h"

#include <stdlib.h>

#include <type_traits>

namespace sknr {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ bf16x8 as_bf8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// round-to-nearest-even FP32 -> bf16 (finite inputs)
__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// Cross products of one 16 x 16 tile (ks K-steps of 32).  XP = number of
// bf16 parts per coordinate (1: hi; 2: hi, lo; 3: hi, mid, lo).  The order
// is fixed: the smallest mirrored pair first (separate accumulators, FP32
// add), then for XP = 3 the mid*mid chain from that sum and the hi*mid
// pair added to it, then the hi*hi chain starting from the total.  Operand
// p[q][s] is part q (0 = hi, 1 = lo for XP = 2; 0 = hi, 1 = mid, 2 = lo for
// XP = 3) of K-step s.
template <int XP, int KR>
__device__ __forceinline__ f32x4 cross_regs(const bf16x8 (&a)[3][KR], const bf16x8 (&b)[3][KR]) {
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  if (XP >= 2) {
    constexpr int LO = XP - 1;  // index of the lo part
    f32x4 t1 = acc, t2 = acc;
#pragma unroll
    for (int s = 0; s < KR; ++s) {
      t1 = mfma_bf16(a[0][s], b[LO][s], t1);
      t2 = mfma_bf16(a[LO][s], b[0][s], t2);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = t1[i] + t2[i];
  }
  if (XP == 3) {
#pragma unroll
    for (int s = 0; s < KR; ++s) acc = mfma_bf16(a[1][s], b[1][s], acc);
    f32x4 t1 = {0.f, 0.f, 0.f, 0.f}, t2 = t1;
#pragma unroll
    for (int s = 0; s < KR; ++s) {
      t1 = mfma_bf16(a[0][s], b[1][s], t1);
      t2 = mfma_bf16(a[1][s], b[0][s], t2);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = acc[i] + (t1[i] + t2[i]);
  }
#pragma unroll
  for (int s = 0; s < KR; ++s) acc = mfma_bf16(a[0][s], b[0][s], acc);
  return acc;
}

// The same tile with operands read from memory per K-step (any dpad):
// pa[q] / pb[q] = uint4 rows of part q of the lane's A / B point, offset
// by the lane's k-slice.
template <int XP>
__device__ __forceinline__ f32x4 cross_mem(const uint4* const (&pa)[3], const uint4* const (&pb)[3], int ks) {
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  if (XP >= 2) {
    constexpr int LO = XP - 1;
    f32x4 t1 = acc, t2 = acc;
    for (int s = 0; s < ks; ++s) {
      t1 = mfma_bf16(as_bf8(pa[0][4 * s]), as_bf8(pb[LO][4 * s]), t1);
      t2 = mfma_bf16(as_bf8(pa[LO][4 * s]), as_bf8(pb[0][4 * s]), t2);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = t1[i] + t2[i];
  }
  if (XP == 3) {
    for (int s = 0; s < ks; ++s) acc = mfma_bf16(as_bf8(pa[1][4 * s]), as_bf8(pb[1][4 * s]), acc);
    f32x4 t1 = {0.f, 0.f, 0.f, 0.f}, t2 = t1;
    for (int s = 0; s < ks; ++s) {
      t1 = mfma_bf16(as_bf8(pa[0][4 * s]), as_bf8(pb[1][4 * s]), t1);
      t2 = mfma_bf16(as_bf8(pa[1][4 * s]), as_bf8(pb[0][4 * s]), t2);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = acc[i] + (t1[i] + t2[i]);
  }
  for (int s = 0; s < ks; ++s) acc = mfma_bf16(as_bf8(pa[0][4 * s]), as_bf8(pb[0][4 * s]), acc);
  return acc;
}

// ============================================================================
// Streaming c-transform sweep in the matrix-core lane layout.  A workgroup
// owns NC = 64*NT outputs (wave w: columns [16*NT*w, 16*NT*(w+1)) of the
// block, NT tiles of 16) and one split of the reduce side, processed in
// tiles of 16 rows.  Lane (g, c) keeps an online (sig, S, Sc) state per
// output tile over the rows 4g..4g+3 of every row tile; the four states of a
// column merge by a butterfly (xor 16, xor 32) with a fixed operand order,
// and the partial is written in the layout of the generic streaming sweep
// ([nsplit][3+ell][n_out]) so that the same split merge and finishing
// kernels complete it.
//
// Cost: XP >= 1 bf16 parts, cross term on matrix cores (KS > 0: K-steps
// known at compile time, the output-side operands stay in registers;
// KS == 0: any dpad, operands reloaded); XP == 0: FP32 squared distance of
// DV-dimensional points on the VALU, in the order of the generic sweep
// (t_k = x_k - y_k, t_0^2 then fma(t_k, t_k, .)), times the cost scale when
// SC.
//
// Weighted sweeps (ELL > 0): W = sum_r p_r V_r is a contraction over the
// reduce rows, run on FP32 matrix cores (16x16x4 f32: A = V^T with M = basis
// index, K = rows; B = p with K = rows, N = columns; lane (g, c) supplies
// V[row 4g+i][basis c] and p[row 4g+i][column c] for MFMA i of a row tile
// and holds W[basis 4g..4g+3][column c]).  The four row groups of a column
// share one shift sig, so every lane rescales only its own column of the
// accumulators.  The shift only has to keep the terms finite: it is
// re-synchronised (cross-lane max) only when some row exceeds it by more
// than 32 / K, a wave-uniform test, so terms stay below 2^32 and the
// relative precision of FP32 is unchanged.  With the VALU cost the V rows of
// the split are staged in LDS, transposed (one 16-byte read gives a lane
// its four rows of a basis column).
// ============================================================================
__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int ELL, int KS, int XP, int NT, int DV = 0, bool SC = false>
__device__ __forceinline__ void sweep_mfma_body(const SweepArgs& A, const int bx, const int by) {
  if (gate_closed(A.st, A.gate)) return;
  extern __shared__ float4 smem4[];
  constexpr int EL = ELL > 0 ? ELL : 1;
  constexpr int NQ = 3 + (ELL > 0 ? ELL : 0);
  constexpr int NB = ELL > 0 ? (ELL + 15) / 16 : 1;  // 16-wide basis blocks of W
  constexpr int NCW = 16 * NT;
  constexpr int NC = WAVES * NCW;
  constexpr int KR = KS > 0 ? KS : 1;
  constexpr int DQ = XP == 0 ? (DV > 0 ? DV : 1) : 1;  // output-side point width (VALU cost)
  constexpr int DX = XP == 0 && DV > 2 ? DV - 2 : 0;   // reduce-side coordinates beyond sR.zw
  constexpr bool VLDS = XP == 0 && ELL > 0;             // V of the split in LDS
  static_assert(XP > 0 || (DV >= 1 && DV <= 8), "VALU cost: 1 <= d <= 8");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, c16 = lane & 15;
  const int r0 = by * A.rows_per_split;
  const int nr = min(A.rows_per_split, A.n_red - r0);
  const EpsConst EC = eps_const(A.st);
  const float K = EC.K;
  const float L = sweep_offset(A.cmax, A.st->maxabs[A.ma_in]);
  const int ks = KS > 0 ? KS : (A.dpad >> 5);
  const int dq = A.dpad >> 3;  // uint4 per packed point
  const float m2cs = A.m2cs;
  const float cscale = A.cscale;
  const float thr = 32.f / K;  // slack of the lazy shift (cost units)

  // reduce-side rows of this split: offset hat potential U + L = h + l as
  // (h, l K), then the scaled squared norm (matrix-core cost) or the first
  // two coordinates (VALU cost; sX holds the rest)
  float4* sR = smem4;
  float* sX = reinterpret_cast<float*>(smem4 + A.rows_per_split);
  // transposed V: sV[l * vrs + row], vrs = rows_per_split + 4 (16-byte rows)
  const int vrs = A.rows_per_split + 4;
  float* sV = sX + (size_t)A.rows_per_split * DX;
  for (int t = threadIdx.x; t < nr; t += TPB) {
    float2 u = A.Uin[r0 + t];
    float2 s = two_sum(L, u.x);
    s.y += u.y;
    s = fast_two_sum(s.x, s.y);
    if (XP > 0) {
      sR[t] = make_float4(s.x, s.y * K, A.Nred[r0 + t], 0.f);
    } else {
      const float* xp = A.Pred + (size_t)(r0 + t) * DQ;
      sR[t] = make_float4(s.x, s.y * K, xp[0], DQ > 1 ? xp[DQ > 1 ? 1 : 0] : 0.f);
#pragma unroll
      for (int k = 0; k < DX; ++k) sX[t * (DX > 0 ? DX : 1) + k] = xp[2 + k];
    }
  }
  if (VLDS) {
    // the split's rows of V are one contiguous block of nr * EL floats
    // (EL a multiple of 8, r0 of 16: 16-byte aligned): eight float4 loads
    // per thread in flight at once, then the transposed LDS writes
    const float4* vb = reinterpret_cast<const float4*>(A.Vred + (size_t)r0 * EL);
    const int total4 = nr * EL / 4;
    for (int base = 0; base < total4; base += 8 * TPB) {
      float4 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = vb[min(base + u * TPB + (int)threadIdx.x, total4 - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i4 = base + u * TPB + (int)threadIdx.x;
        if (i4 < total4) {
          const int r = (4 * i4) / EL, l = 4 * i4 - r * EL;
          sV[l * vrs + r] = v[u].x;
          sV[(l + 1) * vrs + r] = v[u].y;
          sV[(l + 2) * vrs + r] = v[u].z;
          sV[(l + 3) * vrs + r] = v[u].w;
        }
      }
    }
  }
  __syncthreads();

  const int cb = bx * NC + wave * NCW;
  float hy[NT];
  int colc[NT];
  // parts of the output-side points: [0] hi, then lo (XP = 2) or mid, lo
  const uint4* const pout[3] = {A.Hout, XP == 3 ? A.Mout : A.Lout, A.Lout};
  const uint4* const pred[3] = {A.Hred, XP == 3 ? A.Mred : A.Lred, A.Lred};
  bf16x8 bo[NT][3][KR];
  float qy[NT][DQ];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    colc[t] = min(cb + 16 * t + c16, A.n_out - 1);
    if (XP > 0) {
      hy[t] = A.Nout[colc[t]];
      if (KS > 0) {
        const size_t base = (size_t)colc[t] * dq + g;
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
          for (int s = 0; s < KR; ++s) bo[t][q][s] = q < XP ? as_bf8(pout[q][base + 4 * s]) : bo[t][0][s];
      }
    } else {
      hy[t] = 0.f;
#pragma unroll
      for (int k = 0; k < DQ; ++k) qy[t][k] = A.Pout[(size_t)colc[t] * DQ + k];
    }
  }

  // (sig, S + Sc) per output as in the generic sweep; T collects the
  // chunk sums of two row tiles in plain FP32 (at most 8 terms <= 1 each)
  // before one TwoSum adds it into (S, Sc)
  float sig[NT], S[NT], Sc[NT], T[NT];
  f32x4 W[NT][NB];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    sig[t] = SIG0;
    S[t] = 0.f;
    Sc[t] = 0.f;
    T[t] = 0.f;
#pragma unroll
    for (int b = 0; b < NB; ++b) W[t][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  }

  // (the lambdas below capture these locals, not the argument struct, so
  // that the struct stays in kernel-argument registers)
  const float* const Vred = A.Vred;
  // Software pipeline over row tiles: while the log-sum-exp of tile k runs
  // on the VALU, the matrix cores work on tile k+1 (its operands loaded one
  // iteration earlier) and the loads of tile k+2 are in flight.
  bf16x8 ai[3][KR];
  auto load_a = [&](int rt) __attribute__((always_inline)) {
    if (XP > 0 && KS > 0) {
      const size_t ra = (size_t)(r0 + min(rt + c16, nr - 1)) * dq + g;
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int s = 0; s < KR; ++s) ai[q][s] = q < XP ? as_bf8(pred[q][ra + 4 * s]) : ai[0][s];
    }
  };
  auto cross = [&](int rt, f32x4 (&xy)[NT]) __attribute__((always_inline)) {
    if (XP == 0) return;
    if (KS > 0) {
#pragma unroll
      for (int t = 0; t < NT; ++t) xy[t] = cross_regs<XP, KR>(ai, bo[t]);
    } else {
      const size_t ra = (size_t)(r0 + min(rt + c16, nr - 1)) * dq + g;
      const uint4* const pa[3] = {pred[0] + ra, pred[1] + ra, pred[2] + ra};
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const size_t rb = (size_t)colc[t] * dq + g;
        const uint4* const pb[3] = {pout[0] + rb, pout[1] + rb, pout[2] + rb};
        xy[t] = cross_mem<XP>(pa, pb, ks);
      }
    }
  };
  // online log-sum-exp update of one row tile (MASK: rows past nr present)
  auto lse_tile = [&](auto maskc, int rt, const f32x4 (&xy)[NT]) __attribute__((always_inline)) {
    constexpr bool MASK = decltype(maskc)::value;
    float4 rw[4];
    bool ok[4];
    int rowc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rl = rt + 4 * g + i;
      ok[i] = MASK ? rl < nr : true;
      rowc[i] = ok[i] ? rl : nr - 1;
      rw[i] = sR[rowc[i]];
    }
    float xr[4][DX > 0 ? DX : 1];
    if (DX > 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < DX; ++k) xr[i][k] = sX[rowc[i] * (DX > 0 ? DX : 1) + k];
    }
    float p[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      float s[4], cvk[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float cv;
        if (XP > 0) {
          cv = fmaf(m2cs, xy[t][i], rw[i].z + hy[t]);
        } else {
          float dt = rw[i].z - qy[t][0];
          float c2 = dt * dt;
          if (DQ > 1) {
            dt = rw[i].w - qy[t][DQ > 1 ? 1 : 0];
            c2 = fmaf(dt, dt, c2);
          }
#pragma unroll
          for (int k = 0; k < DX; ++k) {
            dt = xr[i][k] - qy[t][2 + k < DQ ? 2 + k : 0];
            c2 = fmaf(dt, dt, c2);
          }
          cv = SC ? c2 * cscale : c2;
        }
        cvk[i] = cv;
        s[i] = (!MASK || ok[i]) ? rw[i].x - cv : SIG0;
      }
      float mx = fmaxf(fmaxf(s[0], s[1]), fmaxf(s[2], s[3]));
      if (ELL > 0) {
        // one shift per column across its four row groups (W sums over
        // them), raised lazily: the test is wave-uniform
        if (__any(mx > sig[t] + thr)) {
          mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
          mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
          if (mx > sig[t]) {
            const float sc = ex2((sig[t] - mx) * K);
            S[t] *= sc;
            Sc[t] *= sc;
            T[t] *= sc;
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
              for (int i = 0; i < 4; ++i) W[t][b][i] *= sc;
            sig[t] = mx;
          }
        }
      } else if (mx > sig[t]) {
        const float sc = ex2((sig[t] - mx) * K);
        S[t] *= sc;
        Sc[t] *= sc;
        T[t] *= sc;
        sig[t] = mx;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // (h - sig) exact, see sweep_offset
        const float pv = ex2(fmaf((rw[i].x - sig[t]) - cvk[i], K, rw[i].y));
        p[t][i] = (!MASK || ok[i]) ? pv : 0.f;
      }
      T[t] += (p[t][0] + p[t][1]) + (p[t][2] + p[t][3]);
    }
    if (ELL > 0) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int l = 16 * b + c16;
        float va[4];
        if (VLDS) {
          // rows rt+4g .. rt+4g+3 lie inside the staged block (rt + 16 <=
          // rows_per_split); rows past nr are unset and replaced by 0
          const float4 v4 = *reinterpret_cast<const float4*>(&sV[(l < EL ? l : 0) * vrs + rt + 4 * g]);
          va[0] = v4.x;
          va[1] = v4.y;
          va[2] = v4.z;
          va[3] = v4.w;
#pragma unroll
          for (int i = 0; i < 4; ++i) va[i] = (l < EL && (!MASK || ok[i])) ? va[i] : 0.f;
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) va[i] = l < EL ? Vred[(size_t)(r0 + rowc[i]) * EL + (l < EL ? l : 0)] : 0.f;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) W[t][b] = mfma_f32(va[i], p[t][i], W[t][b]);
      }
    }
  };

  auto flush = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const float2 ts = two_sum(S[t], T[t]);
      S[t] = ts.x;
      Sc[t] += ts.y;
      T[t] = 0.f;
    }
  };
  auto lse_any = [&](int rt, const f32x4 (&xy)[NT]) __attribute__((always_inline)) {
    if (rt + 16 <= nr) lse_tile(std::integral_constant<bool, false>{}, rt, xy);
    else lse_tile(std::integral_constant<bool, true>{}, rt, xy);
  };

  // two row tiles per iteration; the xy buffers alternate roles
  f32x4 xy0[NT], xy1[NT];
  load_a(0);
  cross(0, xy0);
  if (16 < nr) load_a(16);
  for (int rt = 0; rt < nr; rt += 32) {
    if (rt + 16 < nr) {
      cross(rt + 16, xy1);
      if (rt + 32 < nr) load_a(rt + 32);
    }
    lse_any(rt, xy0);
    if (rt + 16 < nr) {
      if (rt + 32 < nr) {
        cross(rt + 32, xy0);
        if (rt + 48 < nr) load_a(rt + 48);
      }
      lse_any(rt + 16, xy1);
    }
    flush();
  }

  // butterfly over the four row groups of a column: both partners merge
  // (lower, upper) in that order, so they hold identical results
#pragma unroll
  for (int off = 16; off <= 32; off <<= 1) {
    const bool lower = (lane & off) == 0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const float sg2 = __shfl_xor(sig[t], off, 64), S2 = __shfl_xor(S[t], off, 64),
                  C2 = __shfl_xor(Sc[t], off, 64);
      float f1, f2;
      if (lower) {
        lse_merge(sig[t], S[t], Sc[t], sg2, S2, C2, K, f1, f2);
      } else {
        float t1 = sg2, t2 = S2, t3 = C2;
        lse_merge(t1, t2, t3, sig[t], S[t], Sc[t], K, f1, f2);
        sig[t] = t1;
        S[t] = t2;
        Sc[t] = t3;
      }
    }
  }

  // partial of this split: lanes g = 0, 1, 2 write sig, S, Sc; lane (g, c)
  // writes W[basis 16b + 4g + i][column c]
  const int n_out = A.n_out;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = cb + 16 * t + c16;
    if (col < n_out) {
      float* base = A.part + (size_t)by * NQ * n_out + col;
      if (g == 0) store_wt(base, sig[t]);
      else if (g == 1) store_wt(base + (size_t)n_out, S[t]);
      else if (g == 2) store_wt(base + (size_t)2 * n_out, Sc[t]);
#pragma unroll
      for (int b = 0; b < (ELL > 0 ? NB : 0); ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int l = 16 * b + 4 * g + i;
          if (l < EL) store_wt(base + (size_t)(3 + l) * n_out, W[t][b][i]);
        }
    }
  }
}

template <int ELL, int KS, int XP, int NT, int DV = 0, bool SC = false>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(2))) void k_sweep_mfma(SweepArgs A) {
  sweep_mfma_body<ELL, KS, XP, NT, DV, SC>(A, blockIdx.x, blockIdx.y);
}
template <int ELL, int KS, int XP, int NT, int DV = 0, bool SC = false>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(2))) void k_sweep_mfma_b(BatchTab T) {
  int bx, by;
  const int slot = batch_slot(T, blockIdx.x, &bx, &by);
  sweep_mfma_body<ELL, KS, XP, NT, DV, SC>(*static_cast<const SweepArgs*>(T.args[slot]), bx, by);
}

// ----------------------------------------------------------- geometry
// output tiles of 16 per wave (matrix-core cost): 4 for plain sweeps
// (SKNR_MFMA_NT=2 overrides), 2 for weighted sweeps, 1 for 32-wide weighted
// sweeps with three parts (register budget of the output-side operands, the
// W accumulators and the V operands)
//
// VALU-cost weighted sweeps: one output tile per wave and at least 256
// reduce rows per split (SKNR_PW_RMIN overrides).  Measured on the 4096^2
// d = 2 solve: more splits (fewer rows each) cost more in partials written
// and merged (3 + l floats per output per split) than they gain in
// parallelism, and more output tiles per wave halve the workgroup count.
constexpr int kPwNT = 1;
static int pw_rmin() {
  static const int env = getenv("SKNR_PW_RMIN") ? atoi(getenv("SKNR_PW_RMIN")) : 0;
  return env >= 16 ? (env & ~15) : 256;
}

static int mfma_nt(int ell, int parts) {
  static const int env_nt = getenv("SKNR_MFMA_NT") ? atoi(getenv("SKNR_MFMA_NT")) : 0;
  if (parts == 0) return kPwNT;
  if (ell > 16 && parts >= 3) return 1;
  if (ell > 0) return 2;
  return env_nt == 2 ? 2 : 4;
}

size_t mfma_part_floats(int n_out, int n_red, int ell, int parts, int* nsplit, int* rps, int* nblk) {
  const int nc = 64 * mfma_nt(ell, parts);
  const int ncb = (n_out + nc - 1) / nc;
  static const int env_target = getenv("SKNR_SWEEP_TARGET_WG") ? atoi(getenv("SKNR_SWEEP_TARGET_WG")) : 0;
  const int target = env_target > 0 ? env_target : 2048;
  int ns = (target + ncb - 1) / ncb;
  int r = (n_red + ns - 1) / ns;
  r = (r + 15) & ~15;
  const int rmin = (parts == 0 && ell > 0) ? pw_rmin() : 64;
  if (r < rmin) r = rmin;
  // VALU-cost weighted sweeps stage V in LDS: 16 + 4 + 4 ell bytes per row
  // (+ 4 padding rows) within 48 KiB
  const int ellp0 = ell <= 0 ? 0 : (ell <= 8 ? 8 : (ell <= 16 ? 16 : 32));
  const int rcap = (parts == 0 && ell > 0) ? (((49152 - 16 * ellp0) / (20 + 4 * ellp0)) & ~15) : 2048;
  if (r > rcap) r = rcap;
  const int rmax = (n_red + 15) & ~15;
  if (r > rmax) r = rmax;
  ns = (n_red + r - 1) / r;
  *nsplit = ns;
  *rps = r;
  *nblk = merge_blocks(n_out, ell);
  const int ellp = ell <= 0 ? 0 : (ell <= 8 ? 8 : (ell <= 16 ? 16 : 32));
  return (size_t)ns * (3 + ellp) * n_out;
}

template <int ELL, int XP, int NT>
static void go_mfma(const SweepArgs& a, hipStream_t s) {
  const int nc = 64 * NT;
  dim3 grid((a.n_out + nc - 1) / nc, a.nsplit);
  const size_t sm = (size_t)a.rows_per_split * sizeof(float4);
  const int ks = a.dpad >> 5;
  if (g_recorder) {
    record_launch(ks == 1   ? (const void*)k_sweep_mfma_b<ELL, 1, XP, NT>
                  : ks == 2 ? (const void*)k_sweep_mfma_b<ELL, 2, XP, NT>
                            : (const void*)k_sweep_mfma_b<ELL, 0, XP, NT>,
                  a, grid, TPB, sm);
    return;
  }
  if (ks == 1) hipLaunchKernelGGL((k_sweep_mfma<ELL, 1, XP, NT>), grid, dim3(TPB), sm, s, a);
  else if (ks == 2) hipLaunchKernelGGL((k_sweep_mfma<ELL, 2, XP, NT>), grid, dim3(TPB), sm, s, a);
  else hipLaunchKernelGGL((k_sweep_mfma<ELL, 0, XP, NT>), grid, dim3(TPB), sm, s, a);
}

template <int XP>
static void go_mfma_ell(const SweepArgs& a, hipStream_t s) {
  const int e = a.ell;
  if (e == 0) {
    if (mfma_nt(0, XP) == 2) go_mfma<0, XP, 2>(a, s);
    else go_mfma<0, XP, 4>(a, s);
  } else if (e <= 8) go_mfma<8, XP, 2>(a, s);
  else if (e <= 16) go_mfma<16, XP, 2>(a, s);
  else go_mfma<32, XP, (XP >= 3 ? 1 : 2)>(a, s);
}

// weighted sweeps of FP32 point costs with 2 <= d <= 3 (the VALU cost in
// the matrix-core layout, W on FP32 matrix cores)
bool sweep_pw_eligible(int ell, int d) {
  static const int env_pw = getenv("SKNR_PW") ? atoi(getenv("SKNR_PW")) : 1;
  return env_pw != 0 && ell > 0 && (d == 2 || d == 3);
}

template <int ELL, int DV, int NT>
static hipError_t go_pw(const SweepArgs& a, hipStream_t s) {
  dim3 grid((a.n_out + 64 * NT - 1) / (64 * NT), a.nsplit);
  const size_t sm = (size_t)a.rows_per_split * (sizeof(float4) + (DV > 2 ? (DV - 2) * sizeof(float) : 0)) +
                    (size_t)ELL * (a.rows_per_split + 4) * sizeof(float);
  if (sm > 49152 || (a.rows_per_split & 15) || ((uintptr_t)a.Vred & 15)) return hipErrorInvalidValue;
  if (g_recorder) {
    record_launch(a.cscale != 1.0f ? (const void*)k_sweep_mfma_b<ELL, 1, 0, NT, DV, true>
                                   : (const void*)k_sweep_mfma_b<ELL, 1, 0, NT, DV, false>,
                  a, grid, TPB, sm);
    return hipSuccess;
  }
  if (a.cscale != 1.0f) hipLaunchKernelGGL((k_sweep_mfma<ELL, 1, 0, NT, DV, true>), grid, dim3(TPB), sm, s, a);
  else hipLaunchKernelGGL((k_sweep_mfma<ELL, 1, 0, NT, DV, false>), grid, dim3(TPB), sm, s, a);
  return hipSuccess;
}

template <int DV, int NT>
static hipError_t go_pw_ell(const SweepArgs& a, hipStream_t s) {
  if (a.ell <= 8) return go_pw<8, DV, NT>(a, s);
  if (a.ell <= 16) return go_pw<16, DV, NT>(a, s);
  return go_pw<32, DV, NT>(a, s);
}


hipError_t launch_sweep_pw(const SweepArgs& a, hipStream_t s, hipEvent_t mid) {
  if (!sweep_pw_eligible(a.ell, a.d) || a.ell > 32) return hipErrorInvalidValue;
  const hipError_t e = a.d == 2 ? go_pw_ell<2, kPwNT>(a, s) : go_pw_ell<3, kPwNT>(a, s);
  if (e != hipSuccess) return e;
  if (mid && !g_recorder) (void)hipEventRecord(mid, s);
  return launch_sweep_tail(a, s);
}

hipError_t launch_sweep_mfma(const SweepArgs& a, int parts, hipStream_t s, hipEvent_t mid) {
  if (a.dpad <= 0 || (a.dpad & 31) || a.rows_per_split > 2048 || parts < 1 || parts > 3) return hipErrorInvalidValue;
  if (parts == 1) go_mfma_ell<1>(a, s);
  else if (parts == 2) go_mfma_ell<2>(a, s);
  else go_mfma_ell<3>(a, s);
  if (mid && !g_recorder) (void)hipEventRecord(mid, s);
  return launch_sweep_tail(a, s);
}

// ============================================================================
// Packing: centred points v = fl32(x - mu) rounded to `parts` bf16 pieces
// (hi = bf16(v); lo = bf16(v - hi) for two parts; mid = bf16(v - hi),
// lo = bf16(v - hi - mid) for three), rows zero-padded to dpad, and
// n = fl32(scale * ||x~||^2) with x~ = the sum of the pieces, in FP64.
// One thread per point.
// ============================================================================
__global__ void k_pack_points(const float* x, int np, int d, const float* mu, double scale, int dpad, int parts,
                              unsigned short* H, unsigned short* M, unsigned short* Lo, float* nrm) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  double s2 = 0.0;
  for (int k = 0; k < dpad; ++k) {
    unsigned short h = 0, m = 0, l = 0;
    if (k < d) {
      const float v = x[(size_t)p * d + k] - mu[k];
      h = bf16_rne(v);
      const float r1 = v - bf16_val(h);  // exact
      double xt = (double)bf16_val(h);
      if (parts == 2) {
        l = bf16_rne(r1);
        xt += (double)bf16_val(l);
      } else if (parts == 3) {
        m = bf16_rne(r1);
        const float r2 = r1 - bf16_val(m);  // exact
        l = bf16_rne(r2);
        xt += (double)bf16_val(m) + (double)bf16_val(l);
      }
      s2 += xt * xt;
    }
    H[(size_t)p * dpad + k] = h;
    if (parts == 3) M[(size_t)p * dpad + k] = m;
    if (parts >= 2) Lo[(size_t)p * dpad + k] = l;
  }
  nrm[p] = (float)(scale * s2);
}

hipError_t launch_pack_points(const float* x, int np, int d, const float* mu, double scale, int dpad, int parts,
                              unsigned short* H, unsigned short* M, unsigned short* Lo, float* nrm, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_points, dim3((np + 255) / 256), dim3(256), 0, s, x, np, d, mu, scale, dpad, parts, H, M,
                     Lo, nrm);
  return hipGetLastError();
}

// ============================================================================
// FP64 evaluation on the matrix-core cost: the same tiles of 64 rows x 256
// columns as the generic evaluation; each 16-row slice of C~ is built by
// the four waves (64 columns each) into LDS, then every thread runs the
// FP64 terms of its column.
// ============================================================================
template <int XP>
__global__ __launch_bounds__(256) void k_eval_mfma(SweepArgs G, const double* f, const double* g,
                                                   const double* a, const double* b, double eps, double* rowpart,
                                                   double* colpart, double* scal, int n, int m) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g4 = lane >> 4, c16 = lane & 15;
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int i0 = blockIdx.y * 64;
  const int jc = min(j, m - 1);
  const int dq = G.dpad >> 3;
  const int ks = G.dpad >> 5;
  const double inv = 1.0 / eps;
  const double gj = g[jc], bj = b[jc];
  const uint4* const pred[3] = {G.Hred, XP == 3 ? G.Mred : G.Lred, G.Lred};
  const uint4* const pout[3] = {G.Hout, XP == 3 ? G.Mout : G.Lout, G.Lout};
  __shared__ float sC[16][257];
  __shared__ double srow[WAVES][64];
  double cs = 0, cost = 0, mass = 0, ent = 0;
  for (int rt = 0; rt < 64; rt += 16) {
    const size_t ra = (size_t)min(i0 + rt + c16, n - 1) * dq + g4;
    const uint4* const pa[3] = {pred[0] + ra, pred[1] + ra, pred[2] + ra};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int cl = wave * 64 + 16 * t + c16;
      const int jt = min((int)blockIdx.x * 256 + cl, m - 1);
      const size_t rb = (size_t)jt * dq + g4;
      const uint4* const pb[3] = {pout[0] + rb, pout[1] + rb, pout[2] + rb};
      const f32x4 xy = cross_mem<XP>(pa, pb, ks);
      const float ny = G.Nout[jt];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float nx = G.Nred[min(i0 + rt + 4 * g4 + i, n - 1)];
        sC[4 * g4 + i][cl] = fmaf(G.m2cs, xy[i], nx + ny);
      }
    }
    __syncthreads();
    for (int r = 0; r < 16; ++r) {
      const int i = i0 + rt + r;
      double p = 0;
      if (i < n && j < m) {
        const double cij = (double)sC[r][threadIdx.x];
        const double t = (f[i] + gj - cij) * inv;
        p = a[i] * bj * exp(t);
        cs += p;
        cost += p * cij;
        mass += p;
        ent += p * t;
      }
      const double rs = wave_sum(p);
      if (lane == 0) srow[wave][rt + r] = rs;
    }
    __syncthreads();
  }
  if (threadIdx.x < 64) {
    const int i = i0 + threadIdx.x;
    if (i < n) rowpart[(size_t)blockIdx.x * n + i] = srow[0][threadIdx.x] + srow[1][threadIdx.x] +
                                                     srow[2][threadIdx.x] + srow[3][threadIdx.x];
  }
  if (j < m) colpart[(size_t)blockIdx.y * m + j] = cs;
  __shared__ double sbd[16];
  const double c1 = block_sum_d(cost, sbd);
  const double c2 = block_sum_d(mass, sbd);
  const double c3 = block_sum_d(ent, sbd);
  if (threadIdx.x == 0) {
    const size_t bid = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    scal[bid * 3 + 0] = c1;
    scal[bid * 3 + 1] = c2;
    scal[bid * 3 + 2] = c3;
  }
}

hipError_t launch_eval_mfma(const SweepArgs& geo, int parts, const double* f, const double* g, const double* a,
                            const double* b, double eps, double* rowpart, double* colpart, double* scal, int n,
                            int m, int* nrb, int* ncb, hipStream_t s) {
  if (geo.dpad <= 0 || (geo.dpad & 31) || parts < 1 || parts > 3) return hipErrorInvalidValue;
  dim3 grid((m + 255) / 256, (n + 63) / 64);
  *ncb = grid.x;
  *nrb = grid.y;
  if (parts == 1)
    hipLaunchKernelGGL((k_eval_mfma<1>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, rowpart, colpart, scal, n, m);
  else if (parts == 2)
    hipLaunchKernelGGL((k_eval_mfma<2>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, rowpart, colpart, scal, n, m);
  else
    hipLaunchKernelGGL((k_eval_mfma<3>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, rowpart, colpart, scal, n, m);
  return hipGetLastError();
}

// coupling on the matrix-core cost: 16 rows x 256 columns per workgroup
template <int XP>
__global__ __launch_bounds__(256) void k_coupling_mfma(SweepArgs G, const double* f, const double* g,
                                                       const double* a, const double* b, double eps, float* P,
                                                       int n, int m) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g4 = lane >> 4, c16 = lane & 15;
  const int dq = G.dpad >> 3, ks = G.dpad >> 5;
  const int i0 = blockIdx.y * 16;
  const size_t ra = (size_t)min(i0 + c16, n - 1) * dq + g4;
  const uint4* const pa[3] = {G.Hred + ra, (XP == 3 ? G.Mred : G.Lred) + ra, G.Lred + ra};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int j = (int)blockIdx.x * 256 + wave * 64 + 16 * t + c16;
    const int jc = min(j, m - 1);
    const size_t rb = (size_t)jc * dq + g4;
    const uint4* const pb[3] = {G.Hout + rb, (XP == 3 ? G.Mout : G.Lout) + rb, G.Lout + rb};
    const f32x4 xy = cross_mem<XP>(pa, pb, ks);
    const float ny = G.Nout[jc];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ii = i0 + 4 * g4 + i;
      if (ii < n && j < m) {
        const float cf = fmaf(G.m2cs, xy[i], G.Nred[ii] + ny);
        P[(size_t)ii * m + j] = (float)(a[ii] * b[j] * exp((f[ii] + g[j] - (double)cf) / eps));
      }
    }
  }
}

hipError_t launch_coupling_mfma(const SweepArgs& geo, int parts, const double* f, const double* g, const double* a,
                                const double* b, double eps, float* P, int n, int m, hipStream_t s) {
  if (geo.dpad <= 0 || (geo.dpad & 31) || parts < 1 || parts > 3) return hipErrorInvalidValue;
  dim3 grid((m + 255) / 256, (n + 15) / 16);
  if (parts == 1) hipLaunchKernelGGL((k_coupling_mfma<1>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, P, n, m);
  else if (parts == 2) hipLaunchKernelGGL((k_coupling_mfma<2>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, P, n, m);
  else hipLaunchKernelGGL((k_coupling_mfma<3>), grid, dim3(256), 0, s, geo, f, g, a, b, eps, P, n, m);
  return hipGetLastError();
}

}  // namespace sknr
