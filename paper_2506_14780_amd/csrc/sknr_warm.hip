// Small dense FP64 kernels of the spectral warm start (paper Sec. 4):
// block subspace iteration for the top eigenvectors of
//   M = diag(a)^-1 P diag(b)^-1 P^T,
// self-adjoint in L2(a), whose eigenvalues are rho_k^2 (the semi-dual
// Hessian at the optimum is -(1/eps) diag(a)(Id - M)).  The two O(nm k)
// products P^T V and P U run in the weighted c-transform sweeps; what is
// here works on n x k or m x k blocks (k <= 32) and k x k matrices:
// weighted Gram matrices, Cholesky orthonormalisation in L2(a) with the
// constant mode projected out, cyclic Jacobi for the Rayleigh-Ritz step,
// and the block rotations.
#include "sknr_internal.h"
#include "sknr_device.h"

#include <math.h>

namespace sknr {

// counter-based uniform(-1, 1) value number e of stream `seed` (splitmix64)
__device__ __forceinline__ float uniform_pm1(unsigned long long seed, unsigned long long e) {
  unsigned long long x = seed + 0x9E3779B97F4A7C15ull * (e + 1);
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (float)((double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0);
}

// sum over nblk (<= 32) partial blocks of entry e, loads issued together
__device__ __forceinline__ double sum_parts(const double* part, int nblk, int stride, int e) {
  double v[32];
#pragma unroll
  for (int b = 0; b < 32; ++b) v[b] = b < nblk ? part[(size_t)b * stride + e] : 0.0;
  double s = 0;
#pragma unroll
  for (int b = 0; b < 32; ++b) s += v[b];
  return s;
}

// out[e] = sum over blocks (in block order) of part[b * len + e]
__device__ __forceinline__ void sum_partials_body(const SumPartialsArgs& q, const int bx) {
  if (q.st && gate_closed(q.st, q.gate)) return;
  const int e = bx * blockDim.x + threadIdx.x;
  if (e >= q.len) return;
  double s = 0;
  for (int b0 = 0; b0 < q.nblk; b0 += 32) {
    const int nb = min(32, q.nblk - b0);
    s += sum_parts(q.part + (size_t)b0 * q.len, nb, q.len, e);
  }
  q.out[e] = s;
}
__global__ __launch_bounds__(256) void k_sum_partials(SumPartialsArgs q) { sum_partials_body(q, blockIdx.x); }
__global__ __launch_bounds__(256) void k_sum_partials_b(BatchTab T) {
  int bx, by;
  const int slot = batch_slot(T, blockIdx.x, &bx, &by);
  sum_partials_body(*static_cast<const SumPartialsArgs*>(T.args[slot]), bx);
}
hipError_t launch_sum_partials(const double* part, int nblk, int len, double* out, hipStream_t s, DevState* st,
                               int gate) {
  const SumPartialsArgs q{part, nblk, len, out, st, gate};
  const dim3 grid((len + 255) / 256);
  if (g_recorder) {
    record_launch((const void*)k_sum_partials_b, q, grid, 256, 0);
    return hipSuccess;
  }
  hipLaunchKernelGGL(k_sum_partials, grid, dim3(256), 0, s, q);
  return hipGetLastError();
}

// ----------------------------------------------------------------- Gram
// part[blk] = ( sum_i w_i Z_i Z_i^T  (k x k),  sum_i w_i Z_i  (k) ),
// w_i = wgt[i] or 1/wgt[i] (invert), over a contiguous block of rows.
// refill (nullable): bit l of *refill & refill_bits set -> column l of Z
// is first overwritten with fresh uniform(-1, 1) values of stream `seed`
// (zero columns that the orthonormalisation dropped get a new start).
template <int KP>
__global__ __launch_bounds__(256) void k_wgram(float* Z, const double* wgt, int invert, int n, double* part,
                                               int rows_per_blk, const unsigned* refill, unsigned refill_bits,
                                               unsigned long long seed) {
  const unsigned rmask = refill ? (*refill & refill_bits) : 0u;
  constexpr int NE = KP * KP;
  constexpr int PER = (NE + 255) / 256;
  __shared__ __align__(16) float tile[64][KP];
  __shared__ double wrow[64];
  double acc[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) acc[p] = 0;
  double sacc = 0;
  const int beg = blockIdx.x * rows_per_blk;
  const int end = min(beg + rows_per_blk, n);
  for (int t0 = beg; t0 < end; t0 += 64) {
    int nt = min(64, end - t0);
    __syncthreads();
    {
      // rows t0 .. t0+nt-1 of Z are one contiguous block (16-byte
      // aligned): all of a thread's float4 loads in flight at once; rows
      // past nt are zero; refilled columns get their random values (also
      // written back to Z)
      constexpr int T4 = 64 * KP / 4, U4 = (T4 + 255) / 256;
      float4* z4 = reinterpret_cast<float4*>(Z + (size_t)t0 * KP);
      const int valid4 = nt * KP / 4;
      float4 v[U4];
#pragma unroll
      for (int u = 0; u < U4; ++u) v[u] = z4[min((int)threadIdx.x + 256 * u, valid4 - 1)];
#pragma unroll
      for (int u = 0; u < U4; ++u) {
        const int i4 = threadIdx.x + 256 * u;
        if (i4 >= T4) continue;
        float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
        if (i4 < valid4) {
          t = v[u];
          const int l0 = (4 * i4) % KP;
          if ((rmask >> l0) & 0xFu) {
            const size_t e0 = (size_t)t0 * KP + 4 * (size_t)i4;
            if ((rmask >> l0) & 1u) t.x = uniform_pm1(seed, e0);
            if ((rmask >> (l0 + 1)) & 1u) t.y = uniform_pm1(seed, e0 + 1);
            if ((rmask >> (l0 + 2)) & 1u) t.z = uniform_pm1(seed, e0 + 2);
            if ((rmask >> (l0 + 3)) & 1u) t.w = uniform_pm1(seed, e0 + 3);
            z4[i4] = t;
          }
        }
        reinterpret_cast<float4*>(&tile[0][0])[i4] = t;
      }
    }
    if (threadIdx.x < 64) {
      int rr = threadIdx.x;
      double w = 0;
      if (rr < nt) w = invert ? 1.0 / wgt[t0 + rr] : wgt[t0 + rr];
      wrow[rr] = w;
    }
    __syncthreads();
    // all 64 rows of the tile (rows past nt are zero and add exact zeros),
    // eight at a time: the LDS reads of eight rows go out before the sums
    const int scol = (int)threadIdx.x < KP ? (int)threadIdx.x : 0;
    for (int r0 = 0; r0 < 64; r0 += 8) {
      double wv[8];
      float ta[8][PER], tb[8][PER], ts[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        wv[u] = wrow[r0 + u];
        ts[u] = tile[r0 + u][scol];
#pragma unroll
        for (int p = 0; p < PER; ++p) {
          const int e = min((int)threadIdx.x + 256 * p, NE - 1);
          ta[u][p] = tile[r0 + u][e / KP];
          tb[u][p] = tile[r0 + u][e % KP];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
          const int e = threadIdx.x + 256 * p;
          if (e < NE) acc[p] += wv[u] * (double)ta[u][p] * (double)tb[u][p];
        }
        if ((int)threadIdx.x < KP) sacc += wv[u] * (double)ts[u];
      }
    }
  }
  double* out = part + (size_t)blockIdx.x * (NE + KP);
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    int e = threadIdx.x + 256 * p;
    if (e < NE) out[e] = acc[p];
  }
  if ((int)threadIdx.x < KP) out[NE + threadIdx.x] = sacc;
}

// ------------------------------------------- orthonormalisation in L2(a)
// From the Gram partials of Z with weights a: s = Z^T a, B = Z^T D_a Z.
// Projecting out the constant (Z - 1 s^T, since sum a = 1) gives
// B' = B - s s^T; with B' = L L^T, V = (Z - 1 s^T) L^-T is orthonormal in
// L2(a) and orthogonal to the constants.  Writes R = L^-T (k x k), s.
// Rank revealing: a column whose pivot (its squared distance to the span
// of the columns before it) is at most 1e-8 of the largest diagonal entry
// of B' over the columns that were not just refilled (refill mask,
// nullable: fresh random columns are not products M V and would set the
// scale), or 1e-12 in absolute terms, carries no information that the FP32
// products Z = M V resolve (for Z = M V, pivots are ~rho^4, rounding noise
// ~1e-14): it is dropped, i.e. its column of V is exactly zero and no other
// column is orthogonalised against it, so the kept columns stay
// orthonormal.  (A ridge on the diagonal instead shrinks such columns and,
// after the Rayleigh-Ritz rotation, mixes the shrinkage into the good
// ones.)  *ok_out = 0 when every column is dropped.
// One wave, matrix in registers: lane i holds row i of B' and, step by
// step, of L (right-looking Cholesky; the steps unrolled, so every index is
// a constant; step k reads the pivot and column k of L from the lanes that
// hold them); then L goes to LDS and column j of L^-1 is formed by lane j
// with broadcast LDS reads of L.
template <int KP>
__global__ __launch_bounds__(64) void k_orth(const double* part, int nblk, double* R, double* s_out, int* ok_out,
                                             const unsigned* refill) {
  constexpr int NE = KP * KP;
  const int lane = threadIdx.x;
  const int row = lane < KP ? lane : KP - 1;
  __shared__ double Ls[KP][KP + 1];
  // the Gram sums (block order): row `row` of B, its transpose and s
  auto total = [&](int e) {
    if (nblk == 1) return part[e];
    double v = 0;
    for (int b0 = 0; b0 < nblk; b0 += 32) {
      double c = 0;
      for (int b = b0; b < min(nblk, b0 + 32); ++b) c += part[(size_t)b * (NE + KP) + e];
      v += c;
    }
    return v;
  };
  const double s_own = total(NE + row);
  double x[KP];
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    const double bij = total(row * KP + j), bji = total(j * KP + row);
    const double sj = total(NE + j);
    x[j] = 0.5 * (bij + bji) - s_own * sj;  // B' = sym(B) - s s^T
  }
  const unsigned fresh = refill ? *refill : 0u;
  double dgo = 0.0;
#pragma unroll
  for (int j = 0; j < KP; ++j)
    if (j == row) dgo = x[j];
  double bm = (lane < KP && !((fresh >> lane) & 1u)) ? dgo : 0.0;
  for (int o = 32; o > 0; o >>= 1) bm = fmax(bm, __shfl_xor(bm, o, 64));
  const double dcut = fmax(1e-8 * bm, 1e-12);
  // right-looking Cholesky: column k of L from the current B', then the
  // trailing update (rows i > k, columns k < j <= i; the other entries of a
  // lane's row are not used).  A dropped column gets L_kk = 1 and a zero
  // column below the diagonal (no trailing update).
  unsigned drop = 0u;
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const double d = lane_read_d(x[k], k);
    const bool dk = !(d > dcut);  // also NaN
    double lik;
    if (dk) {
      lik = row == k ? 1.0 : 0.0;
    } else {
      const double lk = sqrt(d);
      lik = row == k ? lk : x[k] / lk;
    }
    if (dk) drop |= 1u << k;
#pragma unroll
    for (int j = k + 1; j < KP; ++j) x[j] -= lik * lane_read_d(lik, j);
    x[k] = lik;
  }
  if (lane < KP) {
#pragma unroll
    for (int t = 0; t < KP; ++t) Ls[lane][t] = x[t];
  }
  __syncthreads();
  // L^-1, column j by lane j: x_r = (delta_rj - sum_{t<r} L_rt x_t) / L_rr
  if (lane < KP) {
    const int j = lane;
    double y[KP];
#pragma unroll
    for (int r = 0; r < KP; ++r) {
      double acc = (r == j) ? 1.0 : 0.0;
#pragma unroll
      for (int t = 0; t < r; ++t) acc -= Ls[r][t] * y[t];
      y[r] = acc / Ls[r][r];
    }
    // a dropped column r: row r of L^-1 is zero (V_r = 0); later rows do
    // not read y[r] (L_ir = 0 for i > r)
#pragma unroll
    for (int r = 0; r < KP; ++r)
      if ((drop >> r) & 1u) y[r] = 0.0;
#pragma unroll
    for (int t = 0; t < KP; ++t) R[j * KP + t] = y[t];  // R = L^-T
    s_out[j] = s_own;
  }
  if (lane == 0) *ok_out = __popc(drop) < KP ? 1 : 0;
}

// ------------------------------------------------------ Rayleigh-Ritz
// T = U^T diag(b)^-1 U from Gram partials (U = P^T V, V orthonormal in
// L2(a), so T = V^T D_a M V).  Cyclic Jacobi with a round-robin pairing:
// each step rotates k/2 disjoint index pairs at once.  With the pairs of a
// step, A <- J^T A J splits into independent 2x2 blocks (row pair r,
// column pair t), so one thread updates one block (and one row pair of the
// accumulated Q) per step: two barriers per step.  The sweeps stop when
// ||offdiag||_F^2 <= off2 ||diag||_F^2 (the eigenvalues are then exact to
// about off2 relative, the eigenvectors to about sqrt(off2)).  Then
// eigenpairs sorted descending: Q (k x k, columns = eigenvectors,
// row-major), lam (k).
// Zero rows of T (columns of V that the orthonormalisation dropped) stay
// untouched (their rotations are the identity); *zmask_out (nullable) gets
// bit p set when sorted position p holds such a column.
template <int KP>
__global__ __launch_bounds__(256) void k_jacobi(const double* part, int nblk, double* Qout, double* lam, int sweeps,
                                                int* sweeps_out, unsigned* zmask_out, double off2) {
  constexpr int NE = KP * KP;
  constexpr int NP = KP / 2;
  constexpr int NT = 256;
  __shared__ double A[KP][KP + 1];
  __shared__ double Q[KP][KP + 1];
  __shared__ double cs[NP][2];
  __shared__ int pr[NP][2];
  __shared__ double red[2][NT / 64];
  __shared__ int stop_s;
  __shared__ int zin[KP];
  const int tid = threadIdx.x;
  for (int e = tid; e < NE; e += NT) {
    A[e / KP][e % KP] = sum_parts(part, nblk, NE + KP, e);
    Q[e / KP][e % KP] = (e / KP == e % KP) ? 1.0 : 0.0;
  }
  __syncthreads();
  // T is a Gram matrix: T_kk == 0 exactly iff column k of U (and of V) is 0
  if (tid < KP) zin[tid] = A[tid][tid] == 0.0 ? 1 : 0;
  for (int e = tid; e < NE; e += NT) {
    const int i = e / KP, j = e % KP;
    if (i < j) {
      const double v = 0.5 * (A[i][j] + A[j][i]);
      A[i][j] = v;
      A[j][i] = v;
    }
  }
  __syncthreads();
  int sw = 0;
  for (sw = 0; sw < sweeps; ++sw) {
    double off = 0, dia = 0;
    for (int e = tid; e < NE; e += NT) {
      const double v = A[e / KP][e % KP];
      if (e / KP == e % KP) dia += v * v;
      else off += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o, 64);
      dia += __shfl_xor(dia, o, 64);
    }
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = off;
      red[1][tid >> 6] = dia;
    }
    __syncthreads();
    if (tid == 0) {
      double o2 = 0, d2 = 0;
      for (int w = 0; w < NT / 64; ++w) {
        o2 += red[0][w];
        d2 += red[1][w];
      }
      stop_s = o2 <= off2 * d2 ? 1 : 0;
    }
    __syncthreads();
    if (stop_s) break;
    for (int step = 0; step < KP - 1; ++step) {
      if (tid < NP) {
        const int r = tid;
        auto pos = [&](int i) { return i == 0 ? 0 : 1 + (i - 1 + step) % (KP - 1); };
        int p = pos(r), q = pos(KP - 1 - r);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        pr[r][0] = p;
        pr[r][1] = q;
        // rotation angle in FP32 (the quotient too: th only sets the angle;
        // an apq below FP32 range is no rotation, an overflow of th to inf
        // gives the identity); (c, s) normalised to FP64
        // accuracy (one Newton step on the FP32 reciprocal square root) so
        // that the accumulated Q stays orthogonal to FP64 rounding
        const double apq = A[p][q], dqp = A[q][q] - A[p][p];
        double c = 1.0, sn = 0.0;
        if (fabs(apq) > 1e-30 * (fabs(A[p][p]) + fabs(A[q][q])) && (float)apq != 0.0f) {
          const float th = (float)dqp / (2.0f * (float)apq);
          const float t = copysignf(1.0f, th) / (fabsf(th) + sqrtf(fmaf(th, th, 1.0f)));
          const double td = (double)t;
          const double x = fma(td, td, 1.0);
          double rn = (double)__frsqrt_rn((float)x);
          rn = rn * fma(-0.5 * x, rn * rn, 1.5);
          c = rn;
          sn = td * rn;
        }
        cs[r][0] = c;
        cs[r][1] = sn;
      }
      __syncthreads();
      // A <- J^T A J by 2x2 blocks; J acts on columns (p, q) as
      // (p, q) -> (c p - s q, s p + c q) and the same on rows
      for (int b = tid; b < NP * NP; b += NT) {
        const int r = b / NP, t = b % NP;
        const int p = pr[r][0], q = pr[r][1], u = pr[t][0], v = pr[t][1];
        const double cr = cs[r][0], sr = cs[r][1], ct = cs[t][0], st = cs[t][1];
        const double b00 = A[p][u], b01 = A[p][v], b10 = A[q][u], b11 = A[q][v];
        const double c00 = ct * b00 - st * b01, c01 = st * b00 + ct * b01;
        const double c10 = ct * b10 - st * b11, c11 = st * b10 + ct * b11;
        A[p][u] = cr * c00 - sr * c10;
        A[p][v] = cr * c01 - sr * c11;
        A[q][u] = sr * c00 + cr * c10;
        A[q][v] = sr * c01 + cr * c11;
      }
      // Q <- Q J: row i, column pair t
      for (int e = tid; e < KP * NP; e += NT) {
        const int i = e / NP, t = e % NP;
        const int u = pr[t][0], v = pr[t][1];
        const double ct = cs[t][0], st = cs[t][1];
        const double qiu = Q[i][u], qiv = Q[i][v];
        Q[i][u] = ct * qiu - st * qiv;
        Q[i][v] = st * qiu + ct * qiv;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (tid == 0 && sweeps_out) *sweeps_out = sw;
  // descending order: rank of each eigenvalue (ties by index), in parallel
  __shared__ int order[KP];
  if (tid < KP) {
    const int i = tid;
    const double li = A[i][i];
    int rank = 0;
    for (int j = 0; j < KP; ++j) {
      const double lj = A[j][j];
      rank += (lj > li) || (lj == li && j < i);
    }
    order[rank] = i;
  }
  __syncthreads();
  if (tid < KP) lam[tid] = A[order[tid]][order[tid]];
  if (tid == 0 && zmask_out) {
    unsigned msk = 0;
    for (int p = 0; p < KP; ++p)
      if (zin[order[p]]) msk |= 1u << p;
    *zmask_out = msk;
  }
  for (int e = tid; e < NE; e += NT) {
    const int r = e / KP, i = e % KP;
    Qout[r * KP + i] = Q[r][order[i]];
  }
}

// Rayleigh quotients in place of a Rayleigh-Ritz step: from the Gram
// partials of T (as k_jacobi), lam = the diagonal of T sorted descending,
// Q = identity (the basis is kept as it is), *zmask_out = the columns whose
// diagonal is exactly zero (columns the orthonormalisation dropped), in the
// basis' own column order.
template <int KP>
__global__ __launch_bounds__(64) void k_ritz_diag(const double* part, int nblk, double* Qout, double* lam,
                                                  int* sweeps_out, unsigned* zmask_out) {
  constexpr int NE = KP * KP;
  const int tid = threadIdx.x;
  __shared__ double dg[KP];
  if (tid < KP) dg[tid] = sum_parts(part, nblk, NE + KP, tid * KP + tid);
  __syncthreads();
  if (tid < KP) {
    const double li = dg[tid];
    int rank = 0;
    for (int j = 0; j < KP; ++j) rank += (dg[j] > li) || (dg[j] == li && j < tid);
    lam[rank] = li;
  }
  for (int e = tid; e < NE; e += 64) Qout[e] = (e / KP == e % KP) ? 1.0 : 0.0;
  if (tid == 0) {
    unsigned msk = 0;
    for (int k = 0; k < KP; ++k)
      if (dg[k] == 0.0) msk |= 1u << k;
    if (zmask_out) *zmask_out = msk;
    if (sweeps_out) *sweeps_out = 0;
  }
}

// out_i = ((Z_i - s) R) * rowscale_i   (k x k transform per row, FP64 math).
// KP/4 threads per row, each producing four adjacent outputs (one 16-byte
// store; a row's threads write its KP floats contiguously); every thread
// reads the whole row (L1 hits after the first) and sums over l in order.
template <int KP>
__global__ __launch_bounds__(256) void k_affine(const float* Z, const double* s, const double* R, const double* rs,
                                                int rs_invert, int n, float* out) {
  constexpr int TPR = KP / 4;  // threads per row
  __shared__ double Rs[KP][KP];
  __shared__ double ss[KP];
  for (int e = threadIdx.x; e < KP * KP; e += blockDim.x) Rs[e / KP][e % KP] = R[e];
  if ((int)threadIdx.x < KP) ss[threadIdx.x] = s ? s[threadIdx.x] : 0.0;
  __syncthreads();
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = gt / TPR, j0 = 4 * (gt % TPR);
  if (i >= n) return;
  const float4* zr = reinterpret_cast<const float4*>(Z + (size_t)i * KP);
  float zf[KP];
#pragma unroll
  for (int q = 0; q < KP / 4; ++q) {
    const float4 v = zr[q];
    zf[4 * q] = v.x;
    zf[4 * q + 1] = v.y;
    zf[4 * q + 2] = v.z;
    zf[4 * q + 3] = v.w;
  }
  double sc = 1.0;
  if (rs) sc = rs_invert ? 1.0 / rs[i] : rs[i];
  double v[4] = {0, 0, 0, 0};
#pragma unroll
  for (int l = 0; l < KP; ++l) {
    const double z = (double)zf[l] - ss[l];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] += z * Rs[l][j0 + c];
  }
  *reinterpret_cast<float4*>(out + (size_t)i * KP + j0) =
      make_float4((float)(v[0] * sc), (float)(v[1] * sc), (float)(v[2] * sc), (float)(v[3] * sc));
}

// counter-based uniform(-1, 1) start block for columns >= col0; clears the
// refill mask (nullable): the block has no zero columns
__global__ void k_random_block(float* Z, int n, int KP, int col0, unsigned long long seed, unsigned* zmask) {
  long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (zmask && e == 0) *zmask = 0u;
  if (e >= (long long)n * KP) return;
  int l = (int)(e % KP);
  if (l < col0) return;
  Z[e] = uniform_pm1(seed, (unsigned long long)e);
}

// out (n x ell FP64) = first ell columns of V (n x KP FP32); columns with
// bit l of `zero` set are written as zeros
__global__ void k_take_cols(const float* V, int KP, int n, int ell, unsigned zero, double* out) {
  long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= (long long)n * ell) return;
  int i = (int)(e / ell), l = (int)(e % ell);
  out[e] = ((zero >> l) & 1u) ? 0.0 : (double)V[(size_t)i * KP + l];
}

// out (n x ellp) = first ell columns of V (n x kp), zero padded
__global__ void k_repack(const float* V, int kp, int n, int ell, int ellp, float* out) {
  long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= (long long)n * ellp) return;
  int i = (int)(e / ellp), l = (int)(e % ellp);
  out[e] = l < ell ? V[(size_t)i * kp + l] : 0.f;
}

// ---------------------------------------------------------------- launchers
hipError_t launch_repack(const float* V, int kp, int n, int ell, int ellp, float* out, hipStream_t s) {
  long long cnt = (long long)n * ellp;
  hipLaunchKernelGGL(k_repack, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, V, kp, n, ell, ellp, out);
  return hipGetLastError();
}
hipError_t launch_wgram(int kp, float* Z, const double* w, int invert, int n, double* part, int nblk,
                        const unsigned* refill, unsigned refill_bits, uint64_t seed, hipStream_t s) {
  int rpb = (n + nblk - 1) / nblk;
  if ((uintptr_t)Z & 15) return hipErrorInvalidValue;  // float4 row loads
  unsigned long long sd = (unsigned long long)seed;
  if (kp == 8)
    hipLaunchKernelGGL((k_wgram<8>), dim3(nblk), dim3(256), 0, s, Z, w, invert, n, part, rpb, refill, refill_bits,
                       sd);
  else if (kp == 16)
    hipLaunchKernelGGL((k_wgram<16>), dim3(nblk), dim3(256), 0, s, Z, w, invert, n, part, rpb, refill, refill_bits,
                       sd);
  else
    hipLaunchKernelGGL((k_wgram<32>), dim3(nblk), dim3(256), 0, s, Z, w, invert, n, part, rpb, refill, refill_bits,
                       sd);
  return hipGetLastError();
}
hipError_t launch_orth(int kp, const double* part, int nblk, double* R, double* s_out, int* ok,
                       const unsigned* refill, hipStream_t s) {
  if (kp == 8) hipLaunchKernelGGL((k_orth<8>), dim3(1), dim3(64), 0, s, part, nblk, R, s_out, ok, refill);
  else if (kp == 16) hipLaunchKernelGGL((k_orth<16>), dim3(1), dim3(64), 0, s, part, nblk, R, s_out, ok, refill);
  else hipLaunchKernelGGL((k_orth<32>), dim3(1), dim3(64), 0, s, part, nblk, R, s_out, ok, refill);
  return hipGetLastError();
}
hipError_t launch_jacobi(int kp, const double* part, int nblk, double* Q, double* lam, int* sweeps_out,
                         unsigned* zmask_out, hipStream_t s, double off2) {
  if (kp == 8)
    hipLaunchKernelGGL((k_jacobi<8>), dim3(1), dim3(256), 0, s, part, nblk, Q, lam, 10, sweeps_out, zmask_out, off2);
  else if (kp == 16)
    hipLaunchKernelGGL((k_jacobi<16>), dim3(1), dim3(256), 0, s, part, nblk, Q, lam, 10, sweeps_out, zmask_out,
                       off2);
  else
    hipLaunchKernelGGL((k_jacobi<32>), dim3(1), dim3(256), 0, s, part, nblk, Q, lam, 10, sweeps_out, zmask_out,
                       off2);
  return hipGetLastError();
}
hipError_t launch_ritz_diag(int kp, const double* part, int nblk, double* Q, double* lam, int* sweeps_out,
                            unsigned* zmask_out, hipStream_t s) {
  if (kp == 8) hipLaunchKernelGGL((k_ritz_diag<8>), dim3(1), dim3(64), 0, s, part, nblk, Q, lam, sweeps_out, zmask_out);
  else if (kp == 16)
    hipLaunchKernelGGL((k_ritz_diag<16>), dim3(1), dim3(64), 0, s, part, nblk, Q, lam, sweeps_out, zmask_out);
  else hipLaunchKernelGGL((k_ritz_diag<32>), dim3(1), dim3(64), 0, s, part, nblk, Q, lam, sweeps_out, zmask_out);
  return hipGetLastError();
}
hipError_t launch_affine(int kp, const float* Z, const double* sv, const double* R, const double* rs, int rs_invert,
                         int n, float* out, hipStream_t s) {
  // rows of kp floats: 16-byte aligned (kp a multiple of 4, buffers from
  // 256-byte aligned carving)
  if (((uintptr_t)Z | (uintptr_t)out) & 15) return hipErrorInvalidValue;
  const long long thr = (long long)n * (kp / 4);
  const dim3 grid((unsigned)((thr + 255) / 256));
  if (kp == 8) hipLaunchKernelGGL((k_affine<8>), grid, dim3(256), 0, s, Z, sv, R, rs, rs_invert, n, out);
  else if (kp == 16) hipLaunchKernelGGL((k_affine<16>), grid, dim3(256), 0, s, Z, sv, R, rs, rs_invert, n, out);
  else hipLaunchKernelGGL((k_affine<32>), grid, dim3(256), 0, s, Z, sv, R, rs, rs_invert, n, out);
  return hipGetLastError();
}
hipError_t launch_random_block(int kp, float* Z, int n, int col0, uint64_t seed, unsigned* zmask, hipStream_t s) {
  long long cnt = (long long)n * kp;
  hipLaunchKernelGGL(k_random_block, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, Z, n, kp, col0,
                     (unsigned long long)seed, zmask);
  return hipGetLastError();
}
hipError_t launch_take_cols(const float* V, int kp, int n, int ell, unsigned zero, double* out, hipStream_t s) {
  long long cnt = (long long)n * ell;
  hipLaunchKernelGGL(k_take_cols, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, V, kp, n, ell, zero, out);
  return hipGetLastError();
}

}  // namespace sknr
