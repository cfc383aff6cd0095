// Internal declarations shared by the HIP kernels and the host engine of
// libsknr.  Not part of the public ABI (include/sknr.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sknr {

// ----------------------------------------------------------------- state
// Small device-resident control block of one solver instance.  Kernels of
// one iteration read the gating flags at entry and a one-workgroup
// finishing kernel after each sweep updates the scalars, so a whole chunk
// of iterations can be queued (or captured in a graph) without host round
// trips.
enum DotSlot { DOT_F = 0, DOT_G = 1, DOT_GT = 2, DOT_FSK = 3, DOT_FP = 4, DOT_GP = 5, DOT_TMP = 6, NDOT = 8 };
enum MaxSlot { MA_F = 0, MA_G = 1, MA_GT = 2, MA_FSK = 3, MA_FP = 4, MA_GP = 5, MA_G2 = 6, NMA = 8 };

struct DevState {
  int done;             // stage converged: every gated kernel returns at entry
  int npass;            // column sweeps executed in this stage
  int armed;            // the next checking sweep may declare convergence
  int accept;           // last Newton candidate accepted
  int chol_ok;          // last projected system factorised
  int newton_tried;
  int newton_accepted;
  int gsel;             // SK ping-pong: which g buffer holds g_k at convergence
  double err;           // last L1 marginal error estimate (output side)
  double err_aux;       // sum |mdiff| of the last row sweep (row marginal of P~)
  double dots[NDOT];    // <U, w> of hat potentials (FP64 sums)
  float maxabs[NMA];    // max |U.hi| of hat potentials (for the sweep offset L)
  // constants of the current eps, read by the kernels (so that a captured
  // chunk of iterations serves every stage)
  double eps;           // eps
  double tol;           // L1 marginal tolerance
  float K;              // log2(e)/eps
  float inv_eps;        // 1/eps
  float2 eps_df;        // eps as double-float
  float2 eln2_df;       // eps*ln2 as double-float
  int nr_iters;         // iterations of the last iterative Newton solve (0 for the direct one)
  unsigned tail_ctr;    // arrivals of a sweep's tail workgroups (zero between kernels)
  double err1;          // error of the stage's first checking sweep (npass == 1)
  int pad[2];
};

// Solver of the l x l Newton system (k_nr_solve): Gauss-Jordan with
// Cholesky's pivot test, or the iterative alternatives of Sec. 4
// (disadvantages paragraph): Jacobi-preconditioned conjugate gradients, or
// Newton-Schulz iterative inversion.
enum NrSolverKind { NR_DIRECT = 0, NR_CG = 1, NR_NEWTON_SCHULZ = 2 };
struct NrSolver {
  int kind = NR_DIRECT;
  int max_iter = 0;   // iterative solvers: step cap
  double rtol = 0;    // iterative solvers: stopping threshold
};

// gating bits: a kernel returns immediately unless all requested hold
enum Gate { G_NOT_DONE = 1, G_CHOL_OK = 2, G_ACCEPT = 4, G_NOT_ACCEPT = 8 };
// sweep flags
enum SweepFlag {
  F_CHECK = 1,       // compare the L1 error with tol and set done (col sweeps)
  F_COUNT = 2,       // count this sweep in npass
  F_GSEL = 4,        // record gsel_val into state->gsel when setting done
  F_ACCEPT_DQ = 16,   // after this sweep decide the Newton acceptance test from Q(f') - Q(f)
                      // formed without cancellation (W_CAND sweep)
  F_EXACT_ALL = 32    // single-read pass: take every row through the max-shift path and
                      // every column through the merge's exact per-column path (the
                      // paths for rows and columns that the fixed shifts cannot resolve)
};
// W_CAND: the sweep runs on f with the single basis column expm1((f' - f)/eps)
// and writes the candidate T_c(f') = T_c(f) - eps log1p(w) instead of W
// W_SCALE_MASS: W_o = sum_r pi_ro V_r (the softmax average times the
// output's marginal w_o (1 + ratio_m1) against Uold)
enum WMode { W_NONE = 0, W_SCALE_WEIGHT = 1, W_SCALE_RATIO = 2, W_CAND = 3, W_SCALE_MASS = 4 };

// ---------------------------------------------------------- sweep arguments
// One c-transform sweep: out_o = eps*lw_o - eps*log sum_r exp((Uin_r - C_ro)/eps)
// over the "reduce" side r, for every "output" o, with hat potentials
// U = potential + eps*log(weight) kept as (hi, lo) float pairs.
struct SweepArgs {
  int n_out, n_red;
  // cost: STORED element (r, o) is C[r*ldc + o] for the streaming kernel
  // (output = columns of C) and C[o*ldc + r] for the row kernel.
  const float* C;
  long long ldc;
  // point clouds (SQEUCLID): reduce-side points and output-side points
  const float* Pred;
  const float* Pout;
  int d;
  float cscale;
  double cscale64;       // cost_scale as given (FP64 exact-cost evaluation)
  // matrix-core cost (SQEUCLID with a bf16 cross term): centred points as
  // bf16 rows of dpad entries (dpad a multiple of 32; hi, and lo for the
  // split form, else null) and fl32(cost_scale * ||x~||^2) per point
  const uint4* Hred;
  const uint4* Mred;     // mid part (three-part split only)
  const uint4* Lred;
  const float* Nred;
  const uint4* Hout;
  const uint4* Mout;
  const uint4* Lout;
  const float* Nout;
  int dpad;
  float m2cs;            // -2 * cost_scale (FP32)
  float cmax;            // upper bound of |C| (sweep offset L)
  // potentials
  const float2* Uin;     // reduce-side hat potential (n_red)
  int ma_in;             // maxabs slot of Uin
  // optional scalars of the Newton update f' = f + V c, left as per-block
  // partials by its kernel; the finish kernel stores, before its decisions,
  // dots[aux_dot_slot] = sum of aux_blkdot (<f', a>), maxabs[aux_ma_slot] =
  // max of aux_blkmax, and uses sum of aux_blkddot (<f' - f, a>) in the
  // acceptance test F_ACCEPT_DQ (sums in block order)
  const float* aux_blkmax;
  const double* aux_blkdot;
  const double* aux_blkddot;
  int aux_nblk;
  int aux_dot_slot;
  int aux_ma_slot;
  const float2* lw_out;  // output-side log weights (double-float)
  const float* w_out;    // output-side weights FP32
  const double* w_out64; // output-side weights FP64 (dots)
  const float2* Uold;    // previous output-side hat potential (error / ratio) or null
  float2* Uout;          // new output-side hat potential
  float* mdiff;          // optional: w_o * expm1((Uold_o - Uout_o)/eps)
  int dot_slot;          // slot for <Uout, w_out> (or -1)
  int ma_out;            // slot for max|Uout.hi| (or -1)
  // weighted averages (l-wide): Wout_o = scale_o * sum_r P_ro V_r / sum_r P_ro
  int ell;               // 0 or the compile-time width
  const float* Vred;     // n_red x ell, row-major
  float* Wout;           // n_out x ell
  int wmode;
  // split-K bookkeeping
  int nsplit;
  int rows_per_split;
  float* part;           // [nsplit][3+ell][n_out]
  double* blk_err;       // per output-block partial scalars
  double* blk_dot;
  float* blk_max;
  int nblk;              // number of output blocks (scalar partials)
  DevState* st;
  int gate;
  int flags;
  int gsel_val;
  // fused single-read SK pass over a stored cost (k_sk_fused_stored): the
  // row transform of Uold is written to Uin (the reduce side of this
  // column sweep), with these reduce-side log weights and FP64 weights; the
  // column part's offset L bounds |Uin| by maxabs[ma_in] + lpad_c +
  // eps * lpad_e (a bound known before Uin exists; merge and kernel form it
  // in the same order)
  const float2* lw_red;
  const double* w_red64;
  float lpad_c;
  float lpad_e;
  // fused pass: per reduce-side row, log2 of its largest term relative to
  // L - f^ + eps log w (read for the row's shift, then rewritten)
  float* rowmax;
};

// offset L of a sweep: 3 (cmax + bound on |Uin|), with the fused pass's
// bound when lpad_c / lpad_e are set
__host__ __device__ inline float sweep_offset_bound(const SweepArgs& A, float maxabs_in, double eps) {
  const float b = maxabs_in + A.lpad_c + (float)eps * A.lpad_e;
  return 3.f * (A.cmax + b);
}

// ------------------------------------------------- batched execution
// A tile table spreads one launch over many requests: tile b of the launch
// belongs to slot s with off[s] <= b < off[s + 1], and within the slot it is
// block (x, y) = ((b - off[s]) % gx[s], (b - off[s]) / gx[s]) of that
// request's own grid; args[s] points at the slot's argument block (device
// memory).  Every kernel of an iteration has such a batched twin, and runs
// the same body with the request's own arguments and block coordinates,
// so a request computes exactly what its own launch would.
struct BatchTab {
  const void* const* args;  // [nslot] device pointers to argument blocks
  const int* off;           // [nslot + 1] prefix sums of the slots' tiles
  const int* gx;            // [nslot] grid width of each slot
  int nslot;
};
__device__ __forceinline__ int batch_slot(const BatchTab& T, int b, int* bx, int* by) {
  int lo = 0, hi = T.nslot - 1;
  while (lo < hi) {  // the last slot whose offset is <= b
    const int mid = (lo + hi + 1) >> 1;
    if (T.off[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const int local = b - T.off[lo];
  const int g = T.gx[lo];
  *bx = local % g;
  *by = local / g;
  return lo;
}

// While a recorder is installed on the calling thread, the launchers of the
// iteration kernels append a record (batched twin, argument block, grid,
// block, LDS bytes) instead of launching.
constexpr int kMaxArgBytes = 512;
struct LaunchRec {
  const void* bfunc;  // __global__ void(BatchTab)
  int arg_bytes;
  int gx, gy, block;
  unsigned lds;
  alignas(16) unsigned char args[kMaxArgBytes];
};
struct Recorder {
  LaunchRec* recs = nullptr;  // caller-owned storage
  int cap = 0;
  int n = 0;
  bool unsupported = false;   // a launch without a batched twin was requested
};
extern thread_local Recorder* g_recorder;
template <typename T>
inline void record_launch(const void* bfunc, const T& a, dim3 grid, int block, size_t lds) {
  static_assert(sizeof(T) <= kMaxArgBytes, "argument block too large");
  Recorder* r = g_recorder;
  if (r->n >= r->cap) {
    r->unsupported = true;
    return;
  }
  LaunchRec& L = r->recs[r->n++];
  L.bfunc = bfunc;
  L.arg_bytes = (int)sizeof(T);
  L.gx = (int)grid.x;
  L.gy = (int)grid.y;
  L.block = block;
  L.lds = (unsigned)lds;
  __builtin_memcpy(L.args, &a, sizeof(T));
}

// argument blocks of the kernels without SweepArgs
struct NrAssembleArgs {
  const float* V;
  const float* mdiff;
  const double* a;
  int n;
  const float* W;
  const double* b;
  int m;
  double* part;
  int nrow_blk, rows_per_blk;
  DevState* st;
  int gate;
};
struct NrSolveArgs {
  const double* part;
  int nblk, ell_real;
  float* coef32;
  double* coef64;
  double* Gout;
  double* gout;
  DevState* st;
  int gate, solver, max_it;
  double rtol;
};
struct NrApplyArgs {
  const float2* F;
  const float* V;
  const float* coef;
  const double* a;
  float2* Fp;
  int n;
  double* blk;
  float* blkmax;
  double* blkd;
  float* E1;
  DevState* st;
  int gate;
};
struct SumPartialsArgs {
  const double* part;
  int nblk, len;
  double* out;
  DevState* st;  // gating (nullable: always runs)
  int gate;
};
struct SelectArgs {
  const float2* Fp;
  const float2* Fsk;
  float2* F;
  int n;
  const float2* Gp;
  const float2* Gt;
  float2* G;
  int m;
  DevState* st;
  int gate;
};

// ----------------------------------------------------------- launchers
// All launchers enqueue on `stream` and return hipSuccess or the launch error.
// vec: the stored cost allows float4 access along the output axis
// mid (optional): an event recorded right after the main sweep kernel
hipError_t launch_sweep_stream(const SweepArgs& a, int cost_kind, bool vec, hipStream_t stream,
                               hipEvent_t mid = nullptr);
hipError_t launch_sweep_rows(const SweepArgs& a, hipStream_t stream, hipEvent_t mid = nullptr);
// X (cols x rows, row pitch rows) = the transpose of the stored cost C (rows x cols, row pitch ldc)
hipError_t launch_transpose_cost(const float* C, long long ldc, int rows, int cols, float* X, hipStream_t stream);
// One SK iteration over a stored cost with a single read of C: rows of C
// (side X, not transposed) produce f = T_r(Uold) into Uin, and each row's
// terms join the column log-sum-exp of T_c(f); merge and finish as a
// streaming column sweep.  Eligible: fused_stored_ok().
bool fused_stored_ok(int n_red, int n_out, long long ldc, const float* C);
int fused_stored_splits(int n_red, int n_out);
size_t fused_stored_lds(int n_out, int rows_per_split);  // dynamic LDS bytes of the pass
hipError_t launch_sk_fused_stored(const SweepArgs& a, hipStream_t stream, hipEvent_t mid = nullptr);
size_t sweep_part_floats(int n_out, int n_red, int ell, int cost_kind, int d, bool vec, int* nsplit, int* rps,
                         int* nblk, bool stream_kernel);
// split merge + scalar finishing kernels of a streaming sweep
hipError_t launch_sweep_tail(const SweepArgs& a, hipStream_t stream);
// input checks of prepare(): per weight vector and per point coordinate the
// min, max, sum, bad-entry count and (weights) sum v log v, 5 doubles each,
// (2 + 2d) records (x == nullptr: the two weight records only)
hipError_t launch_input_stats(const double* a, int n, const double* b, int m, const float* x, const float* y, int d,
                              double* out, hipStream_t s);
hipError_t launch_weight_prep(const double* w, int n, float* w32, double* l64, float2* ldf, hipStream_t s);
// The split merge (k_sweep_merge) gives each output merge_lanes(ell)
// lanes, each merging a contiguous range of splits; a workgroup of
// 64 * merge_lanes(ell) threads covers 64 outputs: merge_blocks(n_out)
// blocks, which is also the number of block scalars of the sweep.
// (4 for every width: more lanes per output, in larger workgroups or in
// more of them, measured slower on the 4096^2 sweeps)
constexpr int merge_lanes(int ell) { return ell < 0 ? 0 : 4; }
inline int merge_blocks(int n_out, int ell) {
  (void)ell;
  return (n_out + 63) / 64;
}

// matrix-core cost (cost kinds 2, 3, 4 = bf16 cross term with 1, 2, 3 bf16
// parts per coordinate; `parts` below)
// weighted sweeps of FP32 point costs, 2 <= d <= 3: the matrix-core lane
// layout with the cost on the VALU and W = P^T V on FP32 matrix cores
bool sweep_pw_eligible(int ell, int d);
hipError_t launch_sweep_pw(const SweepArgs& a, hipStream_t s, hipEvent_t mid);
hipError_t launch_sweep_mfma(const SweepArgs& a, int parts, hipStream_t stream, hipEvent_t mid);
size_t mfma_part_floats(int n_out, int n_red, int ell, int parts, int* nsplit, int* rps, int* nblk);
hipError_t launch_pack_points(const float* x, int np, int d, const float* mu, double scale, int dpad, int parts,
                              unsigned short* H, unsigned short* M, unsigned short* Lo, float* nrm, hipStream_t s);
hipError_t launch_eval_mfma(const SweepArgs& geo, int parts, const double* f, const double* g, const double* a,
                            const double* b, double eps, double* rowpart, double* colpart, double* scal, int n,
                            int m, int* nrb, int* ncb, hipStream_t s);
hipError_t launch_coupling_mfma(const SweepArgs& geo, int parts, const double* f, const double* g, const double* a,
                                const double* b, double eps, float* P, int n, int m, hipStream_t s);

// conversions between FP64 paper-convention potentials and hat double-floats
hipError_t launch_to_hat(const double* f, const double* logw, double eps, float2* U, int n,
                         DevState* st, int ma_slot, const double* w, int dot_slot, double* scratch, hipStream_t s);
hipError_t launch_from_hat(const float2* U, const double* logw, double eps, double* f, int n, hipStream_t s);
hipError_t launch_rebase(float2* U, const float2* lw, float2 deps_df, int n, DevState* st, int ma, hipStream_t s);
// *st = z on the device; keep: carry over maxabs[MA_F], maxabs[MA_G],
// dots[DOT_F], dots[DOT_G] from the current state
hipError_t launch_state_reset(DevState* st, const DevState& z, bool keep, hipStream_t s);
hipError_t launch_copy_state_slot(DevState* st, int dst_dot, int src_dot, int dst_ma, int src_ma, hipStream_t s);

// Newton step pieces (FP64 small system)
hipError_t launch_nr_assemble(int ell, const float* V, const float* rdiff, const double* a, int n,
                              const float* W, const double* b, int m, double* part, int nrow_blk,
                              int ncol_blk, DevState* st, int gate, hipStream_t s);
hipError_t launch_nr_solve(int ell, const double* part, int nblk, float* coef32,
                           double* coef64, double* Gout, double* gout, DevState* st, int gate,
                           hipStream_t s, const NrSolver& solver = NrSolver());
// Newton update f' = f + V c (hat form), per-block partials blk = <f', a>,
// blkmax = max|f'.hi|, blkd = <f' - f, a>, and E1[i * 8] = expm1((f' - f)_i /
// eps) (columns 1..7 zero: the single basis column of the W_CAND sweep)
hipError_t launch_nr_apply(int ell, const float2* F, const float* V, const float* coef, const double* a,
                           float2* Fp, int n, double* blk, float* blkmax, double* blkd, float* E1, DevState* st,
                           int gate, hipStream_t s);
// gradients of W_eps: pack columns c0 .. c0+dc of an np x d point array into
// an np x ellp block (zero-padded); grad[p, c0+k] = two_s ((w_p + mdiff_p)
// P[p, c0+k] - Wsum[p, k]); gradw[p] = pot[p] - eps (w_p + mdiff_p) / w_p
hipError_t launch_pack_cols(const float* P, int np, int d, int c0, int dc, int ellp, float* out, hipStream_t s);
hipError_t launch_grad_points(const float* P, int np, int d, int c0, int dc, const double* w, const float* mdiff,
                              const float* Wsum, int ellp, double two_s, double* grad, hipStream_t s);
hipError_t launch_grad_weights(const double* pot, const double* w, const float* mdiff, int np, double eps,
                               double* grad, hipStream_t s);
hipError_t launch_select(const float2* Fp, const float2* Fsk, float2* F, int n, const float2* Gp,
                         const float2* Gt, float2* G, int m, DevState* st, int gate, hipStream_t s);

// FP64 evaluation (final check).  cost_kind: a sweep kind (0 stored, 1 FP32
// points) or kEvalExact, the FP64 squared distance of the FP32 points.
constexpr int kEvalExact = 5;
hipError_t launch_eval(const SweepArgs& geo, int cost_kind, const double* f, const double* g,
                       const double* a, const double* b, double eps, double* rowpart, double* colpart,
                       double* scal, int n, int m, int* nrb, int* ncb, hipStream_t s);
hipError_t launch_eval_finish(const double* rowpart, const double* colpart, const double* scal,
                              const double* a, const double* b, int n, int m, int nrb, int ncb,
                              double* out8, double* blk, hipStream_t s);

// spectral warm start: block subspace iteration helpers (k = kp <= 32)
// refill (nullable device mask, restricted to refill_bits): columns of Z to
// overwrite with fresh random values first; zmask_out (nullable): sorted
// positions whose Ritz vector is a dropped (zero) column
hipError_t launch_wgram(int kp, float* Z, const double* w, int invert, int n, double* part, int nblk,
                        const unsigned* refill, unsigned refill_bits, uint64_t seed, hipStream_t s);
hipError_t launch_orth(int kp, const double* part, int nblk, double* R, double* s_out, int* ok,
                       const unsigned* refill, hipStream_t s);
// off2: the sweeps stop once the squared off-diagonal Frobenius norm is at
// most off2 times the squared diagonal one
hipError_t launch_jacobi(int kp, const double* part, int nblk, double* Q, double* lam, int* sweeps_out,
                         unsigned* zmask_out, hipStream_t s, double off2 = 1e-14);
// the diagonal of T sorted as Ritz-value estimates, Q = I (see k_ritz_diag)
hipError_t launch_ritz_diag(int kp, const double* part, int nblk, double* Q, double* lam, int* sweeps_out,
                            unsigned* zmask_out, hipStream_t s);
hipError_t launch_affine(int kp, const float* Z, const double* sv, const double* R, const double* rs, int rs_invert,
                         int n, float* out, hipStream_t s);
hipError_t launch_random_block(int kp, float* Z, int n, int col0, uint64_t seed, unsigned* zmask, hipStream_t s);
hipError_t launch_take_cols(const float* V, int kp, int n, int ell, unsigned zero, double* out, hipStream_t s);
hipError_t launch_sum_partials(const double* part, int nblk, int len, double* out, hipStream_t s,
                               DevState* st = nullptr, int gate = 0);
// length of the Newton system partials of k_nr_assemble: the upper triangle
// of G (l (l + 1) / 2 entries) then grad (l), for the padded width l
inline int nr_part_len(int ell) {
  const int e = ell <= 8 ? 8 : (ell <= 16 ? 16 : 32);
  return e * (e + 1) / 2 + e;
}
hipError_t launch_repack(const float* V, int kp, int n, int ell, int ellp, float* out, hipStream_t s);
hipError_t launch_f32_to_f64(const float* src, double* dst, long long count, hipStream_t s);
hipError_t launch_f64_to_f32(const double* src, float* dst, long long count, hipStream_t s);
hipError_t launch_coupling(const SweepArgs& geo, int cost_kind, const double* f, const double* g,
                           const double* a, const double* b, double eps, float* P, int n, int m,
                           hipStream_t s);
hipError_t launch_dot64(const double* x, const double* w, int n, double* out, hipStream_t s);
hipError_t launch_shift64(double* x, int n, const double* dots, double sign, hipStream_t s);
hipError_t launch_cost_max(int cost_kind, const float* C, long long ldc, int n, int m, const float* x,
                           const float* y, int d, float* out2, hipStream_t s);

}  // namespace sknr
