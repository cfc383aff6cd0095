// Host engine and C ABI of libsknr (see include/sknr.h).
//
// The engine keeps one problem resident on the device in a fixed
// orientation: side X (size n) carries the semi-dual potential f and is the
// smaller side (Sec. 2: the semi-dual is taken over the smaller space);
// side Y (size m) carries g.  Each Sinkhorn iteration is a fixed sequence of
// kernel launches gated by a small device state block, so chunks of
// iterations run without host round trips; the host polls the state once
// per chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "sknr_host.h"

using namespace sknr;

namespace sknr_host {

thread_local std::string g_last_error;

struct WS {
  // transposed copy of a stored cost (or null): the sweeps whose outputs
  // run along the stored rows use the streaming kernel on it (row pitch ldx)
  const float* X;
  long long ldx;
  float2 *F, *Fsk, *Fp, *G[2], *Gt, *Gp;
  float* mdiff;
  float* mdiffY;  // column-side marginal differences (gradients)
  float *V, *W;
  int ellp;
  float* part;
  double *blk_err, *blk_dot;
  float* blk_max;
  double* ap_dot;   // per-block partials of the Newton update F' (the candidate's finish reduces them)
  float* ap_max;
  double* ap_ddot;  // per-block <F' - F, a>
  float* E1;        // n x 8: expm1((F' - F)/eps) in column 0, the candidate sweep's basis
  double* nrpart;
  double* nrsum;  // partials summed: one (k*k + k) block
  int nr_rows_blk, nr_cols_blk;
  float* coef32;
  double* coef64;
  DevState* st;
  float *wX32, *wY32;
  double *lX64, *lY64;
  float2 *lXdf, *lYdf;
  double *fX64, *gY64;
  double* scratch;
  double *evrow, *evcol, *evscal, *evout, *evblk;
  double* Gout;
  double* gout;
  // warm start (block width up to 32)
  float *Vw, *Zw, *Uw, *Utw;
  double *Rw, *sw, *Qw, *lamw;
  int* okw;
  bool have_Vw;
  // packed points of the matrix-core cost (engine orientation)
  unsigned short *HX, *MX, *LX, *HY, *MY, *LY;
  float *NX, *NY, *mu;
  // sweep geometry
  int ns_c, rps_c, nb_c, ns_r, rps_r, nb_r, ns_cw, rps_cw, nb_cw;
  // fused single-read SK pass (stored cost): per-split row scalars, and
  // max|log a| + max|log b| for the bound on |f^|
  double* fz_dot;
  float* fz_max;
  float* fz_rowmax;  // per row of the reduce side: log2 of its largest term (the pass's shift)
  float lwb;
  unsigned char* argbank;  // argument blocks of a recorded batch unit
};

// split partials of the fused single-read pass (floats), 0 when not eligible
size_t fused_part_floats(const Prepared& P) {
  if (P.kind != SKNR_COST_STORED || P.ctrans || !fused_stored_ok(P.n, P.m, P.ldc, P.C)) return 0;
  return (size_t)fused_stored_splits(P.n, P.m) * 2 * (size_t)P.m;  // one double per column and split
}

int ell_pad(int ell) { return ell <= 0 ? 0 : (ell <= 8 ? 8 : (ell <= 16 ? 16 : 32)); }

// cost kind of the sweep kernels: 0 stored, 1 points FP32, 2 bf16, 3 bf16
// hi/lo split, 4 bf16 hi/mid/lo split (bf16 parts = kind - 1)
int sweep_kind(const Prepared& P) { return P.kind == SKNR_COST_STORED ? 0 : P.xmode; }

bool col_is_stream(const Prepared& P) { return P.kind == SKNR_COST_SQEUCLID || !P.ctrans; }
bool row_is_stream(const Prepared& P) { return P.kind == SKNR_COST_SQEUCLID || P.ctrans; }
// float4 access along the output axis of a streaming sweep over a stored cost
bool stream_vec(const Prepared& P, int n_out) {
  return P.kind == SKNR_COST_STORED && n_out % 4 == 0 && P.ldc % 4 == 0 && ((uintptr_t)P.C % 16) == 0;
}

// a value rounded to the nearest bf16 (round to nearest even), as FP32
float bf16_round(double v) {
  float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  u &= 0xFFFF0000u;
  std::memcpy(&f, &u, 4);
  return f;
}

// --------------------------------------------------------------- prepare
Prepared prepare(const sknr_problem* pr, hipStream_t s, void* scratch) {
  REQUIRE(pr, "problem is NULL");
  REQUIRE(pr->n >= 1 && pr->m >= 1, "n and m must be >= 1");
  REQUIRE(pr->n <= (1 << 26) && pr->m <= (1 << 26), "n, m too large");
  REQUIRE(pr->kind == SKNR_COST_STORED || pr->kind == SKNR_COST_SQEUCLID, "unknown cost kind");
  REQUIRE(pr->a && pr->b, "weights a, b are required");
  REQUIRE(!pr->on_host, "host-resident inputs (on_host) are not accepted by this entry point");
  REQUIRE(scratch, "internal: no scratch for prepare");
  Prepared P;
  P.n0 = (int)pr->n;
  P.m0 = (int)pr->m;
  P.kind = pr->kind;
  P.transposed = pr->n > pr->m;
  P.n = P.transposed ? P.m0 : P.n0;
  P.m = P.transposed ? P.n0 : P.m0;
  P.C = pr->C;
  P.ldc = pr->ldc;
  P.ctrans = P.transposed;
  P.d = pr->d;
  P.cscale = 1.0f;
  P.cscale64 = 1.0;
  const bool pts = pr->kind == SKNR_COST_SQEUCLID;
  if (!pts) {
    REQUIRE(pr->C, "stored cost C is NULL");
    REQUIRE(pr->ldc >= pr->m, "ldc < m");
    P.X = P.Y = nullptr;
  } else {
    REQUIRE(pr->x && pr->y, "points x, y are required");
    REQUIRE(pr->d >= 1 && pr->d <= 1024, "d must be in [1, 1024]");
    double sc = pr->cost_scale == 0.0 ? 1.0 : pr->cost_scale;
    REQUIRE(sc > 0 && std::isfinite(sc), "cost_scale must be positive");
    P.cscale = (float)sc;
    P.cscale64 = sc;
    REQUIRE(pr->xterm >= SKNR_XTERM_AUTO && pr->xterm <= SKNR_XTERM_BF16X6, "unknown xterm");
    P.xmode = pr->xterm == SKNR_XTERM_AUTO ? (pr->d >= 16 ? SKNR_XTERM_BF16X6 : SKNR_XTERM_FP32) : pr->xterm;
    if (P.xmode >= SKNR_XTERM_BF16) P.dpad = (pr->d + 31) & ~31;
    P.X = P.transposed ? pr->y : pr->x;
    P.Y = P.transposed ? pr->x : pr->y;
  }
  // input statistics on the device (and the stored cost's bound), one read
  const int d = pts ? pr->d : 0;
  const int nrec = 2 + 2 * d;
  double* dst = static_cast<double*>(scratch);
  float* dmax = reinterpret_cast<float*>(static_cast<char*>(scratch) + kPrepBytes - 256);
  HIPCHK(launch_input_stats(pr->a, P.n0, pr->b, P.m0, pts ? pr->x : nullptr, pts ? pr->y : nullptr, pts ? d : 1,
                            dst, s));
  if (!pts) HIPCHK(launch_cost_max(0, pr->C, pr->ldc, P.n0, P.m0, nullptr, nullptr, 0, dmax, s));
  std::vector<double> h(5 * (size_t)nrec);
  float hm = 0;
  HIPCHK(hipMemcpyAsync(h.data(), dst, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
  if (!pts) HIPCHK(hipMemcpyAsync(&hm, dmax, sizeof(float), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  auto check_w = [&](int r, int len, const char* name) {
    const double* o = &h[5 * (size_t)r];
    if (o[3] != 0) throw Err{SKNR_EINVAL, std::string(name) + " has a non-positive or non-finite entry"};
    if (std::fabs(o[2] - 1.0) > 1e-9 * std::max<double>(1.0, (double)len))
      throw Err{SKNR_EINVAL, std::string(name) + " does not sum to 1"};
  };
  check_w(0, P.n0, "a");
  check_w(1, P.m0, "b");
  const double* sa = &h[0];
  const double* sb = &h[5];
  P.wX = P.transposed ? pr->b : pr->a;
  P.wY = P.transposed ? pr->a : pr->b;
  const double* sX = P.transposed ? sb : sa;
  const double* sY = P.transposed ? sa : sb;
  P.wminX = sX[0];
  P.wmaxX = sX[1];
  P.entX = sX[4];
  P.wminY = sY[0];
  P.wmaxY = sY[1];
  P.entY = sY[4];
  if (!pts) {
    REQUIRE(std::isfinite(hm), "cost has non-finite entries");
    P.cmax = hm;
  } else {
    double bound = 0;
    P.mu.assign(d, 0.f);
    for (int k = 0; k < d; ++k) {
      const double* ox = &h[5 * (size_t)(2 + k)];
      const double* oy = &h[5 * (size_t)(2 + d + k)];
      REQUIRE(ox[3] == 0, "x has non-finite entries");
      REQUIRE(oy[3] == 0, "y has non-finite entries");
      P.mu[k] = bf16_round((ox[2] + oy[2]) / (double)(P.n0 + P.m0));
      const double span = std::max(std::fabs(ox[1] - oy[0]), std::fabs(oy[1] - ox[0]));
      bound += span * span;
    }
    P.cmax = (float)(bound * P.cscale * 1.001 + 1e-30);
  }
  return P;
}

// --------------------------------------------------------------- workspace
size_t ws_bytes(const Prepared& P, int ellp, int* geo) {
  int n = P.n, m = P.m;
  size_t b = 0;
  auto add = [&](size_t x) { b += (x + 255) & ~size_t(255); };
  int ns, rps, nb, nbmax = 0;
  size_t pmax = 0;
  // weighted sweeps run l-wide (Newton) or up to 32-wide (warm start)
  const int ellw = ellp > 0 ? 32 : 0;
  // T_c (output Y), with and without weights
  // (a stored cost may also run its rows-orientation sweeps on the
  // streaming kernel over a transposed copy: both geometries are sized)
  const bool both = P.kind == SKNR_COST_STORED;
  for (int e : {0, ellp > 0 ? 8 : 0, ellp > 0 ? 16 : 0, ellp, ellw}) {
    for (int k = 0; k < (both ? 2 : 1); ++k) {
      const bool cs = k ? !col_is_stream(P) : col_is_stream(P), rs = k ? !row_is_stream(P) : row_is_stream(P);
      size_t p = sweep_part_floats(m, n, e, sweep_kind(P), P.d, stream_vec(P, m), &ns, &rps, &nb, cs);
      pmax = std::max(pmax, p);
      nbmax = std::max(nbmax, nb);
      p = sweep_part_floats(n, m, e, sweep_kind(P), P.d, stream_vec(P, n), &ns, &rps, &nb, rs);
      pmax = std::max(pmax, p);
      nbmax = std::max(nbmax, nb);
    }
  }
  nbmax = std::max(nbmax, (std::max(n, m) + 255) / 256 + 1);
  pmax = std::max(pmax, fused_part_floats(P));
  add(sizeof(double) * 256);
  add(sizeof(float) * 256);
  add(sizeof(float) * n);
  add((size_t)kMaxUnitLaunches * kMaxArgBytes);
  add(sizeof(float2) * n * 3);
  add(sizeof(float2) * m);
  add(sizeof(float2) * m);
  add(sizeof(float2) * m * 2);
  add(sizeof(float) * n);
  add(sizeof(float) * m);
  add(sizeof(float) * (size_t)n * std::max(ellp, 1));
  add(sizeof(float) * (size_t)m * std::max(ellp, 1));
  add(sizeof(float) * pmax + 16);
  add(sizeof(double) * ((n + 255) / 256));
  add(sizeof(float) * ((n + 255) / 256));
  add(sizeof(double) * ((n + 255) / 256));
  add(sizeof(float) * 8 * (size_t)n);
  add(sizeof(double) * nbmax * 2);
  add(sizeof(float) * nbmax);
  int nrb = 64, ncb = 64;
  add(sizeof(double) * (nrb + ncb) * (size_t)(std::max(ellw, 1) * std::max(ellw, 1) + std::max(ellw, 1)));
  add(sizeof(double) * (size_t)(std::max(ellw, 1) * std::max(ellw, 1) + std::max(ellw, 1)));
  add(sizeof(float) * 32);
  add(sizeof(double) * 32);
  add(sizeof(DevState));
  add(sizeof(float) * (n + m));
  add(sizeof(double) * (n + m));
  add(sizeof(float2) * (n + m));
  add(sizeof(double) * (n + m));
  add(sizeof(double) * ((std::max(n, m) + 255) / 256 + 64));
  int ecb = (P.m0 + 255) / 256, erb = (P.n0 + 63) / 64;
  add(sizeof(double) * (size_t)ecb * P.n0);
  add(sizeof(double) * (size_t)erb * P.m0);
  add(sizeof(double) * (size_t)ecb * erb * 3);
  add(sizeof(double) * 16);
  add(sizeof(double) * ((P.n0 + 255) / 256 + (P.m0 + 255) / 256 + 2));
  add(sizeof(double) * 32 * 32);
  add(sizeof(double) * 32);
  if (ellp > 0) {
    add(sizeof(float) * (size_t)n * 32 * 2);
    add(sizeof(float) * (size_t)m * 32 * 2);
    add(sizeof(double) * 32 * 32 * 2 + sizeof(double) * 96 + 64);
  }
  if (P.xmode >= SKNR_XTERM_BF16) {
    const int parts = P.xmode - 1;
    add(sizeof(unsigned short) * (size_t)n * P.dpad * parts);
    add(sizeof(unsigned short) * (size_t)m * P.dpad * parts);
    add(sizeof(float) * n);
    add(sizeof(float) * m);
    add(sizeof(float) * P.d);
  }
  if (geo) *geo = nbmax;
  return b + 4096;
}

WS make_ws(Lane* c, const Prepared& P, int ellp, hipStream_t s) {
  ++c->ws_gen;
  size_t need = ws_bytes(P, ellp, nullptr);
  if (need > c->arena.cap) {
    if (c->arena_external) throw Err{SKNR_EINTERNAL, "workspace exceeds the reserved block"};
    HIPCHK(hipStreamSynchronize(s));
    c->drop_graphs();  // captured kernels point into the old arena
    if (c->arena.base) HIPCHK(hipFree(c->arena.base));
    c->arena.base = nullptr;
    c->arena.cap = 0;
    size_t cap = need + need / 4;
    hipError_t e = hipMalloc((void**)&c->arena.base, cap);
    if (e != hipSuccess) throw Err{SKNR_ENOMEM, "device allocation of the workspace failed"};
    c->arena.cap = cap;
    HIPCHK(hipMemsetAsync(c->arena.base, 0, cap, s));
  }
  Arena& A = c->arena;
  A.reset();
  int n = P.n, m = P.m;
  WS w{};
  w.ellp = ellp;
  w.F = (float2*)A.take(sizeof(float2) * n);
  w.Fsk = (float2*)A.take(sizeof(float2) * n);
  w.Fp = (float2*)A.take(sizeof(float2) * n);
  w.G[0] = (float2*)A.take(sizeof(float2) * m);
  w.G[1] = (float2*)A.take(sizeof(float2) * m);
  w.Gt = (float2*)A.take(sizeof(float2) * m);
  w.Gp = (float2*)A.take(sizeof(float2) * m);
  w.mdiff = (float*)A.take(sizeof(float) * n);
  w.mdiffY = (float*)A.take(sizeof(float) * m);
  w.V = (float*)A.take(sizeof(float) * (size_t)n * std::max(ellp, 1));
  w.W = (float*)A.take(sizeof(float) * (size_t)m * std::max(ellp, 1));
  int ns, rps, nb, nbmax = 0;
  size_t pmax = 0;
  const int ellw = ellp > 0 ? 32 : 0;
  for (int e : {0, ellp > 0 ? 8 : 0, ellp > 0 ? 16 : 0, ellp, ellw}) {
    pmax = std::max(pmax, sweep_part_floats(m, n, e, sweep_kind(P), P.d, stream_vec(P, m), &ns, &rps, &nb,
                                            col_is_stream(P)));
    nbmax = std::max(nbmax, nb);
    pmax = std::max(pmax, sweep_part_floats(n, m, e, sweep_kind(P), P.d, stream_vec(P, n), &ns, &rps, &nb,
                                            row_is_stream(P)));
    nbmax = std::max(nbmax, nb);
  }
  nbmax = std::max(nbmax, (std::max(n, m) + 255) / 256 + 1);
  pmax = std::max(pmax, fused_part_floats(P));
  w.fz_dot = (double*)A.take(sizeof(double) * 256);
  w.fz_max = (float*)A.take(sizeof(float) * 256);
  w.fz_rowmax = (float*)A.take(sizeof(float) * n);
  w.argbank = (unsigned char*)A.take((size_t)kMaxUnitLaunches * kMaxArgBytes);
  w.part = (float*)A.take(sizeof(float) * pmax + 16);
  w.blk_err = (double*)A.take(sizeof(double) * nbmax);
  w.blk_dot = (double*)A.take(sizeof(double) * nbmax);
  w.blk_max = (float*)A.take(sizeof(float) * nbmax);
  w.ap_dot = (double*)A.take(sizeof(double) * ((n + 255) / 256));
  w.ap_max = (float*)A.take(sizeof(float) * ((n + 255) / 256));
  w.ap_ddot = (double*)A.take(sizeof(double) * ((n + 255) / 256));
  w.E1 = (float*)A.take(sizeof(float) * 8 * (size_t)n);
  // Newton partial blocks: at most 64 row + 64 column blocks
  w.nr_rows_blk = std::min(64, std::max(1, (n + 63) / 64));
  w.nr_cols_blk = std::min(64, std::max(1, (m + 63) / 64));
  int e1 = std::max(ellw, 1);
  w.nrpart = (double*)A.take(sizeof(double) * (128) * (size_t)(e1 * e1 + e1));
  w.nrsum = (double*)A.take(sizeof(double) * (size_t)(e1 * e1 + e1));
  w.coef32 = (float*)A.take(sizeof(float) * 32);
  w.coef64 = (double*)A.take(sizeof(double) * 32);
  w.st = (DevState*)A.take(sizeof(DevState));
  w.wX32 = (float*)A.take(sizeof(float) * n);
  w.wY32 = (float*)A.take(sizeof(float) * m);
  w.lX64 = (double*)A.take(sizeof(double) * n);
  w.lY64 = (double*)A.take(sizeof(double) * m);
  w.lXdf = (float2*)A.take(sizeof(float2) * n);
  w.lYdf = (float2*)A.take(sizeof(float2) * m);
  w.fX64 = (double*)A.take(sizeof(double) * n);
  w.gY64 = (double*)A.take(sizeof(double) * m);
  w.scratch = (double*)A.take(sizeof(double) * ((std::max(n, m) + 255) / 256 + 64));
  int ecb = (P.m0 + 255) / 256, erb = (P.n0 + 63) / 64;
  w.evrow = (double*)A.take(sizeof(double) * (size_t)ecb * P.n0);
  w.evcol = (double*)A.take(sizeof(double) * (size_t)erb * P.m0);
  w.evscal = (double*)A.take(sizeof(double) * (size_t)ecb * erb * 3);
  w.evout = (double*)A.take(sizeof(double) * 16);
  w.evblk = (double*)A.take(sizeof(double) * ((P.n0 + 255) / 256 + (P.m0 + 255) / 256 + 2));
  w.Gout = (double*)A.take(sizeof(double) * 32 * 32);
  w.gout = (double*)A.take(sizeof(double) * 32);
  w.have_Vw = false;
  if (ellp > 0) {
    w.Vw = (float*)A.take(sizeof(float) * (size_t)n * 32);
    w.Zw = (float*)A.take(sizeof(float) * (size_t)n * 32);
    w.Uw = (float*)A.take(sizeof(float) * (size_t)m * 32);
    w.Utw = (float*)A.take(sizeof(float) * (size_t)m * 32);
    w.Rw = (double*)A.take(sizeof(double) * 32 * 32);
    w.Qw = (double*)A.take(sizeof(double) * 32 * 32);
    w.sw = (double*)A.take(sizeof(double) * 32);
    w.lamw = (double*)A.take(sizeof(double) * 64);  // this iteration's Ritz values, then the first's
    w.okw = (int*)A.take(64);
  }
  w.HX = w.MX = w.LX = w.HY = w.MY = w.LY = nullptr;
  w.NX = w.NY = w.mu = nullptr;
  if (P.xmode >= SKNR_XTERM_BF16) {
    const int parts = P.xmode - 1;
    auto pk = [&](int np) { return (unsigned short*)A.take(sizeof(unsigned short) * (size_t)np * P.dpad); };
    w.HX = pk(n);
    w.HY = pk(m);
    if (parts == 3) {
      w.MX = pk(n);
      w.MY = pk(m);
    }
    if (parts >= 2) {
      w.LX = pk(n);
      w.LY = pk(m);
    }
    w.NX = (float*)A.take(sizeof(float) * n);
    w.NY = (float*)A.take(sizeof(float) * m);
    w.mu = (float*)A.take(sizeof(float) * P.d);
    HIPCHK(hipMemcpyAsync(w.mu, P.mu.data(), sizeof(float) * P.d, hipMemcpyHostToDevice, s));
    HIPCHK(launch_pack_points(P.X, n, P.d, w.mu, P.cscale64, P.dpad, parts, w.HX, w.MX, w.LX, w.NX, s));
    HIPCHK(launch_pack_points(P.Y, m, P.d, w.mu, P.cscale64, P.dpad, parts, w.HY, w.MY, w.LY, w.NY, s));
  }
  // weights: FP32 copies, FP64 logs and their double-float splits (device)
  HIPCHK(launch_weight_prep(P.wX, n, w.wX32, w.lX64, w.lXdf, s));
  HIPCHK(launch_weight_prep(P.wY, m, w.wY32, w.lY64, w.lYdf, s));
  // max |log w| per side (log is monotone: at the smallest or largest weight)
  w.lwb = (float)(std::max(std::fabs(std::log(P.wminX)), std::fabs(std::log(P.wmaxX))) +
                  std::max(std::fabs(std::log(P.wminY)), std::fabs(std::log(P.wmaxY))));
  // a large stored cost used with weighted sweeps (SK-NR, warm start): a
  // transposed copy, so that the sweeps along its rows stream (the rows
  // kernel re-reads the l-wide basis for every output row).  Lanes on a
  // lent block (serving) keep the rows kernel, so a served request on a
  // stored cost above 2^24 elements can differ from its solo run in the
  // last bits (both within the sweeps' accuracy)
  w.X = nullptr;
  w.ldx = 0;
  const char* nox = getenv("SKNR_NO_XCOST");
  if (P.kind == SKNR_COST_STORED && ellp > 0 && !c->arena_external && (size_t)n * m >= ((size_t)1 << 24) &&
      !(nox && nox[0] == '1')) {
    const int rows = P.ctrans ? m : n, cols = P.ctrans ? n : m;
    const size_t bytes = sizeof(float) * (size_t)rows * cols;
    if (bytes > c->xcost_cap) {
      HIPCHK(hipStreamSynchronize(s));
      c->drop_graphs();  // captured sweeps may point at the old copy
      if (c->xcost) HIPCHK(hipFree(c->xcost));
      c->xcost = nullptr;
      c->xcost_cap = 0;
      if (hipMalloc((void**)&c->xcost, bytes) == hipSuccess) c->xcost_cap = bytes;
      else (void)hipGetLastError();  // no copy: the rows kernel serves
    }
    if (c->xcost) {
      HIPCHK(launch_transpose_cost(P.C, P.ldc, rows, cols, c->xcost, s));
      w.X = c->xcost;
      w.ldx = rows;
    }
  }
  HIPCHK(hipStreamSynchronize(s));  // host vectors go out of scope
  return w;
}

// ------------------------------------------------------------------ engine
struct Engine {
  Lane* c;
  const Prepared& P;
  WS& w;
  hipStream_t s;
  double eps = 1.0;
  double tol = 1e-6;
  NrSolver nrs;  // solver of the l x l Newton system

  Engine(Lane* c_, const Prepared& P_, WS& w_, hipStream_t s_) : c(c_), P(P_), w(w_), s(s_) {}

  void fill_common(SweepArgs& a) const {
    a.C = P.C;
    a.ldc = P.ldc;
    a.d = P.d;
    a.cscale = P.cscale;
    a.cmax = P.cmax;
    a.dpad = P.dpad;
    a.m2cs = -2.f * P.cscale;
    a.part = w.part;
    a.blk_err = w.blk_err;
    a.blk_dot = w.blk_dot;
    a.blk_max = w.blk_max;
    a.st = w.st;
  }

  void launch_sweep(const SweepArgs& a, bool stream_kernel, bool vec, int ell) {
    hipEvent_t e0 = nullptr, em = nullptr, e1 = nullptr;
    if (c->profile) {
      e0 = c->get_event();
      em = c->get_event();
      e1 = c->get_event();
      HIPCHK(hipEventRecord(e0, s));
    }
    if (stream_kernel) HIPCHK(launch_sweep_stream(a, sweep_kind(P), vec, s, em));
    else HIPCHK(launch_sweep_rows(a, s, em));
    if (c->profile) {
      HIPCHK(hipEventRecord(e1, s));
      char nm[96];
      static const char* kinds[5] = {"stored", "points", "points_bf16", "points_bf16x3", "points_bf16x6"};
      std::snprintf(nm, sizeof nm, "%s_%s%s_l%d", stream_kernel ? "sweep_stream" : "sweep_rows",
                    kinds[sweep_kind(P)], (sweep_kind(P) == 1 && P.d > 8) ? "_gen" : "",
                    ell <= 0 ? 0 : ell_pad(ell));
      const double units = (double)a.n_out * (double)a.n_red;
      // whole sweep (main kernel + merge/finish) and the main kernel alone
      c->pending.push_back(Pending{c->kind_of(nm), e0, e1, units});
      c->pending.push_back(Pending{c->kind_of(std::string(nm) + ":main"), nullptr, em, units});
    }
  }

  // g_out = T_c(U_in) on side Y (eq. foc_g), hat form
  float* col_mdiff = nullptr;  // optional column-side w_o expm1((Uold_o - Uout_o)/eps)

  void sweep_col(const float2* Fin, int ma_in, const float2* Gold, float2* Gout, int dot_slot, int ma_out, int ell,
                 const float* Vred, float* Wout, int wmode, int gate, int flags, int gsel_val = 0) {
    SweepArgs a{};
    fill_common(a);
    a.n_out = P.m;
    a.n_red = P.n;
    a.Pred = P.X;
    a.Pout = P.Y;
    a.Hred = (const uint4*)w.HX;
    a.Mred = (const uint4*)w.MX;
    a.Lred = (const uint4*)w.LX;
    a.Nred = w.NX;
    a.Hout = (const uint4*)w.HY;
    a.Mout = (const uint4*)w.MY;
    a.Lout = (const uint4*)w.LY;
    a.Nout = w.NY;
    a.Uin = Fin;
    a.ma_in = ma_in;
    if (wmode == W_CAND) {
      // the candidate of a Newton step: the update's scalars arrive as its
      // block partials
      a.aux_blkmax = w.ap_max;
      a.aux_blkdot = w.ap_dot;
      a.aux_blkddot = w.ap_ddot;
      a.aux_nblk = (P.n + 255) / 256;
      a.aux_dot_slot = DOT_FP;
      a.aux_ma_slot = MA_FP;
    }
    a.lw_out = w.lYdf;
    a.w_out = w.wY32;
    a.w_out64 = P.wY;
    a.Uold = Gold;
    a.Uout = Gout;
    a.mdiff = col_mdiff;
    a.dot_slot = dot_slot;
    a.ma_out = ma_out;
    a.ell = ell;
    a.Vred = Vred;
    a.Wout = Wout;
    a.wmode = wmode;
    a.gate = gate;
    a.flags = flags;
    a.gsel_val = gsel_val;
    bool st = col_is_stream(P);
    bool vec = stream_vec(P, a.n_out);
    use_transposed(a, st, vec);
    sweep_part_floats(a.n_out, a.n_red, ell, sweep_kind(P), P.d, vec, &a.nsplit, &a.rows_per_split, &a.nblk, st);
    launch_sweep(a, st, vec, ell);
  }

  // f_out = T_r(U_in) on side X (eq. foc_f)
  void sweep_row(const float2* Gin, int ma_in, const float2* Fold, float2* Fout, float* mdiff, int dot_slot,
                 int ma_out, int ell, const float* Vred, float* Wout, int wmode, int gate, int flags) {
    SweepArgs a{};
    fill_common(a);
    a.n_out = P.n;
    a.n_red = P.m;
    a.Pred = P.Y;
    a.Pout = P.X;
    a.Hred = (const uint4*)w.HY;
    a.Mred = (const uint4*)w.MY;
    a.Lred = (const uint4*)w.LY;
    a.Nred = w.NY;
    a.Hout = (const uint4*)w.HX;
    a.Mout = (const uint4*)w.MX;
    a.Lout = (const uint4*)w.LX;
    a.Nout = w.NX;
    a.Uin = Gin;
    a.ma_in = ma_in;
    a.lw_out = w.lXdf;
    a.w_out = w.wX32;
    a.w_out64 = P.wX;
    a.Uold = Fold;
    a.Uout = Fout;
    a.mdiff = mdiff;
    a.dot_slot = dot_slot;
    a.ma_out = ma_out;
    a.ell = ell;
    a.Vred = Vred;
    a.Wout = Wout;
    a.wmode = wmode;
    a.gate = gate;
    a.flags = flags;
    bool st = row_is_stream(P);
    bool vec = stream_vec(P, a.n_out);
    use_transposed(a, st, vec);
    sweep_part_floats(a.n_out, a.n_red, ell, sweep_kind(P), P.d, vec, &a.nsplit, &a.rows_per_split, &a.nblk, st);
    launch_sweep(a, st, vec, ell);
  }
  // a sweep whose outputs run along the stored rows streams over the
  // transposed copy when there is one (element (r, o) = X[r ldx + o])
  void use_transposed(SweepArgs& a, bool& st, bool& vec) const {
    if (st || !w.X) return;
    a.C = w.X;
    a.ldc = w.ldx;
    st = true;
    vec = a.n_out % 4 == 0 && w.ldx % 4 == 0;
  }

  void set_consts(DevState& z) const {
    z.eps = eps;
    z.tol = tol;
    z.K = (float)(1.4426950408889634 / eps);
    z.inv_eps = (float)(1.0 / eps);
    z.eps_df = split_df(eps);
    z.eln2_df = split_df(eps * 0.6931471805599453);
  }
  // fresh state for the current eps, written by a kernel (no host wait)
  void init_state() {
    DevState z{};
    set_consts(z);
    HIPCHK(launch_state_reset(w.st, z, false, s));
  }
  void check_cancel() const {
    if (c->cancel && c->cancel->load(std::memory_order_relaxed)) throw Err{SKNR_ECANCELED, "request cancelled"};
  }
  DevState read_state() {
    HIPCHK(hipMemcpyAsync(c->st_host, w.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (c->profile) c->drain();
    DevState r;
    std::memcpy(&r, c->st_host, sizeof(DevState));
    return r;
  }

  // load FP64 potentials (engine orientation) into hat form
  void load_f(const double* f /*nullable*/) {
    HIPCHK(launch_to_hat(f, w.lX64, eps, w.F, P.n, w.st, MA_F, P.wX, DOT_F, w.scratch, s));
  }
  void load_g(const double* g, float2* dst, int ma, int dot) {
    HIPCHK(launch_to_hat(g, w.lY64, eps, dst, P.m, w.st, ma, P.wY, dot, w.scratch, s));
  }
  // initial potentials at the current eps (engine orientation): f0 when
  // given; else, from g0, f = T_r(g0) (eq. foc_f) with g0 kept as the
  // previous g; else zero
  void start(const double* f0, const double* g0) {
    if (f0 || !g0) {
      load_f(f0);
      load_g(nullptr, w.G[0], MA_G, DOT_G);
      return;
    }
    load_g(g0, w.G[0], MA_G, DOT_G);
    sweep_row(w.G[0], MA_G, nullptr, w.F, nullptr, DOT_F, MA_F, 0, nullptr, nullptr, W_NONE, 0, 0);
  }
  bool have_basis = false;  // w.V holds the basis of an SK-NR stage

  // ---- Newton pieces for one iteration (after Gt, Fsk, mdiff, W exist)
  void newton(int ell, int gate_base) {
    HIPCHK(launch_nr_assemble(ell, w.V, w.mdiff, P.wX, P.n, w.W, P.wY, P.m, w.nrpart, w.nr_rows_blk, w.nr_cols_blk,
                              w.st, gate_base, s));
    HIPCHK(launch_sum_partials(w.nrpart, w.nr_rows_blk + w.nr_cols_blk, nr_part_len(ell), w.nrsum, s, w.st,
                               gate_base));
    HIPCHK(launch_nr_solve(ell, w.nrsum, 1, w.coef32, w.coef64, w.Gout, w.gout, w.st, gate_base, s, nrs));
    HIPCHK(launch_nr_apply(ell, w.F, w.V, w.coef32, P.wX, w.Fp, P.n, w.ap_dot, w.ap_max, w.ap_ddot, w.E1, w.st,
                           gate_base | G_CHOL_OK, s));
  }

  // T_c(F') and the acceptance test of the Newton step: a sweep on F whose
  // basis is the single column expm1((F' - F)/eps), giving T_c(F') =
  // T_c(F) - eps log1p(w) and Q(F') - Q(F) without cancellation
  void candidate(int gate) {
    sweep_col(w.F, MA_F, nullptr, w.Gp, DOT_GP, MA_GP, 8, w.E1, nullptr, W_CAND, gate, F_ACCEPT_DQ);
  }

  // Fused single-read SK pass over a stored cost: f = T_r(G[p]) into F and
  // G[1-p] = T_c(f), testing the pair (f, G[p]) (Sec. 2, eq. SK_iterations)
  bool fused = false;  // plain SK stages use the fused pass (set by the solve)
  bool fused_eligible() const {
    if (P.kind != SKNR_COST_STORED || P.ctrans || !fused_stored_ok(P.n, P.m, P.ldc, P.C)) return false;
    const char* off = getenv("SKNR_NO_FUSED");
    if (off && off[0] == '1') return false;
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return false;
    const int ns = fused_stored_splits(P.n, P.m);
    return (size_t)lds >= fused_stored_lds(P.m, (P.n + ns - 1) / ns);
  }
  void sk_fused(int p) {
    SweepArgs a{};
    fill_common(a);
    a.n_out = P.m;
    a.n_red = P.n;
    a.Uin = w.F;
    a.ma_in = MA_G;
    a.lw_red = w.lXdf;
    a.w_red64 = P.wX;
    a.lpad_c = P.cmax;
    a.lpad_e = w.lwb * 1.01f;
    a.aux_blkdot = w.fz_dot;
    a.aux_blkmax = w.fz_max;
    a.rowmax = w.fz_rowmax;
    a.aux_blkddot = nullptr;
    a.aux_dot_slot = DOT_F;
    a.aux_ma_slot = MA_F;
    a.lw_out = w.lYdf;
    a.w_out = w.wY32;
    a.w_out64 = P.wY;
    a.Uold = w.G[p];
    a.Uout = w.G[1 - p];
    a.mdiff = nullptr;
    a.dot_slot = DOT_G;
    a.ma_out = MA_G;
    a.ell = 0;
    a.wmode = W_NONE;
    a.nsplit = fused_stored_splits(P.n, P.m);
    a.rows_per_split = (P.n + a.nsplit - 1) / a.nsplit;
    a.aux_nblk = a.nsplit;
    a.nblk = merge_blocks(P.m, 0);
    a.gate = G_NOT_DONE;
    a.flags = F_CHECK | F_COUNT | F_GSEL;
    const char* all = getenv("SKNR_FUSED_EXACT_ALL");
    if (all && all[0] == '1') a.flags |= F_EXACT_ALL;
    a.gsel_val = p;
    hipEvent_t e0 = nullptr, em = nullptr, e1 = nullptr;
    if (c->profile) {
      e0 = c->get_event();
      em = c->get_event();
      e1 = c->get_event();
      HIPCHK(hipEventRecord(e0, s));
    }
    HIPCHK(launch_sk_fused_stored(a, s, em));
    if (c->profile) {
      HIPCHK(hipEventRecord(e1, s));
      const double units = (double)P.n * (double)P.m;
      c->pending.push_back(Pending{c->kind_of("sk_fused_stored"), e0, e1, units});
      c->pending.push_back(Pending{c->kind_of("sk_fused_stored:main"), nullptr, em, units});
    }
  }
  // Iterations until the next convergence poll.  A fixed check_every is
  // kept.  Otherwise: the iterations that a geometric decay of the error, at
  // the rate seen since the previous poll, needs to reach the stage's
  // threshold (rounded up to one of a few graph sizes), so that a stage
  // usually ends after two or three polls with few gated iterations; with
  // no rate yet, the chunk doubles up to chunk_max.
  static int next_chunk(int chunk, int chunk_max, int check_every, const DevState& st, double* err_prev,
                        int* np_prev) {
    // the first poll measures the rate from the stage's first check
    if (*err_prev < 0 && st.npass > 1 && st.err1 > 0) {
      *err_prev = st.err1;
      *np_prev = 1;
    }
    int next = std::min(chunk * 2, chunk_max);
    if (check_every <= 0 && *err_prev > 0 && st.err > 0 && st.err < *err_prev && st.npass > *np_prev &&
        st.tol > 0 && st.err > st.tol) {
      const double rate = std::pow(st.err / *err_prev, 1.0 / (st.npass - *np_prev));
      const double need = std::log(st.tol / st.err) / std::log(rate);
      if (std::isfinite(need) && need > 0) {
        static const int sizes[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32};
        next = 32;
        for (int z : sizes)
          if (z >= need) {
            next = z;
            break;
          }
      }
    }
    *err_prev = st.err;
    *np_prev = st.npass;
    return next;
  }

  // A plain SK stage with fused passes: one column sweep g_1 = T_c(f_0)
  // (unarmed test), then pass k computes f_k = T_r(g_k) and g_{k+1} and
  // tests (f_k, g_k) -- the pairs, tests and counts of the two-pass loop,
  // with one read of C per iteration.  G ends in w.G[0].
  int run_stage_fused(int max_iter, int check_every, bool* converged) {
    init_state_keep();
    // no row maxima yet (NaN): the first pass takes each row's max as its shift
    HIPCHK(hipMemsetAsync(w.fz_rowmax, 0xff, sizeof(float) * P.n, s));
    sweep_col(w.F, MA_F, w.G[0], w.G[1], DOT_G, MA_G, 0, nullptr, nullptr, W_NONE, G_NOT_DONE,
              F_CHECK | F_COUNT | F_GSEL, 0);
    int p = 1, launched = 0, chunk = check_every > 0 ? check_every : 4;
    const int chunk_max = check_every > 0 ? check_every : 32;
    DevState st{};
    bool done = false;
    double err_prev = -1.0;  // error at the previous poll, and the check count then
    int np_prev = 0;
    while (launched < max_iter) {
      const int k = std::min(chunk, max_iter - launched);
      for (int t = 0; t < k; ++t) {
        sk_fused(p);
        p = 1 - p;
      }
      launched += k;
      st = read_state();
      check_cancel();
      if (st.done) {
        done = true;
        break;
      }
      chunk = next_chunk(chunk, chunk_max, check_every, st, &err_prev, &np_prev);
    }
    *converged = done;
    last_err = st.err;
    // g_k of the last tested pair: G[gsel] when converged, else the input of
    // the last pass, G[1 - p]
    const int gidx = done ? st.gsel : 1 - p;
    if (gidx != 0) HIPCHK(hipMemcpyAsync(w.G[0], w.G[gidx], sizeof(float2) * P.m, hipMemcpyDeviceToDevice, s));
    return std::max(0, st.npass - 1);
  }

  // One SK iteration (ping-pong on G[p]).
  void sk_iter(int p) {
    sweep_col(w.F, MA_F, w.G[p], w.G[1 - p], DOT_G, MA_G, 0, nullptr, nullptr, W_NONE, G_NOT_DONE,
              F_CHECK | F_COUNT | F_GSEL, p);
    sweep_row(w.G[1 - p], MA_G, nullptr, w.F, nullptr, DOT_F, MA_F, 0, nullptr, nullptr, W_NONE, G_NOT_DONE, 0);
  }
  // One SK-NR iteration; first == true skips the Newton step (first SK
  // iteration of Algorithm 4.1 from f_0).
  void sknr_iter(int ell, bool first) {
    const int ellp = w.ellp;
    sweep_col(w.F, MA_F, w.G[0], w.Gt, DOT_GT, MA_GT, first ? 0 : ellp, w.V, w.W, W_SCALE_WEIGHT, G_NOT_DONE,
              F_CHECK | F_COUNT);
    sweep_row(w.Gt, MA_GT, w.F, w.Fsk, w.mdiff, DOT_FSK, MA_FSK, 0, nullptr, nullptr, W_NONE, G_NOT_DONE, 0);
    if (!first) {
      newton(ell, G_NOT_DONE);
      candidate(G_NOT_DONE | G_CHOL_OK);
    }
    HIPCHK(launch_select(w.Fp, w.Fsk, w.F, P.n, w.Gp, w.Gt, w.G[0], P.m, w.st, G_NOT_DONE, s));
    if (!first)
      sweep_row(w.G[0], MA_G, nullptr, w.F, nullptr, DOT_F, MA_F, 0, nullptr, nullptr, W_NONE,
                G_NOT_DONE | G_ACCEPT, 0);
  }

  // k iterations through the batcher: record one unit (one SK-NR iteration,
  // or the SK pair from parity 0), upload its argument blocks, run it `k /
  // unit` times together with the other requests' units of the same kernel
  // sequence.  Returns the iterations run, or 0 when some launch of the unit
  // has no batched twin (the caller then launches as usual).
  int batch_chunk(int ell, int k) {
    const int u = ell > 0 ? 1 : 2;
    if (!c->batcher || k < u) return 0;
    Recorder rec;
    rec.recs = c->recbuf;
    rec.cap = kMaxUnitLaunches;
    g_recorder = &rec;
    try {
      if (ell > 0) sknr_iter(ell, false);
      else {
        sk_iter(0);
        sk_iter(1);
      }
    } catch (...) {
      g_recorder = nullptr;
      throw;
    }
    g_recorder = nullptr;
    if (rec.unsupported || rec.n == 0) return 0;
    for (int i = 0; i < rec.n; ++i) {
      const LaunchRec& r = rec.recs[i];
      std::memcpy(c->arg_pinned + (size_t)i * kMaxArgBytes, r.args, r.arg_bytes);
      c->units[i] = BatchLaunch{r.bfunc, w.argbank + (size_t)i * kMaxArgBytes, r.gx, r.gy, r.block, r.lds};
    }
    HIPCHK(hipMemcpyAsync(w.argbank, c->arg_pinned, (size_t)rec.n * kMaxArgBytes, hipMemcpyHostToDevice, s));
    HIPCHK(hipEventRecord(c->ev_in, s));
    BatchJob job;
    job.unit = c->units;
    job.nrec = rec.n;
    job.reps = k / u;
    job.ev_in = c->ev_in;
    job.ev_done = c->ev_done;
    const int reps = batcher_run(c->batcher, &job);
    if (job.status != 0) throw Err{SKNR_EDEVICE, std::string("batched launch: ") +
                                                      hipGetErrorString((hipError_t)job.status)};
    HIPCHK(hipStreamWaitEvent(s, c->ev_done, 0));
    return reps * u;
  }

  // k iterations as one captured graph (k even for the SK ping-pong, which
  // then starts and ends on parity 0)
  hipGraphExec_t chunk_graph(int ell, int k) {
    GraphKey key;
    std::memset(&key, 0, sizeof key);
    key.ws = c->arena.base;
    key.C = P.C;
    key.X = P.X;
    key.Y = P.Y;
    key.wX = P.wX;
    key.wY = P.wY;
    key.xcost = w.X;
    key.ldc = P.ldc;
    key.n = P.n;
    key.m = P.m;
    key.d = P.d;
    key.kind = sweep_kind(P);
    key.ell = ell;
    key.ellp = w.ellp;
    key.iters = k;
    key.ctrans = P.ctrans ? 1 : 0;
    key.cscale = P.cscale;
    key.cmax = P.cmax;
    key.stream = (void*)s;
    for (auto& g : c->graphs)
      if (g.key == key) return g.exec;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int t = 0; t < k; ++t) {
      if (ell > 0) sknr_iter(ell, false);
      else sk_iter(t & 1);
    }
    hipGraph_t g;
    HIPCHK(hipStreamEndCapture(s, &g));
    hipGraphExec_t ge;
    hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(e);
    if (c->graphs.size() >= 32) c->drop_graphs();
    c->graphs.push_back(CachedGraph{key, ge});
    return ge;
  }

  // Run one stage of Algorithm 4.1 from the current (F, G[0]); returns
  // iterations and sets *converged.  G ends in w.G[0].
  double last_err = 0;  // the sweeps' FP32 marginal-error estimate at the end of run_stage
  int run_stage(int ell, int max_iter, int check_every, bool resume, bool* converged, int* tried, int* accepted) {
    if (ell == 0 && fused && max_iter >= 1) {
      *tried = *accepted = 0;
      return run_stage_fused(max_iter, check_every, converged);
    }
    if (!c->batcher) return run_stage_impl(ell, max_iter, check_every, resume, converged, tried, accepted);
    // batched chunks: count this lane as iterating while in the loop
    struct Iterating {
      Batcher* b;
      explicit Iterating(Batcher* b_) : b(b_) { batcher_iterating(b, +1); }
      ~Iterating() { batcher_iterating(b, -1); }
    } guard(c->batcher);
    return run_stage_impl(ell, max_iter, check_every, resume, converged, tried, accepted);
  }
  int run_stage_impl(int ell, int max_iter, int check_every, bool resume, bool* converged, int* tried,
                     int* accepted) {
    init_state_keep();
    const bool graphs = c->use_graphs && !c->profile;
    int launched = 0;  // iterations launched (each = one column sweep)
    int p = 0;
    int chunk = check_every > 0 ? check_every : 4;
    const int chunk_max = check_every > 0 ? check_every : (ell > 0 ? 8 : 32);
    bool done = false;
    DevState st{};
    double err_prev = -1.0;  // error at the previous poll, and the check count then
    int np_prev = 0;
    if (ell > 0 && !resume && max_iter >= 1) {
      sknr_iter(ell, true);  // the first iteration of Algorithm 4.1 has no Newton step
      ++launched;
    }
    while (true) {
      int remaining = max_iter - launched;  // full iterations still allowed
      if (remaining <= 0) break;
      int k = std::min(chunk, remaining);
      if (ell == 0 && (k & 1) && k > 1) --k;
      int kb = 0;
      if (c->batcher && (ell > 0 || p == 0)) kb = batch_chunk(ell, k);
      if (kb > 0) {
        k = kb;
      } else if (graphs && k >= 2 && p == 0) {
        HIPCHK(hipGraphLaunch(chunk_graph(ell, k), s));
      } else {
        for (int t = 0; t < k; ++t) {
          if (ell > 0) {
            sknr_iter(ell, false);
          } else {
            sk_iter(p);
            p = 1 - p;
          }
        }
      }
      launched += k;
      st = read_state();
      check_cancel();
      if (st.done) {
        done = true;
        break;
      }
      chunk = next_chunk(chunk, chunk_max, check_every, st, &err_prev, &np_prev);
    }
    if (!done) {
      // the (max_iter+1)-th column sweep: convergence test of f_max_iter
      sweep_col(w.F, MA_F, w.G[ell > 0 ? 0 : p], ell > 0 ? w.Gt : w.G[1 - p], ell > 0 ? DOT_GT : DOT_G,
                ell > 0 ? MA_GT : MA_G, 0, nullptr, nullptr, W_NONE, G_NOT_DONE, F_CHECK | F_COUNT | F_GSEL, p);
      st = read_state();
    }
    *converged = st.done != 0;
    *tried = st.newton_tried;
    *accepted = st.newton_accepted;
    last_err = st.err;
    // bring g_k into G[0]
    int gidx = ell > 0 ? 0 : (st.done ? st.gsel : p);
    if (gidx != 0) HIPCHK(hipMemcpyAsync(w.G[0], w.G[gidx], sizeof(float2) * P.m, hipMemcpyDeviceToDevice, s));
    return std::max(0, st.npass - 1);
  }

  // state re-initialisation that keeps the maxabs / dot slots of (F, G[0])
  void init_state_keep() {
    DevState z{};
    set_consts(z);
    HIPCHK(launch_state_reset(w.st, z, true, s));
  }

  // FP64 potentials in the caller's orientation -> f_out, g_out (device)
  void export_fg(double* f_out, double* g_out) {
    HIPCHK(launch_from_hat(w.F, w.lX64, eps, w.fX64, P.n, s));
    HIPCHK(launch_from_hat(w.G[0], w.lY64, eps, w.gY64, P.m, s));
    double* fo = P.transposed ? g_out : f_out;
    double* go = P.transposed ? f_out : g_out;
    HIPCHK(hipMemcpyAsync(fo, w.fX64, 8 * (size_t)P.n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(go, w.gY64, 8 * (size_t)P.m, hipMemcpyDeviceToDevice, s));
  }

  // cost description for kernels working in the caller's orientation
  SweepArgs caller_geo(const sknr_problem* pr) const {
    SweepArgs geo{};
    geo.C = pr->C;
    geo.ldc = pr->ldc;
    geo.Pred = pr->x;
    geo.Pout = pr->y;
    geo.d = pr->d;
    geo.cscale = P.cscale;
    geo.cscale64 = P.cscale64;
    geo.dpad = P.dpad;
    geo.m2cs = -2.f * P.cscale;
    const bool sw = P.transposed;  // engine side X holds the caller's y
    geo.Hred = (const uint4*)(sw ? w.HY : w.HX);
    geo.Mred = (const uint4*)(sw ? w.MY : w.MX);
    geo.Lred = (const uint4*)(sw ? w.LY : w.LX);
    geo.Nred = sw ? w.NY : w.NX;
    geo.Hout = (const uint4*)(sw ? w.HX : w.HY);
    geo.Mout = (const uint4*)(sw ? w.MX : w.MY);
    geo.Lout = (const uint4*)(sw ? w.LX : w.LY);
    geo.Nout = sw ? w.NX : w.NY;
    return geo;
  }

  // FP64 evaluation in the caller's orientation, on the solver's cost or
  // (exact) on the FP64 squared distance of the FP32 points
  sknr_eval evaluate(const sknr_problem* pr, const double* f, const double* g, bool exact = false) {
    SweepArgs geo = caller_geo(pr);
    int nrb, ncb;
    const int kind = (exact && P.kind == SKNR_COST_SQEUCLID) ? kEvalExact : sweep_kind(P);
    if (kind >= 2 && kind <= 4)
      HIPCHK(launch_eval_mfma(geo, kind - 1, f, g, pr->a, pr->b, eps, w.evrow, w.evcol, w.evscal, P.n0, P.m0,
                              &nrb, &ncb, s));
    else
      HIPCHK(launch_eval(geo, kind, f, g, pr->a, pr->b, eps, w.evrow, w.evcol, w.evscal, P.n0, P.m0, &nrb, &ncb, s));
    HIPCHK(launch_eval_finish(w.evrow, w.evcol, w.evscal, pr->a, pr->b, P.n0, P.m0, nrb, ncb, w.evout, w.evblk, s));
    HIPCHK(launch_dot64(f, pr->a, P.n0, w.evout + 8, s));
    HIPCHK(launch_dot64(g, pr->b, P.m0, w.evout + 9, s));
    double h[16];
    HIPCHK(hipMemcpyAsync(h, w.evout, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    sknr_eval e{};
    e.row_err = h[0];
    e.col_err = h[1];
    e.marginal_err = h[0] + h[1];
    e.transport_cost = h[2];
    e.mass = h[3];
    e.dual_value = h[8] + h[9] - eps * (h[3] - 1.0);
    e.primal_value = h[2] + eps * (h[4] - h[3] + 1.0);
    return e;
  }

  void gauge(const sknr_problem* pr, double* f, double* g) {
    HIPCHK(launch_dot64(f, pr->a, P.n0, w.evout + 10, s));
    HIPCHK(launch_dot64(g, pr->b, P.m0, w.evout + 11, s));
    HIPCHK(launch_shift64(f, P.n0, w.evout + 10, +1.0, s));
    HIPCHK(launch_shift64(g, P.m0, w.evout + 10, -1.0, s));
  }

  // Spectral warm start (Sec. 4) at the current (F, eps): block subspace
  // iteration on M = D_a^-1 P~ D_b^-1 P~^T, P~ = pi(f, f^{C,eps}), with a
  // block of kp = pad(min(32, ell + oversample)) columns kept orthonormal in
  // L2(a) and orthogonal to the constants (rho_0 = 1 is excluded), FP64
  // Rayleigh-Ritz each iteration after the first (whose Rayleigh quotients
  // stand in for Ritz values), stop when the leading ell Ritz values move
  // by less than tol.  Leaves the Ritz vectors in w.Vw (n x kp,
  // descending) and returns the iterations; lam gets the kp Ritz values.
  // Rayleigh-Ritz accuracy (launch_jacobi's off2): 1e-14 (eigenvectors to
  // ~1e-7, the FP32 basis' own resolution) for sknr_spectral_basis; the
  // solve's warm start only needs a basis whose span carries the leading
  // modes and Ritz values for its stop test, and takes 1e-8 (eigenvalues to
  // ~1e-8 relative, eigenvectors to ~1e-4), a sweep fewer per call
  double jacobi_off2 = 1e-14;
  int spectral(int ell, int oversample, int max_it, double tol, uint64_t seed, std::vector<double>* lam) {
    int kp = ell_pad(std::min(32, ell + std::max(0, oversample)));
    if (kp < ell_pad(ell)) kp = ell_pad(ell);
    const int n = P.n, m = P.m;
    const int nbn = std::min(128, std::max(1, (n + 63) / 64));
    const int nbm = std::min(128, std::max(1, (m + 63) / 64));
    const int plen = kp * kp + kp;
    // okw[2]: positions of zero (dropped) columns in the Ritz block.  Each
    // Gram of Z refills them with fresh random values, so the block keeps
    // its full width (at smaller eps more modes are resolved, and the
    // oversampling columns speed up the iteration).
    unsigned* zmask = reinterpret_cast<unsigned*>(w.okw + 2);
    if (w.have_Vw) HIPCHK(hipMemcpyAsync(w.Zw, w.Vw, sizeof(float) * (size_t)n * kp, hipMemcpyDeviceToDevice, s));
    else HIPCHK(launch_random_block(kp, w.Zw, n, 0, seed, zmask, s));
    std::vector<double> lp(kp, 0.0), lc(kp, 0.0);
    int it = 0;
    for (it = 1; it <= max_it; ++it) {
      // V = orthonormalised (Z - 1 s^T) in L2(a)
      HIPCHK(launch_wgram(kp, w.Zw, P.wX, 0, n, w.nrpart, nbn, zmask, ~0u,
                          seed ^ (0x632BE59BD9B4E019ull * (uint64_t)it), s));
      HIPCHK(launch_sum_partials(w.nrpart, nbn, plen, w.nrsum, s));
      HIPCHK(launch_orth(kp, w.nrsum, 1, w.Rw, w.sw, w.okw, zmask, s));
      HIPCHK(launch_affine(kp, w.Zw, w.sw, w.Rw, nullptr, 0, n, w.Vw, s));
      // U = P~^T V (and G~ = T_c(F))
      sweep_col(w.F, MA_F, nullptr, w.Gt, DOT_GT, MA_GT, kp, w.Vw, w.Uw, W_SCALE_WEIGHT, 0, 0);
      // Rayleigh-Ritz: T = U^T D_b^-1 U = V^T D_a M V
      HIPCHK(launch_wgram(kp, w.Uw, P.wY, 1, m, w.nrpart, nbm, nullptr, 0u, 0, s));
      HIPCHK(launch_sum_partials(w.nrpart, nbm, plen, w.nrsum, s));
      // the stop test needs two iterations: the first one's Ritz values stay
      // on the device (lamw + 32) and come back with the second's, one host
      // round trip fewer per warm start
      const bool defer = it == 1 && max_it > 1;
      // the first iteration keeps its basis (a rotation would not change
      // the span that the next iteration works on) and passes the Rayleigh
      // quotients diag(T) to the stop test in place of its Ritz values
      if (defer) HIPCHK(launch_ritz_diag(kp, w.nrsum, 1, w.Qw, w.lamw + 32, w.okw + 1, zmask, s));
      else HIPCHK(launch_jacobi(kp, w.nrsum, 1, w.Qw, w.lamw, w.okw + 1, zmask, s, jacobi_off2));
      if (!defer) {
        HIPCHK(launch_affine(kp, w.Vw, nullptr, w.Qw, nullptr, 0, n, w.Zw, s));
        std::swap(w.Vw, w.Zw);  // V <- V Q (Ritz vectors)
      }
      HIPCHK(launch_affine(kp, w.Uw, nullptr, w.Qw, P.wY, 1, m, w.Utw, s));  // D_b^-1 U Q
      if (defer) {
        check_cancel();
        // Z = M V = D_a^-1 P~ (D_b^-1 U Q)
        sweep_row(w.Gt, MA_GT, w.F, w.Fsk, nullptr, DOT_FSK, MA_FSK, kp, w.Utw, w.Zw, W_SCALE_RATIO, 0, 0);
        continue;
      }
      double both[64];
      const bool first_pair = it == 2 && max_it > 1;  // iteration 1 was deferred
      HIPCHK(hipMemcpyAsync(both, w.lamw, sizeof(double) * (first_pair ? 64 : kp), hipMemcpyDeviceToHost, s));
      int jsw = 0;
      HIPCHK(hipMemcpyAsync(&jsw, w.okw + 1, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      std::copy(both, both + kp, lc.begin());
      if (first_pair) std::copy(both + 32, both + 32 + kp, lp.begin());
      check_cancel();
      if (getenv("SKNR_DEBUG_EIG")) std::fprintf(stderr, "eig it %d jacobi sweeps %d lam0 %.6f lam%d %.6f\n", it, jsw, lc[0], ell - 1, lc[ell - 1]);
      // the move of each leading Ritz value rho_i^2 relative to its gap
      // 1 - rho_i^2, which sets the rate of the mode under SK (Lemma 3.2)
      double dmax = 0;
      for (int i = 0; i < ell; ++i)
        dmax = std::max(dmax, std::fabs(lc[i] - lp[i]) / std::max(1.0 - lc[i], 1e-12));
      lp = lc;
      if (it >= 2 && dmax < tol) break;
      if (it == max_it) break;
      // Z = M V = D_a^-1 P~ (D_b^-1 U Q)
      sweep_row(w.Gt, MA_GT, w.F, w.Fsk, nullptr, DOT_FSK, MA_FSK, kp, w.Utw, w.Zw, W_SCALE_RATIO, 0, 0);
    }
    w.have_Vw = true;
    if (lam) *lam = lc;
    return std::min(it, max_it);
  }
  int spectral_kp(int ell, int oversample) const {
    int kp = ell_pad(std::min(32, ell + std::max(0, oversample)));
    return std::max(kp, ell_pad(ell));
  }
  // Newton basis from the warm-start block: first ell columns, padded
  void use_warm_V(int ell, int oversample) {
    have_basis = true;
    HIPCHK(launch_repack(w.Vw, spectral_kp(ell, oversample), P.n, ell, w.ellp, w.V, s));
  }

  // V (engine orientation, n x ell FP64 device) -> padded FP32 V
  void load_V(const double* V, int ell) {
    have_basis = true;
    std::vector<double> hv((size_t)P.n * ell);
    HIPCHK(hipMemcpyAsync(hv.data(), V, 8 * hv.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<float> pv((size_t)P.n * w.ellp, 0.f);
    for (int i = 0; i < P.n; ++i)
      for (int l = 0; l < ell; ++l) pv[(size_t)i * w.ellp + l] = (float)hv[(size_t)i * ell + l];
    HIPCHK(hipMemcpyAsync(w.V, pv.data(), 4 * pv.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
};

const sknr_problem* stage_problem(Ctx* c, const sknr_problem* pr, hipStream_t s, sknr_problem* tmp) {
  if (!pr || !pr->on_host) return pr;
  REQUIRE(pr->a && pr->b, "weights a, b are required");
  REQUIRE(pr->n >= 1 && pr->m >= 1 && pr->n <= (1 << 26) && pr->m <= (1 << 26), "n, m out of range");
  const bool stored = pr->kind == SKNR_COST_STORED;
  REQUIRE(stored || pr->kind == SKNR_COST_SQEUCLID, "unknown cost kind");
  const size_t n = (size_t)pr->n, m = (size_t)pr->m;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  size_t bytes = al(8 * n) + al(8 * m);
  if (stored) {
    REQUIRE(pr->C && pr->ldc >= pr->m, "stored cost C is NULL or ldc < m");
    bytes += al(4 * n * m);
  } else {
    REQUIRE(pr->x && pr->y && pr->d >= 1 && pr->d <= 1024, "points x, y and 1 <= d <= 1024 are required");
    bytes += al(4 * n * (size_t)pr->d) + al(4 * m * (size_t)pr->d);
  }
  if (bytes > c->stage_cap) {
    HIPCHK(hipStreamSynchronize(s));
    if (c->stage) HIPCHK(hipFree(c->stage));
    c->stage = nullptr;
    c->stage_cap = 0;
    if (hipMalloc((void**)&c->stage, bytes) != hipSuccess) {
      c->stage = nullptr;
      throw Err{SKNR_ENOMEM, "device allocation of the input staging block failed"};
    }
    c->stage_cap = bytes;
  }
  *tmp = *pr;
  tmp->on_host = 0;
  char* q = c->stage;
  auto take = [&](size_t b) {
    char* r = q;
    q += al(b);
    return r;
  };
  double* da = (double*)take(8 * n);
  double* db = (double*)take(8 * m);
  HIPCHK(hipMemcpyAsync(da, pr->a, 8 * n, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(db, pr->b, 8 * m, hipMemcpyHostToDevice, s));
  tmp->a = da;
  tmp->b = db;
  if (stored) {
    float* dC = (float*)take(4 * n * m);
    HIPCHK(hipMemcpy2DAsync(dC, 4 * m, pr->C, 4 * (size_t)pr->ldc, 4 * m, n, hipMemcpyHostToDevice, s));
    tmp->C = dC;
    tmp->ldc = (int64_t)m;
  } else {
    const size_t d = (size_t)pr->d;
    float* dx = (float*)take(4 * n * d);
    float* dy = (float*)take(4 * m * d);
    HIPCHK(hipMemcpyAsync(dx, pr->x, 4 * n * d, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dy, pr->y, 4 * m * d, hipMemcpyHostToDevice, s));
    tmp->x = dx;
    tmp->y = dy;
  }
  return tmp;
}

Prepared prepare_caller_orientation(const sknr_problem* prob, hipStream_t s, void* scratch) {
  Prepared P = prepare(prob, s, scratch);
  if (P.transposed) {
    P.transposed = false;
    P.n = P.n0;
    P.m = P.m0;
    P.ctrans = false;
    P.X = prob->x;
    P.Y = prob->y;
    P.wX = prob->a;
    P.wY = prob->b;
    std::swap(P.wminX, P.wminY);
    std::swap(P.wmaxX, P.wmaxY);
    std::swap(P.entX, P.entY);
  }
  return P;
}


// solver of the l x l Newton system with its defaults filled in
NrSolver nr_solver_of(int kind, int max_iter, double rtol, int ell) {
  NrSolver v;
  v.kind = kind;
  v.max_iter = max_iter > 0 ? max_iter : (kind == NR_CG ? 2 * std::max(ell, 1) : 64);
  v.rtol = rtol > 0 ? rtol : 1e-12;
  return v;
}

// The eps schedule of sknr_solve on one lane (see the header for the
// stage protocol): optional static warm start, per stage the spectral warm
// start (sequential), the rebase of the potentials to the new eps, the SK /
// SK-NR iterations and the FP64 check; the gauge and reported values after
// the last stage.
int solve_on_lane(Lane* L, const sknr_problem* prob, const Prepared& P, const sknr_opts* opts, double* f_out,
                  double* g_out, sknr_result* res) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = L->own;
  int ellp = ell_pad(opts->ell);
  WS w = make_ws(L, P, ellp, s);
  Engine E(L, P, w, s);
  E.jacobi_off2 = 1e-8;
  const int eig_os = opts->eig_oversample > 0 ? opts->eig_oversample : 8;
  const int eig_it = opts->eig_max_iter > 0 ? opts->eig_max_iter : 100;
  const double eig_tol = opts->eig_tol > 0 ? opts->eig_tol : 0.1;
  std::memset(res, 0, sizeof(*res));
  E.tol = opts->tol;
  E.nrs = nr_solver_of(opts->newton_solver, opts->newton_max_iter, opts->newton_rtol, opts->ell);
  E.fused = E.fused_eligible();
  int static_eig_iters = 0;
  // initial potentials: the iteration runs on the engine's f (the semi-dual
  // side); the caller's f0 / g0 swap roles on a transposed problem
  const double* ef0 = P.transposed ? opts->g0 : opts->f0;
  const double* eg0 = P.transposed ? opts->f0 : opts->g0;
  L->sub = Lane::Subspace{};
  if (opts->ell > 0 && opts->warm_mode == SKNR_WARM_STATIC) {
    // plain SK at eps' from the initial potential, then V_l once
    E.eps = opts->eps_prime;
    E.init_state();
    E.start(ef0, eg0);
    bool cv;
    int tr, ac;
    E.run_stage(0, opts->max_iter, opts->check_every, false, &cv, &tr, &ac);
    static_eig_iters = E.spectral(opts->ell, eig_os, eig_it, eig_tol, opts->seed, nullptr);
    E.use_warm_V(opts->ell, eig_os);
  }
  E.eps = opts->eps[0];
  E.init_state();
  E.start(ef0, eg0);
  if (opts->ell > 0 && opts->warm_mode == SKNR_WARM_USER) E.load_V(opts->V0, opts->ell);
  res->n_stages = opts->n_eps;
  res->transposed = P.transposed ? 1 : 0;
  int status = SKNR_OK;
  // adaptive switch: plain SK until a stage needs more than T iterations,
  // SK-NR with the sequential warm start on every stage after it
  const bool adaptive = opts->nr_switch_iters > 0 && opts->ell > 0 && opts->warm_mode == SKNR_WARM_SEQUENTIAL;
  bool nr_on = !adaptive;
  for (int st = 0; st < opts->n_eps; ++st) {
    auto ts = std::chrono::steady_clock::now();
    double eps = opts->eps[st];
    int eig_iters = 0;
    double gain = 0;
    bool gain_ok = true;
    if (st > 0 && opts->ell > 0 && opts->warm_mode == SKNR_WARM_SEQUENTIAL && nr_on) {
      // V_l from the optimum of the previous stage (its eps), Sec. 4
      std::vector<double> lam;
      eig_iters = E.spectral(opts->ell, eig_os, eig_it, eig_tol, opts->seed + st, &lam);
      E.use_warm_V(opts->ell, eig_os);
      // rate gain of Theorem 4.2 over Lemma 3.2 predicted by the Ritz values
      if (!lam.empty()) {
        const double r1 = lam[0];
        const double rl = lam[std::min<size_t>((size_t)opts->ell, lam.size() - 1)];
        gain = (1.0 - rl) / std::max(1.0 - r1, 1e-300);
        if (opts->nr_min_gain > 0 && gain < opts->nr_min_gain) gain_ok = false;
      }
    }
    if (st == 0 && opts->ell > 0 && opts->warm_mode == SKNR_WARM_STATIC) eig_iters = static_eig_iters;
    if (st > 0) {
      double de = eps - E.eps;
      E.init_state();
      HIPCHK(launch_rebase(w.F, w.lXdf, split_df(de), P.n, w.st, MA_F, s));
      HIPCHK(launch_rebase(w.G[0], w.lYdf, split_df(de), P.m, w.st, MA_G, s));
      E.eps = eps;
    }
    bool use_nr = opts->ell > 0 && (st > 0 || opts->first_stage_nr) && nr_on && gain_ok;
    bool conv = false;
    int tried = 0, acc = 0, it = 0;
    sknr_eval ev{};
    // The sweeps estimate the error in FP32 (column marginal via the next
    // c-transform); that ends an intermediate stage, whose potentials only
    // start the next one.  After the last stage the FP64 check decides: if
    // it disagrees, the stage continues with a tighter FP32 threshold.
    const bool last = st == opts->n_eps - 1;
    E.tol = opts->tol;
    for (int attempt = 0; attempt < 8; ++attempt) {
      int tr = 0, ac = 0;
      bool cv = false;
      it += E.run_stage(use_nr ? opts->ell : 0, opts->max_iter - it, opts->check_every, attempt > 0, &cv, &tr, &ac);
      tried += tr;
      acc += ac;
      if (!last) {
        conv = cv;
        ev = sknr_eval{};
        ev.marginal_err = E.last_err;
        break;
      }
      E.export_fg(f_out, g_out);
      ev = E.evaluate(prob, f_out, g_out);
      conv = cv && ev.marginal_err < opts->tol;
      if (conv || !cv || it >= opts->max_iter) break;
      E.tol = E.tol * std::min(0.9, opts->tol / ev.marginal_err);
    }
    if (!conv) status = SKNR_NOT_CONVERGED;
    if (!nr_on && it > opts->nr_switch_iters) nr_on = true;
    sknr_stage_stats& ss = res->stage[st];
    ss.eps = eps;
    ss.iters = it;
    ss.newton_tried = tried;
    ss.newton_accepted = acc;
    ss.eig_iters = eig_iters;
    ss.rate_gain = gain;
    ss.nr_skipped = gain_ok ? 0 : 1;
    ss.marginal_err = ev.marginal_err;
    ss.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - ts).count();
    res->total_iters += it;
    if (st == opts->n_eps - 1) {
      E.gauge(prob, f_out, g_out);
      res->marginal_err = ev.marginal_err;
      res->row_err = ev.row_err;
      res->col_err = ev.col_err;
      res->transport_cost = ev.transport_cost;
      res->dual_value = ev.dual_value;
      res->primal_value = ev.primal_value;
      res->mass = ev.mass;
      if (P.kind == SKNR_COST_SQEUCLID) {
        sknr_eval ex = E.evaluate(prob, f_out, g_out, true);
        res->marginal_err_exact = ex.marginal_err;
        res->transport_cost_exact = ex.transport_cost;
      } else {
        res->marginal_err_exact = ev.marginal_err;
        res->transport_cost_exact = ev.transport_cost;
      }
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  if (E.have_basis) {
    L->sub.V = w.V;
    L->sub.n = P.n;
    L->sub.ellp = w.ellp;
    L->sub.ell = opts->ell;
    L->sub.transposed = P.transposed;
    L->sub.gen = L->ws_gen;
  }
  res->status = status;
  res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return status;
}

void check_opts(const sknr_opts* opts, const Prepared& P) {
  REQUIRE(opts->n_eps >= 1 && opts->n_eps <= SKNR_MAX_STAGES && opts->eps, "eps schedule length out of range");
  for (int s = 0; s < opts->n_eps; ++s) check_eps(opts->eps[s]);
  REQUIRE(opts->tol > 0 && std::isfinite(opts->tol), "tol must be positive");
  REQUIRE(opts->max_iter >= 1, "max_iter must be >= 1");
  REQUIRE(opts->ell >= 0 && opts->ell <= SKNR_MAX_ELL, "ell out of range");
  REQUIRE(opts->ell < std::min(P.n0, P.m0), "ell must be < min(n, m)");
  REQUIRE(opts->nr_switch_iters >= 0, "nr_switch_iters must be >= 0");
  REQUIRE(opts->nr_switch_iters == 0 || opts->ell == 0 || opts->warm_mode == SKNR_WARM_SEQUENTIAL,
          "nr_switch_iters needs WARM_SEQUENTIAL");
  if (opts->ell > 0) {
    REQUIRE(opts->warm_mode == SKNR_WARM_USER || opts->warm_mode == SKNR_WARM_SEQUENTIAL ||
                opts->warm_mode == SKNR_WARM_STATIC, "unknown warm_mode");
    if (opts->warm_mode == SKNR_WARM_USER) REQUIRE(opts->V0, "WARM_USER needs V0");
    if (opts->warm_mode == SKNR_WARM_STATIC) check_eps(opts->eps_prime);
    REQUIRE(!opts->first_stage_nr || opts->warm_mode != SKNR_WARM_SEQUENTIAL,
            "first_stage_nr needs WARM_USER or WARM_STATIC");
  }
  REQUIRE(opts->newton_solver >= SKNR_NEWTON_DIRECT && opts->newton_solver <= SKNR_NEWTON_SCHULZ,
          "unknown newton_solver");
  REQUIRE(opts->newton_max_iter >= 0 && opts->newton_rtol >= 0 && std::isfinite(opts->newton_rtol),
          "newton_max_iter and newton_rtol must be >= 0");
  REQUIRE(opts->nr_min_gain >= 0 && std::isfinite(opts->nr_min_gain), "nr_min_gain must be >= 0");
}

void rebind(Prepared& P, const sknr_problem* pr) {
  P.C = pr->C;
  P.X = P.transposed ? pr->y : pr->x;
  P.Y = P.transposed ? pr->x : pr->y;
  P.wX = P.transposed ? pr->b : pr->a;
  P.wY = P.transposed ? pr->a : pr->b;
}

void lane_init(Lane* L, int device) {
  L->device = device;
  HIPCHK(hipHostMalloc((void**)&L->st_host, sizeof(DevState), hipHostMallocDefault));
  HIPCHK(hipHostMalloc((void**)&L->arg_pinned, (size_t)kMaxUnitLaunches * kMaxArgBytes, hipHostMallocDefault));
  L->recbuf = new LaunchRec[kMaxUnitLaunches];
  L->units = new BatchLaunch[kMaxUnitLaunches];
  HIPCHK(hipEventCreateWithFlags(&L->ev_in, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&L->ev_done, hipEventDisableTiming));
  HIPCHK(hipStreamCreateWithFlags(&L->own, hipStreamNonBlocking));
  const char* ng = getenv("SKNR_NO_GRAPHS");
  L->use_graphs = !(ng && ng[0] == '1');
}

void lane_release(Lane* L) {
  if (L->own) (void)hipStreamSynchronize(L->own);
  L->drop_graphs();
  if (L->arena.base && !L->arena_external) (void)hipFree(L->arena.base);
  L->arena.base = nullptr;
  L->arena.cap = 0;
  if (L->xcost) (void)hipFree(L->xcost);
  L->xcost = nullptr;
  L->xcost_cap = 0;
  if (L->st_host) (void)hipHostFree(L->st_host);
  L->st_host = nullptr;
  if (L->arg_pinned) (void)hipHostFree(L->arg_pinned);
  L->arg_pinned = nullptr;
  delete[] L->recbuf;
  L->recbuf = nullptr;
  delete[] L->units;
  L->units = nullptr;
  if (L->ev_in) (void)hipEventDestroy(L->ev_in);
  if (L->ev_done) (void)hipEventDestroy(L->ev_done);
  L->ev_in = L->ev_done = nullptr;
  L->drain();
  if (L->own) (void)hipStreamDestroy(L->own);
  L->own = nullptr;
  for (auto e : L->evpool) (void)hipEventDestroy(e);
  L->evpool.clear();
}

void check_eps(double eps) { REQUIRE(eps > 0 && std::isfinite(eps), "eps must be positive and finite"); }

}  // namespace sknr_host

using namespace sknr_host;

// ============================================================================
extern "C" {

const char* sknr_version(void) { return "sknr 0.1 (gfx950)"; }

const char* sknr_status_str(int status) {
  switch (status) {
    case SKNR_OK: return "ok";
    case SKNR_NOT_CONVERGED: return "not converged (tolerance not reached within max_iter)";
    case SKNR_EINVAL: return "invalid argument";
    case SKNR_ENOMEM: return "out of device memory or over budget";
    case SKNR_EDEVICE: return "HIP runtime error";
    case SKNR_EBUSY: return "busy";
    case SKNR_ECANCELED: return "cancelled";
    case SKNR_EINTERNAL: return "internal error";
    default: return "unknown status";
  }
}
const char* sknr_last_error(void) { return g_last_error.c_str(); }

int sknr_ctx_create(int device, uint64_t hbm_budget_bytes, void** out) {
  return guarded([&]() -> int {
    REQUIRE(out, "out is NULL");
    int cnt = 0;
    HIPCHK(hipGetDeviceCount(&cnt));
    REQUIRE(device >= 0 && device < cnt, "no such device");
    HIPCHK(hipSetDevice(device));
    Ctx* c = new Ctx();
    try {
      c->device = device;
      size_t fr = 0, tot = 0;
      HIPCHK(hipMemGetInfo(&fr, &tot));
      c->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * fr);
      HIPCHK(hipMalloc(&c->prep, kPrepBytes));
      lane_init(&c->lane, device);
      lane_init(&c->lane_na, device);
      c->lane_na.use_graphs = false;
      noalloc_setup(device);
      HIPCHK(hipEventCreateWithFlags(&c->order_ev, hipEventDisableTiming));
    } catch (...) {
      lane_release(&c->lane);
      lane_release(&c->lane_na);
      if (c->order_ev) (void)hipEventDestroy(c->order_ev);
      if (c->prep) (void)hipFree(c->prep);
      delete c;
      throw;
    }
    *out = c;
    return SKNR_OK;
  });
}

int sknr_ctx_destroy(void* ctx) {
  return guarded([&]() -> int {
    if (!ctx) return SKNR_OK;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    HIPCHK(hipSetDevice(c->device));
    server_destroy(c);
    HIPCHK(hipDeviceSynchronize());
    lane_release(&c->lane);
    c->lane_na.arena.base = nullptr;  // the static array, never freed
    c->lane_na.arena.cap = 0;
    lane_release(&c->lane_na);
    if (c->order_ev) (void)hipEventDestroy(c->order_ev);
    if (c->stage) (void)hipFree(c->stage);
    if (c->prep) (void)hipFree(c->prep);
    delete c;
    return SKNR_OK;
  });
}

int sknr_solve(void* ctx, const sknr_problem* prob, const sknr_opts* opts, double* f_out, double* g_out,
               sknr_result* res) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    REQUIRE(opts && res && f_out && g_out, "opts, res, f_out, g_out are required");
    // run on the context's stream, after the work already queued on the caller's
    hipStream_t cs = as_stream(opts->stream);
    hipStream_t s = c->lane.own;
    HIPCHK(hipEventRecord(c->order_ev, cs));
    HIPCHK(hipStreamWaitEvent(s, c->order_ev, 0));
    sknr_problem staged;
    prob = stage_problem(c, prob, s, &staged);
    Prepared P = prepare(prob, s, c->prep);
    check_opts(opts, P);
    return solve_on_lane(&c->lane, prob, P, opts, f_out, g_out, res);
  });
}

int sknr_c_transform_col(void* ctx, const sknr_problem* prob, double eps, const double* f, const double* g_prev,
                         double* g_out, double* err_out, double* gdot_out, void* stream) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    check_eps(eps);
    REQUIRE(f && g_out, "f and g_out are required");
    hipStream_t s = as_stream(stream);
    sknr_problem staged;
    prob = stage_problem(c, prob, s, &staged);
    Prepared P = prepare_caller_orientation(prob, s, c->prep);
    WS w = make_ws(&c->lane, P, 0, s);
    Engine E(&c->lane, P, w, s);
    E.eps = eps;
    E.init_state();
    E.load_f(f);
    if (g_prev) E.load_g(g_prev, w.G[1], MA_G2, DOT_TMP);
    E.sweep_col(w.F, MA_F, g_prev ? w.G[1] : nullptr, w.G[0], DOT_G, MA_G, 0, nullptr, nullptr, W_NONE, 0, 0);
    HIPCHK(launch_from_hat(w.G[0], w.lY64, eps, g_out, P.m, s));
    DevState st = E.read_state();
    if (err_out) *err_out = g_prev ? st.err : 0.0;
    if (gdot_out) {
      double h;
      HIPCHK(launch_dot64(g_out, prob->b, P.m, w.evout, s));
      HIPCHK(hipMemcpyAsync(&h, w.evout, 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      *gdot_out = h;
    }
    return SKNR_OK;
  });
}

int sknr_c_transform_row(void* ctx, const sknr_problem* prob, double eps, const double* g, double* f_out,
                         void* stream) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    check_eps(eps);
    REQUIRE(g && f_out, "g and f_out are required");
    hipStream_t s = as_stream(stream);
    sknr_problem staged;
    prob = stage_problem(c, prob, s, &staged);
    Prepared P = prepare_caller_orientation(prob, s, c->prep);
    WS w = make_ws(&c->lane, P, 0, s);
    Engine E(&c->lane, P, w, s);
    E.eps = eps;
    E.init_state();
    E.load_g(g, w.G[0], MA_G, DOT_G);
    E.sweep_row(w.G[0], MA_G, nullptr, w.F, nullptr, DOT_F, MA_F, 0, nullptr, nullptr, W_NONE, 0, 0);
    HIPCHK(launch_from_hat(w.F, w.lX64, eps, f_out, P.n, s));
    HIPCHK(hipStreamSynchronize(s));
    return SKNR_OK;
  });
}

int sknr_projected_system(void* ctx, const sknr_problem* prob, double eps, const double* f, const double* V,
                          int32_t ell, double* G_out, double* grad_out, double* qsemi_out, void* stream) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    check_eps(eps);
    REQUIRE(f && V && ell >= 1 && ell <= SKNR_MAX_ELL, "f, V and 1 <= ell <= 32 are required");
    hipStream_t s = as_stream(stream);
    sknr_problem staged;
    prob = stage_problem(c, prob, s, &staged);
    Prepared P = prepare_caller_orientation(prob, s, c->prep);
    int ellp = ell_pad(ell);
    WS w = make_ws(&c->lane, P, ellp, s);
    Engine E(&c->lane, P, w, s);
    E.eps = eps;
    E.init_state();
    E.load_f(f);
    E.load_V(V, ell);
    E.sweep_col(w.F, MA_F, nullptr, w.Gt, DOT_GT, MA_GT, ellp, w.V, w.W, W_SCALE_WEIGHT, 0, 0);
    E.sweep_row(w.Gt, MA_GT, w.F, w.Fsk, w.mdiff, DOT_FSK, MA_FSK, 0, nullptr, nullptr, W_NONE, 0, 0);
    HIPCHK(launch_nr_assemble(ell, w.V, w.mdiff, P.wX, P.n, w.W, P.wY, P.m, w.nrpart, w.nr_rows_blk, w.nr_cols_blk,
                              w.st, 0, s));
    HIPCHK(launch_sum_partials(w.nrpart, w.nr_rows_blk + w.nr_cols_blk, nr_part_len(ell), w.nrsum, s));
    HIPCHK(launch_nr_solve(ell, w.nrsum, 1, w.coef32, w.coef64, w.Gout, w.gout, w.st, 0, s));
    std::vector<double> hG((size_t)ell * ell), hg(ell);
    HIPCHK(hipMemcpyAsync(hG.data(), w.Gout, 8 * hG.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hg.data(), w.gout, 8 * hg.size(), hipMemcpyDeviceToHost, s));
    DevState st = E.read_state();
    if (G_out) std::memcpy(G_out, hG.data(), 8 * hG.size());
    if (grad_out) std::memcpy(grad_out, hg.data(), 8 * hg.size());
    if (qsemi_out) {
      // <f,a> + <g~,b> in paper convention: hat dots minus eps (<log a,a> + <log b,b>)
      const double ca = P.entX, cb = P.entY;
      *qsemi_out = st.dots[DOT_F] + st.dots[DOT_GT] - eps * (ca + cb);
    }
    return SKNR_OK;
  });
}

int sknr_newton_step(void* ctx, const sknr_problem* prob, double eps, double* f_inout, const double* V, int32_t ell,
                     int32_t* accepted, double* q0, double* q1, void* stream) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    check_eps(eps);
    REQUIRE(f_inout && V && ell >= 1 && ell <= SKNR_MAX_ELL, "f, V and 1 <= ell <= 32 are required");
    hipStream_t s = as_stream(stream);
    sknr_problem staged;
    prob = stage_problem(c, prob, s, &staged);
    Prepared P = prepare_caller_orientation(prob, s, c->prep);
    int ellp = ell_pad(ell);
    WS w = make_ws(&c->lane, P, ellp, s);
    Engine E(&c->lane, P, w, s);
    E.eps = eps;
    E.init_state();
    E.load_f(f_inout);
    E.load_V(V, ell);
    E.sweep_col(w.F, MA_F, nullptr, w.Gt, DOT_GT, MA_GT, ellp, w.V, w.W, W_SCALE_WEIGHT, 0, 0);
    E.sweep_row(w.Gt, MA_GT, w.F, w.Fsk, w.mdiff, DOT_FSK, MA_FSK, 0, nullptr, nullptr, W_NONE, 0, 0);
    E.newton(ell, 0);
    E.candidate(G_CHOL_OK);
    DevState st = E.read_state();
    const double ca = P.entX, cb = P.entY;
    if (q0) *q0 = st.dots[DOT_F] + st.dots[DOT_GT] - eps * (ca + cb);
    if (q1) *q1 = st.chol_ok ? st.dots[DOT_FP] + st.dots[DOT_GP] - eps * (ca + cb) : NAN;
    if (accepted) *accepted = st.accept;
    if (st.accept) HIPCHK(launch_from_hat(w.Fp, w.lX64, eps, f_inout, P.n, s));
    HIPCHK(hipStreamSynchronize(s));
    return SKNR_OK;
  });
}

int sknr_newton_coef(void* ctx, const sknr_problem* prob, double eps, const double* f, const double* V, int32_t ell,
                     int32_t solver, int32_t max_iter, double rtol, double* coef_out, int32_t* ok_out,
                     int32_t* iters_out, void* stream) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    check_eps(eps);
    REQUIRE(f && V && coef_out && ok_out && ell >= 1 && ell <= SKNR_MAX_ELL,
            "f, V, coef_out, ok_out and 1 <= ell <= 32 are required");
    REQUIRE(solver >= SKNR_NEWTON_DIRECT && solver <= SKNR_NEWTON_SCHULZ, "unknown solver");
    REQUIRE(max_iter >= 0 && rtol >= 0 && std::isfinite(rtol), "max_iter and rtol must be >= 0");
    hipStream_t s = as_stream(stream);
    sknr_problem staged;
    prob = stage_problem(c, prob, s, &staged);
    Prepared P = prepare_caller_orientation(prob, s, c->prep);
    int ellp = ell_pad(ell);
    WS w = make_ws(&c->lane, P, ellp, s);
    Engine E(&c->lane, P, w, s);
    E.eps = eps;
    E.nrs = nr_solver_of(solver, max_iter, rtol, ell);
    E.init_state();
    E.load_f(f);
    E.load_V(V, ell);
    E.sweep_col(w.F, MA_F, nullptr, w.Gt, DOT_GT, MA_GT, ellp, w.V, w.W, W_SCALE_WEIGHT, 0, 0);
    E.sweep_row(w.Gt, MA_GT, w.F, w.Fsk, w.mdiff, DOT_FSK, MA_FSK, 0, nullptr, nullptr, W_NONE, 0, 0);
    HIPCHK(launch_nr_assemble(ell, w.V, w.mdiff, P.wX, P.n, w.W, P.wY, P.m, w.nrpart, w.nr_rows_blk, w.nr_cols_blk,
                              w.st, 0, s));
    HIPCHK(launch_sum_partials(w.nrpart, w.nr_rows_blk + w.nr_cols_blk, nr_part_len(ell), w.nrsum, s));
    HIPCHK(launch_nr_solve(ell, w.nrsum, 1, w.coef32, w.coef64, nullptr, nullptr, w.st, 0, s, E.nrs));
    std::vector<double> hc(ell);
    HIPCHK(hipMemcpyAsync(hc.data(), w.coef64, 8 * (size_t)ell, hipMemcpyDeviceToHost, s));
    DevState st = E.read_state();
    std::memcpy(coef_out, hc.data(), 8 * (size_t)ell);
    *ok_out = st.chol_ok;
    if (iters_out) *iters_out = st.nr_iters;
    return SKNR_OK;
  });
}

int sknr_evaluate(void* ctx, const sknr_problem* prob, double eps, const double* f, const double* g, sknr_eval* out,
                  void* stream) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    check_eps(eps);
    REQUIRE(f && g && out, "f, g, out are required");
    hipStream_t s = as_stream(stream);
    sknr_problem staged;
    prob = stage_problem(c, prob, s, &staged);
    Prepared P = prepare_caller_orientation(prob, s, c->prep);
    WS w = make_ws(&c->lane, P, 0, s);
    Engine E(&c->lane, P, w, s);
    E.eps = eps;
    *out = E.evaluate(prob, f, g);
    if (P.kind == SKNR_COST_SQEUCLID) {
      sknr_eval ex = E.evaluate(prob, f, g, true);
      out->row_err_exact = ex.row_err;
      out->col_err_exact = ex.col_err;
      out->marginal_err_exact = ex.marginal_err;
      out->transport_cost_exact = ex.transport_cost;
    } else {
      out->row_err_exact = out->row_err;
      out->col_err_exact = out->col_err;
      out->marginal_err_exact = out->marginal_err;
      out->transport_cost_exact = out->transport_cost;
    }
    return SKNR_OK;
  });
}

int sknr_gradient(void* ctx, const sknr_problem* prob, double eps, const double* f, const double* g, double* grad_x,
                  double* grad_y, double* grad_a, double* grad_b, void* stream) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    check_eps(eps);
    REQUIRE(f && g, "f and g are required");
    hipStream_t s = as_stream(stream);
    sknr_problem staged;
    prob = stage_problem(c, prob, s, &staged);
    Prepared P = prepare_caller_orientation(prob, s, c->prep);
    REQUIRE(!(grad_x || grad_y) || P.kind == SKNR_COST_SQEUCLID, "point gradients need a squared-Euclidean problem");
    WS w = make_ws(&c->lane, P, 32, s);
    Engine E(&c->lane, P, w, s);
    E.eps = eps;
    E.init_state();
    E.load_f(f);
    E.load_g(g, w.G[0], MA_G, DOT_G);
    const int d = P.kind == SKNR_COST_SQEUCLID ? P.d : 0;
    const double two_s = 2.0 * P.cscale64;
    // rows: r_i - a_i (mdiff) and sum_j pi_ij y_j, 32 coordinates per pass
    if (grad_x || grad_a) {
      int c0 = 0;
      do {
        const int dc = grad_x ? std::min(32, d - c0) : 0;
        const int ellp = ell_pad(dc);
        if (dc > 0) HIPCHK(launch_pack_cols(P.Y, P.m, d, c0, dc, ellp, w.Utw, s));
        E.sweep_row(w.G[0], MA_G, w.F, w.Fsk, w.mdiff, -1, -1, ellp, dc > 0 ? w.Utw : nullptr, dc > 0 ? w.Zw : nullptr,
                    dc > 0 ? W_SCALE_MASS : W_NONE, 0, 0);
        if (dc > 0) HIPCHK(launch_grad_points(P.X, P.n, d, c0, dc, P.wX, w.mdiff, w.Zw, ellp, two_s, grad_x, s));
        if (c0 == 0 && grad_a) HIPCHK(launch_grad_weights(f, P.wX, w.mdiff, P.n, eps, grad_a, s));
        c0 += 32;
      } while (grad_x && c0 < d);
    }
    // columns: c_j - b_j and sum_i pi_ij x_i
    if (grad_y || grad_b) {
      E.col_mdiff = w.mdiffY;
      int c0 = 0;
      do {
        const int dc = grad_y ? std::min(32, d - c0) : 0;
        const int ellp = ell_pad(dc);
        if (dc > 0) HIPCHK(launch_pack_cols(P.X, P.n, d, c0, dc, ellp, w.Vw, s));
        E.sweep_col(w.F, MA_F, w.G[0], w.Gt, -1, -1, ellp, dc > 0 ? w.Vw : nullptr, dc > 0 ? w.Uw : nullptr,
                    dc > 0 ? W_SCALE_MASS : W_NONE, 0, 0);
        if (dc > 0) HIPCHK(launch_grad_points(P.Y, P.m, d, c0, dc, P.wY, w.mdiffY, w.Uw, ellp, two_s, grad_y, s));
        if (c0 == 0 && grad_b) HIPCHK(launch_grad_weights(g, P.wY, w.mdiffY, P.m, eps, grad_b, s));
        c0 += 32;
      } while (grad_y && c0 < d);
      E.col_mdiff = nullptr;
    }
    HIPCHK(hipStreamSynchronize(s));
    return SKNR_OK;
  });
}

int sknr_coupling(void* ctx, const sknr_problem* prob, double eps, const double* f, const double* g, float* P_out,
                  void* stream) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    check_eps(eps);
    REQUIRE(f && g && P_out, "f, g, P_out are required");
    hipStream_t s = as_stream(stream);
    sknr_problem staged;
    prob = stage_problem(c, prob, s, &staged);
    Prepared P = prepare_caller_orientation(prob, s, c->prep);
    WS w = make_ws(&c->lane, P, 0, s);
    Engine E(&c->lane, P, w, s);
    SweepArgs geo = E.caller_geo(prob);
    const int kind = sweep_kind(P);
    if (kind >= 2 && kind <= 4)
      HIPCHK(launch_coupling_mfma(geo, kind - 1, f, g, prob->a, prob->b, eps, P_out, P.n0, P.m0, s));
    else
      HIPCHK(launch_coupling(geo, P.kind, f, g, prob->a, prob->b, eps, P_out, P.n0, P.m0, s));
    HIPCHK(hipStreamSynchronize(s));
    return SKNR_OK;
  });
}

int sknr_profile(void* ctx, int32_t enable) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    HIPCHK(hipDeviceSynchronize());
    c->lane.drain();
    c->lane.profile = enable != 0;
    c->lane.prof.clear();
    return SKNR_OK;
  });
}

int sknr_profile_read(void* ctx, sknr_kprof* out, int32_t max_entries, int32_t* count) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    REQUIRE(count && (out || max_entries == 0), "count (and out) required");
    HIPCHK(hipDeviceSynchronize());
    c->lane.drain();
    int k = 0;
    for (auto& e : c->lane.prof) {
      if (k < max_entries) {
        std::memset(&out[k], 0, sizeof(sknr_kprof));
        std::snprintf(out[k].name, sizeof(out[k].name), "%s", e.name.c_str());
        out[k].launches = e.launches;
        out[k].total_ms = e.total_ms;
        out[k].units = e.units;
      }
      ++k;
    }
    *count = k;
    return SKNR_OK;
  });
}

int sknr_spectral_basis(void* ctx, const sknr_problem* prob, double eps, const double* f, int32_t ell,
                        int32_t oversample, int32_t max_iter, double tol, uint64_t seed, double* V_out,
                        double* rho_out, int32_t* iters_out, void* stream) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    check_eps(eps);
    REQUIRE(f && V_out && rho_out, "f, V_out, rho_out are required");
    REQUIRE(ell >= 1 && ell <= SKNR_MAX_ELL, "1 <= ell <= 32 required");
    REQUIRE(max_iter >= 1 && tol > 0, "max_iter >= 1 and tol > 0 required");
    hipStream_t s = as_stream(stream);
    sknr_problem staged;
    prob = stage_problem(c, prob, s, &staged);
    Prepared P = prepare_caller_orientation(prob, s, c->prep);
    REQUIRE(ell < std::min(P.n, P.m), "ell must be < min(n, m)");
    WS w = make_ws(&c->lane, P, ell_pad(ell), s);
    Engine E(&c->lane, P, w, s);
    E.eps = eps;
    E.init_state();
    E.load_f(f);
    std::vector<double> lam;
    int it = E.spectral(ell, oversample, max_iter, tol, seed, &lam);
    int kp = E.spectral_kp(ell, oversample);
    // Ritz pairs below what the FP32 products resolve (the bound of the
    // rank-revealing orthonormalisation: ||M v||^2 = rho^4 at most 1e-8 of
    // the top one's, or 1e-12) come back as zero columns with rho = 0; the
    // block may hold random refill directions there
    const double top = lam.empty() ? 0.0 : std::max(0.0, lam[0]);
    const double cut = std::max(1e-8 * top * top, 1e-12);
    unsigned zero = 0;
    for (int i = 0; i < ell; ++i)
      if (!(lam[i] > 0.0 && lam[i] * lam[i] > cut)) zero |= 1u << i;
    HIPCHK(launch_take_cols(w.Vw, kp, P.n, ell, zero, V_out, s));
    HIPCHK(hipStreamSynchronize(s));
    rho_out[0] = 1.0;
    for (int i = 0; i < ell; ++i) rho_out[i + 1] = ((zero >> i) & 1u) ? 0.0 : std::sqrt(lam[i]);
    if (iters_out) *iters_out = it;
    return SKNR_OK;
  });
}

int sknr_get_subspace(void* ctx, double* V_out, int64_t rows, int32_t ell, int32_t* side_out, void* stream) {
  return guarded([&]() -> int {
    Ctx* c = as_ctx(ctx);
    REQUIRE(V_out, "V_out is required");
    const Lane::Subspace& b = c->lane.sub;
    REQUIRE(b.V && b.gen == c->lane.ws_gen,
            "no basis: the last sknr_solve on this context ran no SK-NR stage, or another call has used the "
            "context since");
    REQUIRE(rows == b.n && ell == b.ell, "rows / ell differ from the basis of the last solve (rows = " +
                                             std::to_string(b.n) + ", ell = " + std::to_string(b.ell) + ")");
    hipStream_t s = as_stream(stream);
    HIPCHK(launch_take_cols(b.V, b.ellp, b.n, b.ell, 0u, V_out, s));
    HIPCHK(hipStreamSynchronize(s));
    if (side_out) *side_out = b.transposed ? 1 : 0;
    return SKNR_OK;
  });
}

}  // extern "C"
