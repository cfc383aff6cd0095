"""Parity at the full workload sizes, on sampled outputs.

The oracle cannot solve these problems, but it can evaluate one output of a
c-transform at a time.  Every pair (f, g) that sknr_solve exports satisfies
f = T_r(g) exactly in the algorithm (each SK / SK-NR iteration ends with a
row transform, and the convergence test selects g_k with f_k = T_r(g_k)),
also after the gauge shift.  So for sampled rows i, the oracle's row
c-transform of the GPU's g on the (modelled) cost must reproduce f_i within
the FP32 log-sum-exp tolerance plus the cost model's bound, and the column
transform of f must reproduce g up to the converged marginal error.

Workloads: the benchmark's 4096 x 4096 d = 2 points with the 8-stage ladder;
the 16384^2 stored grid-histogram cost (1 GiB) at eps' = 1e-3 -> eps = 5e-4;
the 20000 x 30000 d = 64 Gaussian clouds with the bf16 hi/lo matrix-core
cost on the ladder 1e-1 -> 1e-2 -> 2e-3 (iteration caps keep the run short;
the identity holds at every iterate).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests._helpers import U32, bf16_cost_model, fp32_sqeuclid, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_2506_14780_amd as sk
    return sk


@pytest.fixture(scope="module")
def ctx(sk):
    c = sk.Context(0)
    yield c
    c.close()


def _rows(n, k=48, seed=0):
    return np.sort(np.random.default_rng(seed).choice(n, size=k, replace=False))


def test_fullsize_points_benchmark_workload(sk, ctx):
    prob = W.gmm_vs_uniform(4096, seed=1)
    ladder = list(W.EPS_LADDER_C2)
    gp = sk.Problem(a=to_dev(prob.a), b=to_dev(prob.b), x=to_dev(prob.x), y=to_dev(prob.y))
    f, g, res = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=200000, ell=16, warm_mode=sk.WARM_SEQUENTIAL)
    f, g = f.cpu().numpy(), g.cpu().numpy()
    eps = ladder[-1]
    print("iters", [s["iters"] for s in res["stages"]], "marginal", res["marginal_err"], flush=True)
    assert res["status"] == 0 and res["marginal_err"] < 1e-6
    rows = _rows(prob.n)
    Cr = fp32_sqeuclid(prob.x[rows], prob.y).astype(np.float64)
    fr = O.c_transform_row(g, Cr, prob.b, eps)
    df = np.abs(f[rows] - fr).max()
    print(f"rows: max|f - T_r(g)| = {df:.3e}", flush=True)
    assert df <= 64 * U32 * eps + 1e-12 * np.abs(f).max()
    cols = _rows(prob.m, seed=1)
    Cc = fp32_sqeuclid(prob.x, prob.y[cols]).astype(np.float64)
    gc = O.c_transform_col(f, Cc, prob.a, eps)
    # |g - T_c(f)| <= eps * |log(1 + marginal residual of column j)|
    lim = eps * np.abs(np.log1p(-np.minimum(res["marginal_err"] / prob.b[cols], 0.5)))
    print(f"cols: max|g - T_c(f)| = {np.abs(g[cols] - gc).max():.3e}", flush=True)
    assert np.all(np.abs(g[cols] - gc) <= lim + 64 * U32 * eps)


def test_fullsize_stored_cost(sk, ctx):
    prob = W.grid_histograms()
    gp = sk.Problem(a=to_dev(prob.a), b=to_dev(prob.b), C=to_dev(prob.C))
    ladder = [1e-3, 5e-4]
    f, g, res = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=150, ell=16, warm_mode=sk.WARM_SEQUENTIAL)
    f, g = f.cpu().numpy(), g.cpu().numpy()
    print("status", res["status"], "iters", [s["iters"] for s in res["stages"]], "marginal", res["marginal_err"],
          flush=True)
    assert res["status"] in (0, 1) and np.all(np.isfinite(f)) and np.all(np.isfinite(g))
    rows = _rows(prob.n)
    fr = O.c_transform_row(g, prob.C[rows].astype(np.float64), prob.b, ladder[-1])
    df = np.abs(f[rows] - fr).max()
    print(f"rows: max|f - T_r(g)| = {df:.3e}", flush=True)
    assert df <= 64 * U32 * ladder[-1] + 1e-12 * np.abs(f).max()


@pytest.mark.parametrize("parts", [2, 3])
def test_fullsize_clouds_matrix_core_cost(sk, ctx, parts):
    prob = W.gaussian_clouds()
    gp = sk.Problem(a=to_dev(prob.a), b=to_dev(prob.b), x=to_dev(prob.x), y=to_dev(prob.y),
                    xterm=sk.XTERM_BF16X3 if parts == 2 else sk.XTERM_BF16X6)
    ladder = [1e-1, 1e-2, 2e-3]
    f, g, res = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=150, ell=16, warm_mode=sk.WARM_SEQUENTIAL)
    f, g = f.cpu().numpy(), g.cpu().numpy()
    print("status", res["status"], "iters", [s["iters"] for s in res["stages"]], "marginal", res["marginal_err"],
          "vs exact", res["marginal_err_exact"], flush=True)
    assert res["status"] in (0, 1) and np.all(np.isfinite(f)) and np.all(np.isfinite(g))
    rows = _rows(prob.n)
    Cm, bound = bf16_cost_model(prob.x[rows], prob.y, 1.0, parts=parts, mu_points=(prob.x, prob.y))
    fr = O.c_transform_row(g, Cm, prob.b, ladder[-1])
    df = np.abs(f[rows] - fr).max()
    print(f"rows: max|f - T_r(g)| = {df:.3e}  (cost bound {bound.max():.3e})", flush=True)
    assert df <= bound.max() + 64 * U32 * ladder[-1] + 1e-12 * np.abs(f).max()


def test_fullsize_gradient_on_sampled_rows_and_columns(sk, ctx):
    """sknr_gradient at the 4096 x 4096 d = 2 benchmark solution: for sampled
    rows i the oracle forms row i of the coupling of the GPU's own (f, g)
    on the FP32 cost and evaluates 2 (r_i x_i - sum_j pi_ij y_j) and
    f_i - eps r_i / a_i; likewise for sampled columns."""
    prob = W.gmm_vs_uniform(4096, seed=1)
    ladder = list(W.EPS_LADDER_C2)
    gp = sk.Problem(a=to_dev(prob.a), b=to_dev(prob.b), x=to_dev(prob.x), y=to_dev(prob.y))
    f, g, res = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=200000, ell=16, warm_mode=sk.WARM_SEQUENTIAL)
    eps = ladder[-1]
    gr = {k: v.cpu().numpy() for k, v in sk.gradient(ctx, gp, eps, f, g).items()}
    f, g = f.cpu().numpy(), g.cpu().numpy()
    x, y = prob.x.astype(np.float64), prob.y.astype(np.float64)
    rows = _rows(prob.n, k=16, seed=3)
    Pr = O.coupling(f[rows], g, fp32_sqeuclid(prob.x[rows], prob.y).astype(np.float64), prob.a[rows], prob.b, eps)
    r = Pr.sum(1)
    gx = 2 * (r[:, None] * x[rows] - Pr @ y)
    ga = f[rows] - eps * r / prob.a[rows]
    cols = _rows(prob.m, k=16, seed=4)
    Pc = O.coupling(f, g[cols], fp32_sqeuclid(prob.x, prob.y[cols]).astype(np.float64), prob.a, prob.b[cols], eps)
    c = Pc.sum(0)
    gy = 2 * (c[:, None] * y[cols] - Pc.T @ x)
    gb = g[cols] - eps * c / prob.b[cols]
    scale = 2 * np.abs(x).max() * prob.a.max()
    ex = np.abs(gr["x"][rows] - gx).max()
    ey = np.abs(gr["y"][cols] - gy).max()
    ea = np.abs(gr["a"][rows] - ga).max()
    eb = np.abs(gr["b"][cols] - gb).max()
    print(f"grad errors x {ex:.3e} y {ey:.3e} (scale {scale:.3e}); a {ea:.3e} b {eb:.3e}", flush=True)
    assert ex <= 1e-5 * scale and ey <= 1e-5 * scale
    assert ea <= 1e-5 * eps and eb <= 1e-5 * eps
