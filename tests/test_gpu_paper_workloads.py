"""Paper-shaped workloads (Sec. 5) on the GPU against the FP64 oracle.

Fig. 5.1's setup: n = 200 samples of N(0, I) against 2n of N((4, 4),
[[1, -0.8], [-0.8, 1]]), uniform weights, squared Euclidean cost (the
paper prints neither its eps values nor its l; the readings here are a
halving ladder from eps = 1 and l = 10):
* left panel: sequential warm start from eps = 1, SK against SK-NR(l);
* middle panel: static warm start, V_l from a plain SK solve at eps' = 1
  used at a smaller eps from f = 0;
* right panel: iteration counts as l grows (l = 0 is SK).
The GPU runs the same algorithm as the oracle with FP32 sweeps, so its
per-stage iteration counts must track the oracle's and its optimum must
match.

The single-cell maps of Sec. 5 (6507 x 3815 and 3815 x 2982, PCA to
R^30, l = 30, eps from 1 decreasing, SK at eps = 1 first) use data that is
not available; a synthetic stand-in at those shapes (workloads.wot_shaped)
runs at full size and is checked on sampled rows against the oracle on the
exact cost.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests._helpers import U32, bf16_cost_model, e_pot, fp32_sqeuclid, gpu_problem

pytestmark = pytest.mark.gpu

LADDER = [1.0, 0.5, 0.25, 0.125]
# the oracle computes V_l exactly (dense eigh); the GPU by subspace
# iteration, here run to Ritz-value stagnation 1e-9 (the solver's default,
# 1e-4, trades basis accuracy for warm-start time)
EIG = dict(eig_tol=1e-9, eig_max_iter=300)


@pytest.fixture(scope="module")
def sk():
    import paper_2506_14780_amd as sk
    return sk


@pytest.fixture(scope="module")
def ctx(sk):
    c = sk.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def fig51():
    prob = W.paper_2d_gaussians(200)
    C = fp32_sqeuclid(prob.x, prob.y).astype(np.float64)
    return prob, C


def _iters(res):
    return [s["iters"] for s in res["stages"]]


def test_fig51_sequential_warm_start(sk, ctx, fig51):
    prob, C = fig51
    gp = gpu_problem(prob)
    f0, g0, r0 = sk.solve(ctx, gp, LADDER, tol=1e-6, max_iter=100000)
    f1, g1, r1 = sk.solve(ctx, gp, LADDER, tol=1e-6, max_iter=100000, ell=10, warm_mode=sk.WARM_SEQUENTIAL, **EIG)
    _, _, rd = sk.solve(ctx, gp, LADDER, tol=1e-6, max_iter=100000, ell=10, warm_mode=sk.WARM_SEQUENTIAL)
    print("GPU SK-NR with the default eigensolver tolerance", _iters(rd), flush=True)
    _, _, ro0 = O.solve_schedule(C, prob.a, prob.b, LADDER, 1e-6, 100000)
    fo, go, ro1 = O.solve_schedule(C, prob.a, prob.b, LADDER, 1e-6, 100000, ell=10)
    print("GPU SK", _iters(r0), "SK-NR", _iters(r1), "| oracle SK", [r.iters for r in ro0], "SK-NR",
          [r.iters for r in ro1], flush=True)
    assert r0["status"] == 0 and r1["status"] == 0
    for a_, b_ in zip(_iters(r0), [r.iters for r in ro0]):
        assert abs(a_ - b_) <= 0.1 * b_ + 2
    for a_, b_ in zip(_iters(r1)[1:], [r.iters for r in ro1][1:]):
        assert a_ <= 1.25 * b_ + 3
    # the paper's left panel: far fewer iterations with the spectral warm start
    assert sum(_iters(r1)[1:]) < 0.5 * sum(_iters(r0)[1:])
    fo, go = O.normalize_gauge(fo, go, prob.a, prob.b)
    assert e_pot(f1.cpu().numpy(), g1.cpu().numpy(), fo, go, C) < 1e-5


def test_fig51_static_warm_start(sk, ctx, fig51):
    prob, C = fig51
    gp = gpu_problem(prob)
    eps = 0.125
    f, g, r = sk.solve(ctx, gp, [eps], tol=1e-6, max_iter=100000, ell=10, warm_mode=sk.WARM_STATIC,
                       eps_prime=1.0, first_stage_nr=True, **EIG)
    _, _, rsk = sk.solve(ctx, gp, [eps], tol=1e-6, max_iter=100000)
    ref = O.sinkhorn(C, prob.a, prob.b, 1.0, 1e-10, 100000)
    V, _ = O.spectral_basis(ref.f, ref.g, C, prob.a, prob.b, 1.0, 10)
    ro = O.sknr(C, prob.a, prob.b, eps, 1e-6, 100000, V=V)
    print("GPU static SK-NR", _iters(r), "SK", _iters(rsk), "| oracle static SK-NR", ro.iters, flush=True)
    assert r["status"] == 0 and r["marginal_err"] < 1e-6
    assert _iters(r)[0] < _iters(rsk)[0]
    assert _iters(r)[0] <= 1.25 * ro.iters + 3


def test_fig51_iterations_fall_as_ell_grows(sk, ctx, fig51):
    prob, C = fig51
    gp = gpu_problem(prob)
    ladder = LADDER[:3]
    tot_gpu, tot_o = [], []
    for ell in (0, 2, 5, 10, 20):
        kw = dict(ell=ell, warm_mode=sk.WARM_SEQUENTIAL, **EIG) if ell > 0 else {}
        _, _, r = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=100000, **kw)
        _, _, ro = O.solve_schedule(C, prob.a, prob.b, ladder, 1e-6, 100000, ell=ell)
        tot_gpu.append(sum(_iters(r)[1:]))
        tot_o.append(sum(r_.iters for r_ in ro[1:]))
        assert r["status"] == 0
    print("l = 0, 2, 5, 10, 20: GPU iterations after the first stage", tot_gpu, "oracle", tot_o, flush=True)
    for a_, b_ in zip(tot_gpu, tot_o):
        assert a_ <= 1.25 * b_ + 4
    assert tot_gpu[-1] < tot_gpu[2] < tot_gpu[0]


def _rows(n, k=16, seed=5):
    return np.sort(np.random.default_rng(seed).choice(n, size=k, replace=False))


def test_wot_shaped_full_size(sk, ctx):
    prob = W.wot_shaped(3815, 2982)
    gp = gpu_problem(prob)
    ladder = [1.0, 0.5, 0.25, 0.125, 0.0625]
    print("case wot_shaped 3815 x 2982 d=30", flush=True)
    f, g, r = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=50000, ell=30, warm_mode=sk.WARM_SEQUENTIAL)
    _, _, r0 = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=50000)
    print("SK-NR(30)", _iters(r), "SK", _iters(r0), "marginal", r["marginal_err"], "exact", r["marginal_err_exact"],
          flush=True)
    assert r["status"] == 0 and r0["status"] == 0
    assert sum(_iters(r)[1:]) < sum(_iters(r0)[1:])
    f, g = f.cpu().numpy(), g.cpu().numpy()
    rows = _rows(prob.n)
    eps = ladder[-1]
    Cm, bound = bf16_cost_model(prob.x[rows], prob.y, 1.0, parts=3, mu_points=(prob.x, prob.y))
    fr = O.c_transform_row(g, Cm, prob.b, eps)
    df = np.abs(f[rows] - fr).max()
    # at L1 marginal error e the row marginal r_i of (f, g) satisfies
    # |r_i - a_i| <= e, so |f_i - T_r(g)_i| = eps |log(r_i / a_i)| is at most
    # about eps e / a_i; plus the matrix-core cost's deviation from its model
    marg = eps * 1.01 * r["marginal_err"] / prob.a.min()
    print(f"rows: max|f - T_r(g)| = {df:.3e} (cost bound {bound.max():.3e}, marginal bound {marg:.3e})", flush=True)
    assert df <= bound.max() + marg + 64 * U32 * eps + 1e-12 * np.abs(f).max()
