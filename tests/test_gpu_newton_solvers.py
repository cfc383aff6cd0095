"""The iterative solvers of the projected Newton system (Sec. 4, the
paragraph on the disadvantages of the algorithm: the NR step made GPU
friendly by iterative inversion of the projected Hessian or by conjugate
gradients) against the direct solve and against the oracle's Cholesky
step, for l = 16 and 30; and full SK-NR schedules with each solver
against the oracle's optimum."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests._helpers import e_pot, fp32_sqeuclid, to_dev

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


@pytest.mark.parametrize("basis", ["eigen", "random"])
@pytest.mark.parametrize("ell", [16, 30])
def test_newton_coef_iterative_solvers_match_direct_and_oracle(sk, ctx, ell, basis):
    """With the low-frequency eigenbasis G is nearly diagonal (a few CG
    steps); a random orthonormal basis gives a dense, worse conditioned G."""
    prob = W.gmm_vs_uniform(500, 700, seed=31)
    C = fp32_sqeuclid(prob.x, prob.y).astype(np.float64)
    eps = 0.03
    r = O.sinkhorn(C, prob.a, prob.b, eps, tol=1e-3, max_iter=5000)
    if basis == "eigen":
        ref = O.sinkhorn(C, prob.a, prob.b, eps, tol=1e-12, max_iter=200000)
        V, _ = O.spectral_basis(ref.f, ref.g, C, prob.a, prob.b, eps, ell, method="dense")
    else:
        V = np.linalg.qr(np.random.default_rng(ell).standard_normal((500, ell)))[0]
    step = O.projected_newton(r.f, C, prob.a, prob.b, eps, V)
    assert step["ok"]
    G = -eps * step["hess"]
    cond = np.linalg.cond(G)
    gp = sk.Problem(a=to_dev(prob.a), b=to_dev(prob.b), x=to_dev(prob.x), y=to_dev(prob.y))
    fd, Vd = to_dev(r.f), to_dev(np.ascontiguousarray(V))
    c0, ok0, it0 = sk.newton_coef(ctx, gp, eps, fd, Vd, sk.NEWTON_DIRECT)
    assert ok0 and it0 == 0
    ref_c = step["coef"]
    scale = np.abs(ref_c).max()
    # c = eps G^-1 grad.  The GPU's G and grad come from FP32 sweeps and meet
    # the projected-system bar (G within 1e-5 of max|G|, grad within 1e-4 of
    # max|grad| plus 1e-6 max a), so to first order
    #   |dc| <= cond(G) (1e-4 + 1e-5) |c| + eps |G^-1| 1e-6 max(a) sqrt(l)
    nrm = np.linalg.norm
    lim = cond * 1.1e-4 * nrm(ref_c) + eps * nrm(np.linalg.inv(G), 2) * 1e-6 * prob.a.max() * np.sqrt(ell)
    print(f"ell {ell} {basis}: cond(G) {cond:.3e}, direct vs oracle {nrm(c0 - ref_c) / nrm(ref_c):.3e} rel "
          f"(bound {lim / nrm(ref_c):.3e})", flush=True)
    assert nrm(c0 - ref_c) <= lim
    for solver, name in ((sk.NEWTON_CG, "CG"), (sk.NEWTON_SCHULZ, "Newton-Schulz")):
        c, ok, it = sk.newton_coef(ctx, gp, eps, fd, Vd, solver)
        d = np.abs(c - c0).max() / scale
        print(f"  {name}: {it} iterations, vs direct {d:.3e} rel, vs oracle "
              f"{np.abs(c - ref_c).max() / scale:.3e} rel", flush=True)
        assert ok and 0 < it
        # the same FP64 system: agreement to the solver's tolerance times cond
        assert d <= 1e-12 * cond * 100 + 1e-13
        assert nrm(c - ref_c) <= lim


def test_rank_deficient_basis(sk, ctx):
    """A basis with a repeated column makes G exactly singular (two equal
    rows, formed by the same FP32 operations) while the system stays
    consistent.  The elimination meets a zero pivot and Newton-Schulz
    cannot drive ||I - G^ X|| below 1: both refuse the step.  CG on a
    consistent positive semi-definite system converges to a solution on the
    span, and its step Delta f = V c equals the direct step of the basis
    without the repeated column (the Newton step depends on span V only)."""
    prob = W.gmm_vs_uniform(300, 320, seed=32)
    C = fp32_sqeuclid(prob.x, prob.y).astype(np.float64)
    eps = 0.05
    r = O.sinkhorn(C, prob.a, prob.b, eps, tol=1e-3, max_iter=5000)
    ref = O.sinkhorn(C, prob.a, prob.b, eps, tol=1e-12, max_iter=200000)
    V5, _ = O.spectral_basis(ref.f, ref.g, C, prob.a, prob.b, eps, 5, method="dense")
    V6 = np.ascontiguousarray(np.column_stack([V5, V5[:, 0]]))
    gp = sk.Problem(a=to_dev(prob.a), b=to_dev(prob.b), x=to_dev(prob.x), y=to_dev(prob.y))
    fd = to_dev(r.f)
    c5, ok5, _ = sk.newton_coef(ctx, gp, eps, fd, to_dev(np.ascontiguousarray(V5)), sk.NEWTON_DIRECT)
    assert ok5
    d5 = V5 @ c5
    _, ok, _ = sk.newton_coef(ctx, gp, eps, fd, to_dev(V6), sk.NEWTON_DIRECT)
    print("direct on the repeated column: ok", ok, flush=True)
    assert not ok
    _, ok, it = sk.newton_coef(ctx, gp, eps, fd, to_dev(V6), sk.NEWTON_SCHULZ)
    print("Newton-Schulz on the repeated column: ok", ok, "iterations", it, flush=True)
    assert not ok
    c6, ok, it = sk.newton_coef(ctx, gp, eps, fd, to_dev(V6), sk.NEWTON_CG)
    d6 = V6 @ c6
    rel = np.abs(d6 - d5).max() / np.abs(d5).max()
    print(f"CG on the repeated column: ok {ok}, {it} iterations, step vs the 5-column step {rel:.3e} rel", flush=True)
    assert ok and rel <= 1e-8


@pytest.mark.parametrize("ell", [16, 30])
def test_schedule_with_each_newton_solver_reaches_the_oracle_optimum(sk, ctx, ell):
    prob = W.gmm_vs_uniform(900, 1000, seed=33)
    ladder = [1e-1, 5e-2, 2.5e-2, 1.25e-2, 6.25e-3]
    C = fp32_sqeuclid(prob.x, prob.y).astype(np.float64)
    fo, go, _ = O.solve_schedule(C, prob.a, prob.b, ladder, 1e-10, 200000)
    gp = sk.Problem(a=to_dev(prob.a), b=to_dev(prob.b), x=to_dev(prob.x), y=to_dev(prob.y))
    its = {}
    for solver in (sk.NEWTON_DIRECT, sk.NEWTON_CG, sk.NEWTON_SCHULZ):
        f, g, res = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=100000, ell=ell, warm_mode=sk.WARM_SEQUENTIAL,
                             newton_solver=solver)
        its[solver] = [s["iters"] for s in res["stages"]]
        acc = [s["newton_accepted"] for s in res["stages"]]
        e = e_pot(f.cpu().numpy(), g.cpu().numpy(), fo, go, C)
        print(f"solver {solver}: iters {its[solver]} accepted {acc} e_pot {e:.2e}", flush=True)
        assert res["status"] == 0 and res["marginal_err"] < 1e-6
        assert e <= 1e-5
        assert sum(acc) > 0
    # the same steps up to the last bits of the coefficients: the counts agree
    for solver in (sk.NEWTON_CG, sk.NEWTON_SCHULZ):
        for a, b in zip(its[solver], its[sk.NEWTON_DIRECT]):
            assert abs(a - b) <= 1 + b // 10
