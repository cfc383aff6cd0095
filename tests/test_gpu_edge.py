"""GPU edge cases of the solver: degenerate shapes (a single point on one
side, 2 x 2, transposed tiny problems), a stored cost with padded rows,
the matrix-core cost forced at small d, the iteration cap, run-to-run
determinism, and the argument validation of the C ABI (every rejected
input returns EINVAL without touching the device state)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests._helpers import bf16_cost_model, e_pot, fp32_sqeuclid, to_dev

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


def _pts(n, m, d, seed):
    rng = np.random.default_rng(seed)
    x = rng.random((n, d)).astype(np.float32)
    y = rng.random((m, d)).astype(np.float32)
    a = rng.dirichlet(np.full(n, 3.0)) if n > 1 else np.ones(1)
    b = rng.dirichlet(np.full(m, 3.0)) if m > 1 else np.ones(1)
    return x, y, a, b


@pytest.mark.parametrize("n,m", [(1, 5), (5, 1), (1, 1), (2, 2), (3, 130), (130, 3), (257, 2)])
def test_degenerate_shapes_match_oracle(sk, ctx, n, m):
    x, y, a, b = _pts(n, m, 2, seed=n * 1000 + m)
    gp = sk.Problem(a=to_dev(a), b=to_dev(b), x=to_dev(x), y=to_dev(y))
    ladder = [2e-1, 1e-1, 5e-2]
    print(f"case n={n} m={m}", flush=True)
    # With one or two points on a side a single term dominates each FP32
    # log-sum-exp.  The sweep exponent folds the low half of the offset
    # potential into the FP32 argument of exp2 (3 instructions per element
    # instead of 7), so that term is exp2 of a small non-zero argument and
    # not exactly 1: its rounding (relative 2^-24) stays in the output, a
    # floor of about eps * 2^-24 per potential and about 2 * 2^-24 = 1.2e-7
    # in the L1 marginal error (a 1 x 1 solve at eps = 0.2 stops at
    # 1.19e-7).  The tolerance sits above that floor; the solver's 1e-6
    # target is not affected.
    tol = 3e-7
    f, g, res = sk.solve(ctx, gp, ladder, tol=tol, max_iter=20000)
    print("status", res["status"], "marginal", res["marginal_err"], flush=True)
    assert res["status"] == 0 and res["marginal_err"] < tol
    C = fp32_sqeuclid(x, y).astype(np.float64)
    fo, go, _ = O.solve_schedule(C, a, b, ladder, 1e-11, 200000)
    fo, go = O.normalize_gauge(fo, go, a, b)
    # gauge-invariant comparison; the cost range is 0 for a single pair
    df = f.cpu().numpy() - fo
    dg = g.cpu().numpy() - go
    dev = max(abs(df.max() + dg.max()), abs(df.min() + dg.min()))
    assert dev <= 1e-5 * max(C.max() - C.min(), ladder[-1])
    # the reported gauge <f,a> = <g,b>
    assert abs(f.cpu().numpy() @ a - g.cpu().numpy() @ b) <= 1e-9 * (1 + abs(f.cpu().numpy() @ a))


def test_stored_cost_with_padded_rows(sk, ctx):
    n, m, ldc = 300, 411, 448
    x, y, a, b = _pts(n, m, 2, seed=9)
    C = O.sqeuclid_cost(x.astype(np.float64), y.astype(np.float64)).astype(np.float32)
    Cpad = np.full((n, ldc), 7.0, np.float32)
    Cpad[:, :m] = C
    Ct = to_dev(Cpad)
    gp = sk.Problem(a=to_dev(a), b=to_dev(b), C=Ct, ldc=ldc)
    gpd = sk.Problem(a=to_dev(a), b=to_dev(b), C=to_dev(C))
    f1, g1, r1 = sk.solve(ctx, gp, [1e-1, 5e-2, 2.5e-2], tol=1e-6, max_iter=20000, ell=8, warm_mode=sk.WARM_SEQUENTIAL)
    f2, g2, r2 = sk.solve(ctx, gpd, [1e-1, 5e-2, 2.5e-2], tol=1e-6, max_iter=20000, ell=8,
                          warm_mode=sk.WARM_SEQUENTIAL)
    assert r1["status"] == 0 and r2["status"] == 0
    assert e_pot(f1.cpu().numpy(), g1.cpu().numpy(), f2.cpu().numpy(), g2.cpu().numpy(), C.astype(np.float64)) < 1e-6


@pytest.mark.parametrize("d", [1, 5])
def test_forced_matrix_core_cost_at_small_d(sk, ctx, d):
    n, m, eps = 300, 260, 0.05
    x, y, a, b = _pts(n, m, d, seed=d)
    Cm, bound = bf16_cost_model(x, y, 1.0, True)
    gp = sk.Problem(a=to_dev(a), b=to_dev(b), x=to_dev(x), y=to_dev(y), xterm=sk.XTERM_BF16X3)
    f = 0.1 * np.random.default_rng(1).standard_normal(n)
    g_gpu = sk.c_transform_col(ctx, gp, eps, to_dev(f))[0].cpu().numpy()
    g_ref = O.c_transform_col(f, Cm, a, eps)
    assert np.abs(g_gpu - g_ref).max() <= bound.max() + 64 * 2.0 ** -24 * eps + 1e-12


def test_iteration_cap_reports_not_converged(sk, ctx):
    prob = W.uniform_square(200, 240, seed=3)
    gp = sk.Problem(a=to_dev(prob.a), b=to_dev(prob.b), x=to_dev(prob.x), y=to_dev(prob.y))
    f, g, res = sk.solve(ctx, gp, [1e-3], tol=1e-9, max_iter=5)
    assert res["status"] == sk.NOT_CONVERGED
    assert res["stages"][0]["iters"] == 5
    assert np.all(np.isfinite(f.cpu().numpy())) and np.all(np.isfinite(g.cpu().numpy()))
    assert res["marginal_err"] > 1e-9


def test_solves_are_deterministic(sk, ctx):
    prob = W.gmm_vs_uniform(700, seed=2)
    gp = sk.Problem(a=to_dev(prob.a), b=to_dev(prob.b), x=to_dev(prob.x), y=to_dev(prob.y))
    runs = [sk.solve(ctx, gp, [1e-1, 5e-2, 2.5e-2, 1.25e-2], tol=1e-6, max_iter=20000, ell=12,
                     warm_mode=sk.WARM_SEQUENTIAL) for _ in range(2)]
    (f1, g1, r1), (f2, g2, r2) = runs
    assert np.array_equal(f1.cpu().numpy(), f2.cpu().numpy())
    assert np.array_equal(g1.cpu().numpy(), g2.cpu().numpy())
    assert [s["iters"] for s in r1["stages"]] == [s["iters"] for s in r2["stages"]]


def test_argument_validation(sk, ctx):
    import torch
    n, m = 50, 60
    x, y, a, b = _pts(n, m, 2, seed=4)
    ok = dict(a=to_dev(a), b=to_dev(b), x=to_dev(x), y=to_dev(y))

    def rejects(kw=None, eps=(0.1,), **opts):
        p = sk.Problem(**(kw or ok))
        with pytest.raises(sk.SknrError) as e:
            sk.solve(ctx, p, list(eps), **opts)
        assert e.value.status == sk.EINVAL, e.value
        return str(e.value)

    bad_a = a.copy()
    bad_a[3] = -bad_a[3]
    print(rejects(dict(ok, a=to_dev(bad_a))), flush=True)                # negative weight
    print(rejects(dict(ok, b=to_dev(b * 1.01))), flush=True)             # weights not summing to 1
    xn = x.copy()
    xn[7, 1] = np.nan
    print(rejects(dict(ok, x=to_dev(xn))), flush=True)                   # non-finite point
    print(rejects(eps=(0.0,)), flush=True)                               # eps <= 0
    print(rejects(eps=(0.1, -1.0)), flush=True)                          # a bad stage
    print(rejects(tol=0.0), flush=True)                                  # tol <= 0
    print(rejects(max_iter=0), flush=True)
    print(rejects(ell=40), flush=True)                                   # ell > 32
    print(rejects(ell=5, warm_mode=7), flush=True)                       # unknown warm mode
    xs, ys, as_, bs = _pts(12, 15, 2, seed=6)
    small = dict(a=to_dev(as_), b=to_dev(bs), x=to_dev(xs), y=to_dev(ys))
    print(rejects(small, ell=12), flush=True)                            # ell >= min(n, m)
    print(rejects(dict(ok, cost_scale=-1.0)), flush=True)
    print(rejects(dict(ok, xterm=9)), flush=True)                        # unknown cross-term mode
    Cn = torch.ones(n, m, dtype=torch.float32, device="cuda")
    Cn[2, 3] = float("inf")
    print(rejects(dict(a=ok["a"], b=ok["b"], C=Cn)), flush=True)         # non-finite cost
    print(rejects(dict(a=ok["a"], b=ok["b"], C=torch.ones(n, m, device="cuda"), ldc=m - 1)), flush=True)
    print(rejects(ell=5, warm_mode=sk.WARM_SEQUENTIAL, nr_switch_iters=-1), flush=True)
    print(rejects(ell=5, warm_mode=sk.WARM_STATIC, eps_prime=0.2, nr_switch_iters=10), flush=True)
    # the context still works afterwards
    f, g, res = sk.solve(ctx, sk.Problem(**ok), [0.1], tol=1e-6)
    assert res["status"] == 0
