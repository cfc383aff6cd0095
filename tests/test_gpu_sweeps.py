"""GPU parity of single steps of the path against the FP64 oracle.

Each test runs one entry point of the C ABI (through the thin binding) on
seeded inputs spanning several tiles with ragged tails, and compares with
the oracle element by element.  Tolerances are derived from the FP32
arithmetic of the kernels (u = 2^-24):
  * stored cost: the kernels read the same FP32 C as the oracle; a
    c-transform output is then exact up to the compensated FP32
    accumulation, |d out| <= 64 u eps + 1e-12 |out|;
  * cost from points: the kernels use the FP32 cost C~, |C~ - C| <=
    2 u |C|, which moves a c-transform by at most max |C~ - C|.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests._helpers import U32, e_pot, fp32_sqeuclid, gpu_problem, to_dev

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


def _stored_problem(n, m, seed):
    rng = np.random.default_rng(seed)
    x = rng.random((n, 2))
    y = rng.random((m, 2))
    C = O.sqeuclid_cost(x, y).astype(np.float32)
    a = rng.dirichlet(np.full(n, 4.0))
    b = rng.dirichlet(np.full(m, 4.0))
    return W.Problem(a=a, b=b, C=C, x=x.astype(np.float32), y=y.astype(np.float32))


@pytest.mark.parametrize("n,m", [(700, 1300), (333, 1299), (1500, 257)])
@pytest.mark.parametrize("eps", [1e-1, 1e-2, 1e-3])
def test_c_transforms_stored_cost(sk, ctx, n, m, eps):
    prob = _stored_problem(n, m, seed=n + m)
    C = prob.C.astype(np.float64)
    gp = gpu_problem(prob, stored=True)
    rng = np.random.default_rng(1)
    f = 0.3 * rng.standard_normal(n)
    g_ref = O.c_transform_col(f, C, prob.a, eps)
    # a previous g near the new one (the regime of the convergence test)
    g_prev = g_ref + 0.5 * eps * rng.standard_normal(m)
    print(f"case stored n={n} m={m} eps={eps}", flush=True)
    g_gpu, err, gdot = sk.c_transform_col(ctx, gp, eps, to_dev(f), to_dev(g_prev))
    dg = np.abs(g_gpu.cpu().numpy() - g_ref)
    tol = 64 * U32 * eps + 1e-12 * np.abs(g_ref).max()
    print(f"  col max|dg|={dg.max():.3e} tol={tol:.3e}", flush=True)
    assert dg.max() <= tol
    # marginal error of (f, g_prev) with g_prev's own coupling: the column marginal of pi(f,g_prev)
    # equals b*exp((g_prev - T_c f)/eps) (F6); compare with the oracle's direct sum
    _, cols = O.marginals(f, g_prev, C, prob.a, prob.b, eps)
    err_ref = np.abs(cols - prob.b).sum()
    # FP32 expm1 of an argument (g_prev - g)/eps = O(1) computed from double-floats
    assert err == pytest.approx(err_ref, rel=1e-6, abs=1e-12)
    # <g,b> is computed from the returned g, so it carries g's error
    assert abs(gdot - g_ref @ prob.b) <= 64 * U32 * eps + 1e-12
    f_gpu = sk.c_transform_row(ctx, gp, eps, to_dev(g_prev))
    f_ref = O.c_transform_row(g_prev, C, prob.b, eps)
    df = np.abs(f_gpu.cpu().numpy() - f_ref)
    tol = 64 * U32 * eps + 1e-12 * np.abs(f_ref).max()
    print(f"  row max|df|={df.max():.3e} tol={tol:.3e}", flush=True)
    assert df.max() <= tol


@pytest.mark.parametrize("n,m,d", [(1000, 1500, 2), (777, 513, 3), (300, 2100, 5), (257, 300, 12), (300, 700, 40),
                                   (200, 333, 70)])
@pytest.mark.parametrize("eps", [1e-1, 1e-3])
def test_c_transforms_points(sk, ctx, n, m, d, eps):
    rng = np.random.default_rng(d * 100 + n)
    x = rng.random((n, d)).astype(np.float32)
    y = rng.random((m, d)).astype(np.float32)
    a = rng.dirichlet(np.full(n, 4.0))
    b = rng.dirichlet(np.full(m, 4.0))
    prob = W.Problem(a=a, b=b, x=x, y=y, cost_scale=1.0 / d if d == 3 else 1.0)
    Ct = fp32_sqeuclid(x, y, prob.cost_scale).astype(np.float64)   # the GPU's FP32 cost
    C = O.sqeuclid_cost(x, y, prob.cost_scale)                      # exact cost
    gp = gpu_problem(prob)
    gp.xterm = sk.XTERM_FP32  # the FP32 cost modelled above (AUTO would pick bf16 for d >= 16)
    f = 0.2 * rng.standard_normal(n)
    print(f"case points n={n} m={m} d={d} eps={eps}", flush=True)
    g_gpu, _, _ = sk.c_transform_col(ctx, gp, eps, to_dev(f))
    g_gpu = g_gpu.cpu().numpy()
    d_model = np.abs(g_gpu - O.c_transform_col(f, Ct, a, eps)).max()
    d_exact = np.abs(g_gpu - O.c_transform_col(f, C, a, eps)).max()
    print(f"  col vs FP32-cost oracle {d_model:.3e}, vs exact cost {d_exact:.3e}", flush=True)
    assert d_model <= 64 * U32 * eps + 1e-12 * np.abs(g_gpu).max()
    assert d_exact <= 4 * U32 * np.abs(C).max() + 64 * U32 * eps
    g = 0.2 * rng.standard_normal(m)
    f_gpu = sk.c_transform_row(ctx, gp, eps, to_dev(g)).cpu().numpy()
    d_model = np.abs(f_gpu - O.c_transform_row(g, Ct, b, eps)).max()
    print(f"  row vs FP32-cost oracle {d_model:.3e}", flush=True)
    assert d_model <= 64 * U32 * eps + 1e-12 * np.abs(f_gpu).max()


def test_evaluate_fp64(sk, ctx):
    prob = _stored_problem(513, 900, seed=4)
    C = prob.C.astype(np.float64)
    eps = 0.05
    r = O.sinkhorn(C, prob.a, prob.b, eps, tol=1e-6, max_iter=5000)
    gp = gpu_problem(prob, stored=True)
    ev = sk.evaluate(ctx, gp, eps, to_dev(r.f), to_dev(r.g))
    rows, cols = O.marginals(r.f, r.g, C, prob.a, prob.b, eps)
    assert ev["row_err"] == pytest.approx(np.abs(rows - prob.a).sum(), rel=1e-9, abs=1e-15)
    assert ev["col_err"] == pytest.approx(np.abs(cols - prob.b).sum(), rel=1e-9, abs=1e-15)
    assert ev["transport_cost"] == pytest.approx(O.transport_cost(r.f, r.g, C, prob.a, prob.b, eps), rel=1e-12)
    assert ev["dual_value"] == pytest.approx(O.dual_value(r.f, r.g, C, prob.a, prob.b, eps), rel=1e-12)
    assert ev["primal_value"] == pytest.approx(O.primal_value(r.f, r.g, C, prob.a, prob.b, eps), rel=1e-12)


def test_coupling(sk, ctx):
    prob = _stored_problem(130, 70, seed=5)
    rng = np.random.default_rng(2)
    f, g = 0.1 * rng.standard_normal(130), 0.1 * rng.standard_normal(70)
    P = sk.coupling(ctx, gpu_problem(prob, stored=True), 0.1, to_dev(f), to_dev(g)).cpu().numpy()
    ref = O.coupling(f, g, prob.C.astype(np.float64), prob.a, prob.b, 0.1)
    assert np.allclose(P, ref, rtol=1e-6, atol=0)


def test_projected_system_matches_oracle(sk, ctx):
    """Semi-dual value, projected gradient and Hessian (G = -eps V^T H V)."""
    prob = _stored_problem(400, 650, seed=6)
    C = prob.C.astype(np.float64)
    eps = 0.02
    rng = np.random.default_rng(3)
    r = O.sinkhorn(C, prob.a, prob.b, eps, tol=1e-4, max_iter=2000)
    f = r.f
    V = np.linalg.qr(rng.standard_normal((400, 5)))[0]
    G, grad, q = sk.projected_system(ctx, gpu_problem(prob, stored=True), eps, to_dev(f), to_dev(V))
    step = O.projected_newton(f, C, prob.a, prob.b, eps, V)
    G_ref = -eps * step["hess"]
    print("G rel err", np.abs(G - G_ref).max() / np.abs(G_ref).max(), "grad", np.abs(grad - step["grad"]).max(),
          flush=True)
    assert np.allclose(G, G_ref, rtol=0, atol=1e-5 * np.abs(G_ref).max())
    assert np.allclose(grad, step["grad"], rtol=0, atol=1e-6 * np.abs(prob.a).max() + 1e-4 * np.abs(step["grad"]).max())
    # Q^semi uses the GPU's T_c(f), accurate to ~64 u eps
    assert abs(q - O.semidual_value(f, C, prob.a, prob.b, eps)) <= 64 * U32 * eps


@pytest.mark.parametrize("n,m,d,ell,scale", [(400, 650, 2, 5, 1.0), (1100, 900, 2, 16, 1.0),
                                             (700, 1333, 3, 32, 0.37), (1300, 517, 3, 12, 1.0)])
def test_projected_system_points(sk, ctx, n, m, d, ell, scale):
    """The projected system on a cost built from points (the weighted sweep
    accumulates W = P~^T V on FP32 matrix cores, in splits of several
    hundred rows with a ragged last split) against the oracle on the FP32
    cost model of the same points."""
    rng = np.random.default_rng(n + m + d)
    x = rng.random((n, d)).astype(np.float32)
    y = rng.random((m, d)).astype(np.float32)
    a = rng.dirichlet(np.full(n, 4.0))
    b = rng.dirichlet(np.full(m, 4.0))
    C = fp32_sqeuclid(x, y, scale).astype(np.float64)
    eps = 0.02
    r = O.sinkhorn(C, a, b, eps, tol=1e-4, max_iter=4000)
    V = np.linalg.qr(rng.standard_normal((n, ell)))[0]
    gp = sk.Problem(a=to_dev(a), b=to_dev(b), x=to_dev(x), y=to_dev(y), cost_scale=scale)
    print(f"case n={n} m={m} d={d} ell={ell} scale={scale}", flush=True)
    G, grad, q = sk.projected_system(ctx, gp, eps, to_dev(r.f), to_dev(V))
    step = O.projected_newton(r.f, C, a, b, eps, V)
    G_ref = -eps * step["hess"]
    print("G rel err", np.abs(G - G_ref).max() / np.abs(G_ref).max(), "grad", np.abs(grad - step["grad"]).max(),
          flush=True)
    assert np.allclose(G, G_ref, rtol=0, atol=1e-5 * np.abs(G_ref).max())
    assert np.allclose(grad, step["grad"], rtol=0, atol=1e-6 * np.abs(a).max() + 1e-4 * np.abs(step["grad"]).max())
    assert abs(q - O.semidual_value(r.f, C, a, b, eps)) <= 64 * U32 * eps


def test_newton_step_matches_oracle(sk, ctx):
    prob = _stored_problem(300, 420, seed=7)
    C = prob.C.astype(np.float64)
    eps = 0.03
    r = O.sinkhorn(C, prob.a, prob.b, eps, tol=1e-3, max_iter=2000)
    ref = O.sinkhorn(C, prob.a, prob.b, eps, tol=1e-12, max_iter=100000)
    V, _ = O.spectral_basis(ref.f, ref.g, C, prob.a, prob.b, eps, 6, method="dense")
    fd = to_dev(r.f.copy())
    acc, q0, q1 = sk.newton_step(ctx, gpu_problem(prob, stored=True), eps, fd, to_dev(V))
    step = O.projected_newton(r.f, C, prob.a, prob.b, eps, V)
    q1_ref = O.semidual_value(r.f + step["delta"], C, prob.a, prob.b, eps)
    q0_ref = O.semidual_value(r.f, C, prob.a, prob.b, eps)
    assert acc == (q1_ref > q0_ref)
    assert abs(q0 - q0_ref) <= 64 * U32 * eps
    assert abs(q1 - q1_ref) <= 64 * U32 * eps + 1e-6 * abs(q1_ref - q0_ref)
    if acc:
        assert np.abs(fd.cpu().numpy() - (r.f + step["delta"])).max() < 1e-5 * np.abs(step["delta"]).max() + 1e-9


def test_newton_step_drops_massless_basis_columns(sk, ctx):
    """A basis with columns that carry no mass (one exactly zero, one at
    1e-9, as the warm start leaves where the spectrum of M lies below FP32
    resolution) gives the Newton step on the span of the other columns,
    where the plain Cholesky of the full projected Hessian would fail and
    lose the step."""
    prob = _stored_problem(300, 420, seed=7)
    C = prob.C.astype(np.float64)
    eps = 0.03
    r = O.sinkhorn(C, prob.a, prob.b, eps, tol=1e-3, max_iter=2000)
    ref = O.sinkhorn(C, prob.a, prob.b, eps, tol=1e-12, max_iter=100000)
    V, _ = O.spectral_basis(ref.f, ref.g, C, prob.a, prob.b, eps, 6, method="dense")
    noise = 1e-9 * np.random.default_rng(3).standard_normal(V.shape[0])
    Vaug = np.column_stack([V[:, 0], np.zeros(V.shape[0]), V[:, 1:4], noise, V[:, 4:]])
    assert O.projected_newton(r.f, C, prob.a, prob.b, eps, V)["ok"]
    fd = to_dev(r.f.copy())
    print("case newton_step massless columns 300x420", flush=True)
    acc, q0, q1 = sk.newton_step(ctx, gpu_problem(prob, stored=True), eps, fd, to_dev(Vaug))
    step = O.projected_newton(r.f, C, prob.a, prob.b, eps, V)
    q1_ref = O.semidual_value(r.f + step["delta"], C, prob.a, prob.b, eps)
    q0_ref = O.semidual_value(r.f, C, prob.a, prob.b, eps)
    assert q1_ref > q0_ref
    assert acc
    assert abs(q1 - q1_ref) <= 64 * U32 * eps + 1e-6 * abs(q1_ref - q0_ref)
    assert np.abs(fd.cpu().numpy() - (r.f + step["delta"])).max() < 1e-5 * np.abs(step["delta"]).max() + 1e-9


def _principal_cosines(V1, V2, a):
    sa = np.sqrt(a)[:, None]
    Q1, _ = np.linalg.qr(sa * V1)
    Q2, _ = np.linalg.qr(sa * V2)
    return np.linalg.svd(Q1.T @ Q2, compute_uv=False)


@pytest.mark.parametrize("ell", [5, 12])
def test_spectral_basis_matches_oracle(sk, ctx, ell):
    """Warm-start basis (Sec. 4): Ritz values rho_k and the span of the top
    ell non-constant eigenvectors of M against the oracle's dense eigh,
    compared by principal angles in L2(a) where the spectral gap is clear."""
    prob = W.uniform_square(600, 700, seed=21)
    C32 = O.sqeuclid_cost(prob.x, prob.y).astype(np.float32)
    C = C32.astype(np.float64)
    eps = 0.05
    ref = O.sinkhorn(C, prob.a, prob.b, eps, tol=1e-11, max_iter=100000)
    Vr, rho_r = O.spectral_basis(ref.f, ref.g, C, prob.a, prob.b, eps, ell + 1, method="dense")
    V, rho, it = sk.spectral_basis(ctx, gpu_problem(prob, stored=True, C32=C32), eps, to_dev(ref.f), ell,
                                   oversample=8, max_iter=300, tol=1e-10)
    V = V.cpu().numpy()
    print("rho gpu", rho[:6], "oracle", rho_r[:6], "iters", it, flush=True)
    assert rho[0] == 1.0
    assert np.allclose(rho[1:], rho_r[1:ell + 1], atol=1e-6)
    # orthonormal in L2(a), orthogonal to the constants
    assert np.allclose(V.T @ (prob.a[:, None] * V), np.eye(ell), atol=1e-5)
    assert np.abs(prob.a @ V).max() < 1e-5
    gap = rho_r[ell] - rho_r[ell + 1]
    if gap > 1e-3:
        cos = _principal_cosines(V, Vr[:, :ell], prob.a)
        print("min cos", cos.min(), flush=True)
        assert cos.min() > 1 - 1e-4


def test_spectral_basis_drops_unresolved_modes(sk, ctx):
    """At large eps most of the top-30 eigenvalues of M lie below what the
    FP32 products resolve (here rho_7^2 ~ 1e-14 at eps = 1).  The basis
    returns them as exact zero columns; the other columns are orthonormal
    in L2(a) and contain the oracle's resolved modes (dense eigh), with
    their rho."""
    tr = W.serving_trace(n_requests=64, rate=1.0, seed=4)
    p = sorted(tr, key=lambda r: r.problem.a.shape[0] * r.problem.b.shape[0])[32].problem
    C = fp32_sqeuclid(p.x, p.y, p.cost_scale).astype(np.float64)
    eps, ell = 1.0, 30
    ref = O.sinkhorn(C, p.a, p.b, eps, tol=1e-11, max_iter=100000)
    Vr, rho_r = O.spectral_basis(ref.f, ref.g, C, p.a, p.b, eps, ell + 1, method="dense")
    print("case spectral basis 484x1447 eps=1 l=30", flush=True)
    V, rho, it = sk.spectral_basis(ctx, gpu_problem(p), eps, to_dev(ref.f), ell, oversample=8, max_iter=300,
                                   tol=1e-8)
    V = V.cpu().numpy()
    nz = np.abs(V).max(axis=0) > 0
    k = int(nz.sum())
    print("kept", k, "rho gpu", rho[:k + 2], "oracle", rho_r[:k + 2], "iters", it, flush=True)
    assert 0 < k < ell
    assert np.all(nz[:k]) and not np.any(nz[k:])          # zero columns sort last
    assert np.all(rho[k + 1:] == 0.0)
    Vk = V[:, :k]
    assert np.allclose(Vk.T @ (p.a[:, None] * Vk), np.eye(k), atol=1e-5)
    assert np.abs(p.a @ Vk).max() < 1e-5
    resolved = int(np.sum(rho_r[1:] ** 2 >= 1e-3 * rho_r[1] ** 2))
    assert 1 <= resolved <= k
    assert np.allclose(rho[1:resolved + 1], rho_r[1:resolved + 1], atol=1e-5)
    cos = _principal_cosines(Vk, Vr[:, :resolved], p.a)
    print("resolved", resolved, "min cos", cos.min(), flush=True)
    assert cos[:resolved].min() > 1 - 1e-4


def test_spectral_basis_points(sk, ctx):
    """The warm-start basis on a cost built from points (its products run
    the 32-wide weighted sweeps in both orientations) against the oracle's
    dense eigh on the FP32 cost model."""
    prob = W.uniform_square(900, 700, seed=22)
    ell = 12
    C = fp32_sqeuclid(prob.x, prob.y, prob.cost_scale).astype(np.float64)
    eps = 0.05
    ref = O.sinkhorn(C, prob.a, prob.b, eps, tol=1e-11, max_iter=100000)
    Vr, rho_r = O.spectral_basis(ref.f, ref.g, C, prob.a, prob.b, eps, ell + 1, method="dense")
    V, rho, it = sk.spectral_basis(ctx, gpu_problem(prob), eps, to_dev(ref.f), ell, oversample=8, max_iter=300,
                                   tol=1e-10)
    V = V.cpu().numpy()
    print("rho gpu", rho[:6], "oracle", rho_r[:6], "iters", it, flush=True)
    assert rho[0] == 1.0
    assert np.allclose(rho[1:], rho_r[1:ell + 1], atol=1e-6)
    assert np.allclose(V.T @ (prob.a[:, None] * V), np.eye(ell), atol=1e-5)
    assert np.abs(prob.a @ V).max() < 1e-5
    gap = rho_r[ell] - rho_r[ell + 1]
    if gap > 1e-3:
        cos = _principal_cosines(V, Vr[:, :ell], prob.a)
        print("min cos", cos.min(), flush=True)
        assert cos.min() > 1 - 1e-4
