"""GPU parity of the W_eps gradients (sknr_gradient) against the FP64 oracle.

At given potentials (f, g) the library returns the partial derivatives of
Q_eps (eq. def_Q) with respect to x, y, a, b (oracle.dual_partials), which
at the optimum are the gradients of W_eps.  The weighted sums sum_j pi_ij
y_j run in the sweep kernels (32 coordinates per pass), so the cases span
the VALU-cost matrix-core instance (d = 2, 3), the streaming kernel (d = 5)
and two passes (d = 40, FP32 cost).  Tolerances: the coupling of the FP32
cost is exact up to the FP32 exponent (relative ~1e-6 per element), the
sums and the final difference r x - sum pi y add FP32 rounding relative to
|r x|.
"""
import numpy as np
import pytest

import oracle as O
from tests._helpers import fp32_sqeuclid, to_dev

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


def _case(n, m, d, seed):
    rng = np.random.default_rng(seed)
    x = rng.random((n, d)).astype(np.float32)
    y = (rng.random((m, d)) + 0.2).astype(np.float32)
    a = rng.dirichlet(np.full(n, 3.0))
    b = rng.dirichlet(np.full(m, 3.0))
    return x, y, a, b


@pytest.mark.parametrize("n,m,d,scale,eps", [(300, 450, 2, 1.0, 0.05), (517, 260, 3, 0.5, 0.02),
                                             (280, 333, 5, 1.0 / 5, 0.05), (260, 300, 40, 1.0 / 40, 0.01)])
def test_gradient_matches_oracle_partials(sk, ctx, n, m, d, scale, eps):
    x, y, a, b = _case(n, m, d, seed=n + d)
    C = fp32_sqeuclid(x, y, scale).astype(np.float64)
    r = O.sinkhorn(C, a, b, eps, tol=1e-3, max_iter=5000)  # near, not at, the optimum
    gp = sk.Problem(a=to_dev(a), b=to_dev(b), x=to_dev(x), y=to_dev(y), cost_scale=scale, xterm=sk.XTERM_FP32)
    print(f"case n={n} m={m} d={d} s={scale} eps={eps}", flush=True)
    gr = {k: v.cpu().numpy() for k, v in sk.gradient(ctx, gp, eps, to_dev(r.f), to_dev(r.g)).items()}
    # oracle partials on the same FP32 cost (dual_partials rebuilds it in FP64 from x, y)
    P = O.coupling(r.f, r.g, C, a, b, eps)
    rr, cc = P.sum(1), P.sum(0)
    xo, yo = x.astype(np.float64), y.astype(np.float64)
    ref = {"x": 2 * scale * (rr[:, None] * xo - P @ yo), "y": 2 * scale * (cc[:, None] * yo - P.T @ xo),
           "a": r.f - eps * rr / a, "b": r.g - eps * cc / b}
    for k in ("x", "y"):
        mag = 2 * scale * (np.abs((rr if k == "x" else cc)[:, None] * (xo if k == "x" else yo)).max()
                           + np.abs(P).sum(1 if k == "x" else 0).max() * np.abs(yo if k == "x" else xo).max())
        err = np.abs(gr[k] - ref[k]).max()
        print(f"  grad_{k}: max err {err:.3e} (scale {mag:.3e})", flush=True)
        assert err <= 1e-5 * mag
    for k, w in (("a", a), ("b", b)):
        err = np.abs(gr[k] - ref[k]).max()
        print(f"  grad_{k}: max err {err:.3e}", flush=True)
        assert err <= 1e-5 * eps * (1 + np.abs((rr / a) if k == "a" else (cc / b)).max()) + 1e-12 * np.abs(ref[k]).max()


def test_gradient_at_the_optimum_is_the_envelope_gradient(sk, ctx):
    """At a converged solve the library's gradient equals the oracle's
    envelope gradient at the oracle's optimum (same FP32 cost)."""
    x, y, a, b = _case(200, 240, 2, seed=5)
    eps = 0.03
    gp = sk.Problem(a=to_dev(a), b=to_dev(b), x=to_dev(x), y=to_dev(y))
    f, g, res = sk.solve(ctx, gp, [0.2, 0.1, 0.05, eps], tol=1e-7, max_iter=100000, ell=8,
                         warm_mode=sk.WARM_SEQUENTIAL)
    gr = sk.gradient(ctx, gp, eps, f, g, a=False, b=False)
    C = fp32_sqeuclid(x, y).astype(np.float64)
    ro = O.sinkhorn(C, a, b, eps, tol=1e-13, max_iter=200000)
    P = O.coupling(ro.f, ro.g, C, a, b, eps)
    gx = 2 * (a[:, None] * x.astype(np.float64) - P @ y.astype(np.float64))
    err = np.abs(gr["x"].cpu().numpy() - gx).max()
    print("envelope grad_x err", err, "max", np.abs(gx).max(), flush=True)
    assert err <= 1e-4 * np.abs(gx).max()


def test_entropic_ot_loss_backward(sk, ctx):
    """entropic_ot_loss: backward against central differences of the loss
    (each side a full solve) and of the oracle's W_eps."""
    import torch
    x, y, a, b = _case(120, 150, 2, seed=9)
    eps = 0.05
    xt = to_dev(x).requires_grad_(True)
    yt, at, bt = to_dev(y), to_dev(a), to_dev(b)
    loss = sk.entropic_ot_loss(ctx, xt, yt, at, bt, [0.2, 0.1, eps], tol=1e-8)
    loss.backward()
    gx = xt.grad.cpu().numpy().astype(np.float64)
    h = 1e-3
    for (i, k) in [(0, 0), (17, 1), (99, 0)]:
        vals = []
        for sgn in (1, -1):
            xp = x.copy()
            xp[i, k] += sgn * h
            with torch.no_grad():
                vals.append(float(sk.entropic_ot_loss(ctx, to_dev(xp), yt, at, bt, [0.2, 0.1, eps], tol=1e-8)))
        fd = (vals[0] - vals[1]) / (np.float32(x[i, k] + h) - np.float32(x[i, k] - h))
        print(f"x[{i},{k}]: backward {gx[i, k]:.6e} fd {fd:.6e}", flush=True)
        assert gx[i, k] == pytest.approx(fd, rel=2e-3, abs=1e-6)
    # the loss is the oracle's W_eps
    C = fp32_sqeuclid(x, y).astype(np.float64)
    ro = O.sinkhorn(C, a, b, eps, tol=1e-13, max_iter=200000)
    assert float(loss.detach()) == pytest.approx(O.dual_value(ro.f, ro.g, C, a, b, eps), rel=1e-6)


def test_gradient_of_a_stored_cost_problem(sk, ctx):
    """Weights only; point gradients of a stored cost are an error."""
    x, y, a, b = _case(90, 70, 2, seed=2)
    C32 = fp32_sqeuclid(x, y)
    C = C32.astype(np.float64)
    eps = 0.05
    r = O.sinkhorn(C, a, b, eps, tol=1e-4, max_iter=5000)
    gp = sk.Problem(a=to_dev(a), b=to_dev(b), C=to_dev(C32))
    gr = sk.gradient(ctx, gp, eps, to_dev(r.f), to_dev(r.g), x=False, y=False)
    P = O.coupling(r.f, r.g, C, a, b, eps)
    assert np.allclose(gr["a"].cpu().numpy(), r.f - eps * P.sum(1) / a, rtol=0, atol=1e-6 * eps * 10)
    assert np.allclose(gr["b"].cpu().numpy(), r.g - eps * P.sum(0) / b, rtol=0, atol=1e-6 * eps * 10)
    # a point-gradient buffer for a stored cost: rejected by the library
    import ctypes
    import torch
    dummy = torch.empty((90, 2), dtype=torch.float64, device="cuda")
    fd, gd = to_dev(r.f), to_dev(r.g)
    ps = gp.c_struct()
    st = sk.lib.sknr_gradient(ctx.handle, ctypes.byref(ps), eps, ctypes.c_void_p(fd.data_ptr()),
                              ctypes.c_void_p(gd.data_ptr()), ctypes.c_void_p(dummy.data_ptr()), None, None, None,
                              None)
    assert st == sk.EINVAL


def test_gradient_matrix_core_cost_d64(sk, ctx):
    """The default cost for d >= 16 (three bf16 parts on matrix cores): the
    gradient against the oracle's formula on the modelled cost C_model
    (tests._helpers.bf16_cost_model), with the coupling's relative slack
    exp(bound / eps) - 1 from the model's per-element bound."""
    from tests._helpers import bf16_cost_model
    n, m, d, eps, scale = 240, 310, 64, 0.05, 1.0 / 64
    rng = np.random.default_rng(64)
    x = rng.standard_normal((n, d)).astype(np.float32)
    y = (rng.standard_normal((m, d)) + 0.3).astype(np.float32)
    a = rng.dirichlet(np.full(n, 3.0))
    b = rng.dirichlet(np.full(m, 3.0))
    Cm, bound = bf16_cost_model(x, y, scale, parts=3)
    r = O.sinkhorn(Cm, a, b, eps, tol=1e-4, max_iter=5000)
    gp = sk.Problem(a=to_dev(a), b=to_dev(b), x=to_dev(x), y=to_dev(y), cost_scale=scale)  # AUTO -> BF16X6
    gr = {k: v.cpu().numpy() for k, v in sk.gradient(ctx, gp, eps, to_dev(r.f), to_dev(r.g)).items()}
    P = O.coupling(r.f, r.g, Cm, a, b, eps)
    rr, cc = P.sum(1), P.sum(0)
    xo, yo = x.astype(np.float64), y.astype(np.float64)
    rel = np.expm1(bound.max() / eps) + 1e-5
    for k, ref, M in (("x", 2 * scale * (rr[:, None] * xo - P @ yo), 2 * scale * (rr[:, None] * np.abs(xo) + np.abs(P) @ np.abs(yo))),
                      ("y", 2 * scale * (cc[:, None] * yo - P.T @ xo), 2 * scale * (cc[:, None] * np.abs(yo) + np.abs(P).T @ np.abs(xo)))):
        err = np.abs(gr[k] - ref)
        print(f"grad_{k}: max err {err.max():.3e}, max allowed {(2 * rel * M).max():.3e}", flush=True)
        assert np.all(err <= 2 * rel * M + 1e-12)
    for k, ref, q in (("a", r.f - eps * rr / a, rr / a), ("b", r.g - eps * cc / b, cc / b)):
        err = np.abs(gr[k] - ref)
        assert np.all(err <= 2 * rel * eps * q + 1e-9)
