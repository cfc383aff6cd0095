"""GPU checks of the boundary's input and output options: host-resident
problem arrays (sknr_problem.on_host), the initial potential g0 (and f0 on
a transposed problem), and the export of the solve's basis V_l
(sknr_get_subspace) with its reuse as WARM_USER's V0 (Algorithm 4.1 takes
V_l as an input; Sec. 4 reuses one basis across eps)."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests._helpers import e_pot, gpu_problem, to_dev

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


def host_problem(sk, prob, stored=False, C32=None):
    a = np.ascontiguousarray(prob.a, np.float64)
    b = np.ascontiguousarray(prob.b, np.float64)
    if stored:
        return sk.Problem(a=a, b=b, C=np.ascontiguousarray(C32, np.float32))
    return sk.Problem(a=a, b=b, x=np.ascontiguousarray(prob.x, np.float32),
                      y=np.ascontiguousarray(prob.y, np.float32), cost_scale=prob.cost_scale)


@pytest.mark.parametrize("stored", [True, False])
def test_host_inputs_match_device_inputs(sk, ctx, stored):
    """The same problem from host arrays and from device tensors gives the
    same solve bit for bit (the call stages an exact copy)."""
    prob = W.uniform_square(200, m=264, seed=11)
    C32 = O.sqeuclid_cost(prob.x, prob.y).astype(np.float32)
    print(f"case host_inputs stored={stored}", flush=True)
    kw = dict(tol=1e-6, max_iter=5000, ell=6, warm_mode=sk.WARM_SEQUENTIAL)
    fd, gd, rd = sk.solve(ctx, gpu_problem(prob, stored=stored, C32=C32), [4e-2, 2e-2], **kw)
    hp = host_problem(sk, prob, stored=stored, C32=C32)
    assert hp.c_struct().on_host == 1
    fh, gh, rh = sk.solve(ctx, hp, [4e-2, 2e-2], **kw)
    assert rh["status"] == 0
    assert np.array_equal(fd.cpu().numpy(), fh.cpu().numpy())
    assert np.array_equal(gd.cpu().numpy(), gh.cpu().numpy())
    assert rd["total_iters"] == rh["total_iters"]
    assert rd["transport_cost"] == rh["transport_cost"]


def test_host_inputs_transposed_with_row_stride(sk, ctx):
    """n > m (solved on the transpose) from a host matrix with a row stride
    larger than m: matches the oracle's optimum."""
    prob = W.uniform_square(300, m=180, seed=12)
    C = O.sqeuclid_cost(prob.x, prob.y)
    C32 = C.astype(np.float32)
    big = np.zeros((300, 200), np.float32)
    big[:, :180] = C32
    hp = sk.Problem(a=np.ascontiguousarray(prob.a), b=np.ascontiguousarray(prob.b), C=big, ldc=200)
    print("case host_inputs transposed ldc=200", flush=True)
    f, g, res = sk.solve(ctx, hp, [2e-2], tol=1e-7, max_iter=20000)
    ref = O.sinkhorn(C32.astype(np.float64), prob.a, prob.b, 2e-2, tol=1e-10, max_iter=100000)
    fr, gr = O.normalize_gauge(ref.f, ref.g, prob.a, prob.b)
    assert res["status"] == 0 and res["transposed"] == 1
    assert e_pot(f.cpu().numpy(), g.cpu().numpy(), fr, gr, C32.astype(np.float64)) < 1e-5


def test_noalloc_rejects_host_inputs(sk, ctx):
    prob = W.uniform_square(64, seed=1)
    hp = host_problem(sk, prob, stored=True, C32=O.sqeuclid_cost(prob.x, prob.y).astype(np.float32))
    import torch
    f = torch.empty(64, dtype=torch.float64, device="cuda")
    g = torch.empty(64, dtype=torch.float64, device="cuda")
    with pytest.raises(sk.SknrError) as e:
        sk.solve_noalloc(ctx, hp, [1e-1], f, g)
    assert e.value.status == sk.EINVAL


def test_g0_start_is_the_row_transform(sk, ctx):
    """g0 alone starts from f = T_r(g0) (eq. foc_f): one SK iteration from
    g0 equals one iteration from f0 = T_r(g0) computed by the row
    transform entry point (up to the FP64 round trip of f0, ~2^-48
    relative), and that start is the oracle's T_r(g0) to the sweep's
    accuracy."""
    prob = W.uniform_square(160, m=224, seed=13)
    C32 = O.sqeuclid_cost(prob.x, prob.y).astype(np.float32)
    C = C32.astype(np.float64)
    eps = 3e-2
    rng = np.random.default_rng(5)
    g0 = rng.uniform(-0.05, 0.05, 224)
    gp = gpu_problem(prob, stored=True, C32=C32)
    print("case g0 start", flush=True)
    fa, ga, ra = sk.solve(ctx, gp, [eps], tol=1e-12, max_iter=1, g0=to_dev(g0))
    f_half = sk.c_transform_row(ctx, gp, eps, to_dev(g0))
    f_ref = O.c_transform_row(g0, C, prob.b, eps)
    assert np.abs(f_half.cpu().numpy() - f_ref).max() <= 64 * 2.0 ** -24 * eps + 1e-12 * np.abs(g0).max()
    fb, gb, rb = sk.solve(ctx, gp, [eps], tol=1e-12, max_iter=1, f0=f_half)
    assert ra["total_iters"] == rb["total_iters"] == 1
    scale = np.abs(fb.cpu().numpy()).max() + eps
    assert np.abs(fa.cpu().numpy() - fb.cpu().numpy()).max() <= 1e-12 * scale
    assert np.abs(ga.cpu().numpy() - gb.cpu().numpy()).max() <= 1e-12 * scale


def test_restart_from_the_optimum(sk, ctx):
    """g0 = g* (and, on a transposed problem, f0 = f*) restarts at the
    optimum: a few iterations, same optimum."""
    for n, m in [(200, 260), (260, 200)]:
        prob = W.uniform_square(n, m=m, seed=14)
        C32 = O.sqeuclid_cost(prob.x, prob.y).astype(np.float32)
        gp = gpu_problem(prob, stored=True, C32=C32)
        print(f"case restart {n}x{m}", flush=True)
        f1, g1, r1 = sk.solve(ctx, gp, [2e-2], tol=1e-7, max_iter=20000)
        assert r1["status"] == 0 and r1["total_iters"] > 20
        # the potential of the side that is not iterated on
        kw = dict(g0=g1) if n <= m else dict(f0=f1)
        f2, g2, r2 = sk.solve(ctx, gp, [2e-2], tol=1e-7, max_iter=20000, **kw)
        assert r2["status"] == 0
        assert r2["total_iters"] <= 3
        assert e_pot(f1.cpu().numpy(), g1.cpu().numpy(), f2.cpu().numpy(), g2.cpu().numpy(),
                     C32.astype(np.float64)) < 1e-6


@pytest.mark.parametrize("n,m", [(240, 300), (300, 240)])
def test_get_subspace_and_reuse(sk, ctx, n, m):
    """The exported V_l is orthonormal in L2(alpha) and orthogonal to the
    constants on the semi-dual side; as V0 (WARM_USER) it runs Newton
    steps to the same optimum."""
    prob = W.uniform_square(n, m=m, seed=15)
    C32 = O.sqeuclid_cost(prob.x, prob.y).astype(np.float32)
    gp = gpu_problem(prob, stored=True, C32=C32)
    ell = 8
    print(f"case get_subspace {n}x{m}", flush=True)
    f, g, res = sk.solve(ctx, gp, [4e-2, 2e-2, 1e-2], tol=1e-6, max_iter=20000, ell=ell,
                         warm_mode=sk.WARM_SEQUENTIAL)
    assert res["status"] == 0
    rows = min(n, m)
    V, side = sk.get_subspace(ctx, rows, ell)
    assert side == (0 if n <= m else 1)
    w = prob.a if n <= m else prob.b
    Vh = V.cpu().numpy()
    assert np.allclose(Vh.T @ (w[:, None] * Vh), np.eye(ell), atol=1e-5)
    assert np.abs(w @ Vh).max() < 1e-5
    # reuse at the last eps from the previous stage's neighbourhood
    f_start, g_start, _ = sk.solve(ctx, gp, [2e-2], tol=1e-6, max_iter=20000)
    kw = dict(f0=f_start) if n <= m else dict(g0=g_start)
    f2, g2, r2 = sk.solve(ctx, gp, [1e-2], tol=1e-6, max_iter=20000, ell=ell, warm_mode=sk.WARM_USER,
                          V0=V, first_stage_nr=True, **kw)
    assert r2["status"] == 0
    assert r2["stages"][0]["newton_accepted"] >= 1
    assert e_pot(f.cpu().numpy(), g.cpu().numpy(), f2.cpu().numpy(), g2.cpu().numpy(),
                 C32.astype(np.float64)) < 1e-5


def test_get_subspace_errors(sk, ctx):
    prob = W.uniform_square(128, seed=16)
    C32 = O.sqeuclid_cost(prob.x, prob.y).astype(np.float32)
    gp = gpu_problem(prob, stored=True, C32=C32)
    print("case get_subspace errors", flush=True)
    sk.solve(ctx, gp, [4e-2, 2e-2], tol=1e-6, max_iter=20000, ell=4, warm_mode=sk.WARM_SEQUENTIAL)
    with pytest.raises(sk.SknrError) as e:  # wrong shape
        sk.get_subspace(ctx, 127, 4)
    assert e.value.status == sk.EINVAL
    V, _ = sk.get_subspace(ctx, 128, 4)
    assert V.shape == (128, 4)
    # another call on the context reuses the workspace
    sk.evaluate(ctx, gp, 2e-2, to_dev(np.zeros(128)), to_dev(np.zeros(128)))
    with pytest.raises(sk.SknrError) as e:
        sk.get_subspace(ctx, 128, 4)
    assert e.value.status == sk.EINVAL
    # a plain SK solve has no basis
    sk.solve(ctx, gp, [2e-2], tol=1e-6, max_iter=20000)
    with pytest.raises(sk.SknrError) as e:
        sk.get_subspace(ctx, 128, 4)
    assert e.value.status == sk.EINVAL
