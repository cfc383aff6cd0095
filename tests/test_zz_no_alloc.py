"""sknr_solve_noalloc (the solve with its workspace in the library's static
device array, for callers that cannot allocate) against sknr_solve on the
same inputs: two calls in a row, the second on a smaller problem, plus a
stored cost and the rejection of a problem whose workspace exceeds the
array.  The two entry points share every kernel and launch geometry, so
the potentials must agree bit for bit and the statistics exactly."""
import ctypes

import numpy as np
import pytest

import workloads as W
from tests._helpers import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_2506_14780_amd as sk
    return sk


def _pair(sk, ctx, gp, ladder, **kw):
    import torch
    n, m = int(gp.a.shape[0]), int(gp.b.shape[0])
    f1, g1, r1 = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=20000, **kw)
    f2 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    g2 = torch.full((m,), float("nan"), dtype=torch.float64, device="cuda")
    r2 = sk.solve_noalloc(ctx, gp, ladder, f2, g2, tol=1e-6, max_iter=20000, **kw)
    torch.cuda.synchronize()
    return (f1.cpu().numpy(), g1.cpu().numpy(), r1), (f2.cpu().numpy(), g2.cpu().numpy(), r2)


def _same(a, b):
    (f1, g1, r1), (f2, g2, r2) = a, b
    assert r1["status"] == 0 and r2["status"] == 0, (r1["status"], r2["status"])
    assert [s["iters"] for s in r1["stages"]] == [s["iters"] for s in r2["stages"]]
    assert [s["newton_accepted"] for s in r1["stages"]] == [s["newton_accepted"] for s in r2["stages"]]
    assert np.array_equal(f1, f2) and np.array_equal(g1, g2)
    assert r1["marginal_err"] == r2["marginal_err"] and r1["transport_cost"] == r2["transport_cost"]


def test_noalloc_matches_solve_twice_in_a_row_second_smaller(sk):
    ctx = sk.Context(0)
    try:
        big = W.gmm_vs_uniform(1500, 1700, seed=21)
        small = W.gmm_vs_uniform(300, 260, seed=22)  # n > m: solved on the transpose
        ladder = [1e-1, 5e-2, 2.5e-2, 1.25e-2]
        for prob in (big, small):
            gp = sk.Problem(a=to_dev(prob.a), b=to_dev(prob.b), x=to_dev(prob.x), y=to_dev(prob.y))
            print(f"case {prob.n}x{prob.m} SK-NR(10)", flush=True)
            _same(*_pair(sk, ctx, gp, ladder, ell=10, warm_mode=sk.WARM_SEQUENTIAL))
        print("case stored 333x401 SK", flush=True)
        st = W.uniform_square(333, 401, seed=23)
        C = ((st.x[:, None, :].astype(np.float64) - st.y[None, :, :]) ** 2).sum(-1).astype(np.float32)
        gp = sk.Problem(a=to_dev(st.a), b=to_dev(st.b), C=to_dev(C))
        _same(*_pair(sk, ctx, gp, [5e-2, 2.5e-2]))
    finally:
        ctx.close()


def test_noalloc_rejects_a_workspace_beyond_the_array(sk):
    import torch
    ctx = sk.Context(0)
    try:
        n = 1 << 16
        prob = W.uniform_square(n, seed=24)
        gp = sk.Problem(a=to_dev(prob.a), b=to_dev(prob.b), x=to_dev(prob.x), y=to_dev(prob.y))
        f = torch.empty(n, dtype=torch.float64, device="cuda")
        g = torch.empty(n, dtype=torch.float64, device="cuda")
        print(f"case {n}x{n} rejected", flush=True)
        with pytest.raises(sk.SknrError) as ei:
            sk.solve_noalloc(ctx, gp, [1e-1], f, g, tol=1e-6, max_iter=10)
        assert "exceeds" in str(ei.value) and ei.value.status == sk.EINVAL
        # the context and the array stay usable
        small = W.gmm_vs_uniform(200, 210, seed=25)
        gp = sk.Problem(a=to_dev(small.a), b=to_dev(small.b), x=to_dev(small.x), y=to_dev(small.y))
        _same(*_pair(sk, ctx, gp, [1e-1, 5e-2]))
    finally:
        ctx.close()
