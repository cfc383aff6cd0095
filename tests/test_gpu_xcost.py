"""SK-NR on a large stored cost (at least 2^24 elements) in both orientations:
the sweeps whose outputs run along the stored rows stream over a transposed
copy of C (the warm start's 32-wide sweeps, the Newton sweeps, the plain
sweeps of SK-NR iterations).  Against the rows kernel on C itself
(SKNR_NO_XCOST=1): the same iteration counts within one and the same
optimum; against plain SK: the same optimum; against the oracle: f = T_r(g)
on sampled rows (Sec. 2, eq. foc_f; Algorithm 4.1)."""
import os

import numpy as np
import pytest

import oracle as O
from tests._helpers import e_pot, to_dev

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


@pytest.mark.parametrize("n,m", [(4000, 5000), (5000, 4000)])
def test_sknr_stored_transposed_copy(sk, ctx, n, m):
    rng = np.random.default_rng(n * 7 + m)
    x = rng.random((n, 2))
    y = rng.random((m, 2))
    C = O.sqeuclid_cost(x, y).astype(np.float32)
    a = rng.dirichlet(np.full(n, 3.0))
    b = rng.dirichlet(np.full(m, 3.0))
    gp = sk.Problem(a=to_dev(a), b=to_dev(b), C=to_dev(C))
    ladder = [5e-2, 2e-2]
    kw = dict(tol=1e-6, max_iter=20000, ell=16, warm_mode=sk.WARM_SEQUENTIAL)
    print(f"case stored {n}x{m} SK-NR(16)", flush=True)
    f1, g1, r1 = sk.solve(ctx, gp, ladder, **kw)
    try:
        os.environ["SKNR_NO_XCOST"] = "1"
        f0, g0, r0 = sk.solve(ctx, gp, ladder, **kw)
    finally:
        os.environ.pop("SKNR_NO_XCOST", None)
    fs, gs, rs = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=20000)
    C64 = C.astype(np.float64)
    it0 = [s["iters"] for s in r0["stages"]]
    it1 = [s["iters"] for s in r1["stages"]]
    f1h, g1h = f1.cpu().numpy(), g1.cpu().numpy()
    e01 = e_pot(f0.cpu().numpy(), g0.cpu().numpy(), f1h, g1h, C64)
    e1s = e_pot(f1h, g1h, fs.cpu().numpy(), gs.cpu().numpy(), C64)
    print(f"rows kernel {it0}, transposed copy {it1}, SK {[s['iters'] for s in rs['stages']]}; "
          f"e_pot {e01:.2e} / vs SK {e1s:.2e}; accepted {[s['newton_accepted'] for s in r1['stages']]}", flush=True)
    assert r0["status"] == 0 and r1["status"] == 0 and rs["status"] == 0
    assert r1["marginal_err"] < 1e-6
    for u, v in zip(it1, it0):
        assert abs(u - v) <= 1
    assert e01 <= 1e-6 and e1s <= 1e-5
    rows = np.sort(np.random.default_rng(2).choice(n, 32, replace=False))
    fr = O.c_transform_row(g1h, C64[rows], b, ladder[-1])
    d = np.abs(f1h[rows] - fr).max()
    print(f"rows: max|f - T_r(g)| = {d:.2e}", flush=True)
    assert d <= 64 * 2.0 ** -24 * ladder[-1] + 1e-12 * np.abs(f1h).max()
