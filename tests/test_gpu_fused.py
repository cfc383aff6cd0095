"""The single-read SK pass over a stored cost (one read of C per iteration:
f = T_r(g) by rows, and each row's terms join the column log-sum-exp of
T_c(f)) against the two-pass iteration (SKNR_NO_FUSED=1) and against the
FP64 oracle: the same pairs are tested, so the iteration counts agree, and
both reach the oracle's optimum.  Shapes cover one, two and four float4
groups of columns per thread, ragged last groups (4100 and 12004 columns),
a single row per split and splits of unequal length."""
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


def _stored(n, m, seed):
    rng = np.random.default_rng(seed)
    x = rng.random((n, 2))
    y = rng.random((m, 2))
    C = O.sqeuclid_cost(x, y).astype(np.float32)
    a = rng.dirichlet(np.full(n, 3.0))
    b = rng.dirichlet(np.full(m, 3.0))
    return C, a, b


@pytest.mark.parametrize("n,m,ladder,full_oracle", [(300, 400, [5e-2, 2e-2], True),
                                                    (1000, 4100, [5e-2, 2e-2, 1e-2], True),
                                                    (4097, 8192, [5e-2, 2e-2], False), (9, 12, [1e-1, 5e-2], True),
                                                    (700, 16384, [5e-2], False), (600, 12004, [5e-2], False)])
def test_fused_pass_matches_two_pass_and_oracle(sk, ctx, n, m, ladder, full_oracle):
    C, a, b = _stored(n, m, seed=n + m)
    gp = sk.Problem(a=to_dev(a), b=to_dev(b), C=to_dev(C))
    print(f"case {n}x{m} ladder {ladder}", flush=True)
    try:
        os.environ["SKNR_NO_FUSED"] = "1"
        f0, g0, r0 = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=100000)
    finally:
        os.environ.pop("SKNR_NO_FUSED", None)
    f1, g1, r1 = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=100000)
    it0 = [s["iters"] for s in r0["stages"]]
    it1 = [s["iters"] for s in r1["stages"]]
    C64 = C.astype(np.float64)
    assert r0["status"] == 0 and r1["status"] == 0 and r1["marginal_err"] < 1e-6
    f1h, g1h = f1.cpu().numpy(), g1.cpu().numpy()
    e01 = e_pot(f0.cpu().numpy(), g0.cpu().numpy(), f1h, g1h, C64)
    print(f"two-pass {it0}, fused {it1}, e_pot between them {e01:.2e}", flush=True)
    for x, y in zip(it1, it0):
        assert abs(x - y) <= 1
    assert e01 <= 1e-5
    if full_oracle:
        _, _, ro = O.solve_schedule(C64, a, b, ladder, 1e-6, 1000000)
        fs, gs, _ = O.solve_schedule(C64, a, b, ladder, 1e-11, 1000000)
        e1 = e_pot(f1h, g1h, fs, gs, C64)
        print(f"oracle {[r.iters for r in ro]}, fused e_pot vs the oracle's optimum {e1:.2e}", flush=True)
        for x, z in zip(it1, [r.iters for r in ro]):
            assert abs(x - z) <= 0.1 * z + 2
        assert e1 <= 1e-5
    else:
        # the oracle on sampled rows: the exported pair satisfies f = T_r(g)
        rows = np.sort(np.random.default_rng(1).choice(n, 32, replace=False))
        fr = O.c_transform_row(g1h, C64[rows], b, ladder[-1])
        d = np.abs(f1h[rows] - fr).max()
        print(f"rows: max|f - T_r(g)| = {d:.2e}", flush=True)
        assert d <= 64 * 2.0 ** -24 * ladder[-1] + 1e-12 * np.abs(f1h).max()


@pytest.mark.parametrize("n,m", [(300, 400), (1000, 4100)])
def test_fused_pass_exact_column_path(sk, ctx, n, m):
    """Every row of every single-read pass through the max-shift path and
    every column through the merge's exact per-column path
    (SKNR_FUSED_EXACT_ALL=1; in normal runs they serve only rows whose sum
    under the fixed shift leaves [2^-24, 2^24] and columns whose plan
    marginal falls below 2^-76): the loop takes the two-pass iteration
    counts to the same optimum."""
    C, a, b = _stored(n, m, seed=n + m + 1)
    gp = sk.Problem(a=to_dev(a), b=to_dev(b), C=to_dev(C))
    ladder = [5e-2, 2e-2]
    print(f"case exact columns {n}x{m}", flush=True)
    try:
        os.environ["SKNR_NO_FUSED"] = "1"
        f0, g0, r0 = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=100000)
    finally:
        os.environ.pop("SKNR_NO_FUSED", None)
    try:
        os.environ["SKNR_FUSED_EXACT_ALL"] = "1"
        f1, g1, r1 = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=100000)
    finally:
        os.environ.pop("SKNR_FUSED_EXACT_ALL", None)
    f2, g2, r2 = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=100000)
    it0 = [s["iters"] for s in r0["stages"]]
    it1 = [s["iters"] for s in r1["stages"]]
    it2 = [s["iters"] for s in r2["stages"]]
    C64 = C.astype(np.float64)
    f1h, g1h = f1.cpu().numpy(), g1.cpu().numpy()
    e01 = e_pot(f0.cpu().numpy(), g0.cpu().numpy(), f1h, g1h, C64)
    e12 = e_pot(f1h, g1h, f2.cpu().numpy(), g2.cpu().numpy(), C64)
    print(f"two-pass {it0}, exact columns {it1}, plan sums {it2}, e_pot {e01:.2e} / {e12:.2e}", flush=True)
    assert r1["status"] == 0 and r1["marginal_err"] < 1e-6
    for x, y, z in zip(it1, it0, it2):
        assert abs(x - y) <= 1 and abs(x - z) <= 1
    assert e01 <= 1e-5 and e12 <= 1e-5


def test_fused_pass_tiny_column_weight(sk, ctx):
    """A column of weight 1e-40 has a plan marginal M_j near 1e-40, below
    the 2^-76 that the pass's FP32 terms resolve: the merge computes that
    column by its exact per-column path in every pass, and the loop
    matches the two-pass iteration and the oracle's optimum."""
    n, m = 300, 400
    C, a, b = _stored(n, m, seed=77)
    b[5] = 1e-40
    b /= b.sum()
    gp = sk.Problem(a=to_dev(a), b=to_dev(b), C=to_dev(C))
    ladder = [5e-2, 2e-2]
    print("case column weight 1e-40", flush=True)
    try:
        os.environ["SKNR_NO_FUSED"] = "1"
        f0, g0, r0 = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=100000)
    finally:
        os.environ.pop("SKNR_NO_FUSED", None)
    f1, g1, r1 = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=100000)
    it0 = [s["iters"] for s in r0["stages"]]
    it1 = [s["iters"] for s in r1["stages"]]
    C64 = C.astype(np.float64)
    f1h, g1h = f1.cpu().numpy(), g1.cpu().numpy()
    e01 = e_pot(f0.cpu().numpy(), g0.cpu().numpy(), f1h, g1h, C64)
    fs, gs, _ = O.solve_schedule(C64, a, b, ladder, 1e-11, 1000000)
    e1 = e_pot(f1h, g1h, fs, gs, C64)
    print(f"two-pass {it0}, fused {it1}, e_pot between them {e01:.2e}, vs the oracle {e1:.2e}", flush=True)
    assert r1["status"] == 0 and r1["marginal_err"] < 1e-6
    for x, y in zip(it1, it0):
        assert abs(x - y) <= 1
    assert e01 <= 1e-5 and e1 <= 1e-5
    # the light column itself: the two loops agree there to well within one
    # step's change near convergence (~eps times the relative marginal error)
    d5 = abs(g1h[5] - g0.cpu().numpy()[5])
    print(f"light column: |g_fused - g_two_pass| = {d5:.2e}", flush=True)
    assert np.isfinite(g1h).all() and d5 <= 1e-4 * ladder[-1]
