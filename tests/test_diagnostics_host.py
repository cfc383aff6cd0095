"""Host-side pins of the diagnostics helpers and the paper-shaped input
generators (no GPU): principal angles between subspaces, the contraction
fit, and the shapes / normalisation / determinism of the generators."""
import math

import numpy as np
import pytest

import workloads as W


def _dg():
    # the helpers tested here run on the host (numpy); importing the package
    # loads the library without touching a GPU
    import paper_2506_14780_amd.diagnostics as dg
    return dg


def _orth_a(V, a):
    # orthonormalise the columns in L2(a)
    L = np.linalg.cholesky(V.T @ (a[:, None] * V))
    return V @ np.linalg.inv(L).T


def test_principal_cosines_pins():
    dg = _dg()
    rng = np.random.default_rng(0)
    n, k = 50, 4
    a = rng.dirichlet(np.full(n, 2.0))
    V = _orth_a(rng.standard_normal((n, k)), a)
    # the same subspace under an orthogonal change of basis: all ones
    Q = np.linalg.qr(rng.standard_normal((k, k)))[0]
    assert np.allclose(dg.principal_cosines(V, V @ Q, a), 1.0, atol=1e-12)
    # an L2(a)-orthogonal complement: all zeros
    X = rng.standard_normal((n, k))
    X -= V @ (V.T @ (a[:, None] * X))
    U = _orth_a(X, a)
    assert np.allclose(dg.principal_cosines(V, U, a), 0.0, atol=1e-12)
    # one shared direction, one at a known angle, the rest orthogonal
    E = _orth_a(rng.standard_normal((n, 3)), a)
    t = 0.3
    V2 = np.stack([E[:, 0], math.cos(t) * E[:, 1] + math.sin(t) * E[:, 2]], axis=1)
    c = dg.principal_cosines(E[:, :2], V2, a)
    assert np.allclose(np.sort(c), np.sort([1.0, math.cos(t)]), atol=1e-12)


def test_contraction_rate_recovers_a_geometric_sequence():
    dg = _dg()
    ks = np.arange(1, 200)
    errs = 3.0 * 0.83 ** ks
    assert dg.contraction_rate(ks, errs) == pytest.approx(0.83, rel=1e-12)
    # points outside the window are ignored (transient and floor)
    e2 = errs.copy()
    e2[:5] = 10.0
    e2[e2 < 1e-8] = 1e-8
    assert dg.contraction_rate(ks, e2) == pytest.approx(0.83, rel=1e-9)
    assert math.isnan(dg.contraction_rate(ks[:2], errs[:2]))


def test_paper_shaped_generators():
    p = W.square_vs_annulus(100, 120, seed=1)
    assert p.x.shape == (100, 2) and p.y.shape == (120, 2) and p.x.dtype == np.float32
    assert np.all(np.abs(p.x) <= 1.0)
    r = np.linalg.norm(p.y.astype(np.float64), axis=1)
    assert r.min() >= 0.5 - 1e-6 and r.max() <= 1.0 + 1e-6
    q = W.two_moons(100, 80, seed=2)
    assert q.x.shape == (100, 2) and q.y.shape == (80, 2)
    w = W.wot_shaped(700, 500, d=30, seed=3)
    assert w.x.shape == (700, 30) and w.y.shape == (500, 30)
    both = np.concatenate([w.x, w.y]).astype(np.float64)
    assert np.abs(both.mean(axis=0)).max() < 1e-5
    assert (both ** 2).sum(1).mean() == pytest.approx(1.0, rel=1e-5)
    for prob in (p, q, w):
        assert prob.a.sum() == pytest.approx(1.0) and prob.b.sum() == pytest.approx(1.0)
    # seeded: the same draw twice
    assert np.array_equal(W.wot_shaped(700, 500, seed=3).x, w.x)
