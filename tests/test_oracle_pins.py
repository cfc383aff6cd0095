"""Pins of the FP64 oracle against facts the mathematics fixes.

None of these re-types an oracle formula: each checks the oracle against a
closed form, a brute force, a library routine of independent provenance,
an invariant stated by the paper, or finite differences of the objective's
plain definition.  Runs on the CPU only.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize
import scipy.special

import oracle as O
import workloads as W


def _rand_problem(n, m, seed, d=2, scale=1.0):
    rng = np.random.default_rng(seed)
    x = rng.random((n, d))
    y = rng.random((m, d))
    a = rng.dirichlet(np.full(n, 4.0))
    b = rng.dirichlet(np.full(m, 4.0))
    return O.sqeuclid_cost(x, y, scale), a, b


# ---------------------------------------------------------------- P1, P2

def test_schroedinger_fixed_point_and_tiny_marginal():
    """Sec. 2 first-order conditions: at the SK limit f = T_r(g) and
    g = T_c(f); Algorithm 4.1's marginal error goes below 1e-12."""
    C, a, b = _rand_problem(40, 55, 0)
    r = O.sinkhorn(C, a, b, eps=0.05, tol=1e-13, max_iter=20000)
    assert r.converged and r.errs[-1] < 1e-12
    assert np.max(np.abs(r.f - O.c_transform_row(r.g, C, b, 0.05))) <= 1e-12 * C.max()
    assert np.max(np.abs(r.g - O.c_transform_col(r.f, C, a, 0.05))) <= 1e-12 * C.max()
    # after the row update the row marginal is exact (iterative proportional fitting)
    rows, cols = O.marginals(r.f, r.g, C, a, b, 0.05)
    assert np.max(np.abs(rows - a)) < 1e-15


# --------------------------------------------------------------------- P3

def test_large_eps_closed_form():
    """eps -> infinity: expanding the c-transforms to first order gives
    pi -> a b^T, f -> C b - (a^T C b)/2, g -> C^T a - (a^T C b)/2 (gauge
    <f,a> = <g,b>), W_eps -> a^T C b, each with an O(1/eps) error."""
    C, a, b = _rand_problem(30, 20, 1)
    acb = a @ C @ b
    f_inf = C @ b - 0.5 * acb
    g_inf = C.T @ a - 0.5 * acb
    errs = []
    for eps in (1e2, 1e3, 1e4):
        r = O.sinkhorn(C, a, b, eps, tol=1e-14, max_iter=200)
        f, g = O.normalize_gauge(r.f, r.g, a, b)
        e = max(np.abs(f - f_inf).max(), np.abs(g - g_inf).max())
        errs.append(e)
        assert e < 5 * C.max() ** 2 / eps
        P = O.coupling(f, g, C, a, b, eps)
        assert np.max(np.abs(P / np.outer(a, b) - 1)) < 5 * C.max() / eps
        assert abs(O.primal_value(f, g, C, a, b, eps) - acb) < 5 * C.max() ** 2 / eps
    # first-order convergence: the error falls by ~10x per decade of eps
    assert 5 < errs[0] / errs[1] < 20 and 5 < errs[1] / errs[2] < 20


# --------------------------------------------------------------------- P4

def test_separable_cost_is_exact_in_one_iteration():
    """C_ij = u_i + v_j: the optimal coupling is a b^T for every eps, and SK
    from f = 0 reaches it after one iteration with f = u + const."""
    prob, u, v = W.separable_cost(25, 33)
    C = prob.C.astype(np.float64)
    for eps in (1.0, 1e-2, 1e-3):
        r = O.sinkhorn(C, prob.a, prob.b, eps, tol=1e-12, max_iter=5)
        assert r.iters == 1 and r.converged
        P = O.coupling(r.f, r.g, C, prob.a, prob.b, eps)
        assert np.allclose(P, np.outer(prob.a, prob.b), rtol=1e-12, atol=0)
        d = r.f - u
        assert np.ptp(d) < 1e-12


# --------------------------------------------------------------------- P5

@pytest.mark.parametrize("n", [3, 5, 7])
def test_brute_force_permutations(n):
    """Uniform weights, n = m <= 7: W_0 = min over permutations of the mean
    matched cost (Birkhoff).  KL >= 0 and KL(pi_sigma || a(x)b) = log n give
    W_0 <= W_eps <= W_0 + eps log n, and <C, pi_eps> lies in the same band."""
    rng = np.random.default_rng(10 + n)
    C = rng.random((n, n))
    a = np.full(n, 1.0 / n)
    W0 = min(np.mean(C[np.arange(n), list(p)]) for p in itertools.permutations(range(n)))
    # plain SK needs >1e5 iterations below eps ~ 3e-2 here (the slowdown the
    # paper is about); SK-NR with a basis of the whole complement of the
    # constants (a full Newton step), warm-started along the eps ladder,
    # converges in a few iterations to the same optimum (Theorem 4.2).
    B = np.linalg.qr(np.c_[np.ones(n), np.random.default_rng(0).standard_normal((n, n - 1))])[0][:, 1:]
    prev_gap = None
    f = None
    for eps in (1e-1, 1e-2, 1e-3):
        r = O.sknr(C, a, a, eps, tol=1e-12, max_iter=20000, V=B, f0=f)
        assert r.converged
        f = r.f
        Weps = O.primal_value(r.f, r.g, C, a, a, eps)
        cost = O.transport_cost(r.f, r.g, C, a, a, eps)
        tol = 1e-9
        assert W0 - tol <= Weps <= W0 + eps * math.log(n) + tol
        assert W0 - tol <= cost <= W0 + eps * math.log(n) + tol
        # strong duality: the primal value equals the dual and semi-dual values
        assert abs(Weps - O.dual_value(r.f, r.g, C, a, a, eps)) < 1e-9
        assert abs(Weps - O.semidual_value(r.f, C, a, a, eps)) < 1e-9
        gap = Weps - W0
        if prev_gap is not None:
            assert gap <= prev_gap + 1e-12
        prev_gap = gap


def test_linear_program_limit_general_weights():
    """Non-uniform weights: W_eps decreases to the LP optimum W_0 (solved by
    scipy's HiGHS) as eps -> 0, with 0 <= W_eps - W_0 <= eps * H-bound."""
    rng = np.random.default_rng(3)
    n, m = 5, 7
    C = rng.random((n, m))
    a = rng.dirichlet(np.ones(n))
    b = rng.dirichlet(np.ones(m))
    A_eq = np.zeros((n + m, n * m))
    for i in range(n):
        A_eq[i, i * m:(i + 1) * m] = 1
    for j in range(m):
        A_eq[n + j, j::m] = 1
    lp = scipy.optimize.linprog(C.ravel(), A_eq=A_eq, b_eq=np.r_[a, b], bounds=(0, None), method="highs")
    W0 = lp.fun
    prev = None
    B = np.linalg.qr(np.c_[np.ones(n), rng.standard_normal((n, n - 1))])[0][:, 1:]
    f = None
    for eps in (1e-1, 1e-2, 1e-3):
        r = O.sknr(C, a, b, eps, tol=1e-12, max_iter=20000, V=B, f0=f)
        assert r.converged
        f = r.f
        Weps = O.primal_value(r.f, r.g, C, a, b, eps)
        # KL(pi_LP || a(x)b) bounds the gap: W_eps <= W_0 + eps KL(pi_LP)
        P0 = lp.x.reshape(n, m)
        with np.errstate(divide="ignore", invalid="ignore"):
            kl = np.nansum(np.where(P0 > 0, P0 * np.log(P0 / np.outer(a, b)), 0.0))
        assert W0 - 1e-9 <= Weps <= W0 + eps * kl + 1e-9
        if prev is not None:
            assert Weps <= prev + 1e-12
        prev = Weps


# --------------------------------------------------------------------- P6

def test_one_dimensional_sorted_matching():
    """d = 1, uniform weights, n = m: the exact OT cost is the mean squared
    gap of the sorted samples (monotone rearrangement); same band as P5."""
    rng = np.random.default_rng(4)
    n = 300
    x = rng.random((n, 1))
    y = rng.random((n, 1)) ** 2
    C = O.sqeuclid_cost(x, y)
    a = np.full(n, 1.0 / n)
    W0 = np.mean((np.sort(x[:, 0]) - np.sort(y[:, 0])) ** 2)
    for eps in (1e-2, 2e-3):
        r = O.sinkhorn(C, a, a, eps, tol=1e-10, max_iter=200000)
        assert r.converged
        Weps = O.primal_value(r.f, r.g, C, a, a, eps)
        assert W0 - 1e-9 <= Weps <= W0 + eps * math.log(n) + 1e-9


# --------------------------------------------------------------------- P7

def test_kernel_domain_matches_log_domain():
    """At moderate eps the scaling form u <- 1/(K (b*v)), v <- 1/(K^T (a*u))
    with K = exp(-C/eps) is the same map as the log-domain c-transforms
    (f = eps log u, g = eps log v)."""
    C, a, b = _rand_problem(50, 70, 5)
    eps = 0.3
    K = np.exp(-C / eps)
    u = np.ones(50)
    f = np.zeros(50)
    for _ in range(25):
        v = 1.0 / (K.T @ (a * u))
        u = 1.0 / (K @ (b * v))
        g = O.c_transform_col(f, C, a, eps)
        f = O.c_transform_row(g, C, b, eps)
        assert np.allclose(eps * np.log(v), g, rtol=1e-12, atol=1e-13)
        assert np.allclose(eps * np.log(u), f, rtol=1e-12, atol=1e-13)


# --------------------------------------------------------------------- P8

def test_semidual_derivatives_by_finite_differences():
    """eq. dQ_semi / d2Q_semi against central differences of Q^semi's
    definition; H 1 = 0 (shift invariance); H is negative semi-definite."""
    C, a, b = _rand_problem(12, 17, 6)
    eps = 0.2
    rng = np.random.default_rng(0)
    f = 0.3 * rng.standard_normal(12)
    q = lambda z: O.semidual_value(z, C, a, b, eps)
    h = 1e-5
    I = np.eye(12)
    g_fd = np.array([(q(f + h * I[i]) - q(f - h * I[i])) / (2 * h) for i in range(12)])
    assert np.allclose(O.semidual_gradient(f, C, a, b, eps), g_fd, atol=1e-9)
    h = 1e-4
    H_fd = np.array([[(q(f + h * I[i] + h * I[j]) - q(f + h * I[i] - h * I[j])
                       - q(f - h * I[i] + h * I[j]) + q(f - h * I[i] - h * I[j])) / (4 * h * h)
                      for j in range(12)] for i in range(12)])
    H = O.semidual_hessian(f, C, a, b, eps)
    assert np.allclose(H, H_fd, atol=2e-6)
    assert np.max(np.abs(H @ np.ones(12))) < 1e-13
    assert np.max(np.linalg.eigvalsh(H)) < 1e-12
    # operator form agrees with the dense one
    V = rng.standard_normal((12, 3))
    assert np.allclose(O.semidual_hessian_apply(f, C, a, b, eps, V), H @ V, atol=1e-13)


def test_projected_newton_step_basis_invariance_and_ascent():
    """The step depends on span(V) only (V -> V T), solves the restricted
    quadratic model, and with V spanning everything but the constants it is
    the full Newton step (checked against scipy's solver on the dense
    Hessian restricted to the complement of 1)."""
    C, a, b = _rand_problem(15, 11, 7)
    eps = 0.1
    rng = np.random.default_rng(1)
    f = O.c_transform_row(O.c_transform_col(np.zeros(15), C, a, eps), C, b, eps)
    V = rng.standard_normal((15, 4))
    T = rng.standard_normal((4, 4)) + 4 * np.eye(4)
    s1 = O.projected_newton(f, C, a, b, eps, V)
    s2 = O.projected_newton(f, C, a, b, eps, V @ T)
    assert s1["ok"] and s2["ok"]
    assert np.allclose(s1["delta"], s2["delta"], atol=1e-11)
    # full space minus constants: Q = orthonormal basis of 1^perp
    Q, _ = np.linalg.qr(np.c_[np.ones(15), rng.standard_normal((15, 14))])
    B = Q[:, 1:]
    H = O.semidual_hessian(f, C, a, b, eps)
    grad = O.semidual_gradient(f, C, a, b, eps)
    ref = -B @ scipy.linalg.solve(B.T @ H @ B, B.T @ grad, assume_a="sym")
    full = O.projected_newton(f, C, a, b, eps, B)
    assert np.allclose(full["delta"], ref, atol=1e-10)
    # with the constant vector inside V the projected Hessian is singular
    bad = O.projected_newton(f, C, a, b, eps, np.c_[np.ones(15), V])
    assert (not bad["ok"]) or np.linalg.cond(bad["hess"]) > 1e12


# --------------------------------------------------------------------- P9

def test_structure_theorem_at_optimum():
    """Theorem 3.1: the Hessian of Q_eps (definition eq. def_Q, by finite
    differences) at the optimum equals -(1/eps)(Id + K_eps) in L2(a)+L2(b);
    K_eps has spectrum in [-1,1], symmetric about 0, with +-1 simple on the
    constants 1+1 and (-1)+1.  spectral_basis's rho are the top |eig(K)|."""
    n, m = 9, 13
    C, a, b = _rand_problem(n, m, 8)
    eps = 0.15
    r = O.sinkhorn(C, a, b, eps, tol=1e-14, max_iter=100000)
    f, g = r.f, r.g
    z0 = np.r_[f, g]
    N = n + m
    Q = lambda z: O.dual_value(z[:n], z[n:], C, a, b, eps)
    h = 1e-4
    I = np.eye(N)
    Hfd = np.array([[(Q(z0 + h * I[i] + h * I[j]) - Q(z0 + h * I[i] - h * I[j])
                      - Q(z0 - h * I[i] + h * I[j]) + Q(z0 - h * I[i] - h * I[j])) / (4 * h * h)
                     for j in range(N)] for i in range(N)])
    w = np.r_[a, b]
    K = -eps * Hfd / w[:, None] - np.eye(N)          # L2-weighted operator form
    P = O.coupling(f, g, C, a, b, eps)
    K_thm = np.zeros((N, N))
    K_thm[:n, n:] = P / a[:, None]
    K_thm[n:, :n] = P.T / b[:, None]
    assert np.allclose(K, K_thm, atol=1e-5)
    # spectrum: K is self-adjoint in L2(w) -> symmetrise
    Ks = np.sqrt(w)[:, None] * K_thm / np.sqrt(w)[None, :]
    ev = np.sort(np.linalg.eigvalsh(0.5 * (Ks + Ks.T)))
    assert ev[-1] == pytest.approx(1.0, abs=1e-10) and ev[0] == pytest.approx(-1.0, abs=1e-10)
    assert ev[-2] < 1 - 1e-6
    nz = ev[np.abs(ev) > 1e-8]
    assert np.allclose(np.sort(nz), np.sort(-nz), atol=1e-10)
    assert np.allclose(K_thm @ np.ones(N), np.ones(N), atol=1e-12)
    assert np.allclose(K_thm @ np.r_[-np.ones(n), np.ones(m)], -np.r_[-np.ones(n), np.ones(m)], atol=1e-12)
    # eigen target of the warm start: rho_k^2 = eig(S), S = A A^T
    V, rho = O.spectral_basis(f, g, C, a, b, eps, ell=3, method="dense")
    top = np.sort(ev)[::-1][: 4]
    assert np.allclose(rho, top, atol=1e-9)
    # V is orthonormal in L2(a) and orthogonal to the constants
    assert np.allclose(V.T @ (a[:, None] * V), np.eye(3), atol=1e-10)
    assert np.allclose(a @ V, 0, atol=1e-10)
    # the semi-dual Hessian at the optimum is -(1/eps) diag(a)(Id - M): eq. semidual_Hessian
    H = O.semidual_hessian(f, C, a, b, eps)
    M = (P / a[:, None]) @ (P.T / b[:, None])
    assert np.allclose(H, -(np.diag(a) @ (np.eye(n) - M)) / eps, atol=1e-10)
    assert np.allclose(M @ V, V * rho[1:] ** 2, atol=1e-9)


def test_arpack_and_dense_bases_agree():
    """spectral_basis by eigsh (operator) and by dense eigh span the same
    space when the gap after rho_l is clear."""
    prob = W.uniform_square(200, seed=11)
    C = O.sqeuclid_cost(prob.x, prob.y)
    r = O.sinkhorn(C, prob.a, prob.b, 0.05, tol=1e-12, max_iter=100000)
    V1, rho1 = O.spectral_basis(r.f, r.g, C, prob.a, prob.b, 0.05, 5, method="dense")
    V2, rho2 = O.spectral_basis(r.f, r.g, C, prob.a, prob.b, 0.05, 5, method="arpack")
    assert np.allclose(rho1, rho2, atol=1e-10)
    # principal angles in L2(a)
    sa = np.sqrt(prob.a)[:, None]
    Q1, _ = np.linalg.qr(sa * V1)
    Q2, _ = np.linalg.qr(sa * V2)
    cosines = np.linalg.svd(Q1.T @ Q2, compute_uv=False)
    assert cosines.min() > 1 - 1e-8


# ------------------------------------------------------------ P10, P11, P12

def _osc(v):
    return float(v.max() - v.min())


def _rates(C, a, b, eps, V, fstar, iters):
    f = np.zeros(C.shape[0])
    errs = []
    for _ in range(iters):
        r = O.sknr(C, a, b, eps, tol=0.0, max_iter=1, V=V, f0=f)
        f = r.f
        errs.append(_osc(f - fstar))
    return np.array(errs)


def test_sk_rate_is_rho1_squared_and_sknr_rate_is_rho_l_plus_1_squared():
    """Lemma 3.2: SK contracts like rho_1^2.  Theorem 4.2: with the exact
    V_l(eps), SK-NR contracts like rho_{l+1}^2.  Ratios of successive
    oscillation errors must match within 10%."""
    prob = W.uniform_square(60, seed=12)
    C = O.sqeuclid_cost(prob.x, prob.y)
    a, b = prob.a, prob.b
    eps = 0.03
    ref = O.sinkhorn(C, a, b, eps, tol=1e-15, max_iter=200000)
    fstar = ref.f
    ell = 3
    V, rho = O.spectral_basis(ref.f, ref.g, C, a, b, eps, ell + 1, method="dense")
    V = V[:, :ell]
    e_sk = _rates(C, a, b, eps, None, fstar, 400)
    ok = (e_sk > 1e-9) & (e_sk < 1e-3)
    ratios = e_sk[1:][ok[1:] & ok[:-1]] / e_sk[:-1][ok[1:] & ok[:-1]]
    assert len(ratios) > 5
    assert ratios[-1] == pytest.approx(rho[1] ** 2, rel=0.1)
    e_nr = _rates(C, a, b, eps, V, fstar, 200)
    ok = (e_nr > 1e-10) & (e_nr < 1e-4)
    ratios = e_nr[1:][ok[1:] & ok[:-1]] / e_nr[:-1][ok[1:] & ok[:-1]]
    assert len(ratios) > 3
    assert ratios[-1] == pytest.approx(rho[ell + 1] ** 2, rel=0.1)
    assert rho[ell + 1] ** 2 < 0.95 * rho[1] ** 2


def test_semidual_value_never_decreases():
    """Proof of Theorem 4.2, step 1: Q^semi(f_k) is non-decreasing along
    SK-NR, also with a poor (random) basis, whose steps the guard rejects
    when they do not increase Q^semi."""
    C, a, b = _rand_problem(40, 50, 13)
    rng = np.random.default_rng(2)
    for V in (rng.standard_normal((40, 5)), None):
        f = np.zeros(40)
        qs = []
        for _ in range(60):
            r = O.sknr(C, a, b, 0.02, tol=0.0, max_iter=1, V=V, f0=f)
            f = r.f
            qs.append(O.semidual_value(f, C, a, b, 0.02))
        assert np.all(np.diff(qs) >= -1e-13)


# -------------------------------------------------------------- P13, P14

def test_transpose_symmetry():
    """Swapping the roles of X and Y (C -> C^T, a <-> b) swaps f and g."""
    C, a, b = _rand_problem(23, 31, 14)
    r1 = O.sinkhorn(C, a, b, 0.05, tol=1e-13, max_iter=100000)
    r2 = O.sinkhorn(C.T, b, a, 0.05, tol=1e-13, max_iter=100000)
    f1, g1 = O.normalize_gauge(r1.f, r1.g, a, b)
    g2, f2 = O.normalize_gauge(r2.f, r2.g, b, a)
    assert np.allclose(f1, f2, atol=1e-11) and np.allclose(g1, g2, atol=1e-11)
    # solve_schedule transposes internally when n > m (semi-dual on the smaller side)
    f3, g3, _ = O.solve_schedule(C.T, b, a, [0.05], 1e-13, 100000)
    fo, go = O.normalize_gauge(g3, f3, a, b)
    assert np.allclose(fo, f1, atol=1e-11) and np.allclose(go, g1, atol=1e-11)


def test_c_transforms_against_scipy_logsumexp():
    """Third implementation: scipy.special.logsumexp with weights."""
    C, a, b = _rand_problem(64, 48, 15)
    rng = np.random.default_rng(3)
    f = rng.standard_normal(64)
    g = rng.standard_normal(48)
    for eps in (1.0, 1e-2, 1e-3):
        gc = -eps * scipy.special.logsumexp((f[:, None] - C) / eps, b=a[:, None], axis=0)
        fr = -eps * scipy.special.logsumexp((g[None, :] - C) / eps, b=b[None, :], axis=1)
        assert np.allclose(O.c_transform_col(f, C, a, eps), gc, rtol=1e-13, atol=1e-13)
        assert np.allclose(O.c_transform_row(g, C, b, eps), fr, rtol=1e-13, atol=1e-13)


def test_gauge_normalisation_keeps_coupling():
    C, a, b = _rand_problem(10, 12, 16)
    rng = np.random.default_rng(4)
    f, g = rng.standard_normal(10), rng.standard_normal(12)
    f2, g2 = O.normalize_gauge(f, g, a, b)
    assert abs(f2 @ a - g2 @ b) < 1e-14
    assert np.allclose(O.coupling(f, g, C, a, b, 0.1), O.coupling(f2, g2, C, a, b, 0.1), rtol=1e-13)


def test_halving_ladder_matches_workload_ladder():
    assert np.allclose(O.halving_ladder(1e-1, 1e-3), W.EPS_LADDER_C2, rtol=0, atol=1e-18)


def test_schedule_sknr_reaches_the_same_optimum_as_sk():
    """Theorem 4.2: SK-NR converges to the same optimum as SK; on a small
    schedule the spectral warm start also needs fewer iterations."""
    prob = W.uniform_square(120, seed=17)
    C = O.sqeuclid_cost(prob.x, prob.y)
    ladder = [0.1, 0.05, 0.025, 0.0125]
    f0, g0, r0 = O.solve_schedule(C, prob.a, prob.b, ladder, 1e-9, 100000, ell=0)
    f1, g1, r1 = O.solve_schedule(C, prob.a, prob.b, ladder, 1e-9, 100000, ell=10)
    f0, g0 = O.normalize_gauge(f0, g0, prob.a, prob.b)
    f1, g1 = O.normalize_gauge(f1, g1, prob.a, prob.b)
    assert np.max(np.abs(f0 - f1)) < 1e-6 and np.max(np.abs(g0 - g1)) < 1e-6
    assert sum(r.iters for r in r1[1:]) < sum(r.iters for r in r0[1:])
    assert all(r.newton_accepted > 0 for r in r1[1:])


# ------------------------------------------------ gradients of W_eps (N3)

def test_dual_partials_by_finite_differences_and_envelope():
    """dual_partials against central differences of Q_eps at fixed (f, g)
    (a definition check), and at the optimum against central differences of
    W_eps itself, re-solved at each perturbed input (the envelope theorem)."""
    rng = np.random.default_rng(31)
    n, m, d, eps, s = 7, 9, 2, 0.3, 0.7
    x = rng.random((n, d))
    y = rng.random((m, d))
    a = rng.dirichlet(np.full(n, 3.0))
    b = rng.dirichlet(np.full(m, 3.0))
    f = 0.2 * rng.standard_normal(n)
    g = 0.2 * rng.standard_normal(m)
    D = O.dual_partials(f, g, x, y, a, b, eps, s)
    Q = lambda xx, yy, aa, bb: O.dual_value(f, g, O.sqeuclid_cost(xx, yy, s), aa, bb, eps)
    h = 1e-6
    for (i, k) in [(0, 0), (3, 1), (6, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[i, k] += h
        xm[i, k] -= h
        assert (Q(xp, y, a, b) - Q(xm, y, a, b)) / (2 * h) == pytest.approx(D["x"][i, k], rel=1e-6, abs=1e-9)
    for (j, k) in [(0, 1), (8, 0)]:
        yp, ym = y.copy(), y.copy()
        yp[j, k] += h
        ym[j, k] -= h
        assert (Q(x, yp, a, b) - Q(x, ym, a, b)) / (2 * h) == pytest.approx(D["y"][j, k], rel=1e-6, abs=1e-9)
    for i in (1, 5):
        ap, am = a.copy(), a.copy()
        ap[i] += h
        am[i] -= h
        assert (Q(x, y, ap, b) - Q(x, y, am, b)) / (2 * h) == pytest.approx(D["a"][i], rel=1e-6, abs=1e-9)
    for j in (2, 7):
        bp, bm = b.copy(), b.copy()
        bp[j] += h
        bm[j] -= h
        assert (Q(x, y, a, bp) - Q(x, y, a, bm)) / (2 * h) == pytest.approx(D["b"][j], rel=1e-6, abs=1e-9)
    # the coupling is dQ/dC
    Cb = O.sqeuclid_cost(x, y, s)
    Cp = Cb.copy()
    Cp[2, 3] += h
    Cm = Cb.copy()
    Cm[2, 3] -= h
    dq = (O.dual_value(f, g, Cp, a, b, eps) - O.dual_value(f, g, Cm, a, b, eps)) / (2 * h)
    assert dq == pytest.approx(D["C"][2, 3], rel=1e-6)

    # envelope: W_eps(x) = max Q; its derivative is the partial at the optimum
    def W(xx):
        C = O.sqeuclid_cost(xx, y, s)
        r = O.sinkhorn(C, a, b, eps, tol=1e-14, max_iter=100000)
        return O.dual_value(r.f, r.g, C, a, b, eps), r
    _, r0 = W(x)
    D0 = O.dual_partials(r0.f, r0.g, x, y, a, b, eps, s)
    h = 1e-5
    for (i, k) in [(0, 0), (4, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[i, k] += h
        xm[i, k] -= h
        fd = (W(xp)[0] - W(xm)[0]) / (2 * h)
        assert fd == pytest.approx(D0["x"][i, k], rel=1e-6, abs=1e-10)


# ------------------------------------------------- the cost of Sec. 5 (input)

@pytest.mark.parametrize("d", [2, 3, 64])
@pytest.mark.parametrize("scale", ["one", "inv_d", 0.37])
def test_sqeuclid_cost_against_cdist_and_euclidean_invariances(d, scale):
    """The squared Euclidean cost of Sec. 5 against scipy's cdist (an
    implementation of independent provenance) for d = 2, 3, 64 and scales
    1, 1/d, 0.37, plus two facts of Euclidean geometry that hold whatever
    the formula: invariance under a common rotation and translation of both
    clouds, and C_ii = 0 when the clouds coincide.  A dropped coordinate, a
    wrong sign, a transposed operand or a mis-applied scale fails one."""
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(30 + d)
    s = {"one": 1.0, "inv_d": 1.0 / d}.get(scale, scale)
    x = rng.standard_normal((17, d))
    y = rng.standard_normal((23, d)) + 0.5
    C = O.sqeuclid_cost(x, y, s)
    assert C.shape == (17, 23)
    np.testing.assert_allclose(C, s * cdist(x, y, "sqeuclidean"), rtol=1e-12, atol=1e-12 * s * d)
    Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    t = rng.standard_normal(d)
    np.testing.assert_allclose(O.sqeuclid_cost(x @ Q + t, y @ Q + t, s), C, rtol=1e-10, atol=1e-10 * s * d)
    assert np.all(np.abs(np.diag(O.sqeuclid_cost(x, x, s))) < 1e-12 * s * d)


# ------------------------------------------------- static warm start (Sec. 5)

def test_static_schedule_reaches_the_sk_optimum_at_the_theorem_4_2_rate():
    """The static warm start of Sec. 5 (V_l computed once, from a plain SK
    solve at eps').  Theorem 4.2: the SK-NR stages reach the SK optimum;
    with eps' equal to the target eps, V_l spans the exact low-frequency
    eigenvectors there and the marginal error contracts like rho_{l+1}^2
    (P11), faster than plain SK's rho_1^2 (Lemma 3.2).  With the paper's
    eps' = 1 the optimum is the same."""
    prob = W.uniform_square(60, seed=12)
    C = O.sqeuclid_cost(prob.x, prob.y)
    a, b = prob.a, prob.b
    eps, ell = 0.03, 3
    ref = O.sinkhorn(C, a, b, eps, tol=1e-14, max_iter=200000)
    fr, gr = O.normalize_gauge(ref.f, ref.g, a, b)
    _, rho = O.spectral_basis(ref.f, ref.g, C, a, b, eps, ell + 1, method="dense")
    f, g, rs = O.solve_schedule(C, a, b, [0.06, eps], 1e-13, 100000, ell=ell, mode="static", eps_prime=eps)
    assert all(r.converged for r in rs)
    assert rs[0].newton_tried == 0 and rs[1].newton_accepted > 0
    f, g = O.normalize_gauge(f, g, a, b)
    assert np.max(np.abs(f - fr)) < 1e-10 and np.max(np.abs(g - gr)) < 1e-10
    e = np.array(rs[1].errs)
    ok = (e > 1e-11) & (e < 1e-5)
    ratios = e[1:][ok[1:] & ok[:-1]] / e[:-1][ok[1:] & ok[:-1]]
    assert len(ratios) >= 3
    assert ratios[-1] == pytest.approx(rho[ell + 1] ** 2, rel=0.15)
    sk = O.sinkhorn(C, a, b, eps, tol=1e-13, max_iter=200000, f0=rs[0].f)
    assert rs[1].iters < sk.iters
    f1, g1, r1 = O.solve_schedule(C, a, b, [0.06, eps], 1e-13, 100000, ell=ell, mode="static", eps_prime=1.0)
    f1, g1 = O.normalize_gauge(f1, g1, a, b)
    assert all(r.converged for r in r1)
    assert np.max(np.abs(f1 - fr)) < 1e-10 and np.max(np.abs(g1 - gr)) < 1e-10
