"""FP64 reference implementation of log-domain Sinkhorn-Knopp and SK-NR(l).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.

Conventions (paper, Sec. 2):

* alpha (``a``, length n) and beta (``b``, length m) are probability
  vectors, C is the n x m cost, eps > 0.
* Potentials are relative to alpha (x) beta: the coupling is
  pi_ij = a_i b_j exp((f_i + g_j - C_ij) / eps)  (eq. Optimal_P_epsilon).
* The c-transforms are the first-order conditions eq. foc_f / foc_g:
  T_r(g)_i = -eps log sum_j b_j exp((g_j - C_ij)/eps)   (row side, f-update)
  T_c(f)_j = -eps log sum_i a_i exp((f_i - C_ij)/eps)   (column side, g-update)

Readings of points the paper leaves open (listed with reasons in the design
notes): the convergence test of Algorithm 4.1 uses the L1 norm; the
low-frequency basis excludes the constant mode and is orthonormal in
L2(alpha); the Newton coordinates are c with Delta f = V c; ties in the
acceptance test reject the step; when n > m the semi-dual is taken on the
smaller side by transposing the problem.

Parity pins for every function live in tests/test_oracle_*.py.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "sqeuclid_cost",
    "logsumexp",
    "c_transform_col",
    "c_transform_row",
    "coupling",
    "marginals",
    "marginal_error",
    "dual_value",
    "semidual_value",
    "transport_cost",
    "primal_value",
    "dual_partials",
    "semidual_gradient",
    "semidual_hessian",
    "semidual_hessian_apply",
    "projected_newton",
    "SolveResult",
    "sinkhorn",
    "sknr",
    "spectral_basis",
    "normalize_gauge",
    "solve_schedule",
    "halving_ladder",
]


# ---------------------------------------------------------------- inputs

def sqeuclid_cost(x: np.ndarray, y: np.ndarray, scale: float = 1.0) -> np.ndarray:
    """C_ij = scale * ||x_i - y_j||^2 in float64 (squared Euclidean cost of
    the paper's experiments, Sec. 5)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    C = np.zeros((x.shape[0], y.shape[0]))
    for k in range(x.shape[1]):
        C += (x[:, k][:, None] - y[:, k][None, :]) ** 2
    return scale * C


def logsumexp(Z: np.ndarray, axis: int) -> np.ndarray:
    """log sum exp along ``axis`` with the usual max shift (an identity)."""
    mx = np.max(Z, axis=axis, keepdims=True)
    out = mx + np.log(np.sum(np.exp(Z - mx), axis=axis, keepdims=True))
    return np.squeeze(out, axis=axis)


# ------------------------------------------------------- c-transforms, Sec. 2

def c_transform_col(f: np.ndarray, C: np.ndarray, a: np.ndarray, eps: float) -> np.ndarray:
    """g = f^{C,eps} (eq. foc_g): g_j = -eps log sum_i a_i exp((f_i - C_ij)/eps)."""
    Z = (f[:, None] - C) / eps + np.log(a)[:, None]
    return -eps * logsumexp(Z, axis=0)


def c_transform_row(g: np.ndarray, C: np.ndarray, b: np.ndarray, eps: float) -> np.ndarray:
    """f = g^{C,eps} (eq. foc_f): f_i = -eps log sum_j b_j exp((g_j - C_ij)/eps)."""
    Z = (g[None, :] - C) / eps + np.log(b)[None, :]
    return -eps * logsumexp(Z, axis=1)


def coupling(f, g, C, a, b, eps) -> np.ndarray:
    """pi_ij = a_i b_j exp((f_i + g_j - C_ij)/eps) (eq. Optimal_P_epsilon)."""
    return a[:, None] * b[None, :] * np.exp((f[:, None] + g[None, :] - C) / eps)


def marginals(f, g, C, a, b, eps):
    """(pi 1_m, pi^T 1_n) of the coupling of (f, g)."""
    P = coupling(f, g, C, a, b, eps)
    return P.sum(axis=1), P.sum(axis=0)


def marginal_error(f, g, C, a, b, eps) -> float:
    """||pi 1_m - a||_1 + ||pi^T 1_n - b||_1: the convergence test of
    Algorithm 4.1, read with the L1 norm."""
    r, c = marginals(f, g, C, a, b, eps)
    return float(np.abs(r - a).sum() + np.abs(c - b).sum())


# ------------------------------------------------------------- objectives

def dual_value(f, g, C, a, b, eps) -> float:
    """Q_eps(f, g) = <f,a> + <g,b> - eps (sum_ij pi_ij - 1)  (eq. def_Q)."""
    P = coupling(f, g, C, a, b, eps)
    return float(f @ a + g @ b - eps * (P.sum() - 1.0))


def semidual_value(f, C, a, b, eps) -> float:
    """Q^semi_eps(f) = <f,a> + <f^{C,eps}, b>  (eq. def_Q_semi)."""
    return float(f @ a + c_transform_col(f, C, a, eps) @ b)


def transport_cost(f, g, C, a, b, eps) -> float:
    """<C, pi>."""
    return float((coupling(f, g, C, a, b, eps) * C).sum())


def primal_value(f, g, C, a, b, eps) -> float:
    """<C, pi> + eps KL(pi || a (x) b)  (eq. primal_EOT) evaluated at the
    coupling of (f, g); KL uses log(pi_ij / (a_i b_j)) = (f_i+g_j-C_ij)/eps."""
    P = coupling(f, g, C, a, b, eps)
    logratio = (f[:, None] + g[None, :] - C) / eps
    return float((P * C).sum() + eps * ((P * logratio).sum() - P.sum() + 1.0))


def dual_partials(f, g, x, y, a, b, eps, scale=1.0) -> dict:
    """Partial derivatives of Q_eps(f, g) (eq. def_Q) with respect to the
    problem data at fixed potentials, for the squared Euclidean cost
    C_ij = scale ||x_i - y_j||^2.  At the optimum they are the derivatives
    of W_eps (eq. primal_EOT / dual_EOT) by the envelope theorem (the
    potentials are stationary), so no implicit differentiation is needed
    for W_eps itself:
      dQ/dC_ij = pi_ij
      dQ/dx_i  = 2 scale sum_j pi_ij (x_i - y_j)
      dQ/dy_j  = 2 scale sum_i pi_ij (y_j - x_i)
      dQ/da_i  = f_i - eps sum_j b_j exp((f_i + g_j - C_ij)/eps)  (= f_i - eps r_i / a_i)
      dQ/db_j  = g_j - eps c_j / b_j
    with r, c the row and column sums of pi."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    C = sqeuclid_cost(x, y, scale)
    P = coupling(f, g, C, a, b, eps)
    r, c = P.sum(1), P.sum(0)
    return {
        "C": P,
        "x": 2.0 * scale * (r[:, None] * x - P @ y),
        "y": 2.0 * scale * (c[:, None] * y - P.T @ x),
        "a": f - eps * r / a,
        "b": g - eps * c / b,
    }


# ------------------------------------- semi-dual derivatives, App. A.1

def _ptilde(f, C, a, b, eps):
    """P~ = pi(f, f^{C,eps}), the coupling entering eq. dQ_semi / d2Q_semi."""
    return coupling(f, c_transform_col(f, C, a, eps), C, a, b, eps)


def semidual_gradient(f, C, a, b, eps) -> np.ndarray:
    """Euclidean gradient of Q^semi (eq. dQ_semi):  a - P~ 1_m."""
    return a - _ptilde(f, C, a, b, eps).sum(axis=1)


def semidual_hessian(f, C, a, b, eps) -> np.ndarray:
    """Dense Euclidean Hessian of Q^semi (eq. d2Q_semi):
    -(1/eps) [diag(P~ 1_m) - P~ diag(b)^-1 P~^T]."""
    P = _ptilde(f, C, a, b, eps)
    return -(np.diag(P.sum(axis=1)) - (P / b[None, :]) @ P.T) / eps


def semidual_hessian_apply(f, C, a, b, eps, V) -> np.ndarray:
    """H V for the Hessian of eq. d2Q_semi without forming H."""
    P = _ptilde(f, C, a, b, eps)
    r = P.sum(axis=1)
    return -(r[:, None] * V - P @ ((P.T @ V) / b[:, None])) / eps


def projected_newton(f, C, a, b, eps, V) -> dict:
    """The Newton-Raphson step of Algorithm 4.1 restricted to span(V).

    gradient  grad_V = V^T grad Q^semi(f)
    Hessian   hess_V = V^T (grad^2 Q^semi(f)) V        (negative definite
              on any V whose span avoids the constant vector)
    step      Delta f = -V hess_V^{-1} grad_V, solved with a Cholesky
              factorisation of -hess_V (Sec. 4, per-iteration complexity).
    Returns dict(grad, hess, coef, delta, ok); ok is False when -hess_V is
    not positive definite (the step is then not taken).
    """
    grad = V.T @ semidual_gradient(f, C, a, b, eps)
    hess = V.T @ semidual_hessian_apply(f, C, a, b, eps, V)
    hess = 0.5 * (hess + hess.T)
    try:
        L = np.linalg.cholesky(-hess)
    except np.linalg.LinAlgError:
        return dict(grad=grad, hess=hess, coef=None, delta=None, ok=False)
    # (-hess) coef = grad  <=>  coef = -hess^{-1} grad
    y = np.linalg.solve(L, grad)
    coef = np.linalg.solve(L.T, y)
    return dict(grad=grad, hess=hess, coef=coef, delta=V @ coef, ok=True)


# -------------------------------------------------------- Algorithm 4.1

@dataclasses.dataclass
class SolveResult:
    f: np.ndarray
    g: np.ndarray
    iters: int
    converged: bool
    errs: list
    newton_tried: int = 0
    newton_accepted: int = 0
    qsemi: list = dataclasses.field(default_factory=list)


def sinkhorn(C, a, b, eps, tol, max_iter, f0=None) -> SolveResult:
    """Log-domain Sinkhorn-Knopp (eq. SK_iterations): Algorithm 4.1 with
    l = 0.  Starts from f0 (zero by default, as in Algorithm 4.1)."""
    return sknr(C, a, b, eps, tol, max_iter, V=None, f0=f0)


def sknr(C, a, b, eps, tol, max_iter, V=None, f0=None) -> SolveResult:
    """Algorithm 4.1, SK-NR(l).

    Each iteration: g_k = f_{k-1}^{C,eps}; f_k = g_k^{C,eps}; stop when the
    marginal error of pi(f_k, g_k) is below ``tol``; otherwise, when
    dim V > 0, take the projected Newton step of ``projected_newton`` and
    keep it only if it strictly increases Q^semi.
    """
    n = C.shape[0]
    f = np.zeros(n) if f0 is None else np.array(f0, dtype=np.float64)
    ell = 0 if V is None else V.shape[1]
    errs, qs = [], []
    tried = accepted = 0
    g = None
    converged = False
    k = 0
    for k in range(1, max_iter + 1):
        g = c_transform_col(f, C, a, eps)
        f = c_transform_row(g, C, b, eps)
        err = marginal_error(f, g, C, a, b, eps)
        errs.append(err)
        if err < tol:
            converged = True
            break
        if ell > 0:
            q0 = semidual_value(f, C, a, b, eps)
            step = projected_newton(f, C, a, b, eps, V)
            tried += 1
            if step["ok"]:
                f1 = f + step["delta"]
                q1 = semidual_value(f1, C, a, b, eps)
                if q1 > q0:
                    f = f1
                    accepted += 1
            qs.append(semidual_value(f, C, a, b, eps))
    return SolveResult(f=f, g=g, iters=k, converged=converged, errs=errs,
                       newton_tried=tried, newton_accepted=accepted, qsemi=qs)


# ------------------------------------------ spectral warm start, Sec. 4

def spectral_basis(f, g, C, a, b, eps, ell, method="auto"):
    """Low-frequency basis V_l for the spectral warm start (Sec. 4).

    At a (near-)optimal pair (f, g) for ``eps``, the semi-dual Hessian is
    -(1/eps)(Id - R R^*) on L2(alpha) (eq. semidual_Hessian), with
    R R^* = M = diag(a)^-1 pi diag(b)^-1 pi^T.  M is self-adjoint in
    L2(alpha); its symmetric form is S = A A^T, A = diag(a)^-1/2 pi
    diag(b)^-1/2, whose eigenvalues are rho_k^2 (Theorem 3.1), rho_0 = 1 for
    the constant mode.  V_l collects the eigenvectors of M for rho_1 .. rho_l
    (the constant mode is dropped), i.e. diag(a)^-1/2 u_k with u_k the
    eigenvectors of S, which are orthonormal in L2(alpha).

    Returns (V, rho) with rho the square roots of the l+1 leading
    eigenvalues of S (rho[0] ~ 1).  ``method`` is "dense" (numpy eigh),
    "arpack" (scipy eigsh on S as an operator) or "auto".
    """
    P = coupling(f, g, C, a, b, eps)
    A = P / np.sqrt(a)[:, None] / np.sqrt(b)[None, :]
    n = A.shape[0]
    if method == "auto":
        method = "dense" if n <= 1500 else "arpack"
    if method == "dense":
        S = A @ A.T
        w, U = np.linalg.eigh(S)
        order = np.argsort(w)[::-1][: ell + 1]
        w, U = w[order], U[:, order]
    else:
        from scipy.sparse.linalg import LinearOperator, eigsh
        op = LinearOperator((n, n), matvec=lambda v: A @ (A.T @ v), dtype=np.float64)
        w, U = eigsh(op, k=ell + 1, which="LA", tol=1e-12, v0=np.sqrt(a))
        order = np.argsort(w)[::-1]
        w, U = w[order], U[:, order]
    V = U[:, 1:ell + 1] / np.sqrt(a)[:, None]
    return V, np.sqrt(np.clip(w, 0.0, None))


# ------------------------------------------------------- output gauge

def normalize_gauge(f, g, a, b):
    """Shift (f, g) by c(1, -1) so that <f,a> = <g,b> (the dual objective is
    invariant under this shift, Sec. 2)."""
    c = 0.5 * (g @ b - f @ a)
    return f + c, g - c


# ---------------------------------------------------------- eps schedules

def halving_ladder(eps0: float, eps_final: float) -> list:
    """eps0, eps0/2, ... halving until the next value would fall below
    eps_final, then eps_final itself."""
    out = [eps0]
    while out[-1] / 2 > eps_final * (1 + 1e-12):
        out.append(out[-1] / 2)
    if abs(out[-1] - eps_final) > 1e-15 * eps_final:
        out.append(eps_final)
    return out


def solve_schedule(C, a, b, eps_list, tol, max_iter, ell=0, mode="sequential",
                   eps_prime=None, f0=None):
    """An eps schedule (Sec. 5): stage s starts from the potential of stage
    s-1 (standard warm start).  With ell > 0 the stages after the first run
    SK-NR(ell) with V_ell computed from the previous stage's optimum
    ("sequential") or once from a vanilla SK solve at ``eps_prime``
    ("static").  The first stage is plain SK.  When n > m the problem is
    solved on its transpose (semi-dual on the smaller side, Sec. 2) and the
    potentials are swapped back.  Returns (f, g, [SolveResult per stage])."""
    C = np.asarray(C, dtype=np.float64)
    transposed = C.shape[0] > C.shape[1]
    if transposed:
        C, a, b = C.T, b, a
        if f0 is not None:
            raise ValueError("f0 with a transposed problem is not supported")
    V_static = None
    if ell > 0 and mode == "static":
        r = sinkhorn(C, a, b, eps_prime, tol, max_iter)
        V_static, _ = spectral_basis(r.f, r.g, C, a, b, eps_prime, ell)
    f = f0
    results = []
    prev = None
    for s, eps in enumerate(eps_list):
        V = None
        if ell > 0 and s > 0:
            V = V_static if mode == "static" else spectral_basis(prev.f, prev.g, C, a, b, eps_list[s - 1], ell)[0]
        r = sknr(C, a, b, eps, tol, max_iter, V=V, f0=f)
        results.append(r)
        f = r.f
        prev = r
    fo, go = results[-1].f, results[-1].g
    if transposed:
        fo, go = go, fo
    return fo, go, results
