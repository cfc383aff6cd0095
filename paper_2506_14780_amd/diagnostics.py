"""Spectral diagnostics of entropic OT and measured convergence rates
(paper Sec. 3: the spectrum of K_eps and the stability of its eigenvectors
across eps; the contraction factors rho_1^2 of SK and rho_{l+1}^2 of SK-NR
in Sec. 3's linearisation lemma and the convergence theorem of Sec. 4).

Everything that touches the n x m problem runs in the library's kernels
through the C ABI: the SK optimum at each eps (``solve``), the Ritz values
and the L2(a)-orthonormal basis of the top eigenvectors
(``spectral_basis``), and the FP64 marginal error of an iterate after a
given number of iterations (``solve`` from a fixed start with an
unreachable tolerance).  The host only loops over eps and iteration counts
and forms k x k matrices (principal angles between two bases).
"""
from __future__ import annotations

import numpy as np

from . import WARM_USER, Context, Problem, solve, spectral_basis

__all__ = ["spectrum", "principal_cosines", "error_history", "contraction_rate"]


def spectrum(ctx: Context, prob: Problem, eps_list, k: int, tol: float = 1e-8, max_iter: int = 20000,
             oversample: int = 8, eig_max_iter: int = 300, eig_tol: float = 1e-10, seed: int = 0):
    """For each eps: the SK optimum of the problem at that eps (one-stage
    solve to ``tol``; FP32 sweeps reach about 1e-7, so a smaller tol runs to
    ``max_iter``), then the top-k non-constant eigenpairs of
    K_eps at the optimum (Ritz values rho_1 >= ... >= rho_k, rho_0 = 1 for
    the constants).  Sec. 3 plots the smallest eigenvalues of Id + K_eps,
    which are 1 - rho_j.

    Returns a list of dicts {eps, rho (k+1 values, host), V (n x k float64
    device tensor, orthonormal in L2(a)), f (device), iters, eig_iters,
    marginal_err}."""
    out = []
    for eps in eps_list:
        f, g, res = solve(ctx, prob, [float(eps)], tol=tol, max_iter=max_iter)
        V, rho, it = spectral_basis(ctx, prob, float(eps), f, k, oversample=oversample, max_iter=eig_max_iter,
                                    tol=eig_tol, seed=seed)
        out.append({"eps": float(eps), "rho": rho, "V": V, "f": f, "iters": res["total_iters"],
                    "eig_iters": it, "marginal_err": res["marginal_err"]})
    return out


def principal_cosines(V1, V2, a) -> np.ndarray:
    """Cosines of the principal angles between span(V1) and span(V2) in
    L2(a) (both n x k with L2(a)-orthonormal columns): the singular values
    of V1^T diag(a) V2, in decreasing order.  All ones: the same subspace."""
    V1 = np.asarray(V1.cpu() if hasattr(V1, "cpu") else V1, dtype=np.float64)
    V2 = np.asarray(V2.cpu() if hasattr(V2, "cpu") else V2, dtype=np.float64)
    a = np.asarray(a.cpu() if hasattr(a, "cpu") else a, dtype=np.float64)
    return np.clip(np.linalg.svd(V1.T @ (a[:, None] * V2), compute_uv=False), 0.0, 1.0)


def error_history(ctx: Context, prob: Problem, eps: float, iters, ell: int = 0, V=None, f0=None):
    """FP64 L1 marginal error of the iterate f_k, k in ``iters``, at a fixed
    eps from the start ``f0`` (None: f = 0): plain SK (ell = 0) or SK-NR
    with the fixed basis V (n x ell float64 device tensor; the first
    iteration of Algorithm 4.1 has no Newton step).  Each k is one solve
    with max_iter = k and a tolerance that is never met, so f_k is the
    library's own k-th iterate."""
    errs = []
    for k in iters:
        kw = dict(tol=1e-300, max_iter=int(k), f0=f0)
        if ell > 0:
            kw.update(ell=int(ell), warm_mode=WARM_USER, V0=V, first_stage_nr=True)
        _, _, res = solve(ctx, prob, [float(eps)], **kw)
        errs.append(res["marginal_err"])
    return np.asarray(errs, dtype=np.float64)


def contraction_rate(iters, errs, lo: float = 1e-7, hi: float = 1e-2) -> float:
    """Per-iteration contraction factor over the iterations whose error lies
    in [lo, hi] (past the transient, above the FP32 floor): the slope of
    log(err) against k by least squares, returned as exp(slope).  NaN if
    fewer than three points qualify."""
    k = np.asarray(iters, dtype=np.float64)
    e = np.asarray(errs, dtype=np.float64)
    sel = (e >= lo) & (e <= hi)
    if sel.sum() < 3:
        return float("nan")
    slope = np.polyfit(k[sel], np.log(e[sel]), 1)[0]
    return float(np.exp(slope))
