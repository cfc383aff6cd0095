"""Write tests/golden/c2_oracle.npz: the FP64 oracle's solution of the
benchmark workload (4096 x 4096 points, d = 2, Gaussian mixture against
uniform, Dirichlet(5) weights, eps 1e-1 -> 1e-3 by halving in 8 stages).

Calls only the oracle and the seeded input generators.  Two runs:

* the schedule of Sec. 5 with the sequential spectral warm start, SK-NR(16)
  from the second stage on, each stage to an L1 marginal error of 1e-6
  (Algorithm 4.1): its per-stage iteration counts and Newton acceptances;
* the last stage continued from that point to an L1 marginal error of
  1e-11 (SK-NR with the same basis reaches the same optimum, Theorem 4.2):
  the optimum (f*, g*) in the gauge <f,a> = <g,b>, its transport cost
  <C, pi>, dual value and marginal error.

The cost is the exact squared distance (FP64) of the FP32 points.
Usage: python tests/golden/make_c2_oracle.py   (several minutes, one core)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

N, SEED, ELL = 4096, 1, 16


def main() -> None:
    prob = W.gmm_vs_uniform(N, seed=SEED)
    C = O.sqeuclid_cost(prob.x.astype(np.float64), prob.y.astype(np.float64))
    a, b = prob.a, prob.b
    ladder = list(W.EPS_LADDER_C2)
    t0 = time.perf_counter()
    f, g, rs = O.solve_schedule(C, a, b, ladder, 1e-6, 100000, ell=ELL, mode="sequential")
    t1 = time.perf_counter()
    print("stages", [r.iters for r in rs], "accepted", [r.newton_accepted for r in rs],
          f"{t1 - t0:.1f} s", flush=True)
    eps = ladder[-1]
    V, _ = O.spectral_basis(rs[-2].f, rs[-2].g, C, a, b, ladder[-2], ELL)
    r = O.sknr(C, a, b, eps, 1e-11, 100000, V=V, f0=rs[-1].f)
    assert r.converged
    fs, gs = O.normalize_gauge(r.f, r.g, a, b)
    print(f"optimum: {r.iters} more iterations, marginal {O.marginal_error(fs, gs, C, a, b, eps):.2e}, "
          f"{time.perf_counter() - t1:.1f} s", flush=True)
    f6, g6 = O.normalize_gauge(f, g, a, b)
    np.savez_compressed(
        os.path.join(HERE, "c2_oracle.npz"),
        n=N, seed=SEED, ell=ELL, eps=np.array(ladder),
        x_sum=float(prob.x.astype(np.float64).sum()), a_sum_sq=float((a * a).sum()),
        iters_tol1e6=np.array([q.iters for q in rs]),
        newton_accepted_tol1e6=np.array([q.newton_accepted for q in rs]),
        transport_cost_tol1e6=O.transport_cost(f6, g6, C, a, b, eps),
        f=fs, g=gs,
        transport_cost=O.transport_cost(fs, gs, C, a, b, eps),
        dual_value=O.dual_value(fs, gs, C, a, b, eps),
        marginal_err=O.marginal_error(fs, gs, C, a, b, eps),
    )


if __name__ == "__main__":
    main()
