"""Write tests/golden/c1_oracle.json: the FP64 oracle on the 256 x 256
workload (points uniform in [0,1]^2, seed 0, uniform weights, squared
Euclidean cost of the FP32 points in FP64, eps = 1e-2).

Calls only the oracle and the seeded input generators.  Protocols of Sec.
5 (Algorithm 4.1): cold SK from f = 0; warm SK from the optimum at eps';
warm SK-NR(l), l in {1, 2, 5, 10, 20, 30}, from the optimum at eps' with
V_l the eigenvectors of M at that optimum (eps' = 2e-2, the previous
stage of a halving ladder, and eps' = 1, the paper's static choice).
Iteration counts at the tolerances 1e-9 (the FP64 target of this
workload) and 1e-6 (the GPU's FP32 target), plus the optimum (f, g) at
1e-12 and its transport cost.

Usage: python tests/golden/make_c1_oracle.py   (about a minute)
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

N, SEED, EPS = 256, 0, 1e-2
ELLS = [1, 2, 5, 10, 20, 30]


def main() -> None:
    prob = W.uniform_square(N, seed=SEED)
    C = O.sqeuclid_cost(prob.x.astype(np.float64), prob.y.astype(np.float64))
    a, b = prob.a, prob.b
    out = {"n": N, "seed": SEED, "eps": EPS, "ells": ELLS, "x_sum": float(prob.x.astype(np.float64).sum())}
    for tol, key in ((1e-9, "tol1e-9"), (1e-6, "tol1e-6")):
        rec = {"cold_sk": O.sinkhorn(C, a, b, EPS, tol, 1000000).iters}
        for ep in (2e-2, 1.0):
            w = O.sinkhorn(C, a, b, ep, 1e-12, 1000000)
            V, rho = O.spectral_basis(w.f, w.g, C, a, b, ep, max(ELLS), method="dense")
            tag = f"eps_prime={ep:g}"
            rec[f"warm_sk {tag}"] = O.sinkhorn(C, a, b, EPS, tol, 1000000, f0=w.f).iters
            rec[f"warm_sknr {tag}"] = {str(l): O.sknr(C, a, b, EPS, tol, 1000000, V=V[:, :l], f0=w.f).iters
                                       for l in ELLS}
            rec[f"rho {tag}"] = [float(r) for r in rho]
        out[key] = rec
        print(key, json.dumps(rec)[:400], flush=True)
    ref = O.sinkhorn(C, a, b, EPS, 1e-12, 1000000)
    f, g = O.normalize_gauge(ref.f, ref.g, a, b)
    out["f"] = f.tolist()
    out["g"] = g.tolist()
    out["transport_cost"] = O.transport_cost(f, g, C, a, b, EPS)
    with open(os.path.join(HERE, "c1_oracle.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
