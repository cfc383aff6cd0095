"""Seeded synthetic inputs for entropic OT problems.

This module only draws random inputs.  It holds none of the solver's
arithmetic, so both the CPU oracle and the GPU path may import it.  Every
array is drawn in float64 from ``numpy.random.default_rng(seed)`` and the
point clouds / stored costs are rounded once to float32, so that both sides
consume bit-identical inputs; weights stay float64 and are normalised to
sum to one.

Shapes and distributions follow the problem families of the paper
(Sec. 5 for the 2-D Gaussian clouds and the single-cell sizes, Sec. 3 for
the uniform square / annulus / two-moons measures) and the benchmark
configurations built on them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem",
    "uniform_square",
    "gmm_vs_uniform",
    "grid_histograms",
    "gaussian_clouds",
    "paper_2d_gaussians",
    "square_vs_annulus",
    "two_moons",
    "wot_shaped",
    "separable_cost",
    "serving_trace",
    "EPS_LADDER_C2",
]

# eps annealing ladder of the 4096x4096 d=2 workload: halve from 1e-1 and
# clamp the last stage at 1e-3.
EPS_LADDER_C2 = (1e-1, 5e-2, 2.5e-2, 1.25e-2, 6.25e-3, 3.125e-3, 1.5625e-3, 1e-3)


@dataclasses.dataclass
class Problem:
    """One OT instance.  Either ``C`` (stored n x m float32 cost) or the
    point clouds ``x`` (n x d) and ``y`` (m x d) are set; ``cost_scale``
    multiplies the squared Euclidean distance when the cost is built from
    points (1.0 means the plain squared distance)."""

    a: np.ndarray
    b: np.ndarray
    x: np.ndarray | None = None
    y: np.ndarray | None = None
    C: np.ndarray | None = None
    cost_scale: float = 1.0
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.a.shape[0])

    @property
    def m(self) -> int:
        return int(self.b.shape[0])

    @property
    def d(self) -> int:
        return 0 if self.x is None else int(self.x.shape[1])


def _norm(w: np.ndarray) -> np.ndarray:
    w = np.asarray(w, dtype=np.float64)
    return w / w.sum()


def uniform_square(n: int = 256, m: int | None = None, seed: int = 0) -> Problem:
    """Points i.i.d. uniform in [0,1]^2 on both sides, uniform weights."""
    m = n if m is None else m
    rng = np.random.default_rng(seed)
    x = rng.random((n, 2)).astype(np.float32)
    y = rng.random((m, 2)).astype(np.float32)
    return Problem(a=np.full(n, 1.0 / n), b=np.full(m, 1.0 / m), x=x, y=y,
                   name=f"uniform_square_{n}x{m}")


def gmm_vs_uniform(n: int = 4096, m: int | None = None, seed: int = 1,
                   components: int = 3, sigma: float = 0.05,
                   dirichlet: float = 5.0, d: int = 2) -> Problem:
    """x from a Gaussian mixture (means ~ U[0.2,0.8]^d, equal weights,
    isotropic sigma), y uniform in [0,1]^d; weights Dirichlet(dirichlet*1)."""
    m = n if m is None else m
    rng = np.random.default_rng(seed)
    means = rng.uniform(0.2, 0.8, size=(components, d))
    comp = rng.integers(0, components, size=n)
    x = (means[comp] + sigma * rng.standard_normal((n, d))).astype(np.float32)
    y = rng.random((m, d)).astype(np.float32)
    a = _norm(rng.dirichlet(np.full(n, dirichlet)))
    b = _norm(rng.dirichlet(np.full(m, dirichlet)))
    return Problem(a=a, b=b, x=x, y=y, name=f"gmm_vs_uniform_{n}x{m}_d{d}")


def grid_histograms(side: int = 128, seed: int = 2, bumps: int = 5,
                    floor: float = 1e-6, build_cost: bool = True) -> Problem:
    """Two densities on a side x side grid of [0,1]^2 (n = m = side^2).

    Each density is a Dirichlet(1)-weighted mixture of ``bumps`` isotropic
    Gaussians with means ~ U[0.15,0.85]^2 and widths ~ U[0.03,0.15],
    plus a ``floor`` and normalised.  The stored cost is the squared grid
    distance halved (so it lies in [0,1]), rounded to float32, row-major.
    """
    rng = np.random.default_rng(seed)
    t = np.arange(side, dtype=np.float64) / (side - 1)
    gx, gy = np.meshgrid(t, t, indexing="ij")
    pts = np.stack([gx.ravel(), gy.ravel()], axis=1)

    def density() -> np.ndarray:
        w = rng.dirichlet(np.ones(bumps))
        mu = rng.uniform(0.15, 0.85, size=(bumps, 2))
        s = rng.uniform(0.03, 0.15, size=bumps)
        dens = np.zeros(pts.shape[0])
        for c in range(bumps):
            r2 = ((pts - mu[c]) ** 2).sum(axis=1)
            dens += w[c] * np.exp(-0.5 * r2 / s[c] ** 2) / (2 * math.pi * s[c] ** 2)
        dens = dens / dens.sum() + floor
        return _norm(dens)

    a = density()
    b = density()
    C = None
    if build_cost:
        N = pts.shape[0]
        C = np.empty((N, N), dtype=np.float32)
        blk = 512
        for i0 in range(0, N, blk):
            p = pts[i0:i0 + blk]
            C[i0:i0 + blk] = (0.5 * ((p[:, None, :] - pts[None, :, :]) ** 2).sum(-1)).astype(np.float32)
    return Problem(a=a, b=b, C=C, x=pts.astype(np.float32), y=pts.astype(np.float32),
                   cost_scale=0.5, name=f"grid_histograms_{side}x{side}")


def gaussian_clouds(n: int = 20000, m: int = 30000, d: int = 64, seed: int = 3,
                    shift: float = 0.5) -> Problem:
    """x ~ N(0, I_d), y ~ N(shift*e_1, I_d), uniform weights."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d)).astype(np.float32)
    y = rng.standard_normal((m, d))
    y[:, 0] += shift
    y = y.astype(np.float32)
    return Problem(a=np.full(n, 1.0 / n), b=np.full(m, 1.0 / m), x=x, y=y,
                   name=f"gaussian_clouds_{n}x{m}_d{d}")


def paper_2d_gaussians(n: int = 200, seed: int = 5) -> Problem:
    """The 2-D experiment of Sec. 5: n samples of N((0,0), I) against 2n
    samples of N((4,4), [[1,-0.8],[-0.8,1]]), uniform weights."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 2))
    L = np.linalg.cholesky(np.array([[1.0, -0.8], [-0.8, 1.0]]))
    y = rng.standard_normal((2 * n, 2)) @ L.T + np.array([4.0, 4.0])
    return Problem(a=np.full(n, 1.0 / n), b=np.full(2 * n, 1.0 / (2 * n)),
                   x=x.astype(np.float32), y=y.astype(np.float32),
                   name=f"paper_2d_gaussians_{n}")


def square_vs_annulus(n: int = 300, m: int | None = None, seed: int = 8, r_in: float = 0.5,
                      r_out: float = 1.0) -> Problem:
    """Sec. 3's square / annulus pair: x uniform on [-1,1]^2, y uniform on
    the annulus r_in <= |y| <= r_out (radius drawn with density ~ r),
    uniform weights."""
    m = n if m is None else m
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, size=(n, 2))
    r = np.sqrt(rng.uniform(r_in ** 2, r_out ** 2, size=m))
    t = rng.uniform(0.0, 2.0 * math.pi, size=m)
    y = np.stack([r * np.cos(t), r * np.sin(t)], axis=1)
    return Problem(a=np.full(n, 1.0 / n), b=np.full(m, 1.0 / m), x=x.astype(np.float32),
                   y=y.astype(np.float32), name=f"square_vs_annulus_{n}x{m}")


def two_moons(n: int = 300, m: int | None = None, seed: int = 9, noise: float = 0.05) -> Problem:
    """Sec. 3's two-moons pair: x uniform on the upper half circle of radius
    1 centred at 0, y uniform on the lower half circle centred at (1, 0.5),
    both with isotropic Gaussian jitter `noise`; uniform weights."""
    m = n if m is None else m
    rng = np.random.default_rng(seed)
    t1 = rng.uniform(0.0, math.pi, size=n)
    x = np.stack([np.cos(t1), np.sin(t1)], axis=1) + noise * rng.standard_normal((n, 2))
    t2 = rng.uniform(0.0, math.pi, size=m)
    y = np.stack([1.0 - np.cos(t2), 0.5 - np.sin(t2)], axis=1) + noise * rng.standard_normal((m, 2))
    return Problem(a=np.full(n, 1.0 / n), b=np.full(m, 1.0 / m), x=x.astype(np.float32),
                   y=y.astype(np.float32), name=f"two_moons_{n}x{m}")


def wot_shaped(n: int = 6507, m: int = 3815, d: int = 30, seed: int = 10, components: int = 6,
               drift: float = 0.35) -> Problem:
    """A synthetic stand-in at the shape of Sec. 5's single-cell maps (day 7
    -> 8: 6507 x 3815; day 8 -> 9: 3815 x 2982; PCA to R^30, normalised).
    Each side is a Gaussian mixture in R^d whose per-axis variances decay
    like the spectrum of a PCA (sigma_k^2 ~ 1/k); the second time point
    moves every component mean by `drift` along a random direction and adds
    one new component.  Both clouds are centred on their joint mean and
    scaled by one factor so that the mean squared norm is 1 (the cost
    ||x - y||^2 is then O(1)).  Uniform weights.  No data of the original
    study is used."""
    rng = np.random.default_rng(seed)
    sd = 1.0 / np.sqrt(np.arange(1, d + 1))
    means = rng.standard_normal((components, d)) * sd * 1.5
    wx = rng.dirichlet(np.full(components, 3.0))
    cx = rng.choice(components, size=n, p=wx)
    x = means[cx] + 0.5 * rng.standard_normal((n, d)) * sd
    step = rng.standard_normal((components, d)) * sd
    step *= drift / np.linalg.norm(step, axis=1, keepdims=True)
    means2 = np.concatenate([means + step, rng.standard_normal((1, d)) * sd * 1.5])
    wy = rng.dirichlet(np.full(components + 1, 3.0))
    cy = rng.choice(components + 1, size=m, p=wy)
    y = means2[cy] + 0.5 * rng.standard_normal((m, d)) * sd
    mu = np.concatenate([x, y]).mean(axis=0)
    x, y = x - mu, y - mu
    s = math.sqrt(np.concatenate([(x ** 2).sum(1), (y ** 2).sum(1)]).mean())
    return Problem(a=np.full(n, 1.0 / n), b=np.full(m, 1.0 / m), x=(x / s).astype(np.float32),
                   y=(y / s).astype(np.float32), name=f"wot_shaped_{n}x{m}_d{d}")


def separable_cost(n: int, m: int, seed: int = 7) -> tuple[Problem, np.ndarray, np.ndarray]:
    """A stored cost C_ij = u_i + v_j (float32-exact sums of small dyadic
    values), random Dirichlet weights.  Returns (problem, u, v)."""
    rng = np.random.default_rng(seed)
    u = np.round(rng.random(n) * 256) / 256.0
    v = np.round(rng.random(m) * 256) / 256.0
    C = (u[:, None] + v[None, :]).astype(np.float32)
    a = _norm(rng.dirichlet(np.full(n, 3.0)))
    b = _norm(rng.dirichlet(np.full(m, 3.0)))
    return Problem(a=a, b=b, C=C, name=f"separable_{n}x{m}"), u, v


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds from trace start
    eps: float              # target regularisation
    problem: Problem


def serving_trace(n_requests: int = 2048, rate: float = 100.0, seed: int = 4,
                  n_min: int = 64, n_max: int = 8192, dims=(2, 3, 64),
                  eps_choices=(1e-1, 1e-2, 1e-3), materialise: bool = True) -> list[Request]:
    """Poisson arrivals at ``rate`` per second; n and m independently
    log-uniform on [n_min, n_max]; d uniform over ``dims``; target eps
    uniform over ``eps_choices``; x, y from 3-component Gaussian mixtures
    (means ~ U[0,1]^d, sigma 0.05); weights Dirichlet(5).  The cost of a
    request is the squared distance divided by d (``cost_scale = 1/d``)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    out = []
    for r in range(n_requests):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        m = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        d = int(dims[rng.integers(0, len(dims))])
        eps = float(eps_choices[rng.integers(0, len(eps_choices))])
        sub = np.random.default_rng([seed, r])
        if materialise:
            mx = sub.random((3, d))
            my = sub.random((3, d))
            x = (mx[sub.integers(0, 3, n)] + 0.05 * sub.standard_normal((n, d))).astype(np.float32)
            y = (my[sub.integers(0, 3, m)] + 0.05 * sub.standard_normal((m, d))).astype(np.float32)
            a = _norm(sub.dirichlet(np.full(n, 5.0)))
            b = _norm(sub.dirichlet(np.full(m, 5.0)))
        else:
            x = y = None
            a = np.zeros(n)
            b = np.zeros(m)
        out.append(Request(rid=r, arrival=float(t[r]), eps=eps,
                           problem=Problem(a=a, b=b, x=x, y=y, cost_scale=1.0 / d,
                                           name=f"req{r}_{n}x{m}_d{d}")))
    return out


def request_ladder(target: float, eps0: float = 1.0) -> list[float]:
    """eps schedule of a serving request: halving from eps0 while above the
    target, then the target itself (Sec. 5 anneals eps from 1 by halving)."""
    out = [eps0]
    while out[-1] * 0.5 > target * (1 + 1e-12):
        out.append(out[-1] * 0.5)
    if out[-1] > target:
        out.append(target)
    return out

