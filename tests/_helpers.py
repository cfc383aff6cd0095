"""Shared test helpers (not the oracle): device transfer, the FP32 cost
model of the GPU path, gauge-invariant error metrics."""
import numpy as np

U32 = 2.0 ** -24


def fp32_sqeuclid(x, y, scale=1.0):
    """The FP32 squared distance as the GPU defines it: t_k = x_k - y_k in
    FP32, acc = t_0^2 then acc = fma(t_k, t_k, acc) for k = 1..d-1, then a
    multiply by ``scale`` when it is not 1.  The fma is modelled by an
    exact float64 product and sum rounded once to float32 (exact up to rare
    double roundings)."""
    x = np.asarray(x, np.float32)
    y = np.asarray(y, np.float32)
    t = (x[:, None, 0] - y[None, :, 0]).astype(np.float32)
    acc = (t * t).astype(np.float32)
    for k in range(1, x.shape[1]):
        t = (x[:, None, k] - y[None, :, k]).astype(np.float32)
        acc = (t.astype(np.float64) * t.astype(np.float64) + acc.astype(np.float64)).astype(np.float32)
    if scale != 1.0:
        acc = (acc * np.float32(scale)).astype(np.float32)
    return acc


def e_pot(f1, g1, f2, g2, C):
    """Gauge-invariant potential error max_ij |df_i + dg_j| / (max C - min C)."""
    df = np.asarray(f1) - np.asarray(f2)
    dg = np.asarray(g1) - np.asarray(g2)
    e = max(abs(df.max() + dg.max()), abs(df.min() + dg.min()))
    return e / (C.max() - C.min())


def to_dev(arr, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(arr))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_problem(prob, stored=False, C32=None):
    """paper_2506_14780_amd.Problem from a workloads.Problem."""
    import paper_2506_14780_amd as sk
    a = to_dev(prob.a.astype(np.float64))
    b = to_dev(prob.b.astype(np.float64))
    if stored:
        C = C32 if C32 is not None else prob.C
        return sk.Problem(a=a, b=b, C=to_dev(np.asarray(C, np.float32)))
    return sk.Problem(a=a, b=b, x=to_dev(prob.x.astype(np.float32)), y=to_dev(prob.y.astype(np.float32)),
                      cost_scale=prob.cost_scale)


def bf16_rne(v):
    """float32 -> the nearest bf16 value (round to nearest even), as float32."""
    u = np.ascontiguousarray(v, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def bf16_cost_model(x, y, scale=1.0, x3=True, mu_points=None, parts=None):
    """The matrix-core cost as the library defines it, in FP64, with a
    rigorous per-element bound on the GPU's deviation from it.

    Centre mu = bf16(mean of all points); v = fl32(x - mu) split into bf16
    parts: hi = bf16(v) (1 part), lo = bf16(v - hi) (2 parts), or mid =
    bf16(v - hi), lo = bf16(v - hi - mid) (3 parts); x~ = the sum of the
    parts; n_i = fl32(scale ||x~_i||^2); model C_ij = n_i + n_j -
    2 fl32(scale) (x~_i . y~_j) over the kept products (hi*hi; + hi*lo +
    lo*hi; or + hi*mid + mid*hi + hi*lo + lo*hi + mid*mid).  The GPU forms
    the dot product on matrix cores (FP32 accumulation, any order: error <=
    (N - 1) u sum|terms| over N products), adds the norms in FP32 and applies
    one fma: bound = 2 s N u T_ij + 2 u (n_i + n_j) + u |C_ij| (the second
    term also covers a last-bit difference of the FP64 norm).
    parts defaults to 2 if x3 else 1.  mu_points: the full point sets (x, y)
    when x or y is only a subset of the rows of the problem."""
    parts = parts if parts is not None else (2 if x3 else 1)
    x = np.asarray(x, np.float32)
    y = np.asarray(y, np.float32)
    d = x.shape[1]
    dpad = (d + 31) // 32 * 32
    px, py = mu_points if mu_points is not None else (x, y)
    mu = bf16_rne(np.float32(np.concatenate([np.asarray(px, np.float32), np.asarray(py, np.float32)])
                             .astype(np.float64).mean(axis=0)))

    def split(p):
        v = (p - mu).astype(np.float32)
        hi = bf16_rne(v)
        r1 = (v - hi).astype(np.float32)
        if parts == 1:
            out = [hi]
        elif parts == 2:
            out = [hi, bf16_rne(r1)]
        else:
            mid = bf16_rne(r1)
            out = [hi, mid, bf16_rne((r1 - mid).astype(np.float32))]
        return [o.astype(np.float64) for o in out]

    X, Y = split(x), split(y)
    s32 = float(np.float32(scale))
    nx = np.float32(scale * (sum(X) ** 2).sum(1)).astype(np.float64)
    ny = np.float32(scale * (sum(Y) ** 2).sum(1)).astype(np.float64)
    pairs = {1: [(0, 0)], 2: [(0, 0), (0, 1), (1, 0)],
             3: [(0, 0), (0, 1), (1, 0), (0, 2), (2, 0), (1, 1)]}[parts]
    E = sum(X[i] @ Y[j].T for i, j in pairs)
    T = sum(np.abs(X[i]) @ np.abs(Y[j]).T for i, j in pairs)
    nprod = len(pairs) * dpad
    C = nx[:, None] + ny[None, :] - 2.0 * s32 * E
    bound = 2.0 * s32 * nprod * U32 * T + 2 * U32 * (nx[:, None] + ny[None, :]) + U32 * np.abs(C)
    return C, bound
