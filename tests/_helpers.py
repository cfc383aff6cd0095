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
