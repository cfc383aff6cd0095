"""GPU tests of the serving runtime (continuous batching).

Every request of a mixed set (n, m, d, cost kind and target eps differ) is
solved alone with sknr_solve and then served in a mix in which later
requests arrive while earlier ones are on the device; the served
potentials must equal the solo ones bit for bit (the kernels of one
request do not depend on the others), and the solo results are themselves
parity-tested against the oracle elsewhere.  Admission by device memory,
cancellation and the error paths are checked on small pools.
"""
import time

import numpy as np
import pytest

import workloads as W
from tests._helpers import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_2506_14780_amd as sk
    return sk


def _mix(n_req=10, seed=17, n_max=1400):
    trace = W.serving_trace(n_requests=n_req, rate=1000.0, seed=seed, n_min=64, n_max=n_max,
                            eps_choices=(1e-1, 1e-2))
    return trace


def _gp(sk, prob, stored=False):
    a, b = to_dev(prob.a), to_dev(prob.b)
    if stored:
        C = (((prob.x[:, None, :].astype(np.float64) - prob.y[None, :, :]) ** 2).sum(-1) * prob.cost_scale)
        return sk.Problem(a=a, b=b, C=to_dev(C.astype(np.float32)))
    return sk.Problem(a=a, b=b, x=to_dev(prob.x), y=to_dev(prob.y), cost_scale=prob.cost_scale)


def _kw(req):
    n, m = req.problem.n, req.problem.m
    return dict(eps=W.request_ladder(req.eps), tol=1e-6, max_iter=20000, ell=min(10, min(n, m) - 1),
                warm_mode=0, seed=req.rid)


def test_serve_alone_equals_mix(sk):
    reqs = _mix()
    stored = {3, 7}  # two requests with a stored cost
    ctx = sk.Context(0)
    solo = []
    for q in reqs:
        kw = _kw(q)
        f, g, res = sk.solve(ctx, _gp(sk, q.problem, q.rid in stored), kw.pop("eps"), **kw)
        solo.append((f.cpu().numpy(), g.cpu().numpy(), res))
        print(f"solo {q.problem.name} eps={q.eps} iters={[s['iters'] for s in res['stages']][-3:]} "
              f"status={res['status']}", flush=True)
    ctx.close()

    ctx = sk.Context(0)
    sk.serve_config(ctx, max_active=4, pool_bytes=256 << 20, batched=True)
    tickets = {}
    first, second = reqs[:5], reqs[5:]
    for q in first:
        kw = _kw(q)
        tickets[q.rid] = sk.submit(ctx, _gp(sk, q.problem, q.rid in stored), kw.pop("eps"), **kw)
    # the rest arrive while the first ones are on the device
    t0 = time.time()
    while sk.serve_stats(ctx)["running"] == 0 and time.time() - t0 < 30:
        time.sleep(0.001)
    st = sk.serve_stats(ctx)
    print("stats after first wave", st, flush=True)
    for q in second:
        kw = _kw(q)
        tickets[q.rid] = sk.submit(ctx, _gp(sk, q.problem, q.rid in stored), kw.pop("eps"), **kw)
    for q, (fs, gs, rs) in zip(reqs, solo):
        f, g, res = sk.wait(ctx, tickets[q.rid], q.problem.n, q.problem.m)
        print(f"mix {q.problem.name} status={res['status']} queue={res['queue_seconds']:.4f}s "
              f"latency={res['latency_seconds']:.4f}s", flush=True)
        assert res["status"] == rs["status"]
        assert [s["iters"] for s in res["stages"]] == [s["iters"] for s in rs["stages"]]
        assert np.array_equal(f.cpu().numpy(), fs)
        assert np.array_equal(g.cpu().numpy(), gs)
        assert res["marginal_err"] == rs["marginal_err"]
        assert res["latency_seconds"] >= res["queue_seconds"] >= 0
    st = sk.serve_stats(ctx)
    print("final stats", st, flush=True)
    assert st["completed"] == len(reqs) and st["queued"] == 0 and st["running"] == 0
    assert st["pool_used"] == 0 and 0 < st["pool_peak"] <= st["pool_bytes"]
    ctx.close()


def test_serve_admission_by_memory(sk):
    """A pool that holds about two of these requests at a time: everything
    still completes, in bounded memory, with results equal to solo runs."""
    reqs = [q for q in _mix(n_req=24, seed=5, n_max=900) if q.problem.n * q.problem.m > 200_000][:6]
    assert len(reqs) >= 3
    ctx = sk.Context(0)
    solo = []
    for q in reqs:
        kw = _kw(q)
        f, g, _ = sk.solve(ctx, _gp(sk, q.problem), kw.pop("eps"), **kw)
        solo.append(f.cpu().numpy())
    ctx.close()
    ctx = sk.Context(0)
    # workspace of the largest request ~ its partial buffers; size the pool
    # from a first single-request run
    sk.serve_config(ctx, max_active=8, pool_bytes=64 << 20)
    kw = _kw(reqs[0])
    t = sk.submit(ctx, _gp(sk, reqs[0].problem), kw.pop("eps"), **kw)
    sk.wait(ctx, t, reqs[0].problem.n, reqs[0].problem.m)
    one = sk.serve_stats(ctx)["pool_peak"]
    ctx.close()
    ctx = sk.Context(0)
    pool = int(2.5 * one)
    sk.serve_config(ctx, max_active=8, pool_bytes=pool)
    tickets = []
    for q in reqs:
        kw = _kw(q)
        tickets.append(sk.submit(ctx, _gp(sk, q.problem), kw.pop("eps"), **kw))
    max_running = 0
    t0 = time.time()
    while sk.serve_stats(ctx)["completed"] < len(reqs) and time.time() - t0 < 120:
        max_running = max(max_running, sk.serve_stats(ctx)["running"])
        time.sleep(0.0005)
    st = sk.serve_stats(ctx)
    print("pool", pool, "one", one, "stats", st, "max running", max_running, flush=True)
    assert st["pool_peak"] <= pool
    assert max_running <= 3
    for q, t, fs in zip(reqs, tickets, solo):
        f, _, res = sk.wait(ctx, t, q.problem.n, q.problem.m)
        assert np.array_equal(f.cpu().numpy(), fs)
    ctx.close()


def test_serve_cancel_and_errors(sk):
    ctx = sk.Context(0)
    sk.serve_config(ctx, max_active=1, pool_bytes=64 << 20)
    big = W.uniform_square(1500, 1700, seed=3)
    gp = _gp(sk, big)
    # a long solve occupies the only lane; the second request stays queued
    t1 = sk.submit(ctx, gp, [1e-1, 5e-2, 2.5e-2, 1.25e-2, 6e-3], tol=1e-9, max_iter=200000, ell=8)
    t2 = sk.submit(ctx, gp, [1e-1], tol=1e-6, max_iter=1000)
    sk.cancel(ctx, t2)
    _, _, r2 = sk.wait(ctx, t2, 1500, 1700, raise_on_error=False)
    assert r2["status"] == sk.ECANCELED
    sk.cancel(ctx, t1)  # running: stops at its next poll
    _, _, r1 = sk.wait(ctx, t1, 1500, 1700, raise_on_error=False)
    assert r1["status"] in (sk.ECANCELED, sk.OK, sk.NOT_CONVERGED)
    # unknown ticket
    with pytest.raises(sk.SknrError) as e:
        sk.poll(ctx, 987654321)
    assert e.value.status == sk.EINVAL
    # a request larger than the pool
    import torch
    n = 4500  # a stored cost of 81 MB
    Cbig = torch.rand(n, n, device="cuda", dtype=torch.float32)
    w = to_dev(np.full(n, 1.0 / n))
    with pytest.raises(sk.SknrError) as e:
        sk.submit(ctx, sk.Problem(a=w, b=w, C=Cbig), [1e-1])
    assert e.value.status == sk.ENOMEM
    # config after start
    with pytest.raises(sk.SknrError) as e:
        sk.serve_config(ctx, 2, 0)
    assert e.value.status == sk.EBUSY
    # the lane still serves after all this
    t3 = sk.submit(ctx, _gp(sk, W.uniform_square(300, 200, seed=4)), [1e-1, 5e-2], tol=1e-6)
    _, _, r3 = sk.wait(ctx, t3, 300, 200)
    assert r3["status"] == sk.OK and r3["marginal_err"] < 1e-6
    ctx.close()


def test_batched_execution_equals_lanes_and_solo(sk):
    """Batched serving (the lanes hand their iteration chunks to one
    batcher, which launches each kernel once for every request with the
    same kernel sequence, over a tile table) against per-lane launches and
    against sknr_solve: the same potentials bit for bit, for a mix of point
    clouds with d = 2, 3 and 64 (VALU, matrix-core-layout and bf16
    matrix-core sweeps) arriving together.  The statistics must show
    batches that carried several requests."""
    trace = W.serving_trace(n_requests=12, rate=1000.0, seed=23, n_min=64, n_max=1200,
                            eps_choices=(1e-1, 1e-2))
    ctx = sk.Context(0)
    solo = []
    for q in trace:
        kw = _kw(q)
        f, g, res = sk.solve(ctx, _gp(sk, q.problem), kw.pop("eps"), **kw)
        solo.append((f.cpu().numpy(), g.cpu().numpy(), res))
    ctx.close()
    for batched in (True, False):
        ctx = sk.Context(0)
        sk.serve_config(ctx, max_active=8, pool_bytes=512 << 20, batched=batched)
        tickets = []
        for q in trace:
            kw = _kw(q)
            tickets.append(sk.submit(ctx, _gp(sk, q.problem), kw.pop("eps"), **kw))
        for q, t, (fs, gs, rs) in zip(trace, tickets, solo):
            f, g, res = sk.wait(ctx, t, q.problem.n, q.problem.m)
            assert res["status"] == rs["status"]
            assert [s["iters"] for s in res["stages"]] == [s["iters"] for s in rs["stages"]]
            assert np.array_equal(f.cpu().numpy(), fs) and np.array_equal(g.cpu().numpy(), gs)
        st = sk.serve_stats(ctx)
        print(f"batched={batched} d={[q.problem.d for q in trace]} stats {st}", flush=True)
        if batched:
            assert st["batches"] > 0 and st["batched_jobs"] > st["batches"]
        else:
            assert st["batches"] == 0
        ctx.close()


def test_served_result_matches_oracle(sk):
    """A served request against the FP64 oracle's optimum of the same
    problem (the oracle on the FP32 cost of the served points, eps ladder of
    the request)."""
    import oracle as O
    from tests._helpers import e_pot, fp32_sqeuclid
    q = [r for r in W.serving_trace(n_requests=40, rate=1000.0, seed=29, n_min=64, n_max=700,
                                    eps_choices=(1e-2,)) if r.problem.d in (2, 3)][0]
    ctx = sk.Context(0)
    sk.serve_config(ctx, max_active=4, pool_bytes=128 << 20)
    kw = _kw(q)
    ladder = kw.pop("eps")
    t = sk.submit(ctx, _gp(sk, q.problem), ladder, **kw)
    f, g, res = sk.wait(ctx, t, q.problem.n, q.problem.m)
    ctx.close()
    C = fp32_sqeuclid(q.problem.x, q.problem.y, q.problem.cost_scale).astype(np.float64)
    fo, go, _ = O.solve_schedule(C, q.problem.a, q.problem.b, ladder, 1e-11, 1000000)
    e = e_pot(f.cpu().numpy(), g.cpu().numpy(), fo, go, C)
    print(f"served {q.problem.name} eps {q.eps}: status {res['status']}, marginal {res['marginal_err']:.2e}, "
          f"e_pot vs the oracle {e:.2e}", flush=True)
    assert res["status"] == 0 and res["marginal_err"] < 1e-6 and e <= 1e-5
