"""Serving loop: admission logic on the CPU; on the GPU, every request's
answer is the same served in the mix as solved alone."""
import threading
import time

import numpy as np
import pytest

from paper_1907_12334_amd import inputs as I
from paper_1907_12334_amd.serve import Admission, Request, work_estimate


def _req(k, P, Q):
    return Request(rid=k, sample_id=k, P=P, Q=Q)


def _adm(budget=1000, foot=lambda P, Q: 10 * (P + Q), **kw):
    return Admission(budget, foot, lambda P, Q: work_estimate(4, P, Q), **kw)


def test_fifo_order_and_batch_cap():
    a = _adm(max_batch=3)
    for k in range(7):
        a.submit(_req(k, 1, 1))
    b1, n1 = a.take("small")
    b2, n2 = a.take("small")
    b3, _ = a.take("small")
    assert [r.rid for r in b1] == [0, 1, 2] and [r.rid for r in b2] == [3, 4, 5] and [r.rid for r in b3] == [6]
    assert n1 == 60 and a.reserved == 60 * 2 + 20


def test_budget_blocks_until_release():
    a = _adm(budget=100)
    for k in range(3):
        a.submit(_req(k, 2, 2))           # 40 bytes each
    b1, n1 = a.take("small")
    assert [r.rid for r in b1] == [0, 1] and n1 == 80
    b2, n2 = a.take("small")
    assert b2 == [] and n2 == 0           # the head does not fit the rest of the budget
    a.release(n1)
    b3, n3 = a.take("small")
    assert [r.rid for r in b3] == [2] and a.reserved == 40


def test_work_cap_and_lanes():
    big = work_estimate(4, 6, 6)
    a = _adm(budget=10 ** 9, max_batch_work=2.5 * work_estimate(4, 3, 3), big_work=big)
    a.submit(_req(0, 6, 6))
    for k in range(1, 5):
        a.submit(_req(k, 3, 3))
    assert a.lane_of(6, 6) == "big" and a.lane_of(3, 3) == "small"
    bb, _ = a.take("big")
    assert [r.rid for r in bb] == [0]
    bs, _ = a.take("small")
    assert [r.rid for r in bs] == [1, 2]  # a third would pass the work cap


def test_oversized_request_is_rejected():
    a = _adm(budget=50)
    with pytest.raises(ValueError):
        a.submit(_req(0, 4, 4))           # 80 bytes > whole budget


def test_wait_batch_wakes_on_submit_and_stops():
    a = _adm()
    got = []

    def worker():
        while True:
            r = a.wait_batch("small")
            if r is None:
                return
            got.extend(x.rid for x in r[0])
            a.release(r[1])

    t = threading.Thread(target=worker)
    t.start()
    for k in range(5):
        a.submit(_req(k, 1, 1))
        time.sleep(0.01)
    time.sleep(0.1)
    a.stop()
    t.join(5)
    assert not t.is_alive() and got == [0, 1, 2, 3, 4] and a.reserved == 0


def test_request_trace_shape():
    t, P, Q, ids = I.request_trace(2000, 5000.0)
    assert np.all(np.diff(t) > 0) and P.min() >= 1 and P.max() <= 9 and Q.min() >= 1
    # geometric size law: about half the requests have l = 1 per direction
    assert 0.4 < np.mean(P == 1) < 0.6 and 0.4 < np.mean(Q == 1) < 0.6
    assert abs(np.mean(np.diff(t)) - 1 / 5000.0) < 0.2 / 5000.0


@pytest.mark.gpu
def test_served_in_mix_equals_alone():
    import torch
    from paper_1907_12334_amd import msg
    from paper_1907_12334_amd.serve import Engine, replay, summarize

    c = 4
    opts = msg.SolveOpts(tol=1e-8, max_cycles=200, precision=msg.MIXED)
    rng = np.random.default_rng(7)
    n = 48
    P = rng.integers(1, 5, size=n)
    Q = rng.integers(1, 5, size=n)
    ids = np.arange(1000, 1000 + n)
    eng = Engine(I.KL10, c, opts, workers=3, big_workers=1, max_batch=8, big_work=work_estimate(c, 4, 4),
                 budget_bytes=8 << 30)
    try:
        reqs = replay(eng, np.zeros(n), P, Q, ids, want_u=True, timeout=300)
    finally:
        eng.close()
    s = summarize(reqs)
    assert s["errors"] == 0 and s["requests"] == n
    assert eng.max_inflight >= 2                 # batches overlapped on the device
    assert all(r.lane in ("small", "big") for r in reqs) and "small_lane" in s
    h = msg.Handle(0)
    worst = 0.0
    for r in reqs[::3]:
        b = msg.Batch(c, [r.P], [r.Q])
        bufs = msg.run(h, I.KL10, b, opts, None, seed=I.BASE_SEED + 5, sample_id=[r.sample_id])
        u = bufs.u.cpu().numpy()
        q = bufs.q.cpu().numpy()
        dq = bufs.dq.cpu().numpy()
        assert int(bufs.status.cpu()[0]) == r.status
        assert np.array_equal(bufs.cycles.cpu().numpy(), r.cycles)
        for a, m in ((u, r.u), (q, r.q), (dq, r.dq)):
            worst = max(worst, float(np.max(np.abs(a - m)) / max(np.max(np.abs(a)), 1e-300)))
    assert worst <= 1e-8, worst


@pytest.mark.gpu
def test_served_answers_match_the_oracle():
    """Requests served from a mix (mixed precision refined to 1e-8, normals
    drawn on the device from the engine's streams): Q and Delta Q on every
    grid within 1e-8 of the FP64 oracle run to 1e-10 on the oracle's own
    normals of the same streams."""
    from oracle import binding as O
    from oracle import normals as N
    from paper_1907_12334_amd import msg
    from paper_1907_12334_amd.serve import Engine, replay

    c, seed = 4, I.BASE_SEED + 5
    opts = msg.SolveOpts(tol=1e-8, max_cycles=200, precision=msg.MIXED)
    t, P, Q, ids = I.request_trace(64, 5000.0)
    keep = (P + Q) <= 7                                   # the oracle stays quick
    P, Q, ids, t = P[keep], Q[keep], ids[keep], t[keep] - t[keep][0]
    eng = Engine(I.KL10, c, opts, workers=3, big_workers=1, budget_bytes=8 << 30, seed=seed)
    try:
        reqs = replay(eng, t, P, Q, ids, timeout=300)
    finally:
        eng.close()
    worst = 0.0
    for r in reqs[::2]:
        xi = N.kl_normals(I.KL10.n_terms, [r.sample_id], seed)[0]
        kx, ky = O.hierarchy_field(c, r.P, r.Q, I.KL10.as_dict(), xi)
        ora = O.fmsg_solve(c, r.P, r.Q, kx, ky, O.opts(tol=1e-10, max_cycles=200))
        assert r.status == 0 and ora["status"] == 0
        dq = O.delta_q(r.P, r.Q, ora["q"])
        worst = max(worst, float(np.max(np.abs(r.q - ora["q"]) / np.abs(ora["q"]))),
                    float(np.max(np.abs(r.dq - dq)) / np.max(np.abs(ora["q"]))))
    print(f"served vs oracle: {len(reqs[::2])} requests, worst {worst:.2e}", flush=True)
    assert worst <= 1e-8, worst
