"""Request scheduler (continuous batching of Lanczos-shaped sessions): every
result of the mixed run equals the same request run alone."""
import random
import time

import numpy as np
import pytest

import seeded_inputs as si
from oracle import hankel
from tests.gpu_util import announce, need_gpu, torch

pytestmark = pytest.mark.gpu


def test_mixed_sessions_equal_alone():
    need_gpu()
    from paper_1402_5287_amd import hmv, serving
    mats = [("hankel", 64, 3322), ("toeplitz", 300, 1024), ("circulant", 1000, 3322),
            ("hankel", 700, 700), ("hankel", 4000, 33220), ("hankel", 8000, 33220)]
    plans, host_h = [], []
    for i, (kind, n, P) in enumerate(mats):
        hl = n if kind == "circulant" else 2 * n - 1
        h = si.uniform(hl, P, (90, i))
        host_h.append(h)
        plans.append(hmv.Plan(kind, hmv.to_device(h), n, P, algo="auto"))
    biggest = max(p.mv_ws_bytes for p in plans)
    # a pool that holds about two of the largest workspaces: admission must wait
    server = hmv.Server(pool_bytes=int(2.3 * biggest), slots=4)
    mids = [server.add_plan(p) for p in plans]
    rng = random.Random(3)
    sessions, host_x = [], {}
    arr = serving.poisson_arrivals(400.0, 10, rng)
    for sid in range(10):
        m = sid if sid < len(mats) else rng.randrange(len(mats))   # every matrix is used
        kind, n, P = mats[m]
        xs, ys = [], []
        for k in range(rng.randint(3, 8)):
            x = si.uniform(n, P, (91, sid, k))
            host_x[(sid, k)] = x
            xs.append(hmv.to_device(x))
            ys.append(torch.zeros((n, hmv.words(P)), dtype=torch.int64, device="cuda"))
        sessions.append(serving.Session(sid=sid, matrix_id=mids[m], arrival=arr[sid], xs=xs, ys=ys))
    announce("serving", len(sessions))
    wall, lats, recs = serving.run(server, sessions, time_limit=120.0)
    torch.cuda.synchronize()
    st = server.stats()
    assert st["completed"] == sum(len(s.xs) for s in sessions)
    assert st["max_in_flight"] >= 2
    assert all(status == 0 for (_, _, _, status) in recs)
    for s in sessions:
        m = mids.index(s.matrix_id)
        kind, n, P = mats[m]
        for k, (x, y) in enumerate(zip(s.xs, s.ys)):
            alone = torch.zeros_like(y)
            plans[m].matvec(x, alone, ws=plans[m].new_workspace())
            torch.cuda.synchronize()
            assert torch.equal(alone, y), (s.sid, k)
            if n <= 300:
                want = hankel.matvec_words(kind, host_h[m], host_x[(s.sid, k)], P)
                assert np.array_equal(hmv.to_host(y), want)
    server.close()


def test_pool_too_small_is_refused():
    need_gpu()
    from paper_1402_5287_amd import hmv
    n, P = 500, 3322
    plan = hmv.Plan("hankel", hmv.to_device(si.uniform(2 * n - 1, P, (92,))), n, P)
    server = hmv.Server(pool_bytes=plan.mv_ws_bytes // 2, slots=2)
    with pytest.raises(hmv.HmvError) as ei:
        server.add_plan(plan)
    assert ei.value.code == hmv.ENOMEM
    server.close()


def test_submit_waits_for_the_producer_stream():
    """x is written by a torch kernel queued behind a long-running one on the
    submitting stream, and the request is submitted right after: the server
    must order the request after that write (the result equals the product
    of the new x, not of the stale buffer)."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    n, P = 1000, 3322
    h = si.uniform(2 * n - 1, P, (93, 0))
    plan = hmv.Plan("hankel", hmv.to_device(h), n, P)
    server = hmv.Server(pool_bytes=4 * plan.mv_ws_bytes, slots=2)
    mid = server.add_plan(plan)
    W = hmv.words(P)
    for k in range(3):
        xsrc = hmv.to_device(si.uniform(n, P, (93, 1, k)))
        x = torch.zeros((n, W), dtype=torch.int64, device="cuda")
        y = torch.zeros_like(x)
        torch.cuda.synchronize()
        announce("serving producer order", k)
        torch.cuda._sleep(200_000_000)          # keeps the stream busy for a while
        x.copy_(xsrc)                           # the producer write, queued behind it
        rid = server.submit(mid, k, x, y)
        done, t0 = [], time.time()
        while not done:
            assert time.time() - t0 < 60.0, "request not retired"
            done = server.poll()
        assert done == [(rid, 0)]
        torch.cuda.synchronize()
        alone = torch.zeros_like(y)
        plan.matvec(xsrc, alone, ws=plan.new_workspace())
        torch.cuda.synchronize()
        assert torch.equal(alone, y), k
        assert torch.count_nonzero(y).item() > 0
    server.close()
    plan.close()


def test_size_aware_admission():
    """With at most one large request in flight, a large request held back by
    the cap lets the small ones behind it start; every result still equals
    the product alone."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    big = hmv.Plan("hankel", hmv.to_device(si.uniform(2 * 2000 - 1, 3322, (94, 0))), 2000, 3322)
    small = hmv.Plan("toeplitz", hmv.to_device(si.uniform(2 * 64 - 1, 3322, (94, 1))), 64, 3322)
    server = hmv.Server(pool_bytes=4 * big.mv_ws_bytes + 4 * small.mv_ws_bytes, slots=4)
    mb, ms = server.add_plan(big), server.add_plan(small)
    with pytest.raises(hmv.HmvError):
        server.set_policy(small.mv_ws_bytes * 2, 5)         # more than the slots
    with pytest.raises(hmv.HmvError):
        server.set_policy(-1, 1)
    server.set_policy(small.mv_ws_bytes * 2, 1)
    jobs = [(mb, 2000, 3322, 0), (mb, 2000, 3322, 1), (mb, 2000, 3322, 2),
            (ms, 64, 3322, 3), (ms, 64, 3322, 4), (ms, 64, 3322, 5)]
    xs, ys = [], []
    for mid, n, P, sid in jobs:
        xs.append(hmv.to_device(si.uniform(n, P, (95, sid))))
        ys.append(torch.zeros((n, hmv.words(P)), dtype=torch.int64, device="cuda"))
    announce("serving size-aware admission")
    for (mid, n, P, sid), x, y in zip(jobs, xs, ys):
        server.submit(mid, sid, x, y)
    st = server.stats()
    # one large and the three small requests run; two large ones wait
    assert st["in_flight"] == 4 and st["waiting"] == 2 and st["large_in_flight"] == 1
    done = []
    t0 = time.time()
    while len(done) < len(jobs):
        assert time.time() - t0 < 60
        done += server.poll()
        time.sleep(1e-4)
    assert all(status == 0 for _, status in done)
    st = server.stats()
    assert st["max_large_in_flight"] == 1 and st["completed"] == len(jobs)
    for (mid, n, P, sid), x, y in zip(jobs, xs, ys):
        plan = big if mid == mb else small
        alone = torch.zeros_like(y)
        plan.matvec(x, alone, ws=plan.new_workspace())
        torch.cuda.synchronize()
        assert torch.equal(alone, y), sid
    server.close()
