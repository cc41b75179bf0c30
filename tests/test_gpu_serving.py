"""Serving loop on the GPU: continuous batching by HBM budget with
least-work-first admission among the requests that fit, overlap of requests on the device (their device intervals from HIP
events intersect), and each request's result bit-identical alone and in a
mix of uneven requests."""
import sys
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _wait(srv, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                p = srv.poll(t)
                if p is not None:
                    out[t] = p
        assert time.time() - t0 < timeout, "requests did not finish"
        time.sleep(0.001)
    return out


def _small_stream(n, seed):
    return [r for _, r in W.serving_stream(n, 1.0, seed=seed, paths=(2000, 12000),
                                           steps=(12, 26, 52), assets=(1, 8))]


def test_alone_vs_mix_bitwise():
    import paper_2206_03719_amd as hs
    reqs = _small_stream(10, seed=3)
    _say("alone: %d requests one at a time" % len(reqs))
    srv = hs.Server(8 << 30, max_slots=1)
    alone = []
    for r in reqs:
        t = srv.submit(r)
        alone.append(_wait(srv, [t])[t][0])
    srv.close()
    _say("mix: the same requests interleaved with others on 4 slots")
    others = _small_stream(12, seed=4)
    srv = hs.Server(8 << 30, max_slots=4)
    order = []
    for i in range(max(len(reqs), len(others))):
        if i < len(others):
            order.append(("o", srv.submit(others[i])))
        if i < len(reqs):
            order.append(("r", srv.submit(reqs[i])))
    res = _wait(srv, [t for _, t in order])
    st = srv.stats()
    srv.close()
    mine = [res[t][0] for k, t in order if k == "r"]
    for a, b in zip(alone, mine):
        assert np.array_equal(a["scenario_price"], b["scenario_price"])
        assert np.array_equal(a["scenario_se"], b["scenario_se"])
        assert np.array_equal(a["delta"], b["delta"], equal_nan=True)
    assert st["completed"] == len(reqs) + len(others) and st["failed"] == 0


def test_server_matches_direct_call():
    import paper_2206_03719_amd as hs
    w = W.best_of_call(n_assets=3, n_paths=3000, n_steps=20)
    direct = hs.price_greeks(w["model"], w["corr"], w["option"], 3000, 20, w["bumps"],
                             seed=w["seed"], precision="fp32")
    srv = hs.Server(1 << 30, max_slots=2)
    t = srv.submit(w)
    r, lat = _wait(srv, [t])[t]
    srv.close()
    assert np.array_equal(r["scenario_price"], direct["scenario_price"])
    assert lat > 0


def test_budget_admission_and_overlap():
    import paper_2206_03719_amd as hs
    reqs = _small_stream(16, seed=5)
    need = [hs.workspace_bytes(r["model"], r["option"], r["n_paths"], r["n_steps"], r["bumps"])
            for r in reqs]
    pool = int(max(need) * 2.5)
    _say("pool %.1f MB for requests of up to %.1f MB" % (pool / 1e6, max(need) / 1e6))
    srv = hs.Server(pool, max_slots=8)
    tickets = [srv.submit(r) for r in reqs]
    seen_running = 0
    t0 = time.time()
    done = {}
    while len(done) < len(tickets):
        st = srv.stats()
        seen_running = max(seen_running, st["running"])
        assert st["pool_in_use"] <= pool
        for t in tickets:
            if t not in done:
                p = srv.poll(t)
                if p is not None:
                    done[t] = p
        assert time.time() - t0 < 120
        time.sleep(0.0005)
    st = srv.stats()
    srv.close()
    _say("  device: at most %d requests at once, %.4f s with two or more"
         % (st["device_max_concurrent"], st["device_overlap_s"]))
    assert st["completed"] == len(reqs)
    assert st["pool_peak"] <= pool
    assert seen_running >= 2
    # overlap on the device itself: the requests' device intervals (HIP
    # events on their streams) intersect
    assert st["device_max_concurrent"] >= 2
    assert st["device_overlap_s"] > 0.0


def test_admission_passes_a_waiting_request():
    # A takes most of the pool; B (as large) waits at the head of the queue;
    # C (small) fits beside A and is admitted past B, so it finishes first
    import paper_2206_03719_amd as hs
    big = W.best_of_call(n_assets=6, n_paths=60000, n_steps=126)
    small = W.best_of_call(n_assets=2, n_paths=4000, n_steps=26)
    nb = hs.workspace_bytes(big["model"], big["option"], 60000, 126, big["bumps"])
    ns = hs.workspace_bytes(small["model"], small["option"], 4000, 26, small["bumps"])
    assert ns * 4 < nb
    srv = hs.Server(nb + 2 * ns, max_slots=4)
    ta = srv.submit(big)
    time.sleep(0.05)
    tb = srv.submit(big)
    tc = srv.submit(small)
    order = []
    t0 = time.time()
    pending = {ta, tb, tc}
    while pending:
        for t in list(pending):
            if srv.poll(t) is not None:
                order.append(t)
                pending.discard(t)
        assert time.time() - t0 < 120
        time.sleep(0.0005)
    srv.close()
    _say("  completion order: %s (a=%d b=%d c=%d)" % (order, ta, tb, tc))
    assert order.index(tc) < order.index(tb)


def test_request_over_budget_runs_in_passes():
    import paper_2206_03719_amd as hs
    w = W.best_of_call(n_assets=4, n_paths=6000, n_steps=30)
    full = hs.workspace_bytes(w["model"], w["option"], 6000, 30, w["bumps"])
    mn = hs.workspace_bytes(w["model"], w["option"], 6000, 30, w["bumps"], minimum=True)
    direct = hs.price_greeks(w["model"], w["corr"], w["option"], 6000, 30, w["bumps"],
                             seed=w["seed"], precision="fp32")
    srv = hs.Server((mn + full) // 2, max_slots=2)
    t = srv.submit(w)
    r, _ = _wait(srv, [t])[t]
    srv.close()
    assert np.array_equal(r["scenario_price"], direct["scenario_price"])


def test_cancel_and_errors():
    import paper_2206_03719_amd as hs
    w = W.best_of_call(n_assets=5, n_paths=20000, n_steps=60)
    srv = hs.Server(4 << 30, max_slots=1)
    t1 = srv.submit(w)
    t2 = srv.submit(w)
    srv.cancel(t2)
    with pytest.raises(hs.HSError) as e:
        srv.poll(t2)
    assert e.value.status == hs.ECANCELLED
    _wait(srv, [t1])
    with pytest.raises(hs.HSError):
        srv.poll(t1)  # retired
    # a request whose minimum workspace (about 10 GiB) exceeds the 4 GiB pool
    big = W.best_of_call(n_assets=20, n_paths=1000000, n_steps=504)
    assert hs.workspace_bytes(big["model"], big["option"], 1000000, 504, big["bumps"],
                              minimum=True) > (4 << 30)
    with pytest.raises(hs.HSError) as e:
        srv.submit(big)
    assert e.value.status == hs.ENOMEM
    srv.close()


def test_small_requests_pass_large_ones_within_the_bound():
    # one slot: a queue of large requests with a small one behind them; the
    # small one (least work) is admitted as soon as the slot frees, ahead of
    # the queued large ones, and every request completes (the pass bound
    # keeps the large ones from waiting for ever)
    import paper_2206_03719_amd as hs
    big = W.best_of_call(n_assets=8, n_paths=100000, n_steps=126)  # ~10 ms each
    small = W.best_of_call(n_assets=2, n_paths=2000, n_steps=26)
    srv = hs.Server(24 << 30, max_slots=1)
    tb = [srv.submit(big) for _ in range(3)]
    ts = srv.submit(small)  # queued behind two large ones while the first runs
    order = []
    t0 = time.time()
    pending = set(tb) | {ts}
    while pending:
        for t in list(pending):
            if srv.poll(t) is not None:
                order.append(t)
                pending.discard(t)
        assert time.time() - t0 < 120
        time.sleep(0.0005)
    st = srv.stats()
    srv.close()
    _say("  completion order: %s (small %d)" % (order, ts))
    assert st["completed"] == 4
    assert order.index(ts) <= 1  # only the request already running finishes before it
