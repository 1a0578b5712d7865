"""Serving on the GPU (continuous batching, perc_server_*): every served result equals the
result of inspecting that configuration alone, bitwise (decision, step count and FP32
first-hit probability), and the oracle's decision and step count; requests join while
others are in flight, wait for slots and pool room, and retire as they finish."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def perc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1401_2130_amd as p
    return p


def alone(perc, lats, W, L, p, seed, cfg):
    key = (W, L)
    if key not in lats:
        lats[key] = perc.Lattice(W, L)
    pg, sg, hg, _ = perc.perc_batch([(lats[key], p, seed, cfg)], hit=True, form="span")
    torch.cuda.synchronize()
    return int(pg[0]), int(sg[0]), np.float32(hg.cpu().numpy()[0])


def check_against_alone_and_oracle(perc, reqs, results):
    lats, refs = {}, {}
    for (W, L, p, seed, cfg, tag) in reqs:
        r = results[tag]
        assert r["status"] == 0, r
        a_perc, a_steps, a_hit = alone(perc, lats, W, L, p, seed, cfg)
        assert (r["perc"], r["steps"]) == (a_perc, a_steps), (tag, r, a_perc, a_steps)
        assert np.float32(r["hit"]).view(np.uint32) == a_hit.view(np.uint32), (tag, r["hit"], a_hit)
        if (W, L) not in refs:
            refs[(W, L)] = oracle.Lattice(W, L)
        occ = refs[(W, L)].sample(p, seed, 1, cfg0=cfg)
        pm, sm, _ = refs[(W, L)].inspect_markov(occ)
        assert (r["perc"], r["steps"]) == (int(pm[0]), int(sm[0])), (tag, r, pm[0], sm[0])


def test_served_equals_alone(perc):
    shapes = [(1, 7), (3, 20), (5, 33), (8, 60), (2, 5), (10, 48), (0, 9), (6, 100), (12, 30)]
    rng = np.random.default_rng(11)
    reqs = []
    for i in range(54):
        W, L = shapes[i % len(shapes)]
        p = float([0.15, 0.3, 0.5, 0.8][rng.integers(4)])
        reqs.append((W, L, p, 40 + i % 3, i, 7000 + i))
    stream = torch.cuda.Stream()
    # few slots and short ticks: requests wait, and join while others are in flight
    srv = perc.perc_server(hbm_bytes=64 << 20, max_slots=5, tick_steps=3, max_w=16, stream=stream)
    results, pending = {}, list(reqs)
    for _ in range(10000):
        for _ in range(min(4, len(pending))):
            W, L, p, seed, cfg, tag = pending.pop(0)
            srv.submit(W, L, p, seed, cfg=cfg, tag=tag)
        srv.tick()
        st = srv.stats()
        assert st["in_flight"] <= 5
        for r in srv.poll():
            assert r["tag"] not in results
            results[r["tag"]] = r
        if len(results) == len(reqs):
            break
    assert len(results) == len(reqs)
    assert srv.stats()["pool_used_bytes"] == 0
    check_against_alone_and_oracle(perc, reqs, results)


def test_run_loop_stream(perc):
    """The native loop over a Poisson stream: all requests complete, each as alone."""
    rng = np.random.default_rng(5)
    n = 120
    t = np.cumsum(rng.exponential(1.0 / 20000.0, size=n))
    W = rng.integers(2, 13, size=n)
    L = rng.integers(10, 160, size=n)
    p = rng.uniform(0.12, 0.45, size=n)
    reqs = [(float(t[i] - t[0]), int(W[i]), int(L[i]), float(p[i]), 1000 + i, 0, i) for i in range(n)]
    stream = torch.cuda.Stream()
    srv = perc.perc_server(hbm_bytes=256 << 20, max_slots=32, tick_steps=8, max_w=16, stream=stream)
    res = srv.run(reqs)
    assert sorted(r["tag"] for r in res) == list(range(n))
    lat_ns = np.array([r["t_done_ns"] - r["t_arrive_ns"] for r in res])
    assert np.all(lat_ns > 0)
    assert np.percentile(lat_ns, 50) <= np.percentile(lat_ns, 99)
    results = {r["tag"]: r for r in res}
    check_against_alone_and_oracle(perc, [(w, l, pp, s, c, tag) for (_, w, l, pp, s, c, tag) in reqs], results)


def test_idle_ticks_and_reuse(perc):
    stream = torch.cuda.Stream()
    srv = perc.perc_server(hbm_bytes=16 << 20, max_slots=2, tick_steps=2, max_w=8, stream=stream)
    assert srv.tick() == 0 and srv.poll() == []  # nothing queued or in flight
    reqs = [(4, 16, 0.5, 9, i, i) for i in range(7)]
    for (W, L, p, seed, cfg, tag) in reqs:
        srv.submit(W, L, p, seed, cfg=cfg, tag=tag)
    results = {}
    for _ in range(1000):
        srv.tick()
        for r in srv.poll():
            results[r["tag"]] = r
        if len(results) == len(reqs):
            break
    check_against_alone_and_oracle(perc, reqs, results)


def test_serving_recipe_sample(perc):
    """The first 96 requests of the serving workload (W 8..64, L 64..4096, p 0.12..0.19,
    Philox seed = request id) through the server in the configuration the benchmark
    uses: every request with N <= 1e6 and a fixed sample of larger ones (every 48th)
    against the oracle's breadth-first search (bits and steps)."""
    from paper_1401_2130_amd import workloads
    base = workloads.serving_requests(96)
    reqs = [(t * 0.0, W, L, p, i, 0, i) for (t, W, L, p, i) in base]  # all arrive at once
    stream = torch.cuda.Stream()
    srv = perc.perc_server(hbm_bytes=32 << 30, max_slots=256, tick_steps=16,
                           max_w=workloads.SERVING.w_range[1], stream=stream)
    res = {r["tag"]: r for r in srv.run(reqs)}
    assert sorted(res) == list(range(96))
    checked = 0
    for (_, W, L, p, seed, cfg, tag) in reqs:
        n = perc.Lattice(W, L).n
        if n > 1_000_000 and tag % 48:
            continue
        ref = oracle.Lattice(W, L)
        pb, sb = ref.inspect_bfs(ref.sample(p, seed, 1, cfg0=cfg))
        r = res[tag]
        assert r["status"] == 0
        assert (r["perc"], r["steps"]) == (int(pb[0]), int(sb[0])), (tag, W, L, p, r)
        checked += 1
    assert checked >= 10


def test_cancel_in_flight_and_queued(perc):
    """Requests cancelled while queued or in flight retire with PERC_ECANCELED; the
    planner drops the in-flight ones from the work list, their slots and pool room are
    reused, and every other request still equals its inspection alone and the oracle."""
    stream = torch.cuda.Stream()
    srv = perc.perc_server(hbm_bytes=64 << 20, max_slots=4, tick_steps=4, max_w=8, lookahead=4, stream=stream)
    # long inspections (percolating fibers of ~100 tubes along the axis) so that the
    # cancelled ones are still in flight after the first tick
    reqs = [(6, 300, 0.6, 21, i, i) for i in range(6)] + [(3, 40, 0.35, 22, i, 100 + i) for i in range(4)]
    for (W, L, p, seed, cfg, tag) in reqs:
        srv.submit(W, L, p, seed, cfg=cfg, tag=tag)
    assert srv.tick() == 0
    assert srv.stats()["in_flight"] == 4
    assert srv.cancel(1) == 1 and srv.cancel(2) == 1  # in flight
    assert srv.cancel(5) == 1                          # still queued
    results = {}
    for r in srv.poll():
        results[r["tag"]] = r
    # a request that arrives after the cancellations takes a freed slot
    late = (6, 300, 0.6, 21, 40, 40)
    srv.submit(*late[:4], cfg=late[4], tag=late[5])
    for _ in range(2000):
        srv.tick()
        for r in srv.poll():
            assert r["tag"] not in results
            results[r["tag"]] = r
        if len(results) == len(reqs) + 1:
            break
    assert sorted(results) == sorted([t for *_, t in reqs] + [40])
    for t in (1, 2, 5):
        assert results[t]["status"] == perc.PERC_ECANCELED
    st = srv.stats()
    assert st["cancelled"] == 3 and st["pool_used_bytes"] == 0 and st["in_flight"] == 0
    kept = [q for q in reqs + [late] if q[5] not in (1, 2, 5)]
    check_against_alone_and_oracle(perc, kept, results)
