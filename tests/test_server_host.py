"""Scheduler logic of the serving loop, on the CPU: the server's host-only mode runs the
same admission, slot and pool bookkeeping with a fake executor (an admitted request
completes at the next tick with zero outputs), so FIFO order, the HBM-footprint
admission and slot reuse are checked without a GPU."""
import numpy as np
import pytest

import paper_1401_2130_amd as perc


def footprint(W, L):
    """Pool bytes of one request: two FP32 state buffers and the code bytes over the
    quad-packed state words (rounded to 64), plus the occupancy words (rounded to 64)."""
    lat = perc.Lattice(W, L)
    C = lat.columns
    cp = max(32, (C + 31) // 32 * 32)
    U = (L + 2) // 3
    sw = ((U + 3) // 4 * 4 * cp + 63) // 64 * 64
    bw = (lat.words + 15) // 16 * 16
    return 9 * sw, 4 * bw


def test_fifo_and_footprint_admission():
    s_bytes, b_bytes = footprint(4, 16)
    # a pool whose state part holds exactly two such requests (the occupancy part, an
    # eighth of the state words, holds more)
    unit = 9 * 16 + 8
    hbm = (2 * s_bytes // (9 * 16) + 1) * unit
    srv = perc.perc_server(hbm_bytes=hbm, max_slots=8, host_only=True)
    for i in range(6):
        srv.submit(4, 16, 0.2, seed=1, cfg=i, tag=100 + i)
    st = srv.stats()
    assert st["queued"] == 6 and st["in_flight"] == 0
    done = []
    in_flight_max = 0
    for _ in range(20):
        n = srv.tick()
        st = srv.stats()
        in_flight_max = max(in_flight_max, st["in_flight"])
        assert st["pool_used_bytes"] <= st["pool_bytes"]
        assert st["in_flight"] * s_bytes <= hbm
        got = srv.poll()
        assert len(got) == n
        done += got
        if len(done) == 6:
            break
    assert [r["tag"] for r in done] == [100 + i for i in range(6)]  # FIFO
    assert in_flight_max == 2  # the pool, not the 8 slots, bounds the concurrency
    assert all(r["status"] == 0 and r["t_done_ns"] >= r["t_admit_ns"] >= r["t_arrive_ns"] for r in done)
    assert srv.stats()["pool_used_bytes"] == 0


def test_slots_bound_concurrency_and_are_reused():
    srv = perc.perc_server(hbm_bytes=1 << 30, max_slots=3, host_only=True)
    for i in range(10):
        srv.submit(2 + i % 3, 10 + i, 0.3, seed=7, cfg=i, tag=i)
    seen = []
    while len(seen) < 10:
        srv.tick()
        assert srv.stats()["in_flight"] <= 3
        seen += srv.poll()
    assert sorted(r["tag"] for r in seen) == list(range(10))
    assert srv.stats()["completed"] == 10


def test_head_of_line_waits_for_room():
    """A big request at the head of the queue is not overtaken by smaller ones."""
    big, _ = footprint(16, 300)
    small, _ = footprint(2, 10)
    unit = 9 * 16 + 8
    hbm = (big // (9 * 16) + 2) * unit
    srv = perc.perc_server(hbm_bytes=hbm, max_slots=16, host_only=True)
    srv.submit(2, 10, 0.3, seed=1, tag=0)
    srv.submit(16, 300, 0.3, seed=1, tag=1)
    srv.submit(2, 10, 0.3, seed=1, tag=2)
    order = []
    for _ in range(10):
        srv.tick()
        order += [r["tag"] for r in srv.poll()]
    assert order == [0, 1, 2]


def test_invalid_requests():
    srv = perc.perc_server(hbm_bytes=1 << 22, max_slots=4, max_w=16, host_only=True)
    for args in ((17, 20, 0.3), (4, 0, 0.3), (4, 20, 1.5), (4, 20, float("nan")), (-1, 20, 0.3)):
        with pytest.raises(perc.PercError) as e:
            srv.submit(*args, seed=1)
        assert e.value.code == perc.PERC_EINVAL
    with pytest.raises(perc.PercError) as e:  # resident state larger than the whole pool
        srv.submit(16, 4000, 0.3, seed=1)
    assert e.value.code == perc.PERC_EBUSY
    assert srv.stats()["rejected"] == 1 and srv.stats()["queued"] == 0
    with pytest.raises(perc.PercError):
        perc.perc_server(max_slots=4, host_only=True)  # host-only needs an explicit pool size
    with pytest.raises(perc.PercError):
        perc.perc_server(hbm_bytes=1 << 22, lookahead=-1, host_only=True)


def test_bounded_queue_sheds_load():
    srv = perc.perc_server(hbm_bytes=1 << 26, max_slots=2, max_queue=3, host_only=True)
    for i in range(3):
        srv.submit(3, 12, 0.25, seed=1, cfg=i, tag=i)
    with pytest.raises(perc.PercError) as e:
        srv.submit(3, 12, 0.25, seed=1, cfg=3, tag=3)
    assert e.value.code == perc.PERC_EBUSY
    st = srv.stats()
    assert st["queued"] == 3 and st["rejected"] == 1
    srv.tick()  # two admitted: room in the queue again
    srv.submit(3, 12, 0.25, seed=1, cfg=3, tag=3)
    got = []
    for _ in range(6):
        srv.tick()
        got += srv.poll()
    assert sorted(r["tag"] for r in got) == [0, 1, 2, 3]
    assert all(r["status"] == perc.PERC_OK for r in got)


def test_run_loop_reports_shed_requests():
    # all requests arrive at once; a queue of 4 and 2 slots refuse the rest
    reqs = [(0.0, 3, 12, 0.25, 5, i, i) for i in range(20)]
    srv = perc.perc_server(hbm_bytes=1 << 26, max_slots=2, max_queue=4, host_only=True)
    res = srv.run(reqs)
    assert sorted(r["tag"] for r in res) == list(range(20))
    busy = [r for r in res if r["status"] == perc.PERC_EBUSY]
    ok = [r for r in res if r["status"] == perc.PERC_OK]
    assert len(busy) + len(ok) == 20 and len(ok) >= 4 and len(busy) >= 1
    assert srv.stats()["rejected"] == len(busy)
    assert all(r["t_done_ns"] >= r["t_arrive_ns"] for r in res)


def test_cancel_queued_and_in_flight():
    srv = perc.perc_server(hbm_bytes=1 << 26, max_slots=2, host_only=True)
    for i in range(5):
        srv.submit(3, 12, 0.25, seed=1, cfg=i, tag=10 + i)
    assert srv.cancel(14) == 1  # still queued: retired at once
    first = srv.poll()
    assert [(r["tag"], r["status"]) for r in first] == [(14, perc.PERC_ECANCELED)]
    assert srv.stats()["queued"] == 4
    srv.tick()  # 10 and 11 admitted
    assert srv.stats()["in_flight"] == 2
    assert srv.cancel(11) == 1  # in flight: stops at the next tick
    assert srv.cancel(11) == 0  # already cancelled
    assert srv.cancel(999) == 0
    got = []
    for _ in range(6):
        srv.tick()
        got += srv.poll()
    status = {r["tag"]: r["status"] for r in got}
    assert status == {10: perc.PERC_OK, 11: perc.PERC_ECANCELED, 12: perc.PERC_OK, 13: perc.PERC_OK}
    st = srv.stats()
    assert st["cancelled"] == 2 and st["completed"] == 3 and st["pool_used_bytes"] == 0
    assert all(r["perc"] == 0 and r["steps"] == 0 for r in got if r["status"] == perc.PERC_ECANCELED)


def test_lookahead_admits_past_a_waiting_head():
    """With lookahead 1 a small request behind a big one that does not fit yet is
    admitted past it; with 0 (strict FIFO) it waits."""
    big, _ = footprint(16, 300)
    small, _ = footprint(2, 10)
    unit = 9 * 16 + 8
    hbm = ((big + small) // (9 * 16) + 3) * unit
    for look, expect in ((0, [0, 1, 2]), (1, [0, 2, 1])):
        srv = perc.perc_server(hbm_bytes=hbm, max_slots=16, lookahead=look, host_only=True)
        srv.submit(16, 300, 0.3, seed=1, tag=0)
        srv.submit(16, 300, 0.3, seed=1, tag=1)  # does not fit beside tag 0
        srv.submit(2, 10, 0.3, seed=1, tag=2)    # fits beside tag 0
        order = []
        for _ in range(10):
            srv.tick()
            order += [r["tag"] for r in srv.poll()]
        assert order == expect, look


def test_run_loop_arrivals():
    rng = np.random.default_rng(3)
    t = np.cumsum(rng.exponential(1e-4, size=40))
    reqs = [(float(t[i]), 3, 12, 0.25, 5, i, 1000 + i) for i in range(40)]
    srv = perc.perc_server(hbm_bytes=1 << 26, max_slots=4, host_only=True)
    res = srv.run(reqs)
    assert sorted(r["tag"] for r in res) == [1000 + i for i in range(40)]
    arrive = {r["tag"]: r["t_arrive_ns"] for r in res}
    # arrival stamps follow the schedule (relative to the first)
    t0 = arrive[1000]
    for i in range(40):
        assert abs((arrive[1000 + i] - t0) - (t[i] - t[0]) * 1e9) < 1e3
    assert all(r["t_done_ns"] >= r["t_arrive_ns"] for r in res)
