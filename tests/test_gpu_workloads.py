"""The benchmark workloads in full on the GPU, against the oracle's stored results.

``tests/golden/oracle_workloads.json`` is written by ``tests/golden/make_golden.py``,
which calls only the CPU oracle: for each (shape, p) group the number of percolating
configurations (the Pi(p) count of Sec. III) and SHA-256 digests of every
configuration's bit and step count. Here the same Philox configurations are inspected
through the C ABI in the execution forms the benchmark times, and every group must
match: count, step sum and maximum, and both digests (so every bit and every step
count is the oracle's). Serving: every stored request (all of the first 2,000 with at
most 1e6 tubes, and every 100th larger one) served in one run must match the oracle's
bit and step count.
"""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_workloads.json")


@pytest.fixture(scope="module")
def perc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1401_2130_amd as p
    return p


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)["workloads"]


def sha(a: np.ndarray, dtype) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.dtype(dtype).newbyteorder("<")).tobytes()).hexdigest()


def check_group(g, bits, steps):
    bits = bits.astype(np.uint8)
    steps = steps.astype(np.int64)
    where = (g["W"], g["L"], g["p"])
    assert int(bits.sum()) == g["n_perc"], where
    assert int(steps.sum()) == g["steps_sum"], where
    assert int(steps.max()) == g["steps_max"], where
    assert sha(bits, np.uint8) == g["bits_sha256"], where
    assert sha(steps, np.int32) == g["steps_sha256"], where


@pytest.mark.parametrize("form", ["plain", "span"])
def test_small_workload(perc, golden, form):
    """W=4 L=16 p=0.1533 x 1000 (seed 1): the plain form (one configuration at a time,
    as benched) and the span form."""
    (g,) = golden["small"]["groups"]
    lat = perc.Lattice(g["W"], g["L"])
    occ = perc.perc_sample(lat, g["p"], g["seed"], g["n"])
    pg, sg, _ = perc.perc_inspect_ex(lat, occ, form=form)
    torch.cuda.synchronize()
    check_group(g, pg.cpu().numpy(), sg.cpu().numpy())


def test_large_workload(perc, golden):
    """W=32 L=1024 at p in {0.14, 0.1533, 0.17} x 256 (seed 2), the headline workload,
    through perc_pi_ex in the span form, one call per p: all 768 configurations."""
    groups = golden["large"]["groups"]
    assert len(groups) == 3
    lat = perc.Lattice(groups[0]["W"], groups[0]["L"])
    for g in groups:
        b = torch.empty(g["n"], dtype=torch.uint8, device="cuda")
        s = torch.empty(g["n"], dtype=torch.int32, device="cuda")
        n_perc, _ = perc.perc_pi_ex(lat, g["p"], g["n"], g["seed"], bits=b, steps=s, form="span")
        assert n_perc == g["n_perc"]
        check_group(g, b.cpu().numpy(), s.cpu().numpy())


def test_large_workload_one_batch(perc, golden):
    """The same 768 configurations as one perc_batch call with one Pi group per p, the
    call the benchmark times."""
    groups = golden["large"]["groups"]
    lat = perc.Lattice(groups[0]["W"], groups[0]["L"])
    n = groups[0]["n"]
    jobs = [(lat, g["p"], g["seed"], c, k) for k, g in enumerate(groups) for c in range(n)]
    pg, sg, _, counts = perc.perc_batch(jobs, n_groups=len(groups), hit=True, form="span")
    torch.cuda.synchronize()
    bits, steps = pg.cpu().numpy(), sg.cpu().numpy()
    assert counts == [g["n_perc"] for g in groups]
    for k, g in enumerate(groups):
        check_group(g, bits[k * n:(k + 1) * n], steps[k * n:(k + 1) * n])


@pytest.mark.parametrize("form", ["persist2", "persist", "span"])
def test_batched_workload(perc, golden, form):
    """W=16 L=256, 21 p x 4096 (seed 3) in one perc_batch call with one group per p:
    all 86,016 configurations, and the Pi(p) counts."""
    groups = golden["batched"]["groups"]
    assert len(groups) == 21
    lat = perc.Lattice(groups[0]["W"], groups[0]["L"])
    n = groups[0]["n"]
    jobs = [(lat, g["p"], g["seed"], c, k) for k, g in enumerate(groups) for c in range(n)]
    pg, sg, _, counts = perc.perc_batch(jobs, n_groups=len(groups), form=form)
    torch.cuda.synchronize()
    bits, steps = pg.cpu().numpy(), sg.cpu().numpy()
    assert counts == [g["n_perc"] for g in groups]
    for k, g in enumerate(groups):
        check_group(g, bits[k * n:(k + 1) * n], steps[k * n:(k + 1) * n])


def test_uneven_workload(perc, golden):
    """35 shapes (W in {8..32} x L/W in {1..64}) x p in {0.1533, 0.16} x 1024 (seed 4)
    mixed in one batch, automatic form: all 71,680 configurations."""
    groups = golden["uneven"]["groups"]
    assert len(groups) == 70
    lats = {}
    jobs = []
    for k, g in enumerate(groups):
        key = (g["W"], g["L"])
        if key not in lats:
            lats[key] = perc.Lattice(*key)
        jobs += [(lats[key], g["p"], g["seed"], c, k) for c in range(g["n"])]
    pg, sg, _, counts = perc.perc_batch(jobs, n_groups=len(groups))
    torch.cuda.synchronize()
    bits, steps = pg.cpu().numpy(), sg.cpu().numpy()
    assert counts == [g["n_perc"] for g in groups]
    off = 0
    for g in groups:
        check_group(g, bits[off:off + g["n"]], steps[off:off + g["n"]])
        off += g["n"]


def test_serving_workload(perc, golden):
    """The first 2,000 requests of the serving recipe through one server run (all
    arriving at once, as many in flight as the pool holds): every stored request's bit
    and step count equal the oracle's."""
    from paper_1401_2130_amd import workloads
    sv = golden["serving"]
    base = workloads.serving_requests(sv["n_requests"])
    reqs = [(0.0, W, L, p, i, 0, i) for (_, W, L, p, i) in base]
    stream = torch.cuda.Stream()
    srv = perc.perc_server(hbm_bytes=96 << 30, max_slots=2048, tick_steps=16,
                           max_w=workloads.SERVING.w_range[1], stream=stream)
    res = {r["tag"]: r for r in srv.run(reqs)}
    assert sorted(res) == list(range(sv["n_requests"]))
    assert len(sv["rows"]) >= 500
    for tag, W, L, p, pb, sb in sv["rows"]:
        r = res[tag]
        assert (r["W"], r["L"], r["p"]) == (W, L, p)
        assert r["status"] == 0
        assert (r["perc"], r["steps"]) == (pb, sb), (tag, W, L, p, r)
