"""The stored oracle results of the benchmark workloads (tests/golden/oracle_workloads.json,
written by tests/golden/make_golden.py from the CPU oracle alone) are what the oracle
computes now: a few groups and serving requests are recomputed on the CPU, with the
Markov iteration where the stored group used the breadth-first search (the two agree
on bits and step counts)."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_1401_2130_amd import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_workloads.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)["workloads"]


def sha(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.dtype(dtype).newbyteorder("<")).tobytes()).hexdigest()


def recompute(g, method):
    ref = oracle.Lattice(g["W"], g["L"])
    occ = ref.sample(g["p"], g["seed"], g["n"], cfg0=g["cfg0"])
    if method == "markov":
        p, s, _ = ref.inspect_markov(occ)
    else:
        p, s = ref.inspect_bfs(occ)
    return p, s


def test_recipes_match(golden):
    assert [g["p"] for g in golden["batched"]["groups"]] == list(workloads.BATCH.ps)
    assert [(g["W"], g["L"]) for g in golden["uneven"]["groups"][::2]] == list(workloads.UNEVEN.shapes)
    assert [g["p"] for g in golden["large"]["groups"]] == list(workloads.LARGE.ps)
    assert golden["small"]["groups"][0]["n"] == workloads.SMALL.n_cfg


def test_small_group_is_the_oracles(golden):
    (g,) = golden["small"]["groups"]
    p, s = recompute(g, "markov")
    assert int(p.sum()) == g["n_perc"]
    assert sha(p, np.uint8) == g["bits_sha256"] and sha(s, np.int32) == g["steps_sha256"]


@pytest.mark.parametrize("k", [15, 17])
def test_batched_groups_are_the_oracles(golden, k):
    """p = 0.175 and 0.185 (inside the transition window) by the Markov iteration."""
    g = golden["batched"]["groups"][k]
    assert g["p"] in (0.175, 0.185)
    g = dict(g, n=128)  # the first 128 configurations by both oracle methods
    p, s = recompute(g, "markov")
    pb, sb = recompute(g, "bfs")
    assert np.array_equal(p, pb) and np.array_equal(s, sb)
    full = golden["batched"]["groups"][k]
    pf, sf = recompute(dict(full), "bfs")
    assert sha(pf, np.uint8) == full["bits_sha256"] and sha(sf, np.int32) == full["steps_sha256"]
    assert np.array_equal(pf[:128], p) and np.array_equal(sf[:128], s)


def test_uneven_smallest_shapes_are_the_oracles(golden):
    for g in golden["uneven"]["groups"][:4]:
        p, s = recompute(g, "bfs")
        assert int(p.sum()) == g["n_perc"]
        assert sha(p, np.uint8) == g["bits_sha256"] and sha(s, np.int32) == g["steps_sha256"]


def test_serving_rows_are_the_oracles(golden):
    sv = golden["serving"]
    rows = [r for r in sv["rows"] if (3 * r[1] * (r[1] + 1) + 1) * ((r[2] + 2) // 3) < 200_000][:25]
    assert len(rows) == 25
    base = {i: (W, L, p) for (_, W, L, p, i) in workloads.serving_requests(sv["n_requests"])}
    for tag, W, L, p, pb, sb in rows:
        assert base[tag] == (W, L, p)
        ref = oracle.Lattice(W, L)
        pm, sm, _ = ref.inspect_markov(ref.sample(p, tag, 1, cfg0=0))
        assert (int(pm[0]), int(sm[0])) == (pb, sb), tag
