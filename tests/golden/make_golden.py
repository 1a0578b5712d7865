#!/usr/bin/env python3
"""Write ``tests/golden/oracle_workloads.json``: the oracle's results on the benchmark
workloads, for the GPU parity tests and the benchmark's parity check.

Calls only the CPU oracle (``oracle/``) and the workload recipes
(``paper_1401_2130_amd/workloads.py``, which hold no arithmetic of the method). For
every (shape, p) group of configurations it records the number that percolate (the
Pi(p) count of Sec. III), the sum and maximum of the step counts, and SHA-256 digests
of the per-configuration bits (uint8) and step counts (little-endian int32) in
configuration order. The small and large plain workloads are decided by the oracle's
Markov iteration (Sec. II.B) and checked against its breadth-first search here; the
batched and uneven sweeps and the serving requests by the breadth-first search, which
the oracle's own tests pin equal to the Markov iteration (bits and step counts).

Usage: ``python tests/golden/make_golden.py [--only small,large,...]`` (about ten
minutes on 8 cores; the Markov iteration of the large workload dominates).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1401_2130_amd import workloads  # noqa: E402

OUT = os.path.join(HERE, "oracle_workloads.json")
# serving requests checked: every one of the first SERVING_N with at most SERVING_NMAX
# tubes, and every SERVING_EVERY-th of the larger ones
SERVING_N, SERVING_NMAX, SERVING_EVERY = 2000, 1_000_000, 100


def digest(a: np.ndarray, dtype) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.dtype(dtype).newbyteorder("<")).tobytes()).hexdigest()


def group_record(W, L, p, seed, cfg0, n, perc, steps, method):
    steps = steps.astype(np.int64)
    return {"W": W, "L": L, "p": p, "seed": seed, "cfg0": cfg0, "n": n, "method": method,
            "n_perc": int(perc.sum()), "steps_sum": int(steps.sum()), "steps_max": int(steps.max()) if n else 0,
            "bits_sha256": digest(perc, np.uint8), "steps_sha256": digest(steps, np.int32)}


def run_groups(wl, method, check_bfs=False, chunk=4096):
    out = []
    for (W, L) in wl.shapes:
        ref = oracle.Lattice(W, L)
        for p in wl.ps:
            t0 = time.time()
            perc_all, steps_all = [], []
            for c0 in range(0, wl.n_cfg, chunk):
                n = min(chunk, wl.n_cfg - c0)
                occ = ref.sample(p, wl.seed, n, cfg0=c0)
                pb, sb = ref.inspect_bfs(occ)
                if method == "markov":
                    pm, sm, _ = ref.inspect_markov(occ)
                    if check_bfs:
                        assert np.array_equal(pm, pb) and np.array_equal(sm, sb), (W, L, p, c0)
                    pb, sb = pm, sm
                perc_all.append(pb)
                steps_all.append(sb)
            rec = group_record(W, L, float(p), wl.seed, 0, wl.n_cfg, np.concatenate(perc_all),
                               np.concatenate(steps_all), method)
            out.append(rec)
            print(f"  W={W} L={L} p={p}: {rec['n_perc']}/{wl.n_cfg} percolate ({time.time() - t0:.1f} s)",
                  flush=True)
    return out


def run_serving():
    reqs = workloads.serving_requests(SERVING_N)
    rows = []
    t0 = time.time()
    for (_, W, L, p, tag) in reqs:
        # at least C (U - 1) tubes (C columns, U unit cells): skip clearly larger fibers
        # without building them
        C = 3 * W * (W + 1) + 1
        if C * ((L + 2) // 3 - 1) > SERVING_NMAX and tag % SERVING_EVERY:
            continue
        ref = oracle.Lattice(W, L)
        if ref.n > SERVING_NMAX and tag % SERVING_EVERY:
            continue
        pb, sb = ref.inspect_bfs(ref.sample(p, tag, 1, cfg0=0))
        rows.append([tag, W, L, p, int(pb[0]), int(sb[0])])
    print(f"  serving: {len(rows)} requests ({time.time() - t0:.1f} s)", flush=True)
    return {"n_requests": SERVING_N, "rule": f"N <= {SERVING_NMAX}, or request id % {SERVING_EVERY} == 0",
            "seed": "request id", "cfg": 0, "method": "bfs",
            "columns": ["tag", "W", "L", "p", "perc", "steps"], "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="small,large,batched,uneven,serving")
    args = ap.parse_args()
    todo = args.only.split(",")
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    data["generator"] = "tests/golden/make_golden.py (oracle/ only)"
    data["digest"] = "SHA-256 of the bits as uint8 and of the step counts as little-endian int32, configuration order"
    wls = data.setdefault("workloads", {})
    spec = {"small": (workloads.SMALL, "markov"), "large": (workloads.LARGE, "markov"),
            "batched": (workloads.BATCH, "bfs"), "uneven": (workloads.UNEVEN, "bfs")}
    for name in todo:
        print(f"{name} ...", flush=True)
        if name == "serving":
            wls[name] = run_serving()
        else:
            wl, method = spec[name]
            wls[name] = {"name": wl.name, "seed": wl.seed, "groups": run_groups(wl, method, check_bfs=True)}
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
