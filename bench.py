#!/usr/bin/env python3
"""Benchmark of the percolation inspection on one MI355X.

Workload: fibers of hex radius W=32 and L=1024 layers (1,081,686 tubes), tubes metallic
with p in {0.14, 0.1533, 0.17}, 256 configurations at each p from Philox seed 2. One
step is the whole hot path over that batch: occupancy sampling on the device, degree
codes and start state, the forward iteration to the stop of every configuration, the
first-hit probabilities and the Pi counts.

Printed (one JSON line on stdout): configurations inspected per second (value),
site-updates per second (N x steps per configuration, the same count for every form),
the plain per-configuration form on a sample for comparison, the roofline of the step
kernel (HIP events on its stream inside the timed region, 8.375 algorithmic bytes per
tube slot advanced one step) and the CPU oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "configs inspected/s and site-updates/s (batched vs plain) + % HBM roofline; p50/p99"
BYTES_PER_TUBE_STEP = 8.375  # x read + write (4 + 4 B), occupancy bit, reach bit read + write
HBM_PEAK_GBS = 8000.0
STEP_KERNEL = "k_span_step"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    with open(os.path.join(ROOT, "paper_1401_2130_amd", "csrc", "kernels.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_from_profiles(tube_steps_per_launch: float):
    """HBM bytes per step launch from the committed PMC summary, if it was taken on
    the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "k_span_step_W32_L1024_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernels_sha") != kernel_source_sha():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(wl, budget_s: float):
    import numpy as np
    import oracle
    (W, L), seed = wl.shapes[0], wl.seed
    ref = oracle.Lattice(W, L)
    cores = oracle.num_threads()
    done, t_total, upd = 0, 0.0, 0
    per_p = {p: 0 for p in wl.ps}
    while t_total < budget_s:
        for p in wl.ps:
            t0 = time.perf_counter()
            occ = ref.sample(p, seed, cores, cfg0=per_p[p])
            perc, steps, _ = ref.inspect_markov(occ, nthreads=cores)
            t_total += time.perf_counter() - t0
            per_p[p] += cores
            done += cores
            upd += int(np.sum(steps.astype(np.int64))) * ref.n
    return {
        "value": done / t_total, "unit": "configs/s", "cores": cores, "kind": "oracle",
        "site_updates_per_s": upd / t_total,
        "sample": (f"configurations 0..{per_p[wl.ps[0]] - 1} at each p of the same workload "
                   f"({done} configurations, {t_total:.1f} s): host Philox sampling + explicit CSR "
                   f"FP64 Markov iteration, one configuration per OpenMP thread"),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", default="span", choices=["span", "persist", "auto"])
    ap.add_argument("--depth", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--graph-steps", type=int, default=0)
    ap.add_argument("--plain-sample", type=int, default=4, help="configurations per p for the plain form")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy this many MiB device to device (counter calibration runs)")
    ap.add_argument("--copy-bandwidth-mib", type=int, default=1024,
                    help="measure device-to-device copy bandwidth on this many MiB (0: skip)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the inspection of a batch runs on a single device and "
              "no multi-GPU path is built (configurations would be sharded across GPUs with one "
              "integer all-reduce of the Pi counts). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1401_2130_amd as perc
    from paper_1401_2130_amd import workloads

    wl = workloads.LARGE
    (W, L), seed, n = wl.shapes[0], wl.seed, wl.n_cfg
    torch.cuda.set_device(0)
    lat = perc.Lattice(W, L)
    stream = torch.cuda.Stream()
    bufs = [(torch.empty(n, dtype=torch.uint8, device="cuda"), torch.empty(n, dtype=torch.int32, device="cuda"),
             torch.empty(n, dtype=torch.float32, device="cuda")) for _ in wl.ps]
    opts = dict(form=args.form, depth=args.depth, block=args.block, graph_steps=args.graph_steps)

    def step():
        counts = []
        for (b, s, h), p in zip(bufs, wl.ps):
            n_perc, _ = perc.perc_pi_ex(lat, p, n, seed, bits=b, steps=s, hit=h, stream=stream, **opts)
            counts.append(n_perc)
        return counts

    if args.copy_calibration_mib:
        src = torch.ones(args.copy_calibration_mib * 2 ** 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {args.copy_calibration_mib} MiB for counter calibration")
        del src, dst

    with torch.cuda.stream(stream):
        for i in range(args.warmup):
            log(f"warmup {i + 1}/{args.warmup}")
            step()
        # timed region: step launches bracketed by HIP events on their stream
        perc.perc_profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            counts = step()
            log(f"step {i + 1}/{args.steps} done")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        prof = perc.perc_profile_read()
        perc.perc_profile_enable(False)
        # the same steps replayed from HIP graphs, without per-launch events
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            step()
        torch.cuda.synchronize()
        elapsed_graph = time.perf_counter() - t0
        log(f"graph-replayed steps: {elapsed_graph / args.steps * 1e3:.1f} ms/step")

    n_total = n * len(wl.ps)
    steps_all = np.concatenate([s.cpu().numpy().astype(np.int64) for _, s, _ in bufs])
    site_updates = int(steps_all.sum()) * lat.n
    value = n_total * args.steps / elapsed

    # plain form: one configuration at a time, the host checks the flags every step
    k = args.plain_sample
    t_plain, upd_plain = 0.0, 0
    with torch.cuda.stream(stream):
        for p in (wl.ps if k > 0 else ()):
            occ = perc.perc_sample(lat, p, seed, k, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st, _ = perc.perc_inspect_ex(lat, occ, form="plain", stream=stream)
            torch.cuda.synchronize()
            t_plain += time.perf_counter() - t0
            upd_plain += int(st.cpu().numpy().astype(np.int64).sum()) * lat.n
    log(f"plain form: {3 * k} configurations in {t_plain:.2f} s")

    # achievable HBM bandwidth on this device: a plain device-to-device copy, timed with
    # events on the same stream (bytes read + written per second)
    copy_gbs = None
    if args.copy_bandwidth_mib > 0:
        src = torch.ones(args.copy_bandwidth_mib * 2 ** 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        with torch.cuda.stream(stream):
            dst.copy_(src)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(5):
                dst.copy_(src)
            e1.record(stream)
        e1.synchronize()
        copy_gbs = 2 * src.numel() * 4 * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        log(f"device copy: {copy_gbs:.0f} GB/s (read + write)")
        del src, dst

    launches = max(prof["step_launches"], 1)
    step_s = prof["step_ms"] / 1e3
    alg_bytes = prof["tube_steps"] * BYTES_PER_TUBE_STEP
    achieved = alg_bytes / step_s / 1e9 if step_s > 0 else 0.0
    traffic = traffic_from_profiles(prof["tube_steps"] / launches)
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "configs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: occupancy drawn on the device from Philox4x32-10, seed 2",
        "config": {"workload": "W=32 L=1024 fiber (1,081,686 tubes), p in {0.14, 0.1533, 0.17} x 256 "
                               "configurations, Philox seed 2",
                   "form": args.form, "depth": args.depth, "block": args.block},
        "site_updates_per_s": site_updates / (elapsed / args.steps),
        "graph_replay": {"configs_per_s": n_total * args.steps / elapsed_graph,
                         "ms_per_step": elapsed_graph / args.steps * 1e3,
                         "note": "same steps from captured HIP graphs, no per-launch events"},
        "pi": {str(p): c / n for p, c in zip(wl.ps, counts)},
        "plain": ({"configs_per_s": 3 * k / t_plain, "site_updates_per_s": upd_plain / t_plain,
                   "sample": f"configurations 0..{k - 1} at each p, one at a time"} if k > 0 else None),
        "batched_over_plain": (value / (3 * k / t_plain)) if k > 0 else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "copy_gbs": copy_gbs, "frac_of_copy": (achieved / copy_gbs) if copy_gbs else None,
                     "kernel": STEP_KERNEL, "launches": prof["step_launches"],
                     "avg_launch_us": prof["step_ms"] / launches * 1e3,
                     "tube_steps_per_launch": prof["tube_steps"] / launches,
                     "bytes_per_tube_step": BYTES_PER_TUBE_STEP},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
