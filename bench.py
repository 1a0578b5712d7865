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
    # the same oracle on one thread: the next configuration at each p
    t1, upd1 = 0.0, 0
    for p in wl.ps:
        t0 = time.perf_counter()
        occ = ref.sample(p, seed, 1, cfg0=per_p[p])
        _, steps, _ = ref.inspect_markov(occ, nthreads=1)
        t1 += time.perf_counter() - t0
        upd1 += int(np.sum(steps.astype(np.int64))) * ref.n
    return {
        "value": done / t_total, "unit": "configs/s", "cores": cores, "kind": "oracle",
        "site_updates_per_s": upd / t_total,
        "sample": (f"configurations 0..{per_p[wl.ps[0]] - 1} at each p of the same workload "
                   f"({done} configurations, {t_total:.1f} s): host Philox sampling + explicit CSR "
                   f"FP64 Markov iteration, one configuration per OpenMP thread"),
        "single_thread": {"value": len(wl.ps) / t1, "unit": "configs/s", "site_updates_per_s": upd1 / t1,
                          "sample": f"configuration {per_p[wl.ps[0]]} at each p ({len(wl.ps)} configurations, {t1:.1f} s)"},
        "host": {"cpu": cpu_model(), "logical_cpus": os.cpu_count()},
    }


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def batched_leg(perc, workloads, stream):
    """Batched Monte Carlo: every configuration of the Pi(p) sweep in one batch (one
    output group per p), settings picked by the autotuner on a sample, then the Eq. 5 fit."""
    import numpy as np
    from paper_1401_2130_amd import fss
    wl = workloads.BATCH
    (W, L), seed, n = wl.shapes[0], wl.seed, wl.n_cfg
    lat = perc.Lattice(W, L)
    p_mid = wl.ps[len(wl.ps) // 2]
    sample = [(lat, p_mid, seed, c) for c in range(512)]
    tuned = perc.perc_autotune(sample, n_target=n * len(wl.ps), stream=stream)
    jobs = [(lat, p, seed, c, g) for g, p in enumerate(wl.ps) for c in range(n)]
    opts = {k: tuned[k] for k in ("form", "depth", "block", "graph_steps")}
    perc.perc_batch(jobs[:1024], n_groups=len(wl.ps), stream=stream, **opts)  # warm-up
    torch_sync()
    t0 = time.perf_counter()
    _, st, _, counts = perc.perc_batch(jobs, n_groups=len(wl.ps), stream=stream, **opts)
    torch_sync()
    wall = time.perf_counter() - t0
    # the same batch once more with the step profiler: kernel time and tube slots
    perc.perc_profile_enable(True)
    perc.perc_batch(jobs, n_groups=len(wl.ps), stream=stream, **opts)
    torch_sync()
    prof = perc.perc_profile_read()
    perc.perc_profile_enable(False)
    steps = st.cpu().numpy().astype(np.int64)
    pis = np.array(counts) / n
    out = {"workload": f"W={W} L={L} ({lat.n} tubes), p = 0.100..0.200 step 0.005 x {n}, Philox seed {seed}",
           "configs": len(jobs), "configs_per_s": len(jobs) / wall, "wall_s": wall,
           "site_updates_per_s": float(steps.sum()) * lat.n / wall, "autotune": tuned,
           "kernel_roofline": {"achieved_gbs": prof["tube_steps"] * BYTES_PER_TUBE_STEP / (prof["step_ms"] / 1e3) / 1e9
                               if prof["step_ms"] > 0 else None,
                               "frac": prof["tube_steps"] * BYTES_PER_TUBE_STEP / (prof["step_ms"] / 1e3) / 1e9
                               / HBM_PEAK_GBS if prof["step_ms"] > 0 else None,
                               "launches": prof["step_launches"], "kernel_ms": prof["step_ms"],
                               "tube_steps": prof["tube_steps"],
                               "note": "tube slots of the steps x 8.375 B over the step-kernel time "
                                       "(the persistent form's one launch also samples and initialises)"},
           "pi": {f"{p:.3f}": float(v) for p, v in zip(wl.ps, pis)}}
    try:
        pc, T, cov = fss.fit_fermi_dirac(wl.ps, pis, n)
        out["eq5_fit"] = {"pc": pc, "T": T, "pc_err": float(np.sqrt(cov[0, 0]))}
    except Exception as e:
        out["eq5_fit"] = {"error": str(e)}
    return out


def uneven_leg(perc, workloads, stream):
    """Uneven batch: 35 shapes x 2 p x 1024 configurations mixed in one batch; effective
    thresholds per shape and the Eq. 7 / Eq. 8 fits."""
    from paper_1401_2130_amd import fss
    wl = workloads.UNEVEN
    lats = [perc.Lattice(*sh) for sh in wl.shapes]
    tuned = perc.perc_autotune([(lat, wl.ps[0], wl.seed, c) for lat in lats for c in range(8)], stream=stream)
    opts = {k: tuned[k] for k in ("form", "depth", "block", "graph_steps")}
    torch_sync()
    t0 = time.perf_counter()
    counts = fss.pi_table(wl.shapes, wl.ps, wl.n_cfg, wl.seed, stream=stream, **opts)
    torch_sync()
    wall = time.perf_counter() - t0
    n_jobs = len(wl.shapes) * len(wl.ps) * wl.n_cfg
    ana = fss.uneven_analysis(counts, wl.n_cfg)
    return {"workload": "W in {8,12,16,24,32} x L/W in {1,2,4,8,16,32,64}, p in {0.1533, 0.16} x 1024, Philox seed 4",
            "configs": n_jobs, "configs_per_s": n_jobs / wall, "wall_s": wall, "autotune": tuned,
            "pc_inf": ana.get("pc_inf"), "eq8": ana.get("eq8"),
            "shapes_with_pc": sum(1 for r in ana["shapes"] if r["pc"] is not None)}


def hist_summary(h) -> dict:
    """Count, mean, quantiles and range of m* from its histogram (bin = m*)."""
    import numpy as np
    h = np.asarray(h, dtype=np.int64)
    tot = int(h.sum())
    if tot == 0:
        return {"percolating": 0}
    m = np.arange(h.size)
    cdf = np.cumsum(h)
    q = lambda f: int(np.searchsorted(cdf, f * tot))
    nz = np.nonzero(h)[0]
    return {"percolating": tot, "mean": float((m * h).sum() / tot), "p5": q(0.05), "p50": q(0.5), "p95": q(0.95),
            "min": int(nz[0]), "max": int(nz[-1])}


def first_passage_leg(perc, workloads, stream, M: int, n_cfg: int = 64):
    """Backward all-sources form of Eq. 3 on n_cfg configurations of the headline fiber in
    one call: M moves timed with HIP events on the launching stream (set-up, backward
    init, M - 1 steps over all configurations and the export inside the timed region)."""
    import torch
    wl = workloads.LARGE
    (W, L) = wl.shapes[0]
    lat = perc.Lattice(W, L)
    p = wl.ps[-1]
    occ = perc.perc_sample(lat, p, wl.seed, n_cfg, stream=stream)
    f = torch.empty((n_cfg, lat.n), dtype=torch.float32, device="cuda")
    perc.perc_first_passage_batch(lat, occ, 8, f=f, stream=stream)  # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    perc.perc_first_passage_batch(lat, occ, M, f=f, stream=stream)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    cols = perc.perc_lattice_columns(lat)
    cells = (L + 2) // 3
    slot_moves = float(M) * cols * cells * n_cfg
    return {"workload": f"W={W} L={L} ({lat.n} tubes), p = {p}, Philox seed {wl.seed}, configurations 0..{n_cfg - 1}",
            "M": M, "configs": n_cfg, "ms": ms, "ms_per_move": ms / M,
            "site_updates_per_s": float(M) * lat.n * n_cfg / (ms / 1e3),
            "achieved_gbs": slot_moves * BYTES_PER_TUBE_STEP / (ms / 1e3) / 1e9,
            "kernel": "k_chunk_step (every cell of every configuration per move)",
            "max_f": float(f.max().item()), "nonzero": int((f > 0).sum().item())}


def ablation_leg(perc, workloads, stream):
    """Regular FCC (no end contacts) against the modified lattice on the same Philox
    configurations: Eq. 5 threshold per near-cubic shape, Eq. 7 intercept at the one
    aspect ratio (literature value for regular FCC: 0.199)."""
    from paper_1401_2130_amd import fss
    wl = workloads.ABLATION
    out = {"workload": f"shapes {list(wl.shapes)} (L = 1.5 W layers), p = 0.120..0.240 step 0.005 x {wl.n_cfg}, "
                       f"Philox seed {wl.seed}, both lattice variants", "variants": {}}
    n_cfg_total, wall = 0, 0.0
    for ends, name in ((False, "regular_fcc"), (True, "modified")):
        torch_sync()
        t0 = time.perf_counter()
        counts = fss.pi_table(wl.shapes, wl.ps, wl.n_cfg, wl.seed, stream=stream, ends=ends)
        torch_sync()
        wall += time.perf_counter() - t0
        n_cfg_total += len(wl.shapes) * len(wl.ps) * wl.n_cfg
        per = []
        for (W, L) in wl.shapes:
            pis = [counts[(W, L, float(p))] / wl.n_cfg for p in wl.ps]
            try:
                pc, T, cov = fss.fit_fermi_dirac(wl.ps, pis, wl.n_cfg)
                per.append({"W": W, "L": L, "pc": pc, "T": T, "pc_err": float(cov[0, 0] ** 0.5)})
            except Exception as e:  # a fit that does not converge is reported, not hidden
                per.append({"W": W, "L": L, "error": str(e)})
        ok = [r for r in per if "pc" in r]
        pinf = fss.fit_eq7([r["W"] for r in ok], [r["L"] for r in ok], [r["pc"] for r in ok])[0] if len(ok) >= 2 else None
        out["variants"][name] = {"per_shape": per, "pc_inf_eq7": pinf}
    out["configs"] = n_cfg_total
    out["configs_per_s"] = n_cfg_total / wall
    return out


def fixed_count_leg(perc, workloads, stream):
    """Fixed-count ensemble (Sec. II.A) on the batched fiber (W=16 L=256): the device
    sampler alone (exactly K metallic tubes, the K smallest of N Philox keys) timed with
    HIP events, then Pi_k at 11 k around the fiber's threshold (one batch) and their
    binomial convolution (Pi_k interpolated linearly in k) to Pi(p) at three p."""
    import numpy as np
    import torch
    from paper_1401_2130_amd import fss
    wl = workloads.BATCH
    (W, L), seed = wl.shapes[0], wl.seed
    lat = perc.Lattice(W, L)
    N, n = lat.n, 1024
    out = torch.empty((n, lat.words), dtype=torch.int32, device="cuda")
    perc.perc_sample_fixed(lat, 0.18, seed, 64, out=out[:64], stream=stream)  # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    perc.perc_sample_fixed(lat, 0.18, seed, n, out=out, stream=stream)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    ks = [int(round(N * (0.170 + 0.0025 * i))) for i in range(11)]
    torch_sync()
    t0 = time.perf_counter()
    counts = fss.pi_fixed_counts(W, L, ks, n, seed, stream=stream)
    torch_sync()
    wall = time.perf_counter() - t0
    pk = counts / n
    ps = [0.1775, 0.18, 0.1825]
    # Pi_k is smooth in k: linear interpolation between the measured k gives every k of
    # the window the binomial weights need
    kk = np.arange(ks[0], ks[-1] + 1)
    conv, miss = fss.binomial_convolution(kk, np.interp(kk, ks, pk), N, ps)
    return {"workload": f"W={W} L={L} ({N} tubes), Philox seed {seed}",
            "sampler": {"configs": n, "ms": ms, "configs_per_s": n / (ms / 1e3), "keys_per_s": n * N / (ms / 1e3)},
            "pi_k": {"k": ks, "pi_k": pk.tolist(), "configs": n * len(ks), "wall_s": wall,
                     "configs_per_s": n * len(ks) / wall},
            "convolution": {f"{p}": {"pi": float(v), "uncovered_mass": float(m)} for p, v, m in zip(ps, conv, miss)}}


def fig6a_leg(perc, workloads, stream):
    """Pi against the fiber length at W = 3 (Fig. 6a): decay rate per p from ln Pi
    linear in L, and the line -ln(rate) against p (its inset)."""
    from paper_1401_2130_amd import fss
    wl = workloads.FIG6A
    torch_sync()
    t0 = time.perf_counter()
    counts = fss.pi_table(wl.shapes, wl.ps, wl.n_cfg, wl.seed, stream=stream)
    torch_sync()
    wall = time.perf_counter() - t0
    Ls = [L for (_, L) in wl.shapes]
    rows, lams, plist = {}, [], []
    for p in wl.ps:
        pis = [counts[(3, L, float(p))] / wl.n_cfg for L in Ls]
        fit = fss.decay_rate(Ls, pis, wl.n_cfg)
        rows[f"{p}"] = {"pi": pis, "decay": fit}
        if fit and fit["lambda"] > 0:
            lams.append(fit["lambda"])
            plist.append(p)
    line = fss.log_rate_slope(plist, lams)
    n_jobs = len(wl.shapes) * len(wl.ps) * wl.n_cfg
    return {"workload": f"W=3, L in {Ls} layers, p in {list(wl.ps)} x {wl.n_cfg}, Philox seed {wl.seed}",
            "configs": n_jobs, "configs_per_s": n_jobs / wall, "per_p": rows,
            "rate_unit": "per layer", "neg_log_rate_vs_p": None if line is None else {"b0": line[0], "b1": line[1]}}


def torch_sync():
    import torch
    torch.cuda.synchronize()


def serving_leg(perc, workloads, n: int, rate_hz: float, stream, grid: int = 0, tick: int = 16):
    """Serve the first n requests of the serving recipe (W, L, p per request; Philox seed
    = request id, configuration 0) with arrivals rescaled to rate_hz; latency = completion
    minus scheduled arrival on the host steady clock."""
    import numpy as np
    base = workloads.serving_requests(n)
    scale = workloads.SERVING.rate_hz / rate_hz
    reqs = [(t * scale, W, L, p, i, 0, i) for (t, W, L, p, i) in base]
    srv = perc.perc_server(hbm_bytes=96 << 30, max_slots=2048, tick_steps=tick, max_w=workloads.SERVING.w_range[1],
                           grid=grid, stream=stream)
    t0 = time.perf_counter()
    res = srv.run(reqs)
    wall = time.perf_counter() - t0
    lat = np.array([r["t_done_ns"] - r["t_arrive_ns"] for r in res], dtype=np.float64) / 1e6
    upd = sum(int(r["steps"]) * perc.Lattice(r["W"], r["L"]).n for r in res)
    span = reqs[-1][0] if reqs else 0.0
    st = srv.stats()
    del srv
    return {"requests": n, "offered_per_s": rate_hz, "arrival_span_s": span, "wall_s": wall,
            "completed_per_s": n / wall, "site_updates_per_s": upd / wall,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "percolating": float(np.mean([r["perc"] for r in res])),
            "ticks": st["ticks"], "tick_steps": tick, "max_slots": 2048, "grid": grid,
            "overloaded": bool(wall > 1.5 * span + 1.0)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", default="span", choices=["span", "span2", "persist", "auto"])
    ap.add_argument("--depth", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0, help="workgroups per step launch (0: the library's choice)")
    ap.add_argument("--graph-steps", type=int, default=0)
    ap.add_argument("--plain-sample", type=int, default=4, help="configurations per p for the plain form")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy this many MiB device to device (counter calibration runs)")
    ap.add_argument("--copy-bandwidth-mib", type=int, default=1024,
                    help="measure device-to-device copy bandwidth on this many MiB (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="serving leg: first requests of the Poisson stream at its own rate (0: skip)")
    ap.add_argument("--serve-low-rate", type=float, default=150.0,
                    help="serving leg at a sustainable rate: the same request mix at this many per second")
    ap.add_argument("--serve-low-requests", type=int, default=450)
    ap.add_argument("--serve-grid", type=int, default=0, help="server step-launch workgroups (0: library default)")
    ap.add_argument("--serve-tick", type=int, default=16, help="steps per server tick")
    ap.add_argument("--batched", type=int, default=1, help="batched Pi(p) leg (W=16 L=256, 21 p x 4096)")
    ap.add_argument("--first-passage", type=int, default=1024,
                    help="moves of the backward all-sources leg on the headline fiber (0: skip)")
    ap.add_argument("--ablation", type=int, default=1, help="regular FCC vs modified lattice thresholds")
    ap.add_argument("--fig6a", type=int, default=1, help="Pi against L at W=3, decay rates")
    ap.add_argument("--fixed-count", type=int, default=1, help="fixed-count ensemble sampler and Pi_k leg")
    ap.add_argument("--uneven", type=int, default=1, help="uneven aspect-ratio sweep leg (35 shapes x 2 p x 1024)")
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
    opts = dict(form=args.form, depth=args.depth, block=args.block, graph_steps=args.graph_steps, grid=args.grid)

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
        # the work-independent count (N x steps per configuration) priced at the same
        # 8.375 B: the kernel touches only the cells up to front + 1 of each step, so this
        # exceeds the bytes it moves; the roofline below uses the cells it does process
        "site_update_bytes": {"gbs": site_updates / (elapsed / args.steps) * BYTES_PER_TUBE_STEP / 1e9,
                              "frac": site_updates / (elapsed / args.steps) * BYTES_PER_TUBE_STEP / 1e9 / HBM_PEAK_GBS},
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
    # the m* (shortest spanning path) distribution of the timed workload, on the device
    result["backbone"] = {"bins": "m* = tubes on the shortest spanning path", "per_p": {}}
    for (b, s, _), p in zip(bufs, wl.ps):
        h = perc.perc_steps_hist(b, s, 4 * L, stream=stream)
        torch.cuda.synchronize()
        result["backbone"]["per_p"][f"{p}"] = hist_summary(h.cpu().numpy())
    if args.first_passage > 0:
        log(f"first-passage leg (M = {args.first_passage}) ...")
        result["first_passage"] = first_passage_leg(perc, workloads, stream, args.first_passage)
        log(f"first passage: {result['first_passage']['ms']:.1f} ms, "
            f"{result['first_passage']['achieved_gbs']:.0f} GB/s")
    if args.batched:
        log("batched Pi(p) leg ...")
        result["batched"] = batched_leg(perc, workloads, stream)
        log(f"batched: {result['batched']['configs_per_s']:.0f} configs/s, fit {result['batched'].get('eq5_fit')}")
    if args.uneven:
        log("uneven aspect-ratio leg ...")
        result["uneven"] = uneven_leg(perc, workloads, stream)
        log(f"uneven: {result['uneven']['configs_per_s']:.0f} configs/s, pc_inf {result['uneven']['pc_inf']}")
    if args.ablation:
        log("ablation leg (regular FCC) ...")
        result["ablation"] = ablation_leg(perc, workloads, stream)
        log(f"ablation: pc_inf regular {result['ablation']['variants']['regular_fcc']['pc_inf_eq7']}, "
            f"modified {result['ablation']['variants']['modified']['pc_inf_eq7']}")
    if args.fixed_count:
        log("fixed-count ensemble leg ...")
        result["fixed_count"] = fixed_count_leg(perc, workloads, stream)
        log(f"fixed count: sampler {result['fixed_count']['sampler']['configs_per_s']:.0f} configs/s")
    if args.fig6a:
        log("Fig. 6a leg (Pi vs L at W=3) ...")
        result["fig6a"] = fig6a_leg(perc, workloads, stream)
        log(f"fig6a: {result['fig6a']['neg_log_rate_vs_p']}")
    if args.serve_requests > 0:
        log(f"serving: {args.serve_requests} requests at {workloads.SERVING.rate_hz:.0f}/s ...")
        result["serving"] = {"offered": serving_leg(perc, workloads, args.serve_requests, workloads.SERVING.rate_hz,
                                                    stream, args.serve_grid, args.serve_tick)}
        if args.serve_low_requests > 0:
            log(f"serving: {args.serve_low_requests} requests at {args.serve_low_rate:.0f}/s ...")
            result["serving"]["sustainable"] = serving_leg(perc, workloads, args.serve_low_requests,
                                                           args.serve_low_rate, stream, args.serve_grid, args.serve_tick)
        result["serving"]["workload"] = ("Poisson arrivals (seed 5), W uniform 8..64, L uniform 64..4096, "
                                         "p uniform 0.12..0.19, Philox seed = request id, configuration 0")
        log(f"serving p50/p99: {result['serving']['offered']['p50_ms']:.1f} / "
            f"{result['serving']['offered']['p99_ms']:.1f} ms")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
