#!/usr/bin/env python3
"""Benchmark of the percolation inspection on one MI355X.

Headline workload: fibers of hex radius W=32 and L=1024 layers (1,081,686 tubes), tubes
metallic with p in {0.14, 0.1533, 0.17}, 256 configurations at each p from Philox seed 2.
One step is the whole hot path over that batch, one perc_batch call of its 768 jobs with
one Pi group per p: occupancy sampling on the device, degree codes and start state, the
forward iteration to the stop of every configuration, the first-hit probabilities and the
Pi counts.

Printed (one JSON line on stdout): configurations inspected per second (value),
site-updates per second (N x steps per configuration, the same count for every form),
the roofline of the step kernel (HIP events on its stream inside the timed region, 8.375
algorithmic bytes per tube slot advanced one step) beside the streaming-copy ceiling,
the other workloads (the small plain one, the batched and uneven sweeps, the serving
stream) each with its own kernel roofline and its Pi counts checked against the oracle's
stored results, and the CPU oracle timed on the host cores.
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
STEP_KERNELS = {"span": "k_span_step", "plain": "k_span_step", "span2": "k_span_step2", "persist": "k_persist",
                "persist2": "k_persist2", "mixed": "k_persist + k_span_step"}


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
    # the measured bytes per tube slot, at this run's tube slots per launch
    return d["hbm_bytes_per_tube_step"] * tube_steps_per_launch


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


GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_workloads.json")


def golden_workloads():
    """The oracle's stored results of the benchmark workloads (tests/golden, written by a
    script that calls only the CPU oracle), or None when the file is absent."""
    if not os.path.exists(GOLDEN):
        return None
    with open(GOLDEN) as fh:
        return json.load(fh)["workloads"]


def parity(groups, counts) -> dict:
    """Pi counts of a leg against the oracle's, group by group."""
    want = [g["n_perc"] for g in groups]
    got = [int(c) for c in counts]
    return {"groups": len(want), "equal": got == want,
            "mismatches": [i for i, (a, b) in enumerate(zip(got, want)) if a != b][:10]}


def kernel_roofline(prof, kernel: str, part: str = "all") -> dict:
    """The step kernel's algorithmic bandwidth over its HIP-event time: of every timed
    launch, or of the persistent launches or the others alone (a mixed batch)."""
    ms, tubes, launches = prof["step_ms"], prof["tube_steps"], prof["step_launches"]
    if part == "persist":
        ms, tubes, launches = prof["persist_ms"], prof["persist_tube_steps"], prof["persist_launches"]
    elif part == "span":
        ms -= prof["persist_ms"]
        tubes -= prof["persist_tube_steps"]
        launches -= prof["persist_launches"]
    gbs = tubes * BYTES_PER_TUBE_STEP / (ms / 1e3) / 1e9 if ms > 0 else None
    return {"bound": "hbm", "kernel": kernel, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS if gbs else None, "launches": launches, "kernel_ms": ms,
            "tube_steps": tubes, "bytes_per_tube_step": BYTES_PER_TUBE_STEP}


def cpu_other_workloads(workloads, budget_s: float) -> dict:
    """The CPU oracle (explicit CSR FP64 Markov iteration, host Philox sampling, one
    configuration per OpenMP thread) on bounded samples of the other workloads: all of
    the small plain workload, and the first configurations of the batched and uneven
    sweeps at every p (uneven: the two smallest and the two largest shapes), each for
    about budget_s seconds."""
    import numpy as np
    import oracle
    cores = oracle.num_threads()
    out = {}

    def run(name, items, per):
        """items: (W, L, p, seed); per: configurations per item and pass"""
        lats, done, t, upd, cfg0 = {}, 0, 0.0, 0, {}
        while True:
            for (W, L, p, seed) in items:
                if (W, L) not in lats:
                    lats[(W, L)] = oracle.Lattice(W, L)
                ref = lats[(W, L)]
                c0 = cfg0.get((W, L, p), 0)
                t0 = time.perf_counter()
                pm, sm, _ = ref.inspect_markov(ref.sample(p, seed, per, cfg0=c0), nthreads=cores)
                t += time.perf_counter() - t0
                cfg0[(W, L, p)] = c0 + per
                done += per
                upd += int(np.sum(sm.astype(np.int64))) * ref.n
            if t >= budget_s or name == "small":
                break
        out[name] = {"value": done / t, "unit": "configs/s", "cores": cores, "kind": "oracle",
                     "site_updates_per_s": upd / t, "configs": done, "seconds": t}

    sm_ = workloads.SMALL
    run("small", [(sm_.shapes[0][0], sm_.shapes[0][1], sm_.ps[0], sm_.seed)], sm_.n_cfg)
    out["small"]["sample"] = "all 1000 configurations of W=4 L=16 p=0.1533 (seed 1)"
    b = workloads.BATCH
    run("batched", [(b.shapes[0][0], b.shapes[0][1], p, b.seed) for p in b.ps], cores)
    out["batched"]["sample"] = (f"configurations 0..{out['batched']['configs'] // len(b.ps) - 1} at each of the 21 p "
                                f"of W=16 L=256 (seed 3)")
    u = workloads.UNEVEN
    shapes = sorted(u.shapes, key=lambda s: s[0] * s[0] * s[1])
    pick = shapes[:2] + shapes[-2:]
    run("uneven", [(W, L, p, u.seed) for (W, L) in pick for p in u.ps], cores)
    out["uneven"]["sample"] = (f"configurations from 0 at both p of shapes {pick} of the aspect-ratio sweep "
                               f"(seed 4), {out['uneven']['configs']} in all")
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def leg_settings(perc, sample, n_target, stream, forced):
    """The autotuner's choice on `sample`, or the forced (form, depth) of a profiling run
    (a profiler's overhead would change the timings the tuner compares)."""
    if forced:
        form, depth = forced
        return {"form": form, "depth": depth, "block": 0, "graph_steps": 0, "ms": None, "forced": True}
    return perc.perc_autotune(sample, n_target=n_target, stream=stream)


def batched_leg(perc, workloads, stream, forced=None):
    """Batched Monte Carlo: every configuration of the Pi(p) sweep in one batch (one
    output group per p), settings picked by the autotuner on a sample, then the Eq. 5 fit."""
    import numpy as np
    from paper_1401_2130_amd import fss
    wl = workloads.BATCH
    (W, L), seed, n = wl.shapes[0], wl.seed, wl.n_cfg
    lat = perc.Lattice(W, L)
    # the tuning sample spans the sweep and fills the device several times over (one
    # workgroup per configuration in the persistent forms): 256 configurations at each
    # of the 21 p
    sample = np.concatenate([perc.philox_jobs(lat, p, seed, 256) for p in wl.ps])
    tuned = leg_settings(perc, sample, n * len(wl.ps), stream, forced)
    jobs = np.concatenate([perc.philox_jobs(lat, p, seed, n, group=g) for g, p in enumerate(wl.ps)])
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
           "kernel_roofline": kernel_roofline(prof, STEP_KERNELS[tuned["form"]]),
           "pi": {f"{p:.3f}": float(v) for p, v in zip(wl.ps, pis)}}
    if tuned["form"] in ("persist", "persist2"):
        out["kernel_roofline"]["note"] = ("the persistent launch also initialises every configuration and sums its "
                                          "first-hit probability: its rate is a lower bound")
    gw = golden_workloads()
    if gw:
        out["oracle_parity"] = parity(gw["batched"]["groups"], counts)
    try:
        pc, T, cov = fss.fit_fermi_dirac(wl.ps, pis, n)
        out["eq5_fit"] = {"pc": pc, "T": T, "pc_err": float(np.sqrt(cov[0, 0]))}
    except Exception as e:
        out["eq5_fit"] = {"error": str(e)}
    return out


def uneven_leg(perc, workloads, stream, forced=None):
    """Uneven batch: 35 shapes x 2 p x 1024 configurations mixed in one batch; effective
    thresholds per shape and the Eq. 7 / Eq. 8 fits."""
    from paper_1401_2130_amd import fss
    wl = workloads.UNEVEN
    lats = [perc.Lattice(*sh) for sh in wl.shapes]
    # the tuning sample spans the sweep: 64 configurations of every shape at both p (6 %
    # of the batch; smaller samples favour the span form over the mixed one, which wins on
    # the whole batch)
    import numpy as np
    sample = np.concatenate([perc.philox_jobs(lat, p, wl.seed, 64) for lat in lats for p in wl.ps])
    tuned = leg_settings(perc, sample, 0, stream, forced)
    opts = {k: tuned[k] for k in ("form", "depth", "block", "graph_steps")}
    torch_sync()
    t0 = time.perf_counter()
    counts = fss.pi_table(wl.shapes, wl.ps, wl.n_cfg, wl.seed, stream=stream, **opts)
    torch_sync()
    wall = time.perf_counter() - t0
    perc.perc_profile_enable(True)
    fss.pi_table(wl.shapes, wl.ps, wl.n_cfg, wl.seed, stream=stream, **opts)
    torch_sync()
    prof = perc.perc_profile_read()
    perc.perc_profile_enable(False)
    n_jobs = len(wl.shapes) * len(wl.ps) * wl.n_cfg
    ana = fss.uneven_analysis(counts, wl.n_cfg)
    out = {"workload": "W in {8,12,16,24,32} x L/W in {1,2,4,8,16,32,64}, p in {0.1533, 0.16} x 1024, Philox seed 4",
           "configs": n_jobs, "configs_per_s": n_jobs / wall, "wall_s": wall, "autotune": tuned,
           "kernel_roofline": kernel_roofline(prof, STEP_KERNELS[tuned["form"]]),
           "pc_inf": ana.get("pc_inf"), "eq8": ana.get("eq8"),
           "shapes_with_pc": sum(1 for r in ana["shapes"] if r["pc"] is not None)}
    if tuned["form"] == "mixed":
        # the span part's step kernel dominates; the persistent part (short-walk fibers,
        # beside it on a second stream) has its own line
        out["kernel_roofline"] = kernel_roofline(prof, "k_span_step", "span")
        out["persist_roofline"] = kernel_roofline(prof, "k_persist", "persist")
        out["persist_roofline"]["note"] = ("the persistent launch also initialises its configurations and sums their "
                                           "first-hit probability: its rate is a lower bound")
    gw = golden_workloads()
    if gw:
        keys = [(g["W"], g["L"], g["p"]) for g in gw["uneven"]["groups"]]
        out["oracle_parity"] = parity(gw["uneven"]["groups"], [counts[k] for k in keys])
    return out


def small_leg(perc, workloads, stream):
    """The small plain workload: W=4 L=16 p=0.1533, 1000 configurations one at a time in
    the plain form (the paper's one-configuration loop, the host checking the stop flags
    after every step), then all at once in the span form; Pi against the oracle."""
    import numpy as np
    wl = workloads.SMALL
    (W, L), p, seed, n = wl.shapes[0], wl.ps[0], wl.seed, wl.n_cfg
    lat = perc.Lattice(W, L)
    occ = perc.perc_sample(lat, p, seed, n, stream=stream)
    bits = torch_empty(n, "uint8")
    steps = torch_empty(n, "int32")
    perc.perc_inspect_ex(lat, occ[:8], 8, perc=bits[:8], steps=steps[:8], form="plain", stream=stream)  # warm-up
    torch_sync()
    t0 = time.perf_counter()
    for i in range(n):
        perc.perc_inspect_ex(lat, occ[i:i + 1], 1, perc=bits[i:i + 1], steps=steps[i:i + 1], form="plain",
                             stream=stream)
    torch_sync()
    wall = time.perf_counter() - t0
    st = steps.cpu().numpy().astype(np.int64)
    n_perc = int(bits.sum().item())
    torch_sync()
    t1 = time.perf_counter()
    n_span, _ = perc.perc_pi_ex(lat, p, n, seed, form="span", stream=stream)
    torch_sync()
    wall_span = time.perf_counter() - t1
    out = {"workload": f"W={W} L={L} ({lat.n} tubes), p = {p} x {n}, Philox seed {seed}",
           "plain": {"configs_per_s": n / wall, "wall_s": wall, "site_updates_per_s": float(st.sum()) * lat.n / wall,
                     "ms_per_config": wall / n * 1e3},
           "span_one_batch": {"configs_per_s": n / wall_span, "wall_s": wall_span},
           "pi": n_perc / n, "n_perc_plain": n_perc, "n_perc_span": n_span}
    gw = golden_workloads()
    if gw:
        out["oracle_parity"] = parity(gw["small"]["groups"], [n_perc])
        out["oracle_parity"]["span_equal"] = n_span == gw["small"]["groups"][0]["n_perc"]
    return out


def torch_empty(n, dtype):
    import torch
    return torch.empty(n, dtype=getattr(torch, dtype), device="cuda")


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


def serving_kernel_roofline(perc, workloads, n: int, stream, grid: int = 0, tick: int = 16) -> dict:
    """The first n requests of the serving recipe all arriving at once, served with the
    step profiler on (steps launched directly between HIP events): the step kernel's
    roofline over the server's ticks, and every served result against the oracle's
    stored ones."""
    base = workloads.serving_requests(n)
    reqs = [(0.0, W, L, p, i, 0, i) for (_, W, L, p, i) in base]
    srv = perc.perc_server(hbm_bytes=96 << 30, max_slots=2048, tick_steps=tick, max_w=workloads.SERVING.w_range[1],
                           grid=grid, stream=stream)
    perc.perc_profile_enable(True)
    res = {r["tag"]: r for r in srv.run(reqs)}
    prof = perc.perc_profile_read()
    perc.perc_profile_enable(False)
    del srv
    out = {"requests": n, "kernel_roofline": kernel_roofline(prof, STEP_KERNEL)}
    gw = golden_workloads()
    if gw:
        rows = [r for r in gw["serving"]["rows"] if r[0] < n]
        bad = [r[0] for r in rows if (res[r[0]]["perc"], res[r[0]]["steps"]) != (r[4], r[5])]
        out["oracle_parity"] = {"requests_checked": len(rows), "rule": gw["serving"]["rule"], "equal": not bad,
                                "mismatches": bad[:10]}
    return out


def serving_leg(perc, workloads, n: int, rate_hz: float, stream, grid: int = 0, tick: int = 16, lookahead: int = 0):
    """Serve the first n requests of the serving recipe (W, L, p per request; Philox seed
    = request id, configuration 0) with arrivals rescaled to rate_hz; latency = completion
    minus scheduled arrival on the host steady clock."""
    import numpy as np
    base = workloads.serving_requests(n)
    scale = workloads.SERVING.rate_hz / rate_hz
    reqs = [(t * scale, W, L, p, i, 0, i) for (t, W, L, p, i) in base]
    srv = perc.perc_server(hbm_bytes=96 << 30, max_slots=2048, tick_steps=tick, max_w=workloads.SERVING.w_range[1],
                           grid=grid, lookahead=lookahead, stream=stream)
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
            "ticks": st["ticks"], "tick_steps": tick, "max_slots": 2048, "grid": grid, "lookahead": lookahead,
            "overloaded": bool(wall > 1.5 * span + 1.0)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", default="span", choices=["span", "span2", "persist", "persist2", "auto"])
    ap.add_argument("--depth", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0, help="workgroups per step launch (0: the library's choice)")
    ap.add_argument("--graph-steps", type=int, default=0)
    ap.add_argument("--plain-sample", type=int, default=64, help="configurations per p for the plain form")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-other-seconds", type=float, default=5.0,
                    help="CPU oracle seconds on each of the batched and uneven samples (0: skip those)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first stream this many MiB with k_stream_copy (counter calibration runs)")
    ap.add_argument("--copy-bandwidth-mib", type=int, default=1024,
                    help="measure the streaming-copy ceiling on this many MiB (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="serving leg: first requests of the Poisson stream at its own rate (0: skip)")
    ap.add_argument("--serve-low-rate", type=float, default=150.0,
                    help="serving leg at a sustainable rate: the same request mix at this many per second")
    ap.add_argument("--serve-low-requests", type=int, default=450)
    ap.add_argument("--serve-grid", type=int, default=0, help="server step-launch workgroups (0: library default)")
    ap.add_argument("--serve-tick", type=int, default=16, help="steps per server tick")
    ap.add_argument("--serve-lookahead", type=int, default=0,
                    help="offered-load run: requests admitted past a waiting head (0: strict FIFO)")
    ap.add_argument("--serve-profile", type=int, default=1, help="profiled all-at-once serving run (kernel roofline)")
    ap.add_argument("--small", type=int, default=1, help="small plain workload leg (W=4 L=16 x 1000, one at a time)")
    ap.add_argument("--only", default="", choices=["", "small", "batched", "uneven", "serving"],
                    help="run this leg alone and print its JSON (profiling runs); not the benchmark line")
    ap.add_argument("--leg-form", default="", choices=["", "span", "span2", "persist", "persist2", "mixed"],
                    help="batched and uneven legs: this form instead of the autotuner's choice (profiling runs)")
    ap.add_argument("--leg-depth", type=int, default=0, help="cells per work item with --leg-form")
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

    torch.cuda.set_device(0)
    if args.copy_calibration_mib:
        # a copy of known size in the same process, for scaling the traffic counters
        src = torch.ones(args.copy_calibration_mib * 2 ** 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        perc.perc_stream_copy(src, dst)
        torch.cuda.synchronize()
        log(f"streamed {args.copy_calibration_mib} MiB for counter calibration (k_stream_copy)")
        del src, dst
    forced = (args.leg_form, args.leg_depth) if args.leg_form else None
    if args.only:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            if args.only == "small":
                res = small_leg(perc, workloads, stream)
            elif args.only == "batched":
                res = batched_leg(perc, workloads, stream, forced)
            elif args.only == "uneven":
                res = uneven_leg(perc, workloads, stream, forced)
            else:
                res = serving_kernel_roofline(perc, workloads, args.serve_requests, stream, args.serve_grid,
                                              args.serve_tick)
        print(json.dumps({args.only: res}), flush=True)
        return
    wl = workloads.LARGE
    (W, L), seed, n = wl.shapes[0], wl.seed, wl.n_cfg
    lat = perc.Lattice(W, L)
    stream = torch.cuda.Stream()
    n_total = n * len(wl.ps)
    bits_all = torch.empty(n_total, dtype=torch.uint8, device="cuda")
    steps_all_t = torch.empty(n_total, dtype=torch.int32, device="cuda")
    hit_all = torch.empty(n_total, dtype=torch.float32, device="cuda")
    bufs = [(bits_all[k * n:(k + 1) * n], steps_all_t[k * n:(k + 1) * n], hit_all[k * n:(k + 1) * n])
            for k in range(len(wl.ps))]
    # one batch of every (p, configuration) job, one Pi group per p
    jobs = np.concatenate([perc.philox_jobs(lat, p, seed, n, group=k) for k, p in enumerate(wl.ps)])
    opts = dict(form=args.form, depth=args.depth, block=args.block, graph_steps=args.graph_steps, grid=args.grid)

    def step():
        _, _, _, counts = perc.perc_batch(jobs, n_groups=len(wl.ps), perc=bits_all, steps=steps_all_t, hit=hit_all,
                                          stream=stream, **opts)
        return counts

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
    log(f"plain form: {len(wl.ps) * k} configurations in {t_plain:.2f} s")

    # the practical HBM ceiling on this device: the library's streaming copy (the step
    # kernel's grid and access pattern, no arithmetic), timed with events on its stream
    copy_gbs = None
    if args.copy_bandwidth_mib > 0:
        src = torch.ones(args.copy_bandwidth_mib * 2 ** 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        perc.perc_stream_copy(src, dst, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(10):
            perc.perc_stream_copy(src, dst, stream=stream)
        e1.record(stream)
        e1.synchronize()
        copy_gbs = 2 * src.numel() * 4 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        log(f"streaming copy: {copy_gbs:.0f} GB/s (read + write)")
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
                   "call": "perc_batch: 768 jobs, one Pi group per p",
                   "form": args.form, "depth": args.depth, "block": args.block},
        # the work-independent count (N x steps per configuration): the kernels process
        # only the cells up to front + 1 of each step, so this is a rate of work done, not a
        # bandwidth; the roofline below prices the cells the step kernel does process
        "site_updates_per_s": site_updates / (elapsed / args.steps),
        "graph_replay": {"configs_per_s": n_total * args.steps / elapsed_graph,
                         "ms_per_step": elapsed_graph / args.steps * 1e3,
                         "note": "same steps from captured HIP graphs, no per-launch events"},
        "pi": {str(p): c / n for p, c in zip(wl.ps, counts)},
        "plain": ({"configs_per_s": len(wl.ps) * k / t_plain, "site_updates_per_s": upd_plain / t_plain,
                   "sample": f"configurations 0..{k - 1} at each p, one at a time"} if k > 0 else None),
        "batched_over_plain": (value / (len(wl.ps) * k / t_plain)) if k > 0 else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "copy_gbs": copy_gbs, "copy_kernel": "k_stream_copy (perc_stream_copy, 1 GiB)",
                     "frac_of_copy": (achieved / copy_gbs) if copy_gbs else None,
                     "kernel": STEP_KERNEL, "launches": prof["step_launches"],
                     "avg_launch_us": prof["step_ms"] / launches * 1e3,
                     "tube_steps_per_launch": prof["tube_steps"] / launches,
                     "bytes_per_tube_step": BYTES_PER_TUBE_STEP},
    }
    gw = golden_workloads()
    if gw:
        result["oracle_parity"] = parity(gw["large"]["groups"], counts)
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
    if args.small:
        log("small plain leg ...")
        result["small"] = small_leg(perc, workloads, stream)
        log(f"small: plain {result['small']['plain']['configs_per_s']:.0f} configs/s")
    if args.batched:
        log("batched Pi(p) leg ...")
        result["batched"] = batched_leg(perc, workloads, stream, forced)
        log(f"batched: {result['batched']['configs_per_s']:.0f} configs/s, fit {result['batched'].get('eq5_fit')}")
    if args.uneven:
        log("uneven aspect-ratio leg ...")
        result["uneven"] = uneven_leg(perc, workloads, stream, forced)
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
                                                    stream, args.serve_grid, args.serve_tick, args.serve_lookahead)}
        if args.serve_low_requests > 0:
            log(f"serving: {args.serve_low_requests} requests at {args.serve_low_rate:.0f}/s ...")
            result["serving"]["sustainable"] = serving_leg(perc, workloads, args.serve_low_requests,
                                                           args.serve_low_rate, stream, args.serve_grid, args.serve_tick)
        if args.serve_profile:
            log("serving: profiled all-at-once run ...")
            result["serving"]["profiled"] = serving_kernel_roofline(perc, workloads, args.serve_requests, stream,
                                                                    args.serve_grid, args.serve_tick)
        result["serving"]["workload"] = ("Poisson arrivals (seed 5), W uniform 8..64, L uniform 64..4096, "
                                         "p uniform 0.12..0.19, Philox seed = request id, configuration 0")
        log(f"serving p50/p99: {result['serving']['offered']['p50_ms']:.1f} / "
            f"{result['serving']['offered']['p99_ms']:.1f} ms")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
        if args.cpu_other_seconds > 0:
            log("cpu baseline (oracle) on the other workloads ...")
            result["cpu_baseline"]["other_workloads"] = cpu_other_workloads(workloads, args.cpu_other_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
