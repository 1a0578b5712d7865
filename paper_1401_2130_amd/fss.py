"""Pi(p) curves and the finite-size-scaling analysis of Sec. III.

The GPU side (``pi_curve``, ``pi_table``) runs all configurations of a sweep in one
``perc_batch`` launch sequence, with one output group per (shape, p), and returns the
integer percolating counts. The fits are host-side statistics on those counts:

* Eq. 5: Pi(p) = 1 / (1 + exp((p_c - p) / T)), the effective threshold p_c of a finite
  fiber being the p where Pi = 1/2 (``fit_fermi_dirac``; ``pc_two_point`` solves it from
  two points on the logit scale);
* Eq. 6-7: p_c = p_c_inf + C(W/L) L^(-1/nu), nu = 0.88 in 3D, one slope per aspect ratio
  and a common intercept (``fit_eq7``);
* Eq. 8: C(W/L) = C0 + C1 (W/L)^alpha (``fit_eq8``), hence Eq. 9:
  p_c = p_c_inf + C0 L^(-1/nu) + C1 W^alpha L^(-alpha - 1/nu) (``eq9``).
"""
from __future__ import annotations

import math
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

NU_3D = 0.88  # universal correlation-length exponent in three dimensions (Sec. III)


def fermi_dirac(p, pc: float, T: float):
    """Eq. 5."""
    return 1.0 / (1.0 + np.exp((pc - np.asarray(p, dtype=np.float64)) / T))


def fit_fermi_dirac(ps: Sequence[float], pis: Sequence[float], n: int) -> Tuple[float, float, np.ndarray]:
    """Weighted least-squares fit of Eq. 5 to Pi estimates from n configurations each
    (binomial standard errors); returns (p_c, T, covariance)."""
    from scipy.optimize import curve_fit
    ps = np.asarray(ps, dtype=np.float64)
    pis = np.asarray(pis, dtype=np.float64)
    pe = np.clip(pis, 0.5 / n, 1.0 - 0.5 / n)
    sigma = np.sqrt(pe * (1.0 - pe) / n)
    inside = (pis > 0.0) & (pis < 1.0)
    if inside.any():
        pc0 = float(ps[inside][np.argmin(np.abs(pis[inside] - 0.5))])
    else:
        pc0 = float(ps[np.argmin(np.abs(pis - 0.5))])
    T0 = max((ps.max() - ps.min()) / 20.0, 1e-4)
    popt, pcov = curve_fit(fermi_dirac, ps, pis, p0=(pc0, T0), sigma=sigma, absolute_sigma=True, maxfev=20000)
    return float(popt[0]), float(popt[1]), pcov


def pc_two_point(p1: float, pi1: float, p2: float, pi2: float) -> Optional[Tuple[float, float]]:
    """(p_c, T) of the Eq. 5 curve through two points with 0 < Pi < 1 (logit(Pi) is linear
    in p); None if a point lies outside (0, 1) or the curve does not rise."""
    if not (0.0 < pi1 < 1.0 and 0.0 < pi2 < 1.0) or p1 == p2:
        return None
    l1, l2 = math.log(pi1 / (1.0 - pi1)), math.log(pi2 / (1.0 - pi2))
    if l2 == l1:
        return None
    T = (p2 - p1) / (l2 - l1)
    if T <= 0.0:
        return None
    return p1 - T * l1, T


def fit_eq7(W: Sequence[float], L: Sequence[float], pc: Sequence[float], nu: float = NU_3D,
            weights: Optional[Sequence[float]] = None) -> Tuple[float, Dict[float, float]]:
    """Eq. 7 with a common intercept: least squares of p_c = p_c_inf + C(r) L^(-1/nu) over
    the aspect ratios r = W/L present. Returns (p_c_inf, {r: C(r)})."""
    W = np.asarray(W, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    pc = np.asarray(pc, dtype=np.float64)
    r = W / L
    keys = sorted(set(np.round(r, 12).tolist()))
    A = np.zeros((len(pc), 1 + len(keys)))
    A[:, 0] = 1.0
    x = L ** (-1.0 / nu)
    for j, k in enumerate(keys):
        A[np.isclose(r, k, rtol=0, atol=1e-12), 1 + j] = x[np.isclose(r, k, rtol=0, atol=1e-12)]
    w = np.ones_like(pc) if weights is None else np.sqrt(np.asarray(weights, dtype=np.float64))
    sol, *_ = np.linalg.lstsq(A * w[:, None], pc * w, rcond=None)
    return float(sol[0]), {k: float(sol[1 + j]) for j, k in enumerate(keys)}


def fit_eq8(ratios: Sequence[float], slopes: Sequence[float]) -> Tuple[float, float, float]:
    """Eq. 8: C(r) = C0 + C1 r^alpha, fitted to per-aspect-ratio slopes; (C0, C1, alpha)."""
    from scipy.optimize import curve_fit
    r = np.asarray(ratios, dtype=np.float64)
    c = np.asarray(slopes, dtype=np.float64)

    def f(x, c0, c1, a):
        return c0 + c1 * np.power(x, a)

    popt, _ = curve_fit(f, r, c, p0=(float(np.min(c)), 0.3, -1.2), maxfev=50000)
    return float(popt[0]), float(popt[1]), float(popt[2])


def eq9(W, L, pc_inf: float, C0: float, C1: float, alpha: float, nu: float = NU_3D):
    """Eq. 9: the effective threshold of a W x L fiber."""
    W = np.asarray(W, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    return pc_inf + C0 * L ** (-1.0 / nu) + C1 * W ** alpha * L ** (-alpha - 1.0 / nu)


def decay_rate(Ls: Sequence[float], pis: Sequence[float], n: int, min_count: int = 8) -> Optional[dict]:
    """Block-product model of Sec. III (Fig. 6a): Pi = prod_i (1 - lambda_i) ~ exp(-lambda L)
    for a long fiber. Weighted least squares of ln Pi = a - lambda L over the points with
    at least min_count percolating and min_count non-percolating configurations out of n
    (variance of ln Pi ~ (1 - Pi) / (n Pi)). Returns {lambda, a, lambda_err, points} or
    None with fewer than two usable points."""
    L = np.asarray(Ls, dtype=np.float64)
    pi = np.asarray(pis, dtype=np.float64)
    use = (pi * n >= min_count) & ((1.0 - pi) * n >= min_count)
    if use.sum() < 2:
        return None
    L, pi = L[use], pi[use]
    w = n * pi / (1.0 - pi)  # 1 / var(ln Pi)
    A = np.stack([np.ones_like(L), -L], axis=1)
    sw = np.sqrt(w)
    sol, *_ = np.linalg.lstsq(A * sw[:, None], np.log(pi) * sw, rcond=None)
    cov = np.linalg.inv((A * w[:, None]).T @ A)
    return {"lambda": float(sol[1]), "a": float(sol[0]), "lambda_err": float(math.sqrt(cov[1, 1])),
            "points": int(use.sum())}


def log_rate_slope(ps: Sequence[float], lams: Sequence[float]) -> Optional[Tuple[float, float]]:
    """Sec. III estimate -ln(lambda) ~ p (the inset of Fig. 6a): least-squares line
    -ln(lambda) = b0 + b1 p over the positive rates; (b0, b1) or None."""
    p = np.asarray(ps, dtype=np.float64)
    lam = np.asarray(lams, dtype=np.float64)
    ok = lam > 0
    if ok.sum() < 2:
        return None
    b1, b0 = np.polyfit(p[ok], -np.log(lam[ok]), 1)
    return float(b0), float(b1)


# ---------------------------------------------------------------------------------
# Fixed-count ensemble (Sec. II.A) and its relation to the Bernoulli ensemble
# ---------------------------------------------------------------------------------

def binomial_window(N: int, p: float, eps: float = 1e-12) -> Tuple[int, int]:
    """Smallest k range [lo, hi] outside which the Binomial(N, p) mass is below eps."""
    from scipy.stats import binom
    lo = int(binom.ppf(eps / 2, N, p))
    hi = int(binom.isf(eps / 2, N, p))
    return max(lo, 0), min(hi, N)


def binomial_convolution(ks: Sequence[int], pi_k: Sequence[float], N: int, ps) -> Tuple[np.ndarray, np.ndarray]:
    """Pi(p) of the Bernoulli ensemble from fixed-count probabilities: a Bernoulli(p)
    configuration has k metallic tubes with probability C(N, k) p^k (1 - p)^(N - k) and,
    given k, is a uniform k-subset, so Pi(p) = sum_k C(N, k) p^k (1 - p)^(N - k) Pi_k.
    ks: the k at which Pi_k is known; returns (Pi(p), binomial mass not covered by ks)."""
    from scipy.stats import binom
    ks = np.asarray(ks, dtype=np.int64)
    pk = np.asarray(pi_k, dtype=np.float64)
    out, miss = [], []
    for p in np.atleast_1d(np.asarray(ps, dtype=np.float64)):
        w = binom.pmf(ks, N, p)
        out.append(float((w * pk).sum()))
        miss.append(max(0.0, 1.0 - float(w.sum())))
    return np.array(out), np.array(miss)


def pi_fixed_counts(W: int, L: int, ks: Sequence[int], n_cfg: int, seed: int, stream=None, **opts) -> np.ndarray:
    """Percolating counts of the fixed-count ensemble (exactly k metallic tubes) at every
    k in ks, n_cfg configurations each: device sampling with perc_sample_fixed, then one
    perc_batch over all of them with one output group per k."""
    import paper_1401_2130_amd as perc
    lat = perc.Lattice(W, L)
    N = lat.n
    keep, jobs = [], []
    for g, k in enumerate(ks):
        if not 0 <= int(k) <= N:
            raise ValueError(f"k = {k} outside [0, {N}]")
        # K = floor(N p + 1/2) with p = k / N is k exactly (N p differs from k by < 1/2)
        bits = perc.perc_sample_fixed(lat, int(k) / N, seed, n_cfg, stream=stream)
        keep.append(bits)
        jobs += [(lat, bits[c], g) for c in range(n_cfg)]
    _, _, _, counts = perc.perc_batch(jobs, n_groups=len(ks), stream=stream, **opts)
    return np.array(counts, dtype=np.int64)


# ---------------------------------------------------------------------------------
# GPU sweeps (one batch each)
# ---------------------------------------------------------------------------------

def pi_table(shapes: Iterable[Tuple[int, int]], ps: Sequence[float], n_cfg: int, seed: int, stream=None,
             ends: bool = True, **opts) -> Dict[Tuple[int, int, float], int]:
    """Percolating counts for every (W, L) x p, configurations 0..n_cfg-1 of the Philox
    stream `seed` (common random numbers across p), all in one perc_batch call (mixed
    shapes in one work list). Returns {(W, L, p): count}."""
    import paper_1401_2130_amd as perc
    shapes = list(shapes)
    lats = {s: perc.Lattice(*s, ends=ends) for s in shapes}
    blocks, keys = [], []
    for (W, L) in shapes:
        for p in ps:
            blocks.append(perc.philox_jobs(lats[(W, L)], float(p), seed, n_cfg, group=len(keys)))
            keys.append((W, L, float(p)))
    jobs = np.concatenate(blocks) if blocks else np.zeros(0, dtype=perc.JOB_DTYPE)
    _, _, _, counts = perc.perc_batch(jobs, n_groups=len(keys), stream=stream, **opts)
    return {k: int(c) for k, c in zip(keys, counts)}


def pi_curve(W: int, L: int, ps: Sequence[float], n_cfg: int, seed: int, stream=None, ends: bool = True,
             **opts) -> np.ndarray:
    """Pi(p) estimates of one fiber at every p (one batch); ends=False: regular FCC."""
    t = pi_table([(W, L)], ps, n_cfg, seed, stream=stream, ends=ends, **opts)
    return np.array([t[(W, L, float(p))] / n_cfg for p in ps])


def uneven_analysis(counts: Dict[Tuple[int, int, float], int], n_cfg: int, nu: float = NU_3D) -> dict:
    """Effective thresholds per shape from two p values (Eq. 5 through two points), then
    Eq. 7 (common intercept) and, with three or more aspect ratios, Eq. 8."""
    by_shape: Dict[Tuple[int, int], List[Tuple[float, float]]] = {}
    for (W, L, p), c in counts.items():
        by_shape.setdefault((W, L), []).append((p, c / n_cfg))
    rows = []
    for (W, L), pts in sorted(by_shape.items()):
        pts.sort()
        sol = pc_two_point(pts[0][0], pts[0][1], pts[-1][0], pts[-1][1]) if len(pts) >= 2 else None
        rows.append({"W": W, "L": L, "pi": [x[1] for x in pts], "pc": None if sol is None else sol[0],
                     "T": None if sol is None else sol[1]})
    ok = [r for r in rows if r["pc"] is not None]
    out = {"shapes": rows, "n_cfg": n_cfg, "nu": nu}
    if len(ok) >= 3:
        pinf, slopes = fit_eq7([r["W"] for r in ok], [r["L"] for r in ok], [r["pc"] for r in ok], nu)
        out["pc_inf"] = pinf
        out["slopes"] = {str(k): v for k, v in slopes.items()}
        if len(slopes) >= 3:
            try:
                out["eq8"] = dict(zip(("C0", "C1", "alpha"), fit_eq8(list(slopes), list(slopes.values()))))
            except Exception as e:  # a fit that does not converge is reported, not raised
                out["eq8"] = {"error": str(e)}
    return out


# ---------------------------------------------------------------------------------
# Paper-scale finite-size scaling (Fig. 3-5): per-shape Eq. 5 fits at 1,024
# configurations per point on a p window found by a coarse pass, then Eq. 7-9
# ---------------------------------------------------------------------------------

def pi_keys(keys: Sequence[Tuple[int, int, float]], n_cfg: int, seed: int, stream=None, ends: bool = True,
            **opts) -> Dict[Tuple[int, int, float], int]:
    """Percolating counts for arbitrary (W, L, p) points, configurations 0..n_cfg-1 of the
    Philox stream `seed`, all in one perc_batch call."""
    import paper_1401_2130_amd as perc
    lats: Dict[Tuple[int, int], object] = {}
    jobs = []
    for g, (W, L, p) in enumerate(keys):
        if (W, L) not in lats:
            lats[(W, L)] = perc.Lattice(W, L, ends=ends)
        jobs += [(lats[(W, L)], float(p), seed, c, g) for c in range(n_cfg)]
    _, _, _, counts = perc.perc_batch(jobs, n_groups=len(keys), stream=stream, **opts)
    return {(int(W), int(L), float(p)): int(c) for (W, L, p), c in zip(keys, counts)}


def fine_window(ps: Sequence[float], pis: Sequence[float], n: int, n_p: int, width: float = 3.0,
                t_min: float = 0.002) -> List[float]:
    """n_p points spanning p_c +- width T of a coarse Eq. 5 fit (p_c from the crossing of
    1/2 if the fit fails; T at least half the coarse spacing), inside [0, 1], rounded to
    1e-4."""
    ps = np.asarray(ps, dtype=np.float64)
    pis = np.asarray(pis, dtype=np.float64)
    try:
        pc, T, _ = fit_fermi_dirac(ps, pis, n)
        if not (0.0 < pc < 1.0) or not (0.0 < T < 0.5):
            raise ValueError("coarse fit out of range")
    except Exception:
        i = int(np.argmin(np.abs(pis - 0.5)))
        pc, T = float(ps[i]), float(ps[1] - ps[0]) if len(ps) > 1 else 0.02
    # the coarse grid cannot place p_c better than its spacing
    if len(ps) > 1:
        t_min = max(t_min, 0.5 * float(np.median(np.diff(np.sort(ps)))))
    T = max(T, t_min)
    lo, hi = max(pc - width * T, 1e-4), min(pc + width * T, 1.0 - 1e-4)
    return [round(float(x), 4) for x in np.linspace(lo, hi, n_p)]


def fss_analysis(counts: Dict[Tuple[int, int, float], int], n_cfg: int, nu: float = NU_3D,
                 min_w: int = 0) -> dict:
    """Eq. 5 per shape (p_c, T and the standard error of p_c); Eq. 7 with a common
    intercept over the aspect ratios W/L that hold two or more shapes (weighted by
    1/err^2, with the intercept's standard error); Eq. 8 on their slopes; Eq. 9
    residuals of every shape; the Fig. 5 check (p_c linear in W^alpha at fixed L); and
    the constants in the paper's length unit (unit cells = 3 layers). Shapes narrower than
    min_w enter the per-shape table only (corrections to scaling are largest there)."""
    from fractions import Fraction
    by_shape: Dict[Tuple[int, int], List[Tuple[float, float]]] = {}
    for (W, L, p), c in counts.items():
        by_shape.setdefault((W, L), []).append((p, c / n_cfg))
    rows = []
    for (W, L), pts in sorted(by_shape.items()):
        pts.sort()
        ps, pis = [x[0] for x in pts], [x[1] for x in pts]
        row = {"W": W, "L": L, "p": ps, "pi": pis}
        try:
            pc, T, cov = fit_fermi_dirac(ps, pis, n_cfg)
            if not (ps[0] <= pc <= ps[-1]) or not (0.0 < T < 1.0):
                raise ValueError(f"threshold {pc:.4g} outside the sampled window {ps[0]}..{ps[-1]}")
            row.update(pc=pc, T=T, pc_err=float(math.sqrt(max(cov[0, 0], 0.0))))
        except Exception as e:  # reported, not raised
            row["error"] = str(e)
        rows.append(row)
    out: dict = {"shapes": rows, "n_cfg": n_cfg, "nu": nu}
    ok = [r for r in rows if "pc" in r and r["pc_err"] > 0 and r["W"] >= min_w]
    out["min_w"] = min_w
    groups: Dict[Fraction, List[dict]] = {}
    for r in ok:
        groups.setdefault(Fraction(r["W"], r["L"]), []).append(r)
    multi = [r for k, g in groups.items() if len(g) >= 2 for r in g]
    if len(multi) >= 3:
        keys = sorted({Fraction(r["W"], r["L"]) for r in multi})
        A = np.zeros((len(multi), 1 + len(keys)))
        A[:, 0] = 1.0
        for i, r in enumerate(multi):
            A[i, 1 + keys.index(Fraction(r["W"], r["L"]))] = r["L"] ** (-1.0 / nu)
        y = np.array([r["pc"] for r in multi])
        w = np.array([1.0 / r["pc_err"] ** 2 for r in multi])
        AtWA = (A * w[:, None]).T @ A
        sol = np.linalg.solve(AtWA, (A * w[:, None]).T @ y)
        cov = np.linalg.inv(AtWA)
        chi2 = float((((A @ sol) - y) ** 2 * w).sum())
        dof = max(len(multi) - A.shape[1], 1)
        scale = max(chi2 / dof, 1.0)  # inflate by the scatter beyond the binomial errors
        out["pc_inf"] = float(sol[0])
        out["pc_inf_err"] = float(math.sqrt(cov[0, 0] * scale))
        out["eq7_chi2_per_dof"] = chi2 / dof
        slopes = {float(k): float(sol[1 + j]) for j, k in enumerate(keys)}
        out["slopes"] = {f"{k:.6g}": v for k, v in slopes.items()}
        if len(slopes) >= 3:
            try:
                C0, C1, alpha = fit_eq8(list(slopes), list(slopes.values()))
                out["eq8"] = {"C0": C0, "C1": C1, "alpha": alpha}
                k = 3.0 ** (-1.0 / nu)
                out["eq8_paper_units"] = {"C0": C0 * k, "C1": C1 * k * 3.0 ** (-alpha), "alpha": alpha}
                res = []
                for r in ok:
                    pred = float(eq9(r["W"], r["L"], out["pc_inf"], C0, C1, alpha, nu))
                    res.append((r["pc"] - pred) / r["pc_err"])
                out["eq9_residual_sigma"] = {"rms": float(np.sqrt(np.mean(np.square(res)))),
                                             "max": float(np.max(np.abs(res)))}
                fig5 = {}
                for L in sorted({r["L"] for r in ok}):
                    g = [r for r in ok if r["L"] == L]
                    if len(g) >= 3:
                        xw = np.array([r["W"] ** alpha for r in g])
                        b1, b0 = np.polyfit(xw, [r["pc"] for r in g], 1)
                        fig5[str(L)] = {"slope": float(b1), "intercept": float(b0),
                                        "eq9_slope": C1 * L ** (-alpha - 1.0 / nu), "shapes": len(g)}
                out["fig5"] = fig5
            except Exception as e:
                out["eq8"] = {"error": str(e)}
    return out


def paper_scale_sweep(shapes: Sequence[Tuple[int, int]], seed: int, n_cfg: int = 1024, n_coarse: int = 128,
                      n_mid: int = 256, coarse_ps: Optional[Sequence[float]] = None, n_p: int = 12, stream=None,
                      log=None, ends: bool = True, **opts) -> dict:
    """Four passes per shape: a coarse p grid (n_coarse configurations), two windows of n_p
    points around the last Eq. 5 threshold (n_mid each), and the final window of n_p
    points at p_c +- 3 T of the last fit (n_cfg configurations per point, the paper's
    1,024).
    Each pass runs in batches of similar-sized shapes (one perc_batch each, progress
    reported per batch); the final counts go to fss_analysis. Passes use different
    Philox seeds, so the final estimates do not reuse the configurations that placed
    their window."""
    import time
    import paper_1401_2130_amd as perc
    shapes = [tuple(s) for s in shapes]
    if coarse_ps is None:
        coarse_ps = [round(0.06 + 0.02 * i, 4) for i in range(33)]
    log = log or (lambda *a: None)
    size = {sh: perc.Lattice(*sh).n for sh in shapes}
    order = sorted(shapes, key=lambda sh: size[sh])
    t0 = time.perf_counter()
    n_jobs = 0

    def run(windows: Dict[Tuple[int, int], List[float]], n: int, pass_seed: int, name: str):
        nonlocal n_jobs
        budget = 5.0e12  # approximate tube-steps per batch (a few seconds of GPU time)
        out: Dict[Tuple[int, int, float], int] = {}
        batch: List[Tuple[int, int]] = []
        acc = 0.0
        for i, sh in enumerate(order):
            batch.append(sh)
            acc += size[sh] * n * len(windows[sh]) * sh[1]
            if acc >= budget or i == len(order) - 1:
                t1 = time.perf_counter()
                keys = [(W, L, p) for (W, L) in batch for p in windows[(W, L)]]
                out.update(pi_keys(keys, n, pass_seed, stream=stream, ends=ends, **opts))
                n_jobs += len(keys) * n
                log(f"{name}: {len(batch)} shapes up to {max(size[b] for b in batch)} tubes, {len(keys)} points x {n} "
                    f"in {time.perf_counter() - t1:.1f} s")
                batch, acc = [], 0.0
        return out

    def refine(counts, windows, n):
        return {sh: fine_window(windows[sh], [counts[(sh[0], sh[1], float(p))] / n for p in windows[sh]], n, n_p)
                for sh in shapes}

    w = {sh: [float(p) for p in coarse_ps] for sh in shapes}
    c = run(w, n_coarse, seed + 3000, "coarse pass")
    w = refine(c, w, n_coarse)
    for k in range(2):  # each middle pass narrows a window by up to the spacing it had
        c = run(w, n_mid, seed + 2000 - 1000 * k, f"middle pass {k + 1}")
        w = refine(c, w, n_mid)
    counts = run(w, n_cfg, seed, "final pass")
    out = fss_analysis(counts, n_cfg)
    out["cuts"] = {}
    for mw in (8, 16, 24):
        a = fss_analysis(counts, n_cfg, min_w=mw)
        out["cuts"][str(mw)] = {k: a.get(k) for k in ("pc_inf", "pc_inf_err", "eq7_chi2_per_dof", "eq8",
                                                      "eq8_paper_units")}
    out["wall_s"] = time.perf_counter() - t0
    out["configs"] = n_jobs
    out["largest_tubes"] = max(size.values())
    out["passes"] = {"coarse": n_coarse, "middle": n_mid, "final": n_cfg, "points": n_p}
    return out


def _main(argv=None) -> int:
    import argparse
    import json
    ap = argparse.ArgumentParser(description="Paper-scale finite-size-scaling sweep (Fig. 3-5, Eq. 5-9) on one GPU")
    ap.add_argument("--out", default="", help="write the result as JSON here")
    ap.add_argument("--n-cfg", type=int, default=1024)
    ap.add_argument("--n-p", type=int, default=12)
    ap.add_argument("--regular-fcc", action="store_true", help="the lattice without end contacts")
    ap.add_argument("--small", action="store_true", help="the reduced shape set (a quick check)")
    a = ap.parse_args(argv)
    import sys
    import torch
    from paper_1401_2130_amd import workloads
    wl = workloads.FSS_SMALL if a.small else workloads.FSS_PAPER
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    res = paper_scale_sweep(wl.shapes, wl.seed, n_cfg=a.n_cfg, n_p=a.n_p, stream=stream, ends=not a.regular_fcc,
                            log=lambda *m: print(*m, file=sys.stderr, flush=True))
    res["workload"] = wl.name
    res["lattice"] = "regular FCC" if a.regular_fcc else "modified FCC"
    text = json.dumps(res)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text + "\n")
    print(json.dumps({k: res.get(k) for k in ("workload", "lattice", "pc_inf", "pc_inf_err", "eq7_chi2_per_dof", "eq8",
                                               "eq8_paper_units", "eq9_residual_sigma", "cuts", "configs", "wall_s",
                                               "largest_tubes")}), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(_main())
