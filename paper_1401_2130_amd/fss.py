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
    jobs, keys = [], []
    for (W, L) in shapes:
        for p in ps:
            g = len(keys)
            keys.append((W, L, float(p)))
            jobs += [(lats[(W, L)], float(p), seed, c, g) for c in range(n_cfg)]
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
