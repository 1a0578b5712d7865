"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

Holds none of the method's arithmetic: workload recipes (fiber shape, metallic
probability, Philox seed, number of configurations) and a numpy generator of random
canonical occupancy words for inspections whose occupancy is given directly. The
paper measures no public dataset; every workload here is synthetic, shaped like the
paper's Monte-Carlo runs (Sec. III: p near the threshold, 1,024 configurations per
point, lattices up to millions of sites).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    shapes: Tuple[Tuple[int, int], ...]  # (W, L) fiber shapes
    ps: Tuple[float, ...]                # metallic probabilities
    seed: int                            # Philox key
    n_cfg: int                           # configurations per (shape, p)
    notes: str = ""


# Plain method, small fiber: W=4, L=16 (324 tubes), p=0.1533, 1000 configurations.
SMALL = Workload("plain-small W4 L16", ((4, 16),), (0.1533,), 1, 1000,
                 "one configuration at a time")
# Plain method, large single configurations: W=32, L=1024 (1,081,686 tubes).
LARGE = Workload("large W32 L1024", ((32, 1024),), (0.14, 0.1533, 0.17), 2, 256,
                 "256 configurations at each of three p")
# Batched Monte Carlo: W=16, L=256 (69,716 tubes), 21 p in 0.10..0.20, 4096 each.
BATCH = Workload("batched W16 L256", ((16, 256),), tuple((100 + 5 * i) / 1000.0 for i in range(21)), 3, 4096,
                 "Pi(p) curve and threshold estimate")
# Uneven batch, aspect-ratio sweep: W in {8,12,16,24,32}, L/W in {1,..,64}, 1024 each.
UNEVEN = Workload("uneven aspect sweep", tuple((w, w * a) for w in (8, 12, 16, 24, 32) for a in (1, 2, 4, 8, 16, 32, 64)),
                  (0.1533, 0.16), 4, 1024, "mixed shapes in one batch; finite-size scaling")


# Ablation (Sec. III comparison with the regular FCC lattice, threshold 0.199 in the
# literature): near-cubic fibers, L = 1.5 W layers (about 2.1 W tube spacings long against
# a 2 W diameter), both lattice variants on the same Philox configurations.
ABLATION = Workload("regular FCC vs modified", ((12, 18), (16, 24), (24, 36), (32, 48)),
                    tuple((120 + 5 * i) / 1000.0 for i in range(25)), 6, 1024,
                    "Pi(p) of both lattice variants; Eq. 5 per shape, Eq. 7 at one aspect ratio")
# Fig. 6a: Pi against the fiber length at W = 3 for several p (exponential decay).
FIG6A = Workload("Pi vs L at W=3", tuple((3, L) for L in (6, 12, 24, 48, 96, 192, 384, 768, 1536, 3072)),
                 (0.2, 0.25, 0.3, 0.35, 0.4, 0.45, 0.5), 7, 2048, "decay rate per p; -ln(rate) against p")


# Paper-scale finite-size scaling (Sec. III, Fig. 3-5; 1,024 configurations per point,
# lattices up to 2.7 M tubes): Fig. 3a W = 5 at L = 30..1920 layers; Fig. 3b L = 1200
# layers (400 unit cells) at W = 3..32; Fig. 4 grid W in {4..48} x L/W in {3, 6, 12, 24}.
FSS_PAPER = Workload("paper-scale FSS", tuple(dict.fromkeys(
    [(5, L) for L in (30, 60, 120, 240, 480, 960, 1920)]
    + [(W, 1200) for W in (3, 5, 8, 12, 16, 24, 32)]
    + [(W, W * a) for W in (4, 6, 8, 12, 16, 24, 32, 48) for a in (3, 6, 12, 24)])),
    (), 8, 1024, "p windows from a coarse pass; Eq. 5 per shape, Eq. 7-9")
FSS_SMALL = Workload("paper-scale FSS (reduced)", tuple((W, W * a) for W in (4, 6, 8, 12) for a in (3, 6, 12)),
                     (), 8, 256, "the same pipeline on small shapes")


@dataclass(frozen=True)
class ServingRecipe:
    rate_hz: float = 2000.0
    w_range: Tuple[int, int] = (8, 64)
    l_range: Tuple[int, int] = (64, 4096)
    p_range: Tuple[float, float] = (0.12, 0.19)
    arrival_seed: int = 5


SERVING = ServingRecipe()


def serving_requests(n: int, recipe: ServingRecipe = SERVING):
    """n requests (arrival time [s], W, L, p, request id) of a Poisson stream."""
    rng = np.random.default_rng(recipe.arrival_seed)
    gaps = rng.exponential(1.0 / recipe.rate_hz, size=n)
    t = np.cumsum(gaps) - gaps[0]
    W = rng.integers(recipe.w_range[0], recipe.w_range[1] + 1, size=n)
    L = rng.integers(recipe.l_range[0], recipe.l_range[1] + 1, size=n)
    p = rng.uniform(recipe.p_range[0], recipe.p_range[1], size=n)
    return [(float(t[i]), int(W[i]), int(L[i]), float(p[i]), i) for i in range(n)]


def random_occupancy(n_sites: int, n_cfg: int, p: float, seed: int, pad_garbage: bool = False) -> np.ndarray:
    """Canonical occupancy words [n_cfg, ceil(n_sites/32)] (uint32): each tube metallic
    with probability p from numpy's PCG64 stream. With pad_garbage the padding bits past
    n_sites are set at random too (they must be ignored)."""
    words = (n_sites + 31) // 32
    rng = np.random.default_rng(seed)
    occ = rng.random((n_cfg, words * 32)) < p
    if not pad_garbage:
        occ[:, n_sites:] = False
    else:
        occ[:, n_sites:] = rng.random((n_cfg, words * 32 - n_sites)) < 0.5
    return np.packbits(occ.astype(np.uint8), axis=1, bitorder="little").view(np.uint32).reshape(n_cfg, words)
