"""The oracle's first-passage probabilities from every tube (Eq. 3 for all sources at
once), pinned on the CPU: hand-derived values on a single column, the identity with the
forward first-hit probability of the inspection for the uniform start mass, explicit
walk enumeration on a small fiber, and total absorption probability 1 exactly for the
tubes whose metallic cluster touches the far surface."""
import itertools
import math

import numpy as np
import pytest

import oracle


def occ_from_mask(lat, mask):
    words = np.zeros(lat.words, np.uint32)
    for s in np.nonzero(mask)[0]:
        words[s >> 5] |= np.uint32(1) << np.uint32(s & 31)
    return words


def test_single_column_by_hand():
    """Three tubes in a column (L = 7: layers 0, 3, 6), all metallic: degrees 1, 2, 2
    (the top tube's second edge is the detector). First-passage probabilities from
    (bottom, middle, top): m=1 (0, 0, 1/2); m=2 (0, 1/4, 0); m=3 (1/4, 0, 1/8);
    m=4 (0, 3/16, 0); m=5 (3/16, 0, 3/32)."""
    lat = oracle.Lattice(0, 7)
    assert lat.n == 3
    b = occ_from_mask(lat, np.ones(3, bool))
    expect = {1: (0, 0, 0.5), 2: (0, 0.25, 0), 3: (0.25, 0, 0.125), 4: (0, 0.1875, 0), 5: (0.1875, 0, 0.09375)}
    for m, v in expect.items():
        np.testing.assert_allclose(lat.first_passage_all(b, m), v, rtol=0, atol=0)


@pytest.mark.parametrize("W,L,p,seed", [(2, 9, 0.6, 1), (3, 13, 0.5, 2), (4, 16, 0.45, 3)])
def test_uniform_start_equals_forward_hit(W, L, p, seed):
    """sum over start tubes of (1/|S0|) f_s^(m*) is the first-hit probability the
    forward inspection reports at its stop m* (R6: same bilinear form)."""
    lat = oracle.Lattice(W, L)
    start, _ = lat.surfaces()
    bits = lat.sample(p, seed, 12)
    perc, steps, hit = lat.inspect_markov(bits)
    checked = 0
    for c in range(12):
        if not perc[c]:
            continue
        occ = np.unpackbits(bits[c].view(np.uint8), bitorder="little")[: lat.n].astype(bool)
        s0 = start & occ
        f = lat.first_passage_all(bits[c], int(steps[c]))
        assert math.isclose(f[s0].sum() / s0.sum(), hit[c], rel_tol=1e-12), (c, f[s0].sum() / s0.sum(), hit[c])
        checked += 1
    assert checked > 0


def test_walk_enumeration():
    """Explicit enumeration of all walks of length <= 4 on a small fiber: the probability
    of a walk is the product of 1/deg along it; it counts for step m if it enters the
    detector first at step m."""
    lat = oracle.Lattice(1, 5)
    ptr, idx = lat.adjacency()
    _, far = lat.surfaces()
    rng = np.random.default_rng(5)
    occ = rng.random(lat.n) < 0.7
    bits = occ_from_mask(lat, occ)
    nbr = [[int(j) for j in idx[ptr[i]:ptr[i + 1]] if occ[j]] for i in range(lat.n)]
    deg = [len(nbr[i]) + (1 if far[i] else 0) for i in range(lat.n)]
    for M in (1, 2, 3, 4):
        want = np.zeros(lat.n)
        for s in range(lat.n):
            if not occ[s]:
                continue
            # walks of M-1 tube-to-tube moves, then the detector edge from a far tube
            frontier = {(s,): 1.0}
            for _ in range(M - 1):
                nxt = {}
                for path, w in frontier.items():
                    i = path[-1]
                    if deg[i] == 0:  # self-loop
                        nxt[path + (i,)] = nxt.get(path + (i,), 0.0) + w
                    for j in nbr[i]:
                        nxt[path + (j,)] = nxt.get(path + (j,), 0.0) + w / deg[i]
                frontier = nxt
            want[s] = sum(w / deg[path[-1]] for path, w in frontier.items() if far[path[-1]])
        np.testing.assert_allclose(lat.first_passage_all(bits, M), want, rtol=1e-12, atol=1e-300)


def test_total_absorption():
    lat = oracle.Lattice(2, 9)
    bits = lat.sample(0.55, 4, 1)[0]
    occ = np.unpackbits(bits.view(np.uint8), bitorder="little")[: lat.n].astype(bool)
    total = sum(lat.first_passage_all(bits, m) for m in range(1, 3000))
    # tubes connected to the far surface through metallic tubes (plain BFS)
    ptr, idx = lat.adjacency()
    _, far = lat.surfaces()
    conn = far & occ
    frontier = list(np.nonzero(conn)[0])
    while frontier:
        i = frontier.pop()
        for j in idx[ptr[i]:ptr[i + 1]]:
            if occ[j] and not conn[j]:
                conn[j] = True
                frontier.append(j)
    np.testing.assert_allclose(total[conn], 1.0, rtol=0, atol=1e-9)
    assert np.all(total[~conn] == 0.0)
