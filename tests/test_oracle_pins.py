"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every expectation here comes from something other than the oracle itself: values
printed with the paper's Fig. 2, brute-force walk enumeration, closed forms for the
one-column fiber, an independent cubic-coordinate description of FCC, symmetries of
the lattice, or exhaustive enumeration checked by an independent Python search.
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------------
# Fig. 2 (Sec. II.B): the seven-tube chain
# ----------------------------------------------------------------------------------

def _fig2_matrix():
    rows = []
    with open(os.path.join(GOLDEN, "fig2_path.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                rows.append([Fraction(t) for t in line.split()])
    return rows


def _walk_first_passage(P, start, target, m_max):
    """Exact P_start[first hit of target at step m] by enumerating every walk."""
    n = len(P)
    out = [Fraction(0)] * (m_max + 1)
    frontier = {(start,): Fraction(1)}
    for m in range(1, m_max + 1):
        nxt = {}
        for walk, pr in frontier.items():
            i = walk[-1]
            for j in range(n):
                if P[i][j] == 0:
                    continue
                q = pr * P[i][j]
                if j == target:
                    out[m] += q
                else:
                    key = walk + (j,)
                    nxt[key] = nxt.get(key, Fraction(0)) + q
        frontier = nxt
    return out


def test_fig2_matrix_rows_sum_to_one():
    P = _fig2_matrix()
    assert len(P) == 7
    for row in P:
        assert sum(row) == 1  # Eq. (2): each row of P sums to one


def test_fig2_first_passage_zero_before_six_positive_at_six():
    P = _fig2_matrix()
    Pd = np.array([[float(v) for v in row] for row in P])
    f = oracle.eq3_backward(Pd, j0=6, M=12)  # tube 7 is index 6
    f1 = f[:, 0]  # starting from tube 1
    assert np.all(f1[:5] == 0.0)  # m = 1..5
    assert f1[5] > 0.0  # m = 6 = N_b
    # exact values from brute-force walk enumeration on the printed matrix
    exact = _walk_first_passage(P, 0, 6, 12)
    for m in range(1, 13):
        assert f1[m - 1] == pytest.approx(float(exact[m]), rel=1e-14, abs=0.0)
    assert exact[6] == Fraction(1, 32)  # the straight walk: 1 * (1/2)^5
    assert exact[7] == 0  # a path graph is bipartite: only even hitting times


def test_fig2_forward_equals_eq3_backward():
    P = _fig2_matrix()
    Pd = np.array([[float(v) for v in row] for row in P])
    f = oracle.eq3_backward(Pd, j0=6, M=20)
    for start in range(6):
        x0 = np.zeros(7); x0[start] = 1.0
        hit = oracle.first_passage_forward(Pd, 6, x0, 20)
        np.testing.assert_allclose(hit, f[:, start], rtol=1e-13, atol=1e-300)


def test_fig2_tube5_insulating_never_reaches():
    P = _fig2_matrix()
    # tube 5 insulating: remove it and renormalise the rows of its neighbours (Eq. 2)
    keep = [0, 1, 2, 3, 5, 6]
    n = len(keep)
    Pd = np.zeros((n, n))
    for a, i in enumerate(keep):
        nbrs = [b for b, j in enumerate(keep) if P[i][j] != 0]
        for b in nbrs:
            Pd[a, b] = 1.0 / len(nbrs)
    f = oracle.eq3_backward(Pd, j0=n - 1, M=40)
    assert np.all(f[:, 0] == 0.0)


# ----------------------------------------------------------------------------------
# Lattice (Sec. II.A, Fig. 1) against an independent cubic description of FCC
# ----------------------------------------------------------------------------------

def _cubic(q, r, k):
    """(q, r, k) -> 3 * cubic FCC coordinates, from the linear map that sends the
    three up-layer contacts to (1,1,0), (0,1,1), (1,0,1) (FCC nearest neighbours)."""
    q = np.asarray(q, np.int64); r = np.asarray(r, np.int64); k = np.asarray(k, np.int64)
    x = q - r + 2 * k
    y = q + 2 * r + 2 * k
    z = -2 * q - r + 2 * k
    return np.stack([x, y, z], axis=1)


_FCC_NN = {v for p in itertools.permutations((1, 1, 0)) for s in itertools.product((1, -1), repeat=3)
           for v in [tuple(a * b for a, b in zip(p, s))]}
_END = {(2, 2, 2), (-2, -2, -2)}


@pytest.mark.parametrize("W,L", [(0, 7), (1, 8), (2, 10), (3, 13), (4, 16)])
def test_lattice_is_fcc_with_end_contacts(W, L):
    lat = oracle.Lattice(W, L)
    q, r, k = lat.coords()
    X3 = _cubic(q, r, k)
    assert np.all(X3 % 3 == 0)  # every site is a point of the cubic lattice
    X = X3 // 3
    assert np.all(X.sum(axis=1) % 2 == 0)  # ... with even coordinate sum: an FCC point
    assert np.all(X.sum(axis=1) == 2 * k)  # layer k is the (111) plane x+y+z = 2k
    assert len(_FCC_NN) == 12
    pos = {tuple(v): i for i, v in enumerate(X)}
    ptr, idx = lat.adjacency()
    for i in range(lat.n):
        nb = set(idx[ptr[i]:ptr[i + 1]].tolist())
        expect = set()
        for v in _FCC_NN | _END:
            j = pos.get((X[i, 0] + v[0], X[i, 1] + v[1], X[i, 2] + v[2]))
            if j is not None:
                expect.add(j)
        assert nb == expect, (i, q[i], r[i], k[i])


@pytest.mark.parametrize("W", [0, 1, 2, 5, 8])
def test_column_count_and_site_count(W):
    L = 10
    lat = oracle.Lattice(W, L)
    q, r, k = lat.coords()
    cols = set(zip(q.tolist(), r.tolist()))
    assert len(cols) == 3 * W * (W + 1) + 1  # hexagon of hex radius W
    # each column (q,r) holds the layers k = (q-r) mod 3, +3, +6, ... below L
    n = sum(len(range((a - b) % 3, L, 3)) for a, b in cols)
    assert n == lat.n
    # canonical order is lexicographic (k, q, r)
    key = list(zip(k.tolist(), q.tolist(), r.tolist()))
    assert key == sorted(key)


def test_bulk_coordination_is_14():
    lat = oracle.Lattice(4, 16)
    q, r, k = lat.coords()
    ptr, idx = lat.adjacency()
    deg = np.diff(ptr)
    hexd = np.maximum(np.maximum(np.abs(q), np.abs(r)), np.abs(q + r))
    interior = (hexd <= 2) & (k >= 3) & (k <= 12)
    assert interior.sum() > 0
    assert np.all(deg[interior] == 14)
    for i in np.nonzero(interior)[0]:
        nb = idx[ptr[i]:ptr[i + 1]]
        same_col = (q[nb] == q[i]) & (r[nb] == r[i])
        assert same_col.sum() == 2  # 2 end contacts
        dk = k[nb] - k[i]
        assert sorted(dk[~same_col].tolist()) == [-1] * 3 + [0] * 6 + [1] * 3  # 12 side contacts


def test_surfaces_one_tube_per_column():
    lat = oracle.Lattice(3, 11)
    q, r, k = lat.coords()
    start, far = lat.surfaces()
    cols = len(set(zip(q.tolist(), r.tolist())))
    assert start.sum() == cols and far.sum() == cols
    assert np.all(k[start] <= 2) and np.all(k[far] >= 8)


# ----------------------------------------------------------------------------------
# Closed form: W = 0 is a single column joined only by end contacts (a 1-D chain)
# ----------------------------------------------------------------------------------

@pytest.mark.parametrize("L", [1, 2, 3, 4, 7, 16, 30])
def test_single_column_closed_form(L):
    lat = oracle.Lattice(0, L)
    n = math.ceil(L / 3)
    assert lat.n == n
    full = np.zeros((1, lat.words), np.uint32)
    for s in range(n):
        full[0, s >> 5] |= np.uint32(1 << (s & 31))
    perc, steps, hm = lat.inspect_markov(full)
    assert perc[0] == 1 and steps[0] == n  # n - 1 bonds, then one step to the detector
    # first-hit probability along the only path: deg(first)=1, inner/top sites deg 2
    assert hm[0] == pytest.approx(1.0 if n == 1 else 0.5 ** (n - 1), rel=1e-15)
    a = lat.exhaustive("markov")
    expect = np.zeros(n + 1, np.int64); expect[n] = 1
    np.testing.assert_array_equal(a, expect)  # Pi(p) = p^n
    for p in (0.1, 0.5, 0.9):
        assert oracle.pi_from_counts(a, p) == pytest.approx(p ** n, rel=1e-12)


# ----------------------------------------------------------------------------------
# Exhaustive enumeration on tiny lattices, checked by an independent Python search
# ----------------------------------------------------------------------------------

def _py_percolates(mask, q, r, k, L):
    X = _cubic(q, r, k) // 3
    n = len(q)
    occ = [(mask >> s) & 1 for s in range(n)]
    pos = {tuple(v): i for i, v in enumerate(X)}
    seen = set(s for s in range(n) if occ[s] and k[s] <= 2)
    stack = list(seen)
    while stack:
        s = stack.pop()
        if k[s] >= L - 3:
            return True
        for v in _FCC_NN | _END:
            j = pos.get((X[s, 0] + v[0], X[s, 1] + v[1], X[s, 2] + v[2]))
            if j is not None and occ[j] and j not in seen:
                seen.add(j); stack.append(j)
    return False


def test_exhaustive_matches_independent_search():
    W, L = 1, 4
    lat = oracle.Lattice(W, L)
    assert lat.n == 8
    q, r, k = lat.coords()
    a_py = np.zeros(lat.n + 1, np.int64)
    for mask in range(1 << lat.n):
        if _py_percolates(mask, q, r, k, L):
            a_py[bin(mask).count("1")] += 1
    np.testing.assert_array_equal(lat.exhaustive("bfs"), a_py)
    np.testing.assert_array_equal(lat.exhaustive("markov"), a_py)


@pytest.mark.parametrize("L", [5, 6, 7, 8])
def test_exhaustive_pi_properties(L):
    lat = oracle.Lattice(1, L)
    a = lat.exhaustive("markov")
    np.testing.assert_array_equal(a, lat.exhaustive("bfs"))
    assert oracle.pi_from_counts(a, 0.0) == 0.0  # Pi(0) = 0
    assert oracle.pi_from_counts(a, 1.0) == 1.0  # Pi(1) = 1: the full lattice connects
    ps = np.linspace(0, 1, 101)
    pis = [oracle.pi_from_counts(a, p) for p in ps]
    assert np.all(np.diff(pis) >= -1e-15)  # monotone in p
    # monotone per set size too: adding a metallic site never breaks a spanning path
    frac = [a[kk] / math.comb(lat.n, kk) for kk in range(lat.n + 1)]
    assert np.all(np.diff(frac) >= -1e-15)


# ----------------------------------------------------------------------------------
# The Markov iteration against the plain definition, and its invariants
# ----------------------------------------------------------------------------------

@pytest.mark.parametrize("W,L,p", [(2, 9, 0.3), (3, 13, 0.2), (4, 16, 0.1533), (6, 30, 0.25), (8, 40, 0.17)])
def test_markov_equals_bfs_equals_unionfind(W, L, p):
    lat = oracle.Lattice(W, L)
    bits = lat.sample(p, seed=11, n_cfg=64)
    pm, sm, _ = lat.inspect_markov(bits)
    pb, sb = lat.inspect_bfs(bits)
    pu = lat.inspect_uf(bits)
    np.testing.assert_array_equal(pm, pb)
    np.testing.assert_array_equal(pm, pu)
    np.testing.assert_array_equal(sm, sb)  # first hit = shortest path + 1 (Sec. II.B)


def test_row_sums_are_one():
    lat = oracle.Lattice(4, 16)
    for seed in range(5):
        bits = lat.sample(0.3, seed=seed, n_cfg=1)
        sums = lat.row_sums(bits)
        np.testing.assert_allclose(sums, 1.0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("K", [0, 1, 5, 16, 40])
def test_mass_conservation_and_support(K):
    lat = oracle.Lattice(4, 22)
    bits = lat.sample(0.35, seed=3, n_cfg=1)
    x, reach = lat.state_after(bits, K)
    start, far = lat.surfaces()
    occ = np.unpackbits(bits[0].view(np.uint8), bitorder="little")[: lat.n].astype(bool)
    if (occ & start).any():
        assert x.sum() == pytest.approx(1.0, abs=1e-12)
    assert np.all(x >= 0)
    assert np.all(reach[x > 0])  # FP can lose positivity but never create it
    assert not np.any(x[:-1][~occ]) and not np.any(reach[:-1][~occ])
    # reach after K steps = sites within distance K of the start set (BFS)
    d = lat.bfs_dist(bits)
    np.testing.assert_array_equal(reach[:-1], (d >= 0) & (d <= K))


def test_rotation_and_mirror_symmetry():
    W, L = 4, 22  # L = 1 mod 3: the mirror k -> L-1-k maps the lattice to itself
    lat = oracle.Lattice(W, L)
    q, r, k = lat.coords()
    index = {(a, b, c): i for i, (a, b, c) in enumerate(zip(q.tolist(), r.tolist(), k.tolist()))}
    rot = np.array([index[(-a - b, a, c)] for a, b, c in zip(q.tolist(), r.tolist(), k.tolist())])
    mir = np.array([index[(b, a, L - 1 - c)] for a, b, c in zip(q.tolist(), r.tolist(), k.tolist())])
    bits = lat.sample(0.3, seed=5, n_cfg=48)
    occ = np.unpackbits(bits.view(np.uint8), axis=1, bitorder="little")[:, : lat.n]

    def permute(perm):
        o2 = np.zeros_like(occ)
        o2[:, perm] = occ
        pad = np.zeros((occ.shape[0], lat.words * 32), np.uint8)
        pad[:, : lat.n] = o2
        return np.packbits(pad, axis=1, bitorder="little").view(np.uint32)

    p0, s0, _ = lat.inspect_markov(bits)
    p1, s1, _ = lat.inspect_markov(permute(rot))
    np.testing.assert_array_equal(p0, p1)
    np.testing.assert_array_equal(s0, s1)
    p2, s2, _ = lat.inspect_markov(permute(mir))
    np.testing.assert_array_equal(p0, p2)
    np.testing.assert_array_equal(s0[p0 == 1], s2[p0 == 1])  # same shortest spanning path


# ----------------------------------------------------------------------------------
# Sampler: integer Bernoulli rule and Philox stream
# ----------------------------------------------------------------------------------

def test_threshold_rule():
    assert oracle.threshold(0.0) == 0
    assert oracle.threshold(1.0) == 2 ** 32
    assert oracle.threshold(0.5) == 2 ** 31
    assert oracle.threshold(0.125) == 2 ** 29
    for p in (0.1, 0.1533, 0.17, 0.2):
        t = oracle.threshold(p)
        assert t <= p * 2 ** 32 < t + 1


def test_bernoulli_frequency_and_extremes():
    lat = oracle.Lattice(16, 64)
    for p in (0.0, 1.0):
        bits = lat.sample(p, seed=9, n_cfg=2)
        occ = np.unpackbits(bits.view(np.uint8), axis=1, bitorder="little")[:, : lat.n]
        assert occ.mean() == p
        pad = np.unpackbits(bits.view(np.uint8), axis=1, bitorder="little")[:, lat.n:]
        assert not pad.any()  # padding bits stay clear
    p = 0.1533
    bits = lat.sample(p, seed=9, n_cfg=8)
    occ = np.unpackbits(bits.view(np.uint8), axis=1, bitorder="little")[:, : lat.n]
    n = occ.size
    pt = oracle.threshold(p) / 2 ** 32
    assert abs(occ.sum() - n * pt) < 5 * math.sqrt(n * pt * (1 - pt))  # <N_m> = Np (Sec. II.A)
    # neighbouring sites are independent: joint frequency of adjacent pairs ~ p^2
    both = (occ[:, :-1] & occ[:, 1:]).sum()
    m = occ[:, :-1].size
    assert abs(both - m * pt * pt) < 5 * math.sqrt(m * pt * pt)


def test_common_random_numbers_monotone():
    lat = oracle.Lattice(6, 30)
    lo = lat.sample(0.15, seed=2, n_cfg=64)
    hi = lat.sample(0.25, seed=2, n_cfg=64)
    assert np.all((lo & ~hi) == 0)  # lower p occupies a subset
    plo, _ = lat.inspect_bfs(lo)
    phi, _ = lat.inspect_bfs(hi)
    assert np.all(plo <= phi)


def test_philox_output_uniform():
    outs = np.array([oracle.philox4x32_10([i, 7, 0, 3], [1, 0]) for i in range(4096)], np.uint32)
    by = outs.view(np.uint8).ravel()
    counts = np.bincount(by, minlength=256)
    exp = by.size / 256
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 255 + 6 * math.sqrt(2 * 255)  # far inside the chi-square tail
    bitsum = np.unpackbits(outs.view(np.uint8)).mean()
    assert abs(bitsum - 0.5) < 0.005
    # different keys and counters give different words
    a = oracle.philox4x32_10([0, 0, 0, 0], [0, 0])
    b = oracle.philox4x32_10([1, 0, 0, 0], [0, 0])
    c = oracle.philox4x32_10([0, 0, 0, 0], [1, 0])
    assert not np.array_equal(a, b) and not np.array_equal(a, c)


def test_philox_known_answers():
    """The oracle's Philox4x32-10 reproduces the published known-answer outputs of the
    generator (tests/golden/philox4x32_10_kat.txt), which fixes its multipliers, Weyl
    increments, round count and word order; the device sampler is bit-exact against the
    oracle (GPU tests), so it is pinned too."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.txt")
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(x, 16) for x in r]
        out = oracle.philox4x32_10(w[0:4], w[4:6])
        assert [int(x) for x in out] == w[6:10], r


def test_philox_key_schedule_shift():
    """Pins the round count and key schedule of the oracle's Philox4x32-10 (Salmon et
    al., SC'11) against the closed forms of the published Weyl increments,
    w0 = floor(2^32 (phi - 1)) and w1 = floor(2^32 (sqrt(3) - 1)): ten rounds f with keys
    k, k + w, ..., k + 9w satisfy round_{k+10w}(f(c, k)) == f(round_k(c), k + w). A wrong
    increment, a wrong round count or a key bumped at the wrong place breaks it."""
    w0 = math.isqrt(5 << 62) - (1 << 31)  # 2^31 (sqrt 5 - 1)
    w1 = math.isqrt(3 << 64) - (1 << 32)  # 2^32 (sqrt 3 - 1)
    m32 = 0xFFFFFFFF

    def rnd(c, k):  # one Philox4x32 round (the published multipliers)
        p0 = 0xD2511F53 * int(c[0])
        p1 = 0xCD9E8D57 * int(c[2])
        return [((p1 >> 32) ^ int(c[1]) ^ k[0]) & m32, p1 & m32, ((p0 >> 32) ^ int(c[3]) ^ k[1]) & m32, p0 & m32]

    def bump(k, n):
        return [(k[0] + n * w0) & m32, (k[1] + n * w1) & m32]

    rng = np.random.default_rng(17)
    for _ in range(64):
        c = [int(x) for x in rng.integers(0, 1 << 32, size=4, dtype=np.uint64)]
        k = [int(x) for x in rng.integers(0, 1 << 32, size=2, dtype=np.uint64)]
        lhs = rnd(oracle.philox4x32_10(c, k), bump(k, 10))
        rhs = [int(x) for x in oracle.philox4x32_10(rnd(c, k), bump(k, 1))]
        assert lhs == rhs
        # the identity discriminates: nine increments do not satisfy it
        assert rnd(oracle.philox4x32_10(c, k), bump(k, 9)) != rhs
