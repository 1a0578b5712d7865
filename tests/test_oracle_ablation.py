"""The oracle's regular FCC lattice (the modified lattice without its end contacts, the
reference the paper compares its threshold with in Sec. III), pinned on the CPU: it is
exactly FCC in an independent cubic description, bulk coordination 12, the one-column
fiber has no bonds, the Markov decision equals BFS and union-find, and removing bonds can
only remove spanning paths."""
import itertools
import math

import numpy as np
import pytest

import oracle

_FCC_NN = {v for p in itertools.permutations((1, 1, 0)) for s in itertools.product((1, -1), repeat=3)
           for v in [tuple(a * b for a, b in zip(p, s))]}


def _cubic(q, r, k):
    q = np.asarray(q, np.int64); r = np.asarray(r, np.int64); k = np.asarray(k, np.int64)
    return np.stack([q - r + 2 * k, q + 2 * r + 2 * k, -2 * q - r + 2 * k], axis=1)


@pytest.mark.parametrize("W,L", [(0, 7), (1, 8), (2, 10), (3, 13)])
def test_regular_lattice_is_fcc(W, L):
    lat = oracle.Lattice(W, L, ends=False)
    q, r, k = lat.coords()
    X3 = _cubic(q, r, k)
    assert np.all(X3 % 3 == 0)
    X = X3 // 3
    pos = {tuple(v): i for i, v in enumerate(X)}
    ptr, idx = lat.adjacency()
    for i in range(lat.n):
        expect = set()
        for v in _FCC_NN:
            j = pos.get((X[i, 0] + v[0], X[i, 1] + v[1], X[i, 2] + v[2]))
            if j is not None:
                expect.add(j)
        assert set(idx[ptr[i]:ptr[i + 1]].tolist()) == expect


def test_same_sites_and_surfaces_as_modified():
    a, b = oracle.Lattice(4, 16), oracle.Lattice(4, 16, ends=False)
    assert a.n == b.n
    for x, y in zip(a.coords(), b.coords()):
        np.testing.assert_array_equal(x, y)
    for x, y in zip(a.surfaces(), b.surfaces()):
        np.testing.assert_array_equal(x, y)
    # the modified lattice has exactly the extra end-contact bonds: one per pair of
    # consecutive tubes of a column
    q, r, k = a.coords()
    cols = set(zip(q.tolist(), r.tolist()))
    assert a.n_bonds - b.n_bonds == a.n - len(cols)


def test_bulk_coordination_is_12():
    lat = oracle.Lattice(4, 16, ends=False)
    q, r, k = lat.coords()
    ptr, idx = lat.adjacency()
    deg = np.diff(ptr)
    hexd = np.maximum(np.maximum(np.abs(q), np.abs(r)), np.abs(q + r))
    interior = (hexd <= 2) & (k >= 3) & (k <= 12)
    assert np.all(deg[interior] == 12)
    for i in range(lat.n):
        nb = idx[ptr[i]:ptr[i + 1]]
        assert not np.any((q[nb] == q[i]) & (r[nb] == r[i]))


@pytest.mark.parametrize("L", [1, 2, 3, 4, 7, 16])
def test_single_column_has_no_bonds(L):
    """W = 0 without end contacts: isolated tubes. Every tube is both start and far only
    for L <= 3 (one tube); beyond, nothing percolates."""
    lat = oracle.Lattice(0, L, ends=False)
    n = math.ceil(L / 3)
    full = np.zeros((1, lat.words), np.uint32)
    for s in range(n):
        full[0, s >> 5] |= np.uint32(1 << (s & 31))
    perc, steps, hit = lat.inspect_markov(full)
    if L <= 3:
        assert perc[0] == 1 and steps[0] == 1 and hit[0] == 1.0
    else:
        assert perc[0] == 0


@pytest.mark.parametrize("W,L,p", [(2, 9, 0.4), (4, 16, 0.25), (6, 30, 0.3)])
def test_markov_equals_bfs_and_uf(W, L, p):
    lat = oracle.Lattice(W, L, ends=False)
    bits = lat.sample(p, seed=12, n_cfg=48)
    pm, sm, _ = lat.inspect_markov(bits)
    pb, sb = lat.inspect_bfs(bits)
    np.testing.assert_array_equal(pm, pb)
    np.testing.assert_array_equal(sm, sb)
    np.testing.assert_array_equal(pm, lat.inspect_uf(bits))


@pytest.mark.parametrize("W,L,p", [(3, 20, 0.2), (5, 40, 0.22)])
def test_removing_bonds_only_removes_paths(W, L, p):
    """Same configurations (the sampler does not depend on the bonds): percolating on the
    regular lattice implies percolating on the modified one, with a path at least as
    short."""
    a, b = oracle.Lattice(W, L), oracle.Lattice(W, L, ends=False)
    bits = a.sample(p, seed=3, n_cfg=96)
    np.testing.assert_array_equal(bits, b.sample(p, seed=3, n_cfg=96))
    pa, sa, _ = a.inspect_markov(bits)
    pb, sb, _ = b.inspect_markov(bits)
    assert np.all(pa >= pb)
    both = (pa == 1) & (pb == 1)
    assert np.all(sb[both] >= sa[both])
    assert pa.sum() > pb.sum()  # at these p the end contacts matter
