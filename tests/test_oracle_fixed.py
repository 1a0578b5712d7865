"""The oracle's fixed-count ensemble (Sec. II.A: Np of the N tubes chosen metallic with
uniform probability), pinned on the CPU: the count is exact, the chosen set is the K
smallest keys (recomputed here from the Philox words and a plain numpy sort), every
tube and every pair is chosen with the hypergeometric frequency, and the percolation
frequency at fixed k matches the exact a_k / C(N, k) of the exhaustive enumeration."""
import math

import numpy as np
import pytest

import oracle


def popcounts(bits):
    return np.unpackbits(bits.view(np.uint8), axis=1).sum(axis=1)


def site_mask(bits, n):
    return np.unpackbits(bits.view(np.uint8), axis=1, bitorder="little")[:, :n].astype(bool)


@pytest.mark.parametrize("W,L,p", [(0, 7, 0.5), (1, 5, 0.25), (2, 9, 0.3), (3, 13, 0.1533), (4, 16, 0.0),
                                   (4, 16, 1.0), (2, 6, 0.5)])
def test_exact_count(W, L, p):
    lat = oracle.Lattice(W, L)
    bits = lat.sample_fixed(p, 11, 20, cfg0=5)
    K = math.floor(lat.n * p + 0.5)
    assert np.all(popcounts(bits) == K)
    if lat.words * 32 > lat.n:  # no bit beyond the last tube
        assert not site_mask(np.ascontiguousarray(bits), lat.words * 32)[:, lat.n:].any()


def test_chosen_set_is_k_smallest_keys():
    lat = oracle.Lattice(2, 10)
    seed, cfg, p = 0x1234_5678_9ABC, 3, 0.35
    n = lat.n
    tag = ((2 << 16) | 10) | 0x80000000
    keys = np.zeros(n, dtype=np.uint64)
    for s in range(n):
        out = oracle.philox4x32_10([s >> 1, cfg, 0, tag], [seed & 0xFFFFFFFF, seed >> 32])
        w = 2 * (s & 1)
        keys[s] = (int(out[w]) << 32) | int(out[w + 1])
    K = math.floor(n * p + 0.5)
    order = np.lexsort((np.arange(n), keys))  # by key, then by index
    expect = np.zeros(n, bool)
    expect[order[:K]] = True
    got = site_mask(lat.sample_fixed(p, seed, 1, cfg0=cfg), n)[0]
    np.testing.assert_array_equal(got, expect)


def test_uniform_inclusion_and_pairs():
    lat = oracle.Lattice(1, 6)  # 14 tubes
    n, p, reps = lat.n, 0.3, 20000
    K = math.floor(n * p + 0.5)
    m = site_mask(lat.sample_fixed(p, 99, reps), n)
    freq = m.mean(axis=0)
    # each tube: hypergeometric inclusion probability K / N, binomial sampling error
    sd = math.sqrt((K / n) * (1 - K / n) / reps)
    assert np.all(np.abs(freq - K / n) < 5 * sd), (freq, K / n)
    pair = (m[:, 0] & m[:, 7]).mean()
    q = K * (K - 1) / (n * (n - 1))
    assert abs(pair - q) < 5 * math.sqrt(q * (1 - q) / reps)


def test_fixed_k_percolation_matches_exhaustive():
    """Pi at exactly k metallic tubes is a_k / C(N, k) (exhaustive enumeration); the
    fixed-count ensemble estimates it without bias."""
    lat = oracle.Lattice(1, 4)  # 8 tubes
    n = lat.n
    a = lat.exhaustive()
    reps = 6000
    for k in (2, 3, 4, 5):
        p = k / n
        bits = lat.sample_fixed(p, 7, reps)
        assert np.all(popcounts(bits) == k)
        perc, _, _ = lat.inspect_markov(bits)
        exact = a[k] / math.comb(n, k)
        sd = math.sqrt(max(exact * (1 - exact), 1e-12) / reps)
        assert abs(perc.mean() - exact) < 5 * sd + 1e-9, (k, perc.mean(), exact)
