"""First-passage outputs of the HIP path (through the C ABI) against the oracle, on the GPU.

* perc_first_passage: the backward all-sources form of Eq. 3. Every entry within
  |f32 - f64| <= (6M + 8) 2^-24 f64 + (M + 1) 2^-146: each backward move adds at most
  6 roundings (a 4-level pairwise sum, 1/deg, the product) relative to the value, and the
  2^-149 floor the kernel keeps on words that were once non-zero adds at most 2^-149 per
  move in absolute terms (the map has row sums <= 1).
* perc_steps_hist: bit-exact against the oracle's step counts.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1401_2130_amd import workloads

pytestmark = pytest.mark.gpu

U24 = 2.0 ** -24


@pytest.fixture(scope="module")
def perc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1401_2130_amd as p
    return p


def dev(words: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(words).view(np.int32)).cuda()


def check_fp(f32, f64, M):
    f32 = f32.astype(np.float64)
    tol = (6 * M + 8) * U24 * f64 + (M + 1) * 2.0 ** -146
    bad = np.nonzero(np.abs(f32 - f64) > tol)[0]
    assert bad.size == 0, (M, bad[:5], f32[bad[:5]], f64[bad[:5]])
    if f64.sum() > 0:
        assert np.abs(f32 - f64).sum() / f64.sum() <= (6 * M + 8) * U24


@pytest.mark.parametrize("W,L,p,M", [(0, 7, 1.0, 5), (2, 9, 0.6, 1), (3, 13, 0.5, 7), (4, 16, 0.45, 16),
                                     (5, 60, 0.4, 64), (16, 37, 0.3, 40), (1, 1, 1.0, 1), (1, 2, 0.8, 3),
                                     (7, 100, 0.0, 4)])
def test_first_passage_all_sources(perc, W, L, p, M):
    """Several tiles (W = 16: 817 columns), ragged last cells (L mod 3 != 0), a one-layer
    fiber where every tube is on both surfaces, an empty fiber."""
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L)
    occ = workloads.random_occupancy(ref.n, 1, p, 700 + 13 * W + L + M)
    f64 = ref.first_passage_all(occ[0], M)
    f32 = perc.perc_first_passage(lat, dev(occ[0]), M)
    torch.cuda.synchronize()
    check_fp(f32.cpu().numpy(), f64, M)
    if p == 0.0:
        assert np.all(f32.cpu().numpy() == 0.0)


def test_first_passage_full_size(perc):
    """W = 32, L = 1024 (1,081,686 tubes, 7 column tiles), M = 64, every entry."""
    (W, L) = workloads.LARGE.shapes[0]
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L)
    occ = ref.sample(0.17, 11, 1)
    M = 64
    f64 = ref.first_passage_all(occ[0], M)
    f32 = perc.perc_first_passage(lat, dev(occ[0]), M)
    torch.cuda.synchronize()
    f32 = f32.cpu().numpy()
    assert (f64 > 0).sum() > 1000
    check_fp(f32, f64, M)


@pytest.mark.parametrize("W,L,p,seed", [(3, 24, 0.45, 5), (4, 16, 0.35, 6)])
def test_mean_over_sources_is_forward_hit(perc, W, L, p, seed):
    """Mean of the backward vector over the metallic start tubes at M = m* equals the
    first-hit probability the forward inspection returns (both on the device)."""
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L)
    start, _ = ref.surfaces()
    occ = ref.sample(p, seed, 16)
    pg, sg, hg = perc.perc_inspect_ex(lat, dev(occ), 16, hit=True)
    pg, sg, hg = pg.cpu().numpy(), sg.cpu().numpy(), hg.cpu().numpy()
    checked = 0
    for c in np.nonzero(pg)[0]:
        m = int(sg[c])
        bits = np.unpackbits(occ[c].view(np.uint8), bitorder="little")[: ref.n].astype(bool)
        s0 = start & bits
        f = perc.perc_first_passage(lat, dev(occ[c]), m).cpu().numpy().astype(np.float64)
        mean = f[s0].sum() / s0.sum()
        assert abs(mean - hg[c]) <= (12 * m + 40) * U24 * hg[c] + 2.0 ** -120, (c, m, mean, hg[c])
        checked += 1
    assert checked > 0


def test_first_passage_rejects_bad_arguments(perc):
    lat = perc.Lattice(2, 6)
    occ = torch.zeros(lat.words, dtype=torch.int32, device="cuda")
    with pytest.raises(perc.PercError):
        perc.perc_first_passage(lat, occ, 0)


@pytest.mark.parametrize("W,L,p,n,nbins", [(4, 16, 0.3, 512, 64), (3, 40, 0.5, 256, 20), (2, 5, 0.0, 8, 4)])
def test_steps_hist_bit_exact(perc, W, L, p, n, nbins):
    """m* histogram of the percolating configurations, last bin open."""
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L)
    occ = ref.sample(p, 21, n)
    pm, sm, _ = ref.inspect_markov(occ)
    pg, sg = perc.perc_inspect(lat, dev(occ), n)
    hist = perc.perc_steps_hist(pg, sg, nbins)
    torch.cuda.synchronize()
    want = np.zeros(nbins, np.int64)
    for i in np.nonzero(pm)[0]:
        want[min(int(sm[i]), nbins - 1)] += 1
    np.testing.assert_array_equal(hist.cpu().numpy(), want)


@pytest.mark.parametrize("W,L,p,M,n", [(3, 13, 0.5, 7, 5), (16, 37, 0.3, 12, 3), (2, 9, 0.6, 1, 4)])
def test_first_passage_batch(perc, W, L, p, M, n):
    """Several configurations in one call: each equals the oracle within the bound and the
    one-configuration call bit for bit."""
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L)
    occ = workloads.random_occupancy(ref.n, n, p, 900 + W + L)
    fb = perc.perc_first_passage_batch(lat, dev(occ), M).cpu().numpy()
    for i in range(n):
        check_fp(fb[i], ref.first_passage_all(occ[i], M), M)
        f1 = perc.perc_first_passage(lat, dev(occ[i]), M).cpu().numpy()
        np.testing.assert_array_equal(f1.view(np.uint32), fb[i].view(np.uint32))
