"""Parity of the HIP path (through the C ABI) with the CPU oracle, on the GPU.

Bar: percolation bits, step counts and Pi counts bit-exact; the sampler bit-exact;
FP32 probabilities within the tolerance derived from the arithmetic:
  * state after K steps: relative 1e-5 (elementwise on entries >= 2^-100, and in L1)
    for K <= 16, the rounding bound (6K + 8) 2^-24 being below it;
  * first-hit probability after m* steps: relative (6 m* + 24) 2^-24.
"""
import math

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


def host_words(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def check_hit(hit_gpu, hit_ref, perc_ref, steps_ref):
    for i in np.nonzero(perc_ref)[0]:
        ref = hit_ref[i]
        if ref < 2.0 ** -100:
            continue
        tol = (6 * steps_ref[i] + 24) * U24
        assert abs(hit_gpu[i] - ref) <= tol * ref, (i, hit_gpu[i], ref, steps_ref[i])
    assert np.all(hit_gpu[perc_ref == 0] == 0.0)


# (form, cells per work item); the library rounds up to a multiple of 8
FORMS = [("plain", 8), ("span", 8), ("span", 5), ("span", 24), ("persist", 8), ("persist", 16), ("persist", 64),
         ("span2", 8), ("span2", 24), ("span2", 64), ("persist2", 8), ("persist2", 64)]


# --------------------------------------------------------------------------------
# sampler
# --------------------------------------------------------------------------------

@pytest.mark.parametrize("W,L,p,seed,cfg0,n", [(4, 16, 0.1533, 1, 0, 64), (3, 10, 0.5, 7, 1000, 16),
                                               (16, 256, 0.17, 3, 4090, 6), (5, 11, 0.0, 2, 0, 3),
                                               (5, 11, 1.0, 2, 0, 3), (2, 7, 0.125, 2 ** 40 + 5, 2 ** 33, 4)])
def test_sampler_bit_exact(perc, W, L, p, seed, cfg0, n):
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L).sample(p, seed, n, cfg0=cfg0)
    got = perc.perc_sample(lat, p, seed, n, cfg0=cfg0)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host_words(got), ref)


@pytest.mark.parametrize("W,L,p,seed,cfg0,n", [(4, 16, 0.1533, 1, 0, 16), (0, 7, 0.5, 3, 2, 8), (2, 9, 0.0, 1, 0, 3),
                                               (2, 9, 1.0, 1, 0, 3), (16, 256, 0.15, 3, 100, 3),
                                               (3, 13, 0.3, 2 ** 40 + 1, 2 ** 33, 4), (32, 64, 0.17, 9, 0, 2)])
def test_fixed_count_sampler_bit_exact(perc, W, L, p, seed, cfg0, n):
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L).sample_fixed(p, seed, n, cfg0=cfg0)
    got = perc.perc_sample_fixed(lat, p, seed, n, cfg0=cfg0)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host_words(got), ref)


def test_fixed_count_ensemble_inspection(perc):
    """Configurations of the fixed-count ensemble inspected on the GPU: bits and steps of
    the oracle on the same configurations."""
    W, L, p, n = 5, 30, 0.3, 64
    lat, ref = perc.Lattice(W, L), oracle.Lattice(W, L)
    occ = perc.perc_sample_fixed(lat, p, 17, n)
    pg, sg = perc.perc_inspect(lat, occ)
    torch.cuda.synchronize()
    pm, sm, _ = ref.inspect_markov(ref.sample_fixed(p, 17, n))
    np.testing.assert_array_equal(pg.cpu().numpy(), pm)
    np.testing.assert_array_equal(sg.cpu().numpy(), sm)


# --------------------------------------------------------------------------------
# inspection: every form and item length against the oracle
# --------------------------------------------------------------------------------

SHAPES = [(0, 1), (0, 2), (0, 3), (0, 10), (1, 4), (1, 5), (2, 6), (2, 13), (3, 9), (4, 16), (4, 17), (5, 30),
          (7, 44), (8, 61)]


@pytest.mark.parametrize("W,L", SHAPES)
@pytest.mark.parametrize("form,depth", FORMS)
def test_inspect_matches_oracle(perc, W, L, form, depth):
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L)
    rows = []
    for p, seed in ((0.15, 1), (0.3, 2), (0.6, 3), (0.95, 4)):
        rows.append(workloads.random_occupancy(ref.n, 24, p, seed + 100 * W + L, pad_garbage=(seed == 2)))
    occ = np.concatenate(rows)
    pm, sm, hm = ref.inspect_markov(occ)
    pb, sb = ref.inspect_bfs(occ)
    assert np.array_equal(pm, pb) and np.array_equal(sm, sb)
    d_occ = dev(occ)
    pg, sg, hg = perc.perc_inspect_ex(lat, d_occ, hit=True, form=form, depth=depth)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(pg.cpu().numpy(), pm)
    np.testing.assert_array_equal(sg.cpu().numpy(), sm)
    check_hit(hg.cpu().numpy().astype(np.float64), hm, pm, sm)


def test_forms_agree_bitwise(perc):
    """Each configuration's bits, steps and FP32 first-hit probability are the same
    alone (plain), spread (span) and one-per-workgroup (persist), at every item length."""
    W, L = 6, 40
    lat = perc.Lattice(W, L)
    occ = workloads.random_occupancy(lat.n, 200, 0.32, 77)
    d_occ = dev(occ)
    results = []
    for form, depth in FORMS:
        p, s, h = perc.perc_inspect_ex(lat, d_occ, hit=True, form=form, depth=depth)
        results.append((p.cpu().numpy(), s.cpu().numpy(), h.cpu().numpy().view(np.uint32)))
    for r in results[1:]:
        for a, b in zip(results[0], r):
            np.testing.assert_array_equal(a, b)
    # a configuration inspected alone equals the same one inside the batch
    for i in (0, 57, 199):
        p1, s1, h1 = perc.perc_inspect_ex(lat, d_occ[i:i + 1].contiguous(), hit=True, form="span")
        assert p1.item() == results[0][0][i] and s1.item() == results[0][1][i]
        assert h1.cpu().numpy().view(np.uint32)[0] == results[0][2][i]


def test_graph_path_on_a_side_stream(perc):
    """A non-default stream lets the span form capture and replay a HIP graph."""
    W, L = 5, 60
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L)
    occ = workloads.random_occupancy(ref.n, 300, 0.35, 5)
    pm, sm, _ = ref.inspect_markov(occ)
    d_occ = dev(occ)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for gs in (1, 3, 8, 32):
            pg, sg, _ = perc.perc_inspect_ex(lat, d_occ, form="span", depth=8, graph_steps=gs, stream=s)
            s.synchronize()
            np.testing.assert_array_equal(pg.cpu().numpy(), pm)
            np.testing.assert_array_equal(sg.cpu().numpy(), sm)


def test_edge_cases(perc):
    W, L = 3, 11
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L)
    n, words = ref.n, ref.words
    start, far = ref.surfaces()
    q, r, k = ref.coords()
    cases = []
    cases.append(np.zeros(n, bool))                    # all insulating: no start tube
    cases.append(np.ones(n, bool))                     # all metallic: percolates in one path
    iso = np.zeros(n, bool); iso[np.nonzero(start)[0][5]] = True
    cases.append(iso)                                  # one isolated start tube: degree 0 self-loop
    col = np.zeros(n, bool); col[(q == 0) & (r == 0)] = True
    cases.append(col)                                  # the central column only: end contacts
    only_far = far.copy()
    cases.append(only_far)                             # far surface only: never starts
    occ = np.stack([np.packbits(np.pad(c, (0, words * 32 - n)).astype(np.uint8), bitorder="little").view(np.uint32)
                    for c in cases])
    pm, sm, hm = ref.inspect_markov(occ)
    assert list(pm) == [0, 1, 0, 1, 0]
    for form in ("plain", "span", "persist", "persist2"):
        pg, sg, hg = perc.perc_inspect_ex(lat, dev(occ), hit=True, form=form)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(pg.cpu().numpy(), pm)
        np.testing.assert_array_equal(sg.cpu().numpy(), sm)
        check_hit(hg.cpu().numpy().astype(np.float64), hm, pm, sm)
    # empty batch
    e = torch.empty((0, words), dtype=torch.int32, device="cuda")
    pg, sg = perc.perc_inspect(lat, e, 0)
    assert pg.numel() == 0


# --------------------------------------------------------------------------------
# state after K steps (the FP32 probabilities themselves)
# --------------------------------------------------------------------------------

@pytest.mark.parametrize("W,L,p,K", [(3, 13, 0.5, 0), (3, 13, 0.5, 1), (4, 16, 0.35, 16), (6, 31, 0.3, 16),
                                     (2, 8, 0.9, 16), (8, 50, 0.25, 16)])
def test_state_after_within_1e5(perc, W, L, p, K):
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L)
    occ = workloads.random_occupancy(ref.n, 1, p, 1000 + K + W)
    x64, r64 = ref.state_after(occ, K)
    x32, r32 = perc.perc_state_after(lat, dev(occ[0]), K)
    torch.cuda.synchronize()
    x32 = x32.cpu().numpy().astype(np.float64)
    r32 = r32.cpu().numpy().astype(bool)
    np.testing.assert_array_equal(r32, r64)
    big = x64 >= 2.0 ** -100
    np.testing.assert_allclose(x32[big], x64[big], rtol=1e-5, atol=0)
    if x64.sum() > 0:
        assert np.abs(x32 - x64).sum() / np.abs(x64).sum() <= 1e-5
    assert np.all(x32[~r64] == 0)


@pytest.mark.parametrize("W,L,p,seed", [(5, 60, 0.4, 9), (6, 120, 0.5, 7)])
@pytest.mark.parametrize("K", [64, 256])
def test_state_after_long_runs_within_1e5(perc, W, L, p, seed, K):
    """The FP32 state stays within 1e-5 of FP64, elementwise and in L1, up to K = 256.
    Each step adds at most a few roundings per tube (a sum of at most 14 terms, one
    product), measured at about 0.35 ulp per step: 5.8e-6 at K = 256 on these shapes."""
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L)
    occ = workloads.random_occupancy(ref.n, 1, p, seed)
    x64, r64 = ref.state_after(occ, K)
    x32, r32 = perc.perc_state_after(lat, dev(occ[0]), K)
    torch.cuda.synchronize()
    x32 = x32.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(r32.cpu().numpy().astype(bool), r64)
    big = x64 >= 2.0 ** -100
    rel = np.abs(x32[big] - x64[big]) / x64[big]
    print(f"K={K}: max elementwise relative error {rel.max():.3e}")
    assert rel.max() <= 1e-5
    assert np.abs(x32 - x64).sum() / np.abs(x64).sum() <= 1e-5


def test_state_after_1024_steps_within_derived_bound(perc):
    """Past K of about 500 the elementwise error passes 1e-5 (2.2e-5 at K = 1024); the
    bound is then the derived (6K + 8) 2^-24, and the reached set stays exact."""
    W, L, K = 6, 120, 1024
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L)
    occ = workloads.random_occupancy(ref.n, 1, 0.5, 7)
    x64, r64 = ref.state_after(occ, K)
    x32, r32 = perc.perc_state_after(lat, dev(occ[0]), K)
    torch.cuda.synchronize()
    x32 = x32.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(r32.cpu().numpy().astype(bool), r64)
    big = x64 >= 2.0 ** -100
    rel = np.abs(x32[big] - x64[big]) / x64[big]
    print(f"K={K}: max elementwise relative error {rel.max():.3e}, bound {(6 * K + 8) * U24:.3e}")
    assert rel.max() <= (6 * K + 8) * U24


# --------------------------------------------------------------------------------
# Pi(p) through perc_pi (sampling on the device) at the workload sizes
# --------------------------------------------------------------------------------

@pytest.mark.parametrize("form", ["span", "persist", "plain"])
def test_pi_small_workload_full(perc, form):
    """W=4, L=16, p=0.1533, seed 1, 1000 configurations: every bit and the count."""
    wl = workloads.SMALL
    (W, L), p, seed, n = wl.shapes[0], wl.ps[0], wl.seed, wl.n_cfg
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L)
    occ = ref.sample(p, seed, n)
    pm, sm, hm = ref.inspect_markov(occ)
    bits = torch.empty(n, dtype=torch.uint8, device="cuda")
    steps = torch.empty(n, dtype=torch.int32, device="cuda")
    hit = torch.empty(n, dtype=torch.float32, device="cuda")
    n_perc, pi = perc.perc_pi_ex(lat, p, n, seed, bits=bits, steps=steps, hit=hit, form=form)
    np.testing.assert_array_equal(bits.cpu().numpy(), pm)
    np.testing.assert_array_equal(steps.cpu().numpy(), sm)
    check_hit(hit.cpu().numpy().astype(np.float64), hm, pm, sm)
    assert n_perc == int(pm.sum()) and pi == pm.sum() / n


def test_pi_large_workload_sampled(perc):
    """W=32, L=1024 at p in {0.14, 0.1533, 0.17}, 256 configurations each, in the span
    launch configuration the benchmark times; every tenth configuration checked
    against the oracle (BFS for bits and steps, the Markov iteration for two)."""
    wl = workloads.LARGE
    (W, L), seed, n = wl.shapes[0], wl.seed, wl.n_cfg
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L)
    for p in wl.ps:
        print(f"large workload p={p}", flush=True)
        bits = torch.empty(n, dtype=torch.uint8, device="cuda")
        steps = torch.empty(n, dtype=torch.int32, device="cuda")
        n_perc, _ = perc.perc_pi_ex(lat, p, n, seed, bits=bits, steps=steps, form="span")
        b = bits.cpu().numpy(); s = steps.cpu().numpy()
        assert n_perc == int(b.sum())
        idx = np.arange(0, n, 10)
        for i in idx:
            occ = ref.sample(p, seed, 1, cfg0=int(i))
            pb, sb = ref.inspect_bfs(occ)
            assert (b[i], s[i]) == (pb[0], sb[0]), (p, i)
        for i in idx[:2]:
            occ = ref.sample(p, seed, 1, cfg0=int(i))
            pm, sm, _ = ref.inspect_markov(occ)
            assert (b[i], s[i]) == (pm[0], sm[0]), (p, i)


def test_pi_batched_workload_sampled(perc):
    """W=16, L=256, 4096 configurations at three of the 21 p values, in the persistent
    form (one launch); a sample checked against the oracle, and common random numbers
    make the bits monotone in p."""
    wl = workloads.BATCH
    (W, L), seed, n = wl.shapes[0], wl.seed, wl.n_cfg
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L)
    prev = None
    for p in (wl.ps[0], wl.ps[10], wl.ps[20]):
        print(f"batched workload p={p}", flush=True)
        bits = torch.empty(n, dtype=torch.uint8, device="cuda")
        steps = torch.empty(n, dtype=torch.int32, device="cuda")
        n_perc, _ = perc.perc_pi_ex(lat, p, n, seed, bits=bits, steps=steps, form="persist")
        b = bits.cpu().numpy(); s = steps.cpu().numpy()
        idx = np.arange(0, n, 64)
        occ = np.concatenate([ref.sample(p, seed, 1, cfg0=int(i)) for i in idx])
        pb, sb = ref.inspect_bfs(occ)
        np.testing.assert_array_equal(b[idx], pb)
        np.testing.assert_array_equal(s[idx], sb)
        if prev is not None:
            assert np.all(prev <= b)
        prev = b


# --------------------------------------------------------------------------------
# uneven batches: several lattice shapes in one launch
# --------------------------------------------------------------------------------

@pytest.mark.parametrize("form,depth", [("span", 8), ("span", 16), ("persist", 8), ("plain", 8), ("persist2", 16)])
def test_batch_of_mixed_shapes(perc, form, depth):
    shapes = [(2, 9), (5, 22), (3, 40), (8, 17), (0, 12), (11, 33)]
    lats = {s: perc.Lattice(*s) for s in shapes}
    refs = {s: oracle.Lattice(*s) for s in shapes}
    rng = np.random.default_rng(4)
    jobs, expect = [], []
    n_groups = len(shapes) * 2
    counts = np.zeros(n_groups, np.int64)
    keep = []
    for gi, s in enumerate(shapes):
        for pi, p in enumerate((0.2, 0.45)):
            grp = 2 * gi + pi
            for cfg in range(6):
                if rng.random() < 0.5:
                    occ = refs[s].sample(p, 31, 1, cfg0=cfg)
                    jobs.append((lats[s], p, 31, cfg, grp))
                else:
                    occ = workloads.random_occupancy(refs[s].n, 1, p, 1000 * gi + 10 * pi + cfg)
                    t = dev(occ[0])
                    keep.append(t)
                    jobs.append((lats[s], t, grp))
                pm, sm, hm = refs[s].inspect_markov(occ)
                expect.append((pm[0], sm[0], hm[0]))
                counts[grp] += pm[0]
    order = rng.permutation(len(jobs))  # shapes interleaved in the batch
    jobs = [jobs[i] for i in order]
    expect = [expect[i] for i in order]
    pg, sg, hg, cnt = perc.perc_batch(jobs, n_groups=n_groups, hit=True, form=form, depth=depth)
    torch.cuda.synchronize()
    pm = np.array([e[0] for e in expect]); sm = np.array([e[1] for e in expect]); hm = np.array([e[2] for e in expect])
    np.testing.assert_array_equal(pg.cpu().numpy(), pm)
    np.testing.assert_array_equal(sg.cpu().numpy(), sm)
    check_hit(hg.cpu().numpy().astype(np.float64), hm, pm, sm)
    assert cnt == counts.tolist()


def test_batch_matches_single_shape_calls_bitwise(perc):
    a, b = perc.Lattice(6, 30), perc.Lattice(9, 21)
    jobs = [(a, 0.3, 5, i, 0) for i in range(40)] + [(b, 0.35, 6, i, 1) for i in range(40)]
    rng = np.random.default_rng(0)
    order = rng.permutation(len(jobs))
    mixed = [jobs[i] for i in order]
    pg, sg, hg, cnt = perc.perc_batch(mixed, n_groups=2, hit=True, form="span")
    for lat, p, seed, grp in ((a, 0.3, 5, 0), (b, 0.35, 6, 1)):
        bits = torch.empty(40, dtype=torch.uint8, device="cuda")
        steps = torch.empty(40, dtype=torch.int32, device="cuda")
        hit = torch.empty(40, dtype=torch.float32, device="cuda")
        n_perc, _ = perc.perc_pi_ex(lat, p, 40, seed, bits=bits, steps=steps, hit=hit, form="persist")
        assert n_perc == cnt[grp]
        sel = [k for k, i in enumerate(order) if jobs[i][0] is lat]
        cfgs = [mixed[k][3] for k in sel]
        np.testing.assert_array_equal(pg.cpu().numpy()[sel], bits.cpu().numpy()[cfgs])
        np.testing.assert_array_equal(sg.cpu().numpy()[sel], steps.cpu().numpy()[cfgs])
        np.testing.assert_array_equal(hg.cpu().numpy().view(np.uint32)[sel], hit.cpu().numpy().view(np.uint32)[cfgs])


def test_wide_fiber_many_tiles(perc):
    """W=40 (4921 columns, ten column tiles with halos): every form against the oracle."""
    W, L = 40, 20
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L)
    occ = np.concatenate([workloads.random_occupancy(ref.n, 8, p, 50 + i) for i, p in enumerate((0.12, 0.2, 0.35))])
    pm, sm, hm = ref.inspect_markov(occ)
    for form, depth in (("span", 8), ("span", 40), ("persist", 16), ("plain", 8)):
        pg, sg, hg = perc.perc_inspect_ex(lat, dev(occ), hit=True, form=form, depth=depth)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(pg.cpu().numpy(), pm)
        np.testing.assert_array_equal(sg.cpu().numpy(), sm)
        check_hit(hg.cpu().numpy().astype(np.float64), hm, pm, sm)
    x64, r64 = ref.state_after(occ[5:6], 12)
    x32, r32 = perc.perc_state_after(lat, dev(occ[5]), 12)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(r32.cpu().numpy().astype(bool), r64)
    big = x64 >= 2.0 ** -100
    np.testing.assert_allclose(x32.cpu().numpy().astype(np.float64)[big], x64[big], rtol=1e-5, atol=0)


def test_fixed_count_curve_and_binomial_convolution(perc):
    """Pi_k of the fixed-count ensemble on the GPU at every k of a 21-tube fiber (W=1,
    L=9): counts equal the oracle's on the same configurations, agree with the exact
    a_k / C(N, k) of the exhaustive enumeration within 5 sigma, and their binomial
    convolution matches the exact Bernoulli Pi(p)."""
    from math import comb
    from paper_1401_2130_amd import fss
    W, L, n, seed = 1, 9, 1024, 8
    ref = oracle.Lattice(W, L)
    N = ref.n
    ks = list(range(N + 1))
    counts = fss.pi_fixed_counts(W, L, ks, n, seed)
    torch.cuda.synchronize()
    a = ref.exhaustive()
    exact = np.array([a[k] / comb(N, k) for k in ks])
    for k in ks:
        pm, _, _ = ref.inspect_markov(ref.sample_fixed(k / N, seed, n))
        assert counts[k] == int(pm.sum()), k
        sig = math.sqrt(max(exact[k] * (1 - exact[k]), 1.0 / n) / n)
        assert abs(counts[k] / n - exact[k]) <= 5 * sig, (k, counts[k] / n, exact[k])
    ps = [0.2, 0.4, 0.6]
    got, miss = fss.binomial_convolution(ks, counts / n, N, ps)
    want = np.array([oracle.pi_from_counts(a, p) for p in ps])
    assert np.all(miss < 1e-12)
    assert np.all(np.abs(got - want) <= 5 / math.sqrt(n))


@pytest.mark.parametrize("p", [0.14, 0.1533, 0.17])
def test_two_step_form_bitwise_at_full_size(perc, p):
    """W=32, L=1024 (7 column tiles): the two-step form gives the bits, steps and FP32
    first-hit probabilities of the one-step span form, configuration by configuration,
    and the oracle's bits and steps on a sample."""
    W, L = workloads.LARGE.shapes[0]
    lat = perc.Lattice(W, L)
    n = 48
    occ = perc.perc_sample(lat, p, 21, n)
    p1, s1, h1 = perc.perc_inspect_ex(lat, occ, n, hit=True, form="span", depth=64)
    p2, s2, h2 = perc.perc_inspect_ex(lat, occ, n, hit=True, form="span2", depth=64)
    p3, s3, h3 = perc.perc_inspect_ex(lat, occ, n, hit=True, form="span2", depth=128)
    torch.cuda.synchronize()
    for a, b in ((p1, p2), (s1, s2), (p1, p3), (s1, s3)):
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    np.testing.assert_array_equal(h1.cpu().numpy().view(np.uint32), h2.cpu().numpy().view(np.uint32))
    np.testing.assert_array_equal(h1.cpu().numpy().view(np.uint32), h3.cpu().numpy().view(np.uint32))
    ref = oracle.Lattice(W, L)
    pick = [0, 17, 40]
    pm, sm, _ = ref.inspect_markov(host_words(occ)[pick])
    np.testing.assert_array_equal(p2.cpu().numpy()[pick], pm)
    np.testing.assert_array_equal(s2.cpu().numpy()[pick], sm)


@pytest.mark.parametrize("form", ["span", "plain"])
def test_largest_serving_fiber(perc, form):
    """W=64, L=4096 (17,040,724 tubes, the largest fiber of the serving mix): bits and
    steps of Philox configurations on both sides of its threshold against the oracle's
    breadth-first search (steps = shortest path + 1, pinned equal to the Markov count)."""
    W, L = 64, 4096
    lat = perc.Lattice(W, L)
    ref = oracle.Lattice(W, L)
    for p in (0.16, 0.17):
        occ = perc.perc_sample(lat, p, 5, 2)
        pg, sg, _ = perc.perc_inspect_ex(lat, occ, 2, form=form)
        torch.cuda.synchronize()
        pb, sb = ref.inspect_bfs(host_words(occ))
        np.testing.assert_array_equal(pg.cpu().numpy(), pb)
        np.testing.assert_array_equal(sg.cpu().numpy(), sb)


def test_two_step_persistent_form_limits(perc):
    """PERC_FORM_PERSIST2 holds the whole cross-section in one workgroup: W = 17 (919
    columns) runs and equals the one-step persistent form bitwise; W = 18 (1027 columns)
    is refused with PERC_EINVAL before any work."""
    lat = perc.Lattice(17, 60)
    occ = perc.perc_sample(lat, 0.2, 13, 64)
    a = perc.perc_inspect_ex(lat, occ, hit=True, form="persist")
    b = perc.perc_inspect_ex(lat, occ, hit=True, form="persist2")
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert np.array_equal(x.cpu().numpy().view(np.uint8), y.cpu().numpy().view(np.uint8))
    wide = perc.Lattice(18, 30)
    occw = perc.perc_sample(wide, 0.2, 13, 4)
    with pytest.raises(perc.PercError) as e:
        perc.perc_inspect_ex(wide, occw, form="persist2")
    assert e.value.code == perc.PERC_EINVAL


@pytest.mark.parametrize("form,depth,graph_steps", [("span", 8, 1), ("span", 80, 8), ("span", 16, 64),
                                                    ("span2", 64, 3)])
def test_lazy_initialisation_long_fibers(perc, form, depth, graph_steps):
    """The span forms compute the degree codes of a configuration's cells as its front
    approaches them (an extension launch at the start of every run of graph_steps
    plans). On thin fibers of about 1,000 cells whose percolating walks cross many
    extensions, with runs from 1 to 64 plans and several item depths: bits and steps
    equal the oracle's breadth-first search, and bits, steps and FP32 first-hit
    probabilities equal the persistent form's (which initialises every cell at once)."""
    for W, L, p, seed in ((3, 3000, 0.55, 41), (2, 3001, 0.7, 42), (5, 2999, 0.4, 43)):
        lat = perc.Lattice(W, L)
        ref = oracle.Lattice(W, L)
        n = 48
        occ = perc.perc_sample(lat, p, seed, n)
        pg, sg, hg = perc.perc_inspect_ex(lat, occ, n, hit=True, form=form, depth=depth, graph_steps=graph_steps)
        pp, sp, hp = perc.perc_inspect_ex(lat, occ, n, hit=True, form="persist")
        torch.cuda.synchronize()
        pb, sb = ref.inspect_bfs(host_words(occ))
        np.testing.assert_array_equal(pg.cpu().numpy(), pb)
        np.testing.assert_array_equal(sg.cpu().numpy(), sb)
        np.testing.assert_array_equal(pg.cpu().numpy(), pp.cpu().numpy())
        np.testing.assert_array_equal(sg.cpu().numpy(), sp.cpu().numpy())
        np.testing.assert_array_equal(hg.cpu().numpy().view(np.uint32), hp.cpu().numpy().view(np.uint32))
        assert pb.sum() > 0 and sb.max() > 300  # some walks run past several extensions
