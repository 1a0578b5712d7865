"""Autotuner and sweep driver on the GPU: the tuned settings are valid, the automatic
form picks them up without changing any result (bits, steps, FP32 hit), and a mixed
Pi table from one batch equals the per-shape Pi counts of perc_pi_ex."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def perc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1401_2130_amd as p
    return p


def test_autotune_then_auto_form_is_bitwise_unchanged(perc):
    lat = perc.Lattice(6, 40)
    best = perc.perc_autotune([(lat, 0.3, 9, c) for c in range(64)], n_target=300)
    assert best["form"] in ("span", "persist", "span2")
    assert best["depth"] % 16 == 0 and 64 <= best["block"] <= 1024 and best["ms"] > 0
    jobs = [(lat, 0.3, 9, c) for c in range(300)]
    pa, sa, ha, _ = perc.perc_batch(jobs, hit=True, form="auto")
    pb, sb, hb, _ = perc.perc_batch(jobs, hit=True, form="span", depth=64)
    pc, sc, hc, _ = perc.perc_batch(jobs, hit=True, **{k: best[k] for k in ("form", "depth", "block", "graph_steps")})
    torch.cuda.synchronize()
    for x, y in ((pa, pb), (sa, sb), (pa, pc), (sa, sc)):
        assert torch.equal(x, y)
    for x, y in ((ha, hb), (ha, hc)):
        assert torch.equal(x.view(torch.int32), y.view(torch.int32))


def test_autotune_mixed_shapes(perc):
    shapes = [perc.Lattice(3, 20), perc.Lattice(9, 30)]
    best = perc.perc_autotune([(shapes[c % 2], 0.35, 2, c) for c in range(40)])
    assert best["form"] in ("span", "persist", "span2")
    with pytest.raises(perc.PercError):
        perc.perc_autotune([])


def test_mixed_form_equals_span(perc):
    """The mixed form (short-walk fibers in the persistent form, the others in the span
    form beside it, outputs scattered back to the jobs' places) and the automatic form,
    which picks it for this batch, give every bit, step count and FP32 first-hit
    probability of the span form and the same group counts; the long-walk fibers' bits
    equal the oracle's breadth-first search."""
    import oracle
    # 1 tile x 6 cells; 2,107 columns = 5 tiles x 134 cells (above 600: the span part)
    narrow, wide = perc.Lattice(8, 16), perc.Lattice(26, 400)
    jobs = np.concatenate([perc.philox_jobs(narrow, 0.25, 5, 2100, group=0),
                           perc.philox_jobs(wide, 0.17, 6, 40, group=1),
                           perc.philox_jobs(narrow, 0.3, 7, 100, group=2)])
    jobs = jobs[np.random.default_rng(1).permutation(len(jobs))]  # the two kinds interleaved
    outs = {f: perc.perc_batch(jobs, n_groups=3, hit=True, form=f) for f in ("span", "mixed", "auto")}
    torch.cuda.synchronize()
    p0, s0, h0, c0 = outs["span"]
    for f in ("mixed", "auto"):
        p1, s1, h1, c1 = outs[f]
        assert torch.equal(p0, p1) and torch.equal(s0, s1), f
        assert torch.equal(h0.view(torch.int32), h1.view(torch.int32)), f
        assert list(c0) == list(c1), f
    # profiled, the two parts run one after the other; the persistent launches are
    # counted apart from the span form's step launches (for the automatic form too, which
    # shows that it took the mixed form: a persistent launch and span steps)
    for f in ("mixed", "auto"):
        perc.perc_profile_enable(True)
        try:
            p2, s2, h2, c2 = perc.perc_batch(jobs, n_groups=3, hit=True, form=f)
            torch.cuda.synchronize()
            prof = perc.perc_profile_read()
        finally:
            perc.perc_profile_enable(False)
        assert torch.equal(p0, p2) and torch.equal(s0, s2) and list(c0) == list(c2), f
        assert 1 <= prof["persist_launches"] < prof["step_launches"], f
        assert 0.0 < prof["persist_ms"] < prof["step_ms"], f
        assert 0 < prof["persist_tube_steps"] < prof["tube_steps"], f
    sel = np.nonzero(jobs["group"] == 1)[0]
    sel = sel[np.argsort(jobs["cfg"][sel])]
    ref = oracle.Lattice(26, 400)
    pb, _ = ref.inspect_bfs(ref.sample(0.17, 6, 40))
    np.testing.assert_array_equal(p0.cpu().numpy()[sel], pb)
    assert c0[1] == int(pb.sum())


def test_pi_table_matches_pi_ex(perc):
    from paper_1401_2130_amd import fss
    shapes, ps, n, seed = [(4, 16), (3, 10), (0, 9)], [0.2, 0.45, 0.9], 200, 77
    table = fss.pi_table(shapes, ps, n, seed)
    for (W, L) in shapes:
        lat = perc.Lattice(W, L)
        for p in ps:
            n_perc, _ = perc.perc_pi_ex(lat, p, n, seed)
            assert table[(W, L, float(p))] == n_perc
    curve = fss.pi_curve(4, 16, ps, n, seed)
    assert np.all(np.diff(curve) >= 0)  # common random numbers: monotone in p


def test_uneven_workload_counts(perc):
    """The uneven aspect-ratio workload (35 shapes x 2 p x 1024 configurations in one
    batch, settings from the autotuner as the benchmark runs it): the counts of four of
    its shapes equal the oracle's breadth-first-search counts over the same Philox
    configurations."""
    import oracle
    from paper_1401_2130_amd import fss, workloads
    wl = workloads.UNEVEN
    lats = [perc.Lattice(*sh) for sh in wl.shapes]
    tuned = perc.perc_autotune([(lat, wl.ps[0], wl.seed, c) for lat in lats for c in range(8)])
    opts = {k: tuned[k] for k in ("form", "depth", "block", "graph_steps")}
    counts = fss.pi_table(wl.shapes, wl.ps, wl.n_cfg, wl.seed, **opts)
    assert len(counts) == len(wl.shapes) * len(wl.ps)
    for (W, L) in [(8, 8), (8, 512), (16, 256), (24, 192)]:
        ref = oracle.Lattice(W, L)
        for p in wl.ps:
            pb, _ = ref.inspect_bfs(ref.sample(p, wl.seed, wl.n_cfg))
            assert counts[(W, L, float(p))] == int(pb.sum()), (W, L, p)


def test_profiler_counts_and_results(perc):
    """The step profiler (perc_profile_*): a profiled batch launches its steps directly and
    gives the bits, steps and FP32 first-hit probabilities of the graph-replayed batch;
    the span form's launches come in pairs, the timed milliseconds are positive, and the
    tube slots it counts lie between what the configurations' step counts allow."""
    import numpy as np
    from paper_1401_2130_amd import workloads

    W, L = 6, 40
    lat = perc.Lattice(W, L)
    occ = workloads.random_occupancy(lat.n, 160, 0.34, 91)
    d_occ = torch.from_numpy(np.ascontiguousarray(occ).view(np.int32)).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        p0, s0, h0 = perc.perc_inspect_ex(lat, d_occ, hit=True, form="span", depth=8, stream=s)
        s.synchronize()
        perc.perc_profile_enable(True)
        try:
            p1, s1, h1 = perc.perc_inspect_ex(lat, d_occ, hit=True, form="span", depth=8, stream=s)
            s.synchronize()
            prof = perc.perc_profile_read()
        finally:
            perc.perc_profile_enable(False)
    np.testing.assert_array_equal(p0.cpu().numpy(), p1.cpu().numpy())
    np.testing.assert_array_equal(s0.cpu().numpy(), s1.cpu().numpy())
    np.testing.assert_array_equal(h0.cpu().numpy().view(np.uint32), h1.cpu().numpy().view(np.uint32))
    assert prof["step_launches"] > 0 and prof["step_launches"] % 2 == 0
    assert prof["step_ms"] > 0.0
    steps = s1.cpu().numpy().astype(np.int64)
    U, C = (L + 2) // 3, lat.columns
    lo = int(np.sum(np.maximum(steps - 1, 0))) * min(U, 2) * C
    hi = int(np.sum(steps + 2)) * U * C
    assert lo <= prof["tube_steps"] <= hi, (lo, prof["tube_steps"], hi)
