"""The work buffer the library keeps between calls (large work memory, lent to one call
at a time, stream-ordered behind the previous borrower's work).

W=16 L=256 with 512 configurations needs about 0.3 GB of work memory in the span form,
above the size from which the buffer is used. Results must not depend on whether a call
borrowed the buffer, allocated its own (buffer lent to another thread), or found it
released by perc_trim; calls on different streams must not overlap in it.
"""
import threading

import pytest
import torch

pytestmark = pytest.mark.gpu

W, L, N = 16, 256, 512


@pytest.fixture(scope="module")
def perc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1401_2130_amd as p
    return p


def run_pi(perc, lat, p, seed, stream=None):
    b = torch.empty(N, dtype=torch.uint8, device="cuda")
    s = torch.empty(N, dtype=torch.int32, device="cuda")
    n, _ = perc.perc_pi_ex(lat, p, N, seed, bits=b, steps=s, form="span", stream=stream)
    torch.cuda.synchronize()
    return n, b.cpu(), s.cpu()


def test_reuse_and_trim(perc):
    lat = perc.Lattice(W, L)
    first = run_pi(perc, lat, 0.16, 11)
    again = run_pi(perc, lat, 0.16, 11)
    perc.perc_trim()
    after_trim = run_pi(perc, lat, 0.16, 11)
    perc.perc_trim()
    perc.perc_trim()  # nothing held: still fine
    for r in (again, after_trim):
        assert r[0] == first[0]
        assert torch.equal(r[1], first[1]) and torch.equal(r[2], first[2])


def test_two_streams_back_to_back(perc):
    """Async inspections on two streams, enqueued without a host wait between them: the
    second borrower must wait for the first's work (each result equals its serial run)."""
    lat = perc.Lattice(W, L)
    occ_a = perc.perc_sample(lat, 0.155, 21, N)
    occ_b = perc.perc_sample(lat, 0.165, 22, N)
    torch.cuda.synchronize()
    ref = []
    for occ in (occ_a, occ_b):
        pg, sg, _ = perc.perc_inspect_ex(lat, occ, form="span")
        torch.cuda.synchronize()
        ref.append((pg.cpu(), sg.cpu()))
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    for _ in range(3):
        outs = []
        for occ, st in ((occ_a, sa), (occ_b, sb)):
            pg = torch.empty(N, dtype=torch.uint8, device="cuda")
            sg = torch.empty(N, dtype=torch.int32, device="cuda")
            perc.perc_inspect_ex(lat, occ, perc=pg, steps=sg, form="span", stream=st)
            outs.append((pg, sg))
        torch.cuda.synchronize()
        for (pg, sg), (rp, rs) in zip(outs, ref):
            assert torch.equal(pg.cpu(), rp) and torch.equal(sg.cpu(), rs)


def test_threads_share_the_buffer(perc):
    """Two host threads inspecting at once on their own streams: one borrows the buffer,
    the other allocates its own while it is lent out; every result equals its serial run."""
    lat = perc.Lattice(W, L)
    cases = [(0.15, 31), (0.16, 32), (0.17, 33), (0.155, 34)]
    ref = {c: run_pi(perc, lat, *c) for c in cases}
    got, errors = {}, []

    def worker(mine):
        try:
            st = torch.cuda.Stream()
            for c in mine * 2:
                b = torch.empty(N, dtype=torch.uint8, device="cuda")
                s = torch.empty(N, dtype=torch.int32, device="cuda")
                n, _ = perc.perc_pi_ex(lat, c[0], N, c[1], bits=b, steps=s, form="span", stream=st)
                st.synchronize()
                got.setdefault(c, []).append((n, b.cpu(), s.cpu()))
        except Exception as e:  # reported below
            errors.append(repr(e))

    th = [threading.Thread(target=worker, args=(cases[i::2],)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    assert not errors, errors
    for c in cases:
        assert len(got[c]) == 2
        for n, b, s in got[c]:
            assert n == ref[c][0]
            assert torch.equal(b, ref[c][1]) and torch.equal(s, ref[c][2])


def test_threads_share_the_side_stream(perc):
    """Two host threads running mixed batches at once (each batch's short-walk part on the
    library's one side stream and its work buffer, the long-walk part on the thread's own
    stream): every result equals its serial run."""
    import numpy as np
    narrow, wide = perc.Lattice(8, 16), perc.Lattice(26, 400)
    batches = [np.concatenate([perc.philox_jobs(narrow, p, seed, 2100, group=0),
                               perc.philox_jobs(wide, 0.17, seed + 1, 24, group=1)])
               for p, seed in ((0.25, 41), (0.3, 43))]
    ref = []
    for jobs in batches:
        pr, sr, _, cr = perc.perc_batch(jobs, n_groups=2, form="mixed")
        torch.cuda.synchronize()
        ref.append((pr.cpu(), sr.cpu(), list(cr)))
    got, errors = {}, []

    def worker(i):
        try:
            st = torch.cuda.Stream()
            for _ in range(2):
                pr, sr, _, cr = perc.perc_batch(batches[i], n_groups=2, form="mixed", stream=st)
                st.synchronize()
                got.setdefault(i, []).append((pr.cpu(), sr.cpu(), list(cr)))
        except Exception as e:  # reported below
            errors.append(repr(e))

    th = [threading.Thread(target=worker, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    assert not errors, errors
    for i in range(2):
        assert len(got[i]) == 2
        for pr, sr, cr in got[i]:
            assert torch.equal(pr, ref[i][0]) and torch.equal(sr, ref[i][1]) and cr == ref[i][2]

