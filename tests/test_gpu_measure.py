"""Measurement hooks on the GPU: the streaming copy behind the HBM ceiling copies exactly
and checks its arguments; the step profiler counts the server's ticks without changing
any served result."""
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


@pytest.mark.parametrize("n,grid", [(16, 0), (4096 * 512 + 48, 0), (12345 * 16, 7), (1 << 24, 4096)])
def test_stream_copy_exact(perc, n, grid):
    src = torch.randint(-2**31, 2**31 - 1, (n // 4,), dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    perc.perc_stream_copy(src, dst, grid=grid)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


def test_stream_copy_arguments(perc):
    a = torch.zeros(64, dtype=torch.int32, device="cuda")
    lib = perc._lib
    assert lib.perc_stream_copy(a.data_ptr(), a.data_ptr() + 128, 24, 0, None) == perc.PERC_EINVAL  # not 16k
    assert lib.perc_stream_copy(a.data_ptr() + 4, a.data_ptr() + 128, 32, 0, None) == perc.PERC_EINVAL  # alignment
    assert lib.perc_stream_copy(a.data_ptr(), a.data_ptr() + 128, 0, 0, None) == perc.PERC_OK


def test_profiled_server_counts_and_results(perc):
    reqs = [(0.0, 6, 200, 0.5, 90 + i, 0, i) for i in range(12)]
    results = []
    for prof in (False, True):
        perc.perc_profile_enable(prof)
        srv = perc.perc_server(hbm_bytes=1 << 28, max_slots=8, tick_steps=8, max_w=8, stream=torch.cuda.Stream())
        res = sorted(srv.run(reqs), key=lambda r: r["tag"])
        pr = perc.perc_profile_read()
        perc.perc_profile_enable(False)
        results.append([(r["perc"], r["steps"], np.float32(r["hit"]).view(np.uint32)) for r in res])
        if prof:
            assert pr["step_launches"] > 0 and pr["step_ms"] > 0
            # every step launch of a request (steps - 1 for a percolating one: the last
            # step is the detector's) advanced at least one cell of its columns
            launched = sum(max(r["steps"] - 1, 0) for r in res)
            assert pr["tube_steps"] >= launched * perc.Lattice(6, 200).columns
    assert results[0] == results[1]
