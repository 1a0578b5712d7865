"""perc_inspect_noalloc (the entry point that allocates nothing) through the C ABI: its
outputs equal perc_inspect_ex's (span form) bit for bit on two calls in a row, the
second with a smaller input, on a batch that needs several waves of the fixed work
array, and it refuses a fiber whose configuration does not fit that array."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1401_2130_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def perc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1401_2130_amd as p
    return p


def call_noalloc(perc, lat, occ, n, with_steps=True, with_hit=True):
    """The C entry point itself, with caller-owned outputs."""
    bits = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    steps = torch.full((n,), -7, dtype=torch.int32, device="cuda") if with_steps else None
    hit = torch.full((n,), -1.0, dtype=torch.float32, device="cuda") if with_hit else None
    torch.cuda.synchronize()
    rc = perc._lib.perc_inspect_noalloc(lat.handle, occ.data_ptr(), n, bits.data_ptr(),
                                        steps.data_ptr() if steps is not None else None,
                                        hit.data_ptr() if hit is not None else None, None)
    assert rc == perc.PERC_OK, perc.perc_last_error()
    return bits, steps, hit


def reference(perc, lat, occ, n):
    pg, sg, hg = perc.perc_inspect_ex(lat, occ, n, hit=True, form="span")
    torch.cuda.synchronize()
    return pg.cpu().numpy(), sg.cpu().numpy(), hg.cpu().numpy()


def check(perc, lat, occ, n, **kw):
    rb, rs, rh = reference(perc, lat, occ, n)
    bits, steps, hit = call_noalloc(perc, lat, occ, n, **kw)
    assert np.array_equal(bits.cpu().numpy(), rb)
    if steps is not None:
        assert np.array_equal(steps.cpu().numpy(), rs)
    if hit is not None:
        assert np.array_equal(hit.cpu().numpy().view(np.uint32), rh.view(np.uint32))
    return rb


def test_two_calls_second_smaller(perc):
    lat = perc.Lattice(8, 150)
    occ = torch.from_numpy(workloads.random_occupancy(lat.n, 48, 0.22, 5, pad_garbage=True).view(np.int32)).cuda()
    b1 = check(perc, lat, occ, 48)
    assert 0 < b1.sum() < 48
    lat2 = perc.Lattice(3, 40)
    occ2 = perc.perc_sample(lat2, 0.35, 9, 11)
    check(perc, lat2, occ2, 11)
    # outputs of the first size again, steps not requested (held in the array)
    check(perc, lat, occ, 48, with_steps=False, with_hit=False)


def test_several_waves_and_no_device_allocation(perc):
    """W=32 L=1024 x 40 configurations need about 400 MB of state: several waves of the
    256 MiB array. The free device memory is the same before and after the call."""
    lat = perc.Lattice(32, 1024)
    occ = perc.perc_sample(lat, 0.17, 2, 40)
    check(perc, lat, occ, 40)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    bits, steps, hit = call_noalloc(perc, lat, occ, 40)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0


def test_too_large_and_bad_arguments(perc):
    lat = perc.Lattice(64, 8192)
    occ = torch.zeros(lat.words, dtype=torch.int32, device="cuda")
    out = torch.empty(1, dtype=torch.uint8, device="cuda")
    rc = perc._lib.perc_inspect_noalloc(lat.handle, occ.data_ptr(), 1, out.data_ptr(), None, None, None)
    assert rc == perc.PERC_EINVAL and "fixed" in perc.perc_last_error()
    assert perc._lib.perc_inspect_noalloc(lat.handle, None, 1, out.data_ptr(), None, None, None) == perc.PERC_EINVAL
    assert perc._lib.perc_inspect_noalloc(lat.handle, occ.data_ptr(), -1, out.data_ptr(), None, None, None) == perc.PERC_EINVAL
    assert perc._lib.perc_inspect_noalloc(lat.handle, occ.data_ptr(), 0, None, None, None, None) == perc.PERC_OK
    # the largest serving fiber fits
    big = perc.Lattice(64, 4096)
    occb = perc.perc_sample(big, 0.19, 77, 1)
    check(perc, big, occb, 1)
