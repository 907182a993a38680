"""The allocation-free domain sums (imexlb_domain_sums_noalloc) against the
context's imexlb_domain_sums, through the C ABI: the same kernels on the
same moment values, so the totals must agree bit for bit, on two calls in a
row (the second on a smaller grid, reusing the device's static partials)."""
import ctypes

import numpy as np
import pytest

from paper_1909_08390_amd import imexlb as I
from paper_1909_08390_amd import workloads as W


def _stacked_moments(s):
    """(n, ux, [uy], T) of the solver's state as one contiguous FP64 device
    tensor, fields of nx*ny values each (the layout the call reads)."""
    import torch
    n, ux, uy, T = s.moments()
    f = (n, ux, uy, T) if s.cfg.d == 2 else (n, ux, T)
    return torch.stack([x.reshape(-1) for x in f]).contiguous()


@pytest.mark.gpu
def test_noalloc_sums_equal_context_sums_on_two_calls():
    import torch
    assert torch.cuda.is_available()
    cases = [
        (I.Config(d=2, nx=300, ny=211, q_phi=5, q_chi=3, K=2, tau=1e-5, dt=1e-4), 3),
        (I.Config(d=1, nx=777, q_phi=8, q_chi=8, K=0, tau=1e-3, dt=2e-4, bc_x=I.PERIODIC), 5),
    ]
    for i, (c, steps) in enumerate(cases):
        print(f"no-alloc sums call {i + 1}: {c.field_shape}, K = {c.K}", flush=True)
        n, ux, uy, T = W.random_fields(c.field_shape, 20 + i)
        s = I.Solver(c)
        s.set_equilibrium(n, ux, uy, T)
        s.step(steps)
        ref = s.domain_sums()
        M = _stacked_moments(s)
        got = I.domain_sums_noalloc(c.d, c.K, M).cpu().numpy()
        print(f"  context {ref}, no-alloc {got}", flush=True)
        assert np.array_equal(got, ref), (got, ref)


def test_noalloc_sums_reject_bad_arguments_before_device_work():
    L = I.lib()
    buf = ctypes.c_void_p(16)  # never dereferenced: every case fails its checks first
    assert L.imexlb_domain_sums_noalloc(3, 2, buf, 10, buf, None) == I.EINVAL
    assert L.imexlb_domain_sums_noalloc(2, -1, buf, 10, buf, None) == I.EINVAL
    assert L.imexlb_domain_sums_noalloc(2, 2, None, 10, buf, None) == I.EINVAL
    assert L.imexlb_domain_sums_noalloc(2, 2, buf, 10, None, None) == I.EINVAL
    assert L.imexlb_domain_sums_noalloc(2, 2, buf, 0, buf, None) == I.EINVAL
    assert L.imexlb_domain_sums_noalloc(2, 2, buf, 1 << 31, buf, None) == I.EINVAL
