"""The plain-copy probe behind the bench's achievable-bandwidth figure
(imexlb_copy_probe): exact copies, a rate, argument checks on device
buffers."""
import ctypes

import pytest

from paper_1909_08390_amd import imexlb as I

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def test_copy_probe_copies_exactly_and_reports_a_rate():
    g = torch.Generator(device="cpu").manual_seed(0)
    nbytes = (1 << 20) + 48  # 65539 16-byte elements: a ragged last work-group
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, generator=g).cuda()
    dst = torch.zeros_like(src)
    gbs = I.copy_probe(src, dst, 3)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    assert 0.0 < gbs < 1e5


def test_copy_probe_rejects_bad_arguments_on_device_buffers():
    L = I.lib()
    buf = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    p = buf.data_ptr()
    out = ctypes.c_double(0.0)

    def call(s, d, nbytes, reps):
        return L.imexlb_copy_probe(ctypes.c_void_p(s), ctypes.c_void_p(d), nbytes, reps, None,
                                   ctypes.byref(out))

    # every case stays inside the 64 KiB buffer even if a check were missing
    assert call(p, p + 4096, 0, 1) == I.EINVAL        # empty
    assert call(p, p + 4096, 15, 1) == I.EINVAL       # not a multiple of 16
    assert call(p + 8, p + 4096, 64, 1) == I.EINVAL   # misaligned source
    assert call(p, p + 4104, 64, 1) == I.EINVAL       # misaligned destination
    assert call(p, p + 32, 64, 1) == I.EINVAL         # overlapping ranges
    assert call(p, p + 4096, 64, 0) == I.EINVAL       # reps < 1
    assert L.imexlb_copy_probe(None, ctypes.c_void_p(p), 64, 1, None, ctypes.byref(out)) == I.EINVAL
    assert call(p, p + 4096, 64, 2) == I.OK
    torch.cuda.synchronize()
    assert out.value > 0.0
