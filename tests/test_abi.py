"""The C-ABI library loads, exports every declared entry point, and rejects
invalid configurations before touching a device (runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1909_08390_amd import imexlb as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "imexlb.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(imexlb_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["imexlb_create", "imexlb_destroy", "imexlb_bind", "imexlb_quadrature",
                     "imexlb_set_equilibrium", "imexlb_set_state", "imexlb_get_state",
                     "imexlb_step", "imexlb_moments", "imexlb_advect",
                     "imexlb_compute_moments", "imexlb_domain_sums", "imexlb_check_state",
                     "imexlb_status_string", "imexlb_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    L = I.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings():
    L = I.lib()
    for st in (I.OK, I.EINVAL, I.ENOMEM, I.EHIP, I.ENONPHYS, I.ESTATE):
        assert L.imexlb_status_string(st)


BAD = [
    dict(d=3),
    dict(nx=0),
    dict(d=1, ny=4),
    dict(q_phi=2),
    dict(q_phi=17),
    dict(q_chi=0),
    dict(K=-1),
    dict(tau=0.0),
    dict(dt=-1.0),
    dict(bc_x=5),
    dict(storage=7),
    dict(lx=0.0),
    # CFL: max |p| dt / dx = 2.857 * 1e-2 * 400 > 1 (Sec. IV)
    dict(dt=1e-2),
]


@pytest.mark.parametrize("over", BAD)
def test_invalid_configuration_rejected_before_device_work(over):
    base = dict(d=1, nx=400, q_phi=5, q_chi=3, K=2, tau=1e-5, dt=2.5e-4)
    base.update(over)
    cfg = I.Config(**base)
    assert I.validate(cfg) == I.EINVAL


def test_null_arguments():
    L = I.lib()
    assert L.imexlb_create(None, None, None) == I.EINVAL
    assert L.imexlb_step(None, 1) == I.EINVAL
    assert L.imexlb_bind(None, None, None) == I.EINVAL


def test_copy_probe_rejects_null_arguments():
    L = I.lib()
    out = ctypes.c_double(0.0)
    assert L.imexlb_copy_probe(None, None, 64, 1, None, ctypes.byref(out)) == I.EINVAL
    assert L.imexlb_copy_probe(None, None, 64, 1, None, None) == I.EINVAL


BAD_TUBES = [
    [],                                   # no tube
    [dict(nx=0)],
    [dict(nx=100, K=-1)],
    [dict(nx=100, tau=0.0)],
    [dict(nx=100, dt=0.0)],
    [dict(nx=100, lx=0.0)],
    [dict(nx=100, bc=3)],
    [dict(nx=64), dict(nx=400, dt=1e-2)],  # CFL of the second tube > 1 (Sec. IV)
]


@pytest.mark.parametrize("tubes", BAD_TUBES)
def test_batch_create_rejects_bad_tubes(tubes):
    assert I.batch_validate([I.TubeSpec(**t) for t in tubes]) == I.EINVAL


@pytest.mark.parametrize("kw", [dict(q_phi=2), dict(q_chi=0), dict(q_phi=17), dict(storage=5)])
def test_batch_create_rejects_bad_quadrature_or_storage(kw):
    assert I.batch_validate([I.TubeSpec(nx=64)], **kw) == I.EINVAL
