"""The C-ABI library loads, exports every declared entry point, and rejects
invalid configurations before touching a device (runs without a GPU)."""
import ctypes
import os
import re
import subprocess

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
                     "imexlb_density_loss", "imexlb_status_string", "imexlb_last_error"]:
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
    assert L.imexlb_density_loss(None, None, None, None, None) == I.EINVAL
    assert L.imexlb_step_recorded(None, None) == I.EINVAL
    assert L.imexlb_step_recorded_to(None, None, None) == I.EINVAL
    assert L.imexlb_adjoint_step_recorded(None, None, None, None, None) == I.EINVAL
    assert L.imexlb_step_record_bytes(None) == 0


def test_config_mirror_matches_header_layout(tmp_path):
    """The ctypes mirrors of imexlb_config and imexlb_tube have the C
    layout: sizes and field offsets printed by a program compiled against
    the header."""
    fields = [f for f, _ in I.CConfig._fields_]
    tfields = [f for f, _ in I.CTube._fields_]
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "imexlb.h"', 'int main(void) {',
             '  printf("%zu\\n", sizeof(imexlb_config));',
             '  printf("%zu\\n", sizeof(imexlb_tube));']
    lines += [f'  printf("%zu\\n", offsetof(imexlb_config, {f}));' for f in fields]
    lines += [f'  printf("%zu\\n", offsetof(imexlb_tube, {f}));' for f in tfields]
    lines += ['  return 0;', '}']
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(I.CConfig), ctypes.sizeof(I.CTube)]
    want += [getattr(I.CConfig, f).offset for f in fields]
    want += [getattr(I.CTube, f).offset for f in tfields]
    assert got == want


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
