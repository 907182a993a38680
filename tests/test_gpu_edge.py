"""Degenerate and extreme configurations against the FP64 oracle.

 * lines of one, two and three cells (every ghost node maps onto the few
   fluid nodes; on a periodic line of one cell every stencil node is that
   cell), in 1D and as 2D grids one cell wide or one cell tall, and a 1 x 1
   grid;
 * the smallest orders (Q_phi = 3, the smallest with exact energy, and
   Q_chi = 1, whose only node is p = 0) and the largest (16 per axis and
   set: 512 planes in 2D);
 * off-equilibrium raw states set through imexlb_set_state;
 * zero steps leave the state unchanged.
FP64 tolerance 1e-12 of the reference's infinity norm, FP32 storage 1e-5,
as for the other parity cases.
"""
import numpy as np
import pytest

import oracle as O
from paper_1909_08390_amd import imexlb as I
from paper_1909_08390_amd import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def ocfg(c: I.Config) -> O.Config:
    return O.Config(d=c.d, nx=c.nx, ny=c.ny, lx=c.lx, ly=c.ly, q_phi=c.q_phi, q_chi=c.q_chi,
                    K=c.K, tau=c.tau, dt=c.dt, bc_x=c.bc_x, bc_y=c.bc_y)


def raw_state(c: I.Config, seed: int):
    """A non-equilibrium plane-set: the equilibrium of random fields with
    each population scaled by a random factor in [0.8, 1.2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n, ux, uy, T = W.random_fields(c.field_shape, seed, n_range=(0.7, 1.3), u_max=0.3,
                                   T_range=(0.8, 1.2))
    F = O.equilibrium(ocfg(c), n, ux, uy if c.d == 2 else None, T)
    return F * rng.uniform(0.8, 1.2, F.shape)


def close(got, ref, tol):
    scale = np.abs(ref).max()
    return np.abs(got - ref).max() <= tol * scale, np.abs(got - ref).max() / scale


CASES = [
    dict(d=1, nx=1, q_phi=5, q_chi=3, K=2, tau=1e-4, dt=1e-4, bc_x=I.OUTFLOW),
    dict(d=1, nx=1, q_phi=8, q_chi=8, K=0, tau=1e-4, dt=1e-4, bc_x=I.PERIODIC),
    dict(d=1, nx=2, q_phi=5, q_chi=3, K=2, tau=1e-4, dt=1e-4, bc_x=I.PERIODIC),
    dict(d=1, nx=3, q_phi=4, q_chi=2, K=2, tau=1e-4, dt=1e-4, bc_x=I.OUTFLOW),
    dict(d=1, nx=37, q_phi=3, q_chi=1, K=2, tau=1e-4, dt=2e-3, bc_x=I.OUTFLOW),
    dict(d=2, nx=1, ny=37, q_phi=5, q_chi=3, K=2, tau=1e-4, dt=2e-4, bc_x=I.OUTFLOW, bc_y=I.PERIODIC),
    dict(d=2, nx=53, ny=1, q_phi=5, q_chi=3, K=2, tau=1e-4, dt=2e-4, bc_x=I.PERIODIC, bc_y=I.OUTFLOW),
    dict(d=2, nx=1, ny=1, q_phi=4, q_chi=3, K=2, tau=1e-4, dt=1e-4, bc_x=I.PERIODIC, bc_y=I.OUTFLOW),
    dict(d=2, nx=35, ny=29, q_phi=3, q_chi=1, K=2, tau=1e-4, dt=2e-3, bc_x=I.OUTFLOW, bc_y=I.OUTFLOW),
    dict(d=2, nx=40, ny=24, q_phi=16, q_chi=16, K=2, tau=1e-4, dt=0.5 / 40 / 6.6309, bc_x=I.OUTFLOW,
         bc_y=I.PERIODIC),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("storage", [I.F64, I.F32])
def test_degenerate_and_extreme_configurations(case, storage):
    _torch()
    c = I.Config(storage=storage, **case)
    F0 = raw_state(c, 7)
    s = I.Solver(c)
    s.set_state(F0)
    steps = 3
    s.step(steps)
    oc = ocfg(c)
    ref = O.step(oc, F0 if storage == I.F64 else F0.astype(np.float32).astype(np.float64), steps)
    tol = 1e-12 if storage == I.F64 else 1e-5
    ok, err = close(s.state.cpu().numpy().astype(np.float64), ref, tol)
    print(f"{c.field_shape} Q {c.q_phi}/{c.q_chi} storage {storage}: max rel err {err:.2e}")
    assert ok, err
    n, ux, uy, T = [x.cpu().numpy() for x in s.moments()]
    on, oux, ouy, oT = O.moments(oc, ref)
    assert close(n, on, tol)[0] and close(T, oT, tol)[0]
    assert np.abs(ux - oux).max() <= tol * max(1.0, np.abs(oux).max())


def test_zero_steps_leave_the_state_unchanged():
    torch = _torch()
    c = I.Config(d=2, nx=70, ny=33, q_phi=5, q_chi=3, K=2, tau=1e-4, dt=1e-4)
    s = I.Solver(c)
    s.set_state(raw_state(c, 3))
    before = s.state.clone()
    m0 = [x.clone() for x in s.moments()]
    s.step(0)
    torch.cuda.synchronize()
    assert torch.equal(s.state, before)
    for a, b in zip(s.moments(), m0):
        assert torch.equal(a, b)


def test_uniform_equilibrium_is_a_fixed_point_on_small_grids():
    """A uniform equilibrium stays exactly uniform: every MP-9 face equals
    the common value (no flux), and the BGK terms vanish."""
    torch = _torch()
    for case in CASES[:8]:
        c = I.Config(**case)
        s = I.Solver(c)
        shape = c.field_shape
        s.set_equilibrium(np.full(shape, 0.9), np.full(shape, 0.2), np.full(shape, -0.1), np.full(shape, 1.1))
        F0 = s.state.clone()
        s.step(4)
        torch.cuda.synchronize()
        err = (s.state - F0).abs().max().item() / F0.abs().max().item()
        assert err < 1e-14, (case, err)
