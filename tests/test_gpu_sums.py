"""Domain sums, the density loss and the physical-state check through the C
ABI, against the FP64 oracle after stepping and against their definitions.

The domain sums are the conserved totals of Sec. II (Eq. Moments): mass
sum n, momentum sum n u and energy sum (D+K)/2 n T + n |u|^2 / 2.  The
reference values are numpy sums of the oracle's moments after the oracle
stepped the same seeded input (they share nothing with the library).
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


def sums_of(n, ux, uy, T, K):
    """The four totals from moment fields (D = 3)."""
    e = 0.5 * (3 + K) * n * T + 0.5 * n * (ux ** 2 + uy ** 2)
    return np.array([n.sum(), (n * ux).sum(), (n * uy).sum(), e.sum()]), \
        np.array([np.abs(n).sum(), np.abs(n * ux).sum(), np.abs(n * uy).sum(), np.abs(e).sum()])


SUM_CASES = [
    # (config, field kind, seed, steps)
    (dict(d=2, nx=96, ny=64, q_phi=6, q_chi=4, K=2, tau=1e-4, dt=5e-4,
          bc_x=I.PERIODIC, bc_y=I.PERIODIC), "smooth", 4, 30),
    (dict(d=2, nx=70, ny=45, q_phi=8, q_chi=8, K=2, tau=1e-6, dt=0.5 / 70 / 4.144547186125894),
     "riemann", 0, 10),
    (dict(d=1, nx=400, q_phi=5, q_chi=3, K=2, tau=1e-5, dt=2.5e-4), "sod", 0, 100),
    (dict(d=1, nx=257, q_phi=8, q_chi=8, K=0, tau=1e-3, dt=2e-4, bc_x=I.PERIODIC), "random", 7, 40),
]


def _fields(c, kind, seed):
    if kind == "smooth":
        return W.smooth_fields(c.field_shape, seed)
    if kind == "random":
        return W.random_fields(c.field_shape, seed)
    if kind == "sod":
        n, ux, T = W.sod_1d(c.nx)
        return n, ux, np.zeros_like(n), T
    st, _ = W.quadrant_states(seed)
    return W.riemann_2d(c.nx, c.ny, st)


@pytest.mark.parametrize("case,kind,seed,steps", SUM_CASES)
def test_domain_sums_match_oracle_after_steps(case, kind, seed, steps):
    """GPU sums after `steps` steps equal numpy sums of the oracle's
    moments after the same steps, to 1e-12 of the summed magnitudes."""
    _torch()
    c = I.Config(**case)
    n, ux, uy, T = _fields(c, kind, seed)
    s = I.Solver(c)
    s.set_equilibrium(n, ux, uy, T)
    s.step(steps)
    got = s.domain_sums()
    oc = ocfg(c)
    F = O.step(oc, O.equilibrium(oc, n, ux, uy if c.d == 2 else None, T), steps)
    on, oux, ouy, oT = O.moments(oc, F)
    ref, mag = sums_of(on, oux, ouy if c.d == 2 else np.zeros_like(on), oT, c.K)
    print(f"{kind} {c.field_shape} {steps} steps: sums {got} vs {ref}")
    assert np.all(np.abs(got - ref) <= 1e-12 * np.maximum(mag, 1.0)), (got, ref)


def test_domain_sums_conserved_on_full_periodic_4096_grid():
    """4096^2 x 128 planes, FP64, periodic in both axes, seeded quadrant
    states: mass, momentum and energy are unchanged after 10 steps (to 1e-12
    of the mass for momentum, relative for mass and energy).  A tile that a
    pass skipped or wrote twice with stale data breaks the telescoping of
    its fluxes, so this covers every tile of the full grid."""
    torch = _torch()
    N = 4096
    c = I.Config(d=2, nx=N, ny=N, q_phi=8, q_chi=8, K=2, tau=1e-7, dt=0.5 / N / 4.144547186125894,
                 bc_x=I.PERIODIC, bc_y=I.PERIODIC)
    st, _ = W.quadrant_states(0)
    n, ux, uy, T = W.riemann_2d(N, N, st)
    s = I.Solver(c)
    s.set_equilibrium(n, ux, uy, T)
    del n, ux, uy, T
    s0 = s.domain_sums()
    s.step(10)
    s1 = s.domain_sums()
    print(f"4096^2 periodic: sums before {s0}, after 10 steps {s1}")
    assert abs(s1[0] - s0[0]) <= 1e-12 * s0[0]
    assert abs(s1[1] - s0[1]) <= 1e-12 * s0[0]
    assert abs(s1[2] - s0[2]) <= 1e-12 * s0[0]
    assert abs(s1[3] - s0[3]) <= 1e-12 * s0[3]
    del s
    torch.cuda.empty_cache()


def test_domain_sums_deterministic():
    """The same state summed twice gives bitwise the same totals."""
    _torch()
    c = I.Config(d=2, nx=300, ny=211, q_phi=5, q_chi=3, K=2, tau=1e-5, dt=1e-4)
    n, ux, uy, T = W.random_fields(c.field_shape, 11)
    s = I.Solver(c)
    s.set_equilibrium(n, ux, uy, T)
    a, b = s.domain_sums(), s.domain_sums()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("shape", [(1,), (5,), (1000,), (333, 101)])
def test_density_loss_matches_definition(shape):
    """loss = 1/2 sum (n - n*)^2 to 1e-13 relative; the gradient is n - n*
    exactly (one subtraction per cell)."""
    torch = _torch()
    d = len(shape)
    c = I.Config(d=d, nx=shape[-1], ny=shape[0] if d == 2 else 1, q_phi=5, q_chi=3, dt=1e-6)
    s = I.Solver(c)
    rng = np.random.default_rng(5)
    n = rng.uniform(0.5, 1.5, shape)
    tgt = rng.uniform(0.5, 1.5, shape)
    loss, g = s.density_loss(tgt, n=n, grad=True)
    torch.cuda.synchronize()
    ref = 0.5 * np.sum((n - tgt) ** 2)
    assert abs(loss.item() - ref) <= 1e-13 * ref
    assert np.array_equal(g.cpu().numpy(), n - tgt)


def test_density_loss_of_current_state():
    """With no density given the loss uses the state's own density."""
    torch = _torch()
    c = I.Config(d=2, nx=40, ny=30, q_phi=6, q_chi=4, K=2, tau=1e-4, dt=5e-4,
                 bc_x=I.PERIODIC, bc_y=I.PERIODIC)
    n, ux, uy, T = W.smooth_fields(c.field_shape, 2)
    s = I.Solver(c)
    s.set_equilibrium(n, ux, uy, T)
    s.step(3)
    tgt = np.full(c.field_shape, 1.0)
    loss, _ = s.density_loss(tgt)
    nn = s.moments()[0].cpu().numpy()
    torch.cuda.synchronize()
    ref = 0.5 * np.sum((nn - tgt) ** 2)
    assert abs(loss.item() - ref) <= 1e-13 * ref


def test_check_physical_flag_in_step():
    """check_physical set: a clean run returns OK with the same state as an
    unchecked run; a NaN injected at one cell from the host makes the step
    return ENONPHYS naming step 1; a negative density likewise."""
    torch = _torch()
    base = dict(d=1, nx=200, q_phi=5, q_chi=3, K=2, tau=1e-5, dt=2.5e-4)
    n, ux, T = W.sod_1d(200)
    plain = I.Solver(I.Config(**base))
    plain.set_equilibrium(n, ux, None, T)
    plain.step(5)
    chk = I.Solver(I.Config(check_physical=1, **base))
    chk.set_equilibrium(n, ux, None, T)
    chk.step(5)
    assert torch.equal(plain.state, chk.state)
    for bad in (float("nan"), -1.0):
        F = chk.state.clone()
        F[:, 17] = bad
        chk.set_state(F)
        with pytest.raises(I.ImexlbError) as e:
            chk.step(3)
        assert e.value.status == I.ENONPHYS
        assert "after step 1 " in str(e.value)
    # unchecked: the same input steps without an error
    F = plain.state.clone()
    F[:, 17] = float("nan")
    plain.set_state(F)
    plain.step(1)
    torch.cuda.synchronize()
