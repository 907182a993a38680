"""Batched 1D tubes: many shock tubes of uneven size, K, tau and dt,
through the C ABI, under every execution plan (per-pass launches, and
persistent launches of several steps with long outflow tubes split into
chunks stepped over extended regions).

 * every tube matches the FP64 oracle stepping that tube alone (1e-12 of the
   reference's infinity norm), for uneven and ragged sizes, K = 0 and 2,
   outflow and periodic ends;
 * every plan gives results bitwise equal to the single-grid 1D path, in
   FP64 and FP32 storage, over 11 steps (odd and even launch counts, a
   shorter last launch, a 4096-cell outflow tube split into 2 or 4 chunks, a
   3001-cell periodic tube kept whole);
 * the autotuner times all plans and leaves state and moments unchanged;
 * the full 256-tube workload (seeded, FP32 storage) stays physical and, on
   sampled tubes, agrees with the FP64 run and with the oracle.
"""
import numpy as np
import pytest

import oracle as O
from paper_1909_08390_amd import imexlb as I
from paper_1909_08390_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def spec_of(t: W.Tube, bc=I.OUTFLOW) -> I.TubeSpec:
    return I.TubeSpec(nx=t.nx, K=t.K, lx=1.0, tau=t.tau, dt=W.tube_dt(t.nx), bc=bc)


def mixed_tubes():
    """Uneven sizes (ragged, below one tile, several tiles), K 0/2, both ends."""
    rng = np.random.Generator(np.random.PCG64(7))
    sizes = [37, 256, 300, 1030, 2049, 613, 4, 1024, 3001, 4096]
    out = []
    for i, nx in enumerate(sizes):
        K = [0, 2][i % 2]
        tau = float(10.0 ** rng.uniform(-6, -2))
        left = (float(rng.uniform(0.5, 2)), float(rng.uniform(-0.3, 0.3)), float(rng.uniform(0.5, 2)))
        right = (float(rng.uniform(0.1, 1)), float(rng.uniform(-0.3, 0.3)), float(rng.uniform(0.1, 1)))
        out.append((W.Tube(nx, K, tau, left, right), I.PERIODIC if i % 3 == 2 else I.OUTFLOW))
    return out


def run_batch(tubes_bc, storage, steps, tiling=None, plan=None):
    torch = _torch()
    specs = [spec_of(t, bc) for t, bc in tubes_bc]
    b = I.Batch(specs, 8, 8, storage)
    f = [W.tube_fields(t) for t, _ in tubes_bc]
    b.set_equilibrium([x[0] for x in f], [x[1] for x in f], [x[2] for x in f])
    if tiling is not None:
        b.set_tiling(*tiling)
    if plan is not None:
        b.set_plan(plan)
    b.step(steps)
    torch.cuda.synchronize()
    return b


def test_every_tube_matches_the_oracle():
    tubes = mixed_tubes()
    b = run_batch(tubes, I.F64, 6)
    n, u, T = [x.cpu().numpy() for x in b.moments()]
    for i, (t, bc) in enumerate(tubes):
        s = spec_of(t, bc)
        oc = O.Config(d=1, nx=t.nx, lx=1.0, q_phi=8, q_chi=8, K=t.K, tau=s.tau, dt=s.dt, bc_x=bc)
        fn, fu, fT = W.tube_fields(t)
        ref = O.step(oc, O.equilibrium(oc, fn, fu, None, fT), 6)
        got = b.tube_state(i).cpu().numpy()
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= TOL * scale, f"tube {i} (nx={t.nx})"
        on, ou, _, oT = O.moments(oc, ref)
        sl = slice(b.cell_offset[i], b.cell_offset[i] + t.nx)
        assert np.abs(n[sl] - on).max() <= TOL * np.abs(on).max()
        assert np.abs(u[sl] - ou).max() <= TOL * max(1.0, np.abs(ou).max())
        assert np.abs(T[sl] - oT).max() <= TOL * np.abs(oT).max()


@pytest.mark.parametrize("storage", [I.F64, I.F32])
def test_every_plan_equals_the_single_grid_path(storage):
    torch = _torch()
    tubes = mixed_tubes()
    steps = 11
    ref, mref = [], []
    for t, bc in tubes:
        s = spec_of(t, bc)
        c = I.Config(d=1, nx=t.nx, q_phi=8, q_chi=8, K=t.K, tau=s.tau, dt=s.dt, bc_x=bc,
                     storage=storage)
        sol = I.Solver(c)
        fn, fu, fT = W.tube_fields(t)
        sol.set_equilibrium(fn, fu, None, fT)
        sol.step(steps)
        torch.cuda.synchronize()
        ref.append(sol.state.cpu().numpy())
        n, u, _, T = sol.moments()
        mref.append((n.cpu().numpy(), u.cpu().numpy(), T.cpu().numpy()))
    plans = I.batch_plans()
    assert any(p.mode == 1 and p.chunk < 4096 for p in plans)
    for plan in plans:
        print(f"plan {plan}", flush=True)
        b = run_batch(tubes, storage, steps, plan=plan)
        assert b.plan() == plan
        n, u, T = [x.cpu().numpy() for x in b.moments()]
        for i in range(len(tubes)):
            got = b.tube_state(i).cpu().numpy()
            assert np.array_equal(got, ref[i]), f"plan {plan}, tube {i}"
            sl = slice(b.cell_offset[i], b.cell_offset[i] + tubes[i][0].nx)
            for a, r in zip((n[sl], u[sl], T[sl]), mref[i]):
                assert np.array_equal(a, r), f"plan {plan}, tube {i} moments"
        del b


def test_tuner_times_every_plan_and_keeps_the_state():
    torch = _torch()
    tubes = [(t, I.OUTFLOW) for t in W.batch_tubes(32, seed=3)]
    b = run_batch(tubes, I.F32, 2)
    before = [b.tube_state(i).clone() for i in range(len(tubes))]
    m0 = [x.clone() for x in b.moments()]
    times = b.tune(3)
    torch.cuda.synchronize()
    assert set(times) == set(I.batch_plans()) and all(v > 0 for v in times.values())
    assert b.plan() == min(times, key=times.get)
    bits = torch.int32 if b.state_dtype == torch.float32 else torch.int64
    for i in range(len(tubes)):
        assert torch.equal(b.tube_state(i).view(bits), before[i].view(bits)), f"tube {i}"
    for a, c in zip(b.moments(), m0):
        assert torch.equal(a.view(torch.int64), c.view(torch.int64))


def test_full_batch_workload_sampled():
    """256 seeded tubes (Nx 256..4096, K 0/2, tau 1e-6..1e-2), FP32 storage
    vs FP64 storage, and the FP64 run vs the oracle on sampled tubes."""
    torch = _torch()
    tubes = [(t, I.OUTFLOW) for t in W.batch_tubes(256, seed=0)]
    b32 = run_batch(tubes, I.F32, 20)
    b64 = run_batch(tubes, I.F64, 20)
    n32, u32, T32 = [x.cpu().numpy() for x in b32.moments()]
    n64, u64, T64 = [x.cpu().numpy() for x in b64.moments()]
    assert np.all(np.isfinite(n32)) and n32.min() > 0 and T32.min() > 0
    rel = lambda a, c: np.abs(a - c).sum() / np.abs(c).sum()
    assert rel(n32, n64) < 1e-5
    assert rel(n32 * T32, n64 * T64) < 1e-5
    assert np.abs(u32 - u64).mean() < 1e-5
    for i in (0, 17, 101, 255):
        t, bc = tubes[i]
        s = spec_of(t, bc)
        oc = O.Config(d=1, nx=t.nx, lx=1.0, q_phi=8, q_chi=8, K=t.K, tau=s.tau, dt=s.dt, bc_x=bc)
        fn, fu, fT = W.tube_fields(t)
        ref = O.step(oc, O.equilibrium(oc, fn, fu, None, fT), 20)
        got = b64.tube_state(i).cpu().numpy()
        assert np.abs(got - ref).max() <= TOL * np.abs(ref).max(), f"tube {i}"
