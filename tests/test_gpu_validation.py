"""The paper's own validations (Sec. V) run through the library on the GPU:
the Sod tube against the exact Riemann solution under resolution and time
step sweeps (Fig. 1), and the 2D Riemann configurations C11 and C12 against
the density ranges the paper prints for its contour plots (Fig. 2).

The checks are the paper's qualitative ones made quantitative:
 * S-sweep at dt = 1e-5, t = 0.15: the L1 density error against the inviscid
   solution falls monotonically from S = 200 to 3200 (it saturates at the
   physical dissipation of tau = 1e-5, as the paper notes);
 * dt-sweep at S = 400: the error does not depend on dt.  The paper's
   largest step, dt = 1e-3, gives max|p| dt / ds = 1.14 on the unit domain,
   above the CFL bound of Sec. IV that the library enforces, so the sweep
   starts at 5e-4, the step the paper adopts;
 * C11 / C12 at 400^2, Q_phi = 5, Q_chi = 3, dt = 5e-4, tau = 1e-5: min and
   max of the density within 2 % of the printed contour range (the printed
   values are plot limits given to 2-3 digits, not data extremes);
 * C12 is symmetric under x <-> y; the GPU arithmetic orders x and y terms
   differently, so symmetry holds to round-off while perturbations are
   small (the shock interaction on the diagonal later amplifies them).
"""
import numpy as np
import pytest

from golden_data import riemann2d
from riemann_exact import sample as riemann_sample

pytestmark = pytest.mark.gpu

T_SOD = 0.15


@pytest.fixture(scope="module")
def I():
    from paper_1909_08390_amd import imexlb
    return imexlb


def sod_l1(I, S, dt):
    import torch
    from paper_1909_08390_amd import workloads as W

    c = I.Config(d=1, nx=S, q_phi=5, q_chi=3, K=2, tau=1e-5, dt=dt)
    s = I.Solver(c)
    n0, u0, T0 = W.sod_1d(S)
    s.set_equilibrium(n0, u0, None, T0)
    steps = int(round(T_SOD / dt))
    s.step(steps)
    torch.cuda.synchronize()
    rho = s.moments()[0].cpu().numpy()
    x = W.centres(S)
    ex, _, _ = riemann_sample(W.SOD_LEFT, W.SOD_RIGHT, 1.4, (x - 0.5) / (steps * dt))
    return float(np.mean(np.abs(rho - ex)))


def test_sod_resolution_sweep_converges(I):
    errs = [sod_l1(I, S, 1e-5) for S in (200, 400, 800, 1600, 3200)]
    print("L1 by S:", errs, flush=True)
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[1] < 1.5e-3


def test_sod_timestep_sweep_is_flat(I):
    errs = [sod_l1(I, 400, dt) for dt in (5e-4, 1e-4, 5e-5, 1e-5)]
    print("L1 by dt:", errs, flush=True)
    assert max(errs) / min(errs) < 1.01


def run_riemann2d(I, c, steps=None):
    import torch
    from paper_1909_08390_amd import workloads as W

    g = riemann2d()[c]
    N, dt = 400, 5e-4
    cfg = I.Config(d=2, nx=N, ny=N, q_phi=5, q_chi=3, K=2, tau=1e-5, dt=dt)
    s = I.Solver(cfg)
    s.set_equilibrium(*W.riemann_2d(N, N, g["states"]))
    s.step(steps if steps is not None else int(round(g["t_end"] / dt)))
    torch.cuda.synchronize()
    assert s.check_state() == I.OK
    return s.moments()[0].cpu().numpy(), g


@pytest.mark.parametrize("c", [11, 12])
def test_riemann2d_density_range_matches_printed_contours(I, c):
    rho, g = run_riemann2d(I, c)
    lo, hi = g["rho_range"]
    print(f"C{c}: rho in [{rho.min():.4f}, {rho.max():.4f}], printed [{lo}, {hi}]", flush=True)
    assert abs(rho.min() - lo) <= 0.02 * lo
    assert abs(rho.max() - hi) <= 0.02 * hi


def test_c12_transpose_symmetry_to_roundoff(I):
    rho, _ = run_riemann2d(I, 12, steps=100)
    assert np.max(np.abs(rho - rho.T)) < 1e-11
