"""Pins of the oracle's MP-9 advection operator (Sec. IV of the paper).

Expected values come from calculus (exact derivatives of polynomials), from
the observed convergence order on a smooth periodic wave, and from the
monotonicity-preserving property -- never from the oracle itself.
"""
import numpy as np
import pytest

import oracle as O


def _cfg1(S, L=1.0, bc=O.PERIODIC, qp=5, qc=3):
    return O.Config(d=1, nx=S, lx=L, q_phi=qp, q_chi=qc, bc_x=bc)


def _plane_field(cfg, f_of_x):
    """A state whose every plane holds f(x) (2D: f(x) for every row)."""
    x = (np.arange(cfg.nx) + 0.5) * cfg.lx / cfg.nx
    line = f_of_x(x)
    F = np.empty(cfg.shape)
    F[...] = line
    return F


@pytest.mark.parametrize("m", list(range(0, 9)))
def test_flux_difference_exact_on_polynomials_up_to_degree_8(m):
    """On point values of a polynomial of degree <= 8 the conservative MP-9
    difference equals p f'(x_s) exactly (when the limiter does not clip).
    The data (x + 3)^m are monotone and convex on [0, 1], well resolved."""
    S = 40
    cfg = _cfg1(S, bc=O.OUTFLOW)
    F = _plane_field(cfg, lambda x: (x + 3.0) ** m)
    VF = O.advect(cfg, F)
    px, _ = O.velocities(cfg)
    x = (np.arange(S) + 0.5) / S
    exact_deriv = m * (x + 3.0) ** (m - 1) if m > 0 else np.zeros(S)
    inner = slice(6, S - 6)  # away from the ghost-node boundary closure
    scale = 4.0 ** m * S
    for v in range(cfg.planes):
        np.testing.assert_allclose(VF[v, inner], px[v] * exact_deriv[inner],
                                   rtol=0, atol=1e-13 * scale)


def test_flux_difference_not_exact_at_degree_9():
    """Control: degree 9 is not reproduced (the stencil is 9th order, no more)."""
    S = 40
    cfg = _cfg1(S, bc=O.OUTFLOW)
    F = _plane_field(cfg, lambda x: (x + 3.0) ** 9)
    VF = O.advect(cfg, F)
    px, _ = O.velocities(cfg)
    x = (np.arange(S) + 0.5) / S
    exact = 9 * (x + 3.0) ** 8
    v = int(np.argmax(px))
    err = np.abs(VF[v, 6:-6] - px[v] * exact[6:-6]).max()
    assert err > 1e-8


def test_ninth_order_convergence_on_smooth_wave():
    """Max error of (p dF/dx) on sin(2 pi x + 0.3) falls at order ~9 (the MP
    limiter keeps the accuracy at smooth extrema)."""
    errs = []
    Ns = [16, 32, 64]
    for S in Ns:
        cfg = _cfg1(S)
        F = _plane_field(cfg, lambda x: np.sin(2 * np.pi * x + 0.3))
        VF = O.advect(cfg, F)
        px, _ = O.velocities(cfg)
        x = (np.arange(S) + 0.5) / S
        exact = 2 * np.pi * np.cos(2 * np.pi * x + 0.3)
        v = int(np.argmax(px))
        errs.append(np.abs(VF[v] / px[v] - exact).max())
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders) > 8.5, (errs, orders)
    assert errs[0] < 5e-6


def test_zero_velocity_plane_has_no_flux():
    cfg = _cfg1(24, qp=5, qc=3)  # Q = 5 and Q = 3 both contain the node p = 0
    rng = np.random.default_rng(1)
    F = rng.uniform(0.5, 1.5, cfg.shape)
    VF = O.advect(cfg, F)
    px, _ = O.velocities(cfg)
    for v in np.where(px == 0.0)[0]:
        assert np.all(VF[v] == 0.0)


def test_periodic_flux_telescopes():
    """Periodic boundaries: sum_s (VF)_s = 0 for every plane (conservation)."""
    cfg = _cfg1(37)
    rng = np.random.default_rng(2)
    F = rng.uniform(0.0, 1.0, cfg.shape)
    VF = O.advect(cfg, F)
    assert np.abs(VF.sum(axis=1)).max() < 1e-11


def test_outflow_uniform_state_has_no_flux():
    cfg = _cfg1(20, bc=O.OUTFLOW)
    F = np.full(cfg.shape, 0.37)
    assert np.all(O.advect(cfg, F) == 0.0)


def test_mirror_symmetry_negative_velocity():
    """Mirroring x -> 1 - x maps the plane of velocity +p onto -p: the
    operator applied to mirrored data is the mirrored (negated) result."""
    cfg = _cfg1(31, bc=O.OUTFLOW)
    rng = np.random.default_rng(3)
    F = rng.uniform(0.0, 1.0, cfg.shape)
    px, _ = O.velocities(cfg)
    # plane permutation that reverses each axis' node order
    perm = np.concatenate([np.arange(cfg.q_phi)[::-1], cfg.q_phi + np.arange(cfg.q_chi)[::-1]])
    np.testing.assert_array_equal(px[perm], -px)
    Fm = F[perm][:, ::-1]
    VF = O.advect(cfg, F)
    VFm = O.advect(cfg, Fm)
    # d/dx of the mirrored field is minus the mirrored derivative, and the
    # velocity is negated: (p dF/dx) is mirrored without sign change.
    np.testing.assert_allclose(VFm, VF[perm][:, ::-1], rtol=1e-13, atol=1e-13)


def _rk3_pure_advection(cfg, F, dt, steps):
    for _ in range(steps):
        u1 = F - dt * O.advect(cfg, F)
        u2 = 0.75 * F + 0.25 * (u1 - dt * O.advect(cfg, u1))
        F = F / 3.0 + 2.0 / 3.0 * (u2 - dt * O.advect(cfg, u2))
    return F


def test_step_advection_creates_no_new_extrema():
    """The MP property: advecting a square pulse (SSP-RK3, CFL 0.2) creates
    no over- or undershoots, while the unlimited 9-point interpolation
    would."""
    S = 64
    cfg = _cfg1(S)
    x = (np.arange(S) + 0.5) / S
    pulse = np.where((x > 0.3) & (x < 0.6), 1.0, 0.0)
    F = np.empty(cfg.shape)
    F[...] = pulse
    px, _ = O.velocities(cfg)
    dt = 0.2 / S / np.abs(px).max()
    F = _rk3_pure_advection(cfg, F, dt, 30)
    assert F.min() > -1e-12 and F.max() < 1 + 1e-12
    # and the pulse has moved: the fastest plane's centre of mass shifted
    v = int(np.argmax(px))
    com0 = np.sum(x * pulse) / pulse.sum()
    com = np.sum(x * F[v]) / F[v].sum()
    assert com - com0 == pytest.approx(px[v] * dt * 30, rel=1e-2)


def test_mp9_face_uniform_and_linear():
    """Constant data give the constant; linear data give the midpoint value."""
    assert O.mp9_face(np.full(9, 0.7)) == 0.7
    f = 0.25 * np.arange(9) + 1.0  # F_{s+j-4}, exact face value F(s + 1/2)
    assert O.mp9_face(f) == pytest.approx(1.0 + 0.25 * 4.5, rel=1e-15)


def test_mp9_face_at_a_jump_is_the_upwind_value():
    """At a jump the limiter returns the upwind node's value exactly (both
    limits collapse onto it; derivations in test_oracle_mp9_pins.py), and a
    scaled and shifted jump gives the scaled and shifted value."""
    assert O.mp9_face(np.array([0, 0, 0, 0, 0, 1, 1, 1, 1], dtype=float)) == 0.0
    assert O.mp9_face(np.array([1, 1, 1, 1, 1, 0, 0, 0, 0], dtype=float)) == 1.0
    assert O.mp9_face(np.array([3, 3, 3, 3, 3, 7, 7, 7, 7], dtype=float)) == 3.0
    assert O.mp9_face(np.array([7, 7, 7, 7, 7, 3, 3, 3, 3], dtype=float)) == 7.0


def test_2d_advection_is_sum_of_axis_operators():
    """Dimensionally unsplit: a field varying only in x gives the 1D x-result
    in every row; one varying only in y gives the 1D y-result per column."""
    nx, ny = 23, 17
    cfg2 = O.Config(d=2, nx=nx, ny=ny, q_phi=4, q_chi=2, bc_x=O.OUTFLOW, bc_y=O.PERIODIC)
    px, py = O.velocities(cfg2)
    rng = np.random.default_rng(4)
    fx = rng.uniform(0, 1, nx)
    F = np.empty(cfg2.shape)
    F[...] = fx[None, None, :]
    VF = O.advect(cfg2, F)
    # reference: 1D operator along x with a single plane of the same velocity
    for v in range(cfg2.planes):
        c1 = O.Config(d=1, nx=nx, q_phi=4, q_chi=2, bc_x=O.OUTFLOW)
        p1, _ = O.velocities(c1)
        # pick the 1D plane with the same x-velocity
        v1 = int(np.where(p1 == px[v])[0][0])
        F1 = np.empty(c1.shape)
        F1[...] = fx
        ref = O.advect(c1, F1)[v1]
        np.testing.assert_array_equal(VF[v], np.broadcast_to(ref, (ny, nx)))
    fy = rng.uniform(0, 1, ny)
    F[...] = fy[None, :, None]
    VF = O.advect(cfg2, F)
    c1 = O.Config(d=1, nx=ny, q_phi=4, q_chi=2, bc_x=O.PERIODIC)
    p1, _ = O.velocities(c1)
    F1 = np.empty(c1.shape)
    F1[...] = fy
    ref1 = O.advect(c1, F1)
    for v in range(cfg2.planes):
        v1 = int(np.where(p1 == py[v])[0][0])
        np.testing.assert_array_equal(VF[v], np.broadcast_to(ref1[v1][:, None], (ny, nx)))
