"""Pins of the oracle's velocity space: Gauss-Hermite quadrature, the
truncated Hermite equilibria and the moments (Sec. II of the paper).

Each expected value here comes from closed-form mathematics (moments of a
standard normal, moments of a Gaussian N(u, T)) or from a library routine
(numpy's probabilists' Gauss-Hermite rule) -- never from the oracle itself.
"""
import math

import numpy as np
import numpy.polynomial.hermite_e as herme
import pytest

import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore")


def double_factorial(n):
    return 1 if n <= 0 else n * double_factorial(n - 2)


@pytest.mark.parametrize("Q", list(range(1, 21)))
def test_quadrature_moments_exact(Q):
    """sum_k w_k p_k^m equals the standard-normal moment (m-1)!! (even m)
    or 0 (odd m) for every m <= 2Q - 1 (Gauss rule exactness)."""
    p, w = O.gauss_hermite(Q)
    assert np.all(np.diff(p) > 0)
    for m in range(0, 2 * Q):
        exact = 0.0 if m % 2 else float(double_factorial(m - 1))
        got = float(np.sum(w * p ** m))
        scale = float(np.sum(w * np.abs(p) ** m))  # size of the summands
        assert got == pytest.approx(exact, rel=1e-12, abs=1e-14 * scale), (Q, m)


@pytest.mark.parametrize("Q", list(range(1, 21)))
def test_quadrature_matches_library_rule(Q):
    """Nodes/weights equal numpy's probabilists' Gauss-Hermite rule, whose
    weights are normalised here by sqrt(2 pi) so that they sum to one."""
    x, wl = herme.hermegauss(Q)
    p, w = O.gauss_hermite(Q)
    np.testing.assert_allclose(p, x, rtol=0, atol=1e-13)
    np.testing.assert_allclose(w, wl / math.sqrt(2 * math.pi), rtol=1e-12, atol=1e-15)


def test_quadrature_q3_closed_form():
    p, w = O.gauss_hermite(3)
    np.testing.assert_allclose(p, [-math.sqrt(3), 0.0, math.sqrt(3)], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 6, 2 / 3, 1 / 6], rtol=1e-14)


def test_quadrature_q5_closed_form():
    """He_5 = x^5 - 10 x^3 + 15 x, so the nodes are 0 and +-sqrt(5 -+ sqrt 10).
    With a = x^2 at a nonzero node, a^2 = 10 a - 15 reduces
    He_6 = x^6 - 15 x^4 + 45 x^2 - 15 to 60 - 20 a, hence
    w = 5!/He_6^2 = 3/(10 (3 - a)^2): (7 + 2 sqrt 10)/60 at a = 5 - sqrt 10,
    (7 - 2 sqrt 10)/60 at a = 5 + sqrt 10, and 120/225 = 8/15 at x = 0."""
    r = math.sqrt(10.0)
    inner, outer = math.sqrt(5 - r), math.sqrt(5 + r)
    p, w = O.gauss_hermite(5)
    np.testing.assert_allclose(p, [-outer, -inner, 0.0, inner, outer], rtol=0, atol=2e-15)
    np.testing.assert_allclose(w, [(7 - 2 * r) / 60, (7 + 2 * r) / 60, 8 / 15,
                                   (7 + 2 * r) / 60, (7 - 2 * r) / 60], rtol=1e-14)


def gaussian_moment(m, u, T):
    """E[X^m] for X ~ N(u, T): sum_j C(m, j) u^(m-j) T^(j/2) (j-1)!! over even j."""
    return sum(math.comb(m, j) * u ** (m - j) * T ** (j // 2) * double_factorial(j - 1)
               for j in range(0, m + 1, 2))


@pytest.mark.parametrize("Q", [3, 4, 5, 8, 12, 16])
def test_equilibrium_factor_reproduces_gaussian_moments(Q):
    """The truncated expansion reproduces the moments of N(u, T) exactly up
    to order Q - 1 (the exactness property stated in Sec. II)."""
    rng = np.random.default_rng(Q)
    p, _ = O.gauss_hermite(Q)
    for _ in range(5):
        u = rng.uniform(-1.0, 1.0)
        T = rng.uniform(0.3, 2.0)
        g = O.g_factor(Q, u, T)
        for m in range(Q):
            exact = gaussian_moment(m, u, T)
            scale = float(np.sum(np.abs(g) * np.abs(p) ** m))
            assert float(np.sum(g * p ** m)) == pytest.approx(exact, rel=1e-11,
                                                              abs=1e-13 * scale), (Q, m)


@pytest.mark.parametrize("Q", [3, 5, 8, 16])
def test_equilibrium_at_rest_reference_temperature_is_weights(Q):
    """u = 0, T = 1: every l >= 1 term vanishes, so g_k = w_k exactly."""
    _, w = O.gauss_hermite(Q)
    np.testing.assert_array_equal(O.g_factor(Q, 0.0, 1.0), w)


def test_equilibrium_order_q_moment_is_not_exact():
    """Control: the order-Q moment is NOT reproduced (truncation is real)."""
    Q, u, T = 5, 0.7, 1.3
    p, _ = O.gauss_hermite(Q)
    g = O.g_factor(Q, u, T)
    assert abs(np.sum(g * p ** Q) - gaussian_moment(Q, u, T)) > 1e-3


@pytest.mark.parametrize("d,qp,qc,K", [(1, 5, 3, 2), (1, 8, 8, 0), (1, 3, 1, 2),
                                       (2, 5, 3, 2), (2, 8, 8, 2), (2, 4, 2, 0)])
def test_moments_of_equilibrium_round_trip(d, qp, qc, K):
    """moments(equilibrium(n, u, T)) = (n, u, T): the discrete equilibria
    carry the given density, velocity and temperature, with the chi
    populations holding the (K + D - d)/2 n T internal/transverse energy."""
    shape = (7,) if d == 1 else (3, 5)
    rng = np.random.default_rng(d * 100 + qp)
    n = rng.uniform(0.2, 2.0, shape)
    ux = rng.uniform(-0.8, 0.8, shape)
    uy = rng.uniform(-0.8, 0.8, shape)
    T = rng.uniform(0.4, 1.8, shape)
    cfg = O.Config(d=d, nx=shape[-1], ny=shape[0] if d == 2 else 1, q_phi=qp, q_chi=qc, K=K)
    F = O.equilibrium(cfg, n, ux, uy if d == 2 else None, T)
    mn, mux, muy, mT = O.moments(cfg, F)
    np.testing.assert_allclose(mn, n, rtol=1e-13)
    np.testing.assert_allclose(mux, ux, rtol=0, atol=1e-13)
    if d == 2:
        np.testing.assert_allclose(muy, uy, rtol=0, atol=1e-13)
    np.testing.assert_allclose(mT, T, rtol=1e-13)


@pytest.mark.parametrize("d", [1, 2])
def test_energy_split_between_phi_and_chi(d):
    """sum_q chi_q = (K + D - d) n T and sum_k phi_k |p_k - u|^2 = d n T."""
    K = 2
    cfg = O.Config(d=d, nx=3, ny=2 if d == 2 else 1, q_phi=6, q_chi=4, K=K)
    shape = cfg.field_shape
    n = np.full(shape, 1.3)
    ux = np.full(shape, 0.25)
    uy = np.full(shape, -0.4)
    T = np.full(shape, 0.9)
    F = O.equilibrium(cfg, n, ux, uy if d == 2 else None, T)
    px, py = O.velocities(cfg)
    nphi = cfg.q_phi ** d
    chi_sum = F[nphi:].sum(axis=0)
    np.testing.assert_allclose(chi_sum, (K + 3 - d) * 1.3 * 0.9, rtol=1e-13)
    xi2 = (px[:nphi] - 0.25) ** 2 + ((py[:nphi] + 0.4) ** 2 if d == 2 else 0.0)
    phi_e = np.tensordot(xi2, F[:nphi], axes=(0, 0))
    np.testing.assert_allclose(phi_e, d * 1.3 * 0.9, rtol=1e-13)


def test_plane_ordering_and_velocities():
    """phi planes first with kx fastest, then chi planes."""
    cfg = O.Config(d=2, nx=1, ny=1, q_phi=3, q_chi=2)
    px, py = O.velocities(cfg)
    pp, _ = O.gauss_hermite(3)
    pc, _ = O.gauss_hermite(2)
    np.testing.assert_array_equal(px[:9], np.tile(pp, 3))
    np.testing.assert_array_equal(py[:9], np.repeat(pp, 3))
    np.testing.assert_array_equal(px[9:], np.tile(pc, 2))
    np.testing.assert_array_equal(py[9:], np.repeat(pc, 2))
