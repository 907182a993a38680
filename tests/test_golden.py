"""Pins against values printed in the paper (Table I, Sec. V) or in a cited
textbook (exact Sod star state), read from tests/golden/."""
import numpy as np
import pytest

from golden_data import riemann2d, sod_star, table1
from paper_1909_08390_amd import workloads as W
from riemann_exact import sample as riemann_sample
from riemann_exact import star_state


def tableaux():
    c = table1()
    a, b, e = c["alpha"], c["beta"], c["eta"]
    A = np.array([[a, 0, 0, 0], [-a, a, 0, 0], [0, 1 - a, a, 0], [b, e, 0.5 - b - e - a, a]])
    At = np.array([[0, 0, 0, 0], [0, 0, 0, 0], [0, 1, 0, 0], [0, 0.25, 0.25, 0]])
    w = np.array([0, 1 / 6, 1 / 6, 2 / 3])
    return A, At, w


def test_table1_constants_give_a_third_order_imex_pair():
    """Order conditions up to 3 of each tableau and the coupling conditions
    of the pair (shared weights), at the printed 14 digits."""
    A, At, w = tableaux()
    c, ct = A.sum(1), At.sum(1)
    for M, cc in ((A, c), (At, ct)):
        assert w.sum() == pytest.approx(1.0, abs=1e-14)
        assert w @ cc == pytest.approx(0.5, abs=1e-13)
        assert w @ cc ** 2 == pytest.approx(1 / 3, abs=1e-13)
        assert w @ M @ cc == pytest.approx(1 / 6, abs=1e-13)
    assert w @ At @ c == pytest.approx(1 / 6, abs=1e-13)
    assert w @ A @ ct == pytest.approx(1 / 6, abs=1e-13)
    assert w @ (c * ct) == pytest.approx(1 / 3, abs=1e-13)
    # a planted error in any constant breaks the pair
    for k in ("alpha", "beta", "eta"):
        bad = dict(table1())
        bad[k] += 1e-6
        a, b, e = bad["alpha"], bad["beta"], bad["eta"]
        Ab = np.array([[a, 0, 0, 0], [-a, a, 0, 0], [0, 1 - a, a, 0], [b, e, 0.5 - b - e - a, a]])
        cb = Ab.sum(1)
        resid = [w @ Ab @ cb - 1 / 6, w @ cb ** 2 - 1 / 3, w @ At @ cb - 1 / 6, w @ (cb * ct) - 1 / 3]
        assert max(abs(r) for r in resid) > 1e-8


def test_implicit_tableau_is_l_stable_and_diagonally_implicit():
    A, _, w = tableaux()
    assert np.allclose(np.triu(A, 1), 0.0)
    z = -1e8
    R = 1.0 + z * w @ np.linalg.solve(np.eye(4) - z * A, np.ones(4))
    assert abs(R) < 1e-6


def test_exact_riemann_solver_reproduces_tabulated_sod_star_state():
    g = sod_star()
    p, u = star_state(W.SOD_LEFT, W.SOD_RIGHT, 1.4)
    assert p == pytest.approx(g["p_star"], abs=6e-6)
    assert u == pytest.approx(g["u_star"], abs=6e-6)
    # densities either side of the contact (x/t = u*), at t = 1
    x = np.array([u - 1e-9, u + 1e-9])
    rho, _, _ = riemann_sample(W.SOD_LEFT, W.SOD_RIGHT, 1.4, x)
    assert rho[0] == pytest.approx(g["rho_star_left"], abs=6e-6)
    assert rho[1] == pytest.approx(g["rho_star_right"], abs=6e-6)


def test_workload_states_are_the_printed_ones():
    r = riemann2d()
    for c in (11, 12):
        assert W.LAX_LIU[c] == r[c]["states"]
    # Sod: rho_L = P_L = T_L = 1, rho_R = 0.125, P_R = 0.1, T_R = 0.8 (Sec. V)
    n, u, T = W.sod_1d(400)
    assert (n[0], u[0], T[0]) == (1.0, 0.0, 1.0)
    assert (n[-1], u[-1]) == (0.125, 0.0)
    assert T[-1] == pytest.approx(0.8, rel=1e-15)
