"""Hand-worked pins of the oracle's MP-9 limiter and outflow ghost nodes
(Sec. IV of the paper).

Every expected value below was derived by hand from the formulas of Sec. IV
on small integer windows; each docstring carries the derivation, so a reader
can check it against the paper line by line.  Notation: the window is
f = (F_{s-4}, ..., F_{s+4}) for the face s+1/2 of a positive velocity,
C_j = F_{j+1} - 2 F_j + F_{j-1}, alpha_MP = 4,
  F^L  = (4, -41, 199, -641, 1879, 1375, -305, 55, -5) . f / 2520,
  F^MP = F_s + mm(F_{s+1} - F_s, 4 (F_s - F_{s-1})),
  F^UL = F_s + 4 (F_s - F_{s-1}),
  F^LC = F_s + (F_s - F_{s-1})/2 + (4/3) mm4(4C_s - C_{s-1}, 4C_{s-1} - C_s, C_s, C_{s-1}),
  F^MD = (F_s + F_{s+1} - mm4(4C_s - C_{s+1}, 4C_{s+1} - C_s, C_s, C_{s+1}))/2,
  F^min = max(min(F_s, F_{s+1}, F^MD), min(F_s, F^UL, F^LC)),
  F^max = min(max(F_s, F_{s+1}, F^MD), max(F_s, F^UL, F^LC)),
and the face is F^L when (F^L - F_s)(F^L - F^MP) <= 0, else
F^L + mm(F^min - F^L, F^max - F^L).

The cases are chosen so that a plausible misreading fails at least one of
them: alpha_MP = 2, a 1/2 in place of 4/3 in F^LC, a 1/2 in place of
alpha_MP in F^UL, a wrong F^MD, and outflow ghosts copied from the second
node instead of the boundary node.  (alpha_MP inside F^MP alone cannot be
pinned by any input: F^MP always lies in [F^min, F^max], so the test only
decides whether F^L is returned as is or clipped into an interval that
already contains it.)
"""
import numpy as np
import pytest

import oracle as O


def test_face_accepted_by_monotonicity_test():
    """f = (0, 0, 5, 5, 4, 0, 5, 4, 1): F_s = 4, F_{s+1} = 0, F_{s-1} = 5.

    F^L = (995 - 3205 + 7516 - 1525 + 220 - 5)/2520 = 3996/2520 = 111/70.
    F^MP = 4 + mm(-4, 4 * (-1)) = 4 - 4 = 0.
    (F^L - F_s)(F^L - F^MP) = (111/70 - 4)(111/70) < 0, so the face is F^L.

    With alpha_MP = 2 instead: F^MP = 4 + mm(-4, -2) = 2 and the test is
    positive; C_{s-1} = -1, C_s = -3, C_{s+1} = 9; F^UL = 2,
    F^LC = 4 - 1/2 + (4/3) mm4(-11, -1, -3, -1) = 13/6, F^MD = 2 (its
    minmod4 has mixed signs), so F^min = max(0, 2) = 2 and the face would
    be 2."""
    assert O.mp9_face([0, 0, 5, 5, 4, 0, 5, 4, 1]) == pytest.approx(111 / 70, rel=2e-16, abs=0)


def test_face_clipped_to_upper_limit():
    """f = (0, 1, 1, 0, 1, 8, 1, 2, 0): F_s = 1, F_{s+1} = 8, F_{s-1} = 0.

    F^L = (-41 + 199 + 1879 + 11000 - 305 + 110)/2520 = 12842/2520 = 6421/1260
    (about 5.096).  F^MP = 1 + mm(7, 4) = 5, and (F^L - 1)(F^L - 5) > 0: clip.
    C_{s-1} = 2, C_s = 6, C_{s+1} = -14.
    F^UL = 1 + 4 * 1 = 5.
    F^LC = 1 + 1/2 + (4/3) mm4(22, 2, 6, 2) = 3/2 + 8/3 = 25/6.
    F^MD = (1 + 8 - mm4(38, -62, 6, -14))/2 = 9/2.
    F^min = max(min(1, 8, 9/2), min(1, 5, 25/6)) = 1,
    F^max = min(max(1, 8, 9/2), max(1, 5, 25/6)) = min(8, 5) = 5 = F^UL.
    Face = F^L + mm(1 - F^L, 5 - F^L) = 5.

    With alpha_MP = 2 (or 1/2 in F^UL) the upper limit is F^LC = 25/6."""
    assert O.mp9_face([0, 1, 1, 0, 1, 8, 1, 2, 0]) == 5.0


def test_face_clipped_to_lower_limit_from_curvature_bound():
    """f = (3, 4, 0, 3, 5, 4, 4, 3, 3): F_s = 5, F_{s+1} = 4, F_{s-1} = 3.

    F^L = (12 - 164 - 1923 + 9395 + 5500 - 1220 + 165 - 15)/2520
        = 11750/2520 = 1175/252 (about 4.6627).
    F^MP = 5 + mm(-1, 8) = 5; (F^L - 5)^2 > 0: clip.
    C_{s-1} = -1, C_s = -3, C_{s+1} = 1.
    F^UL = 5 + 4 * 2 = 13.
    F^LC = 5 + 1 + (4/3) mm4(-11, -1, -3, -1) = 6 - 4/3 = 14/3.
    F^MD = (5 + 4 - mm4(-13, 7, -3, 1))/2 = 9/2.
    F^min = max(min(5, 4, 9/2), min(5, 13, 14/3)) = max(4, 14/3) = 14/3 = F^LC,
    F^max = min(max(5, 4, 9/2), max(5, 13, 14/3)) = 5.
    Face = F^L + mm(14/3 - F^L, 5 - F^L) = 14/3 (both differences positive,
    the first smaller).

    With 1/2 in place of 4/3: F^LC = 11/2, F^min = 5 and the face would be 5."""
    assert O.mp9_face([3, 4, 0, 3, 5, 4, 4, 3, 3]) == pytest.approx(14 / 3, rel=4e-16, abs=0)


def test_face_clipped_to_median_bound():
    """f = (2, 0, 1, 2, 0, 0, 1, 2, 2): F_s = 0, F_{s+1} = 0, F_{s-1} = 2.

    F^L = (8 + 199 - 1282 - 305 + 110 - 10)/2520 = -1280/2520 = -32/63.
    F^MP = 0 + mm(0, -8) = 0; (F^L)^2 > 0: clip.
    C_{s-1} = -3, C_s = 2, C_{s+1} = 1.
    F^UL = 0 + 4 * (-2) = -8.
    F^LC = 0 - 1 + (4/3) mm4(11, -14, 2, -3) = -1.
    F^MD = (0 + 0 - mm4(7, 2, 2, 1))/2 = -1/2.
    F^min = max(min(0, 0, -1/2), min(0, -8, -1)) = -1/2 = F^MD,
    F^max = min(max(0, 0, -1/2), max(0, -8, -1)) = 0.
    Face = F^L + mm(-1/2 - F^L, -F^L) = -1/2: the median bound lets the face
    leave [F_s, F_{s+1}] where the data curve."""
    assert O.mp9_face([2, 0, 1, 2, 0, 0, 1, 2, 2]) == -0.5


def test_face_inside_limits_keeps_linear_value():
    """f = (4, 3, 5, 3, 3, 5, 4, 3, 3): F_s = 3, F_{s+1} = 5, F_{s-1} = 3.

    F^L = (16 - 123 + 995 - 1923 + 5637 + 6875 - 1220 + 165 - 15)/2520
        = 10407/2520 = 3469/840 (about 4.1298).
    F^MP = 3 + mm(2, 0) = 3; (F^L - 3)^2 > 0: clip.
    C_{s-1} = 2, C_s = 2, C_{s+1} = -3.
    F^UL = 3, F^LC = 3 + (4/3) mm4(6, 6, 2, 2) = 17/3,
    F^MD = (3 + 5 - mm4(11, -14, 2, -3))/2 = 4.
    F^min = max(3, 3) = 3, F^max = min(5, 17/3) = 5; F^L lies inside, so
    mm(3 - F^L, 5 - F^L) = 0 and the face is F^L.

    With 1/2 in place of 4/3: F^LC = 4, F^max = 4 and the face would be 4."""
    assert O.mp9_face([4, 3, 5, 3, 3, 5, 4, 3, 3]) == pytest.approx(3469 / 840, rel=2e-16, abs=0)


def test_face_at_upward_jump_is_upwind_value():
    """f = (0, 0, 0, 0, 0, 1, 1, 1, 1): F_s = 0, F_{s+1} = 1, F_{s-1} = 0.

    F^L = (1375 - 305 + 55 - 5)/2520 = 4/9; F^MP = 0 + mm(1, 0) = 0; clip.
    C_{s-1} = 0, C_s = 1, C_{s+1} = -1.  F^UL = 0, F^LC = 0 + (4/3) mm4(4, -1, 1, 0) = 0,
    F^MD = (0 + 1 - mm4(5, -5, 1, -1))/2 = 1/2.
    F^min = max(min(0, 1, 1/2), min(0, 0, 0)) = 0, F^max = min(1, 0) = 0.
    Face = 4/9 + mm(-4/9, -4/9) = 0 exactly: no undershoot or overshoot."""
    assert O.mp9_face([0, 0, 0, 0, 0, 1, 1, 1, 1]) == 0.0


def test_face_at_downward_jump_is_upwind_value():
    """f = (1, 1, 1, 1, 1, 0, 0, 0, 0): F_s = 1, F_{s+1} = 0, F_{s-1} = 1.

    F^L = (4 - 41 + 199 - 641 + 1879)/2520 = 5/9; F^MP = 1 + mm(-1, 0) = 1; clip.
    C_{s-1} = 0, C_s = -1, C_{s+1} = 1.  F^UL = 1, F^LC = 1 + (4/3) mm4(-4, 1, -1, 0) = 1,
    F^MD = (1 + 0 - mm4(-5, 5, -1, 1))/2 = 1/2.
    F^min = max(min(1, 0, 1/2), min(1, 1, 1)) = 1, F^max = min(1, 1) = 1.
    Face = 5/9 + mm(4/9, 4/9) = 1 exactly."""
    assert O.mp9_face([1, 1, 1, 1, 1, 0, 0, 0, 0]) == 1.0


def test_face_tie_returns_linear_value():
    """f = (41, 4, 0, 0, 0, 0, 0, 0, 0): F^L = (4 * 41 - 41 * 4)/2520 = 0 = F_s,
    so (F^L - F_s)(F^L - F^MP) = 0, the first case: the face is F^L = 0.  (The
    clip would give the same: every C near s is 0, so F^min = F^max = F_s.)"""
    assert O.mp9_face([41, 4, 0, 0, 0, 0, 0, 0, 0]) == 0.0


def test_outflow_boundary_cells_two_spikes():
    """Outflow line of S = 12 cells, F = (1, 0, ..., 0, 2), every plane the
    same line, so (VF)_s = p D_s with D_s = S (face_{s+1/2} - face_{s-1/2}).
    Ghost nodes copy the boundary node (Sec. IV, last paragraph): F_{-5..-1} = 1
    and F_{12..16} = 2.

    p > 0 (window F_{s-4..s+4}):
      face -1/2: (1, 1, 1, 1, 1, 1, 0, 0, 0): F_s = F_{s+1} = 1, so F^MP = 1 and
        F^L = 2775/2520 is clipped; C = (0, 0, -1) give F^UL = F^LC = F^MD = 1,
        F^min = F^max = 1: face 1.
      face 1/2: the downward jump (1, 1, 1, 1, 1, 0, 0, 0, 0): face 1.
      face 3/2: (1, 1, 1, 1, 0, 0, 0, 0, 0): F_s = F_{s+1} = 0, F_{s-1} = 1;
        C = (-1, 1, 0), F^UL = -4, F^LC = -1/2, F^MD = 0: F^min = F^max = 0.
      Faces further right are 0 up to face S-3/2, which is the upward jump
      (0, 0, 0, 0, 0, 2, 2, 2, 2): 0; face S-1/2: (0, 0, 0, 0, 2, 2, 2, 2, 2): 2.
      D = (0, -S, 0, ..., 0, 2S): the boundary cell keeps its value (inflow
      from its own copies balances the outflow).
    p < 0 (mirrored window F_{s+5}, ..., F_{s-3}): by the same windows reversed,
      face -1/2 = 1, face 1/2 = 0, faces 3/2 .. S-5/2 = 0, face S-3/2 = 2,
      face S-1/2 = 2: D = (-S, 0, ..., 0, 2S, 0).

    Ghosts copied from the second node instead (0 on both sides) would give
    face -1/2 = 0 for p > 0 (D_0 = S) and face S-1/2 = 0 for p < 0
    (D_{S-1} = -2S)."""
    S = 12
    cfg = O.Config(d=1, nx=S, lx=1.0, q_phi=3, q_chi=3, bc_x=O.OUTFLOW)
    line = np.zeros(S)
    line[0], line[-1] = 1.0, 2.0
    F = np.empty(cfg.shape)
    F[...] = line
    VF = O.advect(cfg, F)
    px, _ = O.velocities(cfg)
    Dpos = np.zeros(S)
    Dpos[1], Dpos[-1] = -S, 2 * S
    Dneg = np.zeros(S)
    Dneg[0], Dneg[-2] = -S, 2 * S
    for v in range(cfg.planes):
        if px[v] > 0:
            expect = px[v] * Dpos
        elif px[v] < 0:
            expect = px[v] * Dneg
        else:
            expect = np.zeros(S)
        np.testing.assert_allclose(VF[v], expect, rtol=1e-15, atol=0)


def test_outflow_2d_boundary_rows_and_columns():
    """The same two-spike line along y in a 2D outflow grid (every column
    holds it): the y-operator gives p_y D at each column; the x-operator sees
    rows of constant value and contributes nothing (its ghosts copy the
    same value)."""
    nx, S = 5, 12
    cfg = O.Config(d=2, nx=nx, ny=S, q_phi=3, q_chi=3, bc_x=O.OUTFLOW, bc_y=O.OUTFLOW)
    col = np.zeros(S)
    col[0], col[-1] = 1.0, 2.0
    F = np.empty(cfg.shape)
    F[...] = col[None, :, None]
    VF = O.advect(cfg, F)
    _, py = O.velocities(cfg)
    Dpos = np.zeros(S)
    Dpos[1], Dpos[-1] = -S, 2 * S
    Dneg = np.zeros(S)
    Dneg[0], Dneg[-2] = -S, 2 * S
    for v in range(cfg.planes):
        D = Dpos if py[v] > 0 else Dneg if py[v] < 0 else np.zeros(S)
        np.testing.assert_allclose(VF[v], np.broadcast_to((py[v] * D)[:, None], (S, nx)),
                                   rtol=1e-15, atol=0)
