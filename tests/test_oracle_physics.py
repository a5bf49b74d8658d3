"""Physics pins of the dense FP64 oracle on the copper bar (Sec. II; eq. (3)-(8))."""
import numpy as np
import pytest

from inputs.geometry import random_complex
from oracle.operators import MU0, Physics, interior_LK
from oracle.rwg import matrix_D, matrix_Ix_and_gram, project_tangential
from oracle.solve import gmres, lu_solve, row_scaling

pytestmark = pytest.mark.slow

A_SIDE, LENGTH, CURRENT = 2e-6, 100e-6, 1.0


def test_efie_elimination_identity(c1_system, c1_rwg):
    """Eliminating c0 rho from (3) must give the RWG EFIE matrix: L_A - D^T L_phi D / k0^2 = L_k0.

    Pins the signs and scalings read for D, B, F (B F = -I) against the
    independently assembled interior single-layer matrix at k = k0.
    """
    S = c1_system
    k0 = S.phys.k0
    L0, _ = interior_LK(c1_rwg, 0, k0)
    lhs = S.LA - S.D.T @ S.Lphi @ S.D / k0 ** 2
    assert np.abs(lhs - L0).max() <= 1e-12 * np.abs(L0).max()
    B, F = np.diag(c1_rwg.area), -np.diag(1.0 / c1_rwg.area)
    assert np.allclose(B @ F, -np.eye(c1_rwg.n_t))


def test_reciprocity(c1_system):
    S = c1_system
    L0, K0 = interior_LK(S.g, 0, S.phys.kc)
    for M in (S.LA, S.Lphi, L0, K0):
        assert np.abs(M - M.T).max() <= 1e-14 * np.abs(M).max()
    assert np.abs(S.Ix + S.Ix.T).max() <= 1e-14 * np.abs(S.Ix).max()


def test_matvec_equals_printed_system(c1_system):
    """The factored product (j = H - M H, ...) equals the matrix of (7) with C of (8),
    block by block (the blocks differ by many orders of magnitude in SI units)."""
    S = c1_system
    A = S.dense()
    ne = S.g.n_e
    for part in (slice(0, ne), slice(ne, None)):
        x = np.zeros(A.shape[0], dtype=complex)
        x[part] = random_complex(A.shape[0], seed=4)[part]
        y, _ = S.matvec(x)
        ref = A @ x
        for rows in (slice(0, ne), slice(ne, None)):
            assert np.linalg.norm(y[rows] - ref[rows]) <= 1e-12 * np.linalg.norm(ref[rows])
    # the internal coupling term alone: C H = (-j k0 L_A Y_eq + I_x/eta0) Z H
    H = random_complex(ne, seed=5)
    parts = S.matvec(np.concatenate([H, np.zeros(S.g.n_t)]))[1]
    CH = -1j * S.phys.k0 * S.LA @ parts['g'] + S.Ix @ parts['e'] / 299792458.0 / (4e-7 * np.pi)
    Cref = A[:ne, :ne] @ H - 1j * S.phys.k0 * S.LA @ H
    assert np.linalg.norm(CH - Cref) <= 1e-11 * np.linalg.norm(Cref)


def _bar_power(g, freq, h, Ix):
    ph = Physics(freq)
    Lc, Kc = interior_LK(g, 0, ph.kc)
    Z = (-1.0 / (1j * ph.omega * ph.eps_c)) * np.linalg.solve(Lc, Kc + 0.5 * Ix)
    e = Z @ h
    return -0.5 * np.real(e @ Ix @ np.conj(h)), Z, ph


@pytest.fixture(scope="module")
def bar_field(c1_rwg):
    """RWG coefficients of n x H for the interior field of a uniform axial current I."""
    g = c1_rwg
    J = CURRENT / A_SIDE ** 2

    def nxH(pts, t):
        H = np.zeros_like(pts)
        H[:, 1] = -J / 2 * pts[:, 2]
        H[:, 2] = J / 2 * pts[:, 1]
        return np.cross(g.normal[t][None, :], H)
    Ix, Gm = matrix_Ix_and_gram(g)
    h, _ = project_tangential(g, nxH)
    return h, Ix, Gm


def test_dc_resistance(c1_rwg, bar_field):
    """At 10 MHz (skin depth 21 um >> 2 um) the power into the bar is I^2 R_DC / 2, R_DC = l/(sigma A)."""
    h, Ix, _ = bar_field
    P, _, ph = _bar_power(c1_rwg, 1e7, h, Ix)
    r_dc = LENGTH / (ph.sigma * A_SIDE ** 2)
    assert abs(r_dc - 0.43103) < 1e-4
    assert abs(2 * P / CURRENT ** 2 / r_dc - 1) < 0.02


def test_skin_effect_sqrt_f(c1_rwg, bar_field):
    """For delta << 2 um the resistance follows the surface resistance R_s = sqrt(omega mu/(2 sigma)):
    R(f) = alpha sqrt(f) + beta (beta: the first-order corner/curvature correction, since
    R_s delta = 1/sigma), alpha within 5% of the Leontovich value, and the power
    ratio to Leontovich tends to 1 (within 10% at 400 GHz)."""
    h, Ix, Gm = bar_field
    f = np.array([1e11, 2e11, 4e11])
    R, ratio = [], []
    for fi in f:
        P, Z, ph = _bar_power(c1_rwg, fi, h, Ix)
        Rs = np.sqrt(ph.omega * MU0 / (2 * ph.sigma))
        Pl = 0.5 * Rs * np.real(np.conj(h) @ Gm @ h)
        R.append(2 * P)
        ratio.append(P / Pl)
    R, ratio = np.array(R), np.array(ratio)
    A = np.stack([np.sqrt(f), np.ones(3)], 1)
    coef, *_ = np.linalg.lstsq(A, R, rcond=None)
    assert np.abs(A @ coef - R).max() < 0.01 * R.max()
    alpha_leon = np.sqrt(np.pi * MU0 / 5.8e7) * np.real(np.conj(h) @ Gm @ h)   # R_s / sqrt(f) * int |H|^2
    assert abs(coef[0] / alpha_leon - 1) < 0.05
    slope = np.polyfit(np.log(f), np.log(R - coef[1]), 1)[0]
    assert abs(slope - 0.5) < 0.02
    assert np.all(np.diff(ratio) < 0) and 1.0 < ratio[-1] < 1.10


def test_passivity(c1_system, c1_mesh):
    """Power into the conductor, -Re(e^T I_x h*)/2 with e = Z h, is >= 0 for every h.

    The discrete form is not exactly semidefinite: testing with the rotated RWG functions
    (I_x) leaves one mode per mesh vertex that carries (almost) no power, and there the
    discretisation puts eigenvalues slightly below zero.  Their size does not fall under
    refinement (about -1.5 % of the largest on a cube at 1, 2 and 3 divisions per side,
    10 GHz), so the pin fixes the count of such modes and bounds the power they carry: the bar
    has exactly N_V = 298 of them at 1, 10 and 100 GHz, separated from the positive ones
    (largest negative -3e-6, smallest positive 1.6e-2 of the largest eigenvalue), together
    0.17 % of the positive power at 10 GHz; a flipped sign of Z makes 590 modes negative."""
    S = c1_system
    Z = S.inner.Z[0]
    Q = -(Z.conj().T @ S.Ix - S.Ix @ Z) / 2.0
    Q = (Q + Q.conj().T) / 2
    ev = np.linalg.eigvalsh(Q)
    neg = ev[ev < 0]
    assert neg.size == len(c1_mesh.verts)
    assert -neg.sum() <= 5e-3 * ev[ev > 0].sum()
    assert ev.min() >= -1e-2 * ev.max()


def test_gmres_matches_lu(c1_system):
    """GMRES on the equilibrated system S A x = r (r: seeded N(0,1) vector) reaches 1e-8 and
    agrees with the dense LU solution within the conditioning bound."""
    S = c1_system
    s = row_scaling(S.g.n_e, S.g.n_t, np.mean(S.g.length))
    A = s[:, None] * S.dense()
    r = random_complex(A.shape[0], seed=0)
    xs = lu_solve(A, r)
    op = lambda v: s * S.matvec(v)[0]
    x, it, hist = gmres(op, r, tol=1e-8, restart=300, max_iter=4000)
    assert hist[-1] <= 1e-8
    assert np.linalg.norm(op(x) - r) <= 1.0001e-8 * np.linalg.norm(r)
    cond = np.linalg.cond(A)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 10 * cond * 1e-8
