"""Pins of the AIM oracle, eq. (11): stencils P, grid convolution H, W = P^T, L_NR."""
import numpy as np
import pytest

from inputs.geometry import random_complex, small_boxes
from oracle import aim
from oracle.operators import Physics, external_dense
from oracle.quad import tri_points
from oracle.rwg import build_rwg


@pytest.fixture(scope="module")
def boxes():
    m = small_boxes(4, seed=1)
    g = build_rwg(m.verts, m.tris, m.obj, m.n_obj)
    ph = Physics(10e9)
    LA, Lphi = external_dense(g, ph)
    return g, ph, LA, Lphi


def test_moment_exactness(boxes):
    """Stencil weights reproduce every moment ((r - r0)/h)^alpha, alpha_c <= 2, of every
    basis function, recomputed here with a different (higher) rule and without the
    oracle's linear solve; the tolerance is relative to the largest moment of the
    basis function."""
    g = boxes[0]
    for N in ((12, 11, 10), (16, 16, 16)):
        grid = aim.make_grid(g.verts, N)
        cE, wE, cT, wT = aim.stencil_weights(grid, g)
        pts, w = tri_points(g.verts[g.tris], 8)
        mono_nodes = np.prod(aim.OFFS[None, :, :].astype(float) ** aim.ALPHAS[:, None, :], axis=2)   # (alpha, node)
        for n in range(g.n_e):
            r0 = grid.node_pos(cE[n])
            rhs = np.zeros((3, 27))
            for t in (g.tplus[n], g.tminus[n]):
                i = int(np.nonzero(g.tri_edge[t] == n)[0][0])
                f = g.tri_sign[t, i] * g.length[n] / (2 * g.area[t]) * (pts[t] - g.verts[g.tris[t, i]])
                mono = np.prod(((pts[t] - r0) / grid.h)[:, None, :] ** aim.ALPHAS[None], axis=2)   # (q, alpha)
                rhs += np.einsum('q,qc,qa->ca', w[t], f, mono)
            lhs = wE[n] @ mono_nodes.T
            assert np.abs(lhs - rhs).max() <= 1e-10 * np.abs(rhs).max()
        for t in range(g.n_t):
            r0 = grid.node_pos(cT[t])
            mono = np.prod(((pts[t] - r0) / grid.h)[:, None, :] ** aim.ALPHAS[None], axis=2)
            rhs = w[t] @ mono / g.area[t]
            assert np.abs(wT[t] @ mono_nodes.T - rhs).max() <= 1e-10 * np.abs(rhs).max()


@pytest.mark.parametrize("N", [(4, 4, 4), (5, 4, 6), (8, 3, 5)])
def test_fft_convolution_equals_direct_sum(N):
    grid = aim.Grid(np.array(N), np.array([1.1e-6, 0.9e-6, 1.3e-6]), np.zeros(3))
    k0 = 2 * np.pi * 10e9 / 299792458.0
    s = random_complex(int(np.prod(N)), seed=3)
    Ghat = np.fft.fftn(aim.circulant_kernel(grid, k0))
    a = aim.convolve_fft(grid, Ghat, s)
    b = aim.convolve_direct(grid, k0, s)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_precorrection_makes_near_entries_exact(boxes):
    g, ph, LA, Lphi = boxes
    grid = aim.make_grid(g.verts, (10, 10, 10))
    op = aim.build_aim(g, grid, ph.k0, lambda a, b: LA[a, b], lambda a, b: Lphi[a, b])
    cE, wE, cT, wT = aim.stencil_weights(grid, g)
    m, n = aim.near_pairs(cE, cE)
    gp = aim.grid_part(grid, ph.k0, cE, wE, cE, wE, m, n)
    assert np.abs(np.asarray(op.LA_nr[m, n]).ravel() + gp - LA[m, n]).max() <= 1e-12 * np.abs(LA).max()
    # the full grid part of a near pair, applied through the FFT path, equals gp
    j = np.zeros(g.n_e, dtype=complex)
    j[n[5]] = 1.0
    far = sum(P.T @ aim.convolve_fft(grid, op.Ghat, P @ j) for P in op.Pc)
    assert abs(far[m[5]] - gp[5]) <= 1e-10 * abs(gp[5])


def test_aim_far_field_accuracy(boxes):
    """For separated basis pairs the grid interaction approaches the exact entry."""
    g, ph, LA, Lphi = boxes
    grid = aim.make_grid(g.verts, (10, 10, 10))
    cE, wE, cT, wT = aim.stencil_weights(grid, g)
    m, n = np.meshgrid(np.arange(g.n_e), np.arange(g.n_e), indexing='ij')
    m, n = m.ravel(), n.ravel()
    cheb = np.abs(cE[m] - cE[n]).max(axis=1)
    errs = []
    for lo, hi in ((4, 5), (6, 7)):
        sel = np.nonzero((cheb >= lo) & (cheb <= hi))[0][:3000]
        gp = aim.grid_part(grid, ph.k0, cE, wE, cE, wE, m[sel], n[sel])
        ex = LA[m[sel], n[sel]]
        errs.append(np.linalg.norm(gp - ex) / np.linalg.norm(ex))
    assert errs[0] < 2e-2 and errs[1] < errs[0]


def test_aim_matvec_close_to_dense(boxes):
    g, ph, LA, Lphi = boxes
    grid = aim.make_grid(g.verts, (10, 10, 10))
    op = aim.build_aim(g, grid, ph.k0, lambda a, b: LA[a, b], lambda a, b: Lphi[a, b])
    j, q = random_complex(g.n_e, 1), random_complex(g.n_t, 2)
    assert np.linalg.norm(op.apply_LA(j) - LA @ j) <= 5e-3 * np.linalg.norm(LA @ j)
    assert np.linalg.norm(op.apply_Lphi(q) - Lphi @ q) <= 5e-3 * np.linalg.norm(Lphi @ q)
