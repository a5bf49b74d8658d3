"""Pins of the oracle's layered-medium near field and layered AIM operator.

* Over a PEC ground, the reflected entries are the free-space kernel to the mirrored
  source with the image current (-J_x, -J_y, +J_z) and the image charge -q.  This is
  written out here with the same TRI(2) rule, so it checks the dyadic contraction and the
  RWG assembly of the reflected entries.
* Over the lossy substrate, the reflected L_A and L_phi are symmetric (reciprocity; this
  fixes G_xz = -G_zx in the contraction), and so is the reflected grid part.
* The layered AIM operator (precorrected near field + layered grid convolution) matches the
  dense layered operator to AIM accuracy.  A wrong sign or a missing cross term in the
  reflected grid part would leave an O(1) error on the near pairs.
"""
import numpy as np
import pytest

from inputs.geometry import box_mesh, merge
from oracle import aim, mgf
from oracle.quad import tri_points
from oracle.rwg import build_rwg

FREQ = 10e9
UM = 1e-6


@pytest.fixture(scope="module")
def two_boxes():
    m = merge([box_mesh((0.0, 0.0, 3 * UM), (4 * UM, 2 * UM, 2 * UM), (2, 1, 1)),
               box_mesh((6 * UM, 1 * UM, 2 * UM), (2 * UM, 2 * UM, 3 * UM), (1, 1, 1))])
    g = build_rwg(m.verts, m.tris, m.obj, m.n_obj)
    grid = aim.make_grid(g.verts, (8, 8, 8))
    return g, grid


def _image_entries(g, k0, z_if, m, n):
    """PEC ground: int int f_m . diag(-1,-1,1) f_n g(|r - M r'|), M mirrors z about z_if."""
    pts, w = tri_points(g.verts[g.tris], 2)
    M = np.array([-1.0, -1.0, 1.0])
    A = np.zeros(len(m), complex)
    for k, (mm, nn) in enumerate(zip(m, n)):
        for t in (g.tplus[mm], g.tminus[mm]):
            i = int(np.argmax(g.tri_edge[t] == mm))
            ft = g.tri_sign[t, i] * g.length[mm] / (2 * g.area[t]) * (pts[t] - g.verts[g.tris[t, i]])
            for u in (g.tplus[nn], g.tminus[nn]):
                j = int(np.argmax(g.tri_edge[u] == nn))
                fu = g.tri_sign[u, j] * g.length[nn] / (2 * g.area[u]) * (pts[u] - g.verts[g.tris[u, j]])
                img = pts[u].copy()
                img[:, 2] = 2 * z_if - img[:, 2]
                R = np.linalg.norm(pts[t][:, None, :] - img[None, :, :], axis=2)
                gk = np.exp(-1j * k0 * R) / (4 * np.pi * R)
                A[k] += np.einsum('p,q,pq,pa,qa->', w[t], w[u], gk, ft, fu * M)
    return A


def test_reflected_entries_pec_images(two_boxes):
    g, grid = two_boxes
    z_if = 0.5 * UM
    st = mgf.Stack([], "pec", z_if=z_if)
    k0 = 2 * np.pi * FREQ / mgf.C0
    rng = np.random.default_rng(0)
    m = rng.integers(0, g.n_e, 40)
    n = rng.integers(0, g.n_e, 40)
    got = aim.reflected_entries(g, FREQ, st, m, n)
    ref = _image_entries(g, k0, z_if, m, n)
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
    t = rng.integers(0, g.n_t, 30)
    u = rng.integers(0, g.n_t, 30)
    pts, w = tri_points(g.verts[g.tris], 2)
    ref_p = []
    for a, b in zip(t, u):
        img = pts[b].copy()
        img[:, 2] = 2 * z_if - img[:, 2]
        R = np.linalg.norm(pts[a][:, None, :] - img[None, :, :], axis=2)
        ref_p.append(-np.einsum('p,q,pq->', w[a], w[b], np.exp(-1j * k0 * R) / (4 * np.pi * R)) / (g.area[a] * g.area[b]))
    np.testing.assert_allclose(aim.reflected_phi_entries(g, FREQ, st, t, u), ref_p, rtol=1e-11)


@pytest.fixture(scope="module")
def reflected_dense(two_boxes):
    """Reflected L_A and L_phi over the lossy substrate on every pair (computed once)."""
    g, grid = two_boxes
    st = mgf.substrate_c4()
    st.z_if = grid.origin[2] - 1 * UM
    m, n = np.meshgrid(np.arange(g.n_e), np.arange(g.n_e), indexing='ij')
    LA = aim.reflected_entries(g, FREQ, st, m.ravel(), n.ravel()).reshape(g.n_e, g.n_e)
    t, u = np.meshgrid(np.arange(g.n_t), np.arange(g.n_t), indexing='ij')
    LP = aim.reflected_phi_entries(g, FREQ, st, t.ravel(), u.ravel()).reshape(g.n_t, g.n_t)
    return st, LA, LP


def test_reflected_operators_are_reciprocal(two_boxes, reflected_dense):
    g, grid = two_boxes
    st, LA, LP = reflected_dense
    m, n = np.meshgrid(np.arange(g.n_e), np.arange(g.n_e), indexing='ij')
    np.testing.assert_allclose(LA, LA.T, rtol=0, atol=1e-10 * np.abs(LA).max())
    assert np.abs(LA).max() > 0
    np.testing.assert_allclose(LP, LP.T, rtol=0, atol=1e-10 * np.abs(LP).max())
    # the reflected grid part is symmetric too
    cE, wE, cT, wT = aim.stencil_weights(grid, g)
    lat = aim._lattice_reflected(grid, FREQ, st)
    GA = aim.grid_part_layered(grid, lat, cE, wE, cE, wE, m.ravel(), n.ravel()).reshape(g.n_e, g.n_e)
    np.testing.assert_allclose(GA, GA.T, rtol=0, atol=1e-10 * np.abs(GA).max())


def test_layered_aim_matches_dense_layered_operator(two_boxes, reflected_dense):
    """Far pairs: AIM approximation of the total kernel; near pairs: exact.  Agreement to AIM accuracy."""
    g, grid = two_boxes
    st, LAr, LPr = reflected_dense
    k0 = 2 * np.pi * FREQ / mgf.C0
    op = aim.build_aim_layered(g, grid, FREQ, st)
    m, n = np.meshgrid(np.arange(g.n_e), np.arange(g.n_e), indexing='ij')
    LA = aim.exact_entries(g, k0, m.ravel(), n.ravel()).reshape(g.n_e, g.n_e) + LAr
    t, u = np.meshgrid(np.arange(g.n_t), np.arange(g.n_t), indexing='ij')
    LP = aim.exact_phi_entries(g, k0, t.ravel(), u.ravel()).reshape(g.n_t, g.n_t) + LPr
    rng = np.random.default_rng(2)
    j = rng.standard_normal(g.n_e) + 1j * rng.standard_normal(g.n_e)
    q = rng.standard_normal(g.n_t) + 1j * rng.standard_normal(g.n_t)
    ea = np.linalg.norm(op.apply_LA(j) - LA @ j) / np.linalg.norm(LA @ j)
    ep = np.linalg.norm(op.apply_Lphi(q) - LP @ q) / np.linalg.norm(LP @ q)
    assert ea < 2e-3 and ep < 2e-3, (ea, ep)
    # the reflected part matters here: dropping it changes the product by far more
    LA0 = aim.exact_entries(g, k0, m.ravel(), n.ravel()).reshape(g.n_e, g.n_e)
    assert np.linalg.norm(LA0 @ j - LA @ j) > 20 * ea * np.linalg.norm(LA @ j)


def test_reflected_rule_converges(two_boxes):
    """The TRI(2) reading of the reflected near entries against higher-order rules.

    The reflected kernel is smooth at the triangle scale.  On the full two-box operator,
    TRI(2) is within 2.7e-3 (L_A) and 5e-4 (L_phi) of TRI(5).  Here a few rows are
    checked (rows 0 and 30, every other column): TRI(2) within 1e-2 of TRI(4), and TRI(3)
    closer to TRI(4) than TRI(2) is.
    """
    g, grid = two_boxes
    st = mgf.substrate_c4()
    st.z_if = grid.origin[2] - 1 * UM
    m, n = np.meshgrid([0, 30], np.arange(0, g.n_e, 2), indexing='ij')
    A = {o: aim.reflected_entries(g, FREQ, st, m.ravel(), n.ravel(), o) for o in (2, 3, 4)}
    e2 = np.linalg.norm(A[2] - A[4]) / np.linalg.norm(A[4])
    e3 = np.linalg.norm(A[3] - A[4]) / np.linalg.norm(A[4])
    assert e2 < 1e-2 and e3 < 0.5 * e2, (e2, e3)
    t, u = np.meshgrid([0, 20], np.arange(0, g.n_t, 2), indexing='ij')
    P = {o: aim.reflected_phi_entries(g, FREQ, st, t.ravel(), u.ravel(), o) for o in (2, 4)}
    assert np.linalg.norm(P[2] - P[4]) / np.linalg.norm(P[4]) < 2e-3
