"""Pins of the mesh, RWG basis and sparse AEFIE matrices (Sec. II, eq. (2)-(3))."""
import numpy as np
import pytest

from inputs.geometry import bar_c1, box_mesh, merge, small_boxes, split_ring_mesh
from oracle.quad import tri_points
from oracle.rwg import MeshError, build_rwg, matrix_D, matrix_Ix_and_gram, rwg_on_triangle


def _meshes():
    ring = merge([split_ring_mesh((0, 0, 0), 20e-6, 4e-6, 1e-6, 4e-6, 37)])
    return [bar_c1(), ring, small_boxes(3, seed=2)]


@pytest.mark.parametrize("mi", range(3))
def test_closed_surface_invariants(mi):
    m = _meshes()[mi]
    g = build_rwg(m.verts, m.tris, m.obj, m.n_obj)
    for i in range(g.n_obj):
        nt = g.obj_tri_off[i + 1] - g.obj_tri_off[i]
        ne = g.obj_edge_off[i + 1] - g.obj_edge_off[i]
        # every closed triangulated surface has N_E = 1.5 N_T (all three meshes printed in Sec. IV)
        assert 2 * ne == 3 * nt
        tris = g.tris[g.obj_tri_off[i]:g.obj_tri_off[i + 1]]
        nv = np.unique(tris).size
        assert nv - ne + nt == 2                      # genus-0 Euler characteristic
        sel = slice(g.obj_tri_off[i], g.obj_tri_off[i + 1])
        assert np.abs((g.area[sel, None] * g.normal[sel]).sum(0)).max() < 1e-12 * g.area[sel].sum()
        vol = np.sum(g.area[sel] * np.einsum('tk,tk->t', g.centroid[sel], g.normal[sel])) / 3.0
        assert vol > 0                                # outward orientation
    D = matrix_D(g)
    assert np.abs(D.sum(axis=0)).max() < 1e-18       # charge conservation: 1^T D = 0
    # div f_n = D[t, n] / A_t: check against the RWG formula on a few triangles
    for t in range(0, g.n_t, max(1, g.n_t // 7)):
        for i in range(3):
            n = g.tri_edge[t, i]
            assert np.isclose(D[t, n] / g.area[t], g.tri_sign[t, i] * g.length[n] / g.area[t])


def test_box_sizes_c1():
    m = bar_c1()
    g = build_rwg(m.verts, m.tris, m.obj, m.n_obj)
    assert (g.n_t, g.n_e) == (592, 888)


def test_mesh_errors():
    v, t = box_mesh((0, 0, 0), (1, 1, 1), (2, 2, 2))
    with pytest.raises(MeshError):                    # not closed
        build_rwg(v, t[:-1], np.zeros(len(t) - 1, np.int32), 1)
    t2 = t.copy()
    t2[0] = t2[0, ::-1]
    with pytest.raises(MeshError):                    # inconsistent orientation
        build_rwg(v, t2, np.zeros(len(t), np.int32), 1)
    with pytest.raises(MeshError):                    # object id out of range
        build_rwg(v, t, np.full(len(t), 3, np.int32), 1)


def test_ix_and_gram():
    m = small_boxes(2, seed=5)
    g = build_rwg(m.verts, m.tris, m.obj, m.n_obj)
    Ix, Gm = matrix_Ix_and_gram(g)
    assert np.abs(Ix + Ix.T).max() < 1e-25 and np.abs(np.diag(Ix)).max() == 0.0
    assert np.abs(Gm - Gm.T).max() < 1e-25
    assert np.linalg.eigvalsh(Gm).min() > 0
    # the edge-midpoint rule is exact for these quadratic integrands: compare with TRI(6)
    V = g.verts[g.tris]
    pts, w = tri_points(V, 6)
    # total Gram entries vs TRI(6) assembled over all triangles
    G2 = np.zeros_like(Gm)
    X2 = np.zeros_like(Ix)
    for t in range(g.n_t):
        f = [rwg_on_triangle(g, t, i, pts[t]) for i in range(3)]
        for i in range(3):
            for j in range(3):
                m_, n_ = g.tri_edge[t, i], g.tri_edge[t, j]
                G2[m_, n_] += np.sum(w[t] * np.einsum('pk,pk->p', f[i], f[j]))
                X2[m_, n_] += np.sum(w[t] * np.einsum('pk,pk->p', np.cross(g.normal[t], f[i]), f[j]))
    assert np.abs(G2 - Gm).max() < 1e-12 * np.abs(Gm).max()
    assert np.abs(X2 - Ix).max() < 1e-12 * np.abs(Gm).max()
