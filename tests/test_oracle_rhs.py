"""Pins of the plane-wave right-hand side of (7): b1[m] = eta0^-1 int f_m . E_inc dS, b2 = 0.

Closed forms used:
  * for a uniform field the RWG integral is exact: int_{T+} f_m dS = (l/2)(c+ - p+) and
    int_{T-} f_m dS = (l/2)(p- - c-), with c the centroid and p the free vertex;
  * on a triangle normal to khat the phase e^{-j k0 khat.r} is constant, so the same
    closed form times that phase is exact.
"""
import numpy as np

from inputs.geometry import box_mesh, merge
from oracle.operators import ETA0, Physics, planewave_rhs
from oracle.rwg import build_rwg

UM = 1e-6


def _box(size, div):
    m = merge([box_mesh((0.0, 0.0, 0.0), size, div)])
    return build_rwg(m.verts, m.tris, m.obj, m.n_obj)


def _closed_form(g, E0, phase_of_tri):
    b = np.zeros(g.n_e + g.n_t, dtype=complex)
    for n in range(g.n_e):
        tot = np.zeros(3, dtype=complex)
        for t, s in ((g.tplus[n], 1.0), (g.tminus[n], -1.0)):
            i = int(np.nonzero(g.tri_edge[t] == n)[0][0])
            p = g.verts[g.tris[t, i]]
            tot += s * 0.5 * g.length[n] * (g.centroid[t] - p) * phase_of_tri(t)
        b[n] = np.dot(tot, E0) / ETA0
    return b


def test_static_limit():
    g = _box((10 * UM, 4 * UM, 3 * UM), (4, 2, 2))
    E0 = np.array([0.3, -1.0, 0.7])
    b = planewave_rhs(g, Physics(1.0), (0.0, 0.6, 0.8), E0)     # k0 |r| ~ 2e-13
    ref = _closed_form(g, E0, lambda t: 1.0)
    assert np.all(b[g.n_e:] == 0)
    assert np.abs(b - ref).max() <= 1e-12 * np.abs(ref).max()
    # a field with no tangential part on a face gives nothing on the edges inside it
    bz = planewave_rhs(g, Physics(1.0), (1.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    top = [n for n in range(g.n_e) if np.allclose(g.normal[[g.tplus[n], g.tminus[n]], 2], 1.0)]
    assert len(top) > 0 and np.abs(bz[top]).max() <= 1e-12 * np.abs(bz).max()


def test_phase_on_faces_normal_to_khat():
    """Travelling along +z at 3 THz across a 20 um tall box: edges inside the top and bottom
    faces see the closed form times e^{-j k0 z} of their face (the sign of the exponent)."""
    g = _box((6 * UM, 6 * UM, 20 * UM), (3, 3, 4))
    ph = Physics(3e12)
    E0 = np.array([1.0, 0.4, 0.0])
    b = planewave_rhs(g, ph, (0.0, 0.0, 1.0), E0)
    ref = _closed_form(g, E0, lambda t: np.exp(-1j * ph.k0 * g.centroid[t, 2]))
    for zn in (1.0, -1.0):
        face = [n for n in range(g.n_e) if np.allclose(g.normal[[g.tplus[n], g.tminus[n]], 2], zn)]
        assert len(face) > 0
        assert np.abs(b[face] - ref[face]).max() <= 1e-12 * np.abs(ref[face]).max()
    assert abs(ph.k0 * 20 * UM - 1.2577) < 1e-3     # a phase of 72 degrees between the faces
