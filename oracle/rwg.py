"""RWG basis and the sparse AEFIE matrices (Sec. II, eq. (2)-(3)).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Readings (the paper defers F, B, D to its reference [Qian2009]):
  * RWG basis on T+ u T-: f_n = l_n/(2A+) (r - p+) on T+, l_n/(2A-) (p- - r) on T-.
    T+ is the triangle whose own vertex cycle runs along the edge from the
    lower to the higher vertex id.
  * unknowns are ordered object by object; inside an object edges are sorted
    by (lower vertex id, higher vertex id).
  * D (N_T x N_E): D[T+, n] = +l_n, D[T-, n] = -l_n  (so div f_n = D[t,n]/A_t).
  * B = diag(A_t),  F = -diag(1/A_t).  With these signs both the "+D^T" of the
    first row of (3) and the continuity row F D J + j k0 c0 rho = 0 hold; the
    charge unknown is then minus the physical surface charge density.
  * I_x[m, n] = integral of (n x f_m) . f_n  (testing f_n with rotated f_m).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class RWG:
    verts: np.ndarray      # (n_vert, 3)
    tris: np.ndarray       # (n_tri, 3)
    obj: np.ndarray        # (n_tri,)
    n_obj: int
    area: np.ndarray       # (n_tri,)
    normal: np.ndarray     # (n_tri, 3) unit outward
    centroid: np.ndarray   # (n_tri, 3)
    diam: np.ndarray       # (n_tri,) longest edge
    edge_v: np.ndarray     # (n_e, 2) lower, higher vertex id
    tplus: np.ndarray      # (n_e,)
    tminus: np.ndarray     # (n_e,)
    length: np.ndarray     # (n_e,)
    edge_obj: np.ndarray   # (n_e,)
    tri_edge: np.ndarray   # (n_tri, 3) RWG index of the edge opposite local vertex i
    tri_sign: np.ndarray   # (n_tri, 3) +1 if the triangle is T+ of that RWG, else -1
    obj_edge_off: np.ndarray  # (n_obj+1,)
    obj_tri_off: np.ndarray   # (n_obj+1,)

    @property
    def n_e(self):
        return int(self.edge_v.shape[0])

    @property
    def n_t(self):
        return int(self.tris.shape[0])


class MeshError(ValueError):
    pass


def build_rwg(verts, tris, obj, n_obj) -> RWG:
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    obj = np.asarray(obj, dtype=np.int64)
    nt = tris.shape[0]
    if np.any(np.diff(obj) < 0):
        raise MeshError("triangles must be grouped by object")
    if obj.min() < 0 or obj.max() >= n_obj:
        raise MeshError("object id out of range")
    v0, v1, v2 = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    cr = np.cross(v1 - v0, v2 - v0)
    two_a = np.linalg.norm(cr, axis=1)
    if np.any(two_a <= 0.0):
        raise MeshError("degenerate triangle %d" % int(np.argmin(two_a)))
    area = 0.5 * two_a
    normal = cr / two_a[:, None]
    centroid = (v0 + v1 + v2) / 3.0
    diam = np.max(np.stack([np.linalg.norm(v1 - v2, axis=1), np.linalg.norm(v2 - v0, axis=1),
                            np.linalg.norm(v0 - v1, axis=1)]), axis=0)

    # directed edges: local edge i is opposite local vertex i
    plus, minus = {}, {}
    for t in range(nt):
        a = tris[t]
        for i in range(3):
            u, w = int(a[(i + 1) % 3]), int(a[(i + 2) % 3])
            key = (min(u, w), max(u, w))
            d = plus if u < w else minus
            if key in d:
                raise MeshError("non-manifold or inconsistently oriented edge %s" % (key,))
            d[key] = (t, i)
    if set(plus) != set(minus):
        raise MeshError("mesh is not closed")
    keys = sorted(plus, key=lambda k: (int(obj[plus[k][0]]), k[0], k[1]))
    ne = len(keys)
    edge_v = np.array(keys, dtype=np.int64).reshape(ne, 2)
    tplus = np.array([plus[k][0] for k in keys], dtype=np.int64)
    tminus = np.array([minus[k][0] for k in keys], dtype=np.int64)
    if np.any(obj[tplus] != obj[tminus]):
        raise MeshError("edge shared by two objects")
    length = np.linalg.norm(verts[edge_v[:, 1]] - verts[edge_v[:, 0]], axis=1)
    tri_edge = np.full((nt, 3), -1, dtype=np.int64)
    tri_sign = np.zeros((nt, 3), dtype=np.int64)
    for n, k in enumerate(keys):
        t, i = plus[k]
        tri_edge[t, i], tri_sign[t, i] = n, 1
        t, i = minus[k]
        tri_edge[t, i], tri_sign[t, i] = n, -1
    edge_obj = obj[tplus]
    obj_edge_off = np.searchsorted(edge_obj, np.arange(n_obj + 1))
    obj_tri_off = np.searchsorted(obj, np.arange(n_obj + 1))
    return RWG(verts, tris, obj, n_obj, area, normal, centroid, diam, edge_v, tplus, tminus,
               length, edge_obj, tri_edge, tri_sign, obj_edge_off, obj_tri_off)


def rwg_on_triangle(g: RWG, t: int, i: int, r):
    """Value of the RWG function attached to local edge i of triangle t at points r."""
    n = g.tri_edge[t, i]
    p = g.verts[g.tris[t, i]]
    return g.tri_sign[t, i] * g.length[n] / (2.0 * g.area[t]) * (np.asarray(r) - p)


def matrix_D(g: RWG):
    """D[T+, n] = +l_n, D[T-, n] = -l_n (dense, N_T x N_E)."""
    D = np.zeros((g.n_t, g.n_e))
    D[g.tplus, np.arange(g.n_e)] += g.length
    D[g.tminus, np.arange(g.n_e)] -= g.length
    return D


def matrix_B(g: RWG):
    return np.diag(g.area)


def matrix_F(g: RWG):
    return -np.diag(1.0 / g.area)


def _edge_midpoints(g: RWG, t):
    a = g.verts[g.tris[t]]
    return np.array([(a[1] + a[2]) / 2, (a[2] + a[0]) / 2, (a[0] + a[1]) / 2])


def matrix_Ix_and_gram(g: RWG):
    """I_x[m,n] = int (n x f_m).f_n dS and Gram[m,n] = int f_m.f_n dS.

    Integrands are quadratic on every triangle, so the three-edge-midpoint rule
    (weights A/3) integrates them exactly.
    """
    Ix = np.zeros((g.n_e, g.n_e))
    G = np.zeros((g.n_e, g.n_e))
    for t in range(g.n_t):
        mids = _edge_midpoints(g, t)
        nrm = g.normal[t]
        f = [rwg_on_triangle(g, t, i, mids) for i in range(3)]
        for i in range(3):
            for j in range(3):
                m, n = g.tri_edge[t, i], g.tri_edge[t, j]
                Ix[m, n] += g.area[t] / 3.0 * np.sum(np.cross(nrm, f[i]) * f[j])
                G[m, n] += g.area[t] / 3.0 * np.sum(f[i] * f[j])
    return Ix, G


def project_tangential(g: RWG, field_fn, order=6):
    """RWG coefficients of a tangential vector field F(r): solve Gram c = <f_m, F>."""
    from .quad import tri_points
    _, Gm = matrix_Ix_and_gram(g)
    b = np.zeros(g.n_e, dtype=complex)
    for t in range(g.n_t):
        pts, w = tri_points(g.verts[g.tris[t]][None], order)
        pts, w = pts[0], w[0]
        F = field_fn(pts, t)
        for i in range(3):
            b[g.tri_edge[t, i]] += np.sum(w[:, None] * rwg_on_triangle(g, t, i, pts) * F)
    return np.linalg.solve(Gm, b), Gm


def interpolate_tangential(g: RWG, field_fn, n=8):
    """RWG interpolant of a tangential field F by edge fluxes (Rao-Wilton-Glisson).

    f_n carries unit normal flux density across its own edge and none across the
    others, so the coefficient of edge n is the mean, along the edge, of F . m_n,
    with m_n the unit vector in the plane of T+ normal to the edge and pointing
    away from the free vertex of T+.  F is evaluated on the T+ side
    (field_fn(points, triangle)).  Unlike the Gram projection, this interpolant
    keeps the flux of F across every edge, hence the triangle-averaged surface
    divergence.
    """
    from .quad import gauss01
    x, w = gauss01(n)
    c = np.zeros(g.n_e, dtype=complex)
    for e in range(g.n_e):
        t = int(g.tplus[e])
        i = int(np.nonzero(g.tri_edge[t] == e)[0][0])
        p = g.verts[g.tris[t, i]]
        a, b = g.verts[g.edge_v[e, 0]], g.verts[g.edge_v[e, 1]]
        tt = (b - a) / np.linalg.norm(b - a)
        m = 0.5 * (a + b) - p
        m = m - np.dot(m, tt) * tt
        m = m / np.linalg.norm(m)
        pts = a[None, :] + x[:, None] * (b - a)[None, :]
        c[e] = np.sum(w * (np.asarray(field_fn(pts, t)) @ m))
    return c
