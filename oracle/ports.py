"""Lumped ports: delta-gap excitation of the right-hand side of (7) and port currents.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper excites its structures "via lumped ports" (Sec. II) and defers the model to
a reference it does not reproduce.  Reading used on both sides of this project: a
port is an ideal voltage source across a cut of one conductor's surface, the closed
ring of mesh edges that lies in the plane through `point` normal to `axis` within
`radius` of `point`.  Its incident field is V delta(s) axis, s the distance from the
plane along axis, so testing with f_m gives

    b1[m] = (V / eta0) int_ring f_m . axis dl = (V / eta0) s_m l_m ,   b2 = 0,

with s_m = sign(nu_m . axis), nu_m the unit vector in the plane of T+ normal to edge m
pointing away from the free vertex of T+ (the direction in which f_m crosses its
edge, with unit normal flux density).  The current through the port in the
direction of axis is the flux of the surface current n x H = sum_m H_m f_m across
the ring:  I = sum_{m in ring} s_m l_m H_m.  With V = 1 the port admittance is I.
"""
from __future__ import annotations

import numpy as np

from .operators import ETA0
from .rwg import RWG


def ring_edges(g: RWG, obj, point, axis, radius):
    """Edges of object obj in the port plane (both end points within 1e-9 of the mean
    edge length of the plane) and within radius of point, with their signs s_m."""
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    point = np.asarray(point, float)
    tol = 1e-9 * float(np.mean(g.length))
    e0, e1 = g.obj_edge_off[obj], g.obj_edge_off[obj + 1]
    edges, signs = [], []
    for m in range(e0, e1):
        a, b = g.verts[g.edge_v[m, 0]], g.verts[g.edge_v[m, 1]]
        if abs(np.dot(a - point, axis)) > tol or abs(np.dot(b - point, axis)) > tol:
            continue
        if np.linalg.norm(0.5 * (a + b) - point) > radius:
            continue
        t = g.tplus[m]
        free = g.verts[g.tris[t, int(np.nonzero(g.tri_edge[t] == m)[0][0])]]
        tt = (b - a) / np.linalg.norm(b - a)
        nu = 0.5 * (a + b) - free
        nu = nu - np.dot(nu, tt) * tt
        nu /= np.linalg.norm(nu)
        c = float(np.dot(nu, axis))
        if abs(c) < 0.5:
            raise ValueError("port plane runs inside a face of the conductor")
        edges.append(m)
        signs.append(1.0 if c > 0 else -1.0)
    if not edges:
        raise ValueError("no mesh edges in the port plane")
    # a closed ring: every vertex of it belongs to exactly two of its edges
    vs, cnt = np.unique(g.edge_v[edges].ravel(), return_counts=True)
    if np.any(cnt != 2):
        raise ValueError("the port edges do not form one closed ring")
    return np.array(edges), np.array(signs)


def port_rhs(g: RWG, ports, V=1.0):
    """Right-hand sides of (7), one column per port (n_sys x n_ports)."""
    B = np.zeros((g.n_e + g.n_t, len(ports)), dtype=complex)
    for p, (obj, point, axis, radius) in enumerate(ports):
        m, s = ring_edges(g, obj, point, axis, radius)
        B[m, p] = V * s * g.length[m] / ETA0
    return B


def port_currents(g: RWG, ports, X):
    """Currents through the ports (n_ports x n_rhs) for solutions X (n_sys x n_rhs)."""
    X = np.asarray(X).reshape(g.n_e + g.n_t, -1)
    out = np.zeros((len(ports), X.shape[1]), dtype=complex)
    for p, (obj, point, axis, radius) in enumerate(ports):
        m, s = ring_edges(g, obj, point, axis, radius)
        out[p] = (s * g.length[m]) @ X[m]
    return out
