"""Sparse interior operators of a conductor at high frequency (Sec. III-A, point 3).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

When the skin depth is small against the object, the paper treats the conductor-kernel
operators L_kc and K_kc of eq. (4) as sparse matrices by ignoring physically distant
interactions, and applies L_kc^{-1} by a sparse direct solve.  The paper names no
cutoff; readings taken here:

  * a triangle pair (t, u) of the object interacts when its centroid distance is at most
    r: dx*dx + dy*dy + dz*dz <= r*r, summed in that order in FP64;
  * L~ and K~ are the Galerkin sums over the interacting pairs only (the same pair
    integrals as the dense operators), and Z~ = -1/(j w eps_c) L~^{-1} (K~ + I_x/2)
    (eq. (4) with the sparse operators);
  * the product applies Z~ as an explicit sparse matrix on the RWG pairs (m, n) that
    share an interacting triangle pair (m an edge of t, n an edge of u, or the reverse),
    Z~_t; the entries off that pattern are dropped.  Z is a local operator once the skin
    depth is small (the fields inside a good conductor decay over a few skin depths), so
    the dropped part falls with r like the kernel's own decay;
  * M~ = Y_eq Z~_t (eq. (6) with the sparse Z); Y_eq (eq. (5), the outer medium's kernel)
    stays dense.
With r at least the object's diameter, every pair interacts and Z~_t is the dense Z.
"""
from __future__ import annotations

import numpy as np

from .operators import (MU0, Interior, Physics, assemble_rwg, interior_LK, tri_pairs,
                        triangle_pair_integrals)
from .quad import QuadParams
from .rwg import RWG, matrix_Ix_and_gram


def interacting(g: RWG, T, U, r):
    """Mask of the triangle pairs (T[b], U[b]) whose centroids are at most r apart."""
    c = g.centroid
    dx = c[T, 0] - c[U, 0]
    dy = c[T, 1] - c[U, 1]
    dz = c[T, 2] - c[U, 2]
    return dx * dx + dy * dy + dz * dz <= r * r


def object_pairs(g: RWG, obj: int):
    """All triangle pairs (t <= u) of one object."""
    return tri_pairs(g, np.arange(g.obj_tri_off[obj], g.obj_tri_off[obj + 1]))


def sparse_LK(g: RWG, obj: int, k, r, qp: QuadParams = QuadParams()):
    """L~_k and K~_k of one object (local edge numbering): eq. (4)-(5) operators summed
    over the interacting triangle pairs only."""
    e0, e1 = g.obj_edge_off[obj], g.obj_edge_off[obj + 1]
    T, U = object_pairs(g, obj)
    keep = interacting(g, T, U, r)
    T, U = T[keep], U[keep]
    IA, IS, IK = triangle_pair_integrals(g, T, U, k, qp, want_k=True)
    Lvec, Ldiv, K = assemble_rwg(g, T, U, IA, IS, IK, e1 - e0, edge_offset=e0)
    return Lvec - Ldiv / (k * k), K


def z_pattern(g: RWG, obj: int, r):
    """Boolean n x n pattern of Z~_t: RWG pairs sharing an interacting triangle pair."""
    e0, e1 = g.obj_edge_off[obj], g.obj_edge_off[obj + 1]
    T, U = object_pairs(g, obj)
    keep = interacting(g, T, U, r)
    T, U = T[keep], U[keep]
    P = np.zeros((e1 - e0, e1 - e0), dtype=bool)
    te = g.tri_edge - e0
    for i in range(3):
        for j in range(3):
            P[te[T, i], te[U, j]] = True
            P[te[U, j], te[T, i]] = True
    return P


def sparse_interior_blocks(g: RWG, phys: Physics, r, qp: QuadParams = QuadParams(), Ix=None):
    """Per object: Z~_t (dense array, zero off the pattern), M~ = Y_eq Z~_t, Y_eq, and the
    pattern (list of boolean arrays)."""
    if Ix is None:
        Ix, _ = matrix_Ix_and_gram(g)
    Zs, Ms, Ys, Ps = [], [], [], []
    w = phys.omega
    for i in range(g.n_obj):
        e0, e1 = g.obj_edge_off[i], g.obj_edge_off[i + 1]
        Ixi = Ix[e0:e1, e0:e1]
        Lc, Kc = sparse_LK(g, i, phys.kc, r, qp)
        Z = (-1.0 / (1j * w * phys.eps_c)) * np.linalg.solve(Lc, Kc + 0.5 * Ixi)
        P = z_pattern(g, i, r)
        Zt = np.where(P, Z, 0.0)
        Ll, Kl = interior_LK(g, i, phys.k0, qp)
        Y = (1.0 / (1j * w * MU0)) * np.linalg.solve(Ll, Kl + 0.5 * Ixi)
        Zs.append(Zt)
        Ys.append(Y)
        Ms.append(Y @ Zt)
        Ps.append(P)
    return Interior(Zs, Ms, Ys), Ps
