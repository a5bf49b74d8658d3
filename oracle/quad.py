"""Triangle quadrature and the triangle-pair integrals of the Galerkin operators.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper computes the entries of L_A, L_phi (Sec. II-A) and of the interior
L, K (eq. (4)-(5)) "through numeric integration" and needs special routines
when the conductivity is high (Sec. II-B).  It does not fix the rules; the
reading used on both sides of this project is:

  * TRI(n): collapsed (Duffy) Gauss-Legendre rule with n x n points,
      r = v0 + u (v1 - v0) + v (1 - u) (v2 - v0),  weight 2A w_u w_v (1 - u).
  * far pairs (centroid distance >= c_near * max diameter): TRI(n_far) x TRI(n_far).
  * near pairs: TRI(n_near) on the lower-index triangle; on the other triangle a
    polar rule around the projection rho0 of each outer point: the triangle is
    split into the three signed sub-triangles (rho0, u1, u2), each swept in
    polar coordinates (angle through u = asinh(tan theta): n_t Gauss points;
    radius rho = s rho_max
    with area element rho d rho d theta, so the 1/R singularity cancels); s is
    integrated on the geometric intervals [0, q^L], [q^L, q^(L-1)], ..., [q, 1]
    (n_r Gauss points each, which also resolves the e^{-R/delta} decay of the
    conductor kernel).
  * the double-layer integrand vanishes for coplanar pairs (its triple product
    is normal to the plane), which is its principal value on flat triangles.

Pair integrals for triangles Ta (test, local vertices p_i) and Tb (source,
local vertices q_j), G = e^{-jkR}/(4 pi R), d = r - r':
    IA[i,j] = int int (r - p_i).(r' - q_j) G
    IS      = int int G
    IK[i,j] = int int (r - p_i) . (grad_r G x (r' - q_j)),
              grad_r G = -(1 + jkR) e^{-jkR} d / (4 pi R^3)
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class QuadParams:
    n_far: int = 4
    n_near: int = 5
    levels: int = 3
    q: float = 0.25
    n_r: int = 5
    n_t: int = 6
    c_near: float = 2.0


def gauss01(n):
    """Gauss-Legendre nodes and weights on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def tri_points(V, n):
    """TRI(n) on a batch of triangles V (B, 3, 3) -> points (B, n*n, 3), weights (B, n*n)."""
    x, w = gauss01(n)
    u = np.repeat(x, n)
    v = np.tile(x, n)
    wt = np.repeat(w, n) * np.tile(w, n) * (1.0 - u)
    a = V[:, 0][:, None, :]
    e1 = (V[:, 1] - V[:, 0])[:, None, :]
    e2 = (V[:, 2] - V[:, 0])[:, None, :]
    pts = a + u[None, :, None] * e1 + (v * (1.0 - u))[None, :, None] * e2
    area2 = np.linalg.norm(np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0]), axis=1)
    return pts, area2[:, None] * wt[None, :]


def radial_rule(levels, q, n_r):
    """Composite Gauss rule on [0,1] with breakpoints 0, q^L, ..., q, 1."""
    bp = [0.0] + [q ** (levels - l) for l in range(levels)] + [1.0]
    x, w = gauss01(n_r)
    s, ws = [], []
    for a, b in zip(bp[:-1], bp[1:]):
        s.append(a + (b - a) * x)
        ws.append((b - a) * w)
    return np.concatenate(s), np.concatenate(ws)


def polar_points(ro, V, levels, q, n_r, n_t):
    """Polar rule on triangles V (B,3,3) around the projections of ro (B,No,3).

    Each signed sub-triangle (rho0, u1, u2) is swept in the polar angle theta,
    measured from the foot of the perpendicular from rho0 to the edge line
    (distance h), through the variable u = asinh(tan theta) (n_t Gauss points
    between the values of u1 and u2; it makes the in-plane 1/R integrand
    constant), and in s = rho / rho_max(theta), rho_max = h / cos(theta), on
    the composite radial rule.  Area element rho d rho d theta = s rho_max^2 ds dtheta, signed with
    the orientation of the sub-triangle.  Returns points (B, No, Ni, 3) and
    weights (B, No, Ni).
    """
    nrm = np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0])
    nrm = nrm / np.linalg.norm(nrm, axis=1)[:, None]
    hgt = np.einsum('bok,bk->bo', ro - V[:, None, 0], nrm)
    rho0 = ro - hgt[..., None] * nrm[:, None, :]
    s, ws = radial_rule(levels, q, n_r)
    x, wx = gauss01(n_t)
    pts, wts = [], []
    for e in range(3):
        u1 = V[:, (e + 1) % 3][:, None, :]
        u2 = V[:, (e + 2) % 3][:, None, :]
        E = u2 - u1
        elen = np.linalg.norm(E, axis=-1)
        et = E / elen[..., None]
        l1 = np.sum((u1 - rho0) * et, axis=-1)
        l2 = np.sum((u2 - rho0) * et, axis=-1)
        hvec = (u1 - rho0) - l1[..., None] * et
        h = np.linalg.norm(hvec, axis=-1)
        sgn = np.sign(np.einsum('bk,bok->bo', nrm, np.cross(u1 - rho0, u2 - rho0)))
        ok = h > 1e-12 * elen
        hs = np.where(ok, h, 1.0)
        eh = hvec / hs[..., None]
        a1 = np.arcsinh(l1 / hs)
        a2 = np.arcsinh(l2 / hs)
        u = a1[..., None] + (a2 - a1)[..., None] * x                 # (B,No,n_t)
        wu = (a2 - a1)[..., None] * wx
        th = np.arctan(np.sinh(u))
        rmax = hs[..., None] * np.cosh(u)                            # h / cos(theta)
        wth = wu / np.cosh(u)                                        # d theta = du / cosh u
        dirv = np.cos(th)[..., None] * eh[:, :, None, :] + np.sin(th)[..., None] * et[:, :, None, :]
        # points (B,No,n_s,n_t,3)
        rho = s[None, None, :, None] * rmax[:, :, None, :]
        p = rho0[:, :, None, None, :] + rho[..., None] * dirv[:, :, None, :, :]
        w = (sgn * ok)[:, :, None, None] * (s * ws)[None, None, :, None] * (rmax ** 2 * wth)[:, :, None, :]
        B_, No = ro.shape[0], ro.shape[1]
        pts.append(p.reshape(B_, No, -1, 3))
        wts.append(w.reshape(B_, No, -1))
    return np.concatenate(pts, axis=2), np.concatenate(wts, axis=2)


def _integrals_direct(ra, wa, rb, wb, Pa, Pb, k, want_k):
    """The three pair integrals as iterated sums over explicit point sets: at every
    test point r of the outer rule, the inner rule over the source triangle, then the
    outer sum.  With f_m ~ (r - p_i) and f_n ~ (r' - q_j):
      IS   = sum_o w_o sum_n w'_n G
      IA_ij = sum_o w_o (r_o - p_i) . [sum_n w'_n G (r'_n - q_j)]
      IK_ij = sum_o w_o (r_o - p_i) . [sum_n w'_n g (d x (r'_n - q_j))],  d = r - r',
    g = dG/dR / R (grad_r G = g d); the inner brackets are formed from the sums
    sum w' G, sum w' G r' and sum w' g d x r', sum w' g d at each test point.

    ra (B,No,3), wa (B,No); rb (B,No,Ni,3), wb (B,No,Ni); Pa, Pb (B,3,3) local vertices.
    """
    d = ra[:, :, None, :] - rb
    R = np.sqrt(np.sum(d * d, axis=-1))
    ekr = np.exp(-1j * k * R)
    WG = wb * (ekr / (4.0 * np.pi * R))                          # (B,No,Ni)
    T0 = WG.sum(axis=2)                                          # inner sum of G
    T1 = np.einsum('bon,bonx->box', WG, rb)                      # inner sum of G r'
    inner = T1[:, :, None, :] - Pb[:, None, :, :] * T0[:, :, None, None]   # (B,No,3j,3)
    A = ra[:, :, None, :] - Pa[:, None, :, :]                    # (B,No,3i,3)
    IS = np.einsum('bo,bo->b', wa, T0)
    IA = np.einsum('bo,boix,bojx->bij', wa, A, inner)
    IK = None
    if want_k:
        Wg = wb * (-(1.0 + 1j * k * R) * ekr / (4.0 * np.pi * R ** 3))
        V1 = np.einsum('bon,bonx->box', Wg, np.cross(d, rb))      # inner sum of g d x r'
        V2 = np.einsum('bon,bonx->box', Wg, d)                   # inner sum of g d
        innerK = V1[:, :, None, :] - np.cross(V2[:, :, None, :], Pb[:, None, :, :])
        IK = np.einsum('bo,boix,bojx->bij', wa, A, innerK)
    return IA, IS, IK


def _integrals(ra, wa, rb, wb, Pa, Pb, k, want_k):
    """The same sums as _integrals_direct, through moments in coordinates centred on Ta.

    With a = r - c, b = r' - c, P_i = p_i - c, Q_j = q_j - c (c = centroid of Ta):
      (a - P_i).(b - Q_j) = a.b - P_i.b - Q_j.a + P_i.Q_j
      (a - P_i).((a - b) x (b - Q_j)) = (Q_j - P_i).(a x b) + Q_j.(P_i x (a - b))
    so IA needs sum G, sum G a, sum G b, sum G a.b and IK needs sum g a x b,
    sum g a, sum g b (G, g the kernel times the weights).
    """
    c = Pa.mean(axis=1)                                       # (B,3)
    a = ra - c[:, None, :]
    b = rb - c[:, None, None, :]
    P = Pa - c[:, None, :]
    Q = Pb - c[:, None, :]
    d = a[:, :, None, :] - b
    R = np.sqrt(np.sum(d * d, axis=-1))
    ekr = np.exp(-1j * k * R)
    WG = wb * (ekr / (4.0 * np.pi * R))                       # (B,No,Ni)
    s0 = WG.sum(axis=2)                                       # (B,No)
    s1 = np.einsum('bon,bonx->box', WG, b)                    # (B,No,3)
    S0 = np.einsum('bo,bo->b', wa, s0)
    Sa = np.einsum('bo,bo,box->bx', wa, s0, a)
    Sb = np.einsum('bo,box->bx', wa, s1)
    Sab = np.einsum('bo,box,box->b', wa, a, s1)
    IA = (Sab[:, None, None] - np.einsum('bix,bx->bi', P, Sb)[:, :, None]
          - np.einsum('bjx,bx->bj', Q, Sa)[:, None, :] + np.einsum('bix,bjx->bij', P, Q) * S0[:, None, None])
    IK = None
    if want_k:
        Wg = wb * (-(1.0 + 1j * k * R) * ekr / (4.0 * np.pi * R ** 3))
        g0 = Wg.sum(axis=2)
        g1 = np.einsum('bon,bonx->box', Wg, b)
        Ya = np.einsum('bo,bo,box->bx', wa, g0, a)
        Yb = np.einsum('bo,box->bx', wa, g1)
        X = np.einsum('bo,box->bx', wa, np.cross(a, g1))
        QmP = Q[:, None, :, :] - P[:, :, None, :]             # (B,i,j,3)
        IK = (np.einsum('bijx,bx->bij', QmP, X)
              + np.einsum('bjx,bix->bij', Q, np.cross(P, (Ya - Yb)[:, None, :])))
    return IA, S0, IK


DEFAULT_DIRECT = True


def pair_integrals(Va, Vb, k, near, coplanar, qp: QuadParams, want_k=True, batch=64, direct=None):
    """IA (B,3,3), IS (B,), IK (B,3,3) for triangle pairs (Va[b], Vb[b]).

    The sums are taken as iterated integrals (_integrals_direct: inner rule at every
    test point, then the outer rule) unless direct=False asks for the centroid-moment
    form (_integrals), a rearrangement of the same sums that the tests pin against the
    iterated one on both rules.
    """
    if direct is None:
        direct = DEFAULT_DIRECT
    B = Va.shape[0]
    IA = np.zeros((B, 3, 3), dtype=complex)
    IS = np.zeros(B, dtype=complex)
    IK = np.zeros((B, 3, 3), dtype=complex)
    for lo in range(0, B, batch):
        sl = slice(lo, min(B, lo + batch))
        va, vb = Va[sl], Vb[sl]
        if near:
            ra, wa = tri_points(va, qp.n_near)
            rb, wb = polar_points(ra, vb, qp.levels, qp.q, qp.n_r, qp.n_t)
        else:
            ra, wa = tri_points(va, qp.n_far)
            rb1, wb1 = tri_points(vb, qp.n_far)
            rb = np.broadcast_to(rb1[:, None], (rb1.shape[0], ra.shape[1]) + rb1.shape[1:])
            wb = np.broadcast_to(wb1[:, None], (wb1.shape[0], ra.shape[1], wb1.shape[1]))
        a, s, kk = (_integrals_direct if direct else _integrals)(ra, wa, rb, wb, va, vb, k, want_k)
        IA[sl], IS[sl] = a, s
        if want_k:
            kk[coplanar[sl]] = 0.0
            IK[sl] = kk
    return IA, IS, IK


def potential_1_over_R(r, V):
    """Closed-form integral of 1/|r - r'| over a flat triangle V (3,3).

    Standard edge-sum formula for the static potential of a uniform source on
    a polygon (Wilton et al. 1984; Graglia 1993): with rho0 the projection of r,
    d its height, and for every edge with unit tangent l, outward in-plane
    normal u, t0 = (rho_edge - rho0).u, l+- the tangential coordinates of its
    end points, R+- their distances to r and R0^2 = t0^2 + d^2:
        sum t0 ln((R+ + l+)/(R- + l-)) - |d| [atan(t0 l+/(R0^2 + |d| R+))
                                              - atan(t0 l-/(R0^2 + |d| R-))]
    """
    r = np.asarray(r, dtype=float)
    nrm = np.cross(V[1] - V[0], V[2] - V[0])
    nrm /= np.linalg.norm(nrm)
    d = float(np.dot(r - V[0], nrm))
    rho0 = r - d * nrm
    ad = abs(d)
    total = 0.0
    for e in range(3):
        a, b = V[e], V[(e + 1) % 3]
        lhat = (b - a) / np.linalg.norm(b - a)
        u = np.cross(lhat, nrm)
        t0 = float(np.dot(a - rho0, u))
        lm, lp = float(np.dot(a - rho0, lhat)), float(np.dot(b - rho0, lhat))
        Rm, Rp = np.linalg.norm(r - a), np.linalg.norm(r - b)
        R0sq = t0 * t0 + d * d
        if abs(t0) > 1e-300:
            total += t0 * np.log((Rp + lp) / (Rm + lm))
        total -= ad * (np.arctan2(t0 * lp, R0sq + ad * Rp) - np.arctan2(t0 * lm, R0sq + ad * Rm))
    return total
