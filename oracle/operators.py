"""Dense FP64 operators of the SLIM formulation and the system product (7)-(8).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Conventions (readings; the paper writes j and leaves them implicit):
  * time dependence e^{j omega t}; G_k(R) = e^{-jkR} / (4 pi R), k0 = omega / c0;
  * conductor permittivity eps_c = eps0 eps_r - j sigma / omega, k_c = omega sqrt(mu eps_c)
    on the branch Im k_c < 0 (the epsilon of eq. (4) is this complex value);
  * c0 = 299792458 m/s, mu0 = 4 pi 1e-7 H/m, eps0 = 1/(mu0 c0^2), eta0 = mu0 c0.

Galerkin matrices (Sec. II-A, II-B), RWG f_m, f_n, pulses on triangles:
  L_A[m,n]   = int int f_m . f_n G_k0
  L_phi[t,u] = 1/(A_t A_u) int_t int_u G_k0
  L_k[m,n]   = int int [f_m . f_n - (div f_m)(div' f_n)/k^2] G_k
  K_k[m,n]   = int int f_m . (grad G_k x f_n')
With these, eq. (4) Z = -1/(j omega eps_c) L_kc^{-1} (K_kc + I_x/2) and eq. (5)
Y_eq = 1/(j omega mu_l) L_kl^{-1} (K_kl + I_x/2) follow from the interior
representation of the fields by n x H and n x E (testing with n x f_m).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .quad import QuadParams, pair_integrals
from .rwg import RWG, matrix_D, matrix_Ix_and_gram

C0 = 299792458.0
MU0 = 4.0e-7 * np.pi
EPS0 = 1.0 / (MU0 * C0 * C0)
ETA0 = MU0 * C0
SIGMA_CU = 5.8e7


@dataclass
class Physics:
    freq: float
    sigma: float = SIGMA_CU
    eps_r: float = 1.0
    mu_r: float = 1.0

    @property
    def omega(self):
        return 2.0 * np.pi * self.freq

    @property
    def k0(self):
        return self.omega / C0

    @property
    def eps_c(self):
        return EPS0 * self.eps_r - 1j * self.sigma / self.omega

    @property
    def kc(self):
        k = self.omega * np.sqrt(MU0 * self.mu_r * self.eps_c + 0j)
        return k if k.imag <= 0 else -k

    @property
    def skin_depth(self):
        return 1.0 / np.sqrt(np.pi * self.freq * MU0 * self.mu_r * self.sigma)


def tri_pairs(g: RWG, tris_a, tris_b=None):
    """All (t, u) with t <= u from one triangle set (tris_b None) or the product of two."""
    ta = np.asarray(tris_a)
    if tris_b is None:
        i, j = np.triu_indices(ta.size)
        return ta[i], ta[j]
    tb = np.asarray(tris_b)
    T, U = np.meshgrid(ta, tb, indexing='ij')
    T, U = T.ravel(), U.ravel()
    keep = T <= U
    return T[keep], U[keep]


def classify(g: RWG, T, U, qp: QuadParams):
    """near: centroid distance < c_near * max(diam); coplanar: same plane (double layer = 0)."""
    d = g.centroid[T] - g.centroid[U]
    dist2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
    dm = np.maximum(g.diam[T], g.diam[U]) * qp.c_near
    near = dist2 < dm * dm
    par = np.abs(np.sum(g.normal[T] * g.normal[U], axis=1)) > 1.0 - 1e-12
    off = np.abs(np.sum(g.normal[T] * d, axis=1)) < 1e-9 * np.maximum(g.diam[T], g.diam[U])
    return near, par & off


def _pair_job(args):
    Va, Vb, k, near, cop, qp, want_k = args
    return pair_integrals(Va, Vb, k, near, cop, qp, want_k)


def triangle_pair_integrals(g: RWG, T, U, k, qp: QuadParams, want_k=True, workers=None):
    """IA, IS, IK for the pairs (T[b], U[b]) (T is the outer / test triangle).

    Independent pair batches are spread over worker processes (OMP-style
    parallelism of a plain loop); the arithmetic is that of quad.pair_integrals.
    """
    import os
    from concurrent.futures import ProcessPoolExecutor
    near, cop = classify(g, T, U, qp)
    n = T.size
    IA = np.zeros((n, 3, 3), dtype=complex)
    IS = np.zeros(n, dtype=complex)
    IK = np.zeros((n, 3, 3), dtype=complex)
    V = g.verts[g.tris]
    if workers is None:
        workers = int(os.environ.get("ORACLE_WORKERS", os.cpu_count() or 1))
    jobs = []
    for flag in (True, False):
        sel = np.nonzero(near == flag)[0]
        step = 2048 if flag else 32768
        for lo in range(0, sel.size, step):
            s = sel[lo:lo + step]
            jobs.append((s, (V[T[s]], V[U[s]], k, flag, cop[s], qp, want_k)))
    if workers > 1 and len(jobs) > 1:
        import multiprocessing
        # fresh interpreters: the workers never inherit a GPU context of the parent
        with ProcessPoolExecutor(max_workers=workers, mp_context=multiprocessing.get_context("spawn")) as ex:
            results = list(ex.map(_pair_job, [j[1] for j in jobs]))
    else:
        results = [_pair_job(j[1]) for j in jobs]
    for (s, _), (a, b, kk) in zip(jobs, results):
        IA[s], IS[s] = a, b
        if want_k:
            IK[s] = kk
    # a triangle with itself: the integrands are symmetric in (i, j); average the
    # two orders so the assembled matrices are exactly symmetric
    same = T == U
    IA[same] = 0.5 * (IA[same] + IA[same].transpose(0, 2, 1))
    IK[same] = 0.5 * (IK[same] + IK[same].transpose(0, 2, 1))
    return IA, IS, IK


def _scatter(te, T, U, vals, coef, n_rows):
    """M[te[t,i], te[u,j]] += vals(i,j) * coef(t,i,u,j), plus the mirror for t != u."""
    M = np.zeros((n_rows, n_rows), dtype=complex)
    off = T != U
    for i in range(3):
        for j in range(3):
            m, n = te[T, i], te[U, j]
            v = vals(i, j) * coef(T, i, U, j)
            np.add.at(M, (m, n), v)
            np.add.at(M, (n[off], m[off]), v[off])
    return M


def assemble_rwg(g: RWG, T, U, IA, IS, IK, n_rows, edge_offset=0):
    """Vector part, divergence part and double layer on RWG indices (minus edge_offset).

    f_m on triangle t with local edge i is s l/(2A) (r - p_i), so
      vector entry += s s' l l'/(4 A A') IA[i,j],  div entry += s s' l l'/(A A') IS,
      double layer += s s' l l'/(4 A A') IK[i,j].
    """
    te = g.tri_edge - edge_offset

    def cv(T_, i, U_, j):
        return (g.tri_sign[T_, i] * g.tri_sign[U_, j] * g.length[g.tri_edge[T_, i]]
                * g.length[g.tri_edge[U_, j]] / (4.0 * g.area[T_] * g.area[U_]))

    def cd(T_, i, U_, j):
        return 4.0 * cv(T_, i, U_, j)

    Lvec = _scatter(te, T, U, lambda i, j: IA[:, i, j], cv, n_rows)
    Ldiv = _scatter(te, T, U, lambda i, j: IS, cd, n_rows)
    Kmat = _scatter(te, T, U, lambda i, j: IK[:, i, j], cv, n_rows) if IK is not None else None
    return Lvec, Ldiv, Kmat


def external_dense(g: RWG, phys: Physics, qp: QuadParams = QuadParams()):
    """Dense L_A (N_E x N_E) and L_phi (N_T x N_T) at k0 over the whole mesh."""
    T, U = tri_pairs(g, np.arange(g.n_t))
    IA, IS, _ = triangle_pair_integrals(g, T, U, phys.k0, qp, want_k=False)
    LA, _, _ = assemble_rwg(g, T, U, IA, IS, None, g.n_e)
    Lphi = np.zeros((g.n_t, g.n_t), dtype=complex)
    v = IS / (g.area[T] * g.area[U])
    Lphi[T, U] = v
    Lphi[U, T] = v
    return LA, Lphi


def interior_LK(g: RWG, obj: int, k, qp: QuadParams = QuadParams()):
    """L_k and K_k of one object (local edge numbering), eq. (4)-(5)."""
    t0, t1 = g.obj_tri_off[obj], g.obj_tri_off[obj + 1]
    e0, e1 = g.obj_edge_off[obj], g.obj_edge_off[obj + 1]
    T, U = tri_pairs(g, np.arange(t0, t1))
    IA, IS, IK = triangle_pair_integrals(g, T, U, k, qp, want_k=True)
    Lvec, Ldiv, K = assemble_rwg(g, T, U, IA, IS, IK, e1 - e0, edge_offset=e0)
    return Lvec - Ldiv / (k * k), K


@dataclass
class Interior:
    Z: list      # per object, n_i x n_i
    M: list      # per object, Y_eq,i Z_i
    Yeq: list


def interior_blocks(g: RWG, phys: Physics, qp: QuadParams = QuadParams(), Ix=None):
    """Z_i (4), Y_eq,i (5) and M_i = Y_eq,i Z_i (6) for every object, by dense LU."""
    if Ix is None:
        Ix, _ = matrix_Ix_and_gram(g)
    Zs, Ms, Ys = [], [], []
    w = phys.omega
    for i in range(g.n_obj):
        e0, e1 = g.obj_edge_off[i], g.obj_edge_off[i + 1]
        Ixi = Ix[e0:e1, e0:e1]
        Lc, Kc = interior_LK(g, i, phys.kc, qp)
        Z = (-1.0 / (1j * w * phys.eps_c)) * np.linalg.solve(Lc, Kc + 0.5 * Ixi)
        Ll, Kl = interior_LK(g, i, phys.k0, qp)
        Y = (1.0 / (1j * w * MU0)) * np.linalg.solve(Ll, Kl + 0.5 * Ixi)
        Zs.append(Z)
        Ys.append(Y)
        Ms.append(Y @ Z)
    return Interior(Zs, Ms, Ys)


@dataclass
class DenseSystem:
    """Everything the system product (7)-(8) needs, dense and in FP64."""
    g: RWG
    phys: Physics
    LA: np.ndarray
    Lphi: np.ndarray
    Ix: np.ndarray
    D: np.ndarray
    inner: Interior

    def apply_blocks(self, blocks, H):
        out = np.zeros_like(H)
        for i, Bi in enumerate(blocks):
            e0, e1 = self.g.obj_edge_off[i], self.g.obj_edge_off[i + 1]
            out[e0:e1] = Bi @ H[e0:e1]
        return out

    def matvec(self, x):
        """y = A x for x = [H; c0 rho] (eq. (7)-(8)); returns y and the parts."""
        g = self.g
        ne = g.n_e
        H, crho = x[:ne], x[ne:]
        e = self.apply_blocks(self.inner.Z, H)
        gq = self.apply_blocks(self.inner.M, H)
        j = H - gq
        q = g.area * crho                       # B c0 rho
        a = self.LA @ j
        phi = self.Lphi @ q
        k0 = self.phys.k0
        y1 = 1j * k0 * a + self.D.T @ phi + self.Ix @ e / ETA0
        y2 = -(self.D @ j) / g.area + 1j * k0 * crho    # F D j + j k0 c0 rho
        return np.concatenate([y1, y2]), dict(e=e, g=gq, j=j, a=a, phi=phi)

    def dense(self):
        """Explicit system matrix of (7) (only for small cases)."""
        g = self.g
        ne, nt = g.n_e, g.n_t
        Z = np.zeros((ne, ne), dtype=complex)
        M = np.zeros((ne, ne), dtype=complex)
        for i in range(g.n_obj):
            e0, e1 = g.obj_edge_off[i], g.obj_edge_off[i + 1]
            Z[e0:e1, e0:e1] = self.inner.Z[i]
            M[e0:e1, e0:e1] = self.inner.M[i]
        k0 = self.phys.k0
        B = np.diag(g.area)
        F = -np.diag(1.0 / g.area)
        A = np.zeros((ne + nt, ne + nt), dtype=complex)
        Y = np.zeros((ne, ne), dtype=complex)
        for i in range(g.n_obj):
            e0, e1 = g.obj_edge_off[i], g.obj_edge_off[i + 1]
            Y[e0:e1, e0:e1] = self.inner.Yeq[i]
        C = (-1j * k0 * self.LA @ Y + self.Ix / ETA0) @ Z          # eq. (8)
        A[:ne, :ne] = 1j * k0 * self.LA + C
        A[:ne, ne:] = self.D.T @ self.Lphi @ B
        A[ne:, :ne] = F @ self.D @ (np.eye(ne) - M)
        A[ne:, ne:] = 1j * k0 * np.eye(nt)
        return A


def dense_system(g: RWG, phys: Physics, qp: QuadParams = QuadParams()):
    LA, Lphi = external_dense(g, phys, qp)
    Ix, _ = matrix_Ix_and_gram(g)
    inner = interior_blocks(g, phys, qp, Ix)
    return DenseSystem(g, phys, LA, Lphi, Ix, matrix_D(g), inner)


def planewave_rhs(g: RWG, phys: Physics, khat, epol, n=4):
    """[E_inc/eta0 tested with f_m; 0] for E_inc = epol e^{-j k0 khat.r} (right side of (7))."""
    from .quad import tri_points
    V = g.verts[g.tris]
    pts, w = tri_points(V, n)
    E = np.asarray(epol, dtype=complex)[None, None, :] * np.exp(
        -1j * phys.k0 * np.einsum('bpk,k->bp', pts, np.asarray(khat, dtype=float)))[..., None]
    b = np.zeros(g.n_e + g.n_t, dtype=complex)
    for i in range(3):
        p = V[np.arange(g.n_t), i][:, None, :]
        f = (g.tri_sign[:, i] * g.length[g.tri_edge[:, i]] / (2.0 * g.area))[:, None, None] * (pts - p)
        np.add.at(b, g.tri_edge[:, i], np.sum(w[..., None] * f * E, axis=(1, 2)) / ETA0)
    return b
