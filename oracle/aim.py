"""Adaptive integral method, eq. (11): L ~ L_NR + W H P (Sec. III-A).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper names the pieces (P projects basis functions onto a uniform grid,
H is the grid convolution done by FFT, W interpolates back, L_NR is the
precorrected near field) and leaves the details to [Bleszynski1996] and
[Phillips1997].  Readings used on both sides of this project:

  * grid: N_c nodes per axis, spacing h_c = max(ext_c/(N_c-3), H/4) with
    H = max_c ext_c/(N_c-3) (ext = vertex bounding box), centred on the box;
  * expansion order M = 2: the stencil of a basis function is the 3x3x3 block
    of nodes centred on the node nearest its centre (RWG: mean of the two
    triangle centroids; pulse: centroid);
  * stencil weights match every moment (r - r0)^alpha, 0 <= alpha_c <= 2, of the
    source about the stencil centre r0; for the Cartesian components of an RWG
    function and for the pulse h_t / A_t;
  * W = P^T (Galerkin testing);
  * grid kernel G(Delta) = e^{-j k0 R}/(4 pi R), R = |Delta o h|, and G(0) = 0;
    aperiodic convolution by zero padding to 2 N_c per axis;
  * near zone: stencil centres within Chebyshev index distance 3;
  * precorrection: L_NR[m,n] = L[m,n] - sum_c P_c[:,m]^T G P_c[:,n] on near pairs.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .quad import tri_points
from .rwg import RWG

NEAR_CHEB = 3


@dataclass
class Grid:
    N: np.ndarray       # (3,) int nodes per axis
    h: np.ndarray       # (3,) spacing
    origin: np.ndarray  # (3,)

    @property
    def n_nodes(self):
        return int(np.prod(self.N))

    def node_pos(self, idx):
        return self.origin + np.asarray(idx) * self.h

    def linear(self, idx):
        idx = np.asarray(idx)
        return (idx[..., 2] * self.N[1] + idx[..., 1]) * self.N[0] + idx[..., 0]


def make_grid(verts, N):
    N = np.asarray(N, dtype=np.int64)
    lo, hi = verts.min(axis=0), verts.max(axis=0)
    ext = hi - lo
    H = np.max(ext / (N - 3))
    h = np.maximum(ext / (N - 3), H / 4.0)
    center = 0.5 * (lo + hi)
    origin = center - h * (N - 1) / 2.0
    return Grid(N, h, origin)


def basis_centres(g: RWG):
    rc = 0.5 * (g.centroid[g.tplus] + g.centroid[g.tminus])
    return rc, g.centroid.copy()


def stencil_centre(grid: Grid, pts):
    idx = np.rint((pts - grid.origin) / grid.h).astype(np.int64)
    if np.any(idx < 1) or np.any(idx > grid.N - 2):
        raise ValueError("stencil leaves the grid")
    return idx


OFFS = np.array([(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)])
ALPHAS = np.array([(ax, ay, az) for az in range(3) for ay in range(3) for ax in range(3)])


def _moment_matrix():
    """V[alpha, node] = prod_c offset_c^alpha_c for the 27 stencil nodes (offsets in units of h)."""
    return np.prod(OFFS[None, :, :].astype(float) ** ALPHAS[:, None, :], axis=2)


def stencil_weights(grid: Grid, g: RWG, order=5):
    """Solve the 27x27 moment systems for every RWG (3 components) and pulse.

    The moments are taken in grid units, sum_g w_g ((r_g - r0)/h)^alpha =
    int f ((r - r0)/h)^alpha dS, which is the same linear condition as in metres
    but keeps the Vandermonde matrix O(1) (in metres its rows differ by h^6).
    Returns (cidx_e (N_E,3), wE (N_E, 3 comps, 27), cidx_t (N_T,3), wT (N_T, 27)).
    """
    rcE, rcT = basis_centres(g)
    cE, cT = stencil_centre(grid, rcE), stencil_centre(grid, rcT)
    V = _moment_matrix()
    Vt = g.verts[g.tris]
    pts, w = tri_points(Vt, order)                       # (N_T, q, 3), (N_T, q)
    # RWG components: moments accumulated from both triangles
    momE = np.zeros((g.n_e, 3, 27))
    for i in range(3):
        n = g.tri_edge[:, i]
        r0 = grid.node_pos(cE[n])                         # (N_T,3)
        rel = (pts - r0[:, None, :]) / grid.h
        mono = np.prod(rel[:, :, None, :] ** ALPHAS[None, None, :, :], axis=3)   # (N_T,q,27)
        f = (g.tri_sign[:, i] * g.length[n] / (2.0 * g.area))[:, None, None] * (pts - Vt[:, i][:, None, :])
        np.add.at(momE, n, np.einsum('tq,tqc,tqa->tca', w, f, mono))
    r0 = grid.node_pos(cT)
    rel = (pts - r0[:, None, :]) / grid.h
    mono = np.prod(rel[:, :, None, :] ** ALPHAS[None, None, :, :], axis=3)
    momT = np.einsum('tq,tqa->ta', w, mono) / g.area[:, None]
    wE = np.linalg.solve(V[None, None], momE[..., None])[..., 0]
    wT = np.linalg.solve(V[None], momT[..., None])[..., 0]
    return cE, wE, cT, wT


def projection_matrices(grid: Grid, g: RWG):
    """Sparse P_x, P_y, P_z (nodes x N_E) and P_rho (nodes x N_T)."""
    cE, wE, cT, wT = stencil_weights(grid, g)
    nodesE = grid.linear(cE[:, None, :] + OFFS[None])      # (N_E,27)
    nodesT = grid.linear(cT[:, None, :] + OFFS[None])
    colsE = np.repeat(np.arange(g.n_e), 27)
    colsT = np.repeat(np.arange(g.n_t), 27)
    Pc = [sp.csr_matrix((wE[:, c, :].ravel(), (nodesE.ravel(), colsE)), shape=(grid.n_nodes, g.n_e))
          for c in range(3)]
    Pr = sp.csr_matrix((wT.ravel(), (nodesT.ravel(), colsT)), shape=(grid.n_nodes, g.n_t))
    return Pc, Pr, (cE, wE, nodesE), (cT, wT, nodesT)


def grid_kernel_value(grid: Grid, k0, delta):
    """G(Delta) = e^{-j k0 R}/(4 pi R), R = |Delta o h|; G(0) = 0."""
    R = np.sqrt(np.sum((np.asarray(delta) * grid.h) ** 2, axis=-1))
    with np.errstate(divide='ignore', invalid='ignore'):
        v = np.exp(-1j * k0 * R) / (4.0 * np.pi * R)
    return np.where(R > 0, v, 0.0)


def circulant_kernel(grid: Grid, k0):
    """G on the zero-padded (2N)^3 grid, index order [z, y, x]; offset N_c unused (0)."""
    axes = []
    for c in range(3):
        n2 = 2 * grid.N[c]
        o = np.arange(n2)
        o = np.where(o < grid.N[c], o, o - n2).astype(float)
        o[grid.N[c]] = np.nan
        axes.append(o)
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing='ij')
    d = np.stack([X, Y, Z], axis=-1)
    G = grid_kernel_value(grid, k0, np.nan_to_num(d, nan=0.0))
    G[np.isnan(d).any(axis=-1)] = 0.0
    return G


def convolve_fft(grid: Grid, Ghat, src):
    """Aperiodic grid convolution phi(g) = sum_g' G(g - g') src(g') via FFT (src in node order)."""
    Nx, Ny, Nz = grid.N
    S = np.zeros((2 * Nz, 2 * Ny, 2 * Nx), dtype=complex)
    S[:Nz, :Ny, :Nx] = src.reshape(Nz, Ny, Nx)
    out = np.fft.ifftn(Ghat * np.fft.fftn(S))
    return out[:Nz, :Ny, :Nx].ravel()


def convolve_direct(grid: Grid, k0, src):
    """Brute-force sum over all node pairs (tiny grids only)."""
    Nx, Ny, Nz = grid.N
    idx = np.stack(np.meshgrid(np.arange(Nx), np.arange(Ny), np.arange(Nz), indexing='ij'), -1)
    idx = idx.transpose(2, 1, 0, 3).reshape(-1, 3)        # node order x fastest
    d = idx[:, None, :] - idx[None, :, :]
    Gm = grid_kernel_value(grid, k0, d)
    return Gm @ src


def near_pairs(cA, cB, symmetric=True):
    """Index pairs (m, n) whose stencil centres are within Chebyshev distance NEAR_CHEB."""
    from scipy.spatial import cKDTree
    tA = cKDTree(cA.astype(float))
    tB = tA if symmetric else cKDTree(cB.astype(float))
    pairs = tA.query_ball_tree(tB, r=NEAR_CHEB + 0.5, p=np.inf)
    m = np.repeat(np.arange(len(pairs)), [len(p) for p in pairs])
    n = np.concatenate([np.asarray(p, dtype=np.int64) for p in pairs]) if len(pairs) else np.zeros(0, np.int64)
    return m, n


def grid_part(grid: Grid, k0, cA, wA, cB, wB, m, n):
    """sum over components and stencil nodes of wA[m] G(node_m - node_n) wB[n] (per pair)."""
    out = np.zeros(m.size, dtype=complex)
    d = OFFS[:, None, :] - OFFS[None, :, :]                 # (27,27,3)
    for lo in range(0, m.size, 20000):
        s = slice(lo, lo + 20000)
        delta = (cA[m[s]] - cB[n[s]])[:, None, None, :] + d[None]
        Gs = grid_kernel_value(grid, k0, delta)             # (B,27,27)
        if wA.ndim == 3:
            out[s] = np.einsum('bcx,bxy,bcy->b', wA[m[s]], Gs, wB[n[s]], optimize=True)
        else:
            out[s] = np.einsum('bx,bxy,by->b', wA[m[s]], Gs, wB[n[s]], optimize=True)
    return out


@dataclass
class AIMOperator:
    grid: Grid
    k0: float
    Pc: list
    Pr: object
    Ghat: np.ndarray
    LA_nr: object     # sparse N_E x N_E
    Lphi_nr: object   # sparse N_T x N_T

    def apply_LA(self, j):
        far = sum(P.T @ convolve_fft(self.grid, self.Ghat, P @ j) for P in self.Pc)
        return self.LA_nr @ j + far

    def apply_Lphi(self, q):
        return self.Lphi_nr @ q + self.Pr.T @ convolve_fft(self.grid, self.Ghat, self.Pr @ q)


def build_aim(g: RWG, grid: Grid, k0, LA_exact, Lphi_exact):
    """O-aim from exact near entries.  LA_exact(m, n) / Lphi_exact(t, u) return entries."""
    Pc, Pr, (cE, wE, _), (cT, wT, _) = projection_matrices(grid, g)
    Ghat = np.fft.fftn(circulant_kernel(grid, k0))
    m, n = near_pairs(cE, cE)
    vA = LA_exact(m, n) - grid_part(grid, k0, cE, wE, cE, wE, m, n)
    t, u = near_pairs(cT, cT)
    vP = Lphi_exact(t, u) - grid_part(grid, k0, cT, wT, cT, wT, t, u)
    LA_nr = sp.csr_matrix((vA, (m, n)), shape=(g.n_e, g.n_e))
    Lphi_nr = sp.csr_matrix((vP, (t, u)), shape=(g.n_t, g.n_t))
    return AIMOperator(grid, k0, Pc, Pr, Ghat, LA_nr, Lphi_nr)


def exact_entries(g: RWG, k0, m, n, qp=None):
    """Exact L_A[m, n] (RWG pairs) from the triangle-pair integrals, without the dense matrix.

    Each triangle pair is integrated with the lower triangle index as test
    triangle (the orientation of the dense assembly) and transposed otherwise.
    """
    from .operators import triangle_pair_integrals
    from .quad import QuadParams
    qp = qp or QuadParams()
    m = np.asarray(m)
    n = np.asarray(n)
    Tm = np.stack([g.tplus[m], g.tminus[m]], 1)
    Tn = np.stack([g.tplus[n], g.tminus[n]], 1)
    keys = []
    for a in range(2):
        for b in range(2):
            t, u = Tm[:, a], Tn[:, b]
            keys.append(np.stack([np.minimum(t, u), np.maximum(t, u)], 1))
    allk = np.unique(np.concatenate(keys), axis=0)
    IA, IS, _ = triangle_pair_integrals(g, allk[:, 0], allk[:, 1], k0, qp, want_k=False)
    key = allk[:, 0] * np.int64(g.n_t) + allk[:, 1]
    out = np.zeros(m.size, dtype=complex)
    for a in range(2):
        for b in range(2):
            t, u = Tm[:, a], Tn[:, b]
            i = np.argmax(g.tri_edge[t] == m[:, None], axis=1)
            j = np.argmax(g.tri_edge[u] == n[:, None], axis=1)
            p = np.searchsorted(key, np.minimum(t, u) * np.int64(g.n_t) + np.maximum(t, u))
            v = np.where(t <= u, IA[p, i, j], IA[p, j, i])
            out += (g.tri_sign[t, i] * g.tri_sign[u, j] * g.length[m] * g.length[n]
                    / (4.0 * g.area[t] * g.area[u])) * v
    return out


def exact_phi_entries(g: RWG, k0, t, u, qp=None):
    """Exact L_phi[t, u] = IS / (A_t A_u) for triangle pairs."""
    from .operators import triangle_pair_integrals
    from .quad import QuadParams
    qp = qp or QuadParams()
    t = np.asarray(t)
    u = np.asarray(u)
    lo, hi = np.minimum(t, u), np.maximum(t, u)
    _, IS, _ = triangle_pair_integrals(g, lo, hi, k0, qp, want_k=False)
    return IS / (g.area[t] * g.area[u])


def convolve_layered_direct(grid: Grid, freq, stack, src, targets=None):
    """Grid potentials over a layered medium by brute force over all node pairs (tiny grids only).

    src: (4, nodes) grid sources of the x, y, z current components and of the
    charge.  targets: node indices (x fastest) at which the potentials are
    summed; None means every node.  With a few targets the sum stays cheap on
    larger grids, since every target is still summed over all sources.  The kernel is the free-space grid kernel above (G(0) = 0) plus the
    reflected dyadic of oracle/mgf.py:
      Phi_x = (g + xx_r) * S_x + G_xz * S_z,   Phi_y = (g + xx_r) * S_y + G_yz * S_z,
      Phi_z = G_zx * S_x + G_zy * S_y + (g + zz_r) * S_z,   Phi_rho = (g + phi_r) * S_rho.
    The reflected parts depend on the in-plane offset and on z + z' (correlation in z).
    """
    from . import mgf
    k0 = 2.0 * np.pi * freq / mgf.C0
    Nx, Ny, Nz = grid.N
    idx = np.stack(np.meshgrid(np.arange(Nx), np.arange(Ny), np.arange(Nz), indexing='ij'), -1)
    idx = idx.transpose(2, 1, 0, 3).reshape(-1, 3)        # node order x fastest
    tgt = idx if targets is None else idx[np.asarray(targets)]
    d = tgt[:, None, :] - idx[None, :, :]
    Gp = grid_kernel_value(grid, k0, d)
    z0 = grid.origin[2] - stack.z_if
    if z0 <= 0:
        raise ValueError("the AIM grid reaches below the interface")
    # reflected kernels on the distinct (|dx|, |dy|, iz + iz') triples
    ax, ay, s = np.abs(d[..., 0]), np.abs(d[..., 1]), tgt[:, None, 2] + idx[None, :, 2]
    key = (ax * Ny + ay) * (2 * Nz) + s
    uk, inv = np.unique(key.ravel(), return_inverse=True)
    rho = np.hypot((uk // (2 * Nz)) // Ny * grid.h[0], (uk // (2 * Nz)) % Ny * grid.h[1])
    zeta = 2.0 * z0 + (uk % (2 * Nz)) * grid.h[2]
    k = mgf.reflected(stack, freq, rho, zeta)
    xx, zz, ph, zxr = (k[n][inv].reshape(key.shape) for n in ("xx", "zz", "phi", "zx"))
    dxm, dym = d[..., 0] * grid.h[0], d[..., 1] * grid.h[1]
    rr = np.hypot(dxm, dym)
    with np.errstate(invalid='ignore', divide='ignore'):
        cx = np.where(rr > 0, dxm / rr, 0.0)
        cy = np.where(rr > 0, dym / rr, 0.0)
    Sx, Sy, Sz, Sr = src
    out = np.zeros((4, tgt.shape[0]), dtype=complex)
    out[0] = (Gp + xx) @ Sx - (cx * zxr) @ Sz
    out[1] = (Gp + xx) @ Sy - (cy * zxr) @ Sz
    out[2] = (cx * zxr) @ Sx + (cy * zxr) @ Sy + (Gp + zz) @ Sz
    out[3] = (Gp + ph) @ Sr
    return out


# ---- layered background: reflected near-field entries and their grid part ----
# Readings (the reflected kernel is smooth at the triangle scale, since every point
# lies above the interface): the reflected parts of the near entries are integrated
# with TRI(2) on both triangles; the precorrection subtracts the reflected dyadic's
# grid part as well, so that L_NR = L_exact - W G_total P on near pairs.

REFL_ORDER = 2


def _tri_rule(g: RWG, order=REFL_ORDER):
    Vt = g.verts[g.tris]
    return tri_points(Vt, order)          # (N_T, q, 3), (N_T, q) with weights summing to A_t


def _reflected_pair_integrals(g: RWG, freq, stack, T, U, order=REFL_ORDER):
    """For triangle pairs (T[b], U[b]), TRI(order) x TRI(order) (TRI(2) by default):
    IA[b, i, j] = int int (r - v_i) . G_r(r, r') . (r' - v_j) and IS[b] = int int phi_r."""
    from . import mgf
    pts, w = _tri_rule(g, order)
    q = pts.shape[1]
    ro = np.repeat(pts[T], q, axis=1).reshape(-1, 3)
    rs = np.tile(pts[U], (1, q, 1)).reshape(-1, 3)
    G, ph = mgf.dyadic_reflected(stack, freq, ro, rs)
    G = G.reshape(T.size, q, q, 3, 3)
    ww = w[T][:, :, None] * w[U][:, None, :]
    dt = pts[T][:, :, None, :] - g.verts[g.tris[T]][:, None, :, :]      # (B, q, 3 vertices, 3)
    du = pts[U][:, :, None, :] - g.verts[g.tris[U]][:, None, :, :]
    IA = np.einsum('bpq,bpia,bpqac,bqjc->bij', ww, dt, G, du)
    IS = np.einsum('bpq,bpq->b', ww, ph.reshape(T.size, q, q))
    return IA, IS


def reflected_entries(g: RWG, freq, stack, m, n, order=REFL_ORDER):
    """Reflected part of L_A[m, n] (RWG pairs) from the triangle-pair integrals above."""
    m = np.asarray(m)
    n = np.asarray(n)
    Tm = np.stack([g.tplus[m], g.tminus[m]], 1)
    Tn = np.stack([g.tplus[n], g.tminus[n]], 1)
    keys = np.unique(np.concatenate([np.stack([Tm[:, a], Tn[:, b]], 1) for a in range(2) for b in range(2)]), axis=0)
    IA, _ = _reflected_pair_integrals(g, freq, stack, keys[:, 0], keys[:, 1], order)
    key = keys[:, 0] * np.int64(g.n_t) + keys[:, 1]
    out = np.zeros(m.size, dtype=complex)
    for a in range(2):
        for b in range(2):
            t, u = Tm[:, a], Tn[:, b]
            i = np.argmax(g.tri_edge[t] == m[:, None], axis=1)
            j = np.argmax(g.tri_edge[u] == n[:, None], axis=1)
            p = np.searchsorted(key, t * np.int64(g.n_t) + u)
            out += (g.tri_sign[t, i] * g.tri_sign[u, j] * g.length[m] * g.length[n]
                    / (4.0 * g.area[t] * g.area[u])) * IA[p, i, j]
    return out


def reflected_phi_entries(g: RWG, freq, stack, t, u, order=REFL_ORDER):
    """Reflected part of L_phi[t, u] = 1/(A_t A_u) int int phi_r, TRI(order) x TRI(order)."""
    t = np.asarray(t)
    u = np.asarray(u)
    _, IS = _reflected_pair_integrals(g, freq, stack, t, u, order)
    return IS / (g.area[t] * g.area[u])


def _lattice_reflected(grid: Grid, freq, stack):
    """Reflected kernels at every (|dx|, |dy|, iz + iz') of the grid: dict of (2Nz-1, Ny, Nx) arrays."""
    from . import mgf
    Nx, Ny, Nz = grid.N
    z0 = grid.origin[2] - stack.z_if
    if z0 <= 0:
        raise ValueError("the AIM grid reaches below the interface")
    s, iy, ix = np.meshgrid(np.arange(2 * Nz - 1), np.arange(Ny), np.arange(Nx), indexing='ij')
    k = mgf.reflected(stack, freq, np.hypot(ix * grid.h[0], iy * grid.h[1]).ravel(),
                      (2 * z0 + s * grid.h[2]).ravel())
    return {key: v.reshape(s.shape) for key, v in k.items()}


def grid_part_layered(grid: Grid, lat, cA, wA, cB, wB, m, n):
    """Reflected grid part of near entries: sum over stencil node pairs of wA . G_r . wB.

    wA/wB: (basis, 3, 27) RWG weights (dyadic) or (basis, 27) pulse weights (scalar kernel).
    G_r between nodes i and j uses the in-plane offset i - j and the z-index sum.
    """
    out = np.zeros(m.size, dtype=complex)
    for lo in range(0, m.size, 5000):
        s = slice(lo, lo + 5000)
        ni = (cA[m[s]][:, None, :] + OFFS[None])[:, :, None, :]                                    # (B,27,1,3)
        nj = (cB[n[s]][:, None, :] + OFFS[None])[:, None, :, :]                                    # (B,1,27,3)
        d = ni - nj
        ax, ay = np.abs(d[..., 0]), np.abs(d[..., 1])
        sz = ni[..., 2] + nj[..., 2]
        if wA.ndim == 2:
            G = lat["phi"][sz, ay, ax]
            out[s] = np.einsum('bi,bij,bj->b', wA[m[s]], G, wB[n[s]])
            continue
        xx, zz, zx = lat["xx"][sz, ay, ax], lat["zz"][sz, ay, ax], lat["zx"][sz, ay, ax]
        dx, dy = d[..., 0] * grid.h[0], d[..., 1] * grid.h[1]
        r = np.hypot(dx, dy)
        with np.errstate(invalid='ignore', divide='ignore'):
            cx = np.where(r > 0, dx / r, 0.0)
            cy = np.where(r > 0, dy / r, 0.0)
        A, B = wA[m[s]], wB[n[s]]                       # (B,3,27)
        v = np.einsum('bi,bij,bj->b', A[:, 0], xx, B[:, 0]) + np.einsum('bi,bij,bj->b', A[:, 1], xx, B[:, 1])
        v += np.einsum('bi,bij,bj->b', A[:, 2], zz, B[:, 2])
        v += np.einsum('bi,bij,bj->b', A[:, 2], cx * zx, B[:, 0]) - np.einsum('bi,bij,bj->b', A[:, 0], cx * zx, B[:, 2])
        v += np.einsum('bi,bij,bj->b', A[:, 2], cy * zx, B[:, 1]) - np.einsum('bi,bij,bj->b', A[:, 1], cy * zx, B[:, 2])
        out[s] = v
    return out


@dataclass
class LayeredAIMOperator:
    grid: Grid
    freq: float
    stack: object
    Pc: list
    Pr: object
    LA_nr: object
    Lphi_nr: object

    def apply_LA(self, j):
        S = np.zeros((4, self.grid.n_nodes), dtype=complex)
        for c in range(3):
            S[c] = self.Pc[c] @ j
        Phi = convolve_layered_direct(self.grid, self.freq, self.stack, S)
        return self.LA_nr @ j + sum(self.Pc[c].T @ Phi[c] for c in range(3))

    def apply_Lphi(self, q):
        S = np.zeros((4, self.grid.n_nodes), dtype=complex)
        S[3] = self.Pr @ q
        Phi = convolve_layered_direct(self.grid, self.freq, self.stack, S)
        return self.Lphi_nr @ q + self.Pr.T @ Phi[3]


def build_aim_layered(g: RWG, grid: Grid, freq, stack):
    """AIM over a layered background: near entries = exact (free + reflected) - grid (free + reflected)."""
    from . import mgf
    k0 = 2.0 * np.pi * freq / mgf.C0
    Pc, Pr, (cE, wE, _), (cT, wT, _) = projection_matrices(grid, g)
    lat = _lattice_reflected(grid, freq, stack)
    m, n = near_pairs(cE, cE)
    vA = (exact_entries(g, k0, m, n) + reflected_entries(g, freq, stack, m, n)
          - grid_part(grid, k0, cE, wE, cE, wE, m, n) - grid_part_layered(grid, lat, cE, wE, cE, wE, m, n))
    t, u = near_pairs(cT, cT)
    vP = (exact_phi_entries(g, k0, t, u) + reflected_phi_entries(g, freq, stack, t, u)
          - grid_part(grid, k0, cT, wT, cT, wT, t, u) - grid_part_layered(grid, lat, cT, wT, cT, wT, t, u))
    LA_nr = sp.csr_matrix((vA, (m, n)), shape=(g.n_e, g.n_e))
    Lphi_nr = sp.csr_matrix((vP, (t, u)), shape=(g.n_t, g.n_t))
    return LayeredAIMOperator(grid, freq, stack, Pc, Pr, LA_nr, Lphi_nr)
