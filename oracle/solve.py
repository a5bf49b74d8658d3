"""Solution of the SLIM system (7): dense LU and restarted FP64 GMRES.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper solves (7) with GMRES [Saad1986] (Sec. III-E) to a relative
residual of 1e-6 (bus) or 1e-4 (SRR, interposer).  Readings: x0 = 0,
restart m, classical Gram-Schmidt applied twice, Givens rotations for the
least-squares problem, and the residual norm of the row-equilibrated system
S A x = S b with S = diag(1/h^2 on the N_E tested-EFIE rows, h on the N_T
continuity rows), h the mean edge length.  In SI units the two row blocks of
(7) differ by about h^3 (cond ~ 1e26 for the 2 um bar); S is exactly the
change of length unit to h, which the paper leaves unstated, and it leaves
the solution unchanged.  gmres() applies no other preconditioner; fgmres()
takes one (the conductor-block preconditioner of precond.py stands in for the
paper's constraint preconditioner [Qian2009], whose definition the paper does
not give).
"""
from __future__ import annotations

import numpy as np


def row_scaling(n_e, n_t, mean_edge):
    """Diagonal S of the equilibrated system S A x = S b (see the module docstring)."""
    return np.concatenate([np.full(n_e, 1.0 / mean_edge ** 2), np.full(n_t, mean_edge)])


def lu_solve(A, b):
    return np.linalg.solve(A, b)


def gmres(matvec, b, tol=1e-8, restart=100, max_iter=5000, x0=None):
    """Restarted GMRES(m); returns x, iterations, true relative residual history."""
    n = b.size
    x = np.zeros(n, dtype=complex) if x0 is None else x0.astype(complex).copy()
    bn = np.linalg.norm(b)
    hist = []
    it = 0
    while it < max_iter:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        hist.append(beta / bn)
        if beta / bn <= tol:
            break
        m = min(restart, max_iter - it)
        V = np.zeros((m + 1, n), dtype=complex)
        Hh = np.zeros((m + 1, m), dtype=complex)
        V[0] = r / beta
        cs = np.zeros(m, dtype=complex)
        sn = np.zeros(m, dtype=complex)
        gvec = np.zeros(m + 1, dtype=complex)
        gvec[0] = beta
        k_used = 0
        for k in range(m):
            w = matvec(V[k])
            for _ in range(2):
                h = V[:k + 1].conj() @ w
                w = w - V[:k + 1].T @ h
                Hh[:k + 1, k] += h
            Hh[k + 1, k] = np.linalg.norm(w)
            if Hh[k + 1, k] != 0:
                V[k + 1] = w / Hh[k + 1, k]
            # rotation [[conj(c), conj(s)], [-s, c]] with c = a/den, s = b/den zeroes b
            for i in range(k):
                t = np.conj(cs[i]) * Hh[i, k] + np.conj(sn[i]) * Hh[i + 1, k]
                Hh[i + 1, k] = -sn[i] * Hh[i, k] + cs[i] * Hh[i + 1, k]
                Hh[i, k] = t
            a, bb = Hh[k, k], Hh[k + 1, k]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            cs[k], sn[k] = (a / den, bb / den) if den > 0 else (1.0, 0.0)
            Hh[k, k] = den
            Hh[k + 1, k] = 0.0
            gvec[k + 1] = -sn[k] * gvec[k]
            gvec[k] = np.conj(cs[k]) * gvec[k]
            it += 1
            k_used = k + 1
            if abs(gvec[k + 1]) / bn <= tol * 0.5 or it >= max_iter:
                break
        y = np.linalg.solve(np.triu(Hh[:k_used, :k_used]), gvec[:k_used])
        x = x + V[:k_used].T @ y
    return x, it, hist


def fgmres(matvec, precond, b, tol=1e-8, restart=100, max_iter=5000):
    """Restarted flexible GMRES with right preconditioning [Saad1993].

    Each basis vector's preconditioned image z_k = precond(v_k) is kept and the
    update is x += sum_k y_k z_k, so a preconditioner that is applied in reduced
    precision (not an exactly linear map) still gives a consistent update.
    Same Gram-Schmidt, rotations and stopping rule as gmres().
    """
    n = b.size
    x = np.zeros(n, dtype=complex)
    bn = np.linalg.norm(b)
    hist = []
    it = 0
    while it < max_iter:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        hist.append(beta / bn)
        if beta / bn <= tol:
            break
        m = min(restart, max_iter - it)
        V = np.zeros((m + 1, n), dtype=complex)
        Zb = np.zeros((m, n), dtype=complex)
        Hh = np.zeros((m + 1, m), dtype=complex)
        V[0] = r / beta
        cs = np.zeros(m, dtype=complex)
        sn = np.zeros(m, dtype=complex)
        gvec = np.zeros(m + 1, dtype=complex)
        gvec[0] = beta
        k_used = 0
        for k in range(m):
            Zb[k] = precond(V[k])
            w = matvec(Zb[k])
            for _ in range(2):
                h = V[:k + 1].conj() @ w
                w = w - V[:k + 1].T @ h
                Hh[:k + 1, k] += h
            Hh[k + 1, k] = np.linalg.norm(w)
            if Hh[k + 1, k] != 0:
                V[k + 1] = w / Hh[k + 1, k]
            for i in range(k):
                t = np.conj(cs[i]) * Hh[i, k] + np.conj(sn[i]) * Hh[i + 1, k]
                Hh[i + 1, k] = -sn[i] * Hh[i, k] + cs[i] * Hh[i + 1, k]
                Hh[i, k] = t
            a, bb = Hh[k, k], Hh[k + 1, k]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            cs[k], sn[k] = (a / den, bb / den) if den > 0 else (1.0, 0.0)
            Hh[k, k] = den
            Hh[k + 1, k] = 0.0
            gvec[k + 1] = -sn[k] * gvec[k]
            gvec[k] = np.conj(cs[k]) * gvec[k]
            it += 1
            k_used = k + 1
            if abs(gvec[k + 1]) / bn <= tol * 0.5 or it >= max_iter:
                break
        y = np.linalg.solve(np.triu(Hh[:k_used, :k_used]), gvec[:k_used])
        x = x + Zb[:k_used].T @ y
    return x, it, hist
