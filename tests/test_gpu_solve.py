"""GMRES and GMRES-IR through the C ABI vs the oracle's dense LU solution (C1 bar)."""
import numpy as np
import pytest

from inputs.geometry import random_complex
from oracle.solve import lu_solve, row_scaling
from tests.gpu_util import context

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("use_precond", [False, True])
@pytest.mark.parametrize("prec", [0, 1])
def test_gmres_matches_lu(c1_mesh, c1_system, prec, use_precond):
    import torch
    ctx, lay = context(c1_mesh, freq=10e9, grid=(0, 0, 0))
    S = c1_system
    s = row_scaling(S.g.n_e, S.g.n_t, np.mean(S.g.length))
    assert abs(lay.mean_edge / np.mean(S.g.length) - 1) < 1e-14
    A = s[:, None] * S.dense()
    r = random_complex(A.shape[0], seed=0)            # right side of the equilibrated system
    xs = lu_solve(A, r)
    b = torch.tensor(r, device='cuda')
    x = torch.zeros_like(b)
    info, ok = ctx.solve(b, x, tol=1e-8, restart=300, max_iter=6000, prec=prec, inner_tol=1e-3,
                         scaled_rhs=True, use_precond=use_precond)
    assert ok and info.rel_residual <= 1e-8
    xg = x.cpu().numpy()
    cond = np.linalg.cond(A)
    assert np.linalg.norm(A @ xg - r) <= 1.01e-8 * np.linalg.norm(r) * 10
    assert np.linalg.norm(xg - xs) / np.linalg.norm(xs) <= 10 * cond * 1e-8
    if prec == 1 and not use_precond:
        assert info.n_matvec_mixed > info.n_matvec_fp64
    if use_precond:
        # one conductor: the block is the whole equilibrated system
        assert info.iterations <= 10 and info.n_precond == info.iterations


def test_gmres_not_converged_returns_best_iterate(c1_mesh):
    import torch
    ctx, lay = context(c1_mesh, freq=10e9, grid=(0, 0, 0))
    b = torch.tensor(random_complex(lay.n_sys, 1), device='cuda')
    x = torch.zeros_like(b)
    info, ok = ctx.solve(b, x, tol=1e-12, restart=20, max_iter=40, prec=0, scaled_rhs=True, use_precond=False)
    assert not ok and info.iterations == 40 and 0 < info.rel_residual < 1


def test_planewave_rhs_matches_oracle(c1_mesh, c1_rwg):
    """Right-hand side of (7) for a plane wave: tested incident field on the RWG rows,
    zero on the continuity rows (oracle: planewave_rhs, same TRI(4) rule, which is
    exact to rounding for this nearly linear integrand)."""
    import torch
    from oracle.operators import Physics, planewave_rhs
    ctx, lay = context(c1_mesh, freq=10e9, grid=(0, 0, 0), precond=0)
    for khat, epol in (((0.0, 0.0, -1.0), (1.0, 0.0, 0.0)), ((0.6, 0.0, 0.8), (0.0, 1.0, 0.0))):
        b = torch.zeros(lay.n_sys, dtype=torch.complex128, device='cuda')
        ctx.rhs_planewave(khat, epol, b)
        torch.cuda.synchronize()
        ref = planewave_rhs(c1_rwg, Physics(10e9), khat, epol)
        got = b.cpu().numpy()
        assert np.abs(got[lay.n_e:]).max() == 0.0
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
