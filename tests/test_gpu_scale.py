"""Sampled parity at a size beyond 2^26 near-field non-zeros.

Four hundred copper conductors in a 256 um cube on a coarse AIM grid (64^3, h
of about 4 um) give more than 2^26 near-field non-zeros per operator. That is
more than one dispatch of the one-wave-per-entry kernels can hold (a dispatch
has fewer than 2^32 work-items). Entries sampled over the whole CSR, tail
included, are compared with the oracle's exact entries minus its grid part,
each computed one by one. The stencil centres are compared index for index.
"""
import numpy as np
import pytest

from inputs.geometry import conductors_c5
from oracle import aim
from oracle.operators import Physics
from oracle.rwg import build_rwg
from tests.gpu_util import context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big_case():
    m = conductors_c5(seed=0, n_obj=400, t_max=2000, cube=256e-6)
    g = build_rwg(m.verts, m.tris, m.obj, m.n_obj)
    grid = aim.make_grid(g.verts, (64, 64, 64))
    cE, wE, cT, wT = aim.stencil_weights(grid, g)
    print("case: 400 conductors, grid 64^3, n_e", g.n_e, flush=True)
    ctx, lay = context(m, freq=5e9, grid=(64, 64, 64))
    return m, g, grid, (cE, wE, cT, wT), ctx, lay


def test_stencil_centres_and_grid(big_case):
    m, g, grid, (cE, wE, cT, wT), ctx, lay = big_case
    assert np.allclose(np.array(lay.grid_h), grid.h, rtol=1e-14, atol=0)
    ce, we, ct, wt = ctx.get_aim(lay.n_e, lay.n_t)
    assert np.array_equal(ce, cE) and np.array_equal(ct, cT)


@pytest.mark.parametrize("which", [0, 1])
def test_near_field_sampled_over_whole_csr(big_case, which):
    m, g, grid, (cE, wE, cT, wT), ctx, lay = big_case
    k0 = Physics(5e9).k0
    rows = lay.n_e if which == 0 else lay.n_t
    nnz = lay.nnz_near_A if which == 0 else lay.nnz_near_phi
    if which == 0:
        assert nnz > 2 ** 26, "the case must need more than one dispatch"
    ptr, col, val = ctx.get_near(which, rows, nnz)
    rng = np.random.default_rng(3)
    z = np.unique(np.concatenate([rng.integers(0, nnz, 150), np.arange(nnz - 40, nnz)]))
    r = np.searchsorted(ptr, z, side='right') - 1
    c = col[z]
    if which == 0:
        ref = aim.exact_entries(g, k0, r, c) - aim.grid_part(grid, k0, cE, wE, cE, wE, r, c)
    else:
        ref = (aim.exact_phi_entries(g, k0, r, c) - aim.grid_part(grid, k0, cT, wT, cT, wT, r, c)) * g.area[c]
    scale = np.abs(ref).max()
    err = np.abs(val[z] - ref)
    assert err.max() <= 1e-9 * scale, (err.max() / scale, int(z[np.argmax(err)]))


def test_conductor_blocks_invert_the_operators_self_part(big_case):
    """A property that holds at any size: for x supported on one conductor, the rows
    of S A x on that conductor are that conductor's block times x. So applying the
    block inverse gives back x, up to the complex64 storage of the inverse.

    This checks the operator and the preconditioner against each other, and it
    fails if either drops part of a conductor's self interaction (the near field,
    the grid part or the internal blocks)."""
    import torch
    from inputs.geometry import random_complex
    m, g, grid, _, ctx, lay = big_case
    assert lay.precond_blocks > 0
    n = lay.n_sys
    h = lay.mean_edge
    s = torch.cat([torch.full((lay.n_e,), 1.0 / h ** 2, dtype=torch.float64),
                   torch.full((lay.n_t,), h, dtype=torch.float64)]).cuda()
    blocks = ctx.get_precond()
    whole = [b for b in blocks if len(b[1]) == len(b[0])]
    rng = np.random.default_rng(2)
    for k in rng.choice(len(whole), 6, replace=False):
        ext = whole[k][0]
        idx = torch.tensor(ext, device='cuda')
        x = torch.zeros(n, dtype=torch.complex128, device='cuda')
        x[idx] = torch.tensor(random_complex(len(ext), int(k)), device='cuda')
        y = torch.zeros_like(x)
        ctx.matvec(0, x, y)
        z = torch.zeros_like(x)
        ctx.precond_apply(y * s, z)
        torch.cuda.synchronize()
        err = float(torch.linalg.norm((z - x)[idx]) / torch.linalg.norm(x))
        assert err <= 1e-2, (int(k), len(ext), err)
