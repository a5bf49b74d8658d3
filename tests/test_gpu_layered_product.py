"""GPU parity of the whole system product (7)-(8) over a layered background.

The oracle's layered AIM operator (oracle/aim.py: build_aim_layered) builds its reflected
near entries with TRI(2) on both triangles, and its reflected grid part from direct
Sommerfeld integrals. The library interpolates a table of the integrated remainders and
adds the closed-form large-k_rho terms back. It convolves the vector components and the
charge on two streams.

Tolerances:
  * FP64: 1e-6 relative, as for the free-space AIM parity (Y_eq conditioning), and 1e-7 for
    phi (the table interpolation, about 1e-9 of the reflected kernels);
  * mixed: 1e-5.
"""
import numpy as np
import pytest

from inputs.geometry import box_mesh, merge, random_complex
from tests.gpu_util import context, rel, run_parts

pytestmark = pytest.mark.gpu

FP64, MIXED = 0, 1
FREQ = 10e9
UM = 1e-6


def _mesh():
    return merge([box_mesh((0.0, 0.0, 3 * UM), (4 * UM, 2 * UM, 2 * UM), (2, 1, 1)),
                  box_mesh((6 * UM, 1 * UM, 2 * UM), (2 * UM, 2 * UM, 3 * UM), (1, 1, 1))])


@pytest.fixture(scope="module")
def layered_case():
    from oracle import aim, mgf
    from oracle.operators import Physics, interior_blocks
    from oracle.rwg import build_rwg, matrix_D, matrix_Ix_and_gram
    m = _mesh()
    g = build_rwg(m.verts, m.tris, m.obj, m.n_obj)
    grid = aim.make_grid(g.verts, (8, 8, 8))
    st = mgf.substrate_c4()
    st.z_if = grid.origin[2] - 1 * UM
    ph = Physics(FREQ)
    op = aim.build_aim_layered(g, grid, FREQ, st)
    Ix, _ = matrix_Ix_and_gram(g)
    inner = interior_blocks(g, ph, Ix=Ix)
    return (m, g, ph, op, Ix, matrix_D(g), inner), st


def _parts(case, x):
    from tests.test_gpu_parity import _oracle_aim_parts
    return _oracle_aim_parts(case, x)


TOL = {FP64: dict(e=1e-11, g=1e-6, a=1e-6, phi=1e-7, y=1e-6), MIXED: dict(e=1e-5, g=1e-5, a=1e-5, phi=1e-5, y=1e-5)}


def _check(got, ref, ne, prec):
    for k in ('e', 'g', 'a', 'phi'):
        assert rel(got[k], ref[k]) <= TOL[prec][k], (prec, k, rel(got[k], ref[k]))
    assert rel(got['y'][:ne], ref['y'][:ne]) <= TOL[prec]['y']
    assert rel(got['y'][ne:], ref['y'][ne:]) <= TOL[prec]['y']


def _set(ctx, st):
    ctx.set_medium(st.z_if, st.layers, st.bottom)


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_layered_product_parity(layered_case, prec):
    case, st = layered_case
    ctx, lay = context(case[0], freq=FREQ, grid=(8, 8, 8), precond=0)
    assert lay.nnz_near_A == case[3].LA_nr.nnz and lay.nnz_near_phi == case[3].Lphi_nr.nnz
    _set(ctx, st)
    for seed in (4, 5):
        x = random_complex(lay.n_e + lay.n_t, seed)
        _check(run_parts(ctx, lay, prec, x), _parts(case, x), lay.n_e, prec)


def test_layered_graph_and_medium_replacement(layered_case):
    """The default (captured, two-stream) product equals the staged one after a medium is set;
    replacing the medium starts again from the free-space near field."""
    import torch
    from oracle import mgf
    case, st = layered_case
    ctx, lay = context(case[0], freq=FREQ, grid=(8, 8, 8), precond=0)
    x = random_complex(lay.n_sys, 9)
    xt = torch.tensor(x, device='cuda')
    y = torch.zeros_like(xt)
    ctx.matvec(FP64, xt, y)                       # captures a free-space graph
    torch.cuda.synchronize()
    free = y.cpu().numpy()
    other = mgf.Stack([(3 * UM, 4.0, 0.0)], "pec", z_if=st.z_if)
    _set(ctx, other)
    _set(ctx, st)                                 # replaces the first medium
    for rep in range(3):
        ctx.matvec(FP64, xt, y)
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        staged = run_parts(ctx, lay, FP64, x)['y']
        assert rel(got, staged) <= 1e-13, rep
    ref = _parts(case, x)['y']
    ne = lay.n_e
    assert rel(got[:ne], ref[:ne]) <= 1e-6 and rel(got[ne:], ref[ne:]) <= 1e-6
    assert rel(free[:ne], ref[:ne]) > 1e-3        # the substrate changes the RWG rows


def _free_case(m, freq, N):
    from oracle import aim
    from oracle.operators import Physics, interior_blocks
    from oracle.rwg import build_rwg, matrix_D, matrix_Ix_and_gram
    g = build_rwg(m.verts, m.tris, m.obj, m.n_obj)
    ph = Physics(freq)
    grid = aim.make_grid(g.verts, N)
    op = aim.build_aim(g, grid, ph.k0, lambda a, b: aim.exact_entries(g, ph.k0, a, b),
                       lambda a, b: aim.exact_phi_entries(g, ph.k0, a, b))
    Ix, _ = matrix_Ix_and_gram(g)
    return (m, g, ph, op, Ix, matrix_D(g), interior_blocks(g, ph, Ix=Ix))


def test_rebuild_starts_in_free_space(layered_case):
    """A build after a medium was set is a free-space operator again (here at another
    frequency and on a larger grid, where the old reflected spectra would not even fit),
    and a medium set after a further rebuild matches the layered oracle."""
    case, st = layered_case
    m = case[0]
    ctx, lay = context(m, freq=FREQ, grid=(8, 8, 8), precond=0)
    _set(ctx, st)
    # 16 x 8 x 8 keeps the grid spacing (0.6 um) of the first build: on a finer grid the
    # stencils of these 2 um triangles would be too small, the near and grid parts would
    # cancel to 1/1700 of their size and complex64 would lose 3e-4 (measured on the CPU)
    lay2 = ctx.build(freq=5e9, grid=(16, 8, 8), precond=0)
    free = _free_case(m, 5e9, (16, 8, 8))
    x = random_complex(lay2.n_sys, 14)
    for prec in (FP64, MIXED):
        _check(run_parts(ctx, lay2, prec, x), _parts(free, x), lay2.n_e, prec)
    lay3 = ctx.build(freq=FREQ, grid=(8, 8, 8), precond=0)
    _set(ctx, st)
    _check(run_parts(ctx, lay3, FP64, x), _parts(case, x), lay3.n_e, FP64)


def test_bad_medium_leaves_context_unchanged(layered_case):
    """An argument error of slim_set_medium keeps the medium that was set: the captured and
    the staged products are bit for bit those from before the failed call."""
    import torch
    from paper_2108_03991_amd import slim
    case, st = layered_case
    ctx, lay = context(case[0], freq=FREQ, grid=(8, 8, 8), precond=0)
    _set(ctx, st)
    x = random_complex(lay.n_sys, 15)
    xt = torch.tensor(x, device='cuda')
    y = torch.zeros_like(xt)
    ctx.matvec(FP64, xt, y)
    torch.cuda.synchronize()
    graph0, staged0 = y.cpu().numpy(), run_parts(ctx, lay, FP64, x)['y']
    for bad in (dict(z_interface=st.z_if, layers=[(-1.0, 11.9, 10.0)], bottom="pec"),
                dict(z_interface=st.z_if + 1.0, layers=st.layers, bottom="pec")):
        with pytest.raises(slim.SlimError) as ei:
            ctx.set_medium(**bad)
        assert ei.value.code == 1
        y.zero_()
        ctx.matvec(FP64, xt, y)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), graph0)
        assert np.array_equal(run_parts(ctx, lay, FP64, x)['y'], staged0)
    ref = _parts(case, x)['y']
    assert rel(graph0[:lay.n_e], ref[:lay.n_e]) <= 1e-6
