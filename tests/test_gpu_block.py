"""The product on a block of right-hand sides (slim_matvec_block) and lumped ports.

Block product: in mixed precision the internal blocks of up to 64 columns run on the
matrix cores with split-BF16 operands (two BF16 terms per FP32 value, three products,
FP32 accumulation: about 2^-16 per product, 4.5e-6 measured on a real block by a CPU
emulation), the external part column by column.  Every column must match the oracle
within the mixed tolerance 1e-5 (relative 2-norm per row block), and the FP64 block
path the oracle within 1e-6, as the single-column products do.  Columns: 20 (one
16-column group and a ragged one of 4) on the AIM case, 70 (a launch of 64 and one of
6) on the dense bar.

Ports: the library's ring edges, signs and right-hand sides against the oracle's
(oracle/ports.py), the currents of given columns, and the admittance matrix of two
ports from GMRES solves against the oracle's dense LU: equal within the solve
tolerance and symmetric (reciprocity).
"""
import numpy as np
import pytest

from inputs.geometry import box_mesh, merge, random_complex
from tests.gpu_util import context, rel
from tests.test_gpu_parity import _oracle_aim_parts, boxes_case  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu

FP64, MIXED = 0, 1


def _block(ctx, lay, prec, X):
    import torch
    Xt = torch.tensor(X.T.copy(), dtype=torch.complex128, device='cuda')      # column-major: [col][row]
    Yt = torch.zeros_like(Xt)
    ctx.matvec_block(prec, Xt, Yt, X.shape[1])
    torch.cuda.synchronize()
    return Yt.cpu().numpy().T


def _check_columns(Y, ref_cols, ne, tol):
    for q, ref in enumerate(ref_cols):
        for rows in (slice(0, ne), slice(ne, None)):
            assert rel(Y[rows, q], ref[rows]) <= tol, (q, rows, rel(Y[rows, q], ref[rows]))


def test_block_product_aim(boxes_case):  # noqa: F811
    m = boxes_case[0]
    ctx, lay = context(m, freq=10e9, grid=(16, 16, 16), precond=0)
    R = 20
    X = np.stack([random_complex(lay.n_sys, 100 + q) for q in range(R)], axis=1)
    ref = [_oracle_aim_parts(boxes_case, X[:, q])['y'] for q in range(R)]
    _check_columns(_block(ctx, lay, MIXED, X), ref, lay.n_e, 1e-5)
    _check_columns(_block(ctx, lay, FP64, X), ref, lay.n_e, 1e-6)
    # a smaller block after a larger one reuses the workspace; one column equals the
    # single-column path's operator
    Y3 = _block(ctx, lay, MIXED, X[:, :3])
    _check_columns(Y3, ref[:3], lay.n_e, 1e-5)


def test_block_product_dense_two_launches(c1_mesh, c1_system):
    ctx, lay = context(c1_mesh, freq=10e9, grid=(0, 0, 0), precond=0)
    R = 70
    X = np.stack([random_complex(lay.n_sys, 200 + q) for q in range(R)], axis=1)
    Yref = np.stack([c1_system.matvec(X[:, q])[0] for q in range(R)], axis=1)
    _check_columns(_block(ctx, lay, MIXED, X), list(Yref.T), lay.n_e, 1e-5)
    Yz = _block(ctx, lay, MIXED, np.zeros((lay.n_sys, 5), complex))
    assert np.all(Yz == 0)


def _two_bars():
    return merge([box_mesh((0.0, 0.0, 0.0), (20e-6, 2e-6, 2e-6), (10, 1, 1)),
                  box_mesh((0.0, 6e-6, 0.0), (20e-6, 2e-6, 2e-6), (10, 1, 1))])


PORTS = [(0, (10e-6, 1e-6, 1e-6), (1.0, 0.0, 0.0), 3e-6), (1, (10e-6, 7e-6, 1e-6), (1.0, 0.0, 0.0), 3e-6)]


def test_ports_rhs_currents_and_admittance():
    import torch
    from oracle.operators import Physics, dense_system
    from oracle.ports import port_currents, port_rhs
    from oracle.rwg import build_rwg
    m = _two_bars()
    g = build_rwg(m.verts, m.tris, m.obj, m.n_obj)
    ctx, lay = context(m, freq=10e9, grid=(0, 0, 0))
    B = torch.zeros((2, lay.n_sys), dtype=torch.complex128, device='cuda')
    ctx.rhs_ports(PORTS, B)
    Bref = port_rhs(g, PORTS)
    assert np.abs(B.cpu().numpy().T - Bref).max() <= 1e-15 * np.abs(Bref).max()
    X = np.stack([random_complex(lay.n_sys, 300 + q) for q in range(3)], axis=1)
    Xt = torch.tensor(X.T.copy(), device='cuda')
    I = ctx.port_currents(PORTS, Xt, 3)
    Iref = port_currents(g, PORTS, X)
    assert np.abs(I - Iref).max() <= 1e-13 * np.abs(Iref).max()
    # admittance from GMRES solves (FP64, preconditioned) against the oracle's dense LU
    S = dense_system(g, Physics(10e9))
    Yref = port_currents(g, PORTS, np.linalg.solve(S.dense(), Bref))
    Xs = torch.zeros_like(B)
    for q in range(2):
        info, ok = ctx.solve(B[q], Xs[q], tol=1e-10, restart=200, max_iter=2000, prec=FP64)
        assert ok, info.rel_residual
    Y = ctx.port_currents(PORTS, Xs, 2)
    assert np.abs(Y - Yref).max() <= 1e-6 * np.abs(Yref).max()
    assert abs(Y[0, 1] - Y[1, 0]) <= 1e-6 * abs(Y[0, 1])          # reciprocity
    assert Y[0, 0].imag > 0 and Y[1, 1].imag > 0                    # open bars: capacitive


def test_port_errors():
    import torch
    from paper_2108_03991_amd import slim
    m = _two_bars()
    ctx, lay = context(m, freq=10e9, grid=(0, 0, 0), precond=0)
    B = torch.zeros(lay.n_sys, dtype=torch.complex128, device='cuda')
    for bad in ([(0, (10.5e-6, 1e-6, 1e-6), (1.0, 0.0, 0.0), 3e-6)],     # between mesh planes: no edge
                [(0, (10e-6, 1e-6, 2e-6), (0.0, 0.0, 1.0), 30e-6)],      # the plane of a face
                [(5, (10e-6, 1e-6, 1e-6), (1.0, 0.0, 0.0), 3e-6)]):      # no such object
        with pytest.raises(slim.SlimError) as ei:
            ctx.rhs_ports(bad, B)
        assert ei.value.code == 1
