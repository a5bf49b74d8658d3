"""Conductor-block preconditioner through the C ABI against the oracle.

 - the partition (integer index work): bit-exact against oracle.precond;
 - P^{-1} v: against the oracle's blocks, built from the dense FP64 system, to
   the complex64 bound derived below;
 - preconditioned solves: convergence and agreement with dense LU.
"""
import numpy as np
import pytest

from inputs.geometry import bar_c1, box_mesh, merge, random_complex, small_boxes
from oracle import precond as opc
from oracle.operators import Physics, dense_system
from oracle.rwg import build_rwg
from oracle.solve import row_scaling
from tests.gpu_util import context

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24          # unit roundoff of FP32 / complex64 parts


def _boxes():
    # a long box (cut under a small cap) and two small ones
    return merge([box_mesh((0.0, 0.0, 0.0), (20e-6, 2e-6, 2e-6), (20, 2, 2)),
                  box_mesh((25e-6, 0.0, 0.0), (4e-6, 2e-6, 2e-6), (4, 2, 2)),
                  box_mesh((32e-6, 0.0, 0.0), (3e-6, 1e-6, 1e-6), (3, 1, 1))])


@pytest.fixture(scope="module")
def boxes_oracle():
    m = _boxes()
    g = build_rwg(m.verts, m.tris, m.obj, m.n_obj)
    A = dense_system(g, Physics(10e9)).dense()
    s = row_scaling(g.n_e, g.n_t, g.length.mean())
    return m, g, s[:, None] * A


CASES = [(0, 2), (120, 0), (120, 2), (60, 3)]


@pytest.mark.parametrize("cap,overlap", CASES)
def test_partition_bit_exact(boxes_oracle, cap, overlap):
    m, g, _ = boxes_oracle
    print("case: boxes partition cap", cap, "overlap", overlap, flush=True)
    ctx, lay = context(m, freq=10e9, grid=(0, 0, 0), precond_cap=cap if cap else 0, precond_overlap=overlap,
                       precond_budget=1 << 33)
    ref = opc.partition(g, cap=cap, overlap=overlap)
    got = ctx.get_precond()
    if cap == 0:
        assert lay.precond_cap == 0
    assert lay.precond_blocks == len(ref) == len(got)
    for (ext, pos), b in zip(got, ref):
        assert np.array_equal(ext, b.ext) and np.array_equal(pos, b.own_pos)


@pytest.mark.parametrize("cap,overlap", CASES)
def test_apply_matches_oracle(boxes_oracle, cap, overlap):
    """z = P^{-1} v against the oracle's FP64 blocks.

    The GPU keeps each FP64 row of the inverse as complex64 (relative error u
    per part) and accumulates s products in FP32. So
    |z - z_ref| <= (s + 3) u (|X| |v|) elementwise, plus the FP64 difference of
    the two inverses. That difference is cond(block) * 1e-15, below u for
    these blocks (cond < 1e7). The test uses the normwise form with a factor 2
    of margin.
    """
    import torch
    m, g, As = boxes_oracle
    print("case: boxes apply cap", cap, "overlap", overlap, flush=True)
    ctx, lay = context(m, freq=10e9, grid=(0, 0, 0), precond_cap=cap if cap else 0, precond_overlap=overlap,
                       precond_budget=1 << 33)
    blocks = opc.build(As, opc.partition(g, cap=cap, overlap=overlap))
    smax = max(len(b.ext) for b in blocks)
    for seed in (0, 1):
        v = random_complex(As.shape[0], seed)
        z_ref = opc.apply(blocks, v)
        bound = np.zeros(As.shape[0])
        for b in blocks:
            bound[b.ext[b.own_pos]] = np.abs(b.rows) @ np.abs(v[b.ext])
        vt = torch.tensor(v, device='cuda')
        zt = torch.full_like(vt, float('nan'))
        ctx.precond_apply(vt, zt)
        torch.cuda.synchronize()
        z = zt.cpu().numpy()
        assert np.all(np.isfinite(z)), "an unknown was not written"
        err = np.linalg.norm(z - z_ref)
        assert err <= 2 * (smax + 3) * U32 * np.linalg.norm(bound), (err, np.linalg.norm(bound))
        assert err <= 1e-4 * np.linalg.norm(z_ref)


@pytest.mark.parametrize("size", ["small", "two_panels"])
def test_single_conductor_inverts_the_system(size):
    """One conductor, dense external operator: P = S A, so P^{-1} S A x = x.
    The second case has more than 2048 unknowns, so its inverse and its (I - M)
    gather are built in several column panels."""
    import torch
    if size == "small":
        m = bar_c1(div=(12, 1, 1), length=30e-6)
    else:
        m = merge([box_mesh((0.0, 0.0, 0.0), (40e-6, 4e-6, 3e-6), (40, 4, 3))])
    ctx, lay = context(m, freq=10e9, grid=(0, 0, 0))
    if size != "small":
        assert lay.n_sys > 2048
    assert lay.precond_blocks == 1
    x = torch.tensor(random_complex(lay.n_sys, 3), device='cuda')
    y = torch.zeros_like(x)
    ctx.matvec(0, x, y)
    h = lay.mean_edge
    s = torch.cat([torch.full((lay.n_e,), 1.0 / h ** 2, dtype=torch.float64),
                   torch.full((lay.n_t,), h, dtype=torch.float64)]).to('cuda')
    z = torch.zeros_like(x)
    ctx.precond_apply(y * s, z)
    torch.cuda.synchronize()
    err = float(torch.linalg.norm(z - x) / torch.linalg.norm(x))
    assert err <= 1e-3, err


@pytest.mark.parametrize("prec", [0, 1])
def test_preconditioned_solve_multi_object_aim(prec):
    """Three copper boxes with the AIM operator (16^3 grid): preconditioned FGMRES
    reaches 1e-8 in a few iterations; without the preconditioner GMRES is far
    slower. The FP64 true residual is checked."""
    import torch
    m = small_boxes(3, seed=2)
    print("case: small_boxes AIM solve prec", prec, flush=True)
    ctx, lay = context(m, freq=10e9, grid=(16, 16, 16))
    b = torch.tensor(random_complex(lay.n_sys, 5), device='cuda')
    x = torch.zeros_like(b)
    info, ok = ctx.solve(b, x, tol=1e-8, restart=50, max_iter=300, prec=prec, inner_tol=1e-4, scaled_rhs=True)
    assert ok and info.rel_residual <= 1e-8 and info.iterations <= 40, (info.iterations, info.rel_residual)
    x0 = torch.zeros_like(b)
    info0, ok0 = ctx.solve(b, x0, tol=1e-8, restart=50, max_iter=3 * info.iterations, prec=prec, inner_tol=1e-4,
                           scaled_rhs=True, use_precond=False)
    assert not ok0 and info0.rel_residual > 1e-8


def test_precond_errors():
    from paper_2108_03991_amd import slim
    import torch
    m = small_boxes(3, seed=2)
    ctx, lay = context(m, freq=10e9, grid=(0, 0, 0), precond=0)
    assert lay.precond_blocks == 0
    v = torch.zeros(lay.n_sys, dtype=torch.complex128, device='cuda')
    z = torch.zeros_like(v)
    with pytest.raises(slim.SlimError) as e:
        ctx.precond_apply(v, z)
    assert e.value.code == 3
    with pytest.raises(slim.SlimError) as e:
        ctx.solve(v + 1, z, use_precond=True)
    assert e.value.code == 3
    with pytest.raises(slim.SlimError) as e:
        context(m, freq=10e9, grid=(0, 0, 0), precond_cap=64, precond_budget=1000)
    assert e.value.code == 4


from tests.test_gpu_parity import boxes_case, _oracle_aim_parts  # noqa: E402,F401  (fixture and oracle product)


@pytest.fixture(scope="module")
def aim_system(boxes_case):
    """Dense equilibrated matrix of the oracle's AIM system (columns of its product)."""
    m, g, ph, op, Ix, D, inner = boxes_case
    n = g.n_e + g.n_t
    A = np.zeros((n, n), dtype=complex)
    for j in range(n):
        e = np.zeros(n, dtype=complex)
        e[j] = 1.0
        A[:, j] = _oracle_aim_parts(boxes_case, e)['y']
    s = row_scaling(g.n_e, g.n_t, g.length.mean())
    return s[:, None] * A


@pytest.mark.parametrize("cap,overlap", [(0, 2), (90, 2)])
def test_apply_matches_oracle_aim(boxes_case, aim_system, cap, overlap):
    """With the AIM operator the blocks are the conductor's part of that operator:
    exact interactions on near pairs, grid interactions on far pairs."""
    import torch
    m, g = boxes_case[0], boxes_case[1]
    print("case: small_boxes AIM apply cap", cap, flush=True)
    ctx, lay = context(m, freq=10e9, grid=(16, 16, 16), precond_cap=cap, precond_overlap=overlap,
                       precond_budget=1 << 33)
    blocks = opc.build(aim_system, opc.partition(g, cap=cap, overlap=overlap))
    if cap:
        assert len(blocks) > g.n_obj
    smax = max(len(b.ext) for b in blocks)
    v = random_complex(aim_system.shape[0], 2)
    z_ref = opc.apply(blocks, v)
    bound = np.zeros(aim_system.shape[0])
    for b in blocks:
        bound[b.ext[b.own_pos]] = np.abs(b.rows) @ np.abs(v[b.ext])
    vt = torch.tensor(v, device='cuda')
    zt = torch.full_like(vt, float('nan'))
    ctx.precond_apply(vt, zt)
    torch.cuda.synchronize()
    z = zt.cpu().numpy()
    err = np.linalg.norm(z - z_ref)
    assert err <= 2 * (smax + 3) * U32 * np.linalg.norm(bound), (err, np.linalg.norm(bound))
    assert err <= 1e-4 * np.linalg.norm(z_ref)
