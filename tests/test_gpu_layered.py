"""GPU parity of the layered-medium grid convolution against the oracle.

The library evaluates the reflected kernels differently from the oracle:
  * it subtracts their large-k_rho limits in closed form;
  * it integrates only the remainder, on its own quadrature path;
  * it sums on the device at the lattice of the AIM grid, then applies them by FFT with
    a correlation in z.
The oracle integrates the Sommerfeld integrals directly and sums over every node pair
by brute force.

Tolerances:
  * lattice kernels: both sides are FP64 quadratures accurate to about 1e-11, so 1e-9
    relative to the largest entry of each kernel;
  * FP64 convolution: 1e-9 relative 2-norm (FFT rounding on top of the kernels);
  * mixed convolution: 1e-5, the complex64 bound of the free-space path.
"""
import numpy as np
import pytest

from inputs.geometry import random_complex, small_boxes
from tests.gpu_util import context, rel

pytestmark = pytest.mark.gpu

FP64, MIXED = 0, 1
FREQ = 10e9


def _stack_c4(z_if):
    from oracle import mgf
    st = mgf.substrate_c4()
    st.z_if = z_if
    return st


def _setup(N, stack_kind="c4", gap=1e-6):
    from oracle import aim, mgf
    m = small_boxes(3, seed=4)
    ctx, lay = context(m, freq=FREQ, grid=N)
    grid = aim.make_grid(m.verts, N)
    assert np.allclose(np.array(lay.grid_origin), grid.origin, rtol=0, atol=1e-18)
    z_if = grid.origin[2] - gap
    if stack_kind == "c4":
        st = _stack_c4(z_if)
        ctx.set_medium(z_if, [(200e-6, 11.9, 10.0)], "pec")
    else:   # PEC ground under 3 um of oxide
        st = mgf.Stack([(3e-6, 4.0, 0.0)], "pec", z_if=z_if)
        ctx.set_medium(z_if, [(3e-6, 4.0, 0.0)], "pec")
    return ctx, grid, st


@pytest.mark.parametrize("N", [(8, 8, 8), (16, 8, 8)])
def test_lattice_kernels_match_oracle(N):
    from oracle import mgf
    ctx, grid, st = _setup(N)
    K = ctx.layered_kernels(grid.N)
    Nx, Ny, Nz = grid.N
    ix, iy, s = np.meshgrid(np.arange(Nx), np.arange(Ny), np.arange(2 * Nz - 1), indexing='ij')
    ix, iy, s = ix.ravel(), iy.ravel(), s.ravel()
    rng = np.random.default_rng(0)
    pick = rng.choice(ix.size, size=min(ix.size, 200), replace=False)
    pick = np.union1d(pick, [0, ix.size - 1])                     # rho = 0 and the largest offset
    rho = np.hypot(ix[pick] * grid.h[0], iy[pick] * grid.h[1])
    zeta = 2 * (grid.origin[2] - st.z_if) + s[pick] * grid.h[2]
    ref = mgf.reflected(st, FREQ, rho, zeta)
    for k, name in enumerate(("xx", "zz", "phi", "zx")):
        got = K[k, s[pick], iy[pick], ix[pick]]
        scale = np.abs(ref[name]).max()
        assert np.abs(got - ref[name]).max() <= 1e-9 * scale, name


@pytest.mark.parametrize("N,kind", [((8, 8, 8), "c4"), ((16, 8, 8), "c4"), ((8, 16, 8), "pec")])
def test_layered_convolution_parity(N, kind):
    import torch
    from oracle.aim import convolve_layered_direct
    ctx, grid, st = _setup(N, kind)
    n3 = grid.n_nodes
    src = random_complex(4 * n3, 21)
    ref = convolve_layered_direct(grid, FREQ, st, src.reshape(4, n3)).ravel()
    dst = torch.zeros(4 * n3, dtype=torch.complex128, device='cuda')
    for prec, tol in ((FP64, 1e-9), (MIXED, 1e-5)):
        ctx.aim_convolve_layered(prec, torch.tensor(src, device='cuda'), dst)
        got = dst.cpu().numpy()
        assert rel(got, ref) <= tol, (prec, rel(got, ref))
        for c in range(4):      # every component on its own
            sl = slice(c * n3, (c + 1) * n3)
            assert rel(got[sl], ref[sl]) <= 10 * tol, (prec, c)


def test_layered_convolution_single_components():
    """A source in one component only: the cross terms G_xz, G_zx, G_zy reach the right outputs."""
    import torch
    from oracle.aim import convolve_layered_direct
    ctx, grid, st = _setup((8, 8, 8))
    n3 = grid.n_nodes
    dst = torch.zeros(4 * n3, dtype=torch.complex128, device='cuda')
    for c in range(4):
        src = np.zeros((4, n3), complex)
        src[c] = random_complex(n3, 30 + c)
        ref = convolve_layered_direct(grid, FREQ, st, src).ravel()
        ctx.aim_convolve_layered(FP64, torch.tensor(src.ravel(), device='cuda'), dst)
        got = dst.cpu().numpy()
        for o in range(4):
            sl = slice(o * n3, (o + 1) * n3)
            if np.linalg.norm(ref[sl]) == 0:
                assert np.all(got[sl] == 0), (c, o)
            else:
                assert rel(got[sl], ref[sl]) <= 1e-9, (c, o)


def test_layered_errors():
    import torch
    from paper_2108_03991_amd import slim
    from oracle import aim
    m = small_boxes(3, seed=4)
    ctx, lay = context(m, freq=FREQ, grid=(8, 8, 8))
    n3 = 512
    buf = torch.zeros(4 * n3, dtype=torch.complex128, device='cuda')
    with pytest.raises(slim.SlimError) as ei:
        ctx.aim_convolve_layered(FP64, buf, buf)            # no medium yet
    assert ei.value.code == 3
    grid = aim.make_grid(m.verts, (8, 8, 8))
    with pytest.raises(slim.SlimError) as ei:               # interface above the lowest node
        ctx.set_medium(grid.origin[2] + 1e-9, [(200e-6, 11.9, 10.0)], "pec")
    assert ei.value.code == 1
    with pytest.raises(slim.SlimError) as ei:
        ctx.set_medium(grid.origin[2] - 1e-6, [(-1.0, 11.9, 10.0)], "pec")
    assert ei.value.code == 1
    with pytest.raises(slim.SlimError) as ei:               # a failed call leaves no medium behind
        ctx.aim_convolve_layered(FP64, buf, buf)
    assert ei.value.code == 3
    plain, _ = context(m, freq=FREQ, grid=(0, 0, 0))
    with pytest.raises(slim.SlimError) as ei:
        plain.set_medium(-1.0, [], "pec")
    assert ei.value.code == 3


def test_layered_convolution_tall_z_sampled():
    """Nz = 128: the layered z step runs length-256 passes and the spectrum product over
    129 kz pairs.  The oracle's brute-force layered sum is taken at 50 sampled target
    nodes (first and last included), each summed over every source node."""
    import torch
    from oracle.aim import convolve_layered_direct
    N = (8, 8, 128)
    ctx, grid, st = _setup(N)
    n3 = grid.n_nodes
    src = random_complex(4 * n3, 22)
    rng = np.random.default_rng(1)
    tg = np.union1d(rng.choice(n3, 48, replace=False), [0, n3 - 1])
    ref = convolve_layered_direct(grid, FREQ, st, src.reshape(4, n3), targets=tg)
    dst = torch.zeros(4 * n3, dtype=torch.complex128, device='cuda')
    for prec, tol in ((FP64, 1e-9), (MIXED, 1e-5)):
        ctx.aim_convolve_layered(prec, torch.tensor(src, device='cuda'), dst)
        got = dst.cpu().numpy().reshape(4, n3)[:, tg]
        for c in range(4):
            assert rel(got[c], ref[c]) <= tol, (prec, c, rel(got[c], ref[c]))
