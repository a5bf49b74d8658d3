"""Pins of the oracle's layered-medium Green's functions (oracle/mgf.py).

The kernels are pinned by things other than their own formulas:
  * Sommerfeld's identity and its rho-derivative, in closed form (integrator and path);
  * PEC ground at the interface and below an air layer, against image theory (all four
    kernels);
  * quasi-static dielectric half-space, against the classical image charge (1 - eps_r) /
    (1 + eps_r), the Laplace-transform closed form of the J_1 kernel, and the vanishing
    TE reflection;
  * a thick lossy slab on PEC, against the lossy half-space (TL recursion);
  * passivity of a lossy stack (sign of sigma);
  * the mixed-potential field E = -j w A - grad phi of x- and z-directed current
    elements, against the field computed directly from the TL voltages and currents.
    This checks the algebra of every entry of the dyadic against K_phi.
"""
import numpy as np
import pytest

from oracle import mgf

F1 = 1e9


def _g(k0, R):
    return np.exp(-1j * k0 * R) / (4 * np.pi * R)


RHO = np.array([0.0, 1e-6, 5e-6, 20e-6, 60e-6, 3e-6])
ZETA = np.array([2e-6, 3e-6, 4e-6, 10e-6, 30e-6, 25e-6])


def test_sommerfeld_identity_and_derivative():
    k0 = 2 * np.pi * F1 / mgf.C0
    R = np.hypot(RHO, ZETA)
    I0 = mgf.sommerfeld(lambda kr, kz: kr / (1j * kz), F1, RHO, ZETA, 0)
    np.testing.assert_allclose(I0, np.exp(-1j * k0 * R) / R, rtol=1e-12)
    I1 = mgf.sommerfeld(lambda kr, kz: kr * kr / (1j * kz), F1, RHO, ZETA, 1)
    ref = (1 + 1j * k0 * R) * np.exp(-1j * k0 * R) * RHO / R**3
    np.testing.assert_allclose(I1, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    # at 10 GHz and millimetre distances (phase matters)
    f = 10e9
    k0 = 2 * np.pi * f / mgf.C0
    rho, zeta = np.array([1e-3, 4e-3]), np.array([2e-3, 1e-4])
    R = np.hypot(rho, zeta)
    I0 = mgf.sommerfeld(lambda kr, kz: kr / (1j * kz), f, rho, zeta, 0)
    np.testing.assert_allclose(I0, np.exp(-1j * k0 * R) / R, rtol=1e-10)


@pytest.mark.parametrize("d", [0.0, 50e-6])
def test_pec_ground_images(d):
    """Over a PEC ground at depth d: xx = -g', zz = +g', phi = -g', zx = 0 with the image at -(z' + 2d)."""
    st = mgf.Stack([(d, 1.0, 0.0)] if d > 0 else [], "pec")
    k0 = 2 * np.pi * F1 / mgf.C0
    g = _g(k0, np.hypot(RHO, ZETA + 2 * d))
    k = mgf.reflected(st, F1, RHO, ZETA)
    tol = 1e-12 * np.abs(g).max()
    np.testing.assert_allclose(k["xx"], -g, atol=tol)
    np.testing.assert_allclose(k["zz"], g, atol=tol)
    np.testing.assert_allclose(k["phi"], -g, atol=tol)
    np.testing.assert_allclose(k["zx"], 0, atol=tol)


def test_quasi_static_dielectric_half_space():
    """eps_r = 4, lossless, 1 MHz, micrometre distances: the static image limits."""
    f = 1e6
    er = 4.0
    st = mgf.Stack([], (er, 0.0))
    k0 = 2 * np.pi * f / mgf.C0
    rho = np.array([0.0, 2e-6, 10e-6, 40e-6])
    zeta = np.array([5e-6, 8e-6, 20e-6, 10e-6])
    R = np.hypot(rho, zeta)
    gam = (1 - er) / (1 + er)
    k = mgf.reflected(st, f, rho, zeta)
    g = _g(k0, R)
    # the static limit fixes the real parts; the imaginary parts are radiation terms of
    # order k / (4 pi), far below |g| here
    k1 = k0 * np.sqrt(er)
    np.testing.assert_allclose(k["phi"].real, (gam * g).real, rtol=1e-7)
    assert np.all(np.abs(k["phi"].imag) < k1 / (4 * np.pi))
    # int_0^inf e^{-k zeta} J_1(k rho) dk = (1 - zeta / R) / rho  (-> 0 at rho = 0)
    with np.errstate(invalid="ignore"):
        zx = np.where(rho > 0, gam * (1 - zeta / R) / np.where(rho > 0, rho, 1) / (4 * np.pi), 0.0)
    np.testing.assert_allclose(k["zx"].real, zx, rtol=1e-7, atol=1e-9 * np.abs(zx).max())
    assert np.all(np.abs(k["zx"].imag) < 1e-7 * np.abs(zx).max())
    assert np.all(np.abs(k["xx"].real) < 1e-7 * np.abs(g))
    assert np.all(np.abs(k["xx"].imag) < k1 / (4 * np.pi))


def test_thick_lossy_slab_equals_half_space():
    f = 10e9
    slab = mgf.Stack([(3e-2, 11.9, 10.0)], "pec")
    half = mgf.Stack([], (11.9, 10.0))
    kr = np.linspace(1.0, 5e3, 400) + 0j
    ge1, gh1 = mgf.gammas(slab, f, kr)
    ge2, gh2 = mgf.gammas(half, f, kr)
    np.testing.assert_allclose(ge1, ge2, atol=1e-12)
    np.testing.assert_allclose(gh1, gh2, atol=1e-12)
    rho, zeta = np.array([0.0, 30e-6]), np.array([4e-6, 10e-6])
    a, b = mgf.reflected(slab, f, rho, zeta), mgf.reflected(half, f, rho, zeta)
    for key in a:
        np.testing.assert_allclose(a[key], b[key], rtol=1e-9, atol=1e-9 * np.abs(a["phi"]).max())


@pytest.mark.parametrize("stack", [mgf.substrate_c4, mgf.table1_bus, mgf.table1_interposer])
def test_lossy_stack_is_passive(stack):
    """For propagating waves (k_rho < k0) a lossy passive stack reflects at most what comes in."""
    st = stack()
    for f in (1e8, 1e9, 1e10):
        k0 = 2 * np.pi * f / mgf.C0
        kr = np.linspace(0.0, 0.999 * k0, 200) + 0j
        ge, gh = mgf.gammas(st, f, kr)
        assert np.all(np.abs(ge) < 1.0) and np.all(np.abs(gh) < 1.0)


def test_two_layer_stack_reduces_to_one_layer():
    """A 'two-layer' stack whose layers are the same material equals one layer of the summed
    thickness (TL recursion through an interface with no contrast)."""
    f = 5e9
    a = mgf.Stack([(100e-6, 11.9, 10.0), (100e-6, 11.9, 10.0)], "pec")
    b = mgf.substrate_c4()
    kr = np.concatenate([np.linspace(0.1, 3e3, 60) + 0j, np.linspace(1.0, 300.0, 20) + 30j])
    for x, y in zip(mgf.gammas(a, f, kr), mgf.gammas(b, f, kr)):
        np.testing.assert_allclose(x, y, rtol=1e-12, atol=1e-14)


def _d(fun, x, h):
    """Central derivative with one Richardson step."""
    d1 = (fun(x + h) - fun(x - h)) / (2 * h)
    d2 = (fun(x + 2 * h) - fun(x - 2 * h)) / (4 * h)
    return (4 * d1 - d2) / 3


@pytest.mark.parametrize("freq,stack", [(1e9, mgf.substrate_c4), (20e9, mgf.substrate_c4), (5e9, mgf.table1_bus)])
def test_mixed_potential_field_equals_tl_field(freq, stack):
    """E of x- and z-directed unit current elements: mixed potentials vs TL voltages/currents."""
    st = stack()
    w = 2 * np.pi * freq
    k0 = w / mgf.C0
    eps0, mu0 = mgf.EPS0, mgf.MU0
    pts = [(7e-6, 3e-6, 6e-6), (20e-6, -8e-6, 15e-6), (2e-6, 1e-6, 3e-6)]   # (x, y, zeta)

    def phi(x, y, zeta):
        return mgf.reflected(st, freq, np.hypot(x, y), zeta)["phi"][0]

    def ge_gh(kr):
        return mgf.gammas(st, freq, kr)

    for x, y, zeta in pts:
        rho = np.hypot(x, y)
        c2 = (x * x - y * y) / (rho * rho)
        k = mgf.reflected(st, freq, rho, zeta)
        h = 2e-3 * np.hypot(rho, zeta)
        dxx = _d(lambda s: _d(lambda t: phi(t, y, zeta), s, h), x, h)
        dxz = _d(lambda s: _d(lambda t: phi(t, y, s), x, h), zeta, h)
        dzz = _d(lambda s: _d(lambda t: phi(x, y, t), s, h), zeta, h)
        # mixed-potential fields (reflected parts)
        Ezx_m = -1j * w * mu0 * (x / rho) * k["zx"][0] + dxz / (1j * w * eps0)
        Ezz_m = -1j * w * mu0 * k["zz"][0] - dzz / (1j * w * eps0)
        Exx_m = -1j * w * mu0 * k["xx"][0] + dxx / (1j * w * eps0)
        # TL fields
        Ezx_t = -1j * (x / rho) / (4 * np.pi * w * eps0) * mgf.sommerfeld(
            lambda kr, kz: ge_gh(kr)[0] * kr * kr, freq, rho, zeta, 1, st)[0]
        Ezz_t = 1 / (4 * np.pi * w * eps0) * mgf.sommerfeld(
            lambda kr, kz: ge_gh(kr)[0] * kr**3 / kz, freq, rho, zeta, 0, st)[0]

        def vsum(order, sgn):
            def F(kr, kz):
                ge, gh = ge_gh(kr)
                Ve = kz / (w * eps0) * ge / 2
                Vh = w * mu0 / kz * gh / 2
                return (Ve + sgn * Vh) * kr
            return mgf.sommerfeld(F, freq, rho, zeta, order, st)[0]
        # kx^2/krho^2 -> (J0 - cos2phi J2)/2 ... ; ky^2/krho^2 -> (J0 + cos2phi J2)/2 (per 2 pi)
        Exx_t = -(1 / (4 * np.pi)) * (vsum(0, +1) - c2 * vsum(2, -1))
        for m_, t_ in ((Ezx_m, Ezx_t), (Ezz_m, Ezz_t), (Exx_m, Exx_t)):
            assert abs(m_ - t_) <= 2e-6 * abs(t_), (x, y, zeta, m_, t_)


def _tiny_grid(N=(5, 4, 3), h=(2e-6, 3e-6, 1.5e-6), z_lo=2e-6):
    from oracle.aim import Grid
    return Grid(np.array(N), np.array(h), np.array([-3e-6, 1e-6, z_lo]))


def test_layered_grid_convolution_pec_images():
    """Over a PEC ground the brute-force layered grid sum is the free-space sum plus image terms."""
    from oracle.aim import convolve_layered_direct, grid_kernel_value
    grid = _tiny_grid()
    st = mgf.Stack([(4e-6, 1.0, 0.0)], "pec", z_if=0.5e-6)
    k0 = 2 * np.pi * F1 / mgf.C0
    rng = np.random.default_rng(0)
    src = rng.standard_normal((4, grid.n_nodes)) + 1j * rng.standard_normal((4, grid.n_nodes))
    out = convolve_layered_direct(grid, F1, st, src)
    Nx, Ny, Nz = grid.N
    idx = np.stack(np.meshgrid(np.arange(Nx), np.arange(Ny), np.arange(Nz), indexing='ij'), -1)
    pos = grid.node_pos(idx.transpose(2, 1, 0, 3).reshape(-1, 3))
    d = pos[:, None, :] - pos[None, :, :]
    Gp = grid_kernel_value(grid, k0, np.rint(d / grid.h).astype(int))
    zimg = 2 * (st.z_if - 4e-6) - pos[None, :, 2]        # image of the source in the PEC plane
    Ri = np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2 + (pos[:, None, 2] - zimg) ** 2)
    gi = np.exp(-1j * k0 * Ri) / (4 * np.pi * Ri)
    ref = np.stack([(Gp - gi) @ src[0], (Gp - gi) @ src[1], (Gp + gi) @ src[2], (Gp - gi) @ src[3]])
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-10 * np.abs(ref).max())


def test_layered_grid_operator_is_reciprocal_and_matches_point_dyadic():
    """Over the lossy substrate: the vector part of the grid operator is symmetric (reciprocity,
    which fixes G_xz = -G_zx), and its entries are the point dyadic at the node pairs."""
    from oracle.aim import convolve_layered_direct, grid_kernel_value
    grid = _tiny_grid(N=(3, 3, 2))
    st = mgf.substrate_c4()
    n = grid.n_nodes
    M = np.zeros((3 * n, 3 * n), dtype=complex)
    for b in range(3):
        for j in range(n):
            src = np.zeros((4, n), dtype=complex)
            src[b, j] = 1.0
            M[:, b * n + j] = convolve_layered_direct(grid, F1, st, src)[:3].ravel()
    np.testing.assert_allclose(M, M.T, rtol=0, atol=1e-12 * np.abs(M).max())
    # entries against the point dyadic
    Nx, Ny, Nz = grid.N
    idx = np.stack(np.meshgrid(np.arange(Nx), np.arange(Ny), np.arange(Nz), indexing='ij'), -1)
    pos = grid.node_pos(idx.transpose(2, 1, 0, 3).reshape(-1, 3))
    k0 = 2 * np.pi * F1 / mgf.C0
    for i, j in [(0, 17), (4, 9), (11, 11), (15, 2)]:
        G, _ = mgf.dyadic_reflected(st, F1, pos[i:i + 1], pos[j:j + 1])
        gp = grid_kernel_value(grid, k0, np.rint((pos[i] - pos[j]) / grid.h).astype(int))
        blk = np.array([[M[a * n + i, b * n + j] for b in range(3)] for a in range(3)])
        np.testing.assert_allclose(blk, G[0] + gp * np.eye(3), rtol=1e-12, atol=1e-12 * np.abs(blk).max())
