"""Reflected parts of the multilayered-medium Green's functions (kernels of L_A,m and L_phi,m in (7)).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper builds the external operators of a layered background with the
multilayered Green's function of [Michalski1990] (Sec. II, after eq. (7);
the layered stacks of Table I).  That reference is not part of the paper, so
the kernels here are derived from transmission-line (TL) theory of a
stratified medium.  Readings:

  * Geometry.  The conductors and every AIM grid node lie in the top
    half-space z > z_if, which is air (eps0, mu0).  Below z_if, layers are
    listed top-down as (thickness, eps_r, sigma); the stack ends in a PEC
    ground or in a lossy half-space.  Time dependence e^{j w t}; a layer's
    permittivity is eps0 eps_r - j sigma / w.
  * Spectral TL model.  Per transverse wavenumber k_rho, TM (e) and TE (h)
    waves see lines of impedance Z_e = k_z / (w eps) and Z_h = w mu / k_z.
    The stack below z_if is a load; Gamma_e and Gamma_h are its voltage
    reflection coefficients seen from the air line.  A PEC ground is a short.
  * Mixed potentials.  A single scalar kernel K_phi serves every charge,
    because the charge is its own unknown (rho_Delta in (7)).  K_phi is the
    kernel of a horizontal source.  The dyadic of the vector potential is then
    fixed by requiring that the field E = -j w A - grad phi of each current
    element equals the TL field.  It has these non-zero entries:
      - xx = yy (TE),
      - zz,
      - zx, zy (A_z from horizontal currents),
      - xz, yz, with G_xz(r, r') = G_zx(r', r) (reciprocity).
    The field of a vertical element needs the xz and yz entries, once K_phi is
    the horizontal kernel.
  * Normalisation.  The free-space parts equal g = e^{-j k0 R} / (4 pi R) of
    the homogeneous-medium operators.  The functions below are the reflected
    parts in the same units: A = mu0 int (g I + G_r) . J, and
    phi = (1/eps0) int (g + phi_r) q.  They depend on rho = |r_t - r_t'| and
    zeta = (z - z_if) + (z' - z_if).

Reflected parts, with k_z = sqrt(k0^2 - k_rho^2) on Im k_z <= 0 and
e = e^{-j k_z zeta}, where S_n[F] = (1/4 pi) int_0^inf F e J_n(k_rho rho) dk_rho:
  xx_r  = S_0[ Gamma_h k_rho / (j k_z) ]
  zz_r  = S_0[ (Gamma_e (k_z^2 - k_rho^2) - Gamma_h k_z^2) / k_rho^2 * k_rho / (j k_z) ]
  phi_r = S_0[ (k0^2 Gamma_h - k_z^2 Gamma_e) / k_rho^2 * k_rho / (j k_z) ]
  zx_r  = S_1[ Gamma_e - Gamma_h ]
The dyadic entries built from zx_r are:
  G_zx = (x - x') / rho * zx_r,    G_zy = (y - y') / rho * zx_r,
  G_xz = -G_zx,                    G_yz = -G_zy.
Over a PEC ground these reduce to the images -g', +g', -g' and 0.

The Sommerfeld integrals are evaluated by direct quadrature, with no
asymptotic extraction and no tabulation: plain and slow.
  * From 0 to a, the path is the arc k_rho = t + j b sin(pi t / a) in the
    first quadrant.  It passes above the branch point k0 and above the
    surface-wave poles, which lie at or below the real axis.
  * From a to infinity, the path runs along the real axis, cut where
    e^{-k_rho zeta} < e^{-40}.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.special import j0, j1, jv

C0 = 299792458.0
MU0 = 4.0e-7 * np.pi
EPS0 = 1.0 / (MU0 * C0 * C0)


@dataclass
class Stack:
    """Layers below the plane z = z_if (top-down) and the termination below them."""
    layers: list = field(default_factory=list)   # [(thickness, eps_r, sigma), ...]
    bottom: object = "pec"                        # "pec" or (eps_r, sigma) of a half-space
    z_if: float = 0.0


def substrate_c4():
    """Silicon 200 um (eps_r 11.9, sigma 10 S/m) on a PEC ground: the substrate of the bus workload."""
    return Stack(layers=[(200e-6, 11.9, 10.0)], bottom="pec", z_if=0.0)


def table1_bus():
    """The high-speed-bus stack of Table I: oxide 30 um (eps_r 4), silicon 495 um (eps_r 11.9,
    10 S/m), PEC."""
    return Stack(layers=[(30e-6, 4.0, 0.0), (495e-6, 11.9, 10.0)], bottom="pec", z_if=0.0)


def table1_interposer():
    """The fan-out-interposer stack of Table I: oxide 27.5 um, silicon 497.5 um (same materials), PEC."""
    return Stack(layers=[(27.5e-6, 4.0, 0.0), (497.5e-6, 11.9, 10.0)], bottom="pec", z_if=0.0)


def _kz(k2, krho):
    """k_z = sqrt(k^2 - k_rho^2) on the branch Im k_z <= 0 (k_rho on or above the real axis)."""
    return -1j * np.sqrt(krho * krho - k2 + 0j)


def _eps(freq, eps_r, sigma):
    return EPS0 * eps_r - 1j * sigma / (2.0 * np.pi * freq)


def gammas(stack: Stack, freq: float, krho):
    """Voltage reflection coefficients (Gamma_e, Gamma_h) of the stack, seen from the air line at z_if."""
    w = 2.0 * np.pi * freq
    krho = np.asarray(krho, dtype=complex)
    # load impedance below the last layer
    if isinstance(stack.bottom, str):
        if stack.bottom != "pec":
            raise ValueError("bottom must be 'pec' or (eps_r, sigma)")
        ZLe = np.zeros_like(krho)
        ZLh = np.zeros_like(krho)
    else:
        eb = _eps(freq, *stack.bottom)
        kzb = _kz(w * w * MU0 * eb, krho)
        ZLe, ZLh = kzb / (w * eb), w * MU0 / kzb
    # transform up through each layer, bottom first: Z_in = Z (Z_L + Z jt) / (Z + Z_L jt),
    # jt = j tan(k_z d) = (1 - E) / (1 + E), E = e^{-2 j k_z d}, |E| <= 1
    for d, er, sg in reversed(stack.layers):
        el = _eps(freq, er, sg)
        kzl = _kz(w * w * MU0 * el, krho)
        E = np.exp(-2j * kzl * d)
        jt = (1.0 - E) / (1.0 + E)
        Ze, Zh = kzl / (w * el), w * MU0 / kzl
        ZLe = Ze * (ZLe + Ze * jt) / (Ze + ZLe * jt)
        ZLh = Zh * (ZLh + Zh * jt) / (Zh + ZLh * jt)
    kz0 = _kz(w * w * MU0 * EPS0, krho)
    Z0e, Z0h = kz0 / (w * EPS0), w * MU0 / kz0
    return (ZLe - Z0e) / (ZLe + Z0e), (ZLh - Z0h) / (ZLh + Z0h)


def _path(stack: Stack, freq: float, rho_max: float, zeta_min: float, gl=16):
    """Quadrature nodes and weights (complex, including dk_rho/dt) of the deformed path."""
    w = 2.0 * np.pi * freq
    k0 = w / C0
    kre = [k0]
    for d, er, sg in stack.layers:
        kre.append(abs((w * np.sqrt(MU0 * _eps(freq, er, sg) + 0j)).real))
    if not isinstance(stack.bottom, str):
        kre.append(abs((w * np.sqrt(MU0 * _eps(freq, *stack.bottom) + 0j)).real))
    a = 2.0 * max(kre) + k0
    b = min(0.5 * a, 1.0 / max(rho_max, 1e-30))
    x, wx = np.polynomial.legendre.leggauss(gl)
    # arc: 24 panels
    n_arc = 24
    edges = np.linspace(0.0, a, n_arc + 1)
    t = (0.5 * (edges[1:] - edges[:-1])[:, None] * (x[None] + 1.0) + edges[:-1, None]).ravel()
    wt = (0.5 * (edges[1:] - edges[:-1])[:, None] * wx[None]).ravel()
    kr_arc = t + 1j * b * np.sin(np.pi * t / a)
    w_arc = wt * (1.0 + 1j * b * (np.pi / a) * np.cos(np.pi * t / a))
    # real tail: panels no wider than a quarter period of J_n(k rho_max) or 1/(4 zeta_min);
    # near a they start at width k0 / 2 and double, to follow the k_z ~ k_rho transition
    k_end = a + 40.0 / zeta_min
    dk = min(0.5 * np.pi / max(rho_max, 1e-30), 0.25 / zeta_min)
    edges = [a]
    wdt = 0.5 * k0
    while wdt < dk and edges[-1] < k_end:
        edges.append(edges[-1] + wdt)
        wdt *= 2.0
    n_tail = max(1, int(np.ceil((k_end - edges[-1]) / dk)))
    edges = np.concatenate([edges[:-1], np.linspace(edges[-1], max(k_end, edges[-1] + dk), n_tail + 1)])
    t = (0.5 * (edges[1:] - edges[:-1])[:, None] * (x[None] + 1.0) + edges[:-1, None]).ravel()
    wt = (0.5 * (edges[1:] - edges[:-1])[:, None] * wx[None]).ravel()
    return np.concatenate([kr_arc, t + 0j]), np.concatenate([w_arc, wt + 0j])


def _bessel_c(n, z):
    """J_n of complex arguments: the power series sum_m (-z^2/4)^m (z/2)^n / (m! (m+n)!) where
    |z| <= 8 (terms stay below 1e3 in size), scipy's jv elsewhere."""
    out = np.empty(z.shape, dtype=complex)
    small = np.abs(z) <= 8.0
    zs = z[small]
    q = -0.25 * zs * zs
    term = (0.5 * zs) ** n / float(np.prod(np.arange(1, n + 1)))
    acc = term.copy()
    for m in range(1, 60):
        term = term * q / (m * (m + n))
        acc += term
        if np.all(np.abs(term) <= 1e-17 * np.maximum(np.abs(acc), 1e-300)):
            break
    out[small] = acc
    if np.any(~small):
        out[~small] = jv(n, z[~small])
    return out


def sommerfeld_many(terms, freq, rho, zeta, stack=None):
    """int_0^inf F(k_rho, k_z) e^{-j k_z zeta} J_n(k_rho rho) dk_rho for every (rho, zeta) pair,
    for each (F, n) in `terms` (one path; the Bessel functions and exponentials are shared).

    F is a callable of (k_rho, k_z) arrays; k_z is the air value.  The path is
    that of the module docstring; `stack` only sets where the arc ends.
    """
    rho = np.atleast_1d(np.asarray(rho, dtype=float))
    zeta = np.atleast_1d(np.asarray(zeta, dtype=float))
    rho, zeta = np.broadcast_arrays(rho, zeta)
    if np.any(zeta <= 0):
        raise ValueError("zeta = z + z' - 2 z_if must be positive (both points above the interface)")
    w = 2.0 * np.pi * freq
    k0 = w / C0
    kr, wk = _path(stack or Stack(), freq, float(rho.max()), float(zeta.min()))
    kz = _kz(k0 * k0, kr)
    Fw = [F(kr, kz) * wk for F, _ in terms]
    orders = sorted({n for _, n in terms})
    outs = [np.zeros(rho.size, dtype=complex) for _ in terms]
    flat_r, flat_z = rho.ravel(), zeta.ravel()
    step = max(1, 2_000_000 // kr.size)
    arc = kr.imag != 0.0
    kr_t = kr[~arc].real
    for lo in range(0, flat_r.size, step):
        s = slice(lo, lo + step)
        E = np.exp(-1j * kz[None, :] * flat_z[s, None])
        for n in orders:
            # complex Bessel functions on the arc, real ones on the real axis
            J = np.empty(E.shape, dtype=complex)
            J[:, arc] = _bessel_c(n, kr[None, arc] * flat_r[s, None])
            x = kr_t[None, :] * flat_r[s, None]
            J[:, ~arc] = j0(x) if n == 0 else (j1(x) if n == 1 else jv(n, x))
            JE = J * E
            for k, (_, nk) in enumerate(terms):
                if nk == n:
                    outs[k][s] = JE @ Fw[k]
    return [o.reshape(rho.shape) for o in outs]


def sommerfeld(F, freq, rho, zeta, order, stack=None):
    """One Sommerfeld integral (see sommerfeld_many)."""
    return sommerfeld_many([(F, order)], freq, rho, zeta, stack)[0]


def reflected(stack: Stack, freq: float, rho, zeta):
    """The four reflected kernels xx_r, zz_r, phi_r, zx_r (see the module docstring)."""
    k0 = 2.0 * np.pi * freq / C0

    def f_xx(kr, kz):
        return gammas(stack, freq, kr)[1] * kr / (1j * kz)

    def f_zz(kr, kz):
        ge, gh = gammas(stack, freq, kr)
        return (ge * (kz * kz - kr * kr) - gh * kz * kz) / (kr * kr) * kr / (1j * kz)

    def f_phi(kr, kz):
        ge, gh = gammas(stack, freq, kr)
        return (k0 * k0 * gh - kz * kz * ge) / (kr * kr) * kr / (1j * kz)

    def f_zx(kr, kz):
        ge, gh = gammas(stack, freq, kr)
        return ge - gh

    c = 1.0 / (4.0 * np.pi)
    xx, zz, ph, zx = sommerfeld_many([(f_xx, 0), (f_zz, 0), (f_phi, 0), (f_zx, 1)], freq, rho, zeta, stack)
    return {"xx": c * xx, "zz": c * zz, "phi": c * ph, "zx": c * zx}


def dyadic_reflected(stack: Stack, freq: float, robs, rsrc):
    """Reflected dyadic (3x3, mu0-normalised) and scalar kernel for point pairs.

    robs, rsrc: (n, 3).  Returns (G (n,3,3), phi (n,)) with G[:, a, b] the
    a-component of A from a b-directed source.
    """
    robs = np.atleast_2d(robs)
    rsrc = np.atleast_2d(rsrc)
    dx = robs[:, 0] - rsrc[:, 0]
    dy = robs[:, 1] - rsrc[:, 1]
    rho = np.hypot(dx, dy)
    zeta = robs[:, 2] + rsrc[:, 2] - 2.0 * stack.z_if
    k = reflected(stack, freq, rho, zeta)
    with np.errstate(invalid="ignore", divide="ignore"):
        cx = np.where(rho > 0, dx / rho, 0.0)
        cy = np.where(rho > 0, dy / rho, 0.0)
    G = np.zeros((rho.size, 3, 3), dtype=complex)
    G[:, 0, 0] = G[:, 1, 1] = k["xx"]
    G[:, 2, 2] = k["zz"]
    G[:, 2, 0] = cx * k["zx"]
    G[:, 2, 1] = cy * k["zx"]
    G[:, 0, 2] = -cx * k["zx"]
    G[:, 1, 2] = -cy * k["zx"]
    return G, k["phi"]
