// Reflected grid kernels of a layered background medium.
//
// The external operators L_A,m and L_phi,m of (7) use the multilayered Green's
// function when the conductors sit above a substrate (Sec. II; Table I).  Source
// and observer both lie in air above the plane z_if.  The free-space part is the
// usual AIM kernel; the reflected part depends on the in-plane distance rho and on
// zeta = z + z' - 2 z_if.  It enters the grid convolution as a convolution in x, y
// and a correlation in z.
//
// The TE/TM reflection coefficients Gamma_h, Gamma_e of the stack come from the
// generalized-reflection recursion.  Four reflected kernels (normalised by mu0 and
// 1/eps0 like g = e^{-jk0R}/(4 pi R)) are the Sommerfeld integrals
//   xx  = S0[Gamma_h],  zz = S0[(Gamma_e (kz^2 - kr^2) - Gamma_h kz^2)/kr^2],
//   phi = S0[(k0^2 Gamma_h - kz^2 Gamma_e)/kr^2],  zx = S1[Gamma_e - Gamma_h],
// where S0[F] = 1/(4 pi) int F e^{-j kz zeta} J0(kr rho) kr/(j kz) dkr and
// S1[F] = 1/(4 pi) int F e^{-j kz zeta} J1(kr rho) dkr.  The dyadic has
// G_zx = (x-x')/rho zx, G_zy = (y-y')/rho zx, G_xz = -G_zx, G_yz = -G_zy.  With a
// single scalar kernel for every charge, these are the entries that make the
// field of every current element exact.
//
// Numerics:
//   * The large-kr limit c of each spectral factor is taken out in closed form:
//     c e^{-jk0R'}/(4 pi R') for the J0 kernels (Sommerfeld's identity), and
//     c rho/(4 pi R'(R'+zeta)) for zx (the static J1 transform).  Only the
//     remainder is integrated; it decays like 1/kr^2.
//   * Path: an arc kr = t + j b sin(pi t/a) over [0, a], above the branch point
//     k0 and the guided-wave poles, then the real axis with panels that grow
//     from k0/4 up to the J_n period of the largest offset.
//   * The host builds the node table (kr, kz, weighted remainders) in FP64.
//   * The device sums it at every lattice offset (|ix|, |iy|) and every
//     lattice value of zeta, in FP64, with LDS-staged node chunks.
//   * Each kernel is then laid out on the (2N)^3 circulant (zx and zy odd in
//     their axis, the index of z + z' unwrapped) and transformed.  The spectrum
//     is kept for kx <= Nx, ky <= Ny and all 2Nz values of kz.
#include <algorithm>

#include "ctx.hpp"

namespace slim {

namespace {

unsigned nblk(int64_t n, int t = 256) { return unsigned((n + t - 1) / t); }

struct Stack {
  std::vector<slim_layer> layers;
  bool pec = true;
  double eb = 1.0, sb = 0.0;
};

cd eps_c(double w, double er, double sg) { return cd(eps0() * er, -sg / w); }
// k_z on the sheet Im k_z <= 0 for k_rho on or above the real axis
cd kz_of(cd k2, cd kr) { return cd(0.0, -1.0) * std::sqrt(kr * kr - k2); }

// TM (e) and TE (h) voltage reflection coefficients seen from air at the interface.
void reflection(const Stack& st, double w, cd kr, cd& ge, cd& gh) {
  const cd k2air = w * w * kMu0 * eps0();
  auto imp = [&](cd eps, cd k2, cd& Ze, cd& Zh, cd& kz) {
    kz = kz_of(k2, kr);
    Ze = kz / (w * eps);
    Zh = w * kMu0 / kz;
  };
  cd Ze0, Zh0, kz0;
  imp(cd(eps0(), 0.0), k2air, Ze0, Zh0, kz0);
  const int nl = int(st.layers.size());
  // reflection inside the last medium above the termination
  cd Re, Rh;
  cd Zel, Zhl, kzl;
  if (nl > 0) {
    const cd el = eps_c(w, st.layers[nl - 1].eps_r, st.layers[nl - 1].sigma);
    imp(el, w * w * kMu0 * el, Zel, Zhl, kzl);
  } else {
    Zel = Ze0; Zhl = Zh0; kzl = kz0;
  }
  if (st.pec) {
    Re = Rh = cd(-1.0, 0.0);
  } else {
    const cd eb = eps_c(w, st.eb, st.sb);
    cd Zeb, Zhb, kzb;
    imp(eb, w * w * kMu0 * eb, Zeb, Zhb, kzb);
    Re = (Zeb - Zel) / (Zeb + Zel);
    Rh = (Zhb - Zhl) / (Zhb + Zhl);
  }
  // up through the layers: propagate to the top of layer l, then cross into the medium above
  for (int l = nl - 1; l >= 0; --l) {
    const cd el = eps_c(w, st.layers[l].eps_r, st.layers[l].sigma);
    imp(el, w * w * kMu0 * el, Zel, Zhl, kzl);
    const cd ph = std::exp(cd(0.0, -2.0) * kzl * st.layers[l].thickness);
    Re *= ph;
    Rh *= ph;
    cd Zea, Zha, kza;
    if (l > 0) {
      const cd ea = eps_c(w, st.layers[l - 1].eps_r, st.layers[l - 1].sigma);
      imp(ea, w * w * kMu0 * ea, Zea, Zha, kza);
    } else {
      Zea = Ze0; Zha = Zh0;
    }
    const cd fe = (Zel - Zea) / (Zel + Zea), fh = (Zhl - Zha) / (Zhl + Zha);
    Re = (fe + Re) / (1.0 + fe * Re);
    Rh = (fh + Rh) / (1.0 + fh * Rh);
  }
  ge = Re;
  gh = Rh;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n)
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& wt) {
  x.resize(n);
  wt.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::abs(dz) < 1e-16) break;
    }
    x[i] = z;
    wt[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

constexpr int kZT = 8;        // zeta values per thread
constexpr int kChunk = 256;   // nodes per LDS chunk

struct LatArgs {
  const double2* node;   // per node: kr, kz, Exx, Ezz, Ephi, Ezx, Wzx (7 complex)
  int n_nodes;
  int Nx, Ny, S;         // lattice: |ix| < Nx, |iy| < Ny, S zeta values
  double hx, hy, hz, zeta0, k0;
  double2 cxx, czz, cphi, czx;
  double2* out;          // [4][S][Ny][Nx]
};

__device__ __forceinline__ double2 cm(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ double2 ca(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// J0, J1 of a complex argument by their power series (|z| <= 8 on the arc: the
// terms stay below 1e3 in size, so the sums keep about 13 digits)
__device__ void bessel01_series(double2 z, double2& j0, double2& j1) {
  const double2 q = make_double2(-0.25 * (z.x * z.x - z.y * z.y), -0.5 * z.x * z.y);   // -z^2/4
  double2 t0 = make_double2(1.0, 0.0), t1 = make_double2(1.0, 0.0);
  double2 s0 = t0, s1 = t1;
  for (int m = 1; m < 60; ++m) {
    t0 = cm(t0, q);
    t0.x /= double(m) * m;
    t0.y /= double(m) * m;
    t1 = cm(t1, q);
    t1.x /= double(m) * (m + 1);
    t1.y /= double(m) * (m + 1);
    s0 = ca(s0, t0);
    s1 = ca(s1, t1);
    if (fabs(t0.x) + fabs(t0.y) + fabs(t1.x) + fabs(t1.y) < 1e-18 * (fabs(s0.x) + fabs(s0.y) + 1e-300)) break;
  }
  j0 = s0;
  j1 = cm(make_double2(0.5 * z.x, 0.5 * z.y), s1);
}

__global__ void __launch_bounds__(256) k_refl_lattice(LatArgs a) {
  __shared__ double2 sh[7][kChunk];
  const int64_t npts = int64_t(a.Nx) * a.Ny;
  const int ntile = (a.S + kZT - 1) / kZT;
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool live = gid < npts * ntile;
  const int64_t p = live ? gid % npts : 0;
  const int tile = live ? int(gid / npts) : 0;
  const int ix = int(p % a.Nx), iy = int(p / a.Nx);
  const double rho = sqrt((ix * a.hx) * (ix * a.hx) + (iy * a.hy) * (iy * a.hy));
  double zeta[kZT];
#pragma unroll
  for (int q = 0; q < kZT; ++q) zeta[q] = a.zeta0 + double(tile * kZT + q) * a.hz;
  double2 acc[4][kZT];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int q = 0; q < kZT; ++q) acc[k][q] = make_double2(0.0, 0.0);
  for (int base = 0; base < a.n_nodes; base += kChunk) {
    __syncthreads();
    const int m = min(kChunk, a.n_nodes - base);
    for (int e = threadIdx.x; e < 7 * m; e += blockDim.x) sh[e % 7][e / 7] = a.node[int64_t(base) * 7 + e];
    __syncthreads();
    if (!live) continue;
    for (int j = 0; j < m; ++j) {
      const double2 kr = sh[0][j], kz = sh[1][j];
      double2 j0, j1;
      if (kr.y == 0.0) {
        j0 = make_double2(::j0(kr.x * rho), 0.0);
        j1 = make_double2(::j1(kr.x * rho), 0.0);
      } else {
        bessel01_series(make_double2(kr.x * rho, kr.y * rho), j0, j1);
      }
      const double2 exx = cm(sh[2][j], j0), ezz = cm(sh[3][j], j0), eph = cm(sh[4][j], j0);
      const double2 ezx = cm(sh[5][j], j1), wzx = cm(sh[6][j], j1);
#pragma unroll
      for (int q = 0; q < kZT; ++q) {
        // e = exp(-j kz zeta), es = exp(-kr zeta)
        double sn, cs;
        sincos(-kz.x * zeta[q], &sn, &cs);
        const double me = exp(kz.y * zeta[q]);
        const double2 e = make_double2(me * cs, me * sn);
        double sn2, cs2;
        sincos(-kr.y * zeta[q], &sn2, &cs2);
        const double ms = exp(-kr.x * zeta[q]);
        const double2 d = make_double2(e.x - ms * cs2, e.y - ms * sn2);
        acc[0][q] = ca(acc[0][q], cm(exx, e));
        acc[1][q] = ca(acc[1][q], cm(ezz, e));
        acc[2][q] = ca(acc[2][q], cm(eph, e));
        acc[3][q] = ca(ca(acc[3][q], cm(ezx, e)), cm(wzx, d));
      }
    }
  }
  if (!live) return;
  const double f = 1.0 / (4.0 * kPi);
#pragma unroll
  for (int q = 0; q < kZT; ++q) {
    const int s = tile * kZT + q;
    if (s >= a.S) break;
    const double R = sqrt(rho * rho + zeta[q] * zeta[q]);
    double sn, cs;
    sincos(a.k0 * R, &sn, &cs);
    const double2 img = make_double2(f * cs / R, -f * sn / R);
    const double st = f * rho / (R * (R + zeta[q]));
    const int64_t o = (int64_t(s) * a.Ny + iy) * a.Nx + ix, plane = int64_t(a.S) * npts;
    a.out[o] = ca(cm(a.cxx, img), make_double2(f * acc[0][q].x, f * acc[0][q].y));
    a.out[plane + o] = ca(cm(a.czz, img), make_double2(f * acc[1][q].x, f * acc[1][q].y));
    a.out[2 * plane + o] = ca(cm(a.cphi, img), make_double2(f * acc[2][q].x, f * acc[2][q].y));
    a.out[3 * plane + o] = make_double2(a.czx.x * st + f * acc[3][q].x, a.czx.y * st + f * acc[3][q].y);
  }
}

// Circulant of one reflected kernel on the (2N)^3 grid, [z][y][x]: kind 0 xx, 1 zz,
// 2 phi (even), 3 zx (odd in x), 4 zy (odd in y).  z index = lattice index of z + z'.
__global__ void k_refl_circulant(const double2* lat, int kind, int Nx, int Ny, int Nz, double hx, double hy,
                                 double2* G) {
  const int64_t X2 = 2 * Nx, Y2 = 2 * Ny, Z2 = 2 * Nz;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= X2 * Y2 * Z2) return;
  const int x = int(i % X2), y = int((i / X2) % Y2), z = int(i / (X2 * Y2));
  double2 v = make_double2(0.0, 0.0);
  if (x != Nx && y != Ny && z != Z2 - 1) {
    const int ox = x < Nx ? x : x - int(X2), oy = y < Ny ? y : y - int(Y2);
    const int ax = ox < 0 ? -ox : ox, ay = oy < 0 ? -oy : oy;
    const int64_t S = Z2 - 1, plane = S * Nx * Ny;
    const int64_t o = (int64_t(z) * Ny + ay) * Nx + ax;
    if (kind < 3) {
      v = lat[kind * plane + o];
    } else {
      const double dx = ox * hx, dy = oy * hy, rho = sqrt(dx * dx + dy * dy);
      if (rho > 0.0) {
        const double c = (kind == 3 ? dx : dy) / rho;
        const double2 r = lat[3 * plane + o];
        v = make_double2(c * r.x, c * r.y);
      }
    }
  }
  G[i] = v;
}

// spectrum of one kernel for kx <= Nx, ky <= Ny, all kz, scaled by 1/(2N)^3
__global__ void k_refl_spectrum(const double2* full, int Nx, int Ny, int Nz, double scale, double2* o128,
                                float2* o64) {
  const int64_t X1 = Nx + 1, Y1 = Ny + 1, Z2 = 2 * Nz;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= X1 * Y1 * Z2) return;
  const int64_t x = i % X1, y = (i / X1) % Y1, z = i / (X1 * Y1);
  const double2 v = full[(z * (2 * Ny) + y) * (2 * Nx) + x];
  o128[i] = make_double2(v.x * scale, v.y * scale);
  o64[i] = make_float2(float(v.x * scale), float(v.y * scale));
}

}  // namespace

void build_layered(Ctx& c, const slim_medium& md, hipStream_t s) {
  SLIM_REQUIRE(c.built && !c.plain, SLIM_E_STATE, "no AIM operator built");
  SLIM_REQUIRE(md.n_layers >= 0 && (md.n_layers == 0 || md.layers), SLIM_E_ARG, "bad layer list");
  Stack st;
  for (int l = 0; l < md.n_layers; ++l) {
    const slim_layer& L = md.layers[l];
    SLIM_REQUIRE(std::isfinite(L.thickness) && L.thickness > 0 && std::isfinite(L.eps_r) && L.eps_r > 0 &&
                     std::isfinite(L.sigma) && L.sigma >= 0,
                 SLIM_E_ARG, "layer " + std::to_string(l) + ": thickness > 0, eps_r > 0, sigma >= 0");
    st.layers.push_back(L);
  }
  st.pec = md.bottom_pec != 0;
  if (!st.pec) {
    SLIM_REQUIRE(std::isfinite(md.bottom_eps_r) && md.bottom_eps_r > 0 && std::isfinite(md.bottom_sigma) &&
                     md.bottom_sigma >= 0,
                 SLIM_E_ARG, "bottom half-space: eps_r > 0, sigma >= 0");
    st.eb = md.bottom_eps_r;
    st.sb = md.bottom_sigma;
  }
  const GridDef& G = c.grid;
  const double z0 = G.origin[2] - md.z_interface;
  SLIM_REQUIRE(std::isfinite(md.z_interface) && z0 > 0.0, SLIM_E_ARG,
               "the AIM grid reaches the interface: its lowest node must lie above z_interface");
  const int Nx = G.N[0], Ny = G.N[1], Nz = G.N[2];
  const double w = c.omega, k0 = c.k0;
  // ---- quadrature path ----
  double kre = k0;
  for (const slim_layer& L : st.layers) kre = std::max(kre, std::abs((w * std::sqrt(kMu0 * eps_c(w, L.eps_r, L.sigma))).real()));
  if (!st.pec) kre = std::max(kre, std::abs((w * std::sqrt(kMu0 * eps_c(w, st.eb, st.sb))).real()));
  const double a = 2.5 * kre + k0;
  const double rho_max = std::sqrt(std::pow((Nx - 1) * G.h[0], 2) + std::pow((Ny - 1) * G.h[1], 2));
  const double b = std::min(0.4 * a, 1.0 / rho_max);
  SLIM_REQUIRE(std::hypot(a, b) * rho_max <= 8.0, SLIM_E_UNSUPPORTED,
               "layered grid kernels: the grid spans too many substrate wavelengths for the quadrature path");
  const double zmin = 2.0 * z0;
  const double k_end = a + 40.0 / zmin;
  const double dk_max = std::min(0.5 * kPi / rho_max, 0.25 / zmin);
  std::vector<double> gx, gw;
  gauss_legendre(8, gx, gw);
  std::vector<cd> kr, wk;
  const int n_arc = 48;
  for (int pnl = 0; pnl < n_arc; ++pnl) {
    const double t0 = a * pnl / n_arc, t1 = a * (pnl + 1) / n_arc;
    for (int i = 0; i < 8; ++i) {
      const double t = 0.5 * (t1 - t0) * (gx[i] + 1.0) + t0;
      kr.push_back(cd(t, b * std::sin(kPi * t / a)));
      wk.push_back(0.5 * (t1 - t0) * gw[i] * cd(1.0, b * kPi / a * std::cos(kPi * t / a)));
    }
  }
  {
    double lo = a, width = 0.25 * k0;
    while (lo < k_end) {
      const double hi = std::min(k_end, lo + std::min(width, dk_max));
      for (int i = 0; i < 8; ++i) {
        kr.push_back(cd(0.5 * (hi - lo) * (gx[i] + 1.0) + lo, 0.0));
        wk.push_back(cd(0.5 * (hi - lo) * gw[i], 0.0));
      }
      lo = hi;
      width *= 1.6;
    }
  }
  // ---- large-k_rho limits: the medium right below the interface seen as a half-space ----
  cd ge_inf, gh_inf;
  {
    bool top_pec = st.layers.empty() && st.pec;
    if (top_pec) {
      ge_inf = gh_inf = cd(-1.0, 0.0);
    } else {
      const cd e1 = st.layers.empty() ? eps_c(w, st.eb, st.sb) : eps_c(w, st.layers[0].eps_r, st.layers[0].sigma);
      ge_inf = (eps0() - e1) / (eps0() + e1);
      gh_inf = cd(0.0, 0.0);
    }
  }
  const cd cxx = gh_inf, czz = -2.0 * ge_inf + gh_inf, cphi = ge_inf, czx = ge_inf - gh_inf;
  // ---- node table ----
  const int n_nodes = int(kr.size());
  std::vector<cd> tab(size_t(n_nodes) * 7);
  for (int n = 0; n < n_nodes; ++n) {
    cd ge, gh;
    reflection(st, w, kr[n], ge, gh);
    const cd k = kr[n], kz = kz_of(cd(k0 * k0, 0.0), k);
    const cd j0w = wk[n] * k / (cd(0.0, 1.0) * kz);
    const cd fzz = (ge * (kz * kz - k * k) - gh * kz * kz) / (k * k);
    const cd fph = (k0 * k0 * gh - kz * kz * ge) / (k * k);
    cd* r = &tab[size_t(n) * 7];
    r[0] = k;
    r[1] = kz;
    r[2] = (gh - cxx) * j0w;
    r[3] = (fzz - czz) * j0w;
    r[4] = (fph - cphi) * j0w;
    r[5] = (ge - gh - czx) * wk[n];
    r[6] = czx * wk[n];
  }
  DevBuf d_tab;
  d_tab.alloc(tab.size() * 16);
  SLIM_HIP(hipMemcpy(d_tab.p, tab.data(), tab.size() * 16, hipMemcpyHostToDevice));
  const int64_t Si = 2 * Nz - 1, npts = int64_t(Nx) * Ny;
  c.d_lay_real.alloc(size_t(4 * Si * npts) * 16);
  LatArgs la{};
  la.node = d_tab.as<double2>();
  la.n_nodes = n_nodes;
  la.Nx = Nx; la.Ny = Ny; la.S = int(Si);
  la.hx = G.h[0]; la.hy = G.h[1]; la.hz = G.h[2];
  la.zeta0 = zmin; la.k0 = k0;
  la.cxx = make_double2(cxx.real(), cxx.imag());
  la.czz = make_double2(czz.real(), czz.imag());
  la.cphi = make_double2(cphi.real(), cphi.imag());
  la.czx = make_double2(czx.real(), czx.imag());
  la.out = c.d_lay_real.as<double2>();
  const int64_t nthreads = npts * ((Si + kZT - 1) / kZT);
  hipLaunchKernelGGL(k_refl_lattice, dim3(nblk(nthreads)), dim3(256), 0, s, la);
  SLIM_HIP(hipGetLastError());
  // ---- spectra: xx, zz, phi, zx, zy ----
  const int64_t full = int64_t(8) * G.nodes();
  const int64_t spec = int64_t(Nx + 1) * (Ny + 1) * (2 * Nz);
  c.d_rhat128.alloc(size_t(5 * spec) * 16);
  c.d_rhat64.alloc(size_t(5 * spec) * 8);
  {
    DevBuf g;
    g.alloc(size_t(full) * 16);
    for (int kind = 0; kind < 5; ++kind) {
      hipLaunchKernelGGL(k_refl_circulant, dim3(nblk(full)), dim3(256), 0, s, c.d_lay_real.as<double2>(), kind, Nx,
                         Ny, Nz, G.h[0], G.h[1], g.as<double2>());
      SLIM_HIP(hipGetLastError());
      fft_forward_3d_c128(c, g.as<double>(), s);
      hipLaunchKernelGGL(k_refl_spectrum, dim3(nblk(spec)), dim3(256), 0, s, g.as<double2>(), Nx, Ny, Nz,
                         1.0 / double(full), c.d_rhat128.as<double2>() + kind * spec,
                         c.d_rhat64.as<float2>() + kind * spec);
      SLIM_HIP(hipGetLastError());
    }
    SLIM_HIP(hipStreamSynchronize(s));
  }
  c.d_lay.alloc(size_t(4 * full) * 16);
  c.layered = true;
  c.lay_zif = md.z_interface;
  c.lay_nodes = n_nodes;
}

}  // namespace slim
