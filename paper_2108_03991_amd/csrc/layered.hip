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
#include <cstdio>

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
  int table;             // 1: rho = ix hx (Ny = 1) and only the integrated remainders are written
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
    if (a.table) {
#pragma unroll
      for (int k = 0; k < 4; ++k) a.out[k * plane + o] = make_double2(f * acc[k][q].x, f * acc[k][q].y);
      continue;
    }
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

namespace {

// Quadrature path and node table for offsets up to rho_max and zeta >= zmin: per node
// (kr, kz, Exx, Ezz, Ephi, Ezx, Wzx), the weighted remainders of the four spectral factors.
struct Limits { cd cxx, czz, cphi, czx; };

std::vector<cd> node_table(const Stack& st, double w, double k0, double rho_max, double zmin, const Limits& L) {
  double kre = k0;
  for (const slim_layer& Ly : st.layers)
    kre = std::max(kre, std::abs((w * std::sqrt(kMu0 * eps_c(w, Ly.eps_r, Ly.sigma))).real()));
  if (!st.pec) kre = std::max(kre, std::abs((w * std::sqrt(kMu0 * eps_c(w, st.eb, st.sb))).real()));
  const double a = 2.5 * kre + k0;
  const double b = std::min(0.4 * a, 1.0 / rho_max);
  SLIM_REQUIRE(std::hypot(a, b) * rho_max <= 8.0, SLIM_E_UNSUPPORTED,
               "layered kernels: the grid spans too many substrate wavelengths for the quadrature path");
  const double k_end = a + 40.0 / zmin;
  const double dk_max = std::min(0.5 * kPi / rho_max, 0.25 / zmin);
  SLIM_REQUIRE(zmin > 0.0 && (k_end - a) / dk_max <= 5.0e5, SLIM_E_UNSUPPORTED,
               "layered kernels: the interface gap is too small against the grid extent (more than 4M path nodes)");
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
  for (double lo = a, width = 0.25 * k0; lo < k_end; width *= 1.6) {
    const double hi = std::min(k_end, lo + std::min(width, dk_max));
    for (int i = 0; i < 8; ++i) {
      kr.push_back(cd(0.5 * (hi - lo) * (gx[i] + 1.0) + lo, 0.0));
      wk.push_back(cd(0.5 * (hi - lo) * gw[i], 0.0));
    }
    lo = hi;
  }
  const size_t n_nodes = kr.size();
  std::vector<cd> tab(n_nodes * 7);
  for (size_t n = 0; n < n_nodes; ++n) {
    cd ge, gh;
    reflection(st, w, kr[n], ge, gh);
    const cd k = kr[n], kz = kz_of(cd(k0 * k0, 0.0), k);
    const cd j0w = wk[n] * k / (cd(0.0, 1.0) * kz);
    const cd fzz = (ge * (kz * kz - k * k) - gh * kz * kz) / (k * k);
    const cd fph = (k0 * k0 * gh - kz * kz * ge) / (k * k);
    cd* r = &tab[n * 7];
    r[0] = k;
    r[1] = kz;
    r[2] = (gh - L.cxx) * j0w;
    r[3] = (fzz - L.czz) * j0w;
    r[4] = (fph - L.cphi) * j0w;
    r[5] = (ge - gh - L.czx) * wk[n];
    r[6] = L.czx * wk[n];
  }
  return tab;
}

double2 d2(cd v) { return make_double2(v.real(), v.imag()); }

// ---- reflected near field ----------------------------------------------------------
// Interpolation table of the integrated remainders over (rho, zeta): [4][nz][nr]
// (xx, zz, phi, zx), rows at zeta = z0 + j dz, columns at rho = i dr.  Cubic
// Lagrange in both directions; rho < 0 mirrors (even kernels, odd zx remainder).
struct Tab {
  const double2* v;
  int nr, nz;
  double dr, z0, dz;
};

__device__ __forceinline__ void lag4(double t, double* L) {
  L[0] = -t * (t - 1.0) * (t - 2.0) / 6.0;
  L[1] = (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0;
  L[2] = -(t + 1.0) * t * (t - 2.0) / 2.0;
  L[3] = (t + 1.0) * t * (t - 1.0) / 6.0;
}

struct Kern { double2 xx, zz, ph, zx; };   // zx: radial factor

__device__ Kern kern_at(const Tab& T, double rho, double zeta, double k0, const double2* lim) {
  int i = int(floor(rho / T.dr));
  i = min(i, T.nr - 3);
  const double t = rho / T.dr - i;
  int j = int(floor((zeta - T.z0) / T.dz));
  j = max(1, min(j, T.nz - 3));
  const double u = (zeta - T.z0) / T.dz - j;
  double Lr[4], Lz[4];
  lag4(t, Lr);
  lag4(u, Lz);
  double2 acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  const int64_t plane = int64_t(T.nr) * T.nz;
  for (int b = 0; b < 4; ++b) {
    const int64_t row = int64_t(j - 1 + b) * T.nr;
    for (int a = 0; a < 4; ++a) {
      int ii = i - 1 + a;
      const double sgn = ii < 0 ? -1.0 : 1.0;
      ii = ii < 0 ? -ii : ii;
      const double wgt = Lr[a] * Lz[b];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double2 v = T.v[k * plane + row + ii];
        const double s = (k == 3 ? sgn : 1.0) * wgt;
        acc[k].x += s * v.x;
        acc[k].y += s * v.y;
      }
    }
  }
  // closed-form large-k_rho parts
  const double R = sqrt(rho * rho + zeta * zeta), f = 1.0 / (4.0 * kPi);
  double sn, cs;
  sincos(k0 * R, &sn, &cs);
  const double2 img = make_double2(f * cs / R, -f * sn / R);
  const double st = f * rho / (R * (R + zeta));
  Kern K;
  K.xx = ca(cm(lim[0], img), acc[0]);
  K.zz = ca(cm(lim[1], img), acc[1]);
  K.ph = ca(cm(lim[2], img), acc[2]);
  K.zx = make_double2(lim[3].x * st + acc[3].x, lim[3].y * st + acc[3].y);
  return K;
}

struct NearRefl {
  const double* xyz; const int32_t* tri; const int32_t* tri_edge; const int8_t* tri_sign;
  const double* len; const double* area; const int32_t* tplus; const int32_t* tminus;
  const int32_t* rows; const int32_t* cols; int64_t nnz;
  const int32_t* cidx; const double* w;     // stencil centres and weights (3 x 27 RWG, 27 pulse)
  const double2* lat; int Nx, Ny, S;        // lattice kernels [4][S][Ny][Nx]
  double hx, hy, zif, k0;
  Tab tab;
  double2 lim[4];
  int rwg;
  double2* vals;                            // near values (complex128): += exact - grid, reflected
};

// TRI(2) on a triangle: P_k = V0 + u e1 + v (1-u) e2, weight w_u w_v (1-u) 2A
__device__ void tri2(const double* xyz, const int32_t* tri, int t, double P[4][3], double W[4], double area) {
  const double g0 = 0.5 - 0.5 / sqrt(3.0), g1 = 0.5 + 0.5 / sqrt(3.0);
  const double* v0 = xyz + 3 * tri[3 * t];
  const double* v1 = xyz + 3 * tri[3 * t + 1];
  const double* v2 = xyz + 3 * tri[3 * t + 2];
  for (int k = 0; k < 4; ++k) {
    const double u = (k / 2) ? g1 : g0, v = (k % 2) ? g1 : g0;
    for (int d = 0; d < 3; ++d) P[k][d] = v0[d] + u * (v1[d] - v0[d]) + v * (1.0 - u) * (v2[d] - v0[d]);
    W[k] = 0.25 * (1.0 - u) * 2.0 * area;
  }
}

__global__ void __launch_bounds__(256) k_near_refl(NearRefl g) {
  const int64_t z = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (z >= g.nnz) return;
  const int m = g.rows[z], n = g.cols[z];
  double2 ex = make_double2(0.0, 0.0);
  // ---- exact reflected part, TRI(2) x TRI(2) ----
  for (int sa = 0; sa < (g.rwg ? 2 : 1); ++sa) {
    const int t = g.rwg ? (sa ? g.tminus[m] : g.tplus[m]) : m;
    double Pt[4][3], Wt[4], ft[4][3];
    tri2(g.xyz, g.tri, t, Pt, Wt, g.area[t]);
    if (g.rwg) {
      int i = 0;
      while (g.tri_edge[3 * t + i] != m) ++i;
      const double* vt = g.xyz + 3 * g.tri[3 * t + i];
      const double cm_ = g.tri_sign[3 * t + i] * g.len[m] / (2.0 * g.area[t]);
      for (int k = 0; k < 4; ++k)
        for (int d = 0; d < 3; ++d) ft[k][d] = cm_ * (Pt[k][d] - vt[d]);
    }
    for (int sb = 0; sb < (g.rwg ? 2 : 1); ++sb) {
      const int u = g.rwg ? (sb ? g.tminus[n] : g.tplus[n]) : n;
      double Pu[4][3], Wu[4], fu[4][3];
      tri2(g.xyz, g.tri, u, Pu, Wu, g.area[u]);
      if (g.rwg) {
        int j = 0;
        while (g.tri_edge[3 * u + j] != n) ++j;
        const double* vu = g.xyz + 3 * g.tri[3 * u + j];
        const double cn_ = g.tri_sign[3 * u + j] * g.len[n] / (2.0 * g.area[u]);
        for (int k = 0; k < 4; ++k)
          for (int d = 0; d < 3; ++d) fu[k][d] = cn_ * (Pu[k][d] - vu[d]);
      }
      for (int k = 0; k < 4; ++k)
        for (int l = 0; l < 4; ++l) {
          const double dx = Pt[k][0] - Pu[l][0], dy = Pt[k][1] - Pu[l][1];
          const double rho = sqrt(dx * dx + dy * dy), zeta = Pt[k][2] + Pu[l][2] - 2.0 * g.zif;
          const Kern K = kern_at(g.tab, rho, zeta, g.k0, g.lim);
          const double ww = Wt[k] * Wu[l];
          if (g.rwg) {
            const double* A = ft[k];
            const double* B = fu[l];
            const double cx = rho > 0.0 ? dx / rho : 0.0, cy = rho > 0.0 ? dy / rho : 0.0;
            const double sxy = A[0] * B[0] + A[1] * B[1], szz = A[2] * B[2];
            const double sc = cx * (A[2] * B[0] - A[0] * B[2]) + cy * (A[2] * B[1] - A[1] * B[2]);
            ex.x += ww * (K.xx.x * sxy + K.zz.x * szz + K.zx.x * sc);
            ex.y += ww * (K.xx.y * sxy + K.zz.y * szz + K.zx.y * sc);
          } else {
            ex.x += ww * K.ph.x;
            ex.y += ww * K.ph.y;
          }
        }
    }
  }
  if (!g.rwg) {   // L_phi = 1/(A_t A_u) int int phi_r
    ex.x /= g.area[m] * g.area[n];
    ex.y /= g.area[m] * g.area[n];
  }
  // ---- grid part of the reflected kernels over the two stencils ----
  double2 gp = make_double2(0.0, 0.0);
  const int nc = g.rwg ? 3 : 1;
  const double* wm = g.w + int64_t(m) * 27 * nc;
  const double* wn = g.w + int64_t(n) * 27 * nc;
  const int64_t plane = int64_t(g.S) * g.Nx * g.Ny;
  for (int a = 0; a < 27; ++a) {
    const int ax = g.cidx[3 * m] + a % 3 - 1, ay = g.cidx[3 * m + 1] + (a / 3) % 3 - 1, az = g.cidx[3 * m + 2] + a / 9 - 1;
    for (int b = 0; b < 27; ++b) {
      const int bx = g.cidx[3 * n] + b % 3 - 1, by = g.cidx[3 * n + 1] + (b / 3) % 3 - 1,
                bz = g.cidx[3 * n + 2] + b / 9 - 1;
      const int ox = ax - bx, oy = ay - by;
      const int64_t o = (int64_t(az + bz) * g.Ny + (oy < 0 ? -oy : oy)) * g.Nx + (ox < 0 ? -ox : ox);
      if (g.rwg) {
        const double2 xx = g.lat[o], zz = g.lat[plane + o], zx = g.lat[3 * plane + o];
        const double dx = ox * g.hx, dy = oy * g.hy, r = sqrt(dx * dx + dy * dy);
        const double cx = r > 0.0 ? dx / r : 0.0, cy = r > 0.0 ? dy / r : 0.0;
        const double A0 = wm[a], A1 = wm[27 + a], A2 = wm[54 + a], B0 = wn[b], B1 = wn[27 + b], B2 = wn[54 + b];
        const double sxy = A0 * B0 + A1 * B1, szz = A2 * B2;
        const double sc = cx * (A2 * B0 - A0 * B2) + cy * (A2 * B1 - A1 * B2);
        gp.x += xx.x * sxy + zz.x * szz + zx.x * sc;
        gp.y += xx.y * sxy + zz.y * szz + zx.y * sc;
      } else {
        const double2 ph = g.lat[2 * plane + o];
        const double ab = wm[a] * wn[b];
        gp.x += ph.x * ab;
        gp.y += ph.y * ab;
      }
    }
  }
  // the pulse near values carry the column factor A_u
  const double sc = g.rwg ? 1.0 : g.area[n];
  g.vals[z].x += sc * (ex.x - gp.x);
  g.vals[z].y += sc * (ex.y - gp.y);
}

__global__ void k_expand_rows(const int64_t* ptr, int64_t nrows, int32_t* rows) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  for (int64_t k = ptr[r]; k < ptr[r + 1]; ++k) rows[k] = int32_t(r);
}

__global__ void k_c128_to_c64_n(const double2* in, float2* out, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2(float(in[i].x), float(in[i].y));
}

}  // namespace

void layered_gammas(const slim_medium& md, double freq, int64_t n, const double* kr, double* out) {
  SLIM_REQUIRE(std::isfinite(freq) && freq > 0, SLIM_E_ARG, "frequency must be positive");
  SLIM_REQUIRE(n >= 0 && (n == 0 || (kr && out)), SLIM_E_ARG, "bad arguments");
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
  const double w = 2.0 * kPi * freq;
  for (int64_t i = 0; i < n; ++i) {
    cd ge, gh;
    reflection(st, w, cd(kr[2 * i], kr[2 * i + 1]), ge, gh);
    out[4 * i] = ge.real();
    out[4 * i + 1] = ge.imag();
    out[4 * i + 2] = gh.real();
    out[4 * i + 3] = gh.imag();
  }
}

static void build_layered_device(Ctx& c, const slim_medium& md, const Stack& st, double d_min, double z0, hipStream_t s);
static bool restore_free_near(Ctx& c, hipStream_t s);

void build_layered(Ctx& c, const slim_medium& md, hipStream_t s) {
  SLIM_REQUIRE(c.built && !c.plain, SLIM_E_STATE, "no AIM operator built");
  SLIM_REQUIRE(md.n_layers >= 0 && (md.n_layers == 0 || md.layers), SLIM_E_ARG, "bad layer list");
  Stack st;
  double d_min = 1e300;
  for (int l = 0; l < md.n_layers; ++l) {
    const slim_layer& L = md.layers[l];
    SLIM_REQUIRE(std::isfinite(L.thickness) && L.thickness > 0 && std::isfinite(L.eps_r) && L.eps_r > 0 &&
                     std::isfinite(L.sigma) && L.sigma >= 0,
                 SLIM_E_ARG, "layer " + std::to_string(l) + ": thickness > 0, eps_r > 0, sigma >= 0");
    st.layers.push_back(L);
    d_min = std::min(d_min, L.thickness);
  }
  st.pec = md.bottom_pec != 0;
  if (!st.pec) {
    SLIM_REQUIRE(std::isfinite(md.bottom_eps_r) && md.bottom_eps_r > 0 && std::isfinite(md.bottom_sigma) &&
                     md.bottom_sigma >= 0,
                 SLIM_E_ARG, "bottom half-space: eps_r > 0, sigma >= 0");
    st.eb = md.bottom_eps_r;
    st.sb = md.bottom_sigma;
  }
  const double z0 = c.grid.origin[2] - md.z_interface;
  SLIM_REQUIRE(std::isfinite(md.z_interface) && z0 > 0.0, SLIM_E_ARG,
               "the AIM grid reaches the interface: its lowest node must lie above z_interface");
  c.layered = false;
  c.drop_graphs();   // captured products hold the free-space convolution
  try {
    build_layered_device(c, md, st, d_min, z0, s);
  } catch (...) {
    // a device failure leaves the context without a medium, with its free-space near
    // field; if even that cannot be restored, the context is marked unbuilt so that no
    // product runs on half-corrected values
    if (!restore_free_near(c, s)) c.built = false;
    throw;
  }
  c.layered = true;
  c.lay_zif = md.z_interface;
}

static bool restore_free_near(Ctx& c, hipStream_t s) {
  // the failed build may still have kernels and copies queued on s that write the
  // near-field values: wait for them before copying the kept values back
  bool ok = hipStreamSynchronize(s) == hipSuccess;
  for (int which = 0; which < 2; ++which) {
    DevBuf& fr = which == 0 ? c.d_nA_free : c.d_nP_free;
    DevBuf& v128 = which == 0 ? c.d_nA_v128 : c.d_nP_v128;
    DevBuf& v64 = which == 0 ? c.d_nA_v64 : c.d_nP_v64;
    const int64_t nnz = which == 0 ? c.nnz_A : c.nnz_P;
    if (!fr.p || nnz == 0) continue;
    if (hipMemcpyAsync(v128.p, fr.p, v128.bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) { ok = false; continue; }
    hipLaunchKernelGGL(k_c128_to_c64_n, dim3(nblk(nnz)), dim3(256), 0, s, v128.as<double2>(), v64.as<float2>(), nnz);
    if (hipGetLastError() != hipSuccess) ok = false;
  }
  if (hipStreamSynchronize(s) != hipSuccess) ok = false;
  return ok;
}

static void build_layered_device(Ctx& c, const slim_medium& md, const Stack& st, double d_min, double z0,
                                 hipStream_t s) {
  const GridDef& G = c.grid;
  const int Nx = G.N[0], Ny = G.N[1], Nz = G.N[2];
  const double w = c.omega, k0 = c.k0;
  // ---- large-k_rho limits: the medium right below the interface seen as a half-space ----
  cd ge_inf, gh_inf;
  if (st.layers.empty() && st.pec) {
    ge_inf = gh_inf = cd(-1.0, 0.0);
  } else {
    const cd e1 = st.layers.empty() ? eps_c(w, st.eb, st.sb) : eps_c(w, st.layers[0].eps_r, st.layers[0].sigma);
    ge_inf = (eps0() - e1) / (eps0() + e1);
    gh_inf = cd(0.0, 0.0);
  }
  Limits lim{gh_inf, -2.0 * ge_inf + gh_inf, ge_inf, ge_inf - gh_inf};
  // ---- kernels on the grid lattice ----
  const double rho_max = std::sqrt(std::pow((Nx - 1) * G.h[0], 2) + std::pow((Ny - 1) * G.h[1], 2));
  const double zmin = 2.0 * z0;
  std::vector<cd> tab = node_table(st, w, k0, rho_max, zmin, lim);
  const int n_nodes = int(tab.size() / 7);
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
  la.cxx = d2(lim.cxx); la.czz = d2(lim.czz); la.cphi = d2(lim.cphi); la.czx = d2(lim.czx);
  la.table = 0;
  la.out = c.d_lay_real.as<double2>();
  hipLaunchKernelGGL(k_refl_lattice, dim3(nblk(npts * ((Si + kZT - 1) / kZT))), dim3(256), 0, s, la);
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
  if (c.opts.verbose) {
    std::fprintf(stderr, "[slim medium] reflected grid kernels and spectra done (%d path nodes)\n", n_nodes);
    std::fflush(stderr);
  }
  // ---- near field: exact reflected part minus its grid part, on the existing CSRs ----
  if (c.nnz_A + c.nnz_P > 0) {
    // table of the integrated remainders over the grid's (rho, zeta) range
    const double zlo = 2.0 * z0, zhi = 2.0 * z0 + 2.0 * (Nz - 1) * G.h[2];
    double dlt = std::min(z0, d_min / 16.0);
    double kmax = k0;
    for (const slim_layer& Ly : st.layers) kmax = std::max(kmax, std::abs(w * std::sqrt(kMu0 * eps_c(w, Ly.eps_r, Ly.sigma))));
    dlt = std::min(dlt, 0.3 / kmax);
    SLIM_REQUIRE(rho_max / dlt <= 4000.0 && (zhi - zlo) / dlt <= 4000.0, SLIM_E_UNSUPPORTED,
                 "layered near field: the grid spans more than 4000 table steps (the step is the smaller of the "
                 "gap between the lowest grid plane and the interface and 1/16 of the thinnest layer)");
    const int nr = int(std::ceil(rho_max / dlt)) + 3, nz = int(std::ceil((zhi - zlo) / dlt)) + 4;
    const double tz0 = zlo - dlt;
    std::vector<cd> tab2 = node_table(st, w, k0, (nr - 1) * dlt, tz0, lim);
    DevBuf d_tab2, d_rt;
    d_tab2.alloc(tab2.size() * 16);
    SLIM_HIP(hipMemcpy(d_tab2.p, tab2.data(), tab2.size() * 16, hipMemcpyHostToDevice));
    d_rt.alloc(size_t(4) * nr * nz * 16);
    LatArgs ta = la;
    ta.node = d_tab2.as<double2>();
    ta.n_nodes = int(tab2.size() / 7);
    ta.Nx = nr; ta.Ny = 1; ta.S = nz;
    ta.hx = dlt; ta.hy = 0.0; ta.hz = dlt; ta.zeta0 = tz0;
    ta.table = 1;
    ta.out = d_rt.as<double2>();
    hipLaunchKernelGGL(k_refl_lattice, dim3(nblk(int64_t(nr) * ((nz + kZT - 1) / kZT))), dim3(256), 0, s, ta);
    SLIM_HIP(hipGetLastError());
    DevBuf d_cidx, d_rows;
    for (int which = 0; which < 2; ++which) {
      const bool rwg = which == 0;
      const int64_t nnz = rwg ? c.nnz_A : c.nnz_P, nrows = rwg ? c.rwg.n_e : c.rwg.n_t;
      if (nnz == 0) continue;
      DevBuf& v128 = rwg ? c.d_nA_v128 : c.d_nP_v128;
      DevBuf& v64 = rwg ? c.d_nA_v64 : c.d_nP_v64;
      DevBuf& fr = rwg ? c.d_nA_free : c.d_nP_free;
      // keep the free-space values once; a later medium starts again from them
      if (!fr.p) {
        fr.alloc(v128.bytes);
        SLIM_HIP(hipMemcpyAsync(fr.p, v128.p, v128.bytes, hipMemcpyDeviceToDevice, s));
      } else {
        SLIM_HIP(hipMemcpyAsync(v128.p, fr.p, v128.bytes, hipMemcpyDeviceToDevice, s));
      }
      const std::vector<int32_t>& ci = rwg ? c.h_cidx_e : c.h_cidx_t;
      d_cidx.alloc(ci.size() * 4);
      SLIM_HIP(hipMemcpy(d_cidx.p, ci.data(), ci.size() * 4, hipMemcpyHostToDevice));
      d_rows.alloc(size_t(nnz) * 4);
      const DevBuf& ptr = rwg ? c.d_nA_ptr : c.d_nP_ptr;
      hipLaunchKernelGGL(k_expand_rows, dim3(nblk(nrows)), dim3(256), 0, s, ptr.as<int64_t>(), nrows,
                         d_rows.as<int32_t>());
      SLIM_HIP(hipGetLastError());
      NearRefl nr_{};
      nr_.xyz = c.d_xyz.as<double>(); nr_.tri = c.d_tri.as<int32_t>(); nr_.tri_edge = c.d_tri_edge.as<int32_t>();
      nr_.tri_sign = c.d_tri_sign.as<int8_t>(); nr_.len = c.d_len.as<double>(); nr_.area = c.d_area.as<double>();
      nr_.tplus = c.d_tplus.as<int32_t>(); nr_.tminus = c.d_tminus.as<int32_t>();
      nr_.rows = d_rows.as<int32_t>(); nr_.cols = (rwg ? c.d_nA_col : c.d_nP_col).as<int32_t>(); nr_.nnz = nnz;
      nr_.cidx = d_cidx.as<int32_t>(); nr_.w = (rwg ? c.d_we_w64 : c.d_wt_w64).as<double>();
      nr_.lat = c.d_lay_real.as<double2>(); nr_.Nx = Nx; nr_.Ny = Ny; nr_.S = int(Si);
      nr_.hx = G.h[0]; nr_.hy = G.h[1]; nr_.zif = md.z_interface; nr_.k0 = k0;
      nr_.tab = Tab{d_rt.as<double2>(), nr, nz, dlt, tz0, dlt};
      nr_.lim[0] = d2(lim.cxx); nr_.lim[1] = d2(lim.czz); nr_.lim[2] = d2(lim.cphi); nr_.lim[3] = d2(lim.czx);
      nr_.rwg = rwg ? 1 : 0;
      nr_.vals = v128.as<double2>();
      // chunks of 2^22 entries, so that a verbose build reports progress
      const int64_t chunk = int64_t(1) << 22;
      for (int64_t k0c = 0; k0c < nnz; k0c += chunk) {
        NearRefl part = nr_;
        part.rows = nr_.rows + k0c;
        part.cols = nr_.cols + k0c;
        part.vals = nr_.vals + k0c;
        part.nnz = std::min(chunk, nnz - k0c);
        hipLaunchKernelGGL(k_near_refl, dim3(nblk(part.nnz)), dim3(256), 0, s, part);
        SLIM_HIP(hipGetLastError());
        if (c.opts.verbose && (k0c / chunk) % 4 == 3) {
          SLIM_HIP(hipStreamSynchronize(s));
          std::fprintf(stderr, "[slim medium] reflected near field %s: %lld / %lld\n", rwg ? "L_A" : "L_phi",
                       (long long)(k0c + part.nnz), (long long)nnz);
          std::fflush(stderr);
        }
      }
      hipLaunchKernelGGL(k_c128_to_c64_n, dim3(nblk(nnz)), dim3(256), 0, s, v128.as<double2>(), v64.as<float2>(), nnz);
      SLIM_HIP(hipGetLastError());
      SLIM_HIP(hipStreamSynchronize(s));
    }
  }
  SLIM_HIP(hipStreamSynchronize(s));
  c.lay_nodes = n_nodes;
}

}  // namespace slim
