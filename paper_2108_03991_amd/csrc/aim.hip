// Adaptive integral method build (eq. (11): L ~ L_NR + W H P, Sec. III-A).
//
// Readings (the paper defers the AIM details to its references):
//  * grid: N_c nodes per axis, h_c = max(ext_c/(N_c - 3), H/4), H = max_c ext_c/(N_c - 3),
//    centred on the vertex bounding box (ext = its extent);
//  * order M = 2: 3x3x3 stencil centred on the node nearest the basis centre
//    (RWG: mean of the two triangle centroids; pulse: centroid);
//  * weights reproduce all moments (r - r0)^alpha, 0 <= alpha_c <= 2: with the
//    tensor Lagrange basis l_a of the three stencil nodes per axis this is
//    w_a = int f(r) l_ax(x - x0) l_ay(y - y0) l_az(z - z0) dS, evaluated with the
//    collapsed Gauss rule TRI(5) (exact: the integrand has degree 7);
//  * W = P^T; grid kernel G(Delta) = e^{-j k0 |Delta o h|}/(4 pi |Delta o h|), G(0) = 0;
//    aperiodic convolution on the zero-padded (2N)^3 grid;
//  * near zone: stencil centres within Chebyshev index distance near_cheb (3);
//  * L_NR = exact near entries - sum_c P_c^T G P_c on the near zone.
#include <algorithm>
#include <cstdio>
#include <numeric>

#include "ctx.hpp"

namespace slim {

void gauss01_host(int n, std::vector<double>& x, std::vector<double>& w);

namespace {

constexpr int kNearMax = 8;   // table reach near_cheb + 2 <= kNearMax

struct Stencils {
  std::vector<int32_t> cidx;     // 3 per basis
  std::vector<double> w;         // ncomp*27 per basis
};

inline double lag(int d, double xi, double h) {
  if (d == -1) return xi * (xi - h) / (2.0 * h * h);
  if (d == 0) return (h * h - xi * xi) / (h * h);
  return xi * (xi + h) / (2.0 * h * h);
}

void lagrange_weights(const GridDef& G, const double r0[3], const double pt[3], double wq, const double f[3], int ncomp,
                      double* out) {
  double lx[3], ly[3], lz[3];
  for (int d = -1; d <= 1; ++d) {
    lx[d + 1] = lag(d, pt[0] - r0[0], G.h[0]);
    ly[d + 1] = lag(d, pt[1] - r0[1], G.h[1]);
    lz[d + 1] = lag(d, pt[2] - r0[2], G.h[2]);
  }
  for (int a = 0; a < 27; ++a) {
    double l = lx[a % 3] * ly[(a / 3) % 3] * lz[a / 9] * wq;
    for (int c = 0; c < ncomp; ++c) out[c * 27 + a] += l * f[c];
  }
}

GridDef make_grid(const Mesh& m, const int N[3]) {
  GridDef g;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < m.n_vert; ++v)
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], m.xyz[3 * v + k]);
      hi[k] = std::max(hi[k], m.xyz[3 * v + k]);
    }
  double H = 0.0;
  for (int k = 0; k < 3; ++k) {
    SLIM_REQUIRE(N[k] >= 4, SLIM_E_ARG, "AIM grid needs at least 4 nodes per axis");
    H = std::max(H, (hi[k] - lo[k]) / (N[k] - 3));
  }
  for (int k = 0; k < 3; ++k) {
    g.N[k] = N[k];
    g.h[k] = std::max((hi[k] - lo[k]) / (N[k] - 3), H / 4.0);
    double center = 0.5 * (lo[k] + hi[k]);
    g.origin[k] = center - g.h[k] * (N[k] - 1) / 2.0;
  }
  return g;
}

void centre_index(const GridDef& G, const double p[3], int32_t* idx) {
  for (int k = 0; k < 3; ++k) {
    double v = std::nearbyint((p[k] - G.origin[k]) / G.h[k]);
    SLIM_REQUIRE(v >= 1 && v <= G.N[k] - 2, SLIM_E_ARG, "stencil leaves the AIM grid");
    idx[k] = int32_t(v);
  }
}

// Stencil weights of every RWG (3 components) and pulse (1, h_t/A_t).
void stencils(const Ctx& c, Stencils& SE, Stencils& ST) {
  const RWGTable& r = c.rwg;
  const Mesh& m = c.mesh;
  const GridDef& G = c.grid;
  std::vector<double> gx, gw;
  gauss01_host(5, gx, gw);
  const int nq = 25;
  double qu[25], qv[25], qw[25];
  for (int i = 0, k = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j, ++k) {
      qu[k] = gx[i];
      qv[k] = gx[j] * (1.0 - gx[i]);
      qw[k] = gw[i] * gw[j] * (1.0 - gx[i]);
    }
  SE.cidx.resize(3 * r.n_e);
  SE.w.assign(81 * r.n_e, 0.0);
  ST.cidx.resize(3 * r.n_t);
  ST.w.assign(27 * r.n_t, 0.0);
  for (int64_t n = 0; n < r.n_e; ++n) {   // serial: centre_index may throw
    double cc[3];
    for (int k = 0; k < 3; ++k) cc[k] = 0.5 * (r.centroid[3 * r.tplus[n] + k] + r.centroid[3 * r.tminus[n] + k]);
    centre_index(G, cc, &SE.cidx[3 * n]);
  }
  for (int64_t t = 0; t < r.n_t; ++t) centre_index(G, &r.centroid[3 * t], &ST.cidx[3 * t]);
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < r.n_e; ++n) {
    double r0[3];
    for (int k = 0; k < 3; ++k) r0[k] = G.origin[k] + SE.cidx[3 * n + k] * G.h[k];
    for (int side = 0; side < 2; ++side) {
      const int64_t t = side == 0 ? r.tplus[n] : r.tminus[n];
      int i = 0;
      for (int k = 0; k < 3; ++k)
        if (r.tri_edge[3 * t + k] == n) i = k;
      const double* v0 = &m.xyz[3 * size_t(m.tri[3 * t])];
      const double* v1 = &m.xyz[3 * size_t(m.tri[3 * t + 1])];
      const double* v2 = &m.xyz[3 * size_t(m.tri[3 * t + 2])];
      const double* p = &m.xyz[3 * size_t(m.tri[3 * t + i])];
      const double coef = r.tri_sign[3 * t + i] * r.len[n] / (2.0 * r.area[t]);
      for (int q = 0; q < nq; ++q) {
        double pt[3], f[3];
        for (int k = 0; k < 3; ++k) {
          pt[k] = v0[k] + qu[q] * (v1[k] - v0[k]) + qv[q] * (v2[k] - v0[k]);
          f[k] = coef * (pt[k] - p[k]);
        }
        lagrange_weights(G, r0, pt, 2.0 * r.area[t] * qw[q], f, 3, &SE.w[81 * n]);
      }
    }
  }
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < r.n_t; ++t) {
    double r0[3];
    for (int k = 0; k < 3; ++k) r0[k] = G.origin[k] + ST.cidx[3 * t + k] * G.h[k];
    const double* v0 = &m.xyz[3 * size_t(m.tri[3 * t])];
    const double* v1 = &m.xyz[3 * size_t(m.tri[3 * t + 1])];
    const double* v2 = &m.xyz[3 * size_t(m.tri[3 * t + 2])];
    const double f[3] = {1.0 / r.area[t], 0.0, 0.0};
    for (int q = 0; q < nq; ++q) {
      double pt[3];
      for (int k = 0; k < 3; ++k) pt[k] = v0[k] + qu[q] * (v1[k] - v0[k]) + qv[q] * (v2[k] - v0[k]);
      lagrange_weights(G, r0, pt, 2.0 * r.area[t] * qw[q], f, 1, &ST.w[27 * t]);
    }
  }
}

// Near pairs: stencil centres within Chebyshev distance R (CSR, sorted columns).
void near_csr(const GridDef& G, const std::vector<int32_t>& cidx, int64_t n, int R, std::vector<int64_t>& ptr,
              std::vector<int32_t>& col) {
  std::vector<int64_t> cell(n);
  for (int64_t i = 0; i < n; ++i)
    cell[i] = (int64_t(cidx[3 * i + 2]) * G.N[1] + cidx[3 * i + 1]) * G.N[0] + cidx[3 * i];
  std::vector<int64_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return cell[a] < cell[b] || (cell[a] == cell[b] && a < b); });
  std::vector<int64_t> sorted_cell(n);
  for (int64_t i = 0; i < n; ++i) sorted_cell[i] = cell[order[i]];
  std::vector<std::vector<int32_t>> rows(n);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) {
    const int32_t* ci = &cidx[3 * i];
    std::vector<int32_t>& out = rows[i];
    for (int dz = -R; dz <= R; ++dz) {
      int z = ci[2] + dz;
      if (z < 0 || z >= G.N[2]) continue;
      for (int dy = -R; dy <= R; ++dy) {
        int y = ci[1] + dy;
        if (y < 0 || y >= G.N[1]) continue;
        int x0 = std::max(0, ci[0] - R), x1 = std::min(G.N[0] - 1, ci[0] + R);
        int64_t c0 = (int64_t(z) * G.N[1] + y) * G.N[0] + x0;
        int64_t c1 = (int64_t(z) * G.N[1] + y) * G.N[0] + x1;
        auto lo = std::lower_bound(sorted_cell.begin(), sorted_cell.end(), c0);
        auto hi = std::upper_bound(lo, sorted_cell.end(), c1);
        for (auto it = lo; it != hi; ++it) out.push_back(int32_t(order[it - sorted_cell.begin()]));
      }
    }
    std::sort(out.begin(), out.end());
  }
  ptr.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) ptr[i + 1] = ptr[i] + int64_t(rows[i].size());
  col.resize(ptr[n]);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) std::copy(rows[i].begin(), rows[i].end(), col.begin() + ptr[i]);
}

// Node-major projection CSR: for every occupied node, the (basis, weights) list.
void node_major(const GridDef& G, const std::vector<int32_t>& cidx, const std::vector<double>& w, int ncomp, int64_t n,
                const std::vector<double>* scale, std::vector<int32_t>& nodes, std::vector<int32_t>& ptr,
                std::vector<int32_t>& idx, std::vector<double>& wout) {
  std::vector<std::pair<int64_t, int64_t>> ent(size_t(n) * 27);   // (node, basis*27 + a)
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < n; ++b)
    for (int a = 0; a < 27; ++a) {
      int dx = a % 3 - 1, dy = (a / 3) % 3 - 1, dz = a / 9 - 1;
      int64_t node = (int64_t(cidx[3 * b + 2] + dz) * G.N[1] + (cidx[3 * b + 1] + dy)) * G.N[0] + (cidx[3 * b] + dx);
      ent[size_t(b) * 27 + a] = {node, b * 27 + a};
    }
  std::sort(ent.begin(), ent.end());
  nodes.clear(); ptr.clear(); idx.resize(ent.size()); wout.resize(ent.size() * ncomp);
  for (size_t e = 0; e < ent.size(); ++e) {
    if (e == 0 || ent[e].first != ent[e - 1].first) {
      nodes.push_back(int32_t(ent[e].first));
      ptr.push_back(int32_t(e));
    }
    int64_t b = ent[e].second / 27, a = ent[e].second % 27;
    idx[e] = int32_t(b);
    double s = scale ? (*scale)[b] : 1.0;
    for (int c = 0; c < ncomp; ++c) wout[e * ncomp + c] = w[b * ncomp * 27 + c * 27 + a] * s;
  }
  ptr.push_back(int32_t(ent.size()));
}

// ---- device kernels of the build ----------------------------------------------
struct PreArgs {
  const int32_t* rows; const int32_t* cols; int64_t nnz;
  const int32_t* cidx; const double* w; int ncomp;
  const double* gtab; int R;       // G over offsets [-R, R]^3, complex128
  double* vals;                    // exact in, exact - grid part out
};

__global__ void k_precorrect(PreArgs g) {
  const int64_t z = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (z >= g.nnz) return;
  const int m = g.rows[z], n = g.cols[z];
  const int D = 2 * g.R + 1;
  const int ddx = g.cidx[3 * m] - g.cidx[3 * n], ddy = g.cidx[3 * m + 1] - g.cidx[3 * n + 1],
            ddz = g.cidx[3 * m + 2] - g.cidx[3 * n + 2];
  double sr = 0.0, si = 0.0;
  const double* wm = g.w + int64_t(m) * 27 * g.ncomp;
  const double* wn = g.w + int64_t(n) * 27 * g.ncomp;
  for (int a = 0; a < 27; ++a) {
    const int ax = a % 3 - 1, ay = (a / 3) % 3 - 1, az = a / 9 - 1;
    double tr[3] = {0, 0, 0}, ti[3] = {0, 0, 0};
    for (int b = 0; b < 27; ++b) {
      const int bx = b % 3 - 1, by = (b / 3) % 3 - 1, bz = b / 9 - 1;
      const int ox = ddx + ax - bx + g.R, oy = ddy + ay - by + g.R, oz = ddz + az - bz + g.R;
      const double* G = g.gtab + 2 * ((int64_t(oz) * D + oy) * D + ox);
      const double gr = G[0], gi = G[1];
      for (int c = 0; c < g.ncomp; ++c) {
        const double wv = wn[c * 27 + b];
        tr[c] += gr * wv;
        ti[c] += gi * wv;
      }
    }
    for (int c = 0; c < g.ncomp; ++c) {
      sr += wm[c * 27 + a] * tr[c];
      si += wm[c * 27 + a] * ti[c];
    }
  }
  g.vals[2 * z] -= sr;
  g.vals[2 * z + 1] -= si;
}

__global__ void k_scale_cols(double* vals, const int32_t* cols, const double* area, int64_t nnz) {
  const int64_t z = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (z >= nnz) return;
  const double a = area[cols[z]];
  vals[2 * z] *= a;
  vals[2 * z + 1] *= a;
}

__global__ void k_to_c64(const double* in, float* out, int64_t n2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n2) out[i] = float(in[i]);
}

// octant [0, Nz] x [0, Ny] x [0, Nx] of the (2N)^3 spectrum, complex128 and complex64
// The octant k in [0, N] of the full spectrum, stored in the order [ky][kz][kx] (a
// batch of adjacent kx lines of the fused z pass reads one contiguous stretch).
__global__ void k_spectrum_octant(const double2* full, int Nx, int Ny, int Nz, double2* o128, float2* o64) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t X1 = Nx + 1, Y1 = Ny + 1, Z1 = Nz + 1;
  if (i >= X1 * Y1 * Z1) return;
  const int64_t x = i % X1, z = (i / X1) % Z1, y = i / (X1 * Z1);
  const double2 v = full[(z * (2 * Ny) + y) * (2 * Nx) + x];
  o128[i] = v;
  o64[i] = make_float2(float(v.x), float(v.y));
}

// Circulant Green's function on the (2N)^3 grid, index order [z][y][x].
__global__ void k_circulant(double* G, int Nx, int Ny, int Nz, double hx, double hy, double hz, double k0) {
  const int64_t X2 = 2 * Nx, Y2 = 2 * Ny, Z2 = 2 * Nz;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= X2 * Y2 * Z2) return;
  int64_t x = i % X2, y = (i / X2) % Y2, z = i / (X2 * Y2);
  double v_r = 0.0, v_i = 0.0;
  if (x != Nx && y != Ny && z != Nz) {
    double dx = double(x < Nx ? x : x - X2) * hx, dy = double(y < Ny ? y : y - Y2) * hy,
           dz = double(z < Nz ? z : z - Z2) * hz;
    double R = sqrt(dx * dx + dy * dy + dz * dz);
    if (R > 0.0) {
      double s, c;
      sincos(k0 * R, &s, &c);
      v_r = c / (4.0 * kPi * R);
      v_i = -s / (4.0 * kPi * R);
    }
  }
  G[2 * i] = v_r;
  G[2 * i + 1] = v_i;
}

__global__ void k_scale_real(double* p, int64_t n, double f) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] *= f;
}

unsigned nblk(int64_t n, int t = 256) { return unsigned((n + t - 1) / t); }

template <class T> void upv(DevBuf& b, const std::vector<T>& v) { b.upload(v); }

std::vector<int32_t> expand_rows(const std::vector<int64_t>& ptr) {
  std::vector<int32_t> r(ptr.back());
  for (size_t i = 0; i + 1 < ptr.size(); ++i)
    for (int64_t z = ptr[i]; z < ptr[i + 1]; ++z) r[z] = int32_t(i);
  return r;
}

}  // namespace

void build_aim(Ctx& c, hipStream_t s) {
  const RWGTable& r = c.rwg;
  const slim_build_opts& o = c.opts;
  c.grid = make_grid(c.mesh, o.grid);
  c.near_cheb = o.near_cheb > 0 ? o.near_cheb : 3;
  SLIM_REQUIRE(c.near_cheb + 2 <= kNearMax, SLIM_E_ARG, "near_cheb too large");
  const GridDef& G = c.grid;
  Stencils SE, ST;
  stencils(c, SE, ST);
  c.h_cidx_e = SE.cidx;
  c.h_cidx_t = ST.cidx;
  c.h_w_e = SE.w;
  c.h_w_t = ST.w;

  // ---- interpolation W (basis-major) ----
  {
    std::vector<int32_t> be(r.n_e), bt(r.n_t);
    for (int64_t n = 0; n < r.n_e; ++n)
      be[n] = int32_t((int64_t(SE.cidx[3 * n + 2] - 1) * G.N[1] + (SE.cidx[3 * n + 1] - 1)) * G.N[0] + (SE.cidx[3 * n] - 1));
    for (int64_t t = 0; t < r.n_t; ++t)
      bt[t] = int32_t((int64_t(ST.cidx[3 * t + 2] - 1) * G.N[1] + (ST.cidx[3 * t + 1] - 1)) * G.N[0] + (ST.cidx[3 * t] - 1));
    upv(c.d_we_base, be);
    upv(c.d_wt_base, bt);
    upv(c.d_we_w64, SE.w);
    upv(c.d_wt_w64, ST.w);
    std::vector<float> f(SE.w.begin(), SE.w.end()), g(ST.w.begin(), ST.w.end());
    upv(c.d_we_w32, f);
    upv(c.d_wt_w32, g);
  }
  // ---- projection P (node-major; pulse weights times A_t: the gather reads c0 rho) ----
  {
    std::vector<int32_t> nodes, ptr, idx;
    std::vector<double> w;
    node_major(G, SE.cidx, SE.w, 3, r.n_e, nullptr, nodes, ptr, idx, w);
    c.n_pe_nodes = int64_t(nodes.size());
    c.nnz_pe = int64_t(idx.size());
    upv(c.d_pe_node, nodes); upv(c.d_pe_ptr, ptr); upv(c.d_pe_idx, idx); upv(c.d_pe_w64, w);
    std::vector<float> wf(w.begin(), w.end());
    upv(c.d_pe_w32, wf);
    node_major(G, ST.cidx, ST.w, 1, r.n_t, &r.area, nodes, ptr, idx, w);
    c.n_pt_nodes = int64_t(nodes.size());
    c.nnz_pt = int64_t(idx.size());
    upv(c.d_pt_node, nodes); upv(c.d_pt_ptr, ptr); upv(c.d_pt_idx, idx); upv(c.d_pt_w64, w);
    std::vector<float> wf2(w.begin(), w.end());
    upv(c.d_pt_w32, wf2);
  }
  // ---- grid kernel table over the precorrection offsets ----
  const int R = c.near_cheb + 2, D = 2 * R + 1;
  std::vector<double> gtab(2 * size_t(D) * D * D);
  for (int z = -R; z <= R; ++z)
    for (int y = -R; y <= R; ++y)
      for (int x = -R; x <= R; ++x) {
        double dx = x * G.h[0], dy = y * G.h[1], dz = z * G.h[2];
        double Rr = std::sqrt(dx * dx + dy * dy + dz * dz);
        size_t k = size_t(((z + R) * D + (y + R)) * D + (x + R));
        cd v = Rr > 0 ? std::exp(cd(0.0, -c.k0 * Rr)) / (4.0 * kPi * Rr) : cd(0.0, 0.0);
        gtab[2 * k] = v.real();
        gtab[2 * k + 1] = v.imag();
      }
  DevBuf d_gtab, d_cidxE, d_cidxT;
  upv(d_gtab, gtab);
  upv(d_cidxE, SE.cidx);
  upv(d_cidxT, ST.cidx);
  // ---- near field: exact entries, precorrection ----
  // L_phi first: its pass keeps the vector-potential integrals of its triangle pairs (when
  // the memory allows), which the L_A pass then reads instead of recomputing the pairs
  // its RWG pairs share (each triangle pair serves up to nine RWG pairs)
  DevBuf ia_tab;
  for (int which : {1, 0}) {
    const bool rwg = which == 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    near_csr(G, rwg ? SE.cidx : ST.cidx, rwg ? r.n_e : r.n_t, c.near_cheb, ptr, col);
    const int64_t nnz = ptr.back();
    std::vector<int32_t> rows = expand_rows(ptr);
    DevBuf d_rows, d_v128;
    DevBuf& d_ptr = rwg ? c.d_nA_ptr : c.d_nP_ptr;
    DevBuf& d_col = rwg ? c.d_nA_col : c.d_nP_col;
    upv(d_ptr, ptr);
    upv(d_col, col);
    upv(d_rows, rows);
    DevBuf& v128 = rwg ? c.d_nA_v128 : c.d_nP_v128;
    DevBuf& v64 = rwg ? c.d_nA_v64 : c.d_nP_v64;
    v128.alloc(size_t(nnz) * 16);
    v64.alloc(size_t(nnz) * 8);
    NearArgs na{};
    na.xyz = c.d_xyz.as<double>(); na.tri = c.d_tri.as<int32_t>(); na.cen = c.d_cen.as<double>();
    na.nrm = c.d_nrm.as<double>(); na.area = c.d_area.as<double>(); na.diam = c.d_diam.as<double>();
    na.tri_edge = c.d_tri_edge.as<int32_t>(); na.tri_sign = c.d_tri_sign.as<int8_t>(); na.len = c.d_len.as<double>();
    na.tplus = c.d_tplus.as<int32_t>(); na.tminus = c.d_tminus.as<int32_t>();
    na.rows = d_rows.as<int32_t>(); na.cols = d_col.as<int32_t>(); na.nnz = nnz;
    na.kr = c.k0; na.ki = 0.0;
    na.out = v128.as<double>();
    if (!rwg) {
      size_t freeb = 0, totalb = 0;
      SLIM_HIP(hipMemGetInfo(&freeb, &totalb));
      const size_t need = size_t(nnz) * 18 * sizeof(double);
      if (nnz > 0 && need + (size_t(8) << 30) < freeb) {
        try {
          ia_tab.alloc(need);
        } catch (const Error&) {
          ia_tab.release();   // the table is an optimisation: without it L_A computes every pair
        }
      }
      na.ia = ia_tab.p ? ia_tab.as<double>() : nullptr;
    } else if (ia_tab.p) {
      na.ia = ia_tab.as<double>();
      na.tp_ptr = c.d_nP_ptr.as<int64_t>();
      na.tp_col = c.d_nP_col.as<int32_t>();
    }
    launch_near_entries(na, rwg, s);
    PreArgs pa{};
    pa.rows = d_rows.as<int32_t>(); pa.cols = d_col.as<int32_t>(); pa.nnz = nnz;
    pa.cidx = rwg ? d_cidxE.as<int32_t>() : d_cidxT.as<int32_t>();
    DevBuf& wdev = rwg ? c.d_we_w64 : c.d_wt_w64;
    pa.w = wdev.as<double>();
    pa.ncomp = rwg ? 3 : 1;
    pa.gtab = d_gtab.as<double>();
    pa.R = R;
    pa.vals = v128.as<double>();
    if (nnz > 0) hipLaunchKernelGGL(k_precorrect, dim3(nblk(nnz)), dim3(256), 0, s, pa);
    SLIM_HIP(hipGetLastError());
    if (!rwg && nnz > 0) {   // q = B c0 rho folded into the columns
      hipLaunchKernelGGL(k_scale_cols, dim3(nblk(nnz)), dim3(256), 0, s, v128.as<double>(), d_col.as<int32_t>(),
                         c.d_area.as<double>(), nnz);
      SLIM_HIP(hipGetLastError());
    }
    if (nnz > 0) hipLaunchKernelGGL(k_to_c64, dim3(nblk(2 * nnz)), dim3(256), 0, s, v128.as<double>(), v64.as<float>(), 2 * nnz);
    SLIM_HIP(hipGetLastError());
    SLIM_HIP(hipStreamSynchronize(s));
    (rwg ? c.nnz_A : c.nnz_P) = nnz;
    if (o.verbose) {
      std::fprintf(stderr, "[slim build] near field %s: %lld non-zeros\n", rwg ? "L_A" : "L_phi", (long long)nnz);
      std::fflush(stderr);
    }
  }
  // ---- Green's function spectrum ----
  fft_init_twiddles(c);
  const int64_t full = int64_t(8) * G.nodes();
  {
    DevBuf g128;
    g128.alloc(size_t(full) * 16);
    hipLaunchKernelGGL(k_circulant, dim3(nblk(full)), dim3(256), 0, s, g128.as<double>(), G.N[0], G.N[1], G.N[2],
                       G.h[0], G.h[1], G.h[2], c.k0);
    SLIM_HIP(hipGetLastError());
    fft_forward_3d_c128(c, g128.as<double>(), s);
    hipLaunchKernelGGL(k_scale_real, dim3(nblk(2 * full)), dim3(256), 0, s, g128.as<double>(), 2 * full, 1.0 / double(full));
    SLIM_HIP(hipGetLastError());
    // The kernel is even in every coordinate, so is its spectrum: keep the octant
    // k_c in [0, N_c] (the z pass reads it with mirrored indices)
    const int64_t oct = int64_t(G.N[0] + 1) * (G.N[1] + 1) * (G.N[2] + 1);
    c.d_ghat128.alloc(size_t(oct) * 16);
    c.d_ghat64.alloc(size_t(oct) * 8);
    hipLaunchKernelGGL(k_spectrum_octant, dim3(nblk(oct)), dim3(256), 0, s, g128.as<double2>(), G.N[0], G.N[1], G.N[2],
                       c.d_ghat128.as<double2>(), c.d_ghat64.as<float2>());
    SLIM_HIP(hipGetLastError());
    SLIM_HIP(hipStreamSynchronize(s));
  }
  // ---- FFT work arrays: 4 components (x, y, z, rho), sized for complex128 ----
  const int64_t N3 = G.nodes();
  c.d_oct_in.alloc(size_t(4 * N3) * 16);
  c.d_oct_in32.alloc(size_t(4 * N3) * 8);
  c.d_oct_out.alloc(size_t(4 * N3) * 16);
  c.d_x1.alloc(size_t(4 * 2 * N3) * 16);
  c.d_x2.alloc(size_t(4 * 4 * N3) * 16);
  SLIM_HIP(hipMemsetAsync(c.d_oct_in.p, 0, c.d_oct_in.bytes, s));
  SLIM_HIP(hipMemsetAsync(c.d_oct_in32.p, 0, c.d_oct_in32.bytes, s));
  SLIM_HIP(hipStreamSynchronize(s));
}

}  // namespace slim
