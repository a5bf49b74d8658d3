// Operator build: physics constants, I_x, interior blocks Z_i (eq. (4)),
// Y_eq,i (eq. (5)) and M_i = Y_eq,i Z_i (eq. (6)) by FP64 LU on the GPU, the
// external operator (dense or AIM), the task queues and the work buffers.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <exception>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>
#include <unordered_map>

#include "ctx.hpp"

namespace slim {

namespace {

struct RocHandle {
  rocblas_handle h = nullptr;
  explicit RocHandle(hipStream_t s) {
    if (rocblas_create_handle(&h) != rocblas_status_success) throw Error(SLIM_E_HIP, "rocblas_create_handle failed");
    rocblas_set_stream(h, s);
  }
  ~RocHandle() { if (h) rocblas_destroy_handle(h); }
};

#define SLIM_ROC(call)                                                                        \
  do {                                                                                        \
    rocblas_status st_ = (call);                                                              \
    if (st_ != rocblas_status_success)                                                        \
      throw ::slim::Error(SLIM_E_HIP, std::string(#call) + " failed: " + std::to_string(int(st_))); \
  } while (0)

}  // namespace

static int ilog2(int v) {
  int k = 0;
  while ((1 << (k + 1)) <= v) ++k;
  return k;
}

// Candidate near triangle pairs (t <= u) in [t0, t1): centroid distance below
// 1.01 c_near max(diam); the device takes the exact decision.
std::vector<int32_t> near_candidates(const RWGTable& r, int64_t t0, int64_t t1, double c_near) {
  std::vector<int32_t> out;
  if (t1 <= t0) return out;
  double dmax = 0.0, lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t t = t0; t < t1; ++t) {
    dmax = std::max(dmax, r.diam[t]);
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], r.centroid[3 * t + k]);
      hi[k] = std::max(hi[k], r.centroid[3 * t + k]);
    }
  }
  const double cell = 1.01 * c_near * dmax;
  int64_t nc[3];
  for (int k = 0; k < 3; ++k) nc[k] = std::max<int64_t>(1, int64_t((hi[k] - lo[k]) / cell) + 1);
  auto cell_of = [&](int64_t t, int64_t* c3) {
    for (int k = 0; k < 3; ++k)
      c3[k] = std::min<int64_t>(nc[k] - 1, std::max<int64_t>(0, int64_t((r.centroid[3 * t + k] - lo[k]) / cell)));
  };
  std::unordered_map<int64_t, std::vector<int32_t>> bins;
  for (int64_t t = t0; t < t1; ++t) {
    int64_t c3[3];
    cell_of(t, c3);
    bins[(c3[2] * nc[1] + c3[1]) * nc[0] + c3[0]].push_back(int32_t(t));
  }
  for (int64_t t = t0; t < t1; ++t) {
    int64_t c3[3];
    cell_of(t, c3);
    for (int64_t dz = -1; dz <= 1; ++dz)
      for (int64_t dy = -1; dy <= 1; ++dy)
        for (int64_t dx = -1; dx <= 1; ++dx) {
          int64_t x = c3[0] + dx, y = c3[1] + dy, z = c3[2] + dz;
          if (x < 0 || y < 0 || z < 0 || x >= nc[0] || y >= nc[1] || z >= nc[2]) continue;
          auto it = bins.find((z * nc[1] + y) * nc[0] + x);
          if (it == bins.end()) continue;
          for (int32_t u : it->second) {
            if (u < t) continue;
            double d2 = 0.0;
            for (int k = 0; k < 3; ++k) {
              double d = r.centroid[3 * t + k] - r.centroid[3 * u + k];
              d2 += d * d;
            }
            double dm = 1.01 * c_near * std::max(r.diam[t], r.diam[u]);
            if (d2 < dm * dm) {
              out.push_back(int32_t(t));
              out.push_back(u);
            }
          }
        }
  }
  return out;
}

// Pattern of the sparse Z~ of one object (edges [e0, e0 + n), triangles [t0, t1)):
// local (row, column) pairs of RWGs that share a triangle pair whose centroids are at
// most rad apart (squared distance dx*dx + dy*dy + dz*dz <= rad*rad, each product and
// sum rounded on its own, as the device decides it), sorted by row then column.
static void z_pattern(const RWGTable& r, int64_t t0, int64_t t1, int32_t e0, int32_t n, double rad,
                      std::vector<int32_t>& rows, std::vector<int32_t>& cols) {
#pragma clang fp contract(off)
  std::vector<std::vector<int32_t>> adj(static_cast<size_t>(n));
  double lo[3] = {1e300, 1e300, 1e300};
  for (int64_t t = t0; t < t1; ++t)
    for (int k = 0; k < 3; ++k) lo[k] = std::min(lo[k], r.centroid[3 * t + k]);
  const double cell = rad;
  auto key = [&](int64_t a, int64_t b, int64_t c) { return (a * 1000003 + b) * 1000003 + c; };
  std::unordered_map<int64_t, std::vector<int32_t>> bins;
  auto cell_of = [&](int64_t t, int64_t* c3) {
    for (int k = 0; k < 3; ++k) c3[k] = int64_t(std::floor((r.centroid[3 * t + k] - lo[k]) / cell));
  };
  for (int64_t t = t0; t < t1; ++t) {
    int64_t c3[3];
    cell_of(t, c3);
    bins[key(c3[0], c3[1], c3[2])].push_back(int32_t(t));
  }
  const double r2 = rad * rad;
  for (int64_t t = t0; t < t1; ++t) {
    int64_t c3[3];
    cell_of(t, c3);
    for (int64_t dz = -1; dz <= 1; ++dz)
      for (int64_t dy = -1; dy <= 1; ++dy)
        for (int64_t dx = -1; dx <= 1; ++dx) {
          auto it = bins.find(key(c3[0] + dx, c3[1] + dy, c3[2] + dz));
          if (it == bins.end()) continue;
          for (int32_t u : it->second) {
            if (u < t) continue;
            const double ddx = r.centroid[3 * t] - r.centroid[3 * size_t(u)];
            const double ddy = r.centroid[3 * t + 1] - r.centroid[3 * size_t(u) + 1];
            const double ddz = r.centroid[3 * t + 2] - r.centroid[3 * size_t(u) + 2];
            const double sx = ddx * ddx, sy = ddy * ddy, sz = ddz * ddz;
            const double d2 = (sx + sy) + sz;
            if (d2 > r2) continue;
            for (int i = 0; i < 3; ++i)
              for (int j = 0; j < 3; ++j) {
                const int32_t m = r.tri_edge[3 * t + i] - e0, q = r.tri_edge[3 * size_t(u) + j] - e0;
                adj[size_t(m)].push_back(q);
                adj[size_t(q)].push_back(m);
              }
          }
        }
  }
  rows.clear();
  cols.clear();
  for (int32_t m = 0; m < n; ++m) {
    std::vector<int32_t>& a = adj[size_t(m)];
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
    for (int32_t q : a) {
      rows.push_back(m);
      cols.push_back(q);
    }
  }
}

// I_x rows: entries with the (up to four) other edges of T+ and T- of each RWG.
// The integrand (n x f_m).f_n is quadratic on a triangle; the three-edge-midpoint
// rule with weights A/3 is exact.
void build_ix(const Mesh& m, const RWGTable& r, std::vector<int32_t>& col, std::vector<double>& val) {
  col.assign(4 * r.n_e, -1);
  val.assign(4 * r.n_e, 0.0);
  std::vector<int> fill(r.n_e, 0);
  const double* X = m.xyz.data();
  for (int64_t t = 0; t < r.n_t; ++t) {
    double v[3][3], mid[3][3];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) v[i][k] = X[3 * size_t(m.tri[3 * t + i]) + k];
    for (int k = 0; k < 3; ++k) {
      mid[0][k] = 0.5 * (v[1][k] + v[2][k]);
      mid[1][k] = 0.5 * (v[2][k] + v[0][k]);
      mid[2][k] = 0.5 * (v[0][k] + v[1][k]);
    }
    const double* nr = &r.normal[3 * t];
    const double A = r.area[t];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        if (i == j) continue;
        int mi = r.tri_edge[3 * t + i], nj = r.tri_edge[3 * t + j];
        double ci = r.tri_sign[3 * t + i] * r.len[mi] / (2.0 * A);
        double cj = r.tri_sign[3 * t + j] * r.len[nj] / (2.0 * A);
        double s = 0.0;
        for (int q = 0; q < 3; ++q) {
          double fi[3], fj[3];
          for (int k = 0; k < 3; ++k) {
            fi[k] = ci * (mid[q][k] - v[i][k]);
            fj[k] = cj * (mid[q][k] - v[j][k]);
          }
          double nx[3] = {nr[1] * fi[2] - nr[2] * fi[1], nr[2] * fi[0] - nr[0] * fi[2], nr[0] * fi[1] - nr[1] * fi[0]};
          s += nx[0] * fj[0] + nx[1] * fj[1] + nx[2] * fj[2];
        }
        s *= A / 3.0;
        int slot = -1;
        for (int q = 0; q < fill[mi]; ++q)
          if (col[4 * mi + q] == nj) slot = q;
        if (slot < 0) {
          SLIM_REQUIRE(fill[mi] < 4, SLIM_E_MESH, "RWG with more than four I_x neighbours");
          slot = fill[mi]++;
          col[4 * mi + slot] = nj;
        }
        val[4 * mi + slot] += s;
      }
  }
}

template <class T> void up(DevBuf& b, const std::vector<T>& v) { b.upload(v); }

// Solve A X = B (n x n, column-major) from rocSOLVER's LU factors of A (in LU,
// pivots ipiv): row swaps, unit-lower solve (rocBLAS), then a blocked upper solve
// by substitution on 32-row diagonal blocks.  The interior EFIE matrices at low
// frequency have pivots spanning about eight decades; explicit inversion of
// diagonal blocks (as in rocBLAS TRSM) loses all accuracy on such factors,
// substitution does not.  The updates are nested: the rows are cut into panels of
// 512, those into panels of 128, those into the 32-row blocks; once a panel is
// solved, the rows above it inside the enclosing panel are updated by one GEMM whose
// inner dimension is the panel's height.  The large updates thus read and write X
// once per 512 solved rows (inner dimension 512, compute-bound) instead of once per
// 32 (memory-bound); the sums are the same, grouped differently.  Every level is
// reached from n > 512 on.
// B has nrhs columns (leading dimension n).
void lu_solve_rhs(rocblas_handle h, int n, double* LU, const rocblas_int* ipiv, double* B, int nrhs, hipStream_t s) {
  auto Z = [](double* p) { return reinterpret_cast<rocblas_double_complex*>(p); };
  SLIM_ROC(rocsolver_zlaswp(h, nrhs, Z(B), n, 1, n, ipiv, 1));
  rocblas_double_complex one{1.0, 0.0}, mone{-1.0, 0.0};
  SLIM_ROC(rocblas_ztrsm(h, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none, rocblas_diagonal_unit, n,
                         nrhs, &one, Z(LU), n, Z(B), n));
  // X[r0:r1) -= U[r0:r1, c0:c1) X[c0:c1)
  auto update = [&](int r0, int r1, int c0, int c1) {
    SLIM_ROC(rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, r1 - r0, nrhs, c1 - c0, &mone,
                           Z(LU) + int64_t(c0) * n + r0, n, Z(B) + c0, n, &one, Z(B) + r0, n));
  };
  // rows [j0, j1), all updates from the rows below j1 applied; level 0 is one block of
  // at most 32 rows, level k > 0 splits into panels of panel[k - 1] rows from the bottom
  constexpr int kLevels = 3;
  static constexpr int panel[kLevels] = {32, 128, 512};
  auto solve = [&](auto&& self, int j0, int j1, int level) -> void {
    if (level == 0) {
      launch_usolve_block(LU, n, j0, j1 - j0, B, n, nrhs, s);
      return;
    }
    const int P = panel[level - 1];
    for (int i1 = j1; i1 > j0;) {
      const int i0 = std::max(j0, i1 - P);
      self(self, i0, i1, level - 1);
      if (i0 > j0) update(j0, i0, i0, i1);
      i1 = i0;
    }
  };
  solve(solve, 0, n, kLevels);
}

void lu_solve(rocblas_handle h, int n, double* LU, const rocblas_int* ipiv, double* B, hipStream_t s) {
  lu_solve_rhs(h, n, LU, ipiv, B, n, s);
}

Ctx::~Ctx() {
  drop_graphs();
  for (auto& v : prof_ev)
    for (hipEvent_t e : v) (void)hipEventDestroy(e);
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_join) (void)hipEventDestroy(ev_join);
  if (ev_zfork) (void)hipEventDestroy(ev_zfork);
  if (ev_zjoin) (void)hipEventDestroy(ev_zjoin);
  for (hipEvent_t e : gev)
    if (e) (void)hipEventDestroy(e);
  if (s_aux) (void)hipStreamDestroy(s_aux);
  if (s_phi) (void)hipStreamDestroy(s_phi);
  if (s_int) (void)hipStreamDestroy(s_int);
}

namespace {

// One stream of the interior-block generation, driven by a host thread of its own:
// FP64 work buffers for blocks up to order `cap`, a rocBLAS handle on the stream, and
// grow-only buffers for the per-object lists.
struct GenWorker {
  hipStream_t s = nullptr;
  std::unique_ptr<RocHandle> rh;
  DevBuf L, B, Z, ipiv, pairs, zrow, zcol, zval;
  void open(int device, int64_t cap) {
    SLIM_HIP(hipSetDevice(device));
    SLIM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    rh.reset(new RocHandle(s));
    const size_t blk = size_t(cap) * size_t(cap) * 16;
    L.alloc(blk);
    B.alloc(blk);
    Z.alloc(blk);
    ipiv.alloc(size_t(std::max<int64_t>(1, cap)) * sizeof(rocblas_int));
  }
  ~GenWorker() {
    rh.reset();
    if (s) (void)hipStreamDestroy(s);
  }
};

// Copy a host list to a device buffer on stream s (grown, never shrunk, so that
// reallocations, which synchronize the device, stay rare); the host data must stay
// alive until the stream has been synchronized.
template <class T> void upload_on(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
  const size_t bytes = v.size() * sizeof(T);
  if (b.bytes < bytes) b.alloc(std::max(bytes, b.bytes + b.bytes / 2));
  if (bytes) SLIM_HIP(hipMemcpyAsync(b.p, v.data(), bytes, hipMemcpyHostToDevice, s));
}

// What every object's generation shares (read-only while the workers run).
struct GenShared {
  const Ctx* c;
  AsmLaunch base;                              // geometry pointers
  rocblas_int* info;                           // 2 per object: L_kc, L_k0 factorizations
  bool hf;
  const std::vector<std::vector<int32_t>>* z_rows;
  const std::vector<std::vector<int32_t>>* z_cols;
  const std::vector<int64_t>* z_off;           // first entry of each object's Z~ in the CSR
};

// Z_i, M_i = Y_eq,i Z_i of object i into the arena (and its Z~ entries with the
// sparse interior operators), on the worker's stream; returns when they are written.
void gen_object(const GenShared& g, GenWorker& w, int i) {
  const Ctx& c = *g.c;
  const RWGTable& r = c.rwg;
  const int n = c.blocks[i].n;
  const size_t bytes = size_t(n) * n * 16;
  hipStream_t s = w.s;
  rocblas_handle h = w.rh->h;
  AsmLaunch L = g.base;
  L.t0 = int32_t(r.obj_tri_off[i]);
  L.t1 = int32_t(r.obj_tri_off[i + 1]);
  L.e0 = c.blocks[i].e0;
  L.ld_e = n;
  const std::vector<int32_t> pairs = near_candidates(r, L.t0, L.t1, c.opts.c_near);
  upload_on(w.pairs, pairs, s);
  L.near_pairs = w.pairs.as<int32_t>();
  L.n_near_pairs = int64_t(pairs.size() / 2);
  // ---- Z_i = -1/(j w eps_c) L_kc^{-1} (K_kc + I_x/2)  (eq. (4)) ----
  SLIM_HIP(hipMemsetAsync(w.L.p, 0, bytes, s));
  SLIM_HIP(hipMemsetAsync(w.Z.p, 0, bytes, s));
  L.k = c.kc[i];
  L.Lk = w.L.as<double>(); L.Kk = w.Z.as<double>(); L.Lvec = nullptr; L.Lphi = nullptr;
  L.skip_mag = 1e-24;   // conductor kernel: far pairs with |e^{-jk R}| < 1e-24 contribute nothing
  L.cut_r2 = g.hf ? c.opts.hf_radius * c.opts.hf_radius : 0.0;   // sparse L~, K~: distant pairs ignored
  launch_assemble(L, s);
  L.cut_r2 = 0.0;
  launch_add_scaled_ix(w.Z.as<double>(), c.d_ix_col.as<int32_t>(), c.d_ix_val.as<double>(), L.e0, n, 0.5, s);
  SLIM_ROC(rocsolver_zgetrf(h, n, n, reinterpret_cast<rocblas_double_complex*>(w.L.p), n, w.ipiv.as<rocblas_int>(),
                            g.info + 2 * i));
  lu_solve(h, n, w.L.as<double>(), w.ipiv.as<rocblas_int>(), w.Z.as<double>(), s);
  cd fz = -1.0 / (cd(0.0, 1.0) * c.omega * c.epsc[i]);
  launch_scale(w.Z.as<double>(), int64_t(n) * n, fz, s);
  if (g.hf) {
    // keep Z~ on its pattern: gather the entries (complex64 hi + lo), then zero the
    // dense copy off the pattern for M = Y_eq Z~
    const std::vector<int32_t>& zr = (*g.z_rows)[size_t(i)];
    const std::vector<int32_t>& zc = (*g.z_cols)[size_t(i)];
    const int64_t nz = int64_t(zr.size());
    upload_on(w.zrow, zr, s);
    upload_on(w.zcol, zc, s);
    if (w.zval.bytes < size_t(std::max<int64_t>(1, nz)) * 16) w.zval.alloc(size_t(std::max<int64_t>(1, nz)) * 16);
    const int64_t z0 = (*g.z_off)[size_t(i)];
    launch_z_gather_mask(w.Z.as<double>(), n, w.zrow.as<int32_t>(), w.zcol.as<int32_t>(), nz, w.zval.as<double>(),
                         c.d_zs_hi.as<Cplx<float>>() + z0, c.d_zs_lo.as<Cplx<float>>() + z0, s);
  }
  // ---- Y_eq,i = 1/(j w mu0) L_k0^{-1} (K_k0 + I_x/2)  (eq. (5), free-space layer) ----
  SLIM_HIP(hipMemsetAsync(w.L.p, 0, bytes, s));
  SLIM_HIP(hipMemsetAsync(w.B.p, 0, bytes, s));
  L.k = cd(c.k0, 0.0);
  L.Lk = w.L.as<double>(); L.Kk = w.B.as<double>();
  L.skip_mag = 0.0;
  launch_assemble(L, s);
  launch_add_scaled_ix(w.B.as<double>(), c.d_ix_col.as<int32_t>(), c.d_ix_val.as<double>(), L.e0, n, 0.5, s);
  SLIM_ROC(rocsolver_zgetrf(h, n, n, reinterpret_cast<rocblas_double_complex*>(w.L.p), n, w.ipiv.as<rocblas_int>(),
                            g.info + 2 * i + 1));
  lu_solve(h, n, w.L.as<double>(), w.ipiv.as<rocblas_int>(), w.B.as<double>(), s);
  // ---- M_i = Y_eq,i Z_i  (eq. (6)); the 1/(j w mu0) factor folded into alpha ----
  cd fy = 1.0 / (cd(0.0, 1.0) * c.omega * kMu0);
  rocblas_double_complex alpha{fy.real(), fy.imag()}, beta{0.0, 0.0};
  SLIM_ROC(rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, n, n, n, &alpha,
                         reinterpret_cast<rocblas_double_complex*>(w.B.p), n,
                         reinterpret_cast<rocblas_double_complex*>(w.Z.p), n, &beta,
                         reinterpret_cast<rocblas_double_complex*>(w.L.p), n));
  const int64_t row0 = g.hf ? n : 0;   // sparse mode: only the rows of M_i are stored
  const int64_t first = c.blocks[i].off + row0 * ((n + 1) & ~1);
  launch_pack_block(w.Z.as<double>(), w.L.as<double>(), n, int(row0), c.d_hi.as<Cplx<float>>() + first,
                    c.d_lo.as<Cplx<float>>() + first, s);
  SLIM_HIP(hipStreamSynchronize(s));   // the host lists above and the work buffers are reused next
}

}  // namespace

static void build_internal(Ctx& c, hipStream_t s) {
  const RWGTable& r = c.rwg;
  // arena layout: the 2n x ld rows of [Z_i; M_i] (rows padded to an even length,
  // 16-byte aligned); with sparse interior operators only the n rows of M_i, and a
  // block's offset is that of its (absent) row 0, so rows n..2n-1 sit where they would
  const bool hf = c.opts.hf_radius > 0.0;
  c.blocks.resize(r.n_obj);
  int64_t off = 0, nmax = 0;
  for (int i = 0; i < r.n_obj; ++i) {
    int64_t n = r.obj_edge_off[i + 1] - r.obj_edge_off[i];
    const int64_t ld = (n + 1) & ~int64_t(1);
    c.blocks[i] = {hf ? off - n * ld : off, int32_t(n), int32_t(r.obj_edge_off[i])};
    off += (hf ? 1 : 2) * n * ld;
    nmax = std::max(nmax, n);
  }
  c.arena_elems = off;
  auto workspace = [](int64_t n) { return 3 * n * n * 16; };   // L, B, Z of one worker
  if (c.opts.mem_budget > 0) {
    int64_t need = off * 16 + workspace(nmax);
    SLIM_REQUIRE(need <= c.opts.mem_budget, SLIM_E_OOM,
                 "device memory budget too small: internal blocks need " + std::to_string(need) + " bytes");
  }
  c.d_hi.alloc(size_t(off) * sizeof(Cplx<float>));
  c.d_lo.alloc(size_t(off) * sizeof(Cplx<float>));
  up(c.d_blocks, c.blocks);
  DevBuf info;
  info.alloc(sizeof(rocblas_int) * size_t(r.n_obj) * 2);
  SLIM_HIP(hipMemsetAsync(info.p, 0, info.bytes, s));
  // sparse Z~ (hf_radius > 0): CSR over all RWG rows, global columns, in object order;
  // per object the local (row, column) list gathers its entries from the dense FP64
  // solution into its own range of the CSR
  std::vector<int64_t> zs_ptr(1, 0), z_off(size_t(r.n_obj) + 1, 0);
  std::vector<int32_t> zs_col;
  if (hf) {
    c.d_zs_hi.release();
    c.d_zs_lo.release();
  }
  std::vector<std::vector<int32_t>> z_rows(hf ? r.n_obj : 0), z_cols(hf ? r.n_obj : 0);
  for (int i = 0; hf && i < r.n_obj; ++i) {
    const int n = c.blocks[i].n;
    z_pattern(r, r.obj_tri_off[i], r.obj_tri_off[i + 1], c.blocks[i].e0, n, c.opts.hf_radius, z_rows[i], z_cols[i]);
    const int64_t nz = int64_t(z_rows[i].size());
    z_off[size_t(i) + 1] = z_off[size_t(i)] + nz;
    for (int64_t k = 0; k < nz; ++k) zs_col.push_back(c.blocks[i].e0 + z_cols[i][size_t(k)]);
    int64_t k = 0;
    for (int m = 0; m < n; ++m) {
      while (k < nz && z_rows[i][size_t(k)] == m) ++k;
      zs_ptr.push_back(z_off[size_t(i)] + k);
    }
  }
  const int64_t z_total = z_off.back();
  if (hf) {
    SLIM_REQUIRE(z_total < (int64_t(1) << 40), SLIM_E_UNSUPPORTED, "sparse interior operator too large");
    c.d_zs_hi.alloc(size_t(std::max<int64_t>(1, z_total)) * sizeof(Cplx<float>));
    c.d_zs_lo.alloc(size_t(std::max<int64_t>(1, z_total)) * sizeof(Cplx<float>));
  }
  SLIM_HIP(hipStreamSynchronize(s));

  GenShared g;
  g.c = &c;
  AsmLaunch& L = g.base;
  L = AsmLaunch{};
  L.xyz = c.d_xyz.as<double>(); L.tri = c.d_tri.as<int32_t>(); L.cen = c.d_cen.as<double>();
  L.nrm = c.d_nrm.as<double>(); L.area = c.d_area.as<double>(); L.diam = c.d_diam.as<double>();
  L.tri_edge = c.d_tri_edge.as<int32_t>(); L.tri_sign = c.d_tri_sign.as<int8_t>(); L.len = c.d_len.as<double>();
  g.info = info.as<rocblas_int>();
  g.hf = hf;
  g.z_rows = &z_rows;
  g.z_cols = &z_cols;
  g.z_off = &z_off;

  // The objects are handed out in decreasing size -- the list order of LPT (Alg. 1);
  // any cost estimate that grows with n_i (the LU's n_i^3, the paper's n_i^2) gives
  // this order -- each to the first worker that is free.  Workers are streams with
  // host threads of their own, so that the many short kernels of small objects
  // (panel factorizations, narrow solves) overlap.  Objects whose workspace does not
  // fit the memory left beside the arena once per worker go first, one at a time.
  std::vector<int> order(size_t(r.n_obj));
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return c.blocks[a].n > c.blocks[b].n; });
  size_t freeb = 0, totalb = 0;
  SLIM_HIP(hipMemGetInfo(&freeb, &totalb));
  int64_t budget = int64_t(freeb) - (int64_t(4) << 30);   // room for rocBLAS workspaces and the lists
  if (c.opts.mem_budget > 0) budget = std::min(budget, c.opts.mem_budget - off * 16);
  budget = std::max(budget, workspace(nmax));
  const int K = std::max(1, std::min(r.n_obj, c.opts.gen_workers > 0 ? c.opts.gen_workers : 8));
  size_t split = 0;
  while (split < order.size() && int64_t(K) * workspace(c.blocks[order[split]].n) > budget) ++split;

  std::atomic<int> done{0};
  std::mutex print_mu;
  auto last_print = std::chrono::steady_clock::now();
  auto run_pool = [&](size_t b0, size_t b1, int workers) {
    if (b1 <= b0) return;
    const int64_t cap = c.blocks[order[b0]].n;
    std::atomic<size_t> next{b0};
    std::atomic<bool> stop{false};
    std::exception_ptr err;
    std::mutex err_mu;
    auto body = [&]() {
      try {
        GenWorker w;
        w.open(c.device, cap);
        for (size_t k = next++; k < b1 && !stop; k = next++) {
          const int i = order[k];
          gen_object(g, w, i);
          const int d = ++done;
          if (c.opts.verbose) {
            std::lock_guard<std::mutex> lk(print_mu);
            auto now = std::chrono::steady_clock::now();
            if (d == r.n_obj || std::chrono::duration<double>(now - last_print).count() > 10.0) {
              std::fprintf(stderr, "[slim build] interior blocks %d / %d (n = %d)\n", d, r.n_obj, c.blocks[i].n);
              std::fflush(stderr);
              last_print = now;
            }
          }
        }
      } catch (...) {
        std::lock_guard<std::mutex> lk(err_mu);
        if (!err) err = std::current_exception();
        stop = true;
      }
    };
    const int nw = int(std::min<size_t>(size_t(workers), b1 - b0));
    if (nw == 1) {
      body();
    } else {
      std::vector<std::thread> th;
      for (int k = 0; k < nw; ++k) th.emplace_back(body);
      for (std::thread& t : th) t.join();
    }
    SLIM_HIP(hipSetDevice(c.device));
    if (err) std::rethrow_exception(err);
  };
  const auto t_gen = std::chrono::steady_clock::now();
  run_pool(0, split, 1);
  run_pool(split, order.size(), K);
  c.gen_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_gen).count();
  c.gen_workers = split < order.size() ? std::min<int>(K, int(order.size() - split)) : 1;

  std::vector<rocblas_int> h_info(2 * size_t(r.n_obj));
  SLIM_HIP(hipMemcpy(h_info.data(), info.p, info.bytes, hipMemcpyDeviceToHost));
  for (int i = 0; i < 2 * r.n_obj; ++i)
    SLIM_REQUIRE(h_info[i] == 0, SLIM_E_NUMERIC,
                 "singular interior matrix of object " + std::to_string(i / 2) + (i % 2 ? " (L_k0)" : " (L_kc)"));
  c.hf_sparse = hf;
  c.z_nnz = hf ? z_total : 0;
  if (hf) {
    SLIM_REQUIRE(int64_t(zs_ptr.size()) == r.n_e + 1 && zs_ptr.back() == z_total, SLIM_E_STATE,
                 "sparse interior operator: row pointers do not cover the edges");
    c.d_zs_ptr.upload(zs_ptr);
    c.d_zs_col.upload(zs_col);
  } else {
    c.d_zs_ptr.release();
    c.d_zs_col.release();
    c.d_zs_hi.release();
    c.d_zs_lo.release();
  }
}

static void build_plain_external(Ctx& c, hipStream_t s) {
  const RWGTable& r = c.rwg;
  const int64_t ne = r.n_e, nt = r.n_t;
  DevBuf LA, LP, d_pairs;
  LA.alloc(size_t(ne * ne) * 16);
  LP.alloc(size_t(nt * nt) * 16);
  SLIM_HIP(hipMemsetAsync(LA.p, 0, LA.bytes, s));
  SLIM_HIP(hipMemsetAsync(LP.p, 0, LP.bytes, s));
  AsmLaunch L{};
  L.xyz = c.d_xyz.as<double>(); L.tri = c.d_tri.as<int32_t>(); L.cen = c.d_cen.as<double>();
  L.nrm = c.d_nrm.as<double>(); L.area = c.d_area.as<double>(); L.diam = c.d_diam.as<double>();
  L.tri_edge = c.d_tri_edge.as<int32_t>(); L.tri_sign = c.d_tri_sign.as<int8_t>(); L.len = c.d_len.as<double>();
  L.t0 = 0; L.t1 = int32_t(nt); L.e0 = 0;
  L.k = cd(c.k0, 0.0);
  L.Lvec = LA.as<double>(); L.Lphi = LP.as<double>();
  L.ld_e = ne; L.ld_t = nt;
  std::vector<int32_t> pairs = near_candidates(r, 0, nt, c.opts.c_near);
  d_pairs.upload(pairs);
  L.near_pairs = d_pairs.as<int32_t>();
  L.n_near_pairs = int64_t(pairs.size() / 2);
  launch_assemble(L, s);
  // L_A and L_phi are symmetric: the column-major arrays are also row-major.
  c.d_LA_hi.alloc(size_t(ne * ne) * 8); c.d_LA_lo.alloc(size_t(ne * ne) * 8);
  c.d_Lphi_hi.alloc(size_t(nt * nt) * 8); c.d_Lphi_lo.alloc(size_t(nt * nt) * 8);
  launch_pack_dense(LA.as<double>(), ne, ne, c.d_LA_hi.as<Cplx<float>>(), c.d_LA_lo.as<Cplx<float>>(), s);
  launch_pack_dense(LP.as<double>(), nt, nt, c.d_Lphi_hi.as<Cplx<float>>(), c.d_Lphi_lo.as<Cplx<float>>(), s);
  SLIM_HIP(hipStreamSynchronize(s));
}

// ---- autotuning of the kernel shapes --------------------------------------------
// The whole mixed product is timed (captured graph, pulse path concurrent) for every
// combination of persistent internal workgroups per compute unit {2, 4, 8}, the
// auto-valued shapes (z-plane padding of the FFT work array {0, 64}, rows per wave
// of the internal kernel {4, 8}), two interleaved rounds, best of each.  Results are
// kept in an optional text cache keyed by (kernel, shape, architecture).
namespace {

// the shape is tuned for the queue form it will run with (static queues and dynamic
// dispatch favour different workgroup counts)
std::string tune_key(const Ctx& c, const char* arch, int cus, bool dynamic) {
  char buf[512];
  std::snprintf(buf, sizeof(buf),
                "product|%s|cus=%d|n_e=%lld|n_t=%lld|n_obj=%d|grid=%dx%dx%d|entries=%lld|nnz=%lld+%lld|queues=%s",
                arch, cus, (long long)c.rwg.n_e, (long long)c.rwg.n_t, c.rwg.n_obj, c.plain ? 0 : c.grid.N[0],
                c.plain ? 0 : c.grid.N[1], c.plain ? 0 : c.grid.N[2], (long long)c.arena_elems, (long long)c.nnz_A,
                (long long)c.nnz_P, dynamic ? "dynamic" : "static");
  return buf;
}

bool tune_cache_lookup(const char* path, const std::string& key, int& per_cu, int& zb, int& rw, int& zpc) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    std::string l(line);
    const size_t bar = l.rfind("|per_cu=");
    if (bar == std::string::npos || l.compare(0, bar, key) != 0 || bar != key.size()) continue;
    int a = 0, b = 0, r = 0, z = 0;
    const int got = std::sscanf(l.c_str() + bar, "|per_cu=%d|zblock=%d|rw=%d|z_per_cu=%d", &a, &b, &r, &z);
    if (got >= 3 && a > 0 && b >= 1 && b <= 64 && (b & (b - 1)) == 0 && (r == 4 || r == 8)) {
      per_cu = a; zb = b; rw = r;
      zpc = got == 4 && z > 0 && z <= a ? z : a;   // older lines: the rows of Z_i on every slot
      found = true;   // the last matching line wins
    }
  }
  std::fclose(f);
  return found;
}

void tune_cache_store(const char* path, const std::string& key, int per_cu, int zb, int rw, int zpc, double ms) {
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;   // an unwritable cache only costs the timing next time
  std::fprintf(f, "%s|per_cu=%d|zblock=%d|rw=%d|z_per_cu=%d|ms=%.4f\n", key.c_str(), per_cu, zb, rw, zpc, ms);
  std::fclose(f);
}

}  // namespace

static void autotune(Ctx& c, const slim_build_opts& o, hipStream_t s) {
  int cus = 256;
  char arch[64] = "unknown";
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c.device) == hipSuccess) {
    if (prop.multiProcessorCount > 0) cus = prop.multiProcessorCount;
    std::snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
    if (char* colon = std::strchr(arch, ':')) *colon = '\0';
  }
  // before any training the learned modes pack on flop counts
  const int pack_mode = o.sched_mode == 1 ? 0 : o.sched_mode == 4 ? 3 : o.sched_mode;
  const std::string key = tune_key(c, arch, cus, pack_mode == 3);
  int per_cu = 0, zb = 0, rw = 0, zpc = 0;
  if (tune_cache_lookup(o.tune_cache, key, per_cu, zb, rw, zpc)) {
    c.slots = per_cu * cus;
    c.slots_z = zpc * cus;
    c.fft_zsh = ilog2(zb);
    c.rw_mixed = rw;
    pack_tiles(c, pack_mode);
    if (o.verbose)
      std::fprintf(stderr, "[slim build] autotune: cached %d per CU (rows of Z_i: %d), z block %d, rw %d\n", per_cu, zpc,
                   zb, rw);
    return;
  }
  SLIM_HIP(hipMemsetAsync(c.d_x64.p, 0, c.d_x64.bytes, s));
  SLIM_HIP(hipStreamSynchronize(s));
  std::vector<int> zbs = o.fft_zblock > 0 || c.plain ? std::vector<int>{1 << c.fft_zsh} : std::vector<int>{1, 8};
  std::vector<int> rws = o.rows_per_wave > 0 ? std::vector<int>{c.rw_mixed} : std::vector<int>{4, 8};
  const int per_cu_set[3] = {2, 4, 8};
  // workgroups of the launch of the rows of Z_i, which runs beside the projection and FFT
  // of j: as many as the other launch, or one per CU (room for the FFT's workgroups).  One
  // per CU only under dynamic dispatch: static queues packed for so few workgroups leave a
  // long tail, and only there can the FP64 launch take the M rows' count instead
  struct Cand { int per_cu, zb, rw, zpc; double ms; };
  std::vector<Cand> cand;
  for (int pc : per_cu_set)
    for (int z : zbs)
      for (int r : rws)
        for (int zpc : {pc, 1})
          if (zpc == pc || (!c.plain && pack_mode == 3)) cand.push_back({pc, z, r, zpc, 1e300});
  for (int round = 0; round < 2; ++round)
    for (Cand& k : cand) {
      if (k.per_cu * cus != c.slots || k.zpc * cus != c.zslots()) {
        c.slots = k.per_cu * cus;
        c.slots_z = k.zpc * cus;
        pack_tiles(c, pack_mode);
      }
      c.fft_zsh = ilog2(k.zb);
      c.rw_mixed = k.rw;
      k.ms = std::min(k.ms, time_product(c, 4));
    }
  const Cand* best = &cand[0];
  for (const Cand& k : cand) {
    if (o.verbose)
      std::fprintf(stderr, "[slim build] autotune: %d per CU (rows of Z_i: %d), z block %d, rw %d -> %.3f ms per product\n",
                   k.per_cu, k.zpc, k.zb, k.rw, k.ms);
    if (k.ms < best->ms) best = &k;
  }
  c.slots = best->per_cu * cus;
  c.slots_z = best->zpc * cus;
  c.fft_zsh = ilog2(best->zb);
  c.rw_mixed = best->rw;
  pack_tiles(c, pack_mode);
  tune_cache_store(o.tune_cache, key, best->per_cu, best->zb, best->rw, best->zpc, best->ms);
}

void build_all(Ctx& c, const slim_build_opts& o) {
  auto t_start = std::chrono::steady_clock::now();
  SLIM_REQUIRE(c.has_mesh, SLIM_E_STATE, "slim_set_mesh must be called before slim_build");
  SLIM_REQUIRE(o.freq > 0.0, SLIM_E_ARG, "frequency must be positive");
  const bool aim = !(o.grid[0] == 0 && o.grid[1] == 0 && o.grid[2] == 0);
  for (int k = 0; aim && k < 3; ++k)
    SLIM_REQUIRE(o.grid[k] >= 8 && o.grid[k] <= 512 && (o.grid[k] & (o.grid[k] - 1)) == 0, SLIM_E_UNSUPPORTED,
                 "AIM grid size must be a power of two between 8 and 512 per axis");
  SLIM_REQUIRE(o.internal_kernel == 0, SLIM_E_UNSUPPORTED,
               "internal_kernel: only the FP32-FMA GEMV (0) is built; a split-BF16 MFMA kernel would read the same "
               "bytes at one right-hand side");
  SLIM_REQUIRE(std::isfinite(o.hf_radius) && o.hf_radius >= 0.0, SLIM_E_ARG, "hf_radius must be finite and >= 0");
  SLIM_REQUIRE(!(o.hf_radius > 0.0 && o.precond), SLIM_E_UNSUPPORTED,
               "the conductor-block preconditioner needs the dense Z_i rows: build with precond = 0 when hf_radius > 0");
  SLIM_REQUIRE(o.gen_workers >= 0 && o.gen_workers <= 64, SLIM_E_ARG, "gen_workers must be in [0, 64]");
  SLIM_REQUIRE(o.fft_zblock == 0 || (o.fft_zblock > 0 && o.fft_zblock <= 64 && (o.fft_zblock & (o.fft_zblock - 1)) == 0),
               SLIM_E_ARG, "fft_zblock must be 0 or a power of two up to 64");
  SLIM_REQUIRE(!aim || o.fft_zblock <= o.grid[2], SLIM_E_ARG, "fft_zblock must not exceed the grid's Nz");
  SLIM_HIP(hipSetDevice(c.device));
  c.built = false;
  // A new build starts in free space: the reflected kernels, their spectra and the
  // kept free-space near values belong to the previous frequency, grid and mesh.
  c.drop_graphs();
  c.layered = false;
  c.lay_zif = 0.0;
  c.lay_nodes = 0;
  c.d_lay_real.release();
  c.d_rhat128.release();
  c.d_rhat64.release();
  c.d_lay.release();
  c.d_nA_free.release();
  c.d_nP_free.release();
  // the block product's workspace is laid out for the old mesh
  c.blk_ldh = 0;
  c.blk_cols = 0;
  c.d_blk_hs.release();
  c.d_blk_h64.release();
  c.d_blk_e.release();
  c.d_blk_j.release();
  c.d_blk_hoff.release();
  c.d_blk_hpos.release();
  c.opts = o;
  c.freq = o.freq;
  c.omega = 2.0 * kPi * o.freq;
  c.k0 = c.omega / kC0;
  const RWGTable& r = c.rwg;
  c.kc.resize(r.n_obj);
  c.epsc.resize(r.n_obj);
  for (int i = 0; i < r.n_obj; ++i) {
    const Material& mt = c.mats.empty() ? Material{} : c.mats[i];
    c.epsc[i] = cd(eps0() * mt.eps_r, -mt.sigma / c.omega);
    cd k = c.omega * std::sqrt(kMu0 * mt.mu_r * c.epsc[i]);
    c.kc[i] = k.imag() <= 0.0 ? k : -k;
  }
  QuadOpts qo;
  qo.n_far = o.n_far; qo.n_near = o.n_near; qo.levels = o.levels; qo.n_r = o.n_r; qo.n_t = o.n_t;
  qo.q = o.q; qo.c_near = o.c_near;
  QuadRulesDev rules;
  make_rules(qo, rules);
  upload_rules(rules);

  hipStream_t s = nullptr;
  SLIM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  struct SG { hipStream_t s; ~SG() { if (s) (void)hipStreamDestroy(s); } } sg{s};
  // geometry
  std::vector<int8_t> sign(r.tri_sign.begin(), r.tri_sign.end());
  up(c.d_xyz, c.mesh.xyz); up(c.d_tri, c.mesh.tri); up(c.d_cen, r.centroid); up(c.d_nrm, r.normal);
  up(c.d_area, r.area); up(c.d_diam, r.diam); up(c.d_tri_edge, r.tri_edge); up(c.d_tri_sign, sign);
  up(c.d_len, r.len); up(c.d_tplus, r.tplus); up(c.d_tminus, r.tminus);
  std::vector<int32_t> ixc;
  std::vector<double> ixv;
  build_ix(c.mesh, r, ixc, ixv);
  up(c.d_ix_col, ixc); up(c.d_ix_val, ixv);

  auto say = [&](const char* what) {
    if (!o.verbose) return;
    std::fprintf(stderr, "[slim build] %s (%.1f s)\n", what,
                 std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count());
    std::fflush(stderr);
  };
  say("geometry uploaded");
  build_internal(c, s);
  say("interior blocks done");
  c.plain = (o.grid[0] == 0 && o.grid[1] == 0 && o.grid[2] == 0);
  if (c.plain) build_plain_external(c, s);
  else build_aim(c, s);
  say("external operator done");

  // vectors
  const int64_t nsys = r.n_e + r.n_t;
  c.drop_graphs();
  c.d_x64.alloc(size_t(nsys) * 8);
  c.d_y64.alloc(size_t(nsys) * 8);
  c.d_e.alloc(size_t(r.n_e) * 16);
  c.d_g.alloc(size_t(r.n_e) * 16);
  c.d_j.alloc(size_t(r.n_e) * 16);
  c.d_a.alloc(size_t(r.n_e) * 16);
  c.d_phi.alloc(size_t(r.n_t) * 16);
  if (!c.s_aux) SLIM_HIP(hipStreamCreateWithFlags(&c.s_aux, hipStreamNonBlocking));
  if (!c.s_phi) SLIM_HIP(hipStreamCreateWithFlags(&c.s_phi, hipStreamNonBlocking));
  if (!c.ev_fork) SLIM_HIP(hipEventCreateWithFlags(&c.ev_fork, hipEventDisableTiming));
  if (!c.ev_join) SLIM_HIP(hipEventCreateWithFlags(&c.ev_join, hipEventDisableTiming));
  if (!c.s_int) SLIM_HIP(hipStreamCreateWithFlags(&c.s_int, hipStreamNonBlocking));
  if (!c.ev_zfork) SLIM_HIP(hipEventCreateWithFlags(&c.ev_zfork, hipEventDisableTiming));
  if (!c.ev_zjoin) SLIM_HIP(hipEventCreateWithFlags(&c.ev_zjoin, hipEventDisableTiming));

  SLIM_REQUIRE(o.sched_mode >= 0 && o.sched_mode <= 4, SLIM_E_ARG, "sched_mode must be 0..4");
  c.tile_rows = o.tile_rows > 0 ? o.tile_rows : 64;
  c.sched_mode = o.sched_mode;
  c.drop_graphs();
  SLIM_REQUIRE(o.rows_per_wave == 0 || o.rows_per_wave == 4 || o.rows_per_wave == 8, SLIM_E_ARG,
               "rows_per_wave must be 0, 4 or 8");
  c.fft_zsh = o.fft_zblock > 0 ? ilog2(o.fft_zblock) : 3;
  c.rw_mixed = o.rows_per_wave > 0 ? o.rows_per_wave : 8;
  SLIM_REQUIRE(o.slots_z >= 0, SLIM_E_ARG, "slots_z must be >= 0");
  if (o.slots > 0) {
    c.slots = o.slots;
    c.slots_z = o.slots_z;
    pack_tiles(c, o.sched_mode);
  } else {
    autotune(c, o, s);
  }
  SLIM_HIP(hipStreamSynchronize(s));
  build_precond(c, s);
  if (o.precond) say("preconditioner done");

  slim_layout& Lo = c.layout;
  Lo = slim_layout{};
  Lo.n_e = r.n_e; Lo.n_t = r.n_t; Lo.n_sys = nsys; Lo.n_obj = r.n_obj;
  for (int k = 0; k < 3; ++k) {
    Lo.grid[k] = c.plain ? 0 : c.grid.N[k];
    Lo.grid_h[k] = c.grid.h[k];
    Lo.grid_origin[k] = c.grid.origin[k];
  }
  Lo.nnz_near_A = c.nnz_A; Lo.nnz_near_phi = c.nnz_P;
  Lo.internal_entries = c.arena_elems;
  Lo.n_tiles = int64_t(c.tiles.size());
  Lo.slots = c.slots;
  Lo.tile_rows = c.tile_rows;
  Lo.mean_edge = r.mean_edge;
  Lo.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  size_t freeb = 0, totalb = 0;
  (void)hipMemGetInfo(&freeb, &totalb);
  Lo.device_bytes = int64_t(totalb - freeb);
  Lo.precond_blocks = c.pc_built ? int64_t(c.pc_blocks.size()) : 0;
  Lo.precond_entries = c.pc_built ? c.pc_entries : 0;
  Lo.precond_cap = c.pc_cap;
  Lo.fft_zblock = c.plain ? 0 : 1 << c.fft_zsh;
  Lo.rows_per_wave = c.rw_mixed;
  Lo.z_nnz = c.z_nnz;
  Lo.slots_z = c.zslots();
  Lo.interior_workers = c.gen_workers;
  Lo.interior_seconds = c.gen_seconds;
  c.built = true;
}

}  // namespace slim
