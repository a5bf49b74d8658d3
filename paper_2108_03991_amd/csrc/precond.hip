// Conductor-block preconditioner of the solve.
//
// The paper right-preconditions GMRES with a constraint preconditioner
// (Sec. III-E) and leaves its definition to a reference.  It is read here as
// block Jacobi over conductors on the row-equilibrated system S A, with
// S = diag(1/h^2 on the RWG rows, h on the pulse rows).  The block of a
// conductor is S A restricted to its own RWG edges and triangles:
//
//   [ (j k0 L_A (I - M_i) + I_x Z_i / eta0) / h^2     D^T L_phi B / h^2 ]
//   [ h F D (I - M_i)                                  h j k0 I          ]
//
// Here L_A and L_phi are the conductor's exact self interactions (not the AIM
// approximation). Each block is inverted in FP64 (LU) and stored as complex64
// rows.
//
// A conductor above the size cap is cut by recursive coordinate bisection
// (RCB) of its triangle centroids:
//  - split along the axis of largest extent (lowest axis on ties);
//  - stable order by that coordinate, the first half takes size/2 triangles;
//  - stop at <= cap unknowns, counting owned edges plus triangles;
//  - an edge belongs to the part that holds its T+.
// Each part is grown by max(overlap, 1) rings of edge-adjacent triangles. The
// extended set holds those triangles and the edges with both triangles among
// them. No current crosses the boundary of a part, so it is solved as an
// isolated piece of conductor. An edge cut open instead would carry current
// whose charge lies outside the block, governed only by j k0 L_A; at low
// frequency its local inverse blows up. A part keeps its own rows of the
// extended block's inverse (restricted additive Schwarz). Every unknown is
// written by exactly one block.
//
// Storing the rows in complex64 makes the preconditioner only approximately
// linear, so the solver uses flexible GMRES.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <numeric>
#include <queue>

#include "ctx.hpp"

namespace slim {

std::vector<int32_t> near_candidates(const RWGTable& r, int64_t t0, int64_t t1, double c_near);   // build.cpp
void lu_solve_rhs(rocblas_handle h, int n, double* LU, const rocblas_int* ipiv, double* B, int nrhs, hipStream_t s);

namespace {

#define SLIM_ROCP(call)                                                                       \
  do {                                                                                        \
    rocblas_status st_ = (call);                                                              \
    if (st_ != rocblas_status_success)                                                        \
      throw ::slim::Error(SLIM_E_HIP, std::string(#call) + " failed: " + std::to_string(int(st_))); \
  } while (0)

unsigned nb256(int64_t n) { return unsigned((n + 255) / 256); }

// ---------------------------------------------------------------------------
// Host partition
// ---------------------------------------------------------------------------
struct Part {
  int32_t obj = 0;
  std::vector<int32_t> ext_e, ext_t;   // global edge / triangle ids, ascending
  std::vector<int32_t> own_pos;        // positions in [ext_e, ext_t] of the owned unknowns
  int64_t n_R = 0;                     // triangles adjacent to ext_e (rows of the L_phi slice)
};

struct Partitioner {
  const RWGTable& r;
  std::vector<int32_t> plus_count;     // edges whose T+ is the triangle
  std::vector<char> mark;
  explicit Partitioner(const RWGTable& r_) : r(r_), plus_count(size_t(r_.n_t), 0), mark(size_t(r_.n_t), 0) {
    for (int64_t e = 0; e < r.n_e; ++e) plus_count[size_t(r.tplus[e])]++;
  }
  int64_t unknowns(const std::vector<int32_t>& tris) const {
    int64_t u = 0;
    for (int32_t t : tris) u += plus_count[size_t(t)] + 1;
    return u;
  }
  void rcb(std::vector<int32_t> tris, int64_t cap, std::vector<std::vector<int32_t>>& out) const {
    if (unknowns(tris) <= cap || tris.size() < 2) {
      out.push_back(std::move(tris));
      return;
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int32_t t : tris)
      for (int k = 0; k < 3; ++k) {
        lo[k] = std::min(lo[k], r.centroid[3 * size_t(t) + k]);
        hi[k] = std::max(hi[k], r.centroid[3 * size_t(t) + k]);
      }
    int axis = 0;
    double best = hi[0] - lo[0];
    for (int k = 1; k < 3; ++k)
      if (hi[k] - lo[k] > best) { best = hi[k] - lo[k]; axis = k; }
    std::vector<int32_t> order = tris;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      return r.centroid[3 * size_t(a) + axis] < r.centroid[3 * size_t(b) + axis];
    });
    const size_t half = order.size() / 2;
    std::vector<int32_t> left(order.begin(), order.begin() + half), right(order.begin() + half, order.end());
    std::sort(left.begin(), left.end());
    std::sort(right.begin(), right.end());
    rcb(std::move(left), cap, out);
    rcb(std::move(right), cap, out);
  }
  std::vector<int32_t> grow(const std::vector<int32_t>& tris, int layers) {
    std::vector<int32_t> cur = tris;
    for (int32_t t : cur) mark[size_t(t)] = 1;
    for (int l = 0; l < layers; ++l) {
      std::vector<int32_t> ring;
      for (int32_t t : cur)
        for (int k = 0; k < 3; ++k) {
          const int32_t e = r.tri_edge[3 * size_t(t) + k];
          for (int32_t u : {r.tplus[size_t(e)], r.tminus[size_t(e)]})
            if (!mark[size_t(u)]) { mark[size_t(u)] = 1; ring.push_back(u); }
        }
      cur.insert(cur.end(), ring.begin(), ring.end());
    }
    for (int32_t t : cur) mark[size_t(t)] = 0;
    std::sort(cur.begin(), cur.end());
    return cur;
  }
  std::vector<int32_t> edges_with_tplus_in(const std::vector<int32_t>& tris) const {
    std::vector<int32_t> e;
    for (int32_t t : tris)
      for (int k = 0; k < 3; ++k) {
        const int32_t ed = r.tri_edge[3 * size_t(t) + k];
        if (r.tplus[size_t(ed)] == t) e.push_back(ed);
      }
    std::sort(e.begin(), e.end());
    return e;
  }
  // edges with both triangles in the set: no current crosses the block boundary
  std::vector<int32_t> edges_inside(const std::vector<int32_t>& tris) {
    for (int32_t t : tris) mark[size_t(t)] = 1;
    std::vector<int32_t> e;
    for (int32_t t : tris)
      for (int k = 0; k < 3; ++k) {
        const int32_t ed = r.tri_edge[3 * size_t(t) + k];
        if (r.tplus[size_t(ed)] == t && mark[size_t(r.tminus[size_t(ed)])]) e.push_back(ed);
      }
    for (int32_t t : tris) mark[size_t(t)] = 0;
    std::sort(e.begin(), e.end());
    return e;
  }
  std::vector<Part> partition(int64_t cap, int overlap) {
    std::vector<Part> parts;
    for (int32_t i = 0; i < r.n_obj; ++i) {
      std::vector<int32_t> tris(size_t(r.obj_tri_off[i + 1] - r.obj_tri_off[i]));
      std::iota(tris.begin(), tris.end(), int32_t(r.obj_tri_off[i]));
      std::vector<std::vector<int32_t>> pl;
      if (cap <= 0) pl.push_back(tris);
      else rcb(tris, cap, pl);
      for (auto& p : pl) {
        Part q;
        q.obj = i;
        q.ext_t = pl.size() == 1 ? p : grow(p, std::max(overlap, 1));
        q.ext_e = edges_inside(q.ext_t);
        const std::vector<int32_t> own_e = edges_with_tplus_in(p);
        for (int32_t e : own_e)
          q.own_pos.push_back(int32_t(std::lower_bound(q.ext_e.begin(), q.ext_e.end(), e) - q.ext_e.begin()));
        for (int32_t t : p)
          q.own_pos.push_back(int32_t(q.ext_e.size() + (std::lower_bound(q.ext_t.begin(), q.ext_t.end(), t) - q.ext_t.begin())));
        // triangles adjacent to the extended edges (rows of the L_phi slice)
        std::vector<int32_t> R;
        for (int32_t e : q.ext_e) { R.push_back(r.tplus[size_t(e)]); R.push_back(r.tminus[size_t(e)]); }
        std::sort(R.begin(), R.end());
        q.n_R = int64_t(std::unique(R.begin(), R.end()) - R.begin());
        parts.push_back(std::move(q));
      }
    }
    return parts;
  }
};

// column panels of the (I - M) gather and of the block inverse (bounds the build buffers)
constexpr int64_t kPanel = 2048;

struct Plan {
  std::vector<Part> parts;
  int64_t cap = 0;
  int64_t stored = 0;          // complex64 entries (rows x padded ext)
  int64_t n_ext = 0, n_own = 0;
  size_t t_la = 0, t_lp = 0, t_mc = 0, t_w = 0, t_b = 0, t_x = 0, t_ipiv = 0, t_emap = 0, t_tmap = 0;
  size_t bytes() const {
    return size_t(stored) * 8 + size_t(n_ext) * (8 + 4) + size_t(n_own) * 4 + t_la + t_lp + t_mc + t_w + t_b + t_x +
           t_ipiv + t_emap + t_tmap + (size_t(1) << 24);
  }
};

Plan make_plan(Partitioner& P, const RWGTable& r, int64_t cap, int overlap) {
  Plan pl;
  pl.cap = cap;
  pl.parts = P.partition(cap, overlap);
  for (const Part& q : pl.parts) {
    const int64_t n = r.obj_edge_off[q.obj + 1] - r.obj_edge_off[q.obj];
    const int64_t t = r.obj_tri_off[q.obj + 1] - r.obj_tri_off[q.obj];
    const int64_t E = int64_t(q.ext_e.size()), s = E + int64_t(q.ext_t.size());
    const int64_t ld = (s + 1) & ~int64_t(1);
    pl.stored += int64_t(q.own_pos.size()) * ld;
    pl.n_ext += s;
    pl.n_own += int64_t(q.own_pos.size());
    pl.t_la = std::max(pl.t_la, size_t(E * n) * 16);
    pl.t_lp = std::max(pl.t_lp, size_t(q.n_R * t) * 16);
    pl.t_mc = std::max(pl.t_mc, size_t(n * std::min<int64_t>(E, kPanel)) * 16);
    pl.t_w = std::max(pl.t_w, size_t(E * E) * 16);
    pl.t_b = std::max(pl.t_b, size_t(s * s) * 16);
    pl.t_x = std::max(pl.t_x, size_t(s * std::min<int64_t>(s, kPanel)) * 16);
    pl.t_ipiv = std::max(pl.t_ipiv, size_t(s) * sizeof(rocblas_int));
    pl.t_emap = std::max(pl.t_emap, size_t(n) * 4);
    pl.t_tmap = std::max(pl.t_tmap, size_t(t) * 4);
  }
  return pl;
}

// ---------------------------------------------------------------------------
// Build kernels (FP64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 arena(const float2* hi, const float2* lo, int64_t i) {
  const float2 h = hi[i], l = lo[i];
  return make_double2(double(h.x) + double(l.x), double(h.y) + double(l.y));
}

// Mc[k + c n] = delta(k, E[c0 + c]) - M_i[k, E[c0 + c]]  for c < w  (n x w, column-major)
__global__ void k_pc_mcols(const float2* hi, const float2* lo, int64_t off, int n, int ld, const int32_t* Eloc, int c0,
                           int w, double2* Mc) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(n) * w) return;
  const int k = int(i % n), c = int(i / n);
  const int q = Eloc[c0 + c];
  const double2 m = arena(hi, lo, off + int64_t(n + k) * ld + q);
  Mc[i] = make_double2((k == q ? 1.0 : 0.0) - m.x, -m.y);
}

struct FillArgs {
  const double2* W; int64_t E;          // L_A[E,:] (I - M)[:,E], E x E column-major
  const double2* LP; int64_t R;         // L_phi rows (R x t), column-major
  const int32_t* Eloc; const int32_t* Tloc; const int32_t* trow;
  int64_t T;
  const float2* hi; const float2* lo; int64_t off; int n, ld;
  int e0, t0;
  const int32_t* ixc; const double* ixv;
  const int32_t* tplus; const int32_t* tminus; const int32_t* tri_edge; const int8_t* tri_sign;
  const double* len; const double* area;
  double k0, inv_eta0, s1, s2;
  double2* B;                           // s x s column-major
};

__global__ void k_pc_fill(FillArgs a) {
  const int64_t s = a.E + a.T;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= s * s) return;
  const int64_t r = i % s, c = i / s;
  double2 v = make_double2(0.0, 0.0);
  if (r < a.E && c < a.E) {
    // (j k0 L_A (I - M) + I_x Z / eta0) / h^2
    const int m = a.Eloc[r], q = a.Eloc[c];
    const double2 w = a.W[r + c * a.E];
    double vr = -a.k0 * w.y, vi = a.k0 * w.x;
    for (int k = 0; k < 4; ++k) {
      const int col = a.ixc[4 * (a.e0 + m) + k];
      if (col < 0) continue;
      const double2 z = arena(a.hi, a.lo, a.off + int64_t(col - a.e0) * a.ld + q);
      const double x = a.ixv[4 * (a.e0 + m) + k] * a.inv_eta0;
      vr += x * z.x;
      vi += x * z.y;
    }
    v = make_double2(vr * a.s1, vi * a.s1);
  } else if (r < a.E) {
    // D^T L_phi B / h^2: l_m (L_phi[T+(m), u] - L_phi[T-(m), u]) A_u
    const int mg = a.e0 + a.Eloc[r];
    const int u = a.Tloc[c - a.E];
    const int rp = a.trow[a.tplus[mg] - a.t0], rm = a.trow[a.tminus[mg] - a.t0];
    const double2 lp = a.LP[rp + int64_t(u) * a.R], lm = a.LP[rm + int64_t(u) * a.R];
    const double f = a.len[mg] * a.area[a.t0 + u] * a.s1;
    v = make_double2(f * (lp.x - lm.x), f * (lp.y - lm.y));
  } else if (c < a.E) {
    // h F D (I - M): -(h / A_t) sum over the triangle's edges of s l (delta - M)
    const int tg = a.t0 + a.Tloc[r - a.E];
    const int q = a.Eloc[c];
    double vr = 0.0, vi = 0.0;
    for (int k = 0; k < 3; ++k) {
      const int eg = a.tri_edge[3 * tg + k];
      const int el = eg - a.e0;
      const double d = double(a.tri_sign[3 * tg + k]) * a.len[eg];
      const double2 m = arena(a.hi, a.lo, a.off + int64_t(a.n + el) * a.ld + q);
      vr += d * ((el == q ? 1.0 : 0.0) - m.x);
      vi += d * (-m.y);
    }
    const double f = -a.s2 / a.area[tg];
    v = make_double2(f * vr, f * vi);
  } else if (r == c) {
    v = make_double2(0.0, a.k0 * a.s2);   // h j k0
  }
  a.B[i] = v;
}

// max over columns of the column sums of |B| (s x s, column-major): one workgroup per column
__global__ void k_pc_colsum(const double2* B, int64_t s, double* out) {
  const int64_t c = blockIdx.x;
  double acc = 0.0;
  for (int64_t r = threadIdx.x; r < s; r += blockDim.x) {
    const double2 v = B[r + c * s];
    acc += sqrt(v.x * v.x + v.y * v.y);
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

// Green's function over a box of integer grid offsets [lo, lo + D) per axis (G(0) = 0)
__global__ void k_pc_gtab(double2* T, int lx, int ly, int lz, int Dx, int Dy, int Dz, double hx, double hy, double hz,
                          double k0) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(Dx) * Dy * Dz) return;
  const int x = int(i % Dx) + lx, y = int((i / Dx) % Dy) + ly, z = int(i / (int64_t(Dx) * Dy)) + lz;
  const double dx = x * hx, dy = y * hy, dz = z * hz;
  const double R = sqrt(dx * dx + dy * dy + dz * dz);
  double2 v = make_double2(0.0, 0.0);
  if (R > 0.0) {
    double sn, cs;
    sincos(k0 * R, &sn, &cs);
    v = make_double2(cs / (4.0 * 3.14159265358979323846 * R), -sn / (4.0 * 3.14159265358979323846 * R));
  }
  T[i] = v;
}

// The AIM operator applies L exactly only on near pairs (stencil centres within
// Chebyshev distance near_cheb) and through the grid elsewhere: replace every
// far entry of the assembled exact rows by its grid value
//   sum_c sum_a sum_b w_c[m, a] G(node_a(m) - node_b(n)) w_c[n, b],
// so that the block is the self part of the operator that is being solved.
struct FarArgs {
  double2* L; int64_t ld; int64_t rows, cols;   // column-major rows x cols
  const int32_t* row_local;                     // row -> local basis index
  int base;                                     // global index of local basis 0
  const int32_t* cidx; const double* w; int ncomp, near_cheb;
  const double2* gtab; int lx, ly, lz, Dx, Dy;
};

__global__ void k_pc_far_grid(FarArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.rows * a.cols) return;
  const int64_t r = i % a.rows, col = i / a.rows;
  const int m = a.base + a.row_local[r], n = a.base + int(col);
  const int dx = a.cidx[3 * m] - a.cidx[3 * n], dy = a.cidx[3 * m + 1] - a.cidx[3 * n + 1],
            dz = a.cidx[3 * m + 2] - a.cidx[3 * n + 2];
  if (max(abs(dx), max(abs(dy), abs(dz))) <= a.near_cheb) return;
  const double* wm = a.w + int64_t(m) * 27 * a.ncomp;
  const double* wn = a.w + int64_t(n) * 27 * a.ncomp;
  double sr = 0.0, si = 0.0;
  for (int p = 0; p < 27; ++p) {
    const int px = p % 3 - 1, py = (p / 3) % 3 - 1, pz = p / 9 - 1;
    double tr[3] = {0, 0, 0}, ti[3] = {0, 0, 0};
    for (int q = 0; q < 27; ++q) {
      const int qx = q % 3 - 1, qy = (q / 3) % 3 - 1, qz = q / 9 - 1;
      const int ox = dx + px - qx - a.lx, oy = dy + py - qy - a.ly, oz = dz + pz - qz - a.lz;
      const double2 G = a.gtab[(int64_t(oz) * a.Dy + oy) * a.Dx + ox];
      for (int c = 0; c < a.ncomp; ++c) {
        const double wv = wn[c * 27 + q];
        tr[c] += G.x * wv;
        ti[c] += G.y * wv;
      }
    }
    for (int c = 0; c < a.ncomp; ++c) {
      sr += wm[c * 27 + p] * tr[c];
      si += wm[c * 27 + p] * ti[c];
    }
  }
  a.L[r + col * a.ld] = make_double2(sr, si);
}

// columns [c0, c0 + w) of the s x s identity (column-major s x w)
__global__ void k_pc_eye(double2* X, int64_t s, int64_t c0, int64_t w) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= s * w) return;
  X[i] = make_double2((i % s) == c0 + (i / s) ? 1.0 : 0.0, 0.0);
}

// own rows of columns [c0, c0 + w) of the inverse (column-major s x w panel) ->
// complex64 rows of length ld >= s; the padding column(s) past s are zeroed by the
// last panel
__global__ void k_pc_pack(const double2* X, int64_t s, int64_t c0, int64_t w, const int32_t* own_pos, int n_own, int ld,
                          float2* out) {
  const int64_t wp = (c0 + w == s) ? w + (ld - s) : w;   // columns written by this panel
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(n_own) * wp) return;
  const int r = int(i / wp);
  const int64_t c = i % wp;
  float2 v = make_float2(0.f, 0.f);
  if (c < w) {
    const double2 x = X[own_pos[r] + c * s];
    v = make_float2(float(x.x), float(x.y));
  }
  out[int64_t(r) * ld + c0 + c] = v;
}

// ---------------------------------------------------------------------------
// Apply kernels
// ---------------------------------------------------------------------------
__global__ void k_pc_gather(const double2* __restrict__ v, const int32_t* __restrict__ ext, int64_t n, float2* __restrict__ vin) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const double2 x = v[ext[q]];
  vin[q] = make_float2(float(x.x), float(x.y));
}

__device__ __forceinline__ float wsum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

typedef float f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ntl(const float2* p) {
  const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

// Persistent block GEMV: each workgroup walks its queue of (block, row0, rows)
// tiles; each wave sweeps 8 rows, lanes stride two 128-column chunks.
__global__ void __launch_bounds__(256) k_pc_gemv(const float2* __restrict__ P, const PcBlk* __restrict__ blks,
                                                 const int4* __restrict__ tiles, const int32_t* __restrict__ slot_start,
                                                 const float2* __restrict__ vin, const int32_t* __restrict__ rowidx,
                                                 double2* __restrict__ z) {
  constexpr int RW = 8;
  const int slot = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int ti = slot_start[slot]; ti < slot_start[slot + 1]; ++ti) {
    const int4 tl = tiles[ti];
    const PcBlk B = blks[tl.x];
    const int ns = B.n_ext, ld = B.ld;
    const float2* vs = vin + B.ext_off;
    const int rend = tl.y + tl.z;
    for (int r0 = tl.y + RW * wave; r0 < rend; r0 += 4 * RW) {
      float ar[RW], ai[RW];
#pragma unroll
      for (int q = 0; q < RW; ++q) { ar[q] = 0.f; ai[q] = 0.f; }
      const int nr = min(RW, rend - r0);
      const int64_t base = B.off + int64_t(r0) * ld;
      for (int col = 2 * lane; col < ld; col += 256) {
        const int col2 = col + 128;
        float2 h0 = make_float2(0.f, 0.f), h1 = h0, h2 = h0, h3 = h0;
        if (col < ns) h0 = vs[col];
        if (col + 1 < ns) h1 = vs[col + 1];
        if (col2 < ns) h2 = vs[col2];
        if (col2 + 1 < ns) h3 = vs[col2 + 1];
        float4 a[RW], b[RW];
#pragma unroll
        for (int q = 0; q < RW; ++q) {
          a[q] = make_float4(0.f, 0.f, 0.f, 0.f);
          b[q] = make_float4(0.f, 0.f, 0.f, 0.f);
          if (q < nr) {
            a[q] = ntl(P + base + int64_t(q) * ld + col);
            if (col2 < ld) b[q] = ntl(P + base + int64_t(q) * ld + col2);
          }
        }
#pragma unroll
        for (int q = 0; q < RW; ++q) {
          ar[q] += a[q].x * h0.x - a[q].y * h0.y + a[q].z * h1.x - a[q].w * h1.y + b[q].x * h2.x - b[q].y * h2.y +
                   b[q].z * h3.x - b[q].w * h3.y;
          ai[q] += a[q].x * h0.y + a[q].y * h0.x + a[q].z * h1.y + a[q].w * h1.x + b[q].x * h2.y + b[q].y * h2.x +
                   b[q].z * h3.y + b[q].w * h3.x;
        }
      }
#pragma unroll
      for (int q = 0; q < RW; ++q) {
        const float sr = wsum(ar[q]), si = wsum(ai[q]);
        if (lane == 0 && q < nr) z[rowidx[B.row_off + r0 + q]] = make_double2(double(sr), double(si));
      }
    }
  }
}

// LPT packing of the row panels of the stored blocks over the slots.
void pc_pack_tiles(Ctx& c, int S) {
  struct Task { int block, row0, rows; double cost; };
  std::vector<Task> tasks;
  double total = 0.0;
  for (const PcBlk& b : c.pc_blocks) total += double(b.n_own) * b.ld;
  const double ideal = std::max(1.0, total / S);
  for (int i = 0; i < int(c.pc_blocks.size()); ++i) {
    const PcBlk& b = c.pc_blocks[i];
    const double w = double(b.n_own) * b.ld;
    const int64_t P = std::max<int64_t>(1, int64_t(std::ceil(w / (0.25 * ideal))));
    int R = int(std::min<int64_t>(b.n_own, std::max<int64_t>(8, (b.n_own + P - 1) / P)));
    R = std::min(b.n_own, ((R + 7) / 8) * 8);
    for (int r0 = 0; r0 < b.n_own; r0 += R) {
      const int rr = std::min(R, b.n_own - r0);
      tasks.push_back({i, r0, rr, double((rr + 7) / 8 * 8) * double((b.ld + 255) / 256 * 256)});
    }
  }
  std::vector<int> order(tasks.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return tasks[a].cost > tasks[b].cost; });
  using E = std::pair<double, int>;
  std::priority_queue<E, std::vector<E>, std::greater<E>> pq;
  for (int s = 0; s < S; ++s) pq.push({0.0, s});
  std::vector<std::vector<int32_t>> q(S);
  for (int k : order) {
    E e = pq.top();
    pq.pop();
    q[e.second].push_back(k);
    pq.push({e.first + tasks[k].cost, e.second});
  }
  std::vector<int32_t> flat, start(S + 1, 0);
  for (int s = 0; s < S; ++s) {
    start[s + 1] = start[s] + int32_t(q[s].size());
    for (int k : q[s]) {
      flat.push_back(tasks[k].block);
      flat.push_back(tasks[k].row0);
      flat.push_back(tasks[k].rows);
      flat.push_back(s);
    }
  }
  c.d_pc_tiles.upload(flat);
  c.d_pc_slot_start.upload(start);
  c.pc_slots = S;
}

}  // namespace

void build_precond(Ctx& c, hipStream_t s) {
  const slim_build_opts& o = c.opts;
  const RWGTable& r = c.rwg;
  c.pc_built = false;
  c.pc_blocks.clear();
  c.pc_ext.clear();
  c.pc_own_ptr.clear();
  c.pc_ext_ptr.clear();
  c.pc_own_pos.clear();
  c.d_pc.release();
  if (!o.precond) return;
  const int overlap = std::max(0, o.precond_overlap);
  Partitioner P(r);
  size_t budget = size_t(std::max<int64_t>(0, o.precond_budget));
  if (budget == 0) {
    size_t freeb = 0, totalb = 0;
    SLIM_HIP(hipMemGetInfo(&freeb, &totalb));
    const size_t reserve = size_t(2) * 101 * size_t(r.n_e + r.n_t) * 16 + (size_t(1) << 30);
    budget = freeb > reserve ? freeb - reserve : 0;
  }
  Plan plan;
  if (o.precond_cap > 0) {
    plan = make_plan(P, r, o.precond_cap, overlap);
    SLIM_REQUIRE(plan.bytes() <= budget, SLIM_E_OOM,
                 "conductor-block preconditioner with cap " + std::to_string(o.precond_cap) + " needs " +
                     std::to_string(plan.bytes()) + " bytes, budget " + std::to_string(budget));
  } else {
    bool found = false;
    // the largest cap whose plan fits, on a ladder with steps of 1/8 to 1/4 (a small
    // change of free memory moves the cap by one short step)
    for (int64_t cap : {int64_t(0), int64_t(65536), int64_t(49152), int64_t(40960), int64_t(32768), int64_t(28672),
                        int64_t(24576), int64_t(20480), int64_t(18432), int64_t(16384), int64_t(14336), int64_t(12288),
                        int64_t(10240), int64_t(8192), int64_t(6144), int64_t(4096), int64_t(3072), int64_t(2048),
                        int64_t(1536), int64_t(1024), int64_t(768), int64_t(512)}) {
      Plan pl = make_plan(P, r, cap, overlap);
      if (o.verbose) {
        std::fprintf(stderr, "[slim build] preconditioner cap %lld: %zu blocks, %.2f GB (budget %.2f GB)\n",
                     (long long)cap, pl.parts.size(), pl.bytes() / 1e9, budget / 1e9);
        std::fflush(stderr);
      }
      if (pl.bytes() <= budget) { plan = std::move(pl); found = true; break; }
    }
    SLIM_REQUIRE(found, SLIM_E_OOM, "no conductor-block preconditioner fits the device memory budget");
  }
  auto t_start = std::chrono::steady_clock::now();

  // ---- host tables ----
  std::vector<int32_t> rowidx;
  c.pc_ext_ptr.assign(1, 0);
  c.pc_own_ptr.assign(1, 0);
  int64_t off = 0;
  for (const Part& q : plan.parts) {
    PcBlk b;
    b.off = off;
    b.ext_off = int64_t(c.pc_ext.size());
    b.row_off = int64_t(rowidx.size());
    b.n_ext = int32_t(q.ext_e.size() + q.ext_t.size());
    b.ld = (b.n_ext + 1) & ~1;
    b.n_own = int32_t(q.own_pos.size());
    for (int32_t e : q.ext_e) c.pc_ext.push_back(e);
    for (int32_t t : q.ext_t) c.pc_ext.push_back(int32_t(r.n_e + t));
    for (int32_t p : q.own_pos) {
      c.pc_own_pos.push_back(p);
      rowidx.push_back(c.pc_ext[size_t(b.ext_off + p)]);
    }
    c.pc_ext_ptr.push_back(int64_t(c.pc_ext.size()));
    c.pc_own_ptr.push_back(int64_t(c.pc_own_pos.size()));
    off += int64_t(b.n_own) * b.ld;
    c.pc_blocks.push_back(b);
  }
  c.pc_cap = plan.cap;
  c.pc_entries = off;

  // ---- device arrays ----
  c.d_pc.alloc(size_t(off) * 8);
  c.d_pc_ext.upload(c.pc_ext);
  c.d_pc_row.upload(rowidx);
  c.d_pc_blk.upload(c.pc_blocks);
  c.d_pc_vin.alloc(std::max<size_t>(1, c.pc_ext.size()) * 8);
  DevBuf la, lp, mc, w, B, X, ipiv, emap, tmap, dE, dT, dpos, dpairs, info, colsum;
  colsum.alloc(std::max<size_t>(8, plan.t_ipiv * 2 + 8));
  c.pc_cond.clear();
  la.alloc(std::max<size_t>(16, plan.t_la));
  lp.alloc(std::max<size_t>(16, plan.t_lp));
  mc.alloc(std::max<size_t>(16, plan.t_mc));
  w.alloc(std::max<size_t>(16, plan.t_w));
  B.alloc(std::max<size_t>(16, plan.t_b));
  X.alloc(std::max<size_t>(16, plan.t_x));
  ipiv.alloc(std::max<size_t>(16, plan.t_ipiv));
  info.alloc(sizeof(rocblas_int) * std::max<size_t>(1, plan.parts.size()));
  SLIM_HIP(hipMemsetAsync(info.p, 0, info.bytes, s));
  rocblas_handle h = nullptr;
  SLIM_REQUIRE(rocblas_create_handle(&h) == rocblas_status_success, SLIM_E_HIP, "rocblas_create_handle failed");
  struct HandleGuard { rocblas_handle h; ~HandleGuard() { rocblas_destroy_handle(h); } } hg{h};
  rocblas_set_stream(h, s);

  AsmLaunch L{};
  L.xyz = c.d_xyz.as<double>(); L.tri = c.d_tri.as<int32_t>(); L.cen = c.d_cen.as<double>();
  L.nrm = c.d_nrm.as<double>(); L.area = c.d_area.as<double>(); L.diam = c.d_diam.as<double>();
  L.tri_edge = c.d_tri_edge.as<int32_t>(); L.tri_sign = c.d_tri_sign.as<int8_t>(); L.len = c.d_len.as<double>();
  L.k = cd(c.k0, 0.0);
  L.skip_mag = 0.0;
  const double hmean = r.mean_edge;
  int32_t pairs_obj = -1;
  std::vector<int32_t> pairs;
  // AIM consistency: stencil centres on the device and a per-conductor Green's function table
  DevBuf d_cidx_e, d_cidx_t, gtab, dR;
  int32_t gtab_obj = -1;
  int gl[3] = {0, 0, 0}, gD[3] = {1, 1, 1};
  if (!c.plain) {
    d_cidx_e.upload(c.h_cidx_e);
    d_cidx_t.upload(c.h_cidx_t);
  }
  for (size_t bi = 0; bi < plan.parts.size(); ++bi) {
    const Part& q = plan.parts[bi];
    const PcBlk& pb = c.pc_blocks[bi];
    const int i = q.obj;
    const Block& ob = c.blocks[size_t(i)];
    const int n = ob.n, ld = (n + 1) & ~1;
    const int64_t t0 = r.obj_tri_off[i], nt = r.obj_tri_off[i + 1] - t0;
    const int64_t E = int64_t(q.ext_e.size()), T = int64_t(q.ext_t.size()), S = E + T;
    // element-wise kernels over S x S and n x E use one work-item per entry (< 2^32 per dispatch)
    SLIM_REQUIRE(S * S < (int64_t(1) << 32) && int64_t(n) * E < (int64_t(1) << 32), SLIM_E_UNSUPPORTED,
                 "preconditioner block of " + std::to_string(S) + " unknowns is too large (cap it with precond_cap)");
    // local index lists and row maps
    std::vector<int32_t> Eloc(static_cast<size_t>(E)), Tloc(static_cast<size_t>(T));
    std::vector<int32_t> em(static_cast<size_t>(n), -1), tm(static_cast<size_t>(nt), -1);
    for (int64_t k = 0; k < E; ++k) { Eloc[size_t(k)] = q.ext_e[size_t(k)] - ob.e0; em[size_t(Eloc[size_t(k)])] = int32_t(k); }
    for (int64_t k = 0; k < T; ++k) Tloc[size_t(k)] = int32_t(q.ext_t[size_t(k)] - t0);
    std::vector<int32_t> R;
    for (int32_t e : q.ext_e) { R.push_back(int32_t(r.tplus[size_t(e)] - t0)); R.push_back(int32_t(r.tminus[size_t(e)] - t0)); }
    std::sort(R.begin(), R.end());
    R.erase(std::unique(R.begin(), R.end()), R.end());
    for (size_t k = 0; k < R.size(); ++k) tm[size_t(R[k])] = int32_t(k);
    const int64_t nR = int64_t(R.size());
    dE.upload(Eloc); dT.upload(Tloc); emap.upload(em); tmap.upload(tm);
    std::vector<int32_t> pos(c.pc_own_pos.begin() + c.pc_own_ptr[bi], c.pc_own_pos.begin() + c.pc_own_ptr[bi + 1]);
    dpos.upload(pos);
    if (pairs_obj != i) {
      pairs = near_candidates(r, t0, t0 + nt, o.c_near);
      dpairs.upload(pairs);
      pairs_obj = i;
    }
    // L_A rows of the extended edges and L_phi rows of their triangles (self interactions at k0)
    SLIM_HIP(hipMemsetAsync(la.p, 0, size_t(E) * n * 16, s));
    SLIM_HIP(hipMemsetAsync(lp.p, 0, size_t(nR) * nt * 16, s));
    L.t0 = int32_t(t0); L.t1 = int32_t(t0 + nt); L.e0 = ob.e0;
    L.Lk = nullptr; L.Kk = nullptr;
    L.Lvec = la.as<double>(); L.Lphi = lp.as<double>();
    L.ld_e = E; L.ld_t = nR;
    L.erow = emap.as<int32_t>(); L.trow = tmap.as<int32_t>();
    L.near_pairs = dpairs.as<int32_t>();
    L.n_near_pairs = int64_t(pairs.size() / 2);
    launch_assemble(L, s);
    if (!c.plain) {
      // the conductor's far pairs as the AIM operator represents them (grid part only)
      if (gtab_obj != i) {
        int lo3[3], hi3[3];
        for (int k = 0; k < 3; ++k) { lo3[k] = 1 << 30; hi3[k] = -(1 << 30); }
        auto span = [&](const std::vector<int32_t>& cidx, int64_t b0, int64_t b1) {
          for (int64_t q2 = b0; q2 < b1; ++q2)
            for (int k = 0; k < 3; ++k) {
              lo3[k] = std::min(lo3[k], cidx[3 * size_t(q2) + k]);
              hi3[k] = std::max(hi3[k], cidx[3 * size_t(q2) + k]);
            }
        };
        span(c.h_cidx_e, ob.e0, ob.e0 + n);
        span(c.h_cidx_t, t0, t0 + nt);
        for (int k = 0; k < 3; ++k) { gl[k] = -(hi3[k] - lo3[k]) - 2; gD[k] = 2 * (hi3[k] - lo3[k]) + 5; }
        const int64_t ntab = int64_t(gD[0]) * gD[1] * gD[2];
        if (size_t(ntab) * 16 > gtab.bytes) gtab.alloc(size_t(ntab) * 16);
        hipLaunchKernelGGL(k_pc_gtab, dim3(nb256(ntab)), dim3(256), 0, s, gtab.as<double2>(), gl[0], gl[1], gl[2], gD[0],
                           gD[1], gD[2], c.grid.h[0], c.grid.h[1], c.grid.h[2], c.k0);
        SLIM_HIP(hipGetLastError());
        gtab_obj = i;
      }
      FarArgs fa2{};
      fa2.gtab = gtab.as<double2>();
      fa2.lx = gl[0]; fa2.ly = gl[1]; fa2.lz = gl[2]; fa2.Dx = gD[0]; fa2.Dy = gD[1];
      fa2.near_cheb = c.near_cheb;
      if (E > 0) {
        fa2.L = la.as<double2>(); fa2.ld = E; fa2.rows = E; fa2.cols = n;
        fa2.row_local = dE.as<int32_t>(); fa2.base = ob.e0;
        fa2.cidx = d_cidx_e.as<int32_t>(); fa2.w = c.d_we_w64.as<double>(); fa2.ncomp = 3;
        hipLaunchKernelGGL(k_pc_far_grid, dim3(nb256(E * n)), dim3(256), 0, s, fa2);
        SLIM_HIP(hipGetLastError());
      }
      if (nR > 0) {
        dR.upload(R);
        fa2.L = lp.as<double2>(); fa2.ld = nR; fa2.rows = nR; fa2.cols = nt;
        fa2.row_local = dR.as<int32_t>(); fa2.base = int(t0);
        fa2.cidx = d_cidx_t.as<int32_t>(); fa2.w = c.d_wt_w64.as<double>(); fa2.ncomp = 1;
        hipLaunchKernelGGL(k_pc_far_grid, dim3(nb256(nR * nt)), dim3(256), 0, s, fa2);
        SLIM_HIP(hipGetLastError());
      }
    }
    // W = L_A[E,:] (I - M)[:, E]  (a part may own triangles only)
    for (int64_t c0 = 0; c0 < E; c0 += kPanel) {
      const int64_t wdt = std::min(kPanel, E - c0);
      hipLaunchKernelGGL(k_pc_mcols, dim3(nb256(int64_t(n) * wdt)), dim3(256), 0, s, c.d_hi.as<float2>(),
                         c.d_lo.as<float2>(), ob.off, n, ld, dE.as<int32_t>(), int(c0), int(wdt), mc.as<double2>());
      SLIM_HIP(hipGetLastError());
      rocblas_double_complex one{1.0, 0.0}, zero{0.0, 0.0};
      SLIM_ROCP(rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, int(E), int(wdt), n, &one,
                              la.as<rocblas_double_complex>(), int(E), mc.as<rocblas_double_complex>(), n, &zero,
                              w.as<rocblas_double_complex>() + c0 * E, int(E)));
    }
    FillArgs fa{};
    fa.W = w.as<double2>(); fa.E = E;
    fa.LP = lp.as<double2>(); fa.R = nR;
    fa.Eloc = dE.as<int32_t>(); fa.Tloc = dT.as<int32_t>(); fa.trow = tmap.as<int32_t>(); fa.T = T;
    fa.hi = c.d_hi.as<float2>(); fa.lo = c.d_lo.as<float2>(); fa.off = ob.off; fa.n = n; fa.ld = ld;
    fa.e0 = ob.e0; fa.t0 = int(t0);
    fa.ixc = c.d_ix_col.as<int32_t>(); fa.ixv = c.d_ix_val.as<double>();
    fa.tplus = c.d_tplus.as<int32_t>(); fa.tminus = c.d_tminus.as<int32_t>();
    fa.tri_edge = c.d_tri_edge.as<int32_t>(); fa.tri_sign = c.d_tri_sign.as<int8_t>();
    fa.len = c.d_len.as<double>(); fa.area = c.d_area.as<double>();
    fa.k0 = c.k0; fa.inv_eta0 = 1.0 / eta0(); fa.s1 = 1.0 / (hmean * hmean); fa.s2 = hmean;
    fa.B = B.as<double2>();
    hipLaunchKernelGGL(k_pc_fill, dim3(nb256(S * S)), dim3(256), 0, s, fa);
    SLIM_HIP(hipGetLastError());
    // 1-norm of the block (for its condition estimate)
    hipLaunchKernelGGL(k_pc_colsum, dim3(unsigned(S)), dim3(256), 0, s, B.as<double2>(), S, colsum.as<double>());
    SLIM_HIP(hipGetLastError());
    std::vector<double> cs(static_cast<size_t>(S));
    SLIM_HIP(hipMemcpyAsync(cs.data(), colsum.p, size_t(S) * 8, hipMemcpyDeviceToHost, s));
    SLIM_HIP(hipStreamSynchronize(s));
    const double nb1 = *std::max_element(cs.begin(), cs.end());
    // FP64 LU and inverse of the block; keep the owned rows in complex64
    SLIM_ROCP(rocsolver_zgetrf(h, int(S), int(S), B.as<rocblas_double_complex>(), int(S), ipiv.as<rocblas_int>(),
                               info.as<rocblas_int>() + bi));
    double nx1 = 0.0;
    for (int64_t c0 = 0; c0 < S; c0 += kPanel) {
      const int64_t wdt = std::min(kPanel, S - c0);
      hipLaunchKernelGGL(k_pc_eye, dim3(nb256(S * wdt)), dim3(256), 0, s, X.as<double2>(), S, c0, wdt);
      SLIM_HIP(hipGetLastError());
      lu_solve_rhs(h, int(S), B.as<double>(), ipiv.as<rocblas_int>(), X.as<double>(), int(wdt), s);
      hipLaunchKernelGGL(k_pc_colsum, dim3(unsigned(wdt)), dim3(256), 0, s, X.as<double2>(), S, colsum.as<double>());
      SLIM_HIP(hipGetLastError());
      const int64_t wp = (c0 + wdt == S) ? wdt + (pb.ld - S) : wdt;
      hipLaunchKernelGGL(k_pc_pack, dim3(nb256(int64_t(pb.n_own) * wp)), dim3(256), 0, s, X.as<double2>(), S, c0,
                         wdt, dpos.as<int32_t>(), pb.n_own, pb.ld, c.d_pc.as<float2>() + pb.off);
      SLIM_HIP(hipGetLastError());
      SLIM_HIP(hipMemcpyAsync(cs.data(), colsum.p, size_t(wdt) * 8, hipMemcpyDeviceToHost, s));
      SLIM_HIP(hipStreamSynchronize(s));
      nx1 = std::max(nx1, *std::max_element(cs.begin(), cs.begin() + wdt));
    }
    c.pc_cond.push_back(nb1 * nx1);
    SLIM_HIP(hipStreamSynchronize(s));   // the index buffers are reused by the next block
    if (o.verbose) {
      static thread_local auto last = std::chrono::steady_clock::now();
      auto now = std::chrono::steady_clock::now();
      if (bi + 1 == plan.parts.size() || std::chrono::duration<double>(now - last).count() > 10.0) {
        std::fprintf(stderr, "[slim build] preconditioner blocks %zu / %zu (size %lld)\n", bi + 1, plan.parts.size(),
                     (long long)S);
        std::fflush(stderr);
        last = now;
      }
    }
  }
  std::vector<rocblas_int> h_info(plan.parts.size());
  if (!h_info.empty())
    SLIM_HIP(hipMemcpy(h_info.data(), info.p, h_info.size() * sizeof(rocblas_int), hipMemcpyDeviceToHost));
  for (size_t k = 0; k < h_info.size(); ++k)
    SLIM_REQUIRE(h_info[k] == 0, SLIM_E_NUMERIC, "singular preconditioner block " + std::to_string(k));
  if (o.verbose && !c.pc_cond.empty()) {
    std::vector<size_t> idx(c.pc_cond.size());
    std::iota(idx.begin(), idx.end(), size_t(0));
    std::sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return c.pc_cond[a] > c.pc_cond[b]; });
    int over = 0;
    for (double k : c.pc_cond) over += k * 0x1p-24 > 0.1;
    std::fprintf(stderr, "[slim build] preconditioner blocks with cond_1 * 2^-24 > 0.1: %d of %zu; largest:", over,
                 c.pc_cond.size());
    for (size_t k = 0; k < std::min<size_t>(8, idx.size()); ++k)
      std::fprintf(stderr, " %.2e (size %d)", c.pc_cond[idx[k]], c.pc_blocks[idx[k]].n_ext);
    std::fprintf(stderr, "\n");
    std::fflush(stderr);
  }
  pc_pack_tiles(c, c.slots > 0 ? c.slots : 1024);
  c.pc_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  c.pc_built = true;
}

void precond_partition(const RWGTable& r, int64_t cap, int overlap, std::vector<int64_t>& ext_ptr,
                       std::vector<int32_t>& ext_idx, std::vector<int64_t>& own_ptr, std::vector<int32_t>& own_pos) {
  Partitioner P(r);
  const std::vector<Part> parts = P.partition(cap, std::max(0, overlap));
  ext_ptr.assign(1, 0);
  own_ptr.assign(1, 0);
  ext_idx.clear();
  own_pos.clear();
  for (const Part& q : parts) {
    for (int32_t e : q.ext_e) ext_idx.push_back(e);
    for (int32_t t : q.ext_t) ext_idx.push_back(int32_t(r.n_e + t));
    own_pos.insert(own_pos.end(), q.own_pos.begin(), q.own_pos.end());
    ext_ptr.push_back(int64_t(ext_idx.size()));
    own_ptr.push_back(int64_t(own_pos.size()));
  }
}

void precond_apply(Ctx& c, const void* v, void* z, hipStream_t s) {
  SLIM_REQUIRE(c.pc_built, SLIM_E_STATE, "no preconditioner was built (build option precond = 0)");
  const int64_t n = int64_t(c.pc_ext.size());
  hipLaunchKernelGGL(k_pc_gather, dim3(nb256(n)), dim3(256), 0, s, reinterpret_cast<const double2*>(v),
                     c.d_pc_ext.as<int32_t>(), n, c.d_pc_vin.as<float2>());
  hipLaunchKernelGGL(k_pc_gemv, dim3(unsigned(c.pc_slots)), dim3(256), 0, s, c.d_pc.as<float2>(),
                     c.d_pc_blk.as<PcBlk>(), c.d_pc_tiles.as<int4>(), c.d_pc_slot_start.as<int32_t>(),
                     c.d_pc_vin.as<float2>(), c.d_pc_row.as<int32_t>(), reinterpret_cast<double2*>(z));
  SLIM_HIP(hipGetLastError());
}

}  // namespace slim
