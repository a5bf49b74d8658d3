// GMRES on the SLIM system (7) (Sec. III-E uses GMRES [Saad1986]) and its
// mixed-precision iterative refinement.
//
// The system is solved in the row-equilibrated form S A x = S b with
// S = diag(1/h^2 on the tested-EFIE rows, h on the continuity rows), h the mean
// edge length: this is the change of length unit to h, which balances the two
// row blocks (in SI units they differ by about h^3).  Optionally right-
// preconditioned by the conductor blocks (precond.hip).  Those are applied in
// complex64, so the cycle is flexible GMRES [Saad1993]: the preconditioned
// vectors z_k = P^{-1} v_k are kept and the update is d = sum_k y_k z_k.
//   FP64: restarted (F)GMRES(m), classical Gram-Schmidt applied twice (CGS2),
//         Givens rotations, FP64 true residual at every restart.
//   MIXED: GMRES-IR -- outer residual r = S (b - A x) with the FP64 operator;
//         inner (F)GMRES(m) with the mixed-precision operator on S A d = r
//         (FP64 Krylov basis and orthogonalisation); x += d.
#include <chrono>
#include <cstdio>

#include "ctx.hpp"

namespace slim {

namespace {

unsigned nblk(int64_t n, int t = 256) { return unsigned((n + t - 1) / t); }
constexpr int kDotBlocks = 1024;

// partial[b][i] = sum over the block's chunk of conj(V_i) w,  i < nv
__global__ void __launch_bounds__(256) k_multidot(const double2* V, int64_t ldv, int nv, const double2* w, int64_t n,
                                                  double2* partial) {
  __shared__ double sr[256], si[256];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  for (int i = 0; i < nv; ++i) {
    double ar = 0.0, ai = 0.0;
    const double2* v = V + i * ldv;
    for (int64_t k = lo + threadIdx.x; k < hi; k += 256) {
      const double2 a = v[k], b = w[k];
      ar += a.x * b.x + a.y * b.y;
      ai += a.x * b.y - a.y * b.x;
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        sr[threadIdx.x] += sr[threadIdx.x + s];
        si[threadIdx.x] += si[threadIdx.x + s];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[int64_t(blockIdx.x) * nv + i] = make_double2(sr[0], si[0]);
    __syncthreads();
  }
}

// out[i] = sum_b partial[b][i] in a fixed order
__global__ void k_reduce_partial(const double2* partial, int nb, int nv, double2* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  double r = 0.0, im = 0.0;
  for (int b = 0; b < nb; ++b) {
    r += partial[int64_t(b) * nv + i].x;
    im += partial[int64_t(b) * nv + i].y;
  }
  out[i] = make_double2(r, im);
}

// w -= sum_i V_i h_i
__global__ void k_multiaxpy(const double2* V, int64_t ldv, int nv, const double2* h, double2* w, int64_t n) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double2 acc = w[k];
  for (int i = 0; i < nv; ++i) {
    const double2 v = V[i * ldv + k], c = h[i];
    acc.x -= v.x * c.x - v.y * c.y;
    acc.y -= v.x * c.y + v.y * c.x;
  }
  w[k] = acc;
}

// out = s .* (b - y)  (s: n_e values 1/h^2, then h); b may be already scaled (bs = 1)
__global__ void k_scaled_residual(const double2* b, const double2* y, double2* out, int64_t ne, int64_t n, double s1,
                                  double s2, int bs) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double s = k < ne ? s1 : s2;
  const double bf = bs ? 1.0 : s;
  out[k] = make_double2(bf * b[k].x - s * y[k].x, bf * b[k].y - s * y[k].y);
}

__global__ void k_scale_rows(double2* v, int64_t ne, int64_t n, double s1, double s2) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double s = k < ne ? s1 : s2;
  v[k].x *= s;
  v[k].y *= s;
}

__global__ void k_cscale(const double2* in, double2* out, int64_t n, double f) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < n) out[k] = make_double2(in[k].x * f, in[k].y * f);
}

// x += sum_i V_i y_i
__global__ void k_update(const double2* V, int64_t ldv, int nv, const double2* y, double2* x, int64_t n) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double2 acc = x[k];
  for (int i = 0; i < nv; ++i) {
    const double2 v = V[i * ldv + k], c = y[i];
    acc.x += v.x * c.x - v.y * c.y;
    acc.y += v.x * c.y + v.y * c.x;
  }
  x[k] = acc;
}

__global__ void k_add(const double2* d, double2* x, int64_t n) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < n) x[k] = make_double2(x[k].x + d[k].x, x[k].y + d[k].y);
}

struct Krylov {
  Ctx& c;
  hipStream_t s;
  int64_t n, ne;
  double s1, s2;
  DevBuf V, Zb, w, partial, hdev, y, r, tmp;
  int m;
  bool pc;
  int n_precond = 0;
  Krylov(Ctx& c_, hipStream_t s_, int m_, bool pc_) : c(c_), s(s_), m(m_), pc(pc_) {
    ne = c.rwg.n_e;
    n = c.rwg.n_e + c.rwg.n_t;
    s1 = 1.0 / (c.rwg.mean_edge * c.rwg.mean_edge);
    s2 = c.rwg.mean_edge;
    V.alloc(size_t(m + 1) * n * 16);
    if (pc) Zb.alloc(size_t(m) * n * 16);
    w.alloc(size_t(n) * 16);
    r.alloc(size_t(n) * 16);
    y.alloc(size_t(n) * 16);
    tmp.alloc(size_t(n) * 16);
    partial.alloc(size_t(kDotBlocks) * (m + 2) * 16);
    hdev.alloc(size_t(m + 2) * 16);
  }
  double2* Vi(int i) { return V.as<double2>() + int64_t(i) * n; }
  double2* Zi(int i) { return Zb.as<double2>() + int64_t(i) * n; }
  void dots(int nv, const double2* vec, std::vector<cd>& out) {
    hipLaunchKernelGGL(k_multidot, dim3(kDotBlocks), dim3(256), 0, s, V.as<double2>(), n, nv, vec, n,
                       partial.as<double2>());
    hipLaunchKernelGGL(k_reduce_partial, dim3(nblk(nv)), dim3(256), 0, s, partial.as<double2>(), kDotBlocks, nv,
                       hdev.as<double2>());
    SLIM_HIP(hipGetLastError());
    out.resize(nv);
    SLIM_HIP(hipMemcpyAsync(out.data(), hdev.p, size_t(nv) * 16, hipMemcpyDeviceToHost, s));
    SLIM_HIP(hipStreamSynchronize(s));
  }
  // sum of |vec_i|^2 (NaN if an entry is not finite)
  double sumsq(const double2* vec) {
    // use the multidot machinery with V_0 := vec
    hipLaunchKernelGGL(k_multidot, dim3(kDotBlocks), dim3(256), 0, s, vec, n, 1, vec, n, partial.as<double2>());
    hipLaunchKernelGGL(k_reduce_partial, dim3(1), dim3(256), 0, s, partial.as<double2>(), kDotBlocks, 1,
                       hdev.as<double2>());
    SLIM_HIP(hipGetLastError());
    cd v;
    SLIM_HIP(hipMemcpyAsync(&v, hdev.p, 16, hipMemcpyDeviceToHost, s));
    SLIM_HIP(hipStreamSynchronize(s));
    return v.real();
  }
  double norm(const double2* vec) { return std::sqrt(std::max(0.0, sumsq(vec))); }
  // out = S A v with the given precision
  void op(slim_prec p, const double2* v, double2* out) {
    matvec(c, p, v, out, nullptr, nullptr, nullptr, nullptr, s);
    hipLaunchKernelGGL(k_scale_rows, dim3(nblk(n)), dim3(256), 0, s, out, ne, n, s1, s2);
    SLIM_HIP(hipGetLastError());
  }
  // One GMRES(m) cycle on S A(p) d = rhs (rhs norm beta) starting from d = 0.
  // Returns iterations done and the estimated residual norm.
  int cycle(slim_prec p, const double2* rhs, double beta, double stop_abs, double2* d, double& est, int max_it) {
    hipLaunchKernelGGL(k_cscale, dim3(nblk(n)), dim3(256), 0, s, rhs, Vi(0), n, 1.0 / beta);
    SLIM_HIP(hipMemsetAsync(d, 0, size_t(n) * 16, s));
    std::vector<cd> Hm(size_t(m + 1) * m, cd(0.0)), cs(m), sn(m), g(m + 1, cd(0.0));
    g[0] = beta;
    std::vector<cd> h, h2;
    int k = 0;
    est = beta;
    for (; k < std::min(m, max_it); ++k) {
      if (pc) {
        precond_apply(c, Vi(k), Zi(k), s);
        n_precond++;
        op(p, Zi(k), w.as<double2>());
      } else {
        op(p, Vi(k), w.as<double2>());
      }
      for (int pass = 0; pass < 2; ++pass) {   // CGS2
        dots(k + 1, w.as<double2>(), h);
        SLIM_HIP(hipMemcpyAsync(hdev.p, h.data(), size_t(k + 1) * 16, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_multiaxpy, dim3(nblk(n)), dim3(256), 0, s, V.as<double2>(), n, k + 1, hdev.as<double2>(),
                           w.as<double2>(), n);
        SLIM_HIP(hipGetLastError());
        for (int i = 0; i <= k; ++i) Hm[size_t(i) * m + k] += h[i];
      }
      double hn = norm(w.as<double2>());
      Hm[size_t(k + 1) * m + k] = hn;
      SLIM_REQUIRE(std::isfinite(hn), SLIM_E_NUMERIC, "GMRES produced a non-finite vector");
      if (hn > 0.0) hipLaunchKernelGGL(k_cscale, dim3(nblk(n)), dim3(256), 0, s, w.as<double2>(), Vi(k + 1), n, 1.0 / hn);
      // rotations [[conj c, conj s], [-s, c]]
      for (int i = 0; i < k; ++i) {
        cd t = std::conj(cs[i]) * Hm[size_t(i) * m + k] + std::conj(sn[i]) * Hm[size_t(i + 1) * m + k];
        Hm[size_t(i + 1) * m + k] = -sn[i] * Hm[size_t(i) * m + k] + cs[i] * Hm[size_t(i + 1) * m + k];
        Hm[size_t(i) * m + k] = t;
      }
      cd a = Hm[size_t(k) * m + k], b = Hm[size_t(k + 1) * m + k];
      double den = std::sqrt(std::norm(a) + std::norm(b));
      cs[k] = den > 0 ? a / den : cd(1.0);
      sn[k] = den > 0 ? b / den : cd(0.0);
      Hm[size_t(k) * m + k] = den;
      Hm[size_t(k + 1) * m + k] = 0.0;
      g[k + 1] = -sn[k] * g[k];
      g[k] = std::conj(cs[k]) * g[k];
      est = std::abs(g[k + 1]);
      if (est <= stop_abs || hn == 0.0) { ++k; break; }
    }
    // back substitution
    std::vector<cd> yv(k);
    for (int i = k - 1; i >= 0; --i) {
      cd acc = g[i];
      for (int j = i + 1; j < k; ++j) acc -= Hm[size_t(i) * m + j] * yv[j];
      yv[i] = acc / Hm[size_t(i) * m + i];
    }
    SLIM_HIP(hipMemcpyAsync(hdev.p, yv.data(), size_t(k) * 16, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_update, dim3(nblk(n)), dim3(256), 0, s, pc ? Zb.as<double2>() : V.as<double2>(), n, k,
                       hdev.as<double2>(), d, n);
    SLIM_HIP(hipGetLastError());
    SLIM_HIP(hipStreamSynchronize(s));
    return k;
  }
};

}  // namespace

slim_status solve_gmres(Ctx& c, const void* b, int scaled_rhs, void* x, const slim_solve_opts& o, slim_solve_info& info,
                        hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  const int m = o.restart > 0 ? o.restart : 50;
  const double tol = o.tol > 0 ? o.tol : 1e-6;
  const int max_iter = o.max_iter > 0 ? o.max_iter : 1000;
  SLIM_REQUIRE(!o.use_precond || c.pc_built, SLIM_E_STATE,
               "use_precond = 1 but no preconditioner was built (build option precond = 0)");
  Krylov K(c, s, m, o.use_precond != 0);
  const double2* B = reinterpret_cast<const double2*>(b);
  double2* X = reinterpret_cast<double2*>(x);
  // ||S b||  (residual of y = 0)
  SLIM_HIP(hipMemsetAsync(K.y.p, 0, size_t(K.n) * 16, s));
  hipLaunchKernelGGL(k_scaled_residual, dim3(nblk(K.n)), dim3(256), 0, s, B, K.y.as<double2>(), K.tmp.as<double2>(),
                     K.ne, K.n, K.s1, K.s2, scaled_rhs);
  SLIM_HIP(hipGetLastError());
  const double bn = K.norm(K.tmp.as<double2>());
  SLIM_REQUIRE(std::isfinite(bn), SLIM_E_NUMERIC, "right-hand side is not finite");
  info = slim_solve_info{};
  if (bn == 0.0) {
    SLIM_HIP(hipMemsetAsync(x, 0, size_t(K.n) * 16, s));
    SLIM_HIP(hipStreamSynchronize(s));
    return SLIM_OK;
  }
  const bool mixed = o.prec == SLIM_MIXED;
  const double inner_tol = o.inner_tol > 0 ? o.inner_tol : 1e-4;
  const int max_outer = o.max_outer > 0 ? o.max_outer : 100000;
  int its = 0, outer = 0;
  double rel = 1.0;
  DevBuf d;
  d.alloc(size_t(K.n) * 16);
  // a zero initial guess has A x = 0: the first residual needs no product (K.y is zero)
  bool x_zero = K.sumsq(reinterpret_cast<const double2*>(x)) == 0.0;
  while (true) {
    // true residual with the FP64 operator
    if (!x_zero) {
      matvec(c, SLIM_FP64, X, K.y.p, nullptr, nullptr, nullptr, nullptr, s);
      info.n_matvec_fp64++;
    }
    x_zero = false;
    hipLaunchKernelGGL(k_scaled_residual, dim3(nblk(K.n)), dim3(256), 0, s, B, K.y.as<double2>(), K.r.as<double2>(),
                       K.ne, K.n, K.s1, K.s2, scaled_rhs);
    SLIM_HIP(hipGetLastError());
    const double rn = K.norm(K.r.as<double2>());
    SLIM_REQUIRE(std::isfinite(rn), SLIM_E_NUMERIC, "residual is not finite");
    rel = rn / bn;
    if (rel <= tol || its >= max_iter || outer >= max_outer) break;
    double est = 0.0;
    const double stop = mixed ? std::max(inner_tol * rn, 0.5 * tol * bn) : 0.5 * tol * bn;
    const int k = K.cycle(mixed ? SLIM_MIXED : SLIM_FP64, K.r.as<double2>(), rn, stop, d.as<double2>(), est,
                          max_iter - its);
    if (mixed) info.n_matvec_mixed += k;
    else info.n_matvec_fp64 += k;
    its += k;
    outer++;
    hipLaunchKernelGGL(k_add, dim3(nblk(K.n)), dim3(256), 0, s, d.as<double2>(), X, K.n);   // x += d
    SLIM_HIP(hipGetLastError());
  }
  SLIM_HIP(hipStreamSynchronize(s));
  info.iterations = its;
  info.n_precond = K.n_precond;
  info.outer_steps = outer;
  info.rel_residual = rel;
  info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return rel <= tol ? SLIM_OK : SLIM_E_NOT_CONVERGED;
}

}  // namespace slim
