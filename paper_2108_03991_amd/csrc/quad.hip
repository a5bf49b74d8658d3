// Triangle-pair integrals of the Galerkin operators (Sec. II-A, II-B) on the GPU.
//
// For a test triangle Ta (local vertices p_i) and a source triangle Tb (local
// vertices q_j), G = e^{-jkR}/(4 pi R) and d = r - r':
//   IA[i][j] = int int (r - p_i).(r' - q_j) G        (vector potential)
//   IS       = int int G                              (scalar potential)
//   IK[i][j] = int int (r - p_i).(grad_r G x (r' - q_j)),
//              grad_r G = -(1 + jkR) e^{-jkR} d / (4 pi R^3)  (double layer)
// The paper leaves the integration rules open.  Rules used here:
//   TRI(n): collapsed Gauss-Legendre, r = v0 + u e1 + v (1-u) e2, weight
//           2A w_u w_v (1-u);
//   far pair (centroid distance >= c_near * max diameter): TRI(n_far) x TRI(n_far);
//   near pair: TRI(n_near) on the lower-index triangle and, around the projection
//           rho0 of each of its points on the other triangle's plane, a polar
//           rule over the three signed sub-triangles (rho0, u1, u2): angle
//           through u = asinh(tan theta) (n_t Gauss points, theta from the foot
//           of the perpendicular on the edge line at distance h), radius
//           rho = s h cosh(u) with s on the composite Gauss rule with breakpoints
//           0, q^L, ..., q, 1 (n_r points per interval); area element
//           s (h cosh u)^2 ds dtheta, dtheta = du / cosh u.
//   The double layer vanishes for coplanar pairs (principal value on flat
//   triangles).  A triangle paired with itself is averaged over (i,j) <-> (j,i).
// The sums are accumulated as moments about the centroid c of Ta:
//   (a - P_i).(b - Q_j) = a.b - P_i.b - Q_j.a + P_i.Q_j,
//   (a - P_i).((a - b) x (b - Q_j)) = (Q_j - P_i).(a x b) + Q_j.(P_i x (a - b)),
// a = r - c, b = r' - c, P_i = p_i - c, Q_j = q_j - c.
#include "common.hpp"
#include "quad.hpp"

namespace slim {

__constant__ QuadRulesDev c_rules;

// ---------------------------------------------------------------------------
// Host: rule tables
// ---------------------------------------------------------------------------
void gauss01_host(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    // Newton iteration on P_n from the Chebyshev-like initial guess
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), pp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; ++j) {
        double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0);
      double dz = p1 / pp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[n - 1 - i] = 0.5 * (z + 1.0);
    w[n - 1 - i] = 1.0 / ((1.0 - z * z) * pp * pp);
  }
}

void make_rules(const QuadOpts& o, QuadRulesDev& R) {
  SLIM_REQUIRE(o.n_far >= 1 && o.n_far <= kMaxTri1 && o.n_near >= 1 && o.n_near <= kMaxTri1, SLIM_E_ARG,
               "triangle rule order out of range");
  SLIM_REQUIRE(o.n_t >= 1 && o.n_t <= kMaxAng && o.n_r >= 1 && (o.levels + 1) * o.n_r <= kMaxRad, SLIM_E_ARG,
               "polar rule size out of range");
  std::vector<double> x, w;
  auto tri = [&](int n, double* U, double* V, double* W) {
    gauss01_host(n, x, w);
    int k = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j, ++k) {
        U[k] = x[i];
        V[k] = x[j] * (1.0 - x[i]);
        W[k] = w[i] * w[j] * (1.0 - x[i]);
      }
  };
  R.n_far = o.n_far * o.n_far;
  R.n_near = o.n_near * o.n_near;
  tri(o.n_far, R.far_u, R.far_v, R.far_w);
  tri(o.n_near, R.near_u, R.near_v, R.near_w);
  gauss01_host(o.n_r, x, w);
  std::vector<double> bp;
  bp.push_back(0.0);
  for (int l = 0; l < o.levels; ++l) bp.push_back(std::pow(o.q, o.levels - l));
  bp.push_back(1.0);
  int k = 0;
  for (size_t b = 0; b + 1 < bp.size(); ++b)
    for (int i = 0; i < o.n_r; ++i, ++k) {
      R.rad_s[k] = bp[b] + (bp[b + 1] - bp[b]) * x[i];
      R.rad_w[k] = (bp[b + 1] - bp[b]) * w[i];
    }
  R.n_rad = k;
  gauss01_host(o.n_t, x, w);
  R.n_ang = o.n_t;
  for (int i = 0; i < o.n_t; ++i) { R.ang_x[i] = x[i]; R.ang_w[i] = w[i]; }
  R.c_near = o.c_near;
}

void upload_rules(const QuadRulesDev& R) { SLIM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_rules), &R, sizeof(R))); }

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
struct V3 { double x, y, z; };
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ V3 ld3(const double* p) { return {p[0], p[1], p[2]}; }

struct Cx { double r, i; };
__device__ __forceinline__ Cx cmul(Cx a, Cx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }

// Weighted moment sums of one pair (see the file header).
struct Moments {
  double S0r, S0i, Sabr, Sabi, g0r, g0i;
  double Sar[3], Sai[3], Sbr[3], Sbi[3], Yar[3], Yai[3], Ybr[3], Ybi[3], Xr[3], Xi[3];
};

__device__ __forceinline__ void mom_zero(Moments& M) {
  double* p = reinterpret_cast<double*>(&M);
#pragma unroll
  for (int i = 0; i < int(sizeof(Moments) / sizeof(double)); ++i) p[i] = 0.0;
}

// Add one point pair (a, b relative to the centroid of Ta) with weight w.
template <bool WANT_K>
__device__ __forceinline__ void mom_add(Moments& M, V3 a, V3 b, double w, double kr, double ki) {
  V3 d = a - b;
  double R = sqrt(dot(d, d));
  // e^{-jkR} = e^{ki R} (cos(kr R) - j sin(kr R))
  double mag = exp(ki * R);
  double sn, cs;
  sincos(kr * R, &sn, &cs);
  Cx e = {mag * cs, -mag * sn};
  double inv4piR = 1.0 / (4.0 * kPi * R);
  Cx G = {w * e.r * inv4piR, w * e.i * inv4piR};
  double ab = dot(a, b);
  M.S0r += G.r; M.S0i += G.i;
  M.Sabr += G.r * ab; M.Sabi += G.i * ab;
  const double av[3] = {a.x, a.y, a.z}, bv[3] = {b.x, b.y, b.z};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    M.Sar[c] += G.r * av[c]; M.Sai[c] += G.i * av[c];
    M.Sbr[c] += G.r * bv[c]; M.Sbi[c] += G.i * bv[c];
  }
  if (WANT_K) {
    // g = -(1 + jkR) e^{-jkR} / (4 pi R^3) times the weight
    Cx one_jkR = {1.0 - ki * R, kr * R};   // 1 + j (kr + j ki) R
    Cx ge = cmul(one_jkR, e);
    double s = -w * inv4piR / (R * R);
    Cx g = {s * ge.r, s * ge.i};
    V3 x = cross(a, b);
    const double xv[3] = {x.x, x.y, x.z};
    M.g0r += g.r; M.g0i += g.i;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      M.Yar[c] += g.r * av[c]; M.Yai[c] += g.i * av[c];
      M.Ybr[c] += g.r * bv[c]; M.Ybi[c] += g.i * bv[c];
      M.Xr[c] += g.r * xv[c]; M.Xi[c] += g.i * xv[c];
    }
  }
}

__device__ __forceinline__ void mom_wave_reduce(Moments& M) {
  double* p = reinterpret_cast<double*>(&M);
#pragma unroll
  for (int i = 0; i < int(sizeof(Moments) / sizeof(double)); ++i) {
    double v = p[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    p[i] = v;
  }
}

// IA, IS, IK from the moments; P, Q local vertices relative to the centroid of Ta.
__device__ void mom_finish(const Moments& M, const V3 P[3], const V3 Q[3], bool want_k, bool coplanar,
                           Cx IA[9], Cx& IS, Cx IK[9]) {
  IS = {M.S0r, M.S0i};
  V3 Sar = {M.Sar[0], M.Sar[1], M.Sar[2]}, Sai = {M.Sai[0], M.Sai[1], M.Sai[2]};
  V3 Sbr = {M.Sbr[0], M.Sbr[1], M.Sbr[2]}, Sbi = {M.Sbi[0], M.Sbi[1], M.Sbi[2]};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double pq = dot(P[i], Q[j]);
      IA[3 * i + j] = {M.Sabr - dot(P[i], Sbr) - dot(Q[j], Sar) + pq * M.S0r,
                       M.Sabi - dot(P[i], Sbi) - dot(Q[j], Sai) + pq * M.S0i};
    }
  if (!want_k) return;
  if (coplanar) {
    for (int i = 0; i < 9; ++i) IK[i] = {0.0, 0.0};
    return;
  }
  V3 Xr = {M.Xr[0], M.Xr[1], M.Xr[2]}, Xi = {M.Xi[0], M.Xi[1], M.Xi[2]};
  V3 Dr = {M.Yar[0] - M.Ybr[0], M.Yar[1] - M.Ybr[1], M.Yar[2] - M.Ybr[2]};
  V3 Di = {M.Yai[0] - M.Ybi[0], M.Yai[1] - M.Ybi[1], M.Yai[2] - M.Ybi[2]};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      V3 qp = Q[j] - P[i];
      IK[3 * i + j] = {dot(qp, Xr) + dot(Q[j], cross(P[i], Dr)), dot(qp, Xi) + dot(Q[j], cross(P[i], Di))};
    }
}

// Classification, computed without contracted multiply-adds so that every
// implementation of the same rule takes the same decision.
__device__ __forceinline__ bool pair_is_near(const double* cen, const double* diam, int t, int u, double c_near) {
  double dx = __dsub_rn(cen[3 * t], cen[3 * u]);
  double dy = __dsub_rn(cen[3 * t + 1], cen[3 * u + 1]);
  double dz = __dsub_rn(cen[3 * t + 2], cen[3 * u + 2]);
  double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
  double dm = __dmul_rn(fmax(diam[t], diam[u]), c_near);
  return d2 < __dmul_rn(dm, dm);
}

// A pair farther apart than the cutoff of the sparse interior operators (squared
// centroid distance summed as dx*dx + dy*dy + dz*dz, no contracted multiply-adds).
__device__ __forceinline__ bool pair_beyond(const double* cen, int t, int u, double cut_r2) {
  if (cut_r2 <= 0.0) return false;
  double dx = __dsub_rn(cen[3 * t], cen[3 * u]);
  double dy = __dsub_rn(cen[3 * t + 1], cen[3 * u + 1]);
  double dz = __dsub_rn(cen[3 * t + 2], cen[3 * u + 2]);
  double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
  return d2 > cut_r2;
}

__device__ __forceinline__ bool pair_is_coplanar(const double* cen, const double* nrm, const double* diam, int t, int u) {
  V3 nt = ld3(nrm + 3 * t), nu = ld3(nrm + 3 * u);
  V3 d = ld3(cen + 3 * t) - ld3(cen + 3 * u);
  return fabs(dot(nt, nu)) > 1.0 - 1e-12 && fabs(dot(nt, d)) < 1e-9 * fmax(diam[t], diam[u]);
}

struct Tri {
  V3 v[3];
  V3 c;        // centroid
  V3 n;        // unit normal
  double two_a;
};

__device__ __forceinline__ Tri load_tri(const double* xyz, const int32_t* tri, const double* cen, const double* nrm,
                                        const double* area, int t) {
  Tri T;
  for (int i = 0; i < 3; ++i) T.v[i] = ld3(xyz + 3 * size_t(tri[3 * t + i]));
  T.c = ld3(cen + 3 * t);
  T.n = ld3(nrm + 3 * t);
  T.two_a = 2.0 * area[t];
  return T;
}

// Far rule: one thread, TRI(n_far) x TRI(n_far).
template <bool WANT_K>
__device__ void far_pair(const Tri& A, const Tri& B, double kr, double ki, Moments& M) {
  mom_zero(M);
  const V3 ea1 = A.v[1] - A.v[0], ea2 = A.v[2] - A.v[0];
  const V3 eb1 = B.v[1] - B.v[0], eb2 = B.v[2] - B.v[0];
  for (int p = 0; p < c_rules.n_far; ++p) {
    V3 ra = A.v[0] + c_rules.far_u[p] * ea1 + c_rules.far_v[p] * ea2;
    V3 a = ra - A.c;
    double wa = A.two_a * c_rules.far_w[p];
    for (int q = 0; q < c_rules.n_far; ++q) {
      V3 rb = B.v[0] + c_rules.far_u[q] * eb1 + c_rules.far_v[q] * eb2;
      mom_add<WANT_K>(M, a, rb - A.c, wa * B.two_a * c_rules.far_w[q], kr, ki);
    }
  }
}

// Wave (64 lanes) cooperative rule; near: polar inner rule, far: product rule.
template <bool WANT_K>
__device__ void wave_pair(const Tri& A, const Tri& B, bool near, double kr, double ki, Moments& M) {
  const int lane = threadIdx.x & 63;
  mom_zero(M);
  const V3 ea1 = A.v[1] - A.v[0], ea2 = A.v[2] - A.v[0];
  if (!near) {
    const V3 eb1 = B.v[1] - B.v[0], eb2 = B.v[2] - B.v[0];
    const int tot = c_rules.n_far * c_rules.n_far;
    for (int it = lane; it < tot; it += 64) {
      int p = it / c_rules.n_far, q = it % c_rules.n_far;
      V3 ra = A.v[0] + c_rules.far_u[p] * ea1 + c_rules.far_v[p] * ea2;
      V3 rb = B.v[0] + c_rules.far_u[q] * eb1 + c_rules.far_v[q] * eb2;
      mom_add<WANT_K>(M, ra - A.c, rb - A.c, A.two_a * c_rules.far_w[p] * B.two_a * c_rules.far_w[q], kr, ki);
    }
  } else {
    const int tot = c_rules.n_near * 3 * c_rules.n_ang;
    for (int it = lane; it < tot; it += 64) {
      int p = it / (3 * c_rules.n_ang);
      int rem = it % (3 * c_rules.n_ang);
      int e = rem / c_rules.n_ang, ia = rem % c_rules.n_ang;
      V3 ra = A.v[0] + c_rules.near_u[p] * ea1 + c_rules.near_v[p] * ea2;
      double wa = A.two_a * c_rules.near_w[p];
      double hgt = dot(ra - B.v[0], B.n);
      V3 rho0 = ra - hgt * B.n;
      V3 u1 = B.v[(e + 1) % 3], u2 = B.v[(e + 2) % 3];
      V3 E = u2 - u1;
      double elen = sqrt(dot(E, E));
      V3 et = (1.0 / elen) * E;
      double l1 = dot(u1 - rho0, et), l2 = dot(u2 - rho0, et);
      V3 hv = (u1 - rho0) - l1 * et;
      double h = sqrt(dot(hv, hv));
      if (!(h > 1e-12 * elen)) continue;
      double sg = dot(B.n, cross(u1 - rho0, u2 - rho0)) >= 0.0 ? 1.0 : -1.0;
      V3 eh = (1.0 / h) * hv;
      double a1 = asinh(l1 / h), a2 = asinh(l2 / h);
      double uu = a1 + (a2 - a1) * c_rules.ang_x[ia];
      double wu = (a2 - a1) * c_rules.ang_w[ia];
      double ch = cosh(uu);
      double rmax = h * ch;
      double wth = wu / ch;
      V3 dir = (1.0 / ch) * eh + tanh(uu) * et;   // cos(theta) e_h + sin(theta) e_t
      V3 a = ra - A.c;
      for (int ir = 0; ir < c_rules.n_rad; ++ir) {
        double s = c_rules.rad_s[ir];
        V3 rb = rho0 + (s * rmax) * dir;
        double w = sg * s * c_rules.rad_w[ir] * rmax * rmax * wth;
        mom_add<WANT_K>(M, a, rb - A.c, wa * w, kr, ki);
      }
    }
  }
  mom_wave_reduce(M);
}

__device__ __forceinline__ void local_pq(const Tri& A, const Tri& B, V3 P[3], V3 Q[3]) {
  for (int i = 0; i < 3; ++i) {
    P[i] = A.v[i] - A.c;
    Q[i] = B.v[i] - A.c;
  }
}

// ---------------------------------------------------------------------------
// Dense assembly (interior L_k, K_k of one object; plain-mode external L_A, L_phi)
// Column-major n x n complex128 (ld = n) outputs, RWG indices local to the
// object (minus e0), triangle indices t in [t0, t1).
// ---------------------------------------------------------------------------
struct AsmArgs {
  const double* xyz; const int32_t* tri; const double* cen; const double* nrm; const double* area;
  const double* diam; const int32_t* tri_edge; const int8_t* tri_sign; const double* len;
  int32_t t0, t1, e0;
  double kr, ki;             // wavenumber
  double inv_k2r, inv_k2i;   // 1/k^2
  double* Lk;                // L_k = Lvec - Ldiv/k^2 (or null)
  double* Kk;                // K_k (or null)
  double* Lvec;              // vector part only (plain L_A) (or null)
  double* Lphi;              // n_t x n_t, IS/(A A') (or null)
  int64_t ld_e, ld_t;
  // optional row selections for Lvec / Lphi: local edge (triangle) -> output row,
  // -1 = not kept; the outputs are then (kept rows) x (all local columns), ld = kept rows
  const int32_t* erow;
  const int32_t* trow;
  double skip_mag;           // skip far pairs with |e^{-jkR}| below this at the closest approach
  double cut_r2;             // > 0: skip pairs whose squared centroid distance exceeds it
};

__device__ __forceinline__ void atomic_c(double* M, int64_t idx, Cx v) {
  atomicAdd(M + 2 * idx, v.r);
  atomicAdd(M + 2 * idx + 1, v.i);
}

template <bool WANT_K>
__device__ void scatter_pair(const AsmArgs& g, int t, int u, Cx IA[9], Cx IS, Cx IK[9]) {
  if (t == u) {  // symmetric average for a triangle with itself
    for (int i = 0; i < 3; ++i)
      for (int j = i + 1; j < 3; ++j) {
        Cx a = IA[3 * i + j], b = IA[3 * j + i];
        IA[3 * i + j] = IA[3 * j + i] = {0.5 * (a.r + b.r), 0.5 * (a.i + b.i)};
        if (WANT_K) {
          a = IK[3 * i + j]; b = IK[3 * j + i];
          IK[3 * i + j] = IK[3 * j + i] = {0.5 * (a.r + b.r), 0.5 * (a.i + b.i)};
        }
      }
  }
  const double At = g.area[t], Au = g.area[u];
  for (int i = 0; i < 3; ++i) {
    int m = g.tri_edge[3 * t + i];
    double sm = g.tri_sign[3 * t + i] * g.len[m];
    for (int j = 0; j < 3; ++j) {
      int n = g.tri_edge[3 * u + j];
      double cv = sm * g.tri_sign[3 * u + j] * g.len[n] / (4.0 * At * Au);
      double cdv = 4.0 * cv;
      Cx a = IA[3 * i + j];
      int64_t ml = m - g.e0, nl = n - g.e0;
      if (g.Lk) {
        // cv IA - (cd IS) / k^2
        Cx dv = {cdv * IS.r, cdv * IS.i};
        Cx dk = cmul(dv, {g.inv_k2r, g.inv_k2i});
        Cx v = {cv * a.r - dk.r, cv * a.i - dk.i};
        atomic_c(g.Lk, ml + nl * g.ld_e, v);
        if (t != u) atomic_c(g.Lk, nl + ml * g.ld_e, v);
      }
      if (g.Lvec) {
        Cx v = {cv * a.r, cv * a.i};
        if (!g.erow) {
          atomic_c(g.Lvec, ml + nl * g.ld_e, v);
          if (t != u) atomic_c(g.Lvec, nl + ml * g.ld_e, v);
        } else {
          // symmetric matrix: entry (m, n) and its mirror (n, m), each kept if its row is selected
          const int rm = g.erow[ml], rn = g.erow[nl];
          if (rm >= 0) atomic_c(g.Lvec, rm + nl * g.ld_e, v);
          if (t != u && rn >= 0) atomic_c(g.Lvec, rn + ml * g.ld_e, v);
        }
      }
      if (WANT_K && g.Kk) {
        Cx v = {cv * IK[3 * i + j].r, cv * IK[3 * i + j].i};
        atomic_c(g.Kk, ml + nl * g.ld_e, v);
        if (t != u) atomic_c(g.Kk, nl + ml * g.ld_e, v);
      }
    }
  }
  if (g.Lphi) {
    Cx v = {IS.r / (At * Au), IS.i / (At * Au)};
    int64_t tl = t - g.t0, ul = u - g.t0;
    if (!g.trow) {
      atomic_c(g.Lphi, tl + ul * g.ld_t, v);
      if (t != u) atomic_c(g.Lphi, ul + tl * g.ld_t, v);
    } else {
      const int rt = g.trow[tl], ru = g.trow[ul];
      if (rt >= 0) atomic_c(g.Lphi, rt + ul * g.ld_t, v);
      if (t != u && ru >= 0) atomic_c(g.Lphi, ru + tl * g.ld_t, v);
    }
  }
}

template <bool WANT_K>
__global__ void __launch_bounds__(256) k_assemble_far(AsmArgs g) {
  const int n = g.t1 - g.t0;
  const int bt = blockIdx.y, bu = blockIdx.x;
  if (bu < bt) return;
  const int t = g.t0 + bt * 16 + (threadIdx.x >> 4);
  const int u = g.t0 + bu * 16 + (threadIdx.x & 15);
  if (t >= g.t0 + n || u >= g.t0 + n || u < t) return;
  if (pair_is_near(g.cen, g.diam, t, u, c_rules.c_near)) return;
  if (pair_beyond(g.cen, t, u, g.cut_r2)) return;
  if (g.skip_mag > 0.0) {
    V3 d = ld3(g.cen + 3 * t) - ld3(g.cen + 3 * u);
    double rmin = sqrt(dot(d, d)) - 0.5 * (g.diam[t] + g.diam[u]);
    if (rmin > 0.0 && exp(g.ki * rmin) < g.skip_mag) return;
  }
  Tri A = load_tri(g.xyz, g.tri, g.cen, g.nrm, g.area, t);
  Tri B = load_tri(g.xyz, g.tri, g.cen, g.nrm, g.area, u);
  Moments M;
  far_pair<WANT_K>(A, B, g.kr, g.ki, M);
  V3 P[3], Q[3];
  local_pq(A, B, P, Q);
  Cx IA[9], IS, IK[9];
  mom_finish(M, P, Q, WANT_K, pair_is_coplanar(g.cen, g.nrm, g.diam, t, u), IA, IS, IK);
  scatter_pair<WANT_K>(g, t, u, IA, IS, IK);
}

// One wave per candidate pair (t <= u); only pairs classified near are done here.
template <bool WANT_K>
__global__ void __launch_bounds__(64) k_assemble_near(AsmArgs g, const int32_t* pairs, int64_t n_pairs) {
  const int64_t p = blockIdx.x;
  if (p >= n_pairs) return;
  const int t = pairs[2 * p], u = pairs[2 * p + 1];
  if (!pair_is_near(g.cen, g.diam, t, u, c_rules.c_near)) return;
  if (pair_beyond(g.cen, t, u, g.cut_r2)) return;
  Tri A = load_tri(g.xyz, g.tri, g.cen, g.nrm, g.area, t);
  Tri B = load_tri(g.xyz, g.tri, g.cen, g.nrm, g.area, u);
  Moments M;
  wave_pair<WANT_K>(A, B, true, g.kr, g.ki, M);
  if ((threadIdx.x & 63) != 0) return;
  V3 P[3], Q[3];
  local_pq(A, B, P, Q);
  Cx IA[9], IS, IK[9];
  mom_finish(M, P, Q, WANT_K, pair_is_coplanar(g.cen, g.nrm, g.diam, t, u), IA, IS, IK);
  scatter_pair<WANT_K>(g, t, u, IA, IS, IK);
}

void launch_assemble(const AsmLaunch& L, hipStream_t s) {
  AsmArgs g;
  g.xyz = L.xyz; g.tri = L.tri; g.cen = L.cen; g.nrm = L.nrm; g.area = L.area; g.diam = L.diam;
  g.tri_edge = L.tri_edge; g.tri_sign = L.tri_sign; g.len = L.len;
  g.t0 = L.t0; g.t1 = L.t1; g.e0 = L.e0;
  g.kr = L.k.real(); g.ki = L.k.imag();
  cd ik2 = 1.0 / (L.k * L.k);
  g.inv_k2r = ik2.real(); g.inv_k2i = ik2.imag();
  g.Lk = L.Lk; g.Kk = L.Kk; g.Lvec = L.Lvec; g.Lphi = L.Lphi;
  g.ld_e = L.ld_e; g.ld_t = L.ld_t;
  g.erow = L.erow; g.trow = L.trow;
  g.skip_mag = L.skip_mag;
  g.cut_r2 = L.cut_r2;
  const int n = L.t1 - L.t0;
  dim3 grid((n + 15) / 16, (n + 15) / 16);
  const bool wk = L.Kk != nullptr;
  if (wk) hipLaunchKernelGGL(k_assemble_far<true>, grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL(k_assemble_far<false>, grid, dim3(256), 0, s, g);
  SLIM_HIP(hipGetLastError());
  // one 64-lane workgroup per candidate pair, at most 2^25 per launch (a dispatch
  // holds fewer than 2^32 work-items)
  const int64_t chunk = int64_t(1) << 25;
  for (int64_t lo = 0; lo < L.n_near_pairs; lo += chunk) {
    const int64_t np = std::min(chunk, L.n_near_pairs - lo);
    const int32_t* pp = L.near_pairs + 2 * lo;
    if (wk) hipLaunchKernelGGL(k_assemble_near<true>, dim3(unsigned(np)), dim3(64), 0, s, g, pp, np);
    else hipLaunchKernelGGL(k_assemble_near<false>, dim3(unsigned(np)), dim3(64), 0, s, g, pp, np);
    SLIM_HIP(hipGetLastError());
  }
}

// ---------------------------------------------------------------------------
// Near-field entries of L_A (RWG pairs) and L_phi (triangle pairs), CSR order.
// One wave per non-zero; triangle-pair integrals oriented with the lower
// triangle index as test triangle, like the dense assembly.
// ---------------------------------------------------------------------------
__device__ void tri_pair_oriented(const NearArgs& g, int t, int u, Cx IA[9], Cx& IS) {
  const int lo = min(t, u), hi = max(t, u);
  Tri A = load_tri(g.xyz, g.tri, g.cen, g.nrm, g.area, lo);
  Tri B = load_tri(g.xyz, g.tri, g.cen, g.nrm, g.area, hi);
  const bool near = pair_is_near(g.cen, g.diam, lo, hi, c_rules.c_near);
  Moments M;
  wave_pair<false>(A, B, near, g.kr, g.ki, M);
  V3 P[3], Q[3];
  local_pq(A, B, P, Q);
  Cx IK[9];
  Cx J[9];
  mom_finish(M, P, Q, false, false, J, IS, IK);
  if (lo == hi) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        Cx a = J[3 * i + j], b = J[3 * j + i];
        IA[3 * i + j] = {0.5 * (a.r + b.r), 0.5 * (a.i + b.i)};
      }
  } else if (t == lo) {
    for (int i = 0; i < 9; ++i) IA[i] = J[i];
  } else {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) IA[3 * i + j] = J[3 * j + i];
  }
}

// position of column u in row t of a CSR with sorted columns, or -1
__device__ __forceinline__ int64_t csr_find(const int64_t* ptr, const int32_t* col, int t, int u) {
  int64_t lo = ptr[t], hi = ptr[t + 1];
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (col[mid] < u) lo = mid + 1;
    else hi = mid;
  }
  return lo < ptr[t + 1] && col[lo] == u ? lo : -1;
}

__global__ void __launch_bounds__(64) k_near_LA(NearArgs g) {
  const int64_t z = blockIdx.x;
  if (z >= g.nnz) return;
  const int m = g.rows[z], n = g.cols[z];
  double accr = 0.0, acci = 0.0;
  const int tm[2] = {g.tplus[m], g.tminus[m]};
  const int tn[2] = {g.tplus[n], g.tminus[n]};
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int t = tm[a], u = tn[b];
      int i = 0, j = 0;
      for (int k = 0; k < 3; ++k) {
        if (g.tri_edge[3 * t + k] == m) i = k;
        if (g.tri_edge[3 * u + k] == n) j = k;
      }
      // the same oriented integrals as tri_pair_oriented computes, from the table when
      // the L_phi pattern holds (t, u) (every lane takes the same branch)
      const int64_t pos = g.ia ? csr_find(g.tp_ptr, g.tp_col, t, u) : -1;
      Cx v;
      if (pos >= 0) {
        v = {g.ia[18 * pos + 2 * (3 * i + j)], g.ia[18 * pos + 2 * (3 * i + j) + 1]};
      } else {
        Cx IA[9], IS;
        tri_pair_oriented(g, t, u, IA, IS);
        v = IA[3 * i + j];
      }
      double cv = g.tri_sign[3 * t + i] * g.tri_sign[3 * u + j] * g.len[m] * g.len[n] / (4.0 * g.area[t] * g.area[u]);
      accr += cv * v.r;
      acci += cv * v.i;
    }
  if ((threadIdx.x & 63) == 0) {
    g.out[2 * z] = accr;
    g.out[2 * z + 1] = acci;
  }
}

__global__ void __launch_bounds__(64) k_near_Lphi(NearArgs g) {
  const int64_t z = blockIdx.x;
  if (z >= g.nnz) return;
  const int t = g.rows[z], u = g.cols[z];
  Cx IA[9], IS;
  tri_pair_oriented(g, t, u, IA, IS);
  if ((threadIdx.x & 63) == 0) {
    g.out[2 * z] = IS.r / (g.area[t] * g.area[u]);
    g.out[2 * z + 1] = IS.i / (g.area[t] * g.area[u]);
    if (g.ia)
      for (int k = 0; k < 9; ++k) {
        g.ia[18 * z + 2 * k] = IA[k].r;
        g.ia[18 * z + 2 * k + 1] = IA[k].i;
      }
  }
}

void launch_near_entries(const NearArgs& g, bool rwg, hipStream_t s) {
  if (g.nnz == 0) return;
  // one 64-lane workgroup per non-zero; a dispatch holds fewer than 2^32 work-items
  // in total, so at most 2^25 workgroups go into one launch
  const int64_t chunk = int64_t(1) << 25;
  for (int64_t lo = 0; lo < g.nnz; lo += chunk) {
    NearArgs h = g;
    h.rows += lo; h.cols += lo; h.out += 2 * lo;
    if (h.ia && !rwg) h.ia += 18 * lo;   // the L_phi pass writes its chunk's rows of the table
    h.nnz = std::min(chunk, g.nnz - lo);
    if (rwg) hipLaunchKernelGGL(k_near_LA, dim3(unsigned(h.nnz)), dim3(64), 0, s, h);
    else hipLaunchKernelGGL(k_near_Lphi, dim3(unsigned(h.nnz)), dim3(64), 0, s, h);
    SLIM_HIP(hipGetLastError());
  }
}

}  // namespace slim
