// Quadrature rule tables and the launch interfaces of the pair-integral kernels.
#pragma once
#include "common.hpp"

namespace slim {

constexpr int kMaxTri1 = 10;            // max points per axis of TRI(n)
constexpr int kMaxRad = 64;             // max radial points of the composite rule
constexpr int kMaxAng = 16;             // max angular points

struct QuadRulesDev {
  int n_far, n_near, n_rad, n_ang;
  double c_near;
  double far_u[kMaxTri1 * kMaxTri1], far_v[kMaxTri1 * kMaxTri1], far_w[kMaxTri1 * kMaxTri1];
  double near_u[kMaxTri1 * kMaxTri1], near_v[kMaxTri1 * kMaxTri1], near_w[kMaxTri1 * kMaxTri1];
  double rad_s[kMaxRad], rad_w[kMaxRad];
  double ang_x[kMaxAng], ang_w[kMaxAng];
};

void make_rules(const QuadOpts& o, QuadRulesDev& R);
void upload_rules(const QuadRulesDev& R);

struct AsmLaunch {
  const double* xyz; const int32_t* tri; const double* cen; const double* nrm; const double* area;
  const double* diam; const int32_t* tri_edge; const int8_t* tri_sign; const double* len;
  int32_t t0, t1, e0;
  cd k;
  double* Lk = nullptr;
  double* Kk = nullptr;
  double* Lvec = nullptr;
  double* Lphi = nullptr;
  int64_t ld_e = 0, ld_t = 0;
  const int32_t* erow = nullptr;          // row selections of Lvec / Lphi (local index -> row, -1 skip)
  const int32_t* trow = nullptr;
  const int32_t* near_pairs = nullptr;   // candidate (t, u) pairs, t <= u
  int64_t n_near_pairs = 0;
  double skip_mag = 0.0;
  double cut_r2 = 0.0;   // > 0: only pairs with squared centroid distance <= cut_r2 (sparse interior operators)
};
void launch_assemble(const AsmLaunch& L, hipStream_t s);

struct NearArgs {
  const double* xyz; const int32_t* tri; const double* cen; const double* nrm; const double* area;
  const double* diam; const int32_t* tri_edge; const int8_t* tri_sign; const double* len;
  const int32_t* tplus; const int32_t* tminus;
  const int32_t* rows; const int32_t* cols;   // COO of the CSR pattern
  int64_t nnz;
  double kr, ki;
  double* out;                                // complex128 values
  // triangle-pair table (optional): the L_phi pass writes the oriented vector-potential
  // integrals IA (3 x 3 complex) of each of its pairs at ia + 18 z; the L_A pass looks its
  // triangle pairs up in that pattern (CSR tp_ptr / tp_col over triangle rows) and
  // computes only the pairs it does not hold
  double* ia = nullptr;
  const int64_t* tp_ptr = nullptr;
  const int32_t* tp_col = nullptr;
};
void launch_near_entries(const NearArgs& g, bool rwg, hipStream_t s);

}  // namespace slim
