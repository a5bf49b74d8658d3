// Shared declarations of the MI355X SLIM library (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/slim.h"

namespace slim {

using cd = std::complex<double>;

// ---- physical constants (SI) ------------------------------------------------
constexpr double kC0 = 299792458.0;
constexpr double kMu0 = 4.0e-7 * 3.14159265358979323846;
constexpr double kPi = 3.14159265358979323846;
inline double eps0() { return 1.0 / (kMu0 * kC0 * kC0); }
inline double eta0() { return kMu0 * kC0; }

// ---- errors -------------------------------------------------------------------
struct Error : std::runtime_error {
  slim_status code;
  Error(slim_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define SLIM_HIP(call)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::slim::Error(SLIM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define SLIM_REQUIRE(cond, code, msg)                  \
  do {                                                 \
    if (!(cond)) throw ::slim::Error((code), (msg));   \
  } while (0)

// ---- device buffer --------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();   // a failed allocation must not surface at the next launch check
      throw Error(SLIM_E_OOM, "hipMalloc of " + std::to_string(n) + " bytes failed");
    }
    bytes = n;
  }
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
  template <class T> void upload(const std::vector<T>& v) {
    alloc(v.size() * sizeof(T));
    if (!v.empty()) SLIM_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  }
};

// ---- mesh / RWG (host) -------------------------------------------------------------
struct Mesh {
  std::vector<double> xyz;       // n_vert*3
  std::vector<int32_t> tri;      // n_tri*3
  std::vector<int32_t> obj;      // n_tri
  int32_t n_obj = 0;
  int64_t n_vert = 0, n_tri = 0;
};

struct RWGTable {
  int64_t n_e = 0, n_t = 0;
  int32_t n_obj = 0;
  std::vector<int32_t> ev;        // 2 n_e (lower, higher vertex)
  std::vector<int32_t> tplus, tminus;
  std::vector<double> len;        // n_e
  std::vector<int32_t> tri_edge;  // 3 n_t: RWG of the edge opposite local vertex i
  std::vector<int8_t> tri_sign;   // 3 n_t
  std::vector<double> area, normal, centroid, diam;  // n_t, 3n_t, 3n_t, n_t
  std::vector<int64_t> obj_edge_off, obj_tri_off;    // n_obj+1
  double mean_edge = 0.0;
};

RWGTable build_rwg(const Mesh& m);

struct Material {
  double sigma = 5.8e7, eps_r = 1.0, mu_r = 1.0;
};

// Triangle-pair quadrature parameters (same meaning as slim_build_opts).
struct QuadOpts {
  int n_far = 4, n_near = 5, levels = 3, n_r = 5, n_t = 6;
  double q = 0.25, c_near = 2.0;
};

}  // namespace slim
