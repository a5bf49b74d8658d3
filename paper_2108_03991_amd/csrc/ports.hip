// Lumped ports (Sec. II: excitation by lumped ports): the ring of mesh edges that a
// port's plane cuts from one conductor, the right-hand-side weights on it, and the
// port currents of solution columns (one workgroup per port and column).
#include <algorithm>
#include <map>

#include "ctx.hpp"

namespace slim {

namespace {

double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// I[p + n_ports col] = sum over the ring of port p of w_m X[m + col nsys]
__global__ void __launch_bounds__(256) k_port_currents(const int32_t* edges, const double* w, const int32_t* start,
                                                       const double2* X, int64_t nsys, int n_ports, double2* I) {
  const int p = blockIdx.x, col = blockIdx.y;
  __shared__ double sr[256], si[256];
  double ar = 0.0, ai = 0.0;
  for (int k = start[p] + threadIdx.x; k < start[p + 1]; k += 256) {
    const double2 v = X[int64_t(col) * nsys + edges[k]];
    ar += w[k] * v.x;
    ai += w[k] * v.y;
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      sr[threadIdx.x] += sr[threadIdx.x + h];
      si[threadIdx.x] += si[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) I[p + int64_t(n_ports) * col] = make_double2(sr[0], si[0]);
}

}  // namespace

void port_ring(const Ctx& c, const slim_port& pt, std::vector<int32_t>& edges, std::vector<double>& w) {
  const RWGTable& r = c.rwg;
  const Mesh& m = c.mesh;
  SLIM_REQUIRE(pt.obj >= 0 && pt.obj < r.n_obj, SLIM_E_ARG, "port object out of range");
  double ax[3] = {pt.axis[0], pt.axis[1], pt.axis[2]};
  const double na = std::sqrt(dot3(ax, ax));
  SLIM_REQUIRE(std::isfinite(na) && na > 0 && std::isfinite(pt.radius) && pt.radius > 0, SLIM_E_ARG,
               "port axis must be non-zero and the radius positive");
  for (double& v : ax) v /= na;
  const double tol = 1e-9 * r.mean_edge;
  const size_t first = edges.size();
  std::map<int32_t, int> valence;
  for (int64_t e = r.obj_edge_off[pt.obj]; e < r.obj_edge_off[pt.obj + 1]; ++e) {
    const double* a = &m.xyz[3 * size_t(r.ev[2 * e])];
    const double* b = &m.xyz[3 * size_t(r.ev[2 * e + 1])];
    double da[3], db[3], mid[3];
    for (int k = 0; k < 3; ++k) {
      da[k] = a[k] - pt.point[k];
      db[k] = b[k] - pt.point[k];
      mid[k] = 0.5 * (a[k] + b[k]) - pt.point[k];
    }
    if (std::fabs(dot3(da, ax)) > tol || std::fabs(dot3(db, ax)) > tol) continue;
    if (dot3(mid, mid) > pt.radius * pt.radius) continue;
    // direction in which f_e crosses its edge: in the plane of T+, normal to the edge,
    // away from the free vertex of T+
    const int32_t t = r.tplus[e];
    int loc = 0;
    while (r.tri_edge[3 * t + loc] != e) ++loc;
    const double* f = &m.xyz[3 * size_t(m.tri[3 * t + loc])];
    double tv[3], nu[3];
    for (int k = 0; k < 3; ++k) tv[k] = b[k] - a[k];
    const double lt = std::sqrt(dot3(tv, tv));
    for (int k = 0; k < 3; ++k) {
      tv[k] /= lt;
      nu[k] = 0.5 * (a[k] + b[k]) - f[k];
    }
    const double along = dot3(nu, tv);
    for (int k = 0; k < 3; ++k) nu[k] -= along * tv[k];
    const double ct = dot3(nu, ax) / std::sqrt(dot3(nu, nu));
    SLIM_REQUIRE(std::fabs(ct) >= 0.5, SLIM_E_ARG, "port plane runs inside a face of object " + std::to_string(pt.obj));
    edges.push_back(int32_t(e));
    w.push_back((ct > 0 ? 1.0 : -1.0) * r.len[e]);
    valence[r.ev[2 * e]]++;
    valence[r.ev[2 * e + 1]]++;
  }
  SLIM_REQUIRE(edges.size() > first, SLIM_E_ARG, "no mesh edge of object " + std::to_string(pt.obj) + " in the port plane");
  for (const auto& kv : valence)
    SLIM_REQUIRE(kv.second == 2, SLIM_E_ARG, "the port edges do not form one closed ring");
}

void port_currents(Ctx& c, const std::vector<int32_t>& edges, const std::vector<double>& w,
                   const std::vector<int32_t>& start, const void* X, int n_rhs, double* I, hipStream_t s) {
  const int n_ports = int(start.size()) - 1;
  DevBuf de, dw, ds, dI;
  de.upload(edges);
  dw.upload(w);
  ds.upload(start);
  dI.alloc(size_t(n_ports) * n_rhs * 16);
  hipLaunchKernelGGL(k_port_currents, dim3(unsigned(n_ports), unsigned(n_rhs)), dim3(256), 0, s, de.as<int32_t>(),
                     dw.as<double>(), ds.as<int32_t>(), reinterpret_cast<const double2*>(X), c.rwg.n_e + c.rwg.n_t,
                     n_ports, dI.as<double2>());
  SLIM_HIP(hipGetLastError());
  SLIM_HIP(hipMemcpyAsync(I, dI.p, dI.bytes, hipMemcpyDeviceToHost, s));
  SLIM_HIP(hipStreamSynchronize(s));
}

}  // namespace slim
