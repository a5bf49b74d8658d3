// Mesh validation and the RWG edge table (Sec. II: RWG basis for J, n x E, n x H).
//
// Every edge of a closed, consistently outward-oriented surface is traversed
// once in each direction by its two triangles.  T+ of the RWG function on an
// edge is the triangle that runs along it from the lower to the higher vertex
// id.  Unknowns are ordered by object, then by (lower, higher) vertex id.
#include <algorithm>
#include <numeric>
#include <unordered_map>

#include "common.hpp"

namespace slim {

namespace {
inline uint64_t edge_key(uint32_t a, uint32_t b) { return (uint64_t(a) << 32) | uint64_t(b); }
}  // namespace

RWGTable build_rwg(const Mesh& m) {
  RWGTable r;
  const int64_t nt = m.n_tri;
  r.n_t = nt;
  r.n_obj = m.n_obj;
  SLIM_REQUIRE(nt > 0, SLIM_E_MESH, "empty mesh");
  for (int64_t t = 0; t < nt; ++t) {
    SLIM_REQUIRE(m.obj[t] >= 0 && m.obj[t] < m.n_obj, SLIM_E_MESH,
                 "object id out of range at triangle " + std::to_string(t));
    SLIM_REQUIRE(t == 0 || m.obj[t] >= m.obj[t - 1], SLIM_E_MESH,
                 "triangles not grouped by object at triangle " + std::to_string(t));
    for (int i = 0; i < 3; ++i)
      SLIM_REQUIRE(m.tri[3 * t + i] >= 0 && m.tri[3 * t + i] < m.n_vert, SLIM_E_MESH,
                   "vertex id out of range at triangle " + std::to_string(t));
  }
  r.area.resize(nt);
  r.normal.resize(3 * nt);
  r.centroid.resize(3 * nt);
  r.diam.resize(nt);
  const double* X = m.xyz.data();
  for (int64_t t = 0; t < nt; ++t) {
    const double* v0 = X + 3 * m.tri[3 * t];
    const double* v1 = X + 3 * m.tri[3 * t + 1];
    const double* v2 = X + 3 * m.tri[3 * t + 2];
    double e1[3], e2[3], c[3];
    for (int k = 0; k < 3; ++k) { e1[k] = v1[k] - v0[k]; e2[k] = v2[k] - v0[k]; }
    c[0] = e1[1] * e2[2] - e1[2] * e2[1];
    c[1] = e1[2] * e2[0] - e1[0] * e2[2];
    c[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double n2 = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    SLIM_REQUIRE(n2 > 0.0, SLIM_E_MESH, "degenerate triangle " + std::to_string(t));
    r.area[t] = 0.5 * n2;
    for (int k = 0; k < 3; ++k) {
      r.normal[3 * t + k] = c[k] / n2;
      r.centroid[3 * t + k] = (v0[k] + v1[k] + v2[k]) / 3.0;
    }
    auto dist = [](const double* a, const double* b) {
      double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
      return std::sqrt(dx * dx + dy * dy + dz * dz);
    };
    r.diam[t] = std::max(std::max(dist(v1, v2), dist(v2, v0)), dist(v0, v1));
  }
  // directed edges: local edge i is opposite local vertex i
  std::unordered_map<uint64_t, int64_t> plus, minus;   // key (lo,hi) -> 3t+i
  plus.reserve(size_t(nt) * 2);
  minus.reserve(size_t(nt) * 2);
  for (int64_t t = 0; t < nt; ++t) {
    for (int i = 0; i < 3; ++i) {
      uint32_t u = m.tri[3 * t + (i + 1) % 3], w = m.tri[3 * t + (i + 2) % 3];
      uint64_t key = edge_key(std::min(u, w), std::max(u, w));
      auto& d = (u < w) ? plus : minus;
      auto ins = d.emplace(key, 3 * t + i);
      SLIM_REQUIRE(ins.second, SLIM_E_MESH,
                   "non-manifold or inconsistently oriented edge (" + std::to_string(std::min(u, w)) +
                       "," + std::to_string(std::max(u, w)) + ") at triangle " + std::to_string(t));
    }
  }
  SLIM_REQUIRE(plus.size() == minus.size(), SLIM_E_MESH, "mesh is not closed");
  struct E { int32_t obj; uint32_t a, b; int64_t p, q; };
  std::vector<E> edges;
  edges.reserve(plus.size());
  for (auto& kv : plus) {
    auto it = minus.find(kv.first);
    SLIM_REQUIRE(it != minus.end(), SLIM_E_MESH,
                 "mesh is not closed at edge (" + std::to_string(kv.first >> 32) + "," +
                     std::to_string(kv.first & 0xffffffffu) + ")");
    int64_t tp = kv.second / 3, tm = it->second / 3;
    SLIM_REQUIRE(m.obj[tp] == m.obj[tm], SLIM_E_MESH, "edge shared by two objects at triangle " + std::to_string(tp));
    edges.push_back({m.obj[tp], uint32_t(kv.first >> 32), uint32_t(kv.first & 0xffffffffu), kv.second, it->second});
  }
  std::sort(edges.begin(), edges.end(), [](const E& x, const E& y) {
    if (x.obj != y.obj) return x.obj < y.obj;
    if (x.a != y.a) return x.a < y.a;
    return x.b < y.b;
  });
  const int64_t ne = int64_t(edges.size());
  r.n_e = ne;
  r.ev.resize(2 * ne);
  r.tplus.resize(ne);
  r.tminus.resize(ne);
  r.len.resize(ne);
  r.tri_edge.assign(3 * nt, -1);
  r.tri_sign.assign(3 * nt, 0);
  double lsum = 0.0;
  for (int64_t n = 0; n < ne; ++n) {
    const E& e = edges[n];
    r.ev[2 * n] = int32_t(e.a);
    r.ev[2 * n + 1] = int32_t(e.b);
    r.tplus[n] = int32_t(e.p / 3);
    r.tminus[n] = int32_t(e.q / 3);
    const double* va = X + 3 * size_t(e.a);
    const double* vb = X + 3 * size_t(e.b);
    double dx = vb[0] - va[0], dy = vb[1] - va[1], dz = vb[2] - va[2];
    r.len[n] = std::sqrt(dx * dx + dy * dy + dz * dz);
    lsum += r.len[n];
    r.tri_edge[e.p] = int32_t(n);
    r.tri_sign[e.p] = 1;
    r.tri_edge[e.q] = int32_t(n);
    r.tri_sign[e.q] = -1;
  }
  r.mean_edge = lsum / double(ne);
  r.obj_edge_off.assign(m.n_obj + 1, 0);
  r.obj_tri_off.assign(m.n_obj + 1, 0);
  for (int64_t n = 0; n < ne; ++n) r.obj_edge_off[edges[n].obj + 1]++;
  for (int64_t t = 0; t < nt; ++t) r.obj_tri_off[m.obj[t] + 1]++;
  for (int i = 0; i < m.n_obj; ++i) {
    r.obj_edge_off[i + 1] += r.obj_edge_off[i];
    r.obj_tri_off[i + 1] += r.obj_tri_off[i];
  }
  for (int i = 0; i < m.n_obj; ++i)
    SLIM_REQUIRE(r.obj_tri_off[i + 1] > r.obj_tri_off[i], SLIM_E_MESH, "object " + std::to_string(i) + " has no triangles");
  return r;
}

}  // namespace slim
