// C ABI entry points (include/slim.h).  Every call catches all exceptions and
// turns them into a status code plus a message kept in the context.
#include <algorithm>
#include <cstring>

#include "ctx.hpp"

using namespace slim;


namespace {

template <class F> slim_status guard(slim_ctx* h, F&& f) {
  if (!h) return SLIM_E_ARG;
  try {
    h->c.last_error.clear();
    return f();
  } catch (const Error& e) {
    h->c.last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    h->c.last_error = "host allocation failed";
    return SLIM_E_OOM;
  } catch (const std::exception& e) {
    h->c.last_error = e.what();
    return SLIM_E_HIP;
  } catch (...) {
    h->c.last_error = "unknown error";
    return SLIM_E_HIP;
  }
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

void slim_default_build_opts(slim_build_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->freq = 10e9;
  o->near_cheb = 3;
  o->n_far = 4;
  o->n_near = 5;
  o->levels = 3;
  o->n_r = 5;
  o->n_t = 6;
  o->q = 0.25;
  o->c_near = 2.0;
  o->sched_mode = 0;
  o->tile_rows = 0;
  o->internal_kernel = 0;
  o->slots = 0;
  o->use_graphs = 1;
  o->precond = 1;
  o->precond_overlap = 2;
  o->precond_cap = 0;
  o->precond_budget = 0;
  o->fft_zblock = 0;
  o->rows_per_wave = 0;
  o->tune_cache = nullptr;
  o->hf_radius = 0.0;
  o->slots_z = 0;
  o->gen_workers = 0;
}

slim_status slim_create(int32_t hip_device, slim_ctx** out) {
  if (!out) return SLIM_E_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return SLIM_E_HIP;
  try {
    slim_ctx* h = new slim_ctx();
    h->c.device = hip_device;
    if (hipSetDevice(hip_device) != hipSuccess) {
      delete h;
      return SLIM_E_HIP;
    }
    // set-up of the allocation-free entry point's workspace on this device (the
    // entry point looks it up itself on a device no context was created on)
    try {
      (void)noalloc_workspace();
    } catch (const Error&) {
    }
    *out = h;
    return SLIM_OK;
  } catch (...) {
    return SLIM_E_OOM;
  }
}

void slim_destroy(slim_ctx* h) {
  if (!h) return;
  (void)hipSetDevice(h->c.device);
  (void)hipDeviceSynchronize();
  delete h;
}

const char* slim_last_error(const slim_ctx* h) { return h ? h->c.last_error.c_str() : "null context"; }

slim_status slim_set_mesh(slim_ctx* h, const double* xyz, int64_t n_vert, const int32_t* tri, int64_t n_tri,
                          const int32_t* obj, int32_t n_obj) {
  return guard(h, [&]() {
    SLIM_REQUIRE(xyz && tri && obj && n_vert > 0 && n_tri > 0 && n_obj > 0, SLIM_E_ARG, "null or empty mesh arrays");
    SLIM_REQUIRE(n_tri < (int64_t(1) << 31) && n_vert < (int64_t(1) << 31), SLIM_E_ARG, "mesh too large for int32 ids");
    Mesh m;
    m.n_vert = n_vert;
    m.n_tri = n_tri;
    m.n_obj = n_obj;
    m.xyz.assign(xyz, xyz + 3 * n_vert);
    m.tri.assign(tri, tri + 3 * n_tri);
    m.obj.assign(obj, obj + n_tri);
    for (double v : m.xyz) SLIM_REQUIRE(std::isfinite(v), SLIM_E_MESH, "non-finite vertex coordinate");
    RWGTable r = build_rwg(m);   // throws SLIM_E_MESH and leaves the context unchanged
    h->c.mesh = std::move(m);
    h->c.rwg = std::move(r);
    h->c.has_mesh = true;
    h->c.built = false;
    h->c.mats.clear();
    return SLIM_OK;
  });
}

slim_status slim_set_materials(slim_ctx* h, const slim_material* per_obj) {
  return guard(h, [&]() {
    SLIM_REQUIRE(h->c.has_mesh, SLIM_E_STATE, "slim_set_mesh must come first");
    std::vector<Material> mats(h->c.mesh.n_obj);
    if (per_obj)
      for (int i = 0; i < h->c.mesh.n_obj; ++i) {
        SLIM_REQUIRE(per_obj[i].sigma >= 0 && per_obj[i].eps_r > 0 && per_obj[i].mu_r > 0, SLIM_E_ARG,
                     "invalid material of object " + std::to_string(i));
        mats[i] = {per_obj[i].sigma, per_obj[i].eps_r, per_obj[i].mu_r};
      }
    h->c.mats = std::move(mats);
    h->c.built = false;
    return SLIM_OK;
  });
}

slim_status slim_build(slim_ctx* h, const slim_build_opts* o) {
  return guard(h, [&]() {
    SLIM_REQUIRE(o, SLIM_E_ARG, "null build options");
    try {
      build_all(h->c, *o);
    } catch (...) {
      h->c.built = false;
      throw;
    }
    return SLIM_OK;
  });
}

slim_status slim_get_layout(const slim_ctx* h, slim_layout* out) {
  if (!h || !out) return SLIM_E_ARG;
  if (!h->c.built) return SLIM_E_STATE;
  *out = h->c.layout;
  return SLIM_OK;
}

slim_status slim_get_rwg(const slim_ctx* h, int32_t* ev, int32_t* tp, int32_t* tm) {
  if (!h) return SLIM_E_ARG;
  if (!h->c.has_mesh) return SLIM_E_STATE;
  const RWGTable& r = h->c.rwg;
  if (ev) std::copy(r.ev.begin(), r.ev.end(), ev);
  if (tp) std::copy(r.tplus.begin(), r.tplus.end(), tp);
  if (tm) std::copy(r.tminus.begin(), r.tminus.end(), tm);
  return SLIM_OK;
}

slim_status slim_matvec(slim_ctx* h, slim_prec prec, const void* x, void* y, void* stream) {
  return slim_matvec_parts(h, prec, x, y, nullptr, nullptr, nullptr, nullptr, stream);
}

slim_status slim_matvec_parts(slim_ctx* h, slim_prec prec, const void* x, void* y, void* e, void* g, void* a, void* phi,
                              void* stream) {
  return guard(h, [&]() {
    SLIM_REQUIRE(h->c.built, SLIM_E_STATE, "operator not built");
    SLIM_REQUIRE(x && y && x != y, SLIM_E_ARG, "x and y must be distinct device buffers");
    SLIM_REQUIRE(prec == SLIM_FP64 || prec == SLIM_MIXED, SLIM_E_ARG, "unknown precision");
    SLIM_HIP(hipSetDevice(h->c.device));
    if (!e && !g && !a && !phi && h->c.opts.use_graphs && !h->c.prof_on) matvec_graph(h->c, prec, x, y, as_stream(stream));
    else matvec(h->c, prec, x, y, e, g, a, phi, as_stream(stream));
    return SLIM_OK;
  });
}

slim_status slim_matvec_block(slim_ctx* h, slim_prec prec, const void* X, void* Y, int32_t n_rhs, void* stream) {
  return guard(h, [&]() {
    SLIM_REQUIRE(h->c.built, SLIM_E_STATE, "operator not built");
    SLIM_REQUIRE(X && Y && X != Y && n_rhs >= 1, SLIM_E_ARG, "X and Y must be distinct device arrays, n_rhs >= 1");
    SLIM_REQUIRE(prec == SLIM_FP64 || prec == SLIM_MIXED, SLIM_E_ARG, "unknown precision");
    SLIM_HIP(hipSetDevice(h->c.device));
    matvec_block(h->c, prec, X, Y, n_rhs, as_stream(stream));
    return SLIM_OK;
  });
}

slim_status slim_internal_apply(slim_ctx* h, slim_prec prec, const void* H, void* e, void* g, double* ms, void* stream) {
  return guard(h, [&]() {
    SLIM_REQUIRE(h->c.built, SLIM_E_STATE, "operator not built");
    SLIM_REQUIRE(H, SLIM_E_ARG, "null H");
    SLIM_HIP(hipSetDevice(h->c.device));
    hipStream_t s = as_stream(stream);
    if (ms) {
      hipEvent_t a, b;
      SLIM_HIP(hipEventCreate(&a));
      SLIM_HIP(hipEventCreate(&b));
      if (prec != SLIM_FP64) launch_cast_c128_to_c64(H, h->c.d_x64.p, h->c.rwg.n_e, s);
      SLIM_HIP(hipEventRecord(a, s));
      internal_apply(h->c, prec, H, e, g, s, true);
      SLIM_HIP(hipEventRecord(b, s));
      SLIM_HIP(hipEventSynchronize(b));
      float t = 0.f;
      SLIM_HIP(hipEventElapsedTime(&t, a, b));
      *ms = t;
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      if (h->c.record) {
        h->c.last_stamps.resize(2 * h->c.tiles.size());
        std::vector<unsigned long long> st(2 * h->c.tiles.size());
        SLIM_HIP(hipMemcpy(st.data(), h->c.d_stamps.p, st.size() * 8, hipMemcpyDeviceToHost));
        for (size_t k = 0; k < st.size(); ++k) h->c.last_stamps[k] = double(st[k]);
      }
    } else {
      internal_apply(h->c, prec, H, e, g, s, true);
    }
    return SLIM_OK;
  });
}

slim_status slim_rhs_planewave(slim_ctx* h, const double khat[3], const double epol[3], void* b, void* stream) {
  return guard(h, [&]() {
    SLIM_REQUIRE(h->c.built, SLIM_E_STATE, "operator not built");
    SLIM_REQUIRE(khat && epol && b, SLIM_E_ARG, "null argument");
    // b1[m] = (1/eta0) int f_m . epol e^{-j k0 khat.r} dS with TRI(4); b2 = 0
    const RWGTable& r = h->c.rwg;
    const Mesh& m = h->c.mesh;
    std::vector<cd> out(r.n_e + r.n_t, cd(0.0));
    std::vector<double> gx = {0.06943184420297371, 0.33000947820757187, 0.6699905217924281, 0.9305681557970262};
    std::vector<double> gw = {0.17392742256872692, 0.3260725774312731, 0.3260725774312731, 0.17392742256872692};
    for (int64_t t = 0; t < r.n_t; ++t) {
      const double* v0 = &m.xyz[3 * size_t(m.tri[3 * t])];
      const double* v1 = &m.xyz[3 * size_t(m.tri[3 * t + 1])];
      const double* v2 = &m.xyz[3 * size_t(m.tri[3 * t + 2])];
      for (int a = 0; a < 4; ++a)
        for (int bq = 0; bq < 4; ++bq) {
          double u = gx[a], v = gx[bq] * (1 - gx[a]), w = 2 * r.area[t] * gw[a] * gw[bq] * (1 - gx[a]);
          double p[3];
          for (int k = 0; k < 3; ++k) p[k] = v0[k] + u * (v1[k] - v0[k]) + v * (v2[k] - v0[k]);
          cd ph = std::exp(cd(0.0, -h->c.k0 * (khat[0] * p[0] + khat[1] * p[1] + khat[2] * p[2])));
          for (int i = 0; i < 3; ++i) {
            const int n = r.tri_edge[3 * t + i];
            const double* pv = &m.xyz[3 * size_t(m.tri[3 * t + i])];
            double cf = r.tri_sign[3 * t + i] * r.len[n] / (2 * r.area[t]);
            double fe = 0.0;
            for (int k = 0; k < 3; ++k) fe += cf * (p[k] - pv[k]) * epol[k];
            out[n] += w * fe * ph / eta0();
          }
        }
    }
    SLIM_HIP(hipMemcpyAsync(b, out.data(), out.size() * 16, hipMemcpyHostToDevice, as_stream(stream)));
    SLIM_HIP(hipStreamSynchronize(as_stream(stream)));
    return SLIM_OK;
  });
}

slim_status slim_rhs_ports(slim_ctx* h, const slim_port* ports, int32_t n_ports, void* B, void* stream) {
  return guard(h, [&]() {
    SLIM_REQUIRE(h->c.built, SLIM_E_STATE, "operator not built");
    SLIM_REQUIRE(ports && B && n_ports >= 1, SLIM_E_ARG, "null or empty port list");
    SLIM_HIP(hipSetDevice(h->c.device));
    const RWGTable& r = h->c.rwg;
    const int64_t nsys = r.n_e + r.n_t;
    std::vector<cd> out(size_t(nsys) * n_ports, cd(0.0));
    for (int p = 0; p < n_ports; ++p) {
      std::vector<int32_t> edges;
      std::vector<double> w;
      port_ring(h->c, ports[p], edges, w);
      for (size_t k = 0; k < edges.size(); ++k) out[size_t(p) * nsys + edges[k]] = cd(w[k] / eta0(), 0.0);
    }
    hipStream_t s = as_stream(stream);
    SLIM_HIP(hipMemcpyAsync(B, out.data(), out.size() * 16, hipMemcpyHostToDevice, s));
    SLIM_HIP(hipStreamSynchronize(s));
    return SLIM_OK;
  });
}

slim_status slim_port_currents(slim_ctx* h, const slim_port* ports, int32_t n_ports, const void* X, int32_t n_rhs,
                               double* I, void* stream) {
  return guard(h, [&]() {
    SLIM_REQUIRE(h->c.built, SLIM_E_STATE, "operator not built");
    SLIM_REQUIRE(ports && X && I && n_ports >= 1 && n_rhs >= 1, SLIM_E_ARG, "null or empty argument");
    SLIM_HIP(hipSetDevice(h->c.device));
    std::vector<int32_t> edges, start(1, 0);
    std::vector<double> w;
    for (int p = 0; p < n_ports; ++p) {
      port_ring(h->c, ports[p], edges, w);
      start.push_back(int32_t(edges.size()));
    }
    port_currents(h->c, edges, w, start, X, n_rhs, I, as_stream(stream));
    return SLIM_OK;
  });
}

slim_status slim_solve(slim_ctx* h, const void* b, int32_t scaled_rhs, void* x, const slim_solve_opts* o,
                       slim_solve_info* info, void* stream) {
  return guard(h, [&]() {
    SLIM_REQUIRE(h->c.built, SLIM_E_STATE, "operator not built");
    SLIM_REQUIRE(b && x && o && b != x, SLIM_E_ARG, "null or aliased argument");
    SLIM_HIP(hipSetDevice(h->c.device));
    slim_solve_info tmp{};
    slim_status st = solve_gmres(h->c, b, scaled_rhs, x, *o, tmp, as_stream(stream));
    if (info) *info = tmp;
    if (st == SLIM_E_NOT_CONVERGED) h->c.last_error = "GMRES did not reach the tolerance";
    return st;
  });
}

slim_status slim_precond_apply(slim_ctx* h, const void* v, void* z, void* stream) {
  return guard(h, [&]() {
    SLIM_REQUIRE(h->c.built, SLIM_E_STATE, "operator not built");
    SLIM_REQUIRE(h->c.pc_built, SLIM_E_STATE, "no preconditioner was built (build option precond = 0)");
    SLIM_REQUIRE(v && z && v != z, SLIM_E_ARG, "null or aliased argument");
    SLIM_HIP(hipSetDevice(h->c.device));
    precond_apply(h->c, v, z, as_stream(stream));
    return SLIM_OK;
  });
}

slim_status slim_get_precond(const slim_ctx* hc, int64_t* n_blocks, int64_t* n_ext, int64_t* n_own, int64_t* ext_ptr,
                             int32_t* ext_idx, int64_t* own_ptr, int32_t* own_pos) {
  if (!hc) return SLIM_E_ARG;
  slim_ctx* h = const_cast<slim_ctx*>(hc);
  return guard(h, [&]() {
    SLIM_REQUIRE(h->c.built, SLIM_E_STATE, "operator not built");
    SLIM_REQUIRE(h->c.pc_built, SLIM_E_STATE, "no preconditioner was built (build option precond = 0)");
    const Ctx& c = h->c;
    if (n_blocks) *n_blocks = int64_t(c.pc_blocks.size());
    if (n_ext) *n_ext = int64_t(c.pc_ext.size());
    if (n_own) *n_own = int64_t(c.pc_own_pos.size());
    if (ext_ptr) std::memcpy(ext_ptr, c.pc_ext_ptr.data(), c.pc_ext_ptr.size() * 8);
    if (ext_idx && !c.pc_ext.empty()) std::memcpy(ext_idx, c.pc_ext.data(), c.pc_ext.size() * 4);
    if (own_ptr) std::memcpy(own_ptr, c.pc_own_ptr.data(), c.pc_own_ptr.size() * 8);
    if (own_pos && !c.pc_own_pos.empty()) std::memcpy(own_pos, c.pc_own_pos.data(), c.pc_own_pos.size() * 4);
    return SLIM_OK;
  });
}

slim_status slim_precond_partition(const double* xyz, int64_t n_vert, const int32_t* tri, int64_t n_tri,
                                   const int32_t* obj, int32_t n_obj, int64_t cap, int32_t overlap, int64_t* n_blocks,
                                   int64_t* n_ext, int64_t* n_own, int64_t* ext_ptr, int32_t* ext_idx, int64_t* own_ptr,
                                   int32_t* own_pos) {
  try {
    if (!xyz || !tri || !obj || n_vert <= 0 || n_tri <= 0 || n_obj <= 0 || overlap < 0) return SLIM_E_ARG;
    if (n_tri >= (int64_t(1) << 31) || n_vert >= (int64_t(1) << 31)) return SLIM_E_ARG;
    Mesh m;
    m.n_vert = n_vert;
    m.n_tri = n_tri;
    m.n_obj = n_obj;
    m.xyz.assign(xyz, xyz + 3 * n_vert);
    m.tri.assign(tri, tri + 3 * n_tri);
    m.obj.assign(obj, obj + n_tri);
    for (double v : m.xyz)
      if (!std::isfinite(v)) return SLIM_E_MESH;
    const RWGTable r = build_rwg(m);
    std::vector<int64_t> ep, op;
    std::vector<int32_t> ei, oi;
    precond_partition(r, cap, overlap, ep, ei, op, oi);
    if (n_blocks) *n_blocks = int64_t(ep.size()) - 1;
    if (n_ext) *n_ext = int64_t(ei.size());
    if (n_own) *n_own = int64_t(oi.size());
    if (ext_ptr) std::memcpy(ext_ptr, ep.data(), ep.size() * 8);
    if (ext_idx && !ei.empty()) std::memcpy(ext_idx, ei.data(), ei.size() * 4);
    if (own_ptr) std::memcpy(own_ptr, op.data(), op.size() * 8);
    if (own_pos && !oi.empty()) std::memcpy(own_pos, oi.data(), oi.size() * 4);
    return SLIM_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (...) {
    return SLIM_E_HIP;
  }
}

slim_status slim_aim_convolve(slim_ctx* h, slim_prec prec, const void* src, void* dst, int32_t ncomp, void* stream) {
  return guard(h, [&]() {
    SLIM_REQUIRE(h->c.built && !h->c.plain, SLIM_E_STATE, "no AIM operator built");
    SLIM_REQUIRE(src && dst && ncomp >= 1 && ncomp <= 4, SLIM_E_ARG, "bad arguments");
    SLIM_HIP(hipSetDevice(h->c.device));
    hipStream_t s = as_stream(stream);
    const int64_t n = ncomp * h->c.grid.nodes();
    const bool f64 = prec == SLIM_FP64;
    void* in = f64 ? h->c.d_oct_in.p : h->c.d_oct_in32.p;
    if (f64) SLIM_HIP(hipMemcpyAsync(in, src, size_t(n) * 16, hipMemcpyDeviceToDevice, s));
    else launch_cast_c128_to_c64(src, in, n, s);
    aim_convolve(h->c, f64, ncomp, s);
    if (f64) SLIM_HIP(hipMemcpyAsync(dst, h->c.d_oct_out.p, size_t(n) * 16, hipMemcpyDeviceToDevice, s));
    else launch_cast_c64_to_c128(h->c.d_oct_out.p, dst, n, s);
    // the projection buffers must stay zero off the occupied nodes
    SLIM_HIP(hipMemsetAsync(in, 0, size_t(4 * h->c.grid.nodes()) * (f64 ? 16 : 8), s));
    SLIM_HIP(hipStreamSynchronize(s));
    return SLIM_OK;
  });
}

slim_status slim_set_medium(slim_ctx* h, const slim_medium* m) {
  return guard(h, [&]() {
    SLIM_REQUIRE(m, SLIM_E_ARG, "null medium");
    SLIM_HIP(hipSetDevice(h->c.device));
    // build_layered validates every argument before it changes any state
    build_layered(h->c, *m, h->c.s_aux);
    return SLIM_OK;
  });
}

slim_status slim_aim_convolve_layered(slim_ctx* h, slim_prec prec, const void* src, void* dst, void* stream) {
  return guard(h, [&]() {
    SLIM_REQUIRE(h->c.built && !h->c.plain, SLIM_E_STATE, "no AIM operator built");
    SLIM_REQUIRE(h->c.layered, SLIM_E_STATE, "no layered medium set");
    SLIM_REQUIRE(src && dst, SLIM_E_ARG, "bad arguments");
    SLIM_HIP(hipSetDevice(h->c.device));
    hipStream_t s = as_stream(stream);
    const int64_t n = 4 * h->c.grid.nodes();
    const bool f64 = prec == SLIM_FP64;
    void* in = f64 ? h->c.d_oct_in.p : h->c.d_oct_in32.p;
    if (f64) SLIM_HIP(hipMemcpyAsync(in, src, size_t(n) * 16, hipMemcpyDeviceToDevice, s));
    else launch_cast_c128_to_c64(src, in, n, s);
    aim_convolve_layered(h->c, f64, s);
    if (f64) SLIM_HIP(hipMemcpyAsync(dst, h->c.d_oct_out.p, size_t(n) * 16, hipMemcpyDeviceToDevice, s));
    else launch_cast_c64_to_c128(h->c.d_oct_out.p, dst, n, s);
    // the projection buffers must stay zero off the occupied nodes
    SLIM_HIP(hipMemsetAsync(in, 0, size_t(n) * (f64 ? 16 : 8), s));
    SLIM_HIP(hipStreamSynchronize(s));
    return SLIM_OK;
  });
}

slim_status slim_layered_gammas(const slim_medium* m, double freq, int64_t n, const double* kr, double* out) {
  if (!m) return SLIM_E_ARG;
  try {
    layered_gammas(*m, freq, n, kr, out);
    return SLIM_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (...) {
    return SLIM_E_ARG;
  }
}

slim_status slim_get_layered_kernels(const slim_ctx* h, double* out) {
  if (!h) return SLIM_E_ARG;
  if (!h->c.layered) return SLIM_E_STATE;
  if (!out) return SLIM_E_ARG;
  if (hipSetDevice(h->c.device) != hipSuccess) return SLIM_E_HIP;
  if (hipMemcpy(out, h->c.d_lay_real.p, h->c.d_lay_real.bytes, hipMemcpyDeviceToHost) != hipSuccess) return SLIM_E_HIP;
  return SLIM_OK;
}

slim_status slim_get_aim(const slim_ctx* h, int32_t* ce, double* we, int32_t* ct, double* wt) {
  if (!h) return SLIM_E_ARG;
  if (!h->c.built || h->c.plain) return SLIM_E_STATE;
  if (ce) std::copy(h->c.h_cidx_e.begin(), h->c.h_cidx_e.end(), ce);
  if (we) std::copy(h->c.h_w_e.begin(), h->c.h_w_e.end(), we);
  if (ct) std::copy(h->c.h_cidx_t.begin(), h->c.h_cidx_t.end(), ct);
  if (wt) std::copy(h->c.h_w_t.begin(), h->c.h_w_t.end(), wt);
  return SLIM_OK;
}

slim_status slim_get_near(const slim_ctx* hc, int32_t which, int64_t* ptr, int32_t* col, double* val) {
  if (!hc) return SLIM_E_ARG;
  slim_ctx* h = const_cast<slim_ctx*>(hc);
  return guard(h, [&]() {
    SLIM_REQUIRE(h->c.built && !h->c.plain, SLIM_E_STATE, "no AIM operator built");
    SLIM_REQUIRE(which == 0 || which == 1, SLIM_E_ARG, "which must be 0 or 1");
    const int64_t rows = which == 0 ? h->c.rwg.n_e : h->c.rwg.n_t;
    const int64_t nnz = which == 0 ? h->c.nnz_A : h->c.nnz_P;
    if (ptr) SLIM_HIP(hipMemcpy(ptr, (which == 0 ? h->c.d_nA_ptr : h->c.d_nP_ptr).p, size_t(rows + 1) * 8, hipMemcpyDeviceToHost));
    if (col) SLIM_HIP(hipMemcpy(col, (which == 0 ? h->c.d_nA_col : h->c.d_nP_col).p, size_t(nnz) * 4, hipMemcpyDeviceToHost));
    if (val) SLIM_HIP(hipMemcpy(val, (which == 0 ? h->c.d_nA_v128 : h->c.d_nP_v128).p, size_t(nnz) * 16, hipMemcpyDeviceToHost));
    return SLIM_OK;
  });
}

slim_status slim_profile(slim_ctx* h, int32_t on) {
  return guard(h, [&]() {
    SLIM_REQUIRE(on >= 0 && on <= 2, SLIM_E_ARG, "profile mode must be 0, 1 or 2");
    const bool graph = on == 2;
    if (graph != h->c.gprof_on) h->c.drop_graphs();   // the event nodes are part of the captured product
    if (graph)
      for (hipEvent_t& e : h->c.gev)
        if (!e) SLIM_HIP(hipEventCreate(&e));
    h->c.prof_on = on == 1;
    h->c.gprof_on = graph;
    for (auto& u : h->c.prof_used) u = 0;
    h->c.prof_calls = 0;
    for (double& v : h->c.gprof_ms) v = 0.0;
    h->c.gprof_calls = 0;
    return SLIM_OK;
  });
}

slim_status slim_profile_read(slim_ctx* h, double* ms, int64_t* n_matvec) {
  return guard(h, [&]() {
    SLIM_REQUIRE(ms, SLIM_E_ARG, "null output");
    if (h->c.gprof_on) {
      for (int st = 0; st < 6; ++st) ms[st] = 0.0;
      for (int k = 0; k < 4; ++k) ms[k] = h->c.gprof_ms[k];
      if (n_matvec) *n_matvec = h->c.gprof_calls;
      return SLIM_OK;
    }
    for (int st = 0; st < 6; ++st) {
      double tot = 0.0;
      const size_t used = h->c.prof_used[st];
      for (size_t k = 0; k + 1 < used; k += 2) {
        SLIM_HIP(hipEventSynchronize(h->c.prof_ev[st][k + 1]));
        float t = 0.f;
        SLIM_HIP(hipEventElapsedTime(&t, h->c.prof_ev[st][k], h->c.prof_ev[st][k + 1]));
        tot += t;
      }
      ms[st] = tot;
    }
    if (n_matvec) *n_matvec = h->c.prof_calls;
    return SLIM_OK;
  });
}

slim_status slim_sched_record(slim_ctx* h, int32_t on) {
  return guard(h, [&]() {
    h->c.record = on != 0;
    return SLIM_OK;
  });
}

slim_status slim_sched_tiles(slim_ctx* h, double* out, int64_t* n_tiles) {
  return guard(h, [&]() {
    SLIM_REQUIRE(n_tiles, SLIM_E_ARG, "null count");
    SLIM_REQUIRE(h->c.built, SLIM_E_STATE, "operator not built");
    const int64_t n = int64_t(h->c.tiles.size());
    const int64_t cap = *n_tiles;
    *n_tiles = n;
    if (!out) return SLIM_OK;
    SLIM_REQUIRE(cap >= n, SLIM_E_ARG, "tile buffer too small");
    for (int64_t k = 0; k < n; ++k) {
      const Tile& t = h->c.tiles[k];
      out[7 * k] = t.block;
      out[7 * k + 1] = t.row0;
      out[7 * k + 2] = t.rows;
      out[7 * k + 3] = h->c.blocks[t.block].n;
      out[7 * k + 4] = t.slot;
      const bool have = int64_t(h->c.last_stamps.size()) == 2 * n;
      out[7 * k + 5] = have ? h->c.last_stamps[2 * k] : 0.0;
      out[7 * k + 6] = have ? h->c.last_stamps[2 * k + 1] : 0.0;
    }
    return SLIM_OK;
  });
}

slim_status slim_sched_set_mode(slim_ctx* h, int32_t mode) {
  return guard(h, [&]() {
    SLIM_REQUIRE(h->c.built, SLIM_E_STATE, "operator not built");
    SLIM_REQUIRE(mode >= 0 && mode <= 4, SLIM_E_ARG, "unknown scheduling mode");
    SLIM_REQUIRE((mode != 1 && mode != 4) || !h->c.mlp_params.empty(), SLIM_E_STATE, "cost model not trained");
    pack_tiles(h->c, mode);
    h->c.last_stamps.clear();
    h->c.layout.n_tiles = int64_t(h->c.tiles.size());
    return SLIM_OK;
  });
}

slim_status slim_sched_set_shape(slim_ctx* h, int32_t slots, int32_t slots_z) {
  return guard(h, [&]() {
    SLIM_REQUIRE(h->c.built, SLIM_E_STATE, "operator not built");
    SLIM_REQUIRE(slots > 0 && slots <= (1 << 16), SLIM_E_ARG, "slots must be in [1, 65536]");
    SLIM_REQUIRE(slots_z >= 0 && slots_z <= (1 << 16), SLIM_E_ARG, "slots_z must be in [0, 65536]");
    h->c.slots = slots;
    h->c.slots_z = slots_z;
    pack_tiles(h->c, h->c.sched_mode);
    h->c.last_stamps.clear();
    h->c.layout.n_tiles = int64_t(h->c.tiles.size());
    h->c.layout.slots = h->c.slots;
    h->c.layout.slots_z = h->c.zslots();
    return SLIM_OK;
  });
}

}  // extern "C"
