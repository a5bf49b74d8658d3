// The library context: host tables and device arenas of one built operator.
#pragma once
#include <memory>

#include "common.hpp"
#include "quad.hpp"

namespace slim {

// AIM grid (eq. (11)): N nodes per axis, spacing h, origin; FFT size 2N.
struct GridDef {
  int N[3] = {0, 0, 0};
  double h[3] = {0, 0, 0};
  double origin[3] = {0, 0, 0};
  int64_t nodes() const { return int64_t(N[0]) * N[1] * N[2]; }
};

// One internal work tile: rows [row0, row0+rows) of the stacked [Z_i; M_i] block.
struct Tile {
  int32_t block, row0, rows, slot;
};

struct Block {
  int64_t off;   // element offset of the 2n x n row-major block in the arena
  int32_t n;     // unknowns of the object
  int32_t e0;    // first global RWG index
};

template <class T> struct Cplx { T x, y; };

// One stored block of the conductor-block preconditioner.
struct PcBlk {
  int64_t off;       // element offset of the n_own x ld complex64 rows
  int64_t ext_off;   // first entry of the block in the gather list
  int64_t row_off;   // first entry of the block in the owned-row list
  int32_t n_ext;     // extended unknowns (columns)
  int32_t ld;        // row length, n_ext rounded up to even
  int32_t n_own;     // stored rows
  int32_t pad;
};

struct Ctx {
  int device = 0;
  std::string last_error;
  bool has_mesh = false, built = false;
  Mesh mesh;
  std::vector<Material> mats;
  RWGTable rwg;
  slim_build_opts opts{};
  slim_layout layout{};
  double freq = 0, omega = 0, k0 = 0;
  cd eps_c_obj;                         // (homogeneous materials: per object below)
  std::vector<cd> kc, epsc;             // per object

  // ---- geometry on the device (build and combine) ----
  DevBuf d_xyz, d_tri, d_cen, d_nrm, d_area, d_diam, d_tri_edge, d_tri_sign, d_len, d_tplus, d_tminus;

  // ---- internal arena (rows of [Z_i; M_i], row-major, hi and lo complex64) ----
  std::vector<Block> blocks;
  DevBuf d_hi, d_lo;                    // Cplx<float>
  DevBuf d_blocks;                      // Block[]
  int64_t arena_elems = 0;
  double gen_seconds = 0.0;             // wall time of the interior-block generation
  int gen_workers = 0;                  // concurrent streams it used for the smaller objects

  // ---- sparse Z~ of the high-frequency form (hf_radius > 0): CSR over all RWG rows,
  //      global columns, hi and lo complex64 values; the arena then holds only M_i ----
  bool hf_sparse = false;
  int64_t z_nnz = 0;
  DevBuf d_zs_ptr, d_zs_col, d_zs_hi, d_zs_lo;

  // ---- work queues of the persistent internal kernel ----
  std::vector<Tile> tiles;              // grouped by slot
  std::vector<int32_t> slot_start;      // slots+1
  DevBuf d_tiles, d_slot_start;         // slot_start: (slots + 1) + (zslots + 1), one range table per phase
  int32_t phase_first[2] = {0, 0};      // tiles of phase 0 (rows of M_i) and phase 1 (rows of Z_i)
  int32_t phase_count[2] = {0, 0};
  bool dynamic = false;                 // dynamic dispatch (scheduling modes 3 and 4)
  DevBuf d_qctr;                        // dispatch counters: GEMV phases 0, 1; block product phases 0, 1;
                                        // FP64 GEMV phase 1 (its own grid)
  int slots = 0;
  int slots_z = 0;                      // workgroups of the launch of the rows of Z_i (0: slots)
  int zslots() const { return slots_z > 0 ? slots_z : slots; }
  // workgroups of the launch of the rows of Z_i in one precision: slots_z is chosen for
  // the mixed path, whose launch runs beside the FFT; the FP64 launch is bound by its
  // arithmetic and latency and takes the M rows' count wherever the queue allows it
  // (dynamic dispatch draws from one list, so any grid serves it)
  int zgrid(bool f64) const { return f64 && dynamic ? std::max(slots, zslots()) : zslots(); }
  int tile_rows = 64;
  int rw_mixed = 8;                     // rows per wave of the mixed internal kernel (4 or 8)
  int sched_mode = 0;
  bool record = false;
  DevBuf d_stamps;                      // 2 x n_tiles uint64 timestamps
  DevBuf d_span;                        // 2 x (slots + zslots) uint64: start and end of every workgroup of both
                                        // launches (graph-path timing)
  std::vector<double> last_stamps;

  // ---- I_x (sparse: the other edges of T+ and T-), per RWG row ----
  DevBuf d_ix_col;                      // 4 n_e int32 (-1 if unused)
  DevBuf d_ix_val;                      // 4 n_e double

  // ---- external: dense (plain mode) ----
  bool plain = false;
  DevBuf d_LA_hi, d_LA_lo, d_Lphi_hi, d_Lphi_lo;   // row-major, hi / lo complex64

  // ---- external: AIM ----
  GridDef grid;
  int near_cheb = 3;
  // projection P (grid-node-major, atomic-free gather)
  DevBuf d_pe_node, d_pe_ptr, d_pe_idx, d_pe_w32, d_pe_w64;   // RWG: (node list, row ptr, basis, 3 weights)
  DevBuf d_pt_node, d_pt_ptr, d_pt_idx, d_pt_w32, d_pt_w64;   // pulses (weights x A_t)
  int64_t n_pe_nodes = 0, n_pt_nodes = 0, nnz_pe = 0, nnz_pt = 0;
  // interpolation W = P^T (basis-major: base node + 27 weights per component)
  DevBuf d_we_base, d_we_w32, d_we_w64, d_wt_base, d_wt_w32, d_wt_w64;
  // Green's function spectrum on the (2N)^3 grid, scaled by 1/(2N)^3
  DevBuf d_ghat64, d_ghat128;           // octant k in [0, N], order [ky][kz][kx]
  DevBuf d_tw64, d_tw128;               // twiddles for each axis length
  // FFT work arrays (4 components)
  DevBuf d_oct_in, d_oct_in32;          // projected sources: complex128 / complex64 (zero off the occupied nodes)
  DevBuf d_oct_out, d_x1, d_x2;         // sized for complex128; complex64 uses the front
  int fft_zsh = 0;                      // log2 of the z planes interleaved per block in d_x2 (0 or 3)
  // layered background: reflected kernels on the lattice [4][2Nz-1][Ny][Nx] (xx, zz, phi, zx radial),
  // their spectra [5][2Nz][Ny+1][Nx+1] (xx, zz, phi, zx, zy; scaled by 1/(2N)^3) and the
  // full-z work array of the layered z step (4 components, sized for complex128)
  bool layered = false;
  double lay_zif = 0.0;
  int lay_nodes = 0;
  DevBuf d_lay_real, d_rhat128, d_rhat64, d_lay;
  DevBuf d_nA_free, d_nP_free;          // free-space near values, kept once a medium changes them
  std::vector<int32_t> h_cidx_e, h_cidx_t;     // stencil centres (host copies)
  std::vector<double> h_w_e, h_w_t;            // stencil weights (host copies)
  // near field
  DevBuf d_nA_ptr, d_nA_col, d_nA_v128, d_nA_v64;
  DevBuf d_nP_ptr, d_nP_col, d_nP_v128, d_nP_v64;     // columns pre-scaled by A_u
  int64_t nnz_A = 0, nnz_P = 0;

  // ---- conductor-block preconditioner ----
  bool pc_built = false;
  std::vector<PcBlk> pc_blocks;
  std::vector<int32_t> pc_ext, pc_own_pos;    // gather list (system indices); owned positions in it
  std::vector<int64_t> pc_ext_ptr, pc_own_ptr;
  DevBuf d_pc, d_pc_ext, d_pc_row, d_pc_blk, d_pc_vin, d_pc_tiles, d_pc_slot_start;
  int pc_slots = 0;
  int64_t pc_entries = 0, pc_cap = 0;
  double pc_seconds = 0.0;
  std::vector<double> pc_cond;                // 1-norm condition number of every block (FP64 inverse)

  // ---- vectors ----
  DevBuf d_x64, d_y64;                  // complex64 copies of x / scratch
  DevBuf d_e, d_g, d_j, d_a, d_phi;     // sized for complex128

  // ---- block of right-hand sides (slim_matvec_block, mixed): workspace grown on demand ----
  DevBuf d_blk_hs, d_blk_h64, d_blk_e, d_blk_j;   // split H planes, complex64 H, e, j (column-major)
  DevBuf d_blk_hoff, d_blk_hpos;                  // per block: start of its H slice; per edge: position
  int64_t blk_ldh = 0;                            // length of a column of a split plane
  int blk_cols = 0;                               // columns the workspace holds

  // ---- graphs ----
  struct GraphKey { int prec; const void* x; void* y; };
  std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs;
  void drop_graphs();
  hipStream_t s_aux = nullptr;
  hipStream_t s_phi = nullptr;          // pulse (phi) path of the product, concurrent with the internal blocks
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipStream_t s_int = nullptr;          // rows of Z_i, concurrent with the projection and convolution of j
  hipEvent_t ev_zfork = nullptr, ev_zjoin = nullptr;

  // ---- per-stage timing ----
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev[6];   // start/end pairs per stage
  size_t prof_used[6] = {0, 0, 0, 0, 0, 0};
  int64_t prof_calls = 0;
  void prof_mark(int stage, hipStream_t s);   // records the next event of the stage
  // graph-path timing: events around each replay on the caller's stream, and the
  // internal kernel's own wall-clock stamps inside the replay
  bool gprof_on = false;
  hipEvent_t gev[2] = {nullptr, nullptr};
  int wall_khz = 0;
  double gprof_ms[4] = {0.0, 0.0, 0.0, 0.0};   // internal (both phases), replay, phase 0, phase 1
  int64_t gprof_calls = 0;

  // ---- cost model ----
  std::vector<float> mlp_params;        // trained FP32 parameters (empty: untrained)
  std::vector<float> mlp_mu, mlp_sd;    // feature standardisation

  ~Ctx();
};

// build.cpp
void build_all(Ctx& c, const slim_build_opts& o);
// aim.cpp
void build_aim(Ctx& c, hipStream_t s);
// kernels.hip
void matvec(Ctx& c, slim_prec prec, const void* x, void* y, void* e_out, void* g_out, void* a_out,
            void* phi_out, hipStream_t s);
void internal_apply(Ctx& c, slim_prec prec, const void* H, void* e, void* g, hipStream_t s, bool h_is_c128);
void matvec_graph(Ctx& c, slim_prec prec, const void* x, void* y, hipStream_t s);
void matvec_block(Ctx& c, slim_prec prec, const void* X, void* Y, int n_rhs, hipStream_t s);
double time_internal(Ctx& c, int reps);   // ms per launch of the mixed internal kernel
double time_product(Ctx& c, int reps);    // ms per mixed product
void launch_cast_c128_to_c64(const void* in, void* out, int64_t n, hipStream_t s);
void launch_cast_c64_to_c128(const void* in, void* out, int64_t n, hipStream_t s);
// rows [row0, 2n) of [Z; M] (column-major n x n inputs) -> hi / lo, row-major, rows padded to even length
void launch_pack_block(const double* Zcm, const double* Mcm, int n, int row0, Cplx<float>* hi, Cplx<float>* lo,
                       hipStream_t s);
// sparse Z~: vals[k] = Z[rows[k] + cols[k] n] (column-major n x n) for k < nnz, hi / lo of
// them, and Z zeroed everywhere else
void launch_z_gather_mask(double* Zcm, int n, const int32_t* rows, const int32_t* cols, int64_t nnz, double* vals,
                          Cplx<float>* hi, Cplx<float>* lo, hipStream_t s);
void launch_add_scaled_ix(double* B, const int32_t* ix_col, const double* ix_val, int e0, int n, double half, hipStream_t s);
void launch_scale(double* M, int64_t n_elems, cd f, hipStream_t s);
void launch_usolve_block(const double* U, int64_t ld, int i0, int nb, double* X, int64_t ldx, int nrhs, hipStream_t s);
void launch_pack_dense(const double* Acm, int64_t rows, int64_t cols, Cplx<float>* hi, Cplx<float>* lo, hipStream_t s);
// fft.hip
void fft_init_twiddles(Ctx& c);
void fft_forward_3d_c128(Ctx& c, double* data_full, hipStream_t s);   // full (2N)^3 in place (build)
// oct_in -> oct_out; layered: free-space kernel plus the reflected dyadic (components
// {0,1,2}, {3} or all four)
void aim_convolve(Ctx& c, bool fp64, int ncomp, hipStream_t s, int comp0 = 0, bool layered = false);
void aim_convolve_layered(Ctx& c, bool fp64, hipStream_t s);   // oct_in -> oct_out, 4 components
// layered.hip
void build_layered(Ctx& c, const slim_medium& m, hipStream_t s);
void layered_gammas(const slim_medium& m, double freq, int64_t n, const double* kr, double* out);   // host only
// ports.cpp: ring edges of a port (appended to edges) and their weights s_m l_m; the
// currents sum_m w_m X[m + col n_sys] of every port (start: n_ports + 1 offsets) into I
void port_ring(const Ctx& c, const slim_port& p, std::vector<int32_t>& edges, std::vector<double>& w);
void port_currents(Ctx& c, const std::vector<int32_t>& edges, const std::vector<double>& w,
                   const std::vector<int32_t>& start, const void* X, int n_rhs, double* I, hipStream_t s);
// mlp.hip: device address of the allocation-free entry point's workspace on the current device
float* noalloc_workspace();
// sched.cpp
void pack_tiles(Ctx& c, int mode);
// precond.hip
void build_precond(Ctx& c, hipStream_t s);
void precond_apply(Ctx& c, const void* v, void* z, hipStream_t s);
void precond_partition(const RWGTable& r, int64_t cap, int overlap, std::vector<int64_t>& ext_ptr,
                       std::vector<int32_t>& ext_idx, std::vector<int64_t>& own_ptr, std::vector<int32_t>& own_pos);
// solve.cpp
slim_status solve_gmres(Ctx& c, const void* b, int scaled_rhs, void* x, const slim_solve_opts& o,
                        slim_solve_info& info, hipStream_t s);

}  // namespace slim

struct slim_ctx {
  slim::Ctx c;
};
