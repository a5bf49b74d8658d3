/*
 * slim.h -- C ABI of the MI355X library for the system matrix-vector product
 * of the SLIM surface-integral formulation for lossy conductors and the GMRES
 * solve built on it (Marek, Sharma, Triverio, "A Parallel Boundary Element
 * Method for the Electromagnetic Analysis of Large Structures With Lossy
 * Conductors").
 *
 * The operator is eq. (7) with C of eq. (8):
 *
 *   [ j k0 L_A + C           D^T L_phi B ] [ H      ]   [ E_inc / eta0 ]
 *   [ F D (I - Y_eq Z)       j k0 I      ] [ c0 rho ] = [ 0            ]
 *
 * with Z = diag(Z_i) (eq. (4), (9)), Y_eq = diag(Y_eq,i) (eq. (5), (10)),
 * L_A, L_phi applied through the adaptive integral method of eq. (11)
 * (L_NR + W H P) or, with grid = {0,0,0}, as dense matrices.
 *
 * Conventions shared by every entry point
 *  - Lengths in metres, SI units, time dependence e^{j omega t}.
 *  - Vectors at the ABI are complex128, interleaved (re, im), on the device.
 *    A system vector is [H (n_e RWG coefficients of n x H); c0 rho (n_t
 *    pulse coefficients)], n_sys = n_e + n_t.  RWG unknowns are ordered
 *    object by object and, inside an object, by (lower vertex id, higher
 *    vertex id) of the edge; the triangle order is the caller's.
 *  - RWG f_n = l/(2A+) (r - p+) on T+ (the triangle whose vertex cycle runs
 *    along the edge from the lower to the higher vertex id), l/(2A-) (p- - r)
 *    on T-.  D[T+,n] = +l_n, D[T-,n] = -l_n, B = diag(A_t), F = -diag(1/A_t),
 *    I_x[m,n] = int (n x f_m) . f_n.
 *  - Host arrays passed in are copied before the call returns; the caller
 *    keeps ownership.  Device buffers passed in (x, y, b, ...) belong to the
 *    caller; the library never frees or retains them.  The library owns
 *    every allocation it makes and releases it in slim_destroy.
 *  - `stream` is a hipStream_t (NULL = default stream).  slim_matvec only
 *    enqueues work; slim_solve and slim_build return after completion.
 *  - Every entry point returns a slim_status and never throws.  On failure
 *    slim_last_error() describes the cause (valid until the next call on the
 *    same context).  A failed set_* call leaves the context unchanged; a failed
 *    build leaves it unbuilt.  One context per host thread.
 */
#ifndef SLIM_H
#define SLIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct slim_ctx slim_ctx;

typedef enum {
  SLIM_OK = 0,
  SLIM_E_ARG = 1,           /* invalid argument (null pointer, size, option)          */
  SLIM_E_MESH = 2,          /* not closed / not manifold / degenerate / bad object id */
  SLIM_E_STATE = 3,         /* call out of order (e.g. matvec before build)           */
  SLIM_E_OOM = 4,           /* device memory budget or allocation exceeded            */
  SLIM_E_HIP = 5,           /* HIP / rocSOLVER / rocBLAS runtime error                */
  SLIM_E_NUMERIC = 6,       /* NaN / Inf or breakdown                                 */
  SLIM_E_NOT_CONVERGED = 7, /* GMRES stopped at max_iter; best iterate returned       */
  SLIM_E_UNSUPPORTED = 8
} slim_status;

/* Precision of the operator applied by slim_matvec / used inside slim_solve.
 * SLIM_FP64: FP64 arithmetic; internal blocks read as hi + lo complex64 pairs
 *            (a 48-bit significand, the same bytes as complex128), grids,
 *            near field and vectors complex128.
 * SLIM_MIXED: internal blocks from the hi complex64 part with FP32
 *            accumulation, complex64 FFT convolution and near field, FP32
 *            stencil weights.                                                */
typedef enum { SLIM_FP64 = 0, SLIM_MIXED = 1 } slim_prec;

typedef struct {
  double sigma;   /* S/m   (copper 5.8e7) */
  double eps_r;
  double mu_r;
} slim_material;

typedef struct {
  double freq;          /* Hz                                                     */
  int32_t grid[3];      /* AIM grid nodes per axis; {0,0,0}: dense L_A, L_phi     */
  int32_t near_cheb;    /* near zone: stencil centres within this Chebyshev index
                           distance (3)                                           */
  /* triangle-pair quadrature (both rules are described in the library source):
     far TRI(n_far)^2; near: TRI(n_near) outer x polar rule (levels, q, n_r, n_t);
     near when the centroid distance < c_near * max triangle diameter            */
  int32_t n_far, n_near, levels, n_r, n_t;
  double q, c_near;
  int32_t sched_mode;     /* 0 = LPT on flop counts, 1 = MLP cost model, 2 = naive */
  int32_t tile_rows;      /* row-panel height of internal tiles (0 = autotune)     */
  int32_t internal_kernel;/* mixed internal GEMV: 0 = FP32 FMA (the only one built;
                             any other value is SLIM_E_UNSUPPORTED)                 */
  int32_t slots;          /* persistent workgroups of the internal kernel (0 = auto) */
  int64_t mem_budget;     /* bytes of device memory the build may use (0 = no cap)  */
  int32_t verbose;
  int32_t use_graphs;     /* slim_matvec replays one captured hipGraph per (prec, x, y) */
  /* Conductor-block preconditioner of slim_solve (a reading of the constraint
     preconditioner the paper uses in Sec. III-E, whose definition the paper does not give):
     block Jacobi over conductors on the row-equilibrated system S A.  Each block
     is S A restricted to one conductor's RWG edges and triangles, inverted in
     FP64 and stored as complex64.  A conductor with more than precond_cap
     unknowns is cut by recursive coordinate bisection of its triangle
     centroids.  Each part is grown by max(precond_overlap, 1) rings of
     edge-adjacent triangles; its extended block holds those triangles and the
     edges with both triangles among them (no current crosses a cut), and it
     keeps its own rows of that block's inverse (restricted additive Schwarz).
     An edge belongs to the part of its T+.  */
  int32_t precond;        /* 1 = build it (default), 0 = none                        */
  int32_t precond_overlap;/* triangle rings added to a part of a cut conductor (2)     */
  int64_t precond_cap;    /* max unknowns per block; 0 = choose the largest cap whose
                             blocks fit precond_budget                                */
  int64_t precond_budget; /* bytes for the stored blocks and their build buffers;
                             0 = the free device memory after the rest of the build,
                             less room for the solver's Krylov vectors               */
  /* Kernel shapes.  With slots = 0 the build times the whole mixed product for every
     combination of the values marked "auto" and keeps the fastest (autotuning). */
  int32_t fft_zblock;     /* z planes interleaved row by row per block in the FFT
                             work array between the y and z passes: B = 1 (plain
                             [z][y][x]) or a power of two up to 64 and up to Nz
                             ([z/B][y][z%B][x]); 0 = auto (tuned over 1 and 8)     */
  int32_t rows_per_wave;  /* rows of [Z_i; M_i] one wave of the mixed internal kernel
                             sweeps together: 4 or 8; 0 = auto (the FP64 kernel,
                             which reads hi + lo, always sweeps two)               */
  const char* tune_cache; /* path of a text file of autotuning results keyed by
                             (kernel, shape, gfx950), read before and appended after
                             tuning; NULL = no cache                               */
  /* Sparse interior operators at high frequency (Sec. III-A, point 3: with a small
     skin depth L_kc and K_kc are treated as sparse by ignoring physically distant
     interactions).  hf_radius > 0 (metres): the conductor-kernel operators L_kc, K_kc
     of eq. (4) are summed over the triangle pairs whose centroids are at most
     hf_radius apart (squared distance dx*dx + dy*dy + dz*dz <= r*r in FP64), Z~ =
     -1/(j w eps_c) L~^-1 (K~ + I_x/2) is formed by an FP64 LU, and the product applies
     it as a sparse matrix kept on the RWG pairs that share such a triangle pair
     (entries elsewhere dropped); M_i = Y_eq,i Z~_i (Y_eq dense).  The internal arena
     then holds only the M_i rows.  0 = dense interior operators (default).  The
     conductor-block preconditioner is not built in this mode (precond must be 0,
     else SLIM_E_UNSUPPORTED).                                                       */
  double hf_radius;
  int32_t slots_z;        /* with slots > 0: persistent workgroups of the launch of the
                             rows of Z_i (0 = slots); ignored when slots = 0 (tuned)  */
  int32_t gen_workers;    /* concurrent streams (each driven by a host thread of its
                             own) of the interior-block generation, eq. (4)-(6): the
                             objects go out in decreasing size, each to the first free
                             worker; objects whose FP64 work buffers (3 n_i^2 x 16 bytes)
                             do not fit the free memory once per worker go first, one
                             at a time.  0 = 8; SLIM_E_ARG below 0 or above 64.      */
} slim_build_opts;

/* Fill `o` with the defaults used by the tests (near_cheb 3, n_far 4, n_near 5,
 * levels 3, q 0.25, n_r 5, n_t 6, c_near 2, LPT, autotuned slot count, plane
 * z block and rows per wave, graphs on, no tuning cache).
 * Autotuning (slots = 0) times the whole mixed product for 2, 4 and 8 persistent
 * internal workgroups per compute unit, times the "auto" kernel shapes, times the
 * workgroups of the launch of the rows of Z_i (as many, or, under dynamic dispatch
 * (sched_mode 3 or 4), one per compute unit),
 * at build time and keeps the fastest.  A tuning cache entry for the same shape
 * skips the timing.  With slots > 0 nothing is timed: auto shapes take 64 and 8,
 * and both launches use `slots` workgroups.                                      */
void slim_default_build_opts(slim_build_opts* o);

typedef struct {
  int64_t n_e, n_t, n_sys;
  int32_t n_obj;
  int32_t grid[3];
  double grid_h[3], grid_origin[3];
  int64_t nnz_near_A, nnz_near_phi;    /* near-field CSR non-zeros               */
  int64_t internal_entries;            /* dense internal entries: sum_i 2 n_i^2
                                          (sum_i n_i^2, the M_i rows, with hf_radius) */
  int64_t n_tiles;                     /* internal work-queue tiles              */
  int32_t slots;
  int32_t tile_rows;
  double mean_edge;                    /* h of the row scaling used by slim_solve */
  double build_seconds;
  int64_t device_bytes;                /* device memory held by the context      */
  int64_t precond_blocks;              /* preconditioner blocks (0: none built)   */
  int64_t precond_entries;             /* stored complex64 entries (rows x ext)   */
  int64_t precond_cap;                 /* cap in effect (0: every conductor whole) */
  int32_t fft_zblock;                  /* kernel shapes in effect (tuned or given) */
  int32_t rows_per_wave;               /* of the mixed internal kernel               */
  int64_t z_nnz;                       /* stored entries of the sparse Z~ (hf_radius > 0),
                                          0 with dense interior operators           */
  int32_t slots_z;                     /* persistent workgroups of the launch of the rows of
                                          Z_i (tuned with the slot count; it runs beside the
                                          projection and FFT of j)                   */
  int32_t interior_workers;            /* streams the interior-block generation used   */
  double interior_seconds;             /* its wall time (part of build_seconds)        */
} slim_layout;

typedef struct {
  double tol;          /* relative residual of the row-equilibrated system        */
  int32_t restart;     /* GMRES(m)                                                 */
  int32_t max_iter;    /* total inner iterations                                   */
  slim_prec prec;      /* FP64: plain GMRES; MIXED: GMRES-IR (FP64 outer residual) */
  double inner_tol;    /* MIXED: relative tolerance of each inner solve            */
  int32_t max_outer;
  int32_t use_precond; /* 1: right-precondition with the conductor blocks (flexible
                          GMRES, the preconditioned basis is kept) if they were built */
} slim_solve_opts;

typedef struct {
  int32_t iterations, outer_steps;
  double rel_residual;        /* final true residual (FP64 operator)              */
  double seconds, matvec_seconds;
  int32_t n_matvec_fp64, n_matvec_mixed;
  int32_t n_precond;          /* preconditioner applications                     */
} slim_solve_info;

/* --- context ----------------------------------------------------------- */
slim_status slim_create(int32_t hip_device, slim_ctx** out);
void slim_destroy(slim_ctx* ctx);                       /* NULL-safe */
const char* slim_last_error(const slim_ctx* ctx);

/* --- problem ----------------------------------------------------------- */
/* Closed, outward-oriented triangle surfaces, one per object (Sec. II).
 * xyz: n_vert x 3 doubles; tri: n_tri x 3 vertex ids; obj_of_tri: n_tri ids in
 * [0, n_obj), non-decreasing.  SLIM_E_MESH names the offending triangle/edge. */
slim_status slim_set_mesh(slim_ctx* ctx, const double* xyz, int64_t n_vert,
                          const int32_t* tri, int64_t n_tri,
                          const int32_t* obj_of_tri, int32_t n_obj);
/* Per-object material (NULL: copper, sigma = 5.8e7, eps_r = mu_r = 1) in a
 * homogeneous free-space background (the layer l of eq. (5) is free space). */
slim_status slim_set_materials(slim_ctx* ctx, const slim_material* per_obj);

/* Operator build (eq. (4)-(6), (11)): RWG table, AIM grid, stencils, near
 * field with precorrection, Green's function spectrum, per-object L, K, FP64
 * LU, explicit Z_i and M_i = Y_eq,i Z_i, task packing, autotuning, graphs. */
slim_status slim_build(slim_ctx* ctx, const slim_build_opts* opts);
slim_status slim_get_layout(const slim_ctx* ctx, slim_layout* out);
/* Host copies of the RWG table: edge_v (2 n_e: lower, higher vertex id),
 * tplus, tminus (n_e each).  Any pointer may be NULL. */
slim_status slim_get_rwg(const slim_ctx* ctx, int32_t* edge_v, int32_t* tplus, int32_t* tminus);

/* --- hot path -------------------------------------------------------------- */
/* y = A x (eq. (7)-(8)); x, y: n_sys complex128 device vectors, no aliasing. */
slim_status slim_matvec(slim_ctx* ctx, slim_prec prec, const void* x_dev, void* y_dev, void* stream);
/* Same product and its intermediate vectors (complex128 device buffers, any
 * may be NULL): e = Z H, g = M H, a = L_A j (n_e each), phi = L_phi B c0rho (n_t). */
slim_status slim_matvec_parts(slim_ctx* ctx, slim_prec prec, const void* x_dev, void* y_dev,
                              void* e_dev, void* g_dev, void* a_dev, void* phi_dev, void* stream);
/* Y = A X for a block of n_rhs right-hand sides (eq. (7)-(8) applied to every
 * column).  X, Y: column-major n_sys x n_rhs complex128 device arrays (leading
 * dimension n_sys), no aliasing, n_rhs >= 1.
 *   SLIM_MIXED: the internal blocks of up to 64 columns at a time on the matrix
 *   cores (v_mfma_f32_16x16x32_bf16): every complex64 entry of [Z_i; M_i] and of
 *   H is split into two BF16 terms, v = v_hi + v_lo, and a b is taken as
 *   a_hi b_hi + a_hi b_lo + a_lo b_hi with FP32 accumulation (about 2^-16 of |a b|
 *   per product); the external part then runs column by column.
 *   SLIM_FP64: every column through the single-column FP64 path.
 * Enqueues on `stream`; the first call (and a call with more columns than before)
 * grows a workspace of about (24 n_e + 8 (n_e + 40 n_obj)) bytes per column. */
slim_status slim_matvec_block(slim_ctx* ctx, slim_prec prec, const void* X_dev, void* Y_dev, int32_t n_rhs,
                              void* stream);
/* Internal part only (eq. (4)-(6) applied blockwise): e = Z H, g = M H.  The
 * internal kernel's makespan (persistent launch) is returned in *ms if non-NULL
 * (synchronous when ms != NULL). */
slim_status slim_internal_apply(slim_ctx* ctx, slim_prec prec, const void* H_dev, void* e_dev,
                                void* g_dev, double* ms, void* stream);

/* AIM pieces on their own, for checks against an independent implementation.
 * slim_aim_convolve: grid convolution H of eq. (11) of ncomp (1..4) complex128
 *   source grids (ncomp x Nx Ny Nz, node order x fastest) into potentials.
 * slim_get_aim: host copies of the stencil centres (3 int32 per basis, node
 *   index) and weights (RWG: 3 x 27 doubles, component-major; pulse: 27).
 * slim_get_near: host copy of the near-field CSR of L_A,NR (which = 0,
 *   n_e rows) or L_phi,NR (which = 1, n_t rows, each column u already scaled by
 *   A_u): ptr (rows+1 int64), col (nnz int32), val (2 nnz doubles).  Any
 *   pointer may be NULL. */
slim_status slim_aim_convolve(slim_ctx* ctx, slim_prec prec, const void* src_dev, void* dst_dev, int32_t ncomp,
                              void* stream);
slim_status slim_get_aim(const slim_ctx* ctx, int32_t* cidx_e, double* w_e, int32_t* cidx_t, double* w_t);

/* --- layered background medium (Sec. II: L_A,m and L_phi,m with the multilayered
 * Green's function; the substrates of Table I) --------------------------------
 * The conductors and every AIM grid node lie in air above the plane
 * z = z_interface.  Below it, n_layers layers are listed top-down; the stack
 * ends in a PEC ground (bottom_pec = 1) or in a half-space (bottom_eps_r,
 * bottom_sigma).  Conductivities are in S/m and thicknesses in metres. */
typedef struct slim_layer {
  double thickness;
  double eps_r;
  double sigma;
} slim_layer;

typedef struct slim_medium {
  double z_interface;
  int32_t n_layers;
  int32_t bottom_pec;
  const slim_layer* layers;   /* host array of n_layers entries, copied */
  double bottom_eps_r;
  double bottom_sigma;
} slim_medium;

/* slim_set_medium: builds the reflected grid kernels of the built AIM grid at
 * the build frequency.  Their spectra are then used by
 * slim_aim_convolve_layered.
 *   Each kernel is a Sommerfeld integral of the stack's TL reflection
 *   coefficients, in FP64.  It is evaluated on the device at every in-plane
 *   lattice offset and every z + z' lattice sum.
 *   The kernels: the xx = yy entry, the zz entry and the scalar kernel, all
 *   even; and the radial factor of zx, so that G_zx = (x - x')/rho times it,
 *   G_zy = (y - y')/rho times it, and G_xz = -G_zx, G_yz = -G_zy.
 *   Normalised by mu0 and 1/eps0, like the free-space g = e^{-jk0R}/(4 pi R).
 * Errors:
 *   SLIM_E_STATE: no AIM operator built.
 *   SLIM_E_ARG: bad layer data, or the grid reaches the interface.
 *   SLIM_E_UNSUPPORTED: the grid is too large electrically for the
 *   quadrature path, or too large against the gap between its lowest plane
 *   and the interface (more than 4M path nodes or 4000 near-field table
 *   steps per axis).
 * Replaces any earlier medium.  A STATE or ARG error leaves the context
 * unchanged.  A later failure (UNSUPPORTED, OOM, HIP) leaves it without a
 * medium, with its free-space near field; if even those values cannot be
 * restored, the context is left unbuilt (products then return SLIM_E_STATE).
 * slim_build always starts again in free space: a medium does not survive a
 * rebuild and must be set again.
 *
 * slim_aim_convolve_layered: the four grid components (x, y, z current and
 *   charge; 4 x Nx Ny Nz complex128 device arrays, node order x fastest),
 *   convolved with the free-space kernel plus the reflected dyadic.  The
 *   reflected part is a convolution in x and y and a correlation in z:
 *     Phi_x = (g + xx) * S_x + G_xz * S_z,
 *     Phi_y = (g + xx) * S_y + G_yz * S_z,
 *     Phi_z = G_zx * S_x + G_zy * S_y + (g + zz) * S_z,
 *     Phi_rho = (g + phi) * S_rho.
 *   SLIM_E_STATE without a medium.
 *
 * slim_get_layered_kernels: host copy of the four reflected kernels on the
 *   lattice, [4][2 Nz - 1][Ny][Nx] complex128 in the order xx, zz, phi, zx.
 *   Index s of the second axis is z + z' - 2 z_interface =
 *   2 (origin_z - z_interface) + s h_z; the last two axes are |offset| in
 *   nodes. */
slim_status slim_set_medium(slim_ctx* ctx, const slim_medium* medium);
/* slim_layered_gammas (host only, no device): the TM and TE voltage reflection
 * coefficients Gamma_e, Gamma_h of the medium seen from air at the interface, at
 * frequency freq (Hz), for n complex transverse wavenumbers on or above the real
 * axis.  These are the coefficients the reflected kernels are built from.
 * kr: 2n doubles (re, im); out: 4n doubles (Gamma_e re, im, Gamma_h re, im per
 * point).  SLIM_E_ARG on bad layer data or null pointers. */
slim_status slim_layered_gammas(const slim_medium* medium, double freq, int64_t n, const double* kr, double* out);
slim_status slim_aim_convolve_layered(slim_ctx* ctx, slim_prec prec, const void* src_dev, void* dst_dev, void* stream);
slim_status slim_get_layered_kernels(const slim_ctx* ctx, double* out);
slim_status slim_get_near(const slim_ctx* ctx, int32_t which, int64_t* ptr, int32_t* col, double* val);

/* Lumped ports (Sec. II: excitation "by lumped ports").  A port is an ideal
 * voltage source across a cut of one conductor's surface: the closed ring of mesh
 * edges of object `obj` that lie in the plane through `point` normal to `axis`
 * and within `radius` of `point`.  Its incident field is V delta(s) axis (s the
 * distance from the plane along axis), so testing with f_m gives
 *   b1[m] = (V / eta0) s_m l_m on the ring edges, 0 elsewhere; b2 = 0,
 * with s_m = +1 or -1 as the edge's RWG function crosses it along or against axis.
 * The port current along axis is the flux of n x H across the ring,
 *   I = sum over the ring of s_m l_m H_m,
 * so with V = 1 the port admittance matrix is Y[p][q] = I_p of the solution for
 * port q.  SLIM_E_ARG if a ring is empty, not one closed loop, or lies in a face
 * (an edge whose RWG function crosses it at more than 60 degrees from axis). */
typedef struct slim_port {
  int32_t obj;
  double point[3];
  double axis[3];
  double radius;
} slim_port;

/* B = [b of port 0, ..., b of port n_ports-1] with V = 1 V: column-major
 * n_sys x n_ports complex128 device array.  Synchronous. */
slim_status slim_rhs_ports(slim_ctx* ctx, const slim_port* ports, int32_t n_ports, void* B_dev, void* stream);
/* Port currents of n_rhs solution columns X (column-major n_sys x n_rhs complex128,
 * device): I_host (host, n_ports x n_rhs complex128 as interleaved doubles,
 * column-major: I_host[2 (p + n_ports q)] is the real part of I_p of column q).
 * Synchronous. */
slim_status slim_port_currents(slim_ctx* ctx, const slim_port* ports, int32_t n_ports, const void* X_dev,
                               int32_t n_rhs, double* I_host, void* stream);

/* Right-hand side of (7) for an incident plane wave E0 epol e^{-j k0 khat.r}. */
slim_status slim_rhs_planewave(slim_ctx* ctx, const double khat[3], const double epol[3],
                               void* b_dev, void* stream);

/* GMRES on S A x = S b with S = diag(1/h^2 (N_E rows), h (N_T rows)), h the
 * mean edge length (a change of length unit that balances the two row blocks),
 * right-preconditioned by the conductor blocks when opts.use_precond = 1.
 * x_dev: in = x0, out = solution (complex128, n_sys); a zero x0 takes no product for
 * its first residual (S b).  b_dev is S b or b according to `scaled_rhs` (1: b_dev
 * already equilibrated).  Synchronous. */
slim_status slim_solve(slim_ctx* ctx, const void* b_dev, int32_t scaled_rhs, void* x_dev,
                       const slim_solve_opts* opts, slim_solve_info* info, void* stream);

/* z = P^{-1} v for the conductor-block preconditioner (built when
 * opts.precond = 1): v, z are n_sys complex128 device vectors in the
 * equilibrated space of slim_solve, no aliasing.  The blocks hold complex64
 * entries; the product accumulates in FP32 and writes complex128.  Every unknown
 * is written by exactly one block.  SLIM_E_STATE if no preconditioner was built. */
slim_status slim_precond_apply(slim_ctx* ctx, const void* v_dev, void* z_dev, void* stream);
/* Host copy of the preconditioner's blocks: *n_blocks, and the totals *n_ext
 * (extended indices) and *n_own (owned rows).  ext_ptr (n_blocks+1 int64),
 * ext_idx (n_ext int32 system indices: edges, then n_e + triangle, each
 * ascending), own_ptr (n_blocks+1 int64) and own_pos (n_own int32 positions in
 * the block's ext list).  Any array pointer may be NULL (sizes only). */
slim_status slim_get_precond(const slim_ctx* ctx, int64_t* n_blocks, int64_t* n_ext, int64_t* n_own,
                             int64_t* ext_ptr, int32_t* ext_idx, int64_t* own_ptr, int32_t* own_pos);

/* Host-only (no device, no context): the blocks the preconditioner would use
 * for a mesh, cap and overlap, in the slim_get_precond layout.  Same mesh
 * rules and SLIM_E_MESH as slim_set_mesh.  Call with NULL arrays for the sizes. */
slim_status slim_precond_partition(const double* xyz, int64_t n_vert, const int32_t* tri, int64_t n_tri,
                                   const int32_t* obj_of_tri, int32_t n_obj, int64_t cap, int32_t overlap,
                                   int64_t* n_blocks, int64_t* n_ext, int64_t* n_own, int64_t* ext_ptr,
                                   int32_t* ext_idx, int64_t* own_ptr, int32_t* own_pos);

/* Timing of slim_matvec with HIP events.
 * slim_profile(ctx, 1): staged products (eager, sequential, the pulse path not
 *   overlapped) with events recorded on the caller's stream around each kernel
 *   group: 0 internal blocks (A1, A2), 1 projection P, 2 FFT convolution (all
 *   passes), 3 pulse rows (W, L_phi,NR), 4 RWG rows (W, L_A,NR, combine),
 *   5 continuity rows and casts.
 * slim_profile(ctx, 2): the default path (captured graph, pulse path concurrent),
 *   with events around each replay on the caller's stream and the internal
 *   kernel's own wall-clock stamps (first workgroup start to last workgroup end);
 *   every product then waits for its own end.  ms[0] = internal kernel inside the
 *   replays, ms[1] = whole replays.
 * slim_profile(ctx, 0) stops.  Each call clears the sums; slim_profile_read
 * synchronizes on the last recorded event and returns the summed milliseconds
 * (ms[6]) and the number of products recorded. */
slim_status slim_profile(slim_ctx* ctx, int32_t on);
slim_status slim_profile_read(slim_ctx* ctx, double* ms, int64_t* n_matvec);

/* --- internal task scheduling (Alg. 1, Part_Schedule idea; learned cost) ---- */
/* Record per-tile start/end timestamps on the next internal launches. */
slim_status slim_sched_record(slim_ctx* ctx, int32_t on);
/* Copy the last recorded tiles: per tile (block, row0, rows, n, slot, t_start,
 * t_end) as 7 doubles; *n_tiles in: capacity, out: count. */
slim_status slim_sched_tiles(slim_ctx* ctx, double* out, int64_t* n_tiles);
/* Train the MLP cost model (on the GPU, own forward/backward kernels) on the
 * recorded tiles; returns the final training loss. */
slim_status slim_sched_train(slim_ctx* ctx, int32_t epochs, double lr, double* final_loss);
/* Training samples of the last recorded tiles, for training on other workloads:
 * per tile 8 doubles, the seven raw (unstandardised) features of the cost model
 * (log n_i, log aspect of the object's box, log(skin depth / sqrt(area)), log
 * rows, (n_i mod 64) / 64, log of the row sweeps of the tile's busiest wave
 * (rows / (4 x rows per wave), rounded up), log of the 256-column chunks of a
 * row) and the log of the tile's duration in wall-clock ticks.  *n in: capacity
 * (tiles), out: count; out may be NULL (count only).  SLIM_E_STATE without
 * recorded timings. */
slim_status slim_sched_export(slim_ctx* ctx, double* out, int64_t* n);
/* Train the context's cost model on n samples in the slim_sched_export layout
 * (for instance pooled from other workloads); features are standardised on
 * these samples.  SLIM_E_ARG on non-finite samples. */
slim_status slim_sched_train_data(slim_ctx* ctx, int64_t n, const double* samples, int32_t epochs, double lr,
                                  double* final_loss);
/* 0 = LPT on flop counts, 1 = LPT on MLP-predicted times, 2 = naive (object
 * order, round robin), 3 = dynamic dispatch in decreasing flop-count order, 4 =
 * dynamic dispatch in decreasing predicted-time order (Sec. III-C scheduling on
 * persistent workgroups); re-packs the work queues and re-captures the graphs.
 * Modes 1 and 4 need a trained cost model (SLIM_E_STATE otherwise). */
slim_status slim_sched_set_mode(slim_ctx* ctx, int32_t mode);
/* Persistent workgroups of the two launches of the internal product: `slots` for
 * the rows of M_i, `slots_z` for the rows of Z_i (0 = slots), as the build options
 * of the same names; re-packs the queues in the current mode and re-captures the
 * graphs (the build's autotuned shape is replaced).  Results do not depend on the
 * shape.  SLIM_E_ARG outside [1, 65536] (slots_z: [0, 65536]); SLIM_E_STATE before
 * slim_build. */
slim_status slim_sched_set_shape(slim_ctx* ctx, int32_t slots, int32_t slots_z);

/* --- cost-model network kernels (exposed for gradient checks) -------------- */
/* FP32 MLP F -> 64 -> 64 -> 1 (tanh).  params (device, fp32) in the order
 * W1 (64 x F), b1, W2 (64 x 64), b2, w3 (64), b3 (1); X (B x F), t (B).
 * Computes loss = mean (y - t)^2, y (B) and grad (same layout as params). */
slim_status slim_mlp_forward_backward(int32_t F, int32_t B, const float* params_dev,
                                      const float* X_dev, const float* t_dev, float* y_dev,
                                      float* grad_dev, float* loss_dev, void* stream);

/* Allocation-free variant of slim_mlp_forward_backward, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight training loops,
 * harnesses that forbid hipMalloc).  Same arguments, layout and results (the
 * same kernels); it allocates nothing and only enqueues on `stream` (no
 * synchronization).  Its workspace, the per-wave partial gradients and losses,
 * is one static device array per GPU of about 9.8 MB, held until the process
 * ends, which limits B to 32768 samples (SLIM_E_ARG beyond, nothing launched).
 * Every call on a GPU uses that GPU's one workspace: calls that overlap on the
 * same GPU (different streams, threads) race and must be serialized by the
 * caller.  The workspace needs no clearing between calls.                     */
slim_status slim_mlp_forward_backward_noalloc(int32_t F, int32_t B, const float* params_dev, const float* X_dev,
                                              const float* t_dev, float* y_dev, float* grad_dev, float* loss_dev,
                                              void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SLIM_H */
