"""Python binding of libslim.so (argument marshalling only).

Every step of the product runs in the HIP library; this module converts
numpy arrays and torch device tensors into the plain pointers and sizes of the
C ABI declared in include/slim.h.  It raises if the library is missing: there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslim.so")

SLIM_FP64, SLIM_MIXED = 0, 1
STATUS = {0: "SLIM_OK", 1: "SLIM_E_ARG", 2: "SLIM_E_MESH", 3: "SLIM_E_STATE", 4: "SLIM_E_OOM", 5: "SLIM_E_HIP",
          6: "SLIM_E_NUMERIC", 7: "SLIM_E_NOT_CONVERGED", 8: "SLIM_E_UNSUPPORTED"}


class SlimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class BuildOpts(C.Structure):
    _fields_ = [("freq", C.c_double), ("grid", C.c_int32 * 3), ("near_cheb", C.c_int32),
                ("n_far", C.c_int32), ("n_near", C.c_int32), ("levels", C.c_int32), ("n_r", C.c_int32),
                ("n_t", C.c_int32), ("q", C.c_double), ("c_near", C.c_double), ("sched_mode", C.c_int32),
                ("tile_rows", C.c_int32), ("internal_kernel", C.c_int32), ("slots", C.c_int32),
                ("mem_budget", C.c_int64), ("verbose", C.c_int32), ("use_graphs", C.c_int32),
                ("precond", C.c_int32), ("precond_overlap", C.c_int32), ("precond_cap", C.c_int64),
                ("precond_budget", C.c_int64), ("fft_zblock", C.c_int32), ("rows_per_wave", C.c_int32),
                ("tune_cache", C.c_char_p), ("hf_radius", C.c_double), ("slots_z", C.c_int32),
                ("gen_workers", C.c_int32)]


class Layout(C.Structure):
    _fields_ = [("n_e", C.c_int64), ("n_t", C.c_int64), ("n_sys", C.c_int64), ("n_obj", C.c_int32),
                ("grid", C.c_int32 * 3), ("grid_h", C.c_double * 3), ("grid_origin", C.c_double * 3),
                ("nnz_near_A", C.c_int64), ("nnz_near_phi", C.c_int64), ("internal_entries", C.c_int64),
                ("n_tiles", C.c_int64), ("slots", C.c_int32), ("tile_rows", C.c_int32), ("mean_edge", C.c_double),
                ("build_seconds", C.c_double), ("device_bytes", C.c_int64), ("precond_blocks", C.c_int64),
                ("precond_entries", C.c_int64), ("precond_cap", C.c_int64), ("fft_zblock", C.c_int32),
                ("rows_per_wave", C.c_int32), ("z_nnz", C.c_int64), ("slots_z", C.c_int32),
                ("interior_workers", C.c_int32), ("interior_seconds", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int32), ("max_iter", C.c_int32), ("prec", C.c_int32),
                ("inner_tol", C.c_double), ("max_outer", C.c_int32), ("use_precond", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("outer_steps", C.c_int32), ("rel_residual", C.c_double),
                ("seconds", C.c_double), ("matvec_seconds", C.c_double), ("n_matvec_fp64", C.c_int32),
                ("n_matvec_mixed", C.c_int32), ("n_precond", C.c_int32)]


class Port(C.Structure):
    _fields_ = [("obj", C.c_int32), ("point", C.c_double * 3), ("axis", C.c_double * 3), ("radius", C.c_double)]


def _ports(ports):
    """(obj, point, axis, radius) tuples -> a ctypes array of slim_port."""
    arr = (Port * len(ports))()
    for k, (obj, point, axis, radius) in enumerate(ports):
        arr[k].obj = int(obj)
        arr[k].point[:] = [float(v) for v in point]
        arr[k].axis[:] = [float(v) for v in axis]
        arr[k].radius = float(radius)
    return arr


class Material(C.Structure):
    _fields_ = [("sigma", C.c_double), ("eps_r", C.c_double), ("mu_r", C.c_double)]


class Layer(C.Structure):
    _fields_ = [("thickness", C.c_double), ("eps_r", C.c_double), ("sigma", C.c_double)]


class Medium(C.Structure):
    _fields_ = [("z_interface", C.c_double), ("n_layers", C.c_int32), ("bottom_pec", C.c_int32),
                ("layers", C.POINTER(Layer)), ("bottom_eps_r", C.c_double), ("bottom_sigma", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libslim.so is not built (run __graft_entry__.build()); there is no fallback")
        # PyTorch ships its own HIP runtime (same SONAMEs as /opt/rocm).  Importing it
        # first makes the dynamic loader bind libslim to that already-loaded runtime, so
        # the process has one HIP runtime and torch's streams and allocations are the
        # library's too.  Loading libslim first would bring in a second runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
        L.slim_create.argtypes = [i32, C.POINTER(vp)]
        L.slim_destroy.argtypes = [vp]
        L.slim_destroy.restype = None
        L.slim_last_error.argtypes = [vp]
        L.slim_last_error.restype = C.c_char_p
        L.slim_default_build_opts.argtypes = [C.POINTER(BuildOpts)]
        L.slim_default_build_opts.restype = None
        L.slim_set_mesh.argtypes = [vp, vp, i64, vp, i64, vp, i32]
        L.slim_set_materials.argtypes = [vp, vp]
        L.slim_build.argtypes = [vp, C.POINTER(BuildOpts)]
        L.slim_get_layout.argtypes = [vp, C.POINTER(Layout)]
        L.slim_get_rwg.argtypes = [vp, vp, vp, vp]
        L.slim_matvec.argtypes = [vp, i32, vp, vp, vp]
        L.slim_matvec_parts.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.slim_internal_apply.argtypes = [vp, i32, vp, vp, vp, dp, vp]
        L.slim_rhs_planewave.argtypes = [vp, dp, dp, vp, vp]
        L.slim_solve.argtypes = [vp, vp, i32, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
        L.slim_sched_record.argtypes = [vp, i32]
        L.slim_sched_tiles.argtypes = [vp, dp, C.POINTER(i64)]
        L.slim_sched_train.argtypes = [vp, i32, C.c_double, dp]
        L.slim_sched_set_mode.argtypes = [vp, i32]
        L.slim_sched_set_shape.argtypes = [vp, i32, i32]
        L.slim_mlp_forward_backward.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp]
        L.slim_mlp_forward_backward_noalloc.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp]
        L.slim_aim_convolve.argtypes = [vp, i32, vp, vp, i32, vp]
        L.slim_get_aim.argtypes = [vp, vp, vp, vp, vp]
        L.slim_get_near.argtypes = [vp, i32, vp, vp, vp]
        L.slim_precond_apply.argtypes = [vp, vp, vp, vp]
        L.slim_get_precond.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.slim_precond_partition.argtypes = [vp, i64, vp, i64, vp, i32, i64, i32, vp, vp, vp, vp, vp, vp, vp]
        L.slim_set_medium.argtypes = [vp, C.POINTER(Medium)]
        L.slim_aim_convolve_layered.argtypes = [vp, i32, vp, vp, vp]
        L.slim_get_layered_kernels.argtypes = [vp, dp]
        L.slim_layered_gammas.argtypes = [C.POINTER(Medium), C.c_double, i64, dp, dp]
        L.slim_profile.argtypes = [vp, i32]
        L.slim_profile_read.argtypes = [vp, dp, C.POINTER(i64)]
        L.slim_matvec_block.argtypes = [vp, i32, vp, vp, i32, vp]
        L.slim_sched_export.argtypes = [vp, dp, C.POINTER(i64)]
        L.slim_sched_train_data.argtypes = [vp, i64, dp, i32, C.c_double, dp]
        L.slim_rhs_ports.argtypes = [vp, C.POINTER(Port), i32, vp, vp]
        L.slim_port_currents.argtypes = [vp, C.POINTER(Port), i32, vp, i32, dp, vp]
        for name in ("slim_create", "slim_set_mesh", "slim_set_materials", "slim_build", "slim_get_layout",
                     "slim_get_rwg", "slim_matvec", "slim_matvec_parts", "slim_internal_apply",
                     "slim_rhs_planewave", "slim_solve", "slim_sched_record", "slim_sched_tiles",
                     "slim_sched_train", "slim_sched_set_mode", "slim_sched_set_shape", "slim_mlp_forward_backward",
                     "slim_profile",
                     "slim_profile_read", "slim_aim_convolve", "slim_get_aim", "slim_get_near",
                     "slim_precond_apply", "slim_get_precond", "slim_precond_partition", "slim_set_medium",
                     "slim_aim_convolve_layered", "slim_get_layered_kernels", "slim_layered_gammas",
                     "slim_matvec_block", "slim_rhs_ports", "slim_port_currents",
                     "slim_mlp_forward_backward_noalloc", "slim_sched_export", "slim_sched_train_data"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


EXPORTS = ["slim_default_build_opts", "slim_create", "slim_destroy", "slim_last_error", "slim_set_mesh",
           "slim_set_materials", "slim_build", "slim_get_layout", "slim_get_rwg", "slim_matvec",
           "slim_matvec_parts", "slim_internal_apply", "slim_rhs_planewave", "slim_solve", "slim_sched_record",
           "slim_sched_tiles", "slim_sched_train", "slim_sched_set_mode", "slim_sched_set_shape",
           "slim_mlp_forward_backward",
           "slim_profile", "slim_profile_read", "slim_aim_convolve", "slim_get_aim", "slim_get_near",
           "slim_precond_apply", "slim_get_precond", "slim_precond_partition", "slim_set_medium",
           "slim_aim_convolve_layered", "slim_get_layered_kernels", "slim_layered_gammas", "slim_matvec_block",
           "slim_rhs_ports", "slim_port_currents", "slim_mlp_forward_backward_noalloc", "slim_sched_export",
           "slim_sched_train_data"]


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream)


def default_build_opts(**kw):
    o = BuildOpts()
    lib().slim_default_build_opts(C.byref(o))
    for k, v in kw.items():
        if k == "grid":
            o.grid[0], o.grid[1], o.grid[2] = (int(x) for x in v)
        elif k == "tune_cache":
            o.tune_cache = None if v is None else os.fsencode(v)
        else:
            setattr(o, k, v)
    return o


def _medium(z_interface, layers, bottom):
    """slim_medium for (layers top-down as (thickness, eps_r, sigma), bottom "pec" or (eps_r, sigma));
    returns the struct and the layer array it points to (keep both alive for the call)."""
    arr = (Layer * max(1, len(layers)))(*[Layer(*map(float, l)) for l in layers])
    m = Medium()
    m.z_interface = float(z_interface)
    m.n_layers = len(layers)
    m.layers = C.cast(arr, C.POINTER(Layer))
    if isinstance(bottom, str):
        if bottom != "pec":
            raise ValueError("bottom must be 'pec' or (eps_r, sigma)")
        m.bottom_pec = 1
    else:
        m.bottom_pec = 0
        m.bottom_eps_r, m.bottom_sigma = (float(v) for v in bottom)
    return m, arr


def layered_gammas(layers, bottom, freq, kr):
    """Host-only: (Gamma_e, Gamma_h) of the stack at complex transverse wavenumbers kr."""
    m, keep = _medium(0.0, layers, bottom)
    kr = np.ascontiguousarray(np.asarray(kr, dtype=np.complex128))
    out = np.zeros(4 * kr.size)
    st = lib().slim_layered_gammas(C.byref(m), float(freq), kr.size,
                                   kr.view(np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                                   out.ctypes.data_as(C.POINTER(C.c_double)))
    if st != 0:
        raise SlimError(st, "slim_layered_gammas failed")
    o = out.view(np.complex128).reshape(-1, 2)
    return o[:, 0].copy(), o[:, 1].copy()


class Context:
    def __init__(self, device=0):
        self._h = C.c_void_p()
        st = lib().slim_create(int(device), C.byref(self._h))
        if st != 0:
            raise SlimError(st, "slim_create failed")

    def close(self):
        if self._h:
            lib().slim_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise SlimError(st, lib().slim_last_error(self._h).decode())

    def set_mesh(self, verts, tris, obj, n_obj):
        v = np.ascontiguousarray(verts, dtype=np.float64)
        t = np.ascontiguousarray(tris, dtype=np.int32)
        o = np.ascontiguousarray(obj, dtype=np.int32)
        self._check(lib().slim_set_mesh(self._h, v.ctypes.data, v.shape[0], t.ctypes.data, t.shape[0],
                                        o.ctypes.data, int(n_obj)))

    def set_materials(self, mats=None):
        if mats is None:
            self._check(lib().slim_set_materials(self._h, None))
            return
        arr = (Material * len(mats))(*[Material(*m) for m in mats])
        self._check(lib().slim_set_materials(self._h, C.cast(arr, C.c_void_p)))

    def build(self, **kw):
        o = default_build_opts(**kw)
        self._check(lib().slim_build(self._h, C.byref(o)))
        return self.layout()

    def layout(self):
        L = Layout()
        self._check(lib().slim_get_layout(self._h, C.byref(L)))
        return L

    def rwg(self, n_e):
        ev = np.zeros(2 * n_e, dtype=np.int32)
        tp = np.zeros(n_e, dtype=np.int32)
        tm = np.zeros(n_e, dtype=np.int32)
        self._check(lib().slim_get_rwg(self._h, ev.ctypes.data, tp.ctypes.data, tm.ctypes.data))
        return ev.reshape(-1, 2), tp, tm

    def matvec(self, prec, x, y, stream=None):
        self._check(lib().slim_matvec(self._h, prec, _ptr(x), _ptr(y), _stream(stream)))

    def matvec_parts(self, prec, x, y, e=None, g=None, a=None, phi=None, stream=None):
        self._check(lib().slim_matvec_parts(self._h, prec, _ptr(x), _ptr(y), _ptr(e), _ptr(g), _ptr(a), _ptr(phi),
                                            _stream(stream)))

    def matvec_block(self, prec, X, Y, n_rhs, stream=None):
        """Y = A X for n_rhs columns (column-major n_sys x n_rhs complex128 device arrays)."""
        self._check(lib().slim_matvec_block(self._h, prec, _ptr(X), _ptr(Y), int(n_rhs), _stream(stream)))

    def rhs_ports(self, ports, B, stream=None):
        """Unit-voltage lumped-port right-hand sides, one column of B per (obj, point, axis, radius)."""
        arr = _ports(ports)
        self._check(lib().slim_rhs_ports(self._h, arr, len(ports), _ptr(B), _stream(stream)))

    def port_currents(self, ports, X, n_rhs, stream=None):
        """Port currents (n_ports x n_rhs complex) of the solution columns X."""
        arr = _ports(ports)
        out = np.zeros(2 * len(ports) * int(n_rhs))
        self._check(lib().slim_port_currents(self._h, arr, len(ports), _ptr(X), int(n_rhs),
                                             out.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)))
        return out.view(np.complex128).reshape(int(n_rhs), len(ports)).T

    def internal_apply(self, prec, H, e=None, g=None, timed=False, stream=None):
        ms = C.c_double(0.0)
        self._check(lib().slim_internal_apply(self._h, prec, _ptr(H), _ptr(e), _ptr(g),
                                              C.byref(ms) if timed else None, _stream(stream)))
        return ms.value if timed else None

    def rhs_planewave(self, khat, epol, b, stream=None):
        k = (C.c_double * 3)(*khat)
        e = (C.c_double * 3)(*epol)
        self._check(lib().slim_rhs_planewave(self._h, k, e, _ptr(b), _stream(stream)))

    def solve(self, b, x, tol=1e-6, restart=50, max_iter=1000, prec=SLIM_FP64, inner_tol=1e-4, max_outer=0,
              scaled_rhs=False, use_precond=True, stream=None):
        o = SolveOpts(tol, restart, max_iter, prec, inner_tol, max_outer, int(bool(use_precond)))
        info = SolveInfo()
        st = lib().slim_solve(self._h, _ptr(b), int(bool(scaled_rhs)), _ptr(x), C.byref(o), C.byref(info),
                              _stream(stream))
        if st not in (0, 7):
            self._check(st)
        return info, st == 0

    def precond_apply(self, v, z, stream=None):
        self._check(lib().slim_precond_apply(self._h, _ptr(v), _ptr(z), _stream(stream)))

    def get_precond(self):
        """Blocks of the preconditioner: list of (ext system indices, owned positions)."""
        nb, ne_, no = C.c_int64(0), C.c_int64(0), C.c_int64(0)
        self._check(lib().slim_get_precond(self._h, C.byref(nb), C.byref(ne_), C.byref(no), None, None, None, None))
        ep = np.zeros(nb.value + 1, np.int64)
        ei = np.zeros(max(1, ne_.value), np.int32)
        op = np.zeros(nb.value + 1, np.int64)
        oi = np.zeros(max(1, no.value), np.int32)
        self._check(lib().slim_get_precond(self._h, C.byref(nb), C.byref(ne_), C.byref(no), ep.ctypes.data,
                                           ei.ctypes.data, op.ctypes.data, oi.ctypes.data))
        return [(ei[ep[k]:ep[k + 1]].copy(), oi[op[k]:op[k + 1]].copy()) for k in range(nb.value)]

    def aim_convolve(self, prec, src, dst, ncomp, stream=None):
        self._check(lib().slim_aim_convolve(self._h, prec, _ptr(src), _ptr(dst), int(ncomp), _stream(stream)))

    def set_medium(self, z_interface, layers=(), bottom="pec"):
        """Layered background: layers top-down as (thickness, eps_r, sigma); bottom "pec" or (eps_r, sigma)."""
        m, keep = _medium(z_interface, layers, bottom)
        self._check(lib().slim_set_medium(self._h, C.byref(m)))

    def aim_convolve_layered(self, prec, src, dst, stream=None):
        self._check(lib().slim_aim_convolve_layered(self._h, prec, _ptr(src), _ptr(dst), _stream(stream)))

    def layered_kernels(self, grid):
        """Reflected kernels on the lattice: (4, 2 Nz - 1, Ny, Nx) complex (xx, zz, phi, zx radial)."""
        Nx, Ny, Nz = (int(v) for v in grid)
        out = np.zeros(2 * 4 * (2 * Nz - 1) * Ny * Nx)
        self._check(lib().slim_get_layered_kernels(self._h, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out.view(np.complex128).reshape(4, 2 * Nz - 1, Ny, Nx)

    def get_aim(self, n_e, n_t):
        ce = np.zeros(3 * n_e, np.int32)
        we = np.zeros(81 * n_e)
        ct = np.zeros(3 * n_t, np.int32)
        wt = np.zeros(27 * n_t)
        self._check(lib().slim_get_aim(self._h, ce.ctypes.data, we.ctypes.data, ct.ctypes.data, wt.ctypes.data))
        return ce.reshape(-1, 3), we.reshape(-1, 3, 27), ct.reshape(-1, 3), wt.reshape(-1, 27)

    def get_near(self, which, rows, nnz):
        ptr = np.zeros(rows + 1, np.int64)
        col = np.zeros(nnz, np.int32)
        val = np.zeros(2 * nnz)
        self._check(lib().slim_get_near(self._h, int(which), ptr.ctypes.data, col.ctypes.data, val.ctypes.data))
        return ptr, col, val.view(np.complex128)

    def profile(self, on=True):
        """on: False/0 stop, True/1 staged per-stage events, 2 graph-path events (see slim.h)."""
        self._check(lib().slim_profile(self._h, int(on)))

    def profile_read(self):
        ms = (C.c_double * 6)()
        n = C.c_int64(0)
        self._check(lib().slim_profile_read(self._h, ms, C.byref(n)))
        return list(ms), n.value

    def sched_record(self, on=True):
        self._check(lib().slim_sched_record(self._h, int(bool(on))))

    def sched_tiles(self):
        n = C.c_int64(0)
        self._check(lib().slim_sched_tiles(self._h, None, C.byref(n)))
        out = np.zeros(7 * n.value, dtype=np.float64)
        self._check(lib().slim_sched_tiles(self._h, out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(n)))
        return out.reshape(-1, 7)

    def sched_train(self, epochs=2000, lr=3e-3):
        loss = C.c_double(0.0)
        self._check(lib().slim_sched_train(self._h, int(epochs), float(lr), C.byref(loss)))
        return loss.value

    def sched_export(self):
        """Samples of the last recorded tiles: (n, 8) = seven raw features and log duration."""
        n = C.c_int64(0)
        self._check(lib().slim_sched_export(self._h, None, C.byref(n)))
        out = np.zeros(8 * n.value)
        self._check(lib().slim_sched_export(self._h, out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(n)))
        return out.reshape(-1, 8)

    def sched_train_data(self, samples, epochs=2000, lr=3e-3):
        """Train the cost model on samples in the sched_export layout; returns the final loss."""
        a = np.ascontiguousarray(samples, dtype=np.float64)
        loss = C.c_double(0.0)
        self._check(lib().slim_sched_train_data(self._h, a.shape[0], a.ctypes.data_as(C.POINTER(C.c_double)),
                                                int(epochs), float(lr), C.byref(loss)))
        return loss.value

    def sched_set_mode(self, mode):
        self._check(lib().slim_sched_set_mode(self._h, int(mode)))

    def sched_set_shape(self, slots, slots_z=0):
        self._check(lib().slim_sched_set_shape(self._h, int(slots), int(slots_z)))


def precond_partition(verts, tris, obj, n_obj, cap, overlap):
    """Host-only block partition of the preconditioner: list of (ext indices, owned positions)."""
    v = np.ascontiguousarray(verts, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    o = np.ascontiguousarray(obj, dtype=np.int32)
    nb, ne_, no = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    args = (v.ctypes.data, v.shape[0], t.ctypes.data, t.shape[0], o.ctypes.data, int(n_obj), int(cap), int(overlap))
    st = lib().slim_precond_partition(*args, C.byref(nb), C.byref(ne_), C.byref(no), None, None, None, None)
    if st != 0:
        raise SlimError(st, "slim_precond_partition failed")
    ep = np.zeros(nb.value + 1, np.int64)
    ei = np.zeros(max(1, ne_.value), np.int32)
    op = np.zeros(nb.value + 1, np.int64)
    oi = np.zeros(max(1, no.value), np.int32)
    st = lib().slim_precond_partition(*args, C.byref(nb), C.byref(ne_), C.byref(no), ep.ctypes.data, ei.ctypes.data,
                                      op.ctypes.data, oi.ctypes.data)
    if st != 0:
        raise SlimError(st, "slim_precond_partition failed")
    return [(ei[ep[k]:ep[k + 1]].copy(), oi[op[k]:op[k + 1]].copy()) for k in range(nb.value)]


def mlp_forward_backward_noalloc(F, B, params, X, t, y, grad, loss, stream=None):
    """The allocation-free variant (enqueues only; B <= 32768; one workspace per GPU)."""
    st = lib().slim_mlp_forward_backward_noalloc(int(F), int(B), _ptr(params), _ptr(X), _ptr(t), _ptr(y), _ptr(grad),
                                                 _ptr(loss), _stream(stream))
    if st != 0:
        raise SlimError(st, "slim_mlp_forward_backward_noalloc failed")


def mlp_forward_backward(F, B, params, X, t, y, grad, loss, stream=None):
    st = lib().slim_mlp_forward_backward(int(F), int(B), _ptr(params), _ptr(X), _ptr(t), _ptr(y), _ptr(grad),
                                         _ptr(loss), _stream(stream))
    if st != 0:
        raise SlimError(st, "slim_mlp_forward_backward failed")
