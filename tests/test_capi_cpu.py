"""Host-side checks of the C ABI library (no GPU needed)."""
import ctypes
import re

import numpy as np

import pytest


def test_library_exports_every_declared_symbol():
    from paper_2108_03991_amd import slim
    L = slim.lib()
    header = open(__file__.replace('tests/test_capi_cpu.py', 'include/slim.h')).read()
    declared = set(re.findall(r'\b(slim_[a-z_0-9]+)\s*\(', header))
    assert declared == set(slim.EXPORTS)
    for name in declared:
        assert hasattr(L, name)


def test_null_arguments_are_rejected():
    from paper_2108_03991_amd import slim
    L = slim.lib()
    assert L.slim_create(0, None) == 1
    assert L.slim_set_mesh(None, None, 0, None, 0, None, 0) == 1
    assert L.slim_matvec(None, 0, None, None, None) == 1
    assert L.slim_build(None, None) == 1
    assert L.slim_get_layout(None, None) == 1
    L.slim_destroy(None)
    assert b"null" in L.slim_last_error(None)
    assert L.slim_mlp_forward_backward(0, 1, None, None, None, None, None, None, None) == 1


def test_default_build_options():
    from paper_2108_03991_amd import slim
    o = slim.default_build_opts()
    assert (o.near_cheb, o.n_far, o.n_near, o.levels, o.n_r, o.n_t) == (3, 4, 5, 3, 5, 6)
    assert o.q == 0.25 and o.c_near == 2.0


def test_single_hip_runtime_in_process():
    """libslim binds to the HIP runtime PyTorch already loaded (same SONAMEs), so torch's
    streams and allocations are the library's own: exactly one libamdhip64 is mapped."""
    from paper_2108_03991_amd import slim
    slim.lib()
    maps = open('/proc/self/maps').read().splitlines()
    hip = {line.split()[-1] for line in maps if 'libamdhip64' in line}
    hsa = {line.split()[-1] for line in maps if 'libhsa-runtime64' in line}
    assert len(hip) == 1 and len(hsa) == 1, (hip, hsa)


@pytest.mark.parametrize("cap,overlap", [(0, 2), (120, 0), (120, 2), (60, 3), (300, 1)])
def test_precond_partition_matches_oracle(cap, overlap):
    """Host logic of the preconditioner: the library's block partition (RCB, growth,
    T+ ownership) equals the oracle's, index for index."""
    from inputs.geometry import box_mesh, merge, small_boxes
    from oracle import precond as opc
    from oracle.rwg import build_rwg
    from paper_2108_03991_amd import slim
    for m in (merge([box_mesh((0.0, 0.0, 0.0), (20e-6, 2e-6, 2e-6), (20, 2, 2)),
                     box_mesh((25e-6, 0.0, 0.0), (4e-6, 2e-6, 2e-6), (4, 2, 2)),
                     box_mesh((32e-6, 0.0, 0.0), (3e-6, 1e-6, 1e-6), (3, 1, 1))]),
              small_boxes(4, seed=5, tri_range=(40, 200))):
        g = build_rwg(m.verts, m.tris, m.obj, m.n_obj)
        ref = opc.partition(g, cap=cap, overlap=overlap)
        got = slim.precond_partition(m.verts, m.tris, m.obj, m.n_obj, cap, overlap)
        assert len(got) == len(ref)
        for (ext, pos), b in zip(got, ref):
            assert np.array_equal(ext, b.ext) and np.array_equal(pos, b.own_pos)


def test_layered_gammas_match_oracle():
    """Host-only: the library's generalized-reflection recursion against the oracle's
    impedance recursion, for several stacks, on the real axis and above it."""
    from oracle import mgf
    from paper_2108_03991_amd import slim
    stacks = [([(200e-6, 11.9, 10.0)], "pec"), ([(30e-6, 4.0, 0.0), (495e-6, 11.9, 10.0)], "pec"),
              ([], (11.9, 10.0)), ([(3e-6, 4.0, 0.0)], (2.0, 0.5)), ([], "pec")]
    for f in (1e9, 20e9):
        k0 = 2 * np.pi * f / mgf.C0
        kr = np.concatenate([np.linspace(0.01, 3e3, 57) + 0j,
                             np.linspace(1.0, 5e2, 23) + 1j * np.linspace(10.0, 80.0, 23),
                             np.array([0.999 * k0, 1.001 * k0, 1e6, 3e7]) + 0j])
        for layers, bottom in stacks:
            ge, gh = slim.layered_gammas(layers, bottom, f, kr)
            ref_e, ref_h = mgf.gammas(mgf.Stack(layers, bottom), f, kr)
            assert np.abs(ge - ref_e).max() <= 1e-12 and np.abs(gh - ref_h).max() <= 1e-12, (layers, bottom, f)
    with pytest.raises(slim.SlimError):
        slim.layered_gammas([(-1.0, 4.0, 0.0)], "pec", 1e9, kr)


def test_every_context_entry_point_rejects_a_null_context():
    """Each entry point that takes a context returns SLIM_E_ARG for NULL, whatever the
    other arguments (zero or NULL here), and touches nothing."""
    import ctypes as C
    from paper_2108_03991_amd import slim
    L = slim.lib()
    header = open(__file__.replace('tests/test_capi_cpu.py', 'include/slim.h')).read()
    names = re.findall(r'slim_status\s+(slim_[a-z_0-9]+)\s*\(\s*slim_ctx\s*\*', header)
    assert len(names) >= 20 and "slim_sched_set_shape" in names and "slim_create" not in names
    for name in names:
        f = getattr(L, name)
        assert f.argtypes, name        # every exported call is declared in the binding
        args = [None]
        for t in f.argtypes[1:]:
            args.append(0.0 if t in (C.c_double, C.c_float) else (0 if t in (C.c_int32, C.c_int64) else None))
        assert f(*args) == 1, name
