"""Benchmark of the SLIM system matrix-vector product on one MI355X.

One step = one full product y = A x of eq. (7)-(8) (internal blocks, AIM
projection, FFT convolution, interpolation, near field, sparse combine) on the
seeded synthetic workload, inputs resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload conductors] [--no-solve]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "AIM+internal matvecs/sec and GMRES time-to-1e-6 at ~1M unknowns, mixed vs FP64"
HBM_PEAK = 8.0e12

WORKLOADS = {
    # name: (generator kwargs, frequency, AIM grid)
    "conductors": (dict(seed=0), 5e9, (256, 256, 256)),
    "line_bundle": (dict(seed=0), 1e9, (128, 128, 128)),
    "srr_array": (dict(), 100e9, (64, 64, 64)),
    "bar": (dict(), 10e9, (0, 0, 0)),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_mesh(name, kw):
    from inputs import geometry
    gen = {"conductors": geometry.conductors_c5, "line_bundle": geometry.line_bundle_c3,
           "srr_array": geometry.srr_array_c2, "bar": geometry.bar_c1}[name]
    return gen(**kw)


def algorithmic_bytes(mesh, lay, mixed):
    """Bytes the method must move per product: every stored operator entry and grid element once."""
    n = np.bincount(mesh.obj)  # triangles per object
    ne_i = (1.5 * n).astype(np.float64)
    sc = 8.0 if mixed else 16.0          # complex element (hi, or hi + lo / complex128)
    b_int = float(np.sum(2.0 * ne_i * ne_i)) * sc + 3.0 * lay.n_e * sc
    out = dict(internal=b_int)
    if lay.grid[0] > 0:
        N3 = float(lay.grid[0] * lay.grid[1] * lay.grid[2])
        out["fft"] = 4 * 26 * N3 * sc + 8 * N3 * sc
        ws = 4.0 if mixed else 8.0
        out["project"] = lay.n_e * 81 * (ws + 4 / 3) + lay.n_t * 27 * (ws + 4) + 4 * N3 * sc
        nnz = lay.nnz_near_A + lay.nnz_near_phi
        out["near_rows"] = nnz * (sc + 4) + (lay.n_e + lay.n_t) * (8 + sc * 4) + lay.n_e * 81 * ws + lay.n_t * 27 * ws
    return out


def cpu_baseline(mesh, lay, freq, grid):
    """The FP64 oracle timed on a bounded sample of the same workload, extrapolated per product."""
    from threadpoolctl import threadpool_info
    from oracle.aim import Grid, circulant_kernel, convolve_fft
    from oracle.operators import Physics, interior_blocks
    from oracle.rwg import build_rwg
    import scipy.sparse as sp
    from inputs.geometry import merge, random_complex
    ph = Physics(freq)
    # internal part: oracle blocks of a few small objects of this workload, GEMVs timed
    counts = np.bincount(mesh.obj)
    order = np.argsort(counts)
    pick = order[len(order) // 2: len(order) // 2 + 3]
    parts = []
    for i in pick:
        sel = np.nonzero(mesh.obj == i)[0]
        vids, inv = np.unique(mesh.tris[sel], return_inverse=True)
        parts.append((mesh.verts[vids], inv.reshape(-1, 3).astype(np.int32)))
    sub = merge(parts)
    g = build_rwg(sub.verts, sub.tris, sub.obj, sub.n_obj)
    inner = interior_blocks(g, ph)
    H = random_complex(g.n_e, 0)
    reps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 3.0:
        for i in range(g.n_obj):
            s = slice(g.obj_edge_off[i], g.obj_edge_off[i + 1])
            inner.Z[i] @ H[s]
            inner.M[i] @ H[s]
        reps += 1
    t_int = (time.perf_counter() - t0) / reps
    ent_sample = sum(2 * Z.size for Z in inner.Z)
    ent_all = float(np.sum(2.0 * (1.5 * counts) ** 2))
    t_internal = t_int * ent_all / ent_sample
    t_ext = 0.0
    note = "internal: oracle Z_i, M_i GEMVs of objects %s (%d entries), scaled by entry count" % (
        list(map(int, pick)), ent_sample)
    if grid[0] > 0:
        # grid convolution: one component on a quarter-size grid, scaled by N^3 log N^3, times 4
        Nq = max(8, grid[0] // 4)
        gq = Grid(np.array([Nq] * 3), np.array([2e-6] * 3), np.zeros(3))
        Ghat = np.fft.fftn(circulant_kernel(gq, ph.k0))
        src = random_complex(Nq ** 3, 1)
        t0 = time.perf_counter()
        convolve_fft(gq, Ghat, src)
        tq = time.perf_counter() - t0
        scale = (grid[0] / Nq) ** 3 * np.log(grid[0]) / np.log(Nq)
        t_fft = 4 * tq * scale
        # near field, projection and interpolation: scipy CSR products (as in the oracle) per non-zero
        rng = np.random.default_rng(0)
        nrow = 200000
        nnz_row = max(1, int(round(lay.nnz_near_A / lay.n_e)))
        cols = rng.integers(0, nrow, size=nrow * nnz_row)
        A = sp.csr_matrix((np.ones(cols.size, complex), (np.repeat(np.arange(nrow), nnz_row), cols)), shape=(nrow, nrow))
        v = random_complex(nrow, 2)
        t0 = time.perf_counter()
        A @ v
        t_nnz = (time.perf_counter() - t0) / A.nnz
        nnz_total = lay.nnz_near_A + lay.nnz_near_phi + 2 * (81 * lay.n_e + 27 * lay.n_t)
        t_ext = t_fft + t_nnz * nnz_total
        note += ("; FFT convolution: oracle on a %d^3 grid scaled by N^3 log N to %d^3, x4 components; "
                 "near field / P / W: scipy CSR product per non-zero x %d non-zeros" % (Nq, grid[0], nnz_total))
    total = t_internal + t_ext
    threads = 1
    for info in threadpool_info():
        if info.get("user_api") == "blas":
            threads = max(threads, int(info.get("num_threads", 1)))
    return dict(value=1.0 / total, unit="matvecs/s", cores=threads, kind="oracle",
                sample=note + "; seconds per product: internal %.3g, external %.3g (extrapolated)" % (t_internal, t_ext))


def sched_study(ctx, lay, x, reps=7, epochs=3000):
    """Makespan of the persistent internal kernel (HIP events) under three packings of the
    same tiles: naive (mesh order, round robin), LPT on flop counts, LPT on times predicted
    by the cost-model network trained on the GPU from this run's own per-tile timestamps."""
    import torch
    from paper_2108_03991_amd import slim
    H = x[:lay.n_e].contiguous()

    def makespan():
        ts = [ctx.internal_apply(slim.SLIM_MIXED, H, timed=True) for _ in range(reps)]
        return float(np.median(ts))

    out = {}
    ctx.sched_set_mode(0)
    ctx.sched_record(True)
    ctx.internal_apply(slim.SLIM_MIXED, H, timed=True)
    tiles = ctx.sched_tiles()
    ctx.sched_record(False)
    dur = tiles[:, 6] - tiles[:, 5]
    slots = int(tiles[:, 4].max()) + 1
    busy = np.bincount(tiles[:, 4].astype(int), weights=dur, minlength=slots)
    out["recorded_tiles"] = int(len(tiles))
    out["ideal_over_lpt_busy"] = float(dur.sum() / slots / busy.max())
    t0 = time.time()
    out["train_loss"] = ctx.sched_train(epochs=epochs, lr=3e-3)
    out["train_s"] = time.time() - t0
    for name, mode in (("naive_ms", 2), ("lpt_ms", 0), ("mlp_ms", 1)):
        ctx.sched_set_mode(mode)
        makespan()
        out[name] = makespan()
    ctx.sched_set_mode(0)
    out["mlp_gain_vs_lpt"] = out["lpt_ms"] / out["mlp_ms"] - 1.0
    return out


def solve_study(ctx, lay, max_iter):
    """GMRES time-to-1e-6 for a plane wave, FP64 and mixed (GMRES-IR), right-preconditioned
    by the conductor blocks; plus how far unpreconditioned GMRES gets in a bounded run."""
    import torch
    from paper_2108_03991_amd import slim
    n = lay.n_sys
    b = torch.zeros(n, dtype=torch.complex128, device="cuda")
    ctx.rhs_planewave((0.0, 0.0, -1.0), (1.0, 0.0, 0.0), b)
    out = {"rhs": "plane wave, E0 = 1 V/m along x, travelling along -z", "tol": 1e-6, "restart": 100, "inner_tol": 1e-6,
           "precond": {"blocks": lay.precond_blocks, "entries": lay.precond_entries, "cap": lay.precond_cap}}
    # the preconditioner apply on its own (HBM-bound GEMV over the stored complex64 rows)
    v = torch.randn(n, dtype=torch.complex128, device="cuda")
    zz = torch.zeros_like(v)
    ctx.precond_apply(v, zz)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(10):
        ctx.precond_apply(v, zz)
    torch.cuda.synchronize()
    dt_pc = (time.perf_counter() - t) / 10
    out["precond"]["apply_ms"] = 1e3 * dt_pc
    out["precond"]["apply_GBps"] = lay.precond_entries * 8 / dt_pc / 1e9
    sols = {}
    for name, prec in (("mixed", slim.SLIM_MIXED), ("fp64", slim.SLIM_FP64)):
        xs = torch.zeros_like(b)
        torch.cuda.synchronize()
        info, ok = ctx.solve(b, xs, tol=1e-6, restart=100, max_iter=max_iter, prec=prec, inner_tol=1e-6)
        out[name] = {"seconds": info.seconds, "iterations": info.iterations, "outer": info.outer_steps,
                     "precond_applies": info.n_precond, "matvecs_mixed": info.n_matvec_mixed,
                     "matvecs_fp64": info.n_matvec_fp64, "rel_residual": info.rel_residual, "converged": bool(ok)}
        sols[name] = xs
        log("solve %s: %s" % (name, out[name]))
    out["mixed_vs_fp64_solution_rel_diff"] = float(torch.linalg.norm(sols["mixed"] - sols["fp64"]) /
                                                   torch.linalg.norm(sols["fp64"]))
    xs = torch.zeros_like(b)
    info, ok = ctx.solve(b, xs, tol=1e-6, restart=50, max_iter=200, prec=slim.SLIM_MIXED, inner_tol=1e-2,
                         use_precond=False)
    out["unpreconditioned_mixed_200_iterations"] = {"rel_residual": info.rel_residual, "seconds": info.seconds,
                                                    "converged": bool(ok)}
    log("solve without preconditioner (200 iterations): %s" % out["unpreconditioned_mixed_200_iterations"])
    return out


def layered_bytes(N, mixed):
    """Algorithmic bytes of one layered convolution of four components.

    Per component, the passes move N^3 elements in x-fwd and x-inv (plus 2 N^3
    each), 6 N^3 in y-fwd and y-inv each, 12 N^3 in the z forward and inverse
    steps each, and 16 N^3 in the spectrum product (read and write of the full
    (2N)^2 x 2N spectrum).  Together with the kernels (the free-space octant and
    five reflected spectra of (N+1)^2 x 2N) that is 58 N^3 elements per component.
    """
    N3 = float(N[0] * N[1] * N[2])
    sc = 8.0 if mixed else 16.0
    kern = (N[0] + 1) * (N[1] + 1) * (N[2] + 1) + 5 * (N[0] + 1) * (N[1] + 1) * 2 * N[2]
    return (4 * 58 * N3 + kern) * sc


def layered_study(steps=10, warmup=2):
    """The bundle-over-substrate workload: the layered product and its convolution.

    The 200-line bundle (1 GHz, AIM grid 128^3) sits above a silicon substrate
    (200 um, eps_r 11.9, sigma 10 S/m) on a PEC ground.  The interface is 1 um
    below the lowest grid plane.  Timed:
      * the whole product (default path) before and after the medium is set;
      * the four-component convolution per entry-point call, layered against
        free space.
    Setting the medium builds the reflected lattice kernels and corrects the
    near field.
    """
    import torch
    from paper_2108_03991_amd import slim
    from inputs.geometry import random_complex
    kw, freq, grid = WORKLOADS["line_bundle"]
    mesh = make_mesh("line_bundle", kw)
    ctx = slim.Context(0)
    ctx.set_mesh(mesh.verts, mesh.tris, mesh.obj, mesh.n_obj)
    lay = ctx.build(freq=freq, grid=grid, verbose=1)
    x = torch.tensor(random_complex(lay.n_sys, 7), dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    y64 = torch.zeros_like(x)

    def product_ms(prec, out):
        for _ in range(warmup):
            ctx.matvec(prec, x, out)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            ctx.matvec(prec, x, out)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t) / steps

    out = {"workload": "line_bundle over silicon (200 um, eps_r 11.9, 10 S/m) on PEC", "aim_grid": list(grid),
           "freq_hz": freq, "n_e": lay.n_e, "n_t": lay.n_t, "z_interface_below_grid_m": 1e-6,
           "free_space_product_ms": {"mixed": product_ms(slim.SLIM_MIXED, y), "fp64": product_ms(slim.SLIM_FP64, y64)}}
    z_if = lay.grid_origin[2] - 1e-6
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.set_medium(z_if, [(200e-6, 11.9, 10.0)], "pec")
    out["medium_build_s"] = time.perf_counter() - t0
    pm, pd = product_ms(slim.SLIM_MIXED, y), product_ms(slim.SLIM_FP64, y64)
    out["layered_product_ms"] = {"mixed": pm, "fp64": pd}
    out["layered_matvecs_per_s"] = {"mixed": 1e3 / pm, "fp64": 1e3 / pd}
    ne = lay.n_e
    ym, yd = y.cpu().numpy(), y64.cpu().numpy()
    out["layered_mixed_vs_fp64_rel_err"] = {
        "y1": float(np.linalg.norm(ym[:ne] - yd[:ne]) / np.linalg.norm(yd[:ne])),
        "y2": float(np.linalg.norm(ym[ne:] - yd[ne:]) / np.linalg.norm(yd[ne:]))}
    # GMRES to 1e-6 over the substrate, right-preconditioned by the (free-space) conductor blocks.
    # The excitation is the incident plane wave alone (the substrate's reflected wave is not
    # added): a fixed right-hand side for the solve time.
    b = torch.zeros_like(x)
    ctx.rhs_planewave((0.0, 0.0, -1.0), (1.0, 0.0, 0.0), b)
    sols = {}
    out["solve"] = {"rhs": "incident plane wave (E0 = 1 V/m along x, along -z), no substrate reflection",
                    "tol": 1e-6, "restart": 100, "inner_tol": 1e-6}
    for name, prec in (("mixed", slim.SLIM_MIXED), ("fp64", slim.SLIM_FP64)):
        xs = torch.zeros_like(b)
        torch.cuda.synchronize()
        info, ok = ctx.solve(b, xs, tol=1e-6, restart=100, max_iter=1000, prec=prec, inner_tol=1e-6)
        out["solve"][name] = {"seconds": info.seconds, "iterations": info.iterations, "outer": info.outer_steps,
                              "rel_residual": info.rel_residual, "converged": bool(ok)}
        sols[name] = xs
        log("layered solve %s: %s" % (name, out["solve"][name]))
    out["solve"]["mixed_vs_fp64_solution_rel_diff"] = float(
        torch.linalg.norm(sols["mixed"] - sols["fp64"]) / torch.linalg.norm(sols["fp64"]))
    n3 = grid[0] * grid[1] * grid[2]
    src = torch.tensor(random_complex(4 * n3, 5), dtype=torch.complex128, device="cuda")
    dst = torch.zeros_like(src)
    for name, prec in (("mixed", slim.SLIM_MIXED), ("fp64", slim.SLIM_FP64)):
        res = {}
        for kind, call in (("layered", lambda: ctx.aim_convolve_layered(prec, src, dst)),
                           ("free_space", lambda: ctx.aim_convolve(prec, src, dst, 4))):
            for _ in range(warmup):
                call()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(steps):
                call()
            torch.cuda.synchronize()
            res[kind + "_ms"] = 1e3 * (time.perf_counter() - t) / steps
        b = layered_bytes(grid, prec == slim.SLIM_MIXED)
        res["layered_algorithmic_bytes"] = b
        res["layered_hbm_frac"] = b / (res["layered_ms"] * 1e-3) / HBM_PEAK
        out["convolution_" + name] = res
    log("layered study: %s" % out)
    ctx.close()
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="conductors", choices=sorted(WORKLOADS))
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the GMRES time-to-1e-6 runs (mixed GMRES-IR vs FP64, plane-wave excitation)")
    ap.add_argument("--solve-max-iter", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sched", type=int, default=0)
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="only run a plain device copy of this many GiB (HBM counter calibration) and exit")
    ap.add_argument("--no-sched-study", action="store_true",
                    help="skip the makespan study (naive / LPT / trained cost model)")
    ap.add_argument("--no-layered", action="store_true",
                    help="skip the layered-medium study (bundle over a silicon substrate)")
    ap.add_argument("--layered-only", action="store_true",
                    help="only run the layered-medium study and print its JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the product is built and applied on a single MI355X "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_probe > 0:
        n = int(args.copy_probe * 2 ** 30) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: 5 copies of %d bytes" % (4 * n))
        return
    from paper_2108_03991_amd import slim
    from inputs.geometry import random_complex

    if args.layered_only:
        print(json.dumps({"layered_substrate": layered_study(args.steps, args.warmup)}), flush=True)
        return
    kw, freq, grid = WORKLOADS[args.workload]
    t0 = time.time()
    mesh = make_mesh(args.workload, kw)
    log("mesh: %d triangles, %d objects (%.1f s)" % (mesh.n_tri, mesh.n_obj, time.time() - t0))
    ctx = slim.Context(0)
    ctx.set_mesh(mesh.verts, mesh.tris, mesh.obj, mesh.n_obj)
    t0 = time.time()
    # the conductor-block preconditioner is only built for the solve
    lay = ctx.build(freq=freq, grid=grid, sched_mode=args.sched, verbose=1, precond=0 if args.no_solve else 1)
    log("build: %.1f s, n_e %d n_t %d nnzA %d nnzP %d tiles %d slots %d" % (
        time.time() - t0, lay.n_e, lay.n_t, lay.nnz_near_A, lay.nnz_near_phi, lay.n_tiles, lay.slots))
    n = lay.n_sys
    x = torch.tensor(random_complex(n, 7), dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    y64 = torch.zeros_like(x)
    stream = torch.cuda.current_stream()

    def timed(prec, steps):
        ctx.profile(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            ctx.matvec(prec, x, y if prec == slim.SLIM_MIXED else y64)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        stages, calls = ctx.profile_read()
        ctx.profile(False)
        return dt, [s / calls for s in stages]

    for _ in range(args.warmup):
        ctx.matvec(slim.SLIM_MIXED, x, y)
        ctx.matvec(slim.SLIM_FP64, x, y64)
    # timed region: the library's default path (one captured hipGraph per product,
    # the pulse path concurrent with the internal blocks), inputs resident in HBM
    rate = {}
    dt = {}
    for name, prec, out in (("mixed", slim.SLIM_MIXED, y), ("fp64", slim.SLIM_FP64, y64)):
        ctx.matvec(prec, x, out)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            ctx.matvec(prec, x, out)
        torch.cuda.synchronize()
        dt[name] = time.perf_counter() - t
        rate[name] = args.steps / dt[name]
    dt_mixed, dt_fp64 = dt["mixed"], dt["fp64"]
    # per-stage breakdown: eager and sequential, HIP events on the launch stream
    dt_pm, st_mixed = timed(slim.SLIM_MIXED, args.steps)
    dt_pd, st_fp64 = timed(slim.SLIM_FP64, args.steps)
    log("mixed %.3f ms/matvec (staged eager %.3f ms: %s)" % (1e3 * dt_mixed / args.steps, 1e3 * dt_pm / args.steps,
                                                           ["%.3f" % s for s in st_mixed]))
    log("fp64  %.3f ms/matvec (staged eager %.3f ms: %s)" % (1e3 * dt_fp64 / args.steps, 1e3 * dt_pd / args.steps,
                                                           ["%.3f" % s for s in st_fp64]))
    # accuracy of the mixed product against the FP64 product, per row block
    ne = lay.n_e
    ym, yd = y.cpu().numpy(), y64.cpu().numpy()
    err = [float(np.linalg.norm(ym[s] - yd[s]) / np.linalg.norm(yd[s])) for s in (slice(0, ne), slice(ne, n))]

    bytes_m = algorithmic_bytes(mesh, lay, True)
    bytes_d = algorithmic_bytes(mesh, lay, False)
    t_int = st_mixed[0] * 1e-3
    achieved = bytes_m["internal"] / t_int
    result = {
        "metric": METRIC,
        "value": args.steps / dt_mixed,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt_mixed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic (seeded geometry generator; random complex x)",
        "config": {
            "workload": args.workload, "seed": kw.get("seed"), "freq_hz": freq, "aim_grid": list(grid),
            "n_e": lay.n_e, "n_t": lay.n_t, "n_obj": lay.n_obj, "nnz_near_A": lay.nnz_near_A,
            "nnz_near_phi": lay.nnz_near_phi, "internal_entries": lay.internal_entries,
            "tiles": lay.n_tiles, "slots": lay.slots, "build_s": lay.build_seconds,
        },
        "fp64": {"value": args.steps / dt_fp64, "unit": "matvecs/s", "ms_per_step": 1e3 * dt_fp64 / args.steps,
                 "stage_ms": st_fp64},
        "stage_ms_mixed": {"internal": st_mixed[0], "project": st_mixed[1], "fft": st_mixed[2],
                           "pulse_rows": st_mixed[3], "rwg_rows": st_mixed[4], "cont_rows": st_mixed[5]},
        "mixed_vs_fp64_rel_err": {"y1": err[0], "y2": err[1]},
        "staged_eager_matvecs_per_s": {"mixed": args.steps / dt_pm, "fp64": args.steps / dt_pd},
        "algorithmic_bytes_mixed": bytes_m,
        "hbm_frac_whole_product": sum(bytes_m.values()) / (dt_mixed / args.steps) / HBM_PEAK,
        "roofline": {"kernel": "k_internal<mixed> (internal blocks)", "bound": "hbm", "achieved": achieved / 1e9,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": None},
    }
    if not args.no_sched_study:
        result["schedule"] = sched_study(ctx, lay, x)
        log("schedule study: %s" % result["schedule"])
    if not args.no_solve:
        result["solve"] = solve_study(ctx, lay, args.solve_max_iter)
        # the second half of the metric: seconds to a 1e-6 FP64 relative residual (null if not reached)
        result["gmres_time_to_1e-6_s"] = {
            k: (result["solve"][k]["seconds"] if result["solve"][k]["converged"] else None) for k in ("mixed", "fp64")}
    if not args.no_layered:
        ctx.close()       # frees the device arenas of this workload first
        torch.cuda.empty_cache()
        result["layered_substrate"] = layered_study()
    if not args.no_cpu_baseline:
        t0 = time.time()
        result["cpu_baseline"] = cpu_baseline(mesh, lay, freq, grid)
        log("cpu baseline %.1f s" % (time.time() - t0))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
