"""Learned scheduling of the internal tiles (the paper's task-scheduling idea, Sec. III-C):
per-tile timestamps -> cost-model network trained on the GPU -> LPT on predicted times.
Checks that every packing gives the same product, that training reduces the loss, that the
library's LPT packer is Alg. 1 on the same costs, and reports the measured makespans
(naive, LPT on flop counts, LPT on the trained model, dynamic dispatch)."""
import numpy as np
import pytest

from inputs.geometry import conductors_c5, random_complex
from tests.gpu_util import context, run_parts

pytestmark = pytest.mark.gpu


def _residual_target(samples):
    """The cost model's regression target: log time per inner iteration of the kernel
    (log duration minus the logs of the row sweeps and column chunks)."""
    return samples[:, 7] - samples[:, 5] - samples[:, 6]


def _check_cover(tiles):
    """Every row of every block is covered exactly once (the two phases together)."""
    cover = {}
    for b, r0, rows, n in tiles[:, :4].astype(int):
        cover.setdefault(b, []).append((r0, rows, n))
    for b, segs in cover.items():
        segs.sort()
        assert segs[0][0] == 0 and all(s[0] + s[1] == t[0] for s, t in zip(segs, segs[1:]))
        assert segs[-1][0] + segs[-1][1] == 2 * segs[0][2]


def test_trained_cost_model_packing():
    import torch
    m = conductors_c5(seed=3, n_obj=160)
    ctx, lay = context(m, freq=5e9, grid=(0, 0, 0), slots=64)
    x = random_complex(lay.n_sys, 2)
    ref = run_parts(ctx, lay, 0, x)
    H = torch.tensor(x[:lay.n_e], device='cuda')
    ctx.sched_record(True)
    ctx.internal_apply(1, H, timed=True)
    tiles = ctx.sched_tiles()
    samples = ctx.sched_export()
    ctx.sched_record(False)
    assert len(tiles) == lay.n_tiles and np.all(tiles[:, 6] >= tiles[:, 5]) and tiles[:, 6].max() > 0
    assert len(samples) == len(tiles)
    _check_cover(tiles)
    loss = ctx.sched_train(epochs=1500, lr=3e-3)
    assert np.isfinite(loss) and loss < np.var(_residual_target(samples))
    times = {}
    for mode in (2, 0, 1, 3, 4):
        ctx.sched_set_mode(mode)
        got = run_parts(ctx, lay, 0, x)
        assert all(np.array_equal(got[k], ref[k]) for k in ref)       # packing never changes the result
        _check_cover(ctx.sched_tiles())
        ctx.internal_apply(1, H, timed=True)
        times[mode] = np.median([ctx.internal_apply(1, H, timed=True) for _ in range(5)])
    print("makespan ms naive %.3f lpt %.3f mlp %.3f dynamic-lpt %.3f dynamic-mlp %.3f (gain of the trained model "
          "over LPT %.1f %%)" % (times[2], times[0], times[1], times[3], times[4], 100 * (times[0] / times[1] - 1)))
    assert times[1] <= times[0] * 1.05      # the learned packing does not lose to LPT on flop counts


def test_lpt_packer_matches_alg1():
    """The library's LPT packing (mode 0) against the oracle's Alg. 1 on the same task costs,
    phase by phase (rows of M_i, then rows of Z_i, each packed on its own): the same
    processor (slot) for every task, in the same order, and the same makespan.  The task
    costs are the kernel-shaped flop estimate of the library (rows rounded up to the
    eight-row sweep, row length up to the 256-column chunk); both sides break ties on the
    lowest slot index and keep equal costs in task order.  The makespan also obeys the LPT
    bound (13) against the lower bound max(sum W / P, max W) of the optimum, and no panel
    carries more than a quarter of the phase's ideal per-slot load, up to the four-row
    granule that panel heights are rounded to (the moldable split)."""
    from oracle.sched import lpt, lpt_bound
    m = conductors_c5(seed=3, n_obj=160)
    ctx, lay = context(m, freq=5e9, grid=(0, 0, 0), slots=64, precond=0)
    all_tiles = ctx.sched_tiles()[:, :5].astype(np.int64)    # block, row0, rows, n, slot (queue order)
    phase = (all_tiles[:, 1] < all_tiles[:, 3]).astype(int)  # 0: rows of M_i (row0 >= n), 1: rows of Z_i
    assert np.all(np.diff(phase) >= 0)                       # phase 0's queues come first
    n_of = {int(b): int(n) for b, n in zip(all_tiles[:, 0], all_tiles[:, 3])}
    ideal = float(sum(n * ((n + 1) & ~1) for n in n_of.values())) / lay.slots
    for ph in (0, 1):
        tiles = all_tiles[phase == ph]
        order = np.lexsort((tiles[:, 1], tiles[:, 0]))       # generation order: block, then row0
        t = tiles[order]
        ld = (t[:, 3] + 1) & ~1
        tau = [float(v) for v in ((t[:, 2] + 7) // 8 * 8) * ((ld + 255) // 256 * 256)]
        C, cmax = lpt(tau, lay.slots)
        slot_of = np.empty(len(tau), dtype=np.int64)
        for p, tasks in enumerate(C):
            slot_of[tasks] = p
        assert np.array_equal(slot_of, t[:, 4])
        # the order inside every queue is the order of assignment
        pos = {int(k): i for i, k in enumerate(order)}
        for p in range(lay.slots):
            q = [pos[k] for k in np.nonzero(tiles[:, 4] == p)[0]]
            assert q == C[p]
        F = np.zeros(lay.slots)
        np.add.at(F, t[:, 4], tau)
        assert F.max() == cmax
        assert cmax <= lpt_bound(lay.slots) * max(sum(tau) / lay.slots, max(tau)) * 1.0000001
        for rows, l in zip(t[:, 2], ld):
            assert rows * l <= 0.25 * ideal + 4 * l


def test_dynamic_queue_order():
    """Dynamic dispatch (modes 3, 4): each phase's list holds every panel of the phase once,
    in decreasing estimated cost, and repeated launches (the dispatch counters are never
    reset) keep giving the same product as the static packing."""
    import torch
    m = conductors_c5(seed=4, n_obj=160)
    ctx, lay = context(m, freq=5e9, grid=(0, 0, 0), slots=128, precond=0)
    x = random_complex(lay.n_sys, 6)
    ref = run_parts(ctx, lay, 0, x)
    ctx.sched_set_mode(3)
    t = ctx.sched_tiles()[:, :5].astype(np.int64)
    _check_cover(t)
    assert np.all(t[:, 4] == -1)
    phase = (t[:, 1] < t[:, 3]).astype(int)
    assert np.all(np.diff(phase) >= 0)
    for ph in (0, 1):
        tt = t[phase == ph]
        ld = (tt[:, 3] + 1) & ~1
        cost = ((tt[:, 2] + 7) // 8 * 8) * ((ld + 255) // 256 * 256)
        assert np.all(np.diff(cost) <= 0)
    H = torch.tensor(x[:lay.n_e], device='cuda')
    for rep in range(5):
        ctx.internal_apply(1, H)
        got = run_parts(ctx, lay, 0, x)
        assert all(np.array_equal(got[k], ref[k]) for k in ref), rep


def _record(ctx, lay, H, modes=(0, 2)):
    """Samples of the internal tiles under the given packings (the last of three timed launches)."""
    out = []
    for mode in modes:
        ctx.sched_set_mode(mode)
        ctx.sched_record(True)
        for _ in range(3):
            ctx.internal_apply(1, H, timed=True)
        out.append(ctx.sched_export())
        ctx.sched_record(False)
    ctx.sched_set_mode(0)
    return np.concatenate(out)


def test_learned_packing_held_out():
    """The cost model trained on tiles recorded on other workloads (three other seeds of the
    conductor distribution, LPT and naive packings; seeds whose meshes keep the dense external
    operator of these plain builds under 100 GB) and used on a held-out one: measured
    makespans of the naive packing, LPT on flop counts and LPT on the model's times (64
    persistent workgroups, where the packing decides the makespan).  The model must not
    lose to LPT on the held-out workload, and every packing gives the same product."""
    import torch
    pooled = []
    for seed in (4, 8, 10):
        m = conductors_c5(seed=seed, n_obj=160)
        ctx, lay = context(m, freq=5e9, grid=(0, 0, 0), slots=64, precond=0)
        H = torch.tensor(random_complex(lay.n_e, seed), device='cuda')
        pooled.append(_record(ctx, lay, H))
        ctx.close()
    data = np.concatenate(pooled)
    assert data.shape[1] == 8 and np.all(np.isfinite(data))
    m = conductors_c5(seed=3, n_obj=160)
    ctx, lay = context(m, freq=5e9, grid=(0, 0, 0), slots=64, precond=0)
    x = random_complex(lay.n_sys, 2)
    ref = run_parts(ctx, lay, 0, x)
    H = torch.tensor(x[:lay.n_e], device='cuda')
    loss = ctx.sched_train_data(data, epochs=3000, lr=3e-3)
    assert np.isfinite(loss) and loss < np.var(_residual_target(data))
    times = {}
    for mode in (2, 0, 1):
        ctx.sched_set_mode(mode)
        got = run_parts(ctx, lay, 0, x)
        assert all(np.array_equal(got[k], ref[k]) for k in ref)
        ctx.internal_apply(1, H, timed=True)
        times[mode] = np.median([ctx.internal_apply(1, H, timed=True) for _ in range(7)])
    print("held-out makespan ms naive %.3f lpt %.3f mlp %.3f (gain of the model over LPT %.1f %%; %d training tiles)"
          % (times[2], times[0], times[1], 100 * (times[0] / times[1] - 1), len(data)))
    assert times[1] <= times[0] * 1.02


def test_fewer_workgroups_for_the_z_rows():
    """The launch of the rows of Z_i on fewer workgroups than the rows of M_i (the shape the
    autotuner may pick so that the FFT's workgroups fit beside it), in static and dynamic
    modes: every row covered once, the same product bit for bit in every mode, and the
    product of a build with equal counts to the bound of two builds (the interior assembly
    sums with atomic adds, so builds agree to rounding amplified by the interior condition
    numbers, not bit for bit)."""
    from tests.gpu_util import rel
    m = conductors_c5(seed=4, n_obj=160)
    ref_ctx, ref_lay = context(m, freq=5e9, grid=(32, 32, 32), slots=256, precond=0)
    x = random_complex(ref_lay.n_sys, 11)
    ref = {prec: run_parts(ref_ctx, ref_lay, prec, x) for prec in (0, 1)}
    ref_ctx.close()
    ctx, lay = context(m, freq=5e9, grid=(32, 32, 32), slots=256, slots_z=96, precond=0)
    assert (lay.slots, lay.slots_z) == (256, 96)
    first = {}
    for mode in (0, 2, 3):
        ctx.sched_set_mode(mode)
        t = ctx.sched_tiles()
        _check_cover(t)
        if mode != 3:
            z = t[t[:, 1] < t[:, 3]]
            assert z[:, 4].max() < 96                 # the rows of Z_i go to the first 96 slots
        for prec, tol in ((0, 1e-6), (1, 1e-5)):      # FP64: g and y carry Y_eq (cond(L_k0) ~ 1e9)
            got = run_parts(ctx, lay, prec, x)
            first.setdefault(prec, got)
            assert all(np.array_equal(got[k], first[prec][k]) for k in got), (mode, prec)
            for k in ("e", "g", "y"):
                assert rel(got[k], ref[prec][k]) <= tol, (mode, prec, k, rel(got[k], ref[prec][k]))


def test_set_shape_keeps_the_product():
    """Re-shaping the two launches after the build (slim_sched_set_shape) re-packs the
    queues and leaves the product unchanged bit for bit, in static and dynamic modes and in
    both precisions -- including the FP64 rows of Z_i, which under dynamic dispatch take the
    M rows' workgroup count and a ticket counter of their own, over repeated products.  A
    Z launch wider than the M launch keeps the block product on the matrix cores correct
    (its grid covers both phases' queues).  Bad shapes are argument errors."""
    import torch
    from paper_2108_03991_amd import slim
    from tests.gpu_util import rel
    m = conductors_c5(seed=4, n_obj=160)
    ctx, lay = context(m, freq=5e9, grid=(32, 32, 32), slots=256, precond=0)
    x = random_complex(lay.n_sys, 12)
    ref = {prec: run_parts(ctx, lay, prec, x) for prec in (0, 1)}
    for mode in (0, 3):
        ctx.sched_set_mode(mode)
        for slots, slots_z in ((512, 128), (256, 512), (384, 0)):
            ctx.sched_set_shape(slots, slots_z)
            assert (ctx.layout().slots, ctx.layout().slots_z) == (slots, slots_z or slots)
            _check_cover(ctx.sched_tiles())
            for prec in (0, 1):
                for rep in range(2):
                    got = run_parts(ctx, lay, prec, x)
                    assert all(np.array_equal(got[k], ref[prec][k]) for k in got), (mode, slots, slots_z, prec, rep)
                    xt = torch.tensor(x, device="cuda")         # the captured product (Z rows beside the FFT)
                    y = torch.zeros_like(xt)
                    ctx.matvec(prec, xt, y)
                    torch.cuda.synchronize()
                    assert np.array_equal(y.cpu().numpy(), ref[prec]["y"]), (mode, slots, slots_z, prec, rep)
            if (slots, slots_z) == (256, 512):
                R = 5
                X = torch.tensor(np.stack([random_complex(lay.n_sys, 40 + q) for q in range(R)]), device="cuda")
                Y = torch.zeros_like(X)
                ctx.matvec_block(1, X, Y, R)
                torch.cuda.synchronize()
                for q in range(R):
                    one = run_parts(ctx, lay, 0, X[q].cpu().numpy())["y"]
                    assert rel(Y[q].cpu().numpy(), one) <= 1e-5, (mode, q)
    for bad in ((0, 0), (-4, 0), (256, -1), (1 << 17, 0)):
        with pytest.raises(slim.SlimError) as ei:
            ctx.sched_set_shape(*bad)
        assert ei.value.code == 1
    fresh = slim.Context(0)
    with pytest.raises(slim.SlimError) as ei:
        fresh.sched_set_shape(256, 0)
    assert ei.value.code == 3
    fresh.close()
