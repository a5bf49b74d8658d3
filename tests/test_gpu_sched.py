"""Learned scheduling of the internal tiles (the paper's task-scheduling idea, Sec. III-C):
per-tile timestamps -> cost-model network trained on the GPU -> LPT on predicted times.
Checks that every packing gives the same product, that training reduces the loss, and
reports the measured makespans (naive, LPT on flop counts, LPT on the trained model)."""
import numpy as np
import pytest

from inputs.geometry import conductors_c5, random_complex
from tests.gpu_util import context, run_parts

pytestmark = pytest.mark.gpu


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
    ctx.sched_record(False)
    assert len(tiles) == lay.n_tiles and np.all(tiles[:, 6] >= tiles[:, 5]) and tiles[:, 6].max() > 0
    # every row of every block is covered exactly once
    cover = {}
    for b, r0, rows, n in tiles[:, :4].astype(int):
        cover.setdefault(b, []).append((r0, rows, n))
    for b, segs in cover.items():
        segs.sort()
        assert segs[0][0] == 0 and all(s[0] + s[1] == t[0] for s, t in zip(segs, segs[1:]))
        assert segs[-1][0] + segs[-1][1] == 2 * segs[0][2]
    loss = ctx.sched_train(epochs=1500, lr=3e-3)
    assert np.isfinite(loss) and loss < np.var(np.log(np.maximum(tiles[:, 6] - tiles[:, 5], 1.0)))
    times = {}
    for mode in (2, 0, 1):
        ctx.sched_set_mode(mode)
        got = run_parts(ctx, lay, 0, x)
        assert all(np.array_equal(got[k], ref[k]) for k in ref)       # packing never changes the result
        ctx.internal_apply(1, H, timed=True)
        times[mode] = np.median([ctx.internal_apply(1, H, timed=True) for _ in range(5)])
    print("makespan ms naive %.3f lpt %.3f mlp %.3f (gain of the trained model over LPT %.1f %%)"
          % (times[2], times[0], times[1], 100 * (times[0] / times[1] - 1)))
    assert times[1] <= times[0] * 1.05      # the learned packing does not lose to LPT on flop counts


def test_lpt_packer_matches_alg1():
    """The library's LPT packing (mode 0) against the oracle's Alg. 1 on the same task costs:
    the same processor (slot) for every task, in the same order, and the same makespan.
    The task costs are the kernel-shaped flop estimate of the library (rows rounded up to
    the eight-row sweep, row length up to the 256-column chunk); both sides break ties on
    the lowest slot index and keep equal costs in task order.  The makespan also obeys
    the LPT bound (13) against the lower bound max(sum W / P, max W) of the optimum, and
    no panel carries more than a quarter of the ideal per-slot load, up to the 16-row
    granule that panel heights are rounded to (the moldable split)."""
    from oracle.sched import lpt, lpt_bound
    m = conductors_c5(seed=3, n_obj=160)
    ctx, lay = context(m, freq=5e9, grid=(0, 0, 0), slots=64, precond=0)
    tiles = ctx.sched_tiles()[:, :5].astype(np.int64)        # block, row0, rows, n, slot (queue order)
    order = np.lexsort((tiles[:, 1], tiles[:, 0]))          # generation order: block, then row0
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
    ideal = float(np.sum(t[:, 2] * ld)) / lay.slots
    for rows, l in zip(t[:, 2], ld):
        assert rows * l <= 0.25 * ideal + 16 * l
