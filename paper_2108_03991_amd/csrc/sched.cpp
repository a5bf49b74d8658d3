// Packing of the internal tasks into the persistent kernel's work queues.
//
// The paper balances the internal workload as a parallel-task scheduling
// problem (Sec. III-C): LPT (Alg. 1) for sequential tasks and Part_Schedule,
// which gives a long task more processors, for moldable ones; the workload of
// object i is estimated as W_i = N_E,i^2.  On one GPU a "processor" is a
// persistent workgroup (slot) and a task is a row panel of the stacked block
// [Z_i; M_i].
//
// The rows fall into two phases that are packed and launched separately: the
// M_i rows (g = M H and j = H - g, which the AIM projection needs) and then the
// Z_i rows (e = Z H, needed only by the final row combine), so that the second
// launch can run concurrently with the projection and the FFT.  In each phase a
// block is split into P_i panels so that no panel exceeds a quarter of the
// phase's ideal per-slot load (the moldable step), and the panels are ordered or
// placed on their estimated time (with the sparse Z~ of the high-frequency form there
// are no dense Z_i rows, and phase 1 is a sparse product instead):
//   mode 0: LPT (Alg. 1) on a flop-count estimate of the kernel as written: rows
//           rounded up to the eight-row wave sweep times the row length rounded up
//           to the 256-column chunk, since lanes past the end of a short row idle
//           (the LPT fallback),
//   mode 1: LPT on the time predicted by the trained cost-model network,
//   mode 2: naive -- objects in mesh order, round robin, one panel height,
//   mode 3: dynamic dispatch in decreasing flop-count order: one queue per phase,
//           each workgroup takes the next panel when it finishes its last one
//           (Alg. 1's rule -- the next task goes to the first processor to become
//           free -- applied with measured rather than estimated finish times),
//   mode 4: dynamic dispatch in decreasing predicted-time order.
// The block product on the matrix cores draws its panels (both phases) the same
// way: from the static queues, or from one dynamic queue in the dynamic modes.
#include <algorithm>
#include <numeric>
#include <queue>

#include "ctx.hpp"

namespace slim {

double mlp_predict_time(const Ctx& c, int block, int rows);   // mlp.hip

void pack_tiles(Ctx& c, int mode) {
  SLIM_REQUIRE(mode >= 0 && mode <= 4, SLIM_E_ARG, "unknown scheduling mode");
  c.drop_graphs();   // captured products point at the old queues
  const int nb = int(c.blocks.size());
  SLIM_REQUIRE(c.slots > 0, SLIM_E_STATE, "slot count not set");
  const bool learned = (mode == 1 || mode == 4) && !c.mlp_params.empty();
  struct Task { int block, row0, rows; double cost; };
  c.tiles.clear();
  c.slot_start.assign(size_t(c.slots + 1) + size_t(c.zslots() + 1), 0);
  for (int phase = 0; phase < 2; ++phase) {
    // phase 0: rows [n, 2n) of every block (M_i); phase 1: rows [0, n) (Z_i), on its own
    // number of workgroups (fewer leave room for the FFT passes that run beside it)
    const int S = phase == 0 ? c.slots : c.zslots();
    std::vector<Task> tasks;
    double total = 0.0;
    for (int i = 0; i < nb; ++i) total += c.blocks[i].n * double((c.blocks[i].n + 1) & ~1);
    const double ideal = total / S;
    for (int i = 0; i < nb && !(phase == 1 && c.hf_sparse); ++i) {   // sparse Z~: no dense rows of Z_i
      const int n = c.blocks[i].n, ld = (n + 1) & ~1, base = phase == 0 ? n : 0;
      int R;
      if (mode == 2) {
        R = std::max(4, c.tile_rows);
      } else {
        // moldable step: P_i panels so that each costs <= ideal / 4 (heights rounded up
        // to four rows; the matrix-core kernel masks the rows of a partial 16-row group)
        const double w = double(n) * ld;
        const int64_t P = std::max<int64_t>(1, int64_t(std::ceil(w / (0.25 * ideal))));
        R = int(std::min<int64_t>(n, std::max<int64_t>(4, (n + P - 1) / P)));
        R = std::min(n, ((R + 3) / 4) * 4);
      }
      for (int r0 = 0; r0 < n; r0 += R) {
        const int rr = std::min(R, n - r0);
        double cost = double((rr + 7) / 8 * 8) * double((ld + 255) / 256 * 256);
        if (learned) cost = mlp_predict_time(c, i, rr);
        tasks.push_back({i, base + r0, rr, cost});
      }
    }
    const size_t first = c.tiles.size();
    int32_t* ss = c.slot_start.data() + (phase == 0 ? 0 : size_t(c.slots + 1));
    ss[0] = int32_t(first);
    if (mode == 2) {
      // naive: round robin in generation order; slot s's queue is contiguous
      std::vector<std::vector<Tile>> q(S);
      for (size_t k = 0; k < tasks.size(); ++k)
        q[k % S].push_back({tasks[k].block, tasks[k].row0, tasks[k].rows, int(k % S)});
      for (int s = 0; s < S; ++s) {
        c.tiles.insert(c.tiles.end(), q[s].begin(), q[s].end());
        ss[s + 1] = int32_t(c.tiles.size());
      }
    } else {
      // decreasing estimated time (equal costs keep the generation order)
      std::vector<int> order(tasks.size());
      std::iota(order.begin(), order.end(), 0);
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return tasks[a].cost > tasks[b].cost; });
      if (mode == 3 || mode == 4) {
        // one queue in that order, drawn from by whichever workgroup is free; the
        // static ranges below (contiguous shares of the list) are unused by the kernels
        for (size_t k = 0; k < order.size(); ++k) {
          const Task& t = tasks[order[k]];
          c.tiles.push_back({t.block, t.row0, t.rows, -1});
        }
        const int64_t cnt = int64_t(order.size());
        for (int s = 0; s < S; ++s) ss[s + 1] = int32_t(first + (s + 1) * cnt / S);
      } else {
        // LPT (Alg. 1): each task to the slot that finishes first (lowest index on ties)
        std::vector<std::vector<Tile>> q(S);
        using E = std::pair<double, int>;
        std::priority_queue<E, std::vector<E>, std::greater<E>> pq;
        for (int s = 0; s < S; ++s) pq.push({0.0, s});
        for (int k : order) {
          E e = pq.top();
          pq.pop();
          q[e.second].push_back({tasks[k].block, tasks[k].row0, tasks[k].rows, e.second});
          pq.push({e.first + tasks[k].cost, e.second});
        }
        for (int s = 0; s < S; ++s) {
          c.tiles.insert(c.tiles.end(), q[s].begin(), q[s].end());
          ss[s + 1] = int32_t(c.tiles.size());
        }
      }
    }
    c.phase_first[phase] = int32_t(first);
    c.phase_count[phase] = int32_t(c.tiles.size() - first);
  }
  c.dynamic = mode == 3 || mode == 4;
  std::vector<int32_t> flat(4 * c.tiles.size());
  for (size_t k = 0; k < c.tiles.size(); ++k) {
    flat[4 * k] = c.tiles[k].block;
    flat[4 * k + 1] = c.tiles[k].row0;
    flat[4 * k + 2] = c.tiles[k].rows;
    flat[4 * k + 3] = c.tiles[k].slot;
  }
  c.d_tiles.upload(flat);
  c.d_slot_start.upload(c.slot_start);
  c.d_stamps.alloc(std::max<size_t>(1, 2 * c.tiles.size()) * sizeof(unsigned long long));
  c.d_span.alloc(2 * size_t(c.slots + std::max(c.slots, c.zslots())) * sizeof(unsigned long long));
  // one ticket counter per (queue, grid size): a launch takes exactly count + grid
  // tickets, so a counter keeps its meaning only while its launches keep one grid size
  c.d_qctr.upload(std::vector<unsigned long long>(5, 0ull));
  c.sched_mode = mode;
}

}  // namespace slim
