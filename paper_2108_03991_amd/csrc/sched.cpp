// Packing of the internal tasks into the persistent kernel's work queues.
//
// The paper balances the internal workload as a parallel-task scheduling
// problem (Sec. III-C): LPT (Alg. 1) for sequential tasks and Part_Schedule,
// which gives a long task more processors, for moldable ones; the workload of
// object i is estimated as W_i = N_E,i^2.  On one GPU a "processor" is a
// persistent workgroup (slot) and a task is a row panel of the stacked block
// [Z_i; M_i].  A block is split into P_i panels so that no panel exceeds a
// quarter of the ideal per-slot load (the moldable step), then all panels are
// placed by LPT on their estimated time:
//   mode 0: flop-count estimate of the kernel as written: rows rounded up to the
//           eight-row wave sweep times the row length rounded up to the 256-column
//           chunk, since lanes past the end of a short row idle (the LPT fallback),
//   mode 1: time predicted by the trained cost-model network,
//   mode 2: naive -- objects in mesh order, round robin, one panel height.
#include <algorithm>
#include <numeric>
#include <queue>

#include "ctx.hpp"

namespace slim {

float mlp_predict_host(const Ctx& c, const float* feat);   // mlp.hip
void tile_features(const Ctx& c, int block, int rows, float* feat);

void pack_tiles(Ctx& c, int mode) {
  c.drop_graphs();   // captured products point at the old queues
  const int nb = int(c.blocks.size());
  SLIM_REQUIRE(c.slots > 0, SLIM_E_STATE, "slot count not set");
  const int S = c.slots;
  struct Task { int block, row0, rows; double cost; };
  std::vector<Task> tasks;
  double total = 0.0;
  for (int i = 0; i < nb; ++i) total += 2.0 * c.blocks[i].n * double((c.blocks[i].n + 1) & ~1);
  const double ideal = total / S;
  if (mode == 2) {
    // naive: fixed panel height, blocks in order, round robin over the slots
    const int R = std::max(4, c.tile_rows);
    for (int i = 0; i < nb; ++i)
      for (int r0 = 0; r0 < 2 * c.blocks[i].n; r0 += R)
        tasks.push_back({i, r0, std::min(R, 2 * c.blocks[i].n - r0), 0.0});
    c.tiles.clear();
    std::vector<std::vector<Tile>> q(S);
    for (size_t k = 0; k < tasks.size(); ++k) q[k % S].push_back({tasks[k].block, tasks[k].row0, tasks[k].rows, int(k % S)});
    c.slot_start.assign(S + 1, 0);
    for (int s = 0; s < S; ++s) {
      c.slot_start[s + 1] = c.slot_start[s] + int32_t(q[s].size());
      c.tiles.insert(c.tiles.end(), q[s].begin(), q[s].end());
    }
  } else {
    // moldable step: P_i panels per block so that each panel costs <= ideal/4; panel
    // heights are whole 16-row groups (the row tile of the matrix-core kernel)
    for (int i = 0; i < nb; ++i) {
      const int n = c.blocks[i].n, ld = (n + 1) & ~1, rows = 2 * n;
      double w = double(rows) * ld;
      int64_t P = std::max<int64_t>(1, int64_t(std::ceil(w / (0.25 * ideal))));
      int R = int(std::min<int64_t>(rows, std::max<int64_t>(16, (rows + P - 1) / P)));
      R = std::min(rows, ((R + 15) / 16) * 16);
      for (int r0 = 0; r0 < rows; r0 += R) {
        const int rr = std::min(R, rows - r0);
        double cost = double((rr + 7) / 8 * 8) * double((ld + 255) / 256 * 256);
        if (mode == 1 && !c.mlp_params.empty()) {
          float f[8];
          tile_features(c, i, rr, f);
          cost = std::exp(double(mlp_predict_host(c, f)));
        }
        tasks.push_back({i, r0, rr, cost});
      }
    }
    // LPT (Alg. 1): decreasing estimated time, earliest-finishing slot (lowest index on ties)
    std::vector<int> order(tasks.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return tasks[a].cost > tasks[b].cost; });
    using E = std::pair<double, int>;
    std::priority_queue<E, std::vector<E>, std::greater<E>> pq;
    for (int s = 0; s < S; ++s) pq.push({0.0, s});
    std::vector<std::vector<Tile>> q(S);
    for (int k : order) {
      E e = pq.top();
      pq.pop();
      q[e.second].push_back({tasks[k].block, tasks[k].row0, tasks[k].rows, e.second});
      pq.push({e.first + tasks[k].cost, e.second});
    }
    c.tiles.clear();
    c.slot_start.assign(S + 1, 0);
    for (int s = 0; s < S; ++s) {
      c.slot_start[s + 1] = c.slot_start[s] + int32_t(q[s].size());
      c.tiles.insert(c.tiles.end(), q[s].begin(), q[s].end());
    }
  }
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
  c.sched_mode = mode;
}

}  // namespace slim
