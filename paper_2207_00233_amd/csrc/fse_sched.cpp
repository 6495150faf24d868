// fse_sched.cpp -- block processing orders of the paper.
//
// Line scan (Section 2): every block with lost samples, left to right, top to
// bottom, one block per wave.
//
// Optimized order (Section 3, Algorithm 1, Eq. (3)): N(b) = number of
// neighbouring blocks not yet extrapolated, where a neighbour outside the
// image counts as not extrapolated (margin blocks +3, corner blocks +5 with
// the 8-neighbourhood); blocks without losses are finished (N = -1).  Each
// wave takes, in raster order, every pending block whose N equals the
// smallest non-negative N and that touches no block already taken for this
// wave; after the wave every taken block is finished and its pending
// neighbours lose one not-extrapolated neighbour.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "fse_sched.h"

namespace fse {

int schedule_blocks(int hb, int wb, const uint8_t* lost, int order, int32_t* wave_of,
                    std::vector<int32_t>* seq) {
  const int nb = hb * wb;
  for (int b = 0; b < nb; ++b) wave_of[b] = -1;
  if (seq) seq->clear();
  if (order == 1) {
    int w = 0;
    for (int b = 0; b < nb; ++b)
      if (lost[b]) {
        wave_of[b] = w++;
        if (seq) seq->push_back(b);
      }
    return w;
  }
  // Neighbour lists (8-neighbourhood, inside the grid).
  auto for_neighbours = [&](int b, auto&& fn) {
    const int i = b / wb, j = b % wb;
    const int i0 = i > 0 ? i - 1 : 0, i1 = i + 1 < hb ? i + 1 : hb - 1;
    const int j0 = j > 0 ? j - 1 : 0, j1 = j + 1 < wb ? j + 1 : wb - 1;
    for (int y = i0; y <= i1; ++y)
      for (int x = j0; x <= j1; ++x)
        if (y != i || x != j) fn(y * wb + x);
  };
  std::vector<int> cnt(nb, 0);
  std::vector<int32_t> pending;
  pending.reserve(nb);
  for (int b = 0; b < nb; ++b) {
    int inside = 0;
    for_neighbours(b, [&](int q) {
      ++inside;
      if (lost[q]) ++cnt[b];
    });
    cnt[b] += 8 - inside;
    if (lost[b]) pending.push_back(b);
    else cnt[b] = -1;
  }
  // `pending` stays in raster order; finished blocks are compacted out.
  std::vector<uint8_t> blocked(nb, 0);
  std::vector<int32_t> taken;
  int wave = 0;
  while (!pending.empty()) {
    int nmin = cnt[pending[0]];
    for (int32_t b : pending)
      if (cnt[b] < nmin) nmin = cnt[b];
    taken.clear();
    for (int32_t b : pending) {
      if (cnt[b] != nmin || blocked[b]) continue;
      taken.push_back(b);
      // a block adjacent to a taken one cannot join this wave
      for_neighbours(b, [&](int q) { blocked[q] = 1; });
    }
    for (int32_t b : taken) {
      wave_of[b] = wave;
      if (seq) seq->push_back(b);
      for_neighbours(b, [&](int q) { blocked[q] = 0; });
    }
    for (int32_t b : taken) {
      cnt[b] = -1;
      for_neighbours(b, [&](int q) {
        if (cnt[q] >= 0) --cnt[q];
      });
    }
    size_t k = 0;
    for (int32_t b : pending)
      if (cnt[b] >= 0) pending[k++] = b;
    pending.resize(k);
    ++wave;
  }
  return wave;
}

// Staggered start of the frames of a batch.  Launch step s runs wave s - off[f]
// of every frame f (when that wave exists), so each frame keeps its own wave
// order and gets exactly its stand-alone result; only which waves share a
// launch changes.  A launch costs about max(latency, blocks / rate), so the
// offsets move the large early waves of short frames onto the steps where the
// long frames only have small waves.  Greedy: frames by decreasing wave count,
// each at the offset (within the longest frame's span) that adds least cost.
std::vector<int> stagger_frames(const std::vector<std::vector<int>>& sizes, double latency_us,
                                double blocks_per_us) {
  const int n = (int)sizes.size();
  int T = 0;
  for (const auto& v : sizes) T = std::max<int>(T, (int)v.size());
  std::vector<int> off(n, 0), order(n);
  for (int f = 0; f < n; ++f) order[f] = f;
  auto total = [&](int f) {
    long t = 0;
    for (int x : sizes[f]) t += x;
    return t;
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (sizes[a].size() != sizes[b].size()) return sizes[a].size() > sizes[b].size();
    return total(a) > total(b);
  });
  auto cost = [&](double x) { return x <= 0 ? 0.0 : std::max(latency_us, x / blocks_per_us); };
  std::vector<double> load(T, 0.0);
  for (int f : order) {
    const int nw = (int)sizes[f].size();
    int best_o = 0;
    double best_c = 0;
    for (int o = 0; o + nw <= T; ++o) {
      double c = 0;
      for (int t = 0; t < nw; ++t) c += cost(load[o + t] + sizes[f][t]) - cost(load[o + t]);
      if (o == 0 || c < best_c - 1e-9) {
        best_c = c;
        best_o = o;
      }
    }
    off[f] = best_o;
    for (int t = 0; t < nw; ++t) load[best_o + t] += sizes[f][t];
  }
  return off;
}

}  // namespace fse
