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

}  // namespace fse
