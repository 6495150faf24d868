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
//
// Refined order (the alternative criterion Section 3 mentions): N(b) counts
// the lost, not yet extrapolated samples of the neighbours (a cell outside
// the image counts a whole block), waves are formed as above, and a finished
// block's samples leave its pending neighbours' N.  With whole-block losses N
// is a fixed multiple of Algorithm 1's N and the two orders coincide.
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
  // The grid padded by one ring of cells outside the image: a neighbour
  // outside counts as not extrapolated, which is the +3 margin / +5 corner
  // rule, and the 8 neighbours of a cell are at fixed offsets.
  const int W2 = wb + 2, H2 = hb + 2, n2 = W2 * H2;
  const int nbr[8] = {-W2 - 1, -W2, -W2 + 1, -1, 1, W2 - 1, W2, W2 + 1};
  std::vector<uint8_t> open(n2, 1);  // 1: not extrapolated (outside, or lost)
  for (int i = 0; i < hb; ++i)
    for (int j = 0; j < wb; ++j) open[(i + 1) * W2 + j + 1] = lost[i * wb + j] ? 1 : 0;
  // N per cell (-1: finished or outside); pending cells by N (0..8) in one
  // bitset per N over the padded index, so a wave visits only the cells with
  // the smallest N, in raster order
  std::vector<int8_t> cnt(n2, -1);
  const int nwords = (n2 + 63) / 64;
  std::vector<uint64_t> bucket((size_t)9 * nwords, 0);
  auto set_bit = [&](int c, int p) { bucket[(size_t)c * nwords + (p >> 6)] |= 1ull << (p & 63); };
  auto clr_bit = [&](int c, int p) {
    bucket[(size_t)c * nwords + (p >> 6)] &= ~(1ull << (p & 63));
  };
  int npending = 0;
  for (int i = 1; i <= hb; ++i)
    for (int j = 1; j <= wb; ++j) {
      const int p = i * W2 + j;
      if (!lost[(i - 1) * wb + j - 1]) continue;
      int c = 0;
      for (int k = 0; k < 8; ++k) c += open[p + nbr[k]];
      cnt[p] = (int8_t)c;
      set_bit(c, p);
      ++npending;
    }
  std::vector<uint8_t> blocked(n2, 0);
  std::vector<int32_t> taken;
  int wave = 0;
  while (npending > 0) {
    int nmin = 0;
    for (;; ++nmin) {
      const uint64_t* w = &bucket[(size_t)nmin * nwords];
      bool any = false;
      for (int k = 0; k < nwords && !any; ++k) any = w[k] != 0;
      if (any) break;
    }
    taken.clear();
    const uint64_t* w = &bucket[(size_t)nmin * nwords];
    for (int k = 0; k < nwords; ++k) {
      for (uint64_t x = w[k]; x; x &= x - 1) {
        const int p = (k << 6) | __builtin_ctzll(x);
        if (blocked[p]) continue;
        taken.push_back(p);
        // a block adjacent to a taken one cannot join this wave
        for (int q = 0; q < 8; ++q) blocked[p + nbr[q]] = 1;
      }
    }
    for (int32_t p : taken) {
      const int b = (p / W2 - 1) * wb + (p % W2 - 1);
      wave_of[b] = wave;
      if (seq) seq->push_back(b);
      for (int q = 0; q < 8; ++q) blocked[p + nbr[q]] = 0;
    }
    for (int32_t p : taken) {
      clr_bit(nmin, p);
      cnt[p] = -1;
      --npending;
      for (int k = 0; k < 8; ++k) {
        const int q = p + nbr[k];
        if (cnt[q] >= 0) {
          clr_bit(cnt[q], q);
          --cnt[q];
          set_bit(cnt[q], q);
        }
      }
    }
    ++wave;
  }
  return wave;
}

int schedule_blocks_refined(int hb, int wb, const int32_t* unknown, int32_t outside,
                            int32_t* wave_of, std::vector<int32_t>* seq) {
  const int nb = hb * wb;
  for (int b = 0; b < nb; ++b) wave_of[b] = -1;
  if (seq) seq->clear();
  // padded grid as above: the ring of outside cells holds `outside` unknown
  // samples that never become known
  const int W2 = wb + 2, H2 = hb + 2, n2 = W2 * H2;
  const int nbr[8] = {-W2 - 1, -W2, -W2 + 1, -1, 1, W2 - 1, W2, W2 + 1};
  std::vector<int64_t> left(n2, outside);  // unknown samples per cell
  for (int i = 0; i < hb; ++i)
    for (int j = 0; j < wb; ++j) left[(i + 1) * W2 + j + 1] = std::max(0, unknown[i * wb + j]);
  // pending cells in raster order of the padded index, with their N
  std::vector<int32_t> pend;
  std::vector<int64_t> cnt(n2, -1);
  for (int i = 1; i <= hb; ++i)
    for (int j = 1; j <= wb; ++j) {
      const int p = i * W2 + j;
      if (left[p] <= 0) continue;
      int64_t c = 0;
      for (int k = 0; k < 8; ++k) c += left[p + nbr[k]];
      cnt[p] = c;
      pend.push_back(p);
    }
  std::vector<uint8_t> blocked(n2, 0);
  std::vector<int32_t> taken;
  int wave = 0;
  while (!pend.empty()) {
    int64_t nmin = cnt[pend[0]];
    for (int32_t p : pend) nmin = std::min(nmin, cnt[p]);
    taken.clear();
    for (int32_t p : pend) {
      if (cnt[p] != nmin || blocked[p]) continue;
      taken.push_back(p);
      for (int q = 0; q < 8; ++q) blocked[p + nbr[q]] = 1;
    }
    for (int32_t p : taken) {
      const int b = (p / W2 - 1) * wb + (p % W2 - 1);
      wave_of[b] = wave;
      if (seq) seq->push_back(b);
      for (int q = 0; q < 8; ++q) blocked[p + nbr[q]] = 0;
    }
    for (int32_t p : taken) {
      cnt[p] = -1;
      for (int k = 0; k < 8; ++k) {
        const int q = p + nbr[k];
        if (cnt[q] >= 0) cnt[q] -= left[p];
      }
      left[p] = 0;
    }
    // drop the finished cells, keeping raster order
    pend.erase(std::remove_if(pend.begin(), pend.end(), [&](int32_t p) { return cnt[p] < 0; }),
               pend.end());
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

// Three-dimensional order: the grid padded by one layer of outside cells on
// every face, so the 26 neighbours of a cell are at fixed offsets; N per
// pending cell = its not-extrapolated neighbours (outside or lost and not yet
// done); each wave takes the cells with the smallest N in raster order
// (frame, row, column) unless a 26-neighbour is already in the wave; after
// the wave every pending neighbour of a taken cell loses one.
int schedule_blocks3(int tb, int hb, int wb, const uint8_t* lost, int order, int32_t* wave_of,
                     std::vector<int32_t>* seq) {
  const int nb = tb * hb * wb;
  for (int b = 0; b < nb; ++b) wave_of[b] = -1;
  if (seq) seq->clear();
  if (nb <= 0) return 0;
  if (order == 1) {
    int w = 0;
    for (int b = 0; b < nb; ++b)
      if (lost[b]) {
        wave_of[b] = w++;
        if (seq) seq->push_back(b);
      }
    return w;
  }
  const int W2 = wb + 2, H2 = hb + 2, T2 = tb + 2, plane = W2 * H2, n2 = plane * T2;
  std::vector<int> nbr;
  for (int a = -1; a <= 1; ++a)
    for (int di = -1; di <= 1; ++di)
      for (int dj = -1; dj <= 1; ++dj)
        if (a || di || dj) nbr.push_back(a * plane + di * W2 + dj);
  auto pad = [&](int t, int i, int j) { return ((t + 1) * H2 + i + 1) * W2 + j + 1; };
  std::vector<uint8_t> open(n2, 1);  // 1: not extrapolated (outside, or lost and pending)
  std::vector<int32_t> cell_of(n2, -1);
  for (int t = 0; t < tb; ++t)
    for (int i = 0; i < hb; ++i)
      for (int j = 0; j < wb; ++j) {
        const int b = (t * hb + i) * wb + j, c = pad(t, i, j);
        open[c] = lost[b] ? 1 : 0;
        cell_of[c] = b;
      }
  std::vector<int> cnt(n2, -1);
  int npending = 0;
  for (int c = 0; c < n2; ++c) {
    if (cell_of[c] < 0 || !lost[cell_of[c]]) continue;
    int k = 0;
    for (int o : nbr) k += open[c + o];
    cnt[c] = k;
    ++npending;
  }
  std::vector<uint8_t> taken(n2, 0);
  std::vector<int> wave;
  int waves = 0;
  while (npending > 0) {
    int nmin = 1 << 30;
    for (int c = 0; c < n2; ++c)
      if (cnt[c] >= 0 && cnt[c] < nmin) nmin = cnt[c];
    wave.clear();
    for (int c = 0; c < n2; ++c) {  // padded raster order = (frame, row, column)
      if (cnt[c] != nmin) continue;
      bool clash = false;
      for (int o : nbr) clash |= taken[c + o] != 0;
      if (clash) continue;
      taken[c] = 1;
      wave.push_back(c);
    }
    for (int c : wave) {
      taken[c] = 0;
      cnt[c] = -1;
      open[c] = 0;
      wave_of[cell_of[c]] = waves;
      if (seq) seq->push_back(cell_of[c]);
      --npending;
      for (int o : nbr)
        if (cnt[c + o] >= 0) --cnt[c + o];
    }
    ++waves;
  }
  return waves;
}

}  // namespace fse
