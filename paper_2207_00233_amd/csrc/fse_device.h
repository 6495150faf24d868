// fse_device.h -- types shared by the HIP kernels and the host runtime of the
// FSE library (device-side layout of frames, work items and kernel args).
#pragma once
#include <stdint.h>

namespace fse {

constexpr int kFft = 64;          // basis grid edge (64 x 64 DFT basis)
constexpr int kHalf = kFft / 2 + 1;          // 33 columns of a real row DFT

// Per-sample state in the device state map.
enum : uint8_t { kKnown = 0, kPending = 1, kRecon = 2 };

struct FrameDesc {
  int64_t off;   // element offset of the frame in the work/state arenas
  int32_t H, W;  // image size
};

// Per-frame input/output pointers of the batched init and finalize kernels.
struct IoDesc {
  const uint8_t* image;  // 8-bit input (device)
  const uint8_t* lost;   // loss mask (device)
  uint8_t* out;          // 8-bit output (device)
  float* of32;           // nullable unquantized outputs (device, contiguous)
  double* of64;
  int64_t off;           // element offset in the work/state arenas
  int64_t flag_off;      // offset of the frame's block flags
  int32_t stride, lstride, ostride;
  int32_t H, W, wb;
};

// Arguments of the fused per-block kernel.  T = float or double.
template <typename T>
struct BlockArgs {
  T* work;                 // working image arena (values of every frame)
  uint8_t* state;          // state arena (kKnown / kPending / kRecon)
  const FrameDesc* frames;
  const int32_t* items;    // 2 ints per work item: frame | priority << 24, (bi << 16) | bj
  const T* radial;         // M*N table rho^dist of Eq. (2)
  const double* radial64;  // the same table in double (re-rank transforms)
  const T* twid;           // 64 x (cos, sin)(2 pi t / 64) in T
  const double* twid64;    // 64 x (cos, sin)(2 pi t / 64) in double
  T* staging;              // nullable: results go here (d > block size)
  int32_t* trace_u;        // nullable: [items * K]
  T* trace_dc;             // nullable: [items * K * 2]
  int32_t M, N, Bh, Bw, d, gox, goy, K;
  T delta, gamma, zscale;  // zscale balances x and w in the packed DFT
  double empty_fill;
  double delta64, gamma64; // the same parameters in double (FP64 transforms, re-rank)
  double* spec64;          // FP64 spectra per work item (re-rank mode), see below
  double rerank_gap;       // relative |R|^2 gap that triggers an exact re-score
  unsigned long long* counters;  // nullable: re-scoring statistics (kCnt*)
};

// Re-scoring statistics of a call (BlockArgs::counters, summed over blocks).
enum : int {
  kCntRescored = 0,   // iterations whose selection was re-scored exactly
  kCntCandidates = 1, // candidates re-scored (over all wavefronts)
  kCntWide = 2,       // wavefront re-scores that took several rounds of candidates
  kCntMaxWave = 3,    // most candidates one wavefront re-scored in one iteration
  kCntSlots = 4
};

// Work item encoding: the first int holds the frame index in its low 24 bits
// and, above them, a flag that raises the wave priority of the item's
// workgroup (items on a batch's critical chain of waves).
constexpr int32_t kItemFrameMask = 0xffffff;
constexpr int kItemPrioShift = 24;

// FP64 spectra of one work item written by the re-rank mode's transforms:
// R0, then W, each the columns k2 = 0..32 of its 64 rows (complex, row
// pitch 33; the spectra of real data are Hermitian, the other columns are
// the conjugates of these).
constexpr int64_t kSpecR0 = 0;                      // in doubles
constexpr int64_t kSpecW = 2 * kFft * kHalf;
constexpr int64_t kSpecStride = 4 * kFft * kHalf;   // doubles per item (256-byte multiple)
static_assert(kSpecStride * 8 % 256 == 0, "items' spectra stay 256-byte aligned");

// Byte offsets of the dynamic LDS regions of the fused block kernel with
// `waves` wavefronts per workgroup (rows = 64 / waves spectrum rows each).
struct LdsLayout {
  int64_t cs;        // compact staging (4 wavefronts): weight classes
  int64_t bx, bw;    // phase B: row DFTs of x and w (M x 33 complex each)
  int64_t hist_dc;   // K complex coefficient increments
  int64_t hist_u;    // K selected indices
  int64_t tw64;      // 64 x (cos, sin) in double
  int64_t twt;       // the same in T
  int64_t slots;     // 2 x waves argmax slots of 32 bytes
  int64_t cand;      // re-rank: 2 x waves exact-candidate slots of 32 bytes
  int64_t misc;      // 32 bytes
  int64_t total;
};

__host__ __device__ inline int64_t align16(int64_t v) { return (v + 15) & ~15LL; }

// `stage_needed` = false for the re-rank kernel, whose FP64 transforms use
// the W region as their grid (fp64_grid below) instead of the float staging.
__host__ __device__ inline LdsLayout lds_layout(int M, int N, int K, int waves, int tsize,
                                                bool stage_needed = true) {
  LdsLayout L;
  const int NP = N | 1;  // odd row pitch of the staged area
  const int rows = kFft / waves;
  // staging: with 4 wavefronts the samples (T) and one weight class per
  // sample, otherwise x and w (T each); then the row DFTs of x and w (M x 33
  // complex each); the 64 x 64 complex exchange buffer of the column DFT
  // reuses the region afterwards
  if (waves == 4) {
    L.cs = align16((int64_t)M * NP * tsize);
    L.bx = align16(L.cs + (int64_t)M * NP);
  } else {
    L.cs = 0;
    L.bx = 2LL * M * NP * tsize;
  }
  L.bw = L.bx + (int64_t)M * kHalf * 2 * tsize;
  const int64_t stage = stage_needed ? L.bw + (int64_t)M * kHalf * 2 * tsize : 0;
  // the W spectrum plus wrap-around rows (rows 64.. repeat 0..), so that a
  // window of a wavefront's rows never wraps: windows of rows / 2 rows with 4
  // wavefronts (split rows), of `rows` rows otherwise
  const int wrap = waves == 4 ? rows / 2 - 1 : rows - 1;
  const int64_t wreg = (int64_t)(kFft + wrap) * kFft * 2 * tsize;
  // the re-rank mode's FP64 transforms use the region first: 64 rows of 33
  // complex doubles
  const int64_t fp64_grid = stage_needed ? 0 : (int64_t)kFft * kHalf * 16;
  const int64_t big = wreg > fp64_grid ? wreg : fp64_grid;
  const int64_t region = align16(stage > big ? stage : big);
  L.hist_dc = region;
  L.hist_u = L.hist_dc + (int64_t)K * 2 * tsize;
  L.tw64 = align16(L.hist_u + (int64_t)K * 4);
  L.twt = L.tw64 + kFft * 2 * 8;
  // the T twiddles serve the transforms only
  L.slots = align16(L.twt + (stage_needed ? kFft * 2 * tsize : 0));
  L.cand = L.slots + 2LL * waves * 32;
  L.misc = L.cand + 2LL * waves * 32;
  L.misc = align16(L.misc);
  L.total = L.misc + 32;
  return L;
}

template <typename T>
inline int64_t lds_bytes(int M, int N, int K, int waves, bool stage_needed = true) {
  return lds_layout(M, N, K, waves, (int)sizeof(T), stage_needed).total;
}

}  // namespace fse
