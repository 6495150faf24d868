// fse_device.h -- types shared by the HIP kernels and the host runtime of the
// FSE library (device-side layout of frames, work items and kernel args).
#pragma once
#include <stdint.h>

namespace fse {

constexpr int kFft = 64;          // basis grid edge (64 x 64 DFT basis)
constexpr int kThreads = 256;     // one workgroup = 4 wavefronts
constexpr int kWaves = 4;
constexpr int kRowsPerWave = kFft / kWaves;  // 16 spectrum rows per wave
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
  const int32_t* items;    // 2 ints per work item: frame, (bi << 16) | bj
  const T* radial;         // M*N table rho^dist of Eq. (2)
  const T* twid;           // 64 x (cos, sin)(2 pi t / 64) in T
  const double* twid64;    // 64 x (cos, sin)(2 pi t / 64) in double
  T* staging;              // nullable: results go here (d > block size)
  int32_t* trace_u;        // nullable: [items * K]
  T* trace_dc;             // nullable: [items * K * 2]
  int32_t M, N, Bh, Bw, d, gox, goy, K;
  T delta, gamma, zscale;  // zscale balances x and w in the packed DFT
  double empty_fill;
};

// Bytes of dynamic LDS the fused kernel needs.
template <typename T>
inline int64_t lds_bytes(int M, int N, int K) {
  const int NP = N | 1;  // odd row pitch for the staged area
  int64_t stage = 2LL * M * NP * sizeof(T) + 2LL * M * kHalf * 2 * sizeof(T);
  int64_t wreg = (int64_t)(kFft + kRowsPerWave - 1) * kFft * 2 * sizeof(T);
  int64_t region = stage > wreg ? stage : wreg;
  region = (region + 15) & ~15LL;
  int64_t hist = (int64_t)K * (2 * sizeof(T)) + (int64_t)K * sizeof(int32_t);
  hist = (hist + 15) & ~15LL;
  int64_t tw = kFft * 2 * sizeof(double) + kFft * 2 * sizeof(T);
  int64_t slots = 2 * kWaves * (3 * sizeof(T) + 4 + (sizeof(T) == 8 ? 4 : 0));
  int64_t misc = 4 * sizeof(double);
  return region + hist + tw + slots + misc;
}

}  // namespace fse
