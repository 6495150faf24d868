// fse_volume.h -- types shared by the HIP kernels and the host runtime of
// three-dimensional FSE (video volumes).
#pragma once
#include <stdint.h>

namespace fse {

// Basis grid of the 3-D form in this build: 8 frames x 32 x 32.
constexpr int kVt = 8, kVh = 32, kVw = 32;
constexpr int kV3 = kVt * kVh * kVw;  // 8192 spectrum entries
constexpr int kVThreads = 512;        // one workgroup per block: 16 entries per thread
constexpr int kVEnt = kV3 / kVThreads;
// LDS grid of the block kernel: rows of 32 complex doubles at a pitch of 33
// (one pad entry), so that lanes walking along different rows or columns hit
// distinct banks; a frame is 32 such rows.
constexpr int kVPitch = 33;
constexpr int kVFrame = kVh * kVPitch;

// Arguments of the 3-D block kernel (FP64).
struct Vol3Args {
  double* work;           // working volume (frames x rows x columns)
  uint8_t* state;         // kKnown / kPending / kRecon per sample
  const int32_t* items;   // 3 ints per work item: block frame, row, column
  double* staging;        // model samples of every item's block, applied after the wave
  const double* radial;   // Mt*M*N table rho^dist (3-D distance from the area centre)
  const double* twid;     // 32 x (cos, sin)(2 pi t / 32)
  int32_t T, H, W;        // volume size
  int32_t Bt, Bh, Bw;     // block size
  int32_t dt, d;          // area border in frames and in samples
  int32_t Mt, M, N, K;    // area size, iterations
  double delta, gamma, empty_fill;
};

// Dynamic LDS of the 3-D block kernel: the 8 x 32 x 32 complex spectrum
// (transform work area, then W) at row pitch kVPitch, the selection history,
// twiddles, slots.
struct Vol3Lds {
  int64_t hist_u, hist_dc, tw, slots, red, total;
};

__host__ __device__ inline Vol3Lds vol3_lds(int K) {
  Vol3Lds L;
  L.hist_u = (int64_t)kVt * kVFrame * 16;
  L.hist_dc = L.hist_u + (((int64_t)K * 4 + 15) & ~15LL);
  L.tw = L.hist_dc + (int64_t)K * 16;
  L.slots = L.tw + 32 * 16;
  L.red = L.slots + 2LL * (kVThreads / 64) * 32;
  L.total = L.red + 8 * (kVThreads / 64);
  return L;
}

}  // namespace fse
