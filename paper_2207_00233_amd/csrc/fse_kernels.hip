// fse_kernels.hip -- HIP kernels (gfx950) of Frequency Selective Extrapolation.
//
// One workgroup of WAVES wavefronts extrapolates one lost block:
//   A  gather the extrapolation area L (block + frame of d samples, paper
//      Section 2) from the working image, classify every sample (known /
//      reconstructed / lost / outside) and apply the weighting function of
//      Eq. (2): x = f * w, w = rho^dist * {1, delta, 0};
//   B  real DFT of every row of x and of w (columns 0..32 of the 64-point
//      transform; the rest follow by conjugate symmetry);
//   C  64-point DFT down the columns of the packed signal z = x + j s w, so
//      one complex transform yields both spectra; unpacked into the residual
//      spectrum R (registers) and the weight spectrum W (LDS);
//   D  K greedy iterations (Section 2 and 4): u = argmax |R|^2, coefficient
//      increment gamma * R[u] / W0, and the residual spectrum update
//      R[k] -= dc * W[k - u], which is the DFT of the spatial update
//      r -= dc * phi_u;
//   E  the model of Eq. (1) evaluated on the lost samples of the block (sums
//      in double), written back as reconstructed samples.
// Spectrum layout in the iteration: wavefront w owns ROWS = 64 / WAVES rows
// k1 (rows ROWS*w .. ROWS*w + ROWS-1; with 4 wavefronts two windows of 8 rows,
// 8w.. and 32 + 8w..), lane l owns column k2 = l, so every lane keeps ROWS
// complex entries in registers and reads W[k - u] from LDS with a per-lane
// column offset.  WAVES = 4 is the throughput shape; WAVES = 8 and 16 halve
// and quarter the serial work per iteration for launches too small to fill
// the GPU.  The re-rank mode's FP64 transforms (rerank_transforms) and the
// matrix-core transforms (forward_transforms_mx) replace phases A-C and are
// described where they are defined.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fse_device.h"
#include "fse_dft.h"

namespace fse {

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// 64 x (cos, sin)(2 pi t / 64) in double and in float, in constant memory:
// the transforms index them with wave-uniform t only, so the reads are
// scalar loads whose values the FMAs take straight from SGPRs (no LDS reads
// or address moves).  Written at plan creation, the same values as
// BlockArgs::twid64 / twid.
__constant__ double c_twid64[2 * kFft];
__constant__ float c_twid32[2 * kFft];

template <typename T>
__device__ __forceinline__ const T* twiddle_const();
template <>
__device__ __forceinline__ const double* twiddle_const<double>() { return c_twid64; }
template <>
__device__ __forceinline__ const float* twiddle_const<float>() { return c_twid32; }

// Scratch of fse_conceal_image_noalloc: a fixed region of device memory in
// the code object (each GPU the library runs on holds its own copy until the
// process ends), so that the call allocates nothing.  Host code never names
// the array itself (its name is a host-side stand-in): it takes the device
// address once per device through hipGetSymbolAddress and passes that.
constexpr size_t kNoAllocScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch_address(void** out) {
  return hipGetSymbolAddress(out, HIP_SYMBOL(scratch));
}

hipError_t upload_twiddle_constants(const double* tbl) {
  float t32[2 * kFft];
  for (int i = 0; i < 2 * kFft; ++i) t32[i] = (float)tbl[i];
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_twid64), tbl, 2 * kFft * sizeof(double));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_twid32), t32, sizeof(t32));
  return e;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// The spectrum entries of one lane.  A vector type keeps them in registers
// even when indexed by a wave-uniform run-time index (register-indexed move).
template <typename T, int R>
using VecR = T __attribute__((ext_vector_type(R)));

template <typename T>
__device__ __forceinline__ T read_lane(T v, int lane);

template <>
__device__ __forceinline__ float read_lane<float>(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

template <>
__device__ __forceinline__ double read_lane<double>(double v, int lane) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One DPP step of a wavefront max: x = max(x, x moved by CTRL).  Lanes
// outside ROWMASK keep their own value, so the step is idempotent there.
// Unsigned max has identity 0, so lanes without a source (or outside
// ROWMASK) may read 0; this lets the move fold into v_max_u32 with DPP.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ unsigned dpp_max_step(unsigned x) {
  unsigned y = (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWMASK, 0xF, true);
  return x > y ? x : y;
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_max_step(double x) {
  long long b = __double_as_longlong(x);
  int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
  int ylo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, 0xF, false);
  int yhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, 0xF, false);
  double y = __longlong_as_double(((long long)yhi << 32) | (unsigned int)ylo);
  return fmax(x, y);
}

// One DPP step of a wavefront sum in double: x += x moved by CTRL (a lane
// without a source adds its own value; only lane 63's sum is used below).
template <int CTRL>
__device__ __forceinline__ double dpp_add_step(double x) {
  long long b = __double_as_longlong(x);
  int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
  int ylo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
  int yhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
  return x + __longlong_as_double(((long long)yhi << 32) | (unsigned int)ylo);
}

// Wavefront sums of C values at once (the C reduction trees interleave),
// returned uniform.  Quads, then rows of 16 (every lane of a row ends with
// the row sum), then row 1 += row 0 and row 3 += row 2 (row_bcast:15), then
// row 3 += row 1 (row_bcast:31): lane 63 holds the wavefront sum.  Lanes
// outside rows 1 and 3 collect partial sums that are not read.
template <int C>
__device__ __forceinline__ void wave_sums(double (&x)[C]) {
#pragma unroll
  for (int c = 0; c < C; ++c) x[c] = dpp_add_step<0xB1>(x[c]);   // quad_perm [1,0,3,2]
#pragma unroll
  for (int c = 0; c < C; ++c) x[c] = dpp_add_step<0x4E>(x[c]);   // quad_perm [2,3,0,1]
#pragma unroll
  for (int c = 0; c < C; ++c) x[c] = dpp_add_step<0x124>(x[c]);  // row_ror:4
#pragma unroll
  for (int c = 0; c < C; ++c) x[c] = dpp_add_step<0x128>(x[c]);  // row_ror:8
#pragma unroll
  for (int c = 0; c < C; ++c) x[c] = dpp_add_step<0x142>(x[c]);  // row_bcast:15
#pragma unroll
  for (int c = 0; c < C; ++c) x[c] = dpp_add_step<0x143>(x[c]);  // row_bcast:31
#pragma unroll
  for (int c = 0; c < C; ++c) x[c] = read_lane(x[c], 63);
}

// Wavefront maximum (exact: max is order-free), returned uniform.
template <typename V>
__device__ __forceinline__ V wave_max(V x) {
  x = dpp_max_step<0xB1, 0xF>(x);   // quad_perm [1,0,3,2]
  x = dpp_max_step<0x4E, 0xF>(x);   // quad_perm [2,3,0,1]
  x = dpp_max_step<0x124, 0xF>(x);  // row_ror:4
  x = dpp_max_step<0x128, 0xF>(x);  // row_ror:8 -> every lane holds its row max
  x = dpp_max_step<0x142, 0xA>(x);  // row_bcast:15 -> rows 1, 3
  x = dpp_max_step<0x143, 0xC>(x);  // row_bcast:31 -> row 3 holds the wave max
  if constexpr (sizeof(V) == 4) {
    return (V)__builtin_amdgcn_readlane((int)x, 63);
  } else {
    return read_lane(x, 63);
  }
}

// Maximum over groups of G adjacent lanes when the data repeat with period G
// (G = 2, 4, 8 or 16); returned uniform (lane 0's group).
template <int G>
__device__ __forceinline__ unsigned group_max(unsigned x) {
  static_assert(G == 2 || G == 4 || G == 8 || G == 16, "group of 2, 4, 8 or 16 lanes");
  x = dpp_max_step<0xB1, 0xF>(x);                          // quad_perm [1,0,3,2]
  if constexpr (G >= 4) x = dpp_max_step<0x4E, 0xF>(x);   // quad_perm [2,3,0,1]
  if constexpr (G >= 8) x = dpp_max_step<0x124, 0xF>(x);  // row_ror:4
  if constexpr (G >= 16) x = dpp_max_step<0x128, 0xF>(x); // row_ror:8
  return (unsigned)__builtin_amdgcn_readfirstlane((int)x);
}

__device__ __forceinline__ unsigned umax3(unsigned a, unsigned b, unsigned c) {
  return max(a, max(b, c));
}

// Median of three as one v_med3_u32 (written out, the compiler splits some
// of them into min/max pairs).
__device__ __forceinline__ unsigned umed3(unsigned a, unsigned b, unsigned c) {
  unsigned r;
  asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// Largest (m1) and second largest (m2) of N distinct keys.  Triples give
// (max3, med3); three (largest, second) pairs merge as largest = max3 of the
// largest ones and second = max(med3 of the largest ones, max3 of the
// seconds) (a loser's second is below the median of the largest ones); two
// pairs as largest = max, second = med3(m, n, max of the seconds).  For 16
// keys: 5 triples, two 3-way merges (the 16th key joins the second one),
// one 2-way merge: 21 instructions.
template <int N>
__device__ __forceinline__ void top2(const unsigned (&k)[N], unsigned& m1, unsigned& m2) {
  if constexpr (N == 16) {
    unsigned a[5], b[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) {
      a[t] = umax3(k[3 * t], k[3 * t + 1], k[3 * t + 2]);
      b[t] = umed3(k[3 * t], k[3 * t + 1], k[3 * t + 2]);
    }
    const unsigned p1 = umax3(a[0], a[1], a[2]);
    const unsigned q1 = max(umed3(a[0], a[1], a[2]), umax3(b[0], b[1], b[2]));
    const unsigned p2 = umax3(a[3], a[4], k[15]);
    const unsigned q2 = max(umed3(a[3], a[4], k[15]), max(b[3], b[4]));
    m1 = max(p1, p2);
    m2 = umed3(p1, p2, max(q1, q2));
  } else {
    m1 = k[0];
    m2 = 0u;
    int j = 1;
    if constexpr (N >= 3) {
      m1 = umax3(k[0], k[1], k[2]);
      m2 = umed3(k[0], k[1], k[2]);
      j = 3;
    }
#pragma unroll
    for (; j + 2 < N; j += 3) {
      const unsigned n1 = umax3(k[j], k[j + 1], k[j + 2]);
      const unsigned n2 = umed3(k[j], k[j + 1], k[j + 2]);
      m2 = umed3(m1, n1, max(m2, n2));
      m1 = max(m1, n1);
    }
#pragma unroll
    for (; j < N; ++j) {
      m2 = umed3(m1, k[j], m2);
      m1 = max(m1, k[j]);
    }
  }
}

// (bits & ~63) | (low & 63) as one bit-field insert (the compiler otherwise
// splits it into two operations).
__device__ __forceinline__ unsigned pack_key(unsigned bits, unsigned low) {
  unsigned r;
  asm("v_bfi_b32 %0, 63, %1, %2" : "=v"(r) : "s"(low), "v"(bits));
  return r;
}

// Argmax slot of the FP32 iteration (16 bytes): the wavefront's best entry.
struct FSlot {
  unsigned key;  // packed selection key
  int k;         // spectrum index k1 * 64 + k2; re-rank: near-tie count << 12
  float re, im;  // residual value
};

// Argmax slot exchanged between wavefronts (32 bytes).
struct Slot {
  double e;     // FP64 path: exact |R|^2 of the wave's best entry; re-rank: exact |R|^2 of
                // the wave's best re-scored candidate
  double re, im;
  unsigned key; // FP32 path: packed selection key of the wave's best entry
  int k;        // its spectrum index k1 * 64 + k2
};

// Spectrum rows of wavefront `wave`: ROWS consecutive rows, or with SPLIT two
// windows of ROWS/2 rows (w ROWS/2 .. and 32 + w ROWS/2 ..), which needs only
// ROWS/2 - 1 wrap-around rows of W in LDS.
template <int WAVES, bool SPLIT>
__device__ __forceinline__ int row_of(int wave, int j) {
  constexpr int ROWS = kFft / WAVES;
  if constexpr (SPLIT)
    return (j < ROWS / 2 ? 0 : kFft / 2 - ROWS / 2) + (ROWS / 2) * wave + j;
  else
    return ROWS * wave + j;
}

// Inverse of row_of: the wavefront that owns spectrum row `row`, and the
// index j of that row in its registers.
template <int WAVES, bool SPLIT>
__device__ __forceinline__ int wave_of_row(int row) {
  constexpr int ROWS = kFft / WAVES;
  if constexpr (SPLIT)
    return (row & (kFft / 2 - 1)) / (ROWS / 2);
  else
    return row / ROWS;
}

template <int WAVES, bool SPLIT>
__device__ __forceinline__ int j_of_row(int row, int wave) {
  constexpr int ROWS = kFft / WAVES;
  if constexpr (SPLIT)
    return (row & (kFft / 2 - 1)) - (ROWS / 2) * wave + (row >= kFft / 2 ? ROWS / 2 : 0);
  else
    return row - ROWS * wave;
}

// Phase A: gather, classify and weight the area (Eq. (2)) into LDS; returns
// W0 = sum of weights (uniform).  COMPACT: the samples are staged as TI with
// one weight class per sample (0 none, 1 known, 2 reconstructed) at pitch
// N | 1; otherwise x = f w and w themselves (T each, x first).
template <typename T, typename TI, int WAVES, bool COMPACT = (WAVES == 4)>
__device__ __forceinline__ T gather_area(unsigned char* smem, const LdsLayout& L, int M, int N,
                                         const T* radial, T delta, const TI* img,
                                         const uint8_t* st, int H, int W, int oy, int ox,
                                         int lane, int wave) {
  const int NP = N | 1;
  T* xs = reinterpret_cast<T*>(smem);
  T* ws = xs + M * NP;
  TI* fs = reinterpret_cast<TI*>(smem);
  uint8_t* cs = reinterpret_cast<uint8_t*>(smem + L.cs);
  Slot* slots = reinterpret_cast<Slot*>(smem + L.slots);
  T wsum = T(0);
  // rows by wavefront, one column per lane (N <= 64): no index division
  const int n = lane;
  const int x = ox + n;
  const bool xin = n < N && x >= 0 && x < W;
  for (int m = wave; m < M; m += WAVES) {
    if (n >= N) continue;
    const int y = oy + m;
    T wv = T(0);
    TI f = TI(0);
    uint8_t c = 0;
    if (xin && y >= 0 && y < H) {
      const int64_t p = (int64_t)y * W + x;
      const uint8_t s = st[p];
      const T fac = s == kKnown ? T(1) : (s == kRecon ? delta : T(0));
      c = s == kKnown ? 1 : (s == kRecon ? 2 : 0);
      f = img[p];
      wv = radial[m * N + n] * fac;
    }
    if constexpr (COMPACT) {
      fs[m * NP + n] = f;
      cs[m * NP + n] = c;
    } else {
      ws[m * NP + n] = wv;
      xs[m * NP + n] = (T)f * wv;
    }
    wsum += wv;
  }
  wsum = wave_sum(wsum);
  if (lane == 0) slots[wave].e = (double)wsum;
  __syncthreads();
  T W0 = T(0);
#pragma unroll
  for (int q = 0; q < WAVES; ++q) W0 += (T)slots[q].e;
  return W0;
}

// Phases A-C: gather and weight the area, transform, unpack.  Computes in T,
// reads the working image in TI.  Returns W0 = sum of weights; when W0 > 0,
// rr/ri hold X[k] and wvr/wvi hold W[k] for k1 = row_of(wave, j), k2 = lane
// (split rows with 4 wavefronts).  With 4 wavefronts (COMPACT) phase A stages
// the samples as TI and one weight class per sample and phase B forms the
// weights again from the radial table, which keeps the staging small enough
// for several blocks per CU; otherwise phase A stages x and w themselves.
// Ends with a barrier, after which the LDS region may be reused.
template <typename T, typename TI, int WAVES>
__device__ __forceinline__ T forward_transforms(unsigned char* smem, const LdsLayout& L, int M,
                                                int N, const T* radial, T delta, T zscale,
                                                const TI* img, const uint8_t* st, int H, int W,
                                                int oy, int ox, int lane, int wave,
                                                VecR<T, kFft / WAVES>& rr,
                                                VecR<T, kFft / WAVES>& ri,
                                                T (&wvr)[kFft / WAVES], T (&wvi)[kFft / WAVES]) {
  constexpr int ROWS = kFft / WAVES;
  constexpr int QB = (kHalf + WAVES - 1) / WAVES;  // row-DFT columns per wavefront
  constexpr bool SPLIT = WAVES == 4;
  constexpr bool COMPACT = WAVES == 4;
  const int NP = N | 1;
  T* xs = reinterpret_cast<T*>(smem);                     // x and w (full staging)
  T* ws = xs + M * NP;
  TI* fs = reinterpret_cast<TI*>(smem);                   // COMPACT: samples
  uint8_t* cs = reinterpret_cast<uint8_t*>(smem + L.cs);  // COMPACT: 0 none, 1 known, 2 recon
  T* bx = reinterpret_cast<T*>(smem + L.bx);
  T* bw = reinterpret_cast<T*>(smem + L.bw);
  T* Zl = reinterpret_cast<T*>(smem);  // 64 x 64 complex, after phase B
  const T* twt = twiddle_const<T>();  // wave-uniform indices: scalar loads

  const T W0 = gather_area<T, TI, WAVES>(smem, L, M, N, radial, delta, img, st, H, W, oy, ox,
                                         lane, wave);
  if (!(W0 > T(0))) return W0;

  // ---- B: real row DFTs, columns k2 = wave + WAVES q, k2 <= 32 ----
  {
    T axr[QB], axi[QB], awr[QB], awi[QB];
#pragma unroll
    for (int q = 0; q < QB; ++q) axr[q] = axi[q] = awr[q] = awi[q] = T(0);
    if (lane < M) {
      auto accumulate = [&](int n, T xv, T wv) {
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          const int t = ((wave + WAVES * q) * n) & (kFft - 1);
          const T c = twt[2 * t], s = twt[2 * t + 1];
          axr[q] = fma(xv, c, axr[q]);
          axi[q] = fma(-xv, s, axi[q]);
          awr[q] = fma(wv, c, awr[q]);
          awi[q] = fma(-wv, s, awi[q]);
        }
      };
      for (int n = 0; n < N; ++n) {
        if constexpr (COMPACT) {
          const uint8_t c = cs[lane * NP + n];
          const T r = radial[lane * N + n];
          const T wv = c == 1 ? r : (c == 2 ? r * delta : T(0));
          accumulate(n, (T)fs[lane * NP + n] * wv, wv);
        } else {
          accumulate(n, xs[lane * NP + n], ws[lane * NP + n]);
        }
      }
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        const int k2 = wave + WAVES * q;
        if (k2 < kHalf) {
          T* px = bx + (lane * kHalf + k2) * 2;
          T* pw = bw + (lane * kHalf + k2) * 2;
          px[0] = axr[q];
          px[1] = axi[q];
          pw[0] = awr[q];
          pw[1] = awi[q];
        }
      }
    }
  }
  __syncthreads();

  // ---- C: column DFT of z = x + j s w for k1 = ROWS wave + j, k2 = lane ----
  {
    const int c = lane <= 32 ? lane : kFft - lane;
    const T sg = lane <= 32 ? T(1) : T(-1);  // conjugate mirrored columns
    auto zval = [&](int m, T& zr, T& zi) {
      const T xr = bx[(m * kHalf + c) * 2], xi = sg * bx[(m * kHalf + c) * 2 + 1];
      const T wr = bw[(m * kHalf + c) * 2], wi = sg * bw[(m * kHalf + c) * 2 + 1];
      zr = fma(-zscale, wi, xr);
      zi = fma(zscale, wr, xi);
    };
#pragma unroll
    for (int j = 0; j < ROWS; ++j) rr[j] = ri[j] = T(0);
    if constexpr (WAVES == 4) {
      // 64 = 4 x 16: with m = m0 + 4 m1 and k1 = j + 16 w,
      //   Z[k1] = sum_m0 e^{-j2pi m0 k1/64} Y_m0[j],
      //   Y_m0[j] = sum_m1 z[m0 + 4 m1] e^{-j2pi m1 j/16};
      // wavefront w computes Y_w (16 points) and the four are shared in LDS.
      for (int m = wave; m < M; m += 4) {
        T zr, zi;
        zval(m, zr, zi);
        const int m1 = m >> 2;
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
          const int t = (4 * m1 * j) & (kFft - 1);
          const T cc = twt[2 * t], ss = twt[2 * t + 1];
          rr[j] = fma(zr, cc, fma(zi, ss, rr[j]));
          ri[j] = fma(zi, cc, fma(-zr, ss, ri[j]));
        }
      }
      __syncthreads();  // every wavefront is done with the phase-B rows
#pragma unroll
      for (int j = 0; j < ROWS; ++j) {
        T* p = Zl + ((wave * ROWS + j) * kFft + lane) * 2;
        p[0] = rr[j];
        p[1] = ri[j];
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < ROWS; ++j) {
        const int k1 = row_of<WAVES, SPLIT>(wave, j);
        T ar = T(0), ai = T(0);
#pragma unroll
        for (int m0 = 0; m0 < 4; ++m0) {
          const T* p = Zl + ((m0 * ROWS + (k1 & (ROWS - 1))) * kFft + lane) * 2;
          const T yr = p[0], yi = p[1];
          const int t = (m0 * k1) & (kFft - 1);
          const T cc = twt[2 * t], ss = twt[2 * t + 1];
          ar = fma(yr, cc, fma(yi, ss, ar));
          ai = fma(yi, cc, fma(-yr, ss, ai));
        }
        rr[j] = ar;
        ri[j] = ai;
      }
    } else {
      for (int m = 0; m < M; ++m) {
        T zr, zi;
        zval(m, zr, zi);
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
          const int t = (row_of<WAVES, SPLIT>(wave, j) * m) & (kFft - 1);
          const T cc = twt[2 * t], ss = twt[2 * t + 1];
          rr[j] = fma(zr, cc, fma(zi, ss, rr[j]));
          ri[j] = fma(zi, cc, fma(-zr, ss, ri[j]));
        }
      }
    }
  }
  __syncthreads();  // phase-B buffers (and the partial DFTs) are dead from here on
#pragma unroll
  for (int j = 0; j < ROWS; ++j) {
    T* p = Zl + (row_of<WAVES, SPLIT>(wave, j) * kFft + lane) * 2;
    p[0] = rr[j];
    p[1] = ri[j];
  }
  __syncthreads();
  // unpack: X[k] = (Z[k] + conj Z[-k]) / 2, W[k] = (Z[k] - conj Z[-k]) / (2 j s)
  {
    const T h = T(0.5), hs = T(0.5) / zscale;
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      const int k1 = row_of<WAVES, SPLIT>(wave, j);
      const T* p = Zl + ((((kFft - k1) & (kFft - 1)) * kFft) + ((kFft - lane) & (kFft - 1))) * 2;
      const T pr = p[0], pi = p[1];
      const T ar = rr[j], ai = ri[j];
      rr[j] = h * (ar + pr);
      ri[j] = h * (ai - pi);
      wvr[j] = hs * (ai + pi);
      wvi[j] = hs * (pr - ar);
    }
  }
  __syncthreads();
  return W0;
}

// ---- Matrix-core transforms (FSE_FP32_F16X3) ----
// Both DFT stages as real products on 16 x 16 x 32 f16 matrix-core tiles with
// float accumulation.  Every operand v is split as v ~ hi + lo with
// hi = f16(v), lo = f16(v - hi) (about 22 significant bits), and a product of
// two split operands takes the three tiles hi*hi, hi*lo, lo*hi.  The operands
// stay inside the f16 range: x is scaled by a power of two to |x| <= 256
// (weights and twiddles are <= 1), so row sums over at most 64 samples stay
// below 2^15, and a lo part that falls below the normal range keeps an
// absolute error of 2^-24.
// (Two bf16 parts carry only ~16 bits: measured, that split flipped too many
// near-tied selections.)  Tile layout (16x16x32): lane l holds row l % 16 of A
// and column l % 16 of B at k = 8 (l / 16) .. + 7, and column l % 16 of D at
// rows 4 (l / 16) .. + 3.
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// element e of (hi, lo) = the split of v
template <typename V>
__device__ __forceinline__ void split_f16(float v, V& hi, V& lo, int e) {
  const _Float16 h = (_Float16)v;
  hi[e] = h;
  lo[e] = (_Float16)(v - (float)h);
}

__device__ __forceinline__ f32x4 mfma_f16x3(f16x8 ah, f16x8 al, f16x8 bh, f16x8 bl, f32x4 d) {
  d = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh, d, 0, 0, 0);
  d = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl, d, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh, d, 0, 0, 0);
}

__device__ __forceinline__ f16x8 neg_f16x8(f16x8 v) {
  return __builtin_bit_cast(f16x8, __builtin_bit_cast(u32x4, v) ^ 0x80008000u);
}

// The row-DFT result of z = x + j s w, transposed (k2-major, 64 x 64) in four
// f16 planes (Re hi, Re lo, Im hi, Im lo); 8-element chunks of a row are
// XOR-swizzled by k2 so that the column reads of 16 lanes spread over banks.
__device__ __forceinline__ int yt_index(int plane, int k2, int m) {
  return plane * kFft * kFft + k2 * kFft + ((((m >> 3) ^ k2) & 7) << 3) + (m & 7);
}

// Phases A-C with 4 wavefronts on matrix cores; same contract as
// forward_transforms<float, TI, 4>.
//  B': [x; w] (64 x N, rows m) times G (N x 64): columns c <= 32 hold
//      cos(2 pi c n / 64), c > 32 hold sin(2 pi (c - 32) n / 64); wavefront w
//      computes rows 16w.. for both x and w.  The real row DFTs are then
//      Y[m][c] = Yc - j Ys, extended to all 64 k2 by conjugate symmetry and
//      combined into Yz = Yx + j s Yw.
//  C': [Zr | Zi] (64 x 128) = [C | S] (64 x 128) times
//      [[Yzr, Yzi], [Yzi, -Yzr]] (128 x 128) with C, S = cos, sin of
//      2 pi k1 m / 64; wavefront w computes rows k1 = 16w.. .
//  Unpack X and W from Z as in the vector path.
template <typename TI>
__device__ __forceinline__ float forward_transforms_mx(unsigned char* smem, const LdsLayout& L,
                                                      int M, int N, const float* radial,
                                                      float delta, float zscale, const TI* img,
                                                      const uint8_t* st, int H, int W, int oy,
                                                      int ox, int lane, int wave,
                                                      VecR<float, 16>& rr, VecR<float, 16>& ri,
                                                      float (&wvr)[16], float (&wvi)[16]) {
  constexpr int WAVES = 4;
  constexpr int ROWS = kFft / WAVES;
  const float W0 = gather_area<float, TI, WAVES>(smem, L, M, N, radial, delta, img, st, H, W, oy,
                                                 ox, lane, wave);
  if (!(W0 > 0.f)) return W0;
  const int NP = N | 1;
  const TI* fs = reinterpret_cast<const TI*>(smem);
  const uint8_t* cs = reinterpret_cast<const uint8_t*>(smem + L.cs);
  const float* twt = reinterpret_cast<const float*>(smem + L.twt);
  _Float16* yt = reinterpret_cast<_Float16*>(smem);  // after B': the four Yz planes
  float* Zl = reinterpret_cast<float*>(smem);    // after C': Z, 64 x 64 complex
  const int cl = lane & 15;      // tile row of A / column of B and D
  const int kq = 8 * (lane >> 4);  // first k of the lane's fragments
  const int rq = 4 * (lane >> 4);  // first D row of the lane

  // x is scaled by 2^-xe so that |x| <= 256 (|x| <= |f| since w <= 1): row
  // sums of at most 64 samples then stay below 2^14 and Yz below 2^15 in f16.
  // 8-bit data give xe = 0; larger reconstructed samples are scaled exactly.
  int xe = 0;
  {
    float fm = 0.f;
    if (lane < N)
      for (int m = wave; m < M; m += WAVES)
        if (cs[m * NP + lane]) fm = fmaxf(fm, fabsf((float)fs[m * NP + lane]));
    Slot* slots = reinterpret_cast<Slot*>(smem + L.slots);
    const unsigned wm = wave_max(__float_as_uint(fm));  // non-negative: bits order as values
    if (lane == 0) slots[wave].key = wm;  // gather_area's readers use .e only
    __syncthreads();
    unsigned bm = slots[0].key;
#pragma unroll
    for (int q = 1; q < WAVES; ++q) bm = max(bm, slots[q].key);
    const float xmax = __uint_as_float(bm);
    if (xmax > 256.f) (void)frexpf(xmax * (1.f / 256.f), &xe);
  }
  const float xs_ = ldexpf(1.f, -xe);

  // ---- B': row DFTs ----
  f32x4 dx[4], dw[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) dx[ct] = dw[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
  {
    const int m = ROWS * wave + cl;
    for (int k0 = 0; k0 < N; k0 += 32) {
      f16x8 xh, xl, wh, wl;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int n = k0 + kq + e;
        float xv = 0.f, wv = 0.f;
        if (m < M && n < N) {
          const uint8_t c = cs[m * NP + n];
          const float r = radial[m * N + n];
          wv = c == 1 ? r : (c == 2 ? r * delta : 0.f);
          xv = (float)fs[m * NP + n] * wv * xs_;
        }
        split_f16(xv, xh, xl, e);
        split_f16(wv, wh, wl, e);
      }
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const int c = 16 * ct + cl;
        const int kk = c <= 32 ? c : c - 32;
        const int part = c <= 32 ? 0 : 1;  // cos or sin
        f16x8 gh, gl;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int t = (kk * (k0 + kq + e)) & (kFft - 1);
          split_f16(twt[2 * t + part], gh, gl, e);
        }
        dx[ct] = mfma_f16x3(xh, xl, gh, gl, dx[ct]);
        dw[ct] = mfma_f16x3(wh, wl, gh, gl, dw[ct]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  __syncthreads();  // the staging is dead; the Yz planes take its place
  {
    const int m0 = ROWS * wave + rq;
    auto put = [&](int k2, const float (&re)[4], const float (&im)[4]) {
      f16x4 rh, rl, ih, il;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        split_f16(re[r], rh, rl, r);
        split_f16(im[r], ih, il, r);
      }
      *reinterpret_cast<f16x4*>(yt + yt_index(0, k2, m0)) = rh;
      *reinterpret_cast<f16x4*>(yt + yt_index(1, k2, m0)) = rl;
      *reinterpret_cast<f16x4*>(yt + yt_index(2, k2, m0)) = ih;
      *reinterpret_cast<f16x4*>(yt + yt_index(3, k2, m0)) = il;
    };
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int c = 16 * ct + cl;  // 0..31; its sine column is 32 + c
      float re[4], im[4], re2[4], im2[4];
      if (c == 0) {
        // k2 = 0 and k2 = 32 (column 32 holds the cosine of k2 = 32)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          re[r] = dx[0][r];
          im[r] = zscale * dw[0][r];
          re2[r] = dx[2][r];
          im2[r] = zscale * dw[2][r];
        }
        put(0, re, im);
        put(32, re2, im2);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float xc = dx[ct][r], xs = dx[ct + 2][r];
          const float wc = dw[ct][r], ws = dw[ct + 2][r];
          re[r] = fmaf(zscale, ws, xc);
          im[r] = fmaf(zscale, wc, -xs);
          re2[r] = fmaf(-zscale, ws, xc);
          im2[r] = fmaf(zscale, wc, xs);
        }
        put(c, re, im);
        put(kFft - c, re2, im2);
      }
    }
  }
  __syncthreads();

  // ---- C': column DFTs ----
  f32x4 dz[8];
#pragma unroll
  for (int ct = 0; ct < 8; ++ct) dz[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
  {
    // A fragments of the 4 k-steps (k = 0..63: cos, 64..127: sin)
    const int k1 = ROWS * wave + cl;
    f16x8 ah[4], al[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int part = ks >> 1;
      const int mb = (32 * ks + kq) & (kFft - 1);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int t = (k1 * (mb + e)) & (kFft - 1);
        split_f16(twt[2 * t + part], ah[ks], al[ks], e);
      }
    }
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) {
      const int k2 = 16 * (ct & 3) + cl;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int part = ks >> 1;
        const int mb = (32 * ks + kq) & (kFft - 1);
        // columns of Zr take (Yzr; Yzi), columns of Zi take (Yzi; -Yzr)
        const int plane = ((ct < 4) == (part == 0)) ? 0 : 2;
        f16x8 bh = *reinterpret_cast<const f16x8*>(yt + yt_index(plane, k2, mb));
        f16x8 bl = *reinterpret_cast<const f16x8*>(yt + yt_index(plane + 1, k2, mb));
        if (ct >= 4 && part == 1) {
          bh = neg_f16x8(bh);
          bl = neg_f16x8(bl);
        }
        dz[ct] = mfma_f16x3(ah[ks], al[ks], bh, bl, dz[ct]);
      }
      __builtin_amdgcn_sched_barrier(0);  // one output tile's operands live at a time
    }
  }
  __syncthreads();  // the Yz planes are dead; Z takes their place
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k1 = ROWS * wave + rq + r, k2 = 16 * ct + cl;
      *reinterpret_cast<float2*>(Zl + (k1 * kFft + k2) * 2) = make_float2(dz[ct][r], dz[ct + 4][r]);
    }
  }
  __syncthreads();
  // unpack: X[k] = (Z[k] + conj Z[-k]) / 2, W[k] = (Z[k] - conj Z[-k]) / (2 j s)
  {
    const float h = ldexpf(0.5f, xe), hs = 0.5f / zscale;  // X back to scale 1
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      const int k1 = row_of<WAVES, true>(wave, j);
      const float2 z = *reinterpret_cast<const float2*>(Zl + (k1 * kFft + lane) * 2);
      const float2 p = *reinterpret_cast<const float2*>(
          Zl + ((((kFft - k1) & (kFft - 1)) * kFft) + ((kFft - lane) & (kFft - 1))) * 2);
      rr[j] = h * (z.x + p.x);
      ri[j] = h * (z.y - p.y);
      wvr[j] = hs * (z.y + p.y);
      wvi[j] = hs * (p.x - z.x);
    }
  }
  __syncthreads();
  return W0;
}

// Twiddle tables into LDS (double for the synthesis, T for the transforms).
template <typename T>
__device__ __forceinline__ void load_twiddles(unsigned char* smem, const LdsLayout& L,
                                              const double* twid64, bool with_t = true) {
  const int tid = threadIdx.x;
  if (tid < 2 * kFft) {
    const double v = twid64[tid];
    reinterpret_cast<double*>(smem + L.tw64)[tid] = v;
    if (with_t) reinterpret_cast<T*>(smem + L.twt)[tid] = (T)v;
  }
}

// FP64 transforms of the re-rank mode, inside the block kernel: W = DFT(w)
// and R0 = DFT(x) in double, written to BlockArgs::spec64 for the exact
// re-scoring; the block kernel reads its float copies of both back from
// there (k1 = row_of(wave, j), k2 = lane).  w and x = f w are real,
// so their spectra are Hermitian (S[-k] = conj S[k]) and columns k2 = 0..32
// hold all of it: the grid is 64 rows x 32 complex slots (33 KB, inside the
// block's own LDS).  w and x go through the same steps one after the other (a
// packed transform of x + j s w would leak the rounding of one into the
// other: a black area would not give X = 0 exactly):
//  A: gather and weight the area (Eq. (2)); row m, slot p holds the sample
//     pair (z[2p], z[2p+1]) as one complex value (zeros outside the area);
//  B: per row, the 32-point DFT Z of those pairs, factorized 8 x 4 (an
//     8-point DFT over n1 of slot 4 n1 + n2, the twiddle e^{-j 2 pi n2 k1 /
//     32}, a 4-point DFT over n2), then the row's real 64-point DFT from the
//     pairs (Z[k], Z[32 - k]): with E and O the DFTs of the even and odd
//     samples, X[k] = E[k] + e^{-j 2 pi k / 64} O[k] and X[32 - k] =
//     conj(E[k] - e^{-j 2 pi k / 64} O[k]).  One thread takes the 4-point
//     DFTs k1 and 8 - k1 of a row, which hold every pair it needs, and puts
//     its eight results back into its own eight slots: slot kHalfSlot[k]
//     holds X[k], the two real values X[0] and X[32] share one slot;
//  C: per slot, the 64-point DFT along the rows, factorized 8 x 8 as in B
//     (output row 8 (K & 7) + (K >> 3) holds frequency K); the shared slot
//     transforms X[.][0] + j X[.][32], whose two columns are separated on the
//     way out;
//  D: out: row K of the spectrum, columns 0..32, to HBM.
// Returns W0 (0 when the area has no support: nothing is written then).
constexpr int kHp = 33;  // grid pitch in complex doubles (one pad slot)
static_assert(kFft * kHp * 16 <= (kFft + 3) * kFft * 8,
              "the half-spectrum grid fits in the block kernel's W region");

// slot of column k2 = 0..32 after the row transforms (0 and 32 share one)
__constant__ unsigned char kHalfSlot[kHalf] = {18, 4,  8,  12, 2,  22, 26, 30, 0,  6,  10,
                                               14, 16, 20, 24, 28, 19, 29, 25, 21, 17, 15,
                                               11, 7,  1,  31, 27, 23, 3,  13, 9,  5,  18};

// entry (k1, k2) of the spectrum of real data stored as columns 0..32
__device__ __forceinline__ double2 half_spec_at(const double* s, int k1, int k2) {
  const bool hi = k2 > kFft / 2;
  const int r = hi ? (kFft - k1) & (kFft - 1) : k1, c = hi ? kFft - k2 : k2;
  const double2 v = *reinterpret_cast<const double2*>(s + 2 * (r * kHalf + c));
  return make_double2(v.x, hi ? -v.y : v.y);
}

namespace {

using dft::dft4;
using dft::dft8;
__device__ __forceinline__ double2 dmul_conj(double2 v, double2 t) { return dft::cmul_conj(v, t); }
__device__ __forceinline__ double2 dconj(double2 v) { return make_double2(v.x, -v.y); }

// X[k] and X[32 - k] of a real row from Z[k] and Z[32 - k] (t = the twiddle
// of k as (cos, sin))
__device__ __forceinline__ void real_pair(double2 zk, double2 zp, double2 t, double2& xk,
                                          double2& xp) {
  const double2 e = make_double2(0.5 * (zk.x + zp.x), 0.5 * (zk.y - zp.y));
  const double2 o = make_double2(0.5 * (zk.y + zp.y), -0.5 * (zk.x - zp.x));
  const double2 to = dmul_conj(o, t);
  xk = make_double2(e.x + to.x, e.y + to.y);
  xp = make_double2(e.x - to.x, to.y - e.y);
}

}  // namespace

// Not inlined: its registers are allocated apart from the iteration loop's.
template <int WAVES>
__device__ __noinline__ double rerank_transforms(unsigned char* smem, int64_t tw_off,
                                                 int64_t red_off, const double* radial64,
                                                 double delta, int M, int N, const float* img,
                                                 const uint8_t* st, int H, int W, int oy, int ox,
                                                 double* spec) {
  constexpr int THREADS = 64 * WAVES;
  static_assert(THREADS >= 256, "one task per thread in every stage");
  double2* G = reinterpret_cast<double2*>(smem);  // 64 rows x kHp
  double* Gd = reinterpret_cast<double*>(smem);
  const double2* tw = reinterpret_cast<const double2*>(smem + tw_off);
  double* red = reinterpret_cast<double*>(smem + red_off);  // WAVES partial sums
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int n = lane, x = ox + n;
  const bool xin = n < N && x >= 0 && x < W;
  double W0 = 0.0;
  for (int pass = 0; pass < 2; ++pass) {  // 0: w, 1: x = f w
    // ---- A: gather and weight ----
    double wsum = 0.0;
    for (int m = wave; m < M; m += WAVES) {
      const int y = oy + m;
      double wv = 0.0, f = 0.0;
      if (xin && y >= 0 && y < H) {
        const int64_t p = (int64_t)y * W + x;
        const uint8_t s = st[p];
        const double fac = s == kKnown ? 1.0 : (s == kRecon ? delta : 0.0);
        wv = radial64[m * N + n] * fac;
        f = (double)img[p];
      }
      wsum += wv;
      Gd[2 * kHp * m + n] = pass ? f * wv : wv;
    }
    if (pass == 0) {
      wsum = wave_sum(wsum);
      if (lane == 0) red[wave] = wsum;
    }
    __syncthreads();
    if (pass == 0) {
#pragma unroll
      for (int q = 0; q < WAVES; ++q) W0 += red[q];
      if (!(W0 > 0.0)) return 0.0;  // uniform
    }

    // ---- B: rows; task (m, n2): 8-point DFT over n1 of slot 4 n1 + n2 ----
    if (tid < 4 * M) {
      const int m = tid >> 2, n2 = tid & 3;
      double2* r = G + m * kHp + n2;
      double2 v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = r[4 * i];
      dft8(v);
#pragma unroll
      for (int kk = 1; kk < 8; ++kk) v[kk] = dmul_conj(v[kk], tw[(2 * n2 * kk) & (kFft - 1)]);
#pragma unroll
      for (int i = 0; i < 8; ++i) r[4 * i] = v[i];
    }
    __syncthreads();
    // task (m, tau): the 4-point DFTs k1 = ka, kb (tau = 0: 0 and 4; else tau
    // and 8 - tau) give Z[ka + 8 k2] and Z[kb + 8 k2]; their real pairs
    // (k, 32 - k) are, for tau = 0: (8, 24), (4, 28), (12, 20) and the
    // self-paired 0 and 16; else (j, 32 - j), (j + 8, 24 - j),
    // (16 - j, 16 + j), (8 - j, 24 + j) with j = tau
    if (tid < 4 * M) {
      const int m = tid >> 2, tau = tid & 3;
      const bool t0 = tau == 0;
      const int ka = tau, kb = t0 ? 4 : 8 - tau;
      double2* ra = G + m * kHp + 4 * ka;
      double2* rb = G + m * kHp + 4 * kb;
      double2 za[4], zb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        za[i] = ra[i];
        zb[i] = rb[i];
      }
      dft4(za[0], za[1], za[2], za[3]);
      dft4(zb[0], zb[1], zb[2], zb[3]);
      const int kA = t0 ? 8 : tau, kB = t0 ? 4 : tau + 8, kC = t0 ? 12 : 16 - tau, kD = 8 - tau;
      double2 x0, x1;
      real_pair(t0 ? za[1] : za[0], t0 ? za[3] : zb[3], tw[kA], x0, x1);
      const double2 zkB = t0 ? zb[0] : za[1], zpB = t0 ? zb[3] : zb[2];
      const double2 zpC = t0 ? zb[2] : za[2];
      ra[0] = x0;
      ra[1] = x1;
      real_pair(zkB, zpB, tw[kB], x0, x1);
      ra[2] = x0;
      ra[3] = x1;
      real_pair(zb[1], zpC, tw[kC], x0, x1);
      rb[0] = x0;
      rb[1] = x1;
      real_pair(zb[0], za[3], tw[kD], x0, x1);
      if (t0) {  // X[0] and X[32] (both real) share a slot; X[16] = conj Z[16]
        x0 = make_double2(za[0].x + za[0].y, za[0].x - za[0].y);
        x1 = dconj(za[2]);
      }
      rb[2] = x0;
      rb[3] = x1;
    }
    __syncthreads();

    // ---- C: columns; task (s, m2): 8-point DFT over m1 of row 8 m1 + m2 ----
    if (tid < 256) {
      const int s = tid & 31, m2 = tid >> 5;
      double2* col = G + s;
      double2 v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        v[i] = 8 * i + m2 < M ? col[(8 * i + m2) * kHp] : make_double2(0.0, 0.0);
      dft8(v);
#pragma unroll
      for (int kk = 1; kk < 8; ++kk) v[kk] = dmul_conj(v[kk], tw[m2 * kk]);
#pragma unroll
      for (int i = 0; i < 8; ++i) col[(8 * i + m2) * kHp] = v[i];
    }
    __syncthreads();
    // task (s, k1): 8-point DFT over m2 of rows 8 k1 ..
    if (tid < 256) {
      const int s = tid & 31, k1 = tid >> 5;
      double2* col = G + 8 * k1 * kHp + s;
      double2 v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = col[i * kHp];
      dft8(v);
#pragma unroll
      for (int i = 0; i < 8; ++i) col[i * kHp] = v[i];
    }
    __syncthreads();

    // ---- D: out: row K, columns 0..32 (lanes 33.. idle) ----
    if (lane <= kFft / 2) {
      const int sl = kHalfSlot[lane];
      double* o = spec + (pass ? kSpecR0 : kSpecW);
      for (int K = wave; K < kFft; K += WAVES) {
        const int Km = (kFft - K) & (kFft - 1);
        const double2 v = G[(8 * (K & 7) + (K >> 3)) * kHp + sl];
        double2 e = v;
        if (lane == 0 || lane == kFft / 2) {  // columns 0 and 32 from the shared slot
          const double2 vm = G[(8 * (Km & 7) + (Km >> 3)) * kHp + sl];
          e = lane == 0 ? make_double2(0.5 * (v.x + vm.x), 0.5 * (v.y - vm.y))
                        : make_double2(0.5 * (v.y + vm.y), -0.5 * (v.x - vm.x));
        }
        *reinterpret_cast<double2*>(o + 2 * (K * kHalf + lane)) = e;
      }
    }
    __syncthreads();  // the grid is free (next pass, then the W region)
  }
  return W0;
}

// RERANK (T = float only): the transforms run in double (rerank_transforms),
// and near-tied selections are re-scored exactly in double.  Its LDS (about
// 40 KB at K = 200) lets four workgroups share a CU, so with 4 wavefronts the
// register budget is set for four workgroups (4 wavefronts per SIMD, 128
// VGPRs); the 8- and 16-wavefront forms serve small launches (a workgroup or
// two per CU) and get the same 128 VGPRs (two and one workgroups per CU).
// MX (T = float, 4 wavefronts, no re-rank): the transforms run on matrix
// cores in split f16.
template <typename T, int WAVES, bool RERANK, bool MX = false>
__global__ __launch_bounds__(64 * WAVES, RERANK ? (WAVES == 4 ? 4 : 16 / WAVES) : (MX ? 4 : 1)) void
fse_block_kernel(BlockArgs<T> a) {
  constexpr int THREADS = 64 * WAVES;
  constexpr int ROWS = kFft / WAVES;
  static_assert(!RERANK || sizeof(T) == 4, "re-rank mode iterates in float");
  static_assert(!MX || (sizeof(T) == 4 && WAVES == 4 && !RERANK),
                "matrix-core transforms: float, 4 wavefronts");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = uniform_int(tid >> 6);
  const int K = a.K;

  // 4 wavefronts: split rows, so that W with its wrap-around rows and the
  // rest of the LDS take at most a quarter of a CU's LDS (FP32)
  constexpr bool SPLIT = WAVES == 4;
  constexpr int WRAP = SPLIT ? ROWS / 2 - 1 : ROWS - 1;
  const LdsLayout L = lds_layout(a.M, a.N, K, WAVES, (int)sizeof(T), !RERANK);
  T* Wl = reinterpret_cast<T*>(smem);  // (64 + WRAP) x 64 complex
  T* hdc = reinterpret_cast<T*>(smem + L.hist_dc);
  int* hu = reinterpret_cast<int*>(smem + L.hist_u);
  double* tw = reinterpret_cast<double*>(smem + L.tw64);
  Slot* slots = reinterpret_cast<Slot*>(smem + L.slots);

  const int item = blockIdx.x;
  const int fw = a.items[2 * item];
  const int fr = fw & kItemFrameMask;
  const int bij = a.items[2 * item + 1];
  // items on the critical chain of waves issue ahead of the other
  // workgroups sharing their SIMDs
  if (fw >> kItemPrioShift) __builtin_amdgcn_s_setprio(2);
  const int bi = (int)((unsigned)bij >> 16), bj = bij & 0xffff;
  const FrameDesc fd = a.frames[fr];
  const int H = fd.H, W = fd.W;
  T* img = a.work + fd.off;
  uint8_t* st = a.state + fd.off;
  const int by0 = bi * a.Bh - a.goy, bx0 = bj * a.Bw - a.gox;

  load_twiddles<T>(smem, L, a.twid64, !RERANK);
  // re-scoring statistics of this wavefront (uniform), added to the call's
  // counters once, after everything else the block does
  unsigned st_rescored = 0u, st_cand = 0u, st_wide = 0u, st_max = 0u;
  // re-rank: no exact re-scoring at or below this key (keys up to 63 carry
  // only row bits: |R|^2 = 0)
  unsigned floor_u = 63u;

  VecR<T, ROWS> rr, ri;
  T wvr[ROWS], wvi[ROWS];
  T W0;
  double W0d = 0.0;
  double* spec = nullptr;  // re-rank: this item's FP64 spectra
  if constexpr (RERANK) {
    spec = a.spec64 + (int64_t)item * kSpecStride;
    W0d = rerank_transforms<WAVES>(smem, L.tw64, L.slots, a.radial64, a.delta64, a.M, a.N, img,
                                   st, H, W, by0 - a.d, bx0 - a.d, spec);
    W0 = (T)W0d;
    if (W0d > 0.0) {  // the spectra as floats, back from this block's own writes
#pragma unroll
      for (int j = 0; j < ROWS; ++j) {
        const int k1 = row_of<WAVES, SPLIT>(wave, j);
        const double2 r = half_spec_at(spec + kSpecR0, k1, lane);
        const double2 w = half_spec_at(spec + kSpecW, k1, lane);
        rr[j] = (T)r.x;
        ri[j] = (T)r.y;
        wvr[j] = (T)w.x;
        wvi[j] = (T)w.y;
      }
    }
  } else if constexpr (MX) {
    W0 = forward_transforms_mx<T>(smem, L, a.M, a.N, a.radial, a.delta, a.zscale, img, st, H, W,
                                  by0 - a.d, bx0 - a.d, lane, wave, rr, ri, wvr, wvi);
  } else {
    W0 = forward_transforms<T, T, WAVES>(smem, L, a.M, a.N, a.radial, a.delta, a.zscale, img, st,
                                         H, W, by0 - a.d, bx0 - a.d, lane, wave, rr, ri, wvr,
                                         wvi);
  }

  if (W0 > T(0)) {
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      const int row = row_of<WAVES, SPLIT>(wave, j);
      T* p = Wl + (row * kFft + lane) * 2;
      p[0] = wvr[j];
      p[1] = wvi[j];
      if (row < WRAP) {  // wrap-around copy: a window of rows never wraps
        T* q = Wl + ((row + kFft) * kFft + lane) * 2;
        q[0] = wvr[j];
        q[1] = wvi[j];
      }
    }
    __syncthreads();

    // ---- D: K greedy iterations ----
    // Each iteration first applies the previous selection's update (a zero
    // update in the first iteration), then selects u = argmax |R|^2 and forms
    // the coefficient increment.
    //  FP64: exact |R|^2, ties to the smallest row-major index.
    //  FP32: |R|^2 compared with its 6 lowest mantissa bits replaced by
    //        63 - k1 (a relative resolution of 2^-17, below the rounding
    //        drift of a float spectrum), so one unsigned max gives value and
    //        row; ties go to the smallest k1, then the smallest k2.
    //  RERANK: when another entry comes within the relative gap of the
    //        maximum, the candidates are re-scored exactly in double from
    //        R0 - sum_i dc_i W[k - u_i] and the best exact one is taken.
    const T gs = a.gamma / W0;
    int u = 0;
    T dcr = T(0), dci = T(0);
    for (int it = 0; it < K; ++it) {
      const int col = (lane - (u & (kFft - 1))) & (kFft - 1);
      const int b = uniform_int((row_of<WAVES, SPLIT>(wave, 0) - (u >> 6)) & (kFft - 1));
      const int b2 = uniform_int((row_of<WAVES, SPLIT>(wave, ROWS / 2) - (u >> 6)) & (kFft - 1));
      const T* wp = Wl + (b * kFft + col) * 2;
      const T* wp2 = Wl + (b2 * kFft + col) * 2;
      // all W reads of the iteration in flight before the first update, so
      // that one LDS latency is exposed per iteration instead of one per pair
      T wvr_[ROWS], wvi_[ROWS];
#pragma unroll
      for (int j = 0; j < ROWS; ++j) {
        if (SPLIT && j >= ROWS / 2) {
          wvr_[j] = wp2[(j - ROWS / 2) * kFft * 2];
          wvi_[j] = wp2[(j - ROWS / 2) * kFft * 2 + 1];
        } else {
          wvr_[j] = wp[j * kFft * 2];
          wvi_[j] = wp[j * kFft * 2 + 1];
        }
      }
      if constexpr (sizeof(T) == 4) __builtin_amdgcn_sched_barrier(0);
      VecR<T, ROWS> e;
#pragma unroll
      for (int j = 0; j < ROWS; ++j) {
        const T wr = wvr_[j], wi = wvi_[j];
        T r = rr[j], q = ri[j];
        r = fma(-dcr, wr, r);
        r = fma(dci, wi, r);
        q = fma(-dcr, wi, q);
        q = fma(-dci, wr, q);
        rr[j] = r;
        ri[j] = q;
        e[j] = fma(r, r, q * q);
      }
      if constexpr (sizeof(T) == 4) {
        unsigned key[ROWS];
#pragma unroll
        for (int j = 0; j < ROWS; ++j)
          key[j] = pack_key(__float_as_uint(e[j]), (unsigned)(63 - row_of<WAVES, SPLIT>(wave, j)));
        unsigned lk, lk2 = 0u;
        if constexpr (RERANK) {
          top2<ROWS>(key, lk, lk2);  // lk2 tests a second near entry in the lane
        } else {
          lk = key[0];
#pragma unroll
          for (int j = 1; j + 1 < ROWS; j += 2) lk = umax3(lk, key[j], key[j + 1]);
          if constexpr (ROWS % 2 == 0) lk = max(lk, key[ROWS - 1]);
        }
        const unsigned wk = wave_max(lk);
        const unsigned long long hit = __ballot(lk == wk);
        const int lw = uniform_int(__builtin_ctzll(hit));
        const int jw = uniform_int(j_of_row<WAVES, SPLIT>(63 - (int)(wk & 63u), wave));
        int near = 0;
        if constexpr (RERANK) {
          // 2 when another entry of this wavefront lies within the gap of its
          // maximum (another lane's maximum, or a lane's second largest key),
          // else 1 (conservative: the block maximum is at least as large)
          const float lim = __uint_as_float(wk) * (float)(1.0 - a.rerank_gap);
          const unsigned thr = __float_as_uint(lim);
          const bool two = __ballot(lk2 >= thr) != 0ull ||
                           __builtin_popcountll(__ballot(lk >= thr)) >= 2;
          near = two ? 2 : 1;
        }
        // the lane holding the maximum writes the slot from its own registers
        // (its key is the wavefront's; the entry by uniform register index)
        FSlot* fs = reinterpret_cast<FSlot*>(smem + L.slots) + (it & 1) * WAVES;
        if (lane == lw) {
          FSlot v;
          v.key = lk;
          v.k = (row_of<WAVES, SPLIT>(wave, jw) << 6) | lane | (near << 12);
          v.re = rr[jw];
          v.im = ri[jw];
          fs[wave] = v;
        }
        __syncthreads();
        // every lane reads the slot of wavefront lane % WAVES (one LDS round
        // trip); the winning wavefront has the largest key (its row is in the
        // key), and its entry is taken from that lane
        const FSlot mine = fs[lane & (WAVES - 1)];
        const unsigned gk = group_max<WAVES>(mine.key);
        const int wwin = uniform_int(wave_of_row<WAVES, SPLIT>(63 - (int)(gk & 63u)));
        u = uniform_int(__builtin_amdgcn_readlane(mine.k, wwin) & 0xfff);
        dcr = gs * read_lane(mine.re, wwin);
        dci = gs * read_lane(mine.im, wwin);
        if constexpr (RERANK) {
          const unsigned thr_g = __float_as_uint(__uint_as_float(gk) * (float)(1.0 - a.rerank_gap));
          // lanes 0 .. WAVES-1 hold one slot each: the wavefronts whose
          // maxima lie within the gap of the block maximum, and those among
          // them that flagged a second entry within the gap of their own
          const unsigned long long in_gap =
              __ballot(mine.key >= thr_g) & ((1ull << WAVES) - 1ull);
          const unsigned long long flagged = __ballot(mine.k >= (2 << 12)) & in_gap;
          // no re-scoring once the float maximum is rounding noise: at or
          // below 2^-40 of the block's first maximum (an all-zero spectrum
          // would otherwise tie every entry)
          const bool live = gk > floor_u;
          if (it == 0) floor_u = (gk >> 23) > 40u ? gk - (40u << 23) : 63u;
          const bool rerank =
              live && (flagged != 0ull || __builtin_popcountll(in_gap) >= 2);
          if (rerank) {  // uniform: every wavefront read the same slots
            // Every wavefront re-scores all of its entries within the gap of
            // the block maximum exactly in double, three at a time (two with
            // 8 or 16 wavefronts) in row-major order, and offers its best
            // one; one barrier joins them.  No candidate is dropped.
            double bex = -1.0, bre = 0.0, bim = 0.0;
            int bkx = 1 << 30;
            // exact |R|^2 of NC candidates (12-bit indices in `packed`):
            // R0 - sum_i dc_i W[k - u_i] in double; the best one (ties to the
            // smallest index) goes to (bex, bre, bim, bkx)
            auto rescore = [&](auto nc_tag, unsigned long long packed) {
              constexpr int NC = decltype(nc_tag)::value;
              int kc[NC];
              double acc[2 * NC], r0r[NC], r0i[NC];
#pragma unroll
              for (int c = 0; c < NC; ++c) {
                kc[c] = (int)((packed >> (12 * c)) & 0xfffull);
                acc[2 * c] = acc[2 * c + 1] = 0.0;
                const double2 r0 = half_spec_at(spec + kSpecR0, kc[c] >> 6, kc[c] & (kFft - 1));
                r0r[c] = r0.x;
                r0i[c] = r0.y;
              }
              // history terms in rounds of kRound x 64 so that all gathers of
              // a round are in flight together (one memory latency per round)
              constexpr int kRound = WAVES == 4 ? 2 : 1;  // register budget
              for (int i0 = 0; i0 < it; i0 += 64 * kRound) {
                double wr[kRound][NC], wi[kRound][NC];
#pragma unroll
                for (int q = 0; q < kRound; ++q) {
                  const int i = i0 + 64 * q + lane;
                  const int uu = i < it ? hu[i] : 0;
#pragma unroll
                  for (int c = 0; c < NC; ++c) {
                    const int d1 = ((kc[c] >> 6) - (uu >> 6)) & (kFft - 1);
                    const int d2 = ((kc[c] & (kFft - 1)) - (uu & (kFft - 1))) & (kFft - 1);
                    const double2 wv = half_spec_at(spec + kSpecW, d1, d2);
                    wr[q][c] = wv.x;
                    wi[q][c] = wv.y;
                  }
                }
#pragma unroll
                for (int q = 0; q < kRound; ++q) {
                  const int i = i0 + 64 * q + lane;
                  const double xr = i < it ? (double)hdc[2 * i] : 0.0;
                  const double xi = i < it ? (double)hdc[2 * i + 1] : 0.0;
#pragma unroll
                  for (int c = 0; c < NC; ++c) {
                    acc[2 * c] = fma(xr, wr[q][c], fma(-xi, wi[q][c], acc[2 * c]));
                    acc[2 * c + 1] = fma(xr, wi[q][c], fma(xi, wr[q][c], acc[2 * c + 1]));
                  }
                }
              }
              wave_sums(acc);
#pragma unroll
              for (int c = 0; c < NC; ++c) {
                const double vr = r0r[c] - acc[2 * c];
                const double vi = r0i[c] - acc[2 * c + 1];
                const double ve = vr * vr + vi * vi;
                if (ve > bex || (ve == bex && kc[c] < bkx)) {
                  bex = ve;
                  bre = vr;
                  bim = vi;
                  bkx = kc[c];
                }
              }
            };
            constexpr int kChunk = WAVES == 4 ? 3 : 2;  // register budget
            unsigned long long packed = 0ull;
            int nc = 0, ncw = 0;
#pragma unroll
            for (int j = 0; j < ROWS; ++j) {
              unsigned long long mm = __ballot(key[j] >= thr_g);
              while (mm) {  // uniform
                const int l = __builtin_ctzll(mm);
                mm &= mm - 1;
                packed |= (unsigned long long)((row_of<WAVES, SPLIT>(wave, j) << 6) | l)
                          << (12 * nc);
                ++ncw;
                if (++nc == kChunk) {
                  rescore(std::integral_constant<int, kChunk>(), packed);
                  nc = 0;
                  packed = 0ull;
                }
              }
            }
            if (nc == 1) rescore(std::integral_constant<int, 1>(), packed);
            if constexpr (kChunk == 3) {
              if (nc == 2) rescore(std::integral_constant<int, 2>(), packed);
            }
            st_rescored += 1u;
            st_cand += (unsigned)ncw;
            st_wide += ncw > kChunk ? 1u : 0u;
            st_max = max(st_max, (unsigned)ncw);
            Slot* ex = reinterpret_cast<Slot*>(smem + L.cand) + (it & 1) * WAVES;
            if (lane == 0) {
              Slot v;
              v.e = bex;
              v.re = bre;
              v.im = bim;
              v.k = bkx;
              v.key = 0u;
              ex[wave] = v;
            }
            __syncthreads();
            Slot bb = ex[0];
#pragma unroll
            for (int q = 1; q < WAVES; ++q) {
              const Slot c = ex[q];
              if (c.e > bb.e || (c.e == bb.e && c.k < bb.k)) bb = c;
            }
            u = uniform_int(bb.k);
            dcr = (T)(a.gamma64 * bb.re / W0d);
            dci = (T)(a.gamma64 * bb.im / W0d);
          }
        }
      } else {
        Slot* sl = slots + (it & 1) * WAVES;
        T lm = e[0];
#pragma unroll
        for (int j = 1; j < ROWS; ++j) lm = fmax(lm, e[j]);
        const T wm = wave_max(lm);
        // first (row, lane) holding the wave maximum
        unsigned long long hit = 0;
        int jw = 0;
#pragma unroll
        for (int j = ROWS - 1; j >= 0; --j) {
          const unsigned long long mj = __ballot(e[j] == wm);
          if (mj) {
            hit = mj;
            jw = j;
          }
        }
        jw = uniform_int(jw);
        const int lw = uniform_int(__builtin_ctzll(hit));
        if (lane == lw) {  // the lane holding the maximum writes the slot
          Slot v;
          v.e = wm;
          v.re = rr[jw];
          v.im = ri[jw];
          v.k = (row_of<WAVES, SPLIT>(wave, jw) << 6) | lane;
          sl[wave] = v;
        }
        __syncthreads();
        // the largest |R|^2, ties to the smallest index k: consecutive rows
        // per wavefront cover increasing k, so a strict > keeps the smallest;
        // split rows compare the indices
        Slot best = sl[0];
#pragma unroll
        for (int q = 1; q < WAVES; ++q) {
          const Slot c = sl[q];
          if constexpr (SPLIT) {
            if (c.e > best.e || (c.e == best.e && c.k < best.k)) best = c;
          } else {
            if (c.e > best.e) best = c;
          }
        }
        u = uniform_int(best.k);
        dcr = gs * (T)best.re;
        dci = gs * (T)best.im;
      }
      if (tid == 0) {
        hu[it] = u;
        hdc[2 * it] = dcr;
        hdc[2 * it + 1] = dci;
      }
    }
    __syncthreads();
  }

  // ---- E: model samples on B_i (Eq. (1)), sums in double ----
  const bool empty = !(W0 > T(0));
  const int nb = a.Bh * a.Bw;
  for (int s = tid; s < nb; s += THREADS) {
    const int dy = s / a.Bw, dx = s - dy * a.Bw;
    const int y = by0 + dy, x = bx0 + dx;
    if (y < 0 || y >= H || x < 0 || x >= W) continue;
    const int64_t p = (int64_t)y * W + x;
    if (st[p] != kPending) continue;
    double acc;
    if (empty) {
      acc = a.empty_fill;
    } else {
      const int m = a.d + dy, n = a.d + dx;
      acc = 0.0;
      for (int i = 0; i < K; ++i) {
        const int uu = hu[i];
        const int t = ((uu >> 6) * m + (uu & (kFft - 1)) * n) & (kFft - 1);
        acc = fma((double)hdc[2 * i], tw[2 * t], acc);
        acc = fma(-(double)hdc[2 * i + 1], tw[2 * t + 1], acc);
      }
    }
    if (a.staging) {
      a.staging[(int64_t)item * nb + s] = (T)acc;
    } else {
      img[p] = (T)acc;
      st[p] = kRecon;
    }
  }
  if (a.trace_u) {
    for (int i = tid; i < K; i += THREADS) {
      a.trace_u[(int64_t)item * K + i] = empty ? -1 : hu[i];
      a.trace_dc[((int64_t)item * K + i) * 2] = empty ? T(0) : hdc[2 * i];
      a.trace_dc[((int64_t)item * K + i) * 2 + 1] = empty ? T(0) : hdc[2 * i + 1];
    }
  }
  if (RERANK && a.counters && lane == 0 && st_rescored > 0u) {
    // one update per wavefront and block (re-scored iterations counted once,
    // by wavefront 0); nothing waits for these atomics
    if (wave == 0) atomicAdd(&a.counters[kCntRescored], (unsigned long long)st_rescored);
    if (st_cand) atomicAdd(&a.counters[kCntCandidates], (unsigned long long)st_cand);
    if (st_wide) atomicAdd(&a.counters[kCntWide], (unsigned long long)st_wide);
    atomicMax(&a.counters[kCntMaxWave], (unsigned long long)st_max);
  }
}

// Apply staged block results after a wave (used when d exceeds the block
// size, so that blocks of one wave may see each other's areas).
template <typename T>
__global__ void fse_scatter_kernel(T* work, uint8_t* state, const FrameDesc* frames,
                                   const int32_t* items, const T* staging, int Bh, int Bw,
                                   int gox, int goy) {
  const int item = blockIdx.x;
  const int fr = items[2 * item] & kItemFrameMask, bij = items[2 * item + 1];
  const int bi = (int)((unsigned)bij >> 16), bj = bij & 0xffff;
  const FrameDesc fd = frames[fr];
  const int nb = Bh * Bw;
  for (int s = threadIdx.x; s < nb; s += blockDim.x) {
    const int dy = s / Bw, dx = s - dy * Bw;
    const int y = bi * Bh - goy + dy, x = bj * Bw - gox + dx;
    if (y < 0 || y >= fd.H || x < 0 || x >= fd.W) continue;
    const int64_t p = fd.off + (int64_t)y * fd.W + x;
    if (state[p] != kPending) continue;
    work[p] = staging[(int64_t)item * nb + s];
    state[p] = kRecon;
  }
}

// Working image and state map of every frame from its 8-bit input (when
// `convert`), and (each nullable) the flag of every block that holds a lost
// sample and the number of lost samples per block (zeroed by the caller).
// blockIdx.y = frame.
template <typename T>
__global__ void fse_init_kernel(const IoDesc* io, T* work, uint8_t* state, uint8_t* flags,
                                int32_t* counts, bool convert, int Bh, int Bw, int gox, int goy) {
  const IoDesc d = io[blockIdx.y];
  for (int y = blockIdx.x; y < d.H; y += gridDim.x) {  // rows; lanes along the row
    const uint8_t* lr = d.lost + (int64_t)y * d.lstride;
    const uint8_t* ir = d.image + (int64_t)y * d.stride;
    const int64_t o = d.off + (int64_t)y * d.W;
    const int64_t frow = d.flag_off + (int64_t)((y + goy) / Bh) * d.wb;
    for (int x = threadIdx.x; x < d.W; x += blockDim.x) {
      const bool l = lr[x] != 0;
      if (convert) {
        work[o + x] = l ? T(0) : (T)ir[x];
        state[o + x] = l ? kPending : kKnown;
      }
      if (l && flags) flags[frow + (x + gox) / Bw] = 1;
      if (l && counts) atomicAdd(counts + frow + (x + gox) / Bw, 1);
    }
  }
}

// Output of every frame: known samples copied, lost samples rounded
// half-to-even and clamped to [0, 255].  blockIdx.y = frame.
template <typename T>
__global__ void fse_finalize_kernel(const IoDesc* io, const uint8_t* state, const T* work) {
  const IoDesc d = io[blockIdx.y];
  for (int y = blockIdx.x; y < d.H; y += gridDim.x) {  // rows; lanes along the row
    const int64_t o = d.off + (int64_t)y * d.W;
    const int64_t oi = (int64_t)y * d.W;
    const uint8_t* ir = d.image + (int64_t)y * d.stride;
    uint8_t* outr = d.out + (int64_t)y * d.ostride;
    for (int x = threadIdx.x; x < d.W; x += blockDim.x) {
      const T v = work[o + x];
      uint8_t b;
      if (state[o + x] == kKnown) {
        b = ir[x];
      } else {
        T r = rint(v);
        r = r < T(0) ? T(0) : (r > T(255) ? T(255) : r);
        b = (uint8_t)r;
      }
      outr[x] = b;
      if (d.of32) d.of32[oi + x] = (float)v;
      if (d.of64) d.of64[oi + x] = (double)v;
    }
  }
}

// ---------------------------------------------------------------- launchers

template <typename K, typename... Args>
static hipError_t launch_with_lds(K kernel, size_t& attr_bytes, int n_items, int threads,
                                  size_t lds, hipStream_t s, Args... args) {
  if (lds > attr_bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_bytes = lds;
  }
  hipLaunchKernelGGL(kernel, dim3(n_items), dim3(threads), lds, s, args...);
  return hipGetLastError();
}

template <typename T, int WAVES, bool RERANK, bool MX = false>
static hipError_t launch_block_w(const BlockArgs<T>& a, int n_items, hipStream_t s) {
  static size_t attr_bytes = 0;  // largest dynamic LDS size enabled so far
  const size_t lds = (size_t)lds_bytes<T>(a.M, a.N, a.K, WAVES, !RERANK);
  return launch_with_lds(fse_block_kernel<T, WAVES, RERANK, MX>, attr_bytes, n_items, 64 * WAVES,
                         lds, s, a);
}

// mode: 0 = plain, 1 = FP32 iterations on FP64 spectra with re-ranking,
// 2 = FP32 with matrix-core f16x3 transforms (4 wavefronts only)
template <typename T>
hipError_t launch_block(const BlockArgs<T>& a, int n_items, int waves, hipStream_t s,
                        int mode = 0);

template <>
hipError_t launch_block<double>(const BlockArgs<double>& a, int n_items, int waves, hipStream_t s,
                                int mode) {
  if (n_items <= 0) return hipSuccess;
  if (mode != 0) return hipErrorInvalidValue;
  switch (waves) {
    case 4: return launch_block_w<double, 4, false>(a, n_items, s);
    case 8: return launch_block_w<double, 8, false>(a, n_items, s);
    case 16: return launch_block_w<double, 16, false>(a, n_items, s);
    default: return hipErrorInvalidValue;
  }
}

template <>
hipError_t launch_block<float>(const BlockArgs<float>& a, int n_items, int waves, hipStream_t s,
                               int mode) {
  if (n_items <= 0) return hipSuccess;
  if (mode == 2) {
    if (waves != 4) return hipErrorInvalidValue;
    return launch_block_w<float, 4, false, true>(a, n_items, s);
  }
  if (mode == 1) {
    switch (waves) {
      case 4: return launch_block_w<float, 4, true>(a, n_items, s);
      case 8: return launch_block_w<float, 8, true>(a, n_items, s);
      case 16: return launch_block_w<float, 16, true>(a, n_items, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (waves) {
    case 4: return launch_block_w<float, 4, false>(a, n_items, s);
    case 8: return launch_block_w<float, 8, false>(a, n_items, s);
    case 16: return launch_block_w<float, 16, false>(a, n_items, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_scatter(T* work, uint8_t* state, const FrameDesc* frames, const int32_t* items,
                          int n_items, const T* staging, int Bh, int Bw, int gox, int goy,
                          hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(fse_scatter_kernel<T>, dim3(n_items), dim3(256), 0, s, work, state, frames,
                     items, staging, Bh, Bw, gox, goy);
  return hipGetLastError();
}

// Workgroups per frame of the init and finalize kernels: one row each, at
// most 256 (a workgroup strides over the rows), at least enough for the
// largest frame's rows at 64 pixels per row.
static int grid_rows(int64_t max_pixels) {
  int64_t g = (max_pixels + 4095) / 4096;
  if (g > 256) g = 256;
  return (int)(g < 1 ? 1 : g);
}

template <typename T>
hipError_t launch_init(const IoDesc* io, int nframes, int64_t max_pixels, T* work,
                       uint8_t* state, uint8_t* flags, int32_t* counts, bool convert, int Bh,
                       int Bw, int gox, int goy, hipStream_t s) {
  hipLaunchKernelGGL(fse_init_kernel<T>, dim3(grid_rows(max_pixels), nframes), dim3(256), 0, s,
                     io, work, state, flags, counts, convert, Bh, Bw, gox, goy);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_finalize(const IoDesc* io, int nframes, int64_t max_pixels,
                           const uint8_t* state, const T* work, hipStream_t s) {
  hipLaunchKernelGGL(fse_finalize_kernel<T>, dim3(grid_rows(max_pixels), nframes), dim3(256), 0,
                     s, io, state, work);
  return hipGetLastError();
}

template hipError_t launch_scatter<float>(float*, uint8_t*, const FrameDesc*, const int32_t*, int,
                                          const float*, int, int, int, int, hipStream_t);
template hipError_t launch_scatter<double>(double*, uint8_t*, const FrameDesc*, const int32_t*,
                                           int, const double*, int, int, int, int, hipStream_t);
template hipError_t launch_init<float>(const IoDesc*, int, int64_t, float*, uint8_t*, uint8_t*,
                                       int32_t*, bool, int, int, int, int, hipStream_t);
template hipError_t launch_init<double>(const IoDesc*, int, int64_t, double*, uint8_t*, uint8_t*,
                                        int32_t*, bool, int, int, int, int, hipStream_t);
template hipError_t launch_finalize<float>(const IoDesc*, int, int64_t, const uint8_t*,
                                           const float*, hipStream_t);
template hipError_t launch_finalize<double>(const IoDesc*, int, int64_t, const uint8_t*,
                                            const double*, hipStream_t);

}  // namespace fse
