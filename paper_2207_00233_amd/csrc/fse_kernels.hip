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
// Spectrum layout in the iteration: wavefront w owns rows k1 = ROWS*w ..
// ROWS*w + ROWS-1 (ROWS = 64 / WAVES), lane l owns column k2 = l, so every lane
// keeps ROWS complex entries in registers and reads W[k - u] from LDS with a
// per-lane column offset.  WAVES = 4 is the throughput shape; WAVES = 16
// quarters the serial work per iteration for waves too small to fill the GPU.
#include <hip/hip_runtime.h>

#include "fse_device.h"

namespace fse {

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

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

__device__ __forceinline__ unsigned umax3(unsigned a, unsigned b, unsigned c) {
  return max(a, max(b, c));
}

// (bits & ~63) | (low & 63) as one bit-field insert (the compiler otherwise
// splits it into two operations).
__device__ __forceinline__ unsigned pack_key(unsigned bits, unsigned low) {
  unsigned r;
  asm("v_bfi_b32 %0, 63, %1, %2" : "=v"(r) : "s"(low), "v"(bits));
  return r;
}

// Argmax slot exchanged between wavefronts (32 bytes).
struct Slot {
  double e;     // FP64 path: exact |R|^2 of the wave's best entry
  double re, im;
  unsigned key; // FP32 path: packed selection key of the wave's best entry
  int k;        // its spectrum index k1 * 64 + k2
};

template <typename T, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void fse_block_kernel(BlockArgs<T> a) {
  constexpr int THREADS = 64 * WAVES;
  constexpr int ROWS = kFft / WAVES;
  constexpr int QB = (kHalf + WAVES - 1) / WAVES;  // row-DFT columns per wavefront
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = uniform_int(tid >> 6);
  const int M = a.M, N = a.N, NP = N | 1, K = a.K;

  const LdsLayout L = lds_layout(M, N, K, WAVES, (int)sizeof(T));
  T* xs = reinterpret_cast<T*>(smem);
  T* ws = xs + M * NP;
  T* bx = reinterpret_cast<T*>(smem + L.bx);
  T* bw = reinterpret_cast<T*>(smem + L.bw);
  T* Wl = reinterpret_cast<T*>(smem);  // (64 + ROWS - 1) x 64 complex, after phase C
  T* hdc = reinterpret_cast<T*>(smem + L.hist_dc);
  int* hu = reinterpret_cast<int*>(smem + L.hist_u);
  double* tw = reinterpret_cast<double*>(smem + L.tw64);
  T* twt = reinterpret_cast<T*>(smem + L.twt);
  Slot* slots = reinterpret_cast<Slot*>(smem + L.slots);

  const int item = blockIdx.x;
  const int fr = a.items[2 * item];
  const int bij = a.items[2 * item + 1];
  const int bi = bij >> 16, bj = bij & 0xffff;
  const FrameDesc fd = a.frames[fr];
  const int H = fd.H, W = fd.W;
  T* img = a.work + fd.off;
  uint8_t* st = a.state + fd.off;
  const int by0 = bi * a.Bh - a.goy, bx0 = bj * a.Bw - a.gox;
  const int oy = by0 - a.d, ox = bx0 - a.d;

  if (tid < 2 * kFft) {
    const double v = a.twid64[tid];
    tw[tid] = v;
    twt[tid] = (T)v;
  }

  // ---- A: gather, classify, weight (Eq. (2)) ----
  T wsum = T(0);
  for (int i = tid; i < M * N; i += THREADS) {
    const int m = i / N, n = i - m * N;
    const int y = oy + m, x = ox + n;
    T wv = T(0), xv = T(0);
    if (y >= 0 && y < H && x >= 0 && x < W) {
      const int64_t p = (int64_t)y * W + x;
      const uint8_t s = st[p];
      const T fac = s == kKnown ? T(1) : (s == kRecon ? a.delta : T(0));
      wv = a.radial[i] * fac;
      xv = img[p] * wv;
    }
    ws[m * NP + n] = wv;
    xs[m * NP + n] = xv;
    wsum += wv;
  }
  wsum = wave_sum(wsum);
  if (lane == 0) slots[wave].e = (double)wsum;
  __syncthreads();
  T W0 = T(0);
#pragma unroll
  for (int q = 0; q < WAVES; ++q) W0 += (T)slots[q].e;

  if (W0 > T(0)) {
    // ---- B: real row DFTs, columns k2 = wave + WAVES q, k2 <= 32 ----
    {
      T axr[QB], axi[QB], awr[QB], awi[QB];
#pragma unroll
      for (int q = 0; q < QB; ++q) axr[q] = axi[q] = awr[q] = awi[q] = T(0);
      if (lane < M) {
        for (int n = 0; n < N; ++n) {
          const T xv = xs[lane * NP + n], wv = ws[lane * NP + n];
#pragma unroll
          for (int q = 0; q < QB; ++q) {
            const int t = ((wave + WAVES * q) * n) & (kFft - 1);
            const T c = twt[2 * t], s = twt[2 * t + 1];
            axr[q] = fma(xv, c, axr[q]);
            axi[q] = fma(-xv, s, axi[q]);
            awr[q] = fma(wv, c, awr[q]);
            awi[q] = fma(-wv, s, awi[q]);
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
    VecR<T, ROWS> rr, ri;
    {
      const int c = lane <= 32 ? lane : kFft - lane;
      const T sg = lane <= 32 ? T(1) : T(-1);  // conjugate mirrored columns
      const T zs = a.zscale;
#pragma unroll
      for (int j = 0; j < ROWS; ++j) rr[j] = ri[j] = T(0);
      for (int m = 0; m < M; ++m) {
        const T xr = bx[(m * kHalf + c) * 2], xi = sg * bx[(m * kHalf + c) * 2 + 1];
        const T wr = bw[(m * kHalf + c) * 2], wi = sg * bw[(m * kHalf + c) * 2 + 1];
        const T zr = fma(-zs, wi, xr), zi = fma(zs, wr, xi);
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
          const int t = ((ROWS * wave + j) * m) & (kFft - 1);
          const T cc = twt[2 * t], ss = twt[2 * t + 1];
          rr[j] = fma(zr, cc, fma(zi, ss, rr[j]));
          ri[j] = fma(zi, cc, fma(-zr, ss, ri[j]));
        }
      }
    }
    __syncthreads();  // phase-B buffers are dead from here on
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      T* p = Wl + ((ROWS * wave + j) * kFft + lane) * 2;
      p[0] = rr[j];
      p[1] = ri[j];
    }
    __syncthreads();
    // unpack: X[k] = (Z[k] + conj Z[-k]) / 2, W[k] = (Z[k] - conj Z[-k]) / (2 j s)
    T wvr[ROWS], wvi[ROWS];
    {
      const T h = T(0.5), hs = T(0.5) / a.zscale;
#pragma unroll
      for (int j = 0; j < ROWS; ++j) {
        const int k1 = ROWS * wave + j;
        const T* p = Wl + ((((kFft - k1) & (kFft - 1)) * kFft) + ((kFft - lane) & (kFft - 1))) * 2;
        const T pr = p[0], pi = p[1];
        const T ar = rr[j], ai = ri[j];
        rr[j] = h * (ar + pr);
        ri[j] = h * (ai - pi);
        wvr[j] = hs * (ai + pi);
        wvi[j] = hs * (pr - ar);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      const int row = ROWS * wave + j;
      T* p = Wl + (row * kFft + lane) * 2;
      p[0] = wvr[j];
      p[1] = wvi[j];
      if (row < ROWS - 1) {  // wrap-around copy: a wave's ROWS rows never wrap
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
    const T gs = a.gamma / W0;
    int u = 0;
    T dcr = T(0), dci = T(0);
    for (int it = 0; it < K; ++it) {
      const int col = (lane - (u & (kFft - 1))) & (kFft - 1);
      const int b = uniform_int((ROWS * wave - (u >> 6)) & (kFft - 1));
      const T* wp = Wl + (b * kFft + col) * 2;
      VecR<T, ROWS> e;
#pragma unroll
      for (int j = 0; j < ROWS; ++j) {
        const T wr = wp[j * kFft * 2], wi = wp[j * kFft * 2 + 1];
        T r = rr[j], q = ri[j];
        r = fma(-dcr, wr, r);
        r = fma(dci, wi, r);
        q = fma(-dcr, wi, q);
        q = fma(-dci, wr, q);
        rr[j] = r;
        ri[j] = q;
        e[j] = fma(r, r, q * q);
      }
      Slot* sl = slots + (it & 1) * WAVES;
      if constexpr (sizeof(T) == 4) {
        unsigned key[ROWS];
#pragma unroll
        for (int j = 0; j < ROWS; ++j)
          key[j] = pack_key(__float_as_uint(e[j]), (unsigned)(63 - (ROWS * wave + j)));
        unsigned lk = key[0];
#pragma unroll
        for (int j = 1; j + 1 < ROWS; j += 2) lk = umax3(lk, key[j], key[j + 1]);
        if constexpr (ROWS % 2 == 0) lk = max(lk, key[ROWS - 1]);
        const unsigned wk = wave_max(lk);
        const unsigned long long hit = __ballot(lk == wk);
        const int lw = uniform_int(__builtin_ctzll(hit));
        const int jw = uniform_int(63 - (int)(wk & 63u) - ROWS * wave);
        const T sr = read_lane((T)rr[jw], lw);
        const T si = read_lane((T)ri[jw], lw);
        if (lane == 0) {
          Slot v;
          v.key = wk;
          v.k = ((ROWS * wave + jw) << 6) | lw;
          v.re = sr;
          v.im = si;
          sl[wave] = v;
        }
        __syncthreads();
        // the winning wavefront: largest key (its row is in the key)
        unsigned gk = lane < WAVES ? sl[lane].key : 0u;
        gk = wave_max(gk);
        const int wwin = uniform_int((63 - (int)(gk & 63u)) / ROWS);
        const Slot best = sl[wwin];
        u = uniform_int(best.k);
        dcr = gs * (T)best.re;
        dci = gs * (T)best.im;
      } else {
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
        const T sr = read_lane((T)rr[jw], lw);
        const T si = read_lane((T)ri[jw], lw);
        if (lane == 0) {
          Slot v;
          v.e = wm;
          v.re = sr;
          v.im = si;
          v.k = ((ROWS * wave + jw) << 6) | lw;
          sl[wave] = v;
        }
        __syncthreads();
        // wavefronts cover increasing k, so a strict > keeps the smallest k
        Slot best = sl[0];
#pragma unroll
        for (int q = 1; q < WAVES; ++q) {
          const Slot c = sl[q];
          if (c.e > best.e) best = c;
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
}

// Apply staged block results after a wave (used when d exceeds the block
// size, so that blocks of one wave may see each other's areas).
template <typename T>
__global__ void fse_scatter_kernel(T* work, uint8_t* state, const FrameDesc* frames,
                                   const int32_t* items, const T* staging, int Bh, int Bw,
                                   int gox, int goy) {
  const int item = blockIdx.x;
  const int fr = items[2 * item], bij = items[2 * item + 1];
  const int bi = bij >> 16, bj = bij & 0xffff;
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

// Working image and state map of every frame from its 8-bit input, and the
// flag of every block that holds a lost sample.  blockIdx.y = frame.
template <typename T>
__global__ void fse_init_kernel(const IoDesc* io, T* work, uint8_t* state, uint8_t* flags,
                                int Bh, int Bw, int gox, int goy) {
  const IoDesc d = io[blockIdx.y];
  const int64_t n = (int64_t)d.H * d.W;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / d.W), x = (int)(i - (int64_t)y * d.W);
    const bool l = d.lost[(int64_t)y * d.lstride + x] != 0;
    work[d.off + i] = l ? T(0) : (T)d.image[(int64_t)y * d.stride + x];
    state[d.off + i] = l ? kPending : kKnown;
    if (l && flags) flags[d.flag_off + (int64_t)((y + goy) / Bh) * d.wb + (x + gox) / Bw] = 1;
  }
}

// Output of every frame: known samples copied, lost samples rounded
// half-to-even and clamped to [0, 255].  blockIdx.y = frame.
template <typename T>
__global__ void fse_finalize_kernel(const IoDesc* io, const uint8_t* state, const T* work) {
  const IoDesc d = io[blockIdx.y];
  const int64_t n = (int64_t)d.H * d.W;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / d.W), x = (int)(i - (int64_t)y * d.W);
    const T v = work[d.off + i];
    uint8_t o;
    if (state[d.off + i] == kKnown) {
      o = d.image[(int64_t)y * d.stride + x];
    } else {
      T r = rint(v);
      r = r < T(0) ? T(0) : (r > T(255) ? T(255) : r);
      o = (uint8_t)r;
    }
    d.out[(int64_t)y * d.ostride + x] = o;
    if (d.of32) d.of32[i] = (float)v;
    if (d.of64) d.of64[i] = (double)v;
  }
}

// ---------------------------------------------------------------- launchers

template <typename T, int WAVES>
static hipError_t launch_block_w(const BlockArgs<T>& a, int n_items, size_t lds, hipStream_t s) {
  static size_t attr_bytes = 0;  // largest dynamic LDS size enabled so far
  if (lds > attr_bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)fse_block_kernel<T, WAVES>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_bytes = lds;
  }
  hipLaunchKernelGGL((fse_block_kernel<T, WAVES>), dim3(n_items), dim3(64 * WAVES), lds, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_block(const BlockArgs<T>& a, int n_items, int waves, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const size_t lds = (size_t)lds_bytes<T>(a.M, a.N, a.K, waves);
  switch (waves) {
    case 4: return launch_block_w<T, 4>(a, n_items, lds, s);
    case 16: return launch_block_w<T, 16>(a, n_items, lds, s);
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

static int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 2048) g = 2048;
  return (int)(g < 1 ? 1 : g);
}

template <typename T>
hipError_t launch_init(const IoDesc* io, int nframes, int64_t max_pixels, T* work,
                       uint8_t* state, uint8_t* flags, int Bh, int Bw, int gox, int goy,
                       hipStream_t s) {
  hipLaunchKernelGGL(fse_init_kernel<T>, dim3(grid_for(max_pixels), nframes), dim3(256), 0, s,
                     io, work, state, flags, Bh, Bw, gox, goy);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_finalize(const IoDesc* io, int nframes, int64_t max_pixels,
                           const uint8_t* state, const T* work, hipStream_t s) {
  hipLaunchKernelGGL(fse_finalize_kernel<T>, dim3(grid_for(max_pixels), nframes), dim3(256), 0,
                     s, io, state, work);
  return hipGetLastError();
}

template hipError_t launch_block<float>(const BlockArgs<float>&, int, int, hipStream_t);
template hipError_t launch_block<double>(const BlockArgs<double>&, int, int, hipStream_t);
template hipError_t launch_scatter<float>(float*, uint8_t*, const FrameDesc*, const int32_t*, int,
                                          const float*, int, int, int, int, hipStream_t);
template hipError_t launch_scatter<double>(double*, uint8_t*, const FrameDesc*, const int32_t*,
                                           int, const double*, int, int, int, int, hipStream_t);
template hipError_t launch_init<float>(const IoDesc*, int, int64_t, float*, uint8_t*, uint8_t*,
                                       int, int, int, int, hipStream_t);
template hipError_t launch_init<double>(const IoDesc*, int, int64_t, double*, uint8_t*, uint8_t*,
                                        int, int, int, int, hipStream_t);
template hipError_t launch_finalize<float>(const IoDesc*, int, int64_t, const uint8_t*,
                                           const float*, hipStream_t);
template hipError_t launch_finalize<double>(const IoDesc*, int, int64_t, const uint8_t*,
                                            const double*, hipStream_t);

}  // namespace fse
