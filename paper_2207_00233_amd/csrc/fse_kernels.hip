// fse_kernels.hip -- HIP kernels (gfx950) of Frequency Selective Extrapolation.
//
// One workgroup (256 threads, 4 wavefronts) extrapolates one lost block:
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
// Spectrum layout in the iteration: wave w owns rows k1 = 16w .. 16w+15, lane
// l owns column k2 = l, so every lane keeps 16 complex entries in registers
// and reads W[k - u] from LDS with a per-lane column offset.
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

// 16 spectrum entries of one lane.  A vector type keeps them in registers
// even when indexed by a wave-uniform run-time index (register-indexed move).
template <typename T>
using Vec16 = T __attribute__((ext_vector_type(16)));

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

struct Lds {
  int64_t region, hist;
};

template <typename T>
__device__ __forceinline__ Lds lds_layout(int M, int N, int K) {
  const int NP = N | 1;
  int64_t stage = 2LL * M * NP * sizeof(T) + 2LL * M * kHalf * 2 * sizeof(T);
  int64_t wreg = (int64_t)kFft * kFft * 2 * sizeof(T);
  int64_t region = stage > wreg ? stage : wreg;
  region = (region + 15) & ~15LL;
  int64_t hist = (int64_t)K * (2 * sizeof(T)) + (int64_t)K * sizeof(int32_t);
  hist = (hist + 15) & ~15LL;
  return {region, hist};
}

template <typename T>
__global__ __launch_bounds__(kThreads) void fse_block_kernel(BlockArgs<T> a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = uniform_int(tid >> 6);
  const int M = a.M, N = a.N, NP = N | 1, K = a.K;

  const Lds L = lds_layout<T>(M, N, K);
  T* xs = reinterpret_cast<T*>(smem);
  T* ws = xs + M * NP;
  T* bx = ws + M * NP;
  T* bw = bx + M * kHalf * 2;
  T* Wl = reinterpret_cast<T*>(smem);  // 64 x 64 complex, after phase C
  T* hdc = reinterpret_cast<T*>(smem + L.region);
  int* hu = reinterpret_cast<int*>(hdc + 2 * K);
  double* tw = reinterpret_cast<double*>(smem + L.region + L.hist);  // 128
  double* slots = tw + 2 * kFft;  // 2 x 4 x {e, k, re, im}
  double* misc = slots + 2 * kWaves * 4;

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

  if (tid < 2 * kFft) tw[tid] = a.twid64[tid];

  // ---- A: gather, classify, weight (Eq. (2)) ----
  T wsum = T(0);
  for (int i = tid; i < M * N; i += kThreads) {
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
  if (lane == 0) misc[wave] = (double)wsum;
  __syncthreads();
  const T W0 = ((T)misc[0] + (T)misc[1]) + ((T)misc[2] + (T)misc[3]);

  // twiddles in the working precision (wave-uniform reads broadcast)
  auto twc = [&](int t) { return (T)tw[2 * t]; };
  auto tws = [&](int t) { return (T)tw[2 * t + 1]; };

  if (W0 > T(0)) {
    // ---- B: real row DFTs, columns k2 = wave + 4q (q = 0..8), k2 <= 32 ----
    {
      T axr[9], axi[9], awr[9], awi[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) axr[q] = axi[q] = awr[q] = awi[q] = T(0);
      if (lane < M) {
        for (int n = 0; n < N; ++n) {
          const T xv = xs[lane * NP + n], wv = ws[lane * NP + n];
#pragma unroll
          for (int q = 0; q < 9; ++q) {
            const int k2 = wave + 4 * q;
            const int t = (k2 * n) & (kFft - 1);
            const T c = twc(t), s = tws(t);
            axr[q] += xv * c;
            axi[q] -= xv * s;
            awr[q] += wv * c;
            awi[q] -= wv * s;
          }
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          const int k2 = wave + 4 * q;
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

    // ---- C: column DFT of z = x + j s w for k1 = 16 wave + j, k2 = lane ----
    Vec16<T> rr, ri;
    {
      const int c = lane <= 32 ? lane : kFft - lane;
      const T sg = lane <= 32 ? T(1) : T(-1);  // conjugate mirrored columns
      const T zs = a.zscale;
#pragma unroll
      for (int j = 0; j < kRowsPerWave; ++j) rr[j] = ri[j] = T(0);
      for (int m = 0; m < M; ++m) {
        const T xr = bx[(m * kHalf + c) * 2], xi = sg * bx[(m * kHalf + c) * 2 + 1];
        const T wr = bw[(m * kHalf + c) * 2], wi = sg * bw[(m * kHalf + c) * 2 + 1];
        const T zr = xr - zs * wi, zi = xi + zs * wr;
#pragma unroll
        for (int j = 0; j < kRowsPerWave; ++j) {
          const int t = ((kRowsPerWave * wave + j) * m) & (kFft - 1);
          const T cc = twc(t), ss = tws(t);
          rr[j] += zr * cc + zi * ss;
          ri[j] += zi * cc - zr * ss;
        }
      }
    }
    __syncthreads();  // phase-B buffers are dead from here on
#pragma unroll
    for (int j = 0; j < kRowsPerWave; ++j) {
      T* p = Wl + ((kRowsPerWave * wave + j) * kFft + lane) * 2;
      p[0] = rr[j];
      p[1] = ri[j];
    }
    __syncthreads();
    // unpack: X[k] = (Z[k] + conj Z[-k]) / 2, W[k] = (Z[k] - conj Z[-k]) / (2 j s)
    T wvr[kRowsPerWave], wvi[kRowsPerWave];
    {
      const T h = T(0.5), hs = T(0.5) / a.zscale;
#pragma unroll
      for (int j = 0; j < kRowsPerWave; ++j) {
        const int k1 = kRowsPerWave * wave + j;
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
    for (int j = 0; j < kRowsPerWave; ++j) {
      T* p = Wl + ((kRowsPerWave * wave + j) * kFft + lane) * 2;
      p[0] = wvr[j];
      p[1] = wvi[j];
    }
    __syncthreads();

    // ---- D: K greedy iterations ----
    const T gs = a.gamma / W0;
    int u = 0;
    T dcr = T(0), dci = T(0);
    for (int it = 0; it < K; ++it) {
      T be = T(-1);
      int bjx = 0;
      if (it > 0) {
        const int u1 = u >> 6, u2 = u & (kFft - 1);
        const int col = (lane - u2) & (kFft - 1);
        const int b = uniform_int((kRowsPerWave * wave - u1) & (kFft - 1));
        if (b <= kFft - kRowsPerWave) {
          const T* wp = Wl + (b * kFft + col) * 2;
#pragma unroll
          for (int j = 0; j < kRowsPerWave; ++j) {
            const T wr = wp[j * kFft * 2], wi = wp[j * kFft * 2 + 1];
            rr[j] -= dcr * wr - dci * wi;
            ri[j] -= dcr * wi + dci * wr;
            const T e = rr[j] * rr[j] + ri[j] * ri[j];
            if (e > be) { be = e; bjx = j; }
          }
        } else {
#pragma unroll
          for (int j = 0; j < kRowsPerWave; ++j) {
            const T* wp = Wl + ((((b + j) & (kFft - 1)) * kFft) + col) * 2;
            const T wr = wp[0], wi = wp[1];
            rr[j] -= dcr * wr - dci * wi;
            ri[j] -= dcr * wi + dci * wr;
            const T e = rr[j] * rr[j] + ri[j] * ri[j];
            if (e > be) { be = e; bjx = j; }
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < kRowsPerWave; ++j) {
          const T e = rr[j] * rr[j] + ri[j] * ri[j];
          if (e > be) { be = e; bjx = j; }
        }
      }
      // wavefront argmax; ties go to the smallest row-major index
      int kk = ((kRowsPerWave * wave + bjx) << 6) | lane;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const T oe = __shfl_xor(be, off);
        const int ok = __shfl_xor(kk, off);
        if (oe > be || (oe == be && ok < kk)) { be = oe; kk = ok; }
      }
      kk = uniform_int(kk);
      const int jw = (kk >> 6) & (kRowsPerWave - 1), lw = kk & (kFft - 1);
      const T sr = read_lane((T)rr[jw], lw);
      const T si = read_lane((T)ri[jw], lw);
      double* sl = slots + (it & 1) * kWaves * 4;
      if (lane == 0) {
        sl[wave * 4 + 0] = (double)be;
        sl[wave * 4 + 1] = (double)kk;
        sl[wave * 4 + 2] = (double)sr;
        sl[wave * 4 + 3] = (double)si;
      }
      __syncthreads();
      double ge = sl[0];
      int gk = (int)sl[1];
      double gr = sl[2], gi = sl[3];
#pragma unroll
      for (int q = 1; q < kWaves; ++q) {
        const double e = sl[q * 4];
        const int k = (int)sl[q * 4 + 1];
        if (e > ge || (e == ge && k < gk)) {
          ge = e; gk = k; gr = sl[q * 4 + 2]; gi = sl[q * 4 + 3];
        }
      }
      u = gk;
      dcr = gs * (T)gr;
      dci = gs * (T)gi;
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
  for (int s = tid; s < nb; s += kThreads) {
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
        acc += (double)hdc[2 * i] * tw[2 * t] - (double)hdc[2 * i + 1] * tw[2 * t + 1];
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
    for (int i = tid; i < K; i += kThreads) {
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

// Working image and state map of one frame from the 8-bit input.
template <typename T>
__global__ void fse_init_kernel(const uint8_t* image, int stride, const uint8_t* lost,
                                int lstride, T* work, uint8_t* state, int H, int W) {
  const int64_t n = (int64_t)H * W;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
    const bool l = lost[(int64_t)y * lstride + x] != 0;
    work[i] = l ? T(0) : (T)image[(int64_t)y * stride + x];
    state[i] = l ? kPending : kKnown;
  }
}

// Blocks holding at least one lost sample.
__global__ void fse_block_flags_kernel(const uint8_t* lost, int lstride, int H, int W, int Bh,
                                       int Bw, int gox, int goy, int wb, int nblocks,
                                       uint8_t* flags) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblocks) return;
  const int bi = b / wb, bj = b - bi * wb;
  const int y0 = bi * Bh - goy, x0 = bj * Bw - gox;
  uint8_t f = 0;
  for (int dy = 0; dy < Bh && !f; ++dy) {
    const int y = y0 + dy;
    if (y < 0 || y >= H) continue;
    for (int dx = 0; dx < Bw; ++dx) {
      const int x = x0 + dx;
      if (x >= 0 && x < W && lost[(int64_t)y * lstride + x]) { f = 1; break; }
    }
  }
  flags[b] = f;
}

// Output: known samples copied, lost samples rounded half-to-even and clamped.
template <typename T>
__global__ void fse_finalize_kernel(const uint8_t* image, int stride, const uint8_t* state,
                                    const T* work, uint8_t* out, int ostride, float* of32,
                                    double* of64, int H, int W) {
  const int64_t n = (int64_t)H * W;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
    const T v = work[i];
    uint8_t o;
    if (state[i] == kKnown) {
      o = image[(int64_t)y * stride + x];
    } else {
      T r = rint(v);
      r = r < T(0) ? T(0) : (r > T(255) ? T(255) : r);
      o = (uint8_t)r;
    }
    out[(int64_t)y * ostride + x] = o;
    if (of32) of32[i] = (float)v;
    if (of64) of64[i] = (double)v;
  }
}

// ---------------------------------------------------------------- launchers

template <typename T>
hipError_t launch_block(const BlockArgs<T>& a, int n_items, size_t lds, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  static size_t attr_bytes = 0;  // largest dynamic LDS size enabled so far
  if (lds > attr_bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)fse_block_kernel<T>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_bytes = lds;
  }
  hipLaunchKernelGGL(fse_block_kernel<T>, dim3(n_items), dim3(kThreads), lds, s, a);
  return hipGetLastError();
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
  if (g > 65536) g = 65536;
  return (int)(g < 1 ? 1 : g);
}

template <typename T>
hipError_t launch_init(const uint8_t* image, int stride, const uint8_t* lost, int lstride,
                       T* work, uint8_t* state, int H, int W, hipStream_t s) {
  hipLaunchKernelGGL(fse_init_kernel<T>, dim3(grid_for((int64_t)H * W)), dim3(256), 0, s, image,
                     stride, lost, lstride, work, state, H, W);
  return hipGetLastError();
}

hipError_t launch_block_flags(const uint8_t* lost, int lstride, int H, int W, int Bh, int Bw,
                              int gox, int goy, int hb, int wb, uint8_t* flags, hipStream_t s) {
  const int nb = hb * wb;
  hipLaunchKernelGGL(fse_block_flags_kernel, dim3((nb + 255) / 256), dim3(256), 0, s, lost,
                     lstride, H, W, Bh, Bw, gox, goy, wb, nb, flags);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_finalize(const uint8_t* image, int stride, const uint8_t* state,
                           const T* work, uint8_t* out, int ostride, float* of32, double* of64,
                           int H, int W, hipStream_t s) {
  hipLaunchKernelGGL(fse_finalize_kernel<T>, dim3(grid_for((int64_t)H * W)), dim3(256), 0, s,
                     image, stride, state, work, out, ostride, of32, of64, H, W);
  return hipGetLastError();
}

template hipError_t launch_block<float>(const BlockArgs<float>&, int, size_t, hipStream_t);
template hipError_t launch_block<double>(const BlockArgs<double>&, int, size_t, hipStream_t);
template hipError_t launch_scatter<float>(float*, uint8_t*, const FrameDesc*, const int32_t*, int,
                                          const float*, int, int, int, int, hipStream_t);
template hipError_t launch_scatter<double>(double*, uint8_t*, const FrameDesc*, const int32_t*,
                                           int, const double*, int, int, int, int, hipStream_t);
template hipError_t launch_init<float>(const uint8_t*, int, const uint8_t*, int, float*, uint8_t*,
                                       int, int, hipStream_t);
template hipError_t launch_init<double>(const uint8_t*, int, const uint8_t*, int, double*,
                                        uint8_t*, int, int, hipStream_t);
template hipError_t launch_finalize<float>(const uint8_t*, int, const uint8_t*, const float*,
                                           uint8_t*, int, float*, double*, int, int, hipStream_t);
template hipError_t launch_finalize<double>(const uint8_t*, int, const uint8_t*, const double*,
                                            uint8_t*, int, float*, double*, int, int,
                                            hipStream_t);

}  // namespace fse
