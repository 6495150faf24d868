// fse_volume.hip -- HIP kernels (gfx950) of three-dimensional Frequency
// Selective Extrapolation for video volumes (the 3-D form the paper's
// conclusion names), FP64.
//
// One workgroup of 256 threads extrapolates one lost block of a wave:
//   A  gather the Mt x M x N area (the block plus dt frames and d samples),
//      classify and weight it (Eq. (2) with the 3-D distance), and place
//      z = x + j s w (x = f w) at the first corner of the 8 x 32 x 32 grid in
//      LDS, so that one complex transform gives both spectra;
//   B  the 3-D DFT of z in place: along the columns (one thread per row of a
//      frame), along the rows (one thread per column of a frame), along the
//      frames (four lines of 8 per thread); then X = (Z[k] + conj Z[-k]) / 2
//      into registers and W = (Z[k] - conj Z[-k]) / (2 j s) back into LDS;
//   D  K greedy iterations: R[k] -= dc W[k - u] (indices mod 8, 32, 32),
//      u = argmax |R|^2 (ties to the smallest (k1 32 + k2) 32 + k3),
//      dc = gamma R[u] / W0;
//   E  the model on the block's lost samples, sum_i Re(dc_i phi_{u_i}) with
//      phi_k[t,m,n] = exp(+j 2 pi (4 k1 t + k2 m + k3 n) / 32) (the 8-point
//      frame axis is every fourth point of the 32-point table), into a
//      staging buffer that a second kernel applies after the wave, so every
//      block of a wave reads the volume as it was at the wave's start.
// Thread tid owns the 32 spectrum entries k3 = tid % 32, k2 = tid / 32 + 8q
// (q = 0..3), k1 = 0..7.
#include <hip/hip_runtime.h>

#include "fse_device.h"
#include "fse_volume.h"

namespace fse {

namespace {

constexpr double kZScale = 128.0;  // balances x and w in z = x + j s w

struct VSlot {  // a wavefront's best entry (32 bytes)
  double e, re, im;
  int k, pad;
};

__device__ __forceinline__ double2 cmul_conj(double2 v, double2 t) {
  // v * conj(t) with t = (cos, sin): the forward-transform kernel e^{-j a}
  return make_double2(fma(v.x, t.x, v.y * t.y), fma(v.y, t.x, -v.x * t.y));
}

}  // namespace

__global__ __launch_bounds__(kVThreads, 1) void fse_volume_block_kernel(Vol3Args a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const Vol3Lds L = vol3_lds(a.K);
  double2* Z = reinterpret_cast<double2*>(smem);  // [k1][k2][k3] (or [t][m][n])
  int* hu = reinterpret_cast<int*>(smem + L.hist_u);
  double2* hdc = reinterpret_cast<double2*>(smem + L.hist_dc);
  double2* tw = reinterpret_cast<double2*>(smem + L.tw);
  VSlot* slots = reinterpret_cast<VSlot*>(smem + L.slots);
  double* red = reinterpret_cast<double*>(smem + L.red);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int item = blockIdx.x;
  const int bt = a.items[3 * item], bi = a.items[3 * item + 1], bj = a.items[3 * item + 2];
  const int z0 = bt * a.Bt - a.dt, y0 = bi * a.Bh - a.d, x0 = bj * a.Bw - a.d;
  const int Mt = a.Mt, M = a.M, N = a.N, K = a.K;

  if (tid < 32) tw[tid] = make_double2(a.twid[2 * tid], a.twid[2 * tid + 1]);
  for (int i = tid; i < kV3; i += kVThreads) Z[i] = make_double2(0.0, 0.0);
  __syncthreads();

  // ---- A: gather, classify, weight ----
  double wsum = 0.0;
  const int area = Mt * M * N;
  for (int i = tid; i < area; i += kVThreads) {
    const int n = i % N, m = (i / N) % M, t = i / (M * N);
    const int z = z0 + t, y = y0 + m, x = x0 + n;
    double wv = 0.0, f = 0.0;
    if (z >= 0 && z < a.T && y >= 0 && y < a.H && x >= 0 && x < a.W) {
      const int64_t p = ((int64_t)z * a.H + y) * a.W + x;
      const uint8_t s = a.state[p];
      const double fac = s == kKnown ? 1.0 : (s == kRecon ? a.delta : 0.0);
      wv = a.radial[i] * fac;
      f = a.work[p];
    }
    wsum += wv;
    Z[(t * kVh + m) * kVw + n] = make_double2(f * wv, kZScale * wv);
  }
  for (int off = 32; off >= 1; off >>= 1) wsum += __shfl_xor(wsum, off);
  if (lane == 0) red[wave] = wsum;
  __syncthreads();
  double W0 = 0.0;
#pragma unroll
  for (int q = 0; q < kVThreads / 64; ++q) W0 += red[q];

  const int g = tid >> 5, k3 = tid & 31;
  if (W0 > 0.0) {
    // ---- B: 3-D DFT in place ----
    {  // columns n -> k3, one thread per row (t, m) = (g, k3)
      const int t = g, m = k3;
      if (t < Mt && m < M) {
        double2 v[kVw];  // the row is in registers: results go straight back
        double2* row = Z + (t * kVh + m) * kVw;
#pragma unroll
        for (int n = 0; n < kVw; ++n) v[n] = row[n];
        for (int k = 0; k < kVw; ++k) {
          double2 acc = make_double2(0.0, 0.0);
#pragma unroll
          for (int n = 0; n < kVw; ++n) {
            const double2 c = cmul_conj(v[n], tw[(k * n) & 31]);
            acc.x += c.x;
            acc.y += c.y;
          }
          row[k] = acc;
        }
      }
    }
    __syncthreads();
    {  // rows m -> k2, one thread per column (t, n) = (g, k3)
      const int t = g, n = k3;
      if (t < Mt) {
        double2 v[kVh];
#pragma unroll
        for (int m = 0; m < kVh; ++m) v[m] = Z[(t * kVh + m) * kVw + n];
        for (int k = 0; k < kVh; ++k) {
          double2 acc = make_double2(0.0, 0.0);
#pragma unroll
          for (int m = 0; m < kVh; ++m) {
            const double2 c = cmul_conj(v[m], tw[(k * m) & 31]);
            acc.x += c.x;
            acc.y += c.y;
          }
          Z[(t * kVh + k) * kVw + n] = acc;
        }
      }
    }
    __syncthreads();
    // frames t -> k1: lines (k2, k3), four per thread (frames >= Mt are 0)
    for (int q = 0; q < 4; ++q) {
      const int line = tid + kVThreads * q;
      double2 v[kVt], o[kVt];
#pragma unroll
      for (int t = 0; t < kVt; ++t) v[t] = Z[t * kVh * kVw + line];
#pragma unroll
      for (int k = 0; k < kVt; ++k) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int t = 0; t < kVt; ++t) {
          const double2 c = cmul_conj(v[t], tw[(4 * k * t) & 31]);
          acc.x += c.x;
          acc.y += c.y;
        }
        o[k] = acc;
      }
#pragma unroll
      for (int k = 0; k < kVt; ++k) Z[k * kVh * kVw + line] = o[k];
    }
    __syncthreads();
  }

  // unpack: X into registers, W back into LDS
  double rr[kVt][4], ri[kVt][4];
  if (W0 > 0.0) {
    double wr[kVt][4], wi[kVt][4];
    const double h = 0.5, hs = 0.5 / kZScale;
#pragma unroll
    for (int k1 = 0; k1 < kVt; ++k1)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k2 = g + 8 * q;
        const double2 zk = Z[(k1 * kVh + k2) * kVw + k3];
        const double2 zn = Z[((((kVt - k1) & 7) * kVh) + ((kVh - k2) & 31)) * kVw + ((kVw - k3) & 31)];
        rr[k1][q] = h * (zk.x + zn.x);
        ri[k1][q] = h * (zk.y - zn.y);
        wr[k1][q] = hs * (zk.y + zn.y);
        wi[k1][q] = hs * (zn.x - zk.x);
      }
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < kVt; ++k1)
#pragma unroll
      for (int q = 0; q < 4; ++q) Z[(k1 * kVh + g + 8 * q) * kVw + k3] = make_double2(wr[k1][q], wi[k1][q]);
    __syncthreads();

    // ---- D: K greedy iterations ----
    const double gs = a.gamma / W0;
    int u = 0;
    double dcr = 0.0, dci = 0.0;
    for (int it = 0; it < K; ++it) {
      const int u1 = u >> 10, u2 = (u >> 5) & 31, u3 = u & 31;
      const int c3 = (k3 - u3) & 31;
      double be = -1.0, bre = 0.0, bim = 0.0;
      int bk = 0;
#pragma unroll
      for (int k1 = 0; k1 < kVt; ++k1) {
        const int p1 = ((k1 - u1) & 7) * (kVh * kVw);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int k2 = g + 8 * q;
          const double2 w = Z[p1 + ((k2 - u2) & 31) * kVw + c3];
          double r = rr[k1][q], s = ri[k1][q];
          r = fma(-dcr, w.x, fma(dci, w.y, r));
          s = fma(-dcr, w.y, fma(-dci, w.x, s));
          rr[k1][q] = r;
          ri[k1][q] = s;
          const double e = fma(r, r, s * s);
          if (e > be) {  // entries in increasing index order: the first maximum stays
            be = e;
            bre = r;
            bim = s;
            bk = (k1 * kVh + k2) * kVw + k3;
          }
        }
      }
      // wavefront: the largest |R|^2, ties to the smallest index
      for (int off = 32; off >= 1; off >>= 1) {
        const double oe = __shfl_xor(be, off), ore = __shfl_xor(bre, off),
                     oim = __shfl_xor(bim, off);
        const int ok = __shfl_xor(bk, off);
        if (oe > be || (oe == be && ok < bk)) {
          be = oe;
          bre = ore;
          bim = oim;
          bk = ok;
        }
      }
      VSlot* sl = slots + (it & 1) * (kVThreads / 64);
      if (lane == 0) {
        VSlot v;
        v.e = be;
        v.re = bre;
        v.im = bim;
        v.k = bk;
        v.pad = 0;
        sl[wave] = v;
      }
      __syncthreads();
      VSlot best = sl[0];
#pragma unroll
      for (int q = 1; q < kVThreads / 64; ++q) {
        const VSlot c = sl[q];
        if (c.e > best.e || (c.e == best.e && c.k < best.k)) best = c;
      }
      u = __builtin_amdgcn_readfirstlane(best.k);
      dcr = gs * best.re;
      dci = gs * best.im;
      if (tid == 0) {
        hu[it] = u;
        hdc[it] = make_double2(dcr, dci);
      }
    }
    __syncthreads();
  }

  // ---- E: the model on the block's lost samples ----
  const int blk = a.Bt * a.Bh * a.Bw;
  for (int s = tid; s < blk; s += kVThreads) {
    const int dz = s / (a.Bh * a.Bw), dy = (s / a.Bw) % a.Bh, dx = s % a.Bw;
    double acc;
    if (!(W0 > 0.0)) {
      acc = a.empty_fill;
    } else {
      const int t = a.dt + dz, m = a.d + dy, n = a.d + dx;
      acc = 0.0;
      for (int i = 0; i < K; ++i) {
        const int uu = hu[i];
        const int ix = (4 * (uu >> 10) * t + ((uu >> 5) & 31) * m + (uu & 31) * n) & 31;
        const double2 c = tw[ix], dc = hdc[i];
        acc = fma(dc.x, c.x, acc);
        acc = fma(-dc.y, c.y, acc);
      }
    }
    a.staging[(int64_t)item * blk + s] = acc;
  }
}

// The staged model samples of the items of a wave become reconstructed
// samples (lost samples inside the volume only).
__global__ void fse_volume_scatter_kernel(Vol3Args a) {
  const int item = blockIdx.x;
  const int bt = a.items[3 * item], bi = a.items[3 * item + 1], bj = a.items[3 * item + 2];
  const int blk = a.Bt * a.Bh * a.Bw;
  for (int s = threadIdx.x; s < blk; s += blockDim.x) {
    const int dz = s / (a.Bh * a.Bw), dy = (s / a.Bw) % a.Bh, dx = s % a.Bw;
    const int z = bt * a.Bt + dz, y = bi * a.Bh + dy, x = bj * a.Bw + dx;
    if (z >= a.T || y >= a.H || x >= a.W) continue;
    const int64_t p = ((int64_t)z * a.H + y) * a.W + x;
    if (a.state[p] != kPending) continue;
    a.work[p] = a.staging[(int64_t)item * blk + s];
    a.state[p] = kRecon;
  }
}

// Working volume and state map from the 8-bit input (lost samples 0 / pending).
__global__ void fse_volume_init_kernel(const uint8_t* vol, const uint8_t* lost, double* work,
                                       uint8_t* state, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const bool l = lost[i] != 0;
    work[i] = l ? 0.0 : (double)vol[i];
    state[i] = l ? kPending : kKnown;
  }
}

// 8-bit output: lost samples rounded half to even and clamped, known copied.
__global__ void fse_volume_finalize_kernel(const uint8_t* vol, const uint8_t* state,
                                           const double* work, uint8_t* out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (state[i] == kKnown) {
      out[i] = vol[i];
    } else {
      const double v = rint(work[i]);
      out[i] = (uint8_t)(v < 0.0 ? 0.0 : (v > 255.0 ? 255.0 : v));
    }
  }
}

hipError_t launch_volume_block(const Vol3Args& a, int n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  static size_t attr = 0;
  const size_t lds = (size_t)vol3_lds(a.K).total;
  if (lds > attr) {
    hipError_t e = hipFuncSetAttribute((const void*)fse_volume_block_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = lds;
  }
  hipLaunchKernelGGL(fse_volume_block_kernel, dim3(n_items), dim3(kVThreads), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_volume_scatter(const Vol3Args& a, int n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(fse_volume_scatter_kernel, dim3(n_items), dim3(256), 0, s, a);
  return hipGetLastError();
}

static int grid_for(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

hipError_t launch_volume_init(const uint8_t* vol, const uint8_t* lost, double* work,
                              uint8_t* state, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fse_volume_init_kernel, dim3(grid_for(n)), dim3(256), 0, s, vol, lost, work,
                     state, n);
  return hipGetLastError();
}

hipError_t launch_volume_finalize(const uint8_t* vol, const uint8_t* state, const double* work,
                                  uint8_t* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fse_volume_finalize_kernel, dim3(grid_for(n)), dim3(256), 0, s, vol, state,
                     work, out, n);
  return hipGetLastError();
}

}  // namespace fse
