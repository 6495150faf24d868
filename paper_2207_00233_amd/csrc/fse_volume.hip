// fse_volume.hip -- HIP kernels (gfx950) of three-dimensional Frequency
// Selective Extrapolation for video volumes (the 3-D form the paper's
// conclusion names), FP64.
//
// One workgroup of 512 threads (8 wavefronts, two per SIMD) extrapolates one
// lost block of a wave:
//   A  gather the Mt x M x N area (the block plus dt frames and d samples),
//      classify and weight it (Eq. (2) with the 3-D distance), and place
//      z = x + j s w (x = f w) at the first corner of the 8 x 32 x 32 grid in
//      LDS (rows of 32 at a pitch of 33), so that one complex transform
//      gives both spectra;
//   B  the 3-D DFT of z in place: 32-point FFTs along the rows (one thread per
//      row of a frame, the 32 values in registers, factorized as 8-point DFTs
//      over n1 of z[4 n1 + n2], twiddles e^{-j 2 pi n2 k1 / 32}, 4-point DFTs
//      over n2), the same along the columns (one thread per column), 8-point
//      DFTs along the frames (two lines per thread); then
//      X = (Z[k] + conj Z[-k]) / 2 into registers and
//      W = (Z[k] - conj Z[-k]) / (2 j s) back into LDS;
//   D  K greedy iterations: R[k] -= dc W[k - u] (indices mod 8, 32, 32),
//      u = argmax |R|^2 (ties to the smallest (k1 32 + k2) 32 + k3),
//      dc = gamma R[u] / W0: every thread scans its entries in increasing
//      index order keeping the first largest, a wavefront takes the largest
//      (exact double compare, ties by index), one slot per wavefront, one
//      barrier, every lane reduces the eight slots;
//   E  the model on the block's lost samples, sum_i Re(dc_i phi_{u_i}) with
//      phi_k[t,m,n] = exp(+j 2 pi (4 k1 t + k2 m + k3 n) / 32) (the 8-point
//      frame axis is every fourth point of the 32-point table), into a
//      staging buffer that a second kernel applies after the wave, so every
//      block of a wave reads the volume as it was at the wave's start.
// Thread tid owns the 16 spectrum entries k3 = tid % 32 and (k1, k2) =
// row r + 16 j of the 256 rows (k1 32 + k2), r = tid / 32, j = 0..15: k1 =
// j / 2, k2 = r + 16 (j % 2).
#include <hip/hip_runtime.h>

#include "fse_device.h"
#include "fse_dft.h"
#include "fse_volume.h"

namespace fse {

namespace {

constexpr double kZScale = 128.0;  // balances x and w in z = x + j s w
constexpr int kVWaves = kVThreads / 64;

struct VSlot {  // a wavefront's best entry (32 bytes)
  double e, re, im;
  int k, pad;
};

using dft::cmul_conj;
using dft::dft4;
using dft::dft8;

// 32-point DFT of the line at `p` with element stride `stride` (LDS), in
// registers, written back in natural order; elements with index >= n_in are
// taken as zero (not read).
__device__ __forceinline__ void fft32_line(double2* p, int stride, int n_in, const double2* tw) {
  double2 v[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) v[i] = i < n_in ? p[i * stride] : make_double2(0.0, 0.0);
  // position 4 k1 + n2 <- A[n2][k1] = DFT8 over n1 of v[4 n1 + n2], twiddled
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    double2 t[8];
#pragma unroll
    for (int n1 = 0; n1 < 8; ++n1) t[n1] = v[4 * n1 + n2];
    dft8(t);
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) v[4 * k1 + n2] = (n2 && k1) ? cmul_conj(t[k1], tw[n2 * k1]) : t[k1];
  }
  // position 4 k1 + k2 <- X[k1 + 8 k2] = DFT4 over n2
#pragma unroll
  for (int k1 = 0; k1 < 8; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
#pragma unroll
  for (int k = 0; k < 32; ++k) p[k * stride] = v[4 * (k & 7) + (k >> 3)];
}

// One DPP step of a maximum in double: x = max(x, x moved by CTRL); lanes
// without a source (or outside ROWS) keep their own value.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_fmax(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  const int ylo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false);
  const int yhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false);
  return fmax(x, __hiloint2double(yhi, ylo));
}

template <int CTRL>
__device__ __forceinline__ int dpp_imin(int x) {
  return min(x, __builtin_amdgcn_update_dpp(x, x, CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ double read_lane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

}  // namespace

__global__ __launch_bounds__(kVThreads, 1) void fse_volume_block_kernel(Vol3Args a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const Vol3Lds L = vol3_lds(a.K);
  double2* Z = reinterpret_cast<double2*>(smem);  // [t][m][n] / [k1][k2][k3], pitch kVPitch
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
  for (int i = tid; i < kVt * kVFrame; i += kVThreads) Z[i] = make_double2(0.0, 0.0);
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
    Z[t * kVFrame + m * kVPitch + n] = make_double2(f * wv, kZScale * wv);
  }
  for (int off = 32; off >= 1; off >>= 1) wsum += __shfl_xor(wsum, off);
  if (lane == 0) red[wave] = wsum;
  __syncthreads();
  double W0 = 0.0;
#pragma unroll
  for (int q = 0; q < kVWaves; ++q) W0 += red[q];

  const int k3 = tid & 31, r = tid >> 5;
  if (W0 > 0.0) {
    // ---- B: 3-D DFT in place ----
    if (tid < kVt * kVh) {  // rows: thread (t, m), 32-point DFT along n
      const int t = tid >> 5, m = tid & 31;
      if (t < Mt && m < M) fft32_line(Z + t * kVFrame + m * kVPitch, 1, N, tw);
    }
    __syncthreads();
    if (tid < kVt * kVw) {  // columns: thread (t, n), 32-point DFT along m
      const int t = tid >> 5, n = tid & 31;
      if (t < Mt) fft32_line(Z + t * kVFrame + n, kVPitch, M, tw);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (kVh * kVw) / kVThreads; ++q) {  // frames: lines (m, n)
      const int line = tid + kVThreads * q;
      double2* p = Z + (line >> 5) * kVPitch + (line & 31);
      double2 v[8];
#pragma unroll
      for (int t = 0; t < kVt; ++t) v[t] = t < Mt ? p[t * kVFrame] : make_double2(0.0, 0.0);
      dft8(v);
#pragma unroll
      for (int t = 0; t < kVt; ++t) p[t * kVFrame] = v[t];
    }
    __syncthreads();
  }

  // unpack: X into registers, W back into LDS
  double rr[kVEnt], ri[kVEnt];
  if (W0 > 0.0) {
    double wr[kVEnt], wi[kVEnt];
    const double h = 0.5, hs = 0.5 / kZScale;
#pragma unroll
    for (int j = 0; j < kVEnt; ++j) {
      const int k1 = j >> 1, k2 = r + 16 * (j & 1);
      const double2 zk = Z[k1 * kVFrame + k2 * kVPitch + k3];
      const double2 zn =
          Z[((kVt - k1) & 7) * kVFrame + ((kVh - k2) & 31) * kVPitch + ((kVw - k3) & 31)];
      rr[j] = h * (zk.x + zn.x);
      ri[j] = h * (zk.y - zn.y);
      wr[j] = hs * (zk.y + zn.y);
      wi[j] = hs * (zn.x - zk.x);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kVEnt; ++j)
      Z[(j >> 1) * kVFrame + (r + 16 * (j & 1)) * kVPitch + k3] = make_double2(wr[j], wi[j]);
    __syncthreads();

    // ---- D: K greedy iterations ----
    const double gs = a.gamma / W0;
    const int kbase = r * 32 + k3;  // index of entry j: kbase + 512 j
    int u = 0;
    double dcr = 0.0, dci = 0.0;
    for (int it = 0; it < K; ++it) {
      const int u1 = u >> 10, u2 = (u >> 5) & 31, u3 = u & 31;
      const int c3 = (k3 - u3) & 31;
      const int a0 = ((r - u2) & 31) * kVPitch + c3, a1 = ((r + 16 - u2) & 31) * kVPitch + c3;
      double e[kVEnt];
#pragma unroll
      for (int j = 0; j < kVEnt; ++j) {
        const int k1 = j >> 1;
        const double2 w = Z[((k1 - u1) & 7) * kVFrame + ((j & 1) ? a1 : a0)];
        double x = rr[j], y = ri[j];
        x = fma(-dcr, w.x, fma(dci, w.y, x));
        y = fma(-dcr, w.y, fma(-dci, w.x, y));
        rr[j] = x;
        ri[j] = y;
        e[j] = fma(x, x, y * y);
      }
      double t8[kVEnt / 2];  // the thread's largest |R|^2 as a tree of maxima
#pragma unroll
      for (int j = 0; j < kVEnt / 2; ++j) t8[j] = fmax(e[2 * j], e[2 * j + 1]);
#pragma unroll
      for (int w = kVEnt / 4; w >= 1; w >>= 1)
#pragma unroll
        for (int j = 0; j < w; ++j) t8[j] = fmax(t8[2 * j], t8[2 * j + 1]);
      const double be = t8[0];
      // wavefront: the largest |R|^2; the entry holding it is the lowest
      // entry index j, then the lowest lane, among those equal to it (for
      // equal values the smallest index (k1 32 + k2) 32 + k3 = kbase + 512 j)
      // quads, rows of 16, then rows 1 and 3 (row_bcast:15), row 3
      // (row_bcast:31): lane 63 holds the wavefront's maximum
      double gm = dpp_fmax<0xB1>(be);  // quad_perm [1,0,3,2]
      gm = dpp_fmax<0x4E>(gm);         // quad_perm [2,3,0,1]
      gm = dpp_fmax<0x124>(gm);        // row_ror:4
      gm = dpp_fmax<0x128>(gm);        // row_ror:8
      gm = dpp_fmax<0x142, 0xA>(gm);   // row_bcast:15
      gm = dpp_fmax<0x143, 0xC>(gm);   // row_bcast:31
      gm = read_lane_d(gm, 63);
      int jw = kVEnt, lw = 0;
#pragma unroll
      for (int j = kVEnt - 1; j >= 0; --j) {  // lowest j wins
        const unsigned long long m = __ballot(e[j] == gm);
        if (m) {
          jw = j;
          lw = __builtin_ctzll(m);
        }
      }
      jw = __builtin_amdgcn_readfirstlane(jw);
      lw = __builtin_amdgcn_readfirstlane(lw);
      const double sx = rr[jw], sy = ri[jw];  // uniform register index
      VSlot* sl = slots + (it & 1) * kVWaves;
      if (lane == lw) {
        VSlot v;
        v.e = be;
        v.re = sx;
        v.im = sy;
        v.k = kbase + 512 * jw;
        v.pad = 0;
        sl[wave] = v;
      }
      __syncthreads();
      // block: lane l reads slot l % 8 (the data repeat with period 8, so
      // quad and row-of-8 DPP steps reduce all eight): the largest |R|^2, then
      // the smallest index among the slots holding it
      const VSlot mine = sl[lane & 7];
      double ge = dpp_fmax<0xB1>(mine.e);  // quad_perm [1,0,3,2]
      ge = dpp_fmax<0x4E>(ge);             // quad_perm [2,3,0,1]
      ge = dpp_fmax<0x124>(ge);            // row_ror:4
      int gk = mine.e == ge ? (mine.k << 3) | (lane & 7) : 0x7fffffff;
      gk = dpp_imin<0xB1>(gk);
      gk = dpp_imin<0x4E>(gk);
      gk = dpp_imin<0x124>(gk);
      gk = __builtin_amdgcn_readfirstlane(gk);
      u = gk >> 3;
      const VSlot& win = sl[gk & 7];
      dcr = gs * win.re;
      dci = gs * win.im;
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
