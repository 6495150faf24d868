// fse_peaks.hip -- microbenchmarks of the device's vector FMA rate (float and
// double), LDS read bandwidth and HBM copy bandwidth, timed with HIP events,
// for the measured roofline peaks.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fse.h"
#include "fse_peaks.h"

namespace {

constexpr int kThreads = 256;
constexpr int kChains = 16;  // independent FMA chains per thread

// x <- x a + b on kChains independent values per thread; the result is stored
// only if it takes an impossible value, so the work cannot be dropped.
template <typename T>
__global__ __launch_bounds__(kThreads) void peak_fma_kernel(T* out, int iters, T a, T b) {
  T x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = (T)(threadIdx.x + c);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = fma(x[c], a, b);
  }
  T s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  if (s == (T)-1) out[blockIdx.x] = s;
}

// Eight 16-byte LDS reads per thread and step; a wavefront's 64 lanes read
// 1 KB of consecutive bytes (no bank conflicts), the window moves each step.
__global__ __launch_bounds__(kThreads) void peak_lds_kernel(float* out, int iters) {
  __shared__ float4 buf[4096];  // 64 KB
  for (int i = threadIdx.x; i < 4096; i += kThreads)
    buf[i] = make_float4((float)i, (float)(i + 1), (float)(i + 2), (float)(i + 3));
  __syncthreads();
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int i = 0; i < iters; ++i) {
    const int base = (threadIdx.x + 64 * i) & 2047;  // + 256 j stays below 4096
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float4 v = buf[base + kThreads * j];
      acc.x += v.x;
      acc.y += v.y;
      acc.z += v.z;
      acc.w += v.w;
    }
  }
  if (acc.x + acc.y + acc.z + acc.w == -1.f) out[blockIdx.x] = acc.x;
}

template <typename F>
int best_ms(F launch, int reps, float* best) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return FSE_ERR_DEVICE;
  *best = 1e30f;
  int rc = FSE_OK;
  for (int r = 0; r < reps && rc == FSE_OK; ++r) {
    float ms = 0.f;
    if (hipEventRecord(e0, nullptr) != hipSuccess || launch() != hipSuccess ||
        hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      rc = FSE_ERR_DEVICE;
    else if (r > 0)  // the first run warms up
      *best = std::min(*best, ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // namespace

extern "C" int32_t fse_measure_peaks(fse_peaks* out) {
  if (!out) return FSE_ERR_INVALID;
  *out = fse_peaks{};
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return FSE_ERR_DEVICE;
  const int ncu = prop.multiProcessorCount;
  out->compute_units = ncu;
  const int grid = ncu * 16;  // 16 workgroups of 4 wavefronts per CU
  void* sink = nullptr;
  if (hipMalloc(&sink, (size_t)grid * sizeof(double)) != hipSuccess) return FSE_ERR_DEVICE;
  int rc = FSE_OK;
  float ms = 0.f;
  {
    const int iters = 4096;
    rc = best_ms([&] {
      hipLaunchKernelGGL(peak_fma_kernel<float>, dim3(grid), dim3(kThreads), 0, nullptr,
                         (float*)sink, iters, 0.9999999f, 1e-7f);
      return hipGetLastError();
    }, 4, &ms);
    if (rc == FSE_OK)
      out->fp32_fma_tflops = 2.0 * grid * kThreads * (double)iters * kChains / (ms * 1e-3) / 1e12;
  }
  if (rc == FSE_OK) {
    const int iters = 4096;
    rc = best_ms([&] {
      hipLaunchKernelGGL(peak_fma_kernel<double>, dim3(grid), dim3(kThreads), 0, nullptr,
                         (double*)sink, iters, 0.9999999, 1e-7);
      return hipGetLastError();
    }, 4, &ms);
    if (rc == FSE_OK)
      out->fp64_fma_tflops = 2.0 * grid * kThreads * (double)iters * kChains / (ms * 1e-3) / 1e12;
  }
  if (rc == FSE_OK) {
    const int iters = 2048, lds_grid = ncu * 8;
    rc = best_ms([&] {
      hipLaunchKernelGGL(peak_lds_kernel, dim3(lds_grid), dim3(kThreads), 0, nullptr,
                         (float*)sink, iters);
      return hipGetLastError();
    }, 4, &ms);
    if (rc == FSE_OK)
      out->lds_read_tbps = 16.0 * 8 * lds_grid * kThreads * (double)iters / (ms * 1e-3) / 1e12;
  }
  (void)hipFree(sink);
  if (rc != FSE_OK) return rc;
  const size_t bytes = (size_t)1 << 30;
  void *src = nullptr, *dst = nullptr;
  if (hipMalloc(&src, bytes) != hipSuccess || hipMalloc(&dst, bytes) != hipSuccess) {
    if (src) (void)hipFree(src);
    (void)hipGetLastError();
    return FSE_ERR_NOMEM;
  }
  if (hipMemset(src, 1, bytes) != hipSuccess) rc = FSE_ERR_DEVICE;
  if (rc == FSE_OK) {
    rc = best_ms([&] { return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, nullptr); },
                 4, &ms);
    if (rc == FSE_OK) out->hbm_copy_tbps = 2.0 * (double)bytes / (ms * 1e-3) / 1e12;
  }
  (void)hipFree(src);
  (void)hipFree(dst);
  return rc;
}
