// fse_volume.cpp -- host runtime of three-dimensional FSE (fse_plan3,
// fse_conceal_volume, fse_schedule3): tables, device buffers, the
// 26-neighbourhood processing order and one launch (plus the staging
// scatter) per wave.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "fse.h"
#include "fse_device.h"
#include "fse_internal.h"
#include "fse_sched.h"
#include "fse_volume.h"

namespace fse {
hipError_t launch_volume_block(const Vol3Args& a, int n_items, hipStream_t s);
hipError_t launch_volume_scatter(const Vol3Args& a, int n_items, hipStream_t s);
hipError_t launch_volume_init(const uint8_t* vol, const uint8_t* lost, double* work,
                              uint8_t* state, int64_t n, hipStream_t s);
hipError_t launch_volume_finalize(const uint8_t* vol, const uint8_t* state, const double* work,
                                  uint8_t* out, int64_t n, hipStream_t s);
}  // namespace fse

using namespace fse;

struct fse_plan3_s {
  fse_params3 p;
  int Mt = 0, M = 0, N = 0, device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  DevBuf radial, twid, vol, lost, work, state, out, items, staging;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // device time of a call
  std::mutex mu;  // one call at a time
  int sticky = FSE_OK;
};

namespace {

int validate3(const fse_params3* p) {
  if (!p) return FSE_ERR_INVALID;
  if (p->block_t < 1 || p->block_h < 1 || p->block_w < 1 || p->border_t < 0 || p->border_d < 0)
    return FSE_ERR_INVALID;
  if (!(p->rho > 0.0 && p->rho <= 1.0) || !(p->delta >= 0.0 && p->delta <= 1.0) ||
      !(p->gamma > 0.0 && p->gamma <= 1.0) || !std::isfinite(p->empty_fill))
    return FSE_ERR_INVALID;
  if (p->iterations < 1 || p->iterations > FSE_MAX_ITERATIONS) return FSE_ERR_INVALID;
  if (p->order != FSE_ORDER_OPTIMIZED && p->order != FSE_ORDER_LINESCAN) return FSE_ERR_INVALID;
  if (p->fft_t < 1 || p->fft_h < 1 || p->fft_w < 1) return FSE_ERR_INVALID;
  if (p->block_t + 2 * p->border_t > p->fft_t || p->block_h + 2 * p->border_d > p->fft_h ||
      p->block_w + 2 * p->border_d > p->fft_w)
    return FSE_ERR_INVALID;
  if (p->fft_t != kVt || p->fft_h != kVh || p->fft_w != kVw) return FSE_ERR_UNSUPPORTED;
  if (p->precision != FSE_FP64) return FSE_ERR_UNSUPPORTED;
  return FSE_OK;
}

}  // namespace

extern "C" {

int32_t fse_plan3(const fse_params3* p, void* hip_stream, fse_plan3_t* out) {
  if (!out) return FSE_ERR_INVALID;
  *out = nullptr;
  int rc = validate3(p);
  if (rc) return rc;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return FSE_ERR_DEVICE;
  if (vol3_lds(p->iterations).total > (int64_t)prop.sharedMemPerBlock) return FSE_ERR_UNSUPPORTED;
  fse_plan3_s* pl = new fse_plan3_s();
  pl->p = *p;
  pl->Mt = p->block_t + 2 * p->border_t;
  pl->M = p->block_h + 2 * p->border_d;
  pl->N = p->block_w + 2 * p->border_d;
  pl->device = dev;
  if (hip_stream) {
    pl->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&pl->stream, hipStreamNonBlocking) != hipSuccess) {
      delete pl;
      return FSE_ERR_DEVICE;
    }
    pl->own_stream = true;
  }
  // rho^dist with the 3-D distance from the area's centre (Eq. (2))
  std::vector<double> radial((size_t)pl->Mt * pl->M * pl->N);
  for (int t = 0; t < pl->Mt; ++t)
    for (int m = 0; m < pl->M; ++m)
      for (int n = 0; n < pl->N; ++n) {
        const double dt = t - 0.5 * (pl->Mt - 1), dm = m - 0.5 * (pl->M - 1),
                     dn = n - 0.5 * (pl->N - 1);
        radial[((size_t)t * pl->M + m) * pl->N + n] =
            std::pow(p->rho, std::sqrt(dt * dt + dm * dm + dn * dn));
      }
  // (cos, sin)(2 pi t / 32), exactly symmetric, zeros at the quarter points
  const double two_pi = 6.283185307179586476925286766559;
  std::vector<double> tw(2 * 32);
  for (int t = 0; t <= 16; ++t) {
    tw[2 * t] = std::cos(two_pi * t / 32.0);
    tw[2 * t + 1] = std::sin(two_pi * t / 32.0);
  }
  for (int t = 17; t < 32; ++t) {
    tw[2 * t] = tw[2 * (32 - t)];
    tw[2 * t + 1] = -tw[2 * (32 - t) + 1];
  }
  tw[2 * 8] = tw[2 * 24] = 0.0;
  tw[2 * 16 + 1] = 0.0;
  if (pl->radial.reserve(radial.size() * sizeof(double)) || pl->twid.reserve(tw.size() * 8) ||
      hipMemcpy(pl->radial.ptr, radial.data(), radial.size() * sizeof(double),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(pl->twid.ptr, tw.data(), tw.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
    fse_plan3_destroy(pl);
    return FSE_ERR_DEVICE;
  }
  if (hipEventCreate(&pl->ev0) != hipSuccess || hipEventCreate(&pl->ev1) != hipSuccess) {
    fse_plan3_destroy(pl);
    return FSE_ERR_DEVICE;
  }
  *out = pl;
  return FSE_OK;
}

int32_t fse_plan3_destroy(fse_plan3_t pl) {
  if (!pl) return FSE_OK;
  (void)hipSetDevice(pl->device);
  if (pl->stream) (void)hipStreamSynchronize(pl->stream);
  for (DevBuf* b : {&pl->radial, &pl->twid, &pl->vol, &pl->lost, &pl->work, &pl->state, &pl->out,
                    &pl->items, &pl->staging})
    b->release();
  if (pl->ev0) (void)hipEventDestroy(pl->ev0);
  if (pl->ev1) (void)hipEventDestroy(pl->ev1);
  if (pl->own_stream && pl->stream) (void)hipStreamDestroy(pl->stream);
  delete pl;
  return FSE_OK;
}

int32_t fse_conceal_volume(fse_plan3_t pl, const fse_volume* v) {
  if (!pl || !v || !v->volume || !v->lost || !v->out) return FSE_ERR_INVALID;
  if (v->frames < 1 || v->height < 1 || v->width < 1 || v->frames > 65535 ||
      v->height > 65535 || v->width > 65535)
    return FSE_ERR_INVALID;
  std::lock_guard<std::mutex> lk(pl->mu);
  if (pl->sticky) return pl->sticky;
  if (hipSetDevice(pl->device) != hipSuccess) return FSE_ERR_DEVICE;
  const fse_params3& p = pl->p;
  const int T = v->frames, H = v->height, W = v->width;
  const int64_t n = (int64_t)T * H * W;
  const int tb = (T + p.block_t - 1) / p.block_t, hb = (H + p.block_h - 1) / p.block_h,
            wb = (W + p.block_w - 1) / p.block_w;
  const int64_t nb = (int64_t)tb * hb * wb;
  if (nb > (1LL << 31) / 4) return FSE_ERR_INVALID;
  hipStream_t s = pl->stream;
  auto fail = [&](int rc) {
    if (rc == FSE_ERR_DEVICE) pl->sticky = rc;
    return rc;
  };
  // lost blocks and the processing order on the host
  std::vector<uint8_t> blost((size_t)nb, 0);
  for (int z = 0; z < T; ++z)
    for (int y = 0; y < H; ++y) {
      const uint8_t* row = v->lost + ((int64_t)z * H + y) * W;
      const int64_t base = ((int64_t)(z / p.block_t) * hb + y / p.block_h) * wb;
      for (int x = 0; x < W; ++x)
        if (row[x]) blost[base + x / p.block_w] = 1;
    }
  std::vector<int32_t> wave_of((size_t)nb), seq;
  const int nwaves = schedule_blocks3(tb, hb, wb, blost.data(), p.order, wave_of.data(), &seq);
  const int64_t n_items = (int64_t)seq.size();
  std::vector<int32_t> items((size_t)std::max<int64_t>(1, n_items) * 3);
  std::vector<int64_t> wave_start((size_t)nwaves + 1, 0);
  int best = 0;
  for (int64_t i = 0, w = 0; i < n_items; ++i) {
    const int32_t b = seq[i];
    items[3 * i] = b / (hb * wb);
    items[3 * i + 1] = (b / wb) % hb;
    items[3 * i + 2] = b % wb;
    while (w < wave_of[b]) wave_start[++w] = i;
  }
  wave_start[nwaves] = n_items;  // every wave holds at least one block
  for (int w = 0; w < nwaves; ++w)
    best = std::max<int>(best, (int)(wave_start[w + 1] - wave_start[w]));
  const int blk = p.block_t * p.block_h * p.block_w;
  if (pl->vol.reserve(n) || pl->lost.reserve(n) || pl->work.reserve(n * sizeof(double)) ||
      pl->state.reserve(n) || pl->out.reserve(n) ||
      pl->items.reserve(items.size() * sizeof(int32_t)) ||
      pl->staging.reserve((size_t)std::max(1, best) * blk * sizeof(double))) {
    (void)hipGetLastError();  // an allocation that failed leaves the plan usable
    return FSE_ERR_NOMEM;
  }
  if (hipMemcpyAsync(pl->vol.ptr, v->volume, n, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(pl->lost.ptr, v->lost, n, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(pl->items.ptr, items.data(), items.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      launch_volume_init((const uint8_t*)pl->vol.ptr, (const uint8_t*)pl->lost.ptr,
                         (double*)pl->work.ptr, (uint8_t*)pl->state.ptr, n, s) != hipSuccess)
    return fail(FSE_ERR_DEVICE);
  Vol3Args a{};
  a.work = (double*)pl->work.ptr;
  a.state = (uint8_t*)pl->state.ptr;
  a.staging = (double*)pl->staging.ptr;
  a.radial = (const double*)pl->radial.ptr;
  a.twid = (const double*)pl->twid.ptr;
  a.T = T;
  a.H = H;
  a.W = W;
  a.Bt = p.block_t;
  a.Bh = p.block_h;
  a.Bw = p.block_w;
  a.dt = p.border_t;
  a.d = p.border_d;
  a.Mt = pl->Mt;
  a.M = pl->M;
  a.N = pl->N;
  a.K = p.iterations;
  a.delta = p.delta;
  a.gamma = p.gamma;
  a.empty_fill = p.empty_fill;
  if (hipEventRecord(pl->ev0, s) != hipSuccess) return fail(FSE_ERR_DEVICE);
  for (int w = 0; w < nwaves; ++w) {
    const int64_t i0 = wave_start[w], cnt = wave_start[w + 1] - i0;
    if (cnt <= 0) continue;
    a.items = (const int32_t*)pl->items.ptr + 3 * i0;
    if (launch_volume_block(a, (int)cnt, s) != hipSuccess ||
        launch_volume_scatter(a, (int)cnt, s) != hipSuccess)
      return fail(FSE_ERR_DEVICE);
  }
  if (launch_volume_finalize((const uint8_t*)pl->vol.ptr, (const uint8_t*)pl->state.ptr,
                             (const double*)pl->work.ptr, (uint8_t*)pl->out.ptr, n,
                             s) != hipSuccess ||
      hipEventRecord(pl->ev1, s) != hipSuccess ||
      hipMemcpyAsync(v->out, pl->out.ptr, n, hipMemcpyDeviceToHost, s) != hipSuccess ||
      (v->out_f64 && hipMemcpyAsync(v->out_f64, pl->work.ptr, n * sizeof(double),
                                    hipMemcpyDeviceToHost, s) != hipSuccess) ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(FSE_ERR_DEVICE);
  if (v->stats) {
    v->stats->waves = nwaves;
    v->stats->lost_blocks = (int32_t)n_items;
    v->stats->max_wave_blocks = best;
    v->stats->reserved = 0;
    float ms = 0.f;
    v->stats->latency_ms =
        hipEventElapsedTime(&ms, pl->ev0, pl->ev1) == hipSuccess ? (double)ms : -1.0;
  }
  return FSE_OK;
}

int32_t fse_schedule3(int32_t tb, int32_t hb, int32_t wb, const uint8_t* lost, int32_t order,
                      int32_t* wave_of, int32_t* seq) {
  if (tb < 0 || hb < 0 || wb < 0) return FSE_ERR_INVALID;
  if (order != FSE_ORDER_OPTIMIZED && order != FSE_ORDER_LINESCAN) return FSE_ERR_INVALID;
  const int64_t nb = (int64_t)tb * hb * wb;
  if (nb > (1LL << 31) / 4) return FSE_ERR_INVALID;
  if (nb == 0) return 0;
  if (!lost || !wave_of) return FSE_ERR_INVALID;
  std::vector<int32_t> s;
  const int nw = schedule_blocks3(tb, hb, wb, lost, order, wave_of, seq ? &s : nullptr);
  if (seq) std::copy(s.begin(), s.end(), seq);
  return nw;
}

}  // extern "C"
