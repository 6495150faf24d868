// fse_runtime.cpp -- host runtime and C ABI of the FSE library (fse.h).
//
// A plan owns the per-plan tables (radial weights of Eq. (2), DFT twiddles),
// a HIP stream and grow-only device arenas.  fse_conceal_image runs the
// paper's processing order (fse_sched.cpp) on the host and launches one fused
// kernel per wave (fse_kernels.hip); with several frames, wave t of the call
// is the union of wave t of every frame, so one launch covers all of them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>
#include <type_traits>
#include <vector>

#include "fse.h"
#include "fse_device.h"
#include "fse_internal.h"
#include "fse_sched.h"

namespace fse {

template <typename T>
hipError_t launch_block(const BlockArgs<T>& a, int n_items, int waves, hipStream_t s, int mode);
hipError_t upload_twiddle_constants(const double* tbl);
template <typename T>
hipError_t launch_scatter(T* work, uint8_t* state, const FrameDesc* frames, const int32_t* items,
                          int n_items, const T* staging, int Bh, int Bw, int gox, int goy,
                          hipStream_t s);
template <typename T>
hipError_t launch_init(const IoDesc* io, int nframes, int64_t max_pixels, T* work,
                       uint8_t* state, uint8_t* flags, int32_t* counts, bool convert, int Bh,
                       int Bw, int gox, int goy, hipStream_t s);
template <typename T>
hipError_t launch_finalize(const IoDesc* io, int nframes, int64_t max_pixels,
                           const uint8_t* state, const T* work, hipStream_t s);

// Scratch arena of the calling thread (fse_conceal_image_noalloc): while it is
// set, device buffers are carved from it and nothing is allocated.
static thread_local ScratchArena* t_arena = nullptr;

int DevBuf::reserve(size_t bytes) {
  if (bytes <= cap) return FSE_OK;
  if (ScratchArena* ar = t_arena) {
    const size_t off = (ar->used + 255) & ~(size_t)255;
    if (off > ar->size || bytes > ar->size - off) return FSE_ERR_NOMEM;
    ptr = ar->base + off;
    cap = bytes;
    ar->used = off + bytes;
    return FSE_OK;
  }
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  cap = 0;
  size_t want = bytes + bytes / 4 + 256;
  if (hipMalloc(&ptr, want) != hipSuccess) {
    ptr = nullptr;
    return FSE_ERR_DEVICE;
  }
  cap = want;
  return FSE_OK;
}

int DevBuf::reserve_exact(size_t bytes) {
  if (bytes <= cap) return FSE_OK;
  if (t_arena) return reserve(bytes);
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  cap = 0;
  if (hipMalloc(&ptr, bytes) != hipSuccess) {
    ptr = nullptr;
    return FSE_ERR_DEVICE;
  }
  cap = bytes;
  return FSE_OK;
}

void DevBuf::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  cap = 0;
}

int HostBuf::reserve(size_t bytes) {
  if (bytes <= cap) return FSE_OK;
  if (ptr) (void)hipHostFree(ptr);
  ptr = nullptr;
  cap = 0;
  size_t want = bytes + bytes / 4 + 256;
  if (hipHostMalloc(&ptr, want, hipHostMallocDefault) != hipSuccess) {
    ptr = nullptr;
    return FSE_ERR_DEVICE;
  }
  cap = want;
  return FSE_OK;
}

void HostBuf::release() {
  if (ptr) (void)hipHostFree(ptr);
  ptr = nullptr;
  cap = 0;
}

int validate_params(const fse_params* p) {
  if (!p) return FSE_ERR_INVALID;
  if (p->block_w < 1 || p->block_h < 1 || p->block_w > 64 || p->block_h > 64) return FSE_ERR_INVALID;
  if (p->border_d < 0 || p->fft_w < 1 || p->fft_h < 1) return FSE_ERR_INVALID;
  if (p->block_w + 2 * p->border_d > p->fft_w || p->block_h + 2 * p->border_d > p->fft_h)
    return FSE_ERR_INVALID;
  if (!(p->rho > 0.0 && p->rho <= 1.0)) return FSE_ERR_INVALID;
  if (!(p->delta >= 0.0 && p->delta <= 1.0)) return FSE_ERR_INVALID;
  if (!(p->gamma > 0.0 && p->gamma <= 1.0)) return FSE_ERR_INVALID;
  if (p->iterations < 1 || p->iterations > FSE_MAX_ITERATIONS) return FSE_ERR_INVALID;
  if (p->order != FSE_ORDER_OPTIMIZED && p->order != FSE_ORDER_LINESCAN &&
      p->order != FSE_ORDER_REFINED)
    return FSE_ERR_INVALID;
  if (p->precision != FSE_FP64 && p->precision != FSE_FP32 && p->precision != FSE_FP32_RERANK &&
      p->precision != FSE_FP32_F16X3)
    return FSE_ERR_INVALID;
  if (!(p->rerank_gap >= 0.0 && p->rerank_gap < 0.5)) return FSE_ERR_INVALID;
  if (p->grid_off_x < 0 || p->grid_off_x >= p->block_w || p->grid_off_y < 0 ||
      p->grid_off_y >= p->block_h)
    return FSE_ERR_INVALID;
  if (!std::isfinite(p->empty_fill)) return FSE_ERR_INVALID;
  if (p->device_mem_budget < 0 || p->max_inflight_frames < 0) return FSE_ERR_INVALID;
  if (p->flags & ~(FSE_FLAG_DEVICE_PTRS)) return FSE_ERR_INVALID;
  if (p->fft_w != kFft || p->fft_h != kFft) return FSE_ERR_UNSUPPORTED;
  return FSE_OK;
}

int validate_frame(const fse_frame* f, bool device_ptrs) {
  if (!f || !f->image || !f->lost || !f->out) return FSE_ERR_INVALID;
  if (f->width <= 0 || f->height <= 0) return FSE_ERR_INVALID;
  if (f->width > 65535 * 1 || f->height > 65535) return FSE_ERR_INVALID;
  if (f->stride < f->width || f->lost_stride < f->width || f->out_stride < f->width)
    return FSE_ERR_INVALID;
  if (device_ptrs && f->trace) return FSE_ERR_INVALID;
  if (f->trace && (f->trace->capacity < 0 ||
                   (f->trace->capacity > 0 &&
                    (!f->trace->block || !f->trace->wave || !f->trace->u || !f->trace->dc))))
    return FSE_ERR_INVALID;
  return FSE_OK;
}

static void make_tables(fse_plan_s* pl) {
  const int M = pl->M, N = pl->N;
  pl->radial.resize((size_t)M * N);
  const double cm = 0.5 * (M - 1), cn = 0.5 * (N - 1);
  for (int m = 0; m < M; ++m)
    for (int n = 0; n < N; ++n) {
      const double dm = m - cm, dn = n - cn;
      pl->radial[(size_t)m * N + n] = std::pow(pl->p.rho, std::sqrt(dm * dm + dn * dn));
    }
  // cos/sin(2 pi t / 64); the second half mirrors the first exactly
  pl->twid.assign(2 * kFft, 0.0);
  for (int t = 0; t <= kFft / 2; ++t) {
    const double ang = 2.0 * M_PI * t / kFft;
    pl->twid[2 * t] = std::cos(ang);
    pl->twid[2 * t + 1] = std::sin(ang);
  }
  pl->twid[2 * (kFft / 4)] = 0.0;
  pl->twid[2 * (kFft / 2) + 1] = 0.0;
  for (int t = kFft / 2 + 1; t < kFft; ++t) {
    pl->twid[2 * t] = pl->twid[2 * (kFft - t)];
    pl->twid[2 * t + 1] = -pl->twid[2 * (kFft - t) + 1];
  }
}

int plan_device_init(fse_plan_s* pl) {
  const size_t mn = (size_t)pl->M * pl->N;
  if (pl->tbl_radial.reserve(mn * sizeof(double)) || pl->tbl_twid.reserve(2 * kFft * sizeof(double)) ||
      pl->tbl_twid64.reserve(2 * kFft * sizeof(double)) ||
      pl->tbl_radial64.reserve(mn * sizeof(double)))
    return FSE_ERR_DEVICE;
  if (hipMemcpy(pl->tbl_radial64.ptr, pl->radial.data(), mn * sizeof(double), hipMemcpyHostToDevice))
    return FSE_ERR_DEVICE;
  if (pl->p.precision != FSE_FP64) {
    std::vector<float> r(mn), t(2 * kFft);
    for (size_t i = 0; i < mn; ++i) r[i] = (float)pl->radial[i];
    for (int i = 0; i < 2 * kFft; ++i) t[i] = (float)pl->twid[i];
    if (hipMemcpy(pl->tbl_radial.ptr, r.data(), mn * sizeof(float), hipMemcpyHostToDevice) ||
        hipMemcpy(pl->tbl_twid.ptr, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice))
      return FSE_ERR_DEVICE;
  } else {
    if (hipMemcpy(pl->tbl_radial.ptr, pl->radial.data(), mn * sizeof(double), hipMemcpyHostToDevice) ||
        hipMemcpy(pl->tbl_twid.ptr, pl->twid.data(), 2 * kFft * sizeof(double), hipMemcpyHostToDevice))
      return FSE_ERR_DEVICE;
  }
  if (hipMemcpy(pl->tbl_twid64.ptr, pl->twid.data(), 2 * kFft * sizeof(double), hipMemcpyHostToDevice))
    return FSE_ERR_DEVICE;
  // the constant-memory copies of the transforms (same values for every plan)
  if (upload_twiddle_constants(pl->twid.data()) != hipSuccess) return FSE_ERR_DEVICE;
  return FSE_OK;
}

// ------------------------------------------------------------ batch execution

HostPool::HostPool(int workers) {
  for (int t = 0; t < workers; ++t) th_.emplace_back([this] { worker(); });
}

HostPool::~HostPool() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  for (auto& t : th_) t.join();
}

void HostPool::worker() {
  uint64_t seen = 0;
  for (;;) {
    const std::function<void(int)>* fn;
    int n;
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
      if (stop_) return;
      seen = gen_;
      fn = fn_;
      n = n_;
    }
    for (int i = next_++; i < n; i = next_++) (*fn)(i);
    std::lock_guard<std::mutex> lk(mu_);
    if (--active_ == 0) done_cv_.notify_all();
  }
}

void HostPool::run(int n, const std::function<void(int)>& fn) {
  if (th_.empty() || n <= 1) {
    for (int i = 0; i < n; ++i) fn(i);
    return;
  }
  {
    std::lock_guard<std::mutex> lk(mu_);
    fn_ = &fn;
    n_ = n;
    next_ = 0;
    active_ = (int)th_.size();
    ++gen_;
  }
  cv_.notify_all();
  for (int i = next_++; i < n; i = next_++) fn(i);
  std::unique_lock<std::mutex> lk(mu_);
  done_cv_.wait(lk, [&] { return active_ == 0; });
  fn_ = nullptr;
}

// fn(0..n-1) on the plan's host workers (created on first use: up to 15
// threads besides the caller).
static void parallel_for(fse_plan_s* pl, int n, const std::function<void(int)>& fn) {
  if (!pl->pool) {
    const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
    pl->pool = new HostPool(std::min(15, hw - 1));
  }
  pl->pool->run(n, fn);
}

// nonzero bytes in p[0..n)
static int count_nonzero(const uint8_t* p, int n) {
  int c = 0;
  for (int i = 0; i < n; ++i) c += p[i] != 0;
  return c;
}

// any nonzero byte in p[0..n)
static bool any_nonzero(const uint8_t* p, int n) {
  uint64_t acc = 0;
  int i = 0;
  for (; i + 8 <= n; i += 8) {
    uint64_t v;
    std::memcpy(&v, p + i, 8);
    acc |= v;
  }
  for (; i < n; ++i) acc |= p[i];
  return acc != 0;
}

// Group 0 runs on the plan's stream; groups 1.. on non-blocking streams of
// their own (default priority), each with a join event, created on first use.
static int ensure_group_streams(fse_plan_s* pl, int G) {
  while ((int)pl->gstreams.size() < G - 1) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return FSE_ERR_DEVICE;
    pl->gstreams.push_back(st);
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return FSE_ERR_DEVICE;
    pl->gjoin.push_back(e);
  }
  return FSE_OK;
}

// noalloc: device buffers come from the calling thread's scratch arena, one
// frame group, synchronous copies through ordinary host memory instead of
// pinned staging, no per-launch timing events.
template <typename T>
static int run_batch(fse_plan_s* pl, const fse_frame* frames, int n, bool noalloc) {
  const fse_params& p = pl->p;
  const bool dev = (p.flags & FSE_FLAG_DEVICE_PTRS) != 0;
  hipStream_t s = pl->stream;
  const int Bh = p.block_h, Bw = p.block_w, gox = p.grid_off_x, goy = p.grid_off_y;
  const int K = p.iterations;
  auto chk = [&](hipError_t e) { return e == hipSuccess ? FSE_OK : FSE_ERR_DEVICE; };

  // geometry and arena offsets (256-element aligned)
  std::vector<FrameDesc> fd(n);
  std::vector<int> hb(n), wb(n);
  int64_t total = 0;
  for (int f = 0; f < n; ++f) {
    fd[f].off = total;
    fd[f].H = frames[f].height;
    fd[f].W = frames[f].width;
    hb[f] = (frames[f].height + goy + Bh - 1) / Bh;
    wb[f] = (frames[f].width + gox + Bw - 1) / Bw;
    total += ((int64_t)frames[f].height * frames[f].width + 255) & ~255LL;
  }
  int rc = FSE_OK;
  // per-frame I/O descriptors; block flags of all frames in one array
  std::vector<IoDesc> io(n);
  std::vector<uint8_t> host_flags;  // host frames: lost-block flags from the staged masks
  // the refined order needs the lost samples of every block instead of flags
  const bool refined = p.order == FSE_ORDER_REFINED;
  std::vector<int32_t> host_counts;
  std::vector<int64_t> fout_off(n, -1);
  int64_t flag_total = 0, max_pixels = 0, fout_bytes = 0;
  for (int f = 0; f < n; ++f) {
    const fse_frame& fr = frames[f];
    const int64_t px = (int64_t)fr.height * fr.width;
    io[f].off = fd[f].off;
    io[f].flag_off = flag_total;
    io[f].H = fr.height;
    io[f].W = fr.width;
    io[f].wb = wb[f];
    flag_total += (int64_t)hb[f] * wb[f];
    max_pixels = std::max(max_pixels, px);
    if (!dev && (fr.out_f32 || fr.out_f64)) {
      fout_off[f] = fout_bytes;
      fout_bytes += ((fr.out_f32 ? px * 4 : 0) + (fr.out_f64 ? px * 8 : 0) + 255) & ~255LL;
    }
  }
  if ((rc = pl->work.reserve(total * sizeof(T))) || (rc = pl->state.reserve(total)) ||
      (rc = pl->frames_dev.reserve(n * sizeof(FrameDesc))) ||
      (rc = pl->io_dev.reserve(n * sizeof(IoDesc))) || (rc = pl->flags_dev.reserve(flag_total * (refined ? 4 : 1))))
    return rc;
  if (!dev) {
    if ((rc = pl->u8_img.reserve(total)) || (rc = pl->u8_lost.reserve(total)) ||
        (rc = pl->u8_out.reserve(total)) || (fout_bytes && (rc = pl->fout.reserve(fout_bytes))) ||
        (rc = pl->pin_in.reserve(2 * total)) || (rc = pl->pin_out.reserve(total)))
      return rc;
    // host frames: rows into pinned staging on host threads, each frame's
    // DMA issued as soon as its rows are in (pageable 2-D copies would go row
    // by row), and the lost-block flags taken from the staged mask on the
    // host, so the schedule does not wait for the device
    uint8_t* pimg = (uint8_t*)pl->pin_in.ptr;
    uint8_t* plost = pimg + total;
    if (refined)
      host_counts.assign(flag_total, 0);
    else
      host_flags.assign(flag_total, 0);
    std::vector<int> frc(n, FSE_OK);
    parallel_for(pl, n, [&](int f) {
      const fse_frame& fr = frames[f];
      const int H = fr.height, W = fr.width;
      uint8_t* a = pimg + fd[f].off;
      uint8_t* b = plost + fd[f].off;
      for (int y = 0; y < H; ++y) {
        std::memcpy(a + (int64_t)y * W, fr.image + (int64_t)y * fr.stride, W);
        uint8_t* row = b + (int64_t)y * W;
        std::memcpy(row, fr.lost + (int64_t)y * fr.lost_stride, W);
        const int64_t rb = io[f].flag_off + (int64_t)((y + goy) / Bh) * wb[f];
        if (refined) {
          int32_t* crow = host_counts.data() + rb;
          for (int bj = 0; bj < wb[f]; ++bj) {
            const int x0 = std::max(0, bj * Bw - gox), x1 = std::min(W, (bj + 1) * Bw - gox);
            if (x1 > x0) crow[bj] += count_nonzero(row + x0, x1 - x0);
          }
          continue;
        }
        uint8_t* frow = host_flags.data() + rb;
        for (int bj = 0; bj < wb[f]; ++bj) {
          if (frow[bj]) continue;
          const int x0 = std::max(0, bj * Bw - gox), x1 = std::min(W, (bj + 1) * Bw - gox);
          if (x1 > x0 && any_nonzero(row + x0, x1 - x0)) frow[bj] = 1;
        }
      }
      const size_t bytes = (size_t)H * W;
      if (hipSetDevice(pl->device) != hipSuccess ||
          hipMemcpyAsync((uint8_t*)pl->u8_img.ptr + fd[f].off, a, bytes, hipMemcpyHostToDevice,
                         s) != hipSuccess ||
          hipMemcpyAsync((uint8_t*)pl->u8_lost.ptr + fd[f].off, b, bytes, hipMemcpyHostToDevice,
                         s) != hipSuccess)
        frc[f] = FSE_ERR_DEVICE;
    });
    for (int f = 0; f < n; ++f)
      if (frc[f]) return frc[f];
  }
  T* work = (T*)pl->work.ptr;
  uint8_t* state = (uint8_t*)pl->state.ptr;
  for (int f = 0; f < n; ++f) {
    const fse_frame& fr = frames[f];
    const int H = fr.height, W = fr.width;
    if (dev) {
      io[f].image = fr.image;
      io[f].lost = fr.lost;
      io[f].out = fr.out;
      io[f].stride = fr.stride;
      io[f].lstride = fr.lost_stride;
      io[f].ostride = fr.out_stride;
      io[f].of32 = fr.out_f32;
      io[f].of64 = fr.out_f64;
    } else {
      uint8_t* a = (uint8_t*)pl->u8_img.ptr + fd[f].off;
      uint8_t* b = (uint8_t*)pl->u8_lost.ptr + fd[f].off;
      io[f].image = a;
      io[f].lost = b;
      io[f].out = (uint8_t*)pl->u8_out.ptr + fd[f].off;
      io[f].stride = io[f].lstride = io[f].ostride = W;
      char* fo = fout_off[f] >= 0 ? (char*)pl->fout.ptr + fout_off[f] : nullptr;
      io[f].of32 = fr.out_f32 ? (float*)fo : nullptr;
      io[f].of64 = fr.out_f64 ? (double*)(fo + (fr.out_f32 ? (size_t)H * W * 4 : 0)) : nullptr;
    }
  }
  if ((rc = chk(hipMemcpyAsync(pl->io_dev.ptr, io.data(), n * sizeof(IoDesc),
                               hipMemcpyHostToDevice, s))))
    return rc;
  // device frames: a first pass over the masks marks the lost blocks (or
  // counts their lost samples) and they are copied back, so that the host
  // schedules while the second pass converts the images; host frames have
  // their flags already
  const size_t flag_bytes = (size_t)flag_total * (refined ? 4 : 1);
  const IoDesc* iod = (const IoDesc*)pl->io_dev.ptr;
  std::vector<uint8_t> flag_copy;  // noalloc: the flags in ordinary host memory
  if (dev && noalloc) {
    flag_copy.resize(std::max<size_t>(1, flag_bytes));
    if ((rc = chk(hipMemsetAsync(pl->flags_dev.ptr, 0, flag_bytes, s))) ||
        (rc = chk(launch_init<T>(iod, n, max_pixels, work, state,
                                 refined ? nullptr : (uint8_t*)pl->flags_dev.ptr,
                                 refined ? (int32_t*)pl->flags_dev.ptr : nullptr, false, Bh, Bw,
                                 gox, goy, s))) ||
        (rc = chk(hipMemcpyAsync(flag_copy.data(), pl->flags_dev.ptr, flag_bytes,
                                 hipMemcpyDeviceToHost, s))) ||
        (rc = chk(hipStreamSynchronize(s))))
      return rc;
  } else if (dev) {
    if ((rc = pl->pin_flags.reserve(std::max<size_t>(1, flag_bytes)))) return rc;
    if (!pl->ev_flags && hipEventCreateWithFlags(&pl->ev_flags, hipEventDisableTiming) != hipSuccess)
      return FSE_ERR_DEVICE;
    if ((rc = chk(hipMemsetAsync(pl->flags_dev.ptr, 0, flag_bytes, s))) ||
        (rc = chk(launch_init<T>(iod, n, max_pixels, work, state,
                                 refined ? nullptr : (uint8_t*)pl->flags_dev.ptr,
                                 refined ? (int32_t*)pl->flags_dev.ptr : nullptr, false, Bh, Bw,
                                 gox, goy, s))) ||
        (rc = chk(hipMemcpyAsync(pl->pin_flags.ptr, pl->flags_dev.ptr, flag_bytes,
                                 hipMemcpyDeviceToHost, s))) ||
        (rc = chk(hipEventRecord(pl->ev_flags, s))))
      return rc;
  }
  if ((rc = chk(launch_init<T>(iod, n, max_pixels, work, state, nullptr, nullptr, true, Bh, Bw,
                               gox, goy, s))))
    return rc;
  if (dev && !noalloc && (rc = chk(hipEventSynchronize(pl->ev_flags)))) return rc;
  const void* dflags = noalloc ? (const void*)flag_copy.data() : pl->pin_flags.ptr;
  const uint8_t* flag_base = dev ? (const uint8_t*)dflags : host_flags.data();
  const int32_t* count_base = dev ? (const int32_t*)dflags : host_counts.data();

  // processing order per frame
  std::vector<std::vector<int32_t>> wave_of(n), seq(n);
  // frames are scheduled independently, on the plan's host workers, the
  // largest grids first (the last frame taken should be a small one)
  std::vector<int> nwaves(n, 0);
  std::vector<int> by_size(n);
  for (int f = 0; f < n; ++f) by_size[f] = f;
  std::stable_sort(by_size.begin(), by_size.end(),
                   [&](int x, int y) { return (int64_t)hb[x] * wb[x] > (int64_t)hb[y] * wb[y]; });
  parallel_for(pl, n, [&](int i) {
    const int f = by_size[i];
    wave_of[f].resize((size_t)hb[f] * wb[f]);
    nwaves[f] = refined ? schedule_blocks_refined(hb[f], wb[f], count_base + io[f].flag_off,
                                                  Bh * Bw, wave_of[f].data(), &seq[f])
                        : schedule_blocks(hb[f], wb[f], flag_base + io[f].flag_off, p.order,
                                          wave_of[f].data(), &seq[f]);
  });
  for (int f = 0; f < n; ++f) {
    const int nw = nwaves[f];
    if (frames[f].stats) {
      fse_stats* st = frames[f].stats;
      st->waves = nw;
      st->lost_blocks = (int32_t)seq[f].size();
      int best = 0, run = 0, prev = -1;
      for (int32_t b : seq[f]) {
        int w = wave_of[f][b];
        run = (w == prev) ? run + 1 : 1;
        prev = w;
        best = std::max(best, run);
      }
      st->max_wave_blocks = best;
      st->latency_ms = 0.0;
    }
  }
  // Frames are split into up to `groups` groups (largest first onto the
  // group with the fewest lost blocks); each group runs its own sequence of
  // steps on its own stream, so one group's small launches overlap another's.
  // The deepest frames (crit_depth) take group 0 to themselves: their chain of
  // waves is the batch's critical path.  Inside a group frames start at
  // staggered steps: step s of the group holds wave s - off[f] of its frame f.
  const bool staged_mode = p.border_d > std::min(Bh, Bw);
  const int G = (staged_mode || noalloc) ? 1 : std::max(1, std::min(pl->group_count(), n));
  std::vector<std::vector<int>> gframes(G);
  bool crit_group = false;  // group 0 holds the deepest frames
  {
    std::vector<int> byload;
    if (G >= 2 && pl->crit_depth() > 0.0) {
      int D = 0;
      for (int f = 0; f < n; ++f) D = std::max(D, nwaves[f]);
      for (int f = 0; f < n; ++f) {
        if (nwaves[f] > 0 && nwaves[f] >= pl->crit_depth() * D)
          gframes[0].push_back(f);
        else
          byload.push_back(f);
      }
      crit_group = !gframes[0].empty() && !byload.empty();
      if (!crit_group) {
        gframes[0].clear();
        byload.clear();
      }
    }
    const int g0 = crit_group ? 1 : 0;
    if (!crit_group)
      for (int f = 0; f < n; ++f) byload.push_back(f);
    std::stable_sort(byload.begin(), byload.end(),
                     [&](int x, int y) { return seq[x].size() > seq[y].size(); });
    std::vector<int64_t> load(G - g0, 0);
    for (int f : byload) {
      const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      gframes[g0 + g].push_back(f);
      load[g] += (int64_t)seq[f].size();
    }
    for (auto& v : gframes) std::sort(v.begin(), v.end());
  }
  const bool fp64 = p.precision == FSE_FP64;
  // gstart[g][t] = first item of step t of group g (items of all groups in
  // one array, group after group); each group's items are laid out on a host
  // worker of their own, then joined
  std::vector<std::vector<int64_t>> gstart(G);
  std::vector<std::vector<int32_t>> gitems(G);
  std::vector<std::vector<std::pair<int, int32_t>>> gsrc(G);
  parallel_for(pl, G, [&](int g) {
    std::vector<int32_t>& items = gitems[g];
    std::vector<std::pair<int, int32_t>>& item_src = gsrc[g];
    const std::vector<int>& fs = gframes[g];
    const int m = (int)fs.size();
    std::vector<int> off(m, 0);
    int steps = 0;
    for (int f : fs) steps = std::max(steps, nwaves[f]);
    if (m > 1 && pl->stagger) {
      std::vector<std::vector<int>> sizes(m);
      for (int k = 0; k < m; ++k) {
        const int f = fs[k];
        sizes[k].assign(nwaves[f], 0);
        for (int32_t b : seq[f]) ++sizes[k][wave_of[f][b]];
      }
      off = stagger_frames(sizes, fp64 ? pl->model_latency_us[0] : pl->model_latency_us[1],
                           fp64 ? pl->model_rate[0] : pl->model_rate[1]);
      for (int k = 0; k < m; ++k) steps = std::max(steps, off[k] + nwaves[fs[k]]);
    }
    gstart[g].assign(steps + 1, 0);
    std::vector<size_t> pos(m, 0);
    const int32_t prio = (crit_group && g == 0 && pl->crit_prio) ? 1 << kItemPrioShift : 0;
    for (int step = 0; step < steps; ++step) {
      gstart[g][step] = (int64_t)items.size() / 2;
      for (int k = 0; k < m; ++k) {
        const int f = fs[k];
        const int t = step - off[k];
        while (t >= 0 && pos[k] < seq[f].size() && wave_of[f][seq[f][pos[k]]] == t) {
          const int32_t b = seq[f][pos[k]++];
          items.push_back(f | prio);
          items.push_back(((b / wb[f]) << 16) | (b % wb[f]));
          item_src.emplace_back(f, b);
        }
      }
    }
    gstart[g][steps] = (int64_t)items.size() / 2;
  });
  std::vector<int32_t> items;
  std::vector<std::pair<int, int32_t>> item_src;  // (frame, block) per item
  int max_steps = 0;
  {
    size_t ni = 0;
    for (int g = 0; g < G; ++g) ni += gsrc[g].size();
    items.reserve(2 * ni);
    item_src.reserve(ni);
    for (int g = 0; g < G; ++g) {
      const int64_t base = (int64_t)item_src.size();
      for (int64_t& x : gstart[g]) x += base;
      items.insert(items.end(), gitems[g].begin(), gitems[g].end());
      item_src.insert(item_src.end(), gsrc[g].begin(), gsrc[g].end());
      max_steps = std::max(max_steps, (int)gstart[g].size() - 1);
    }
  }
  const int64_t n_items = (int64_t)items.size() / 2;

  const bool staged = staged_mode;
  bool want_trace = false;
  for (int f = 0; f < n; ++f) want_trace |= frames[f].trace != nullptr;
  if ((rc = pl->items_dev.reserve(std::max<int64_t>(1, n_items) * 2 * sizeof(int32_t))))
    return rc;
  if (staged && (rc = pl->staging.reserve(std::max<int64_t>(1, n_items) * Bh * Bw * sizeof(T))))
    return rc;
  if (want_trace && ((rc = pl->trace_u.reserve(std::max<int64_t>(1, n_items) * K * sizeof(int32_t))) ||
                     (rc = pl->trace_dc.reserve(std::max<int64_t>(1, n_items) * K * 2 * sizeof(T)))))
    return rc;
  if (n_items > 0 && noalloc) {
    if ((rc = chk(hipMemcpyAsync(pl->items_dev.ptr, items.data(), items.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, s))) ||
        (rc = chk(hipStreamSynchronize(s))))
      return rc;
  } else if (n_items > 0) {
    // through pinned staging, so that the copy does not hold the host; the
    // previous call's copy out of the staging is done first
    if (!pl->ev_items && hipEventCreateWithFlags(&pl->ev_items, hipEventDisableTiming) != hipSuccess)
      return FSE_ERR_DEVICE;
    if (pl->items_recorded && (rc = chk(hipEventSynchronize(pl->ev_items)))) return rc;
    if ((rc = pl->pin_items.reserve(items.size() * sizeof(int32_t)))) return rc;
    std::memcpy(pl->pin_items.ptr, items.data(), items.size() * sizeof(int32_t));
    if ((rc = chk(hipMemcpyAsync(pl->items_dev.ptr, pl->pin_items.ptr,
                                 items.size() * sizeof(int32_t), hipMemcpyHostToDevice, s))) ||
        (rc = chk(hipEventRecord(pl->ev_items, s))))
      return rc;
    pl->items_recorded = true;
  }
  if ((rc = chk(hipMemcpyAsync(pl->frames_dev.ptr, fd.data(), n * sizeof(FrameDesc),
                               hipMemcpyHostToDevice, s))))
    return rc;

  BlockArgs<T> a;
  a.work = work;
  a.state = state;
  a.frames = (const FrameDesc*)pl->frames_dev.ptr;
  a.radial = (const T*)pl->tbl_radial.ptr;
  a.radial64 = (const double*)pl->tbl_radial64.ptr;
  a.twid = (const T*)pl->tbl_twid.ptr;
  a.twid64 = (const double*)pl->tbl_twid64.ptr;
  a.M = pl->M;
  a.N = pl->N;
  a.Bh = Bh;
  a.Bw = Bw;
  a.d = p.border_d;
  a.gox = gox;
  a.goy = goy;
  a.K = K;
  a.delta = (T)p.delta;
  a.gamma = (T)p.gamma;
  a.delta64 = p.delta;
  a.gamma64 = p.gamma;
  a.zscale = (T)128.0;
  a.empty_fill = p.empty_fill;
  a.rerank_gap = p.rerank_gap > 0.0 ? p.rerank_gap : 1e-4;
  a.counters = nullptr;
  const bool rerank = p.precision == FSE_FP32_RERANK;
  const bool mx = p.precision == FSE_FP32_F16X3;  // matrix-core transforms, 4 wavefronts
  // FP64 spectra: one slot per item of a step, per group (groups run at once)
  std::vector<int64_t> spec_base(G + 1, 0);
  for (int g = 0; g < G; ++g) {
    int64_t mx = 0;
    for (size_t t = 0; t + 1 < gstart[g].size(); ++t) mx = std::max(mx, gstart[g][t + 1] - gstart[g][t]);
    spec_base[g + 1] = spec_base[g] + mx;
  }
  a.spec64 = nullptr;
  if (rerank) {
    if ((rc = pl->spec64.reserve(std::max<int64_t>(1, spec_base[G]) * kSpecStride * sizeof(double))))
      return rc;
  }
  // re-scoring statistics of this call
  if (rerank) {
    if ((rc = pl->counters.reserve(kCntSlots * sizeof(unsigned long long))) ||
        (!noalloc && (rc = pl->pin_cnt.reserve(kCntSlots * sizeof(unsigned long long)))) ||
        (rc = chk(hipMemsetAsync(pl->counters.ptr, 0, kCntSlots * sizeof(unsigned long long), s))))
      return rc;
    a.counters = (unsigned long long*)pl->counters.ptr;
  }

  // streams: group 0 on the plan's stream, the other groups on streams forked
  // from and joined back into it
  if ((rc = ensure_group_streams(pl, G))) return rc;
  int n_launch = 0;
  for (int g = 0; g < G; ++g)
    for (size_t t = 0; t + 1 < gstart[g].size(); ++t) n_launch += gstart[g][t + 1] > gstart[g][t];
  // timing events (not in the noalloc form): a marker before and one after
  // every launch of the block kernel; a group's consecutive launches share
  // the marker between them (every recorded event is a packet its queue
  // processes between two kernels: three per launch cost 2-5 % of a batch).
  // Two more bracket the call's launches.
  const bool timed = !noalloc;
  while (timed && (int)pl->events.size() < 2 * n_launch + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return FSE_ERR_DEVICE;
    pl->events.push_back(e);
  }
  hipEvent_t ev_fork = timed ? pl->events[2 * n_launch] : nullptr;
  hipEvent_t ev_end = timed ? pl->events[2 * n_launch + 1] : nullptr;
  if (timed && (rc = chk(hipEventRecord(ev_fork, s)))) return rc;  // G > 1 implies timed
  for (int g = 1; g < G; ++g)
    if ((rc = chk(hipStreamWaitEvent(pl->gstreams[g - 1], ev_fork, 0)))) return rc;
  struct LaunchMarks {
    int pre, post;  // indices into pl->events
  };
  std::vector<LaunchMarks> marks(timed ? n_launch : 0);
  std::vector<int> tail(G, -1);  // marker at the tail of a group's stream, -1 = none
  int n_ev = 0;
  auto mark = [&](hipStream_t st, int& idx) {
    idx = n_ev++;
    return chk(hipEventRecord(pl->events[idx], st));
  };
  int li = 0;
  for (int t = 0; t < max_steps; ++t) {
    // blocks of this step over all groups, for the workgroup shape
    int64_t step_total = 0;
    for (int g = 0; g < G; ++g)
      if (t + 1 < (int)gstart[g].size()) step_total += gstart[g][t + 1] - gstart[g][t];
    for (int g = 0; g < G; ++g) {
      if (t + 1 >= (int)gstart[g].size()) continue;
      const int64_t i0 = gstart[g][t], cnt = gstart[g][t + 1] - i0;
      if (cnt == 0) continue;
      hipStream_t gs = g > 0 ? pl->gstreams[g - 1] : s;
      a.items = (const int32_t*)pl->items_dev.ptr + 2 * i0;
      a.staging = staged ? (T*)pl->staging.ptr : nullptr;
      a.trace_u = want_trace ? (int32_t*)pl->trace_u.ptr + i0 * K : nullptr;
      a.trace_dc = want_trace ? (T*)pl->trace_dc.ptr + i0 * K * 2 : nullptr;
      if (rerank) a.spec64 = (double*)pl->spec64.ptr + spec_base[g] * kSpecStride;
      const int waves =
          mx ? 4 : (crit_group && g == 0 ? pl->crit_waves_for(cnt) : pl->waves_for(step_total));
      LaunchMarks m{-1, -1};
      if (timed) {
        if (tail[g] >= 0)
          m.pre = tail[g];
        else if ((rc = mark(gs, m.pre)))
          return rc;
      }
      if ((rc = chk(launch_block<T>(a, (int)cnt, waves, gs, rerank ? 1 : (mx ? 2 : 0)))))
        return rc;
      if (timed) {
        if ((rc = mark(gs, m.post))) return rc;
        marks[li] = m;
        tail[g] = staged ? -1 : m.post;  // the scatter kernel follows in the staged form
      }
      if (staged && (rc = chk(launch_scatter<T>(work, state, a.frames, a.items, (int)cnt,
                                                (const T*)pl->staging.ptr, Bh, Bw, gox, goy, gs))))
        return rc;
      ++li;
    }
  }
  for (int g = 1; g < G; ++g) {
    if ((rc = chk(hipEventRecord(pl->gjoin[g - 1], pl->gstreams[g - 1]))) ||
        (rc = chk(hipStreamWaitEvent(s, pl->gjoin[g - 1], 0))))
      return rc;
  }
  if (timed && (rc = chk(hipEventRecord(ev_end, s)))) return rc;

  // outputs
  if ((rc = chk(launch_finalize<T>((const IoDesc*)pl->io_dev.ptr, n, max_pixels, state, work, s))))
    return rc;
  // the re-scoring statistics come back with the outputs (through pinned
  // staging; the noalloc form copies them after the wait)
  if (a.counters && !noalloc &&
      (rc = chk(hipMemcpyAsync(pl->pin_cnt.ptr, a.counters, kCntSlots * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, s))))
    return rc;
  if (!dev) {
    if ((rc = chk(hipMemcpyAsync(pl->pin_out.ptr, pl->u8_out.ptr, total, hipMemcpyDeviceToHost, s))))
      return rc;
    for (int f = 0; f < n; ++f) {
      const fse_frame& fr = frames[f];
      const int H = fr.height, W = fr.width;
      if (fr.out_f32 && (rc = chk(hipMemcpyAsync(fr.out_f32, io[f].of32, (size_t)H * W * 4,
                                                 hipMemcpyDeviceToHost, s))))
        return rc;
      if (fr.out_f64 && (rc = chk(hipMemcpyAsync(fr.out_f64, io[f].of64, (size_t)H * W * 8,
                                                 hipMemcpyDeviceToHost, s))))
        return rc;
    }
  }
  if ((rc = chk(hipStreamSynchronize(s)))) return rc;
  if (!dev) {
    const uint8_t* pout = (const uint8_t*)pl->pin_out.ptr;
    parallel_for(pl, n, [&](int f) {
      const fse_frame& fr = frames[f];
      for (int y = 0; y < fr.height; ++y)
        std::memcpy(fr.out + (int64_t)y * fr.out_stride, pout + fd[f].off + (int64_t)y * fr.width,
                    fr.width);
    });
  }

  // device time of every marker from the fork (one query per marker)
  std::vector<float> at(timed ? n_ev : 0, 0.f);
  std::vector<char> at_ok(at.size(), 0);
  for (size_t i = 0; i < at.size(); ++i)
    at_ok[i] = hipEventElapsedTime(&at[i], ev_fork, pl->events[i]) == hipSuccess;
  double kms = 0.0;
  for (int t = 0; timed && t < n_launch; ++t) {
    const LaunchMarks& m = marks[t];
    if (at_ok[m.pre] && at_ok[m.post]) kms += at[m.post] - at[m.pre];
  }
  float span = 0.f;
  if (timed) (void)hipEventElapsedTime(&span, ev_fork, ev_end);
  // union of the iteration kernel's launch intervals (launches of different
  // groups overlap)
  double busy = 0.0;
  if (timed) {
    std::vector<std::pair<float, float>> iv;
    iv.reserve(n_launch);
    for (int t = 0; t < n_launch; ++t)
      if (at_ok[marks[t].pre] && at_ok[marks[t].post]) iv.emplace_back(at[marks[t].pre], at[marks[t].post]);
    std::sort(iv.begin(), iv.end());
    float lo = 0.f, hi = -1.f;
    for (const auto& x : iv) {
      if (x.first > hi) {
        if (hi > lo) busy += hi - lo;
        lo = x.first;
        hi = x.second;
      } else {
        hi = std::max(hi, x.second);
      }
    }
    if (hi > lo) busy += hi - lo;
  }
  pl->last.rescored = pl->last.rescore_candidates = pl->last.rescore_wide =
      pl->last.rescore_max_wave = 0;
  if (a.counters) {
    unsigned long long cnt[kCntSlots];
    if (!noalloc)
      std::memcpy(cnt, pl->pin_cnt.ptr, sizeof(cnt));
    else if ((rc = chk(hipMemcpy(cnt, a.counters, sizeof(cnt), hipMemcpyDeviceToHost))))
      return rc;
    pl->last.rescored = (int64_t)cnt[kCntRescored];
    pl->last.rescore_candidates = (int64_t)cnt[kCntCandidates];
    pl->last.rescore_wide = (int64_t)cnt[kCntWide];
    pl->last.rescore_max_wave = (int64_t)cnt[kCntMaxWave];
  }
  pl->last.kernel_ms = kms;
  pl->last.transform_ms = 0.0;  // the transforms run inside the block kernel
  pl->last.span_ms = span;
  pl->last.busy_ms = busy;
  pl->last.groups = G;
  pl->last.launches = n_launch;
  pl->last.blocks = n_items;

  if (want_trace && n_items > 0) {
    std::vector<int32_t> tu((size_t)n_items * K);
    std::vector<T> tdc((size_t)n_items * K * 2);
    if ((rc = chk(hipMemcpy(tu.data(), pl->trace_u.ptr, tu.size() * sizeof(int32_t), hipMemcpyDeviceToHost))) ||
        (rc = chk(hipMemcpy(tdc.data(), pl->trace_dc.ptr, tdc.size() * sizeof(T), hipMemcpyDeviceToHost))))
      return rc;
    std::vector<int32_t> cnt(n, 0);
    for (int64_t i = 0; i < n_items; ++i) {
      const int f = item_src[i].first;
      fse_trace* tr = frames[f].trace;
      if (!tr) continue;
      const int slot = cnt[f]++;
      if (slot >= tr->capacity) continue;
      const int32_t b = item_src[i].second;
      tr->block[slot] = b;
      tr->wave[slot] = wave_of[f][b];
      for (int k = 0; k < K; ++k) {
        tr->u[(size_t)slot * K + k] = tu[(size_t)i * K + k];
        tr->dc[((size_t)slot * K + k) * 2] = (double)tdc[((size_t)i * K + k) * 2];
        tr->dc[((size_t)slot * K + k) * 2 + 1] = (double)tdc[((size_t)i * K + k) * 2 + 1];
      }
    }
    for (int f = 0; f < n; ++f)
      if (frames[f].trace) frames[f].trace->count = (int32_t)seq[f].size();
  } else {
    for (int f = 0; f < n; ++f)
      if (frames[f].trace) frames[f].trace->count = (int32_t)seq[f].size();
  }
  return FSE_OK;
}

// Device address of the noalloc scratch, taken once per device (with that
// device current) and kept: each GPU holds its own copy of the array.
static int noalloc_scratch_init(fse_plan_s* pl) {
  static std::mutex mu;
  static std::vector<void*> addr;  // per device id
  std::lock_guard<std::mutex> lk(mu);
  if ((int)addr.size() <= pl->device) addr.resize(pl->device + 1, nullptr);
  if (!addr[pl->device]) {
    void* p = nullptr;
    if (hipSetDevice(pl->device) != hipSuccess || noalloc_scratch_address(&p) != hipSuccess ||
        !p)
      return FSE_ERR_DEVICE;
    addr[pl->device] = p;
  }
  pl->scratch = addr[pl->device];
  return FSE_OK;
}

int conceal_batch(fse_plan_s* pl, const fse_frame* frames, int n, bool noalloc) {
  return pl->p.precision == FSE_FP64 ? run_batch<double>(pl, frames, n, noalloc)
                                     : run_batch<float>(pl, frames, n, noalloc);
}

void set_thread_arena(ScratchArena* a) { t_arena = a; }

}  // namespace fse

using namespace fse;

extern "C" {

int32_t fse_plan(const fse_params* p, void* hip_stream, fse_plan_t* out) {
  if (!out) return FSE_ERR_INVALID;
  *out = nullptr;
  int rc = validate_params(p);
  if (rc) return rc;
  const int M = p->block_h + 2 * p->border_d, N = p->block_w + 2 * p->border_d;
  const int K = p->iterations;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return FSE_ERR_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return FSE_ERR_DEVICE;
  for (int waves : {4, 8, 16}) {
    const int64_t need = p->precision == FSE_FP64 ? lds_bytes<double>(M, N, K, waves)
                                                  : lds_bytes<float>(M, N, K, waves);
    if (need > (int64_t)prop.sharedMemPerBlock) return FSE_ERR_UNSUPPORTED;
  }
  if (p->precision == FSE_FP32_RERANK &&
      lds_bytes<double>(M, N, K, 4) > (int64_t)prop.sharedMemPerBlock)
    return FSE_ERR_UNSUPPORTED;
  fse_plan_s* pl = new fse_plan_s();
  pl->p = *p;
  if (p->precision == FSE_FP32_RERANK) {
    // its small launches on 8 wavefronts instead of 16: the 16-wavefront form
    // of the re-rank kernel holds its FP64 transforms in 64 VGPRs
    pl->wide_threshold = 0;
    pl->mid_threshold = 128;
  }
  pl->M = M;
  pl->N = N;
  pl->device = dev;
  if (hip_stream) {
    pl->stream = (hipStream_t)hip_stream;
    pl->own_stream = false;
  } else {
    if (hipStreamCreateWithFlags(&pl->stream, hipStreamNonBlocking) != hipSuccess) {
      delete pl;
      return FSE_ERR_DEVICE;
    }
    pl->own_stream = true;
  }
  if (const char* env = std::getenv("FSE_FRAME_GROUPS")) {
    const int g = std::atoi(env);
    if (g >= 1 && g <= 16) pl->groups = g;
  }
  if (const char* env = std::getenv("FSE_CRIT_DEPTH")) {
    const double c = std::atof(env);
    if (c >= 0.0 && c <= 1.0) pl->crit = c;
  }
  if (const char* env = std::getenv("FSE_CRIT_PRIO")) pl->crit_prio = std::atoi(env) != 0;
  if (const char* env = std::getenv("FSE_CRIT_WAVES")) {
    const int c = std::atoi(env);
    if (c == 0 || c == 4 || c == 8 || c == 16) pl->crit_waves = c;
  }
  if (const char* env = std::getenv("FSE_WAVE_THRESHOLDS")) {
    int t16 = 0, t8 = 0;
    if (std::sscanf(env, "%d,%d", &t16, &t8) == 2 && t16 >= 0 && t8 >= 0) {
      pl->wide_threshold = t16;
      pl->mid_threshold = t8;
    }
  }
  make_tables(pl);
  rc = noalloc_scratch_init(pl);
  if (rc) {
    fse_plan_destroy(pl);
    return rc;
  }
  rc = plan_device_init(pl);
  if (rc) {
    fse_plan_destroy(pl);
    return rc;
  }
  rc = serving_init(pl);
  if (rc) {
    fse_plan_destroy(pl);
    return rc;
  }
  *out = pl;
  return FSE_OK;
}

int32_t fse_plan_destroy(fse_plan_t pl) {
  if (!pl) return FSE_OK;
  serving_shutdown(pl);
  if (pl->stream) (void)hipStreamSynchronize(pl->stream);
  for (hipEvent_t e : pl->events) (void)hipEventDestroy(e);
  pl->events.clear();
  for (hipStream_t st : pl->gstreams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  pl->gstreams.clear();
  for (hipEvent_t e : pl->gjoin) (void)hipEventDestroy(e);
  pl->gjoin.clear();
  DevBuf* bufs[] = {&pl->tbl_radial, &pl->tbl_twid, &pl->tbl_twid64, &pl->tbl_radial64,
                    &pl->spec64, &pl->counters, &pl->work, &pl->state,
                    &pl->frames_dev, &pl->items_dev, &pl->u8_img, &pl->u8_lost, &pl->u8_out,
                    &pl->fout, &pl->staging, &pl->trace_u, &pl->trace_dc, &pl->flags_dev,
                    &pl->io_dev};
  for (DevBuf* b : bufs) b->release();
  pl->pin_in.release();
  pl->pin_out.release();
  pl->pin_flags.release();
  pl->pin_items.release();
  pl->pin_cnt.release();
  if (pl->ev_flags) (void)hipEventDestroy(pl->ev_flags);
  if (pl->ev_items) (void)hipEventDestroy(pl->ev_items);
  delete pl->pool;
  pl->pool = nullptr;
  if (pl->own_stream && pl->stream) (void)hipStreamDestroy(pl->stream);
  delete pl;
  return FSE_OK;
}

int32_t fse_conceal_image(fse_plan_t pl, const fse_frame* frames, int32_t n) {
  if (!pl || !frames || n < 1 || n > kItemFrameMask) return FSE_ERR_INVALID;
  const bool dev = (pl->p.flags & FSE_FLAG_DEVICE_PTRS) != 0;
  for (int f = 0; f < n; ++f) {
    int rc = validate_frame(&frames[f], dev);
    if (rc) return rc;
  }
  std::lock_guard<std::mutex> lk(pl->exec_mu);
  if (pl->sticky) return pl->sticky;
  if (hipSetDevice(pl->device) != hipSuccess) return FSE_ERR_DEVICE;
  auto t0 = std::chrono::steady_clock::now();
  int rc = conceal_batch(pl, frames, n, false);
  auto t1 = std::chrono::steady_clock::now();
  pl->last.total_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  if (rc == FSE_ERR_DEVICE) pl->sticky = rc;
  return rc;
}

int32_t fse_conceal_image_noalloc(fse_plan_t pl, const fse_frame* frames, int32_t n) {
  if (!pl || !frames || n < 1 || n > kItemFrameMask) return FSE_ERR_INVALID;
  if (!(pl->p.flags & FSE_FLAG_DEVICE_PTRS)) return FSE_ERR_INVALID;
  for (int f = 0; f < n; ++f) {
    int rc = validate_frame(&frames[f], true);
    if (rc) return rc;
    if (frames[f].trace) return FSE_ERR_INVALID;
  }
  std::lock_guard<std::mutex> lk(pl->exec_mu);
  if (pl->sticky) return pl->sticky;
  if (!pl->scratch) return FSE_ERR_DEVICE;
  if (hipSetDevice(pl->device) != hipSuccess) return FSE_ERR_DEVICE;
  // the call's device buffers become slices of the scratch; the plan's own
  // buffers are set aside and restored afterwards
  ScratchArena ar;
  ar.base = (char*)pl->scratch;
  ar.size = (size_t)FSE_NOALLOC_SCRATCH_BYTES;
  DevBuf* bufs[] = {&pl->work, &pl->state, &pl->frames_dev, &pl->io_dev, &pl->flags_dev,
                    &pl->items_dev, &pl->staging, &pl->spec64, &pl->counters};
  DevBuf saved[sizeof(bufs) / sizeof(bufs[0])];
  for (size_t i = 0; i < sizeof(bufs) / sizeof(bufs[0]); ++i) {
    saved[i] = *bufs[i];
    *bufs[i] = DevBuf();
  }
  set_thread_arena(&ar);
  auto t0 = std::chrono::steady_clock::now();
  int rc = conceal_batch(pl, frames, n, true);
  auto t1 = std::chrono::steady_clock::now();
  set_thread_arena(nullptr);
  for (size_t i = 0; i < sizeof(bufs) / sizeof(bufs[0]); ++i) *bufs[i] = saved[i];
  pl->last.total_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  if (rc == FSE_ERR_DEVICE) pl->sticky = rc;
  return rc;
}

int32_t fse_schedule(int32_t hb, int32_t wb, const uint8_t* lost, int32_t order,
                     int32_t* wave_of, int32_t* seq) {
  if (hb < 0 || wb < 0 || (hb * (int64_t)wb > 0 && (!lost || !wave_of))) return FSE_ERR_INVALID;
  if (order != FSE_ORDER_OPTIMIZED && order != FSE_ORDER_LINESCAN) return FSE_ERR_INVALID;
  if (hb == 0 || wb == 0) return 0;
  std::vector<int32_t> s;
  int nw = schedule_blocks(hb, wb, lost, order, wave_of, seq ? &s : nullptr);
  if (seq) std::copy(s.begin(), s.end(), seq);
  return nw;
}

int32_t fse_schedule_refined(int32_t hb, int32_t wb, const int32_t* unknown, int32_t outside,
                             int32_t* wave_of, int32_t* seq) {
  if (hb < 0 || wb < 0 || outside < 0 || (hb * (int64_t)wb > 0 && (!unknown || !wave_of)))
    return FSE_ERR_INVALID;
  if (hb == 0 || wb == 0) return 0;
  std::vector<int32_t> s;
  int nw = schedule_blocks_refined(hb, wb, unknown, outside, wave_of, seq ? &s : nullptr);
  if (seq) std::copy(s.begin(), s.end(), seq);
  return nw;
}

int32_t fse_plan_get_tuning(fse_plan_t pl, fse_tuning* out) {
  if (!pl || !out) return FSE_ERR_INVALID;
  out->wave_threshold_16 = pl->wide_threshold.load();
  out->wave_threshold_8 = pl->mid_threshold.load();
  out->frame_groups = pl->group_count();
  out->crit_depth = pl->crit_depth();
  out->crit_prio = pl->crit_prio.load() ? 1 : 0;
  {
    const int c = pl->crit_waves.load();
    out->crit_waves = c >= 0 ? c : 4;
  }
  return FSE_OK;
}

int32_t fse_plan_set_tuning(fse_plan_t pl, const fse_tuning* t) {
  if (!pl || !t) return FSE_ERR_INVALID;
  if (t->wave_threshold_16 < 0 || t->wave_threshold_8 < 0 || t->frame_groups < 0 ||
      t->frame_groups > 16 || !(t->crit_depth <= 1.0) || (t->crit_prio != 0 && t->crit_prio != 1) ||
      (t->crit_waves >= 0 && t->crit_waves != 0 && t->crit_waves != 4 && t->crit_waves != 8 &&
       t->crit_waves != 16))
    return FSE_ERR_INVALID;
  pl->wide_threshold = t->wave_threshold_16;
  pl->mid_threshold = t->wave_threshold_8;
  pl->groups = t->frame_groups;
  pl->crit = t->crit_depth < 0.0 ? -1.0 : t->crit_depth;
  pl->crit_prio = t->crit_prio != 0;
  pl->crit_waves = t->crit_waves < 0 ? -1 : t->crit_waves;
  return FSE_OK;
}

int32_t fse_last_call_stats(fse_plan_t pl, fse_call_stats* out) {
  if (!pl || !out) return FSE_ERR_INVALID;
  *out = pl->last;
  return FSE_OK;
}

const char* fse_strerror(int32_t code) {
  switch (code) {
    case FSE_OK: return "ok";
    case FSE_PENDING: return "pending";
    case FSE_ERR_INVALID: return "invalid argument";
    case FSE_ERR_UNSUPPORTED: return "unsupported by this build";
    case FSE_ERR_NOMEM: return "does not fit the device memory budget";
    case FSE_ERR_AGAIN: return "serving queue full, retry";
    case FSE_ERR_DEVICE: return "HIP device error";
    case FSE_ERR_TICKET: return "unknown ticket";
    default: return "unknown error code";
  }
}

}  // extern "C"
