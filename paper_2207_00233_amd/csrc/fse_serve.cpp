// fse_serve.cpp -- asynchronous serving (fse_submit / fse_poll) with
// continuous batching.
//
// fse_submit copies the frame into library-owned pinned memory, derives the
// block flags (lost-sample counts) and the processing order on the caller's
// thread, and queues it.
// One worker thread per plan:
//   - admits queued frames while the device memory budget (device_mem_budget)
//     and the slot count (max_inflight_frames) allow, uploads them and builds
//     their working image and state map.  The budget covers every device
//     buffer the worker holds: the per-pixel arenas (working image, state map,
//     8-bit input, mask and output) and the per-step buffers (FP64 spectra in
//     re-rank mode, staging when d exceeds the block, work items), which get
//     a fixed share of it; a frame is admitted only while its pixels fit the
//     arenas and its largest wave fits, beside the largest waves of the frames
//     already admitted, the per-step share;
//   - launches one step at a time: a step holds the next wave of every
//     admitted frame, so frames that arrive while others run join the very
//     next steps and their work overlaps on the device;
//   - keeps at most kAhead steps in flight, so that new arrivals are not
//     queued behind a long backlog of already launched steps;
//   - finalizes a frame after its last wave, copies the result back and
//     completes its ticket.
// Every frame gets exactly the result fse_conceal_image gives it alone: a
// block only reads its own frame, and each frame's waves stay in order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "fse_device.h"
#include "fse_internal.h"
#include "fse_sched.h"

namespace fse {

template <typename T>
hipError_t launch_block(const BlockArgs<T>& a, int n_items, int waves, hipStream_t s, int mode);
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

namespace {

using Clock = std::chrono::steady_clock;
constexpr int kAhead = 2;  // launched steps the worker may run ahead of the GPU

// First-fit allocator over element offsets of the serving arenas.
class Arena {
 public:
  void reset(int64_t n) {
    free_.clear();
    if (n > 0) free_[0] = n;
    cap_ = n;
  }
  int64_t capacity() const { return cap_; }
  int64_t alloc(int64_t n) {
    n = (n + 255) & ~255LL;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const int64_t off = it->first, left = it->second - n;
        free_.erase(it);
        if (left > 0) free_[off + n] = left;
        used_[off] = n;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    int64_t n = u->second;
    used_.erase(u);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  int64_t used_elems() const {
    int64_t s = 0;
    for (auto& kv : used_) s += kv.second;
    return s;
  }

 private:
  std::map<int64_t, int64_t> free_, used_;
  int64_t cap_ = 0;
};

// Pinned host buffers reused by size.
class PinnedPool {
 public:
  ~PinnedPool() {
    for (auto& kv : free_)
      for (void* p : kv.second) (void)hipHostFree(p);
  }
  void* get(size_t bytes) {
    bytes = (bytes + 4095) & ~size_t(4095);
    auto& v = free_[bytes];
    if (!v.empty()) {
      void* p = v.back();
      v.pop_back();
      sizes_[p] = bytes;
      return p;
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
    sizes_[p] = bytes;
    return p;
  }
  void put(void* p) {
    if (!p) return;
    auto it = sizes_.find(p);
    if (it == sizes_.end()) return;
    free_[it->second].push_back(p);
    sizes_.erase(it);
  }

 private:
  std::map<size_t, std::vector<void*>> free_;
  std::unordered_map<void*, size_t> sizes_;
};

enum class St { kQueued, kActive, kFinishing, kDone, kFailed };

struct Req {
  uint64_t ticket = 0;
  fse_frame user{};          // caller's output pointers (input is copied)
  int H = 0, W = 0, hb = 0, wb = 0;
  uint8_t* pin_in = nullptr;  // image (H*W) then lost (H*W)
  uint8_t* pin_out = nullptr; // u8 out (H*W) then unquantized values (H*W*sizeof(T))
  std::vector<int32_t> seq;        // lost blocks in processing order
  std::vector<int32_t> wave_start; // start of every wave in seq, plus the end
  int nwaves = 0, next_wave = 0;
  int max_wave = 0;  // blocks of the largest wave (per-step buffer share)
  int64_t off = -1;  // element offset in the arenas
  int slot = -1;     // index in the device frame tables
  hipEvent_t done_ev = nullptr;
  St st = St::kQueued;
  int err = FSE_OK;
  Clock::time_point t_submit;
  double latency_ms = 0;
};

}  // namespace

struct Serving {
  fse_plan_s* pl = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  bool stop = false;
  bool started = false;
  int sticky = FSE_OK;
  uint64_t next_ticket = 1;
  std::deque<std::shared_ptr<Req>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Req>> all;  // submitted, not yet polled
  // worker-owned
  std::vector<std::shared_ptr<Req>> active;
  std::vector<int> free_slots;
  Arena arena;
  PinnedPool pinned;
  DevBuf d_work, d_state, d_img, d_lost, d_out, d_frames, d_io, d_staging, d_spec64;
  int64_t elem_bytes = 0;
  struct Step {
    DevBuf items;
    HostBuf host;
    hipEvent_t ev = nullptr;
    bool used = false;
  } ring[kAhead + 1];
  int ring_pos = 0;
  HostBuf host_desc;  // per-slot staging of FrameDesc + IoDesc updates
  int max_slots = 64;
  int64_t budget = 0;
  // per-step buffers: bytes per block of a step, their share of the budget in
  // blocks, and the blocks reserved for the largest waves of admitted frames
  int64_t per_block_step = 0;
  int64_t step_blocks_cap = 0;
  int64_t step_blocks = 0;
  // accounting reported by fse_serving_stats
  int64_t device_bytes = 0;   // device memory the worker holds
  int64_t peak_admitted = 0;  // most bytes ever committed to admitted frames
  int peak_frames = 0;        // most frames admitted at once
  int64_t peak_step_blocks = 0;  // most per-step blocks committed at once
  int64_t admitted_total = 0;
};

static int tsize(const fse_plan_s* pl) { return pl->p.precision == FSE_FP64 ? 8 : 4; }
// (FSE_FP32_RERANK iterates in float: its working image is float.)

int serving_init(fse_plan_s* pl) {
  Serving* sv = new Serving();
  sv->pl = pl;
  const fse_params& p = pl->p;
  sv->max_slots = p.max_inflight_frames > 0 ? p.max_inflight_frames : 64;
  sv->budget = p.device_mem_budget > 0 ? p.device_mem_budget : (int64_t)4 << 30;
  sv->elem_bytes = tsize(pl) + 4;  // work, state, image, lost, out
  // per step and block: FP64 spectra (re-rank), staged results (d > block),
  // and the work item in each of the kAhead + 1 step slots
  const bool rerank = p.precision == FSE_FP32_RERANK;
  const bool staged = p.border_d > std::min(p.block_h, p.block_w);
  sv->per_block_step = (rerank ? kSpecStride * (int64_t)sizeof(double) : 0) +
                       (staged ? (int64_t)p.block_h * p.block_w * tsize(pl) : 0) +
                       (kAhead + 1) * 2 * (int64_t)sizeof(int32_t);
  // their share: a quarter of the budget when they hold spectra or staged
  // results, else 1/64 (work items only)
  const int64_t share = (rerank || staged) ? sv->budget / 4 : sv->budget / 64;
  sv->step_blocks_cap = share / sv->per_block_step;
  pl->serving = sv;
  return FSE_OK;
}

// Bytes committed to the admitted frames (caller holds mu).
static int64_t committed_bytes(const Serving* sv) {
  return sv->arena.used_elems() * sv->elem_bytes + sv->step_blocks * sv->per_block_step;
}

// Device resources are created on first use so plans used only for
// synchronous calls do not hold the serving arena.
static int serving_start(Serving* sv) {
  fse_plan_s* pl = sv->pl;
  const fse_params& p = pl->p;
  const bool rerank = p.precision == FSE_FP32_RERANK;
  const bool staged = p.border_d > std::min(p.block_h, p.block_w);
  const int64_t nb = std::max<int64_t>(1, sv->step_blocks_cap);
  // descriptors and the per-step buffers first, the pixel arenas get the rest
  const int64_t fixed = (int64_t)sv->max_slots * (sizeof(FrameDesc) + sizeof(IoDesc)) +
                        sv->step_blocks_cap * sv->per_block_step;
  const int64_t elems = std::max<int64_t>(0, sv->budget - fixed) / sv->elem_bytes;
  sv->arena.reset(elems);
  if (sv->d_work.reserve_exact(elems * tsize(pl)) || sv->d_state.reserve_exact(elems) ||
      sv->d_img.reserve_exact(elems) || sv->d_lost.reserve_exact(elems) ||
      sv->d_out.reserve_exact(elems) ||
      sv->d_frames.reserve_exact(sv->max_slots * sizeof(FrameDesc)) ||
      sv->d_io.reserve_exact(sv->max_slots * sizeof(IoDesc)) ||
      (rerank && sv->d_spec64.reserve_exact(nb * kSpecStride * sizeof(double))) ||
      (staged && sv->d_staging.reserve_exact(nb * p.block_h * p.block_w * tsize(pl))) ||
      sv->host_desc.reserve((size_t)sv->max_slots * (sizeof(FrameDesc) + sizeof(IoDesc))))
    return FSE_ERR_DEVICE;
  for (auto& st : sv->ring)
    if (st.items.reserve_exact(nb * 2 * sizeof(int32_t)) ||
        st.host.reserve(nb * 2 * sizeof(int32_t)))
      return FSE_ERR_DEVICE;
  sv->device_bytes = 0;
  for (const DevBuf* b : {&sv->d_work, &sv->d_state, &sv->d_img, &sv->d_lost, &sv->d_out,
                          &sv->d_frames, &sv->d_io, &sv->d_spec64, &sv->d_staging})
    sv->device_bytes += (int64_t)b->cap;
  for (auto& st : sv->ring) sv->device_bytes += (int64_t)st.items.cap;
  for (auto& st : sv->ring)
    if (hipEventCreateWithFlags(&st.ev, hipEventDisableTiming) != hipSuccess) return FSE_ERR_DEVICE;
  for (int s = sv->max_slots - 1; s >= 0; --s) sv->free_slots.push_back(s);
  return FSE_OK;
}

template <typename T>
static int worker_admit(Serving* sv, const std::shared_ptr<Req>& r) {
  fse_plan_s* pl = sv->pl;
  hipStream_t s = pl->stream;
  const int64_t px = (int64_t)r->H * r->W;
  T* work = (T*)sv->d_work.ptr;
  uint8_t* state = (uint8_t*)sv->d_state.ptr;
  uint8_t* img = (uint8_t*)sv->d_img.ptr + r->off;
  uint8_t* lost = (uint8_t*)sv->d_lost.ptr + r->off;
  if (hipMemcpyAsync(img, r->pin_in, px, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(lost, r->pin_in + px, px, hipMemcpyHostToDevice, s) != hipSuccess)
    return FSE_ERR_DEVICE;
  FrameDesc fd;
  fd.off = r->off;
  fd.H = r->H;
  fd.W = r->W;
  IoDesc io{};
  io.image = img;
  io.lost = lost;
  io.out = (uint8_t*)sv->d_out.ptr + r->off;
  io.off = r->off;
  io.stride = io.lstride = io.ostride = r->W;
  io.H = r->H;
  io.W = r->W;
  io.wb = r->wb;
  // descriptors go through the slot's own pinned staging area: a slot is
  // reused only after its previous frame completed, so no copy is in flight
  char* hd = (char*)sv->host_desc.ptr + (size_t)r->slot * (sizeof(fd) + sizeof(io));
  std::memcpy(hd, &fd, sizeof(fd));
  std::memcpy(hd + sizeof(fd), &io, sizeof(io));
  if (hipMemcpyAsync((FrameDesc*)sv->d_frames.ptr + r->slot, hd, sizeof(fd),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync((IoDesc*)sv->d_io.ptr + r->slot, hd + sizeof(fd), sizeof(io),
                     hipMemcpyHostToDevice, s) != hipSuccess)
    return FSE_ERR_DEVICE;
  if (launch_init<T>((const IoDesc*)sv->d_io.ptr + r->slot, 1, px, work, state, nullptr, nullptr,
                     true, pl->p.block_h, pl->p.block_w, pl->p.grid_off_x, pl->p.grid_off_y,
                     s) != hipSuccess)
    return FSE_ERR_DEVICE;
  return FSE_OK;
}

template <typename T>
static int worker_finalize(Serving* sv, const std::shared_ptr<Req>& r) {
  fse_plan_s* pl = sv->pl;
  hipStream_t s = pl->stream;
  const int64_t px = (int64_t)r->H * r->W;
  const T* work = (const T*)sv->d_work.ptr;
  if (launch_finalize<T>((const IoDesc*)sv->d_io.ptr + r->slot, 1, px,
                         (const uint8_t*)sv->d_state.ptr, work, s) != hipSuccess ||
      hipMemcpyAsync(r->pin_out, (uint8_t*)sv->d_out.ptr + r->off, px, hipMemcpyDeviceToHost,
                     s) != hipSuccess)
    return FSE_ERR_DEVICE;
  if ((r->user.out_f32 || r->user.out_f64) &&
      hipMemcpyAsync(r->pin_out + px, work + r->off, px * sizeof(T), hipMemcpyDeviceToHost, s) !=
          hipSuccess)
    return FSE_ERR_DEVICE;
  if (hipEventRecord(r->done_ev, s) != hipSuccess) return FSE_ERR_DEVICE;
  r->st = St::kFinishing;
  return FSE_OK;
}

template <typename T>
static void worker_complete(Serving* sv, const std::shared_ptr<Req>& r) {
  const int64_t px = (int64_t)r->H * r->W;
  const fse_frame& u = r->user;
  for (int y = 0; y < r->H; ++y)
    std::memcpy(u.out + (int64_t)y * u.out_stride, r->pin_out + (int64_t)y * r->W, r->W);
  const T* v = (const T*)(r->pin_out + px);
  if (u.out_f32)
    for (int64_t i = 0; i < px; ++i) u.out_f32[i] = (float)v[i];
  if (u.out_f64)
    for (int64_t i = 0; i < px; ++i) u.out_f64[i] = (double)v[i];
  r->latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - r->t_submit).count();
  if (u.stats) u.stats->latency_ms = r->latency_ms;
}

template <typename T>
static void worker_loop(Serving* sv) {
  fse_plan_s* pl = sv->pl;
  hipStream_t s = pl->stream;
  const fse_params& p = pl->p;
  (void)hipSetDevice(pl->device);
  const bool staged = p.border_d > std::min(p.block_h, p.block_w);
  BlockArgs<T> a{};
  a.work = (T*)sv->d_work.ptr;
  a.state = (uint8_t*)sv->d_state.ptr;
  a.frames = (const FrameDesc*)sv->d_frames.ptr;
  a.radial = (const T*)pl->tbl_radial.ptr;
  a.twid = (const T*)pl->tbl_twid.ptr;
  a.twid64 = (const double*)pl->tbl_twid64.ptr;
  a.M = pl->M;
  a.N = pl->N;
  a.Bh = p.block_h;
  a.Bw = p.block_w;
  a.d = p.border_d;
  a.gox = p.grid_off_x;
  a.goy = p.grid_off_y;
  a.K = p.iterations;
  a.delta = (T)p.delta;
  a.gamma = (T)p.gamma;
  a.delta64 = p.delta;
  a.gamma64 = p.gamma;
  a.zscale = (T)128.0;
  a.empty_fill = p.empty_fill;
  a.trace_u = nullptr;
  a.trace_dc = nullptr;
  a.spec64 = nullptr;
  a.radial64 = (const double*)pl->tbl_radial64.ptr;
  a.rerank_gap = p.rerank_gap > 0.0 ? p.rerank_gap : 1e-4;
  a.counters = nullptr;
  const bool rerank = p.precision == FSE_FP32_RERANK;
  const bool mx = p.precision == FSE_FP32_F16X3;  // matrix-core transforms, 4 wavefronts

  auto fail_all = [&](int err) {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->sticky = err;
    for (auto& r : sv->active) {
      r->st = St::kFailed;
      r->err = err;
    }
    for (auto& r : sv->queue) {
      r->st = St::kFailed;
      r->err = err;
    }
    sv->active.clear();
    sv->queue.clear();
    sv->cv_done.notify_all();
  };

  for (;;) {
    // ---- admission ----
    std::vector<std::shared_ptr<Req>> admitted;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      if (sv->queue.empty() && sv->active.empty())
        sv->cv_work.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
      if (sv->stop && sv->active.empty()) {
        for (auto& r : sv->queue) {
          r->st = St::kFailed;
          r->err = FSE_ERR_DEVICE;
        }
        sv->queue.clear();
        sv->cv_done.notify_all();
        return;
      }
      while (!sv->stop && !sv->queue.empty() && !sv->free_slots.empty()) {
        auto& r = sv->queue.front();
        // the frame's largest wave must fit the per-step share beside the
        // largest waves of the frames already admitted
        if (sv->step_blocks + r->max_wave > sv->step_blocks_cap) break;
        const int64_t off = sv->arena.alloc((int64_t)r->H * r->W);
        if (off < 0) break;  // wait until running frames free the arena
        sv->step_blocks += r->max_wave;
        r->off = off;
        r->slot = sv->free_slots.back();
        sv->free_slots.pop_back();
        r->st = St::kActive;
        admitted.push_back(r);
        sv->active.push_back(r);
        sv->queue.pop_front();
        sv->admitted_total += 1;
        sv->peak_admitted = std::max(sv->peak_admitted, committed_bytes(sv));
        sv->peak_frames = std::max(sv->peak_frames, (int)sv->active.size());
        sv->peak_step_blocks = std::max(sv->peak_step_blocks, sv->step_blocks);
      }
    }
    for (auto& r : admitted)
      if (worker_admit<T>(sv, r)) return fail_all(FSE_ERR_DEVICE);

    // ---- one step: the next wave of every active frame ----
    Serving::Step& stp = sv->ring[sv->ring_pos];
    if (stp.used && hipEventSynchronize(stp.ev) != hipSuccess) return fail_all(FSE_ERR_DEVICE);
    stp.used = false;
    int64_t n_items = 0;
    for (auto& r : sv->active)
      if (r->st == St::kActive && r->next_wave < r->nwaves)
        n_items += r->wave_start[r->next_wave + 1] - r->wave_start[r->next_wave];
    if (n_items > 0) {
      if (stp.host.reserve(n_items * 2 * sizeof(int32_t)) ||
          stp.items.reserve(n_items * 2 * sizeof(int32_t)) ||
          (staged && sv->d_staging.reserve(n_items * p.block_h * p.block_w * sizeof(T))) ||
          (rerank && sv->d_spec64.reserve(n_items * kSpecStride * sizeof(double))))
        return fail_all(FSE_ERR_DEVICE);
      a.spec64 = rerank ? (double*)sv->d_spec64.ptr : nullptr;
      int32_t* it = (int32_t*)stp.host.ptr;
      int64_t k = 0;
      for (auto& r : sv->active) {
        if (r->st != St::kActive || r->next_wave >= r->nwaves) continue;
        for (int q = r->wave_start[r->next_wave]; q < r->wave_start[r->next_wave + 1]; ++q) {
          const int32_t b = r->seq[q];
          it[2 * k] = r->slot;
          it[2 * k + 1] = ((b / r->wb) << 16) | (b % r->wb);
          ++k;
        }
        ++r->next_wave;
      }
      a.items = (const int32_t*)stp.items.ptr;
      a.staging = staged ? (T*)sv->d_staging.ptr : nullptr;
      const int waves = mx ? 4 : pl->waves_for(n_items);
      if (hipMemcpyAsync(stp.items.ptr, stp.host.ptr, n_items * 2 * sizeof(int32_t),
                         hipMemcpyHostToDevice, s) != hipSuccess)
        return fail_all(FSE_ERR_DEVICE);
      if (launch_block<T>(a, (int)n_items, waves, s, rerank ? 1 : (mx ? 2 : 0)) != hipSuccess)
        return fail_all(FSE_ERR_DEVICE);
      if (staged && launch_scatter<T>(a.work, a.state, a.frames, a.items, (int)n_items, a.staging,
                                      p.block_h, p.block_w, p.grid_off_x, p.grid_off_y,
                                      s) != hipSuccess)
        return fail_all(FSE_ERR_DEVICE);
      if (hipEventRecord(stp.ev, s) != hipSuccess) return fail_all(FSE_ERR_DEVICE);
      stp.used = true;
      sv->ring_pos = (sv->ring_pos + 1) % (kAhead + 1);
    }
    // ---- frames whose last wave has been launched ----
    for (auto& r : sv->active)
      if (r->st == St::kActive && r->next_wave >= r->nwaves)
        if (worker_finalize<T>(sv, r)) return fail_all(FSE_ERR_DEVICE);
    // ---- completions ----
    bool any_done = false;
    for (size_t i = 0; i < sv->active.size();) {
      auto r = sv->active[i];
      hipError_t q = r->st == St::kFinishing ? hipEventQuery(r->done_ev) : hipErrorNotReady;
      if (q == hipSuccess) {
        worker_complete<T>(sv, r);
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->arena.release(r->off);
        sv->step_blocks -= r->max_wave;
        sv->free_slots.push_back(r->slot);
        r->st = St::kDone;
        sv->active.erase(sv->active.begin() + i);
        any_done = true;
      } else if (q != hipErrorNotReady) {
        return fail_all(FSE_ERR_DEVICE);
      } else {
        ++i;
      }
    }
    if (any_done) {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->cv_done.notify_all();
    }
    // nothing launched and only finishing frames: wait for the oldest one
    if (n_items == 0 && admitted.empty() && !any_done) {
      std::shared_ptr<Req> oldest;
      for (auto& r : sv->active)
        if (r->st == St::kFinishing) {
          oldest = r;
          break;
        }
      if (oldest) {
        if (hipEventSynchronize(oldest->done_ev) != hipSuccess) return fail_all(FSE_ERR_DEVICE);
      } else {
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv_work.wait_for(lk, std::chrono::microseconds(200));
      }
    }
  }
}

void serving_shutdown(fse_plan_s* pl) {
  Serving* sv = pl->serving;
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  (void)hipStreamSynchronize(pl->stream);
  for (auto& kv : sv->all) {
    Req& r = *kv.second;
    if (r.pin_in) sv->pinned.put(r.pin_in);
    if (r.pin_out) sv->pinned.put(r.pin_out);
    if (r.done_ev) (void)hipEventDestroy(r.done_ev);
  }
  sv->all.clear();
  for (auto& st : sv->ring) {
    if (st.ev) (void)hipEventDestroy(st.ev);
    st.items.release();
    st.host.release();
  }
  DevBuf* bufs[] = {&sv->d_work, &sv->d_state, &sv->d_img, &sv->d_lost, &sv->d_out,
                    &sv->d_frames, &sv->d_io, &sv->d_staging, &sv->d_spec64};
  for (DevBuf* b : bufs) b->release();
  sv->host_desc.release();
  delete sv;
  pl->serving = nullptr;
}

}  // namespace fse

using namespace fse;

extern "C" {

int32_t fse_submit(fse_plan_t pl, const fse_frame* f, uint64_t* ticket) {
  if (!pl || !f || !ticket) return FSE_ERR_INVALID;
  if (pl->p.flags & FSE_FLAG_DEVICE_PTRS) return FSE_ERR_INVALID;
  int rc = validate_frame(f, false);
  if (rc) return rc;
  Serving* sv = pl->serving;
  const fse_params& p = pl->p;
  const int64_t px = (int64_t)f->height * f->width;
  // can never fit: more pixels than the arenas hold (checked against the
  // budget here, against the arenas once the worker has started)
  if (((px + 255) & ~255LL) > sv->budget / sv->elem_bytes) return FSE_ERR_NOMEM;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->sticky) return sv->sticky;
    int pending = (int)sv->queue.size();
    for (auto& kv : sv->all)
      if (kv.second->st == St::kActive || kv.second->st == St::kFinishing) ++pending;
    if (pending >= sv->max_slots) return FSE_ERR_AGAIN;
    if (!sv->started) {
      if (hipSetDevice(pl->device) != hipSuccess) return FSE_ERR_DEVICE;
      rc = serving_start(sv);
      if (rc) return rc;
      sv->started = true;
      if (p.precision == FSE_FP64)
        sv->worker = std::thread(worker_loop<double>, sv);
      else
        sv->worker = std::thread(worker_loop<float>, sv);
    }
  }
  auto r = std::make_shared<Req>();
  r->t_submit = Clock::now();
  r->user = *f;
  r->H = f->height;
  r->W = f->width;
  r->hb = (f->height + p.grid_off_y + p.block_h - 1) / p.block_h;
  r->wb = (f->width + p.grid_off_x + p.block_w - 1) / p.block_w;
  const size_t out_bytes = (size_t)px * (1 + tsize(pl));
  {
    std::lock_guard<std::mutex> lk(sv->mu);  // the pool is shared with the worker
    r->pin_in = (uint8_t*)sv->pinned.get(2 * px);
    r->pin_out = (uint8_t*)sv->pinned.get(out_bytes);
  }
  if (!r->pin_in || !r->pin_out || hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming) != hipSuccess) {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->pinned.put(r->pin_in);
    sv->pinned.put(r->pin_out);
    return FSE_ERR_DEVICE;
  }
  // lost samples per block (the refined order counts them; the others only
  // need to know which blocks have any)
  std::vector<int32_t> counts((size_t)r->hb * r->wb, 0);
  for (int y = 0; y < r->H; ++y) {
    std::memcpy(r->pin_in + (int64_t)y * r->W, f->image + (int64_t)y * f->stride, r->W);
    const uint8_t* lrow = f->lost + (int64_t)y * f->lost_stride;
    uint8_t* dst = r->pin_in + px + (int64_t)y * r->W;
    const int bi = (y + p.grid_off_y) / p.block_h;
    int x = 0;
    for (; x + 8 <= r->W; x += 8) {  // skip runs of known samples 8 at a time
      uint64_t w8;
      std::memcpy(&w8, lrow + x, 8);
      if (!w8) {
        std::memset(dst + x, 0, 8);
        continue;
      }
      for (int q = x; q < x + 8; ++q) {
        dst[q] = lrow[q] ? 1 : 0;
        if (lrow[q]) counts[(size_t)bi * r->wb + (q + p.grid_off_x) / p.block_w] += 1;
      }
    }
    for (; x < r->W; ++x) {
      dst[x] = lrow[x] ? 1 : 0;
      if (lrow[x]) counts[(size_t)bi * r->wb + (x + p.grid_off_x) / p.block_w] += 1;
    }
  }
  std::vector<int32_t> wave_of(counts.size());
  if (p.order == FSE_ORDER_REFINED) {
    r->nwaves = schedule_blocks_refined(r->hb, r->wb, counts.data(), p.block_h * p.block_w,
                                        wave_of.data(), &r->seq);
  } else {
    std::vector<uint8_t> flags(counts.size());
    for (size_t b = 0; b < counts.size(); ++b) flags[b] = counts[b] > 0;
    r->nwaves = schedule_blocks(r->hb, r->wb, flags.data(), p.order, wave_of.data(), &r->seq);
  }
  r->wave_start.assign(r->nwaves + 1, 0);
  for (size_t q = 0, t = 0; t <= (size_t)r->nwaves; ++t) {
    while (q < r->seq.size() && wave_of[r->seq[q]] < (int)t) ++q;
    r->wave_start[t] = (int32_t)q;
  }
  for (int t = 0; t < r->nwaves; ++t)
    r->max_wave = std::max(r->max_wave, r->wave_start[t + 1] - r->wave_start[t]);
  if (f->stats) {
    f->stats->waves = r->nwaves;
    f->stats->lost_blocks = (int32_t)r->seq.size();
    f->stats->max_wave_blocks = r->max_wave;
    f->stats->latency_ms = 0.0;
  }
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    // a frame whose pixels or largest wave exceed what the budget ever holds
    const bool too_big = r->max_wave > sv->step_blocks_cap ||
                         (sv->started && ((px + 255) & ~255LL) > sv->arena.capacity());
    if (too_big) {
      sv->pinned.put(r->pin_in);
      sv->pinned.put(r->pin_out);
      (void)hipEventDestroy(r->done_ev);
      return FSE_ERR_NOMEM;
    }
  }
  if (f->trace) f->trace->count = 0;  // traces are recorded by fse_conceal_image only
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    r->ticket = sv->next_ticket++;
    sv->queue.push_back(r);
    sv->all[r->ticket] = r;
    *ticket = r->ticket;
  }
  sv->cv_work.notify_all();
  return FSE_OK;
}

int32_t fse_plan_serving_stats(fse_plan_t pl, fse_serving_stats* out) {
  if (!pl || !out) return FSE_ERR_INVALID;
  Serving* sv = pl->serving;
  std::lock_guard<std::mutex> lk(sv->mu);
  out->budget = sv->budget;
  out->device_bytes = sv->started ? sv->device_bytes : 0;
  out->peak_committed = sv->peak_admitted;
  out->admitted_frames = sv->admitted_total;
  out->peak_frames = sv->peak_frames;
  out->reserved = 0;
  out->step_blocks_cap = sv->step_blocks_cap;
  out->peak_step_blocks = sv->peak_step_blocks;
  return FSE_OK;
}

int32_t fse_poll(fse_plan_t pl, uint64_t ticket, int32_t timeout_us) {
  if (!pl) return FSE_ERR_INVALID;
  Serving* sv = pl->serving;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return FSE_ERR_TICKET;
  auto r = it->second;
  auto done = [&] { return r->st == St::kDone || r->st == St::kFailed; };
  if (!done() && timeout_us != 0) {
    if (timeout_us < 0)
      sv->cv_done.wait(lk, done);
    else
      sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done);
  }
  if (!done()) return FSE_PENDING;
  const int rc = r->st == St::kDone ? FSE_OK : r->err;
  sv->pinned.put(r->pin_in);
  sv->pinned.put(r->pin_out);
  r->pin_in = r->pin_out = nullptr;
  if (r->done_ev) (void)hipEventDestroy(r->done_ev);
  r->done_ev = nullptr;
  sv->all.erase(it);
  return rc;
}

}  // extern "C"
