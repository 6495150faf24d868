// fse_internal.h -- plan object and helpers shared by the host runtime files.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "fse.h"

namespace fse {

// Bump allocator over a fixed device region (the scratch of the noalloc entry
// point): while a thread has one set, DevBuf::reserve carves from it.
struct ScratchArena {
  char* base = nullptr;
  size_t size = 0;
  size_t used = 0;
};
void set_thread_arena(ScratchArena* a);

// Grow-only device allocation (or a slice of the thread's scratch arena).
struct DevBuf {
  void* ptr = nullptr;
  size_t cap = 0;
  int reserve(size_t bytes);        // grows with 25 % slack
  int reserve_exact(size_t bytes);  // grows to exactly `bytes` (for memory budgets)
  void release();
};

// Grow-only pinned host allocation.
struct HostBuf {
  void* ptr = nullptr;
  size_t cap = 0;
  int reserve(size_t bytes);
  void release();
};

// Persistent host worker threads of a plan: run(n, fn) calls fn(0..n-1) on the
// workers and the calling thread and returns when all calls have returned.
// One run at a time (the plan serializes its synchronous calls).
class HostPool {
 public:
  explicit HostPool(int workers);
  ~HostPool();
  void run(int n, const std::function<void(int)>& fn);

 private:
  void worker();
  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(int)>* fn_ = nullptr;
  int n_ = 0;
  std::atomic<int> next_{0};
  int active_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};

struct Serving;

int validate_params(const fse_params* p);
int validate_frame(const fse_frame* f, bool device_ptrs);

}  // namespace fse

struct fse_plan_s {
  fse_params p;
  int M = 0, N = 0, device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<double> radial;  // M*N, rho^dist (Eq. (2))
  std::vector<double> twid;    // 64 x (cos, sin)(2 pi t / 64)
  fse::DevBuf tbl_radial, tbl_twid, tbl_twid64, tbl_radial64;
  fse::DevBuf spec64;          // FP64 spectra of a step (re-rank mode)
  fse::DevBuf counters;        // re-scoring statistics of a call (kCntSlots x uint64)
  fse::DevBuf work, state, frames_dev, items_dev, u8_img, u8_lost, u8_out, fout, staging,
      trace_u, trace_dc, flags_dev, io_dev;
  fse::HostBuf pin_in, pin_out;  // pinned staging of host frames (inputs, 8-bit outputs)
  // pinned staging of the lost-block flags (device frames) and of the work
  // items of a call; ev_flags / ev_items mark their copies done
  fse::HostBuf pin_flags, pin_items;
  fse::HostBuf pin_cnt;  // pinned copy of the re-scoring statistics
  hipEvent_t ev_flags = nullptr, ev_items = nullptr;
  bool items_recorded = false;
  fse::HostPool* pool = nullptr;  // host workers (scheduling, host frame copies)
  std::vector<hipEvent_t> events;
  // wavefronts per block by launch size: at most wide_threshold blocks -> 16,
  // at most mid_threshold -> 8, else 4 (fewer blocks than the GPU holds leave
  // SIMDs idle; more wavefronts per block shorten each block's iteration)
  // (the tuning fields are atomic: fse_plan_set_tuning may change them while
  // the serving worker issues launches).  128: the autotuner's best on the
  // 64-frame batch in the FP32 modes (1-2 % ahead of 256); the re-rank mode
  // takes 0 and 128 instead (fse_plan), measured faster in batches and in
  // serving
  std::atomic<int> wide_threshold{128};
  std::atomic<int> mid_threshold{0};
  int waves_for(int64_t n_items) const {
    return n_items <= wide_threshold.load(std::memory_order_relaxed)
               ? 16
               : (n_items <= mid_threshold.load(std::memory_order_relaxed) ? 8 : 4);
  }
  bool stagger = true;       // staggered frame starts inside a batch
  // frames of a batch run in up to `groups` groups on streams of their own
  // (0: the default, 3, measured on MI355X with the 64-frame batch in every
  // precision; with the critical group below, 3 groups ran 2-8 % ahead of 2
  // and 4; 3 streams also fit HIP's default 4 hardware queues)
  std::atomic<int> groups{0};
  int group_count() const {
    const int g = groups.load(std::memory_order_relaxed);
    return g > 0 ? g : 3;
  }
  // frames whose schedule has at least crit_depth() x the waves of the
  // deepest frame of a batch form group 0 (when there are other frames): their
  // chain of waves bounds the batch, so they start first, their launches take
  // a wavefront count of their own (crit_waves) instead of the step total's,
  // and their workgroups raise their wave priority (crit_prio).  0 = off;
  // < 0 = the default, 0.9 (measured on MI355X with the 64-frame batch: 7-20 %
  // ahead of no critical group in every precision)
  std::atomic<double> crit{-1.0};
  double crit_depth() const {
    const double c = crit.load(std::memory_order_relaxed);
    return c >= 0.0 ? c : 0.9;
  }
  std::atomic<bool> crit_prio{true};
  // wavefronts per block of group 0's launches: 4/8/16; 0 = waves_for() of
  // the group's own launch size; < 0 = the default, 4 (measured on MI355X
  // with the 64-frame batch: 16 wavefronts shorten a block's iterations but
  // cost 1.7x its vector instructions, and group 0 shares the GPU with the
  // other groups)
  std::atomic<int> crit_waves{-1};
  int crit_waves_for(int64_t n_items) const {
    int c = crit_waves.load(std::memory_order_relaxed);
    if (c < 0) c = 4;
    return c > 0 ? c : waves_for(n_items);
  }
  std::vector<hipStream_t> gstreams;
  std::vector<hipEvent_t> gjoin;
  // launch cost model used to stagger frames: max(latency, blocks / rate),
  // [0] = FP64, [1] = FP32; measured on MI355X for 16x16 blocks, d = 14, K = 200
  double model_latency_us[2] = {260.0, 150.0};
  double model_rate[2] = {1.0, 3.1};  // blocks per microsecond
  fse_call_stats last{};
  int sticky = 0;
  std::mutex exec_mu;  // one synchronous call at a time
  fse::Serving* serving = nullptr;
  void* scratch = nullptr;  // device address of the noalloc scratch on this plan's device
};

namespace fse {
int conceal_batch(fse_plan_s* pl, const fse_frame* frames, int n, bool noalloc);
// Device address of the noalloc scratch on the current device (the array is a
// file-scope __device__ symbol of the kernel file).
hipError_t noalloc_scratch_address(void** out);
int serving_init(fse_plan_s* pl);
void serving_shutdown(fse_plan_s* pl);
}  // namespace fse
