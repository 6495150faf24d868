// fse_sched.h -- block processing orders (paper Section 2 and Algorithm 1).
#pragma once
#include <cstdint>
#include <vector>

namespace fse {

// Wave index per block of an hb x wb grid (-1 for blocks without losses);
// `seq` (nullable) receives the lost blocks in processing order.  order: 0 =
// Algorithm 1, 1 = line scan (2, the refined order, takes sample counts:
// schedule_blocks_refined).  Returns the number of waves.
int schedule_blocks(int hb, int wb, const uint8_t* lost, int order, int32_t* wave_of,
                    std::vector<int32_t>* seq);

// Refined order (the sample-count criterion suggested in Section 3): as
// Algorithm 1, with N(b) = the lost, not yet extrapolated samples of the 8
// neighbours; a neighbour cell outside the image counts `outside` samples (a
// whole block).  unknown[b] = lost samples of block b (0: nothing to do).
int schedule_blocks_refined(int hb, int wb, const int32_t* unknown, int32_t outside,
                            int32_t* wave_of, std::vector<int32_t>* seq);

// Processing order of a tb x hb x wb block grid of a video volume (frames,
// rows, columns) for three-dimensional FSE: Algorithm 1 over the
// 26-neighbourhood (a missing neighbour at the volume's faces counts as not
// extrapolated), or line scan (order 1).  Same outputs as schedule_blocks.
int schedule_blocks3(int tb, int hb, int wb, const uint8_t* lost, int order, int32_t* wave_of,
                     std::vector<int32_t>* seq);

// Start offsets (in launch steps) for the frames of a batch; sizes[f][t] is the
// number of blocks of wave t of frame f.  See fse_sched.cpp.
std::vector<int> stagger_frames(const std::vector<std::vector<int>>& sizes, double latency_us,
                                double blocks_per_us);

}  // namespace fse
