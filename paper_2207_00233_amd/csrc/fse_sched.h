// fse_sched.h -- block processing orders (paper Section 2 and Algorithm 1).
#pragma once
#include <cstdint>
#include <vector>

namespace fse {

// Wave index per block of an hb x wb grid (-1 for blocks without losses);
// `seq` (nullable) receives the lost blocks in processing order.  order: 0 =
// Algorithm 1, 1 = line scan.  Returns the number of waves.
int schedule_blocks(int hb, int wb, const uint8_t* lost, int order, int32_t* wave_of,
                    std::vector<int32_t>* seq);

// Start offsets (in launch steps) for the frames of a batch; sizes[f][t] is the
// number of blocks of wave t of frame f.  See fse_sched.cpp.
std::vector<int> stagger_frames(const std::vector<std::vector<int>>& sizes, double latency_us,
                                double blocks_per_us);

}  // namespace fse
