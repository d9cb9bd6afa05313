// lane_br6.hip -- the lane kernel of the branch subproblem (BR6, n = 6), in a translation
// unit of its own (it compiles beside the other sources), with the LDS set-up its
// parameter blocks need.
#include <hip/hip_runtime.h>

#include "lane_kernels.hpp"

void mt_launch_br6(const LaneArgs &a, hipStream_t st) { launch_lane<mt::BR6, 6>(a, st); }

// the parameters of a 256-lane workgroup take 72 KB of LDS, above the default limit
void mt_prepare_br6()
{
    (void)hipFuncSetAttribute((const void *)lane_kernel<mt::BR6, 6>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(sizeof(double) * mt::BR6::kLdsDoubles * kLaneBlock));
}
