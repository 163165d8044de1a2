// Launchers of the three-site gate kernels.
#pragma once
#include "common.h"

namespace mpsk {

// T1 = B_s B_{s+1}, then theta (2a x 4d) with the U(8) mix; FP64 or dd
hipError_t launch_theta3(Task2* d_tasks, const Ent* d_ents, int nent, int maxA, int maxC, int maxD, bool dd,
                         hipStream_t st);
// theta of split 2 from the finished split 1 (ents[i] = {split-1 slot, split-2 slot})
hipError_t launch_mid3(Task2* d_tasks, const Ent* d_ents, int nent, int maxN1, int maxK1, bool dd, hipStream_t st);

}  // namespace mpsk
