// Double-double (hi + lo) variants of the gate-update kernels.
#pragma once
#include "common.h"
#include "launch.h"

namespace mpsk {

bool dd_available();
hipError_t launch_gate1_dd(Task1* d_tasks, int ntask, long maxel, hipStream_t st);
hipError_t launch_theta2_dd(Task2* d_tasks, const Ent* d_ents, int nent, int maxM, int maxN, hipStream_t st);
hipError_t launch_dd_enter(Task2* d_tasks, const Ent* d_ents, int nent, int maxM, int maxN, hipStream_t st);
hipError_t launch_jacobi_step_dd(Task2* d_tasks, const Ent* d_ents, int nent, int maxN, int step, double tol_mult,
                                 int maxin, hipStream_t st);
hipError_t launch_znorm_dd(Task2* d_tasks, const Ent* d_ents, int nent, int maxJM, int maxK, hipStream_t st);
// chi_max and eps are read from each task
hipError_t launch_truncate_dd(Task2* d_tasks, const Ent* d_ents, int nent, double floor_rel, hipStream_t st);
hipError_t launch_split_dd(Task2* d_tasks, const Ent* d_ents, int nent, int maxM, int maxN, int maxK, hipStream_t st,
                           bool right = true);
hipError_t launch_amplitude_dd(const AmpArgs& args, const double2* const* B_lo, int count, hipStream_t st);

}  // namespace mpsk
