// Launchers of the double-double refinement by simultaneous first-order corrections.
#pragma once
#include "common.h"

namespace mpsk {

// One refinement pass for each listed task (ents[].sweep = the task's pass index):
// flags[pass % 3] receives 0 (converged: the applied correction was the last one
// needed), bit 0 (another pass needed) or bit 1 (a near-degenerate pair: nothing
// was applied, the pairwise dd Jacobi polish must take over).
hipError_t launch_ddref_pass(Task2* d_tasks, const Ent* d_ents, int nent, int maxM, int maxN, double tol_mult,
                             hipStream_t st);
// zero the three rotation flags of each listed task
hipError_t launch_flags_clear(Task2* d_tasks, const Ent* d_ents, int nent, hipStream_t st);

}  // namespace mpsk
