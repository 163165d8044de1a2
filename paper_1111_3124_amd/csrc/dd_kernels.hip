// Double-double variants (not yet enabled: every entry reports unavailability).
#include "dd_kernels.h"

namespace mpsk {

bool dd_available() { return false; }
hipError_t launch_gate1_dd(Task1*, int, long, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_theta2_dd(Task2*, int, int, int, hipStream_t) { return hipErrorNotSupported; }
int run_dd_refine(Task2*, int, int, int, int, int, double, int*, int*, hipStream_t, int*, bool*) { return -1; }
hipError_t launch_truncate_dd(Task2*, int, int, double, double, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_split_dd(Task2*, int, int, int, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_amplitude_dd(const AmpArgs&, const double2* const*, int, hipStream_t) { return hipErrorNotSupported; }

}  // namespace mpsk
