// Kernels of one process in the Feynman-diagram gauge (its own translation unit).
#include "me2_kernels.h"
#include "procs/ggttg_fd.h"

namespace hme {

ProcInfo info_ggttg_fd() { return make_info<P_ggttg_fd>(); }

// precision 1 (single-precision amplitudes) has its own kernel; 0 and 2 share the
// double-precision one and differ in the colour-sum type only.
hipError_t launch_me2_ggttg_fd(const LaunchArgs& a, int precision) {
  return precision != 1 ? launch_me2<P_ggttg_fd, double>(a) : launch_me2<P_ggttg_fd, float>(a);
}

}  // namespace hme
