// Kernels of one process in the Feynman-diagram gauge (its own translation unit).
#include "me2_kernels.h"
#include "procs/ggttgg_fd.h"

namespace hme {

ProcInfo info_ggttgg_fd() { return make_info<P_ggttgg_fd>(); }

// precision 1 (single-precision amplitudes) has its own kernel; 0 and 2 share the
// double-precision one and differ in the colour-sum type only.
hipError_t launch_me2_ggttgg_fd(const LaunchArgs& a, int precision) {
  return precision != 1 ? launch_me2<P_ggttgg_fd, double>(a) : launch_me2<P_ggttgg_fd, float>(a);
}

}  // namespace hme
