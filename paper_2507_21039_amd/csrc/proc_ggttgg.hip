// Kernels of one process (its own translation unit so processes compile in parallel).
#include "me2_kernels.h"
#include "procs/ggttgg.h"

namespace hme {

ProcInfo info_ggttgg() { return make_info<P_ggttgg>(); }

// precision 1 (single-precision amplitudes) has its own kernel; 0 and 2 share the
// double-precision one and differ in the colour-sum type only.
hipError_t launch_me2_ggttgg(const LaunchArgs& a, int precision) {
  return precision != 1 ? launch_me2<P_ggttgg, double>(a) : launch_me2<P_ggttgg, float>(a);
}

hipError_t launch_hel_ggttgg(const double* mom, int nev, const ProcParams& prm, double* out, hipStream_t s) {
  return launch_hel<P_ggttgg>(mom, nev, prm, out, s);
}

}  // namespace hme
