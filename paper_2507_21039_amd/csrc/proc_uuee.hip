// Kernels of one process (its own translation unit so processes compile in parallel).
#include "me2_kernels.h"
#include "procs/uuee.h"

namespace hme {

ProcInfo info_uuee() { return make_info<P_uuee>(); }

// precision 1 (single-precision amplitudes) has its own kernel; 0 and 2 share the
// double-precision one and differ in the colour-sum type only.
hipError_t launch_me2_uuee(const LaunchArgs& a, int precision) {
  return precision != 1 ? launch_me2<P_uuee, double>(a) : launch_me2<P_uuee, float>(a);
}

hipError_t launch_hel_uuee(const double* mom, int nev, const ProcParams& prm, double* out, hipStream_t s) {
  return launch_hel<P_uuee>(mom, nev, prm, out, s);
}

}  // namespace hme
