// Kernels of one process (its own translation unit so processes compile in parallel).
#include "me2_kernels.h"
#include "procs/uueegg.h"

namespace hme {

ProcInfo info_uueegg() { return make_info<P_uueegg>(); }

// precision 1 (single-precision amplitudes) has its own kernel; 0 and 2 share the
// double-precision one and differ in the colour-sum type only.
hipError_t launch_me2_uueegg(const LaunchArgs& a, int precision) {
  return precision != 1 ? launch_me2<P_uueegg, double>(a) : launch_me2<P_uueegg, float>(a);
}

hipError_t launch_hel_uueegg(const double* mom, int nev, const ProcParams& prm, double* out, hipStream_t s) {
  return launch_hel<P_uueegg>(mom, nev, prm, out, s);
}

}  // namespace hme
