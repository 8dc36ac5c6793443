// Test-only: the compensated (double-double) helpers as the device compiler sees them.  The
// test compiles this file for gfx950 to LLVM IR and checks that no multiply or add in them
// carries the contraction flag (a fused multiply-add formed across them breaks the
// error-free transformations).
#include "../../paper_2507_21039_amd/csrc/helas.h"

__global__ void dd_probe(const double* in, double* out) {
  hme::dd Q[4];
  for (int mu = 0; mu < 4; ++mu) Q[mu] = hme::dd_add(hme::two_sum(in[mu], in[4 + mu]), hme::two_prod(in[9], in[mu]));
  out[0] = hme::dd_minkowski_sq(Q, in[8]);
  out[1] = hme::dd_val(hme::dd_add(hme::dd_scale(2.0, Q[0]), hme::dd_neg(Q[1])));
}
