// Derivation of the run-time parameters from the SM card.
#pragma once

#include <cmath>
#include <string>

#include "../../include/hme.h"
#include "process.h"

namespace hme {

// sin^2(thetaW) from (mZ, alpha, G_F): mW^2 = mZ^2/2 + sqrt(mZ^4/4 - pi alpha mZ^2 / (sqrt(2) G_F)),
// cos^2 = mW^2 / mZ^2; e^2 = 4 pi alpha; lepton Z couplings gL = -1/2 + sin^2, gR = sin^2;
// up-quark Z couplings gL = 1/2 - 2/3 sin^2, gR = -2/3 sin^2.
inline bool derive_params(const hme_sm_card& c, ProcParams& p, std::string& why) {
  if (!(c.mZ > 0) || !(c.alpha_inv > 0) || !(c.Gf > 0) || !(c.mT >= 0) || !(c.wZ >= 0)) {
    why = "card: mZ, 1/alpha, G_F must be positive and mT, wZ non-negative";
    return false;
  }
  const double pi = 3.14159265358979323846;
  const double alpha = 1.0 / c.alpha_inv;
  const double mZ2 = c.mZ * c.mZ;
  const double disc = mZ2 * mZ2 / 4 - pi * alpha * mZ2 / (std::sqrt(2.0) * c.Gf);
  if (!(disc > 0)) {
    why = "card: (mZ, alpha, G_F) give no real W mass";
    return false;
  }
  const double mW2 = mZ2 / 2 + std::sqrt(disc);
  const double cw2 = mW2 / mZ2, sw2 = 1 - cw2;
  const double e2 = 4 * pi * alpha;
  p.mT = c.mT;
  p.mZ = c.mZ;
  p.wZ = c.wZ;
  p.gL = -0.5 + sw2;
  p.gR = sw2;
  p.cA = e2;
  p.cZ = e2 / (sw2 * cw2);
  p.gLu = 0.5 - 2.0 / 3.0 * sw2;
  p.gRu = -2.0 / 3.0 * sw2;
  return true;
}

}  // namespace hme
