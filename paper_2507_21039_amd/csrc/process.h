// Run-time parameters shared by all generated processes.
#pragma once

namespace hme {

// Masses, widths and electroweak couplings derived on the host from the SM card
// (mZ, width Z, 1/alpha, G_F, m_top, width top).  The strong coupling is not
// here: every QCD amplitude is computed with g_s = 1 and |M|^2 is scaled by
// g_s^(2n) once per event.
struct ProcParams {
  double mT;      // top mass (internal top propagators use zero width)
  double mZ, wZ;  // Z mass and width (s-channel Z only)
  double gL, gR;  // Z couplings to charged leptons: -1/2 + sin^2(thetaW), sin^2(thetaW)
  double cA, cZ;  // e^2 and e^2 / (sin^2 cos^2) for the photon and Z exchange
  double gLu, gRu;  // Z couplings to up quarks: 1/2 - 2/3 sin^2(thetaW), -2/3 sin^2(thetaW)
};

}  // namespace hme
