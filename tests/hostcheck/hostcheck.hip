// Test-only: evaluates the generated process code on the host CPU (all helicities,
// no filter) so the generator can be checked against the oracle without a GPU.
// The library never uses this; its only compute path is the GPU kernel.
#include <cstdint>
#include <string>

#include "../../paper_2507_21039_amd/csrc/params.h"
#include "../../paper_2507_21039_amd/csrc/procs/eemumu.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggtt.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggttg.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggttgg.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggttg_fd.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggttgg_fd.h"
#include "../../paper_2507_21039_amd/csrc/procs/uuee.h"
#include "../../paper_2507_21039_amd/csrc/procs/uueeg.h"
#include "../../paper_2507_21039_amd/csrc/procs/uueegg.h"
#include "../../paper_2507_21039_amd/csrc/procs/uueeggg.h"

namespace {
template <class Proc, class T>
void run(const hme::ProcParams& prm, double alpha_s, int64_t nevt, const double* mom, double* out, double* per_hel) {
  const double pi = 3.14159265358979323846;
  double norm = 1.0 / (Proc::iden * Proc::colour_denom);
  for (int k = 0; k < Proc::gs_power / 2; ++k) norm *= 4 * pi * alpha_s;
  for (int64_t e = 0; e < nevt; ++e) {
    double p[Proc::npar][4];
    for (int k = 0; k < Proc::npar; ++k)
      for (int mu = 0; mu < 4; ++mu) p[k][mu] = mom[(e * Proc::npar + k) * 4 + mu];
    T tab[Proc::ntab > 0 ? Proc::ntab : 1];
    double sums[8 * (Proc::nsum > 0 ? Proc::nsum : 1)];
    for (int i = 0; i < Proc::nsum; ++i) Proc::momentum_sum(p, i, sums);
    for (int j = 0; j < Proc::nitems; ++j) Proc::table_entry(p, prm, j, sums, tab);
    for (int i = 0; i < 4 * Proc::nrec; ++i) Proc::template recycled_entry<T>(i, (hme::tab_of<T>)tab, tab);
    double acc = 0;
    for (int h = 0; h < Proc::nhel; ++h) {
      hme::cx<T> jamp[Proc::ncol];
      for (auto& j : jamp) j = {T(0), T(0)};
      Proc::template amplitudes<T>(p, prm, (unsigned)h, (hme::tab_of<T>)tab, jamp);
      const double v = (double)Proc::template colour_sum<T>(jamp) * norm;
      if (per_hel) per_hel[e * Proc::nhel + h] = v;
      acc += v;
    }
    out[e] = acc;
  }
}
template <class Proc>
void jamps(const hme::ProcParams& prm, const double* mom, int h, double* out) {
  double p[Proc::npar][4];
  for (int k = 0; k < Proc::npar; ++k)
    for (int mu = 0; mu < 4; ++mu) p[k][mu] = mom[k * 4 + mu];
  double tab[Proc::ntab > 0 ? Proc::ntab : 1];
  double sums[8 * (Proc::nsum > 0 ? Proc::nsum : 1)];
  for (int i = 0; i < Proc::nsum; ++i) Proc::momentum_sum(p, i, sums);
  for (int j = 0; j < Proc::nitems; ++j) Proc::table_entry(p, prm, j, sums, tab);
  for (int i = 0; i < 4 * Proc::nrec; ++i) Proc::template recycled_entry<double>(i, (hme::tab_ptr)tab, tab);
  hme::cx<double> jamp[Proc::ncol];
  for (auto& j : jamp) j = {0.0, 0.0};
  Proc::template amplitudes<double>(p, prm, (unsigned)h, (hme::tab_ptr)tab, jamp);
  for (int c = 0; c < Proc::ncol; ++c) out[2 * c] = jamp[c].r, out[2 * c + 1] = jamp[c].i;
}
struct HostChannels {
  double* w;
  template <class C> void term(int d, const C& a) const { w[d] += (double)a.r * a.r + (double)a.i * a.i; }
};

// per-diagram sum over all helicities and terms of |a|^2 (unnormalised), FP64
template <class Proc>
void channels(const hme::ProcParams& prm, int64_t nevt, const double* mom, double* out) {
  for (int64_t e = 0; e < nevt; ++e) {
    double p[Proc::npar][4];
    for (int k = 0; k < Proc::npar; ++k)
      for (int mu = 0; mu < 4; ++mu) p[k][mu] = mom[(e * Proc::npar + k) * 4 + mu];
    double tab[Proc::ntab > 0 ? Proc::ntab : 1];
    double sums[8 * (Proc::nsum > 0 ? Proc::nsum : 1)];
    for (int i = 0; i < Proc::nsum; ++i) Proc::momentum_sum(p, i, sums);
    for (int j = 0; j < Proc::nitems; ++j) Proc::table_entry(p, prm, j, sums, tab);
    for (int i = 0; i < 4 * Proc::nrec; ++i) Proc::template recycled_entry<double>(i, (hme::tab_ptr)tab, tab);
    double* w = out + e * Proc::ndiag;
    for (int d = 0; d < Proc::ndiag; ++d) w[d] = 0;
    for (int h = 0; h < Proc::nhel; ++h) {
      hme::cx<double> jamp[Proc::ncol];
      for (auto& j : jamp) j = {0.0, 0.0};
      Proc::template amplitudes<double>(p, prm, (unsigned)h, (hme::tab_ptr)tab, jamp, HostChannels{w});
    }
  }
}
}  // namespace

extern "C" int hostcheck_channels(int process, const double* card, int64_t nevt, const double* mom, double* out) {
  hme_sm_card c{card[0], card[1], card[2], card[3], card[4], card[5]};
  hme::ProcParams prm;
  std::string why;
  if (!hme::derive_params(c, prm, why)) return -1;
  switch (process) {
    case 1: channels<hme::P_ggtt>(prm, nevt, mom, out); break;
    case 2: channels<hme::P_ggttg>(prm, nevt, mom, out); break;
    case 3: channels<hme::P_ggttgg>(prm, nevt, mom, out); break;
    case 5: channels<hme::P_uuee>(prm, nevt, mom, out); break;
    case 6: channels<hme::P_uueeg>(prm, nevt, mom, out); break;
    case 7: channels<hme::P_uueegg>(prm, nevt, mom, out); break;
    case 8: channels<hme::P_uueeggg>(prm, nevt, mom, out); break;
    default: return -1;
  }
  return 0;
}

// the colour-flow amplitudes (jamps, FP64) of one event and one helicity
extern "C" int hostcheck_jamps(int process, const double* card, const double* mom, int h, double* out) {
  hme_sm_card c{card[0], card[1], card[2], card[3], card[4], card[5]};
  hme::ProcParams prm;
  std::string why;
  if (!hme::derive_params(c, prm, why)) return -1;
  switch (process) {
    case 1: jamps<hme::P_ggtt>(prm, mom, h, out); break;
    case 2: jamps<hme::P_ggttg>(prm, mom, h, out); break;
    case 3: jamps<hme::P_ggttgg>(prm, mom, h, out); break;
    case 5: jamps<hme::P_uuee>(prm, mom, h, out); break;
    case 6: jamps<hme::P_uueeg>(prm, mom, h, out); break;
    case 7: jamps<hme::P_uueegg>(prm, mom, h, out); break;
    case 8: jamps<hme::P_uueeggg>(prm, mom, h, out); break;
    default: return -1;
  }
  return 0;
}

extern "C" int hostcheck_me2(int process, int precision, const double* card, double alpha_s, int64_t nevt,
                             const double* mom, double* out, double* per_hel) {
  hme_sm_card c{card[0], card[1], card[2], card[3], card[4], card[5]};
  hme::ProcParams prm;
  std::string why;
  if (!hme::derive_params(c, prm, why)) return -1;
  const bool f64 = precision != 1;
  switch (process) {
    case 0: f64 ? run<hme::P_eemumu, double>(prm, alpha_s, nevt, mom, out, per_hel)
                : run<hme::P_eemumu, float>(prm, alpha_s, nevt, mom, out, per_hel); break;
    case 1: f64 ? run<hme::P_ggtt, double>(prm, alpha_s, nevt, mom, out, per_hel)
                : run<hme::P_ggtt, float>(prm, alpha_s, nevt, mom, out, per_hel); break;
    case 2: f64 ? run<hme::P_ggttg, double>(prm, alpha_s, nevt, mom, out, per_hel)
                : run<hme::P_ggttg, float>(prm, alpha_s, nevt, mom, out, per_hel); break;
    case 3: f64 ? run<hme::P_ggttgg, double>(prm, alpha_s, nevt, mom, out, per_hel)
                : run<hme::P_ggttgg, float>(prm, alpha_s, nevt, mom, out, per_hel); break;
    case 102: f64 ? run<hme::P_ggttg_fd, double>(prm, alpha_s, nevt, mom, out, per_hel)
                  : run<hme::P_ggttg_fd, float>(prm, alpha_s, nevt, mom, out, per_hel); break;
    case 103: f64 ? run<hme::P_ggttgg_fd, double>(prm, alpha_s, nevt, mom, out, per_hel)
                  : run<hme::P_ggttgg_fd, float>(prm, alpha_s, nevt, mom, out, per_hel); break;
    case 5: f64 ? run<hme::P_uuee, double>(prm, alpha_s, nevt, mom, out, per_hel)
                : run<hme::P_uuee, float>(prm, alpha_s, nevt, mom, out, per_hel); break;
    case 6: f64 ? run<hme::P_uueeg, double>(prm, alpha_s, nevt, mom, out, per_hel)
                : run<hme::P_uueeg, float>(prm, alpha_s, nevt, mom, out, per_hel); break;
    case 7: f64 ? run<hme::P_uueegg, double>(prm, alpha_s, nevt, mom, out, per_hel)
                : run<hme::P_uueegg, float>(prm, alpha_s, nevt, mom, out, per_hel); break;
    case 8: f64 ? run<hme::P_uueeggg, double>(prm, alpha_s, nevt, mom, out, per_hel)
                : run<hme::P_uueeggg, float>(prm, alpha_s, nevt, mom, out, per_hel); break;
    default: return -1;
  }
  return 0;
}
