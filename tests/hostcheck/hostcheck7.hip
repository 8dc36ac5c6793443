// Test-only: evaluates the generated g g -> t tbar g g g pieces on the host CPU (all
// helicities, no filter): the pieces write their partial jamps to slots, the generated
// gather adds them up per flow, as the piece and colour kernels do through their
// workspace, so the split can be checked against the oracle without a GPU.  The
// library never uses this.
#include <cstdint>
#include <string>

#include "../../paper_2507_21039_amd/csrc/colour_blocked.h"
#include "../../paper_2507_21039_amd/csrc/params.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggttggg_c0.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggttggg_c1.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggttggg_c2.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggttggg_c3.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggttggg_c4.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggttggg_c5.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggttggg_c6.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggttggg_c7.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggttggg_c8.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggttggg_c9.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggttggg_c10.h"
#include "../../paper_2507_21039_amd/csrc/procs/ggttggg_c11.h"

namespace {
using P = hme::P_ggttggg;
static_assert(P::nchunk == 12, "update the piece list");

// one helicity's slots as a column the fold can write (stride 1)
template <class T> struct HostColumn {
  hme::cx<T>* slots;
  hme::cx<T> operator[](int64_t i) const { return slots[i]; }
  void put(int64_t i, hme::cx<T> v) const { slots[i] = v; }
};

// the same slots read at the device layout's offsets (entry s at s * nhel)
struct StrideNhel {
  const hme::cx<double>* slots;
  hme::cx<double> operator[](int64_t i) const { return slots[i / P::nhel]; }
};

// the pieces' partial jamps, one slot each, for one helicity; every slot written once
template <class T> struct SlotSink {
  hme::cx<T>* slots;
  bool* written;
  void put(int slot, hme::cx<T> v) {
    if (slot < 0 || slot >= P::nslot || written[slot]) throw "slot out of range or written twice";
    written[slot] = true;
    slots[slot] = v;
  }
};

template <class C, class T>
void add_piece(const hme::ProcParams& prm, unsigned h, hme::tab_of<T> tab, SlotSink<T>& sink) {
  C::template amplitudes<T>(prm, h, tab, sink);
}

template <class T>
void run(const hme::ProcParams& prm, double alpha_s, int64_t nevt, const double* mom, double* out) {
  const double pi = 3.14159265358979323846;
  double norm = 1.0 / (P::iden * P::colour_denom);
  for (int k = 0; k < P::gs_power / 2; ++k) norm *= 4 * pi * alpha_s;
  for (int64_t e = 0; e < nevt; ++e) {
    double p[P::npar][4];
    for (int k = 0; k < P::npar; ++k)
      for (int mu = 0; mu < 4; ++mu) p[k][mu] = mom[(e * P::npar + k) * 4 + mu];
    T tab[P::ntab];
    double sums[8 * P::nsum];
    for (int i = 0; i < P::nsum; ++i) P::momentum_sum(p, i, sums);
    for (int j = 0; j < P::nitems; ++j) P::table_entry(p, prm, j, sums, tab);
    for (int i = 0; i < 4 * P::nrec; ++i) P::template recycled_entry<T>(i, (hme::tab_of<T>)tab, tab);
    double acc = 0;
    for (int h = 0; h < P::nhel; ++h) {
      static hme::cx<T> slots[P::nslot];
      static bool written[P::nslot];
      for (bool& x : written) x = false;
      SlotSink<T> sink{slots, written};
      const auto t = (hme::tab_of<T>)tab;
      add_piece<hme::P_ggttggg_c0, T>(prm, h, t, sink);
      add_piece<hme::P_ggttggg_c1, T>(prm, h, t, sink);
      add_piece<hme::P_ggttggg_c2, T>(prm, h, t, sink);
      add_piece<hme::P_ggttggg_c3, T>(prm, h, t, sink);
      add_piece<hme::P_ggttggg_c4, T>(prm, h, t, sink);
      add_piece<hme::P_ggttggg_c5, T>(prm, h, t, sink);
      add_piece<hme::P_ggttggg_c6, T>(prm, h, t, sink);
      add_piece<hme::P_ggttggg_c7, T>(prm, h, t, sink);
      add_piece<hme::P_ggttggg_c8, T>(prm, h, t, sink);
      add_piece<hme::P_ggttggg_c9, T>(prm, h, t, sink);
      add_piece<hme::P_ggttggg_c10, T>(prm, h, t, sink);
      add_piece<hme::P_ggttggg_c11, T>(prm, h, t, sink);
      for (bool x : written)
        if (!x) throw "slot never written";
      if constexpr (sizeof(T) == 8) {
        // the FP64 path of the GPU: fold in place, then the blocked colour sum
        P::template fold<T>(HostColumn<T>{slots}, 1);
        acc += hme::colour_sum_blocked<P, hme::kColourBlock>(StrideNhel{slots}) * norm;
      } else {
        hme::cx<T> jamp[P::ncol];
        P::template gather<T, T>(slots, 1, jamp);
        acc += (double)P::template colour_sum<T>(jamp) * norm;
      }
    }
    out[e] = acc;
  }
}
}  // namespace

extern "C" int hostcheck7_me2(int precision, const double* card, double alpha_s, int64_t nevt, const double* mom,
                              double* out) {
  hme_sm_card c{card[0], card[1], card[2], card[3], card[4], card[5]};
  hme::ProcParams prm;
  std::string why;
  if (!hme::derive_params(c, prm, why)) return -1;
  try {
    if (precision == 1)
      run<float>(prm, alpha_s, nevt, mom, out);
    else
      run<double>(prm, alpha_s, nevt, mom, out);
  } catch (const char*) {
    return -2;
  }
  return 0;
}
