// |M|^2 kernels: one event per group of LPE lanes, one good helicity per lane.
//
// A wavefront of 64 lanes holds 64 / LPE events.  Lane j of an event evaluates
// the good helicities j, j + LPE, ... (the paper's helicity sum over
// non-vanishing spin configurations, section "Parallel scattering amplitudes"):
// external wavefunctions, the generated diagram sequence, the jamps and their
// colour sum, all in registers.  The per-helicity |M_h|^2 are then summed
// across the LPE lanes with butterfly shuffles in FP64, scaled by
// g_s^(2n) / (IDEN * colour denominator), and lane 0 of the group stores the
// event's result.  With LPE = 64 every lane of a wavefront reads the same
// event record, so the momenta are wave-uniform.  The helicity-independent
// quantities (momentum sums, propagator denominators) are computed once per
// event by its lanes into an LDS table before the helicity loop.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "colour_mfma.h"
#include "helas.h"
#include "process.h"

namespace hme {

template <class Proc>
HME_FN void load_event(const double* __restrict__ mom, int64_t ev, double (&p)[Proc::npar][4]) {
  const double* src = mom + ev * (Proc::npar * 4);
#pragma unroll
  for (int k = 0; k < Proc::npar; ++k)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) p[k][mu] = src[k * 4 + mu];
}

template <class T> constexpr int me2_min_waves() { return sizeof(T) == 4 ? 3 : 2; }

// Per-event choice of one helicity and one colour flow from caller-supplied uniform numbers
// (the information an event generator keeps with each event; section "Event generation
// interface").  Helicity: the first good helicity, in increasing index order, whose running
// sum of |M_h|^2 exceeds rnd_hel x sum_h |M_h|^2.  Colour flow: the first flow whose running
// sum of W_c = sum_h |J_c,h|^2 exceeds rnd_col x sum_c W_c.
struct SelectArgs {
  const double* rnd_hel = nullptr;
  const double* rnd_col = nullptr;
  int* sel_hel = nullptr;
  int* sel_col = nullptr;
  double* chan_w = nullptr;  // channel weights [nevt][ndiag] (a kernel variant of its own)
};

// Single-diagram-enhancement channel weights (section "Event generation interface": what an
// event generator's multi-channel integration reads besides |M|^2): for each Feynman diagram d,
// W_d = sum over good helicities and over the diagram's amplitude terms of |a|^2 (colour
// stripped; a diagram with a four-gluon vertex has one term per colour structure), normalised to
// sum to 1 over the diagrams.  The observer sums each term's |a|^2 over the event's LPE lanes
// (one helicity each) and adds it to the event's LDS row.
template <class T, int LPE> struct ChannelObserver {
  volatile HME_LDS float* w;
  bool valid;
  HME_FN void term(int d, const cx<T>& a) const {
    float s = valid ? (float)a.r * (float)a.r + (float)a.i * (float)a.i : 0.f;
#pragma unroll
    for (int off = LPE / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    // every lane of the segment holds the sum and writes the same value: no branch in the
    // straight-line amplitude code
    w[d] = w[d] + s;
  }
};

// Sums over the 64 lanes of a wavefront of v[c] for every c < K (K a power of two), by
// recursive halving: at the step with lane offset O each lane keeps one half of its values
// (the upper half when its lane bit O is set) and adds the partner lane's copy of that half,
// so a step costs K/2 shuffles instead of K.  When one value is left the remaining steps are
// plain butterflies.  On return v[s], s < max(K / 64, 1), holds the total of value
// halving_index<K, 32>(lane) + s.
template <int K, int O, class V> HME_FN void halving_sum(V* v, int lane) {
  if constexpr (O > 0) {
    if constexpr (K >= 2) {
      const bool up = lane & O;
#pragma unroll
      for (int i = 0; i < K / 2; ++i) {
        const V keep = up ? v[K / 2 + i] : v[i];
        const V send = up ? v[i] : v[K / 2 + i];
        v[i] = keep + __shfl_xor(send, O, 64);
      }
      halving_sum<K / 2, O / 2>(v, lane);
    } else {
      v[0] += __shfl_xor(v[0], O, 64);
      halving_sum<1, O / 2>(v, lane);
    }
  }
}

template <int K, int O> HME_FN int halving_index(int lane) {
  if constexpr (O == 0) {
    return 0;
  } else if constexpr (K >= 2) {
    return ((lane & O) ? K / 2 : 0) + halving_index<K / 2, O / 2>(lane);
  } else {
    return halving_index<1, O / 2>(lane);
  }
}

constexpr int pow2_at_least(int n) { return n <= 1 ? 1 : 2 * pow2_at_least((n + 1) / 2); }

// Adds sum over the wavefront's lanes of |jamp[c]|^2 into w[c] (LDS, one array per
// wavefront) for every flow c: recursive halving over the flows padded to a power of two;
// each total is written by the lane that holds it (lanes holding the same total write the
// same value).  Zero jamps on lanes without a helicity.
template <int NCOL, class T>
HME_FN void add_flow_weights(const cx<T> (&jamp)[NCOL], int lane, volatile HME_LDS double* w) {
  constexpr int K = pow2_at_least(NCOL);
  T v[K];
#pragma unroll
  for (int c = 0; c < K; ++c) v[c] = c < NCOL ? jamp[c].r * jamp[c].r + jamp[c].i * jamp[c].i : T(0);
  halving_sum<K, 32>(v, lane);
  const int c0 = halving_index<K, 32>(lane);
#pragma unroll
  for (int s = 0; s < (K >= 64 ? K / 64 : 1); ++s)
    if (c0 + s < NCOL) w[c0 + s] += (double)v[s];
}

// Running sum over w[0..ncol) in flow order (one lane): the first flow whose running sum
// exceeds r times the total; the last flow of nonzero weight if rounding leaves none.
HME_FN int choose_flow(const volatile HME_LDS double* w, int ncol, double r) {
  double wtot = 0.0;
  for (int c = 0; c < ncol; ++c) wtot += w[c];
  const double target = r * wtot;
  double cum = 0.0;
  int kc = -1, last = 0;
  for (int c = 0; c < ncol; ++c) {
    const double v = w[c];
    cum += v;
    if (kc < 0 && cum > target) kc = c;
    if (v > 0) last = c;
  }
  return kc < 0 ? last : kc;
}

// orders this wavefront's LDS writes before its own later reads from other lanes
HME_FN void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The event's LPE lanes (an aligned segment of the wavefront) hold one helicity each; lanes
// past the last good helicity pass valid = false.  Every lane of the segment must call this.
// wlds: with LPE = 64 and 16 or more flows, the wavefront's LDS array of ncol flow weights
// (the flow sums then take the halving reduction); otherwise unused.
template <class Proc, class T, int LPE>
HME_FN void choose_helicity_and_flow(const cx<T> (&jamp)[Proc::ncol], bool valid, double mh, int sub, int64_t ev,
                                     int64_t evc, int64_t nevt, const int* __restrict__ goodhel, int ngood,
                                     const SelectArgs& sel, volatile HME_LDS double* wlds) {
  // inclusive running sum of |M_h|^2 over the segment, in good-helicity order
  double cum = valid ? mh : 0.0;
#pragma unroll
  for (int d = 1; d < LPE; d <<= 1) {
    const double t = __shfl_up(cum, d, LPE);
    if (sub >= d) cum += t;
  }
  const double total = __shfl(cum, LPE - 1, LPE);
  const double target_h = sel.rnd_hel[evc] * total;
  const uint64_t over = __ballot(valid && cum > target_h);
  const int base = (int)(threadIdx.x & 63) - sub;
  const uint64_t seg = (~0ull >> (64 - LPE)) << base;
  const uint64_t hit = over & seg;
  const int kh = hit ? __builtin_ctzll(hit) - base : ngood - 1;
  if constexpr (LPE == 64 && Proc::ncol >= 16) {
    for (int c = sub; c < Proc::ncol; c += 64) wlds[c] = 0.0;
    wave_lds_sync();
    cx<T> jz[Proc::ncol];
#pragma unroll
    for (int c = 0; c < Proc::ncol; ++c) jz[c] = valid ? jamp[c] : cx<T>{T(0), T(0)};
    add_flow_weights<Proc::ncol, T>(jz, sub, wlds);
    wave_lds_sync();
    if (sub == 0 && ev < nevt) {
      sel.sel_hel[ev] = goodhel[kh];
      sel.sel_col[ev] = choose_flow(wlds, Proc::ncol, sel.rnd_col[evc]);
    }
    return;
  }
  // colour-flow weights summed over the segment's helicities
  double wtot = 0.0;
#pragma unroll
  for (int c = 0; c < Proc::ncol; ++c)
    wtot += valid ? (double)jamp[c].r * (double)jamp[c].r + (double)jamp[c].i * (double)jamp[c].i : 0.0;
#pragma unroll
  for (int off = LPE / 2; off > 0; off >>= 1) wtot += __shfl_xor(wtot, off, 64);
  const double target_c = sel.rnd_col[evc] * wtot;
  double cum_c = 0.0;
  int kc = -1, last = 0;
#pragma unroll
  for (int c = 0; c < Proc::ncol; ++c) {
    double w = valid ? (double)jamp[c].r * (double)jamp[c].r + (double)jamp[c].i * (double)jamp[c].i : 0.0;
#pragma unroll
    for (int off = LPE / 2; off > 0; off >>= 1) w += __shfl_xor(w, off, 64);
    cum_c += w;
    if (kc < 0 && cum_c > target_c) kc = c;
    if (w > 0) last = c;
  }
  if (kc < 0) kc = last;  // rounding left the target at or above the last running sum
  if (sub == 0 && ev < nevt) {
    sel.sel_hel[ev] = goodhel[kh];
    sel.sel_col[ev] = kc;
  }
}

// The per-event table, built by the event's LPE lanes (an aligned segment of one wavefront):
// first the compensated momentum sums into ms (8 doubles each), then the table items from them,
// then the recycled wavefunctions from the items.
// A barrier over the block must follow before the table is read.
template <class Proc, int LPE, class S>
HME_FN void build_event_table(const double (&p)[Proc::npar][4], const ProcParams& prm, int sub, double* ms, S* tab) {
  for (int i = sub; i < Proc::nsum; i += LPE) Proc::momentum_sum(p, i, ms);
  wave_lds_sync();
  for (int j = sub; j < Proc::nitems; j += LPE) Proc::table_entry(p, prm, j, ms, tab);
  if constexpr (Proc::nrec > 0) {
    // helicity recycling: the two-state wavefunctions for every helicity pair, from the kits
    wave_lds_sync();
    for (int i = sub; i < 4 * Proc::nrec; i += LPE) Proc::template recycled_entry<S>(i, (tab_of<S>)tab, tab);
  }
}

// Mode 0: |M|^2; 1: also the helicity and colour-flow choice; 2: also the channel weights.
template <class Proc, class T, int LPE, int Mode = 0>
__global__ void __launch_bounds__(256, me2_min_waves<T>())
    me2_kernel(const double* __restrict__ mom, double* __restrict__ out, int64_t nevt,
               const int* __restrict__ goodhel, int ngood, ProcParams prm, double norm, int colour_f32,
               const int64_t* __restrict__ nevt_dev, SelectArgs sel) {
  constexpr bool Select = Mode == 1, Channels = Mode == 2;
  constexpr int EPW = 64 / LPE;   // events per wavefront
  constexpr int EPB = 256 / LPE;  // events per block
  // per-event table of momentum sums and propagator denominators, shared by the event's lanes,
  // and the compensated momentum sums it is built from
  __shared__ T table[EPB * (Proc::ntab > 0 ? Proc::ntab : 1)];
  __shared__ double msums[EPB * 8 * (Proc::nsum > 0 ? Proc::nsum : 1)];
  // with single-precision amplitudes, the colour sums of processes with 24 or more flows run
  // on the matrix cores (one event per wavefront, the 64 lanes are 64 helicity columns)
  constexpr bool kMfmaColour = LPE == 64 && Proc::ncol >= 24 && sizeof(T) == 4;
  __shared__ __attribute__((aligned(16))) __bf16 cnh[kMfmaColour ? ColourTiles<Proc>::words : 8];
  __shared__ __attribute__((aligned(16))) __bf16 cnl[kMfmaColour ? ColourTiles<Proc>::words : 8];
  // flow weights of the selection variant (one array per wavefront, events of 64 lanes)
  __shared__ double wsel[4][Select && LPE == 64 && Proc::ncol >= 16 ? Proc::ncol : 1];
  // channel weights of the events of the block
  __shared__ float wch[Channels ? EPB : 1][Channels ? Proc::ndiag : 1];
  const int lane = threadIdx.x & 63;
  // the event count comes from device memory when a captured graph launches a batch of
  // varying size with a fixed grid; blocks past the end leave at once
  if (nevt_dev) nevt = *nevt_dev;
  if ((int64_t)blockIdx.x * EPB >= nevt) return;  // uniform per block
  // wave index in the block, made explicitly wave-uniform so that with LPE = 64 the
  // event record is fetched with scalar loads
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ev = ((int64_t)blockIdx.x * 4 + wib) * EPW + lane / LPE;
  const int sub = lane % LPE;
  const int64_t evc = ev < nevt ? ev : nevt - 1;  // ragged tail: recompute the last event, store nothing
  double p[Proc::npar][4];
  load_event<Proc>(mom, evc, p);
  T* tab = table + (threadIdx.x / LPE) * Proc::ntab;
  double* ms = msums + (threadIdx.x / LPE) * 8 * Proc::nsum;
  build_event_table<Proc, LPE>(p, prm, sub, ms, tab);
  if constexpr (kMfmaColour) colour_tiles_fill<Proc>(cnh, cnl, threadIdx.x, 256);
  __syncthreads();
  double acc = 0.0;
  if constexpr (Mode != 0) {
    // one helicity per lane (the launcher checks ngood <= LPE); every lane runs, a lane past
    // the last good helicity evaluates the last one again and contributes zero
    const bool valid = sub < ngood;
    cx<T> jamp[Proc::ncol];
#pragma unroll
    for (int c = 0; c < Proc::ncol; ++c) jamp[c] = {T(0), T(0)};
    const unsigned hsel = (unsigned)goodhel[valid ? sub : ngood - 1];
    [[maybe_unused]] volatile HME_LDS float* wd = nullptr;
    if constexpr (Channels) {
      wd = (volatile HME_LDS float*)&wch[threadIdx.x / LPE][0];
      for (int d = sub; d < Proc::ndiag; d += LPE) wd[d] = 0.f;
      wave_lds_sync();
      Proc::template amplitudes<T>(p, prm, hsel, (tab_of<T>)tab, jamp, ChannelObserver<T, LPE>{wd, valid});
    } else {
      Proc::template amplitudes<T>(p, prm, hsel, (tab_of<T>)tab, jamp);
    }
    double mh;
    if constexpr (kMfmaColour) {
      mh = (double)colour_sum_wave<Proc>(jamp, NumerLds<Proc>{(const HME_LDS __bf16*)cnh, (const HME_LDS __bf16*)cnl});
    } else if (colour_f32) {
      cx<float> jf[Proc::ncol];
#pragma unroll
      for (int c = 0; c < Proc::ncol; ++c) jf[c] = cast<float>(jamp[c]);
      mh = (double)Proc::template colour_sum<float>(jf);
    } else {
      mh = (double)Proc::template colour_sum<T>(jamp);
    }
    acc = valid ? mh : 0.0;
    if constexpr (Select)
      choose_helicity_and_flow<Proc, T, LPE>(jamp, valid, mh, sub, ev, evc, nevt, goodhel, ngood, sel,
                                             (volatile HME_LDS double*)&wsel[wib][0]);
    if constexpr (Channels) {
      // normalise the event's row and write it
      wave_lds_sync();
      double tot = 0.0;
      for (int d = sub; d < Proc::ndiag; d += LPE) tot += (double)wd[d];
#pragma unroll
      for (int off = LPE / 2; off > 0; off >>= 1) tot += __shfl_xor(tot, off, 64);
      if (ev < nevt)
        for (int d = sub; d < Proc::ndiag; d += LPE) sel.chan_w[ev * Proc::ndiag + d] = (double)wd[d] / tot;
    }
  } else if constexpr (kMfmaColour) {
    // every lane runs every pass (the matrix cores take the whole wavefront); a lane past the
    // last good helicity evaluates the last one again and drops its result (each helicity
    // column of the product depends on that lane's jamps only)
    for (int g = 0; g < ngood; g += 64) {
      const int k = g + sub;
      const bool valid = k < ngood;
      cx<T> jamp[Proc::ncol];
#pragma unroll
      for (int c = 0; c < Proc::ncol; ++c) jamp[c] = {T(0), T(0)};
      Proc::template amplitudes<T>(p, prm, (unsigned)goodhel[valid ? k : ngood - 1], (tab_of<T>)tab, jamp);
      const float s = colour_sum_wave<Proc>(jamp, NumerLds<Proc>{(const HME_LDS __bf16*)cnh, (const HME_LDS __bf16*)cnl});
      acc += valid ? (double)s : 0.0;
    }
  } else {
    for (int k = sub; k < ngood; k += LPE) {
      cx<T> jamp[Proc::ncol];
#pragma unroll
      for (int c = 0; c < Proc::ncol; ++c) jamp[c] = {T(0), T(0)};
      Proc::template amplitudes<T>(p, prm, (unsigned)goodhel[k], (tab_of<T>)tab, jamp);
      if (colour_f32) {  // wave-uniform: the colour algebra in single precision
        cx<float> jf[Proc::ncol];
#pragma unroll
        for (int c = 0; c < Proc::ncol; ++c) jf[c] = cast<float>(jamp[c]);
        acc += (double)Proc::template colour_sum<float>(jf);
      } else {
        acc += (double)Proc::template colour_sum<T>(jamp);
      }
    }
  }
#pragma unroll
  for (int off = LPE / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (sub == 0 && ev < nevt) out[ev] = acc * norm;
}

// |M_h|^2 (colour-summed, unnormalised) for every helicity of a few events; used once at
// set-up to find the helicities that vanish identically.  One block of 64 lanes per
// event; the event's table is built in LDS exactly as in me2_kernel.
template <class Proc>
__global__ void __launch_bounds__(64) hel_kernel(const double* __restrict__ mom, int nev, ProcParams prm,
                                                 double* __restrict__ out) {
  __shared__ double table[Proc::ntab > 0 ? Proc::ntab : 1];
  __shared__ double msums[8 * (Proc::nsum > 0 ? Proc::nsum : 1)];
  const int ev = blockIdx.x;
  if (ev >= nev) return;  // uniform per block
  double p[Proc::npar][4];
  load_event<Proc>(mom, ev, p);
  build_event_table<Proc, 64>(p, prm, threadIdx.x, msums, table);
  __syncthreads();
  for (int h = threadIdx.x; h < Proc::nhel; h += blockDim.x) {
    cx<double> jamp[Proc::ncol];
    for (int c = 0; c < Proc::ncol; ++c) jamp[c] = {0.0, 0.0};
    Proc::template amplitudes<double>(p, prm, (unsigned)h, (tab_ptr)table, jamp);
    out[(size_t)ev * Proc::nhel + h] = Proc::template colour_sum<double>(jamp);
  }
}

// ------------------------------------------------------------------ launchers

struct LaunchArgs {
  const double* mom;
  double* out;
  int64_t nevt;
  const int* goodhel;
  int ngood;
  ProcParams prm;
  double norm;
  hipStream_t stream;
  int colour_f32;  // colour sum in single precision (for double-precision amplitudes)
  const int64_t* nevt_dev = nullptr;  // if set, the kernel reads the event count here (nevt sizes the grid)
  void* ws = nullptr;                 // jamp workspace of a process evaluated in pieces
  int64_t ws_events = 0;              // events the workspace holds (the sub-batch size)
  SelectArgs sel{};                   // helicity / colour-flow choice (sel.sel_hel == nullptr: none)
};

struct ProcInfo {
  int npar, nhel, ncol, ndiag, namp, gs_power;
  double iden, colour_denom, flops_per_hel, flops_per_event;
  int nchunk;  // 0: one kernel; otherwise pieces + colour kernel over a jamp workspace
  int nslot;   // workspace slots per (event, good helicity) of a process in pieces
};

template <class Proc> ProcInfo make_info() {
  return ProcInfo{Proc::npar, Proc::nhel, Proc::ncol, Proc::ndiag, Proc::namp, Proc::gs_power,
                  Proc::iden, Proc::colour_denom, Proc::flops_per_hel, Proc::flops_per_event, Proc::nchunk,
                  Proc::nslot};
}

// lanes per event: the smallest of 4, 8, 16, 32, 64 that holds all good helicities (64 loops over more)
inline int lanes_per_event(int ngood) {
  if (ngood <= 4) return 4;
  if (ngood <= 8) return 8;
  if (ngood <= 16) return 16;
  if (ngood <= 32) return 32;
  return 64;
}

template <class Proc, class T, int LPE> hipError_t launch_lpe(const LaunchArgs& a) {
  constexpr int threads = 256;
  constexpr int EPB = threads / LPE;  // events per block
  const int64_t blocks = (a.nevt + EPB - 1) / EPB;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (a.sel.sel_hel || a.sel.chan_w) {
    // the choice and the channel weights need one helicity per lane, and one of them per call
    if (a.ngood > LPE || (a.sel.sel_hel && a.sel.chan_w)) return hipErrorInvalidValue;
    if (a.sel.sel_hel)
      me2_kernel<Proc, T, LPE, 1><<<dim3((unsigned)blocks), dim3(threads), 0, a.stream>>>(
          a.mom, a.out, a.nevt, a.goodhel, a.ngood, a.prm, a.norm, a.colour_f32, a.nevt_dev, a.sel);
    else
      me2_kernel<Proc, T, LPE, 2><<<dim3((unsigned)blocks), dim3(threads), 0, a.stream>>>(
          a.mom, a.out, a.nevt, a.goodhel, a.ngood, a.prm, a.norm, a.colour_f32, a.nevt_dev, a.sel);
  } else {
    me2_kernel<Proc, T, LPE, 0><<<dim3((unsigned)blocks), dim3(threads), 0, a.stream>>>(
        a.mom, a.out, a.nevt, a.goodhel, a.ngood, a.prm, a.norm, a.colour_f32, a.nevt_dev, a.sel);
  }
  return hipGetLastError();
}

// LDS of a block of me2_kernel with LPE lanes per event (the per-event tables and sums of its
// 256 / LPE events, the channel-weight rows): a lane count whose block would not fit in 64 KiB
// is not built, and its events take the next larger lane count (lanes past the last good
// helicity idle).
template <class Proc, class T, int LPE> constexpr bool lpe_fits() {
  constexpr size_t per_event = sizeof(T) * (Proc::ntab > 0 ? Proc::ntab : 1) + 64 * (Proc::nsum > 0 ? Proc::nsum : 1) +
                               8 * Proc::ndiag;
  return (256 / LPE) * per_event <= (size_t)64 << 10;
}

template <class Proc, class T> hipError_t launch_me2(const LaunchArgs& a) {
  // processes with 24 or more colour flows and 64 or more helicities always fill whole
  // wavefronts (idle lanes are masked; the matrix-core colour sum takes one event per wavefront)
  if constexpr (Proc::nhel >= 64 && Proc::ncol >= 24) {
    return launch_lpe<Proc, T, 64>(a);
  } else {
    switch (lanes_per_event(a.ngood)) {
      case 4:
        if constexpr (lpe_fits<Proc, T, 4>()) return launch_lpe<Proc, T, 4>(a);
        [[fallthrough]];
      case 8:
        if constexpr (lpe_fits<Proc, T, 8>()) return launch_lpe<Proc, T, 8>(a);
        [[fallthrough]];
      case 16:
        if constexpr (lpe_fits<Proc, T, 16>()) return launch_lpe<Proc, T, 16>(a);
        [[fallthrough]];
      case 32: return launch_lpe<Proc, T, 32>(a);
      default: return launch_lpe<Proc, T, 64>(a);
    }
  }
}

template <class Proc>
hipError_t launch_hel(const double* mom, int nev, const ProcParams& prm, double* out, hipStream_t s) {
  hel_kernel<Proc><<<dim3(nev), dim3(64), 0, s>>>(mom, nev, prm, out);
  return hipGetLastError();
}

}  // namespace hme
