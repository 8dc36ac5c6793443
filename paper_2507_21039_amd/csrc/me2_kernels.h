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
};

// The event's LPE lanes (an aligned segment of the wavefront) hold one helicity each; lanes
// past the last good helicity pass valid = false.  Every lane of the segment must call this.
template <class Proc, class T, int LPE>
HME_FN void choose_helicity_and_flow(const cx<T> (&jamp)[Proc::ncol], bool valid, double mh, int sub, int64_t ev,
                                     int64_t evc, int64_t nevt, const int* __restrict__ goodhel, int ngood,
                                     const SelectArgs& sel) {
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

template <class Proc, class T, int LPE, bool Select = false>
__global__ void __launch_bounds__(256, me2_min_waves<T>())
    me2_kernel(const double* __restrict__ mom, double* __restrict__ out, int64_t nevt,
               const int* __restrict__ goodhel, int ngood, ProcParams prm, double norm, int colour_f32,
               const int64_t* __restrict__ nevt_dev, SelectArgs sel) {
  constexpr int EPW = 64 / LPE;   // events per wavefront
  constexpr int EPB = 256 / LPE;  // events per block
  // per-event table of momentum sums and propagator denominators, shared by the event's lanes
  __shared__ double table[EPB * (Proc::ntab > 0 ? Proc::ntab : 1)];
  // with single-precision amplitudes, the colour sums of processes with 24 or more flows run
  // on the matrix cores (one event per wavefront, the 64 lanes are 64 helicity columns)
  constexpr bool kMfmaColour = LPE == 64 && Proc::ncol >= 24 && sizeof(T) == 4;
  __shared__ __attribute__((aligned(16))) __bf16 cnh[kMfmaColour ? ColourTiles<Proc>::words : 8];
  __shared__ __attribute__((aligned(16))) __bf16 cnl[kMfmaColour ? ColourTiles<Proc>::words : 8];
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
  double* tab = table + (threadIdx.x / LPE) * Proc::ntab;
  for (int j = sub; j < Proc::nitems; j += LPE) Proc::table_entry(p, prm, j, tab);
  if constexpr (kMfmaColour) colour_tiles_fill<Proc>(cnh, cnl, threadIdx.x, 256);
  __syncthreads();
  double acc = 0.0;
  if constexpr (Select) {
    // one helicity per lane (the launcher checks ngood <= LPE); every lane runs, a lane past
    // the last good helicity evaluates the last one again and contributes zero
    const bool valid = sub < ngood;
    cx<T> jamp[Proc::ncol];
#pragma unroll
    for (int c = 0; c < Proc::ncol; ++c) jamp[c] = {T(0), T(0)};
    Proc::template amplitudes<T>(p, prm, (unsigned)goodhel[valid ? sub : ngood - 1], (tab_ptr)tab, jamp);
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
    choose_helicity_and_flow<Proc, T, LPE>(jamp, valid, mh, sub, ev, evc, nevt, goodhel, ngood, sel);
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
      Proc::template amplitudes<T>(p, prm, (unsigned)goodhel[valid ? k : ngood - 1], (tab_ptr)tab, jamp);
      const float s = colour_sum_wave<Proc>(jamp, NumerLds<Proc>{(const HME_LDS __bf16*)cnh, (const HME_LDS __bf16*)cnl});
      acc += valid ? (double)s : 0.0;
    }
  } else {
    for (int k = sub; k < ngood; k += LPE) {
      cx<T> jamp[Proc::ncol];
#pragma unroll
      for (int c = 0; c < Proc::ncol; ++c) jamp[c] = {T(0), T(0)};
      Proc::template amplitudes<T>(p, prm, (unsigned)goodhel[k], (tab_ptr)tab, jamp);
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
  const int ev = blockIdx.x;
  if (ev >= nev) return;  // uniform per block
  double p[Proc::npar][4];
  load_event<Proc>(mom, ev, p);
  for (int j = threadIdx.x; j < Proc::nitems; j += blockDim.x) Proc::table_entry(p, prm, j, table);
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

// lanes per event: the smallest of 4, 16, 32, 64 that holds all good helicities (64 loops over more)
inline int lanes_per_event(int ngood) {
  if (ngood <= 4) return 4;
  if (ngood <= 16) return 16;
  if (ngood <= 32) return 32;
  return 64;
}

template <class Proc, class T, int LPE> hipError_t launch_lpe(const LaunchArgs& a) {
  constexpr int threads = 256;
  constexpr int EPB = threads / LPE;  // events per block
  const int64_t blocks = (a.nevt + EPB - 1) / EPB;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (a.sel.sel_hel) {
    if (a.ngood > LPE) return hipErrorInvalidValue;  // the choice needs one helicity per lane
    me2_kernel<Proc, T, LPE, true><<<dim3((unsigned)blocks), dim3(threads), 0, a.stream>>>(
        a.mom, a.out, a.nevt, a.goodhel, a.ngood, a.prm, a.norm, a.colour_f32, a.nevt_dev, a.sel);
  } else {
    me2_kernel<Proc, T, LPE, false><<<dim3((unsigned)blocks), dim3(threads), 0, a.stream>>>(
        a.mom, a.out, a.nevt, a.goodhel, a.ngood, a.prm, a.norm, a.colour_f32, a.nevt_dev, a.sel);
  }
  return hipGetLastError();
}

template <class Proc, class T> hipError_t launch_me2(const LaunchArgs& a) {
  // processes with 64 or more helicities always fill whole wavefronts (idle lanes are masked)
  if constexpr (Proc::nhel >= 64) {
    return launch_lpe<Proc, T, 64>(a);
  } else {
    switch (lanes_per_event(a.ngood)) {
      case 4: return launch_lpe<Proc, T, 4>(a);
      case 16: return launch_lpe<Proc, T, 16>(a);
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
