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

template <class Proc, class T, int LPE>
__global__ void __launch_bounds__(256)
    me2_kernel(const double* __restrict__ mom, double* __restrict__ out, int64_t nevt,
               const int* __restrict__ goodhel, int ngood, ProcParams prm, double norm, int colour_f32,
               const int64_t* __restrict__ nevt_dev) {
  constexpr int EPW = 64 / LPE;   // events per wavefront
  constexpr int EPB = 256 / LPE;  // events per block
  // per-event table of momentum sums and propagator denominators, shared by the event's lanes
  __shared__ double table[EPB * (Proc::ntab > 0 ? Proc::ntab : 1)];
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
  __syncthreads();
  double acc = 0.0;
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

// ------------------------------------------------- processes evaluated in pieces
//
// For the largest process one straight-line kernel would not compile in reasonable
// time, and its 120 jamps would not fit in registers beside the wavefunctions.  The
// generator then cuts the amplitude schedule into pieces, each a kernel.  A piece keeps
// at most a fixed number of flows in registers; a flow's partial sum leaves its register
// after its last term in the piece, or earlier when the register is needed, and is
// written to a slot of its own in a device workspace
//     ws[event][slot][good helicity]   (cx<float>, events of one sub-batch)
// so that the LPE lanes of an event, which hold consecutive helicities, write
// consecutive addresses (plain coalesced stores; no read-modify-write, no atomics).  A
// last kernel adds up each flow's slots, forms the colour sum and reduces over
// helicities as me2_kernel does.  Single precision only.

// Events in a sub-batch: at most nevt (which sizes the grid); when a captured graph reads
// the batch's event count from device memory, only those left after the sub-batch's
// first event e0 (none if the batch ends before it).
HME_FN int64_t sub_batch_events(int64_t nevt, const int64_t* nevt_dev, int64_t e0) {
  if (nevt_dev) {
    const int64_t left = *nevt_dev - e0;
    if (left < nevt) nevt = left;
  }
  return nevt;
}

// Where a piece's partial jamps go: slot `slot` of this lane's (event, helicity) column,
// written once with a plain store (no other code writes it).
struct WorkspaceSink {
  cx<float>* base;
  int64_t stride;  // entries between consecutive slots (the number of good helicities)
  HME_FN void put(int slot, cx<float> v) const { base[slot * stride] = v; }
};

// the per-event table in LDS, built by the event's lanes (as in me2_kernel)
template <class Proc, int LPE>
HME_FN void build_table(const double (&p)[Proc::npar][4], const ProcParams& prm, int sub, double* tab) {
  for (int j = sub; j < Proc::nitems; j += LPE) Proc::table_entry(p, prm, j, tab);
}

// Pieces are compiled for 2 waves per SIMD (at most 256 VGPRs): the generator's budgets keep
// them within it or a few registers above, which the compiler then spills; one wave per SIMD
// with AGPRs costs far more (measured: 1.1-1.3 ms against 0.63-0.8 ms per 8,192 events).
#ifndef HME_PIECE_WAVES
#define HME_PIECE_WAVES 2
#endif
template <class Proc, class Chunk, int LPE>
__global__ void __launch_bounds__(256, HME_PIECE_WAVES)
    chunk_kernel(const double* __restrict__ mom, cx<float>* __restrict__ ws, int64_t nevt,
                 const int* __restrict__ goodhel, int ngood, ProcParams prm, const int64_t* __restrict__ nevt_dev,
                 int64_t e0) {
  constexpr int EPW = 64 / LPE, EPB = 256 / LPE;
  __shared__ double table[EPB * Proc::ntab];
  const int lane = threadIdx.x & 63;
  nevt = sub_batch_events(nevt, nevt_dev, e0);
  if ((int64_t)blockIdx.x * EPB >= nevt) return;  // uniform per block
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ev = ((int64_t)blockIdx.x * 4 + wib) * EPW + lane / LPE;
  const int sub = lane % LPE;
  const int64_t evc = ev < nevt ? ev : nevt - 1;  // ragged tail: recompute the last event, store nothing
  double p[Proc::npar][4];
  load_event<Proc>(mom, evc, p);
  double* tab = table + (threadIdx.x / LPE) * Proc::ntab;
  build_table<Proc, LPE>(p, prm, sub, tab);
  __syncthreads();
  if (ev >= nevt) return;  // no barrier follows
  cx<float>* w = ws + (size_t)ev * Proc::nslot * ngood;
  for (int k = sub; k < ngood; k += LPE) {
    WorkspaceSink sink{w + k, ngood};
    Chunk::template amplitudes<float>(prm, (unsigned)goodhel[k], (tab_ptr)tab, sink);
  }
}

// colour sum of the workspace jamps; per_hel = 0: out[ev] = norm * sum over helicities,
// per_hel = 1: out[ev * ngood + k] = colour sum of good helicity k (unnormalised)
template <class Proc, int LPE>
__global__ void __launch_bounds__(256)
    colour_kernel(const cx<float>* __restrict__ ws, double* __restrict__ out, int64_t nevt, int ngood,
                  double norm, int per_hel, const int64_t* __restrict__ nevt_dev, int64_t e0) {
  constexpr int EPW = 64 / LPE, EPB = 256 / LPE;
  const int lane = threadIdx.x & 63;
  nevt = sub_batch_events(nevt, nevt_dev, e0);
  if ((int64_t)blockIdx.x * EPB >= nevt) return;
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ev = ((int64_t)blockIdx.x * 4 + wib) * EPW + lane / LPE;
  const int sub = lane % LPE;
  const int64_t evc = ev < nevt ? ev : nevt - 1;
  const cx<float>* w = ws + (size_t)evc * Proc::nslot * ngood;
  double acc = 0.0;
  for (int k = sub; k < ngood; k += LPE) {
    cx<float> jamp[Proc::ncol];
    Proc::template gather<float, float>(w + k, ngood, jamp);
    const double v = (double)Proc::template colour_sum<float>(jamp);
    if (per_hel && ev < nevt) out[(size_t)ev * ngood + k] = v;
    acc += v;
  }
#pragma unroll
  for (int off = LPE / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (!per_hel && sub == 0 && ev < nevt) out[ev] = acc * norm;
}

struct ChunkArgs {
  const double* mom;  // momenta of the sub-batch's first event
  cx<float>* ws;      // workspace, nevt * nslot * ngood entries
  int64_t nevt;       // events in the sub-batch
  const int* goodhel;
  int ngood;
  ProcParams prm;
  hipStream_t stream;
  const int64_t* nevt_dev;  // if set: the batch's event count (device), of which this sub-batch
  int64_t e0;               // starts at event e0
};

template <class Proc> constexpr int chunk_lpe() { return Proc::nhel >= 64 ? 64 : 32; }

template <class Proc, class Chunk> hipError_t launch_chunk(const ChunkArgs& a) {
  constexpr int LPE = chunk_lpe<Proc>(), EPB = 256 / LPE;
  const int64_t blocks = (a.nevt + EPB - 1) / EPB;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  chunk_kernel<Proc, Chunk, LPE><<<dim3((unsigned)blocks), dim3(256), 0, a.stream>>>(
      a.mom, a.ws, a.nevt, a.goodhel, a.ngood, a.prm, a.nevt_dev, a.e0);
  return hipGetLastError();
}

template <class Proc>
hipError_t launch_colour(const cx<float>* ws, double* out, int64_t nevt, int ngood, double norm, int per_hel,
                         const int64_t* nevt_dev, int64_t e0, hipStream_t s) {
  constexpr int LPE = chunk_lpe<Proc>(), EPB = 256 / LPE;
  const int64_t blocks = (nevt + EPB - 1) / EPB;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  colour_kernel<Proc, LPE><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(ws, out, nevt, ngood, norm, per_hel,
                                                                         nevt_dev, e0);
  return hipGetLastError();
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
  me2_kernel<Proc, T, LPE><<<dim3((unsigned)blocks), dim3(threads), 0, a.stream>>>(
      a.mom, a.out, a.nevt, a.goodhel, a.ngood, a.prm, a.norm, a.colour_f32, a.nevt_dev);
  return hipGetLastError();
}

template <class Proc, class T> hipError_t launch_me2(const LaunchArgs& a) {
  // processes with 64 or more helicities always fill whole wavefronts (idle lanes are masked)
  if constexpr (Proc::nhel >= 64) return launch_lpe<Proc, T, 64>(a);
  switch (lanes_per_event(a.ngood)) {
    case 4: return launch_lpe<Proc, T, 4>(a);
    case 16: return launch_lpe<Proc, T, 16>(a);
    case 32: return launch_lpe<Proc, T, 32>(a);
    default: return launch_lpe<Proc, T, 64>(a);
  }
}

template <class Proc>
hipError_t launch_hel(const double* mom, int nev, const ProcParams& prm, double* out, hipStream_t s) {
  hel_kernel<Proc><<<dim3(nev), dim3(64), 0, s>>>(mom, nev, prm, out);
  return hipGetLastError();
}

}  // namespace hme
