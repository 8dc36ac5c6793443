// Kernels of a process evaluated in pieces (gg -> t tbar g g g): the piece kernels, the
// jamp workspace they write, and the colour kernels over it (on the vector ALUs or on the
// matrix cores, colour_mfma.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "colour_blocked.h"
#include "colour_mfma.h"
#include "me2_kernels.h"

namespace hme {

// ------------------------------------------------- processes evaluated in pieces
//
// For the largest process one straight-line kernel would not compile in reasonable
// time, and its 120 jamps would not fit in registers beside the wavefunctions.  The
// generator then cuts the amplitude schedule into pieces, each a kernel.  A piece keeps
// at most a fixed number of flows in registers; a flow's partial sum leaves its register
// after its last term in the piece, or earlier when the register is needed, and is
// written to a slot of its own in a device workspace
//     ws[event][slot][helicity column]   (cx<float> or cx<double>, events of one sub-batch)
// with Proc::nhel columns of which the good helicities take the first ngood, so that the
// LPE lanes of an event, which hold consecutive helicities, write consecutive addresses
// (plain coalesced stores; no read-modify-write, no atomics) and every slot sits at a
// compile-time offset from the event's column (the colour kernel's 789 loads then need no
// address registers of their own).  A last kernel adds up each flow's slots, forms the
// colour sum and reduces over helicities as me2_kernel does.

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
// written once with a plain store (no other code writes it).  T: the type of the amplitudes
// (float for HME_MIXED_FAST, double for HME_FP64 and HME_MIXED_PAPER).
template <class T> struct WorkspaceSink {
  cx<T>* base;
  int64_t stride;  // entries between consecutive slots (Proc::nhel, a compile-time constant)
  HME_FN void put(int slot, cx<T> v) const { base[slot * stride] = v; }
};

// One lane's helicity column of an event's workspace, read with buffer loads: the event's
// slots in a buffer descriptor (wave-uniform base, bounds = the event's slots), the lane's
// column as the vector offset and each slot's offset, a compile-time constant in the gather,
// as the scalar offset.  The gather's 789 loads then take no address registers or address
// arithmetic, which leaves the registers for loads in flight.
template <class S> struct WsColumn {
  __amdgpu_buffer_rsrc_t rsrc;
  int lane_bytes;
  // word 3 of a raw (untyped, unswizzled) buffer descriptor on the gfx9 family
  static constexpr int kRawBufferFlags = 0x00020000;
  template <class Proc> HME_FN static WsColumn make(const cx<S>* event_base, int column) {
    constexpr int bytes = Proc::nslot * Proc::nhel * (int)sizeof(cx<S>);
    return WsColumn{__builtin_amdgcn_make_buffer_rsrc(const_cast<cx<S>*>(event_base), 0, bytes, kRawBufferFlags),
                    column * (int)sizeof(cx<S>)};
  }
  // writes entry i of the column (the same offsets as operator[])
  HME_FN void put(int64_t i, cx<S> v) const {
    const int off = (int)(i * (int64_t)sizeof(cx<S>));
    if constexpr (sizeof(S) == 4) {
      typedef unsigned u32x2 __attribute__((vector_size(8)));
      const u32x2 d = {__float_as_uint(v.r), __float_as_uint(v.i)};
      __builtin_amdgcn_raw_buffer_store_b64(d, rsrc, lane_bytes, off, 0);
    } else {
      typedef unsigned u32x4 __attribute__((vector_size(16)));
      const u32x4 d = {(unsigned)__double2loint(v.r), (unsigned)__double2hiint(v.r),
                       (unsigned)__double2loint(v.i), (unsigned)__double2hiint(v.i)};
      __builtin_amdgcn_raw_buffer_store_b128(d, rsrc, lane_bytes, off, 0);
    }
  }
  HME_FN cx<S> operator[](int64_t i) const {
    const int off = (int)(i * (int64_t)sizeof(cx<S>));
    // the words are copied out of the vector before reinterpretation (a bit cast of a vector
    // element in place reads element 0 with this compiler)
    if constexpr (sizeof(S) == 4) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(rsrc, lane_bytes, off, 0);
      const unsigned re = v[0], im = v[1];
      return cx<S>{__uint_as_float(re), __uint_as_float(im)};
    } else {
      const auto v = __builtin_amdgcn_raw_buffer_load_b128(rsrc, lane_bytes, off, 0);
      const unsigned r0 = v[0], r1 = v[1], i0 = v[2], i1 = v[3];
      return cx<S>{__hiloint2double((int)r1, (int)r0), __hiloint2double((int)i1, (int)i0)};
    }
  }
};

// The jamps of one helicity column k of an event's workspace w.  Double-precision slots (16 B)
// are read through a buffer descriptor with constant slot offsets.  Single-precision slots are
// read through a plain pointer with the stride hidden from the optimiser: with constant offsets
// the compiler keeps a 64-bit address per load in flight and runs out of registers, while a
// running pointer advanced by scalar strides keeps the gather's loads in flight (measured on the
// compiled code: 25 against 541 waits for all loads of the colour kernel).
template <class Proc, class T, class S>
HME_FN void gather_column(const cx<S>* w, int k, cx<T> (&jamp)[Proc::ncol]) {
  if constexpr (sizeof(S) == 8) {
    Proc::template gather<T, S>(WsColumn<S>::template make<Proc>(w, k), Proc::nhel, jamp);
  } else {
    int64_t stride = Proc::nhel;
    asm volatile("" : "+s"(stride));
    Proc::template gather<T, S>(w + k, stride, jamp);
  }
}

// Single-precision pieces are compiled for 2 waves per SIMD (at most 256 VGPRs): the generator's
// budgets keep them within it or a few registers above, which the compiler then spills; one wave
// per SIMD with AGPRs costs far more for them (measured: 1.1-1.3 ms against 0.63-0.8 ms per
// 8,192 events).  Double-precision pieces run the same schedule (the same partial-jamp slots)
// with twice the registers, at one wave per SIMD.
#ifndef HME_PIECE_WAVES
#define HME_PIECE_WAVES 2
#endif
template <class T> constexpr int piece_waves() { return sizeof(T) == 4 ? HME_PIECE_WAVES : 1; }

template <class Proc, class Chunk, int LPE, class T>
__global__ void __launch_bounds__(256, piece_waves<T>())
    chunk_kernel(const double* __restrict__ mom, cx<T>* __restrict__ ws, int64_t nevt,
                 const int* __restrict__ goodhel, int ngood, ProcParams prm, const int64_t* __restrict__ nevt_dev,
                 int64_t e0) {
  constexpr int EPW = 64 / LPE, EPB = 256 / LPE;
  __shared__ T table[EPB * Proc::ntab];
  __shared__ double msums[EPB * 8 * Proc::nsum];
  const int lane = threadIdx.x & 63;
  nevt = sub_batch_events(nevt, nevt_dev, e0);
  if ((int64_t)blockIdx.x * EPB >= nevt) return;  // uniform per block
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ev = ((int64_t)blockIdx.x * 4 + wib) * EPW + lane / LPE;
  const int sub = lane % LPE;
  const int64_t evc = ev < nevt ? ev : nevt - 1;  // ragged tail: recompute the last event, store nothing
  double p[Proc::npar][4];
  load_event<Proc>(mom, evc, p);
  T* tab = table + (threadIdx.x / LPE) * Proc::ntab;
  build_event_table<Proc, LPE>(p, prm, sub, msums + (threadIdx.x / LPE) * 8 * Proc::nsum, tab);
  __syncthreads();
  if (ev >= nevt) return;  // no barrier follows
  cx<T>* w = ws + (size_t)ev * Proc::nslot * Proc::nhel;
  for (int k = sub; k < ngood; k += LPE) {
    WorkspaceSink<T> sink{w + k, Proc::nhel};
    Chunk::template amplitudes<T>(prm, (unsigned)goodhel[k], (tab_of<T>)tab, sink);
  }
}

// colour sum of the workspace jamps; per_hel = 0: out[ev] = norm * sum over helicities,
// per_hel = 1: out[ev * ngood + k] = colour sum of good helicity k (unnormalised)
// S: the workspace type, C: the type of the colour sum (VALU)
template <class Proc, int LPE, class S, class C>
__global__ void __launch_bounds__(256)
    colour_kernel(const cx<S>* __restrict__ ws, double* __restrict__ out, int64_t nevt, int ngood,
                  double norm, int per_hel, const int64_t* __restrict__ nevt_dev, int64_t e0) {
  constexpr int EPW = 64 / LPE, EPB = 256 / LPE;
  static_assert(LPE == 64, "one event per wavefront: the workspace descriptor is wave-uniform");
  const int lane = threadIdx.x & 63;
  nevt = sub_batch_events(nevt, nevt_dev, e0);
  if ((int64_t)blockIdx.x * EPB >= nevt) return;
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ev = ((int64_t)blockIdx.x * 4 + wib) * EPW + lane / LPE;
  const int sub = lane % LPE;
  const int64_t evc = ev < nevt ? ev : nevt - 1;
  const cx<S>* w = ws + (size_t)evc * Proc::nslot * Proc::nhel;
  double acc = 0.0;
  for (int k = sub; k < ngood; k += LPE) {
    cx<C> jamp[Proc::ncol];
    gather_column<Proc, C, S>(w, k, jamp);
    const double v = (double)Proc::template colour_sum<C>(jamp);
    if (per_hel && ev < nevt) out[(size_t)ev * ngood + k] = v;
    acc += v;
  }
#pragma unroll
  for (int off = LPE / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (!per_hel && sub == 0 && ev < nevt) out[ev] = acc * norm;
}

// FP64 colour sum in two kernels.  The 120 double jamps of a helicity need 480 registers, so
// the gather form spills; instead fold_kernel adds each flow's slots (in slot order, the same
// sums as the gather) and writes the result over the flow's first slot, with a few groups of
// loads live at a time, and colour_blocked_kernel, a launch later, reads those 120 values back
// in blocks for the symmetric colour sum.  Each lane folds and reads only its own helicity
// column, and no slot is read after it is written within a kernel.
template <class Proc>
__global__ void __launch_bounds__(256)
    fold_kernel(cx<double>* ws, int64_t nevt, int ngood, const int64_t* __restrict__ nevt_dev, int64_t e0) {
  const int lane = threadIdx.x & 63;
  nevt = sub_batch_events(nevt, nevt_dev, e0);
  const int64_t ev = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (ev >= nevt) return;  // wave-uniform; no barrier follows
  cx<double>* w = ws + (size_t)ev * Proc::nslot * Proc::nhel;
  for (int k = lane; k < ngood; k += 64) Proc::template fold<double>(WsColumn<double>::template make<Proc>(w, k), Proc::nhel);
}

template <class Proc>
__global__ void __launch_bounds__(256)
    colour_blocked_kernel(const cx<double>* __restrict__ ws, double* __restrict__ out, int64_t nevt, int ngood,
                          double norm, int per_hel, const int64_t* __restrict__ nevt_dev, int64_t e0) {
  const int lane = threadIdx.x & 63;
  nevt = sub_batch_events(nevt, nevt_dev, e0);
  const int64_t ev = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (ev >= nevt) return;  // wave-uniform; no barrier follows
  const cx<double>* w = ws + (size_t)ev * Proc::nslot * Proc::nhel;
  double acc = 0.0;
  for (int k = lane; k < ngood; k += 64) {
    const double v = colour_sum_blocked<Proc, kColourBlock>(WsColumn<double>::template make<Proc>(w, k));
    if (per_hel) out[(size_t)ev * ngood + k] = v;
    acc += v;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (!per_hel && lane == 0) out[ev] = acc * norm;
}

// Select: also picks one helicity and one colour flow per event (the rule of
// choose_helicity_and_flow, with up to NPASS helicities per lane): |M_h|^2 of each pass is
// kept in registers, the flow weights sum_h |J_c,h|^2 are summed over the wavefront by
// recursive halving and accumulated in LDS.  sel's pointers are offset to the sub-batch's
// first event.  (Measured: with the choice this kernel takes about three times its plain
// time, most of that already with the helicity part alone; a separate kernel for the flow
// weights, gathering the jamps again, was slower.)
template <class Proc, bool Select, class S>
__global__ void __launch_bounds__(256)
    colour_mfma_kernel(const cx<S>* __restrict__ ws, double* __restrict__ out, int64_t nevt, int ngood,
                       double norm, int per_hel, const int64_t* __restrict__ nevt_dev, int64_t e0,
                       const int* __restrict__ goodhel, SelectArgs sel) {
  constexpr int NCOL = Proc::ncol;
  constexpr int NPASS = (Proc::nhel + 63) / 64;
  __shared__ __attribute__((aligned(16))) __bf16 nh[ColourTiles<Proc>::words];
  __shared__ __attribute__((aligned(16))) __bf16 nl[ColourTiles<Proc>::words];
  __shared__ double wflow[Select ? 4 : 1][Select ? NCOL : 1];
  nevt = sub_batch_events(nevt, nevt_dev, e0);
  if ((int64_t)blockIdx.x * 4 >= nevt) return;  // uniform per block
  colour_tiles_fill<Proc>(nh, nl, threadIdx.x, 256);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ev = (int64_t)blockIdx.x * 4 + wib;
  if (ev >= nevt) return;  // wave-uniform; no barrier follows
  const cx<S>* w = ws + (size_t)ev * Proc::nslot * Proc::nhel;
  double acc = 0.0;
  [[maybe_unused]] double mpass[Select ? NPASS : 1];
  if constexpr (Select) {
    for (int c = lane; c < NCOL; c += 64) wflow[wib][c] = 0.0;
    wave_lds_sync();
  }
  for (int g = 0; g < ngood; g += 64) {
    const int k = g + lane;
    const bool valid = k < ngood;
    cx<float> jamp[NCOL];
    gather_column<Proc, float, S>(w, valid ? k : 0, jamp);
    if (!valid) {
#pragma unroll
      for (int f = 0; f < NCOL; ++f) jamp[f] = {0.f, 0.f};
    }
    const float s = colour_sum_wave<Proc>(jamp, NumerLds<Proc>{(const HME_LDS __bf16*)nh, (const HME_LDS __bf16*)nl});
    if (per_hel && valid) out[(size_t)ev * ngood + k] = (double)s;
    acc += valid ? (double)s : 0.0;
    if constexpr (Select) {
#pragma unroll
      for (int q = 0; q < NPASS; ++q)
        if (q == g / 64) mpass[q] = valid ? (double)s : 0.0;
      // flow weights |J_c|^2 summed over the wavefront (invalid lanes hold zero jamps)
      add_flow_weights<NCOL, float>(jamp, lane, (volatile HME_LDS double*)&wflow[wib][0]);
    }
  }
  if constexpr (Select) {
    const int npass = (ngood + 63) / 64;
    for (int q = npass; q < NPASS; ++q) mpass[q] = 0.0;
    // helicity: total, then a running sum over the passes in good-helicity order
    double tot = 0.0;
#pragma unroll
    for (int q = 0; q < NPASS; ++q) tot += mpass[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off, 64);
    const double target_h = sel.rnd_hel[ev] * tot;
    double carry = 0.0;
    int kh = -1;
#pragma unroll
    for (int q = 0; q < NPASS; ++q) {
      double cum = mpass[q];
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const double t = __shfl_up(cum, d, 64);
        if (lane >= d) cum += t;
      }
      cum += carry;
      const uint64_t hit = __ballot(q * 64 + lane < ngood && cum > target_h);
      if (kh < 0 && hit) kh = q * 64 + __builtin_ctzll(hit);
      carry = __shfl(cum, 63, 64);
    }
    if (kh < 0) kh = ngood - 1;
    // colour flow: lane 0 runs over the LDS weights in flow order
    wave_lds_sync();
    if (lane == 0) {
      sel.sel_hel[ev] = goodhel[kh];
      sel.sel_col[ev] = choose_flow((volatile HME_LDS double*)&wflow[wib][0], NCOL, sel.rnd_col[ev]);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (!per_hel && lane == 0) out[ev] = acc * norm;
}

struct ChunkArgs {
  const double* mom;  // momenta of the sub-batch's first event
  void* ws;           // workspace, nevt * nslot * nhel entries of cx<float> (f64 = 0) or cx<double>
  int64_t nevt;       // events in the sub-batch
  const int* goodhel;
  int ngood;
  ProcParams prm;
  hipStream_t stream;
  const int64_t* nevt_dev;  // if set: the batch's event count (device), of which this sub-batch
  int64_t e0;               // starts at event e0
  int f64 = 0;              // double-precision amplitudes and workspace
};

template <class Proc> constexpr int chunk_lpe() { return Proc::nhel >= 64 ? 64 : 32; }

template <class Proc, class Chunk> hipError_t launch_chunk(const ChunkArgs& a) {
  constexpr int LPE = chunk_lpe<Proc>(), EPB = 256 / LPE;
  const int64_t blocks = (a.nevt + EPB - 1) / EPB;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (a.f64)
    chunk_kernel<Proc, Chunk, LPE, double><<<dim3((unsigned)blocks), dim3(256), 0, a.stream>>>(
        a.mom, static_cast<cx<double>*>(a.ws), a.nevt, a.goodhel, a.ngood, a.prm, a.nevt_dev, a.e0);
  else
    chunk_kernel<Proc, Chunk, LPE, float><<<dim3((unsigned)blocks), dim3(256), 0, a.stream>>>(
        a.mom, static_cast<cx<float>*>(a.ws), a.nevt, a.goodhel, a.ngood, a.prm, a.nevt_dev, a.e0);
  return hipGetLastError();
}

// colour sum of the workspace (cx<S>): on the matrix cores (mfma != 0, single precision) or on
// the vector ALUs in the type C
template <class Proc, class S, class C>
hipError_t launch_colour(const cx<S>* ws, double* out, int64_t nevt, int ngood, double norm, int per_hel,
                         const int64_t* nevt_dev, int64_t e0, hipStream_t s, int mfma, const int* goodhel = nullptr,
                         const SelectArgs& sel = SelectArgs{}) {
  constexpr int LPE = chunk_lpe<Proc>(), EPB = 256 / LPE;
  const int64_t blocks = (nevt + EPB - 1) / EPB;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (sel.sel_hel && (!mfma || per_hel || !goodhel || ngood > Proc::nhel)) return hipErrorInvalidValue;
  if (mfma) {
    static_assert(LPE == 64, "the matrix-core colour sum takes one event per wavefront");
    if (sel.sel_hel)
      colour_mfma_kernel<Proc, true, S><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(ws, out, nevt, ngood, norm,
                                                                                      per_hel, nevt_dev, e0, goodhel, sel);
    else
      colour_mfma_kernel<Proc, false, S><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(ws, out, nevt, ngood, norm,
                                                                                       per_hel, nevt_dev, e0, goodhel, sel);
  } else if constexpr (sizeof(S) == 8 && sizeof(C) == 8) {
    static_assert(LPE == 64, "one event per wavefront");
    // (the fold writes the workspace in place)
    fold_kernel<Proc><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(const_cast<cx<S>*>(ws), nevt, ngood, nevt_dev, e0);
    colour_blocked_kernel<Proc><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(ws, out, nevt, ngood, norm, per_hel,
                                                                             nevt_dev, e0);
  } else {
    colour_kernel<Proc, LPE, S, C><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(ws, out, nevt, ngood, norm, per_hel,
                                                                                 nevt_dev, e0);
  }
  return hipGetLastError();
}

}  // namespace hme
