// Kernels of a process evaluated in pieces (gg -> t tbar g g g): the piece kernels, the
// jamp workspace they write, and the colour kernels over it, among them the colour sum on
// the matrix cores.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "me2_kernels.h"

namespace hme {

// ------------------------------------------------- colour sum on the matrix cores
//
// The 120-flow colour sum of the pieces' process as a matrix product: per event, the
// jamps of 64 helicities form J (flows x helicities, real and imaginary parts apart),
// Z = N J with N the integer colour numerators, and |M_h|^2 * denom = sum over flows of
// J (.) Z in column h (N is symmetric).  Z runs on v_mfma_f32_32x32x16_bf16 with FP32
// accumulation: each J entry is split into three bf16 terms (hi + mid + lo carry its 24
// bits) and each numerator into two (hi + lo == N exactly), and the four products that
// matter at FP32 precision are accumulated (N_lo x J_lo, below 2^-24 relative, is left
// out).  One wavefront per event; lanes l and l ^ 32 exchange the halves of their jamp
// columns that the operand layouts assign to the other (A: lane l holds row l % 32,
// k = 8 (l / 32) .. + 7; B: column l % 32, the same k; C: register r of lane l holds row
// 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32).

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

// Exchange halves between lanes l and l ^ 32 (v_permlane32_swap): afterwards a holds
// (a of lanes 0-31, b of lanes 0-31) and b holds (a of lanes 32-63, b of lanes 32-63).
// The empty asm keeps the compiler from sharing one exchange (and the operands built
// from it) between row tiles, which would keep them all live at once.
HME_FN void swap_halves(float& a, float& b) {
  asm volatile("" : "+v"(a), "+v"(b));
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}

// x = h + m + l to about 24 significant bits, each term a bf16
HME_FN void split_bf16x3(float x, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)x;
  const float r = x - (float)h;
  m = (__bf16)r;
  l = (__bf16)(r - (float)m);
}

// One 32-row tile of Z = N J (rows 32 MTI .. + 31) and its contraction with J; see
// colour_mfma_kernel.  jv(p, f) is part p (0 re, 1 im) of this lane's jamp of flow f.
// K chunk kc (flows 16 kc .. + 15) of one row tile: z[t][p] += N[rows, chunk] J_p[chunk, tile t]
template <int mt, int S, int kc, class JV>
HME_FN void colour_k_chunk(const JV& jv, const HME_LDS __bf16* nh, const HME_LDS __bf16* nl, int col, int half,
                           f32x16_t (&z)[2][2]) {
  const int ro = (32 * mt + col) * S + 16 * kc + 8 * half;
  const bf16x8_t ah = *reinterpret_cast<const HME_LDS bf16x8_t*>(&nh[ro]);
  const bf16x8_t al = *reinterpret_cast<const HME_LDS bf16x8_t*>(&nl[ro]);
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    // B operands: tile 0 holds the helicities of lanes 0-31, tile 1 those of lanes 32-63;
    // lane l supplies flows 16 kc + 8 (l / 32) + j of column l % 32
    bf16x8_t b[2][3];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      float x0 = jv(p, 16 * kc + j), x1 = jv(p, 16 * kc + 8 + j);
      swap_halves(x0, x1);
      __bf16 h, m, l;
      split_bf16x3(x0, h, m, l);
      b[0][0][j] = h;
      b[0][1][j] = m;
      b[0][2][j] = l;
      split_bf16x3(x1, h, m, l);
      b[1][0][j] = h;
      b[1][1][j] = m;
      b[1][2][j] = l;
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      z[t][p] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, b[t][0], z[t][p], 0, 0, 0);
      z[t][p] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, b[t][1], z[t][p], 0, 0, 0);
      z[t][p] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, b[t][2], z[t][p], 0, 0, 0);
      z[t][p] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, b[t][0], z[t][p], 0, 0, 0);
      z[t][p] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, b[t][1], z[t][p], 0, 0, 0);
    }
  }
}

template <int mt, int S, class JV, int... KCI>
HME_FN void colour_k_chunks(std::integer_sequence<int, KCI...>, const JV& jv, const HME_LDS __bf16* nh,
                            const HME_LDS __bf16* nl, int col, int half, f32x16_t (&z)[2][2]) {
  (colour_k_chunk<mt, S, KCI>(jv, nh, nl, col, half, z), ...);
}

template <int MTI, int NC, int S, class JV>
HME_FN void colour_row_tile(const JV& jv, const HME_LDS __bf16* nh, const HME_LDS __bf16* nl, int col, int half,
                            float& s0, float& s1) {
  constexpr int mt = MTI, KC = NC / 16;
  f32x16_t z[2][2];  // [helicity tile][re, im]: rows 32 mt .. + 31 of Z
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int r = 0; r < 16; ++r) z[t][p][r] = 0.f;
  colour_k_chunks<mt, S>(std::make_integer_sequence<int, KC>{}, jv, nh, nl, col, half, z);
  // contract: register r of lane l holds row f0 + 4 (l / 32) of Z, f0 as below, in the
  // column l % 32 of each tile; the matching jamps come from the same exchange
#pragma unroll
  for (int p = 0; p < 2; ++p) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int f0 = 32 * mt + 8 * (r / 4) + r % 4;
      float x0 = jv(p, f0), x1 = jv(p, f0 + 4);
      swap_halves(x0, x1);
      s0 += x0 * z[0][p][r];
      s1 += x1 * z[1][p][r];
    }
  }
}

template <int NC, int S, class JV, int... MTI>
HME_FN void colour_rows_impl(std::integer_sequence<int, MTI...>, const JV& jv, const HME_LDS __bf16* nh,
                             const HME_LDS __bf16* nl, int col, int half, float& s0, float& s1) {
  (colour_row_tile<MTI, NC, S>(jv, nh, nl, col, half, s0, s1), ...);
}

// Padded size and LDS layout of the colour numerators for the matrix-core colour sum.
template <class Proc> struct ColourTiles {
  static constexpr int NC = (Proc::ncol + 31) / 32 * 32;  // padded with zero rows and columns
  static constexpr int S = NC + 8;                        // row stride (bf16), a 16-byte multiple
  static constexpr int words = NC * S;                    // bf16 per table (hi and lo)
};

// Fill the two bf16 numerator tables (hi + lo == numerator exactly) in LDS; every thread
// of the block takes part, a barrier must follow.
template <class Proc> HME_FN void colour_tiles_fill(__bf16* nh, __bf16* nl, int tid, int nthreads) {
  constexpr int NCOL = Proc::ncol, NC = ColourTiles<Proc>::NC, S = ColourTiles<Proc>::S;
  for (int i = tid; i < NC * NC; i += nthreads) {
    const int r = i / NC, c = i % NC;
    const float v = (r < NCOL && c < NCOL) ? (float)Proc::numer[r * NCOL + c] : 0.f;
    const __bf16 h = (__bf16)v;
    nh[r * S + c] = h;
    nl[r * S + c] = (__bf16)(v - (float)h);
  }
}

// Colour sum (times colour_denom) of this lane's helicity on the matrix cores.  All 64
// lanes of the wavefront must call it together, each with its own helicity's jamps
// (zeros for a lane without one).
template <class Proc>
HME_FN float colour_sum_wave(const cx<float> (&jamp)[Proc::ncol], const __bf16* nh, const __bf16* nl) {
  constexpr int NCOL = Proc::ncol, NC = ColourTiles<Proc>::NC, S = ColourTiles<Proc>::S, MT = NC / 32;
  const int lane = threadIdx.x & 63, col = lane & 31, half = lane >> 5;
  // part p (0 re, 1 im) of the jamp of flow f; zero in the padding
  auto jv = [&](int p, int f) -> float { return f < NCOL ? (p ? jamp[f].i : jamp[f].r) : 0.f; };
  // partial sums over this lane's rows for the column l % 32 of helicity tiles 0 and 1;
  // rows 32 mt .. + 31 of Z one tile at a time (a compile-time sequence, so that every
  // jamp index is a constant and the jamps stay in registers)
  float s0 = 0.f, s1 = 0.f;
  colour_rows_impl<NC, S>(std::make_integer_sequence<int, MT>{}, jv, (const HME_LDS __bf16*)nh,
                          (const HME_LDS __bf16*)nl, col, half, s0, s1);
  // lane l's helicity is column l % 32 of tile l / 32; its rows are split between l and l ^ 32
  swap_halves(s0, s1);
  return s0 + s1;
}

// 2 waves per SIMD at least (256 VGPRs + AGPRs): every generated schedule is sized for it
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

template <class Proc>
__global__ void __launch_bounds__(256)
    colour_mfma_kernel(const cx<float>* __restrict__ ws, double* __restrict__ out, int64_t nevt, int ngood,
                       double norm, int per_hel, const int64_t* __restrict__ nevt_dev, int64_t e0) {
  constexpr int NCOL = Proc::ncol;
  __shared__ __attribute__((aligned(16))) __bf16 nh[ColourTiles<Proc>::words];
  __shared__ __attribute__((aligned(16))) __bf16 nl[ColourTiles<Proc>::words];
  nevt = sub_batch_events(nevt, nevt_dev, e0);
  if ((int64_t)blockIdx.x * 4 >= nevt) return;  // uniform per block
  colour_tiles_fill<Proc>(nh, nl, threadIdx.x, 256);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ev = (int64_t)blockIdx.x * 4 + wib;
  if (ev >= nevt) return;  // wave-uniform; no barrier follows
  const cx<float>* w = ws + (size_t)ev * Proc::nslot * ngood;
  double acc = 0.0;
  for (int g = 0; g < ngood; g += 64) {
    const int k = g + lane;
    const bool valid = k < ngood;
    cx<float> jamp[NCOL];
    Proc::template gather<float, float>(w + (valid ? k : 0), ngood, jamp);
    if (!valid) {
#pragma unroll
      for (int f = 0; f < NCOL; ++f) jamp[f] = {0.f, 0.f};
    }
    const float s = colour_sum_wave<Proc>(jamp, nh, nl);
    if (per_hel && valid) out[(size_t)ev * ngood + k] = (double)s;
    acc += valid ? (double)s : 0.0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (!per_hel && lane == 0) out[ev] = acc * norm;
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

// colour sum of the workspace: on the matrix cores (mfma != 0) or on the vector ALUs
template <class Proc>
hipError_t launch_colour(const cx<float>* ws, double* out, int64_t nevt, int ngood, double norm, int per_hel,
                         const int64_t* nevt_dev, int64_t e0, hipStream_t s, int mfma) {
  constexpr int LPE = chunk_lpe<Proc>(), EPB = 256 / LPE;
  const int64_t blocks = (nevt + EPB - 1) / EPB;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (mfma) {
    static_assert(LPE == 64, "the matrix-core colour sum takes one event per wavefront");
    colour_mfma_kernel<Proc><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(ws, out, nevt, ngood, norm, per_hel,
                                                                           nevt_dev, e0);
  } else {
    colour_kernel<Proc, LPE><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(ws, out, nevt, ngood, norm, per_hel,
                                                                           nevt_dev, e0);
  }
  return hipGetLastError();
}

}  // namespace hme
