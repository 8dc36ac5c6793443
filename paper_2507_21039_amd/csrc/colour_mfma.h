// Colour sum on the matrix cores, one wavefront of 64 helicity columns at a time; used by
// the 120-flow colour kernel and by the single-precision kernel of the 24-flow process.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "helas.h"

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
template <int mt, int kc, class JV, class AS>
HME_FN void colour_k_chunk(const JV& jv, const AS& numer, int col, int half, f32x16_t (&z)[2][2]) {
  bf16x8_t ah, al;
  numer.load(32 * mt + col, 16 * kc + 8 * half, ah, al);
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

template <int mt, class JV, class AS, int... KCI>
HME_FN void colour_k_chunks(std::integer_sequence<int, KCI...>, const JV& jv, const AS& numer, int col, int half,
                            f32x16_t (&z)[2][2]) {
  (colour_k_chunk<mt, KCI>(jv, numer, col, half, z), ...);
}

template <int MTI, int NC, class JV, class AS>
HME_FN void colour_row_tile(const JV& jv, const AS& numer, int col, int half, float& s0, float& s1) {
  constexpr int mt = MTI, KC = NC / 16;
  f32x16_t z[2][2];  // [helicity tile][re, im]: rows 32 mt .. + 31 of Z
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int r = 0; r < 16; ++r) z[t][p][r] = 0.f;
  colour_k_chunks<mt>(std::make_integer_sequence<int, KC>{}, jv, numer, col, half, z);
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

template <int NC, class JV, class AS, int... MTI>
HME_FN void colour_rows_impl(std::integer_sequence<int, MTI...>, const JV& jv, const AS& numer, int col, int half,
                             float& s0, float& s1) {
  (colour_row_tile<MTI, NC>(jv, numer, col, half, s0, s1), ...);
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

// The A operand: 8 numerators of one row as bf16 hi + lo, from the tables in LDS
template <class Proc> struct NumerLds {
  const HME_LDS __bf16* nh;
  const HME_LDS __bf16* nl;
  HME_FN void load(int row, int k0, bf16x8_t& ah, bf16x8_t& al) const {
    const int o = row * ColourTiles<Proc>::S + k0;
    ah = *reinterpret_cast<const HME_LDS bf16x8_t*>(&nh[o]);
    al = *reinterpret_cast<const HME_LDS bf16x8_t*>(&nl[o]);
  }
};

// Colour sum (times colour_denom) of this lane's helicity on the matrix cores.  All 64
// lanes of the wavefront must call it together, each with its own helicity's jamps
// (a lane without a helicity of its own may pass any finite values and drop the result:
// each helicity column of the product depends on that lane's jamps only).
template <class Proc, class AS>
HME_FN float colour_sum_wave(const cx<float> (&jamp)[Proc::ncol], const AS& numer) {
  constexpr int NCOL = Proc::ncol, NC = ColourTiles<Proc>::NC, MT = NC / 32;
  const int lane = threadIdx.x & 63, col = lane & 31, half = lane >> 5;
  // part p (0 re, 1 im) of the jamp of flow f; zero in the padding
  auto jv = [&](int p, int f) -> float { return f < NCOL ? (p ? jamp[f].i : jamp[f].r) : 0.f; };
  // partial sums over this lane's rows for the column l % 32 of helicity tiles 0 and 1;
  // rows 32 mt .. + 31 of Z one tile at a time (a compile-time sequence, so that every
  // jamp index is a constant and the jamps stay in registers)
  float s0 = 0.f, s1 = 0.f;
  colour_rows_impl<NC>(std::make_integer_sequence<int, MT>{}, jv, numer, col, half, s0, s1);
  // lane l's helicity is column l % 32 of tile l / 32; its rows are split between l and l ^ 32
  swap_halves(s0, s1);
  return s0 + s1;
}

}  // namespace hme
