// FP64 colour sum of a process evaluated in pieces, over the jamps its workspace column holds
// after the fold (host and device code).
#pragma once

#include <cstdint>

#include "helas.h"

namespace hme {

// FP64 colour sum of one helicity column whose jamps the fold has left at the flows' first
// slots (Proc::jslot; entry s of the column at col[s * Proc::nhel]): the symmetric form
// sum_i N_ii |J_i|^2 + 2 sum_{i<j} N_ij Re(conj(J_i) J_j) taken over blocks of B flows, two blocks
// live at a time (the 120 double jamps of a helicity would need 480 registers at once).
template <class Proc, int B, class Col> HME_FN double colour_sum_blocked(const Col& col) {
  constexpr int NCOL = Proc::ncol, NB = (NCOL + B - 1) / B;
  double acc = 0.0;
  // the block loops stay loops (unrolled, the compiler would issue every block's loads at once)
#pragma unroll 1
  for (int bi = 0; bi < NB; ++bi) {
    cx<double> a[B];
#pragma unroll
    for (int i = 0; i < B; ++i)
      a[i] = bi * B + i < NCOL ? cast<double>(col[(int64_t)Proc::jslot[bi * B + i] * Proc::nhel]) : cx<double>{0.0, 0.0};
    // the diagonal block
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const int fi = bi * B + i;
      if (fi >= NCOL) break;
      double zr = 0.0, zi = 0.0;
#pragma unroll
      for (int j = i; j < B; ++j) {
        const int fj = bi * B + j;
        if (fj >= NCOL) break;
        const double n = (double)Proc::numer[fi * NCOL + fj] * (i == j ? 1.0 : 2.0);
        zr = fmadd(n, a[j].r, zr);
        zi = fmadd(n, a[j].i, zi);
      }
      acc = fmadd(a[i].r, zr, fmadd(a[i].i, zi, acc));
    }
    // the blocks to its right
#pragma unroll 1
    for (int bj = bi + 1; bj < NB; ++bj) {
      cx<double> b[B];
#pragma unroll
      for (int j = 0; j < B; ++j)
        b[j] = bj * B + j < NCOL ? cast<double>(col[(int64_t)Proc::jslot[bj * B + j] * Proc::nhel]) : cx<double>{0.0, 0.0};
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const int fi = bi * B + i;
        if (fi >= NCOL) break;
        double zr = 0.0, zi = 0.0;
#pragma unroll
        for (int j = 0; j < B; ++j) {
          const int fj = bj * B + j;
          if (fj >= NCOL) break;
          const double n = 2.0 * (double)Proc::numer[fi * NCOL + fj];
          zr = fmadd(n, b[j].r, zr);
          zi = fmadd(n, b[j].i, zi);
        }
        acc = fmadd(a[i].r, zr, fmadd(a[i].i, zi, acc));
      }
    }
  }
  return acc;
}

// flows per block of the FP64 colour sum: two blocks of 20 double jamps (160 registers) keep the
// kernel at 2 waves/SIMD (measured per 65,536 events of g g -> t tbar g g g: blocks of 12, 20
// and 24 flows 152.7, 151.9 and 161.4 ms; 16 compiles to re-reads of every jamp at each use)
constexpr int kColourBlock = 20;

}  // namespace hme
