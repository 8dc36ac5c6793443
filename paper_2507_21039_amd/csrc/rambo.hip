// Phase-space points on the device: flat n-body phase space (RAMBO, Kleiss, Stirling and
// Ellis, Comput. Phys. Commun. 40 (1986) 359) from counter-based random numbers
// (Philox4x32-10, Salmon et al., SC'11), one thread per event, written straight into the
// [nevt][npar][4] layout hme_compute reads.  The paper's standalone throughput includes
// this step (section "Standalone application"); here it stays on the GPU.
//
// Event i draws from Philox counter (i_lo, i_hi, attempt, block) with key (seed, "RAMB");
// each counter gives four 32-bit words, turned into two doubles in (0, 1) with 53 random
// bits each.  An event rejected by the cut moves on to the next attempt, so every event is
// a function of (seed, i) alone, independent of batch size, order and device.  Each point
// carries its phase-space weight (the massless volume times the massive correction of the
// RAMBO paper), and hme_weighted_sum reduces weight x |M|^2 to a flat Monte Carlo estimate
// of the cross section.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/hme.h"

namespace hme {
void set_last_error(const std::string& msg);
}

namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;
constexpr uint32_t kRamboKey = 0x52414D42u;  // "RAMB"
constexpr int kMaxAttempts = 10000;

__device__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(kPhiloxM0, c[0]), lo0 = kPhiloxM0 * c[0];
    const uint32_t hi1 = __umulhi(kPhiloxM1, c[2]), lo1 = kPhiloxM1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
}

// two doubles in (0, 1): 27 + 26 bits of two words each, offset by half an ulp
__device__ void uniform_pair(const uint32_t (&w)[4], double& u0, double& u1) {
  const double scale = 1.0 / 9007199254740992.0;  // 2^-53
  u0 = ((double)(w[0] >> 5) * 67108864.0 + (double)(w[1] >> 6) + 0.5) * scale;
  u1 = ((double)(w[2] >> 5) * 67108864.0 + (double)(w[3] >> 6) + 0.5) * scale;
}

__device__ double pseudorapidity(const double* p) {
  const double pt2 = p[1] * p[1] + p[2] * p[2];
  const double P = sqrt(pt2 + p[3] * p[3]);
  // 1/2 ln((P + pz) / (P - pz)), the small side rewritten to avoid cancellation
  const double plus = p[3] >= 0 ? P + p[3] : pt2 / fmax(P - p[3], 1e-300);
  const double minus = p[3] >= 0 ? pt2 / fmax(P + p[3], 1e-300) : P - p[3];
  return 0.5 * log(plus / minus);
}

struct FinalMasses {
  double m[5];
};

template <int NOUT>
__global__ void __launch_bounds__(256)
    rambo_kernel(double* __restrict__ mom, double* __restrict__ weight, int64_t first_event, int64_t nevt,
                 double sqrt_s, uint32_t seed, FinalMasses masses_in, double w0, int cut, double cut_value,
                 int max_attempts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nevt) return;
  double masses[NOUT];
  double msum = 0;
#pragma unroll
  for (int j = 0; j < NOUT; ++j) {
    masses[j] = masses_in.m[j];
    msum += masses[j];
  }
  const int64_t ev = first_event + i;
  const uint32_t lo = (uint32_t)((uint64_t)ev & 0xFFFFFFFFu), hi = (uint32_t)((uint64_t)ev >> 32);
  const double pi = 3.14159265358979323846;
  double* out = mom + i * (2 + NOUT) * 4;
  double k[NOUT][4];
  double wgt = w0;
  bool done = false;
  for (int attempt = 0; attempt < max_attempts && !done; ++attempt) {
    // isotropic massless momenta with exponential energies (4 uniforms per particle)
    double q[NOUT][4], Q[4] = {0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < NOUT; ++j) {
      double u[4];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        uint32_t c[4] = {lo, hi, (uint32_t)attempt, (uint32_t)(2 * j + b)};
        philox4x32_10(c, seed, kRamboKey);
        uniform_pair(c, u[2 * b], u[2 * b + 1]);
      }
      const double cth = 2 * u[0] - 1, sth = sqrt(fmax(0.0, 1 - cth * cth)), phi = 2 * pi * u[1];
      const double q0 = -log(u[2] * u[3]);
      q[j][0] = q0;
      q[j][1] = q0 * sth * cos(phi);
      q[j][2] = q0 * sth * sin(phi);
      q[j][3] = q0 * cth;
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) Q[mu] += q[j][mu];
    }
    // conformal transformation to the centre-of-mass frame at sqrt_s
    const double M = sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
    const double b[3] = {-Q[1] / M, -Q[2] / M, -Q[3] / M};
    const double x = sqrt_s / M, gamma = Q[0] / M, a = 1 / (1 + gamma);
    double P2[NOUT], E[NOUT];
#pragma unroll
    for (int j = 0; j < NOUT; ++j) {
      const double bq = b[0] * q[j][1] + b[1] * q[j][2] + b[2] * q[j][3];
      k[j][0] = x * (gamma * q[j][0] + bq);
#pragma unroll
      for (int d = 0; d < 3; ++d) k[j][1 + d] = x * (q[j][1 + d] + b[d] * q[j][0] + a * bq * b[d]);
      P2[j] = k[j][1] * k[j][1] + k[j][2] * k[j][2] + k[j][3] * k[j][3];
      E[j] = sqrt(P2[j]);
    }
    // common rescaling of the three-momenta that puts the massive particles on shell
    if (msum > 0) {
      double xi = sqrt(fmax(0.0, 1 - (msum / sqrt_s) * (msum / sqrt_s)));
      for (int it = 0; it < 100; ++it) {
        double f = -sqrt_s, df = 0;
#pragma unroll
        for (int j = 0; j < NOUT; ++j) {
          const double e = sqrt(masses[j] * masses[j] + xi * xi * P2[j]);
          f += e;
          df += xi * P2[j] / e;
        }
        const double step = f / df;
        xi -= step;
        // quadratic convergence: after a step this small the remaining error is below rounding
        if (fabs(step) <= 1e-14 * fabs(xi)) break;
      }
      // weight of the massive point: w0 xi^(2n-3) prod(|k_j| / E_j) sqrt_s / sum(|k_j|^2 / E_j)
      double prod = 1, sum = 0, xpow = xi;
#pragma unroll
      for (int j = 0; j < NOUT; ++j) {
#pragma unroll
        for (int d = 1; d < 4; ++d) k[j][d] *= xi;
        k[j][0] = sqrt(masses[j] * masses[j] + xi * xi * P2[j]);
        const double kabs = xi * E[j];
        prod *= kabs / k[j][0];
        sum += kabs * kabs / k[j][0];
      }
#pragma unroll
      for (int j = 1; j < NOUT - 1; ++j) xpow *= xi * xi;
      wgt = w0 * xpow * prod * sqrt_s / sum;
    } else {
#pragma unroll
      for (int j = 0; j < NOUT; ++j) k[j][0] = E[j];
    }
    // cuts on the first two final-state gluons (final-state particles 2 and 3)
    if (cut == HME_CUT_GLUON_PT && NOUT >= 3) {
      const int g = NOUT >= 3 ? 2 : 0;
      done = sqrt(k[g][1] * k[g][1] + k[g][2] * k[g][2]) > cut_value;
    } else if (cut == HME_CUT_GLUON_DR && NOUT >= 4) {
      const int g1 = NOUT >= 4 ? 2 : 0, g2 = NOUT >= 4 ? 3 : 0;
      const double deta = pseudorapidity(k[g1]) - pseudorapidity(k[g2]);
      double dphi = fabs(atan2(k[g1][2], k[g1][1]) - atan2(k[g2][2], k[g2][1]));
      if (dphi > pi) dphi = 2 * pi - dphi;
      done = sqrt(deta * deta + dphi * dphi) > cut_value;
    } else {
      done = true;
    }
  }
  // a single attempt (no retry) keeps a rejected point with weight 0; an event whose attempts
  // all failed gets NaN momenta and weight
  const bool keep = done || max_attempts == 1;
  const double half = 0.5 * sqrt_s, nan = __builtin_nan("");
  out[0] = half, out[1] = 0, out[2] = 0, out[3] = half;
  out[4] = half, out[5] = 0, out[6] = 0, out[7] = -half;
#pragma unroll
  for (int j = 0; j < NOUT; ++j)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) out[8 + 4 * j + mu] = keep ? k[j][mu] : nan;
  if (weight) weight[i] = done ? wgt : (keep ? 0.0 : nan);
}

// sum_i w_i m_i and sum_i (w_i m_i)^2 in one workgroup: a fixed order of additions, so the
// result does not depend on the launch or the run
constexpr int kSumThreads = 1024;

__global__ void __launch_bounds__(kSumThreads)
    weighted_sum_kernel(const double* __restrict__ me2, const double* __restrict__ weight, int64_t nevt,
                        double* __restrict__ out) {
  __shared__ double part[2][kSumThreads / 64];
  double s1 = 0, s2 = 0;
  // eight loads in flight per thread before the (sequential, fixed-order) additions
  constexpr int kBatch = 8;
  int64_t i = threadIdx.x;
  for (; i + (kBatch - 1) * kSumThreads < nevt; i += kBatch * kSumThreads) {
    double v[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) v[b] = weight[i + b * kSumThreads] * me2[i + b * kSumThreads];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      s1 += v[b];
      s2 += v[b] * v[b];
    }
  }
  for (; i < nevt; i += kSumThreads) {
    const double v = weight[i] * me2[i];
    s1 += v;
    s2 += v * v;
  }
  for (int off = 32; off > 0; off >>= 1) {
    s1 += __shfl_xor(s1, off);
    s2 += __shfl_xor(s2, off);
  }
  const int wave = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) part[0][wave] = s1, part[1][wave] = s2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0;
    for (int w = 0; w < kSumThreads / 64; ++w) a += part[0][w], b += part[1][w];
    out[0] = a;
    out[1] = b;
  }
}

template <int NOUT>
hipError_t launch_rambo(double* mom, double* weight, int64_t first_event, int64_t nevt, double sqrt_s, uint32_t seed,
                        const FinalMasses& masses, double w0, int cut, double cut_value, int max_attempts,
                        hipStream_t s) {
  const int64_t blocks = (nevt + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  rambo_kernel<NOUT><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(mom, weight, first_event, nevt, sqrt_s, seed, masses,
                                                                   w0, cut, cut_value, max_attempts);
  return hipGetLastError();
}

// massless n-body phase-space volume (2 pi)^(4 - 3n) (pi / 2)^(n - 1) s^(n - 2) / ((n - 1)! (n - 2)!)
double massless_volume(int n, double s) {
  const double pi = 3.14159265358979323846;
  double v = std::pow(2 * pi, 4 - 3 * n) * std::pow(pi / 2, n - 1) * std::pow(s, n - 2);
  for (int k = 2; k <= n - 1; ++k) v /= k;
  for (int k = 2; k <= n - 2; ++k) v /= k;
  return v;
}

int rambo_fail(int code, const std::string& msg) {
  hme::set_last_error(msg);
  return code;
}

}  // namespace

extern "C" int hme_rambo(int process, const hme_sm_card* card, double sqrt_s, uint64_t seed, int64_t first_event,
                         int64_t nevt, int cut, double cut_value, double* momenta, double* weights, void* hip_stream) {
  static const int kNout[] = {2, 2, 3, 4, 5, 2, 3, 4, 5};  // final-state particles per process
  if (process < 0 || process > HME_UUEEGGG) return rambo_fail(HME_E_ARG, "hme_rambo: unknown process");
  if (!card) return rambo_fail(HME_E_ARG, "hme_rambo: card is NULL");
  if (nevt < 0 || first_event < 0) return rambo_fail(HME_E_ARG, "hme_rambo: negative nevt or first_event");
  const int cut_kind = cut & ~HME_CUT_NO_RETRY;
  if ((cut & ~(HME_CUT_NO_RETRY | 0xff)) != 0 || cut_kind < HME_CUT_NONE || cut_kind > HME_CUT_GLUON_DR)
    return rambo_fail(HME_E_ARG, "hme_rambo: unknown cut");
  const int nout = kNout[process];
  // massive final-state top pair for g g -> t tbar + n g; every other final state is massless
  const bool tops = process >= HME_GGTT && process <= HME_GGTTGGG;
  const double mt = tops ? card->mT : 0.0;
  if (!(mt >= 0)) return rambo_fail(HME_E_ARG, "hme_rambo: negative top mass");
  if (!(sqrt_s > 2 * mt) || !(sqrt_s > 0) || !std::isfinite(sqrt_s))
    return rambo_fail(HME_E_ARG, "hme_rambo: sqrt_s not above the final-state masses");
  if (nevt == 0) return HME_OK;
  if (!momenta || (reinterpret_cast<uintptr_t>(momenta) & 7u) || (reinterpret_cast<uintptr_t>(weights) & 7u))
    return rambo_fail(HME_E_ARG, "hme_rambo: NULL or misaligned output buffer");
  const auto stream = static_cast<hipStream_t>(hip_stream);
  const FinalMasses fm{{mt, mt, 0, 0, 0}};
  const uint32_t key = (uint32_t)(seed & 0xFFFFFFFFu);
  const double w0 = massless_volume(nout, sqrt_s * sqrt_s);
  const int attempts = (cut & HME_CUT_NO_RETRY) ? 1 : kMaxAttempts;
  hipError_t e;
  switch (nout) {
    case 2: e = launch_rambo<2>(momenta, weights, first_event, nevt, sqrt_s, key, fm, w0, cut_kind, cut_value, attempts,
                                stream); break;
    case 3: e = launch_rambo<3>(momenta, weights, first_event, nevt, sqrt_s, key, fm, w0, cut_kind, cut_value, attempts,
                                stream); break;
    case 4: e = launch_rambo<4>(momenta, weights, first_event, nevt, sqrt_s, key, fm, w0, cut_kind, cut_value, attempts,
                                stream); break;
    default: e = launch_rambo<5>(momenta, weights, first_event, nevt, sqrt_s, key, fm, w0, cut_kind, cut_value,
                                 attempts, stream); break;
  }
  if (e != hipSuccess) return rambo_fail(HME_E_HIP, std::string("hme_rambo: ") + hipGetErrorString(e));
  return HME_OK;
}

extern "C" int hme_weighted_sum(const double* me2, const double* weights, int64_t nevt, double* out,
                                void* hip_stream) {
  if (nevt < 0) return rambo_fail(HME_E_ARG, "hme_weighted_sum: negative nevt");
  if (!out || (reinterpret_cast<uintptr_t>(out) & 7u))
    return rambo_fail(HME_E_ARG, "hme_weighted_sum: NULL or misaligned out");
  if (nevt > 0 && (!me2 || !weights || (reinterpret_cast<uintptr_t>(me2) & 7u) ||
                   (reinterpret_cast<uintptr_t>(weights) & 7u)))
    return rambo_fail(HME_E_ARG, "hme_weighted_sum: NULL or misaligned input");
  weighted_sum_kernel<<<dim3(1), dim3(kSumThreads), 0, static_cast<hipStream_t>(hip_stream)>>>(me2, weights, nevt,
                                                                                              out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return rambo_fail(HME_E_HIP, std::string("hme_weighted_sum: ") + hipGetErrorString(e));
  return HME_OK;
}

// Flat Monte Carlo cross section from the two sums of hme_weighted_sum (host arithmetic):
// sigma = (1 / (2 s)) (1 / N) sum_i w_i |M_i|^2, the flux factor of massless colliding
// partons times the mean of weight x |M|^2 (the integral over flat phase space of the paper's
// standalone application), converted from GeV^-2 to pb with (hbar c)^2 = 0.3893793721e9 GeV^2 pb;
// its error from the variance of w |M|^2 over the N points.
extern "C" int hme_flat_cross_section(const double* sums, int64_t npoints, double sqrt_s, double* sigma_pb,
                                      double* error_pb) {
  if (!sums || !sigma_pb || !error_pb) return rambo_fail(HME_E_ARG, "hme_flat_cross_section: NULL argument");
  if (npoints <= 0) return rambo_fail(HME_E_ARG, "hme_flat_cross_section: npoints must be positive");
  if (!(sqrt_s > 0)) return rambo_fail(HME_E_ARG, "hme_flat_cross_section: sqrt_s must be positive");
  constexpr double kGeV2ToPb = 0.3893793721e9;
  const double flux = 2.0 * sqrt_s * sqrt_s;
  const double n = (double)npoints;
  const double mean = sums[0] / n;
  double var = sums[1] / n - mean * mean;
  if (var < 0) var = 0;
  *sigma_pb = mean / flux * kGeV2ToPb;
  *error_pb = std::sqrt(var / n) / flux * kGeV2ToPb;
  return HME_OK;
}
