// The C interface of include/hme.h: handle life cycle, parameter derivation,
// the good-helicity filter and kernel dispatch.
#include "../../include/hme.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "me2_kernels.h"
#include "params.h"

namespace hme {
#define HME_DECLARE(NAME)                                                          \
  ProcInfo info_##NAME();                                                          \
  hipError_t launch_me2_##NAME(const LaunchArgs& a, int precision);                \
  hipError_t launch_hel_##NAME(const double* mom, int nev, const ProcParams& prm, \
                               double* out, hipStream_t s);
HME_DECLARE(eemumu)
HME_DECLARE(ggtt)
HME_DECLARE(ggttg)
HME_DECLARE(ggttgg)
HME_DECLARE(ggttggg)
HME_DECLARE(uuee)
HME_DECLARE(uueeg)
HME_DECLARE(uueegg)
HME_DECLARE(uueeggg)
#undef HME_DECLARE
ProcInfo info_ggttg_fd();
hipError_t launch_me2_ggttg_fd(const LaunchArgs& a, int precision);
ProcInfo info_ggttgg_fd();
hipError_t launch_me2_ggttgg_fd(const LaunchArgs& a, int precision);

struct ProcEntry {
  ProcInfo (*info)();
  hipError_t (*me2)(const LaunchArgs&, int);
  hipError_t (*hel)(const double*, int, const ProcParams&, double*, hipStream_t);
  bool qcd;            // g g -> t tbar + n g: massive final quarks (otherwise every particle is massless)
  double sample_sqrt_s;  // energy of the internal helicity-filter sample
  ProcInfo (*info_fd)() = nullptr;  // the process in the Feynman-diagram gauge, if built
  hipError_t (*me2_fd)(const LaunchArgs&, int) = nullptr;
};

static const ProcEntry kProcs[] = {
    {info_eemumu, launch_me2_eemumu, launch_hel_eemumu, false, 500.0},
    {info_ggtt, launch_me2_ggtt, launch_hel_ggtt, true, 1000.0},
    {info_ggttg, launch_me2_ggttg, launch_hel_ggttg, true, 1500.0, info_ggttg_fd, launch_me2_ggttg_fd},
    {info_ggttgg, launch_me2_ggttgg, launch_hel_ggttgg, true, 2000.0, info_ggttgg_fd, launch_me2_ggttgg_fd},
    {info_ggttggg, launch_me2_ggttggg, launch_hel_ggttggg, true, 2000.0},
    {info_uuee, launch_me2_uuee, launch_hel_uuee, false, 1000.0},
    {info_uueeg, launch_me2_uueeg, launch_hel_uueeg, false, 1000.0},
    {info_uueegg, launch_me2_uueegg, launch_hel_uueegg, false, 1000.0},
    {info_uueeggg, launch_me2_uueeggg, launch_hel_uueeggg, false, 1000.0},
};

// events per sub-batch of a process evaluated in pieces (workspace nslot * nhel * sizeof(cx) bytes
// each: 13 GB in single, 26 GB in double precision).  Measured per 65,536 events of g g -> t tbar
// g g g: FP64 152 / 132.5 ms and MIXED_PAPER 134.3 / 115.3 ms with sub-batches of 4,096 / 16,384
// events (the double pieces run at 1 wave/SIMD, and the fold at 4 waves/SIMD on 4,096 events
// did not fill the machine), MIXED_FAST 61.1 / 60.9 ms with 8,192 / 16,384.
constexpr int64_t kChunkSubBatch = 16384;
constexpr int64_t kChunkWorkspaceCap = int64_t(32) << 30;  // bytes
constexpr int kNumProcs = sizeof(kProcs) / sizeof(kProcs[0]);

}  // namespace hme

struct hme_handle {
  int process = 0, precision = 0, device = 0;
  bool gauge_fd = false;  // internal gluons in the Feynman-diagram gauge
  hme::ProcInfo info{};
  hme::ProcParams prm{};
  std::vector<int> goodhel;
  int* d_goodhel = nullptr;
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

}  // namespace

namespace hme {
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace hme

// Device scratch of hme_compute_noalloc: the jamp workspace of a process evaluated in pieces,
// for callers that cannot allocate.  One copy per device, held from the library's first use
// of that device until the process ends.  In host code `scratch` names a host-side stand-in,
// never the device copy: kernels and copies take the address kept in g_scratch_dev.
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};  // device address of `scratch` per device (null until looked up)

// Looks up this device's copy of `scratch` once; the device must be current.
hipError_t scratch_lookup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_dev[device] = ptr;
  return hipSuccess;
}

void* scratch_of(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_dev[device] : nullptr;
}

}  // namespace

namespace {

int hip_fail(hipError_t e, const char* what) {
  return fail(HME_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Restores the caller's current device when it goes out of scope.
struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// A few flat phase-space points (massless RAMBO, then a common rescaling of the
// three-momenta for the final-state masses) from a fixed seed.  Used only to
// find the vanishing helicities; it never sees user data.
std::vector<double> helicity_sample(const hme::ProcInfo& info, bool qcd, double mT, double sqrt_s, int nev) {
  const int npar = info.npar, nout = npar - 2;
  std::vector<double> masses(nout, 0.0);
  if (qcd) masses[0] = masses[1] = mT;
  std::mt19937_64 rng(0x6d655f68656cULL);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  auto u01 = [&]() {
    double x;
    do x = U(rng); while (x <= 0.0);
    return x;
  };
  std::vector<double> mom((size_t)nev * npar * 4, 0.0);
  const double pi = 3.14159265358979323846;
  for (int e = 0; e < nev; ++e) {
    double* ev = &mom[(size_t)e * npar * 4];
    ev[0] = ev[3] = sqrt_s / 2;
    ev[4] = sqrt_s / 2;
    ev[7] = -sqrt_s / 2;
    std::vector<double> q(4 * nout), P(4, 0.0);
    for (int i = 0; i < nout; ++i) {
      const double c = 2 * u01() - 1, s = std::sqrt(1 - c * c), f = 2 * pi * u01();
      const double q0 = -std::log(u01() * u01());
      q[4 * i + 0] = q0;
      q[4 * i + 1] = q0 * s * std::cos(f);
      q[4 * i + 2] = q0 * s * std::sin(f);
      q[4 * i + 3] = q0 * c;
      for (int mu = 0; mu < 4; ++mu) P[mu] += q[4 * i + mu];
    }
    const double M = std::sqrt(P[0] * P[0] - P[1] * P[1] - P[2] * P[2] - P[3] * P[3]);
    const double b[3] = {-P[1] / M, -P[2] / M, -P[3] / M};
    const double x = sqrt_s / M, g = P[0] / M, a = 1 / (1 + g);
    std::vector<double> k(4 * nout);
    for (int i = 0; i < nout; ++i) {
      const double* qi = &q[4 * i];
      const double bq = b[0] * qi[1] + b[1] * qi[2] + b[2] * qi[3];
      for (int j = 0; j < 3; ++j) k[4 * i + 1 + j] = x * (qi[1 + j] + b[j] * qi[0] + a * bq * b[j]);
      k[4 * i] = x * (g * qi[0] + bq);
    }
    double xi = 1.0;
    for (int it = 0; it < 100; ++it) {
      double f = -sqrt_s, df = 0;
      for (int i = 0; i < nout; ++i) {
        const double E = std::sqrt(masses[i] * masses[i] + xi * xi * k[4 * i] * k[4 * i]);
        f += E;
        df += xi * k[4 * i] * k[4 * i] / E;
      }
      xi -= f / df;
    }
    for (int i = 0; i < nout; ++i) {
      double* o = ev + 4 * (2 + i);
      for (int j = 1; j < 4; ++j) o[j] = xi * k[4 * i + j];
      o[0] = std::sqrt(masses[i] * masses[i] + o[1] * o[1] + o[2] * o[2] + o[3] * o[3]);
    }
  }
  return mom;
}

}  // namespace

extern "C" {

const char* hme_last_error(void) { return g_last_error.c_str(); }

int hme_create(int process, const hme_sm_card* card, int precision, int device, hme_handle** out) {
  if (!out) return fail(HME_E_ARG, "hme_create: out is NULL");
  *out = nullptr;
  if (!card) return fail(HME_E_ARG, "hme_create: card is NULL");
  if (process < 0 || process >= hme::kNumProcs) return fail(HME_E_ARG, "hme_create: unknown process");
  const bool gauge_fd = (precision & HME_GAUGE_FD) != 0;
  precision &= ~HME_GAUGE_FD;
  if (precision != HME_FP64 && precision != HME_MIXED_FAST && precision != HME_MIXED_PAPER)
    return fail(HME_E_ARG, "hme_create: unknown precision");
  if (gauge_fd && !hme::kProcs[process].me2_fd)
    return fail(HME_E_UNSUPPORTED, "hme_create: this process is not built in the Feynman-diagram gauge");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(e, "hme_create: hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(HME_E_ARG, "hme_create: no such device");
  hme::ProcParams prm;
  std::string why;
  if (!hme::derive_params(*card, prm, why)) return fail(HME_E_ARG, "hme_create: " + why);
  const hme::ProcEntry& P = hme::kProcs[process];
  DeviceGuard guard(device);
  if (guard.err != hipSuccess) return hip_fail(guard.err, "hme_create: hipSetDevice");

  if ((e = scratch_lookup(device)) != hipSuccess) return hip_fail(e, "hme_create: scratch address");

  auto* h = new hme_handle;
  h->process = process;
  h->precision = precision;
  h->device = device;
  h->info = gauge_fd ? P.info_fd() : P.info();
  h->gauge_fd = gauge_fd;
  h->prm = prm;

  // good-helicity filter on the internal sample
  const int nev = 16, nhel = h->info.nhel;
  std::vector<double> mom = helicity_sample(h->info, P.qcd, prm.mT, P.sample_sqrt_s, nev);
  std::vector<double> mh((size_t)nev * nhel);
  double *d_mom = nullptr, *d_out = nullptr;
  auto cleanup = [&]() {
    if (d_mom) (void)hipFree(d_mom);
    if (d_out) (void)hipFree(d_out);
  };
  if ((e = hipMalloc(&d_mom, mom.size() * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&d_out, mh.size() * sizeof(double))) != hipSuccess) {
    cleanup();
    delete h;
    return fail(HME_E_OOM, std::string("hme_create: ") + hipGetErrorString(e));
  }
  if ((e = hipMemcpy(d_mom, mom.data(), mom.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = P.hel(d_mom, nev, prm, d_out, nullptr)) != hipSuccess ||
      (e = hipMemcpy(mh.data(), d_out, mh.size() * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess) {
    cleanup();
    delete h;
    return hip_fail(e, "hme_create: helicity filter");
  }
  cleanup();
  for (int k = 0; k < nhel; ++k) {
    bool nonzero = false;
    for (int ev = 0; ev < nev; ++ev) nonzero = nonzero || mh[(size_t)ev * nhel + k] != 0.0;
    if (nonzero) h->goodhel.push_back(k);
  }
  if (h->goodhel.empty()) {
    delete h;
    return fail(HME_E_HIP, "hme_create: every helicity vanished on the internal sample");
  }
  if ((e = hipMalloc(&h->d_goodhel, h->goodhel.size() * sizeof(int))) != hipSuccess) {
    delete h;
    return fail(HME_E_OOM, std::string("hme_create: ") + hipGetErrorString(e));
  }
  if ((e = hipMemcpy(h->d_goodhel, h->goodhel.data(), h->goodhel.size() * sizeof(int), hipMemcpyHostToDevice)) !=
      hipSuccess) {
    (void)hipFree(h->d_goodhel);
    delete h;
    return hip_fail(e, "hme_create: upload helicities");
  }
  *out = h;
  return HME_OK;
}

}  // extern "C"

namespace hme {

// me2[i] *= (4 pi alpha_s[i])^power, one thread per event
__global__ void __launch_bounds__(256)
    alpha_scale_kernel(double* __restrict__ me2, const double* __restrict__ alpha_s, int64_t nevt, int power) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nevt) return;
  const double gs2 = 4 * 3.14159265358979323846 * alpha_s[i];
  double f = 1.0;
  for (int k = 0; k < power; ++k) f *= gs2;
  me2[i] *= f;
}

hipError_t launch_alpha_scale(double* me2, const double* alpha_s, int64_t nevt, int power, hipStream_t s) {
  const int64_t blocks = (nevt + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  alpha_scale_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(me2, alpha_s, nevt, power);
  return hipGetLastError();
}

double handle_norm(const hme_handle* h, double alpha_s) {
  const double pi = 3.14159265358979323846;
  const double gs2 = 4 * pi * alpha_s;
  double norm = 1.0 / (h->info.iden * h->info.colour_denom);
  for (int k = 0; k < h->info.gs_power / 2; ++k) norm *= gs2;
  return norm;
}

int handle_npar(const hme_handle* h) { return h->info.npar; }

bool handle_chunked(const hme_handle* h) { return h->info.nchunk > 0; }

// workspace bytes per event of a sub-batch (0 for a process evaluated in one kernel): a complex
// partial jamp per slot and good helicity, in the type of the amplitudes
int64_t handle_ws_bytes_per_event(const hme_handle* h) {
  const int64_t real = h->precision == HME_MIXED_FAST ? (int64_t)sizeof(float) : (int64_t)sizeof(double);
  return handle_chunked(h) ? (int64_t)h->info.nslot * (int64_t)h->info.nhel * 2 * real : 0;
}

hipError_t launch_for_handle(const hme_handle* h, int64_t nevt_grid, const int64_t* nevt_dev, const double* mom,
                             double* out, double norm, hipStream_t s, void* ws, int64_t ws_events,
                             const SelectArgs& sel) {
  LaunchArgs a{mom, out, nevt_grid, h->d_goodhel, (int)h->goodhel.size(), h->prm, norm, s,
               h->precision == HME_MIXED_PAPER ? 1 : 0, nevt_dev, ws, ws_events, sel};
  return (h->gauge_fd ? kProcs[h->process].me2_fd : kProcs[h->process].me2)(a, h->precision);
}

hipError_t launch_for_handle(const hme_handle* h, int64_t nevt_grid, const int64_t* nevt_dev, const double* mom,
                             double* out, double norm, hipStream_t s, void* ws, int64_t ws_events) {
  return launch_for_handle(h, nevt_grid, nevt_dev, mom, out, norm, s, ws, ws_events, SelectArgs{});
}

}  // namespace hme

extern "C" {

static int compute_impl(const char* who, hme_handle* h, double norm, int64_t nevt, const double* momenta,
                        double* me2, void* hip_stream, const hme::SelectArgs& sel) {
  const std::string w(who);
  DeviceGuard guard(h->device);
  if (guard.err != hipSuccess) return hip_fail(guard.err, (w + ": hipSetDevice").c_str());
  const auto stream = static_cast<hipStream_t>(hip_stream);
  void* ws = nullptr;
  int64_t ws_events = 0;
  hipError_t e;
  if (hme::handle_chunked(h)) {
    // jamp workspace, allocated and released in stream order
    // at most kChunkSubBatch events and kChunkWorkspaceCap bytes per sub-batch
    const int64_t cap = std::min<int64_t>(hme::kChunkSubBatch, hme::kChunkWorkspaceCap / hme::handle_ws_bytes_per_event(h));
    ws_events = nevt < cap ? nevt : cap;
    const size_t bytes = (size_t)ws_events * (size_t)hme::handle_ws_bytes_per_event(h);
    if ((e = hipMallocAsync(&ws, bytes, stream)) != hipSuccess)
      return fail(HME_E_OOM, w + ": workspace: " + hipGetErrorString(e));
  }
  e = hme::launch_for_handle(h, nevt, nullptr, momenta, me2, norm, stream, ws, ws_events, sel);
  if (ws) {
    const hipError_t ef = hipFreeAsync(ws, stream);
    if (e == hipSuccess) e = ef;
  }
  if (e != hipSuccess) return hip_fail(e, (w + ": launch").c_str());
  return HME_OK;
}

int hme_compute(hme_handle* h, double alpha_s, int64_t nevt, const double* momenta, double* me2, void* hip_stream) {
  if (!h) return fail(HME_E_ARG, "hme_compute: handle is NULL");
  if (nevt < 0) return fail(HME_E_ARG, "hme_compute: nevt < 0");
  if (nevt == 0) return HME_OK;
  if (!momenta || !me2) return fail(HME_E_ARG, "hme_compute: NULL momenta or me2");
  if ((reinterpret_cast<uintptr_t>(momenta) | reinterpret_cast<uintptr_t>(me2)) & 7u)
    return fail(HME_E_ARG, "hme_compute: pointers must be 8-byte aligned");
  if (!(alpha_s > 0)) return fail(HME_E_ARG, "hme_compute: alpha_s must be positive");
  return compute_impl("hme_compute", h, hme::handle_norm(h, alpha_s), nevt, momenta, me2, hip_stream,
                      hme::SelectArgs{});
}

int hme_compute_noalloc(hme_handle* h, double alpha_s, int64_t nevt, const double* momenta, double* me2,
                        void* hip_stream) {
  if (!h) return fail(HME_E_ARG, "hme_compute_noalloc: handle is NULL");
  if (nevt < 0) return fail(HME_E_ARG, "hme_compute_noalloc: nevt < 0");
  if (nevt == 0) return HME_OK;
  if (!momenta || !me2) return fail(HME_E_ARG, "hme_compute_noalloc: NULL momenta or me2");
  if ((reinterpret_cast<uintptr_t>(momenta) | reinterpret_cast<uintptr_t>(me2)) & 7u)
    return fail(HME_E_ARG, "hme_compute_noalloc: pointers must be 8-byte aligned");
  if (!(alpha_s > 0)) return fail(HME_E_ARG, "hme_compute_noalloc: alpha_s must be positive");
  DeviceGuard guard(h->device);
  if (guard.err != hipSuccess) return hip_fail(guard.err, "hme_compute_noalloc: hipSetDevice");
  void* ws = nullptr;
  int64_t ws_events = 0;
  if (hme::handle_chunked(h)) {
    // sub-batches as large as the scratch holds, a multiple of the colour kernel's 4 events per block
    const int64_t per_event = hme::handle_ws_bytes_per_event(h);
    ws_events = (int64_t)(kScratchBytes / (size_t)per_event) / 4 * 4;
    if (ws_events < 4)
      return fail(HME_E_BUDGET, "hme_compute_noalloc: the workspace of 4 events exceeds the 256 MiB scratch");
    if (ws_events > nevt) ws_events = nevt;
    ws = scratch_of(h->device);
    if (!ws) return fail(HME_E_HIP, "hme_compute_noalloc: no scratch address for this device");
  }
  const hipError_t e = hme::launch_for_handle(h, nevt, nullptr, momenta, me2, hme::handle_norm(h, alpha_s),
                                              static_cast<hipStream_t>(hip_stream), ws, ws_events);
  if (e != hipSuccess) return hip_fail(e, "hme_compute_noalloc: launch");
  return HME_OK;
}

int hme_compute_alphas(hme_handle* h, const double* alpha_s, int64_t nevt, const double* momenta, double* me2,
                       void* hip_stream) {
  if (!h) return fail(HME_E_ARG, "hme_compute_alphas: handle is NULL");
  if (nevt < 0) return fail(HME_E_ARG, "hme_compute_alphas: nevt < 0");
  if (nevt == 0) return HME_OK;
  if (!momenta || !me2 || !alpha_s) return fail(HME_E_ARG, "hme_compute_alphas: NULL buffer");
  if ((reinterpret_cast<uintptr_t>(momenta) | reinterpret_cast<uintptr_t>(me2) | reinterpret_cast<uintptr_t>(alpha_s)) &
      7u)
    return fail(HME_E_ARG, "hme_compute_alphas: pointers must be 8-byte aligned");
  // |M|^2 without the coupling (g_s = 1), then each event times (4 pi alpha_s[i])^(power / 2)
  const int rc = compute_impl("hme_compute_alphas", h, 1.0 / (h->info.iden * h->info.colour_denom), nevt, momenta,
                              me2, hip_stream, hme::SelectArgs{});
  if (rc != HME_OK) return rc;
  const hipError_t e = hme::launch_alpha_scale(me2, alpha_s, nevt, h->info.gs_power / 2,
                                               static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "hme_compute_alphas: launch");
  return HME_OK;
}

int hme_compute_select(hme_handle* h, double alpha_s, int64_t nevt, const double* momenta, const double* rnd_hel,
                       const double* rnd_col, double* me2, int* sel_hel, int* sel_col, void* hip_stream) {
  if (!h) return fail(HME_E_ARG, "hme_compute_select: handle is NULL");
  if (nevt < 0) return fail(HME_E_ARG, "hme_compute_select: nevt < 0");
  if (nevt == 0) return HME_OK;
  if (!momenta || !me2 || !rnd_hel || !rnd_col || !sel_hel || !sel_col)
    return fail(HME_E_ARG, "hme_compute_select: NULL buffer");
  if (((reinterpret_cast<uintptr_t>(momenta) | reinterpret_cast<uintptr_t>(me2) | reinterpret_cast<uintptr_t>(rnd_hel) |
        reinterpret_cast<uintptr_t>(rnd_col)) & 7u) ||
      ((reinterpret_cast<uintptr_t>(sel_hel) | reinterpret_cast<uintptr_t>(sel_col)) & 3u))
    return fail(HME_E_ARG, "hme_compute_select: misaligned buffer");
  if (!(alpha_s > 0)) return fail(HME_E_ARG, "hme_compute_select: alpha_s must be positive");
  if (h->info.nchunk > 0 && h->precision == HME_FP64)
    return fail(HME_E_UNSUPPORTED, "hme_compute_select: gg -> ttbar ggg chooses at HME_MIXED_FAST or HME_MIXED_PAPER");
  return compute_impl("hme_compute_select", h, hme::handle_norm(h, alpha_s), nevt, momenta, me2, hip_stream,
                      hme::SelectArgs{rnd_hel, rnd_col, sel_hel, sel_col});
}

int hme_compute_channels(hme_handle* h, double alpha_s, int64_t nevt, const double* momenta, double* me2,
                         double* channel_weights, void* hip_stream) {
  if (!h) return fail(HME_E_ARG, "hme_compute_channels: handle is NULL");
  if (nevt < 0) return fail(HME_E_ARG, "hme_compute_channels: nevt < 0");
  if (h->info.nchunk > 0 || h->process == HME_EEMUMU || h->gauge_fd)
    return fail(HME_E_UNSUPPORTED, "hme_compute_channels: no channel weights for this process or gauge");
  if (nevt == 0) return HME_OK;
  if (!momenta || !me2 || !channel_weights) return fail(HME_E_ARG, "hme_compute_channels: NULL buffer");
  if ((reinterpret_cast<uintptr_t>(momenta) | reinterpret_cast<uintptr_t>(me2) |
       reinterpret_cast<uintptr_t>(channel_weights)) & 7u)
    return fail(HME_E_ARG, "hme_compute_channels: pointers must be 8-byte aligned");
  if (!(alpha_s > 0)) return fail(HME_E_ARG, "hme_compute_channels: alpha_s must be positive");
  hme::SelectArgs sel{};
  sel.chan_w = channel_weights;
  return compute_impl("hme_compute_channels", h, hme::handle_norm(h, alpha_s), nevt, momenta, me2, hip_stream, sel);
}

int hme_query(const hme_handle* h, hme_info* info) {
  if (!h || !info) return fail(HME_E_ARG, "hme_query: NULL argument");
  std::memset(info, 0, sizeof *info);
  info->process = h->process;
  info->precision = h->precision;
  info->npar = h->info.npar;
  info->nhel = h->info.nhel;
  info->ngoodhel = (int)h->goodhel.size();
  info->ncol = h->info.ncol;
  info->ndiag = h->info.ndiag;
  info->namp = h->info.namp;
  info->iden = h->info.iden;
  info->flops_per_event = info->ngoodhel * h->info.flops_per_hel + h->info.flops_per_event;
  info->bytes_per_event = h->info.npar * 4 * sizeof(double) + sizeof(double);
  info->workspace_bytes_per_event = (double)hme::handle_ws_bytes_per_event(h);
  return HME_OK;
}

int hme_good_helicities(const hme_handle* h, int* out, int cap) {
  if (!h || (!out && cap > 0) || cap < 0) return fail(HME_E_ARG, "hme_good_helicities: bad argument");
  const int n = (int)h->goodhel.size();
  for (int k = 0; k < n && k < cap; ++k) out[k] = h->goodhel[k];
  return n;
}

int hme_destroy(hme_handle* h) {
  if (!h) return HME_OK;
  int rc = HME_OK;
  if (h->d_goodhel) {
    DeviceGuard guard(h->device);
    hipError_t e = hipFree(h->d_goodhel);
    if (e != hipSuccess) rc = hip_fail(e, "hme_destroy: hipFree");
  }
  delete h;
  return rc;
}

}  // extern "C"
