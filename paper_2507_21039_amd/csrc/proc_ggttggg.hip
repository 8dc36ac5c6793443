// g g -> t tbar g g g: the helicity filter, the colour kernel and the sequence of
// piece kernels (each piece in its own generated translation unit).
#include "piece_kernels.h"
#include "procs/ggttggg.h"
#include "procs/ggttggg_chunks.h"

namespace hme {

using P7 = P_ggttggg;
static_assert(sizeof(chunks_ggttggg) / sizeof(chunks_ggttggg[0]) == P7::nchunk, "piece table out of date");

ProcInfo info_ggttggg() { return make_info<P7>(); }

// the 120 x 120 colour sum on the matrix cores (bf16 splits, FP32 accumulation)
constexpr int kColourOnMatrixCores = 1;

// All pieces, then the colour sum, for consecutive sub-batches of ws_events events.  nevt
// sizes the launches; with nevt_dev set (a captured graph) the kernels take the batch's
// event count from device memory and sub-batches past its end do nothing.  precision: 1 single
// precision pieces and workspace, colour sum on the matrix cores; 0 double precision pieces and
// workspace, colour sum in double on the vector ALUs; 2 double precision pieces and workspace,
// colour sum on the matrix cores (single precision).
static hipError_t run_pieces(const double* mom, double* out, int64_t nevt, const int64_t* nevt_dev,
                             const int* goodhel, int ngood, const ProcParams& prm, double norm, int per_hel,
                             void* ws, int64_t ws_events, hipStream_t s, int precision,
                             const SelectArgs& sel = SelectArgs{}) {
  const int f64 = precision != 1;
  if (sel.sel_hel && precision == 0) return hipErrorInvalidValue;  // the choice runs on the matrix-core kernel
  for (int64_t e0 = 0; e0 < nevt; e0 += ws_events) {
    const int64_t n = nevt - e0 < ws_events ? nevt - e0 : ws_events;
    ChunkArgs c{mom + e0 * P7::npar * 4, ws, n, goodhel, ngood, prm, s, nevt_dev, e0};
    c.f64 = f64;
    for (int k = 0; k < P7::nchunk; ++k) {
      const hipError_t e = chunks_ggttggg[k](c);
      if (e != hipSuccess) return e;
    }
    SelectArgs sub{};
    if (sel.sel_hel) sub = SelectArgs{sel.rnd_hel + e0, sel.rnd_col + e0, sel.sel_hel + e0, sel.sel_col + e0};
    double* o = out + (per_hel ? e0 * ngood : e0);
    hipError_t e;
    if (precision == 1)
      e = launch_colour<P7, float, float>(static_cast<const cx<float>*>(ws), o, n, ngood, norm, per_hel, nevt_dev, e0,
                                          s, kColourOnMatrixCores, goodhel, sub);
    else if (precision == 2)
      e = launch_colour<P7, double, float>(static_cast<const cx<double>*>(ws), o, n, ngood, norm, per_hel, nevt_dev,
                                           e0, s, 1, goodhel, sub);
    else
      e = launch_colour<P7, double, double>(static_cast<const cx<double>*>(ws), o, n, ngood, norm, per_hel, nevt_dev,
                                            e0, s, 0, goodhel, sub);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_me2_ggttggg(const LaunchArgs& a, int precision) {
  if (!a.ws || a.ws_events <= 0 || a.sel.chan_w) return hipErrorInvalidValue;
  return run_pieces(a.mom, a.out, a.nevt, a.nevt_dev, a.goodhel, a.ngood, a.prm, a.norm, 0, a.ws, a.ws_events,
                    a.stream, precision, a.sel);
}

// |M_h|^2 of every helicity for nev events (set-up only; synchronous, own workspace)
hipError_t launch_hel_ggttggg(const double* mom, int nev, const ProcParams& prm, double* out, hipStream_t s) {
  int hel[P7::nhel];
  for (int h = 0; h < P7::nhel; ++h) hel[h] = h;
  int* d_hel = nullptr;
  cx<float>* ws = nullptr;
  hipError_t e = hipMalloc(&d_hel, sizeof hel);
  if (e == hipSuccess) e = hipMalloc(&ws, (size_t)nev * P7::nslot * P7::nhel * sizeof(cx<float>));
  if (e == hipSuccess) e = hipMemcpy(d_hel, hel, sizeof hel, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = run_pieces(mom, out, nev, nullptr, d_hel, P7::nhel, prm, 1.0, 1, ws, nev, s, 1);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (ws) (void)hipFree(ws);
  if (d_hel) (void)hipFree(d_hel);
  return e;
}

}  // namespace hme
