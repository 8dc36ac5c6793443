// Serving: a persistent request loop with continuous batching, fixed per-slot HBM
// regions (the memory budget), and one captured hipGraph per (process, slot, size
// bucket).  See include/hme.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/hme.h"

namespace hme {
double handle_norm(const hme_handle* h, double alpha_s);
int handle_npar(const hme_handle* h);
int64_t handle_ws_bytes_per_event(const hme_handle* h);
hipError_t launch_for_handle(const hme_handle* h, int64_t nevt_grid, const int64_t* nevt_dev, const double* mom,
                             double* out, double norm, hipStream_t s, void* ws, int64_t ws_events);
void set_last_error(const std::string& msg);
}  // namespace hme

namespace {

constexpr int kNumProcesses = 9;  // every process of hme_process
constexpr int64_t kMaxSubBatch = 4096;  // events per sub-batch of a process evaluated in pieces
constexpr int kMaxBatchReq = 64;      // request parts per batch
constexpr int64_t kPiecePart = 8192;  // events per part of a request of a process evaluated in pieces
constexpr int64_t kMinBucket = 256;   // smallest graph size bucket (events)

struct ReqDesc {
  const double* mom;  // caller's momenta [nevt][npar][4]
  double* out;        // caller's |M|^2 [nevt]
  int64_t nevt;
  int64_t offset;  // first event of this request inside the slot
  double norm;     // g_s^(2n) / (IDEN * colour denominator) for this request's alpha_s
};

// One batch as the device sees it; lives in pinned host memory and is copied to the
// slot's device copy by the first node of the graph.
struct BatchDesc {
  int64_t nevt_total;
  int64_t nreq;
  ReqDesc req[kMaxBatchReq];
};

// Copy each request's momenta into the slot, contiguously.  grid.y = request index.
__global__ void gather_kernel(const BatchDesc* __restrict__ b, double* __restrict__ slot_mom, int npar) {
  const int r = blockIdx.y;
  if (r >= b->nreq) return;
  const ReqDesc d = b->req[r];
  const int64_t n = d.nevt * npar * 4;
  double* dst = slot_mom + d.offset * npar * 4;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = d.mom[i];
}

// Scale each request's raw |M|^2 by its normalisation and write them back to the caller.
__global__ void scatter_kernel(const BatchDesc* __restrict__ b, const double* __restrict__ slot_out) {
  const int r = blockIdx.y;
  if (r >= b->nreq) return;
  const ReqDesc d = b->req[r];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.nevt; i += (int64_t)gridDim.x * blockDim.x)
    d.out[i] = slot_out[d.offset + i] * d.norm;
}

struct Request {
  uint64_t id;
  int process;
  double alpha_s;
  int64_t nevt;
  const double* mom;
  double* out;
  bool done = false;
  int status = HME_OK;
  std::string error;               // message of a failed batch, handed to the waiting thread
  hipEvent_t ready = nullptr;      // recorded on the producer stream at submit (hme_submit_after)
  int parts_left = 0;              // parts not finished yet
  int parts_running = 0;           // parts in a batch on the device now
  std::chrono::steady_clock::time_point t_submit, t_done;
};

// A contiguous range of a request's events, scheduled on its own: a request larger than a
// slot, or a large request of a process evaluated in pieces, runs as several parts that can
// share the device with other requests' parts.
struct Part {
  std::shared_ptr<Request> r;
  int64_t offset, nevt;
};

struct Server;

struct Batch {
  Server* srv;
  int slot;
  std::vector<Part> parts;
};

struct Slot {
  hipStream_t stream = nullptr;
  // slot_bytes: gathered momenta of a batch, then its raw |M|^2; a process evaluated in
  // pieces also uses the last ws_bytes as its jamp workspace
  char* d_mem = nullptr;
  BatchDesc* d_desc = nullptr;  // device copy of the descriptor
  BatchDesc* h_desc = nullptr; // pinned host descriptor
  bool busy = false;
  bool heavy = false;  // busy with a process evaluated in pieces
  std::map<std::pair<int, int64_t>, hipGraphExec_t> graphs;  // (process, bucket) -> graph
  std::vector<hipGraph_t> graph_defs;
};

}  // namespace

struct hme_server {};

namespace {

struct Server : hme_server {
  int device = 0, precision = 0;
  int64_t slot_bytes = 0;
  int64_t ws_bytes = 0, ws_events = 0;  // workspace of the processes evaluated in pieces
  hme_handle* handles[kNumProcesses] = {};  // NULL: process not served at this precision
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_sched;  // pending work or a freed slot
  std::condition_variable cv_done;   // a request completed
  std::deque<Part> pending;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> requests;
  uint64_t next_id = 1;
  int inflight = 0;
  bool stop = false;
  std::thread scheduler;
  hme_server_stats stats{};

  // events of `process` one slot holds: momenta (npar * 32 bytes) and |M|^2 (8 bytes) per
  // event, beside the workspace for a process evaluated in pieces
  int64_t capacity(int process) const {
    const int npar = hme::handle_npar(handles[process]);
    if (hme::handle_ws_bytes_per_event(handles[process]) > 0) {
      if (ws_events <= 0) return 0;
      return (slot_bytes - ws_bytes - 512) / (npar * 32 + 8);
    }
    return (slot_bytes - 256) / (npar * 32 + 8);
  }

  // events per part (and per batch) of `process`: what a slot holds, at most kPiecePart for a
  // process evaluated in pieces (so that its large requests interleave with other work)
  int64_t part_events(int process) const {
    const int64_t cap = capacity(process);
    return hme::handle_ws_bytes_per_event(handles[process]) > 0 ? std::min(cap, kPiecePart) : cap;
  }

  static int64_t bucket_for(int64_t n, int64_t cap) {
    int64_t b = kMinBucket;
    while (b < n) b *= 2;
    return std::min(b, cap);
  }

  // Capture gather -> |M|^2 -> scatter for one (process, bucket) on a slot.
  hipError_t graph_for(Slot& sl, int process, int64_t bucket, hipGraphExec_t* out) {
    auto key = std::make_pair(process, bucket);
    auto it = sl.graphs.find(key);
    if (it != sl.graphs.end()) {
      *out = it->second;
      return hipSuccess;
    }
    const int npar = hme::handle_npar(handles[process]);
    // the batch's momenta at the start of the slot, its |M|^2 right after (256-byte aligned)
    double* d_mom = reinterpret_cast<double*>(sl.d_mem);
    double* d_out = reinterpret_cast<double*>(sl.d_mem + ((bucket * npar * 32 + 255) & ~int64_t(255)));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t e1 = hipMemcpyAsync(sl.d_desc, sl.h_desc, sizeof(BatchDesc), hipMemcpyHostToDevice, sl.stream);
    const unsigned gx = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, bucket * npar * 4 / 1024));
    if (e1 == hipSuccess) {
      gather_kernel<<<dim3(gx, kMaxBatchReq), dim3(256), 0, sl.stream>>>(sl.d_desc, d_mom, npar);
      e1 = hipGetLastError();
    }
    const bool pieces = hme::handle_ws_bytes_per_event(handles[process]) > 0;
    void* d_ws = pieces ? sl.d_mem + (slot_bytes - ws_bytes) : nullptr;
    if (e1 == hipSuccess)
      e1 = hme::launch_for_handle(handles[process], bucket, &sl.d_desc->nevt_total, d_mom, d_out, 1.0, sl.stream,
                                 d_ws, pieces ? ws_events : 0);
    if (e1 == hipSuccess) {
      const unsigned sx = (unsigned)std::min<int64_t>(256, std::max<int64_t>(1, bucket / 1024));
      scatter_kernel<<<dim3(sx, kMaxBatchReq), dim3(256), 0, sl.stream>>>(sl.d_desc, d_out);
      e1 = hipGetLastError();
    }
    e = hipStreamEndCapture(sl.stream, &g);
    if (e1 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return e1;
    }
    if (e != hipSuccess) return e;
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return e;
    }
    sl.graphs[key] = ex;
    sl.graph_defs.push_back(g);
    {
      std::lock_guard<std::mutex> lk(mu);
      stats.graphs++;
    }
    *out = ex;
    return hipSuccess;
  }

  static void on_batch_done(void* user) {
    // runs on a HIP runtime thread after the batch's graph finished; no HIP calls here
    Batch* b = static_cast<Batch*>(user);
    Server* s = b->srv;
    const auto now = std::chrono::steady_clock::now();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (auto& pt : b->parts) {
        auto& r = pt.r;
        r->parts_running--;
        if (--r->parts_left == 0) {
          r->done = true;
          r->t_done = now;
          s->stats.completed++;
        }
      }
      s->slots[b->slot].busy = false;
      s->slots[b->slot].heavy = false;
      s->inflight--;
    }
    s->cv_done.notify_all();
    s->cv_sched.notify_all();
    delete b;
  }

  void fail_batch(Batch* b, hipError_t e) {
    const std::string msg = std::string("server batch: ") + hipGetErrorString(e);
    std::lock_guard<std::mutex> lk(mu);
    for (auto& pt : b->parts) {
      auto& r = pt.r;
      r->parts_running--;
      r->status = HME_E_HIP;
      r->error = msg;
      if (--r->parts_left == 0) {
        r->done = true;
        r->t_done = std::chrono::steady_clock::now();
        stats.completed++;
      }
    }
    slots[b->slot].busy = false;
    slots[b->slot].heavy = false;
    inflight--;
  }

  // The pending part to start on a free slot, or pending.end().  Preference: the oldest part
  // of a request with no part on the device, else the oldest part.  Two limits keep slots
  // open for requests that arrive meanwhile: batches of a process evaluated in pieces (long
  // ones, which take most of the device while they run) hold at most half of the slots, and a
  // further part of a request already on the device starts only while another slot stays free.
  std::deque<Part>::iterator pick_part() {
    int nfree = 0, nheavy = 0;
    for (const Slot& sl : slots) {
      nfree += !sl.busy;
      nheavy += sl.busy && sl.heavy;
    }
    const int nslots = (int)slots.size();
    auto fresh = pending.end(), any = pending.end();
    for (auto it = pending.begin(); it != pending.end(); ++it) {
      if (nfree == 0) break;
      const bool heavy = hme::handle_ws_bytes_per_event(handles[it->r->process]) > 0;
      if (heavy && nslots > 1 && nheavy >= std::max(1, nslots / 2)) continue;
      if (it->r->parts_running == 0) {
        fresh = it;
        break;
      }
      if (any == pending.end() && (nfree >= 2 || nslots == 1)) any = it;
    }
    return fresh != pending.end() ? fresh : any;
  }

  void run() {
    hipError_t e0 = hipSetDevice(device);
    (void)e0;
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      int free_slot = -1;
      std::deque<Part>::iterator hit;
      cv_sched.wait(lk, [&] {
        if (stop && pending.empty()) return true;
        free_slot = -1;
        for (size_t k = 0; k < slots.size(); ++k)
          if (!slots[k].busy) {
            free_slot = (int)k;
            break;
          }
        if (free_slot < 0) return false;
        hit = pick_part();
        return hit != pending.end();
      });
      if (pending.empty()) {
        if (stop) break;
        continue;
      }
      // continuous batching: the chosen part, then later parts of the same process while
      // they fit (a request's own parts only if nothing else is waiting)
      const Part head = *hit;
      pending.erase(hit);
      Batch* b = new Batch{this, free_slot, {head}};
      head.r->parts_running++;
      const int process = head.r->process;
      const int64_t cap = part_events(process);
      int64_t total = head.nevt;
      for (auto it = pending.begin(); it != pending.end() && (int)b->parts.size() < kMaxBatchReq;) {
        if (it->r->process == process && total + it->nevt <= cap && it->r != head.r) {
          total += it->nevt;
          it->r->parts_running++;
          b->parts.push_back(*it);
          it = pending.erase(it);
        } else {
          ++it;
        }
      }
      Slot& sl = slots[free_slot];
      sl.busy = true;
      sl.heavy = hme::handle_ws_bytes_per_event(handles[process]) > 0;
      inflight++;
      stats.batches++;
      stats.events += total;
      lk.unlock();

      BatchDesc* d = sl.h_desc;
      d->nevt_total = total;
      d->nreq = (int64_t)b->parts.size();
      int64_t off = 0;
      const int npar = hme::handle_npar(handles[process]);
      for (size_t i = 0; i < b->parts.size(); ++i) {
        const Part& pt = b->parts[i];
        const auto& r = pt.r;
        d->req[i] = ReqDesc{r->mom + pt.offset * npar * 4, r->out + pt.offset, pt.nevt, off,
                            hme::handle_norm(handles[r->process], r->alpha_s)};
        off += pt.nevt;
      }
      hipGraphExec_t ex = nullptr;
      hipError_t e = graph_for(sl, process, bucket_for(total, capacity(process)), &ex);
      // requests submitted with a producer stream: the gather reads their momenta only after
      // the work queued on that stream before the submit (each part's batch waits on it)
      for (auto& pt : b->parts) {
        if (!pt.r->ready || e != hipSuccess) continue;
        e = hipStreamWaitEvent(sl.stream, pt.r->ready, 0);
      }
      if (e == hipSuccess) e = hipGraphLaunch(ex, sl.stream);
      if (e == hipSuccess) e = hipLaunchHostFunc(sl.stream, &Server::on_batch_done, b);
      if (e != hipSuccess) {
        fail_batch(b, e);
        delete b;
        cv_done.notify_all();
      }
      lk.lock();
    }
  }
};

int srv_fail(int code, const std::string& msg) {
  hme::set_last_error(msg);
  return code;
}

}  // namespace

extern "C" {

int hme_server_create(const hme_sm_card* card, int precision, int device, size_t hbm_budget_bytes, int nstreams,
                      hme_server** out) {
  if (!out) return srv_fail(HME_E_ARG, "hme_server_create: out is NULL");
  *out = nullptr;
  if (!card) return srv_fail(HME_E_ARG, "hme_server_create: card is NULL");
  if (nstreams < 1 || nstreams > 8) return srv_fail(HME_E_ARG, "hme_server_create: nstreams must be 1..8");
  if (precision & HME_GAUGE_FD) return srv_fail(HME_E_UNSUPPORTED, "hme_server_create: Feynman gauge only");
  if (hbm_budget_bytes < (size_t)nstreams * (1u << 20))
    return srv_fail(HME_E_BUDGET, "hme_server_create: budget below 1 MiB per stream");
  auto* s = new Server;
  s->device = device;
  s->precision = precision;
  s->slot_bytes = (int64_t)(hbm_budget_bytes / nstreams) & ~int64_t(255);
  for (int p = 0; p < kNumProcesses; ++p) {
    int rc = hme_create(p, card, precision, device, &s->handles[p]);
    if (rc == HME_E_UNSUPPORTED) continue;  // not served at this precision
    if (rc != HME_OK) {
      for (int q = 0; q < p; ++q) hme_destroy(s->handles[q]);
      delete s;
      return rc;
    }
    // the workspace: half the slot at most, whole 64-event groups, 256-byte aligned
    const int64_t per_event = hme::handle_ws_bytes_per_event(s->handles[p]);
    if (per_event > 0) {
      int64_t n = std::min<int64_t>(kMaxSubBatch, s->slot_bytes / 2 / per_event) & ~int64_t(63);
      if (s->ws_events == 0 || n < s->ws_events) {
        s->ws_events = n;
        s->ws_bytes = (n * per_event + 255) & ~int64_t(255);
      }
    }
  }
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(device);
  s->slots.resize(nstreams);
  hipError_t e = hipSuccess;
  for (auto& sl : s->slots) {
    if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess) break;
    if ((e = hipMalloc(&sl.d_mem, s->slot_bytes)) != hipSuccess) break;
    if ((e = hipMalloc(&sl.d_desc, sizeof(BatchDesc))) != hipSuccess) break;
    if ((e = hipHostMalloc(&sl.h_desc, sizeof(BatchDesc), hipHostMallocDefault)) != hipSuccess) break;
    std::memset(sl.h_desc, 0, sizeof(BatchDesc));
  }
  (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    s->stop = true;
    hme_server_destroy(s);
    return srv_fail(HME_E_OOM, std::string("hme_server_create: ") + hipGetErrorString(e));
  }
  s->stats.slot_capacity_bytes = s->slot_bytes;
  s->scheduler = std::thread([s] { s->run(); });
  *out = s;
  return HME_OK;
}

static int submit_impl(hme_server* srv, int process, double alpha_s, int64_t nevt, const double* momenta_dev,
                       double* me2_dev, bool after, void* producer_stream, uint64_t* req_id) {
  auto* s = static_cast<Server*>(srv);
  if (!s || !req_id) return srv_fail(HME_E_ARG, "hme_submit: NULL server or req_id");
  if (process < 0 || process >= kNumProcesses) return srv_fail(HME_E_ARG, "hme_submit: unknown process");
  if (!s->handles[process]) return srv_fail(HME_E_UNSUPPORTED, "hme_submit: process not served at this precision");
  if (nevt < 0) return srv_fail(HME_E_ARG, "hme_submit: nevt < 0");
  if (!(alpha_s > 0)) return srv_fail(HME_E_ARG, "hme_submit: alpha_s must be positive");
  if (nevt > 0 && (!momenta_dev || !me2_dev)) return srv_fail(HME_E_ARG, "hme_submit: NULL momenta or me2");
  if ((reinterpret_cast<uintptr_t>(momenta_dev) | reinterpret_cast<uintptr_t>(me2_dev)) & 7u)
    return srv_fail(HME_E_ARG, "hme_submit: pointers must be 8-byte aligned");
  if (s->capacity(process) < 1) return srv_fail(HME_E_BUDGET, "hme_submit: a slot holds no event of this process");
  auto r = std::make_shared<Request>();
  r->t_submit = std::chrono::steady_clock::now();
  r->process = process;
  r->alpha_s = alpha_s;
  r->nevt = nevt;
  r->mom = momenta_dev;
  r->out = me2_dev;
  if (after && nevt > 0) {
    int prev = 0;
    (void)hipGetDevice(&prev);
    hipError_t e = hipSetDevice(s->device);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&r->ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(r->ready, static_cast<hipStream_t>(producer_stream));
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
      if (r->ready) (void)hipEventDestroy(r->ready);
      return srv_fail(HME_E_HIP, std::string("hme_submit_after: ") + hipGetErrorString(e));
    }
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      if (r->ready) (void)hipEventDestroy(r->ready);
      return srv_fail(HME_E_ARG, "hme_submit: server is shutting down");
    }
    r->id = s->next_id++;
    s->requests[r->id] = r;
    s->stats.submitted++;
    if (nevt == 0) {
      r->done = true;
      r->t_done = r->t_submit;
      s->stats.completed++;
    } else {
      const int64_t part = s->part_events(process);
      for (int64_t o = 0; o < nevt; o += part) {
        s->pending.push_back(Part{r, o, std::min(part, nevt - o)});
        r->parts_left++;
      }
    }
  }
  s->cv_sched.notify_one();
  *req_id = r->id;
  return HME_OK;
}

int hme_submit(hme_server* srv, int process, double alpha_s, int64_t nevt, const double* momenta_dev, double* me2_dev,
               uint64_t* req_id) {
  return submit_impl(srv, process, alpha_s, nevt, momenta_dev, me2_dev, false, nullptr, req_id);
}

int hme_submit_after(hme_server* srv, int process, double alpha_s, int64_t nevt, const double* momenta_dev,
                     double* me2_dev, void* producer_stream, uint64_t* req_id) {
  return submit_impl(srv, process, alpha_s, nevt, momenta_dev, me2_dev, true, producer_stream, req_id);
}

int hme_wait(hme_server* srv, uint64_t req_id, double timeout_s) {
  return hme_wait_timed(srv, req_id, timeout_s, nullptr);
}

int hme_wait_timed(hme_server* srv, uint64_t req_id, double timeout_s, double* latency_s) {
  auto* s = static_cast<Server*>(srv);
  if (!s) return srv_fail(HME_E_ARG, "hme_wait: NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->requests.find(req_id);
  if (it == s->requests.end()) return srv_fail(HME_E_ARG, "hme_wait: unknown request id");
  std::shared_ptr<Request> r = it->second;
  if (timeout_s < 0) {
    s->cv_done.wait(lk, [&] { return r->done; });
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return r->done; })) {
    return srv_fail(HME_E_TIMEOUT, "hme_wait: timed out");
  }
  s->requests.erase(req_id);
  // the producer-stream event of hme_submit_after: every part's batch has waited on it by now
  if (r->ready) {
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    (void)hipEventDestroy(r->ready);
    (void)hipSetDevice(prev);
    r->ready = nullptr;
  }
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  if (r->status != HME_OK) return srv_fail(r->status, "hme_wait: " + r->error);
  return r->status;
}

int hme_server_stats_get(const hme_server* srv, hme_server_stats* out) {
  auto* s = static_cast<const Server*>(srv);
  if (!s || !out) return srv_fail(HME_E_ARG, "hme_server_stats_get: NULL argument");
  std::lock_guard<std::mutex> lk(const_cast<Server*>(s)->mu);
  *out = s->stats;
  return HME_OK;
}

int hme_server_destroy(hme_server* srv) {
  auto* s = static_cast<Server*>(srv);
  if (!s) return HME_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_sched.notify_all();
  if (s->scheduler.joinable()) s->scheduler.join();
  {
    // wait for the last batches' callbacks
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->inflight == 0; });
  }
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->device);
  for (auto& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    for (auto& kv : sl.graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto g : sl.graph_defs) (void)hipGraphDestroy(g);
    if (sl.d_mem) (void)hipFree(sl.d_mem);
    if (sl.d_desc) (void)hipFree(sl.d_desc);
    if (sl.h_desc) (void)hipHostFree(sl.h_desc);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  for (auto& kv : s->requests)  // requests never waited for
    if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
  (void)hipSetDevice(prev);
  for (auto* h : s->handles)
    if (h) hme_destroy(h);
  delete s;
  return HME_OK;
}

}  // extern "C"
