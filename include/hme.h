/* hme: tree-level squared matrix elements |M|^2 on AMD MI355X (gfx950).
 *
 * The operation is the per-event, helicity- and colour-summed squared matrix
 * element of a fixed parton-level process, evaluated from the external momenta
 * by helicity amplitudes: external wavefunctions, off-shell currents and
 * amplitudes per Feynman diagram, summed into colour-flow amplitudes (jamps),
 * contracted with the constant colour matrix and summed over the non-vanishing
 * helicities (arXiv:2507.21039, section "Parallel scattering amplitudes"; the
 * colour inner product and the precision modes, section "Numerical
 * stability").  The interface follows the paper's Bridge: a handle is created
 * once per process, executed once per batch of events, and destroyed (section
 * "Event generation interface").
 *
 * Output normalisation: |M|^2 averaged over the initial helicities and colours
 * and divided by the symmetry factor of identical final-state particles
 * (IDEN, reported by hme_query): 4 for e+e- -> mu+mu-; 256, 256, 512, 1536 for
 * g g -> t tbar + 0..3 g.
 *
 * Momenta: device memory, double[nevt][npar][4] with components (E, px, py, pz)
 * in GeV, particles in the order
 *   e+ e- -> mu+ mu- : e+ (in), e- (in), mu+, mu-
 *   g g -> t tbar + n g : g (in), g (in), t, tbar, g ...
 * Physics is not validated: momenta are taken to be on shell and conserving;
 * NaN in gives NaN out.
 *
 * Errors: every call returns HME_OK (0) or a negative code; no exception
 * crosses the interface.  hme_last_error() returns a message for the calling
 * thread's last failure.
 */
#ifndef HME_H
#define HME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hme_handle hme_handle;

/* Standard Model inputs: Z mass and width, 1/alpha, Fermi constant, top mass and width (GeV).
 * sin^2(thetaW) follows from (mZ, alpha, G_F); internal top propagators use zero width. */
typedef struct {
  double mZ, wZ, alpha_inv, Gf, mT, wT;
} hme_sm_card;

/* HME_GGTTGGG (1240 diagrams, 120 colour flows) is evaluated in pieces over a jamp
 * workspace (see hme_compute), at every precision. */
/* HME_UUEE .. HME_UUEEGGG: the Drell-Yan family u ubar -> e+ e- + n g (n = 0..3), the paper's
 * second standalone workload (section "SIMT GPU results"): massless quarks and leptons, the
 * lepton pair through a photon and a Z in the s channel, particles 0 u, 1 ubar (incoming),
 * 2 e+, 3 e-, 4.. gluons (outgoing).  |M|^2 is averaged over the 4 initial spin and 9 colour
 * states and divided by n! for the identical gluons. */
enum hme_process {
  HME_EEMUMU = 0, HME_GGTT = 1, HME_GGTTG = 2, HME_GGTTGG = 3, HME_GGTTGGG = 4,
  HME_UUEE = 5, HME_UUEEG = 6, HME_UUEEGG = 7, HME_UUEEGGG = 8
};

/* HME_FP64: every step in double precision.
 * HME_MIXED_FAST: vertices, propagators, jamps and the colour sum in single
 *   precision; external wavefunctions, propagator denominators and the
 *   helicity/event sums in double.
 * HME_MIXED_PAPER: the paper's mixed mode (section "Numerical stability"):
 *   amplitudes and jamps in double, cast to single precision for the colour
 *   algebra; helicity/event sums in double. */
enum hme_precision { HME_FP64 = 0, HME_MIXED_FAST = 1, HME_MIXED_PAPER = 2, HME_MIXED = HME_MIXED_FAST };

/* Flag OR'd into the precision of hme_create: internal gluon propagators in the Feynman-diagram
 * gauge (Hagiwara, Kanzaki, Li, Mawatari and Nakamura, Eur. Phys. J. C 80 (2020) 584) instead of
 * the Feynman gauge; the paper names it for single-precision stability (section "Numerical
 * stability").  |M|^2 is gauge invariant: the same value up to rounding.  Built for HME_GGTTG
 * and HME_GGTTGG (HME_E_UNSUPPORTED otherwise); not for hme_compute_channels (the weights of
 * single diagrams depend on the gauge) nor the server. */
enum { HME_GAUGE_FD = 0x100 };

enum hme_status {
  HME_OK = 0,
  HME_E_ARG = -1,        /* null or misaligned pointer, negative size, unknown process or precision */
  HME_E_HIP = -2,        /* a HIP runtime call failed (message has the HIP error string) */
  HME_E_OOM = -3,        /* device allocation failed */
  HME_E_BUDGET = -4,     /* request larger than the server's memory budget */
  HME_E_TIMEOUT = -5,    /* wait timed out */
  HME_E_UNSUPPORTED = -6 /* process or precision not built into this library */
};

typedef struct {
  int process, precision, npar, nhel, ngoodhel, ncol, ndiag, namp;
  double iden;             /* averaging and symmetry factor applied to the output */
  double flops_per_event;  /* algorithmic floating-point operations per event (all good helicities) */
  double bytes_per_event;  /* HBM traffic per event: momenta in + |M|^2 out */
  double workspace_bytes_per_event; /* jamp workspace of a process evaluated in pieces (else 0) */
} hme_info;

/* Create a handle for `process` on HIP device `device`.  Uploads nothing but a
 * small helicity table; finds the helicities whose |M_h|^2 vanishes identically
 * by evaluating every helicity on a fixed internal sample of 16 events (never on
 * user data) and keeps the others.  The handle owns its device tables.
 * On failure *out is NULL. */
int hme_create(int process, const hme_sm_card* card, int precision, int device, hme_handle** out);

/* Compute |M|^2 for nevt events, asynchronously on `hip_stream` (a hipStream_t,
 * NULL for the default stream).  `momenta` and `me2` are caller-owned device
 * pointers, 8-byte aligned, [nevt][npar][4] and [nevt] doubles.  alpha_s is the
 * strong coupling for this call.  nevt = 0 is a successful no-op; any nevt >= 1
 * is valid (partial wavefronts are masked).  Not thread-safe per handle.
 * HME_GGTTGGG also takes a device workspace of min(nevt, S) events times
 * hme_info.workspace_bytes_per_event (partial-jamp slots x helicities x the size of a
 * complex jamp: 789 x 128 x 8 bytes = 0.81 MB per event at HME_MIXED_FAST, twice that in the
 * double-precision modes), allocated and released on `hip_stream` in stream order (HME_E_OOM if
 * that fails); larger batches run as consecutive sub-batches of S = 16384 events (13 GB of
 * workspace at HME_MIXED_FAST, 26 GB in the double-precision modes). */
int hme_compute(hme_handle* h, double alpha_s, int64_t nevt, const double* momenta, double* me2, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): hme_compute with the same arguments,
 * results and errors, that allocates nothing.  The jamp workspace of HME_GGTTGGG comes from a
 * 256 MiB device array inside the library (one per device, held until the process ends,
 * its address looked up once per device by hme_create) instead of hipMallocAsync: batches
 * run in sub-batches of as many events as it holds (320 at 0.81 MB per event, 160 in the
 * double-precision modes).  A process
 * whose workspace for 4 events exceeds 256 MiB is rejected with HME_E_BUDGET.  Other
 * processes use no workspace and run exactly as in hme_compute.  Every call on a device
 * shares that device's array: calls that overlap in time on one device (different streams,
 * threads or handles) race and give undefined results; calls in one stream are ordered. */
int hme_compute_noalloc(hme_handle* h, double alpha_s, int64_t nevt, const double* momenta, double* me2,
                        void* hip_stream);

/* Same as hme_compute, and also the single-diagram-enhancement channel weights of every event
 * (the paper's section "Event generation interface": with |M|^2, an event generator's
 * multi-channel integration reads one weight per Feynman diagram).  channel_weights: device
 * array [nevt][ndiag] doubles (hme_info.ndiag, diagrams in the generator's order), 8-byte
 * aligned.  Weight of diagram d: W_d / sum_d' W_d', with W_d the sum over good helicities and
 * over the diagram's amplitude terms of |a|^2, a the term with its colour factor stripped (a
 * diagram with a four-gluon vertex has one term per colour structure; for the Drell-Yan family
 * a diagram is the photon and the Z exchange together), accumulated in single precision.
 * |M|^2 is computed as in hme_compute (equal up to rounding: the compiler may fuse the
 * operations differently).  HME_E_UNSUPPORTED for HME_EEMUMU and HME_GGTTGGG; other errors as
 * hme_compute. */
int hme_compute_channels(hme_handle* h, double alpha_s, int64_t nevt, const double* momenta, double* me2,
                         double* channel_weights, void* hip_stream);

/* Fill `info` with the handle's process constants. */
int hme_query(const hme_handle* h, hme_info* info);

/* Copy up to `cap` good helicity indices into `out` (bit k of an index, counted
 * from the most significant of npar bits, is 1 for helicity +1 of particle k);
 * returns the number of good helicities or a negative code. */
int hme_good_helicities(const hme_handle* h, int* out, int cap);

/* Release the handle and its device tables (NULL is accepted). */
int hme_destroy(hme_handle* h);

/* Message describing the calling thread's most recent failure ("" if none). */
const char* hme_last_error(void);

/* Same as hme_compute with a strong coupling per event (running alpha_s evaluated by the
 * caller at each event's scale): alpha_s is a device array of nevt doubles (8-byte aligned).
 * Event i gets |M|^2 computed with g_s = 1 times (4 pi alpha_s[i])^(n/2) for a g_s^n
 * coupling factor of |M|^2 (equal to hme_compute at that scalar alpha_s up to the rounding
 * of the last product).  Values of alpha_s[i] are not checked.  Errors as hme_compute. */
int hme_compute_alphas(hme_handle* h, const double* alpha_s, int64_t nevt, const double* momenta, double* me2,
                       void* hip_stream);

/* Same as hme_compute, and also picks one helicity and one colour flow per event, the
 * information an event generator keeps with each unweighted event (the paper's section
 * "Event generation interface": the Bridge returns them with |M|^2).
 * rnd_hel, rnd_col: device arrays of nevt uniform numbers in [0, 1) supplied by the caller.
 * sel_hel[i]: the chosen helicity index (numbered as in hme_good_helicities): the first good
 *   helicity, in increasing index order, at which the running sum of |M_h|^2 exceeds
 *   rnd_hel[i] times their total (probability |M_h|^2 / sum_h |M_h|^2).
 * sel_col[i]: the chosen colour flow c (flows are the orderings of the gluons along the quark
 *   line, particle order, in lexicographic order; 0 for e+e- -> mu+mu-): the first flow at
 *   which the running sum of W_c = sum_h |J_c,h|^2 (squared colour-flow amplitudes summed over
 *   the good helicities) exceeds rnd_col[i] times their total.
 * me2 is bitwise the output of hme_compute.  Device buffers: me2, rnd_* 8-byte aligned,
 * sel_* 4-byte aligned; asynchronous on hip_stream.  Errors as hme_compute. */
int hme_compute_select(hme_handle* h, double alpha_s, int64_t nevt, const double* momenta, const double* rnd_hel,
                       const double* rnd_col, double* me2, int* sel_hel, int* sel_col, void* hip_stream);

/* ------------------------------------------------------------------ phase space
 * Flat phase-space points on the device (RAMBO: Kleiss, Stirling, Ellis, Comput. Phys.
 * Commun. 40 (1986) 359), the sampling of the paper's standalone application (section
 * "Standalone application"), so that generation and |M|^2 both stay on the GPU.
 *
 * hme_rambo writes nevt events [nevt][npar][4] (E, px, py, pz in GeV) for `process` into the
 * caller's device buffer `momenta` (8-byte aligned), on the current device, asynchronously on
 * `hip_stream`: two massless partons along +z and -z with sqrt_s / 2 each, then the final
 * state (top mass card->mT for the top pair of the QCD processes, massless otherwise).
 * Event i (numbered from first_event) draws from Philox4x32-10 (Salmon et al., SC'11) with
 * key (seed mod 2^32, 0x52414D42) and counter (i mod 2^32, i / 2^32, attempt, 2 j + b) for
 * final-state particle j: each counter gives two doubles (27 + 26 bits of two words each,
 * plus half an ulp) used as cos(theta), phi and the two factors of the exponential energy.
 * An event the cut rejects moves on to attempt + 1, so every event depends on (seed, i)
 * alone; after 10000 rejected attempts its final-state momenta and weight are NaN.
 * With HME_CUT_NO_RETRY or-ed into `cut` every event keeps its first attempt, and a
 * rejected one gets weight 0 (unbiased flat Monte Carlo with cuts).
 * weights (device, may be NULL): the phase-space weight of each point in GeV^(2n-4) for n
 * final-state particles, (2 pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!) for massless
 * ones, times xi^(2n-3) prod_j (|k_j| / E_j) sqrt_s / sum_j (|k_j|^2 / E_j) with massive ones
 * (xi: the common rescaling of the three-momenta).
 * cut: HME_CUT_NONE; HME_CUT_GLUON_PT: transverse momentum of final-state particle 2 (the
 * first gluon) above cut_value; HME_CUT_GLUON_DR: Delta R (pseudorapidity, azimuth) of
 * final-state particles 2 and 3 above cut_value.  A cut on gluons that the process lacks
 * accepts every point.
 * Returns HME_E_ARG for an unknown process or cut, nevt < 0, sqrt_s not above the final-state
 * masses, or a NULL / misaligned buffer with nevt > 0. */
enum hme_cut { HME_CUT_NONE = 0, HME_CUT_GLUON_PT = 1, HME_CUT_GLUON_DR = 2, HME_CUT_NO_RETRY = 0x100 };

int hme_rambo(int process, const hme_sm_card* card, double sqrt_s, uint64_t seed, int64_t first_event, int64_t nevt,
              int cut, double cut_value, double* momenta, double* weights, void* hip_stream);

/* out[0] = sum_i weights[i] me2[i], out[1] = sum_i (weights[i] me2[i])^2 over nevt events, all
 * three device buffers of doubles, asynchronously on `hip_stream` (one workgroup, a fixed
 * order of additions: the same inputs give the same bits).  With the weights of hme_rambo
 * and |M|^2 of hme_compute, the flat Monte Carlo cross section is out[0] / (2 s nevt) in
 * GeV^-2, its statistical error sqrt(out[1] / nevt - (out[0] / nevt)^2) / sqrt(nevt) / (2 s).
 * Returns HME_E_ARG for nevt < 0 or a NULL / misaligned buffer. */
int hme_weighted_sum(const double* me2, const double* weights, int64_t nevt, double* out, void* hip_stream);

/* The flat Monte Carlo cross section and its statistical error, in pb, from the two sums of
 * hme_weighted_sum over npoints points (sums: a HOST pointer to those two doubles, copied back by
 * the caller): sigma = sums[0] / (2 s npoints) times (hbar c)^2 = 0.3893793721e9 GeV^2 pb (flux
 * of massless colliding partons, s = sqrt_s^2), error = sqrt(sums[1] / npoints -
 * (sums[0] / npoints)^2) / sqrt(npoints) / (2 s) in the same units.  Host arithmetic only.
 * Returns HME_E_ARG for NULL pointers, npoints <= 0 or sqrt_s <= 0. */
int hme_flat_cross_section(const double* sums, int64_t npoints, double sqrt_s, double* sigma_pb, double* error_pb);

/* ------------------------------------------------------------------ serving
 * A persistent request loop over every process of the library on one device
 * (the paper's multi-event interface and gridpack workers, section "Event
 * generation interface" and "Gridpacks", feed many batches of varying size; the
 * server keeps the tables resident and batches requests as they arrive).
 *
 * The server owns `nstreams` slots; slot k owns hbm_budget_bytes / nstreams of
 * device memory (gathered momenta and |M|^2 of one batch) and its own stream.  A
 * scheduler thread takes the oldest pending part of a request that has no part on the
 * device (else the oldest part) and, while they fit in a free slot, later pending parts of
 * the same process (continuous batching); a request runs as one part, or as several when it
 * is larger than a slot holds or, for HME_GGTTGGG, larger than 8192 events, so that large
 * requests share the device with others instead of holding a slot for their whole length.
 * Two limits keep slots open for requests that arrive meanwhile: HME_GGTTGGG batches hold
 * at most half of the slots (at least one), and a further part of a request already on the
 * device starts only while another slot stays free.  The scheduler then launches the batch as one
 * captured hipGraph per (process, slot, size bucket): descriptor upload, gather
 * kernel, |M|^2 kernel, scatter kernel (which also applies each request's alpha_s
 * normalisation).  Batches on different slots overlap on the device.  Per-event
 * arithmetic does not depend on the batch, so a request's |M|^2 are bitwise those of
 * hme_compute on it alone.
 * HME_GGTTGGG's jamp workspace, for sub-batches of up to 4096 events, takes at most half
 * of each slot.
 * The server is thread-safe. */

typedef struct hme_server hme_server;

typedef struct {
  uint64_t submitted, completed, batches, events, graphs;
  int64_t slot_capacity_bytes; /* device bytes per slot */
} hme_server_stats;

/* Create a server for all processes at one precision.  hbm_budget_bytes is the
 * total device working memory (split over nstreams slots, 1 <= nstreams <= 8). */
int hme_server_create(const hme_sm_card* card, int precision, int device, size_t hbm_budget_bytes, int nstreams,
                      hme_server** out);

/* Queue |M|^2 of nevt events of `process`.  momenta_dev / me2_dev are caller-owned
 * device pointers that must stay valid until hme_wait returns for *req_id.
 * Returns HME_E_BUDGET if a slot cannot hold a single event of the process (a request larger
 * than a slot runs in parts); nothing is copied at submit time.  The server's streams do not wait for any stream of the caller: the
 * momenta must already be complete in device memory (for instance the stream that wrote them
 * synchronized) when hme_submit is called; use hme_submit_after otherwise. */
int hme_submit(hme_server* s, int process, double alpha_s, int64_t nevt, const double* momenta_dev, double* me2_dev,
               uint64_t* req_id);

/* As hme_submit, for momenta still being produced on the caller's stream `producer_stream`
 * (a hipStream_t on the server's device, NULL for the default stream): the server records an
 * event on that stream at submit time, and the request's batch reads the momenta only after
 * the work queued there before the call has finished.  HME_E_HIP if the event cannot be
 * recorded. */
int hme_submit_after(hme_server* s, int process, double alpha_s, int64_t nevt, const double* momenta_dev,
                     double* me2_dev, void* producer_stream, uint64_t* req_id);

/* Wait for a request: HME_OK once its |M|^2 are in me2_dev (the request is then
 * forgotten), HME_E_TIMEOUT if timeout_s (< 0: forever) passes first, HME_E_ARG
 * for an unknown id, HME_E_HIP if its batch failed (hme_last_error on the waiting thread
 * then names the failing HIP call). */
int hme_wait(hme_server* s, uint64_t req_id, double timeout_s);

/* As hme_wait; on HME_OK also stores the request's latency from hme_submit to the end of
 * its batch on the device (host steady clock, seconds) in *latency_s (if not NULL). */
int hme_wait_timed(hme_server* s, uint64_t req_id, double timeout_s, double* latency_s);

int hme_server_stats_get(const hme_server* s, hme_server_stats* out);

/* Drain all queued and in-flight work, then release the server (NULL is accepted). */
int hme_server_destroy(hme_server* s);

#ifdef __cplusplus
}
#endif

#endif /* HME_H */
