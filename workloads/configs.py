"""The five synthetic workloads: process, batch size, energy, seed and cuts.

Particle order inside an event (momenta [nevt][npar][4], E/px/py/pz in GeV):
  e+ e- -> mu+ mu-      : 1 e+ (in, +z), 2 e- (in, -z), 3 mu+, 4 mu-
  g g -> t tbar + n g   : 1 g (in, +z), 2 g (in, -z), 3 t, 4 tbar, 5.. g
This follows the gg -> t tbar listing of the paper's section "Parallel
scattering amplitudes" (gluons first, then top, then antitop).

Everything here is input shaping: no matrix-element arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import rambo

EEMUMU, GGTT, GGTTG, GGTTGG, GGTTGGG = 0, 1, 2, 3, 4
UUEE, UUEEG, UUEEGG, UUEEGGG = 5, 6, 7, 8  # u ubar -> e+ e- + n g (Drell-Yan family)
PROCESS_NAMES = {
    EEMUMU: "e+e- -> mu+mu-",
    GGTT: "gg -> ttbar",
    GGTTG: "gg -> ttbar g",
    GGTTGG: "gg -> ttbar gg",
    GGTTGGG: "gg -> ttbar ggg",
    UUEE: "uu~ -> e+e-",
    UUEEG: "uu~ -> e+e- g",
    UUEEGG: "uu~ -> e+e- gg",
    UUEEGGG: "uu~ -> e+e- ggg",
}
NPAR = {EEMUMU: 4, GGTT: 4, GGTTG: 5, GGTTGG: 6, GGTTGGG: 7, UUEE: 4, UUEEG: 5, UUEEGG: 6, UUEEGGG: 7}
DY = (UUEE, UUEEG, UUEEGG, UUEEGGG)

# Standard Model inputs shared by every evaluation (input data, not derived
# quantities): mZ, width Z, 1/alpha, G_F, m_top, width top (GeV units).
SM_CARD = dict(mZ=91.188, wZ=2.441, alpha_inv=132.5, Gf=1.16639e-5, mT=173.0, wT=0.0)
ALPHA_S = 0.118


def card_array(card=None) -> np.ndarray:
    c = dict(SM_CARD)
    if card:
        c.update(card)
    return np.array([c["mZ"], c["wZ"], c["alpha_inv"], c["Gf"], c["mT"], c["wT"]], dtype=np.float64)


def final_masses(process: int, mT: float = SM_CARD["mT"]):
    if process == EEMUMU or process in DY:
        return [0.0] * (NPAR[process] - 2)  # massless leptons and gluons
    ng = NPAR[process] - 4
    return [mT, mT] + [0.0] * ng


def _cut_gluon_pt(p):
    g = p[:, 2]
    return np.hypot(g[:, 1], g[:, 2]) > 20.0


def _cut_gluon_dr(p):
    return rambo.delta_r(p[:, 2], p[:, 3]) > 0.4


# the same cuts as codes of the on-device generator: (kind, value); kinds 1 = pT of the
# first final-state gluon, 2 = Delta R of the first two final-state gluons
CUT_CODES = {"none": (0, 0.0), "pT(g) > 20 GeV": (1, 20.0), "dR(g,g) > 0.4": (2, 0.4)}


@dataclass
class Workload:
    name: str
    process: int
    nevt: int
    sqrt_s: float
    seed: int
    cut: object = None
    cut_text: str = "none"
    extra: dict = field(default_factory=dict)

    def momenta(self, nevt: int | None = None, first_event: int = 0, mT: float = SM_CARD["mT"],
                retry: bool = True, with_weight: bool = False):
        n = self.nevt if nevt is None else nevt
        return rambo.generate(n, self.sqrt_s, [0.0, 0.0], final_masses(self.process, mT),
                              self.seed, self.cut, first_event=first_event, retry=retry,
                              with_weight=with_weight)


WORKLOADS = {
    "eemumu": Workload("eemumu", EEMUMU, 16384, 500.0, 1),
    "ggtt": Workload("ggtt", GGTT, 524288, 1000.0, 2),
    "ggttg": Workload("ggttg", GGTTG, 1048576, 1500.0, 3, _cut_gluon_pt, "pT(g) > 20 GeV"),
    "ggttgg": Workload("ggttgg", GGTTGG, 1048576, 2000.0, 4, _cut_gluon_dr, "dR(g,g) > 0.4"),
    # the served mix's largest process on its own, at the largest request size (no cuts)
    "ggttggg": Workload("ggttggg", GGTTGGG, 65536, 2000.0, 5),
    # the Drell-Yan family u ubar -> e+ e- + n g (the paper's second standalone workload): flat
    # RAMBO points at sqrt(s) = 1 TeV, seed 6, pT > 20 GeV on the first gluon (n = 1) and
    # Delta R > 0.4 between the first two gluons (n >= 2), as for the top-pair processes
    "uuee": Workload("uuee", UUEE, 1048576, 1000.0, 6),
    "uueeg": Workload("uueeg", UUEEG, 1048576, 1000.0, 6, _cut_gluon_pt, "pT(g) > 20 GeV"),
    "uueegg": Workload("uueegg", UUEEGG, 1048576, 1000.0, 6, _cut_gluon_dr, "dR(g,g) > 0.4"),
    "uueeggg": Workload("uueeggg", UUEEGGG, 1048576, 1000.0, 6, _cut_gluon_dr, "dR(g,g) > 0.4"),
    # served mix: request sizes log-uniform in [256, 65536], processes uniform over
    # the four gg -> ttbar + n g, Poisson arrivals with mean 200 requests/s
    "served": Workload("served", GGTTGGG, 0, 2000.0, 5,
                       extra=dict(rate_hz=200.0, min_batch=256, max_batch=65536,
                                  processes=[GGTT, GGTTG, GGTTGG, GGTTGGG])),
}


def served_requests(nreq: int, seed: int = 5, processes=None):
    """Request stream for the served mix: (arrival_s, process, nevt, first_event).

    processes: the process ids drawn uniformly (default: the four gg -> ttbar + n g).
    """
    from .philox import philox4x32, uniform_pairs
    w = WORKLOADS["served"]
    idx = np.arange(nreq, dtype=np.uint32)
    words = philox4x32((idx, np.uint32(0), np.uint32(0), np.uint32(0)),
                       (np.uint32(seed), np.uint32(0x53455256)))
    u0, u1 = uniform_pairs(words)
    words2 = philox4x32((idx, np.uint32(0), np.uint32(0), np.uint32(1)),
                        (np.uint32(seed), np.uint32(0x53455256)))
    u2, _ = uniform_pairs(words2)
    gaps = -np.log(u0) / w.extra["rate_hz"]
    arrival = np.cumsum(gaps)
    plist = np.array(processes if processes is not None else w.extra["processes"])
    procs = plist[np.minimum((u1 * len(plist)).astype(int), len(plist) - 1)]
    lo, hi = np.log(w.extra["min_batch"]), np.log(w.extra["max_batch"] + 1)
    nevt = np.minimum(np.floor(np.exp(lo + u2 * (hi - lo))).astype(np.int64), w.extra["max_batch"])
    first = np.concatenate([[0], np.cumsum(nevt)[:-1]])
    return arrival, procs, nevt, first
