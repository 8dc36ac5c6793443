"""GPU parity of the per-event strong coupling (hme_compute_alphas, C ABI).

Each event carries its own alpha_s (five values spread over the batch).  Against
hme_compute at that scalar alpha_s: the same kernel with the coupling applied in a separate
product, so equal to 1e-14 relative (a few roundings of (4 pi alpha_s)^(n/2)).  Against the
FP64 oracle evaluated at each event's alpha_s: the FP64 gate of the main parity tests (1e-12
in every event, events beyond it decided by the long double oracle) and the single-precision
bars for gg -> ttbar ggg.
"""
import numpy as np
import pytest

import oracle
import paper_2507_21039_amd as hme
from workloads import configs

from test_parity_gpu import fp64_gate

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ALPHAS = np.array([0.09, 0.105, 0.118, 0.13, 0.16])
CASES = [("eemumu", hme.EEMUMU, hme.FP64, 2001), ("ggtt", hme.GGTT, hme.FP64, 4001),
         ("ggttg", hme.GGTTG, hme.FP64, 2001), ("ggttgg", hme.GGTTGG, hme.FP64, 601),
         ("ggttgg", hme.GGTTGG, hme.MIXED_FAST, 601), ("ggttggg", hme.GGTTGGG, hme.MIXED_FAST, 203)]


@pytest.mark.parametrize("key,proc,prec,nevt", CASES)
def test_per_event_alpha_s(key, proc, prec, nevt):
    card = configs.card_array()
    p = configs.WORKLOADS[key].momenta(nevt, first_event=77)
    which = np.arange(nevt) % len(ALPHAS)
    a = ALPHAS[which]
    print(f"[gpu] alphas {key} precision={prec} nevt={nevt}", flush=True)
    with hme.Handle(proc, card, prec) as h:
        mom = torch.from_numpy(p).cuda()
        got = h.compute_alphas(mom, torch.from_numpy(a).cuda()).cpu().numpy()
        per_value = {v: h.compute(mom, alpha_s=float(v)).cpu().numpy() for v in ALPHAS}
    for j, v in enumerate(ALPHAS):
        sel = which == j
        assert np.abs(got[sel] / per_value[v][sel] - 1).max() <= 1e-14
        idx = np.flatnonzero(sel)[:40]
        ref = oracle.me2(proc, p[idx], card, float(v))
        rel = np.abs(got[idx] / ref - 1)
        if prec == hme.FP64:
            fp64_gate(proc, p[idx], got[idx], ref, card, float(v))
        else:
            assert np.quantile(rel, 0.99) <= 1e-5 and rel.max() <= 1e-3
    if proc == hme.EEMUMU:  # no strong coupling: identical to hme_compute
        assert np.array_equal(got, per_value[0.118])
