"""GPU parity of the single-diagram-enhancement channel weights (hme_compute_channels) through
the C ABI: per event and diagram, W_d / sum W against the oracle's diagram-by-diagram
evaluation (diagrams matched by name), in every precision, across wavefront boundaries with a
ragged tail; |M|^2 of the same call equal to that of hme_compute up to rounding.

Tolerance: the device sums each term's |a|^2 over the helicities in single precision, so
weights above 1e-6 agree to 1e-5 relative (5e-4 with single-precision amplitudes) and every
weight to 1e-9 absolute (1e-6)."""
import numpy as np
import pytest

import oracle
import paper_2507_21039_amd as hme
from paper_2507_21039_amd.gen import diagrams
from workloads import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [("ggtt", hme.GGTT, 0, "tt", 301), ("ggttg", hme.GGTTG, 1, "tt", 301), ("ggttgg", hme.GGTTGG, 2, "tt", 261),
         ("uuee", hme.UUEE, 0, "dy", 301), ("uueeg", hme.UUEEG, 1, "dy", 301), ("uueegg", hme.UUEEGG, 2, "dy", 261),
         ("uueeggg", hme.UUEEGGG, 3, "dy", 97)]


@pytest.mark.parametrize("key,proc,ng,family,n", CASES)
@pytest.mark.parametrize("prec", [hme.FP64, hme.MIXED_FAST, hme.MIXED_PAPER])
def test_channel_weights(card, key, proc, ng, family, n, prec):
    print(f"[gpu] channel weights {key} precision={prec} n={n}", flush=True)
    p = configs.WORKLOADS[key].momenta(n, first_event=3)
    gkeys = diagrams.diagram_keys(ng, family)
    okeys = oracle.diagram_keys(proc)
    ref = oracle.channel_weights(proc, p, card)[:, [okeys.index(k) for k in gkeys]]
    ref /= ref.sum(axis=1, keepdims=True)
    with hme.Handle(proc, card, prec) as h:
        assert h.query()["ndiag"] == len(gkeys)
        t = torch.from_numpy(p).cuda()
        me2, w = h.compute_channels(t)
        plain = h.compute(t)
        torch.cuda.synchronize()
    # the same operations as hme_compute; the observer's extra use of each amplitude term can
    # change which products the compiler fuses, so single precision agrees to its rounding
    rel = (me2 / plain - 1).abs().max().item()
    assert rel <= (1e-4 if prec == hme.MIXED_FAST else 1e-13), rel
    w = w.cpu().numpy()
    assert np.all(np.isfinite(w)) and np.all(w >= 0)
    assert np.abs(w.sum(axis=1) - 1).max() <= 1e-12
    rtol, atol = (5e-4, 1e-6) if prec == hme.MIXED_FAST else (1e-5, 1e-9)
    big = ref > 1e-6
    assert np.abs(w[big] / ref[big] - 1).max() <= rtol
    assert np.abs(w - ref).max() <= atol + rtol * ref.max()


def test_channel_weights_unsupported_and_edges(card):
    for proc, prec in ((hme.EEMUMU, hme.FP64), (hme.GGTTGGG, hme.MIXED_FAST)):
        with hme.Handle(proc, card, prec) as h:
            with pytest.raises(hme.HmeError) as e:
                h.compute_channels(torch.zeros((4, hme.NPAR[proc], 4), dtype=torch.float64, device="cuda"))
            assert e.value.code == hme.HME_E_UNSUPPORTED
    with hme.Handle(hme.GGTTG, card, hme.FP64) as h:
        p = torch.from_numpy(configs.WORKLOADS["ggttg"].momenta(70)).cuda()
        _, whole = h.compute_channels(p)
        for a, b in [(0, 1), (1, 33), (33, 70)]:
            _, part = h.compute_channels(p[a:b].contiguous())
            assert torch.equal(part, whole[a:b])
