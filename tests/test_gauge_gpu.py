"""The Feynman-diagram gauge variant (HME_GAUGE_FD) on the GPU through the C ABI: gauge
invariance against the oracle (which works in the Feynman gauge) with the usual gates in every
precision, and its argument errors."""
import numpy as np
import pytest

import oracle
import paper_2507_21039_amd as hme
from workloads import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

AS = 0.118


@pytest.mark.parametrize("key,proc,n", [("ggttg", hme.GGTTG, 6007), ("ggttgg", hme.GGTTGG, 2003)])
def test_fd_gauge_parity(card, key, proc, n):
    print(f"[gpu] feynman-diagram gauge {key} n={n}", flush=True)
    p = configs.WORKLOADS[key].momenta(n, first_event=77)
    ref = oracle.me2(proc, p, card, AS)
    t = torch.from_numpy(p).cuda()
    out = {}
    for prec in (hme.FP64, hme.MIXED_PAPER, hme.MIXED_FAST):
        with hme.Handle(proc, card, prec | hme.GAUGE_FD) as h:
            out[prec] = h.compute(t, alpha_s=AS)
            torch.cuda.synchronize()
            out[prec] = out[prec].cpu().numpy()
    rel = np.abs(out[hme.FP64] / ref - 1)
    bad = np.nonzero(~(rel <= 1e-12))[0]
    if bad.size:
        ld = oracle.me2(proc, p[bad], card, AS, extended=True)
        err = np.abs(out[hme.FP64][bad] / ld - 1)
        print(f"  {bad.size} arbitrated, gpu-vs-ld max {err.max():.3g}")
        assert np.all(err <= 1e-12)
    paper = np.abs(out[hme.MIXED_PAPER] / ref - 1)
    fast = np.abs(out[hme.MIXED_FAST] / ref - 1)
    print(f"  fp64 max {rel.max():.3g}; mixed_paper max {paper.max():.3g}; mixed_fast max {fast.max():.3g} "
          f"p99 {np.quantile(fast, 0.99):.3g}")
    assert paper.max() <= 1e-5
    assert np.quantile(fast, 0.99) <= 1e-5 and fast.max() <= 1e-3


def test_fd_gauge_errors(card):
    for proc in (hme.EEMUMU, hme.GGTT, hme.GGTTGGG, hme.UUEEGG):
        with pytest.raises(hme.HmeError) as e:
            hme.Handle(proc, card, hme.FP64 | hme.GAUGE_FD)
        assert e.value.code == hme.HME_E_UNSUPPORTED
    with hme.Handle(hme.GGTTG, card, hme.FP64 | hme.GAUGE_FD) as h:
        with pytest.raises(hme.HmeError) as e:
            h.compute_channels(torch.zeros((4, 5, 4), dtype=torch.float64, device="cuda"))
        assert e.value.code == hme.HME_E_UNSUPPORTED
    with pytest.raises(hme.HmeError) as e:
        hme.Server(card, hme.MIXED_FAST | hme.GAUGE_FD, hbm_budget_bytes=64 << 20, nstreams=1)
    assert e.value.code == hme.HME_E_UNSUPPORTED
