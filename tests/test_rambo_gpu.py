"""GPU parity of the on-device phase-space generator and cross-section sum (through the C ABI).

The host reference is workloads/rambo.py (numpy, extended-precision arithmetic); the device
computes in double, so momenta agree to rounding of the conformal boost and the rescaling:
|dp| <= 1e-10 sqrt_s per component, weights to 1e-11 relative.  Which attempt an event
keeps is an integer decision and must agree exactly (a cut value within rounding of its
threshold would be the one legitimate exception; none occurs at these seeds).
"""
import math

import numpy as np
import pytest

import oracle
import paper_2507_21039_amd as hme
from workloads import configs, rambo

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

P_TOL = 1e-10
W_TOL = 1e-11


def device_events(w, nevt, first_event=0, card=None, retry=True, seed=None):
    kind, value = configs.CUT_CODES[w.cut_text]
    cut = kind | (0 if retry else hme.CUT_NO_RETRY)
    print(f"[gpu] rambo {w.name} nevt={nevt} first={first_event} cut={cut}", flush=True)
    p, wt = hme.rambo(w.process, card if card is not None else configs.card_array(), w.sqrt_s,
                      w.seed if seed is None else seed, nevt, first_event, cut, value, weights=True)
    torch.cuda.synchronize()
    return p.cpu().numpy(), wt.cpu().numpy()


def compare(w, p_dev, w_dev, p_host, w_host):
    assert np.isfinite(p_dev).all() and np.isfinite(w_dev).all()
    assert np.abs(p_dev - p_host).max() <= P_TOL * w.sqrt_s
    pos = w_host > 0
    assert np.array_equal(w_dev > 0, pos)
    assert np.abs(w_dev[pos] / w_host[pos] - 1).max() <= W_TOL


@pytest.mark.parametrize("name,nevt,first", [("eemumu", 16384, 0), ("ggtt", 20011, 7), ("ggttg", 12007, 100),
                                             ("ggttgg", 6007, 3), ("ggttggg", 4099, 65000), ("uueeg", 6007, 9),
                                             ("uueeggg", 4099, 1000)])
def test_rambo_matches_host(name, nevt, first):
    w = configs.WORKLOADS[name]
    p_dev, w_dev = device_events(w, nevt, first)
    p_host, w_host = w.momenta(nevt, first_event=first, with_weight=True)
    compare(w, p_dev, w_dev, p_host, w_host)


@pytest.mark.parametrize("name", ["ggttg", "ggttgg"])
def test_rambo_no_retry_matches_host(name):
    w = configs.WORKLOADS[name]
    p_dev, w_dev = device_events(w, 8191, retry=False)
    p_host, w_host = w.momenta(8191, retry=False, with_weight=True)
    assert 0 < (w_host == 0).sum() < 8191
    compare(w, p_dev, w_dev, p_host, w_host)


def test_rambo_high_event_numbers_and_batch_split():
    w = configs.WORKLOADS["ggttgg"]
    first = (1 << 32) - 700  # the counter's high word changes inside the batch
    p_dev, w_dev = device_events(w, 1500, first)
    p_host, w_host = w.momenta(1500, first_event=first, with_weight=True)
    compare(w, p_dev, w_dev, p_host, w_host)
    p_tail, w_tail = device_events(w, 800, first + 700)
    assert np.array_equal(p_tail, p_dev[700:]) and np.array_equal(w_tail, w_dev[700:])


def test_rambo_hard_cut_retries_and_exhaustion():
    w = configs.WORKLOADS["ggttg"]
    card = configs.card_array()
    # pT of the gluon above 650 GeV at 1.5 TeV: about 3% acceptance, tens of attempts per event
    p, wt = hme.rambo(w.process, card, w.sqrt_s, 9, 2048, 0, hme.CUT_GLUON_PT, 650.0, weights=True)
    torch.cuda.synchronize()
    cut = lambda k: np.hypot(k[:, 2, 1], k[:, 2, 2]) > 650.0
    p_host, w_host = rambo.generate(2048, w.sqrt_s, [0, 0], configs.final_masses(w.process), 9, cut,
                                    with_weight=True)
    compare(w, p.cpu().numpy(), wt.cpu().numpy(), p_host, w_host)
    # the gluon's energy stays below (s - 4 mT^2) / (2 sqrt_s) = 710 GeV: every event exhausts its attempts
    p, wt = hme.rambo(w.process, card, w.sqrt_s, 9, 256, 0, hme.CUT_GLUON_PT, 760.0, weights=True)
    torch.cuda.synchronize()
    p, wt = p.cpu().numpy(), wt.cpu().numpy()
    assert np.isnan(p[:, 2:]).all() and np.isnan(wt).all()
    assert np.array_equal(p[:, 0], np.tile([750.0, 0, 0, 750.0], (256, 1)))


def test_rambo_full_size_properties():
    """ggttgg at 2^20 events with the Delta R cut, as the end-to-end benchmark draws them."""
    w = configs.WORKLOADS["ggttgg"]
    kind, value = configs.CUT_CODES[w.cut_text]
    card = configs.card_array()
    print(f"[gpu] rambo full size {w.nevt}", flush=True)
    p, wt = hme.rambo(w.process, card, w.sqrt_s, w.seed, w.nevt, 0, kind, value, weights=True)
    fin = p[:, 2:]
    assert bool(torch.isfinite(p).all()) and bool((wt > 0).all())
    tot = fin.sum(1)
    assert float((tot - torch.tensor([w.sqrt_s, 0, 0, 0], dtype=torch.float64, device=p.device)).abs().max()) \
        <= 1e-9 * w.sqrt_s
    m2 = fin[..., 0] ** 2 - (fin[..., 1:] ** 2).sum(-1)
    mass = torch.tensor([card[4] ** 2, card[4] ** 2, 0, 0], dtype=torch.float64, device=p.device)
    assert float((m2 - mass).abs().max()) <= 1e-8 * w.sqrt_s ** 2
    # sampled events one by one against the host generator
    idx = np.sort(np.random.default_rng(5).choice(w.nevt, 48, replace=False))
    ti = torch.from_numpy(idx).to(p.device)
    p_np, w_np = p[ti].cpu().numpy(), wt[ti].cpu().numpy()
    for j, i in enumerate(idx):
        ph, wh = w.momenta(1, first_event=int(i), with_weight=True)
        assert np.abs(p_np[j] - ph[0]).max() <= P_TOL * w.sqrt_s and abs(w_np[j] / wh[0] - 1) <= W_TOL
    # the cut holds on every event
    dr = rambo.delta_r(fin[:, 2].cpu().numpy(), fin[:, 3].cpu().numpy())
    assert dr.min() > value


def test_weighted_sum_and_cross_section_parity(card):
    """Device phase space + |M|^2 + sum against the host generator + oracle + extended sum."""
    w = configs.WORKLOADS["ggttg"]
    nevt = 20011
    p, wt = device_events(w, nevt, retry=False)
    pt, wtt = torch.from_numpy(p).cuda(), torch.from_numpy(wt).cuda()
    with hme.Handle(w.process, card, hme.FP64) as h:
        me = h.compute(pt)
        sums = hme.weighted_sum(me, wtt)
        sums2 = hme.weighted_sum(me, wtt)
        torch.cuda.synchronize()
    s_dev = sums.cpu().numpy()
    assert np.array_equal(s_dev, sums2.cpu().numpy())
    v = wt * me.cpu().numpy()
    assert s_dev[0] == pytest.approx(math.fsum(v), rel=1e-13)
    assert s_dev[1] == pytest.approx(math.fsum(v * v), rel=1e-13)
    sig_dev, err_dev = hme.cross_section_pb(s_dev, nevt, w.sqrt_s)
    p_host, w_host = w.momenta(nevt, retry=False, with_weight=True)
    sig, err = oracle.cross_section(oracle.me2(w.process, p_host, card), w_host, w.sqrt_s)
    assert sig_dev == pytest.approx(sig, rel=1e-11) and err_dev == pytest.approx(err, rel=1e-9)


def test_eemumu_cross_section_on_device_closed_form(card):
    w = configs.WORKLOADS["eemumu"]
    nevt = 1 << 23
    print(f"[gpu] eemumu cross section nevt={nevt}", flush=True)
    p, wt = hme.rambo(w.process, card, w.sqrt_s, 77, nevt, 0, hme.CUT_NONE, 0.0, weights=True)
    with hme.Handle(w.process, card, hme.FP64) as h:
        sums = hme.weighted_sum(h.compute(p), wt)
        sig, err = hme.cross_section_pb(sums.cpu().numpy(), nevt, w.sqrt_s)
    ew = oracle.ew(card)
    sw2, cw2, e = ew["sw2"], ew["cw2"], ew["e"]
    mZ, wZ, s = card[0], card[1], w.sqrt_s ** 2
    gL, gR = -0.5 + sw2, sw2
    A = lambda gi, gj: 1 / s + gi * gj / (sw2 * cw2) / (s - mZ ** 2 + 1j * mZ * wZ)
    exact = e ** 4 * s * sum(abs(A(a, b)) ** 2 for a in (gL, gR) for b in (gL, gR)) / (48 * math.pi)
    exact *= oracle.GEV2_TO_PB
    assert err < 3e-4 * exact and abs(sig - exact) <= 5 * err, (sig, exact, err)
