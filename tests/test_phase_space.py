"""Pins for the phase-space weights and the cross-section estimate (CPU only).

Phase-space volumes in the measure (2 pi)^4 delta^4(P - sum k) prod d^3k / ((2 pi)^3 2E):
  two bodies: Phi_2(s; ma, mb) = sqrt(lambda(s, ma^2, mb^2)) / (8 pi s);
  n bodies by splitting off one particle:
  Phi_n(s; m1, rest) = int dM^2 / (2 pi) Phi_2(s; m1, M) Phi_(n-1)(M^2; rest).
The mean RAMBO weight over its points is the volume Phi_n, and for two massive bodies every
weight equals Phi_2.  e+e- -> mu+mu- through photon and Z has the total cross section
e^4 s (|A_LL|^2 + |A_RR|^2 + |A_LR|^2 + |A_RL|^2) / (48 pi) (the angular integral of the
helicity closed form, int dOmega u^2 = int dOmega t^2 = 4 pi s^2 / 3, over 2 s and 32 pi^2).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from workloads import configs, rambo

MT = configs.SM_CARD["mT"]


def lam(a, b, c):
    return a * a + b * b + c * c - 2 * (a * b + b * c + c * a)


def phi2(s, ma, mb):
    return math.sqrt(max(lam(s, ma * ma, mb * mb), 0.0)) / (8 * math.pi * s)


def phi_n(s, masses):
    """Phase-space volume by recursive splitting (nested adaptive quadrature)."""
    if len(masses) == 2:
        return phi2(s, *masses)
    m1, rest = masses[0], masses[1:]
    lo, hi = sum(rest) ** 2, (math.sqrt(s) - m1) ** 2
    val, _ = integrate.quad(lambda M2: phi2(s, m1, math.sqrt(M2)) * phi_n(M2, rest) / (2 * math.pi), lo, hi,
                            epsabs=0, epsrel=1e-10, limit=200)
    return val


def test_massless_volume_closed_forms():
    s = 1500.0 ** 2
    assert rambo.massless_volume(2, s) == pytest.approx(1 / (8 * math.pi), rel=1e-15)
    assert rambo.massless_volume(3, s) == pytest.approx(s / (256 * math.pi ** 3), rel=1e-15)
    for n in (4, 5):
        assert rambo.massless_volume(n, s) == pytest.approx(phi_n(s, [0.0] * n), rel=1e-8)


@pytest.mark.parametrize("mT", [MT, 0.0])
def test_two_body_weight_is_the_volume(mT):
    w = configs.WORKLOADS["ggtt"]
    _, wt = w.momenta(2000, mT=mT, with_weight=True)
    assert np.abs(wt / phi2(w.sqrt_s ** 2, mT, mT) - 1).max() <= 1e-14


@pytest.mark.parametrize("name,nevt", [("ggttg", 200000), ("ggttgg", 100000)])
def test_mean_massive_weight_is_the_volume(name, nevt):
    w = configs.WORKLOADS[name]
    masses = configs.final_masses(w.process)
    _, wt = rambo.generate(nevt, w.sqrt_s, [0.0, 0.0], masses, seed=11, with_weight=True)
    vol = phi_n(w.sqrt_s ** 2, masses[2:] + masses[:2])  # gluons first, the top pair last
    err = wt.std() / math.sqrt(nevt)
    assert err < 2e-3 * vol
    assert abs(wt.mean() - vol) <= 5 * err, (wt.mean(), vol, err)
    # the weight depends on the masses: the massless volume is well outside the error
    assert abs(rambo.massless_volume(len(masses), w.sqrt_s ** 2) - vol) > 50 * err


def test_no_retry_keeps_first_attempt_with_zero_weight():
    w = configs.WORKLOADS["ggttg"]
    p_retry, w_retry = w.momenta(3000, with_weight=True)
    p, wt = w.momenta(3000, retry=False, with_weight=True)
    ok = w.cut(p[:, 2:])
    assert 0.5 < ok.mean() < 1.0
    assert np.all(wt[~ok] == 0) and np.all(wt[ok] > 0)
    # accepted first attempts are the retried generator's events
    assert np.array_equal(p[ok], p_retry[ok]) and np.array_equal(wt[ok], w_retry[ok])


def test_eemumu_cross_section_closed_form(card):
    w = configs.WORKLOADS["eemumu"]
    nevt = 400000
    p, wt = w.momenta(nevt, with_weight=True)
    me = oracle.me2(oracle.EEMUMU, p, card)
    sigma, err = oracle.cross_section(me, wt, w.sqrt_s)
    ew = oracle.ew(card)
    sw2, cw2, e = ew["sw2"], ew["cw2"], ew["e"]
    mZ, wZ, s = card[0], card[1], w.sqrt_s ** 2
    gL, gR = -0.5 + sw2, sw2

    def A(gi, gj):
        return 1 / s + gi * gj / (sw2 * cw2) / (s - mZ ** 2 + 1j * mZ * wZ)

    exact = e ** 4 * s * sum(abs(A(a, b)) ** 2 for a in (gL, gR) for b in (gL, gR)) / (48 * math.pi)
    exact *= oracle.GEV2_TO_PB
    assert err < 2e-3 * exact
    assert abs(sigma - exact) <= 5 * err, (sigma, exact, err)
    # a dropped flux factor of 2 or a photon-only cross section lies far outside the error
    assert abs(4 * math.pi * (e ** 2 / (4 * math.pi)) ** 2 / (3 * s) * oracle.GEV2_TO_PB - sigma) > 50 * err
