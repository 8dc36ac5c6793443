"""Pins for the oracle's |M|^2: closed forms, gauge and Lorentz invariance, Bose and C
symmetry, colour-dressed versus colour-ordered evaluation, colour-matrix identities.

Closed forms used (all averaged over initial spins and colours):
  e+e- -> mu+mu- via photon and Z, massless: helicity amplitudes give
    4 e^4 [(|A_LL|^2 + |A_RR|^2) u^2 + (|A_LR|^2 + |A_RL|^2) t^2] / 4,
    A_ij = 1/s + g_i g_j / (sw^2 cw^2 (s - mZ^2 + i mZ wZ)), g_L = -1/2 + sw^2, g_R = sw^2
    (t = (p_e- - p_mu-)^2, u = (p_e- - p_mu+)^2).
  g g -> Q Qbar (Combridge 1979; Ellis, Stirling, Webber, "QCD and collider physics",
    eq. 10.12): g^4 (1/(6 t1 t2) - 3/8) (t1^2 + t2^2 + rho - rho^2/(4 t1 t2)),
    t1 = 2 p1.p3 / s, t2 = 2 p2.p3 / s, rho = 4 m^2 / s.
  g g -> g g: (9/2) g^4 (3 - t u / s^2 - s u / t^2 - s t / u^2).
"""
import itertools

import numpy as np
import pytest

import oracle
from workloads import configs

AS = 0.118
G4 = (4 * np.pi * AS) ** 2


def mdot(a, b):
    return a[..., 0] * b[..., 0] - (a[..., 1:] * b[..., 1:]).sum(-1)


def test_eemumu_closed_form_all_events(card):
    p = configs.WORKLOADS["eemumu"].momenta()
    assert p.shape == (16384, 4, 4)
    me = oracle.me2(oracle.EEMUMU, p, card)
    ew = oracle.ew(card)
    sw2, cw2, e = ew["sw2"], ew["cw2"], ew["e"]
    mZ, wZ = card[0], card[1]
    pep, pem, pmp, pmm = p[:, 0], p[:, 1], p[:, 2], p[:, 3]
    s = mdot(pep + pem, pep + pem)
    t = mdot(pem - pmm, pem - pmm)
    u = mdot(pem - pmp, pem - pmp)
    gL, gR = -0.5 + sw2, sw2

    def A(gi, gj):
        return 1 / s + gi * gj / (sw2 * cw2) / (s - mZ ** 2 + 1j * mZ * wZ)

    cf = e ** 4 * ((abs(A(gL, gL)) ** 2 + abs(A(gR, gR)) ** 2) * u ** 2
                   + (abs(A(gL, gR)) ** 2 + abs(A(gR, gL)) ** 2) * t ** 2)
    assert np.abs(me / cf - 1).max() <= 1e-13


@pytest.mark.parametrize("mT", [173.0, 0.0])
def test_ggtt_closed_form(mT):
    card = configs.card_array(dict(mT=mT))
    p = configs.WORKLOADS["ggtt"].momenta(20000, mT=mT)
    me = oracle.me2(oracle.GGTT, p, card, AS)
    s = mdot(p[:, 0] + p[:, 1], p[:, 0] + p[:, 1])
    # beams along +-z at sqrt(s)/2: 2 p1.p3 / s = (E3 - pz3)/sqrt(s), 2 p2.p3 / s = (E3 + pz3)/sqrt(s);
    # the smaller of E3 -+ pz3 is rewritten as (m^2 + pT^2)/(E3 +- pz3) to avoid cancellation
    E3, pz3 = p[:, 2, 0], p[:, 2, 3]
    mt2 = mT ** 2 + p[:, 2, 1] ** 2 + p[:, 2, 2] ** 2
    em = np.where(pz3 > 0, mt2 / (E3 + pz3), E3 - pz3)
    ep = np.where(pz3 > 0, E3 + pz3, mt2 / (E3 - pz3))
    t1 = em / np.sqrt(s)
    t2 = ep / np.sqrt(s)
    rho = 4 * mT ** 2 / s
    cf = G4 * (1 / (6 * t1 * t2) - 3 / 8) * (t1 ** 2 + t2 ** 2 + rho - rho ** 2 / (4 * t1 * t2))
    rel = np.abs(me / cf - 1)
    # the closed form itself cancels in 1/(6 t1 t2) - 3/8 near t1 t2 = 4/9; allow for that
    cond = 1 + np.abs(1 / (6 * t1 * t2)) / np.abs(1 / (6 * t1 * t2) - 3 / 8)
    assert np.max(rel / cond) <= 2e-14


def test_gggg_closed_form(card):
    p = configs.WORKLOADS["ggtt"].momenta(4, mT=0.0)
    me = oracle.me2(oracle.GGGG, p, card, AS, mode=oracle.DRESSED) * 2  # undo the 1/2! for identical gluons
    s = mdot(p[:, 0] + p[:, 1], p[:, 0] + p[:, 1])
    t = mdot(p[:, 0] - p[:, 2], p[:, 0] - p[:, 2])
    u = mdot(p[:, 0] - p[:, 3], p[:, 0] - p[:, 3])
    cf = 4.5 * G4 * (3 - t * u / s ** 2 - s * u / t ** 2 - s * t / u ** 2)
    assert np.abs(me / cf - 1).max() <= 1e-13


@pytest.mark.parametrize("proc,key,nevt", [(oracle.GGTT, "ggtt", 200), (oracle.GGTTG, "ggttg", 40),
                                           (oracle.GGTTGG, "ggttgg", 16)])
def test_dressed_equals_ordered(card, proc, key, nevt):
    """|M|^2 summed over every external colour assignment with explicit generators (the plain
    definition) equals the colour-ordered amplitudes contracted with the colour matrix."""
    p = configs.WORKLOADS[key].momenta(nevt, first_event=100)
    a = oracle.me2(proc, p, card, AS, mode=oracle.DRESSED)
    b = oracle.me2(proc, p, card, AS, mode=oracle.ORDERED)
    assert np.abs(a / b - 1).max() <= 1e-12


@pytest.mark.parametrize("key,n", [("ggttg", 3), ("ggttgg", 4), ("ggttggg", 5)])
def test_dressed_amplitude_is_sum_over_orderings(card, key, n):
    """Colour decomposition amplitude by amplitude: for explicit gluon colours a_k and quark colours
    (i, j), the colour-dressed amplitude (every Feynman diagram with explicit generators and
    structure constants) equals sum over orderings s of (T^a_s1 ... T^a_sn)_ij A(s), for random
    spin and colour assignments.  This pins the n = 5 ordered amplitudes (four-gluon terms
    included) to the plain definition, where the summed |M|^2 would take hours."""
    T, _ = oracle.su3()
    perms = list(itertools.permutations(range(n)))
    rng = np.random.default_rng(20 + n)
    p = configs.WORKLOADS[key].momenta(3, first_event=200)
    checked = 0
    for ev in p:
        for _ in range(3):
            sp = rng.integers(0, 2, n + 2)
            A = oracle.partial_amps(ev, card, sp)
            scale = np.abs(A).max()
            for _ in range(12):
                col = rng.integers(0, 8, n)
                i3, j4 = (int(x) for x in rng.integers(0, 3, 2))
                dressed = oracle.dressed_amp(ev, card, sp, col, i3, j4)
                ordered = 0j
                for s, perm in enumerate(perms):
                    M = np.eye(3, dtype=complex)
                    for g in perm:
                        M = M @ T[col[g]]
                    ordered += M[i3, j4] * A[s]
                assert abs(dressed - ordered) <= 1e-13 * scale
                checked += abs(dressed) > 1e-3 * scale
    assert checked >= 20  # most assignments give a nonzero amplitude


def _random_spins(rng, npar):
    return rng.integers(0, 2, npar)


@pytest.mark.parametrize("proc,key", [(oracle.GGTTG, "ggttg"), (oracle.GGTTGG, "ggttgg")])
def test_ward_identity_ordered(card, proc, key):
    """Each colour-ordered amplitude vanishes when one gluon polarisation is replaced by its momentum."""
    rng = np.random.default_rng(3)
    npar = oracle.NPAR[proc]
    p = configs.WORKLOADS[key].momenta(3)
    for ev in p:
        for trial in range(4):
            sp = _random_spins(rng, npar)
            ref = np.abs(oracle.partial_amps(ev, card, sp)).max()
            # scale of the amplitude with the polarisation replaced: |k| times the amplitude
            for g in range(npar - 2):
                w = oracle.partial_amps(ev, card, sp, gauge_leg=g)
                assert np.abs(w).max() <= 1e-11 * ref * ev[0, 0]


def test_ward_identity_ordered_ggttggg(card):
    rng = np.random.default_rng(4)
    p = configs.Workload("x", configs.GGTTGGG, 0, 2000.0, 5).momenta(2)
    for ev in p:
        sp = _random_spins(rng, 7)
        ref = np.abs(oracle.partial_amps(ev, card, sp)).max()
        for g in range(5):
            w = oracle.partial_amps(ev, card, sp, gauge_leg=g)
            assert np.abs(w).max() <= 1e-11 * ref * ev[0, 0]


def test_ward_identity_dressed(card):
    rng = np.random.default_rng(5)
    ev = configs.WORKLOADS["ggttgg"].momenta(1)[0]
    checked = 0
    for col in itertools.product(range(8), repeat=4):
        if rng.random() > 0.05:
            continue
        sp = _random_spins(rng, 6)
        i3, j4 = rng.integers(0, 3, 2)
        a = oracle.dressed_amp(ev, card, sp, col, i3, j4)
        if abs(a) == 0:
            continue
        for g in range(4):
            w = oracle.dressed_amp(ev, card, sp, col, i3, j4, gauge_leg=g)
            assert abs(w) <= 1e-11 * abs(a) * ev[0, 0] + 1e-300
        checked += 1
        if checked >= 12:
            break
    assert checked >= 5


def boost_matrix(beta_vec):
    b2 = beta_vec @ beta_vec
    g = 1 / np.sqrt(1 - b2)
    L = np.eye(4)
    L[0, 0] = g
    L[0, 1:] = L[1:, 0] = g * beta_vec
    L[1:, 1:] += (g - 1) * np.outer(beta_vec, beta_vec) / b2
    return L


def rotation_matrix(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    R = np.eye(4)
    R[1:, 1:] = q
    return R


@pytest.mark.parametrize("proc,key,nevt", [(oracle.GGTTG, "ggttg", 40), (oracle.GGTTGG, "ggttgg", 40),
                                           (oracle.EEMUMU, "eemumu", 200)])
def test_lorentz_invariance(card, proc, key, nevt):
    rng = np.random.default_rng(6)
    p = configs.WORKLOADS[key].momenta(nevt)
    ref = oracle.me2(proc, p, card, AS)
    for trial in range(3):
        v = rng.normal(size=3)
        v *= rng.uniform(0.1, 0.9) / np.linalg.norm(v)
        L = boost_matrix(v) @ rotation_matrix(rng)
        q = np.einsum("ij,enj->eni", L, p)
        me = oracle.me2(proc, q, card, AS)
        assert np.abs(me / ref - 1).max() <= 1e-11


def test_lorentz_invariance_ggttggg(card):
    rng = np.random.default_rng(7)
    p = configs.Workload("x", configs.GGTTGGG, 0, 2000.0, 5).momenta(8)
    ref = oracle.me2(oracle.GGTTGGG, p, card, AS)
    v = np.array([0.3, -0.5, 0.2])
    q = np.einsum("ij,enj->eni", boost_matrix(v) @ rotation_matrix(rng), p)
    assert np.abs(oracle.me2(oracle.GGTTGGG, q, card, AS) / ref - 1).max() <= 1e-11


@pytest.mark.parametrize("proc,key", [(oracle.GGTTG, "ggttg"), (oracle.GGTTGG, "ggttgg")])
def test_bose_and_charge_symmetry(card, proc, key):
    p = configs.WORKLOADS[key].momenta(60)
    ref = oracle.me2(proc, p, card, AS)
    npar = oracle.NPAR[proc]
    # swap the incoming gluons
    q = p.copy()
    q[:, [0, 1]] = p[:, [1, 0]]
    assert np.abs(oracle.me2(proc, q, card, AS) / ref - 1).max() <= 1e-12
    # swap top and antitop (charge conjugation)
    q = p.copy()
    q[:, [2, 3]] = p[:, [3, 2]]
    assert np.abs(oracle.me2(proc, q, card, AS) / ref - 1).max() <= 1e-12
    # permute the outgoing gluons
    if npar > 5:
        q = p.copy()
        q[:, [4, 5]] = p[:, [5, 4]]
        assert np.abs(oracle.me2(proc, q, card, AS) / ref - 1).max() <= 1e-12


def test_extended_precision_agrees(card):
    p = configs.WORKLOADS["ggttgg"].momenta(200)
    a = oracle.me2(oracle.GGTTGG, p, card, AS)
    b = oracle.me2(oracle.GGTTGG, p, card, AS, extended=True)
    assert np.abs(a / b - 1).max() <= 1e-12


def test_colour_matrix_identities():
    from fractions import Fraction
    # n = 2 by hand from Sum_b T^b T^a T^b = -T^a / (2 N): C = (1/3) [[16, -2], [-2, 16]]
    C2 = oracle.colour_matrix(2)
    assert np.allclose(C2, np.array([[16, -2], [-2, 16]]) / 3.0, atol=1e-15, rtol=0)
    for n in range(2, 6):
        C = oracle.colour_matrix(n)
        perms = list(itertools.permutations(range(n)))
        assert np.allclose(C, C.T, atol=0)
        # diagonal: N C_F^n = 3 (4/3)^n
        assert np.allclose(np.diag(C), 3 * (4.0 / 3.0) ** n, rtol=1e-15)
        # relabelling the summed gluon colours: C(s, t) depends on s^-1 t only
        index = {p: i for i, p in enumerate(perms)}
        inv0 = {}
        for i, s in enumerate(perms):
            for j, t in enumerate(perms):
                rel = tuple(s.index(x) for x in t)
                if rel in inv0:
                    assert abs(C[i, j] - inv0[rel]) <= 1e-13
                else:
                    inv0[rel] = C[i, j]
        # rational with a small denominator
        num = C * 4 * 3 ** (n - 1)
        assert np.abs(num - np.round(num)).max() <= 1e-9


@pytest.mark.parametrize("proc,key,nevt", [(oracle.EEMUMU, "eemumu", 20), (oracle.GGTT, "ggtt", 20),
                                           (oracle.GGTTG, "ggttg", 10), (oracle.GGTTGG, "ggttgg", 4)])
def test_helicity_basis_sums_to_linear_basis(card, proc, key, nevt):
    """Circular gluon polarisations summed over helicities give the linear-polarisation sum."""
    p = configs.WORKLOADS[key].momenta(nevt)
    tot = oracle.me2(proc, p, card, AS)
    for e in range(nevt):
        assert oracle.me2_hel(proc, p[e], card, AS).sum() == pytest.approx(tot[e], rel=1e-13)


def test_eemumu_helicity_closed_form(card):
    """Massless e+e- -> mu+mu-: only opposite helicities on each fermion line survive; with
    bit 3-k for particle k (e+, e-, mu+, mu-) set for helicity +1, index 10 is (e-_L, mu-_L),
    5 (e-_R, mu-_R), 9 (e-_L, mu-_R), 6 (e-_R, mu-_L), with values e^4 |A_ij|^2 u^2 or t^2."""
    p = configs.WORKLOADS["eemumu"].momenta(50)
    ew = oracle.ew(card)
    sw2, cw2, e = ew["sw2"], ew["cw2"], ew["e"]
    mZ, wZ = card[0], card[1]
    gL, gR = -0.5 + sw2, sw2
    for ev in p:
        hel = oracle.me2_hel(oracle.EEMUMU, ev, card)
        s = mdot(ev[0] + ev[1], ev[0] + ev[1])
        t = mdot(ev[1] - ev[3], ev[1] - ev[3])
        u = mdot(ev[1] - ev[2], ev[1] - ev[2])
        A = lambda gi, gj: 1 / s + gi * gj / (sw2 * cw2) / (s - mZ ** 2 + 1j * mZ * wZ)
        want = np.zeros(16)
        want[10] = e ** 4 * abs(A(gL, gL)) ** 2 * u ** 2
        want[5] = e ** 4 * abs(A(gR, gR)) ** 2 * u ** 2
        want[9] = e ** 4 * abs(A(gL, gR)) ** 2 * t ** 2
        want[6] = e ** 4 * abs(A(gR, gL)) ** 2 * t ** 2
        assert np.abs(hel - want).max() <= 1e-13 * want.sum()


def test_ggtt_helicity_selection_rules():
    """Massless quarks: helicity is conserved along the quark line and the two incoming gluons
    need opposite helicities (all-outgoing MHV counting), so only 4 of 16 configurations
    survive; two-to-two kinematics is planar, so flipping every helicity leaves |M_h|^2."""
    card0 = configs.card_array(dict(mT=0.0))
    p = configs.WORKLOADS["ggtt"].momenta(30, mT=0.0)
    allowed = {0b0101, 0b0110, 0b1001, 0b1010}
    for ev in p:
        hel = oracle.me2_hel(oracle.GGTT, ev, card0, AS)
        for h in range(16):
            if h not in allowed:
                assert hel[h] <= 1e-26 * hel.sum()
        assert min(hel[h] for h in allowed) > 1e-6 * hel.sum()
    card = configs.card_array()
    for ev in configs.WORKLOADS["ggtt"].momenta(30):
        hel = oracle.me2_hel(oracle.GGTT, ev, card, AS)
        assert np.abs(hel - hel[::-1]).max() <= 1e-13 * hel.sum()
