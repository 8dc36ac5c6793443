"""Pins for the oracle's Drell-Yan family u ubar -> e+ e- + n g (photon and Z, n = 0..3).

  n = 0: the closed form of massless f fbar -> l+ l- through a photon and a Z, helicity by
    helicity: with A_ij = Q_u Q_e / s + g_i^u g_j^e / (sw^2 cw^2 (s - mZ^2 + i mZ wZ))
    (g_L = T3 - Q sw^2, g_R = -Q sw^2), the averaged |M_h|^2 is e^4 |A_ij|^2 u^2 / 3 for equal
    chiralities i = j and e^4 |A_ij|^2 t^2 / 3 otherwise (t = (p_u - p_e-)^2,
    u = (p_u - p_e+)^2; the colour sum gives 3, the average 1/36).
  n >= 1: gauge invariance of every colour-ordered amplitude (gluon polarisation replaced by
    its momentum), the colour-dressed sum over every colour assignment (the plain definition)
    against the colour-ordered amplitudes with the colour matrix, amplitude by amplitude for
    random colour assignments, Lorentz invariance, Bose symmetry of the gluons, and the
    helicity-basis sum equal to the linear-polarisation sum.
"""
import itertools

import numpy as np
import pytest

import oracle
from workloads import configs

from test_oracle_physics import boost_matrix, mdot, rotation_matrix

AS = 0.118
KEYS = {oracle.UUEE: "uuee", oracle.UUEEG: "uueeg", oracle.UUEEGG: "uueegg", oracle.UUEEGGG: "uueeggg"}


def _A(s, gi, gj, ew, card):
    sw2, cw2 = ew["sw2"], ew["cw2"]
    mZ, wZ = card[0], card[1]
    return (2.0 / 3.0) * (-1.0) / s + gi * gj / (sw2 * cw2) / (s - mZ ** 2 + 1j * mZ * wZ)


def test_uuee_helicity_closed_form(card):
    p = configs.WORKLOADS["uuee"].momenta(400)
    ew = oracle.ew(card)
    sw2, e = ew["sw2"], ew["e"]
    gLu, gRu = 0.5 - 2.0 / 3.0 * sw2, -2.0 / 3.0 * sw2
    gLe, gRe = -0.5 + sw2, sw2
    tot = oracle.me2(oracle.UUEE, p, card, AS)
    for k, ev in enumerate(p):
        hel = oracle.me2_hel(oracle.UUEE, ev, card, AS)
        s = mdot(ev[0] + ev[1], ev[0] + ev[1])
        t = mdot(ev[0] - ev[3], ev[0] - ev[3])
        u = mdot(ev[0] - ev[2], ev[0] - ev[2])
        want = np.zeros(16)
        # index bit 3-k set for helicity +1 of particle k (u, ubar, e+, e-)
        want[0b0110] = e ** 4 * abs(_A(s, gLu, gLe, ew, card)) ** 2 * u ** 2 / 3  # u_L, e-_L
        want[0b1001] = e ** 4 * abs(_A(s, gRu, gRe, ew, card)) ** 2 * u ** 2 / 3  # u_R, e-_R
        want[0b0101] = e ** 4 * abs(_A(s, gLu, gRe, ew, card)) ** 2 * t ** 2 / 3  # u_L, e-_R
        want[0b1010] = e ** 4 * abs(_A(s, gRu, gLe, ew, card)) ** 2 * t ** 2 / 3  # u_R, e-_L
        assert np.abs(hel - want).max() <= 1e-13 * want.max()
        assert tot[k] == pytest.approx(want.sum(), rel=1e-13)


@pytest.mark.parametrize("proc,nevt", [(oracle.UUEE, 100), (oracle.UUEEG, 60), (oracle.UUEEGG, 6)])
def test_dy_dressed_equals_ordered(card, proc, nevt):
    p = configs.WORKLOADS[KEYS[proc]].momenta(nevt, first_event=50)
    a = oracle.me2(proc, p, card, AS, mode=oracle.DRESSED)
    b = oracle.me2(proc, p, card, AS, mode=oracle.ORDERED)
    assert np.abs(a / b - 1).max() <= 1e-12


@pytest.mark.parametrize("proc,n", [(oracle.UUEEG, 1), (oracle.UUEEGG, 2), (oracle.UUEEGGG, 3)])
def test_dy_dressed_amplitude_is_sum_over_orderings(card, proc, n):
    """For explicit gluon colours a_k, u colour i and ubar colour j, the colour-dressed amplitude
    equals sum over orderings s of (T^a_s1 ... T^a_sn)_ji A(s) (the ordering read from the ubar end)."""
    T, _ = oracle.su3()
    perms = list(itertools.permutations(range(n)))
    rng = np.random.default_rng(40 + n)
    p = configs.WORKLOADS[KEYS[proc]].momenta(3, first_event=300)
    nonzero = 0
    for ev in p:
        for _ in range(3):
            sp = rng.integers(0, 2, n + 4)
            # opposite helicities on the quark and on the lepton line (the others vanish exactly)
            sp[1], sp[3] = 1 - sp[0], 1 - sp[2]
            A = oracle.partial_amps_dy(ev, card, sp)
            scale = np.abs(A).max()
            for _ in range(10):
                col = rng.integers(0, 8, n)
                i1, j2 = (int(x) for x in rng.integers(0, 3, 2))
                dressed = oracle.dressed_amp_dy(ev, card, sp, col, i1, j2)
                ordered = 0j
                for s, perm in enumerate(perms):
                    M = np.eye(3, dtype=complex)
                    for g in perm:
                        M = M @ T[col[g]]
                    ordered += M[j2, i1] * A[s]
                assert abs(dressed - ordered) <= 1e-13 * scale
                nonzero += abs(dressed) > 1e-3 * scale
    assert nonzero >= 10  # many assignments have a vanishing colour factor


@pytest.mark.parametrize("proc,n", [(oracle.UUEEG, 1), (oracle.UUEEGG, 2), (oracle.UUEEGGG, 3)])
def test_dy_ward_identity(card, proc, n):
    """Every colour-ordered amplitude vanishes when a gluon polarisation becomes its momentum."""
    rng = np.random.default_rng(50 + n)
    p = configs.WORKLOADS[KEYS[proc]].momenta(3, first_event=400)
    for ev in p:
        for _ in range(3):
            sp = rng.integers(0, 2, n + 4)
            sp[1], sp[3] = 1 - sp[0], 1 - sp[2]
            ref = np.abs(oracle.partial_amps_dy(ev, card, sp)).max()
            for g in range(n):
                w = oracle.partial_amps_dy(ev, card, sp, gauge_leg=g)
                assert np.abs(w).max() <= 1e-11 * ref * ev[0, 0]


def test_dy_ward_identity_dressed(card):
    rng = np.random.default_rng(60)
    ev = configs.WORKLOADS["uueegg"].momenta(1)[0]
    checked = 0
    for _ in range(120):
        sp = rng.integers(0, 2, 6)
        sp[1], sp[3] = 1 - sp[0], 1 - sp[2]
        col = rng.integers(0, 8, 2)
        i1, j2 = (int(x) for x in rng.integers(0, 3, 2))
        a = oracle.dressed_amp_dy(ev, card, sp, col, i1, j2)
        if abs(a) == 0:
            continue
        for g in range(2):
            w = oracle.dressed_amp_dy(ev, card, sp, col, i1, j2, gauge_leg=g)
            assert abs(w) <= 1e-11 * abs(a) * ev[0, 0]
        checked += 1
    assert checked >= 10


@pytest.mark.parametrize("proc,nevt", [(oracle.UUEEG, 40), (oracle.UUEEGG, 20), (oracle.UUEEGGG, 6)])
def test_dy_lorentz_invariance(card, proc, nevt):
    rng = np.random.default_rng(70)
    p = configs.WORKLOADS[KEYS[proc]].momenta(nevt)
    ref = oracle.me2(proc, p, card, AS)
    for _ in range(2):
        v = rng.normal(size=3)
        v *= rng.uniform(0.1, 0.9) / np.linalg.norm(v)
        q = np.einsum("ij,enj->eni", boost_matrix(v) @ rotation_matrix(rng), p)
        assert np.abs(oracle.me2(proc, q, card, AS) / ref - 1).max() <= 1e-11


@pytest.mark.parametrize("proc,nevt", [(oracle.UUEEGG, 30), (oracle.UUEEGGG, 6)])
def test_dy_gluon_bose_symmetry(card, proc, nevt):
    p = configs.WORKLOADS[KEYS[proc]].momenta(nevt)
    ref = oracle.me2(proc, p, card, AS)
    npar = oracle.NPAR[proc]
    for perm in itertools.permutations(range(4, npar)):
        q = p.copy()
        q[:, 4:] = p[:, list(perm)]
        assert np.abs(oracle.me2(proc, q, card, AS) / ref - 1).max() <= 1e-12


@pytest.mark.parametrize("proc,nevt", [(oracle.UUEE, 10), (oracle.UUEEG, 6), (oracle.UUEEGG, 3), (oracle.UUEEGGG, 1)])
def test_dy_helicity_basis_sums_to_linear_basis(card, proc, nevt):
    """Circular gluon polarisations summed over helicities give the linear-polarisation sum, and
    the massless quark and lepton lines keep 4 x 2^n helicity configurations (opposite helicities
    on each line, every gluon helicity)."""
    p = configs.WORKLOADS[KEYS[proc]].momenta(nevt)
    tot = oracle.me2(proc, p, card, AS)
    n = oracle.NPAR[proc] - 4
    for e in range(nevt):
        hel = oracle.me2_hel(proc, p[e], card, AS)
        assert hel.sum() == pytest.approx(tot[e], rel=1e-13)
        assert int(np.count_nonzero(hel > 1e-12 * hel.max())) == 4 * 2 ** n
