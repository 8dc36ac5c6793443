"""Pins for the oracle's building blocks: Dirac and SU(3) algebra, external states, EW inputs.

Each check is a textbook identity, so a wrong matrix entry, sign or phase in the
oracle's explicit representations fails here.
"""
import numpy as np
import pytest

import oracle
from workloads import configs

G = np.diag([1.0, -1.0, -1.0, -1.0])


def gammas():
    return [oracle.gamma(mu) for mu in range(4)], oracle.gamma(5)


def test_clifford_algebra():
    g, g5 = gammas()
    for mu in range(4):
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(anti, 2 * G[mu, nu] * np.eye(4), atol=0)
        assert np.allclose(g5 @ g[mu] + g[mu] @ g5, 0, atol=0)
    assert np.allclose(g5 @ g5, np.eye(4), atol=0)
    assert np.allclose(1j * g[0] @ g[1] @ g[2] @ g[3], g5, atol=1e-15)
    # hermiticity: gamma0 gamma^mu gamma0 = gamma^mu dagger
    for mu in range(4):
        assert np.allclose(g[0] @ g[mu] @ g[0], g[mu].conj().T, atol=0)


def test_su3_algebra():
    T, f = oracle.su3()
    for a in range(8):
        for b in range(8):
            assert abs(np.trace(T[a] @ T[b]) - (0.5 if a == b else 0.0)) < 1e-15
            comm = T[a] @ T[b] - T[b] @ T[a]
            assert np.allclose(comm, 1j * np.einsum("c,cij->ij", f[a, b], T), atol=1e-15)
    # textbook values of the structure constants (1-based: f123 = 1, f147 = 1/2, f458 = sqrt(3)/2)
    assert abs(f[0, 1, 2] - 1.0) < 1e-15
    assert abs(f[0, 3, 6] - 0.5) < 1e-15
    assert abs(f[3, 4, 7] - np.sqrt(3) / 2) < 1e-15
    assert np.allclose(f, -np.transpose(f, (1, 0, 2)), atol=0)
    assert np.allclose(f, np.transpose(f, (1, 2, 0)), atol=1e-15)
    # Casimirs: sum_a T^a T^a = C_F 1 with C_F = 4/3;  f^{acd} f^{bcd} = C_A delta^{ab}, C_A = 3
    assert np.allclose(np.einsum("aij,ajk->ik", T, T), 4.0 / 3.0 * np.eye(3), atol=1e-15)
    assert np.allclose(np.einsum("acd,bcd->ab", f, f), 3.0 * np.eye(8), atol=1e-14)


def random_momenta(rng, m, n=20, special=True):
    out = []
    for i in range(n):
        P = rng.uniform(1, 500)
        v = rng.normal(size=3)
        v *= P / np.linalg.norm(v)
        out.append(v)
    if special:  # exactly along the beam axis, both directions
        out += [np.array([0.0, 0.0, 300.0]), np.array([0.0, 0.0, -300.0])]
    return [np.concatenate([[np.sqrt(m * m + v @ v)], v]) for v in out]


def slash(p):
    g, _ = gammas()
    return g[0] * p[0] - g[1] * p[1] - g[2] * p[2] - g[3] * p[3]


@pytest.mark.parametrize("m", [0.0, 173.0])
def test_spinor_identities(m):
    rng = np.random.default_rng(1)
    g, g5 = gammas()
    # helicity operator Sigma . p-hat with Sigma^k = gamma5 gamma0 gamma^k
    for p in random_momenta(rng, m):
        ps = slash(p)
        us = {l: oracle.external(0, p, m, l) for l in (-1, 1)}
        vs = {l: oracle.external(1, p, m, l) for l in (-1, 1)}
        ubs = {l: oracle.external(2, p, m, l) for l in (-1, 1)}
        vbs = {l: oracle.external(3, p, m, l) for l in (-1, 1)}
        scale = p[0]
        for l in (-1, 1):
            assert np.abs((ps - m * np.eye(4)) @ us[l]).max() <= 1e-13 * scale
            assert np.abs((ps + m * np.eye(4)) @ vs[l]).max() <= 1e-13 * scale
            assert np.abs(ubs[l] @ (ps - m * np.eye(4))).max() <= 1e-13 * scale
            assert np.abs(vbs[l] @ (ps + m * np.eye(4))).max() <= 1e-13 * scale
            assert abs(ubs[l] @ us[l] - 2 * m) <= 1e-13 * scale
            assert abs(vbs[l] @ vs[l] + 2 * m) <= 1e-13 * scale
            phat = p[1:] / np.linalg.norm(p[1:])
            hel = sum(phat[k - 1] * (g5 @ g[0] @ g[k]) for k in (1, 2, 3))
            assert np.abs(hel @ us[l] - l * us[l]).max() <= 1e-13 * np.sqrt(scale)
        compl_u = sum(np.outer(us[l], ubs[l]) for l in (-1, 1))
        compl_v = sum(np.outer(vs[l], vbs[l]) for l in (-1, 1))
        assert np.abs(compl_u - (ps + m * np.eye(4))).max() <= 1e-13 * scale
        assert np.abs(compl_v - (ps - m * np.eye(4))).max() <= 1e-13 * scale


def test_polarisation_vectors():
    rng = np.random.default_rng(2)
    for k in random_momenta(rng, 0.0):
        e = [oracle.external(4, k, 0.0, s) for s in (0, 1)]
        for s in (0, 1):
            assert abs(e[s] @ G @ k) <= 1e-13 * k[0]
            assert abs(e[s] @ G @ e[s] + 1) <= 1e-14
            assert abs(e[s][0]) == 0
        assert abs(e[0] @ G @ e[1]) <= 1e-14
        # completeness: sum_s e^i e^j = delta^ij - k^i k^j / |k|^2
        kh = k[1:] / np.linalg.norm(k[1:])
        tr = sum(np.outer(e[s][1:].real, e[s][1:].real) for s in (0, 1))
        assert np.abs(tr - (np.eye(3) - np.outer(kh, kh))).max() <= 1e-14


def test_electroweak_inputs():
    # mZ = 91.188, 1/alpha = 132.5, G_F = 1.16639e-5 give mW = 80.418 and sin^2(theta_W) = 0.22226
    ew = oracle.ew(configs.card_array())
    mW = 91.188 * np.sqrt(ew["cw2"])
    assert abs(mW - 80.418) < 5e-4
    assert abs(ew["sw2"] - 0.2222629) < 1e-6
    assert abs(ew["e"] - np.sqrt(4 * np.pi / 132.5)) < 1e-15


def test_iden():
    # initial spins x initial colours x (identical final-state gluons)!
    assert [oracle.iden(p) for p in range(10)] == [4, 256, 256, 512, 1536, 36, 36, 72, 216, 512]
