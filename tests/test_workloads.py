"""Seeded input generators: Philox known answers, RAMBO kinematics, cuts, determinism."""
import os

import numpy as np
import pytest

from workloads import configs, rambo
from workloads.philox import philox4x32

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox4x32(tuple(np.uint32(x) for x in v[0:4]), tuple(np.uint32(x) for x in v[4:6]))
        assert [int(o) for o in out] == v[6:10]


def mdot(a, b):
    return a[..., 0] * b[..., 0] - (a[..., 1:] * b[..., 1:]).sum(-1)


@pytest.mark.parametrize("name", ["eemumu", "ggtt", "ggttg", "ggttgg", "ggttggg"])
def test_rambo_conservation_and_mass_shell(name):
    w = configs.WORKLOADS[name]
    p = w.momenta(4000)
    total = p[:, 0] + p[:, 1] - p[:, 2:].sum(axis=1)
    assert np.abs(total).max() <= 1e-13 * w.sqrt_s
    masses = np.array([0.0, 0.0] + configs.final_masses(w.process))
    m2 = mdot(p, p)
    assert np.abs(m2 - masses ** 2).max() <= 1e-13 * w.sqrt_s ** 2 / 4
    assert np.all(p[..., 0] > 0)


def test_rambo_two_body_is_isotropic():
    # flat two-body phase space: cos(theta) uniform on [-1, 1], phi uniform
    p = configs.WORKLOADS["eemumu"].momenta(40000)
    ct = p[:, 3, 3] / np.linalg.norm(p[:, 3, 1:], axis=1)
    hist, _ = np.histogram(ct, bins=10, range=(-1, 1))
    expected = len(ct) / 10
    chi2 = ((hist - expected) ** 2 / expected).sum()
    assert chi2 < 35.0  # 9 degrees of freedom, p ~ 1e-4
    assert np.allclose(p[:, 2, 0], 250.0) and np.allclose(p[:, 3, 0], 250.0)


def test_cuts_are_applied():
    p = configs.WORKLOADS["ggttg"].momenta(3000)
    assert np.all(np.hypot(p[:, 4, 1], p[:, 4, 2]) > 20.0)
    p = configs.WORKLOADS["ggttgg"].momenta(3000)
    assert np.all(rambo.delta_r(p[:, 4], p[:, 5]) > 0.4)


def test_events_independent_of_batching():
    w = configs.WORKLOADS["ggttgg"]
    whole = w.momenta(600)
    parts = np.concatenate([w.momenta(250), w.momenta(350, first_event=250)])
    assert np.array_equal(whole, parts)


def test_served_request_stream():
    arrival, procs, nevt, first = configs.served_requests(4000)
    assert np.all(np.diff(arrival) > 0)
    assert abs(np.mean(np.diff(arrival)) - 1 / 200.0) < 0.0005
    assert nevt.min() >= 256 and nevt.max() <= 65536
    assert set(np.unique(procs)) == {configs.GGTT, configs.GGTTG, configs.GGTTGG, configs.GGTTGGG}
