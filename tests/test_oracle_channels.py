"""Pins for the oracle's diagram-by-diagram evaluation (channel weights).

The oracle enumerates the tree diagrams itself and evaluates each with its colour factor
stripped from the Feynman rules and kept apart.  Pins: the diagram counts (3 / 16 / 123 for
g g -> t tbar + 0..2 g, 1 / 2 / 8 / 50 for u ubar -> e+ e- + 0..3 g with photon and Z together),
distinct diagram keys, the sum over diagrams and terms of colour x value equal to the
colour-dressed amplitude (the plain definition) for random colours and spins, and the Bose
symmetry of the per-diagram weights under the exchange of two final-state gluons."""
import numpy as np
import pytest

import oracle
from workloads import configs

PROCS = [(oracle.GGTT, "ggtt", 3), (oracle.GGTTG, "ggttg", 16), (oracle.GGTTGG, "ggttgg", 123),
         (oracle.UUEE, "uuee", 1), (oracle.UUEEG, "uueeg", 2), (oracle.UUEEGG, "uueegg", 8),
         (oracle.UUEEGGG, "uueeggg", 50)]


@pytest.mark.parametrize("proc,key,nd", PROCS)
def test_diagram_counts_and_keys(proc, key, nd):
    keys = oracle.diagram_keys(proc)
    assert len(keys) == nd and len(set(keys)) == nd


def _dressed(proc, p, card, spins, col, row, column):
    import ctypes
    L = oracle.lib()
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    out = np.empty(2)
    sp = np.ascontiguousarray(spins, dtype=np.int32)
    cl = np.ascontiguousarray(col if len(col) else [0], dtype=np.int32)
    mom = np.ascontiguousarray(p)
    if proc in oracle.DY:
        rc = L.oracle_dressed_amp_dy(len(p), card.ctypes.data_as(dp), mom.ctypes.data_as(dp), sp.ctypes.data_as(ip),
                                     cl.ctypes.data_as(ip), column, row, -1, out.ctypes.data_as(dp))
    else:
        rc = L.oracle_dressed_amp(len(p), card.ctypes.data_as(dp), mom.ctypes.data_as(dp), sp.ctypes.data_as(ip),
                                  cl.ctypes.data_as(ip), row, column, -1, 0, out.ctypes.data_as(dp))
    assert rc == 0
    return complex(out[0], out[1])


@pytest.mark.parametrize("proc,key,nd", PROCS)
def test_sum_of_diagrams_is_the_dressed_amplitude(card, proc, key, nd):
    rng = np.random.default_rng(proc)
    p = configs.WORKLOADS[key].momenta(3, first_event=20)
    npar = p.shape[1]
    n = npar - 4 if proc in oracle.DY else npar - 2
    got, want = [], []
    for e in range(3):
        for _ in range(8):
            spins = rng.integers(0, 2, npar)
            col = rng.integers(0, 8, n)
            r, c = (int(x) for x in rng.integers(0, 3, 2))
            got.append(oracle.diagram_sum(proc, p[e], card, spins, col, r, c))
            want.append(_dressed(proc, p[e], card, spins, col, r, c))
    got, want = np.array(got), np.array(want)
    scale = np.abs(want).max()
    assert scale > 0
    # exact zeros of the colour algebra come out as rounding noise on both sides
    assert np.abs(got - want).max() <= 1e-12 * scale


def test_sum_of_diagrams_ggttggg(card):
    """g g -> t tbar g g g (1240 diagrams, 1890 terms) on two colour and spin assignments."""
    p = configs.WORKLOADS["ggttggg"].momenta(1)[0]
    for spins, col, r, c in (([0, 1, 1, 0, 1, 0, 1], [0, 3, 5, 2, 7], 0, 2), ([1, 1, 0, 0, 0, 1, 1], [1, 1, 4, 6, 2], 2, 1)):
        a = oracle.diagram_sum(oracle.GGTTGGG, p, card, spins, col, r, c)
        b = _dressed(oracle.GGTTGGG, p, card, spins, col, r, c)
        assert abs(a - b) <= 1e-11 * max(abs(b), 1e-300)


@pytest.mark.parametrize("proc,key,g1,g2", [(oracle.GGTTGG, "ggttgg", 4, 5), (oracle.UUEEGG, "uueegg", 4, 5),
                                            (oracle.UUEEGGG, "uueeggg", 5, 6)])
def test_channel_weights_bose_symmetry(card, proc, key, g1, g2):
    """Swapping the momenta of two final gluons maps the weight of each diagram onto the diagram
    with the two gluons' labels swapped."""
    p = configs.WORKLOADS[key].momenta(4, first_event=7)
    q = p.copy()
    q[:, [g1, g2]] = q[:, [g2, g1]]
    keys = oracle.diagram_keys(proc)
    w, ws = oracle.channel_weights(proc, p, card), oracle.channel_weights(proc, q, card)

    def swap(k):
        import re
        canon = re.sub(r"g(\d+)", lambda m: "g" + str({g1: g2, g2: g1}.get(int(m.group(1)), int(m.group(1)))), k)
        return canon

    def canonical(k):
        # re-sort the children of every vertex after relabelling
        def parse(s, i):
            if s[i] == "g":
                j = i + 1
                while j < len(s) and s[j].isdigit():
                    j += 1
                return s[i:j], j
            close = ")" if s[i] == "(" else "]"
            parts, j = [], i + 1
            while True:
                t, j = parse(s, j)
                parts.append(t)
                if s[j] == close:
                    break
                j += 1
            return s[i] + ",".join(sorted(parts)) + close, j + 1
        return ";".join(e if e == "W" else parse(e, 0)[0] for e in k.split(";"))

    index = {k: i for i, k in enumerate(keys)}
    perm = [index[canonical(swap(k))] for k in keys]
    assert np.allclose(ws[:, perm], w, rtol=1e-12, atol=0)
    assert np.all(w > 0)
