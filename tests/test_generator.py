"""The generator of the GPU path: diagram counts, exact colour matrices, and the generated
call sequences evaluated on the host CPU against the oracle.

The host evaluation compiles the generated process headers for the CPU (test-only
build, tests/hostcheck); it checks the generator and the Lorentz routines before
any GPU run.  The parity tests proper run the same code on the GPU.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2507_21039_amd.gen import colour, diagrams
from workloads import configs

HERE = os.path.dirname(os.path.abspath(__file__))
HOSTLIB = os.path.join(HERE, "_build", "libhostcheck.so")


def test_diagram_counts():
    # 3 / 16 / 123 / 1240 tree diagrams for g g -> t tbar + 0..3 g (four-gluon vertex counted once)
    assert [len(diagrams.diagrams(tuple([0, 1] + list(range(4, 4 + n))))) for n in range(4)] == [3, 16, 123, 1240]


def test_drell_yan_diagram_counts():
    # u ubar -> e+ e- + n g: the electroweak boson inserted anywhere along the quark line of the
    # gluon trees; photon and Z together 1 / 2 / 8 / 50 (apart: 2 / 4 / 16 / 100)
    assert [len(diagrams.diagrams_dy(tuple(range(4, 4 + n)))) for n in range(4)] == [1, 2, 8, 50]
    for n in range(4):
        g = diagrams.build_graph(n, "dy")
        assert g.ndiag == [1, 2, 8, 50][n]
        assert {a.diagram for a in g.amps} == set(range(g.ndiag))
        for a in g.amps:
            assert all(abs(c.re) + abs(c.im) == 1 for c in a.colour.terms.values())


def test_helicity_and_colour_counts():
    assert [2 ** (4 + n) for n in range(4)] == [16, 32, 64, 128]
    assert [len(colour.orderings(range(n + 2))) for n in range(4)] == [2, 6, 24, 120]


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_exact_colour_matrix_matches_oracle(n):
    basis, C = colour.colour_matrix(range(n))
    exact = np.array([[float(x) for x in row] for row in C])
    assert np.abs(exact - oracle.colour_matrix(n)).max() <= 1e-13 * np.abs(exact).max()
    N, D = colour.integer_form(C)
    assert D == {2: 3, 3: 9, 4: 54, 5: 324}[n]
    assert all(x == N[i][i] for i, row in enumerate(N) for x in [row[i]])


def test_jamp_coefficients_are_units():
    for n in range(3):
        g = diagrams.build_graph(n)
        for a in g.amps:
            for c in a.colour.terms.values():
                assert abs(c.re) + abs(c.im) == 1


def _hostlib():
    os.makedirs(os.path.dirname(HOSTLIB), exist_ok=True)
    src = os.path.join(HERE, "hostcheck", "hostcheck.hip")
    deps = [src] + [os.path.join(HERE, "..", "paper_2507_21039_amd", "csrc", f)
                    for f in ("helas.h", "params.h", "process.h", "procs/ggttgg.h", "procs/uueeggg.h",
                              "procs/ggttgg_fd.h")]
    if not os.path.exists(HOSTLIB) or os.path.getmtime(HOSTLIB) < max(os.path.getmtime(d) for d in deps):
        subprocess.run(["/opt/rocm/bin/hipcc", "-O1", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                        "-x", "hip", src, "-o", HOSTLIB], check=True)
    L = ctypes.CDLL(HOSTLIB)
    dp = ctypes.POINTER(ctypes.c_double)
    L.hostcheck_me2.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_double, ctypes.c_int64, dp, dp, dp]
    L.hostcheck_jamps.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp]
    return L


@pytest.fixture(scope="module")
def hostlib():
    if not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not available")
    return _hostlib()


def host_me2(L, proc, prec, p, card, alpha_s=0.118):
    dp = ctypes.POINTER(ctypes.c_double)
    p = np.ascontiguousarray(p)
    card = np.ascontiguousarray(card)
    out = np.empty(len(p))
    assert L.hostcheck_me2(proc, prec, card.ctypes.data_as(dp), alpha_s, len(p), p.ctypes.data_as(dp),
                           out.ctypes.data_as(dp), None) == 0
    return out


@pytest.mark.parametrize("key,proc,n", [("eemumu", 0, 4000), ("ggtt", 1, 4000), ("ggttg", 2, 600),
                                        ("ggttgg", 3, 150), ("uuee", 5, 2000), ("uueeg", 6, 1000),
                                        ("uueegg", 7, 300), ("uueeggg", 8, 60)])
def test_generated_code_on_host_matches_oracle(hostlib, card, key, proc, n):
    p = configs.WORKLOADS[key].momenta(n)
    ref = oracle.me2(proc, p, card)
    got = host_me2(hostlib, proc, 0, p, card)
    rel = np.abs(got / ref - 1)
    far = rel > 1e-13  # decided by the long double oracle (the FP64 oracle's own rounding)
    if far.any():
        ld = oracle.me2(proc, p[far], card, extended=True)
        assert np.abs(got[far] / ld - 1).max() <= 1e-13
    mixed = host_me2(hostlib, proc, 1, p, card)
    assert np.abs(mixed / ref - 1).max() <= 1e-5


@pytest.mark.parametrize("key,proc,n,first", [("ggttg", 2, 3000, 0), ("ggttgg", 3, 1500, 500000),
                                              ("uueegg", 7, 4000, 0)])
def test_generated_fp64_against_extended_precision(hostlib, card, key, proc, n, first):
    """The generated FP64 code against the long double oracle (the exact value of the same
    double inputs, every internal line's momentum summed over the side without the barred
    spinor's particle, as the oracle does).  The per-event table forms momentum sums and
    Q^2 - m^2 in compensated arithmetic, so the generated code stays within 2e-14 even on
    events where the FP64 oracle, which forms Q^2 - m^2 directly, is off by 1e-13 or more (the
    gg -> ttbar gg and u ubar -> e+ e- g g samples below hold such events)."""
    p = configs.WORKLOADS[key].momenta(n, first_event=first)
    ld = oracle.me2(proc, p, card, extended=True)
    got = host_me2(hostlib, proc, 0, p, card)
    ora = oracle.me2(proc, p, card)
    err_gen = np.abs(got / ld - 1)
    err_ora = np.abs(ora / ld - 1)
    print(f"generated max {err_gen.max():.3g}, FP64 oracle max {err_ora.max():.3g}")
    assert err_gen.max() <= 2e-14
    if key in ("ggttgg", "uueegg"):
        assert err_ora.max() > 1e-13  # the sample does exercise the ill-conditioned case


HOSTLIB7 = os.path.join(HERE, "_build", "libhostcheck7.so")


@pytest.fixture(scope="module")
def hostlib7():
    if not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not available")
    src = os.path.join(HERE, "hostcheck", "hostcheck7.hip")
    procs = os.path.join(HERE, "..", "paper_2507_21039_amd", "csrc", "procs")
    deps = [src] + [os.path.join(procs, f) for f in os.listdir(procs) if f.startswith("ggttggg")] + [
        os.path.join(procs, "..", f) for f in ("colour_blocked.h", "helas.h", "params.h", "process.h")]
    if not os.path.exists(HOSTLIB7) or os.path.getmtime(HOSTLIB7) < max(os.path.getmtime(d) for d in deps):
        os.makedirs(os.path.dirname(HOSTLIB7), exist_ok=True)
        subprocess.run(["/opt/rocm/bin/hipcc", "-O1", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                        "-x", "hip", src, "-o", HOSTLIB7], check=True)
    L = ctypes.CDLL(HOSTLIB7)
    dp = ctypes.POINTER(ctypes.c_double)
    L.hostcheck7_me2.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_int64, dp, dp]
    return L


def test_pieces_cover_every_term_once():
    """The split of g g -> t tbar g g g: every amplitude term in exactly one piece; every
    workspace slot written by exactly one statement and gathered into exactly one flow."""
    import json
    import re
    procs = os.path.join(HERE, "..", "paper_2507_21039_amd", "csrc", "procs")
    info = json.load(open(os.path.join(procs, "processes.json")))["ggttggg"]
    assert info["nchunk"] >= 2 and info["ncol"] == 120
    nterms = 0
    puts = []
    for c in range(info["nchunk"]):
        text = open(os.path.join(procs, f"ggttggg_c{c}.h")).read()
        nterms += int(re.search(r"// (\d+) of the 1890 amplitude terms", text).group(1))
        puts += [int(x) for x in re.findall(r"sink\.put\((\d+),", text)]
    assert nterms == 1890
    assert sorted(puts) == list(range(info["nslot"]))
    main = open(os.path.join(procs, "ggttggg.h")).read()
    # the gather loads slot s into a temporary s<s> (col[s * stride]) and sums temporaries per flow
    loads = {int(a): int(b) for a, b in re.findall(r"const auto s(\d+) = col\[(\d+) \* stride\];", main)}
    assert all(a == b for a, b in loads.items())
    assert sorted(loads) == list(range(info["nslot"]))
    gathered = {}
    for flow, rhs in re.findall(r"jamp\[(\d+)\] = (cast<T>\(s.*);", main):
        gathered[int(flow)] = [int(x) for x in re.findall(r"cast<T>\(s(\d+)\)", rhs)]
    assert sorted(gathered) == list(range(120))
    assert sorted(x for v in gathered.values() for x in v) == list(range(info["nslot"]))


def test_generated_pieces_on_host_match_oracle(hostlib7, card):
    """g g -> t tbar g g g evaluated piece by piece (as the GPU does through its workspace) on the host."""
    dp = ctypes.POINTER(ctypes.c_double)
    p = np.ascontiguousarray(configs.WORKLOADS["ggttggg"].momenta(6))
    ref = oracle.me2(configs.GGTTGGG, p, card)
    for prec, tol in ((0, 1e-13), (1, 1e-5)):
        out = np.empty(len(p))
        assert hostlib7.hostcheck7_me2(prec, card.ctypes.data_as(dp), 0.118, len(p), p.ctypes.data_as(dp),
                                       out.ctypes.data_as(dp)) == 0
        assert np.abs(out / ref - 1).max() <= tol, prec


def test_generation_does_not_depend_on_hash_seed():
    """The generated code is a function of the process alone (no set-iteration order leaks in)."""
    import sys
    code = ("import sys, hashlib; sys.path.insert(0, %r)\n"
            "from paper_2507_21039_amd.gen import diagrams, emit\n"
            "from paper_2507_21039_amd.gen.__main__ import PROCESSES\n"
            "g = diagrams.build_graph(2)\n"
            "h, info = emit.emit_qcd('P', g, 'x', **PROCESSES['ggttgg']['opts'])\n"
            "h2, _ = emit.emit_qcd('P', g, 'x', order=(None, {'cache': 20, 'flow_cost': 50.0}), chunks=4)\n"
            "print(hashlib.sha256((h + h2).encode()).hexdigest())\n") % os.path.join(HERE, "..")
    outs = []
    for seed in ("1", "2"):
        env = dict(os.environ, PYTHONHASHSEED=seed)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                                   check=True).stdout)
    assert outs[0] == outs[1]


@pytest.mark.parametrize("proc,key,npar", [(0, "eemumu", 4), (1, "ggtt", 4), (2, "ggttg", 5), (3, "ggttgg", 6),
                                           (5, "uuee", 4), (6, "uueeg", 5), (7, "uueegg", 6)])
def test_generated_helicities_match_oracle_helicity_basis(hostlib, card, proc, key, npar):
    """Each helicity's |M_h|^2 of the generated code equals the oracle's physical-helicity value
    (index bit npar-1-k set for helicity +1 of particle k): helicity labels, not just their sum."""
    dp = ctypes.POINTER(ctypes.c_double)
    p = np.ascontiguousarray(configs.WORKLOADS[key].momenta(4))
    nhel = 1 << npar
    out, per_hel = np.empty(len(p)), np.empty(len(p) * nhel)
    assert hostlib.hostcheck_me2(proc, 0, card.ctypes.data_as(dp), 0.118, len(p), p.ctypes.data_as(dp),
                                 out.ctypes.data_as(dp), per_hel.ctypes.data_as(dp)) == 0
    per_hel = per_hel.reshape(len(p), nhel)
    for e in range(len(p)):
        ref = oracle.me2_hel(proc, p[e], card, 0.118)
        assert np.abs(per_hel[e] - ref).max() <= 1e-13 * ref.sum()


@pytest.mark.parametrize("proc,key,npar", [(1, "ggtt", 4), (2, "ggttg", 5), (3, "ggttgg", 6)])
def test_generated_flows_match_oracle_orderings(hostlib, card, proc, key, npar):
    """Jamp c of the generated code is the oracle's colour-ordered amplitude for the c-th
    lexicographic ordering of the gluons, up to one factor common to all flows."""
    dp = ctypes.POINTER(ctypes.c_double)
    ncol = math.factorial(npar - 2)
    p = np.ascontiguousarray(configs.WORKLOADS[key].momenta(2)[1])
    pairs = []
    for h in range(1 << npar):
        out = np.empty(2 * ncol)
        assert hostlib.hostcheck_jamps(proc, card.ctypes.data_as(dp), p.ctypes.data_as(dp), h,
                                       out.ctypes.data_as(dp)) == 0
        A = oracle.partial_amps_hel(p, card, [(h >> (npar - 1 - k)) & 1 for k in range(npar)])
        pairs.append((out[0::2] + 1j * out[1::2], A))
    top = max(np.abs(A).max() for _, A in pairs)
    checked = 0
    for J, A in pairs:
        big = np.abs(A) > 1e-6 * top  # vanishing helicities hold rounding noise only
        if not big.any():
            continue
        ratio = np.abs(J[big]) ** 2 / np.abs(A[big]) ** 2
        assert np.abs(ratio / ratio[0] - 1).max() <= 1e-9
        checked += 1
    assert checked >= (1 << npar) // 2


def test_compensated_helpers_are_not_contracted_on_the_device(tmp_path):
    """The double-double helpers keep their error-free transformations in device code: compiled
    for gfx950, none of their multiplies or adds may be fused into a multiply-add (a product
    rounded once inside a later sum, e.g. round(a^2) + b turned into fma(a, a, b))."""
    if not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not available")
    src = os.path.join(HERE, "devicecheck", "dd_contract.hip")
    ll = tmp_path / "dd.ll"
    subprocess.run(["/opt/rocm/bin/hipcc", "-O3", "-std=c++17", "--offload-arch=gfx950", "--cuda-device-only",
                    "-S", "-emit-llvm", src, "-o", str(ll)], check=True, capture_output=True)
    body = ll.read_text()
    assert "@llvm.fma.f64" in body  # the exact products are there
    import re
    # a fusion needs the add to allow contraction: no add or subtract in them may allow it
    flagged = re.findall(r"= (?:fadd|fsub) (?:[a-z]+ )*contract", body)
    assert not flagged, flagged[:4]


CHANNEL_CASES = [(1, "ggtt", 0, "tt"), (2, "ggttg", 1, "tt"), (3, "ggttgg", 2, "tt"), (5, "uuee", 0, "dy"),
                 (6, "uueeg", 1, "dy"), (7, "uueegg", 2, "dy"), (8, "uueeggg", 3, "dy")]


@pytest.mark.parametrize("proc,key,ng,family", CHANNEL_CASES)
def test_generated_channel_weights_match_oracle(hostlib, card, proc, key, ng, family):
    """Per-diagram sums over helicities and terms of |a|^2 of the generated code (its amplitude
    observer) against the oracle's diagram-by-diagram evaluation; diagrams matched by name."""
    dp = ctypes.POINTER(ctypes.c_double)
    hostlib.hostcheck_channels.argtypes = [ctypes.c_int, dp, ctypes.c_int64, dp, dp]
    p = np.ascontiguousarray(configs.WORKLOADS[key].momenta(3, first_event=40))
    gkeys = diagrams.diagram_keys(ng, family)
    okeys = oracle.diagram_keys(proc)
    assert sorted(gkeys) == sorted(okeys)
    got = np.empty((len(p), len(gkeys)))
    assert hostlib.hostcheck_channels(proc, card.ctypes.data_as(dp), len(p), p.ctypes.data_as(dp),
                                      got.ctypes.data_as(dp)) == 0
    want = oracle.channel_weights(proc, p, card)[:, [okeys.index(k) for k in gkeys]]
    assert np.abs(got / want - 1).max() <= 1e-12


@pytest.mark.parametrize("proc,key,n", [(2, "ggttg", 2000), (3, "ggttgg", 300)])
def test_feynman_diagram_gauge_on_host(hostlib, card, proc, key, n):
    """The generated code in the Feynman-diagram gauge (internal gluon propagators with the light-like
    gauge vector n = (sign Q0, -Q/|Q|)) equals the oracle, which works in the Feynman gauge: |M|^2 is
    gauge invariant, so a mistake in the gauge terms shows as a difference.  Double precision within
    2e-14 of the long double oracle; single precision within 1e-5."""
    p = configs.WORKLOADS[key].momenta(n, first_event=300)
    ld = oracle.me2(proc, p, card, extended=True)
    fd64 = host_me2(hostlib, 100 + proc, 0, p, card)
    fd32 = host_me2(hostlib, 100 + proc, 1, p, card)
    assert np.abs(fd64 / ld - 1).max() <= 2e-14
    assert np.abs(fd32 / ld - 1).max() <= 1e-5
