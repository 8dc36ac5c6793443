"""Test infrastructure: the FP64 CPU oracle for |M|^2 (and its checks).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It shares no code with the GPU library and never imports it.

The C++ source `oracle.cpp` is compiled with the host compiler into
`liboracle.so` next to it (``build()``); loading builds it when it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

EEMUMU, GGTT, GGTTG, GGTTGG, GGTTGGG = 0, 1, 2, 3, 4
UUEE, UUEEG, UUEEGG, UUEEGGG = 5, 6, 7, 8  # u ubar -> e+ e- + n g (Drell-Yan family)
GGGG = 9  # g g -> g g, test only
NPAR = {EEMUMU: 4, GGTT: 4, GGTTG: 5, GGTTGG: 6, GGTTGGG: 7, UUEE: 4, UUEEG: 5, UUEEGG: 6, UUEEGGG: 7, GGGG: 4}
DY = (UUEE, UUEEG, UUEEGG, UUEEGGG)
ORDERED, DRESSED = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, OpenMP, no FMA contraction)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", _LIB + ".tmp", _SRC]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            ip = ctypes.POINTER(ctypes.c_int)
            for name in ("oracle_me2", "oracle_me2_ld"):
                f = getattr(L, name)
                f.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_int64, dp, dp, ctypes.c_int, ctypes.c_int]
                f.restype = ctypes.c_int
            L.oracle_colour_matrix.argtypes = [ctypes.c_int, dp]
            L.oracle_partial_amps.argtypes = [ctypes.c_int, dp, dp, ip, ctypes.c_int, dp]
            L.oracle_partial_amps_hel.argtypes = [ctypes.c_int, dp, dp, ip, dp]
            L.oracle_me2_hel.argtypes = [ctypes.c_int, dp, ctypes.c_double, dp, dp]
            L.oracle_dressed_amp.argtypes = [ctypes.c_int, dp, dp, ip, ip, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int, dp]
            L.oracle_partial_amps_dy.argtypes = [ctypes.c_int, dp, dp, ip, ctypes.c_int, ctypes.c_int, dp]
            L.oracle_dressed_amp_dy.argtypes = [ctypes.c_int, dp, dp, ip, ip, ctypes.c_int, ctypes.c_int,
                                                ctypes.c_int, dp]
            L.oracle_diagram_keys.argtypes = [ctypes.c_int, ctypes.c_char_p, ctypes.c_int]
            L.oracle_channel_weights.argtypes = [ctypes.c_int, dp, ctypes.c_int64, dp, dp, ctypes.c_int]
            L.oracle_diagram_sum.argtypes = [ctypes.c_int, dp, dp, ip, ip, ctypes.c_int, ctypes.c_int, dp]
            L.oracle_external.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_int, dp]
            L.oracle_gamma.argtypes = [ctypes.c_int, dp]
            L.oracle_su3.argtypes = [dp, dp]
            L.oracle_ew.argtypes = [dp, dp]
            L.oracle_iden.argtypes = [ctypes.c_int, dp]
            _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


def me2(process: int, momenta, card, alpha_s: float = 0.118, mode: int = ORDERED,
        nthreads: int | None = None, extended: bool = False) -> np.ndarray:
    """|M|^2 averaged over initial spins/colours and divided by the final-state symmetry factor."""
    mom = np.ascontiguousarray(momenta, dtype=np.float64)
    if mom.ndim != 3 or mom.shape[1] != NPAR[process] or mom.shape[2] != 4:
        raise ValueError(f"momenta must be [nevt, {NPAR[process]}, 4]")
    card = np.ascontiguousarray(card, dtype=np.float64)
    out = np.empty(mom.shape[0], dtype=np.float64)
    f = lib().oracle_me2_ld if extended else lib().oracle_me2
    rc = f(process, _dp(card), float(alpha_s), mom.shape[0], _dp(mom), _dp(out), mode,
           nthreads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle_me2 failed with {rc}")
    return out


def colour_matrix(n: int) -> np.ndarray:
    import math
    k = math.factorial(n)
    out = np.empty(k * k, dtype=np.float64)
    if lib().oracle_colour_matrix(n, _dp(out)) != 0:
        raise ValueError("bad n")
    return out.reshape(k, k)


def partial_amps(momentum, card, spins, gauge_leg: int = -1) -> np.ndarray:
    import math
    mom = np.ascontiguousarray(momentum, dtype=np.float64)
    npar = mom.shape[0]
    card = np.ascontiguousarray(card, dtype=np.float64)
    sp = np.ascontiguousarray(spins, dtype=np.int32)
    out = np.empty(2 * math.factorial(npar - 2), dtype=np.float64)
    if lib().oracle_partial_amps(npar, _dp(card), _dp(mom), _ip(sp), gauge_leg, _dp(out)) != 0:
        raise ValueError("bad arguments")
    return out[0::2] + 1j * out[1::2]


def me2_hel(process: int, momentum, card, alpha_s: float = 0.118) -> np.ndarray:
    """|M_h|^2 of every helicity configuration of one event (physical helicities), normalised so
    that they sum to me2; index h has bit npar-1-k set when particle k has helicity +1."""
    mom = np.ascontiguousarray(momentum, dtype=np.float64)
    card = np.ascontiguousarray(card, dtype=np.float64)
    out = np.empty(1 << NPAR[process], dtype=np.float64)
    if mom.shape != (NPAR[process], 4) or lib().oracle_me2_hel(process, _dp(card), float(alpha_s), _dp(mom),
                                                               _dp(out)) != 0:
        raise ValueError("bad arguments")
    return out


def partial_amps_hel(momentum, card, spins) -> np.ndarray:
    """Colour-ordered partial amplitudes (g_s = 1) for physical helicities spins[k] in {0: -1, 1: +1}."""
    import math
    mom = np.ascontiguousarray(momentum, dtype=np.float64)
    card = np.ascontiguousarray(card, dtype=np.float64)
    sp = np.ascontiguousarray(spins, dtype=np.int32)
    out = np.empty(2 * math.factorial(mom.shape[0] - 2), dtype=np.float64)
    if lib().oracle_partial_amps_hel(mom.shape[0], _dp(card), _dp(mom), _ip(sp), _dp(out)) != 0:
        raise ValueError("bad arguments")
    return out[0::2] + 1j * out[1::2]


def dressed_amp(momentum, card, spins, colours, i3: int = 0, j4: int = 0, gauge_leg: int = -1,
                pure_gluon: bool = False) -> complex:
    mom = np.ascontiguousarray(momentum, dtype=np.float64)
    card = np.ascontiguousarray(card, dtype=np.float64)
    sp = np.ascontiguousarray(spins, dtype=np.int32)
    col = np.ascontiguousarray(colours, dtype=np.int32)
    out = np.empty(2, dtype=np.float64)
    if lib().oracle_dressed_amp(mom.shape[0], _dp(card), _dp(mom), _ip(sp), _ip(col), i3, j4, gauge_leg,
                                int(pure_gluon), _dp(out)) != 0:
        raise ValueError("bad arguments")
    return complex(out[0], out[1])


def partial_amps_dy(momentum, card, spins, gauge_leg: int = -1, helicity_basis: bool = False) -> np.ndarray:
    """Colour-ordered partial amplitudes (g_s = 1) of u ubar -> e+ e- + n g for one event and one spin
    configuration (spins[k] in {0, 1}; gluons linear e1 / e2, or helicity -1 / +1 with
    helicity_basis), the n! gluon orderings in lexicographic order."""
    import math
    mom = np.ascontiguousarray(momentum, dtype=np.float64)
    npar = mom.shape[0]
    card = np.ascontiguousarray(card, dtype=np.float64)
    sp = np.ascontiguousarray(spins, dtype=np.int32)
    out = np.empty(2 * math.factorial(npar - 4), dtype=np.float64)
    if lib().oracle_partial_amps_dy(npar, _dp(card), _dp(mom), _ip(sp), gauge_leg, int(helicity_basis),
                                    _dp(out)) != 0:
        raise ValueError("bad arguments")
    return out[0::2] + 1j * out[1::2]


def dressed_amp_dy(momentum, card, spins, colours, i1: int = 0, j2: int = 0, gauge_leg: int = -1) -> complex:
    """Colour-dressed amplitude (g_s = 1) of u ubar -> e+ e- + n g: gluon colours (0..7), u colour i1,
    ubar colour j2 (0..2), linear gluon polarisations."""
    mom = np.ascontiguousarray(momentum, dtype=np.float64)
    card = np.ascontiguousarray(card, dtype=np.float64)
    sp = np.ascontiguousarray(spins, dtype=np.int32)
    col = np.ascontiguousarray(list(colours) if len(colours) else [0], dtype=np.int32)
    out = np.empty(2, dtype=np.float64)
    if lib().oracle_dressed_amp_dy(mom.shape[0], _dp(card), _dp(mom), _ip(sp), _ip(col), i1, j2, gauge_leg,
                                   _dp(out)) != 0:
        raise ValueError("bad arguments")
    return complex(out[0], out[1])


def external(kind: int, p, m: float, lam: int) -> np.ndarray:
    """kind 0 u, 1 v, 2 ubar, 3 vbar (helicity lam = +-1); 4 linear polarisation lam in {0, 1}."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    out = np.empty(8, dtype=np.float64)
    if lib().oracle_external(kind, _dp(p), float(m), int(lam), _dp(out)) != 0:
        raise ValueError("bad kind")
    return out[0::2] + 1j * out[1::2]


def gamma(mu: int) -> np.ndarray:
    out = np.empty(32, dtype=np.float64)
    if lib().oracle_gamma(mu, _dp(out)) != 0:
        raise ValueError("bad index")
    return (out[0::2] + 1j * out[1::2]).reshape(4, 4)


def su3():
    T = np.empty(8 * 9 * 2, dtype=np.float64)
    f = np.empty(512, dtype=np.float64)
    lib().oracle_su3(_dp(T), _dp(f))
    return (T[0::2] + 1j * T[1::2]).reshape(8, 3, 3), f.reshape(8, 8, 8)


def ew(card):
    card = np.ascontiguousarray(card, dtype=np.float64)
    out = np.empty(3, dtype=np.float64)
    lib().oracle_ew(_dp(card), _dp(out))
    return dict(sw2=out[0], cw2=out[1], e=out[2])


def iden(process: int) -> float:
    out = np.empty(1, dtype=np.float64)
    if lib().oracle_iden(process, _dp(out)) != 0:
        raise ValueError("bad process")
    return float(out[0])


GEV2_TO_PB = 0.3893793721e9  # (hbar c)^2 in GeV^2 pb


def cross_section(me2_values, weights, sqrt_s: float):
    """Flat Monte Carlo cross section and its statistical error, both in pb.

    sigma = (1 / (2 s)) (1 / N) sum_i w_i |M_i|^2: the flux factor of massless
    colliding partons times the mean over N phase-space points of weight times
    |M|^2 (points that fail the cuts count with weight 0), as the paper's
    standalone application integrates over flat phase space (section
    "Standalone application").  Summed in extended precision.
    """
    v = np.asarray(weights, dtype=np.longdouble) * np.asarray(me2_values, dtype=np.longdouble)
    n = v.size
    flux = 2.0 * sqrt_s * sqrt_s
    mean = v.sum() / n
    var = max((v * v).sum() / n - mean * mean, 0.0)
    return float(mean / flux * GEV2_TO_PB), float(np.sqrt(var / n) / flux * GEV2_TO_PB)


def diagram_keys(process: int) -> list:
    """Keys of the process's tree diagrams in the order of channel_weights (gluon g<particle>,
    three-gluon vertex (x,y), four-gluon vertex [x,y,z], electroweak boson W; elements of the
    quark line from its barred end, joined by ';')."""
    buf = ctypes.create_string_buffer(1 << 20)
    n = lib().oracle_diagram_keys(process, buf, len(buf))
    if n < 0:
        raise ValueError("no quark-line diagrams for this process")
    return buf.value.decode().split("\n")


def channel_weights(process: int, momenta, card, nthreads: int | None = None) -> np.ndarray:
    """Per event and diagram: sum over spins and over the diagram's terms of |value|^2 (colour
    stripped, g_s = 1), diagrams in the order of diagram_keys; [nevt, ndiag]."""
    mom = np.ascontiguousarray(momenta, dtype=np.float64)
    card = np.ascontiguousarray(card, dtype=np.float64)
    nd = len(diagram_keys(process))
    out = np.empty((mom.shape[0], nd), dtype=np.float64)
    if lib().oracle_channel_weights(process, _dp(card), mom.shape[0], _dp(mom), _dp(out),
                                    nthreads or default_threads()) != 0:
        raise ValueError("bad arguments")
    return out


def diagram_sum(process: int, momentum, card, spins, col, row: int, column: int) -> complex:
    """Sum over diagrams and terms of colour factor x value for explicit colours (equals the
    colour-dressed amplitude)."""
    mom = np.ascontiguousarray(momentum, dtype=np.float64)
    card = np.ascontiguousarray(card, dtype=np.float64)
    sp = np.ascontiguousarray(spins, dtype=np.int32)
    cl = np.ascontiguousarray(col if len(col) else [0], dtype=np.int32)
    out = np.empty(2)
    if lib().oracle_diagram_sum(process, _dp(card), _dp(mom), _ip(sp), _ip(cl), row, column, _dp(out)) != 0:
        raise ValueError("bad arguments")
    return complex(out[0], out[1])
