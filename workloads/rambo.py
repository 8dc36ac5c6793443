"""Flat n-body phase space (RAMBO) with per-event counter-based randomness.

Algorithm: R. Kleiss, W. J. Stirling, S. D. Ellis, "A new Monte Carlo treatment
of multiparticle phase space at high energies", Comput. Phys. Commun. 40 (1986)
359: massless momenta from isotropic exponential energies, a conformal boost to
the centre-of-mass frame at the requested energy, then a common rescaling of the
three-momenta (solved by Newton iteration) to put massive particles on shell.

The paper's standalone harness samples its phase-space points this way (section
"Standalone application").  This module is an input generator only.

Event i draws its numbers from Philox counters (i_lo, i_hi, attempt, block), key
(seed, 0x52414D42).  When a cut rejects event i, that event alone moves on to
the next attempt, so every event is independent of batch size and order.
"""
from __future__ import annotations

import math

import numpy as np

from .philox import philox4x32, uniform_pairs

_KEY1 = 0x52414D42  # "RAMB"


def _uniforms(seed: int, event_idx: np.ndarray, attempt: np.ndarray, nblocks: int):
    """Return uniforms of shape [len(event_idx), 2 * nblocks] in (0, 1)."""
    ev = event_idx.astype(np.uint64)
    lo = (ev & np.uint64(0xFFFFFFFF)).astype(np.uint32)[:, None]
    hi = (ev >> np.uint64(32)).astype(np.uint32)[:, None]
    att = attempt.astype(np.uint32)[:, None]
    blk = np.arange(nblocks, dtype=np.uint32)[None, :]
    words = philox4x32((lo, hi, att, blk), (np.uint32(seed & 0xFFFFFFFF), np.uint32(_KEY1)))
    u0, u1 = uniform_pairs(words)
    out = np.empty((len(event_idx), 2 * nblocks), dtype=np.float64)
    out[:, 0::2] = u0
    out[:, 1::2] = u1
    return out


def rambo_massless(u: np.ndarray, sqrt_s: float, nout: int) -> np.ndarray:
    """Massless RAMBO for a batch.  u: [nevt, 4*nout] uniforms.  Returns [nevt, nout, 4].

    The arithmetic runs in extended precision (numpy longdouble): the conformal
    boost cancels large terms when the isotropic momenta are nearly collinear,
    and the extra bits keep the returned momenta on shell and conserving to
    double rounding.
    """
    nevt = u.shape[0]
    u = np.asarray(u, dtype=np.longdouble).reshape(nevt, nout, 4)
    c = 2.0 * u[..., 0] - 1.0
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    f = 8.0 * np.arctan(np.longdouble(1.0)) * u[..., 1]
    q0 = -np.log(u[..., 2] * u[..., 3])
    q = np.stack([q0, q0 * s * np.cos(f), q0 * s * np.sin(f), q0 * c], axis=-1)
    Q = q.sum(axis=1)  # [nevt, 4]
    M = np.sqrt(Q[:, 0] ** 2 - Q[:, 1] ** 2 - Q[:, 2] ** 2 - Q[:, 3] ** 2)
    b = -Q[:, 1:] / M[:, None]
    x = np.longdouble(sqrt_s) / M
    gamma = Q[:, 0] / M
    a = 1.0 / (1.0 + gamma)
    bq = np.einsum("ek,enk->en", b, q[..., 1:])
    p = np.empty_like(q)
    p[..., 0] = x[:, None] * (gamma[:, None] * q[..., 0] + bq)
    p[..., 1:] = x[:, None, None] * (
        q[..., 1:] + b[:, None, :] * q[..., 0:1] + (a[:, None] * bq)[..., None] * b[:, None, :]
    )
    return p


def massless_volume(n: int, s: float) -> float:
    """Volume of massless n-body phase space at invariant mass squared s (the RAMBO paper):
    (2 pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!), with (2 pi)^4 delta^4 and
    d^3p / ((2 pi)^3 2E) per particle in the measure."""
    return ((2 * math.pi) ** (4 - 3 * n) * (math.pi / 2) ** (n - 1) * s ** (n - 2)
            / (math.factorial(n - 1) * math.factorial(n - 2)))


def put_on_shell(p: np.ndarray, masses, sqrt_s: float, with_weight: bool = False):
    """Rescale massless momenta [nevt, nout, 4] so that particle j has mass masses[j].

    Solves sum_j sqrt(m_j^2 + xi^2 E_j^2) = sqrt_s for xi by Newton iteration
    to extended-precision rounding, then k_j = (sqrt(m_j^2 + xi^2 E_j^2), xi * p_j).
    With with_weight, also returns the phase-space weight of each point: the massless
    volume times xi^(2n-3) prod_j |k_j| / k_j^0 * sqrt_s / sum_j |k_j|^2 / k_j^0.
    """
    m = np.asarray(masses, dtype=np.longdouble)[None, :]
    p = np.asarray(p, dtype=np.longdouble)
    n = p.shape[1]
    if np.sum(m) >= sqrt_s:
        raise ValueError("sum of final-state masses exceeds sqrt(s)")
    P2 = p[..., 1] ** 2 + p[..., 2] ** 2 + p[..., 3] ** 2
    w0 = massless_volume(n, sqrt_s * sqrt_s)
    if not np.any(m > 0):
        k = p.copy()
        k[..., 0] = np.sqrt(P2)
        k = k.astype(np.float64)
        return (k, np.full(p.shape[0], w0)) if with_weight else k
    E = np.sqrt(P2)
    xi = np.full(p.shape[0], np.sqrt(max(0.0, 1.0 - float(np.sum(m) / sqrt_s) ** 2)), dtype=np.longdouble)
    for _ in range(200):
        e = np.sqrt(m * m + (xi[:, None] * E) ** 2)
        f = e.sum(axis=1) - sqrt_s
        df = (xi[:, None] * E * E / e).sum(axis=1)
        step = f / df
        xi = xi - step
        if np.all(np.abs(step) <= 1e-17 * np.abs(xi)):
            break
    k = np.empty_like(p)
    k[..., 1:] = xi[:, None, None] * p[..., 1:]
    k[..., 0] = np.sqrt(m * m + (xi * xi)[:, None] * P2)
    if not with_weight:
        return k.astype(np.float64)
    kabs = xi[:, None] * E
    w = (w0 * xi ** (2 * n - 3) * np.prod(kabs / k[..., 0], axis=1) * sqrt_s
         / np.sum(kabs * kabs / k[..., 0], axis=1))
    return k.astype(np.float64), w.astype(np.float64)


def pseudorapidity(p: np.ndarray) -> np.ndarray:
    pt2 = p[..., 1] ** 2 + p[..., 2] ** 2
    P = np.sqrt(pt2 + p[..., 3] ** 2)
    # eta = 1/2 ln((P + pz)/(P - pz)); rewrite the small side to avoid cancellation
    plus = np.where(p[..., 3] >= 0, P + p[..., 3], pt2 / np.maximum(P - p[..., 3], 1e-300))
    minus = np.where(p[..., 3] >= 0, pt2 / np.maximum(P + p[..., 3], 1e-300), P - p[..., 3])
    return 0.5 * np.log(plus / minus)


def delta_r(pa: np.ndarray, pb: np.ndarray) -> np.ndarray:
    deta = pseudorapidity(pa) - pseudorapidity(pb)
    dphi = np.abs(np.arctan2(pa[..., 2], pa[..., 1]) - np.arctan2(pb[..., 2], pb[..., 1]))
    dphi = np.where(dphi > np.pi, 2.0 * np.pi - dphi, dphi)
    return np.sqrt(deta * deta + dphi * dphi)


def generate(nevt: int, sqrt_s: float, in_masses, out_masses, seed: int, cut=None,
             first_event: int = 0, max_attempts: int = 10000, retry: bool = True,
             with_weight: bool = False):
    """Generate events [nevt, nin + nout, 4] (E, px, py, pz) in GeV.

    The two incoming partons are massless and collide along the z axis at
    sqrt_s / 2 each: parton 1 moves along +z, parton 2 along -z.
    ``cut`` maps final-state momenta [n, nout, 4] to a boolean mask of accepted
    events.  Event numbers run from ``first_event``.  With ``retry`` False every
    event keeps its first attempt and a rejected one gets weight 0.  With
    ``with_weight`` returns (momenta, phase-space weights [nevt]).
    """
    if any(m != 0 for m in in_masses):
        raise ValueError("only massless incoming partons are supported")
    nout = len(out_masses)
    nin = len(in_masses)
    ev_idx = np.arange(first_event, first_event + nevt, dtype=np.int64)
    out = np.empty((nevt, nin + nout, 4), dtype=np.float64)
    wgt = np.empty(nevt, dtype=np.float64)
    half = 0.5 * sqrt_s
    out[:, 0] = (half, 0.0, 0.0, half)
    out[:, 1] = (half, 0.0, 0.0, -half)
    todo = np.arange(nevt)
    attempt = np.zeros(nevt, dtype=np.int64)
    nblocks = 2 * nout  # 4 uniforms per particle, 2 uniforms per Philox call
    while todo.size:
        u = _uniforms(seed, ev_idx[todo], attempt[todo], nblocks)
        p, w = put_on_shell(rambo_massless(u, sqrt_s, nout), out_masses, sqrt_s, with_weight=True)
        ok = np.ones(todo.size, dtype=bool) if cut is None else np.asarray(cut(p), dtype=bool)
        if not retry:
            out[todo, nin:] = p
            wgt[todo] = np.where(ok, w, 0.0)
            break
        out[todo[ok], nin:] = p[ok]
        wgt[todo[ok]] = w[ok]
        attempt[todo[~ok]] += 1
        todo = todo[~ok]
        if todo.size and attempt[todo].min() >= max_attempts:
            raise RuntimeError("cut acceptance too low")
    return (out, wgt) if with_weight else out


def acceptance(nevt: int, sqrt_s: float, out_masses, seed: int, cut) -> float:
    """Fraction of first-attempt RAMBO points that pass ``cut`` (for reports)."""
    u = _uniforms(seed, np.arange(nevt, dtype=np.int64), np.zeros(nevt, dtype=np.int64),
                  2 * len(out_masses))
    p = put_on_shell(rambo_massless(u, sqrt_s, len(out_masses)), out_masses, sqrt_s)
    return float(np.mean(cut(p)))
