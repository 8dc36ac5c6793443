"""Emit one HIP header per process from the generated call graph.

Each header defines a struct with the process constants, a straight-line
`amplitudes<T>()` (external wavefunctions, off-shell currents with propagators,
amplitudes, jamp accumulation for one helicity) and `colour_sum<T>()` (the
quadratic form jamp^dagger C jamp with C's integer numerators).  T is the type
of the vertex/propagator arithmetic: double for the FP64 mode, float for the
mixed mode, in which the external wavefunctions and the propagator
denominators are still formed in double and cast.

The emitter also returns a static count of the real floating-point operations
per helicity (a complex multiply is 6, an add 2, a real-complex multiply 2),
used as the algorithmic FLOP figure of the kernel.
"""
from __future__ import annotations

import math

from . import colour as colour_mod
from .colour import Gauss
from .diagrams import ATOP, TOP

# real flops of each routine, counted from the formulas in helas.h
FLOPS = {
    "ffv_amp": 8 + 8 * 6 + 7 * 2,  # shorthands, 8 complex products, 7 complex adds
    "ffv_psi": 8 + 8 * 6 + 4 * 2 + 2 + 4 * (2 + 2 * 6 + 2 * 2 + 2 * 2) + 4 * 2,  # V-slash f, (K-slash+m), den
    "ffv_psibar": 8 + 8 * 6 + 4 * 2 + 2 + 4 * (2 + 2 * 6 + 2 * 2 + 2 * 2) + 4 * 2,
    "ffv_vec": 16 * 6 + 12 * 2 + 4 * 2,
    "vvv_amp": 12 + 3 * (4 * 6 + 3 * 2) + 3 * 8 + 3 * 6 + 2 * 2,  # momentum diffs, 3 dots c.c, 3 dots r.c, 3 cmul, 2 cadd
    "vvv_vec": 12 + (4 * 6 + 3 * 2) + 2 * 14 + 3 * 2 + 4 * (2 + 6 + 6 + 2 * 2),
    "vvvv_amp": 4 * (4 * 6 + 3 * 2) + 2 * 6 + 2,
    "vvvv_vec": 2 * (4 * 6 + 3 * 2) + 2 * 2 + 4 * (6 + 6 + 2),
}
EXT_FLOPS = {"vxxxxx": 20, "ixxxxx": 30, "oxxxxx": 30}  # includes sqrt/div as one each
DEN_FLOPS = 9  # momentum square (7) and the reciprocal of (Q^2 - m^2) (2)


def _word_index(basis):
    return {w: i for i, w in enumerate(basis)}


def _coef_code(c: Gauss, a: str) -> str:
    if (c.re, c.im) == (1, 0):
        return f"+ {a}"
    if (c.re, c.im) == (-1, 0):
        return f"- {a}"
    if (c.re, c.im) == (0, 1):
        return f"+ mul_i({a})"
    if (c.re, c.im) == (0, -1):
        return f"- mul_i({a})"
    return f"+ cx<T>{{T({c.re}), T({c.im})}} * {a}"


def _common_phase(amps):
    """If every coefficient is a unit times i, return -i (to multiply by) so they become real."""
    allim = all(c.re == 0 for a in amps for c in a.colour.terms.values())
    return Gauss(0, -1) if allim else Gauss(1, 0)


def emit_qcd(name: str, g, label: str) -> tuple[str, dict]:
    npar = g.npar
    gl = tuple(sorted(g.gluons))
    basis, C = colour_mod.colour_matrix(gl)
    N, D = colour_mod.integer_form(C)
    widx = _word_index(basis)
    ncol = len(basis)
    phase = _common_phase(g.amps)

    node_ids = {k: i for i, k in enumerate(g.nodes)}
    lines = []
    emitted = set()
    flops = 0
    masks_needed = {}

    def var(key):
        return f"w{node_ids[key]}"

    def mom(mask, sign=1):
        masks_needed[mask] = True
        return f"Q{mask}" if sign > 0 else f"mQ{mask}"

    def den_name(mask):
        return f"d{mask}"

    def emit_node(key):
        nonlocal flops
        if key in emitted:
            return
        n = g.nodes[key]
        for a in n.args:
            emit_node(a)
        v = var(key)
        if n.kind == "ext_v":
            k = key[1]
            nsv = -1 if k < 2 else 1
            lines.append(f"  const vw4<T> {v} = cast<T>(vxxxxx(p[{k}], hel({k}), {nsv}));")
            flops += EXT_FLOPS["vxxxxx"]
        elif n.kind == "ext_o":
            lines.append(f"  const sp4<T> {v} = cast<T>(oxxxxx(p[{TOP}], prm.mT, hel({TOP}), +1));")
            flops += EXT_FLOPS["oxxxxx"]
        elif n.kind == "ext_i":
            lines.append(f"  const sp4<T> {v} = cast<T>(ixxxxx(p[{ATOP}], prm.mT, hel({ATOP}), -1));")
            flops += EXT_FLOPS["ixxxxx"]
        elif n.kind == "vvv":
            a, b = n.args
            ma, mb = g.nodes[a].mask, g.nodes[b].mask
            lines.append(f"  const vw4<T> {v} = vvv_vec<T>({var(a)}, {mom(ma)}, {var(b)}, {mom(mb)}, "
                         f"{den_name(n.mask)});")
            masks_needed[n.mask] = True
            flops += FLOPS["vvv_vec"]
        elif n.kind == "vvvv":
            a, b, c = n.args
            s = n.extra[0]
            lines.append(f"  const vw4<T> {v} = vvvv_vec<{s}, T>({var(a)}, {var(b)}, {var(c)}, {den_name(n.mask)});")
            masks_needed[n.mask] = True
            flops += FLOPS["vvvv_vec"]
        elif n.kind == "psi":
            inner, t = n.args
            lines.append(f"  const sp4<T> {v} = ffv_psi<T>({var(inner)}, {var(t)}, {mom(n.mask)}, mT, "
                         f"{den_name(n.mask)});")
            flops += FLOPS["ffv_psi"]
        elif n.kind == "psibar":
            inner, t = n.args
            lines.append(f"  const sp4<T> {v} = ffv_psibar<T>({var(inner)}, {var(t)}, {mom(n.mask, -1)}, mT, "
                         f"{den_name(n.mask)});")
            flops += FLOPS["ffv_psibar"]
        elif n.kind == "qq":
            a, b = n.args
            lines.append(f"  const vw4<T> {v} = ffv_vec<T>({var(a)}, {var(b)}, {den_name(n.mask)});")
            masks_needed[n.mask] = True
            flops += FLOPS["ffv_vec"]
        else:
            raise ValueError(n.kind)
        emitted.add(key)

    jamp_terms = 0
    from .diagrams import schedule
    for ia in schedule(g):
        amp = g.amps[ia]
        for k in amp.args:
            emit_node(k)
        if amp.kind == "ffv":
            fb, f, t = amp.args
            call = f"ffv_amp<T>({var(fb)}, {var(f)}, {var(t)})"
            flops += FLOPS["ffv_amp"]
        elif amp.kind == "vvv":
            a, b, q = amp.args
            call = (f"vvv_amp<T>({var(a)}, {mom(g.nodes[a].mask)}, {var(b)}, {mom(g.nodes[b].mask)}, "
                    f"{var(q)}, {mom(g.nodes[q].mask)})")
            flops += FLOPS["vvv_amp"]
        else:
            a, b, c, q = amp.args
            call = f"vvvv_amp<{amp.extra[0]}, T>({var(a)}, {var(b)}, {var(c)}, {var(q)})"
            flops += FLOPS["vvvv_amp"]
        lines.append(f"  {{  // diagram {amp.diagram + 1}")
        lines.append(f"    const cx<T> a = {call};")
        for w, c in sorted(amp.colour.terms.items(), key=lambda x: widx[x[0]]):
            cc = c * phase
            j = widx[w]
            lines.append(f"    jamp[{j}] = jamp[{j}] {_coef_code(cc, 'a')};")
            jamp_terms += 1
        lines.append("  }")
    flops += 2 * jamp_terms

    # momenta and denominators used above
    pre = []
    for k in range(npar):
        sgn = "" if k < 2 else "-"
        pre.append(f"  const T q{1 << k}[4] = {{{sgn}T(p[{k}][0]), {sgn}T(p[{k}][1]), {sgn}T(p[{k}][2]), "
                   f"{sgn}T(p[{k}][3])}};")
    # masks are bit sets over particles; build sums in increasing popcount
    needed = set(masks_needed)
    # closure: every mask's momentum from lowest bit + rest
    allm = set()

    def need(m):
        if m in allm or m == 0:
            return
        allm.add(m)
        low = m & -m
        if m != low:
            need(low)
            need(m ^ low)

    for m in needed:
        need(m)
    mom_lines = []
    for m in sorted(allm, key=lambda x: (bin(x).count("1"), x)):
        if m & (m - 1) == 0:
            if m != 0:
                mom_lines.append(f"  const T* Q{m} = q{m};")
            continue
        low = m & -m
        mom_lines.append(f"  const T Q{m}[4] = {{Q{low}[0] + Q{m ^ low}[0], Q{low}[1] + Q{m ^ low}[1], "
                         f"Q{low}[2] + Q{m ^ low}[2], Q{low}[3] + Q{m ^ low}[3]}};")
    # negated momenta for barred currents, denominators
    den_lines = []
    for m in sorted(needed):
        node_kinds = {n.kind for n in g.nodes.values() if n.mask == m}
        fermion = bool(node_kinds & {"psi", "psibar"})
        if fermion:
            if "psibar" in node_kinds:
                den_lines.append(f"  const T mQ{m}[4] = {{-Q{m}[0], -Q{m}[1], -Q{m}[2], -Q{m}[3]}};")
            den_lines.append(f"  const T d{m} = T(1.0 / (sq(p, {m}) - prm.mT * prm.mT));")
        elif any(n.kind in ("vvv", "vvvv", "qq") for n in g.nodes.values() if n.mask == m):
            den_lines.append(f"  const T d{m} = T(1.0 / sq(p, {m}));")
    nden = sum(1 for l in den_lines if " d" in l.split("=")[0])
    flops_den = DEN_FLOPS * nden

    # colour sum with symmetric integer numerators
    cs = []
    cs_flops = 0
    for i in range(ncol):
        terms = []
        for j in range(i, ncol):
            v = N[i][j] * (1 if i == j else 2)
            if v == 0:
                continue
            terms.append((j, v))
        if not terms:
            continue
        zr = " + ".join(f"T({v}) * jamp[{j}].r" for j, v in terms)
        zi = " + ".join(f"T({v}) * jamp[{j}].i" for j, v in terms)
        cs.append(f"  s += jamp[{i}].r * ({zr}) + jamp[{i}].i * ({zi});")
        cs_flops += 4 * len(terms) + 4
    hdr = f"""// Generated by paper_2507_21039_amd.gen for {label}.  Do not edit.
// {g.ndiag} Feynman diagrams, {len(g.amps)} amplitude terms (each four-gluon vertex split into its
// three structures), {len(g.nodes)} wavefunctions, {ncol} colour flows.
#pragma once
#include "../helas.h"
#include "../process.h"

namespace hme {{

struct {name} {{
  static constexpr int npar = {npar};
  static constexpr int nhel = {2 ** npar};
  static constexpr int ncol = {ncol};
  static constexpr int ndiag = {g.ndiag};
  static constexpr int namp = {len(g.amps)};
  static constexpr int gs_power = {2 * len(gl)};  // |M|^2 carries g_s^gs_power
  static constexpr double iden = {iden_qcd(len(gl) - 2)};  // spin and colour average, identical gluons
  static constexpr double colour_denom = {D};
  static constexpr double flops_per_hel = {flops + cs_flops};
  static constexpr double flops_per_event = {flops_den};  // helicity-independent part

  HME_FN static double sq(const double (&p)[{npar}][4], unsigned mask) {{
    double Q[4] = {{0, 0, 0, 0}};
    for (int k = 0; k < {npar}; ++k)
      if (mask >> k & 1)
        for (int mu = 0; mu < 4; ++mu) Q[mu] += (k < 2 ? p[k][mu] : -p[k][mu]);
    return Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3];
  }}

  // jamps of one helicity (jamp[] must be zeroed by the caller)
  template <class T>
  HME_FN static void amplitudes(const double (&p)[{npar}][4], const ProcParams& prm, unsigned h,
                                cx<T> (&jamp)[{ncol}]) {{
    auto hel = [h](int k) {{ return (h >> ({npar - 1} - k) & 1u) ? 1 : -1; }};
    const T mT = T(prm.mT);
""" + "\n".join(pre) + "\n" + "\n".join(mom_lines) + "\n" + "\n".join(den_lines) + "\n" + "\n".join(lines) + f"""
  }}

  // sum over colour flows of conj(jamp) C jamp times colour_denom
  template <class T> HME_FN static T colour_sum(const cx<T> (&jamp)[{ncol}]) {{
    T s = 0;
""" + "\n".join(cs) + """
    return s;
  }
};

}  // namespace hme
"""
    info = dict(name=name, npar=npar, ncol=ncol, ndiag=g.ndiag, namp=len(g.amps), nwf=len(g.nodes),
                flops_per_hel=flops + cs_flops, flops_colour=cs_flops, flops_den=flops_den, colour_denom=D,
                numerators=N, jamp_terms=jamp_terms)
    return hdr, info


def iden_qcd(nfinal_gluons: int) -> float:
    return 4.0 * 64.0 * math.factorial(nfinal_gluons)


def emit_eemumu(name: str = "P_eemumu") -> tuple[str, dict]:
    """e+ e- -> mu+ mu- through a photon and a Z in the s channel (2 diagrams, 1 colour flow).

    Particles: 0 e+ (incoming, vbar), 1 e- (incoming, u), 2 mu+ (outgoing, v), 3 mu- (outgoing, ubar).
    Vertices -i e Q gamma^mu (Q = -1) and -i e/(sw cw) gamma^mu (gL P_L + gR P_R); propagators
    -i g/s and -i (g - q q / mZ^2) / (s - mZ^2 + i mZ wZ).  Both diagrams carry the same overall
    factor i, dropped here, leaving e^2 and e^2/(sw^2 cw^2) as the two couplings.
    """
    flops = (2 * EXT_FLOPS["oxxxxx"] + 2 * EXT_FLOPS["ixxxxx"] + FLOPS["ffv_vec"] + FLOPS["ffv_amp"]
             + (FLOPS["ffv_vec"] + 8 + 30) + (FLOPS["ffv_amp"] + 4) + 6 + 2 + 4)
    hdr = f"""// Generated by paper_2507_21039_amd.gen for e+ e- -> mu+ mu-.  Do not edit.
// 2 Feynman diagrams (photon and Z in the s channel), 1 colour flow.
#pragma once
#include "../helas.h"
#include "../process.h"

namespace hme {{

struct {name} {{
  static constexpr int npar = 4;
  static constexpr int nhel = 16;
  static constexpr int ncol = 1;
  static constexpr int ndiag = 2;
  static constexpr int namp = 2;
  static constexpr int gs_power = 0;
  static constexpr double iden = 4.0;  // average over the initial helicities
  static constexpr double colour_denom = 1.0;
  static constexpr double flops_per_hel = {flops};
  static constexpr double flops_per_event = 20.0;  // s, 1/s, Z propagator denominator

  template <class T>
  HME_FN static void amplitudes(const double (&p)[4][4], const ProcParams& prm, unsigned h, cx<T> (&jamp)[1]) {{
    auto hel = [h](int k) {{ return (h >> (3 - k) & 1u) ? 1 : -1; }};
    const sp4<T> w0 = cast<T>(oxxxxx(p[0], 0.0, hel(0), -1));  // vbar(e+)
    const sp4<T> w1 = cast<T>(ixxxxx(p[1], 0.0, hel(1), +1));  // u(e-)
    const sp4<T> w2 = cast<T>(ixxxxx(p[2], 0.0, hel(2), -1));  // v(mu+)
    const sp4<T> w3 = cast<T>(oxxxxx(p[3], 0.0, hel(3), +1));  // ubar(mu-)
    const double qd[4] = {{p[0][0] + p[1][0], p[0][1] + p[1][1], p[0][2] + p[1][2], p[0][3] + p[1][3]}};
    const double s = qd[0] * qd[0] - qd[1] * qd[1] - qd[2] * qd[2] - qd[3] * qd[3];
    const T q[4] = {{T(qd[0]), T(qd[1]), T(qd[2]), T(qd[3])}};
    // complex 1 / (s - mZ^2 + i mZ wZ)
    const double dr = s - prm.mZ * prm.mZ, di = prm.mZ * prm.wZ, dn = 1.0 / (dr * dr + di * di);
    const cx<T> dz = {{T(dr * dn), T(-di * dn)}};
    const vw4<T> ja = ffv_vec<T>(w0, w1, T(1.0 / s));
    const vw4<T> jz = ffvlr_vec_massive<T>(w0, w1, T(prm.gL), T(prm.gR), q, T(prm.mZ), dz);
    const cx<T> a = T(prm.cA) * ffv_amp<T>(w3, w2, ja) + T(prm.cZ) * ffvlr_amp<T>(w3, w2, jz, T(prm.gL), T(prm.gR));
    jamp[0] = jamp[0] + a;
  }}

  template <class T> HME_FN static T colour_sum(const cx<T> (&jamp)[1]) {{
    return jamp[0].r * jamp[0].r + jamp[0].i * jamp[0].i;
  }}
}};

}}  // namespace hme
"""
    info = dict(name=name, npar=4, ncol=1, ndiag=2, namp=2, nwf=6, flops_per_hel=flops, flops_colour=4,
                flops_den=20, colour_denom=1, numerators=[[1]], jamp_terms=1)
    return hdr, info
