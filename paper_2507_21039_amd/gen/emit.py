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
import re

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
# the momentum combinations and propagator factors of a vertex, read from the per-event table
FLOPS["vvv_vec_k"] = FLOPS["vvv_vec"] - 18
FLOPS["ffv_psi_k"] = FLOPS["ffv_psi"] - 10
FLOPS["ffv_psibar_k"] = FLOPS["ffv_psibar"] - 10
FLOPS["vvv_amp_k"] = FLOPS["vvv_amp"] - 12
# fermion vertices whose vector comes in light-cone form from the table: no shorthands (8); an
# external gluon's real vp = -vm also makes two complex products real ones (amplitude) or four
# (currents)
for _r in ("ffv_amp", "ffv_psi_k", "ffv_psibar_k"):
    FLOPS[_r + ":lc"] = FLOPS[_r] - 8
    FLOPS[_r + ":lcx"] = FLOPS[_r] - 8 - (8 if _r == "ffv_amp" else 16)
LC_KIT_FLOPS = 8  # light-cone form of an external gluon's kit (both helicities), per event
LC_REC_FLOPS = 8  # light-cone form of a recycled current (one helicity pair), per event
GATHER_GROUP = 24  # workspace loads written ahead of their use in the gather
VK_SIZE = {"vvv": 12, "psi": 5, "amp3": 12, "fd": 8}  # doubles per vertex kit
VK_FLOPS = {"vvv": 24, "psi": 7, "amp3": 12, "fd": 16}  # per event, in the table
FD_FLOPS = 2 * 14 + 4 * 2 * 4  # the gauge projection of a gluon current: two dots, four updates
EXT_FLOPS = {"vxxxxx": 20, "ixxxxx": 30, "oxxxxx": 30,  # includes sqrt/div as one each
             "ewkit": 2 * 30 + 120 + 40}  # lepton spinors, lepton current, photon + Z couplings
EW_ITEMS = 8  # electroweak current per (quark, e+, e-) helicity, 8 doubles each
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


def _closure(g, keys):
    out = set()
    stack = list(keys)
    while stack:
        k = stack.pop()
        if k in out or k[0] == "E":
            continue
        out.add(k)
        stack.extend(g.nodes[k].args)
    return out


NODE_FLOPS = {"vvv": "vvv_vec_k", "vvvv": "vvvv_vec", "psi": "ffv_psi_k", "psibar": "ffv_psibar_k", "qq": "ffv_vec"}
KIT_FLOPS = {"ext_v": 0, "ext_o": 0, "ext_i": 0, "ext_w": 0}  # a wavefunction is read from its per-event kit


UNIT = "@@UNIT@@"
_READ = re.compile(r"(qv<T>\(tab, \d+\)|dv<T>\(tab, [^)]*\)|load_kit<T, \d+>\(tab \+ [^)]*\)|"
                   r"(vxxxxx|oxxxxx|ixxxxx)_kit<T>\(tab \+ (\w+), hel\((\d+)\))")


def prefetch_units(lines, enable, kits: bool = True):
    """Split the body into units (one wavefunction or one amplitude term each).

    With enable, every table read of a unit (momentum sums, denominators and, with
    kits, the external-state kits) becomes a local loaded one unit earlier, fenced so
    the loads are issued before the previous unit's arithmetic.
    """
    units, cur = [], None
    for l in lines:
        if l == UNIT:
            cur = []
            units.append(cur)
        else:
            cur.append(l)
    if not enable:
        return [l for u in units for l in u]
    decls, bodies = [], []
    for k, u in enumerate(units):
        d = []
        seen = {}

        def repl(m):
            txt = m.group(0)
            if txt in seen:
                return seen[txt]
            nm = f"t{k}_{len(seen)}"
            if txt.startswith("qv"):
                d.append(f"  const m4<T> {nm} = {txt};")
                seen[txt] = nm
                return nm
            if txt.startswith("dv"):
                d.append(f"  const T {nm} = {txt};")
                seen[txt] = nm
                return nm
            if txt.startswith("load_kit"):
                n = txt.split("<T, ", 1)[1].split(">", 1)[0]
                d.append(f"  const kitv<T, {n}> {nm} = {txt};")
                seen[txt] = nm
                return nm
            kind, off, part = m.group(2), m.group(3), m.group(4)
            if not kits:
                return txt
            n = 5 if kind == "vxxxxx" else 8  # the half of the kit for the lane's helicity
            d.append(f"  const kitv<T, {n}> {nm} = load_kit<T, {n}>(tab + {off} + (hel({part}) > 0 ? 0 : {n}));")
            seen[txt] = f"{kind}_from<T>({nm}, hel({part})"
            return seen[txt]

        body = [_READ.sub(repl, l) for l in u]
        decls.append(d)
        bodies.append(body)
    out = decls[0] + ["  HME_FENCE();"] if units else []
    for k in range(len(units)):
        if k + 1 < len(units):
            out += decls[k + 1]
        out.append("  HME_FENCE();")
        out += bodies[k]
    return out


def emit_qcd(name: str, g, label: str, budget=(4, 12), prefetch=("", "all"), chunks: int = 0,
             file_stem: str = "", jbudget: int = 32, order=None, recycle: bool = False, gauge: str = "feynman"):
    """Emit the process header.

    budget: number of off-shell wavefunctions kept live at once, for the double and the
    single precision schedule.  When a schedule needs more, the wavefunction whose next
    use is farthest away is dropped and recomputed when needed again (Belady's rule).
    External wavefunctions are rebuilt at every use from a per-event kit in the LDS table.
    prefetch: per precision, "" (table reads at their use), "table" (momentum sums and
    denominators read one unit ahead) or "all" (kits too).  The defaults are the fastest
    measured on MI355X for g g -> t tbar g g: budget 4 without prefetch keeps the FP64
    kernel at 2 waves per SIMD; FP32 gains more from hiding LDS latency.
    order: the amplitude order, either one for both precisions or a pair (double, float); each
    is None (diagrams.schedule), a list of amplitude indices, or {"cache": n, "flow_cost": c}
    for diagrams.schedule_cached with that LRU model size and cost of a new partial jamp.
    chunks: if nonzero, cut the single-precision schedule into that many contiguous pieces,
    each emitted as its own struct (returned in info["chunk_headers"]) that adds its terms to
    the jamps of the flows it touches; the main header then holds the table and the colour
    sum only.  Used where one straight-line kernel would be too large to compile and to keep
    its jamps in registers.  jbudget: flows a piece accumulates in registers at once.
    recycle: helicity recycling.  A wavefunction built from two external states takes only 4
    values per event (one per helicity pair), so the event's lanes compute those once into the
    per-event table and every lane reads the one of its helicities instead of computing it.
    gauge: "feynman" (gluon propagator -i g/Q^2) or "fd", the Feynman-diagram gauge of Hagiwara,
    Kanzaki, Li, Mawatari and Nakamura (Eur. Phys. J. C 80 (2020) 584): every internal gluon
    current J becomes J - nt (Q.J) - Q (nt.J), nt = n / (n.Q), n = (sign Q0, -Q3vec / |Q3vec|),
    which removes the gauge cancellations between diagrams that cost digits in single precision.
    External gluons keep their helicity vectors (n.eps = 0 for them already).
    """
    fd = gauge == "fd"
    if isinstance(budget, int):
        budget = (budget, budget)
    if isinstance(prefetch, str):
        prefetch = (prefetch, prefetch)
    npar = g.npar
    gl = tuple(sorted(g.gluons))
    basis, C = colour_mod.colour_matrix(gl)
    N, D = colour_mod.integer_form(C)
    widx = _word_index(basis)
    ncol = len(basis)
    phase = _common_phase(g.amps)

    node_ids = {k: i for i, k in enumerate(g.nodes)}
    qidx = {}  # (mask, sign) -> index of a momentum sum in the table
    didx = {}  # mask -> (index, massive)

    def mom(mask, sign=1):
        key = (mask, sign)
        if key not in qidx:
            qidx[key] = len(qidx)
        return f"qv<T>(tab, {qidx[key]})"

    def den(mask, massive):
        if mask not in didx:
            didx[mask] = (len(didx), massive)
        return f"dv<T>(tab, DOFF + {didx[mask][0]})"

    vkidx = {}  # vertex-kit key -> offset in the vertex-kit region of the table
    vk_list = []  # (kind, mask0, mask1, mask2, sign, offset)
    vk_off = [0]

    def vkit(kind, m0, m1=0, m2=0, sign=1):
        key = (kind, m0, m1, m2, sign)
        if key not in vkidx:
            vkidx[key] = vk_off[0]
            vk_list.append((kind, m0, m1, m2, sign, vk_off[0]))
            vk_off[0] += VK_SIZE[kind]
        n = VK_SIZE[kind]
        return f"load_kit<T, {n}>(tab + VOFF + {vkidx[key]})"

    from .diagrams import schedule, schedule_cached
    node_cost = {kind: FLOPS[NODE_FLOPS[kind]] for kind in NODE_FLOPS}

    # recycled wavefunctions: two external arguments (gluons, quark ends), 4 helicity pairs each
    rec = {}  # node key -> index
    if recycle:
        for key, n in g.nodes.items():
            if key[0] != "E" and all(a[0] == "E" and g.nodes[a].kind in ("ext_v", "ext_o", "ext_i")
                                     for a in n.args) and len(n.args) == 2:
                rec[key] = len(rec)
    # the recycled currents (vectors) also keep their light-cone form, for the fermion vertices
    rec_lc = {key: i for i, key in enumerate(k for k in rec if g.nodes[k].kind in ("vvv", "qq"))}
    # recycled wavefunctions: kind (0 three-gluon current, 1 spinor current, 2 barred spinor
    # current, 3 quark pair), the particles of the two external arguments, and the offset of
    # the vertex kit (kinds 0-2, in the vertex-kit region) or the index of the denominator (3);
    # their kits are registered here, before the schedules
    rec_info = []
    for key in rec:
        n = g.nodes[key]
        pa, pb = (x[1] for x in n.args)
        if n.kind == "vvv":
            ma, mb = g.nodes[n.args[0]].mask, g.nodes[n.args[1]].mask
            vkit("vvv", ma, mb, n.mask)
            kk = vkidx[("vvv", ma, mb, n.mask, 1)]
        elif n.kind in ("psi", "psibar"):
            sg = 1 if n.kind == "psi" else -1
            vkit("psi", n.mask, sign=sg)
            kk = vkidx[("psi", n.mask, 0, 0, sg)]
        else:
            den(n.mask, False)
            kk = didx[n.mask][0]
        fk = 0
        if fd and n.kind in ("vvv", "qq"):
            vkit("fd", n.mask)
            fk = vkidx[("fd", n.mask, 0, 0, 1)]
        rec_info.append(({"vvv": 0, "psi": 1, "psibar": 2, "qq": 3}[n.kind], pa, pb, kk, fk, rec_lc.get(key, -1)))

    def pick_order(spec):
        if spec is None:
            return schedule(g)
        if isinstance(spec, dict):  # cache-aware schedule: LRU model size, cost of a new partial sum
            fc = spec.get("flow_cost", 0.0)
            return schedule_cached(g, node_cost, spec["cache"], jbudget if fc else 0, fc)
        return list(spec)

    if not (isinstance(order, tuple) and len(order) == 2 and all(x is None or isinstance(x, dict) for x in order)):
        order = (order, order)
    order_d, order_f = pick_order(order[0]), pick_order(order[1])
    full_order = order_f

    def emit_schedule(budget, order=None, wmap=None, jbudget=None, partials=None):
        """One amplitude schedule under a live-wavefunction budget; returns the body lines.

        order: the amplitude terms to evaluate (default: all, in schedule order);
        wmap: colour flow -> index into the jamp array (default: all flows in basis order).
        jbudget: if set, at most this many flows are accumulated in registers (jr[]); a flow
        leaves its register after its last term in `order`, or earlier when the register is
        needed (the flow whose next term is farthest away: Belady's rule, which gives the
        fewest partial sums), as a partial sum written by sink.put to a slot of its own;
        `partials` maps each flow to its slots and counts them ("n").
        """
        lines = []
        flops_exec = 0
        flops_dag = 0
        import bisect
        order = full_order if order is None else order
        wmap = widx if wmap is None else wmap
        amp_nodes = [_closure(g, g.amps[i].args) for i in order]
        uses = {}
        for t, s in enumerate(amp_nodes):
            for k in s:
                uses.setdefault(k, []).append(t)

        def next_use(k, t):
            u = uses[k]
            i = bisect.bisect_right(u, t)
            return u[i] if i < len(u) else 1 << 30

        live = {}  # node key -> variable name of its current value
        version = {}
        now = [0]
        computed_once = set()

        def ext_expr(key, out_lines, lc=False):
            """Build an external wavefunction from its kit into a fresh local, return the name."""
            nonlocal flops_exec
            k = key[1]
            kind = g.nodes[key].kind
            nm = f"e{k}_{len(out_lines)}"
            if kind == "ext_v" and lc:
                out_lines.append(f"    const vlcx<T> {nm} = vxxxxx_lc_kit<T>(tab + KLOFF{k}, hel({k}));")
            elif kind == "ext_w":
                out_lines.append(f"    const vw4<T> {nm} = ew_from_kit<T>(tab + KOFFW, hel(0), hel(2), hel(3));")
            elif kind == "ext_v":
                nsv = -1 if k < 2 else 1
                out_lines.append(f"    const vw4<T> {nm} = vxxxxx_kit<T>(tab + KOFF{k}, hel({k}), {nsv});")
            elif kind == "ext_o":
                out_lines.append(f"    const sp4<T> {nm} = oxxxxx_kit<T>(tab + KOFF{k}, hel({k}));")
            else:
                out_lines.append(f"    const sp4<T> {nm} = ixxxxx_kit<T>(tab + KOFF{k}, hel({k}));")
            flops_exec += KIT_FLOPS[kind]
            return nm

        def arg(key, pre, lc=False):
            """The expression of an argument; lc: the vector of a fermion vertex, taken in
            light-cone form where the table holds it (external gluons, recycled currents)."""
            if key[0] == "E":
                return ext_expr(key, pre, lc)
            if key in rec:  # the lane's helicity pair of a recycled wavefunction
                a, b = (k[1] for k in g.nodes[key].args)
                typ = "sp4" if g.nodes[key].kind in ("psi", "psibar") else "vw4"
                nm = f"r{rec[key]}_{len(pre)}"
                pair = f"(hel({a}) > 0 ? 16 : 0) + (hel({b}) > 0 ? 8 : 0)"
                if lc and typ == "vw4":
                    pre.append(f"    const vlc<T> {nm} = recycled_vlc<T>(tab + RLOFF + {32 * rec_lc[key]}, {pair});")
                else:
                    pre.append(f"    const {typ}<T> {nm} = recycled_{typ}<T>(tab + ROFF + {32 * rec[key]}, {pair});")
                return nm
            return live[key]

        def lc_form(key):
            """Which form a fermion vertex gets its vector in: ':lcx' (external gluon), ':lc'
            (recycled current) or '' (a current of this kernel, converted at the use)."""
            if key[0] == "E" and g.nodes[key].kind == "ext_v":
                return ":lcx"
            if key in rec and g.nodes[key].kind not in ("psi", "psibar"):
                return ":lc"
            return ""

        def need(key, pinned):
            nonlocal flops_exec, flops_dag
            if key[0] == "E" or key in live or key in rec:
                return
            n = g.nodes[key]
            for a in n.args:
                need(a, pinned | {key})
            pre = []
            fermion_vertex = n.kind in ("psi", "psibar")
            args = [arg(a, pre, lc=fermion_vertex and i == 1) for i, a in enumerate(n.args)]
            version[key] = version.get(key, -1) + 1
            v = f"w{node_ids[key]}" + (f"_{version[key]}" if version[key] else "")
            if n.kind == "vvv":
                ma, mb = g.nodes[n.args[0]].mask, g.nodes[n.args[1]].mask
                expr = f"vvv_vec_k<T>({args[0]}, {args[1]}, {vkit('vvv', ma, mb, n.mask)})"
                call = f"vw4<T> {v} = " + (f"fd_project<T>({expr}, {vkit('fd', n.mask)});" if fd else expr + ";")
            elif n.kind == "vvvv":
                expr = f"vvvv_vec<{n.extra[0]}, T>({args[0]}, {args[1]}, {args[2]}, {den(n.mask, False)})"
                call = f"vw4<T> {v} = " + (f"fd_project<T>({expr}, {vkit('fd', n.mask)});" if fd else expr + ";")
            elif n.kind == "psi":
                call = f"sp4<T> {v} = ffv_psi_k<T>({args[0]}, {args[1]}, {vkit('psi', n.mask)});"
            elif n.kind == "psibar":
                call = f"sp4<T> {v} = ffv_psibar_k<T>({args[0]}, {args[1]}, {vkit('psi', n.mask, sign=-1)});"
            elif n.kind == "qq":
                expr = f"ffv_vec<T>({args[0]}, {args[1]}, {den(n.mask, False)})"
                call = f"vw4<T> {v} = " + (f"fd_project<T>({expr}, {vkit('fd', n.mask)});" if fd else expr + ";")
            else:
                raise ValueError(n.kind)
            typ = call.split(" ", 1)[0]
            name_rest = call.split(" ", 1)[1]
            lines.append(UNIT)
            lines.append(f"  {typ} {v};")
            lines.append("  {")
            lines.extend(pre)
            lines.append(f"    {name_rest.replace(v + ' =', v + ' =', 1)}")
            lines.append("  }")
            f = (FLOPS[NODE_FLOPS[n.kind] + (lc_form(n.args[1]) if fermion_vertex else "")]
                 + (FD_FLOPS if fd and n.kind in ("vvv", "vvvv", "qq") else 0))
            flops_exec += f
            if key not in computed_once:
                flops_dag += f
                computed_once.add(key)
            live[key] = v
            while len(live) > budget:
                cands = [x for x in live if x not in pinned and x != key and x not in n.args]
                if not cands:
                    break
                victim = max(cands, key=lambda x: next_use(x, now[0]))
                del live[victim]

        jamp_terms = 0
        jslot = {}  # flow -> register slot (jamp budget mode)
        jfree = list(range(jbudget or 0))[::-1]
        wtouch = {}
        for t, ia in enumerate(order):
            for w in g.amps[ia].colour.terms:
                wtouch.setdefault(w, []).append(t)
        nflush = [0]

        def next_touch(w, t):
            u = wtouch[w]
            i = bisect.bisect_right(u, t)
            return u[i] if i < len(u) else 1 << 30

        def flush(w):
            slot = jslot.pop(w)
            jfree.append(slot)
            partials.setdefault(w, []).append(partials["n"])
            lines.append(f"    sink.put({partials['n']}, jr[{slot}]);")
            partials["n"] += 1
            nflush[0] += 1

        for t, ia in enumerate(order):
            now[0] = t
            amp = g.amps[ia]
            for k in amp.args:
                need(k, set(amp.args))
            pre = []
            args = [arg(k, pre, lc=amp.kind == "ffv" and i == 2) for i, k in enumerate(amp.args)]
            if amp.kind == "ffv":
                call = f"ffv_amp<T>({args[0]}, {args[1]}, {args[2]})"
                f = FLOPS["ffv_amp" + lc_form(amp.args[2])]
            elif amp.kind == "vvv":
                a, b, q = amp.args
                call = (f"vvv_amp_k<T>({args[0]}, {args[1]}, {args[2]}, "
                        f"{vkit('amp3', g.nodes[a].mask, g.nodes[b].mask, g.nodes[q].mask)})")
                f = FLOPS["vvv_amp_k"]
            else:
                call = f"vvvv_amp<{amp.extra[0]}, T>({args[0]}, {args[1]}, {args[2]}, {args[3]})"
                f = FLOPS["vvvv_amp"]
            flops_exec += f
            flops_dag += f
            lines.append(UNIT)
            lines.append(f"  {{  // diagram {amp.diagram + 1}")
            lines.extend(pre)
            lines.append(f"    const cx<T> a = {call};")
            if not jbudget:
                lines.append(f"    obs.term({amp.diagram}, a);")
            if jbudget:
                mine = set(amp.colour.terms)
                for w, c in sorted(amp.colour.terms.items(), key=lambda x: widx[x[0]]):
                    code = _coef_code(c * phase, 'a')
                    if w in jslot:
                        lines.append(f"    jr[{jslot[w]}] = jr[{jslot[w]}] {code};")
                    else:
                        if not jfree:
                            cands = [x for x in jslot if x not in mine]
                            flush(max(cands, key=lambda x: next_touch(x, t)))
                        jslot[w] = jfree.pop()
                        init = code[2:] if code.startswith("+ ") else "-" + code[2:]
                        lines.append(f"    jr[{jslot[w]}] = {init};")
                    jamp_terms += 1
                for w in sorted(jslot, key=lambda x: widx[x]):
                    if next_touch(w, t) >= 1 << 30:
                        flush(w)
            else:
                for w, c in sorted(amp.colour.terms.items(), key=lambda x: wmap[x[0]]):
                    j = wmap[w]
                    lines.append(f"    jamp[{j}] = jamp[{j}] {_coef_code(c * phase, 'a')};")
                    jamp_terms += 1
            lines.append("  }")
            for x in list(live):
                if next_use(x, t) >= 1 << 30:
                    del live[x]
        flops_exec += 2 * jamp_terms
        ext_name = {"ext_v": "vxxxxx", "ext_o": "oxxxxx", "ext_i": "ixxxxx", "ext_w": "ewkit"}
        # (the external states come from the per-event kits: their flops are in the table's count)
        flops_dag += 2 * jamp_terms
        assert not jslot
        if jbudget:
            return lines, flops_exec, flops_dag, jamp_terms, nflush[0]
        return lines, flops_exec, flops_dag, jamp_terms

    if chunks:
        # chunked form: contiguous pieces of the schedule, each with the flows it touches
        K = chunks
        size = (len(full_order) + K - 1) // K
        pieces = [full_order[c * size:(c + 1) * size] for c in range(K)]
        chunk_out = []
        partials = {"n": 0}
        for c, piece in enumerate(pieces):
            words = sorted({w for i in piece for w in g.amps[i].colour.terms}, key=lambda w: widx[w])
            lines_c, fexec_c, fdag_c, jt_c, nfl = emit_schedule(budget[1], piece, None, jbudget, partials)
            chunk_out.append((words, nfl, lines_c, fexec_c, fdag_c, jt_c))
        assert set(partials) - {"n"} == set(basis)
        nslot = partials["n"]
        lines_d = lines_f = []
        flops_exec_d = flops_exec_f = sum(x[3] for x in chunk_out)
        # a wavefunction recomputed by several chunks counts once in the DAG figure
        flops_dag = emit_schedule(budget[1])[2]
        jamp_terms = sum(x[5] for x in chunk_out)
    else:
        lines_d, flops_exec_d, flops_dag, jamp_terms = emit_schedule(budget[0], order_d)
        lines_f, flops_exec_f, _, _ = emit_schedule(budget[1], order_f)

    nq, nd = len(qidx), len(didx)
    dy = g.family == "dy"
    ext = [k for k in range(npar) if ("E", k) in g.nodes]  # particles with a kit of their own
    koff = {}
    off = 4 * nq + nd
    for k in ext:
        koff[k] = off
        # both helicities; a gluon's kit is followed by its light-cone form
        off += 20 if g.nodes[("E", k)].kind == "ext_v" else 16
    if dy:
        koff["W"] = off
        off += 8 * EW_ITEMS
    voff = off
    roff = off + vk_off[0]  # recycled wavefunctions: 4 helicity pairs x 8 reals each
    rlcoff = roff + 32 * len(rec)  # light-cone forms of the recycled currents, the same layout
    ntab = rlcoff + 32 * len(rec_lc)

    def finish(lines, pf):
        lines = [l.replace("DOFF", str(4 * nq)).replace("VOFF", str(voff)).replace("RLOFF", str(rlcoff))
                 .replace("ROFF", str(roff)) for l in lines]
        for k in koff:
            lines = [l.replace(f"KLOFF{k}", str(koff[k] + 10)).replace(f"KOFF{k}", str(koff[k])) for l in lines]
        return "\n".join(prefetch_units(lines, bool(pf), kits=(pf != "table")))

    body_d = finish(lines_d, prefetch[0])
    body_f = finish(lines_f, prefetch[1])
    chunk_headers = []
    for c, (words, nfl, lines_c, fexec_c, fdag_c, jt_c) in enumerate(chunk_out if chunks else []):
        body_c = finish(lines_c, prefetch[1])
        chunk_headers.append(f"""// Generated by paper_2507_21039_amd.gen for {label}, piece {c} of {len(chunk_out)}.  Do not edit.
// {len(pieces[c])} of the {len(g.amps)} amplitude terms, adding to {len(words)} of the {ncol} colour flows.
#pragma once
#include "{file_stem}.h"

namespace hme {{

struct {name}_c{c} {{
  using Base = {name};
  static constexpr int nw = {len(words)};       // colour flows this piece adds to
  static constexpr int nflush = {nfl};  // partial jamps it hands to the sink
  static constexpr int jbudget = {jbudget};  // flows accumulated in registers at once
  static constexpr double flops_per_hel_executed = {fexec_c};

  // This piece's terms of the jamps of one helicity.  Each partial sum of a flow leaves
  // through sink.put(slot, value), to a workspace slot no other code writes; the colour
  // kernel adds up the slots of every flow (Base::gather).
  template <class T, class Sink>
  HME_FN static void amplitudes(const ProcParams& prm, unsigned h, tab_of<T> tab, Sink& sink) {{
    auto hel = [h](int k) {{ return (h >> ({npar - 1} - k) & 1u) ? 1 : -1; }};
    const T mT = T(prm.mT);
    cx<T> jr[{jbudget}];
{body_c}
  }}
}};

}}  // namespace hme
""")
    qmask = [0] * nq
    qsign = [0] * nq
    for (m, sgn), i in qidx.items():
        qmask[i], qsign[i] = m, sgn
    dmask = [0] * nd
    dmassive = [0] * nd
    for m, (i, massive) in didx.items():
        dmask[i], dmassive[i] = m, int(massive)
    # kit kinds: 0 vector; fermions 1 ubar (outgoing), 2 v (outgoing), 3 vbar (incoming),
    # 4 u (incoming); -1 none (the leptons of the Drell-Yan family live in the electroweak kit)
    kind_code = {"ext_v": 0, "ext_o": 3 if dy else 1, "ext_i": 4 if dy else 2}
    kits = [(koff[k], kind_code[g.nodes[("E", k)].kind], k) if k in koff else (0, -1, k) for k in range(npar)]
    flops_table = DEN_FLOPS * nd + 4 * nq + 40 * len(ext)
    flops_table += LC_KIT_FLOPS * sum(1 for k in ext if g.nodes[("E", k)].kind == "ext_v")
    flops_table += 4 * sum(FLOPS[NODE_FLOPS[g.nodes[k].kind]] + (FD_FLOPS if fd and g.nodes[k].kind in ("vvv", "qq") else 0)
                           for k in rec)  # each helicity pair once
    flops_table += 4 * LC_REC_FLOPS * len(rec_lc)
    rec_rows = [(kind, pa, pb, koff[pa], koff[pb], kk, fk, lc) for kind, pa, pb, kk, fk, lc in rec_info]
    nrec = len(rec)
    qmass = "0.0" if dy else "prm.mT"  # mass of the quark line
    row_end = 1 if dy else TOP  # particle of the barred spinor at the quark line's end
    fmass = "0.0" if dy else "k < 2 ? 0.0 : prm.mT"  # masses of the external fermions
    ew_items = ""
    if dy:
        ew_items = (f"    if (j >= nq + nd + {npar} + nvk) {{\n"
                    "      // the electroweak current of the lepton pair (u-quark charge 2/3, electron -1)\n"
                    "      const EwCouplings c{prm.cA * (-2.0 / 3.0), prm.cZ, prm.gLu, prm.gRu, prm.gL, prm.gR, prm.mZ, prm.wZ};\n"
                    f"      const int item = j - nq - nd - {npar} - nvk;\n"
                    f"      ew_kit(p[2], p[3], c, item, tab + {koff['W']} + 8 * item);\n"
                    "      return;\n"
                    "    }\n")
    flops_table += 0  # the electroweak kit is counted per helicity, with the external states

    # colour sum with symmetric integer numerators
    cs = []
    cs_flops = 0
    for i in range(ncol):
        terms = [(j, N[i][j] * (1 if i == j else 2)) for j in range(i, ncol) if N[i][j] != 0]
        if not terms:
            continue
        zr = " + ".join(f"T({v}) * jamp[{j}].r" for j, v in terms)
        zi = " + ".join(f"T({v}) * jamp[{j}].i" for j, v in terms)
        cs.append(f"    s += jamp[{i}].r * ({zr}) + jamp[{i}].i * ({zi});")
        cs_flops += 4 * len(terms) + 4

    nvk = len(vk_list)
    nitems = nq + nd + npar + nvk + (EW_ITEMS if dy else 0)
    # the momentum sums the table reads, one per internal line: a mask and its complement
    # are the two sides of one line, and the sum is always taken over the side without the
    # barred spinor's particle (a mask holding it reads that sum negated)
    full = (1 << npar) - 1
    sum_masks = []

    def slot(m):
        neg = bool(m >> row_end & 1)
        c = (~m & full) if neg else m
        if c not in sum_masks:
            sum_masks.append(c)
        return 2 * sum_masks.index(c) + int(neg)

    qcode = [slot(m) for m in qmask]
    dcode = [slot(m) for m in dmask]
    vk_c = [[slot(x[1 + i]) if (i == 0 or x[0] in ("vvv", "amp3")) else 0 for x in vk_list] for i in range(3)]
    nsum = len(sum_masks)
    flops_table += sum(VK_FLOPS[x[0]] for x in vk_list)
    vk_kind_code = {"vvv": 0, "psi": 1, "amp3": 2, "fd": 3}
    numer_list = ", ".join(str(N[i][j]) for i in range(ncol) for j in range(ncol))
    assert all(abs(N[i][j]) < 32768 for i in range(ncol) for j in range(ncol))
    gather_code = ""
    if chunks:
        # flows in groups of about GATHER_GROUP slots: a group's loads are written before its
        # sums, so that many loads are in flight whatever order the compiler would pick
        gl_lines, fold_lines, group, nload = [], [], [], 0

        def flush():
            if not group:
                return
            for out in (gl_lines, fold_lines):
                out.append("    {")
                for _, sls in group:
                    out.extend(f"      const auto s{sl} = col[{sl} * stride];" for sl in sls)
            for i, sls in group:
                total = " + ".join(f"cast<T>(s{sl})" for sl in sls)
                gl_lines.append(f"      jamp[{i}] = {total};")
                fold_lines.append(f"      col.put({sls[0]} * stride, {total});")
            gl_lines.append("    }")
            fold_lines.append("    }")
            group.clear()

        for i, w in enumerate(basis):
            sls = sorted(partials[w])
            if group and nload + len(sls) > GATHER_GROUP:
                flush()
                nload = 0
            group.append((i, sls))
            nload += len(sls)
        flush()
        jslot = [sorted(partials[w])[0] for w in basis]
        gather_code = (
            "  // the jamps of one helicity from the workspace column `col` (slot s at col[s * stride];\n"
            "  // col: a pointer to cx<S>, or an accessor with the same indexing): each flow is the sum of\n"
            "  // its partial slots, added in slot order; the loads of a group of flows come first\n"
            "  template <class T, class S, class Col>\n"
            f"  HME_FN static void gather(const Col& col, int64_t stride, cx<T> (&jamp)[{ncol}]) {{\n"
            + "\n".join(gl_lines) + "\n  }\n\n"
            "  // the same sums, each written over its flow's first slot (jslot): the column then holds\n"
            "  // the jamps at those slots (col: an accessor with put; no slot is read after it is written)\n"
            f"  static constexpr short jslot[{ncol}] = {{{', '.join(map(str, jslot))}}};\n"
            "  template <class T, class Col>\n"
            "  HME_FN static void fold(const Col& col, int64_t stride) {\n"
            + "\n".join(fold_lines) + "\n  }\n\n")
        amp_section = (f"  // the amplitude terms are split into {len(chunk_out)} contiguous pieces of the schedule\n"
                       f"  // ({name}_c0 .. {name}_c{len(chunk_out) - 1}); each runs as its own kernel and adds\n"
                       f"  // its terms to the jamps kept in a device workspace between kernels\n"
                       f"  static constexpr int nchunk = {len(chunk_out)};\n"
                       f"  static constexpr int nslot = {nslot};  // partial-sum slots per helicity\n\n"
                       + gather_code)
    else:
        amp_section = f"""  static constexpr int nchunk = 0, nslot = 0;  // one kernel evaluates every amplitude term

  // jamps of one helicity (jamp[] must be zeroed by the caller); the schedule depends on the
  // arithmetic type (budget {budget[0]} / prefetch "{prefetch[0]}" for double, {budget[1]} / "{prefetch[1]}" for float).
  // obs.term(d, a) sees every amplitude term a of diagram d (the default observer does nothing).
  template <class T, class Obs = NoObserver>
  HME_FN static void amplitudes(const double (&p)[{npar}][4], const ProcParams& prm, unsigned h,
                                tab_of<T> tab, cx<T> (&jamp)[{ncol}], Obs obs = Obs{{}}) {{
    if constexpr (sizeof(T) == 8)
      amplitudes_d<T>(prm, h, tab, jamp, obs);
    else
      amplitudes_f<T>(prm, h, tab, jamp, obs);
  }}

  template <class T, class Obs>
  HME_FN static void amplitudes_d(const ProcParams& prm, unsigned h, tab_of<T> tab, cx<T> (&jamp)[{ncol}], Obs& obs) {{
    auto hel = [h](int k) {{ return (h >> ({npar - 1} - k) & 1u) ? 1 : -1; }};
    const T mT = T(prm.mT);
{body_d}
  }}

  template <class T, class Obs>
  HME_FN static void amplitudes_f(const ProcParams& prm, unsigned h, tab_of<T> tab, cx<T> (&jamp)[{ncol}], Obs& obs) {{
    auto hel = [h](int k) {{ return (h >> ({npar - 1} - k) & 1u) ? 1 : -1; }};
    const T mT = T(prm.mT);
{body_f}
  }}

"""
    hdr = f"""// Generated by paper_2507_21039_amd.gen for {label}.  Do not edit.
// {g.ndiag} Feynman diagrams{" (photon and Z exchange counted together)" if dy else ""}, {len(g.amps)} amplitude terms (each four-gluon vertex split into its
// three structures), {len(g.nodes)} wavefunctions, {ncol} colour flows; at most {budget[0]} (double) or
// {budget[1]} (float) off-shell wavefunctions live at once (others are recomputed when needed again).
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
  static constexpr double iden = {iden_dy(len(gl)) if dy else iden_qcd(len(gl) - 2)};  // spin and colour average, identical gluons
  static constexpr double colour_denom = {D};
  // algorithmic flops per helicity: every call once (wavefunctions once), jamp additions and
  // the colour sum counted as 4 ncol^2 (the dense quadratic form; the symmetric VALU form
  // executes {cs_flops}); executed: with recomputation, the symmetric colour sum (double)
  static constexpr double flops_per_hel = {flops_dag + 4 * ncol * ncol};
  static constexpr double flops_per_hel_executed = {flops_exec_d + cs_flops};
  static constexpr double flops_per_event = {flops_table};  // helicity-independent table

  // Per-event table (LDS): {nq} momentum sums (incoming momenta of the particles in the mask,
  // negated for barred currents), {nd} propagator denominators 1/(Q^2 - m^2), and for every
  // external particle a kit holding its state for either helicity (gluon: the five nonzero real
  // parts of eps or conj(eps); fermion: the four complex components of ubar or v).
  // Momentum sums are read through codes 2 s + n: sum s of sum_mask (n = 1: negated).
  static constexpr int nq = {nq}, nd = {nd}, nitems = {nitems}, ntab = {ntab};
  static constexpr short qcode[{max(nq, 1)}] = {{{", ".join(map(str, qcode)) or "0"}}};
  static constexpr int qsign[{max(nq, 1)}] = {{{", ".join(map(str, qsign))}}};
  static constexpr short dcode[{max(nd, 1)}] = {{{", ".join(map(str, dcode)) or "0"}}};
  static constexpr int dmassive[{max(nd, 1)}] = {{{", ".join(map(str, dmassive))}}};
  static constexpr int kit_off[{npar}] = {{{", ".join(str(k[0]) for k in kits)}}};
  static constexpr int kit_kind[{npar}] = {{{", ".join(str(k[1]) for k in kits)}}};  // 0 vector, 1 ubar, 2 v, 3 vbar, 4 u, -1 none

  // vertex kits after the external-state kits: kind 0 three-gluon current (den (Qa - Qb),
  // den (Qa + 2 Qb), den (2 Qa + Qb) with den = 1 / Q^2 of mask 2), kind 1 quark propagator
  // (den sign (K0 + K3, K0 - K3, K1, K2), den mT with K of mask 0 and den = 1 / (K^2 - mT^2)),
  // kind 2 three-gluon amplitude (Qa - Qb, Qb - Qc, Qc - Qa), kind 3 Feynman-diagram gauge
  // projection of a gluon line (nt = n / (n.Q) with n = (sign Q0, -Q3vec / |Q3vec|), then Q)
  static constexpr int nvk = {nvk}, voff = {voff};
  static constexpr int vk_kind[{max(nvk, 1)}] = {{{", ".join(str(vk_kind_code[x[0]]) for x in vk_list) or "0"}}};
  static constexpr short vk_c0[{max(nvk, 1)}] = {{{", ".join(map(str, vk_c[0])) or "0"}}};
  static constexpr short vk_c1[{max(nvk, 1)}] = {{{", ".join(map(str, vk_c[1])) or "0"}}};
  static constexpr short vk_c2[{max(nvk, 1)}] = {{{", ".join(map(str, vk_c[2])) or "0"}}};
  static constexpr int vk_sign[{max(nvk, 1)}] = {{{", ".join(str(x[4]) for x in vk_list) or "1"}}};
  static constexpr int vk_off[{max(nvk, 1)}] = {{{", ".join(str(x[5]) for x in vk_list) or "0"}}};

  // helicity recycling: {nrec} wavefunctions built from two external states, stored for each
  // helicity pair after the vertex kits (8 reals per pair: the 4 complex components); kind 0
  // three-gluon current, 1 spinor current, 2 barred spinor current, 3 quark pair; particles and
  // kit offsets of the two arguments; vertex-kit offset (kinds 0-2) or denominator index (3)
  static constexpr int nrec = {nrec}, roff = {roff};
  static constexpr int rec_kind[{max(nrec, 1)}] = {{{", ".join(str(x[0]) for x in rec_rows) or "0"}}};
  static constexpr int rec_pa[{max(nrec, 1)}] = {{{", ".join(str(x[1]) for x in rec_rows) or "0"}}};
  static constexpr int rec_pb[{max(nrec, 1)}] = {{{", ".join(str(x[2]) for x in rec_rows) or "0"}}};
  static constexpr int rec_oa[{max(nrec, 1)}] = {{{", ".join(str(x[3]) for x in rec_rows) or "0"}}};
  static constexpr int rec_ob[{max(nrec, 1)}] = {{{", ".join(str(x[4]) for x in rec_rows) or "0"}}};
  static constexpr int rec_k[{max(nrec, 1)}] = {{{", ".join(str(x[5]) for x in rec_rows) or "0"}}};
  static constexpr int rec_fd[{max(nrec, 1)}] = {{{", ".join(str(x[6]) for x in rec_rows) or "0"}}};  // gauge kit (kinds 0, 3)
  // currents (kinds 0, 3): index of the light-cone copy at rlcoff + 32 i, same pair layout
  static constexpr int rlcoff = {rlcoff};
  static constexpr int rec_lc[{max(nrec, 1)}] = {{{", ".join(str(x[7]) for x in rec_rows) or "0"}}};
  static constexpr bool fd_gauge = {"true" if fd else "false"};  // Feynman-diagram gauge for internal gluons

  // item i < 4 nrec: recycled wavefunction i / 4 for the helicity pair i % 4 (bit 1: first
  // argument +1, bit 0: second +1), from the kits in t, written into w (the same table)
  template <class S> HME_FN static void recycled_entry(int i, tab_of<S> t, S* w) {{
    using T = S;
    const int r = i >> 2, ha = (i & 2) ? 1 : -1, hb = (i & 1) ? 1 : -1;
    const int na = rec_pa[r] < 2 ? -1 : 1, nb = rec_pb[r] < 2 ? -1 : 1;
    S* o = w + roff + 32 * r + 8 * (i & 3);
    const auto tab = t;
    switch (rec_kind[r]) {{
      case 0: {{
        vw4<T> x = vvv_vec_k<T>(vxxxxx_kit<T>(tab + rec_oa[r], ha, na), vxxxxx_kit<T>(tab + rec_ob[r], hb, nb),
                                load_kit<T, 12>(tab + voff + rec_k[r]));
        if constexpr (fd_gauge) x = fd_project<T>(x, load_kit<T, 8>(tab + voff + rec_fd[r]));
        store_wf(x, o);
        store_lc(vlc_of(x), w + rlcoff + 32 * rec_lc[r] + 8 * (i & 3));
        break;
      }}
      case 1:
        store_wf(ffv_psi_k<T>(ixxxxx_kit<T>(tab + rec_oa[r], ha), vxxxxx_kit<T>(tab + rec_ob[r], hb, nb),
                              load_kit<T, 5>(tab + voff + rec_k[r])), o);
        break;
      case 2:
        store_wf(ffv_psibar_k<T>(oxxxxx_kit<T>(tab + rec_oa[r], ha), vxxxxx_kit<T>(tab + rec_ob[r], hb, nb),
                                 load_kit<T, 5>(tab + voff + rec_k[r])), o);
        break;
      default: {{
        vw4<T> x = ffv_vec<T>(oxxxxx_kit<T>(tab + rec_oa[r], ha), ixxxxx_kit<T>(tab + rec_ob[r], hb),
                              dv<T>(tab, {4 * nq} + rec_k[r]));
        if constexpr (fd_gauge) x = fd_project<T>(x, load_kit<T, 8>(tab + voff + rec_fd[r]));
        store_wf(x, o);
        store_lc(vlc_of(x), w + rlcoff + 32 * rec_lc[r] + 8 * (i & 3));
        break;
      }}
    }}
  }}

  // Sums of incoming momenta (outgoing ones negated) over the masks the table needs, each
  // component as an unevaluated sum hi + lo (two-sum chain: as accurate as a sum in twice the
  // precision).  An internal line has two sides; momenta given in double precision conserve
  // momentum only up to rounding, so the two sums differ slightly, by 1e-12 relative in Q^2 of
  // an almost on-shell line.  Every line therefore takes the sum over the side without particle
  // {row_end} (the barred spinor of the quark line), whichever current it is built in.
  static constexpr int nsum = {nsum};
  static constexpr unsigned sum_mask[{max(nsum, 1)}] = {{{", ".join(map(str, sum_masks)) or "0"}}};

  // sum i (i < nsum) into o[8 i .. 8 i + 7] as (hi, lo) per component; the lanes of an event
  // compute disjoint sums before any table item reads them
  HME_FN static void momentum_sum(const double (&p)[{npar}][4], int i, double* o) {{
    _Pragma("clang fp contract(off)")
    const unsigned m = sum_mask[i];
    double hi[4] = {{0.0, 0.0, 0.0, 0.0}}, lo[4] = {{0.0, 0.0, 0.0, 0.0}};
#pragma unroll
    for (int j = 0; j < {npar}; ++j) {{
      const double s = (m >> j & 1u) ? (j < 2 ? 1.0 : -1.0) : 0.0;
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {{
        const dd t = two_sum(hi[mu], s * p[j][mu]);  // s p is exact
        hi[mu] = t.hi;
        lo[mu] += t.lo;
      }}
    }}
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {{
      const dd t = quick_two_sum(hi[mu], lo[mu]);
      o[8 * i + 2 * mu] = t.hi;
      o[8 * i + 2 * mu + 1] = t.lo;
    }}
  }}

  // the momentum sum of code c (2 s + n) from the sums in `sums`
  HME_FN static void mask_sum(const double* sums, int c, dd* Q) {{
    const double* q = sums + 8 * (c >> 1);
    const double g = (c & 1) ? -1.0 : 1.0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) Q[mu] = dd{{g * q[2 * mu], g * q[2 * mu + 1]}};
  }}

  // the quantities below are formed in compensated arithmetic and rounded once
  // (differences of momentum sums, and Q^2 - m^2 of almost on-shell propagators)
  template <class S> HME_FN static void vertex_kit(const double* sums, const ProcParams& prm, int v, S* o) {{
    dd A[4], B[4], C[4];
    mask_sum(sums, vk_c0[v], A);
    if (vk_kind[v] == 3) {{
      // Feynman-diagram gauge: nt = n / (n.Q), n = (sign Q0, -Q3vec / |Q3vec|), n.Q = |Q0| + |Q3vec|;
      // a line at rest (an s-channel gluon in the centre-of-mass frame) has no direction of its
      // own and takes the z axis (any fixed direction is a gauge choice)
      double q[4];
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) q[mu] = dd_val(A[mu]);
      const double qa = sqrt(q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
      const double nq = 1.0 / (fabs(q[0]) + qa);
      o[0] = S((q[0] >= 0 ? 1.0 : -1.0) * nq);
#pragma unroll
      for (int mu = 1; mu < 4; ++mu) o[mu] = S(qa > 0 ? -q[mu] / qa * nq : (mu == 3 ? -nq : 0.0));
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) o[4 + mu] = S(q[mu]);
      return;
    }}
    if (vk_kind[v] == 1) {{
      const double den = 1.0 / dd_minkowski_sq(A, {qmass});
      const double ds = den * vk_sign[v];
      o[0] = S(ds * dd_val(dd_add(A[0], A[3])));
      o[1] = S(ds * dd_val(dd_add(A[0], dd_neg(A[3]))));
      o[2] = S(ds * dd_val(A[1]));
      o[3] = S(ds * dd_val(A[2]));
      o[4] = S(den * {qmass});
      return;
    }}
    mask_sum(sums, vk_c1[v], B);
    mask_sum(sums, vk_c2[v], C);
    if (vk_kind[v] == 0) {{
      const double den = 1.0 / dd_minkowski_sq(C, 0.0);
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {{
        o[mu] = S(den * dd_val(dd_add(A[mu], dd_neg(B[mu]))));
        o[4 + mu] = S(den * dd_val(dd_add(A[mu], dd_scale(2.0, B[mu]))));
        o[8 + mu] = S(den * dd_val(dd_add(dd_scale(2.0, A[mu]), B[mu])));
      }}
    }} else {{
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {{
        o[mu] = S(dd_val(dd_add(A[mu], dd_neg(B[mu]))));
        o[4 + mu] = S(dd_val(dd_add(B[mu], dd_neg(C[mu]))));
        o[8 + mu] = S(dd_val(dd_add(C[mu], dd_neg(A[mu]))));
      }}
    }}
  }}

  // item j of the table (j < nitems), from the event and its momentum sums; the lanes of an
  // event compute disjoint items
  template <class S>
  HME_FN static void table_entry(const double (&p)[{npar}][4], const ProcParams& prm, int j, const double* sums,
                                 S* tab) {{
{ew_items}    if (j >= nq + nd + {npar}) {{
      const int v = j - nq - nd - {npar};
      vertex_kit(sums, prm, v, tab + voff + vk_off[v]);
      return;
    }}
    if (j >= nq + nd) {{
      // static indexing of p (a dynamic index would put the event record in scratch)
#pragma unroll
      for (int k = 0; k < {npar}; ++k) {{
        if (j - nq - nd != k) continue;
        if (kit_kind[k] == 0) {{
          vector_kit(p[k], k < 2 ? -1 : 1, tab + kit_off[k]);
          vector_lc_kit(p[k], k < 2 ? -1 : 1, tab + kit_off[k] + 10);
        }}
        else if (kit_kind[k] > 0) fermion_kit(p[k], {fmass}, kit_kind[k], tab + kit_off[k]);
      }}
      return;
    }}
    const bool isq = j < nq;
    dd Q[4];
    mask_sum(sums, isq ? qcode[j] : dcode[j - nq], Q);
    if (isq) {{
      const double sg = qsign[j];
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) tab[4 * j + mu] = S(sg * dd_val(Q[mu]));
    }} else {{
      tab[4 * nq + (j - nq)] = S(1.0 / dd_minkowski_sq(Q, dmassive[j - nq] ? {qmass} : 0.0));
    }}
  }}

{amp_section}  // the colour matrix times colour_denom (integer numerators, row-major, symmetric)
  static constexpr short numer[{ncol * ncol}] = {{{numer_list}}};

  // sum over colour flows of conj(jamp) C jamp times colour_denom
  template <class T> HME_FN static T colour_sum(const cx<T> (&jamp)[{ncol}]) {{
    T s = 0;
{chr(10).join(cs)}
    return s;
  }}
}};

}}  // namespace hme
"""
    info = dict(name=name, npar=npar, ncol=ncol, ndiag=g.ndiag, namp=len(g.amps), nwf=len(g.nodes),
                flops_per_hel=flops_dag + 4 * ncol * ncol, flops_per_hel_executed=flops_exec_d + cs_flops,
                flops_per_hel_executed_f32=flops_exec_f + cs_flops,
                flops_colour=4 * ncol * ncol, flops_colour_symmetric=cs_flops, flops_table=flops_table, colour_denom=D, numerators=N,
                jamp_terms=jamp_terms, budget=list(budget), prefetch=list(prefetch), ntab=ntab,
                nchunk=len(chunk_headers), nslot=nslot if chunks else 0, jbudget=jbudget if chunks else 0,
                chunk_headers=chunk_headers)
    return hdr, info


def iden_qcd(nfinal_gluons: int) -> float:
    return 4.0 * 64.0 * math.factorial(nfinal_gluons)


def iden_dy(nfinal_gluons: int) -> float:
    """u ubar initial state: 4 spin states, 9 colour states; identical final gluons."""
    return 4.0 * 9.0 * math.factorial(nfinal_gluons)


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
  static constexpr int nchunk = 0, nslot = 0;
  static constexpr int gs_power = 0;
  static constexpr double iden = 4.0;  // average over the initial helicities
  static constexpr double colour_denom = 1.0;
  static constexpr double flops_per_hel = {flops};
  static constexpr double flops_per_event = 20.0;  // s, 1/s, Z propagator denominator

  static constexpr int nq = 0, nd = 0, nitems = 0, ntab = 0, nsum = 0, nrec = 0;  // no per-event table
  template <class S> HME_FN static void recycled_entry(int, tab_of<S>, S*) {{}}
  HME_FN static void momentum_sum(const double (&)[4][4], int, double*) {{}}
  template <class S>
  HME_FN static void table_entry(const double (&)[4][4], const ProcParams&, int, const double*, S*) {{}}

  template <class T, class Obs = NoObserver>
  HME_FN static void amplitudes(const double (&p)[4][4], const ProcParams& prm, unsigned h,
                                tab_of<T>, cx<T> (&jamp)[1], Obs obs = Obs{{}}) {{
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
