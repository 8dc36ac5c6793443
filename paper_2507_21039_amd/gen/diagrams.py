"""Tree-level Feynman diagrams of g g -> t tbar + n g and their HELAS-style call graph.

Every diagram has one quark line, from the outgoing top (barred spinor, particle
index 2) to the outgoing antitop (spinor, particle index 3), with gluon trees
attached along it.  A gluon tree is a leaf (external gluon), a three-gluon
vertex joining two trees, or a four-gluon vertex joining three trees.  Counting
each four-gluon vertex once gives 3 / 16 / 123 / 1240 diagrams for n = 0..3
extra gluons.

For evaluation each four-gluon vertex splits into its three Lorentz/colour
structures, so a diagram becomes one or more amplitude terms.  The generator
builds the wavefunctions (external states, off-shell currents with their
propagators) once and reuses them across diagrams, then closes each diagram
with one amplitude call.  This is the sequence the paper describes in section
"Parallel scattering amplitudes": external wavefunctions, off-shell propagators
merged pairwise, a final vertex giving a complex amplitude, repeated for each
diagram, then the colour inner product.

The Drell-Yan family u ubar -> e+ e- + n g has the same structure with one more element on
the quark line (from vbar(ubar), particle 1, to u(u), particle 0): the electroweak boson
that carries the lepton pair.  Its photon and Z exchanges are one wavefunction here (the
lepton current times the photon and Z propagators and couplings, summed for the quark's
chirality, which a massless line conserves), so a diagram counts the photon and the Z
together: 1 / 2 / 8 / 50 diagrams for n = 0..3 (2 / 4 / 16 / 100 counting them apart).

Feynman rules with the strong coupling stripped (every amplitude carries g_s^n):
quark-gluon vertex i gamma^mu T^a, three-gluon vertex f^{abc} V^{mu nu rho},
four-gluon vertex -i [f^{abe} f^{cde} L1 + f^{ace} f^{bde} L2 + f^{ade} f^{bce} L3],
gluon propagator -i g/Q^2, quark propagator i (K-slash + m)/(K^2 - m^2).  The
Lorentz routines compute the bare structures; the factors of i and the colour
expansion (f^{abc} T^c = -i [T^a, T^b]) are collected here into the jamp
coefficients.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from functools import lru_cache

from .colour import I, MINUS_I, ONE, Gauss, Poly

TOP, ATOP = 2, 3  # particle indices of t and tbar (0-based)
EW = ("W",)  # the electroweak boson (photon and Z) as an element of a quark-line sequence


# ------------------------------------------------------------------ gluon trees
# ('L', k) | ('3', X, Y) | ('4', X, Y, Z)          -- topologies (for counting)
# ('L', k) | ('3', X, Y) | ('4', X, Y, Z, s)       -- versions (s = 1, 2, 3 structure)


def leaves(t) -> frozenset:
    if t == EW:
        return frozenset()
    if t[0] == "L":
        return frozenset([t[1]])
    return frozenset().union(*(leaves(x) for x in t[1:] if isinstance(x, tuple)))


def _set_partitions_2(S):
    S = sorted(S)
    lo, rest = S[0], S[1:]
    for r in range(0, len(rest)):
        for comb in itertools.combinations(rest, r):
            A = frozenset((lo,) + comb)
            B = frozenset(S) - A
            if B:
                yield A, B


def _set_partitions_3(S):
    for A, R in _set_partitions_2(S):
        if len(R) < 2:
            continue
        for B, C in _set_partitions_2(R):
            yield A, B, C


@lru_cache(maxsize=None)
def trees(S: frozenset):
    """All gluon tree topologies over the gluon set S (unordered children, canonical order)."""
    if len(S) == 1:
        return (("L", next(iter(S))),)
    out = []
    for A, B in _set_partitions_2(S):
        for X in trees(A):
            for Y in trees(B):
                out.append(("3", X, Y))
    for A, B, C in _set_partitions_3(S):
        for X in trees(A):
            for Y in trees(B):
                for Z in trees(C):
                    out.append(("4", X, Y, Z))
    return tuple(out)


def versions(t):
    """Expand the four-gluon vertices of a topology into their three structures."""
    if t == EW or t[0] == "L":
        return [t]
    if t[0] == "3":
        return [("3", x, y) for x in versions(t[1]) for y in versions(t[2])]
    return [("4", x, y, z, s) for x in versions(t[1]) for y in versions(t[2]) for z in versions(t[3])
            for s in (1, 2, 3)]


def ordered_set_partitions(S):
    S = sorted(S)
    n = len(S)
    for k in range(1, n + 1):
        # assign each element a block index, blocks non-empty, then order the blocks
        for assign in itertools.product(range(k), repeat=n):
            if len(set(assign)) != k:
                continue
            # canonical: blocks labelled by order of first appearance -> then permute labels
            first = []
            for a in assign:
                if a not in first:
                    first.append(a)
            if first != list(range(k)):
                continue
            blocks = [frozenset(S[i] for i in range(n) if assign[i] == b) for b in range(k)]
            for perm in itertools.permutations(range(k)):
                yield tuple(blocks[p] for p in perm)


def diagrams(gluons):
    """All diagrams as tuples of gluon-tree topologies along the quark line (from the top end)."""
    out = []
    for blocks in ordered_set_partitions(gluons):
        for ts in itertools.product(*(trees(b) for b in blocks)):
            out.append(tuple(ts))
    return out


def diagrams_dy(gluons):
    """Diagrams of u ubar -> e+ e- + gluons: gluon trees along the quark line with the
    electroweak boson inserted at any position (sequences read from the ubar end)."""
    out = []
    parts = list(ordered_set_partitions(gluons)) if gluons else [()]
    for blocks in parts:
        for ts in itertools.product(*(trees(b) for b in blocks)):
            for pos in range(len(ts) + 1):
                out.append(tuple(ts[:pos]) + (EW,) + tuple(ts[pos:]))
    return out


def tree_key(t) -> str:
    """Name of a gluon tree independent of enumeration order: g<particle>, (x,y) for a three-gluon
    vertex, [x,y,z] for a four-gluon vertex (children's names sorted); W for the electroweak boson."""
    if t == EW:
        return "W"
    if t[0] == "L":
        return f"g{t[1]}"
    ks = sorted(tree_key(x) for x in t[1:] if isinstance(x, tuple))
    return ("(" if t[0] == "3" else "[") + ",".join(ks) + (")" if t[0] == "3" else "]")


def diagram_keys(ngluon_final: int, family: str = "tt") -> list:
    """Names of the diagrams in the generator's order (the columns of the channel weights): the
    elements of the quark line from its barred end (the top, or the ubar), joined by ';'."""
    if family == "dy":
        ds = diagrams_dy(tuple(range(4, 4 + ngluon_final)))
    else:
        ds = diagrams(tuple([0, 1] + list(range(4, 4 + ngluon_final))))
    return [";".join(tree_key(t) for t in d) for d in ds]


# ------------------------------------------------------------------ colour of wavefunctions


@lru_cache(maxsize=None)
def tree_poly(v) -> Poly:
    """Colour polynomial of a gluon-tree version, including vertex and propagator phases.

    three-gluon current:  f^{xyr} T^r = -i[X, Y], propagator -i      -> -(XY - YX)
    four-gluon current s: -i * (-[[.,.],.]) from f f T, propagator -i -> +[[X,Y],Z], [[X,Z],Y], [[Y,Z],X]
    """
    if v == EW:
        return Poly.unit()  # colourless
    if v[0] == "L":
        return Poly.letter(v[1])
    if v[0] == "3":
        return tree_poly(v[1]).comm(tree_poly(v[2])).scale(Gauss(-1, 0))
    X, Y, Z = tree_poly(v[1]), tree_poly(v[2]), tree_poly(v[3])
    s = v[4]
    if s == 1:
        return X.comm(Y).comm(Z)
    if s == 2:
        return X.comm(Z).comm(Y)
    return Y.comm(Z).comm(X)


# ------------------------------------------------------------------ call graph


@dataclass(frozen=True)
class Node:
    key: tuple
    kind: str  # 'ext_v', 'ext_i', 'ext_o', 'ext_w', 'vvv', 'vvvv', 'psi', 'psibar', 'qq'
    args: tuple  # keys of input nodes
    mask: int  # set of external particles the wavefunction covers
    extra: tuple = ()


@dataclass
class Amp:
    kind: str  # 'ffv', 'vvv', 'vvvv'
    args: tuple
    extra: tuple
    colour: Poly
    diagram: int


@dataclass
class Graph:
    npar: int
    gluons: tuple
    family: str = "tt"  # "tt": g g -> t tbar + n g; "dy": u ubar -> e+ e- + n g
    nodes: dict = field(default_factory=dict)  # key -> Node, insertion = topological order
    amps: list = field(default_factory=list)
    ndiag: int = 0

    def add(self, node: Node):
        if node.key not in self.nodes:
            self.nodes[node.key] = node
        return node.key


def _bit(k):
    return 1 << k


def build_graph(ngluon_final: int, family: str = "tt") -> Graph:
    """Call graph for g g -> t tbar + ngluon_final g (family "tt") or for
    u ubar -> e+ e- + ngluon_final g (family "dy").

    Particle indices, tt: 0, 1 incoming gluons; 2 top; 3 antitop; 4.. outgoing gluons.  The
    quark line runs from ubar(t) (row spinor) to v(tbar) (column spinor).
    dy: 0 u (incoming); 1 ubar (incoming); 2 e+; 3 e-; 4.. outgoing gluons.  The quark line
    runs from vbar(ubar) (row spinor) to u(u) (column spinor); the external node ("E", "W") is
    the electroweak current of the lepton pair.
    """
    npar = 4 + ngluon_final
    dy = family == "dy"
    gluons = tuple(range(4, npar)) if dy else tuple([0, 1] + list(range(4, npar)))
    row_end, col_end = (1, 0) if dy else (TOP, ATOP)
    g = Graph(npar=npar, gluons=gluons, family=family)
    for k in gluons:
        g.add(Node(("E", k), "ext_v", (), _bit(k)))
    g.add(Node(("E", row_end), "ext_o", (), _bit(row_end)))
    g.add(Node(("E", col_end), "ext_i", (), _bit(col_end)))
    if dy:
        g.add(Node(("E", "W"), "ext_w", (), _bit(2) | _bit(3)))

    def tree_node(v):
        if v == EW:
            return ("E", "W")
        if v[0] == "L":
            return ("E", v[1])
        if v[0] == "3":
            a, b = tree_node(v[1]), tree_node(v[2])
            return g.add(Node(("J", v), "vvv", (a, b), g.nodes[a].mask | g.nodes[b].mask))
        a, b, c = tree_node(v[1]), tree_node(v[2]), tree_node(v[3])
        return g.add(Node(("J", v), "vvvv", (a, b, c), g.nodes[a].mask | g.nodes[b].mask | g.nodes[c].mask,
                          (v[4],)))

    def psi_node(seq):
        """Spinor current: the trees in seq attached to v(tbar), seq read from the top end."""
        if not seq:
            return ("E", col_end)
        inner = psi_node(seq[1:])
        t = tree_node(seq[0])
        return g.add(Node(("F", seq), "psi", (inner, t), g.nodes[inner].mask | g.nodes[t].mask))

    def psibar_node(seq):
        """Barred spinor current: ubar(t) with the trees in seq attached, seq read from the top end."""
        if not seq:
            return ("E", row_end)
        inner = psibar_node(seq[:-1])
        t = tree_node(seq[-1])
        return g.add(Node(("Fb", seq), "psibar", (inner, t), g.nodes[inner].mask | g.nodes[t].mask))

    def psi_poly(seq):
        p = Poly.unit()
        for v in seq:
            # a gluon attachment: vertex i and propagator i -> -1; the electroweak boson:
            # propagator i (its vertex factor, the same in every diagram, is left out)
            p = (p * tree_poly(v)).scale(I if v == EW else Gauss(-1, 0))
        return p

    def missing(seq, bar):
        """Number of fermion currents that closing with this sequence would add."""
        cnt = 0
        while seq:
            key = ("Fb", seq) if bar else ("F", seq)
            if key in g.nodes:
                break
            cnt += 1
            seq = seq[:-1] if bar else seq[1:]
        return cnt

    qq_key = None
    diags = diagrams_dy(gluons) if dy else diagrams(gluons)
    g.ndiag = len(diags)
    # close short quark lines first so that longer ones find their currents
    order = sorted(range(len(diags)), key=lambda d: (len(diags[d]), d))
    for d in order:
        topo = diags[d]
        for vs in itertools.product(*(versions(t) for t in topo)):
            if len(vs) == 1 and not dy:
                root = vs[0]
                if qq_key is None:
                    qq_key = g.add(Node(("Q",), "qq", (("E", TOP), ("E", ATOP)), _bit(TOP) | _bit(ATOP)))
                if root[0] == "3":
                    a, b = tree_node(root[1]), tree_node(root[2])
                    col = tree_poly(root[1]).comm(tree_poly(root[2])).scale(MINUS_I)
                    g.amps.append(Amp("vvv", (a, b, qq_key), (), col, d))
                else:
                    a, b, c = tree_node(root[1]), tree_node(root[2]), tree_node(root[3])
                    X, Y, Z = tree_poly(root[1]), tree_poly(root[2]), tree_poly(root[3])
                    s = root[4]
                    col = (X.comm(Y).comm(Z) if s == 1 else X.comm(Z).comm(Y) if s == 2 else Y.comm(Z).comm(X))
                    g.amps.append(Amp("vvvv", (a, b, c, qq_key), (s,), col.scale(I), d))
                continue
            k = len(vs)
            best = None
            for j in range(k):
                bar, mid, right = vs[:j], vs[j], vs[j + 1:]
                cost = missing(bar, True) + missing(right, False)
                bal = abs(len(bar) - len(right))
                cand = (cost, bal, j)
                if best is None or cand < best:
                    best = cand
            j = best[2]
            bar, mid, right = vs[:j], vs[j], vs[j + 1:]
            fb = psibar_node(bar)
            f = psi_node(right)
            t = tree_node(mid)
            # the closing vertex: i for a gluon; the electroweak vertex factor is left out
            colour = (psi_poly(bar) * tree_poly(mid) * psi_poly(right)).scale(ONE if mid == EW else I)
            g.amps.append(Amp("ffv", (fb, f, t), (), colour, d))
    return g


def stats(g: Graph):
    kinds = {}
    for n in g.nodes.values():
        kinds[n.kind] = kinds.get(n.kind, 0) + 1
    akinds = {}
    for a in g.amps:
        akinds[a.kind] = akinds.get(a.kind, 0) + 1
    return dict(ndiag=g.ndiag, namp=len(g.amps), nodes=kinds, amps=akinds)


def schedule(g: Graph) -> list:
    """Order the amplitude terms to keep few wavefunctions live at once.

    Greedy list scheduling: repeatedly take the amplitude that needs the fewest
    wavefunctions not yet computed, net of the wavefunctions whose last
    consumer it is.  External wavefunctions are not counted (they are cheap and
    live throughout).  Returns indices into g.amps.
    """
    nodes_of = []
    for a in g.amps:
        s = set()
        stack = list(a.args)
        while stack:
            k = stack.pop()
            if k in s:
                continue
            s.add(k)
            stack.extend(g.nodes[k].args)
        nodes_of.append(frozenset(s))
    pending = {k: 0 for k in g.nodes}  # remaining amplitudes that need each node
    for s in nodes_of:
        for k in s:
            pending[k] += 1
    remaining = set(range(len(g.amps)))
    done = set()
    live = set()
    order = []
    while remaining:
        best = None
        for i in remaining:
            s = nodes_of[i]
            new = [k for k in s if k not in done and k[0] != "E"]
            freed = sum(1 for k in (live | s) if k[0] != "E" and pending[k] == (1 if k in s else 0))
            cand = (len(new) - freed, len(new), i)
            if best is None or cand < best:
                best = cand
        i = best[2]
        order.append(i)
        remaining.discard(i)
        for k in nodes_of[i]:
            pending[k] -= 1
        done |= nodes_of[i]
        live = {k for k in (live | nodes_of[i]) if pending[k] > 0}
    return order


def schedule_cached(g: Graph, node_cost: dict, cache: int, flow_regs: int = 0, flow_cost: float = 0.0) -> list:
    """Order the amplitude terms for a kernel that keeps only `cache` off-shell wavefunctions.

    Greedy: repeatedly take the amplitude term whose evaluation is cheapest given what an
    LRU model of the registers holds: the cost of computing every wavefunction of its
    closure that is not held (node_cost[kind]), plus flow_cost for every colour flow it
    adds to that is not among the `flow_regs` most recently used flows (a new partial sum
    when jamps are accumulated in a bounded set of registers).  The emitter then evicts
    with Belady's rule on the order chosen here.  Returns indices into g.amps.
    """
    from collections import OrderedDict
    closures = []
    for a in g.amps:
        s, stack = set(), list(a.args)
        while stack:
            k = stack.pop()
            if k in s or k[0] == "E":
                continue
            s.add(k)
            stack.extend(g.nodes[k].args)
        closures.append(s)
    cost = {k: node_cost[n.kind] for k, n in g.nodes.items() if k[0] != "E"}
    # fixed iteration orders (node creation order, flow order of the colour terms), so the
    # schedule does not depend on Python's hash seed
    rank = {k: i for i, k in enumerate(g.nodes)}
    closures = [sorted(c, key=rank.__getitem__) for c in closures]
    flows = [list(a.colour.terms) for a in g.amps]
    held, regs = OrderedDict(), OrderedDict()
    remaining = set(range(len(g.amps)))
    order = []
    while remaining:
        best = None
        for i in remaining:
            c = sum(cost[k] for k in closures[i] if k not in held)
            if flow_regs:
                c += flow_cost * sum(1 for w in flows[i] if w not in regs)
            if best is None or (c, i) < best:
                best = (c, i)
        i = best[1]
        order.append(i)
        remaining.discard(i)
        for k in closures[i]:
            held[k] = True
            held.move_to_end(k)
        while len(held) > cache:
            held.popitem(last=False)
        if flow_regs:
            for w in flows[i]:
                regs[w] = True
                regs.move_to_end(w)
            while len(regs) > flow_regs:
                regs.popitem(last=False)
    return order
