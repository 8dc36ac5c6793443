"""Exact SU(3) colour algebra for one quark line with n gluons.

Colour basis: the ordered products (T^{a_s1} ... T^{a_sn})_{i j}, one per ordering
s of the gluons, read from the outgoing quark (row index i) to the outgoing
antiquark (column index j).  A colour factor is a polynomial in non-commuting
letters (gluon labels) with Gaussian-integer coefficients; f^{abc} contracted
into a generator becomes a commutator, f^{abc} T^c = -i [T^a, T^b], so every
Feynman diagram maps to such a polynomial.  These jamp coefficients feed the
colour-flow amplitudes (the paper's "jamps", section "Parallel scattering
amplitudes").

The colour matrix C(s, t) = sum over colours of (T..T)_s conj((T..T)_t)
= Tr(T^{s1} .. T^{sn} T^{tn} .. T^{t1}) is computed exactly with the Fierz
identity T^a_{ij} T^a_{kl} = 1/2 (d_il d_kj - 1/N d_ij d_kl), N = 3, as
fractions.  The paper's colour algebra contracts colour-ordered amplitudes with
this integer-over-denominator matrix (section "Numerical stability").
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction
from functools import lru_cache

NC = 3


class Gauss:
    """Gaussian integer a + b i (exact)."""

    __slots__ = ("re", "im")

    def __init__(self, re: int = 0, im: int = 0):
        self.re = re
        self.im = im

    def __add__(self, o):
        return Gauss(self.re + o.re, self.im + o.im)

    def __sub__(self, o):
        return Gauss(self.re - o.re, self.im - o.im)

    def __mul__(self, o):
        if isinstance(o, int):
            return Gauss(self.re * o, self.im * o)
        return Gauss(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    __rmul__ = __mul__

    def __neg__(self):
        return Gauss(-self.re, -self.im)

    def __eq__(self, o):
        return self.re == o.re and self.im == o.im

    def __hash__(self):
        return hash((self.re, self.im))

    def iszero(self):
        return self.re == 0 and self.im == 0

    def __repr__(self):
        return f"({self.re}{self.im:+d}i)"

    def complex(self):
        return complex(self.re, self.im)


ONE = Gauss(1, 0)
I = Gauss(0, 1)
MINUS_I = Gauss(0, -1)


class Poly:
    """Linear combination of words (tuples of gluon labels) with Gaussian-integer coefficients."""

    __slots__ = ("terms",)

    def __init__(self, terms=None):
        self.terms = {}
        if terms:
            for w, c in terms.items():
                if not c.iszero():
                    self.terms[w] = c

    @staticmethod
    def letter(k):
        return Poly({(k,): ONE})

    @staticmethod
    def unit():
        return Poly({(): ONE})

    def __add__(self, o):
        t = dict(self.terms)
        for w, c in o.terms.items():
            t[w] = t[w] + c if w in t else c
        return Poly(t)

    def __sub__(self, o):
        return self + o.scale(Gauss(-1, 0))

    def scale(self, g: Gauss):
        return Poly({w: c * g for w, c in self.terms.items()})

    def __mul__(self, o):
        t = {}
        for w1, c1 in self.terms.items():
            for w2, c2 in o.terms.items():
                w = w1 + w2
                c = c1 * c2
                t[w] = t[w] + c if w in t else c
        return Poly(t)

    def comm(self, o):
        return self * o - o * self

    def __repr__(self):
        return " + ".join(f"{c}*{''.join(map(str, w))}" for w, c in sorted(self.terms.items()))


# ------------------------------------------------------------------ traces


def _canon_trace(word):
    """Canonical cyclic rotation of a trace word (tuple)."""
    if not word:
        return ()
    n = len(word)
    return min(word[i:] + word[:i] for i in range(n))


def _canon_product(traces):
    return tuple(sorted(_canon_trace(t) for t in traces))


@lru_cache(maxsize=None)
def _eval_traces(traces) -> Fraction:
    """Sum over all colour indices of a product of traces in which each label appears twice."""
    traces = list(traces)
    # empty traces give N
    value = Fraction(1)
    rest = []
    for t in traces:
        if len(t) == 0:
            value *= NC
        elif len(t) == 1:
            return Fraction(0)  # Tr T^a = 0
        else:
            rest.append(t)
    if not rest:
        return value
    t0 = rest[0]
    a = t0[0]
    # find the partner of the first letter
    for k in range(1, len(t0)):
        if t0[k] == a:
            A, B = t0[1:k], t0[k + 1:]
            # Tr(T^a A T^a B) = 1/2 [Tr(A) Tr(B) - 1/N Tr(A B)]
            t1 = _canon_product(rest[1:] + [A, B])
            t2 = _canon_product(rest[1:] + [A + B])
            return value * (Fraction(1, 2) * _eval_traces(t1) - Fraction(1, 2 * NC) * _eval_traces(t2))
    for j in range(1, len(rest)):
        t1 = rest[j]
        if a in t1:
            k = t1.index(a)
            A = t0[1:]
            B = t1[k + 1:] + t1[:k]
            others = rest[1:j] + rest[j + 1:]
            # Tr(T^a A) Tr(T^a B) = 1/2 [Tr(A B) - 1/N Tr(A) Tr(B)]
            p1 = _canon_product(others + [A + B])
            p2 = _canon_product(others + [A, B])
            return value * (Fraction(1, 2) * _eval_traces(p1) - Fraction(1, 2 * NC) * _eval_traces(p2))
    raise ValueError("colour label appears only once")


def orderings(gluons):
    """All orderings of the gluon labels, lexicographic."""
    return list(itertools.permutations(sorted(gluons)))


def colour_matrix(gluons):
    """Exact colour matrix over the ordering basis: list of lists of Fractions."""
    basis = orderings(gluons)
    C = []
    for s in basis:
        row = []
        for t in basis:
            word = tuple(s) + tuple(reversed(t))
            row.append(_eval_traces(_canon_product([word])))
        C.append(row)
    return basis, C


def integer_form(C):
    """Write C = N / D with integer numerators N and the smallest common denominator D."""
    D = 1
    for row in C:
        for x in row:
            D = D * x.denominator // math.gcd(D, x.denominator)
    N = [[int(x * D) for x in row] for row in C]
    return N, D
