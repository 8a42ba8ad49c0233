"""Exact SU(N) colour factors for one quark line, by the Fierz identity.

The matrix element of one quark line with k gluons is a sum over the k!
gluon orderings sigma of (t^{a_sigma1} ... t^{a_sigmak})_{i jbar} A(sigma); its
colour-summed square needs C_{sigma tau} = Tr(t^{sigma_1}..t^{sigma_k} t^{tau_k}..t^{tau_1})
summed over the gluon colours.  Each trace is reduced symbolically with
    t^a_{ij} t^a_{kl} = 1/2 (delta_il delta_kj - 1/N delta_ij delta_kl),
which in trace form reads
    Tr(t^a X t^a Y)     = 1/2 Tr X Tr Y - 1/(2N) Tr(XY)
    Tr(t^a X) Tr(t^a Y) = 1/2 Tr(XY)    - 1/(2N) Tr X Tr Y
with Tr(1) = N.  All arithmetic is in exact rationals.
"""
from fractions import Fraction
from functools import lru_cache
import itertools


def _canon(traces):
    """Canonical form of a product of traces: rotate each word, sort the factors."""
    out = []
    for w in traces:
        if not w:
            out.append(())
            continue
        rots = [w[i:] + w[:i] for i in range(len(w))]
        out.append(min(rots))
    return tuple(sorted(out))


@lru_cache(maxsize=None)
def _eval(traces, N):
    traces = list(traces)
    # pick the first label that still appears
    for ti, w in enumerate(traces):
        if w:
            a = w[0]
            break
    else:
        return Fraction(N) ** len(traces)
    half = Fraction(1, 2)
    invn = Fraction(1, 2 * N)
    # locate both occurrences of a
    occ = [(i, j) for i, w in enumerate(traces) for j, x in enumerate(w) if x == a]
    assert len(occ) == 2
    (i1, j1), (i2, j2) = occ
    rest = [w for k, w in enumerate(traces) if k not in (i1, i2)]
    if i1 == i2:
        w = traces[i1]
        w = w[j1:] + w[:j1]                       # a X a Y with X = w[1:j], Y = w[j+1:]
        j = (j2 - j1) % len(w)
        X, Y = w[1:j], w[j + 1:]
        t1 = _eval(_canon(rest + [X, Y]), N)
        t2 = _eval(_canon(rest + [X + Y]), N)
        return half * t1 - invn * t2
    wa = traces[i1][j1:] + traces[i1][:j1]      # a X
    wb = traces[i2][j2:] + traces[i2][:j2]      # a Y
    X, Y = wa[1:], wb[1:]
    t1 = _eval(_canon(rest + [X + Y]), N)
    t2 = _eval(_canon(rest + [X, Y]), N)
    return half * t1 - invn * t2


def trace(word, N=3):
    """Tr of a product of generators whose labels each occur twice, summed over labels."""
    return _eval(_canon([tuple(word)]), N)


def orderings(k):
    return list(itertools.permutations(range(k)))


def colour_matrix(k, N=3):
    """C[sigma][tau] as Fractions, orderings in lexicographic order."""
    perms = orderings(k)
    return [[trace(list(s) + list(reversed(t)), N) for t in perms] for s in perms]


def integer_form(C):
    """(numerators, common denominator) of a rational matrix."""
    den = 1
    for row in C:
        for v in row:
            den = den * v.denominator // _gcd(den, v.denominator)
    return [[int(v * den) for v in row] for row in C], den


def _gcd(a, b):
    while b:
        a, b = b, a % b
    return a
