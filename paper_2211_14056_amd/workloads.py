"""Seeded synthetic workload descriptions (no physics arithmetic here).

The mixed persistent batch: 64 requests, each a process drawn uniformly from
{gg -> ttbar, gg -> ttbar g, gg -> ttbar gg} and an event count drawn
log-uniformly from that process's range, from numpy's PCG64 generator.
"""
import math

import numpy as np

MIXED_RANGES = {'gg_tt': (1e3, 1e6), 'gg_ttg': (1e4, 4e6), 'gg_ttgg': (1e4, 1e6)}


def mixed_batch(n_requests=64, seed=5, scale=1.0):
    """[(process, n_events)]; `scale` shrinks the counts for small test runs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    procs = list(MIXED_RANGES)
    out = []
    for _ in range(n_requests):
        proc = procs[int(rng.integers(0, len(procs)))]
        lo, hi = MIXED_RANGES[proc]
        n = int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi))) * scale))
        out.append((proc, max(n, 1)))
    return out


# Stand-ins for tabulated parton densities (no PDF grids are available here): the smooth
# toy form  x f(x, Q^2) = A x^(-a(L)) (1 - x)^(b(L)),  L = ln(Q^2 / Q0^2),  a(L) = a0 + a1 L,
# b(L) = b0 + b1 L, Q0^2 = 1.69 GeV^2, tabulated on nodes equally spaced in ln x (x from 1e-6
# to 1) and ln Q^2 (Q^2 from Q0^2 to 1e8 GeV^2), the layout of a grid file.  Only the node
# values enter the computation.  'g' is the gluon, 'q' a light quark (valence-like: vanishing
# at small x), 'qbar' its antiquark (sea-like).
TOY_PDFS = {
    'g': dict(A=1.7, a0=0.18, a1=0.03, b0=5.0, b1=0.4),
    'q': dict(A=0.9, a0=-0.45, a1=0.01, b0=3.2, b1=0.3),
    'qbar': dict(A=0.15, a0=0.16, a1=0.02, b0=7.0, b1=0.4),
}
TOY_PDF = dict(TOY_PDFS['g'], q0sq=1.69, xmin=1e-6, q2max=1e8)
_GRID = dict(q0sq=1.69, xmin=1e-6, q2max=1e8)


def toy_xf(kind, x, q2):
    """The toy form of parton `kind` at (x, Q^2) (numpy arrays)."""
    t = TOY_PDFS[kind]
    L = np.log(q2 / _GRID['q0sq'])
    return t['A'] * x ** (-(t['a0'] + t['a1'] * L)) * (1.0 - x) ** (t['b0'] + t['b1'] * L)


def toy_xg(x, q2):
    """The toy gluon at (x, Q^2)."""
    return toy_xf('g', x, q2)


def toy_pdf_grid(nx=121, nq=61, kind='g'):
    """(ln x nodes [nx], ln Q^2 nodes [nq], x f at the nodes [nq][nx]) of a toy density."""
    lx = np.linspace(np.log(_GRID['xmin']), 0.0, nx)
    lq = np.linspace(np.log(_GRID['q0sq']), np.log(_GRID['q2max']), nq)
    X, Q2 = np.meshgrid(np.exp(lx), np.exp(lq))
    X[:, -1] = 1.0
    return lx, lq, toy_xf(kind, X, Q2)
