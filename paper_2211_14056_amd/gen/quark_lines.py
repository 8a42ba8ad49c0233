"""Generated matrix elements for the processes with two quark lines: q qbar -> t tbar (+g, +gg)
and q g -> t tbar q (+g), a massless light quark of one flavour.

The paper's generated code evaluates each Feynman diagram from external wavefunctions,
vertices and propagators, and sums the diagrams into colour-flow amplitudes contracted with a
colour matrix (sect. 2, Fig. 2).  This module does the same from a process definition:

  diagrams   every tree of QCD vertices (q q g, three- and four-gluon) joining the external
             legs, enumerated over subsets of legs (all momenta incoming).  A subset has a type
             from its fermion numbers per flavour (gluon; column or row spinor of the light
             quark or of the top).  Sub-trees shared between diagrams are evaluated once.
  colour     each diagram's colour tensor (products of t^a and f^abc, every index explicit)
             is decomposed on a basis of products of two generator strings along the two
             quark lines, (t^alpha)_{row_L col_T} (t^beta)_{row_T col_L} and
             (t^alpha)_{row_L col_L} (t^beta)_{row_T col_T}, alpha and beta ordered gluon
             sequences that share out the gluons; the colour matrix is the Gram matrix of the
             basis.  Decomposition and Gram matrix are computed numerically here with explicit
             SU(3) generators, the coefficients identified as small rationals and checked.
  Lorentz    straight-line code (ir.Block) per helicity configuration: off-shell currents
             with the coupling g taken out (every diagram carries g^(n-2)), propagators
             1/(P^2 - m^2) and momentum sums computed once per event in FP64.
  helicities configurations that conserve the chirality of the massless light-quark line, and
             of those the half with the incoming quark at helicity +1; parity supplies the
             other half (the colour-summed |M|^2 is unchanged when every helicity flips).

Conventions (Feynman gauge, all momenta incoming):
  fermion propagator i (pslash + m)/(p^2 - m^2), p along the fermion flow (P for a column
  current, -P for a row current); gluon propagator -i g_{mu nu}/P^2; q q g vertex
  i g gamma^mu t^a; three-gluon g f^{abc}[g^{mu nu}(k-p)^rho + g^{nu rho}(p-q)^mu +
  g^{rho mu}(q-k)^nu]; four-gluon -i g^2 sum over the three f f structures.
"""
import itertools
from fractions import Fraction

import numpy as np

from . import ir
from .ir import C, CZERO, cadd, cmat, cmul, cneg, csum, creal

PROCESSES = {
    'qq_tt': [('q', True), ('qbar', True), ('t', False), ('tbar', False)],
    'qq_ttg': [('q', True), ('qbar', True), ('t', False), ('tbar', False), ('g', False)],
    'qq_ttgg': [('q', True), ('qbar', True), ('t', False), ('tbar', False), ('g', False), ('g', False)],
    'qg_ttq': [('q', True), ('g', True), ('t', False), ('tbar', False), ('q', False)],
    'qg_ttqg': [('q', True), ('g', True), ('t', False), ('tbar', False), ('q', False), ('g', False)],
}
# spin x colour average of the initial state, identical final-state particles
AVERAGE = {'qq': 36.0, 'qg': 96.0}

GLUON, COL, ROW = 'g', 'col', 'row'


# ------------------------------------------------------------------ SU(3)
def _gell_mann():
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


TA = _gell_mann() / 2.0
# f^{abc} = -2 i Tr([t^a, t^b] t^c)
FABC = np.real(-2j * (np.einsum('aij,bjk,cki->abc', TA, TA, TA) - np.einsum('bij,ajk,cki->abc', TA, TA, TA)))


# ------------------------------------------------------------------ process structure
class Leg:
    def __init__(self, i, kind, incoming):
        self.i, self.kind, self.incoming = i, kind, incoming
        if kind == 'g':
            self.type, self.flav = GLUON, None
        else:
            self.flav = 'top' if kind in ('t', 'tbar') else 'light'
            anti = kind in ('tbar', 'qbar')
            self.type = COL if (incoming and not anti) or (not incoming and anti) else ROW

    @property
    def dim(self):
        return 8 if self.type == GLUON else 3


def subset_type(S, legs):
    n = {'light': 0, 'top': 0}
    for i in S:
        L = legs[i]
        if L.type == COL:
            n[L.flav] += 1
        elif L.type == ROW:
            n[L.flav] -= 1
    if n['light'] == 0 and n['top'] == 0:
        return GLUON, None
    for f, o in (('light', 'top'), ('top', 'light')):
        if n[o] == 0 and n[f] in (1, -1):
            return (COL if n[f] == 1 else ROW), f
    return None, None


def _pairs(S):
    first, rest = S[0], S[1:]
    for r in range(len(rest)):
        for extra in itertools.combinations(rest, r):
            A = (first,) + extra
            B = tuple(x for x in S if x not in A)
            if B:
                yield A, B


def _triples(S):
    for A, BC in _pairs(S):
        if len(BC) >= 2:
            for B, C_ in _pairs(BC):
                yield A, B, C_


class Node:
    """One sub-tree: an off-shell current over `legs` made at `vertex` from `children`."""

    def __init__(self, nid, legs, typ, flav, vertex, children, struct=0):
        self.id, self.legs, self.type, self.flav = nid, tuple(legs), typ, flav
        self.vertex, self.children, self.struct = vertex, tuple(children), struct
        self.colour = None


def enumerate_diagrams(proc):
    """(legs, nodes, diagrams): nodes of every sub-tree over subsets of legs 1..n-1, and the
    full diagrams as (row node, gluon node) joined with leg 0 at its q q g vertex."""
    legs = [Leg(i, k, inc) for i, (k, inc) in enumerate(PROCESSES[proc])]
    assert legs[0].type == COL and legs[0].flav == 'light'
    n = len(legs)
    nodes = []
    by_set = {}

    def add(S, typ, flav, vertex, children, struct=0):
        nd = Node(len(nodes), S, typ, flav, vertex, children, struct)
        nodes.append(nd)
        by_set.setdefault(S, []).append(nd)

    rest = tuple(range(1, n))
    for i in rest:
        add((i,), legs[i].type, legs[i].flav, 'ext', ())
    for size in range(2, n):
        for S in itertools.combinations(rest, size):
            typ, flav = subset_type(S, legs)
            if typ is None:
                continue
            for A, B in _pairs(S):
                for a in by_set.get(A, []):
                    for b in by_set.get(B, []):
                        if typ == GLUON:
                            if a.type == GLUON and b.type == GLUON:
                                add(S, typ, flav, 'v3', (a, b))
                            elif a.type == COL and b.type == ROW and a.flav == b.flav:
                                add(S, typ, flav, 'pair', (a, b))
                            elif a.type == ROW and b.type == COL and a.flav == b.flav:
                                add(S, typ, flav, 'pair', (b, a))
                        else:
                            for f_, g_ in ((a, b), (b, a)):
                                if g_.type == GLUON and f_.type == typ and f_.flav == flav:
                                    add(S, typ, flav, typ, (f_, g_))
            if typ == GLUON:
                for A, B, C_ in _triples(S):
                    for a in by_set.get(A, []):
                        for b in by_set.get(B, []):
                            for c in by_set.get(C_, []):
                                if a.type == b.type == c.type == GLUON:
                                    for s in (1, 2, 3):
                                        add(S, typ, flav, 'v4', (a, b, c), s)
    diagrams = []
    for A, B in _pairs(rest):
        for RS, GS in ((A, B), (B, A)):
            for r in by_set.get(RS, []):
                for g_ in by_set.get(GS, []):
                    if r.type == ROW and r.flav == 'light' and g_.type == GLUON:
                        diagrams.append((r, g_))
    # diagrams that share a row sub-tree next to each other: its value is live for a shorter span
    diagrams.sort(key=lambda rg: (rg[0].id, rg[1].id))
    return legs, nodes, diagrams


# ------------------------------------------------------------------ colour
def _sorted_axes(T, legs_in):
    """T[..legs_in.., open] -> axes in sorted leg order (open index last)."""
    order = sorted(range(len(legs_in)), key=lambda k: legs_in[k])
    return np.transpose(T, order + [len(legs_in)]), tuple(sorted(legs_in))


def node_colour(nd, legs):
    if nd.colour is not None:
        return nd.colour
    if nd.vertex == 'ext':
        d = legs[nd.legs[0]].dim
        nd.colour = np.eye(d, dtype=np.complex128)
        return nd.colour
    ch = [node_colour(c, legs) for c in nd.children]
    L = [c.legs for c in nd.children]
    if nd.vertex == 'pair':                    # psi (col, open j), chi (row, open i): chi_i t^a_ij psi_j
        T = np.einsum('...j,aij->...ia', ch[0], TA)                          # [Lc..., i, a]
        T = np.tensordot(T, ch[1], axes=([T.ndim - 2], [ch[1].ndim - 1]))    # [Lc..., a, Lr...]
        T = np.moveaxis(T, len(L[0]), -1)                                    # [Lc..., Lr..., a]
        legs_in = L[0] + L[1]
    elif nd.vertex == 'v3':                    # f^{abc} X_b Y_c
        T = np.einsum('abc,...b->...ac', FABC, ch[0])
        T = np.tensordot(T, ch[1], axes=([T.ndim - 1], [ch[1].ndim - 1]))    # [La..., a, Lb...]
        T = np.moveaxis(T, len(L[0]), -1)
        legs_in = L[0] + L[1]
    elif nd.vertex == 'v4':
        ff = {1: np.einsum('abe,cde->abcd', FABC, FABC), 2: np.einsum('ace,bde->abcd', FABC, FABC),
              3: np.einsum('ade,bce->abcd', FABC, FABC)}[nd.struct]
        T = np.tensordot(ch[0], ff, axes=([ch[0].ndim - 1], [1]))           # [La..., a, c, d]
        T = np.tensordot(T, ch[1], axes=([T.ndim - 2], [ch[1].ndim - 1]))    # [La..., a, d, Lb...]
        nb = len(L[1])
        T = np.moveaxis(T, len(L[0]) + 1, -1)                                # [La..., a, Lb..., d]
        T = np.tensordot(T, ch[2], axes=([T.ndim - 1], [ch[2].ndim - 1]))    # [La..., a, Lb..., Lc...]
        T = np.moveaxis(T, len(L[0]), -1)
        legs_in = L[0] + L[1] + L[2]
    elif nd.vertex == COL:                     # t^a_ij X_j  (X col, G gluon)
        T = np.einsum('aij,...j->...ia', TA, ch[0])                          # [Lf..., i, a]
        T = np.tensordot(T, ch[1], axes=([T.ndim - 1], [ch[1].ndim - 1]))    # [Lf..., i, Lg...]
        T = np.moveaxis(T, len(L[0]), -1)
        legs_in = L[0] + L[1]
    elif nd.vertex == ROW:                     # X_i t^a_ij
        T = np.einsum('...i,aij->...ja', ch[0], TA)
        T = np.tensordot(T, ch[1], axes=([T.ndim - 1], [ch[1].ndim - 1]))
        T = np.moveaxis(T, len(L[0]), -1)
        legs_in = L[0] + L[1]
    else:
        raise ValueError(nd.vertex)
    T, srt = _sorted_axes(T, legs_in)
    assert srt == nd.legs
    nd.colour = T
    return T


def diagram_colour(r, g_, legs):
    """Full colour tensor [leg 0, legs 1..n-1] of leg 0 (column, index j) joined to row r
    (open i) and gluon g (open a): X_i t^a_ij delta_j,c0 Y_a."""
    X, Y = node_colour(r, legs), node_colour(g_, legs)
    T = np.einsum('...i,aij->...ja', X, TA)                                  # [Lr..., j, a]
    T = np.tensordot(T, Y, axes=([T.ndim - 1], [Y.ndim - 1]))                # [Lr..., j, Lg...]
    T = np.moveaxis(T, len(r.legs), 0)                                       # [j = leg 0, Lr..., Lg...]
    T, srt = _sorted_axes(np.moveaxis(T, 0, -1), list(r.legs) + list(g_.legs))   # open = leg 0 last
    return np.moveaxis(T, -1, 0)                                             # [leg 0, legs 1..n-1]


def colour_basis(legs):
    """Basis tensors [leg 0, ..., leg n-1] and their labels."""
    n = len(legs)
    rowL = [L.i for L in legs if L.flav == 'light' and L.type == ROW][0]
    rowT = [L.i for L in legs if L.flav == 'top' and L.type == ROW][0]
    colT = [L.i for L in legs if L.flav == 'top' and L.type == COL][0]
    glu = [L.i for L in legs if L.type == GLUON]
    basis, labels = [], []
    for k in range(len(glu) + 1):
        for alpha in itertools.permutations(glu, k):
            rem = [x for x in glu if x not in alpha]
            for beta in itertools.permutations(rem):
                for kind in ('cross', 'self'):
                    basis.append(_basis_tensor(legs, alpha, beta, kind, rowL, rowT, colT))
                    labels.append((kind, alpha, tuple(beta)))
    return basis, labels


def _basis_tensor(legs, alpha, beta, kind, rowL, rowT, colT):
    """(t^alpha)_{rowL X} (t^beta)_{rowT Y} with (X, Y) = (colT, col0) for 'cross' and
    (col0, colT) for 'self', as an explicit tensor over all legs."""
    n = len(legs)
    dims = [L.dim for L in legs]
    letters = 'abcdefgh'
    # einsum: string alpha from rowL to X, string beta from rowT to Y
    ops, subs = [], []
    idx = {L.i: letters[L.i] for L in legs}
    X, Y = (colT, 0) if kind == 'cross' else (0, colT)
    inner = iter('pqrstuvw')

    def chain(start, seq, end):
        cur = idx[start]
        for gl in seq:
            nxt = next(inner)
            ops.append(TA)
            subs.append(idx[gl] + cur + nxt)
            cur = nxt
        ops.append(np.eye(3))
        subs.append(cur + idx[end])

    chain(rowL, alpha, X)
    chain(rowT, beta, Y)
    out = ''.join(idx[i] for i in range(n))
    T = np.einsum(','.join(subs) + '->' + out, *ops)
    assert list(T.shape) == dims
    return T


def _rational(x, tol=1e-12):
    fr = Fraction(x).limit_denominator(10000)
    return fr if abs(float(fr) - x) <= tol * max(1.0, abs(x)) else None


def _crational(z):
    a, b = _rational(z.real), _rational(z.imag)
    assert a is not None and b is not None, z
    return a, b


def decompose(proc):
    """Diagrams, basis labels, coefficient matrix c[r][d] (exact complex rationals as
    (re, im) Fractions) and the colour matrix G (Fractions)."""
    legs, nodes, diagrams = enumerate_diagrams(proc)
    basis, labels = colour_basis(legs)
    Bm = np.stack([b.reshape(-1) for b in basis], 1)                       # [colours, NB]
    # drop basis elements dependent on earlier ones
    keep, Q = [], np.zeros((Bm.shape[0], 0), dtype=np.complex128)
    for j in range(Bm.shape[1]):
        v = Bm[:, j]
        r = v - Q @ (Q.conj().T @ v) if Q.shape[1] else v
        if np.linalg.norm(r) > 1e-9 * np.linalg.norm(v):
            keep.append(j)
            Q = np.concatenate([Q, (r / np.linalg.norm(r))[:, None]], 1)
    Bm = Bm[:, keep]
    labels = [labels[j] for j in keep]
    coeff = []
    for r, g_ in diagrams:
        T = diagram_colour(r, g_, legs).reshape(-1)
        c, *_ = np.linalg.lstsq(Bm, T, rcond=None)
        assert np.linalg.norm(Bm @ c - T) <= 1e-10 * max(1.0, np.linalg.norm(T)), 'colour not in the basis'
        coeff.append([_crational(z) for z in c])
    Gn = Bm.conj().T @ Bm
    assert np.abs(Gn.imag).max() < 1e-12 and np.abs(Gn - Gn.T).max() < 1e-12
    G = [[_rational(float(Gn[i, j].real)) for j in range(len(keep))] for i in range(len(keep))]
    assert all(x is not None for row in G for x in row)
    return legs, nodes, diagrams, labels, coeff, G


def helicity_configs(legs):
    """Helicity configurations evaluated: chirality conserved along the massless line, the
    incoming quark at +1 (parity gives the rest)."""
    rowL = [L.i for L in legs if L.flav == 'light' and L.type == ROW][0]
    out = []
    for h in itertools.product((-1, 1), repeat=len(legs)):
        if h[0] != 1:
            continue
        # column u(+) of the incoming quark: an incoming antiquark row vbar carries -h0,
        # an outgoing quark row ubar carries +h0
        need = -h[0] if legs[rowL].incoming else h[0]
        if h[rowL] != need:
            continue
        out.append(h)
    return out


# ------------------------------------------------------------------ Lorentz code
def _lc(b, J):
    """(J0+J3, J0-J3, J1+iJ2, J1-iJ2) for a complex vector J."""
    Jp = cadd(b, J[0], J[3])
    Jm = C(b.sub(J[0].re, J[3].re), b.sub(J[0].im, J[3].im))
    iJ2 = C(b.neg(J[2].im), J[2].re)
    Jt = cadd(b, J[1], iJ2)
    Jtb = C(b.sub(J[1].re, iJ2.re), b.sub(J[1].im, iJ2.im))
    return Jp, Jm, Jt, Jtb


def slash_col(b, J, psi):
    """Jslash psi (chiral representation)."""
    Jp, Jm, Jt, Jtb = _lc(b, J)
    return [csum(b, [(Jm, psi[2]), (cneg(b, Jtb), psi[3])]), csum(b, [(cneg(b, Jt), psi[2]), (Jp, psi[3])]),
            csum(b, [(Jp, psi[0]), (Jtb, psi[1])]), csum(b, [(Jt, psi[0]), (Jm, psi[1])])]


def slash_row(b, chi, J):
    """chi Jslash."""
    Jp, Jm, Jt, Jtb = _lc(b, J)
    return [csum(b, [(chi[2], Jp), (chi[3], Jt)]), csum(b, [(chi[2], Jtb), (chi[3], Jm)]),
            csum(b, [(chi[0], Jm), (cneg(b, chi[1]), Jt)]), csum(b, [(cneg(b, chi[0]), Jtb), (chi[1], Jp)])]


def current(b, chi, psi):
    """chi gamma^mu psi, upper index."""
    cp = csum(b, [(chi[1], psi[3]), (chi[2], psi[0])])
    cm = csum(b, [(chi[0], psi[2]), (chi[3], psi[1])])
    ct = csum(b, [(cneg(b, chi[1]), psi[2]), (chi[3], psi[0])])
    ctb = csum(b, [(cneg(b, chi[0]), psi[3]), (chi[2], psi[1])])
    J0 = cadd(b, cp, cm)
    J3 = C(b.sub(cm.re, cp.re), b.sub(cm.im, cp.im))
    J1 = cneg(b, cadd(b, ct, ctb))
    d = C(b.sub(ct.re, ctb.re), b.sub(ct.im, ctb.im))            # J2 = -i (ct - ctb)
    J2 = C(d.im, b.neg(d.re))
    return [J0, J1, J2, J3]


def mdot(b, x, y):
    return csum(b, [(x[0], y[0]), (cneg(b, x[1]), y[1]), (cneg(b, x[2]), y[2]), (cneg(b, x[3]), y[3])])


def cscale_r(b, x, s):
    return C(b.mul(x.re, s), b.mul(x.im, s))


def times_i(b, x):
    return C(b.neg(x.im), x.re)


class Emitter:
    """Straight-line code for one helicity configuration of one process."""

    def __init__(self, proc, legs, nodes, diagrams, labels, coeff, G):
        self.proc, self.legs, self.nodes, self.diagrams = proc, legs, nodes, diagrams
        self.labels, self.coeff, self.G = labels, coeff, G
        # every leg subset of a node (singletons too: the three-gluon vertex needs the momenta
        # of external gluons); K holds its incoming momentum sum and 1/(P^2 - m^2)
        self.subsets = sorted({nd.legs for nd in nodes}, key=lambda s: (len(s), s))
        self.sidx = {S: i for i, S in enumerate(self.subsets)}

    def kin_ref(self, b, S, c):
        # K[5 s + c]: c = 0..3 incoming momentum sum, 4 = 1/(P^2 - m^2) of the subset's type
        return b.var(f'K[{5 * self.sidx[S] + c}]')

    def P(self, b, S):
        return [creal(self.kin_ref(b, S, c)) for c in range(4)]

    def body(self):
        """Straight-line code of one helicity configuration.  Sub-trees are emitted when a
        diagram first needs them (so their live ranges start late) and every diagram is folded
        into the colour-flow amplitudes as soon as it is formed (so no diagram stays live)."""
        b = ir.Block('t')
        legs = self.legs
        W = {}
        for L in legs:
            W[L.i] = [C(b.var(f'W[{4 * L.i + c}].re'), b.var(f'W[{4 * L.i + c}].im')) for c in range(4)]
        val = {}
        mass = {'light': None, 'top': b.var('mt')}

        def value(nd):
            if nd.id in val:
                return val[nd.id]
            if nd.vertex == 'ext':
                val[nd.id] = W[nd.legs[0]]
                return val[nd.id]
            for c in nd.children:
                value(c)
            ch = [val[c.id] for c in nd.children]
            inv = self.kin_ref(b, nd.legs, 4)
            if nd.vertex == 'pair':
                J = current(b, ch[1], ch[0])
                out = [cscale_r(b, x, inv) for x in J]
            elif nd.vertex == 'v3':
                A, B = nd.children
                p, q = self.P(b, A.legs), self.P(b, B.legs)
                JA, JB = ch
                # k = -(p + q): k - p = -(2p + q), p - q, q - k = p + 2q
                kmp = [C(b.neg(b.add(b.add(p[c].re, p[c].re), q[c].re)), ir.ZERO) for c in range(4)]
                pmq = [C(b.sub(p[c].re, q[c].re), ir.ZERO) for c in range(4)]
                qmk = [C(b.add(p[c].re, b.add(q[c].re, q[c].re)), ir.ZERO) for c in range(4)]
                a1 = cmat(b, mdot(b, kmp, JB))
                a2 = cmat(b, mdot(b, JA, JB))
                a3 = cmat(b, mdot(b, qmk, JA))
                V = [csum(b, [(JA[c], a1), (pmq[c], a2), (JB[c], a3)]) for c in range(4)]
                # (-i) V / P^2
                out = [cscale_r(b, C(V[c].im, b.neg(V[c].re)), inv) for c in range(4)]
            elif nd.vertex == 'v4':
                Jb, Jc, Jd = ch
                if nd.struct == 1:                   # Jc (Jb.Jd) - Jd (Jb.Jc)
                    x, y = cmat(b, mdot(b, Jb, Jd)), cmat(b, mdot(b, Jb, Jc))
                    L4 = [csum(b, [(Jc[c], x), (cneg(b, Jd[c]), y)]) for c in range(4)]
                elif nd.struct == 2:                 # Jb (Jc.Jd) - Jd (Jb.Jc)
                    x, y = cmat(b, mdot(b, Jc, Jd)), cmat(b, mdot(b, Jb, Jc))
                    L4 = [csum(b, [(Jb[c], x), (cneg(b, Jd[c]), y)]) for c in range(4)]
                else:                                # Jb (Jc.Jd) - Jc (Jb.Jd)
                    x, y = cmat(b, mdot(b, Jc, Jd)), cmat(b, mdot(b, Jb, Jd))
                    L4 = [csum(b, [(Jb[c], x), (cneg(b, Jc[c]), y)]) for c in range(4)]
                out = [cscale_r(b, cneg(b, L4[c]), inv) for c in range(4)]
            elif nd.vertex == COL:                  # -(P + m)(Jslash psi) / (P^2 - m^2)
                psi, J = ch
                x = [cmat(b, v) for v in slash_col(b, J, psi)]
                out = self._prop_col(b, nd, x, inv, mass[nd.flav])
            elif nd.vertex == ROW:                  # -(chi Jslash)(-P + m) / (P^2 - m^2)
                chi, J = ch
                x = [cmat(b, v) for v in slash_row(b, chi, J)]
                out = self._prop_row(b, nd, x, inv, mass[nd.flav])
            else:
                raise ValueError(nd.vertex)
            val[nd.id] = [cmat(b, v) for v in out]
            return val[nd.id]

        nb = len(self.labels)
        jamp = [None] * nb
        for d, (r, g_) in enumerate(self.diagrams):
            chiJ = slash_row(b, value(r), value(g_))
            amp = csum(b, [(chiJ[s_], W[0][s_]) for s_ in range(4)])
            D = cmat(b, times_i(b, amp))                    # i (chi Jslash u0)
            for rr in range(nb):
                re, im = self.coeff[d][rr]
                if re == 0 and im == 0:
                    continue
                term = [(C(ir.const(float(re)), ir.const(float(im))), D)]
                jamp[rr] = cmat(b, csum(b, term, jamp[rr]))
        jamp = [x if x is not None else CZERO for x in jamp]
        tot = []
        for i in range(nb):
            y_re, y_im = [], []
            for j in range(nb):
                g = self.G[i][j]
                if g == 0:
                    continue
                y_re.append((ir.const(float(g)), jamp[j].re))
                y_im.append((ir.const(float(g)), jamp[j].im))
            yr, yi = b.sumprod(y_re), b.sumprod(y_im)
            tot += [(jamp[i].re, yr), (jamp[i].im, yi)]
        res = b.sumprod(tot)
        return b, res

    def _prop_col(self, b, nd, x, inv, m):
        P = self.P(b, nd.legs)
        Pp = b.add(P[0].re, P[3].re)
        Pm = b.sub(P[0].re, P[3].re)
        Pt = C(P[1].re, P[2].re)
        Ptb = C(P[1].re, b.neg(P[2].re))
        # Pslash x = (Pm x2 - Ptb x3, -Pt x2 + Pp x3, Pp x0 + Ptb x1, Pt x0 + Pm x1)
        y = [csum(b, [(creal(Pm), x[2]), (cneg(b, Ptb), x[3])]), csum(b, [(cneg(b, Pt), x[2]), (creal(Pp), x[3])]),
             csum(b, [(creal(Pp), x[0]), (Ptb, x[1])]), csum(b, [(Pt, x[0]), (creal(Pm), x[1])])]
        if m is not None:
            y = [cadd(b, y[s], C(b.mul(m, x[s].re), b.mul(m, x[s].im))) for s in range(4)]
        ninv = b.neg(inv)
        return [cscale_r(b, y[s], ninv) for s in range(4)]

    def _prop_row(self, b, nd, x, inv, m):
        P = self.P(b, nd.legs)
        # x (-Pslash + m): row times slash of -P
        Pp = b.add(P[0].re, P[3].re)
        Pm = b.sub(P[0].re, P[3].re)
        Pt = C(P[1].re, P[2].re)
        Ptb = C(P[1].re, b.neg(P[2].re))
        # x Pslash = (x2 Pp + x3 Pt, x2 Ptb + x3 Pm, x0 Pm - x1 Pt, -x0 Ptb + x1 Pp)
        y = [csum(b, [(x[2], creal(Pp)), (x[3], Pt)]), csum(b, [(x[2], Ptb), (x[3], creal(Pm))]),
             csum(b, [(x[0], creal(Pm)), (cneg(b, x[1]), Pt)]), csum(b, [(cneg(b, x[0]), Ptb), (x[1], creal(Pp))])]
        y = [cneg(b, v) for v in y]
        if m is not None:
            y = [cadd(b, y[s], C(b.mul(m, x[s].re), b.mul(m, x[s].im))) for s in range(4)]
        ninv = b.neg(inv)
        return [cscale_r(b, y[s], ninv) for s in range(4)]


def emit(proc):
    """C++ source for one process and its summary (diagram and basis counts, flops)."""
    legs, nodes, diagrams, labels, coeff, G = decompose(proc)
    em = Emitter(proc, legs, nodes, diagrams, labels, coeff, G)
    b, res = em.body()
    hels = helicity_configs(legs)
    n = len(legs)
    name = f'me_{proc}'
    avg = AVERAGE[proc[:2]]
    ng = sum(1 for L in legs[2:] if L.type == GLUON and not L.incoming)
    sym = 2.0 if ng == 2 else 1.0
    # leg kinds: 0 u (in quark), 1 vbar (in antiquark), 2 ubar (out quark), 3 v (out antiquark),
    # 4 eps (in gluon), 5 eps* (out gluon)
    kinds = []
    for Lg in legs:
        if Lg.type == GLUON:
            kinds.append(4 if Lg.incoming else 5)
        elif Lg.type == COL:
            kinds.append(0 if Lg.incoming else 3)
        else:
            kinds.append(1 if Lg.incoming else 2)
    masks, tops = [], []
    for S in em.subsets:
        masks.append(sum(1 << i for i in S))
        typ, flav = subset_type(S, legs)
        tops.append(1 if flav == 'top' else 0)
    ns = len(em.subsets)
    L = [f'// {proc}: {len(diagrams)} Feynman diagrams ({len(nodes) - (n - 1)} sub-trees), '
         f'{len(labels)} colour-flow amplitudes, {len(hels)} helicity configurations evaluated',
         f'static __constant__ const signed char {name}_hel[{len(hels)}][{n}] = {{'
         + ', '.join('{' + ', '.join(str(x) for x in h) + '}' for h in hels) + '};',
         'namespace mf {',
         f'struct QL_{proc} {{',
         f'    static constexpr int NEXT = {n}, NSUB = {ns}, NHEL = {len(hels)};',
         f'    static constexpr double NORM = {2.0 / (avg * sym)!r};   // parity x 1 / (average x symmetry)',
         '    // leg kinds: 0 u (in quark), 1 vbar (in antiquark), 2 ubar (out quark), 3 v (out antiquark),',
         '    // 4 eps (in gluon), 5 eps* (out gluon); the top legs are massive',
         f'    static constexpr int KIND[{n}] = {{' + ', '.join(str(k) for k in kinds) + '};',
         f'    static constexpr bool MASSIVE[{n}] = {{'
         + ', '.join('true' if Lg.flav == 'top' else 'false' for Lg in legs) + '};',
         '    // leg subsets of the off-shell currents: K[5 s .. 5 s + 3] = incoming momentum sum,',
         '    // K[5 s + 4] = 1/(P^2 - m^2) with m = m_t for a top current',
         f'    static constexpr int SUB_MASK[{ns}] = {{' + ', '.join(map(str, masks)) + '};',
         f'    static constexpr bool SUB_TOP[{ns}] = {{' + ', '.join('true' if t else 'false' for t in tops) + '};',
         f'    __device__ static __forceinline__ int hel(int h, int l) {{ return {name}_hel[h][l]; }}',
         '    template <typename R>',
         '    __device__ static __forceinline__ R body(const cplx<R>* W, const R* K, R mt)',
         '    {']
    L += ['        ' + x for x in b.lines]
    L.append(f'        return {b.ref(res)};')
    L += ['    }', '};', '}  // namespace mf']
    summary = dict(diagrams=len(diagrams), subtrees=len(nodes) - (n - 1), colour_flows=len(labels),
                   helicities=len(hels), flops_per_hel=b.flops, per_event=b.flops * len(hels))
    return '\n'.join(L) + '\n', summary
