"""Tree-level |M|^2 with explicit colour for processes with two quark lines.  Test infrastructure only.

The quark-initiated parts of pp -> t tbar (+ jets) (the paper's workload, sect. 3, Table 1):
q qbar -> t tbar (+ g, + g g) and q g -> t tbar q (+ g), with a massless light quark q of one
flavour and the massive top.  Definition: the sum of all tree Feynman diagrams of QCD in
Feynman gauge with the rules of me_explicit (Peskin & Schroeder, Fig. 16.7), every colour
index explicit, ME = (1/avg)(1/S) sum over helicities and colours of |M|^2.

Organisation (each diagram counted exactly once).  All momenta are taken incoming
(k = p for incoming legs, -p for outgoing ones).  Every leg has a type: a gluon, or an end
of a fermion line of flavour light or top that is a column spinor (incoming quark u(p),
outgoing antiquark v(p): fermion number +1) or a row spinor (incoming antiquark vbar(p),
outgoing quark ubar(p): fermion number -1).  A subset S of legs carries fermion numbers
(n_light, n_top); it defines an off-shell current of type gluon for (0, 0), column or row
spinor of a flavour for +-1 of that flavour and 0 of the other, and none otherwise.  A
current is the sum over the unordered splits of S into blocks whose types meet at a QCD
vertex (gluon: two gluons, three gluons, or a column and a row of one flavour; column or
row: the same kind of fermion current and a gluon), times the propagator of its type.
The amplitude is the vertex of leg 0 (an incoming light quark, column u) with the split of
all other legs into a light row current and a gluon current.

Propagators and vertices (momenta along the fermion flow: P for a column current, -P for a
row current, P its incoming momentum sum):
  fermion  i (pslash + m)/(p^2 - m^2);   gluon  -i g_{mu nu} delta^{ab} / P^2;
  q q g    i g gamma^mu t^a;  three- and four-gluon vertices as in me_explicit.
Currents carry one explicit colour index per external leg in them (3 for quarks, 8 for
gluons) plus the open index of their off-shell leg.
"""
import itertools

import torch

from . import colour
from .kinematics import mdot
from .processes import PROCESSES, g_strong, helicities
from .wavefunctions import GAMMA, bar, polarisation, u_spinor, v_spinor

C128 = torch.complex128
TA = torch.tensor(colour.T, dtype=C128)                  # t^a_{ij}
FABC = torch.tensor(colour.F, dtype=C128)                # f^{abc}
_FF1 = torch.einsum('abe,cde->abcd', FABC, FABC)
_FF2 = torch.einsum('ace,bde->abcd', FABC, FABC)
_FF3 = torch.einsum('ade,bce->abcd', FABC, FABC)
METRIC = torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=C128)
LEG = 'ABCDEFGH'                                         # colour index letter of leg i

GLUON, COL, ROW = 'g', 'col', 'row'


class Current:
    """T[z, colour of each leg in `legs` (sorted), open colour, 4]; type, flavour, P [z, 4]."""

    def __init__(self, legs, kind, flav, T, P):
        self.legs, self.kind, self.flav, self.T, self.P = tuple(legs), kind, flav, T, P

    @property
    def e(self):
        return ''.join(LEG[l] for l in self.legs)


def _out(*cs):
    return ''.join(LEG[l] for l in sorted(itertools.chain(*(c.legs for c in cs))))


def _lower(J):
    return J * METRIC


def _gluon_from_pair(col, row, g):
    """i g rowbar gamma^mu t^a col: [z, ext, a, mu]."""
    e1, e2, eo = col.e, row.e, _out(col, row)
    X = torch.einsum(f'z{e2}is,mst->z{e2}imt', row.T, GAMMA)
    Y = torch.einsum(f'aij,z{e1}jt->z{e1}ait', TA, col.T)
    return 1j * g * torch.einsum(f'z{e2}imt,z{e1}ait->z{eo}am', X, Y)


def _v3(c1, c2, g):
    k = -(c1.P + c2.P)
    X, Y, Z = (k - c1.P).to(C128), (c1.P - c2.P).to(C128), (c2.P - k).to(C128)
    e1, e2, eo = c1.e, c2.e, _out(c1, c2)
    XJ2 = torch.einsum(f'zm,z{e2}cm->z{e2}c', X * METRIC, c2.T)
    ZJ1 = torch.einsum(f'zm,z{e1}bm->z{e1}b', Z * METRIC, c1.T)
    J1J2 = torch.einsum(f'z{e1}bm,z{e2}cm->z{e1}{e2}bc', _lower(c1.T), c2.T)
    t1 = torch.einsum(f'z{e1}acm,z{e2}c->z{eo}am', torch.einsum(f'abc,z{e1}bm->z{e1}acm', FABC, c1.T), XJ2)
    t2 = torch.einsum(f'z{e1}{e2}a,zm->z{eo}am', torch.einsum(f'abc,z{e1}{e2}bc->z{e1}{e2}a', FABC, J1J2), Y)
    t3 = torch.einsum(f'z{e2}abm,z{e1}b->z{eo}am', torch.einsum(f'abc,z{e2}cm->z{e2}abm', FABC, c2.T), ZJ1)
    return g * (t1 + t2 + t3)


def _v4(c1, c2, c3, g):
    e1, e2, e3, eo = c1.e, c2.e, c3.e, _out(c1, c2, c3)
    D12 = torch.einsum(f'z{e1}bm,z{e2}cm->z{e1}{e2}bc', _lower(c1.T), c2.T)
    D13 = torch.einsum(f'z{e1}bm,z{e3}dm->z{e1}{e3}bd', _lower(c1.T), c3.T)
    D23 = torch.einsum(f'z{e2}cm,z{e3}dm->z{e2}{e3}cd', _lower(c2.T), c3.T)
    G1, G2, G3 = _FF2 + _FF3, _FF1 - _FF3, -_FF1 - _FF2
    H1 = torch.einsum(f'abcd,z{e2}{e3}cd->z{e2}{e3}ab', G1, D23)
    H2 = torch.einsum(f'abcd,z{e1}{e3}bd->z{e1}{e3}ac', G2, D13)
    H3 = torch.einsum(f'abcd,z{e1}{e2}bc->z{e1}{e2}ad', G3, D12)
    t1 = torch.einsum(f'z{e2}{e3}ab,z{e1}bm->z{eo}am', H1, c1.T)
    t2 = torch.einsum(f'z{e1}{e3}ac,z{e2}cm->z{eo}am', H2, c2.T)
    t3 = torch.einsum(f'z{e1}{e2}ad,z{e3}dm->z{eo}am', H3, c3.T)
    return -1j * g * g * (t1 + t2 + t3)


def _slash_gluon(J):
    """gamma_mu J^{a mu}: [z, ext, a, s, t]"""
    return torch.einsum('...m,mst->...st', _lower(J), GAMMA)


def _fermion_prop(p, m):
    """i (pslash + m) / (p^2 - m^2): [z, s, t]"""
    den = (mdot(p, p) - m * m).to(C128)
    num = torch.einsum('zm,mst->zst', p.to(C128) * METRIC, GAMMA) + m * torch.eye(4, dtype=C128)
    return 1j * num / den.view(-1, 1, 1)


def _col_from(col, glu, g, m):
    """S(P) (i g Jslash t^a) psi: [z, ext, i, s]"""
    e1, e2, eo = col.e, glu.e, _out(col, glu)
    Js = _slash_gluon(glu.T)                                              # [z, e2, a, s, t]
    Y = torch.einsum(f'aij,z{e1}jt->z{e1}ait', TA, col.T)
    v = 1j * g * torch.einsum(f'z{e2}ast,z{e1}ait->z{eo}is', Js, Y)
    P = col.P + glu.P
    return torch.einsum('zst,z...t->z...s', _fermion_prop(P, m), v), P


def _row_from(row, glu, g, m):
    """chi (i g Jslash t^a) S(-P): [z, ext, j, t]"""
    e1, e2, eo = row.e, glu.e, _out(row, glu)
    Js = _slash_gluon(glu.T)
    X = torch.einsum(f'z{e1}is,aij->z{e1}ajs', row.T, TA)
    v = 1j * g * torch.einsum(f'z{e1}ajs,z{e2}ast->z{eo}jt', X, Js)
    P = row.P + glu.P
    return torch.einsum('z...s,zst->z...t', v, _fermion_prop(-P, m)), P


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
            for B, C in _pairs(BC):
                yield A, B, C


def external_legs(proc, p, hel, params, ward=None):
    """Per leg: (type, flavour, tensor [z, colour, colour, 4], incoming momentum).  ward: a gluon
    leg whose polarisation is replaced by its momentum (gauge-invariance check)."""
    info = PROCESSES[proc]
    m = params['m_t']
    legs = []
    eye3 = torch.eye(3, dtype=C128)
    eye8 = torch.eye(8, dtype=C128)
    z = p.shape[0]
    for i, (kind, incoming) in enumerate(info['legs']):
        k = p[:, i] if incoming else -p[:, i]
        if kind == 'g':
            if ward == i:
                e = p[:, i].to(C128)
            else:
                e = polarisation(p[:, i], hel[i])
                if not incoming:
                    e = e.conj()
            T = eye8.view(1, 8, 8, 1) * e.view(z, 1, 1, 4)
            legs.append((GLUON, None, T, k))
            continue
        flav = 'top' if kind in ('t', 'tbar') else 'light'
        mass = m if flav == 'top' else 0.0
        anti = kind in ('tbar', 'qbar')
        if incoming and not anti:
            s, kindc = u_spinor(p[:, i], mass, hel[i]), COL
        elif incoming and anti:
            s, kindc = bar(v_spinor(p[:, i], mass, hel[i])), ROW
        elif not anti:
            s, kindc = bar(u_spinor(p[:, i], mass, hel[i])), ROW
        else:
            s, kindc = v_spinor(p[:, i], mass, hel[i]), COL
        T = eye3.view(1, 3, 3, 1) * s.view(z, 1, 1, 4)
        legs.append((kindc, flav, T, k))
    return legs


def _type_of(S, legs):
    n = {'light': 0, 'top': 0}
    for i in S:
        kind, flav = legs[i][0], legs[i][1]
        if kind == COL:
            n[flav] += 1
        elif kind == ROW:
            n[flav] -= 1
    if n['light'] == 0 and n['top'] == 0:
        return GLUON, None
    for f, o in (('light', 'top'), ('top', 'light')):
        if n[o] == 0 and n[f] in (1, -1):
            return (COL if n[f] == 1 else ROW), f
    return None, None


def amplitude(proc, p, hel, params, ward=None):
    """Explicit-colour amplitude M[z, colour of legs 0..n-1] for one helicity configuration."""
    g = g_strong(params)
    m = params['m_t']
    legs = external_legs(proc, p, hel, params, ward)
    n = len(legs)
    assert legs[0][0] == COL and legs[0][1] == 'light'
    mass = {'light': 0.0, 'top': m}
    cur = {}
    for i in range(1, n):
        kind, flav, T, k = legs[i]
        cur[(i,)] = Current((i,), kind, flav, T, k)
    rest = tuple(range(1, n))
    for size in range(2, n):
        for S in itertools.combinations(rest, size):
            kind, flav = _type_of(S, legs)
            if kind is None:
                continue
            V = None
            P = sum(legs[i][3] for i in S)
            if kind == GLUON:
                for A, B in _pairs(S):
                    a, b = cur.get(A), cur.get(B)
                    if a is None or b is None:
                        continue
                    if a.kind == GLUON and b.kind == GLUON:
                        t = _v3(a, b, g)
                    elif a.kind == COL and b.kind == ROW and a.flav == b.flav:
                        t = _gluon_from_pair(a, b, g)
                    elif a.kind == ROW and b.kind == COL and a.flav == b.flav:
                        t = _gluon_from_pair(b, a, g)
                    else:
                        continue
                    V = t if V is None else V + t
                for A, B, C in _triples(S):
                    cs = [cur.get(X) for X in (A, B, C)]
                    if any(c is None or c.kind != GLUON for c in cs):
                        continue
                    t = _v4(*cs, g)
                    V = t if V is None else V + t
                if V is None:
                    continue
                P2 = mdot(P, P).to(C128)
                T = (-1j / P2).view(-1, *([1] * (V.dim() - 1))) * V
            else:
                for A, B in _pairs(S):
                    for F_, G_ in ((A, B), (B, A)):
                        f, gl = cur.get(F_), cur.get(G_)
                        if f is None or gl is None or gl.kind != GLUON or f.kind != kind or f.flav != flav:
                            continue
                        t, _ = (_col_from if kind == COL else _row_from)(f, gl, g, mass[flav])
                        V = t if V is None else V + t
                if V is None:
                    continue
                T = V
            cur[S] = Current(S, kind, flav, T, P)
    # vertex of leg 0 (column u, light) with a light row current and a gluon current
    _, _, T0, _ = legs[0]
    M = None
    for A, B in _pairs(rest):
        for R_, G_ in ((A, B), (B, A)):
            r, gl = cur.get(R_), cur.get(G_)
            if r is None or gl is None or r.kind != ROW or r.flav != 'light' or gl.kind != GLUON:
                continue
            Js = _slash_gluon(gl.T)
            e1, e2 = r.e, gl.e
            eo = LEG[0] + _out(r, gl)
            X = torch.einsum(f'z{e2}ast,z{LEG[0]}jt->z{e2}as{LEG[0]}j', Js, T0)
            Y = torch.einsum(f'z{e2}as{LEG[0]}j,aij->z{e2}s{LEG[0]}i', X, TA)
            t = 1j * g * torch.einsum(f'z{e1}is,z{e2}s{LEG[0]}i->z{eo}', r.T, Y)
            M = t if M is None else M + t
    return M


def matrix_element(proc, p, params, hel_list=None):
    """Spin- and colour-summed and averaged |M|^2 per event, float64 [N]."""
    info = PROCESSES[proc]
    hels = hel_list if hel_list is not None else helicities(proc)
    tot = torch.zeros(p.shape[0], dtype=torch.float64)
    for h in hels:
        M = amplitude(proc, p, h, params)
        tot = tot + (M.abs() ** 2).reshape(p.shape[0], -1).sum(-1)
    return tot / (info['avg'] * info['sym'])
