"""Tree-level |M|^2 with explicit colour: the sum of all Feynman diagrams.  Test infrastructure only.

Definition.  ME = (1/avg) (1/S) sum_{helicities} sum_{all colour indices} |M|^2,
M = sum of all tree Feynman diagrams of QCD with one massive quark line (or of
QED for e+e- -> mu+mu-), Feynman gauge, physical external gluons.

Feynman rules (Peskin & Schroeder, Fig. 16.7; D_mu = d_mu - i g A^a_mu t^a):
  quark propagator        i (pslash + m) / (p^2 - m^2)
  gluon propagator        -i g^{mu nu} delta^{ab} / k^2
  quark-gluon vertex      i g gamma^mu t^a
  three-gluon vertex      g f^{abc} [g^{mu nu}(k-p)^rho + g^{nu rho}(p-q)^mu + g^{rho mu}(q-k)^nu]
                          (legs (a,mu,k), (b,nu,p), (c,rho,q), momenta incoming)
  four-gluon vertex       -i g^2 [f^{abe}f^{cde}(g^{mu rho}g^{nu sigma} - g^{mu sigma}g^{nu rho})
                                + f^{ace}f^{bde}(g^{mu nu}g^{rho sigma} - g^{mu sigma}g^{nu rho})
                                + f^{ade}f^{bce}(g^{mu nu}g^{rho sigma} - g^{mu rho}g^{nu sigma})]

The diagram sum is organised as an off-shell recursion over subsets of external
gluons (each tree is counted exactly once: the root vertex of a gluon sub-tree
splits its leg set into an unordered pair or triple of non-empty blocks; along
the quark line the blocks are attached in every order).  No colour-ordered
decomposition is used: every current carries explicit adjoint indices for each
external gluon it contains and for its off-shell leg, and quark currents carry
explicit fundamental indices.  The colour sum is the squared norm of the
resulting tensor M[a_1..a_k, i, j].

Momenta in the recursion are incoming: k_i = p_i for incoming legs and -p_i for
outgoing ones; external gluons are eps(p) if incoming and eps*(p) if outgoing;
the outgoing top is ubar(p_t), the outgoing antitop v(p_tbar).
"""
import itertools
import math

import numpy as np
import torch

from . import colour
from .kinematics import mdot
from .processes import PROCESSES, g_strong, e_charge, helicities
from .wavefunctions import GAMMA, u_spinor, v_spinor, bar, polarisation

C128 = torch.complex128
TA = torch.tensor(colour.T, dtype=C128)                   # t^a_{ij}
FABC = torch.tensor(colour.F, dtype=C128)                 # f^{abc}
_FF1 = torch.einsum('abe,cde->abcd', FABC, FABC)
_FF2 = torch.einsum('ace,bde->abcd', FABC, FABC)
_FF3 = torch.einsum('ade,bce->abcd', FABC, FABC)
METRIC = torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=C128)
LETTERS = 'ABCDEFGH'


def _ext(labels):
    return ''.join(LETTERS[l] for l in labels)


def _sorted_ext(*groups):
    return _ext(sorted(itertools.chain(*groups)))


class _GluonCurrent:
    """J[n, a_ext..., a, mu] with upper Lorentz index; P = incoming momentum sum."""

    def __init__(self, labels, J, P):
        self.labels, self.J, self.P = tuple(labels), J, P


def _dot_vec(X, cur):
    """X.J over the Lorentz index (X real [N,4])."""
    e = _ext(cur.labels)
    return torch.einsum(f'nm,n{e}bm->n{e}b', X.to(C128) * METRIC, cur.J)


def _v3(c1, c2, g):
    """Amputated three-gluon vertex contracted with two currents (leg a free)."""
    P1, P2 = c1.P, c2.P
    k = -(P1 + P2)
    X, Y, Z = k - P1, P1 - P2, P2 - k
    e1, e2 = _ext(c1.labels), _ext(c2.labels)
    eo = _sorted_ext(c1.labels, c2.labels)
    XJ2 = _dot_vec(X, c2)
    ZJ1 = _dot_vec(Z, c1)
    J1J2 = torch.einsum(f'n{e1}bm,n{e2}cm->n{e1}{e2}bc', c1.J * METRIC, c2.J)
    fJ1 = torch.einsum(f'abc,n{e1}bm->n{e1}acm', FABC, c1.J)
    t1 = torch.einsum(f'n{e1}acm,n{e2}c->n{eo}am', fJ1, XJ2)
    fJJ = torch.einsum(f'abc,n{e1}{e2}bc->n{e1}{e2}a', FABC, J1J2)
    t2 = torch.einsum(f'n{e1}{e2}a,nm->n{eo}am', fJJ, Y.to(C128))
    fJ2 = torch.einsum(f'abc,n{e2}cm->n{e2}abm', FABC, c2.J)
    t3 = torch.einsum(f'n{e2}abm,n{e1}b->n{eo}am', fJ2, ZJ1)
    return g * (t1 + t2 + t3)


def _v4(c1, c2, c3, g):
    """Amputated four-gluon vertex contracted with three currents (leg a free)."""
    e1, e2, e3 = _ext(c1.labels), _ext(c2.labels), _ext(c3.labels)
    eo = _sorted_ext(c1.labels, c2.labels, c3.labels)
    D12 = torch.einsum(f'n{e1}bm,n{e2}cm->n{e1}{e2}bc', c1.J * METRIC, c2.J)
    D13 = torch.einsum(f'n{e1}bm,n{e3}dm->n{e1}{e3}bd', c1.J * METRIC, c3.J)
    D23 = torch.einsum(f'n{e2}cm,n{e3}dm->n{e2}{e3}cd', c2.J * METRIC, c3.J)
    # f^{abe}f^{cde}(J2^mu D13 - J3^mu D12) + f^{ace}f^{bde}(J1^mu D23 - J3^mu D12)
    #   + f^{ade}f^{bce}(J1^mu D23 - J2^mu D13)
    G1 = _FF2 + _FF3          # multiplies J1^mu (J2.J3)
    G2 = _FF1 - _FF3          # multiplies J2^mu (J1.J3)
    G3 = -_FF1 - _FF2         # multiplies J3^mu (J1.J2)
    H1 = torch.einsum(f'abcd,n{e2}{e3}cd->n{e2}{e3}ab', G1, D23)
    t1 = torch.einsum(f'n{e2}{e3}ab,n{e1}bm->n{eo}am', H1, c1.J)
    H2 = torch.einsum(f'abcd,n{e1}{e3}bd->n{e1}{e3}ac', G2, D13)
    t2 = torch.einsum(f'n{e1}{e3}ac,n{e2}cm->n{eo}am', H2, c2.J)
    H3 = torch.einsum(f'abcd,n{e1}{e2}bc->n{e1}{e2}ad', G3, D12)
    t3 = torch.einsum(f'n{e1}{e2}ad,n{e3}dm->n{eo}am', H3, c3.J)
    return -1j * g * g * (t1 + t2 + t3)


def _pairs(S):
    """Unordered splits of the tuple S into two non-empty blocks."""
    first, rest = S[0], S[1:]
    for r in range(0, len(rest)):
        for extra in itertools.combinations(rest, r):
            A = (first,) + extra
            B = tuple(x for x in S if x not in A)
            if B:
                yield A, B


def _triples(S):
    """Unordered splits of S into three non-empty blocks."""
    for A, BC in _pairs(S):
        if len(BC) >= 2:
            for B, C in _pairs(BC):
                yield A, B, C


def gluon_currents(eps, kin, g):
    """All explicit-colour gluon currents for subsets of the gluons.

    eps: list of [N,4] complex external polarisations; kin: list of [N,4]
    incoming momenta.  Returns dict tuple(sorted labels) -> _GluonCurrent.
    """
    k = len(eps)
    N = eps[0].shape[0]
    eye = torch.eye(8, dtype=C128)
    cur = {}
    for i in range(k):
        J = eye.view(1, 8, 8, 1) * eps[i].view(N, 1, 1, 4)
        cur[(i,)] = _GluonCurrent((i,), J, kin[i])
    for size in range(2, k + 1):
        for S in itertools.combinations(range(k), size):
            P = sum(kin[i] for i in S)
            V = 0
            for A, B in _pairs(S):
                V = V + _v3(cur[A], cur[B], g)
            for A, B, C in _triples(S):
                V = V + _v4(cur[A], cur[B], cur[C], g)
            P2 = mdot(P, P).to(C128)
            J = (-1j / P2).view(N, *([1] * (V.dim() - 1))) * V
            cur[S] = _GluonCurrent(S, J, P)
    return cur


def quark_line(ubar_t, v_tb, p_t, m, cur, k, g):
    """M[n, a_1..a_k, i, j] for ubar(p_t) ... v(p_tbar) with all gluon blocks attached."""
    N = ubar_t.shape[0]
    eye3 = torch.eye(3, dtype=C128)
    Q = {(): eye3.view(1, 3, 3, 1) * ubar_t.view(N, 1, 1, 4)}      # [n, i, k, s]
    P_of = {S: cur[S].P for S in cur}
    full = tuple(range(k))

    def vertex(Qprev, prev_labels, B):
        """i g gamma^mu t^a J^a_mu(B) applied on the right of a row quark current."""
        c = cur[B]
        eB = _ext(B)
        ep = _ext(prev_labels)
        eo = _sorted_ext(prev_labels, B)
        Js = torch.einsum(f'n{eB}am,mst->n{eB}ast', c.J * METRIC, GAMMA)
        TJ = torch.einsum(f'akl,n{eB}ast->n{eB}klst', TA, Js)
        return 1j * g * torch.einsum(f'n{ep}iks,n{eB}klst->n{eo}ilt', Qprev, TJ)

    def subsets(S):
        for r in range(1, len(S) + 1):
            for B in itertools.combinations(S, r):
                yield B

    for size in range(1, k):
        for S in itertools.combinations(full, size):
            acc = 0
            for B in subsets(S):
                prev = tuple(x for x in S if x not in B)
                acc = acc + vertex(Q[prev], prev, B)
            p = p_t - sum(P_of[(i,)] for i in S)
            den = (mdot(p, p) - m * m).to(C128)
            prop = 1j * (torch.einsum('nm,mst->nst', p.to(C128) * METRIC, GAMMA)
                         + m * torch.eye(4, dtype=C128)) / den.view(N, 1, 1)
            e = _ext(S)
            Q[S] = torch.einsum(f'n{e}ils,nst->n{e}ilt', acc, prop)
    M = 0
    for B in subsets(full):
        prev = tuple(x for x in full if x not in B)
        M = M + vertex(Q[prev], prev, B)
    e = _ext(full)
    return torch.einsum(f'n{e}ijt,nt->n{e}ij', M, v_tb)


def amplitude_qcd(p, hel, params, ward=None):
    """Explicit-colour amplitude tensor M[n, a_1..a_k, i, j] for one helicity.

    p: [N, n_ext, 4] physical momenta (legs: g, g, t, tbar, g...).
    ward: optional gluon index whose polarisation is replaced by its momentum.
    """
    n_ext = p.shape[1]
    m = params['m_t']
    g = g_strong(params)
    gl_legs = [0, 1] + list(range(4, n_ext))
    eps, kin = [], []
    for gi, leg in enumerate(gl_legs):
        incoming = leg < 2
        if ward == gi:
            e = p[:, leg].to(C128)
        else:
            e = polarisation(p[:, leg], hel[leg])
            if not incoming:
                e = e.conj()
        eps.append(e)
        kin.append(p[:, leg] if incoming else -p[:, leg])
    ubar_t = bar(u_spinor(p[:, 2], m, hel[2]))
    v_tb = v_spinor(p[:, 3], m, hel[3])
    cur = gluon_currents(eps, kin, g)
    return quark_line(ubar_t, v_tb, p[:, 2], m, cur, len(gl_legs), g)


def amplitude_ee(p, hel, params):
    """e-(p0) e+(p1) -> mu-(p2) mu+(p3) through an s-channel photon (QED, massless)."""
    e = e_charge(params)
    u1 = u_spinor(p[:, 0], 0.0, hel[0])
    vb2 = bar(v_spinor(p[:, 1], 0.0, hel[1]))
    ub3 = bar(u_spinor(p[:, 2], 0.0, hel[2]))
    v4 = v_spinor(p[:, 3], 0.0, hel[3])
    jin = torch.einsum('ns,mst,nt->nm', vb2, GAMMA, u1)        # vbar gamma^mu u
    jout = torch.einsum('ns,mst,nt->nm', ub3, GAMMA, v4)
    P = p[:, 0] + p[:, 1]
    s = mdot(P, P)
    # (-i e gamma^mu) (-i g_{mu nu}/s) (-i e gamma^nu)
    return (1j * e * e / s) * (jin * METRIC * jout).sum(-1)


def matrix_element(proc, p, params, hel_list=None):
    """Spin/colour summed and averaged |M|^2 per event, float64 [N]."""
    info = PROCESSES[proc]
    hels = hel_list if hel_list is not None else helicities(proc)
    tot = torch.zeros(p.shape[0], dtype=torch.float64)
    for h in hels:
        if info['kind'] == 'ee':
            A = amplitude_ee(p, h, params)
            tot = tot + (A.abs() ** 2)
        else:
            M = amplitude_qcd(p, h, params)
            tot = tot + (M.abs() ** 2).reshape(p.shape[0], -1).sum(-1)
    return tot / (info['avg'] * info['sym'])
