"""Colour-ordered |M|^2: partial amplitudes and the colour matrix.  Test infrastructure only.

For one quark line with k gluons the full amplitude decomposes exactly as
    M_{i jbar}(a_1..a_k) = sum_{sigma in S_k} (t^{a_sigma1} ... t^{a_sigmak})_{i jbar} A(sigma)
and the colour-summed square is sum_{sigma,tau} A(sigma) C_{sigma tau} A(tau)^*,
C from ``colour.colour_matrix``.

Derivation of the ordered rules from the Feynman rules listed in
``me_explicit`` (P&S conventions): contract each gluon current with t^a into a
matrix JJ = t^a J^a, and use f^{abc} t^a = -i [t^b, t^c].  The three- and
four-gluon vertices then become commutators of matrix currents; expanding them
gives JJ(S) = sum over orderings rho of S of (t..t)_rho j(rho) with ordered
currents
    j(rho) = (1/P_rho^2) [ -g sum_{rho = pi pi'} K(j(pi), P_pi; j(pi'), P_pi')
                           + g^2 sum_{rho = pi1 pi2 pi3} W(j(pi1), j(pi2), j(pi3)) ],
    K(J1,P1;J2,P2) = J1 ((-2P1-P2).J2) + (J1.J2)(P1-P2) + J2 ((P1+2P2).J1),
    W(J1,J2,J3)    = 2 J2 (J1.J3) - J3 (J1.J2) - J1 (J2.J3),
(sums over contiguous splits; single-gluon currents are the polarisations) and
    A(sigma) = sum over splits of sigma into contiguous blocks b1..br of
               ubar(p_t) [i g jslash(b1)] [i S(p_1)] [i g jslash(b2)] ... [i g jslash(br)] v(p_tbar),
    S(p) = (pslash + m)/(p^2 - m^2),  p_l = p_t - (incoming momenta of blocks 1..l).
The explicit-colour module uses none of this; agreement of the two is a test.
"""
import itertools

import numpy as np
import torch

from . import colour
from .kinematics import mdot
from .processes import PROCESSES, g_strong, helicities
from .wavefunctions import GAMMA, u_spinor, v_spinor, bar, polarisation

C128 = torch.complex128
METRIC = torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=C128)


def cdot(a, b):
    """Minkowski product of complex/real four-vectors [..., 4] (no conjugation)."""
    return (a.to(C128) * METRIC * b.to(C128)).sum(-1)


def K3(J1, P1, J2, P2):
    a = -2.0 * P1 - P2
    c = P1 + 2.0 * P2
    return (J1 * cdot(a, J2).unsqueeze(-1) + cdot(J1, J2).unsqueeze(-1) * (P1 - P2).to(C128)
            + J2 * cdot(c, J1).unsqueeze(-1))


def W4(J1, J2, J3):
    return (2.0 * J2 * cdot(J1, J3).unsqueeze(-1) - J3 * cdot(J1, J2).unsqueeze(-1)
            - J1 * cdot(J2, J3).unsqueeze(-1))


def pslash(p):
    return torch.einsum('nm,mst->nst', p.to(C128) * METRIC, GAMMA)


def partial_amplitudes(p, hel, params, ward=None):
    """A[sigma] for one helicity: complex [N, k!] in ``colour.orderings(k)`` order."""
    n_ext = p.shape[1]
    m = params['m_t']
    g = g_strong(params)
    gl_legs = [0, 1] + list(range(4, n_ext))
    k = len(gl_legs)
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
    N = p.shape[0]

    jmemo = {}

    def mom(rho):
        return sum(kin[i] for i in rho)

    def j(rho):
        if rho in jmemo:
            return jmemo[rho]
        if len(rho) == 1:
            out = eps[rho[0]]
        else:
            acc = 0
            for s in range(1, len(rho)):
                a, b = rho[:s], rho[s:]
                acc = acc - g * K3(j(a), mom(a), j(b), mom(b))
            for s1 in range(1, len(rho) - 1):
                for s2 in range(s1 + 1, len(rho)):
                    a, b, c = rho[:s1], rho[s1:s2], rho[s2:]
                    acc = acc + g * g * W4(j(a), j(b), j(c))
            P = mom(rho)
            out = acc / mdot(P, P).to(C128).unsqueeze(-1)
        jmemo[rho] = out
        return out

    qmemo = {(): ubar_t}

    def vert(row, rho):
        return 1j * g * torch.einsum('ns,nst->nt', row, pslash(j(rho)))

    def q(prefix):
        """Row spinor: ubar with the gluons of ``prefix`` attached, propagator included."""
        if prefix in qmemo:
            return qmemo[prefix]
        acc = 0
        for s in range(len(prefix)):
            acc = acc + vert(q(prefix[:s]), prefix[s:])
        pp = p[:, 2] - mom(prefix)
        den = (mdot(pp, pp) - m * m).to(C128)
        mm = m.view(-1, 1, 1) if torch.is_tensor(m) else m
        prop = 1j * (pslash(pp) + mm * torch.eye(4, dtype=C128)) / den.view(N, 1, 1)
        out = torch.einsum('ns,nst->nt', acc, prop)
        qmemo[prefix] = out
        return out

    amps = []
    for sigma in colour.orderings(k):
        acc = 0
        for s in range(k):
            acc = acc + vert(q(sigma[:s]), sigma[s:])
        amps.append((acc * v_tb).sum(-1))
    return torch.stack(amps, -1)


_CMAT = {}


def colour_matrix(k):
    """Brute-force colour matrix of k gluons as a tensor (computed once per k)."""
    if k not in _CMAT:
        _CMAT[k] = torch.tensor(colour.colour_matrix(k), dtype=torch.float64)
    return _CMAT[k]


def matrix_element(proc, p, params, hel_list=None, return_per_helicity=False):
    """Spin/colour summed and averaged |M|^2 per event [N] from partial amplitudes."""
    info = PROCESSES[proc]
    assert info['kind'] == 'qcd'
    k = info['n_ext'] - 2
    C = colour_matrix(k).to(C128)
    hels = hel_list if hel_list is not None else helicities(proc)
    tot = torch.zeros(p.shape[0], dtype=torch.float64)
    per = []
    for h in hels:
        A = partial_amplitudes(p, h, params)
        val = torch.einsum('ns,st,nt->n', A, C, A.conj()).real
        per.append(val)
        tot = tot + val
    tot = tot / (info['avg'] * info['sym'])
    if return_per_helicity:
        return tot, torch.stack(per, -1)
    return tot
