"""Pins of the oracle for the processes with two quark lines (oracle/me_quarks.py).

* q qbar -> t tbar against the textbook spin- and colour-averaged form
  (4/9) g^4 [(m^2 - t)^2 + (m^2 - u)^2 + 2 m^2 s] / s^2 (R. K. Ellis, W. J. Stirling,
  B. R. Webber, QCD and Collider Physics, ch. 10), and its massless limit (4/9) g^4 (t^2+u^2)/s^2.
* q qbar -> t tbar g and q g -> t tbar q against the five Feynman diagrams written out one by
  one here (gluon emission from each of the four quark legs, and the three-gluon vertex), every
  colour index explicit, per helicity configuration: an independent evaluation of the same
  sum of diagrams (no recursion, no shared code with the oracle beyond the external
  wavefunctions and the SU(3) matrices, which are pinned elsewhere).
* Gauge invariance: for every process with a gluon, each gluon's polarisation replaced by its
  momentum makes the whole colour tensor vanish, per helicity.
* Lorentz invariance of the summed |M|^2 and the exact alpha_s^n scaling.
* The phase-space and cut conventions: legs 4, 5, ... (gluons and the light quark) are cut.
* Planted mistakes in the oracle's vertices fail one of these.
"""
import math

import numpy as np
import pytest
import torch

from oracle import colour, cuts, integrand, me_quarks, philox, processes
from oracle.kinematics import mdot
from oracle.wavefunctions import GAMMA, bar, polarisation, u_spinor, v_spinor

P = processes.DEFAULT_PARAMS
C128 = torch.complex128
TA = torch.tensor(colour.T, dtype=C128)
FABC = torch.tensor(colour.F, dtype=C128)
G = torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=C128)


def events(proc, n, seed, params=P):
    x = philox.uniforms(seed, n, processes.dims(proc))
    p, _ = integrand.momenta(proc, params, torch.tensor(np.ascontiguousarray(x.T)))
    return p


def mandelstam(p):
    s = mdot(p[:, 0] + p[:, 1], p[:, 0] + p[:, 1]).numpy()
    t = mdot(p[:, 0] - p[:, 2], p[:, 0] - p[:, 2]).numpy()
    u = mdot(p[:, 0] - p[:, 3], p[:, 0] - p[:, 3]).numpy()
    return s, t, u


@pytest.mark.parametrize('mt', [173.0, 0.0])
def test_qq_tt_textbook_form(mt):
    par = dict(P, m_t=mt)
    p = events('qq_tt', 200, 4, par)
    me = me_quarks.matrix_element('qq_tt', p, par).numpy()
    s, t, u = mandelstam(p)
    g4 = (4 * math.pi * P['alpha_s']) ** 2
    m2 = mt * mt
    ref = (4.0 / 9.0) * g4 * ((m2 - t) ** 2 + (m2 - u) ** 2 + 2 * m2 * s) / s ** 2
    assert np.abs(me / ref - 1).max() < 1e-12


# ------------------------------------------------------------ five diagrams, written out
def _slash(a):
    return torch.einsum('zm,mst->zst', a.to(C128) * G, GAMMA)


def _prop(q, m):
    den = (mdot(q, q) - m * m).to(C128).view(-1, 1, 1)
    return 1j * (_slash(q) + m * torch.eye(4, dtype=C128)) / den


def five_diagrams(u1, k1, rowL, kL, ub3, k3, v4, k4, eps, kg, g, m):
    """Explicit-colour amplitude M[z, c(u1), c(rowL), c(ub3), c(v4), a] of the five diagrams of
    light quark line (column u1, row rowL) x top line (row ub3, column v4) x one gluon (eps),
    all momenta k incoming.  Colour: the light line carries (row index, column index)."""
    ig = 1j * g
    gsl = _slash(eps)                                       # eps-slash
    Jtop = torch.einsum('zs,mst,zt->zm', ub3, GAMMA, v4)    # ubar3 gamma^mu v4
    Jlig = torch.einsum('zs,mst,zt->zm', rowL, GAMMA, u1)   # rowL gamma^mu u1
    sL = mdot(k1 + kL, k1 + kL).to(C128)                    # gluon off the light line
    sT = mdot(k3 + k4, k3 + k4).to(C128)                    # gluon off the top line
    # D1: emission next to u1 (fermion momentum k1 + kg), then the exchanged gluon
    L1 = torch.einsum('zs,mst,ztu,zuv,zv->zm', rowL, GAMMA, _prop(k1 + kg, 0.0), gsl, u1)
    D1 = ig * ig * ig * (-1j) * (L1 * G * Jtop).sum(-1) / sT
    # D2: emission next to rowL (fermion momentum -(kL + kg))
    L2 = torch.einsum('zs,zst,ztu,muv,zv->zm', rowL, gsl, _prop(-(kL + kg), 0.0), GAMMA, u1)
    D2 = ig * ig * ig * (-1j) * (L2 * G * Jtop).sum(-1) / sT
    # D3: emission next to ub3 (fermion momentum -(k3 + kg))
    T3 = torch.einsum('zs,zst,ztu,muv,zv->zm', ub3, gsl, _prop(-(k3 + kg), m), GAMMA, v4)
    D3 = ig * ig * ig * (-1j) * (Jlig * G * T3).sum(-1) / sL
    # D4: emission next to v4 (fermion momentum k4 + kg)
    T4 = torch.einsum('zs,mst,ztu,zuv,zv->zm', ub3, GAMMA, _prop(k4 + kg, m), gsl, v4)
    D4 = ig * ig * ig * (-1j) * (Jlig * G * T4).sum(-1) / sL
    # D5: three-gluon vertex; legs (b, nu, kb = k1 + kL) from the light line, (c, rho,
    # kc = k3 + k4) from the top line, (a, mu, kg) the external gluon
    kb, kc = (k1 + kL).to(C128), (k3 + k4).to(C128)
    ka = kg.to(C128)
    B = -1j * Jlig / sL.view(-1, 1)                          # propagated light-line current
    Cc = -1j * Jtop / sT.view(-1, 1)                         # propagated top-line current
    dot = lambda x, y: (x * G * y).sum(-1)                   # noqa: E731
    V = (dot(B, Cc) * dot(kb - kc, eps) + dot(Cc, eps) * dot(kc - ka, B) + dot(eps, B) * dot(ka - kb, Cc))
    D5 = g * (ig * ig) * V
    # colour: light line (row r, column c), top line (row R, column C), gluon a
    tt = torch.einsum('bri,aic->rcab', TA, TA)               # (t^b t^a)_{rc}
    c1 = torch.einsum('rcab,bRC->rcRCa', tt, TA)             # D1: rowL t^b S t^a u1
    c2 = torch.einsum('ari,bic,bRC->rcRCa', TA, TA, TA)      # D2: rowL t^a S t^b u1
    c3 = torch.einsum('brc,aRI,bIC->rcRCa', TA, TA, TA)      # D3: ub3 t^a S t^b v4
    c4 = torch.einsum('brc,bRI,aIC->rcRCa', TA, TA, TA)      # D4: ub3 t^b S t^a v4
    c5 = torch.einsum('bca,brk,cRC->rkRCa', FABC, TA, TA)   # D5: f^{bca} t^b_{light} t^c_{top}
    M = (D1.view(-1, 1, 1, 1, 1, 1) * c1 + D2.view(-1, 1, 1, 1, 1, 1) * c2 + D3.view(-1, 1, 1, 1, 1, 1) * c3
         + D4.view(-1, 1, 1, 1, 1, 1) * c4 + D5.view(-1, 1, 1, 1, 1, 1) * c5)
    return M                                                  # [z, r, c, R, C, a]


def _five_diagram_me_per_helicity(proc, p, h):
    m, g = P['m_t'], processes.g_strong(P)
    u1 = u_spinor(p[:, 0], 0.0, h[0])
    ub3 = bar(u_spinor(p[:, 2], m, h[2]))
    v4 = v_spinor(p[:, 3], m, h[3])
    if proc == 'qq_ttg':
        rowL, kL = bar(v_spinor(p[:, 1], 0.0, h[1])), p[:, 1]
        eps, kg = polarisation(p[:, 4], h[4]).conj(), -p[:, 4]
    else:                                                    # q g -> t tbar q
        rowL, kL = bar(u_spinor(p[:, 4], 0.0, h[4])), -p[:, 4]
        eps, kg = polarisation(p[:, 1], h[1]), p[:, 1]
    M = five_diagrams(u1, p[:, 0], rowL, kL, ub3, -p[:, 2], v4, -p[:, 3], eps, kg, g, m)
    return (M.abs() ** 2).reshape(p.shape[0], -1).sum(-1)


@pytest.mark.parametrize('proc', ['qq_ttg', 'qg_ttq'])
def test_five_diagrams_written_out(proc):
    p = events(proc, 6, 11)
    hels = processes.helicities(proc)
    tot_ref = torch.zeros(p.shape[0], dtype=torch.float64)
    for h in hels:
        ref = _five_diagram_me_per_helicity(proc, p, h)
        got = (me_quarks.amplitude(proc, p, h, P).abs() ** 2).reshape(p.shape[0], -1).sum(-1)
        scale = ref.max().item() + 1e-300
        assert (got - ref).abs().max().item() <= 1e-12 * max(scale, 1e-300) + 1e-30, h
        tot_ref += ref
    info = processes.PROCESSES[proc]
    me = me_quarks.matrix_element(proc, p, P)
    assert ((me / (tot_ref / (info['avg'] * info['sym'])) - 1).abs().max().item()) < 1e-12


# ------------------------------------------------------------ gauge invariance
@pytest.mark.parametrize('proc,n', [('qq_ttg', 3), ('qg_ttq', 3), ('qq_ttgg', 2), ('qg_ttqg', 2)])
def test_ward_identity_every_gluon(proc, n):
    p = events(proc, n, 13)
    legs = processes.PROCESSES[proc]['legs']
    hels = processes.helicities(proc)
    gl = [i for i, (k, _) in enumerate(legs) if k == 'g']
    for h in hels[::5]:
        M = me_quarks.amplitude(proc, p, h, P)
        scale = M.abs().max().item()
        if scale == 0.0:
            continue
        for leg in gl:
            W = me_quarks.amplitude(proc, p, h, P, ward=leg)
            # the momentum has the size of sqrt(s) where the polarisation has size 1
            assert W.abs().max().item() < 1e-11 * scale * P['sqrt_s'], (h, leg)


# ------------------------------------------------------------ symmetries
def _boost_z(p, y):
    ch, sh = math.cosh(y), math.sinh(y)
    q = p.clone()
    q[..., 0] = ch * p[..., 0] + sh * p[..., 3]
    q[..., 3] = sh * p[..., 0] + ch * p[..., 3]
    return q


def _rotate(p, a):
    c, s = math.cos(a), math.sin(a)
    q = p.clone()
    q[..., 1] = c * p[..., 1] - s * p[..., 2]
    q[..., 2] = s * p[..., 1] + c * p[..., 2]
    return q


@pytest.mark.parametrize('proc', ['qq_ttg', 'qg_ttqg'])
def test_lorentz_invariance_and_alpha_s_scaling(proc):
    p = events(proc, 3, 17)
    me = me_quarks.matrix_element(proc, p, P)
    for q in (_boost_z(p, 0.7), _rotate(p, 1.1), _rotate(_boost_z(p, -0.4), 2.3)):
        assert ((me_quarks.matrix_element(proc, q, P) / me - 1).abs().max().item()) < 1e-10
    nq = processes.PROCESSES[proc]['n_ext'] - 2
    me2 = me_quarks.matrix_element(proc, p, dict(P, alpha_s=0.2))
    assert ((me2 / me / (0.2 / P['alpha_s']) ** nq - 1).abs().max().item()) < 1e-12


def test_light_quark_is_cut_like_a_gluon():
    p = events('qg_ttq', 2000, 19)
    ok = cuts.passes(p, P)
    from oracle.kinematics import pt, eta
    exp = (pt(p[:, 4]) > P['pt_min']) & (eta(p[:, 4]).abs() < P['eta_max'])
    assert torch.equal(ok, exp)
    assert 0 < ok.sum().item() < 2000


# ------------------------------------------------------------ planted mistakes
def test_planted_mistakes_are_caught(monkeypatch):
    orig_v3 = me_quarks._v3

    def v3_wrong_sign(c1, c2, g):
        return -orig_v3(c1, c2, g)

    with monkeypatch.context() as mp:
        mp.setattr(me_quarks, '_v3', v3_wrong_sign)
        with pytest.raises(AssertionError):
            test_five_diagrams_written_out('qq_ttg')
        with pytest.raises(AssertionError):
            test_ward_identity_every_gluon('qq_ttgg', 2)
    orig_prop = me_quarks._fermion_prop
    with monkeypatch.context() as mp:
        mp.setattr(me_quarks, '_fermion_prop', lambda p, m: orig_prop(p, 0.0))   # top mass dropped
        with pytest.raises(AssertionError):
            test_five_diagrams_written_out('qq_ttg')
    orig_ta = me_quarks.TA
    with monkeypatch.context() as mp:
        mp.setattr(me_quarks, 'TA', orig_ta.transpose(1, 2).contiguous())        # t^a transposed
        with pytest.raises(AssertionError):
            test_five_diagrams_written_out('qg_ttq')
