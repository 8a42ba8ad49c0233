"""Numerical anchors the oracle must reproduce (CPU only).

Each number below was computed from a published closed form, independently of
the oracle's code, and is asserted here as a literal:

* e+e- -> mu+mu- (massless QED, s-channel photon): e^4 = (4 pi alpha)^2 at
  alpha = 1/137, and sigma = 4 pi alpha^2/(3 s) at sqrt(s) = 100 GeV
  (Peskin & Schroeder eqs. 5.13-5.14);
* LO gg -> t tbar (Combridge 1979; Ellis, Stirling, Webber, heavy-quark table) at
  sqrt(s_hat) = 1 TeV, m_t = 173 GeV, alpha_s = 0.118: the averaged |M|^2 at
  cos theta = 0 and 0.5, and the partonic cross section;
* massless n-body phase-space volumes V_n = (2 pi)^(4-3n) (pi/2)^(n-1)
  s^(n-2)/((n-1)!(n-2)!) at sqrt(s) = 1 TeV, and the two-body massive volume
  beta/(8 pi);
* the three-body volume with masses (m_t, m_t, 0), from the recursive
  factorisation of phase space by quadrature.

The processes are the gluon channels of the paper's benchmarks (sect. 3,
Table 1); the paper itself prints no formula or number for them.
"""
import math

import numpy as np
import pytest
import torch

from oracle import closed_forms as cf, me_explicit, me_ordered, phase_space as ps, philox, processes

P = processes.DEFAULT_PARAMS
PEE = processes.EE_PARAMS
S = P['sqrt_s'] ** 2

E4 = 8.4135367e-3                     # (4 pi / 137)^2
ME_C0 = 0.38824112473715              # gg -> ttbar, cos theta = 0
ME_C05 = 0.75045320685473             # gg -> ttbar, cos theta = 0.5
SIGMA_TT_GEV = 2.91959689250e-8       # GeV^-2
SIGMA_TT_PB = 11.36831                # pb
SIGMA_EE_GEV = 2.23175993e-8          # GeV^-2
SIGMA_EE_PB = 8.690013                # pb
V = {2: 3.978873577297e-2, 3: 1.259825563797e2, 4: 1.329656430279e5}
W2_MASSIVE = 3.733116510149e-2        # beta / (8 pi)
PHI3_MM0 = 74.856205781               # GeV^2


def rel(a, b):
    return abs(a / b - 1.0)


def test_ee_anchors():
    assert rel(cf.ee_mumu_me(0.0, PEE['alpha']), E4) < 1e-7
    s = PEE['sqrt_s'] ** 2
    assert rel(cf.ee_mumu_sigma(s, PEE['alpha']), SIGMA_EE_GEV) < 1e-8
    assert rel(cf.ee_mumu_sigma(s, PEE['alpha']) * cf.GEV2_TO_PB, SIGMA_EE_PB) < 1e-6


def _tt_events(cos_list, phi=0.7):
    E = P['sqrt_s'] / 2
    q = math.sqrt(E * E - P['m_t'] ** 2)
    p = torch.zeros(len(cos_list), 4, 4, dtype=torch.float64)
    for i, c in enumerate(cos_list):
        s_ = math.sqrt(1 - c * c)
        p[i, 0] = torch.tensor([E, 0, 0, E], dtype=torch.float64)
        p[i, 1] = torch.tensor([E, 0, 0, -E], dtype=torch.float64)
        p[i, 2] = torch.tensor([E, q * s_ * math.cos(phi), q * s_ * math.sin(phi), q * c], dtype=torch.float64)
        p[i, 3] = torch.tensor([E, -q * s_ * math.cos(phi), -q * s_ * math.sin(phi), -q * c], dtype=torch.float64)
    return p


@pytest.mark.parametrize('mode', ['ordered', 'explicit'])
def test_gg_tt_worked_values(mode):
    p = _tt_events([0.0, 0.5])
    fn = me_ordered.matrix_element if mode == 'ordered' else me_explicit.matrix_element
    me = fn('gg_tt', p, P).numpy()
    assert rel(me[0], ME_C0) < 1e-12
    assert rel(me[1], ME_C05) < 1e-12
    assert rel(cf.gg_tt_me_costheta(0.0, S, P['m_t'], P['alpha_s']), ME_C0) < 1e-13
    assert rel(cf.gg_tt_me_costheta(0.5, S, P['m_t'], P['alpha_s']), ME_C05) < 1e-13


def test_gg_tt_sigma_anchor():
    sig = cf.gg_tt_sigma(S, P['m_t'], P['alpha_s'])
    assert rel(sig, SIGMA_TT_GEV) < 1e-11
    assert rel(sig * cf.GEV2_TO_PB, SIGMA_TT_PB) < 1e-6


@pytest.mark.parametrize('n', [2, 3, 4])
def test_massless_volume_anchors(n):
    assert rel(ps.massless_volume(n, S), V[n]) < 1e-12
    # the sampler's weight is that constant on every event
    u = torch.tensor(philox.uniforms(3, 64, 3 * n - 4).T.copy())
    _, w = ps.phase_space(u, P['sqrt_s'], [0.0] * n)
    assert torch.all((w / V[n] - 1).abs() < 1e-12)


def test_two_body_massive_weight_anchor():
    u = torch.tensor(philox.uniforms(4, 64, 2).T.copy())
    _, w = ps.phase_space(u, P['sqrt_s'], [P['m_t'], P['m_t']])
    assert torch.all((w / W2_MASSIVE - 1).abs() < 1e-12)


def test_three_body_massive_volume_anchor():
    # statistical: the mean weight estimates the volume, within 4 Monte Carlo errors
    N = 200000
    u = torch.tensor(philox.uniforms(21, N, 5).T.copy())
    _, w = ps.phase_space(u, P['sqrt_s'], [P['m_t'], P['m_t'], 0.0])
    w = w.numpy()
    err = w.std() / math.sqrt(N)
    assert abs(w.mean() - PHI3_MM0) < 4 * err, (w.mean(), err)
    assert err < 2e-3 * PHI3_MM0
