"""Pins for the oracle's generation cuts (CPU only).

The cuts are those of the gg -> ttbar g(g) workloads: every final gluon needs
pT > 20 GeV and |eta| < 2.5, and the two final gluons of gg -> ttbar gg need
Delta R > 0.4 (the paper's benchmarks are these processes, sect. 3, Table 1).
The definitions pinned here:

* pT = sqrt(px^2 + py^2);
* eta is the PSEUDOrapidity atanh(pz/|p|), a function of the three-momentum only
  (for a massless on-shell gluon it equals the rapidity; the events below give the
  gluon an energy different from |p| so that the two readings differ);
* Delta R = sqrt(Delta eta^2 + Delta phi^2) with Delta phi wrapped into [-pi, pi];
* strict inequalities; the tops are never cut.

Events are built by hand at known pT, eta and phi just inside and just outside
each boundary.  Each plausible mistake (rapidity for eta, an unwrapped Delta phi,
>= for >, cutting the tops, Delta R on the tops, |eta| replaced by eta) is planted
in a copy of the oracle's function and must fail at least one pin.
"""
import math

import pytest
import torch

from oracle import cuts, kinematics

P = dict(pt_min=20.0, eta_max=2.5, dr_min=0.4)
EPS = 1e-9


def gluon(pt, eta, phi, e_scale=1.0):
    """Momentum (E, px, py, pz) of pseudorapidity eta; E = e_scale * |p|."""
    pz = pt * math.sinh(eta)
    pabs = pt * math.cosh(eta)
    return [e_scale * pabs, pt * math.cos(phi), pt * math.sin(phi), pz]


def event(gluons, tops=None):
    """p[1, n_ext, 4]: beams along +-z, tops, then the final gluons."""
    E = 500.0
    legs = [[E, 0, 0, E], [E, 0, 0, -E]]
    legs += tops if tops is not None else [[400.0, 100.0, 50.0, 30.0], [400.0, -100.0, -50.0, -30.0]]
    legs += gluons
    return torch.tensor([legs], dtype=torch.float64)


SAFE_A = (100.0, 0.3, 0.5)
SAFE_B = (80.0, -1.0, 2.5)


# (name, event, params, expected pass) -- each case is one boundary probed from one side
def cases():
    out = []
    for sgn in (1, -1):
        out.append((f'pt above, ttg', event([gluon(20.0 * (1 + EPS), 0.1, 0.2)]), P, True))
        out.append((f'pt below, ttg', event([gluon(20.0 * (1 - EPS), 0.1, 0.2)]), P, False))
        out.append((f'eta inside {sgn}', event([gluon(50.0, sgn * (2.5 - 1e-7), 1.0)]), P, True))
        out.append((f'eta outside {sgn}', event([gluon(50.0, sgn * (2.5 + 1e-7), 1.0)]), P, False))
        # pseudorapidity, not rapidity: a gluon with E = 3 |p| has rapidity atanh(tanh(eta)/3) ~ 0.34
        # at eta = 2.4 and 2.6 alike, so only the pseudorapidity decides
        out.append((f'off-shell eta 2.6 {sgn}', event([gluon(50.0, sgn * 2.6, 1.0, e_scale=3.0)]), P, False))
        out.append((f'off-shell eta 2.4 {sgn}', event([gluon(50.0, sgn * 2.4, 1.0, e_scale=3.0)]), P, True))
        # one gluon of two fails pT or eta
        out.append((f'second gluon pt below {sgn}',
                    event([gluon(*SAFE_A), gluon(19.0, sgn * 1.0, -2.0)]), P, False))
        out.append((f'second gluon eta outside {sgn}',
                    event([gluon(*SAFE_A), gluon(60.0, sgn * 2.7, -2.0)]), P, False))
    # Delta R with Delta phi straddling +-pi: phi_a = pi - 0.1, phi_b = -pi + 0.1, so the
    # wrapped Delta phi is 0.2 (unwrapped: 2 pi - 0.2)
    dphi = 0.2
    for dr, want in ((0.4 * (1 + 1e-7), True), (0.4 * (1 - 1e-7), False)):
        deta = math.sqrt(dr * dr - dphi * dphi)
        for sgn in (1, -1):
            a = gluon(60.0, 0.3, sgn * (math.pi - 0.1))
            b = gluon(70.0, 0.3 + deta, -sgn * (math.pi - 0.1))
            out.append((f'dR {dr:.9f} across pi {sgn}', event([a, b]), P, want))
    # the same Delta R away from the branch cut
    for dr, want in ((0.4 * (1 + 1e-7), True), (0.4 * (1 - 1e-7), False)):
        deta = math.sqrt(dr * dr - 0.09)
        out.append((f'dR {dr:.9f} plain', event([gluon(60.0, -0.5, 1.0), gluon(70.0, -0.5 - deta, 1.3)]), P, want))
    # large Delta phi, small Delta eta: passes (a wrapped Delta phi never exceeds pi)
    out.append(('dR back to back', event([gluon(60.0, 0.0, 0.0), gluon(60.0, 0.0, math.pi - 1e-3)]), P, True))
    # strict inequalities at values that are exact in floating point
    out.append(('pt exactly at the cut', event([[20.0, 20.0, 0.0, 0.0]]), P, False))
    out.append(('eta exactly at the cut', event([gluon(50.0, 0.0, 0.3)]), dict(P, eta_max=0.0), False))
    out.append(('dR exactly at the cut', event([gluon(50.0, 0.4, 0.3), gluon(90.0, 0.4, 0.3)]),
                dict(P, dr_min=0.0), False))
    # tops are not cut: soft, forward tops pass; top pair collinear passes
    soft_tops = [[173.0 * math.cosh(5.0), 1.0, 0.0, 173.0 * math.sinh(5.0)], [400.0, 0.5, 0.2, -300.0]]
    out.append(('soft forward tops, ttg', event([gluon(*SAFE_A)], tops=soft_tops), P, True))
    out.append(('soft forward tops, ttgg', event([gluon(*SAFE_A), gluon(*SAFE_B)], tops=soft_tops), P, True))
    coll_tops = [[400.0, 100.0, 0.0, 30.0], [400.0, 100.0, 0.0, 30.0]]
    out.append(('collinear tops', event([gluon(*SAFE_A), gluon(*SAFE_B)], tops=coll_tops), P, True))
    # gluon close to a top: Delta R between a gluon and a top is not cut
    top_along = [[500.0, 100.0 * math.cos(0.5), 100.0 * math.sin(0.5), 100.0 * math.sinh(0.3)],
                 [400.0, -100.0, -50.0, -30.0]]
    out.append(('gluon along a top', event([gluon(*SAFE_A), gluon(*SAFE_B)], tops=top_along), P, True))
    # gg -> ttbar: no final gluons, always passes
    out.append(('no gluons', event([]), P, True))
    return out


CASES = cases()


def failures(fn):
    bad = []
    for name, p, prm, want in CASES:
        got = bool(fn(p, prm)[0])
        if got != want:
            bad.append(name)
    return bad


def test_cut_boundaries():
    assert failures(cuts.passes) == []


def test_cuts_vectorised_over_events():
    # the same decisions when the events of one process come in one batch
    for n_gl in (1, 2):
        sel = [(p, want) for _, p, prm, want in CASES if prm is P and p.shape[1] == 4 + n_gl]
        p = torch.cat([s[0] for s in sel])
        want = torch.tensor([s[1] for s in sel])
        assert torch.equal(cuts.passes(p, P), want)


def test_boundary_events_are_what_they_claim():
    # the constructed gluons have the pT, eta and phi asked for (independent formulas)
    g = torch.tensor([gluon(37.0, -1.7, 2.9, e_scale=2.0)], dtype=torch.float64)
    assert abs(math.hypot(g[0, 1].item(), g[0, 2].item()) - 37.0) < 1e-12
    pabs = math.sqrt(g[0, 1] ** 2 + g[0, 2] ** 2 + g[0, 3] ** 2)
    assert abs(0.5 * math.log((pabs + g[0, 3].item()) / (pabs - g[0, 3].item())) + 1.7) < 1e-12
    assert abs(math.atan2(g[0, 2].item(), g[0, 1].item()) - 2.9) < 1e-12


# ---------------------------------------------------------------- planted mistakes
def _variant(eta_fn=kinematics.eta, wrap=True, strict=True, cut_tops=False, abs_eta=True, gluon_pair=True):
    """A copy of the cut function with one definition changed."""
    def passes(p, params):
        N, n_ext = p.shape[0], p.shape[1]
        ok = torch.ones(N, dtype=torch.bool)
        gl = list(range(4, n_ext))
        legs = ([2, 3] if cut_tops else []) + gl
        gt = (lambda a, b: a > b) if strict else (lambda a, b: a >= b)
        for leg in legs:
            ok &= gt(kinematics.pt(p[:, leg]), params['pt_min'])
            e = eta_fn(p[:, leg])
            ok &= gt(params['eta_max'], e.abs() if abs_eta else e)
        if len(gl) == 2:
            a, b = (p[:, gl[0]], p[:, gl[1]]) if gluon_pair else (p[:, 2], p[:, gl[0]])
            dphi = kinematics.phi(a) - kinematics.phi(b)
            if wrap:
                dphi = torch.remainder(dphi + math.pi, 2.0 * math.pi) - math.pi
            deta = eta_fn(a) - eta_fn(b)
            ok &= gt(torch.sqrt(deta * deta + dphi * dphi), params['dr_min'])
        return ok
    return passes


def _rapidity(p):
    return 0.5 * torch.log((p[..., 0] + p[..., 3]) / (p[..., 0] - p[..., 3]))


def test_unplanted_variant_matches_oracle():
    assert failures(_variant()) == []


@pytest.mark.parametrize('mistake', [
    dict(eta_fn=_rapidity),
    dict(wrap=False),
    dict(strict=False),
    dict(cut_tops=True),
    dict(abs_eta=False),
    dict(gluon_pair=False),
], ids=['rapidity', 'unwrapped-dphi', 'non-strict', 'tops-cut', 'signed-eta', 'dR-to-top'])
def test_planted_cut_mistakes_fail_a_pin(mistake):
    assert failures(_variant(**mistake)) != []
