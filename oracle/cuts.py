"""Generation cuts on the final-state gluons.  Test infrastructure only.

pT = sqrt(px^2 + py^2), eta = atanh(pz/|p|), Delta R = sqrt(Delta eta^2 + Delta phi^2)
with Delta phi wrapped into [-pi, pi].  An event passes if every final gluon has
pT > pt_min and |eta| < eta_max and, with two final gluons, Delta R > dr_min
(strict inequalities).  Tops are not cut.
"""
import math

import torch

from .kinematics import pt, eta, phi


def passes(p, params):
    """Boolean [N] for momenta p[N, n_ext, 4] (final gluons are legs 4, 5, ...)."""
    N, n_ext = p.shape[0], p.shape[1]
    ok = torch.ones(N, dtype=torch.bool)
    gl = list(range(4, n_ext))
    for leg in gl:
        ok &= pt(p[:, leg]) > params['pt_min']
        ok &= eta(p[:, leg]).abs() < params['eta_max']
    if len(gl) == 2:
        a, b = p[:, gl[0]], p[:, gl[1]]
        dphi = phi(a) - phi(b)
        dphi = torch.remainder(dphi + math.pi, 2.0 * math.pi) - math.pi
        deta = eta(a) - eta(b)
        ok &= torch.sqrt(deta * deta + dphi * dphi) > params['dr_min']
    return ok
