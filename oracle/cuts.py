"""Generation cuts on the final-state light partons (gluons and light quarks).  Test infrastructure only.

pT = sqrt(px^2 + py^2), eta = atanh(pz/|p|), Delta R = sqrt(Delta eta^2 + Delta phi^2)
with Delta phi wrapped into [-pi, pi].  An event passes if every final light parton has
pT > pt_min and |eta| < eta_max and every pair of them has Delta R > dr_min
(strict inequalities).  Tops are not cut.
"""
import math

import torch

from .kinematics import pt, eta, phi


def passes(p, params):
    """Boolean [N] for momenta p[N, n_ext, 4] (final light partons are legs 4, 5, ...)."""
    N, n_ext = p.shape[0], p.shape[1]
    ok = torch.ones(N, dtype=torch.bool)
    gl = list(range(4, n_ext))
    for leg in gl:
        ok &= pt(p[:, leg]) > params['pt_min']
        ok &= eta(p[:, leg]).abs() < params['eta_max']
    for i in range(len(gl)):
        for j in range(i + 1, len(gl)):
            a, b = p[:, gl[i]], p[:, gl[j]]
            dphi = phi(a) - phi(b)
            dphi = torch.remainder(dphi + math.pi, 2.0 * math.pi) - math.pi
            deta = eta(a) - eta(b)
            ok &= torch.sqrt(deta * deta + dphi * dphi) > params['dr_min']
    return ok
