"""Partonic cross-section integrand.  Test infrastructure only.

F = conv * (1/(2 s)) * W * ME * Theta(cuts)   [pb], with conv = (hbar c)^2 =
0.3893793721e9 pb GeV^2, W the phase-space weight and ME the spin/colour
averaged |M|^2 (including the 1/S identical-particle factor).  The Vegas
Jacobian multiplies F in the Vegas driver.
"""
import numpy as np
import torch

from . import me_explicit, me_ordered, me_quarks
from .closed_forms import GEV2_TO_PB
from .cuts import passes
from .phase_space import phase_space, incoming
from .processes import PROCESSES, out_masses


def momenta(proc, params, u):
    """u [N, d] float64 tensor -> p [N, n_ext, 4], weight [N]."""
    k, w = phase_space(u, params['sqrt_s'], out_masses(proc, params))
    p = torch.cat([incoming(u.shape[0], params['sqrt_s']), k], 1)
    return p, w


def me(proc, p, params):
    """ME per event: explicit diagrams for e+e- -> mu+mu-, colour-ordered form for gg-initiated
    QCD, explicit colour for the processes with two quark lines."""
    kind = PROCESSES[proc]['kind']
    if kind == 'ee':
        return me_explicit.matrix_element(proc, p, params)
    if kind == 'qcd4':
        return me_quarks.matrix_element(proc, p, params)
    return me_ordered.matrix_element(proc, p, params)


def integrand(proc, params, y, apply_cuts=True):
    """y [d][N] numpy -> (F [N] numpy in pb, pass mask [N] numpy bool, ME [N])."""
    u = torch.tensor(np.ascontiguousarray(y.T), dtype=torch.float64)
    p, w = momenta(proc, params, u)
    m = me(proc, p, params)
    ok = passes(p, params) if apply_cuts else torch.ones(p.shape[0], dtype=torch.bool)
    s = params['sqrt_s'] ** 2
    F = GEV2_TO_PB * w * m / (2.0 * s) * ok.to(torch.float64)
    return F.numpy(), ok.numpy(), m.numpy()
