"""Parton densities from a tabulated grid, and hadronic events.  Test infrastructure only.

The paper's workload is hadronic (pp -> t tbar + jets, sect. 3, Table 1): partonic matrix
elements convoluted with parton densities, which its generator interpolates from PDF grids
on the device (the PDF step before the matrix element, sect. 1).  No grid files are
available, so smooth toy densities tabulated like grid files stand in.

Interpolation (a reading of the usual log-bicubic scheme of grid-based PDF libraries): with
t = ln x and s = ln Q^2, and (x, Q^2) clamped into the grid,
  * per Q^2 node, a cubic Hermite in t on the cell [t_i, t_i+1] holding t, with node
    slopes from finite differences of the node values: the mean of the two adjacent secant
    slopes inside the grid, the one secant slope at its ends;
  * then the same cubic Hermite in s over the values of the Q^2 nodes j-1 .. j+2 around the
    cell [s_j, s_j+1] holding s.
The grid stores x f(x, Q^2); f = (x f) / x.

Hadronic events (readings): collider energy sqrt(S); one parton channel per call, parton 1
from beam 1 (+z) with density f_a and parton 2 from beam 2 with density f_b (gg: both the
gluon; q qbar -> t tbar (+ jets): quark and antiquark; q g -> t tbar q (+ g): quark and
gluon); factorisation scale mu_F = m_t; two more
uniforms (u_tau, u_y) before the partonic ones:
  tau = tau0^(1 - u_tau), tau0 = (2 m_t)^2 / S,      jacobian tau ln(1/tau0),
  y = (u_y - 1/2) ln(1/tau),                          jacobian ln(1/tau),
  x1 = sqrt(tau) e^y, x2 = sqrt(tau) e^-y, s_hat = tau S;
the partonic event is generated in the partonic c.m. frame at sqrt(s_hat) (parton 1
along +z); the cuts are applied in the lab frame, which is reached by a boost of rapidity
y along z (pseudorapidities of the massless gluons shift by y; pT and Delta R do not
change).  The integrand, in pb,
  F = J_tau J_y f_a(x1) f_b(x2) (hbar c)^2 / (2 s_hat) W ME Theta.
"""
import math

import numpy as np
import torch

from .closed_forms import GEV2_TO_PB
from .cuts import passes
from .integrand import me as partonic_me
from .phase_space import incoming, phase_space
from .processes import out_masses


def _slope(v, t, k):
    """Node slope of values v at nodes t (mean of adjacent secants; one secant at the ends)."""
    n = len(t)
    if k == 0:
        return (v[1] - v[0]) / (t[1] - t[0])
    if k == n - 1:
        return (v[n - 1] - v[n - 2]) / (t[n - 1] - t[n - 2])
    return 0.5 * ((v[k + 1] - v[k]) / (t[k + 1] - t[k]) + (v[k] - v[k - 1]) / (t[k] - t[k - 1]))


def _cell(t, v):
    """Index i with t[i] <= v < t[i+1], within [0, len(t) - 2]."""
    i = int(np.searchsorted(t, v, side='right')) - 1
    return min(max(i, 0), len(t) - 2)


def _hermite(v, t, i, s, m_i, m_j):
    h = t[i + 1] - t[i]
    u = (s - t[i]) / h
    return ((2 * u ** 3 - 3 * u ** 2 + 1) * v[i] + (u ** 3 - 2 * u ** 2 + u) * h * m_i
            + (-2 * u ** 3 + 3 * u ** 2) * v[i + 1] + (u ** 3 - u ** 2) * h * m_j)


def interp_1d(t, v, s):
    """Cubic Hermite interpolation of node values v at nodes t, at s (clamped into [t0, tn])."""
    s = min(max(s, t[0]), t[-1])
    i = _cell(t, s)
    return _hermite(v, t, i, s, _slope(v, t, i), _slope(v, t, i + 1))


def xf(grid, x, q2):
    """x f(x, Q^2) from the grid (lx [nx], lq [nq], values [nq][nx]); plain loops over points."""
    lx, lq, val = grid
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    q2 = np.broadcast_to(np.asarray(q2, dtype=np.float64), x.shape)
    out = np.empty(x.shape)
    for n in range(x.size):
        t = min(max(math.log(x.flat[n]), lx[0]), lx[-1])
        s = min(max(math.log(q2.flat[n]), lq[0]), lq[-1])
        j = _cell(lq, s)
        rows = [jj for jj in (j - 1, j, j + 1, j + 2) if 0 <= jj < len(lq)]
        col = {jj: interp_1d(lx, val[jj], t) for jj in rows}
        # the Q^2 Hermite needs the row values at j, j + 1 and the slopes there
        vq = np.array([col.get(jj, 0.0) for jj in range(len(lq))])

        def sl(k):
            return _slope(vq, lq, k)
        out.flat[n] = _hermite(vq, lq, j, s, sl(j), sl(j + 1))
    return out


def hadronic_variables(u_tau, u_y, S, tau0):
    """(x1, x2, y, s_hat, jacobian) from the two hadronic uniforms (numpy arrays)."""
    ltau0 = math.log(tau0)
    tau = np.exp((1.0 - u_tau) * ltau0)
    lti = -np.log(tau)
    y = (u_y - 0.5) * lti
    x1 = np.sqrt(tau) * np.exp(y)
    x2 = np.sqrt(tau) * np.exp(-y)
    jac = tau * (-ltau0) * lti
    return x1, x2, y, tau * S, jac


def lab_passes(p, y, params):
    """Cuts in the lab frame for partonic-frame momenta p [N, n_ext, 4] and boost rapidity y [N]."""
    boosted = p.clone()
    ch, sh = torch.cosh(torch.as_tensor(y)), torch.sinh(torch.as_tensor(y))
    E, pz = p[..., 0], p[..., 3]
    boosted[..., 0] = ch.unsqueeze(-1) * E + sh.unsqueeze(-1) * pz
    boosted[..., 3] = sh.unsqueeze(-1) * E + ch.unsqueeze(-1) * pz
    return passes(boosted, params)


def hadronic_integrand(proc, params, grid, S, u, with_me=True, grid_b=None):
    """u [d + 2][N] (u_tau, u_y, partonic uniforms) -> (F [N] in pb, pass mask, ME, momenta in the
    partonic c.m. frame [N, n_ext, 4], weight w = J f1 f2 W S / s_hat).  With with_me False the
    matrix element is not evaluated and F and ME are None.  grid is the density of parton 1,
    grid_b that of parton 2 (the same grid when None)."""
    u = np.asarray(u, dtype=np.float64)
    mt = params['m_t']
    tau0 = (2.0 * mt) ** 2 / S
    x1, x2, y, shat, jac = hadronic_variables(u[0], u[1], S, tau0)
    f1 = xf(grid, x1, mt * mt) / x1
    f2 = xf(grid if grid_b is None else grid_b, x2, mt * mt) / x2
    rs = torch.tensor(np.sqrt(shat))
    up = torch.tensor(np.ascontiguousarray(u[2:].T))
    k, W = phase_space(up, rs, out_masses(proc, params))
    p = torch.cat([incoming(up.shape[0], rs), k], 1)
    ok = lab_passes(p, y, params).numpy()
    Wn = W.numpy()
    w = jac * f1 * f2 * Wn * S / shat
    if not with_me:
        return None, ok, None, p, w
    m = partonic_me(proc, p, params)
    F = np.where(ok, jac * f1 * f2 * GEV2_TO_PB / (2.0 * shat) * Wn * m.numpy(), 0.0)
    return F, ok, m.numpy(), p, w


def sigma_pp_qq_tt_quadrature(grid_q, grid_qbar, S, params, n=64):
    """q(beam 1) qbar(beam 2) -> ttbar part of sigma(pp) in pb: Gauss-Legendre quadrature in
    (u_tau, u_y) of J f_q(x1) f_qbar(x2) times the closed-form LO partonic cross section
    8 pi alpha_s^2 beta (1 + rho/2) / (27 s_hat), rho = 4 m^2 / s_hat (no cuts act on tops)."""
    mt = params['m_t']
    tau0 = (2 * mt) ** 2 / S
    xg, wg = np.polynomial.legendre.leggauss(n)
    u = 0.5 * (xg + 1)
    w = 0.5 * wg
    tot = 0.0
    a2 = params['alpha_s'] ** 2
    for ui, wi in zip(u, w):
        x1, x2, y, shat, jac = hadronic_variables(np.full(n, ui), u, S, tau0)
        f = xf(grid_q, x1, mt * mt) / x1 * xf(grid_qbar, x2, mt * mt) / x2
        rho = 4 * mt * mt / shat
        beta = np.sqrt(np.maximum(1 - rho, 0.0))
        sig = 8 * math.pi * a2 * beta * (1 + rho / 2) / (27 * shat)
        tot += wi * (w * jac * f * sig).sum()
    return tot * GEV2_TO_PB


def sigma_pp_gg_tt_quadrature(grid, S, params, n=64):
    """gg -> ttbar part of sigma(pp) in pb: Gauss-Legendre quadrature in (u_tau, u_y) of
    J f(x1) f(x2) times the closed-form LO partonic cross section (no cuts act on tops)."""
    from .closed_forms import gg_tt_sigma
    mt = params['m_t']
    tau0 = (2 * mt) ** 2 / S
    xg, wg = np.polynomial.legendre.leggauss(n)
    u = 0.5 * (xg + 1)
    w = 0.5 * wg
    tot = 0.0
    for ui, wi in zip(u, w):
        x1, x2, y, shat, jac = hadronic_variables(np.full(n, ui), u, S, tau0)
        f = xf(grid, x1, mt * mt) / x1 * xf(grid, x2, mt * mt) / x2
        sig = np.array([gg_tt_sigma(sh, mt, params['alpha_s']) for sh in shat])
        tot += wi * (w * jac * f * sig).sum()
    return tot * GEV2_TO_PB
