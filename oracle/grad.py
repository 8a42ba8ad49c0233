"""Reverse-mode gradient of the matrix element with respect to the random inputs and (m_t, alpha_s).

Test infrastructure only.  The paper notes that its custom operator has no
derivative and that adding one is straightforward (sect. 2); this module gives
the reference derivative by torch autograd (float64/complex128) through the
Vegas map, the phase space and the colour-ordered matrix element, and by
central finite differences for cross-checks.

Definitions (readings):
* ME(x; m_t, alpha_s) = matrix element at the momenta generated from x through
  the Vegas map (edges fixed) and the phase space (massive rescaling uses m_t).
* grad_x[d][n] = gbar_n dME_n/dx_{d,n}; grad_theta[n] = gbar_n (dME_n/dm_t,
  dME_n/dalpha_s), the m_t derivative being the total one at fixed x.
* ME scales as alpha_s^k (k gluons), so dME/dalpha_s = k ME / alpha_s; the
  scaling itself is tested by evaluating the oracle at two alpha_s values.
"""
import numpy as np
import torch

from . import me_ordered
from .integrand import momenta
from .phase_space import phase_space, incoming
from .processes import PROCESSES, out_masses


def vegas_map_torch(x, edges):
    """Differentiable Vegas map: x [N, d] tensor, edges [d][nb+1] numpy -> y [N, d]."""
    e = torch.tensor(np.asarray(edges), dtype=torch.float64)
    nb = e.shape[1] - 1
    t = x * nb
    i = torch.clamp(torch.floor(t.detach()).long(), max=nb - 1)
    lo = torch.stack([e[k][i[:, k]] for k in range(x.shape[1])], 1)
    hi = torch.stack([e[k][i[:, k] + 1] for k in range(x.shape[1])], 1)
    return lo + (t - i.to(torch.float64)) * (hi - lo)


def me_of_x(proc, params, x, edges=None, m_t=None):
    """ME [N] as a differentiable function of x [N, d] (and per-event m_t [N] if given)."""
    y = x if edges is None else vegas_map_torch(x, edges)
    N = x.shape[0]
    info = PROCESSES[proc]
    mt = params['m_t'] if m_t is None else m_t
    if m_t is None:
        masses = out_masses(proc, params)
    else:
        zeros = torch.zeros(N, dtype=torch.float64)
        masses = torch.stack([m_t, m_t] + [zeros] * info['n_out_gluons'], 1)
    k, w = phase_space(y, params['sqrt_s'], masses)
    p = torch.cat([incoming(N, params['sqrt_s']), k], 1)
    pp = dict(params)
    pp['m_t'] = mt
    return me_ordered.matrix_element(proc, p, pp)


def vjp(proc, params, x, gbar, edges=None):
    """x [d][N] numpy, gbar [N] -> (ME [N], grad_x [d][N], grad_theta [N][2])."""
    xt = torch.tensor(np.ascontiguousarray(np.asarray(x).T), dtype=torch.float64, requires_grad=True)
    N = xt.shape[0]
    mt = torch.full((N,), float(params['m_t']), dtype=torch.float64, requires_grad=True)
    me = me_of_x(proc, params, xt, edges, m_t=mt)
    gb = torch.as_tensor(np.asarray(gbar), dtype=torch.float64)
    (me * gb).sum().backward()
    k = PROCESSES[proc]['n_ext'] - 2
    dal = gb * k * me.detach() / params['alpha_s']
    gtheta = torch.stack([mt.grad, dal], 1)
    return me.detach().numpy(), xt.grad.numpy().T.copy(), gtheta.numpy()


def finite_difference(proc, params, x, edges=None, h=1e-6, hm_rel=1e-6):
    """Central differences of ME: (dME/dx [d][N], dME/dm_t [N])."""
    x = np.asarray(x, dtype=np.float64)
    d, N = x.shape

    def f(xx, mt):
        with torch.no_grad():
            pp = dict(params)
            pp['m_t'] = mt
            t = torch.tensor(np.ascontiguousarray(xx.T), dtype=torch.float64)
            return me_of_x(proc, pp, t, edges).numpy()

    gx = np.empty((d, N))
    for k in range(d):
        xp, xm = x.copy(), x.copy()
        xp[k] += h
        xm[k] -= h
        gx[k] = (f(xp, params['m_t']) - f(xm, params['m_t'])) / (2 * h)
    hm = hm_rel * params['m_t']
    gm = (f(x, params['m_t'] + hm) - f(x, params['m_t'] - hm)) / (2 * hm)
    return gx, gm
