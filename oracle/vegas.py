"""Vegas adaptive importance sampling (FP64).  Test infrastructure only.

The paper integrates with Vegas (sect. 1, citing G. P. Lepage, J. Comput. Phys.
27 (1978) 192 and CLNS-80/447); it gives no details.  This follows Lepage's
original separable-grid algorithm:

map     per dimension, i = floor(x nb), y = e_i + (x nb - i) (e_{i+1} - e_i),
        Jacobian J = prod_d nb (e_{i+1} - e_i)
estimate I_k = <F>, sigma_k^2 = (<F^2> - I_k^2)/(N - 1)
histogram h_{d,i} = sum of F^2 over the events whose x_d falls in bin i
smooth  hb_0 = (h_0 + h_1)/2, hb_i = (h_{i-1} + h_i + h_{i+1})/3, hb_last = (h_{-2} + h_{-1})/2
damp    rho_i = hb_i / sum hb,  r_i = ((1 - rho_i)/(-ln rho_i))^alpha  (r_i = 0 if rho_i = 0)
rebin   new edge k (k = 1..nb-1) where the running sum of r over old bins reaches
        k sum(r)/nb, linearly interpolated inside the old bin; e_0 = 0, e_nb = 1
combine I = sum(I_k/sigma_k^2)/sum(1/sigma_k^2), sigma = (sum 1/sigma_k^2)^(-1/2),
        chi2/dof = sum (I_k - I)^2/sigma_k^2 / (K - 1)
A dimension whose histogram is all zero keeps its grid.
"""
import math

import numpy as np


def uniform_grid(d, nb):
    return np.tile(np.linspace(0.0, 1.0, nb + 1), (d, 1))


def vegas_map(x, edges):
    """x [d][N] -> y [d][N], bin [d][N] (int), J [N]."""
    d, N = x.shape
    nb = edges.shape[1] - 1
    y = np.empty_like(x)
    b = np.empty(x.shape, dtype=np.int64)
    J = np.ones(N)
    for k in range(d):
        t = x[k] * nb
        i = np.minimum(np.floor(t).astype(np.int64), nb - 1)
        w = edges[k, i + 1] - edges[k, i]
        y[k] = edges[k, i] + (t - i) * w
        b[k] = i
        J *= nb * w
    return y, b, J


def accumulate(F, bins, nb):
    """(sum F, sum F^2, hist[d][nb] of F^2)."""
    F = np.asarray(F, dtype=np.float64)
    d = bins.shape[0]
    h = np.zeros((d, nb))
    for k in range(d):
        for i in range(nb):
            sel = bins[k] == i
            h[k, i] = (F[sel] ** 2).sum()
    return F.sum(), (F * F).sum(), h


def estimate(sum_f, sum_f2, N):
    I = sum_f / N
    var = (sum_f2 / N - I * I) / (N - 1)
    return I, var


def refine(edges, h, alpha=1.5):
    edges = np.array(edges, dtype=np.float64)
    d, nb1 = edges.shape
    nb = nb1 - 1
    new = edges.copy()
    for k in range(d):
        hk = h[k]
        if not (hk > 0).any():
            continue
        hb = np.empty(nb)
        hb[0] = (hk[0] + hk[1]) / 2.0
        hb[nb - 1] = (hk[nb - 2] + hk[nb - 1]) / 2.0
        for i in range(1, nb - 1):
            hb[i] = (hk[i - 1] + hk[i] + hk[i + 1]) / 3.0
        rho = hb / hb.sum()
        r = np.zeros(nb)
        for i in range(nb):
            if rho[i] <= 0.0:
                r[i] = 0.0
            elif rho[i] >= 1.0:
                r[i] = 1.0
            else:
                r[i] = ((1.0 - rho[i]) / (-math.log(rho[i]))) ** alpha
        total = r.sum()
        delta = total / nb
        old = edges[k]
        cum = 0.0
        i = 0
        for e in range(1, nb):
            target = e * delta
            while i < nb and cum + r[i] < target:
                cum += r[i]
                i += 1
            if i >= nb:
                new[k, e] = old[nb]
                continue
            if r[i] > 0.0:
                new[k, e] = old[i] + (target - cum) / r[i] * (old[i + 1] - old[i])
            else:
                new[k, e] = old[i]
        new[k, 0] = 0.0
        new[k, nb] = 1.0
    return new


def combine(Is, vars_):
    Is = np.asarray(Is)
    w = 1.0 / np.asarray(vars_)
    I = (Is * w).sum() / w.sum()
    sig = w.sum() ** -0.5
    chi2 = ((Is - I) ** 2 * w).sum() / max(len(Is) - 1, 1)
    return I, sig, chi2


def integrate(func, d, n, iters, seed, nb=50, alpha=1.5, uniforms=None):
    """Plain Vegas driver: func(y [d][N]) -> F [N]; returns (I, sigma, chi2, per-iter, edges)."""
    from .philox import uniforms as philox_uniforms
    draw = uniforms or philox_uniforms
    edges = uniform_grid(d, nb)
    Is, vs = [], []
    for it in range(iters):
        x = draw(seed, n, d, offset=it * n)
        y, b, J = vegas_map(x, edges)
        F = func(y) * J
        sf, sf2, h = accumulate(F, b, nb)
        I, v = estimate(sf, sf2, n)
        Is.append(I)
        vs.append(v)
        edges = refine(edges, h, alpha)
    I, sig, chi2 = combine(Is, vs)
    return I, sig, chi2, list(zip(Is, vs)), edges
