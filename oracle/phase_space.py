"""Phase-space sampling (FP64).  Test infrastructure only.

The paper does not describe its phase-space generator; the sampler used here is
RAMBO on diet (S. Plaetzer, "RAMBO on diet", arXiv:1308.2922), which maps
3n-4 uniform numbers onto massless n-body phase space with constant weight,
followed by the massive rescaling of RAMBO (R. Kleiss, W. J. Stirling,
S. D. Ellis, Comput. Phys. Commun. 40 (1986) 359).  Classic 4n-number RAMBO
(same reference) is provided for cross-checks only.

Conventions (readings the paper leaves open):
* uniforms: the n-2 intermediate-mass numbers first, then (cos theta, phi)
  pairs in emission order; cos theta = 2u-1, phi = 2 pi u';
* particles are emitted in the order of the ``masses`` list; for the gg
  processes that is t, tbar, then the final gluons;
* the two incoming partons run along +z and -z with E = sqrt(s)/2 each;
* sqrt(s) is one value for all events or a tensor with one value per event
  (hadronic events, whose partonic energy varies);
* the weight is the phase-space measure
  dPhi_n = (2pi)^4 delta^4(P - sum p) prod d^3p/((2pi)^3 2E)  per point.

All functions take torch float64 tensors and are differentiable by autograd:
the two one-dimensional root solves are done by bisection (obviously convergent)
and then one Newton step is taken under autograd, which leaves the value
unchanged to rounding and gives the implicit-function derivative.
"""
import math
import torch

from .kinematics import boost

TWO_PI = 2.0 * math.pi


def massless_volume(n, s):
    """Volume of massless n-body phase space at c.m. energy squared s."""
    return (TWO_PI ** (4 - 3 * n) * (math.pi / 2.0) ** (n - 1) * s ** (n - 2)
            / (math.factorial(n - 1) * math.factorial(n - 2)))


def _per_event(sqrt_s, N):
    """sqrt(s) as a [N] float64 tensor: one value for all events, or one per event (the
    partonic energy of hadronic events)."""
    if torch.is_tensor(sqrt_s):
        return sqrt_s.to(torch.float64).expand(N).clone() if sqrt_s.dim() == 0 else sqrt_s.to(torch.float64)
    return torch.full((N,), float(sqrt_s), dtype=torch.float64)


def _bisect(f, lo, hi, iters=200):
    """Root of an increasing function f on [lo, hi] (elementwise tensors)."""
    lo = lo.clone()
    hi = hi.clone()
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        pos = f(mid) > 0
        hi = torch.where(pos, mid, hi)
        lo = torch.where(pos, lo, mid)
    return 0.5 * (lo + hi)


def _mass_ratio(u, a):
    """Solve u = (a+1) r^(2a) - a r^(2(a+1)) for r in [0,1] (a = n - i >= 1).

    The right-hand side is the cumulative distribution of r = M_i/M_{i-1} for
    massless n-body phase space factorised into a 2-body decay times the
    (a+1)-body remainder, whose volume grows as M^(2a-2); it is increasing on
    [0, 1] from 0 to 1.
    """
    def G(r, uu):
        return (a + 1) * r ** (2 * a) - a * r ** (2 * (a + 1)) - uu

    with torch.no_grad():
        ud = u.detach()
        r0 = _bisect(lambda r: G(r, ud), torch.zeros_like(ud), torch.ones_like(ud))
    # one Newton step under autograd: value unchanged, derivative = implicit one
    dG = 2 * a * (a + 1) * r0 ** (2 * a - 1) * (1 - r0 * r0)
    return r0 - G(r0, u) / dG


def rambo_diet_massless(u, sqrt_s):
    """Massless n-body momenta from 3n-4 uniforms.

    u: [N, 3n-4] float64.  Returns p [N, n, 4] in the c.m. frame and the
    (constant) weight [N].
    """
    N, d = u.shape
    n = (d + 4) // 3
    assert 3 * n - 4 == d and n >= 2
    rs = _per_event(sqrt_s, N)
    M = [rs]
    for i in range(2, n):
        r = _mass_ratio(u[:, i - 2], n - i)
        M.append(r * M[-1])
    M.append(torch.zeros(N, dtype=torch.float64))   # M_n = 0
    Q = torch.zeros(N, 4, dtype=torch.float64)
    Q[:, 0] = rs
    ps = []
    for i in range(1, n):
        Mi, Mn = M[i - 1], M[i]
        q = (Mi * Mi - Mn * Mn) / (2.0 * Mi)
        cth = 2.0 * u[:, (n - 2) + 2 * (i - 1)] - 1.0
        ph = TWO_PI * u[:, (n - 2) + 2 * (i - 1) + 1]
        sth = torch.sqrt(torch.clamp(1.0 - cth * cth, min=0.0))
        nvec = torch.stack([sth * torch.cos(ph), sth * torch.sin(ph), cth], -1)
        p_rest = torch.cat([q.unsqueeze(-1), q.unsqueeze(-1) * nvec], -1)
        Qn_rest = torch.cat([torch.sqrt(q * q + Mn * Mn).unsqueeze(-1), -q.unsqueeze(-1) * nvec], -1)
        # Q has invariant mass M_i by construction; use it (no cancellation)
        p_lab = boost(p_rest, Q, Mi)
        Q = boost(Qn_rest, Q, Mi)
        ps.append(p_lab)
    ps.append(Q)
    p = torch.stack(ps, 1)
    w = massless_volume(n, rs * rs)
    return p, w


def massive_rescale(p, masses, sqrt_s):
    """RAMBO massive rescaling of massless c.m. momenta p [N, n, 4].

    Solve sum_i sqrt(m_i^2 + xi^2 E_i^2) = sqrt(s) for xi in (0, 1], set
    k_i = (sqrt(m_i^2 + xi^2 E_i^2), xi p_i) and return (k, weight factor)
    with weight factor
      (sum|k_i|/sqrt s)^(2n-3) * prod(|k_i|/k_i0) * sqrt s / sum(|k_i|^2/k_i0).
    """
    n = p.shape[1]
    m = masses if torch.is_tensor(masses) else torch.tensor(masses, dtype=torch.float64)
    if m.dim() == 1:
        m = m.unsqueeze(0)                       # [1, n] or per-event [N, n]
    if not m.requires_grad and float(m.abs().sum()) == 0.0:
        return p, torch.ones(p.shape[0], dtype=torch.float64)
    E = p[..., 0]
    m2 = m * m

    def F(xi, EE):
        return torch.sqrt(m2 + (xi.unsqueeze(-1) * EE) ** 2).sum(-1) - sqrt_s

    with torch.no_grad():
        Ed = E.detach()
        xi0 = _bisect(lambda x: F(x, Ed), torch.zeros(p.shape[0], dtype=torch.float64),
                      torch.ones(p.shape[0], dtype=torch.float64))
    dF = ((xi0.unsqueeze(-1) * E * E) / torch.sqrt(m2 + (xi0.unsqueeze(-1) * E) ** 2)).sum(-1)
    xi = xi0 - F(xi0, E) / dF
    k0 = torch.sqrt(m2 + (xi.unsqueeze(-1) * E) ** 2)
    kvec = xi.unsqueeze(-1).unsqueeze(-1) * p[..., 1:]
    k = torch.cat([k0.unsqueeze(-1), kvec], -1)
    kabs = torch.sqrt((kvec * kvec).sum(-1))
    fac = ((kabs.sum(-1) / sqrt_s) ** (2 * n - 3) * (kabs / k0).prod(-1)
           * sqrt_s / (kabs * kabs / k0).sum(-1))
    return k, fac


def phase_space(u, sqrt_s, masses):
    """Outgoing momenta [N, n, 4] and phase-space weight [N] for 3n-4 uniforms."""
    p, w = rambo_diet_massless(u, sqrt_s)
    k, fac = massive_rescale(p, masses, sqrt_s)
    return k, w * fac


def incoming(N, sqrt_s):
    """Two incoming massless partons along +z and -z, [N, 2, 4] (sqrt_s one value or [N])."""
    E = 0.5 * _per_event(sqrt_s, N)
    z = torch.zeros(N, dtype=torch.float64)
    a = torch.stack([E, z, z, E], -1)
    b = torch.stack([E, z, z, -E], -1)
    return torch.stack([a, b], 1)


def classic_rambo(u, sqrt_s):
    """Classic massless RAMBO with 4 uniforms per particle, u [N, 4n]; weight = volume."""
    N, d = u.shape
    n = d // 4
    uu = u.view(N, n, 4)
    c = 2.0 * uu[..., 0] - 1.0
    ph = TWO_PI * uu[..., 1]
    q0 = -torch.log(uu[..., 2] * uu[..., 3])
    s = torch.sqrt(1.0 - c * c)
    q = torch.stack([q0, q0 * s * torch.cos(ph), q0 * s * torch.sin(ph), q0 * c], -1)
    Q = q.sum(1)
    M = torch.sqrt(Q[:, 0] ** 2 - (Q[:, 1:] ** 2).sum(-1))
    b = -Q[:, 1:] / M.unsqueeze(-1)
    x = sqrt_s / M
    gam = Q[:, 0] / M
    a = 1.0 / (1.0 + gam)
    bq = (b.unsqueeze(1) * q[..., 1:]).sum(-1)
    p0 = x.unsqueeze(-1) * (gam.unsqueeze(-1) * q[..., 0] + bq)
    pv = x.unsqueeze(-1).unsqueeze(-1) * (q[..., 1:] + b.unsqueeze(1) * q[..., :1]
                                          + (a.unsqueeze(-1) * bq).unsqueeze(-1) * b.unsqueeze(1))
    p = torch.cat([p0.unsqueeze(-1), pv], -1)
    w = torch.full((N,), massless_volume(n, float(sqrt_s) ** 2), dtype=torch.float64)
    return p, w
