"""Minkowski-space helpers (metric +,-,-,-).  Test infrastructure only.

Four-vectors are torch tensors with the Lorentz index LAST: [..., 4] = (E, px, py, pz).
"""
import torch

METRIC = torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=torch.float64)


def mdot(a, b):
    """Minkowski product a.b = a0 b0 - a.b (works for complex and real)."""
    g = METRIC.to(a.dtype) if not a.is_complex() else METRIC.to(torch.complex128)
    return (a * g * b).sum(-1)


def msq(a):
    return mdot(a, a)


def boost(p, q, M=None):
    """Boost p (given in the rest frame of q) to the frame in which q has momentum q.

    Standard pure boost with velocity q_vec/q0:
      E' = (q0 E + q.p)/M,   p' = p + q_vec (E + E')/(q0 + M),   M = sqrt(q^2).
    M may be passed when the invariant mass of q is known exactly; computing it
    as sqrt(q0^2 - |q|^2) cancels for a strongly boosted light system.
    """
    if M is None:
        M = torch.sqrt(msq(q))
    qp = (q[..., 1:] * p[..., 1:]).sum(-1)
    E = (q[..., 0] * p[..., 0] + qp) / M
    fac = (p[..., 0] + E) / (q[..., 0] + M)
    vec = p[..., 1:] + q[..., 1:] * fac.unsqueeze(-1)
    return torch.cat([E.unsqueeze(-1), vec], -1)


def general_boost(p, beta):
    """Boost p by velocity vector beta[...,3] (|beta|<1)."""
    b2 = (beta * beta).sum(-1)
    gam = 1.0 / torch.sqrt(1.0 - b2)
    bp = (beta * p[..., 1:]).sum(-1)
    gam2 = torch.where(b2 > 0, (gam - 1.0) / torch.where(b2 > 0, b2, torch.ones_like(b2)), torch.zeros_like(b2))
    E = gam * (p[..., 0] + bp)
    vec = p[..., 1:] + (gam2 * bp + gam * p[..., 0]).unsqueeze(-1) * beta
    return torch.cat([E.unsqueeze(-1), vec], -1)


def rotate(p, R):
    """Spatial rotation by a 3x3 matrix R."""
    vec = p[..., 1:] @ R.T
    return torch.cat([p[..., :1], vec], -1)


def pt(p):
    return torch.sqrt(p[..., 1] ** 2 + p[..., 2] ** 2)


def pabs(p):
    return torch.sqrt(p[..., 1] ** 2 + p[..., 2] ** 2 + p[..., 3] ** 2)


def eta(p):
    """Pseudorapidity atanh(pz/|p|)."""
    return torch.atanh(p[..., 3] / pabs(p))


def phi(p):
    return torch.atan2(p[..., 2], p[..., 1])
