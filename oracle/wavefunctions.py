"""External wavefunctions in HELAS conventions (FP64/complex128).  Test infrastructure only.

The paper's generated code builds each matrix element from external
wavefunctions, vertices and propagators (sect. 2, Fig. 2: the wavefunction and
vertex function files fed to the code writer); it does not print their form.
The forms below follow H. Murayama, I. Watanabe, K. Hagiwara, "HELAS: HELicity
Amplitude Subroutines for Feynman diagram evaluations", KEK-91-11 (chiral
representation of the Dirac matrices):

  gamma^0 = [[0, 1], [1, 0]],  gamma^k = [[0, sigma^k], [-sigma^k, 0]]
  chi_+(p) = (|p|+pz, px+i py) / sqrt(2|p|(|p|+pz))
  chi_-(p) = (-px+i py, |p|+pz) / sqrt(2|p|(|p|+pz))
  (p along -z: chi_+ = (0, 1), chi_- = (-1, 0); p = 0: chi along +z;
   |p|+pz is evaluated as pT^2/(|p|-pz) when pz < 0, its cancellation-free form)
  u(p, l) = ( w_{-l} chi_l ,  w_{+l} chi_l ),   w_{+-} = sqrt(E +- |p|)
  v(p, l) = ( -l w_{+l} chi_{-l} ,  l w_{-l} chi_{-l} )
  eps(k, l) = (-l e1 - i e2)/sqrt(2),
     e1 = (0, cos th cos ph, cos th sin ph, -sin th),  e2 = (0, -sin ph, cos ph, 0)

w_- is evaluated as m / w_+ (equal to sqrt(E - |p|) on shell, exact zero for
massless particles).  Incoming gluons carry eps, outgoing gluons eps*.
Spinors are column vectors [..., 4]; barred spinors are rows psi^dagger gamma^0.
"""
import math
import torch

C128 = torch.complex128


def _sigma():
    s1 = torch.tensor([[0, 1], [1, 0]], dtype=C128)
    s2 = torch.tensor([[0, -1j], [1j, 0]], dtype=C128)
    s3 = torch.tensor([[1, 0], [0, -1]], dtype=C128)
    return s1, s2, s3


def gamma_matrices():
    """gamma^mu as a [4 (mu), 4, 4] complex tensor (chiral representation)."""
    z = torch.zeros(2, 2, dtype=C128)
    one = torch.eye(2, dtype=C128)
    g = [torch.cat([torch.cat([z, one], 1), torch.cat([one, z], 1)], 0)]
    for s in _sigma():
        g.append(torch.cat([torch.cat([z, s], 1), torch.cat([-s, z], 1)], 0))
    return torch.stack(g, 0)


GAMMA = gamma_matrices()
GAMMA5 = torch.diag(torch.tensor([-1, -1, 1, 1], dtype=C128))


def slash(a):
    """a_mu gamma^mu for a[..., 4] (upper-index components) -> [..., 4, 4]."""
    a = a.to(C128)
    g = torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=C128)
    return torch.einsum('...m,mij->...ij', a * g, GAMMA)


def chi(p, lam):
    """Two-component helicity eigenstate of sigma.p_hat with eigenvalue lam."""
    px, py, pz = p[..., 1], p[..., 2], p[..., 3]
    pt2 = px * px + py * py
    pa = torch.sqrt(pt2 + pz * pz)
    # |p| + pz, written as pT^2/(|p| - pz) for pz < 0 (same value, no cancellation)
    s = torch.where(pz >= 0, pa + pz, pt2 / torch.where(pa - pz > 0, pa - pz, torch.ones_like(pa)))
    ok = s > 0
    ss = torch.where(ok, s, torch.ones_like(s))
    pas = torch.where(pa > 0, pa, torch.ones_like(pa))
    norm = torch.sqrt(2.0 * pas * ss)
    zero = torch.zeros_like(px)
    if lam > 0:
        c0 = torch.complex(s, zero) / norm
        c1 = torch.complex(px, py) / norm
        d0 = torch.zeros_like(c0)
        d1 = torch.ones_like(c0)
    else:
        c0 = torch.complex(-px, py) / norm
        c1 = torch.complex(s, zero) / norm
        d0 = -torch.ones_like(c0)
        d1 = torch.zeros_like(c0)
    # p along -z (pa>0, s=0): limits given above; p = 0: quantise along +z
    at_rest = pa == 0
    if lam > 0:
        r0, r1 = torch.ones_like(c0), torch.zeros_like(c0)
    else:
        r0, r1 = torch.zeros_like(c0), torch.ones_like(c0)
    c0 = torch.where(ok, c0, torch.where(at_rest, r0, d0))
    c1 = torch.where(ok, c1, torch.where(at_rest, r1, d1))
    return torch.stack([c0, c1], -1)


def _omegas(p, m):
    pa = torch.sqrt(p[..., 1] ** 2 + p[..., 2] ** 2 + p[..., 3] ** 2)
    wp = torch.sqrt(p[..., 0] + pa)
    wm = m / wp
    return wp, wm


def u_spinor(p, m, lam):
    wp, wm = _omegas(p, m)
    c = chi(p, lam)
    lo, hi = (wm, wp) if lam > 0 else (wp, wm)      # w_{-l}, w_{+l}
    return torch.cat([lo.unsqueeze(-1) * c, hi.unsqueeze(-1) * c], -1)


def v_spinor(p, m, lam):
    wp, wm = _omegas(p, m)
    c = chi(p, -lam)
    wpl, wml = (wp, wm) if lam > 0 else (wm, wp)    # w_{+l}, w_{-l}
    return torch.cat([(-lam * wpl).unsqueeze(-1) * c, (lam * wml).unsqueeze(-1) * c], -1)


def bar(psi):
    """Dirac adjoint psi^dagger gamma^0 (row spinor)."""
    return torch.einsum('...i,ij->...j', psi.conj(), GAMMA[0])


def polarisation(k, lam):
    """eps^mu(k, lam) for a massless vector boson, [..., 4] complex."""
    kx, ky, kz = k[..., 1], k[..., 2], k[..., 3]
    ka = torch.sqrt(kx * kx + ky * ky + kz * kz)
    kt = torch.sqrt(kx * kx + ky * ky)
    has_t = kt > 0
    kts = torch.where(has_t, kt, torch.ones_like(kt))
    cph = torch.where(has_t, kx / kts, torch.ones_like(kt))
    sph = torch.where(has_t, ky / kts, torch.zeros_like(kt))
    cth = kz / ka
    sth = kt / ka
    zero = torch.zeros_like(kx)
    e1 = torch.stack([zero, cth * cph, cth * sph, -sth], -1)
    e2 = torch.stack([zero, -sph, cph, zero], -1)
    return torch.complex(-lam * e1, -e2) / math.sqrt(2.0)
