"""Pins for the oracle's external wavefunctions and colour algebra (CPU only).

Dirac equation, normalisation and completeness of spinors; transversality,
normalisation and completeness of polarisation vectors; SU(3) identities and
Casimir values of the colour matrices.
"""
import math

import numpy as np
import pytest
import torch

from oracle import colour
from oracle.wavefunctions import (GAMMA, GAMMA5, bar, chi, polarisation, slash,
                                  u_spinor, v_spinor)

C128 = torch.complex128


def _momenta(m, N=50, seed=0):
    g = torch.Generator().manual_seed(seed)
    pv = (torch.rand(N, 3, generator=g, dtype=torch.float64) - 0.5) * 800
    pv[0] = torch.tensor([0.0, 0.0, -300.0])    # along -z
    pv[1] = torch.tensor([0.0, 0.0, 250.0])     # along +z
    E = torch.sqrt((pv ** 2).sum(-1) + m * m)
    return torch.cat([E.unsqueeze(-1), pv], -1)


def _eye(N):
    return torch.eye(4, dtype=C128).expand(N, 4, 4)


@pytest.mark.parametrize('m', [0.0, 173.0])
def test_dirac_equation(m):
    p = _momenta(m)
    ps = slash(p)
    for lam in (-1, 1):
        u = u_spinor(p, m, lam)
        v = v_spinor(p, m, lam)
        scale = p[:, 0].view(-1, 1) * torch.sqrt(p[:, 0]).view(-1, 1)
        assert ((torch.einsum('nij,nj->ni', ps - m * _eye(len(p)), u)).abs() / scale).max() < 1e-13
        assert ((torch.einsum('nij,nj->ni', ps + m * _eye(len(p)), v)).abs() / scale).max() < 1e-13


@pytest.mark.parametrize('m', [0.0, 173.0])
def test_spinor_normalisation_and_completeness(m):
    p = _momenta(m)
    N = len(p)
    su = torch.zeros(N, 4, 4, dtype=C128)
    sv = torch.zeros(N, 4, 4, dtype=C128)
    for lam in (-1, 1):
        u = u_spinor(p, m, lam)
        v = v_spinor(p, m, lam)
        ub = bar(u)
        vb = bar(v)
        assert ((torch.einsum('ni,ni->n', ub, u) - 2 * m).abs() / p[:, 0]).max() < 1e-13
        assert ((torch.einsum('ni,ni->n', vb, v) + 2 * m).abs() / p[:, 0]).max() < 1e-13
        # u^dagger u = 2E
        assert ((torch.einsum('ni,ni->n', u.conj(), u).real - 2 * p[:, 0]).abs() / p[:, 0]).max() < 1e-13
        su = su + torch.einsum('ni,nj->nij', u, ub)
        sv = sv + torch.einsum('ni,nj->nij', v, vb)
    e = p[:, 0].view(-1, 1, 1)
    assert ((su - (slash(p) + m * _eye(N))).abs() / e).max() < 1e-13
    assert ((sv - (slash(p) - m * _eye(N))).abs() / e).max() < 1e-13


def test_massless_spinors_are_chiral_helicity_states():
    p = _momenta(0.0)
    for lam in (-1, 1):
        u = u_spinor(p, 0.0, lam)
        # gamma5 u = lam u for massless u (right-handed = +1)
        g5u = torch.einsum('ij,nj->ni', GAMMA5, u)
        assert (g5u - lam * u).abs().max() < 1e-10
        # helicity eigenstate of the two-spinor
        c = chi(p, lam)
        pv = p[:, 1:].to(C128)
        sig = [torch.tensor(s, dtype=C128) for s in ([[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]])]
        sp = sum(pv[:, k].view(-1, 1, 1) * sig[k] for k in range(3))
        pa = torch.sqrt((p[:, 1:] ** 2).sum(-1)).view(-1, 1)
        assert (torch.einsum('nij,nj->ni', sp, c) - lam * pa * c).abs().max() < 1e-9


def test_polarisation_vectors():
    k = _momenta(0.0)
    N = len(k)
    g = torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=C128)
    # reference vector n = (1, -khat) for the light-cone completeness relation
    kh = k[:, 1:] / k[:, :1]
    n = torch.cat([torch.ones(N, 1, dtype=torch.float64), -kh], -1)
    comp = torch.zeros(N, 4, 4, dtype=C128)
    for lam in (-1, 1):
        e = polarisation(k, lam)
        assert ((e * g * k.to(C128)).sum(-1)).abs().max() < 1e-12
        assert ((e * g * e.conj()).sum(-1) + 1).abs().max() < 1e-14
        assert ((e * g * e).sum(-1)).abs().max() < 1e-14
        comp = comp + torch.einsum('ni,nj->nij', e, e.conj())
    kn = (k * g.real * n).sum(-1).view(-1, 1, 1)
    gmn = torch.diag(g).expand(N, 4, 4)
    rhs = -gmn + (torch.einsum('ni,nj->nij', k, n) + torch.einsum('ni,nj->nij', n, k)) / kn
    assert (comp - rhs.to(C128)).abs().max() < 1e-12


def test_su3_algebra():
    T, F = colour.T, colour.F
    # [t^a, t^b] = i f^abc t^c, Tr t^a t^b = delta/2, f totally antisymmetric
    comm = np.einsum('aij,bjk->abik', T, T) - np.einsum('bij,ajk->abik', T, T)
    assert np.abs(comm - 1j * np.einsum('abc,cik->abik', F, T)).max() < 1e-14
    assert np.abs(np.einsum('aij,bji->ab', T, T) - 0.5 * np.eye(8)).max() < 1e-15
    assert np.abs(F + F.transpose(1, 0, 2)).max() < 1e-15
    assert np.abs(F + F.transpose(0, 2, 1)).max() < 1e-15
    # textbook values (Gell-Mann basis)
    assert abs(F[0, 1, 2] - 1) < 1e-15
    assert abs(F[3, 4, 7] - math.sqrt(3) / 2) < 1e-15
    assert abs(F[0, 3, 6] - 0.5) < 1e-15
    # Casimirs: t^a t^a = C_F 1, f^acd f^bcd = C_A delta
    assert np.abs(np.einsum('aij,ajk->ik', T, T) - 4 / 3 * np.eye(3)).max() < 1e-14
    assert np.abs(np.einsum('acd,bcd->ab', F, F) - 3 * np.eye(8)).max() < 1e-13


@pytest.mark.parametrize('k,den', [(2, 3), (3, 9), (4, 54)])
def test_colour_matrix_properties(k, den):
    C = colour.colour_matrix(k)
    Cf, d = colour.colour_matrix_exact(k)
    assert d == den
    assert np.allclose(C, C.T, rtol=0, atol=1e-13)
    assert np.linalg.eigvalsh(C).min() > 0
    # diagonal = N C_F^k (t^a t^a = C_F repeatedly)
    assert np.allclose(np.diag(C), 3 * (4 / 3) ** k, rtol=1e-13)
    # every numerator an exact small integer: exact in bf16 (|n| <= 256 or power of two)
    for row in Cf:
        for v in row:
            n = int(v * den)
            assert abs(n) <= 256 or (abs(n) & (abs(n) - 1)) == 0


def test_colour_matrix_k2_casimir_form():
    # off-diagonal: Tr(t^a t^b t^a t^b) = N C_F (C_F - C_A/2) = -2/3
    C = colour.colour_matrix(2)
    assert abs(C[0, 1] + 2 / 3) < 1e-14


def test_colour_matrix_k3_k4_numerators():
    _, d3 = colour.colour_matrix_exact(3)
    C3 = np.rint(colour.colour_matrix(3) * 9).astype(int)
    assert set(np.unique(C3)) == {64, 10, 1, -8}
    C4 = np.rint(colour.colour_matrix(4) * 54).astype(int)
    assert set(np.unique(C4)) == {512, 80, 71, 62, 8, -1, -10, -28, -64}
