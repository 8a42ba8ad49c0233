"""Pins for the oracle's phase-space sampler (CPU only).

Independent references: the recursive phase-space factorisation
Phi_n(s) = int dq^2/(2 pi) Phi_2(s; m_1, q) Phi_{n-1}(q^2; m_2..m_n) with
Phi_2(s; a, b) = lambda^(1/2)(s, a^2, b^2)/(8 pi s) (PDG kinematics review),
evaluated by numerical quadrature; the massless one-particle energy spectrum
f(x) = (n-1)(n-2) x (1-x)^(n-3), x = 2E/sqrt(s); isotropy; and classic RAMBO.
"""
import math

import numpy as np
import pytest
import torch
from scipy import integrate

from oracle import phase_space as ps
from oracle import philox
from oracle.kinematics import msq

SQRT_S = 1000.0
MT = 173.0


def lam(a, b, c):
    return a * a + b * b + c * c - 2 * a * b - 2 * a * c - 2 * b * c


def phi2(s, ma, mb):
    l = lam(s, ma * ma, mb * mb)
    return math.sqrt(max(l, 0.0)) / (8 * math.pi * s)


def phi3_m00(s, m):
    f = lambda q2: phi2(s, m, math.sqrt(q2)) * phi2(q2, 0.0, 0.0) / (2 * math.pi)
    return integrate.quad(f, 0.0, (math.sqrt(s) - m) ** 2, epsabs=0, epsrel=1e-12, limit=200)[0]


def phi3_000(s):
    return phi3_m00(s, 0.0)


def phi4_mm00(s, m):
    f = lambda q2: phi2(s, m, math.sqrt(q2)) * phi3_m00(q2, m) / (2 * math.pi)
    return integrate.quad(f, m * m, (math.sqrt(s) - m) ** 2, epsabs=0, epsrel=1e-10, limit=200)[0]


def phi4_0000(s):
    f = lambda q2: phi2(s, 0.0, math.sqrt(q2)) * phi3_000(q2) / (2 * math.pi)
    return integrate.quad(f, 0.0, s, epsabs=0, epsrel=1e-12, limit=200)[0]


def _sample(n, N, seed, masses=None):
    u = torch.tensor(philox.uniforms(seed, N, 3 * n - 4).T.copy())
    if masses is None:
        return ps.rambo_diet_massless(u, SQRT_S)
    return ps.phase_space(u, SQRT_S, masses)


def test_two_body_volume_textbook():
    # int dPhi_2 = 1/(8 pi) for massless particles
    assert abs(ps.massless_volume(2, SQRT_S ** 2) - 1 / (8 * math.pi)) < 1e-17


@pytest.mark.parametrize('n,ref', [(3, phi3_000), (4, phi4_0000)])
def test_massless_volume_vs_recursive_quadrature(n, ref):
    s = SQRT_S ** 2
    assert abs(ps.massless_volume(n, s) / ref(s) - 1) < 1e-9


@pytest.mark.parametrize('n', [2, 3, 4])
def test_massless_weight_constant_and_momentum_conservation(n):
    p, w = _sample(n, 5000, 3)
    assert torch.all(w == ps.massless_volume(n, SQRT_S ** 2))
    tot = p.sum(1)
    assert (tot[:, 0] - SQRT_S).abs().max() < 1e-12 * SQRT_S
    assert tot[:, 1:].abs().max() < 1e-12 * SQRT_S
    assert (msq(p).abs() / p[..., 0] ** 2).max() < 1e-12


@pytest.mark.parametrize('n', [3, 4])
def test_massless_energy_spectrum_every_particle(n):
    N = 200000
    p, _ = _sample(n, N, 5 + n)
    x = (2 * p[..., 0] / SQRT_S).numpy()
    m1, m2 = 2 / n, 6 / (n * (n + 1))
    sd1 = math.sqrt(m2 - m1 * m1) / math.sqrt(N)
    for i in range(n):
        assert abs(x[:, i].mean() - m1) < 5 * sd1, (i, x[:, i].mean(), m1)
        assert abs((x[:, i] ** 2).mean() - m2) < 5 * 2 * sd1, i


@pytest.mark.parametrize('n', [3, 4])
def test_massless_isotropy_every_particle(n):
    N = 200000
    p, _ = _sample(n, N, 21 + n)
    c = (p[..., 3] / torch.sqrt((p[..., 1:] ** 2).sum(-1))).numpy()
    for i in range(n):
        assert abs(c[:, i].mean()) < 5 * math.sqrt(1 / 3 / N)
        assert abs((c[:, i] ** 2).mean() - 1 / 3) < 5 * math.sqrt(4 / 45 / N)


def test_massless_three_body_dalitz_plot_is_flat():
    """With a constant weight, massless three-body events fill the Dalitz triangle
    x1 + x2 >= 1, x1, x2 <= 1 (x_i = 2E_i/sqrt(s), equivalently s23 = s(1 - x1),
    s13 = s(1 - x2)) uniformly: the three-body phase-space density is flat in two
    invariant masses.  Checked by a chi-square over the 45 cells of a 10 x 10 grid
    that lie wholly inside the triangle, and by the fraction on the diagonal cells."""
    N = 200000
    p, w = _sample(3, N, 41)
    assert float(w.std()) <= 1e-12 * float(w.mean())
    x = (2 * p[..., 0] / SQRT_S).numpy()
    x1, x2 = x[:, 0], x[:, 1]
    assert (x1 + x2 >= 1 - 1e-12).all() and (x1 <= 1 + 1e-12).all() and (x2 <= 1 + 1e-12).all()
    i = np.minimum((x1 * 10).astype(int), 9)
    j = np.minimum((x2 * 10).astype(int), 9)
    counts = np.zeros((10, 10))
    np.add.at(counts, (i, j), 1)
    full = np.add.outer(np.arange(10), np.arange(10)) >= 10
    expect = N * 0.01 / 0.5
    chi2 = float((((counts[full] - expect) ** 2) / expect).sum())
    assert full.sum() == 45 and chi2 < 45 + 5 * math.sqrt(2 * 45), chi2
    # the 10 cells the diagonal cuts hold half a full cell's area each
    diag = np.add.outer(np.arange(10), np.arange(10)) == 9
    frac = counts[diag].sum() / N
    assert abs(frac - 0.1) < 5 * math.sqrt(0.1 * 0.9 / N), frac


def test_diet_matches_classic_rambo_pair_invariants():
    n, N = 4, 200000
    p, _ = _sample(n, N, 31)
    u = torch.tensor(philox.uniforms(32, N, 4 * n).T.copy())
    q, _ = ps.classic_rambo(u, SQRT_S)
    s = SQRT_S ** 2
    for a, b in [(0, 1), (0, 3), (2, 3)]:
        x = (msq(p[:, a] + p[:, b]) / s).numpy()
        y = (msq(q[:, a] + q[:, b]) / s).numpy()
        assert abs(x.mean() - 2 / (n * (n - 1))) < 5 * x.std() / math.sqrt(N)
        err = math.sqrt(x.var() / N + y.var() / N)
        assert abs((x ** 2).mean() - (y ** 2).mean()) < 5 * math.sqrt((x ** 2).var() / N + (y ** 2).var() / N)
        assert abs(x.mean() - y.mean()) < 5 * err


def test_two_body_massive_weight_exact():
    p, w = _sample(2, 1000, 4, masses=[MT, MT])
    beta = math.sqrt(1 - 4 * MT * MT / SQRT_S ** 2)
    assert torch.allclose(w, torch.full_like(w, beta / (8 * math.pi)), rtol=1e-14, atol=0)
    pabs = torch.sqrt((p[..., 1:] ** 2).sum(-1))
    assert (pabs / (beta * SQRT_S / 2) - 1).abs().max() < 1e-14


@pytest.mark.parametrize('n,masses', [(3, [MT, MT, 0.0]), (4, [MT, MT, 0.0, 0.0])])
def test_massive_on_shell_and_conservation(n, masses):
    p, w = _sample(n, 20000, 9, masses=masses)
    m2 = torch.tensor(masses) ** 2
    assert ((msq(p) - m2).abs() / p[..., 0] ** 2).max() < 1e-10
    tot = p.sum(1)
    assert (tot[:, 0] - SQRT_S).abs().max() < 1e-12 * SQRT_S
    assert tot[:, 1:].abs().max() < 1e-12 * SQRT_S
    assert torch.all(w > 0)


@pytest.mark.parametrize('n,masses,ref', [
    (3, [MT, MT, 0.0], lambda s: None),
    (4, [MT, MT, 0.0, 0.0], lambda s: phi4_mm00(s, MT)),
])
def test_massive_volume_vs_quadrature(n, masses, ref):
    s = SQRT_S ** 2
    if n == 3:
        # Phi_3(s; m, m, 0) = int dq^2/(2pi) Phi_2(s; m, q) Phi_2(q^2; m, 0)
        f = lambda q2: phi2(s, MT, math.sqrt(q2)) * phi2(q2, MT, 0.0) / (2 * math.pi)
        want = integrate.quad(f, MT * MT, (SQRT_S - MT) ** 2, epsabs=0, epsrel=1e-12, limit=200)[0]
    else:
        want = ref(s)
    N = 200000
    _, w = _sample(n, N, 40 + n, masses=masses)
    w = w.numpy()
    assert abs(w.mean() - want) < 5 * w.std() / math.sqrt(N), (w.mean(), want)


def test_mass_ratio_solver_inverts_cdf():
    u = torch.tensor(np.linspace(0.001, 0.999, 101))
    for a in (1, 2, 3):
        r = ps._mass_ratio(u, a)
        back = (a + 1) * r ** (2 * a) - a * r ** (2 * (a + 1))
        assert (back - u).abs().max() < 1e-14


def test_conservation_for_strongly_boosted_light_subsystem():
    # tiny intermediate-mass uniforms give a light, strongly boosted remainder
    # system; momentum must still balance to FP64 rounding
    n = 4
    u = torch.tensor(philox.uniforms(6, 64, 3 * n - 4).T.copy())
    u[:, 0] = 0.5
    u[:, 1] = torch.logspace(-14, -4, 64, dtype=torch.float64)
    p, w = ps.phase_space(u, SQRT_S, [MT, MT, 0.0, 0.0])
    tot = p.sum(1)
    assert (tot[:, 0] - SQRT_S).abs().max() < 1e-12 * SQRT_S
    assert tot[:, 1:].abs().max() < 1e-12 * SQRT_S
