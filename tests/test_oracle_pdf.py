"""Pins of the oracle's grid interpolation and hadronic events against what the method fixes.

* The interpolation returns the node values at the nodes; it reproduces exactly any
  product of quadratics in (ln x, ln Q^2) inside the grid (node slopes from adjacent
  secants are exact for quadratics on equally spaced nodes, and a cubic Hermite with exact
  slopes reproduces a quadratic); its error against the smooth toy density falls by at
  least six when the node spacing halves (third order); points outside the grid take the
  edge values.
* The hadronic variables: x1 x2 = tau, ln(x1/x2)/2 = y, and the Jacobian integrates the
  unit function to the area of the (tau, y) region, 1 - tau0 + tau0 ln tau0 (Gauss-Legendre).
* The boost to the lab frame shifts every massless gluon's pseudorapidity by y exactly.
* The whole hadronic integrand: the Monte Carlo estimate of the gg -> ttbar part of
  sigma(pp) agrees, within four Monte Carlo errors, with a two-dimensional quadrature of
  f(x1) f(x2) times the closed-form partonic cross section; the same for the q qbar -> ttbar
  part with the toy quark and antiquark densities, whose closed form
  8 pi alpha_s^2 beta (1 + rho/2) / (27 s) is pinned against the oracle's |M|^2 integrated
  over the two-body phase space.
* Planted mistakes in the interpolation fail one of these.
"""
import math

import numpy as np
import pytest
import torch

from oracle import pdf, philox, processes
from oracle.kinematics import eta
from paper_2211_14056_amd import workloads as wl

P = processes.DEFAULT_PARAMS
S = 13000.0 ** 2


def _quadratic_grid(nx=21, nq=15):
    lx = np.linspace(-9.0, 0.0, nx)
    lq = np.linspace(0.5, 12.0, nq)
    A = lambda t: 1.3 - 0.2 * t + 0.05 * t * t          # noqa: E731
    B = lambda s: 0.7 + 0.1 * s - 0.004 * s * s          # noqa: E731
    return (lx, lq, np.outer(B(lq), A(lx))), A, B


def test_nodes_are_reproduced():
    g = wl.toy_pdf_grid(31, 17)
    lx, lq, v = g
    for i in (0, 3, 17, 29, 30):
        for j in (0, 5, 16):
            got = pdf.xf(g, math.exp(lx[i]), math.exp(lq[j]))[0]
            assert abs(got - v[j, i]) <= 1e-13 * max(abs(v[j, i]), 1e-300)


def test_products_of_quadratics_are_exact_inside():
    g, A, B = _quadratic_grid()
    lx, lq, _ = g
    rng = np.random.default_rng(1)
    t = rng.uniform(lx[1], lx[-2], 200)
    s = rng.uniform(lq[1], lq[-2], 200)
    got = pdf.xf(g, np.exp(t), np.exp(s))
    ref = A(t) * B(s)
    assert np.abs(got / ref - 1).max() < 1e-12


def test_third_order_convergence_to_the_smooth_density():
    rng = np.random.default_rng(2)
    x = np.exp(rng.uniform(math.log(1e-5), math.log(0.3), 300))
    q2 = np.exp(rng.uniform(math.log(10.0), math.log(1e6), 300))
    ref = wl.toy_xg(x, q2)
    errs = []
    for nx, nq in ((31, 16), (61, 31), (121, 61)):
        g = wl.toy_pdf_grid(nx, nq)
        errs.append(np.abs(pdf.xf(g, x, q2) / ref - 1).max())
    assert errs[1] < errs[0] / 6 and errs[2] < errs[1] / 6, errs
    assert errs[2] < 5e-4


def test_points_outside_the_grid_take_the_edge_values():
    g = wl.toy_pdf_grid(31, 17)
    lx, lq, v = g
    assert pdf.xf(g, 1e-9, math.exp(lq[4]))[0] == pytest.approx(v[4, 0], rel=1e-13)
    assert pdf.xf(g, 1e-3, 1e12)[0] == pytest.approx(pdf.xf(g, 1e-3, math.exp(lq[-1]))[0], rel=1e-13)
    assert pdf.xf(g, 1e-3, 0.5)[0] == pytest.approx(pdf.xf(g, 1e-3, math.exp(lq[0]))[0], rel=1e-13)


def test_hadronic_variables_and_jacobian():
    tau0 = (2 * P['m_t']) ** 2 / S
    xg, wg = np.polynomial.legendre.leggauss(40)
    u = 0.5 * (xg + 1)
    w = 0.5 * wg
    U1, U2 = np.meshgrid(u, u)
    W = np.outer(w, w)
    x1, x2, y, shat, jac = pdf.hadronic_variables(U1, U2, S, tau0)
    assert np.allclose(x1 * x2, shat / S, rtol=1e-14)
    assert np.allclose(0.5 * np.log(x1 / x2), y, rtol=1e-12, atol=1e-15)
    assert (x1 <= 1).all() and (x2 <= 1).all()
    area = (W * jac).sum()
    assert area == pytest.approx(1 - tau0 + tau0 * math.log(tau0), rel=1e-9)


def test_lab_boost_shifts_gluon_pseudorapidity():
    u = torch.tensor(philox.uniforms(3, 50, processes.dims('gg_ttgg')).T.copy())
    from oracle.phase_space import incoming, phase_space
    k, _ = phase_space(u, 700.0, processes.out_masses('gg_ttgg', P))
    p = torch.cat([incoming(50, 700.0), k], 1)
    y = torch.linspace(-1.5, 1.5, 50, dtype=torch.float64)
    ch, sh = torch.cosh(y), torch.sinh(y)
    for leg in (4, 5):
        b = p[:, leg].clone()
        b[:, 0] = ch * p[:, leg, 0] + sh * p[:, leg, 3]
        b[:, 3] = sh * p[:, leg, 0] + ch * p[:, leg, 3]
        assert torch.allclose(eta(b), eta(p[:, leg]) + y, atol=1e-10)


@pytest.mark.slow
def test_hadronic_monte_carlo_matches_quadrature_of_closed_form():
    grid = wl.toy_pdf_grid()
    ref = pdf.sigma_pp_gg_tt_quadrature(grid, S, P)
    n = 40_000
    u = philox.uniforms(8, n, processes.dims('gg_tt') + 2)
    F, ok, _, _, _ = pdf.hadronic_integrand('gg_tt', P, grid, S, u)
    assert ok.all()                       # tops are not cut
    I, err = F.mean(), F.std() / math.sqrt(n)
    assert abs(I - ref) < 4 * err, (I, err, ref)
    assert err / I < 0.02


def test_planted_interpolation_mistakes_are_caught():
    orig_slope, orig_herm = pdf._slope, pdf._hermite

    def left_secant(v, t, k):
        if k == 0:
            return (v[1] - v[0]) / (t[1] - t[0])
        return (v[k] - v[k - 1]) / (t[k] - t[k - 1])

    def swapped_basis(v, t, i, s, m_i, m_j):
        h = t[i + 1] - t[i]
        u = (s - t[i]) / h
        return ((2 * u ** 3 - 3 * u ** 2 + 1) * v[i] + (u ** 3 - u ** 2) * h * m_i
                + (-2 * u ** 3 + 3 * u ** 2) * v[i + 1] + (u ** 3 - 2 * u ** 2 + u) * h * m_j)

    for name, fn in (('_slope', left_secant), ('_hermite', swapped_basis)):
        setattr(pdf, name, fn)
        try:
            with pytest.raises(AssertionError):
                test_products_of_quadratics_are_exact_inside()
        finally:
            pdf._slope, pdf._hermite = orig_slope, orig_herm


def test_qq_tt_partonic_cross_section_closed_form():
    """The closed form 8 pi alpha_s^2 beta (1 + rho/2) / (27 s) used by the qq channel's
    quadrature equals the oracle's |M|^2 integrated over the two-body phase space
    (Gauss-Legendre in cos theta, weight beta / (16 pi) per unit cos theta, flux 1/(2 s))."""
    from oracle import me_quarks
    from oracle.closed_forms import GEV2_TO_PB
    mt, a = P['m_t'], P['alpha_s']
    for rs in (350.0, 400.0, 1000.0, 5000.0):
        s = rs * rs
        c, wc = np.polynomial.legendre.leggauss(24)
        n = c.size
        E = rs / 2
        pa = math.sqrt(E * E - mt * mt)
        st = np.sqrt(1 - c * c)
        p = torch.zeros(n, 4, 4, dtype=torch.float64)
        p[:, 0] = torch.tensor([E, 0, 0, E])
        p[:, 1] = torch.tensor([E, 0, 0, -E])
        p[:, 2, 0], p[:, 2, 1], p[:, 2, 3] = E, torch.tensor(pa * st), torch.tensor(pa * c)
        p[:, 3, 0], p[:, 3, 1], p[:, 3, 3] = E, torch.tensor(-pa * st), torch.tensor(-pa * c)
        me = me_quarks.matrix_element('qq_tt', p, dict(P, sqrt_s=rs)).numpy()
        beta = pa / E
        sig = (wc * me).sum() * beta / (16 * math.pi) / (2 * s)
        rho = 4 * mt * mt / s
        ref = 8 * math.pi * a * a * beta * (1 + rho / 2) / (27 * s)
        assert abs(sig / ref - 1) < 1e-12, (rs, sig, ref)
    assert GEV2_TO_PB > 0


@pytest.mark.slow
def test_hadronic_qq_channel_monte_carlo_matches_quadrature():
    """q(beam 1) qbar(beam 2) -> ttbar with the toy quark and antiquark densities: the oracle's
    hadronic integrand averaged over 4e4 events within four Monte Carlo errors of the
    quadrature of f_q f_qbar times the closed form."""
    gq, gqb = wl.toy_pdf_grid(kind='q'), wl.toy_pdf_grid(kind='qbar')
    ref = pdf.sigma_pp_qq_tt_quadrature(gq, gqb, S, P)
    n = 40_000
    u = philox.uniforms(9, n, processes.dims('qq_tt') + 2)
    F, ok, _, _, _ = pdf.hadronic_integrand('qq_tt', P, gq, S, u, grid_b=gqb)
    assert ok.all()
    I, err = F.mean(), F.std() / math.sqrt(n)
    assert abs(I - ref) < 4 * err, (I, err, ref)
    assert err / I < 0.02
