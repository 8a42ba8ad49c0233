"""Pins of the oracle for g g -> t tbar g g g (five gluons, 120 colour orderings, 128 helicities).

The colour-ordered oracle is general in the number of gluons; at five gluons it is pinned
by what the method and the mathematics fix, on single events (one helicity of the oracle
takes ~0.3 s here):
* explicit colour (every SU(3) index summed, Feynman rules as for fewer gluons) equals the
  colour-ordered form with the brute-force colour matrix, per helicity;
* the gluon Ward identity for every partial amplitude (each gluon's polarisation replaced by
  its momentum);
* the Parke-Taylor form of the MHV partial amplitudes in the massless limit, in absolute
  normalisation, and zero for the configurations that must vanish;
* Bose symmetry of the three final gluons, per helicity (swapping two gluons swaps their
  helicities), and the exact alpha_s^5 scaling;
* the colour matrix: symmetric, positive definite, diagonal N C_F^5 = 4096/324;
* the stored |M|^2 values the GPU tests compare against are the oracle's.
"""
import math
import os

import numpy as np
import pytest
import torch

from oracle import colour, cuts, integrand, me_explicit, me_ordered, philox, processes

P = processes.DEFAULT_PARAMS
PROC = 'gg_ttggg'


def events(n, seed, params=P):
    x = philox.uniforms(seed, n, processes.dims(PROC))
    p, _ = integrand.momenta(PROC, params, torch.tensor(np.ascontiguousarray(x.T)))
    return p


def test_colour_matrix_five_gluons():
    C = colour.colour_matrix(5)
    assert np.abs(C - C.T).max() < 1e-12
    assert np.linalg.eigvalsh(C).min() > 0
    assert np.abs(np.diag(C) - 3 * (4 / 3) ** 5).max() < 1e-10
    num = C * 324
    assert np.abs(num - np.round(num)).max() < 1e-8


def test_explicit_colour_equals_colour_ordered_five_gluons():
    p = events(1, 3)
    hels = processes.helicities(PROC)
    for h in (hels[5], hels[37], hels[70], hels[101]):
        a = me_explicit.matrix_element(PROC, p, P, hel_list=[h])
        b = me_ordered.matrix_element(PROC, p, P, hel_list=[h])
        assert ((a / b - 1).abs()).max() < 1e-12, h


def test_ward_identity_five_gluons():
    p = events(1, 5)
    hels = processes.helicities(PROC)[3::29]
    scale = max(me_ordered.partial_amplitudes(p, h, P).abs().max() for h in hels) * P['sqrt_s']
    for h in hels:
        for j in range(5):
            Aw = me_ordered.partial_amplitudes(p, h, P, ward=j)
            assert Aw.abs().max() < 1e-13 * scale, (h, j)


def test_parke_taylor_mhv_five_gluons():
    """|A(sigma)|^2 = 2^5 g^10 s(tbar, j)^3 s(t, j) / [s(t, g_s1) s(g_s1, g_s2) ... s(g_s5, tbar) s(tbar, t)]
    at m_t = 0 for the MHV configurations (all momenta outgoing, incoming helicities
    flipped, exactly one gluon j with the antiquark's helicity); zero for equal quark
    helicities and for no gluon with the antiquark's helicity."""
    P0 = dict(P, m_t=0.0)
    p = events(1, 31, params=P0)
    gl = [0, 1, 4, 5, 6]
    po = p.clone()
    po[:, :2] = -p[:, :2]

    def sij(a, b):
        x = po[:, a] + po[:, b]
        return (x[:, 0] ** 2 - x[:, 1] ** 2 - x[:, 2] ** 2 - x[:, 3] ** 2).abs()

    g2 = 4 * math.pi * P0['alpha_s']
    orders = colour.orderings(5)
    mhv, zero = [], []
    for hel in processes.helicities(PROC):
        h = list(hel)
        h[0], h[1] = -h[0], -h[1]
        gh = [h[l] for l in gl]
        if h[2] != h[3] and gh.count(h[3]) == 1:
            mhv.append((hel, gl[gh.index(h[3])]))
        elif (h[2] == h[3] or gh.count(h[3]) == 0) and len(zero) < 6:
            zero.append(hel)
    assert len(mhv) == 10
    scale = 0.0
    for hel, j in mhv:
        A = me_ordered.partial_amplitudes(p, hel, P0)
        scale = max(scale, float(A.abs().max()))
        num = sij(3, j) ** 3 * sij(2, j)
        for si, sigma in enumerate(orders):
            chain = [2] + [gl[i] for i in sigma] + [3]
            den = torch.ones(1, dtype=torch.float64)
            for a, b in zip(chain, chain[1:] + chain[:1]):
                den = den * sij(a, b)
            want = 2 ** 5 * g2 ** 5 * num / den
            assert ((A[:, si].abs() ** 2 / want - 1).abs()).max() < 1e-10, (hel, sigma)
    for hel in zero:
        assert me_ordered.partial_amplitudes(p, hel, P0).abs().max() < 1e-13 * scale, hel


def test_bose_symmetry_and_coupling_scaling_five_gluons():
    p = events(1, 8)
    hels = processes.helicities(PROC)
    for h in (hels[9], hels[77]):
        a = me_ordered.matrix_element(PROC, p, P, hel_list=[h])
        for i, j in ((4, 5), (5, 6), (4, 6)):
            q = p.clone()
            q[:, [i, j]] = p[:, [j, i]]
            hs = list(h)
            hs[i], hs[j] = h[j], h[i]
            b = me_ordered.matrix_element(PROC, q, P, hel_list=[tuple(hs)])
            assert ((b / a - 1).abs()).max() < 1e-12, (h, i, j)
    h = hels[40]
    a = me_ordered.matrix_element(PROC, p, P, hel_list=[h])
    b = me_ordered.matrix_element(PROC, p, dict(P, alpha_s=0.2), hel_list=[h])
    assert abs(float(b / a) / (0.2 / P['alpha_s']) ** 5 - 1) < 1e-13


@pytest.mark.slow
def test_stored_values_are_the_oracles():
    """tests/golden/gg_ttggg_me.txt (the GPU tests' reference at five gluons) holds what the
    oracle gives: cut decisions on every stored event, |M|^2 at both top masses on three."""
    v = np.loadtxt(os.path.join(os.path.dirname(os.path.abspath(__file__)), 'golden', 'gg_ttggg_me.txt'))
    assert v.shape == (128, 3)
    x = philox.uniforms(13, 128, processes.dims(PROC))
    p, _ = integrand.momenta(PROC, P, torch.tensor(np.ascontiguousarray(x.T)))
    assert np.array_equal(cuts.passes(p, P).numpy(), v[:, 2].astype(bool))
    sel = [0, 57, 127]
    assert np.abs(integrand.me(PROC, p[sel], P).numpy() / v[sel, 0] - 1).max() < 1e-14
    assert np.abs(integrand.me(PROC, p[sel], dict(P, m_t=0.0)).numpy() / v[sel, 1] - 1).max() < 1e-14
