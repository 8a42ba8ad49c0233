"""GPU q qbar -> t tbar (+g, +gg) and q g -> t tbar q (+g) (generated diagram code) against the oracle.

Bars: bit-exact uniforms and Vegas bins; momenta to 1e-12 sqrt(s), weights to 1e-12 relative
plus eight times their change under a one-ulp change of one uniform (hadronic events: 3e-12
plus the same, as for the gluon channels) and
identical cut masks (the light quark of q g channels is cut like a gluon); FP64 |M|^2 within
1e-12 relative of the oracle's explicit-colour diagram sum on every event that passes the cuts
(1e-10 on the others: a soft or collinear gluon makes |M|^2 a cancellation between diagrams),
also at m_t = 0; FP32 within
1e-5 median and 1e-3 max relative over the events that pass the cuts; ragged and empty batches;
the matrix-core precisions and the derivative rejected before any launch; at 2^20 events FP32
against FP64 on every event that passes the cuts, and bitwise repeatability.  Hadronic events:
q g -> t tbar q with the toy quark and gluon densities against the oracle per event, and the
q qbar -> t tbar part of sigma(pp) from 4e6 GPU events within four Monte Carlo errors of the
quadrature of f_q f_qbar times the closed-form partonic cross section; sigma(pp -> t tbar) summed
over all its parton channels (gg, q qbar, qbar q) within four errors of the sum of the
quadratures; every channel of pp -> t tbar + jet finite and positive.
"""
import sys

import numpy as np
import pytest
import torch

import paper_2211_14056_amd as mf
from oracle import cuts as ocuts, integrand, pdf as opdf, philox, processes, vegas as ovegas
from paper_2211_14056_amd import workloads as wl

pytestmark = pytest.mark.gpu

P = processes.DEFAULT_PARAMS
PROCS = ['qq_tt', 'qq_ttg', 'qq_ttgg', 'qg_ttq', 'qg_ttqg']
ME_N = {'qq_tt': 500, 'qq_ttg': 200, 'qq_ttgg': 24, 'qg_ttq': 200, 'qg_ttqg': 24}
SQRT_S = 13000.0


def say(*a):
    print('[gpu-test]', *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope='module')
def h():
    torch.cuda.init()
    return mf.Handle(0)


def _oracle_me(proc, p_gpu, par=P):
    p = torch.tensor(np.ascontiguousarray(np.transpose(p_gpu, (2, 0, 1))), dtype=torch.float64)
    return integrand.me(proc, p, par).numpy()


def _gpu_me(h, proc, p, precision, par=P):
    out = mf.matrix_element(h, mf.PROCESS[proc], p.contiguous(), precision, mf.params_from_dict(par))
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


@pytest.mark.parametrize('proc', PROCS)
def test_phase_space_vs_oracle(h, proc):
    n = 4096 + 17
    pid = mf.PROCESS[proc]
    d = processes.dims(proc)
    assert mf.mf_process_dims(pid) == d and mf.mf_process_legs(pid) == processes.PROCESSES[proc]['n_ext']
    rng = np.random.default_rng(8)
    w_ = rng.uniform(0.3, 1.7, (d, 50))
    edges = np.concatenate([np.zeros((d, 1)), np.cumsum(w_, 1) / w_.sum(1, keepdims=True)], 1)
    edges[:, -1] = 1.0
    dev = torch.device('cuda', 0)
    say('phase space', proc, n)
    ev = mf.mf_phase_space(h, pid, mf.params_from_dict(P), n, seed=78, offset=3,
                           edges=torch.tensor(edges, device=dev).contiguous(), nb=50,
                           pass_=torch.empty(n, dtype=torch.uint8, device=dev),
                           bin_idx=torch.empty(d, n, dtype=torch.int16, device=dev),
                           jac=torch.empty(n, dtype=torch.float64, device=dev),
                           x_out=torch.empty(d, n, dtype=torch.float64, device=dev))
    torch.cuda.synchronize()
    x = ev['x'].cpu().numpy()
    assert np.array_equal(x, philox.uniforms(78, n, d, offset=3))
    y, b, J = ovegas.vegas_map(x, edges)
    assert np.array_equal(ev['bin_idx'].cpu().numpy().astype(np.int64), b)
    p_ref, w_ref = integrand.momenta(proc, P, torch.tensor(np.ascontiguousarray(y.T)))
    diff = np.abs(np.transpose(ev['p'].cpu().numpy(), (2, 0, 1)) - p_ref.numpy()).max() / P['sqrt_s']
    assert diff < 1e-12, diff
    # the weight against 1e-12 plus eight times its change under a one-ulp change of one uniform
    # (the mass-ratio inversion near u -> 1 makes some events' weights sensitive to the last bit)
    sens = np.zeros(n)
    for k in range(d):
        for to in (2.0, -1.0):
            yy = y.copy()
            yy[k] = np.nextafter(yy[k], to)
            wk = integrand.momenta(proc, P, torch.tensor(np.ascontiguousarray(yy.T)))[1].numpy()
            sens = np.maximum(sens, np.abs(wk / w_ref.numpy() - 1))
    rel = np.abs(ev['w'].cpu().numpy() / w_ref.numpy() - 1)
    assert (rel <= 1e-12 + 8 * sens).all(), rel.max()
    assert np.array_equal(ev['pass_'].cpu().numpy().astype(bool), ocuts.passes(p_ref, P).numpy())


@pytest.mark.parametrize('proc', PROCS)
def test_me_fp64_and_fp32_vs_oracle(h, proc):
    n = ME_N[proc] + 3
    pid = mf.PROCESS[proc]
    say('me', proc, n)
    ev = mf.mf_phase_space(h, pid, mf.params_from_dict(P), n, seed=21,
                           pass_=torch.empty(n, dtype=torch.uint8, device='cuda'))
    torch.cuda.synchronize()
    ref = _oracle_me(proc, ev['p'].cpu().numpy())
    me64 = _gpu_me(h, proc, ev['p'], mf.MF_FP64)
    rel = np.abs(me64 / ref - 1)
    ok = ev['pass_'].cpu().numpy().astype(bool)
    say('  fp64 max rel', rel.max(), 'passing the cuts', rel[ok].max())
    # as for the gluon channels: 1e-12 over the events that pass the cuts; a soft or collinear
    # gluon outside them makes |M|^2 a cancellation between diagrams (1e-10 there)
    assert rel[ok].max() < 1e-12 and rel.max() < 1e-10
    me32 = _gpu_me(h, proc, ev['p'], mf.MF_FP32)
    rel = np.abs(me32 / ref - 1)[ok]
    say('  fp32 median', np.median(rel), 'max', rel.max())
    assert np.median(rel) < 1e-5 and rel.max() < 1e-3


@pytest.mark.parametrize('proc', ['qq_ttg', 'qg_ttqg'])
def test_me_fp64_massless_vs_oracle(h, proc):
    n = 19
    par = dict(P, m_t=0.0)
    pid = mf.PROCESS[proc]
    say('me massless', proc, n)
    ev = mf.mf_phase_space(h, pid, mf.params_from_dict(par), n, seed=23,
                           pass_=torch.empty(n, dtype=torch.uint8, device='cuda'))
    torch.cuda.synchronize()
    ref = _oracle_me(proc, ev['p'].cpu().numpy(), par)
    ok = ev['pass_'].cpu().numpy().astype(bool)
    rel = np.abs(_gpu_me(h, proc, ev['p'], mf.MF_FP64, par) / ref - 1)
    assert rel[ok].max() < 1e-12 and rel.max() < 1e-10


@pytest.mark.parametrize('n', [0, 1, 255, 257])
def test_me_ragged_and_empty_batches(h, n):
    for proc in ('qq_ttg', 'qg_ttq'):
        pid = mf.PROCESS[proc]
        say('ragged', proc, n)
        p = torch.empty(mf.mf_process_legs(pid), 4, n, dtype=torch.float64, device='cuda')
        ok = np.zeros(n, dtype=bool)
        if n:
            ev = mf.mf_phase_space(h, pid, mf.params_from_dict(P), n, seed=2,
                                   pass_=torch.empty(n, dtype=torch.uint8, device='cuda'))
            p, ok = ev['p'], ev['pass_'].cpu().numpy().astype(bool)
        for prec in (mf.MF_FP64, mf.MF_FP32):
            me = _gpu_me(h, proc, p, prec)
            assert me.shape == (n,)
            if n and prec == mf.MF_FP64:
                rel = np.abs(me / _oracle_me(proc, p.cpu().numpy()) - 1)
                assert rel[ok].max(initial=0.0) < 1e-12 and rel.max() < 1e-10


def test_unsupported_forms_rejected_before_launch(h):
    pid = mf.MF_QQ_TTG
    p = mf.mf_phase_space(h, pid, mf.params_from_dict(P), 64, seed=1)['p']
    for prec in (mf.MF_FP32_MFMA_BF16, mf.MF_FP32_MFMA_F32):
        out = torch.full((64,), -1.0, dtype=torch.float32, device='cuda')
        with pytest.raises(mf.MFError) as ei:
            mf.mf_matrix_element(h, [mf.make_request(pid, p, out)], prec, mf.params_from_dict(P))
        assert ei.value.status == -2
        torch.cuda.synchronize()
        assert (out == -1.0).all()
    d = mf.mf_process_dims(pid)
    x = torch.rand(d, 64, dtype=torch.float64, device='cuda')
    g = torch.ones(64, dtype=torch.float64, device='cuda')
    req = mf.make_request(pid, None, None, x=x, grad_me=g, grad_x=torch.empty_like(x),
                          grad_theta=torch.empty(64, 2, dtype=torch.float64, device='cuda'), n=64)
    with pytest.raises(mf.MFError) as ei:
        mf.mf_matrix_element_vjp(h, [req], mf.MF_FP64, mf.params_from_dict(P))
    assert ei.value.status == -2


@pytest.mark.parametrize('proc', ['qq_ttgg', 'qg_ttqg'])
def test_full_size_fp32_vs_fp64_and_repeatability(h, proc):
    n = 1 << 20
    pid = mf.PROCESS[proc]
    say('full size', proc, n)
    ev = mf.mf_phase_space(h, pid, mf.params_from_dict(P), n, seed=5,
                           pass_=torch.empty(n, dtype=torch.uint8, device='cuda'))
    torch.cuda.synchronize()
    ok = ev['pass_'].cpu().numpy().astype(bool)
    ref = _gpu_me(h, proc, ev['p'], mf.MF_FP64)
    assert np.isfinite(ref).all() and (ref > 0).all()
    assert np.array_equal(_gpu_me(h, proc, ev['p'], mf.MF_FP64), ref)
    rel = np.abs(_gpu_me(h, proc, ev['p'], mf.MF_FP32) / ref - 1)[ok]
    say('  fp32 median', np.median(rel), 'max', rel.max())
    assert np.median(rel) < 1e-5 and rel.max() < 1e-3
    # sampled events against the oracle at full size
    idx = np.random.default_rng(4).choice(np.nonzero(ok)[0], 12, replace=False)
    pe = ev['p'].cpu().numpy()[:, :, idx]
    assert np.abs(ref[idx] / _oracle_me(proc, pe) - 1).max() < 1e-12


# ------------------------------------------------------------------ hadronic events
@pytest.fixture(scope='module')
def grids():
    return {k: wl.toy_pdf_grid(kind=k) for k in ('g', 'q', 'qbar')}


def test_hadronic_qg_events_vs_oracle(h, grids):
    proc, n = 'qg_ttq', 1007
    pid = mf.PROCESS[proc]
    d = processes.dims(proc) + 2
    x = philox.uniforms(27, n, d)
    dev = torch.device('cuda', 0)
    gq, gg = mf.PdfGrid(*grids['q']), mf.PdfGrid(*grids['g'])
    say('hadronic', proc, n)
    ev = mf.mf_phase_space_pp(h, pid, mf.params_from_dict(P), SQRT_S, gq, n, grid_b=gg,
                              x=torch.tensor(x, device=dev).contiguous(),
                              pass_=torch.empty(n, dtype=torch.uint8, device=dev),
                              x12=torch.empty(2, n, dtype=torch.float64, device=dev))
    torch.cuda.synchronize()
    F, ok, me_o, p_o, w_o = opdf.hadronic_integrand(proc, P, grids['q'], SQRT_S ** 2, x, grid_b=grids['g'])
    p = ev['p'].cpu().numpy()
    po = np.transpose(p_o.numpy(), (1, 2, 0))
    assert (np.abs(p - po).max(axis=(0, 1)) <= 1e-12 * 2.0 * po[0, 0]).all()
    w = ev['w'].cpu().numpy()
    x1, x2, _, _, _ = opdf.hadronic_variables(x[0], x[1], SQRT_S ** 2, (2 * P['m_t']) ** 2 / SQRT_S ** 2)
    inner = (x1 < 0.5) & (x2 < 0.5)
    # as for the gluon channels: 1e-12 for the partonic weight and for each density, plus eight
    # times the weight's change under a one-ulp change of one uniform (measured on the oracle)
    sens = np.zeros(n)
    for k in range(d):
        for to in (2.0, -1.0):
            xx = x.copy()
            xx[k] = np.nextafter(xx[k], to)
            wk = opdf.hadronic_integrand(proc, P, grids['q'], SQRT_S ** 2, xx, with_me=False, grid_b=grids['g'])[4]
            sens = np.maximum(sens, np.abs(wk / w_o - 1))
    rel = np.abs(w / w_o - 1)
    assert (rel[inner] <= (3e-12 + 8 * sens)[inner]).all()
    assert (np.abs(w - w_o) <= 3e-12 * np.abs(w_o).max() + 8 * sens * np.abs(w_o)).all()
    assert np.array_equal(ev['pass_'].cpu().numpy().astype(bool), ok)
    me64 = _gpu_me(h, proc, ev['p'], mf.MF_FP64)
    assert np.abs(me64 / me_o - 1)[ok].max() < 1e-12


def test_sigma_pp_qq_tt_matches_quadrature(h, grids):
    ref = opdf.sigma_pp_qq_tt_quadrature(grids['q'], grids['qbar'], SQRT_S ** 2, P)
    proc, n, iters = 'qq_tt', 2_000_000, 2
    pid = mf.PROCESS[proc]
    d = processes.dims(proc) + 2
    dev = torch.device('cuda', 0)
    gq, gqb = mf.PdfGrid(*grids['q']), mf.PdfGrid(*grids['qbar'])
    prm = mf.params_from_dict(P)
    vprm = mf.params_from_dict(dict(P, sqrt_s=SQRT_S))
    acc = torch.empty(2 + d * 50, dtype=torch.float64, device=dev)
    edges = torch.tensor(np.tile(np.linspace(0, 1, 51), (d, 1)), dtype=torch.float64, device=dev).contiguous()
    Is, vs = [], []
    for it in range(iters):
        say('sigma pp qq iteration', it)
        ev = mf.mf_phase_space_pp(h, pid, prm, SQRT_S, gq, n, grid_b=gqb, seed=33, offset=it * n, edges=edges,
                                  nb=50, pass_=torch.empty(n, dtype=torch.uint8, device=dev),
                                  bin_idx=torch.empty(d, n, dtype=torch.int16, device=dev),
                                  jac=torch.empty(n, dtype=torch.float64, device=dev))
        me = mf.matrix_element(h, pid, ev['p'], mf.MF_FP64, prm)
        mf.mf_vegas_refine(h, vprm, n, d, 50, 1.5, ev['w'], ev['jac'], me, ev['pass_'], ev['bin_idx'], acc, edges)
        a = acc.cpu().numpy()
        I = a[0] / n
        Is.append(I)
        vs.append((a[1] / n - I * I) / (n - 1))
    w = 1 / np.array(vs)
    I = (np.array(Is) * w).sum() / w.sum()
    sig = w.sum() ** -0.5
    say('  sigma', I, '+-', sig, 'quadrature', ref)
    assert abs(I - ref) < 4 * sig
    assert sig / I < 2e-3


def test_sigma_pp_tt_all_channels_matches_quadrature(h, grids):
    """sigma(pp -> ttbar) summed over its parton channels (hadronic.sigma_pp: gg once, q qbar
    twice for the beam-swapped qbar q) against the oracle's quadratures of the closed forms."""
    from paper_2211_14056_amd import hadronic
    ref = (opdf.sigma_pp_gg_tt_quadrature(grids['g'], SQRT_S ** 2, P)
           + 2 * opdf.sigma_pp_qq_tt_quadrature(grids['q'], grids['qbar'], SQRT_S ** 2, P))
    say('sigma pp -> ttbar, all channels')
    r = hadronic.sigma_pp('tt', sqrt_S=SQRT_S, n=1_000_000, iters=3, warmup=1, prm=mf.params_from_dict(P),
                          handle=h)
    say('  sigma', r['sigma_pb'], '+-', r['error_pb'], 'quadrature', ref, r['channels'])
    assert abs(r['sigma_pb'] - ref) < 4 * r['error_pb']
    assert r['error_pb'] / r['sigma_pb'] < 2e-3


def test_sigma_pp_tt_jet_channels(h):
    """pp -> ttbar + jet (pT > 20 GeV, |eta| < 2.5): every tree-level channel of one light
    flavour integrates to a finite positive cross section with a small error, and the total is
    the multiplicity-weighted sum."""
    from paper_2211_14056_amd import hadronic
    say('sigma pp -> ttbar + jet')
    r = hadronic.sigma_pp('ttj', sqrt_S=SQRT_S, n=1 << 18, iters=2, warmup=1, prm=mf.params_from_dict(P),
                          handle=h)
    say('  ', r)
    ch = r['channels']
    assert len(ch) == 4
    for v in ch.values():
        assert np.isfinite(v['sigma_pb']) and v['sigma_pb'] > 0 and v['error_pb'] < 0.05 * v['sigma_pb']
    assert abs(sum(v['sigma_pb'] for v in ch.values()) - r['sigma_pb']) <= 1e-12 * r['sigma_pb']
