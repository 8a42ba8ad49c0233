"""GPU g g -> t tbar g g g (the table-driven recursion, one wavefront per event) against the oracle.

Bars: bit-exact uniforms and Vegas bins, momenta to 1e-12 sqrt(s), weights to 1e-12 relative
plus eight times their sensitivity to a one-ulp change of a uniform (measured on the oracle),
and identical cut masks; FP64 |M|^2 within 1e-12 relative of the
oracle on every event, for 16, 32 and 64 lanes per event, with m_t = 173 GeV and m_t = 0; FP32
within 1e-5 median and 1e-3 max relative over the events that pass the cuts; ragged and empty
batches; the matrix-core precisions rejected before any launch.  The oracle's |M|^2 at five
gluons takes ~35 s per call, so its values on 128 seeded events are stored
(tests/golden/gg_ttggg_me.txt, written by tests/golden/make_gg_ttggg_me.py from the oracle
alone); the momenta they belong to are recomputed here by the oracle's phase space.
At 2^18 events: FP32 against FP64 on every event that passes the cuts, the three
lanes-per-event layouts against each other, and bitwise repeatability.
"""
import os
import sys

import numpy as np
import pytest
import torch

import paper_2211_14056_amd as mf
from oracle import cuts as ocuts, integrand, philox, processes

pytestmark = pytest.mark.gpu

PROC = 'gg_ttggg'
P = processes.DEFAULT_PARAMS
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), 'golden', 'gg_ttggg_me.txt')
LPES = [16, 32, 64]


def say(*a):
    print('[gpu-test]', *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope='module')
def h():
    torch.cuda.init()
    return mf.Handle(0)


@pytest.fixture(scope='module')
def golden():
    v = np.loadtxt(GOLDEN)
    return v[:, 0], v[:, 1], v[:, 2].astype(bool)


@pytest.fixture(scope='module')
def p_oracle():
    """the stored events' momenta from the oracle's phase space, GPU layout [7][4][128]"""
    x = philox.uniforms(13, 128, processes.dims(PROC))
    p, _ = integrand.momenta(PROC, P, torch.tensor(np.ascontiguousarray(x.T)))
    assert ocuts.passes(p, P).numpy().sum() > 100
    return torch.tensor(np.ascontiguousarray(np.transpose(p.numpy(), (1, 2, 0))), device='cuda')


def _me(h, p, precision, lpe=0, par=P):
    h.set_launch(proc=mf.MF_GG_TTGGG, precision=precision, block=lpe)
    try:
        out = mf.matrix_element(h, mf.MF_GG_TTGGG, p.contiguous(), precision, mf.params_from_dict(par))
        torch.cuda.synchronize()
    finally:
        h.set_launch(proc=mf.MF_GG_TTGGG, precision=precision, block=0)
    return out.double().cpu().numpy()


def _weight_ulp_sensitivity(y):
    """per event: the largest relative change of the oracle's weight when one uniform moves by
    one ulp (y [d][N], after the Vegas map)"""
    def w_of(yy):
        return integrand.momenta(PROC, P, torch.tensor(np.ascontiguousarray(yy.T)))[1].numpy()
    w0 = w_of(y)
    s = np.zeros(y.shape[1])
    for k in range(y.shape[0]):
        for to in (2.0, -1.0):
            yy = y.copy()
            yy[k] = np.nextafter(yy[k], to)
            s = np.maximum(s, np.abs(w_of(yy) / w0 - 1))
    return s


def test_phase_space_ttggg_vs_oracle(h):
    n = 4096 + 17
    d = processes.dims(PROC)
    assert mf.mf_process_dims(mf.MF_GG_TTGGG) == d == 11
    rng = np.random.default_rng(6)
    w_ = rng.uniform(0.3, 1.7, (d, 50))
    edges = np.concatenate([np.zeros((d, 1)), np.cumsum(w_, 1) / w_.sum(1, keepdims=True)], 1)
    edges[:, -1] = 1.0
    dev = torch.device('cuda', 0)
    say('phase space', PROC, n)
    ev = mf.mf_phase_space(h, mf.MF_GG_TTGGG, mf.params_from_dict(P), n, seed=77, offset=5,
                           edges=torch.tensor(edges, device=dev).contiguous(), nb=50,
                           pass_=torch.empty(n, dtype=torch.uint8, device=dev),
                           bin_idx=torch.empty(d, n, dtype=torch.int16, device=dev),
                           jac=torch.empty(n, dtype=torch.float64, device=dev),
                           x_out=torch.empty(d, n, dtype=torch.float64, device=dev))
    torch.cuda.synchronize()
    x = ev['x'].cpu().numpy()
    assert np.array_equal(x, philox.uniforms(77, n, d, offset=5))
    from oracle import vegas as ovegas
    y, b, J = ovegas.vegas_map(x, edges)
    assert np.array_equal(ev['bin_idx'].cpu().numpy().astype(np.int64), b)
    assert np.allclose(ev['jac'].cpu().numpy(), J, rtol=1e-13, atol=0)
    p_ref, w_ref = integrand.momenta(PROC, P, torch.tensor(np.ascontiguousarray(y.T)))
    diff = np.abs(np.transpose(ev['p'].cpu().numpy(), (2, 0, 1)) - p_ref.numpy()).max() / P['sqrt_s']
    assert diff < 1e-12, diff
    # the mass ratios of the phase space invert a distribution function whose slope vanishes
    # at u -> 1, so the weight can move by ~4e-13 for a one-ulp change of a uniform; both
    # sides round u-sized values a few times there, hence 1e-12 plus eight such changes
    rel = np.abs(ev['w'].cpu().numpy() / w_ref.numpy() - 1)
    assert (rel <= 1e-12 + 8 * _weight_ulp_sensitivity(y)).all(), rel.max()
    ok_ref = ocuts.passes(p_ref, P).numpy()
    assert np.array_equal(ev['pass_'].cpu().numpy().astype(bool), ok_ref)


def test_phase_space_of_the_stored_events(h, p_oracle):
    """the GPU phase space on the stored events' uniforms gives the momenta the stored |M|^2
    belongs to"""
    x = philox.uniforms(13, 128, processes.dims(PROC))
    ev = mf.mf_phase_space(h, mf.MF_GG_TTGGG, mf.params_from_dict(P), 128,
                           x=torch.tensor(x, device='cuda').contiguous())
    torch.cuda.synchronize()
    assert (ev['p'] - p_oracle).abs().max().item() < 1e-12 * P['sqrt_s']


@pytest.mark.parametrize('lpe', LPES)
def test_me_fp64_vs_oracle(h, golden, p_oracle, lpe):
    me_ref, _, _ = golden
    say('me fp64', PROC, 'lanes per event', lpe)
    me = _me(h, p_oracle, mf.MF_FP64, lpe)
    rel = np.abs(me / me_ref - 1)
    say('  max rel', rel.max())
    assert rel.max() < 1e-12


def test_me_fp64_massless_vs_oracle(h, golden, p_oracle):
    _, me0_ref, _ = golden
    say('me fp64 massless', PROC)
    me = _me(h, p_oracle, mf.MF_FP64, 0, dict(P, m_t=0.0))
    rel = np.abs(me / me0_ref - 1)
    say('  max rel', rel.max())
    assert rel.max() < 1e-12


@pytest.mark.parametrize('lpe', LPES)
def test_me_fp32_vs_oracle(h, golden, p_oracle, lpe):
    me_ref, _, ok = golden
    say('me fp32', PROC, 'lanes per event', lpe)
    me = _me(h, p_oracle, mf.MF_FP32, lpe)
    rel = np.abs(me / me_ref - 1)[ok]
    say('  median', np.median(rel), 'max', rel.max())
    assert np.median(rel) < 1e-5 and rel.max() < 1e-3


@pytest.mark.parametrize('n', [0, 1, 3, 37, 127])
def test_me_ragged_and_empty_batches(h, golden, p_oracle, n):
    me_ref, _, _ = golden
    say('ragged', PROC, n)
    for lpe in LPES:
        p = p_oracle[:, :, :n].contiguous()
        me = _me(h, p, mf.MF_FP64, lpe)
        assert me.shape == (n,)
        if n:
            assert np.abs(me / me_ref[:n] - 1).max() < 1e-12


def test_matrix_core_precisions_rejected(h, p_oracle):
    for prec in (mf.MF_FP32_MFMA_BF16, mf.MF_FP32_MFMA_F32):
        out = torch.full((128,), -1.0, dtype=torch.float32, device='cuda')
        with pytest.raises(mf.MFError) as ei:
            mf.mf_matrix_element(h, [mf.make_request(mf.MF_GG_TTGGG, p_oracle, out)], prec, mf.params_from_dict(P))
        assert ei.value.status == -2
        torch.cuda.synchronize()
        assert (out == -1.0).all()
    with pytest.raises(mf.MFError) as ei:
        h.set_launch(proc=mf.MF_GG_TTGGG, precision=mf.MF_FP64, block=128)
    assert ei.value.status == -1


def test_full_size_layouts_precisions_and_repeatability(h):
    n = 1 << 18
    say('full size', PROC, n)
    prm = mf.params_from_dict(P)
    ev = mf.mf_phase_space(h, mf.MF_GG_TTGGG, prm, n, seed=5,
                           pass_=torch.empty(n, dtype=torch.uint8, device='cuda'))
    torch.cuda.synchronize()
    ok = ev['pass_'].cpu().numpy().astype(bool)
    ref = _me(h, ev['p'], mf.MF_FP64, 64)
    assert np.isfinite(ref).all() and (ref > 0).all()
    for lpe in (16, 32):
        say('  fp64 lanes per event', lpe)
        assert np.abs(_me(h, ev['p'], mf.MF_FP64, lpe) / ref - 1).max() < 1e-12
    assert np.array_equal(_me(h, ev['p'], mf.MF_FP64, 64), ref)
    say('  fp32')
    rel = np.abs(_me(h, ev['p'], mf.MF_FP32, 0) / ref - 1)[ok]
    say('  median', np.median(rel), 'max', rel.max())
    assert np.median(rel) < 1e-5 and rel.max() < 1e-3
