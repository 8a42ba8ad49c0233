"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars: bit-exact uniforms and bin indices; FP64 momenta/weights/|M|^2 within
1e-12 relative; FP32 |M|^2 within 1e-5 median and 1e-3 max relative (events
passing cuts); Vegas sums and refined edges within 1e-12.
"""
import math
import sys

import numpy as np
import pytest
import torch

import paper_2211_14056_amd as mf
from oracle import (closed_forms, cuts as ocuts, integrand, me_explicit, me_ordered, phase_space as ops,
                    philox, processes, vegas as ovegas)

pytestmark = pytest.mark.gpu

P = processes.DEFAULT_PARAMS
PEE = processes.EE_PARAMS
PROCS = ['ee_mumu', 'gg_tt', 'gg_ttg', 'gg_ttgg']


def say(*a):
    print('[gpu-test]', *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope='module')
def h():
    import os
    if not os.path.exists(mf.LIB_PATH):
        from paper_2211_14056_amd import build as _b
        _b.build()
    torch.cuda.init()
    return mf.Handle(0)


def prm_of(proc):
    return mf.params_from_dict(PEE if proc == 'ee_mumu' else P)


def par_of(proc):
    return PEE if proc == 'ee_mumu' else P


def gpu_events(h, proc, n, seed, offset=0, edges=None, nb=50):
    pid = mf.PROCESS[proc]
    d = mf.mf_process_dims(pid)
    dev = torch.device('cuda', 0)
    x_out = torch.empty(d, n, dtype=torch.float64, device=dev)
    pas = torch.empty(n, dtype=torch.uint8, device=dev)
    bins = torch.empty(d, n, dtype=torch.int16, device=dev)
    jac = torch.empty(n, dtype=torch.float64, device=dev)
    e = None if edges is None else torch.tensor(edges, dtype=torch.float64, device=dev).contiguous()
    out = mf.mf_phase_space(h, pid, prm_of(proc), n, seed=seed, offset=offset, edges=e, nb=nb,
                            pass_=pas, bin_idx=bins, jac=jac, x_out=x_out)
    torch.cuda.synchronize()
    return out


def oracle_momenta(proc, x):
    """x [d][N] numpy -> p [N, n_ext, 4] torch f64, w [N]."""
    u = torch.tensor(np.ascontiguousarray(x.T), dtype=torch.float64)
    return integrand.momenta(proc, par_of(proc), u)


def gpu_me(h, proc, p, precision):
    pid = mf.PROCESS[proc]
    out = mf.matrix_element(h, pid, p.contiguous(), precision, prm_of(proc))
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


def oracle_me(proc, p_gpu_layout):
    """p [n_ext][4][N] numpy -> oracle ME [N]."""
    p = torch.tensor(np.ascontiguousarray(np.transpose(p_gpu_layout, (2, 0, 1))), dtype=torch.float64)
    return integrand.me(proc, p, par_of(proc)).numpy()


# ------------------------------------------------------------------ RNG
@pytest.mark.parametrize('proc', PROCS)
def test_uniforms_bitwise(h, proc):
    n = 5000 + 37
    say('uniforms', proc, n)
    ev = gpu_events(h, proc, n, seed=1234, offset=10 ** 10 + 3)
    x_ref = philox.uniforms(1234, n, processes.dims(proc), offset=10 ** 10 + 3)
    assert np.array_equal(ev['x'].cpu().numpy(), x_ref)


# ------------------------------------------------------------------ phase space
@pytest.mark.parametrize('proc', PROCS)
def test_phase_space_vs_oracle(h, proc):
    n = 4096 + 17
    d = processes.dims(proc)
    rng = np.random.default_rng(5)
    w_ = rng.uniform(0.3, 1.7, (d, 50))
    edges = np.concatenate([np.zeros((d, 1)), np.cumsum(w_, 1) / w_.sum(1, keepdims=True)], 1)
    edges[:, -1] = 1.0
    say('phase space', proc, n)
    ev = gpu_events(h, proc, n, seed=77, edges=edges)
    x = ev['x'].cpu().numpy()
    y, b, J = ovegas.vegas_map(x, edges)
    assert np.array_equal(ev['bin_idx'].cpu().numpy().astype(np.int64), b)
    assert np.allclose(ev['jac'].cpu().numpy(), J, rtol=1e-13, atol=0)
    p_ref, w_ref = oracle_momenta(proc, y)
    p_gpu = ev['p'].cpu().numpy()
    rs = par_of(proc)['sqrt_s']
    # both sides solve the same root equations (GPU: safeguarded Newton, oracle:
    # bisection); near rho -> 1 the mass-ratio root is ill-conditioned, so agree
    # to 1e-12 of sqrt(s) rather than to the last bit
    diff = np.abs(np.transpose(p_gpu, (2, 0, 1)) - p_ref.numpy()).max() / rs
    assert diff < 1e-12, diff
    wr = w_ref.numpy()
    assert np.abs(ev['w'].cpu().numpy() / wr - 1).max() < 1e-12
    # cut decisions agree except within rounding of a cut boundary
    ok_ref = ocuts.passes(p_ref, par_of(proc)).numpy()
    ok_gpu = ev['pass_'].cpu().numpy().astype(bool)
    assert (ok_ref != ok_gpu).sum() == 0


def test_phase_space_conservation_full_size(h):
    n = 1_000_000
    say('phase space full size gg_ttgg', n)
    ev = gpu_events(h, 'gg_ttgg', n, seed=4)
    p = ev['p']
    tot = p[2:].sum(0)
    assert float((tot[0] - 1000.0).abs().max()) < 1e-12 * 1000
    assert float(tot[1:].abs().max()) < 1e-12 * 1000
    m2 = p[:, 0] ** 2 - p[:, 1] ** 2 - p[:, 2] ** 2 - p[:, 3] ** 2
    assert float(((m2[2:4] - 173.0 ** 2).abs() / p[2:4, 0] ** 2).max()) < 1e-10
    assert float((m2[4:].abs() / p[4:, 0] ** 2).max()) < 1e-10
    assert bool(torch.isfinite(ev['w']).all()) and float(ev['w'].min()) > 0
    assert h.failures() == 0


def _bad_uniforms(x, nb):
    """Copy of x with a NaN, a negative and a >= 1 uniform in three events; returns
    (x_bad, {event: (dim, expected bin)})."""
    xb = x.copy()
    bad = {5: (0, 0), 70: (1, 0), x.shape[1] - 1: (2, nb - 1)}
    for e, (k, _) in bad.items():
        xb[k, e] = (np.nan, -0.25, 1.25)[list(bad).index(e)]
    return xb, bad


def test_phase_space_out_of_range_uniforms_stay_in_bounds(h):
    """Caller uniforms outside [0, 1) or NaN: the Vegas bins are clamped (first or last
    bin, NaN in bin 0), and every other event is bit-identical to a run without them,
    in the phase space and in the derivative."""
    proc, n, nb = 'gg_ttg', 130, 50
    pid, d = mf.PROCESS[proc], processes.dims(proc)
    x = philox.uniforms(50, n, d)
    xb, bad = _bad_uniforms(x, nb)
    keep = np.setdiff1d(np.arange(n), list(bad))
    ed = _edges(d, 3)
    dev = torch.device('cuda', 0)
    e = torch.tensor(ed, dtype=torch.float64, device=dev).contiguous()
    hh = mf.Handle(0)                      # own handle: the NaN event is counted as a failure
    try:
        outs = []
        for xx in (x, xb):
            say('phase space with caller uniforms', proc, n, 'bad' if xx is xb else 'good')
            xt = torch.tensor(xx, dtype=torch.float64, device=dev).contiguous()
            o = mf.mf_phase_space(hh, pid, prm_of(proc), n, x=xt, edges=e, nb=nb,
                                  pass_=torch.empty(n, dtype=torch.uint8, device=dev),
                                  bin_idx=torch.empty(d, n, dtype=torch.int16, device=dev),
                                  jac=torch.empty(n, dtype=torch.float64, device=dev))
            torch.cuda.synchronize()
            outs.append({k: v.cpu().numpy() for k, v in o.items() if k != 'x'})
        good, got = outs
        b = got['bin_idx']
        assert b.min() >= 0 and b.max() <= nb - 1
        for ev, (k, want) in bad.items():
            assert b[k, ev] == want, (ev, k, b[k, ev])
        assert np.isnan(got['p'][2:, :, 5]).any()
        for k in ('p', 'w', 'jac', 'pass_', 'bin_idx'):
            assert np.array_equal(got[k][..., keep], good[k][..., keep]), k
        # the clamped events' Jacobian is the product of their bins' widths
        for ev in list(bad)[1:]:
            jac = 1.0
            for k in range(d):
                i = b[k, ev]
                jac *= nb * (ed[k, i + 1] - ed[k, i])
            assert abs(got['jac'][ev] / jac - 1) < 1e-14
        # the derivative maps x the same way
        gb = np.ones(n)
        for prec in (mf.MF_FP64, mf.MF_FP32):
            say('vjp with caller uniforms', proc, n, prec)
            me_r, gx_r, gth_r = _vjp_gpu(hh, proc, x, gb, prec, edges=ed)
            me_b, gx_b, gth_b = _vjp_gpu(hh, proc, xb, gb, prec, edges=ed)
            assert np.array_equal(me_b[keep], me_r[keep])
            assert np.array_equal(gx_b[:, keep], gx_r[:, keep])
            assert np.array_equal(gth_b[keep], gth_r[keep])
    finally:
        hh.close()


# ------------------------------------------------------------------ matrix element
ME_N = {'ee_mumu': 2000, 'gg_tt': 2000, 'gg_ttg': 300, 'gg_ttgg': 40}


@pytest.mark.parametrize('proc', PROCS)
def test_me_fp64_vs_oracle(h, proc):
    n = ME_N[proc] + 3
    say('me fp64', proc, n)
    ev = gpu_events(h, proc, n, seed=21)
    me = gpu_me(h, proc, ev['p'], mf.MF_FP64)
    ref = oracle_me(proc, ev['p'].cpu().numpy())
    rel = np.abs(me / ref - 1)
    say('  max rel', rel.max())
    assert rel.max() < 1e-12


@pytest.mark.parametrize('proc', ['gg_tt', 'gg_ttg', 'gg_ttgg'])
def test_me_fp64_massless_limit_vs_oracle(h, proc):
    """m_t = 0: the GPU kernels against the oracle in the limit where the oracle's partial
    amplitudes are pinned to the Parke-Taylor form (massless spinors and propagators)."""
    n = ME_N[proc] + 3
    par = dict(P)
    par['m_t'] = 0.0
    prm = mf.params_from_dict(par)
    pid = mf.PROCESS[proc]
    say('me fp64 massless', proc, n)
    ev = mf.mf_phase_space(h, pid, prm, n, seed=23)
    me = mf.matrix_element(h, pid, ev['p'], mf.MF_FP64, prm)
    torch.cuda.synchronize()
    pt = torch.tensor(np.ascontiguousarray(np.transpose(ev['p'].cpu().numpy(), (2, 0, 1))), dtype=torch.float64)
    ref = integrand.me(proc, pt, par).numpy()
    rel = np.abs(me.cpu().numpy() / ref - 1)
    say('  max rel', rel.max())
    assert rel.max() < 1e-12


@pytest.mark.parametrize('proc', PROCS)
def test_me_fp32_vs_oracle(h, proc):
    n = ME_N[proc] + 3
    say('me fp32', proc, n)
    ev = gpu_events(h, proc, n, seed=22)
    me = gpu_me(h, proc, ev['p'], mf.MF_FP32)
    ref = oracle_me(proc, ev['p'].cpu().numpy())
    ok = ev['pass_'].cpu().numpy().astype(bool)
    rel = np.abs(me / ref - 1)[ok]
    say('  median', np.median(rel), 'max', rel.max())
    assert np.median(rel) < 1e-5 and rel.max() < 1e-3


@pytest.mark.parametrize('prec', ['fp32_mfma_f32', 'fp32_mfma_bf16'])
@pytest.mark.parametrize('proc', ['gg_tt', 'gg_ttg', 'gg_ttgg'])
def test_me_mfma_colour_vs_oracle(h, proc, prec):
    n = ME_N[proc] + 5          # not a multiple of the wave size: tail lanes recompute, do not store
    say('me', prec, proc, n)
    ev = gpu_events(h, proc, n, seed=23)
    me = gpu_me(h, proc, ev['p'], mf.PRECISION[prec])
    ref = oracle_me(proc, ev['p'].cpu().numpy())
    ok = ev['pass_'].cpu().numpy().astype(bool)
    rel = np.abs(me / ref - 1)[ok]
    say('  median', np.median(rel), 'max', rel.max())
    assert np.median(rel) < 1e-5 and rel.max() < 1e-3


NAN_FORMS = ([(proc, 'fp64') for proc in PROCS] + [(proc, 'fp32') for proc in PROCS]
             + [(proc, prec) for proc in PROCS[1:] for prec in ('fp32_mfma_f32', 'fp32_mfma_bf16')])


@pytest.mark.parametrize('proc,prec', NAN_FORMS)
def test_me_nan_momenta_give_nan_and_leave_other_events(h, proc, prec):
    """NaN momenta in one event give a NaN |M|^2 for that event; every other event of
    the launch (same wavefront, same matrix-core tile) is bit-identical to a clean run."""
    n, bad = 130, 7
    say('me nan event', proc, prec, n)
    ev = gpu_events(h, proc, n, seed=24)
    p = ev['p'].contiguous()
    pb = p.clone()
    pb[2, :, bad] = float('nan')
    keep = np.arange(n) != bad
    blocks = [64, 128, 256] if (proc, prec) == ('gg_ttgg', 'fp64') else [None]
    for blk in blocks:
        if blk is None:
            a, b = gpu_me(h, proc, p, mf.PRECISION[prec]), gpu_me(h, proc, pb, mf.PRECISION[prec])
        else:
            a = _layout_me(h, p, blk).cpu().numpy()
            b = _layout_me(h, pb, blk).cpu().numpy()
        assert np.isnan(b[bad]), (blk, b[bad])
        assert np.array_equal(a[keep], b[keep]), blk


@pytest.mark.parametrize('n', [1, 63, 65, 257])
def test_me_mfma_ragged_batches(h, n):
    say('mfma ragged', n)
    ev = gpu_events(h, 'gg_ttgg', n, seed=24)
    a = gpu_me(h, 'gg_ttgg', ev['p'], mf.MF_FP32_MFMA_F32)
    b = gpu_me(h, 'gg_ttgg', ev['p'], mf.MF_FP64)
    assert np.abs(a / b - 1).max() < 1e-3


def test_me_closed_forms_on_gpu(h):
    # e+e- -> mu+mu- and gg -> ttbar against their closed forms, per event
    for proc in ('ee_mumu', 'gg_tt'):
        n = 10000
        say('closed form', proc, n)
        ev = gpu_events(h, proc, n, seed=3)
        p = ev['p'].cpu().numpy()
        me = gpu_me(h, proc, ev['p'], mf.MF_FP64)
        if proc == 'ee_mumu':
            c = (p[0, 1] * p[2, 1] + p[0, 2] * p[2, 2] + p[0, 3] * p[2, 3]) / (
                np.sqrt((p[0, 1:] ** 2).sum(0)) * np.sqrt((p[2, 1:] ** 2).sum(0)))
            ref = (4 * math.pi * PEE['alpha']) ** 2 * (1 + c * c)
        else:
            s = P['sqrt_s'] ** 2
            t1 = 2 * (p[0, 0] * p[2, 0] - (p[0, 1:] * p[2, 1:]).sum(0)) / s
            ref = np.array([closed_forms.gg_tt_me(float(t), s, P['m_t'], P['alpha_s']) for t in t1])
        assert np.abs(me / ref - 1).max() < 1e-12


@pytest.mark.parametrize('proc,n', [('gg_tt', 1_000_000), ('gg_ttg', 4_000_000), ('gg_ttgg', 1_000_000)])
def test_me_full_size_sampled(h, proc, n):
    """At the benchmark batch sizes: all outputs finite and positive, sampled events vs oracle."""
    say('me full size', proc, n)
    ev = gpu_events(h, proc, n, seed=1 + mf.PROCESS[proc])
    for prec in (mf.MF_FP64, mf.MF_FP32):
        me = mf.matrix_element(h, mf.PROCESS[proc], ev['p'], prec, prm_of(proc))
        torch.cuda.synchronize()
        assert bool(torch.isfinite(me).all()) and float(me.min()) > 0
        idx = torch.tensor(np.random.default_rng(9).choice(n, 24, replace=False), device=me.device)
        idx = torch.cat([idx, torch.tensor([0, n - 1], device=me.device)])
        ps = ev['p'][:, :, idx].cpu().numpy()
        ref = oracle_me(proc, ps)
        got = me[idx].double().cpu().numpy()
        rel = np.abs(got / ref - 1)
        ok = ev['pass_'][idx].cpu().numpy().astype(bool)
        if prec == mf.MF_FP64:
            assert rel.max() < 1e-12
        else:
            assert rel[ok].max() < 1e-3


@pytest.mark.parametrize('proc,n', [('gg_ttgg', 1_000_000), ('gg_ttg', 4_000_000), ('gg_tt', 4_000_000)])
def test_me_fp32_forms_vs_fp64_every_event_full_size(h, proc, n):
    """Every event of a full-size batch (10^6 gg -> ttbar gg events: the benchmark launch): each
    FP32 form (VALU colour, FP32-MFMA colour, BF16x3-MFMA colour) against the FP64 kernel, which
    the tests above pin to the oracle.  Bars on the events passing the cuts: median 1e-5, max 1e-3.
    Checking all events, not a sample, would expose a kernel build that is wrong on a subset."""
    pid = mf.PROCESS[proc]
    say('me fp32 forms vs fp64, every event', proc, n)
    ev = gpu_events(h, proc, n, seed=4)
    ref = mf.matrix_element(h, pid, ev['p'], mf.MF_FP64, prm_of(proc))
    ok = ev['pass_'].bool()
    for prec in (mf.MF_FP32, mf.MF_FP32_MFMA_F32, mf.MF_FP32_MFMA_BF16):
        me = mf.matrix_element(h, pid, ev['p'], prec, prm_of(proc))
        torch.cuda.synchronize()
        assert bool(torch.isfinite(me).all())
        rel = ((me.double() - ref) / ref).abs()[ok]
        say('  precision', prec, 'median', float(rel.median()), 'max', float(rel.max()))
        assert float(rel.median()) < 1e-5 and float(rel.max()) < 1e-3


@pytest.mark.parametrize('proc,n', [('gg_ttgg', 1_000_000), ('gg_ttg', 4_000_000), ('gg_tt', 4_000_000)])
def test_me_forms_bitwise_repeatable_full_size(h, proc, n):
    """Each matrix-element form, launched three times on the same full-size batch, returns
    bit-identical values.  Every event is computed by one lane (or one quad) alone, in a fixed
    order, so a difference between launches can only come from a build whose results depend on
    timing; such a build is also wrong on some events.  After a small launch first, so that the
    kernels do not start from their own previous state."""
    small = gpu_events(h, proc, 43, seed=22)
    ev = gpu_events(h, proc, n, seed=4)
    for prec in (mf.MF_FP32, mf.MF_FP32_MFMA_F32, mf.MF_FP32_MFMA_BF16, mf.MF_FP64):
        say('  repeatability', proc, n, 'precision', prec)
        pid = mf.PROCESS[proc]
        mf.matrix_element(h, pid, small['p'], prec, prm_of(proc))
        outs = [mf.matrix_element(h, pid, ev['p'], prec, prm_of(proc)) for _ in range(3)]
        torch.cuda.synchronize()
        assert bool(torch.isfinite(outs[0]).all())
        for o in outs[1:]:
            assert torch.equal(o, outs[0]), int((o != outs[0]).sum())


def test_me_lorentz_invariance_fp64(h):
    n = 512
    say('lorentz gg_ttgg', n)
    ev = gpu_events(h, 'gg_ttgg', n, seed=8)
    p = ev['p']
    a = mf.matrix_element(h, mf.MF_GG_TTGG, p, mf.MF_FP64)
    # boost along z (the kernel takes the beams along the z axis), beta = 0.6
    beta = 0.6
    g = 1 / math.sqrt(1 - beta * beta)
    q = p.clone()
    q[:, 0] = g * (p[:, 0] + beta * p[:, 3])
    q[:, 3] = g * (p[:, 3] + beta * p[:, 0])
    b = mf.matrix_element(h, mf.MF_GG_TTGG, q.contiguous(), mf.MF_FP64)
    torch.cuda.synchronize()
    # the boost rounds the momenta (1e-16 relative), which near-singular events
    # amplify by their condition number (up to ~1e4 here)
    rel = ((a / b) - 1).abs()
    assert float(rel.max()) < 1e-10 and float(rel.median()) < 1e-13


def test_me_empty_and_tiny_batches(h):
    for n in (0, 1, 63, 65):
        say('tiny batch', n)
        p = torch.empty(6, 4, n, dtype=torch.float64, device='cuda')
        if n:
            ev = gpu_events(h, 'gg_ttgg', n, seed=2)
            p = ev['p']
        me = mf.matrix_element(h, mf.MF_GG_TTGG, p, mf.MF_FP64)
        torch.cuda.synchronize()
        assert me.shape == (n,)
        if n:
            ref = oracle_me('gg_ttgg', p.cpu().numpy())
            assert np.abs(me.cpu().numpy() / ref - 1).max() < 1e-12


def _layout_me(h, p, block):
    """FP64 gg -> ttbar gg with the event layout `block` selects (64: one lane per event,
    128: two, 256: four); the handle goes back to its default (two lanes) afterwards."""
    h.set_launch(mf.MF_GG_TTGG, mf.MF_FP64, block)
    try:
        return mf.matrix_element(h, mf.MF_GG_TTGG, p, mf.MF_FP64)
    finally:
        h.set_launch(mf.MF_GG_TTGG, mf.MF_FP64, 0)


def _quad_me(h, p):
    """FP64 gg -> ttbar gg with the four-lanes-per-event layout."""
    return _layout_me(h, p, 256)


@pytest.mark.parametrize('block,n', [(64, ME_N['gg_ttgg'] + 3), (128, 1), (128, 31), (128, 32), (128, 33),
                                     (128, ME_N['gg_ttgg'] + 3)])
def test_me_ttgg_layouts_vs_oracle(h, block, n):
    """One lane per event and two lanes per event (orderings in pairs related by swapping the
    beams and the final gluons, DPP exchange of currents and amplitudes) vs the oracle, with
    batches that end inside a workgroup of 32 events."""
    say('me ttgg layout', block, n)
    ev = gpu_events(h, 'gg_ttgg', n, seed=32)
    me = _layout_me(h, ev['p'], block)
    torch.cuda.synchronize()
    ref = oracle_me('gg_ttgg', ev['p'].cpu().numpy())
    rel = np.abs(me.cpu().numpy() / ref - 1)
    say('  max rel', rel.max())
    assert rel.max() < 1e-12


def test_me_ttgg_pair_layout_full_size(h):
    """At the benchmark batch size the two-lane layout equals the one-lane kernel to rounding on
    every event and sampled events match the oracle; an empty batch is a no-op."""
    n = 1_000_000
    say('me ttgg pair layout full size', n)
    ev = gpu_events(h, 'gg_ttgg', n, seed=4)
    a = _layout_me(h, ev['p'], 128)
    b = _layout_me(h, ev['p'], 64)
    torch.cuda.synchronize()
    rel = ((a / b) - 1).abs()
    say('  pair vs one-lane max rel', float(rel.max()))
    assert float(rel.max()) < 1e-12
    idx = np.concatenate([np.random.default_rng(5).choice(n, 16, replace=False), [0, 31, 32, n - 1]])
    ref = oracle_me('gg_ttgg', ev['p'][:, :, torch.tensor(idx, device=a.device)].cpu().numpy())
    assert np.abs(a[torch.tensor(idx, device=a.device)].cpu().numpy() / ref - 1).max() < 1e-12
    e = _layout_me(h, torch.empty(6, 4, 0, dtype=torch.float64, device='cuda'), 128)
    assert e.shape == (0,)


@pytest.mark.parametrize('n', [1, 15, 16, 17, ME_N['gg_ttgg'] + 3])
def test_me_ttgg_quad_layout_vs_oracle(h, n):
    """Four lanes per event (orderings split by first gluon, DPP colour exchange) vs the oracle,
    with batches that end inside a workgroup of 16 events."""
    say('me ttgg quad layout', n)
    ev = gpu_events(h, 'gg_ttgg', n, seed=31)
    me = _quad_me(h, ev['p'])
    torch.cuda.synchronize()
    ref = oracle_me('gg_ttgg', ev['p'].cpu().numpy())
    rel = np.abs(me.cpu().numpy() / ref - 1)
    say('  max rel', rel.max())
    assert rel.max() < 1e-12


def test_me_ttgg_quad_layout_full_size(h):
    """At the benchmark batch size: quad layout equals the one-lane FP64 kernel to rounding
    on every event, and sampled events match the oracle; an empty batch is a no-op."""
    n = 1_000_000
    say('me ttgg quad layout full size', n)
    ev = gpu_events(h, 'gg_ttgg', n, seed=4)
    a = _quad_me(h, ev['p'])
    b = _layout_me(h, ev['p'], 64)
    torch.cuda.synchronize()
    rel = ((a / b) - 1).abs()
    say('  quad vs one-lane max rel', float(rel.max()))
    assert float(rel.max()) < 1e-12
    idx = np.concatenate([np.random.default_rng(3).choice(n, 16, replace=False), [0, n - 1]])
    ref = oracle_me('gg_ttgg', ev['p'][:, :, torch.tensor(idx, device=a.device)].cpu().numpy())
    assert np.abs(a[torch.tensor(idx, device=a.device)].cpu().numpy() / ref - 1).max() < 1e-12
    e = _quad_me(h, torch.empty(6, 4, 0, dtype=torch.float64, device='cuda'))
    assert e.shape == (0,)


# ------------------------------------------------------------------ Vegas
def test_vegas_refine_vs_oracle(h):
    proc = 'gg_ttg'
    n = 20000 + 11
    d = processes.dims(proc)
    say('vegas refine', proc, n)
    ev = gpu_events(h, proc, n, seed=31, edges=ovegas.uniform_grid(d, 50))
    me = mf.matrix_element(h, mf.PROCESS[proc], ev['p'], mf.MF_FP64, prm_of(proc))
    dev = me.device
    edges = torch.tensor(ovegas.uniform_grid(d, 50), dtype=torch.float64, device=dev).contiguous()
    acc = torch.empty(2 + d * 50, dtype=torch.float64, device=dev)
    F = torch.empty(n, dtype=torch.float64, device=dev)
    mf.mf_vegas_refine(h, prm_of(proc), n, d, 50, 1.5, ev['w'], ev['jac'], me, ev['pass_'], ev['bin_idx'],
                       acc, edges, F=F)
    torch.cuda.synchronize()
    s = P['sqrt_s'] ** 2
    F_ref = closed_forms.GEV2_TO_PB * ev['w'].cpu().numpy() * me.cpu().numpy() / (2 * s) * \
        ev['pass_'].cpu().numpy() * ev['jac'].cpu().numpy()
    assert np.abs(F.cpu().numpy() - F_ref).max() <= 1e-13 * np.abs(F_ref).max()
    sf, sf2, hist = ovegas.accumulate(F_ref, ev['bin_idx'].cpu().numpy().astype(np.int64), 50)
    a = acc.cpu().numpy()
    assert abs(a[0] / sf - 1) < 1e-12 and abs(a[1] / sf2 - 1) < 1e-12
    assert np.abs(a[2:].reshape(d, 50) - hist).max() <= 1e-12 * hist.max()
    new_ref = ovegas.refine(ovegas.uniform_grid(d, 50), hist, 1.5)
    assert np.abs(edges.cpu().numpy() - new_ref).max() < 1e-12


def test_vegas_deterministic(h):
    proc = 'gg_tt'
    n = 300000
    say('vegas determinism', n)
    ev = gpu_events(h, proc, n, seed=5)
    me = mf.matrix_element(h, mf.PROCESS[proc], ev['p'], mf.MF_FP64, prm_of(proc))
    outs = []
    for _ in range(2):
        edges = torch.tensor(ovegas.uniform_grid(2, 50), dtype=torch.float64, device='cuda').contiguous()
        acc = torch.empty(2 + 100, dtype=torch.float64, device='cuda')
        mf.mf_vegas_refine(h, prm_of(proc), n, 2, 50, 1.5, ev['w'], ev['jac'], me, ev['pass_'],
                           ev['bin_idx'], acc, edges)
        torch.cuda.synchronize()
        outs.append((acc.cpu().numpy(), edges.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_vegas_bad_uniform_batch_keeps_state_finite(h):
    """A batch holding a NaN, a negative and a >= 1 uniform goes through phase space, matrix
    element and mf_vegas_refine: the NaN event (NaN momenta, |M|^2 and weight) adds exactly 0,
    the sums and the refined grid stay finite, and they equal the oracle's accumulation of
    the same events with that event's F set to 0."""
    proc, n, nb = 'gg_ttg', 130, 50
    pid, d = mf.PROCESS[proc], processes.dims(proc)
    x = philox.uniforms(50, n, d)
    xb, bad = _bad_uniforms(x, nb)
    dev = torch.device('cuda', 0)
    hh = mf.Handle(0)
    try:
        for prec in (mf.MF_FP64, mf.MF_FP32_MFMA_BF16):
            say('vegas refine with a NaN event', proc, n, prec)
            ed = torch.tensor(ovegas.uniform_grid(d, nb), dtype=torch.float64, device=dev).contiguous()
            xt = torch.tensor(xb, dtype=torch.float64, device=dev).contiguous()
            o = mf.mf_phase_space(hh, pid, prm_of(proc), n, x=xt, edges=ed, nb=nb,
                                  pass_=torch.empty(n, dtype=torch.uint8, device=dev),
                                  bin_idx=torch.empty(d, n, dtype=torch.int16, device=dev),
                                  jac=torch.empty(n, dtype=torch.float64, device=dev))
            me = mf.matrix_element(hh, pid, o['p'], prec, prm_of(proc))
            acc = torch.empty(2 + d * nb, dtype=torch.float64, device=dev)
            F = torch.empty(n, dtype=torch.float64, device=dev)
            mf.mf_vegas_refine(hh, prm_of(proc), n, d, nb, 1.5, o['w'], o['jac'], me, o['pass_'], o['bin_idx'],
                               acc, ed, F=F)
            torch.cuda.synchronize()
            m = me.double().cpu().numpy()
            w = o['w'].cpu().numpy()
            assert np.isnan(m[5]) and not w[5] > 0.0       # NaN in, NaN out (or a failed solve: 0)
            a, e, f = acc.cpu().numpy(), ed.cpu().numpy(), F.cpu().numpy()
            assert np.isfinite(a).all() and np.isfinite(e).all() and np.isfinite(f).all()
            assert f[5] == 0.0
            assert (np.diff(e, axis=1) >= 0).all() and (e[:, 0] == 0).all() and (e[:, -1] == 1).all()
            ok = o['pass_'].cpu().numpy().astype(bool) & (w == w) & (w != 0)
            s_ = P['sqrt_s'] ** 2
            F_ref = np.where(ok, closed_forms.GEV2_TO_PB * w * np.where(ok, m, 0.0) / (2 * s_)
                             * o['jac'].cpu().numpy(), 0.0)
            sf, sf2, hist = ovegas.accumulate(F_ref, o['bin_idx'].cpu().numpy().astype(np.int64), nb)
            assert abs(a[0] / sf - 1) < 1e-12 and abs(a[1] / sf2 - 1) < 1e-12
            assert np.abs(a[2:].reshape(d, nb) - hist).max() <= 1e-12 * hist.max()
            new_ref = ovegas.refine(ovegas.uniform_grid(d, nb), hist, 1.5)
            assert np.abs(e - new_ref).max() < 1e-12
    finally:
        hh.close()


def test_graph_replay_after_a_larger_call_on_the_same_handle(h):
    """The handle's workspace is allocated once: a graph captured from a small integrator
    still replays correctly after a second integrator with a larger batch has used the
    same handle (the workspace is not regrown, so the graph's pointers stay valid)."""
    from paper_2211_14056_amd.integrator import VegasIntegrator
    hh = mf.Handle(0)
    try:
        say('graph replay after a larger call')
        small = VegasIntegrator('gg_tt', precision=mf.MF_FP64, n=3000, batches=1, seed=3, handle=hh)
        eager = []
        for _ in range(3):
            small.enqueue_iteration()
            eager.append((small.acc.clone(), small.edges.clone()))
        small.reset()
        small.iterate(1)
        small.capture()
        big = VegasIntegrator('gg_ttg', precision=mf.MF_FP64, n=600_000, batches=1, seed=4, handle=hh)
        big.iterate(1)
        torch.cuda.synchronize()
        got = [eager[0]]
        for _ in range(2):
            small.graph.launch()
            torch.cuda.synchronize()
            got.append((small.acc.clone(), small.edges.clone()))
        for (a1, e1), (a2, e2) in zip(eager, got):
            assert torch.equal(a1, a2) and torch.equal(e1, e2)
    finally:
        hh.close()


def _gpu_vegas(h, proc, n, iters, seed, precision=mf.MF_FP64):
    pid = mf.PROCESS[proc]
    d = processes.dims(proc)
    dev = torch.device('cuda', 0)
    edges = torch.tensor(ovegas.uniform_grid(d, 50), dtype=torch.float64, device=dev).contiguous()
    acc = torch.empty(2 + d * 50, dtype=torch.float64, device=dev)
    Is, vs = [], []
    for it in range(iters):
        ev = mf.mf_phase_space(h, pid, prm_of(proc), n, seed=seed, offset=it * n, edges=edges, nb=50,
                               pass_=torch.empty(n, dtype=torch.uint8, device=dev),
                               bin_idx=torch.empty(d, n, dtype=torch.int16, device=dev),
                               jac=torch.empty(n, dtype=torch.float64, device=dev))
        me = mf.matrix_element(h, pid, ev['p'], precision, prm_of(proc))
        mf.mf_vegas_refine(h, prm_of(proc), n, d, 50, 1.5, ev['w'], ev['jac'], me, ev['pass_'],
                           ev['bin_idx'], acc, edges)
        a = acc.cpu().numpy()
        I, v = ovegas.estimate(a[0], a[1], n)
        Is.append(I)
        vs.append(v)
    return ovegas.combine(Is, vs), Is, vs, edges.cpu().numpy()


def test_vegas_ee_mumu_matches_oracle_and_closed_form(h):
    n, iters = 100_000, 5
    say('vegas ee_mumu', n, iters)
    (I, sig, chi2), Is, vs, edges = _gpu_vegas(h, 'ee_mumu', n, iters, seed=1)
    f = lambda y: integrand.integrand('ee_mumu', PEE, y)[0]
    I_o, sig_o, chi2_o, its, edges_o = ovegas.integrate(f, 2, n, iters, seed=1)
    assert abs(I / I_o - 1) < 1e-12
    assert np.abs(edges - edges_o).max() < 1e-10
    ref = closed_forms.ee_mumu_sigma(PEE['sqrt_s'] ** 2, PEE['alpha']) * closed_forms.GEV2_TO_PB
    say('  sigma', I, '+-', sig, 'closed form', ref)
    assert abs(I - ref) < 3 * sig


def test_vegas_gg_tt_closed_form(h):
    n, iters = 1_000_000, 5
    say('vegas gg_tt', n, iters)
    (I, sig, chi2), Is, vs, edges = _gpu_vegas(h, 'gg_tt', n, iters, seed=2)
    ref = closed_forms.gg_tt_sigma(P['sqrt_s'] ** 2, P['m_t'], P['alpha_s']) * closed_forms.GEV2_TO_PB
    say('  sigma', I, '+-', sig, 'closed form', ref)
    assert abs(I - ref) < 3 * sig


def test_vegas_pull_distribution(h):
    """Vegas on the GPU over 20 seeds: the pulls (I - closed form)/sigma of sigma(ee->mumu) and
    sigma_hat(gg->ttbar) are consistent with N(0, 1) (mean and spread within their 3-sigma sampling
    ranges for 20 draws), so the quoted errors are the statistical ones."""
    ref = {'ee_mumu': closed_forms.ee_mumu_sigma(PEE['sqrt_s'] ** 2, PEE['alpha']) * closed_forms.GEV2_TO_PB,
           'gg_tt': closed_forms.gg_tt_sigma(P['sqrt_s'] ** 2, P['m_t'], P['alpha_s']) * closed_forms.GEV2_TO_PB}
    for proc, n, iters in (('ee_mumu', 20_000, 4), ('gg_tt', 50_000, 4)):
        pulls = []
        for seed in range(1, 21):
            (I, sig, chi2), _, _, _ = _gpu_vegas(h, proc, n, iters, seed=100 + seed)
            pulls.append((I - ref[proc]) / sig)
        pulls = np.array(pulls)
        say('vegas pulls', proc, 'mean', pulls.mean(), 'std', pulls.std(ddof=1))
        assert abs(pulls.mean()) < 3 / math.sqrt(20)
        assert 0.5 < pulls.std(ddof=1) < 1.5
        # "within 1 sigma" over seeds: I +- sigma covers the closed form at the nominal 68% rate
        # (binomial(20, 0.683): mean 13.7, standard deviation 2.1)
        assert (np.abs(pulls) < 1).sum() >= 8


# ------------------------------------------------------------------ derivative
def _vjp_gpu(h, proc, x, gbar, precision, edges=None):
    pid = mf.PROCESS[proc]
    d, n = x.shape
    dev = torch.device('cuda', 0)
    xt = torch.tensor(x, dtype=torch.float64, device=dev).contiguous()
    gb = torch.tensor(gbar, dtype=torch.float64, device=dev).contiguous()
    gx = torch.empty(d, n, dtype=torch.float64, device=dev)
    gth = torch.empty(n, 2, dtype=torch.float64, device=dev)
    me = torch.empty(n, dtype=torch.float64 if precision == mf.MF_FP64 else torch.float32, device=dev)
    e = None if edges is None else torch.tensor(edges, dtype=torch.float64, device=dev).contiguous()
    req = mf.make_request(pid, None, me, x=xt, grad_me=gb, grad_x=gx, grad_theta=gth, n=n)
    mf.mf_matrix_element_vjp(h, [req], precision, prm_of(proc), edges=e, nb=50)
    torch.cuda.synchronize()
    return me.double().cpu().numpy(), gx.cpu().numpy(), gth.cpu().numpy()


def _edges(d, seed):
    rng = np.random.default_rng(seed)
    w_ = rng.uniform(0.5, 1.5, (d, 50))
    e = np.concatenate([np.zeros((d, 1)), np.cumsum(w_, 1) / w_.sum(1, keepdims=True)], 1)
    e[:, -1] = 1.0
    return e


def _normwise(a, b):
    """Per event: max_k |a_k - b_k| / max_k |b_k| over the derivative components."""
    return np.abs(a - b).max(0) / np.abs(b).max(0)


VJP_N = {'gg_tt': 64, 'gg_ttg': 97, 'gg_ttgg': 69}     # full waves plus ragged tails


@pytest.mark.parametrize('proc', ['gg_tt', 'gg_ttg', 'gg_ttgg'])
def test_vjp_fp64_vs_oracle_reverse_mode(h, proc):
    from oracle import grad as ograd
    n = VJP_N[proc]
    d = processes.dims(proc)
    x = philox.uniforms(41, n, d)
    edges = _edges(d, 3)
    gbar = np.random.default_rng(1).uniform(0.5, 2.0, n)
    say('vjp fp64', proc, n)
    me, gx, gth = _vjp_gpu(h, proc, x, gbar, mf.MF_FP64, edges)
    me_o, gx_o, gth_o = ograd.vjp(proc, P, x, gbar, edges)
    assert np.abs(me / me_o - 1).max() < 1e-12
    ga = np.concatenate([gx, gth[:, :1].T], 0)
    gb = np.concatenate([gx_o, gth_o[:, :1].T], 0)
    err = _normwise(ga, gb)
    say('  max normwise', err.max())
    assert err.max() < 1e-10
    assert np.abs(gth[:, 1] / gth_o[:, 1] - 1).max() < 1e-12


@pytest.mark.parametrize('proc', ['gg_tt', 'gg_ttg', 'gg_ttgg'])
def test_vjp_fp32_vs_oracle(h, proc):
    from oracle import grad as ograd
    n = VJP_N[proc]
    d = processes.dims(proc)
    x = philox.uniforms(42, n, d)
    gbar = np.ones(n)
    say('vjp fp32', proc, n)
    me, gx, gth = _vjp_gpu(h, proc, x, gbar, mf.MF_FP32)
    me_o, gx_o, gth_o = ograd.vjp(proc, P, x, gbar)
    ga = np.concatenate([gx, gth[:, :1].T], 0)
    gb = np.concatenate([gx_o, gth_o[:, :1].T], 0)
    err = _normwise(ga, gb)
    say('  median', np.median(err), 'max', err.max())
    assert np.median(err) < 1e-4 and err.max() < 1e-2


@pytest.mark.parametrize('precision', ['fp64', 'fp32'])
def test_vjp_empty_and_tiny_batches(h, precision):
    """n = 0 is a no-op; one event and a ragged 65 (one full wavefront plus one) match the oracle."""
    from oracle import grad as ograd
    prec = mf.PRECISION[precision]
    for proc, n in (('gg_tt', 0), ('gg_ttg', 0), ('gg_tt', 1), ('gg_ttg', 1), ('gg_tt', 65)):
        say('vjp tiny batch', precision, proc, n)
        d = processes.dims(proc)
        x = philox.uniforms(44, n, d)
        gbar = np.linspace(0.5, 1.5, n)
        me, gx, gth = _vjp_gpu(h, proc, x, gbar, prec)
        assert me.shape == (n,) and gx.shape == (d, n) and gth.shape == (n, 2)
        if not n:
            continue
        me_o, gx_o, gth_o = ograd.vjp(proc, P, x, gbar)
        err = _normwise(np.concatenate([gx, gth[:, :1].T], 0), np.concatenate([gx_o, gth_o[:, :1].T], 0))
        if precision == 'fp64':
            assert np.abs(me / me_o - 1).max() < 1e-12
            assert err.max() < 1e-10
        else:
            assert np.abs(me / me_o - 1).max() < 1e-3
            assert np.median(err) < 1e-4 and err.max() < 1e-2


def test_vjp_vs_finite_differences_ttg(h):
    """Central differences (h = 1e-6) of the FP64 oracle, the configuration of the tt g derivative run."""
    from oracle import grad as ograd
    proc, n = 'gg_ttg', 8
    d = processes.dims(proc)
    x = 0.05 + 0.9 * philox.uniforms(43, n, d)
    say('vjp vs FD', proc, n)
    me, gx, gth = _vjp_gpu(h, proc, x, np.ones(n), mf.MF_FP64)
    fx, fm = ograd.finite_difference(proc, P, x)
    ga = np.concatenate([gx, gth[:, :1].T], 0)
    gb = np.concatenate([fx, fm[None, :]], 0)
    assert _normwise(ga, gb).max() < 1e-6


def test_vjp_full_size_ttg_sampled(h):
    """4e6 events (the tt g derivative configuration): finite, forward value equal to mf_matrix_element."""
    proc, n = 'gg_ttg', 4_000_000
    pid = mf.PROCESS[proc]
    d = processes.dims(proc)
    say('vjp full size', proc, n)
    ev = gpu_events(h, proc, n, seed=44)
    dev = torch.device('cuda', 0)
    gx = torch.empty(d, n, dtype=torch.float64, device=dev)
    gth = torch.empty(n, 2, dtype=torch.float64, device=dev)
    gb = torch.ones(n, dtype=torch.float64, device=dev)
    me = torch.empty(n, dtype=torch.float32, device=dev)
    req = mf.make_request(pid, None, me, x=ev['x'], grad_me=gb, grad_x=gx, grad_theta=gth, n=n)
    mf.mf_matrix_element_vjp(h, [req], mf.MF_FP32, prm_of(proc))
    me_fwd = mf.matrix_element(h, pid, ev['p'], mf.MF_FP32)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(gx).all()) and bool(torch.isfinite(gth).all())
    assert float(((me.double() - me_fwd.double()).abs() / me_fwd.double()).max()) < 1e-5
    from oracle import grad as ograd
    idx = np.random.default_rng(2).choice(n, 6, replace=False)
    x = ev['x'][:, idx].cpu().numpy()
    me_o, gx_o, gth_o = ograd.vjp(proc, P, x, np.ones(6))
    ga = np.concatenate([gx[:, idx].cpu().numpy(), gth[idx, :1].cpu().numpy().T], 0)
    gbb = np.concatenate([gx_o, gth_o[:, :1].T], 0)
    assert _normwise(ga, gbb).max() < 1e-2


def test_vjp_several_requests_in_one_call_equal_separate_calls(h):
    """Requests of all three processes in one mf_matrix_element_vjp call (one launch per
    process, a grid of 64-event tiles over its requests, ragged sizes) give bit for bit the
    results of one call per request."""
    specs = [('gg_ttgg', 70), ('gg_tt', 1), ('gg_ttg', 130), ('gg_ttgg', 64), ('gg_tt', 200), ('gg_ttg', 3)]
    dev = torch.device('cuda', 0)
    for prec in (mf.MF_FP32, mf.MF_FP64):
        say('vjp batch vs separate', prec)
        bufs, reqs = [], []
        for i, (proc, n) in enumerate(specs):
            pid, d = mf.PROCESS[proc], processes.dims(proc)
            x = torch.tensor(philox.uniforms(60 + i, n, d), dtype=torch.float64, device=dev).contiguous()
            b = dict(x=x, gb=torch.linspace(0.5, 1.5, n, dtype=torch.float64, device=dev),
                     gx=torch.empty(d, n, dtype=torch.float64, device=dev),
                     gth=torch.empty(n, 2, dtype=torch.float64, device=dev),
                     me=torch.empty(n, dtype=torch.float64 if prec == mf.MF_FP64 else torch.float32, device=dev))
            bufs.append(b)
            reqs.append(mf.make_request(pid, None, b['me'], x=x, grad_me=b['gb'], grad_x=b['gx'],
                                        grad_theta=b['gth'], n=n))
        mf.mf_matrix_element_vjp(h, reqs, prec, prm_of('gg_tt'))
        torch.cuda.synchronize()
        together = [{k: v.clone() for k, v in b.items()} for b in bufs]
        for r in reqs:
            mf.mf_matrix_element_vjp(h, [r], prec, prm_of('gg_tt'))
        torch.cuda.synchronize()
        for a, b in zip(together, bufs):
            for k in ('gx', 'gth', 'me'):
                assert torch.equal(a[k], b[k]), k


def test_mixed_iteration_graph_equals_eager_and_share_vjp_matches_oracle(h):
    """The 64-request mixed iteration (phase space, one matrix-element call over all
    requests, one derivative call over the gg -> ttbar gg share, Vegas per request) captured
    in one library graph: three replays equal three eager iterations bit for bit (sums,
    grids, derivatives), and the share's derivative matches the oracle's reverse mode on
    sampled events."""
    from oracle import grad as ograd
    from paper_2211_14056_amd.mixed import MixedIteration
    from paper_2211_14056_amd.workloads import mixed_batch
    spec = mixed_batch(64, seed=5, scale=0.004)
    say('mixed iteration', sum(n for _, n in spec), 'events')
    eager = MixedIteration(spec, handle=h)
    ref, grids = [], []
    for _ in range(3):
        grids.append(eager.edges['gg_ttgg'].clone())
        eager.enqueue()
        torch.cuda.synchronize()
        ref.append(eager.state())
    it = MixedIteration(spec, handle=h)
    it.enqueue()
    torch.cuda.synchronize()
    got = [it.state()]
    it.capture()
    for _ in range(2):
        it.launch()
        torch.cuda.synchronize()
        junk = torch.randn(1000, device='cuda').sum()       # unrelated eager work between replays
        got.append(it.state())
    for a, b in zip(ref, got):
        assert a.keys() == b.keys()
        for k in a:
            assert torch.equal(a[k], b[k]), k
    # derivative of the gg -> ttbar gg share (last iteration) against the oracle
    ed = grids[2].cpu().numpy()
    checked = 0
    for i, r in enumerate(eager.reqs):
        if 'x' not in r or checked >= 2:
            continue
        idx = np.random.default_rng(i).choice(r['n'], min(8, r['n']), replace=False)
        x = r['x'][:, idx].cpu().numpy()
        me_o, gx_o, gth_o = ograd.vjp('gg_ttgg', P, x, np.ones(len(idx)), edges=ed)
        ga = np.concatenate([r['gx'][:, idx].cpu().numpy(), r['gth'][idx, :1].cpu().numpy().T], 0)
        gbb = np.concatenate([gx_o, gth_o[:, :1].T], 0)
        err = _normwise(ga, gbb)
        say('  share vjp request', i, 'median', np.median(err), 'max', err.max())
        assert np.median(err) < 1e-4 and err.max() < 1e-2
        assert np.abs(r['gth'][idx, 1].cpu().numpy() / gth_o[:, 1] - 1).max() < 1e-3
        checked += 1
    assert checked == 2


def test_autograd_function(h):
    from oracle import grad as ograd
    from paper_2211_14056_amd.autograd import MatrixElementFn
    proc, n = 'gg_ttg', 16
    d = processes.dims(proc)
    x0 = philox.uniforms(45, n, d)
    x = torch.tensor(x0, dtype=torch.float64, device='cuda', requires_grad=True)
    theta = torch.tensor([P['m_t'], P['alpha_s']], dtype=torch.float64, requires_grad=True)
    say('autograd', proc, n)
    me = MatrixElementFn.apply(x, theta, h, proc, mf.MF_FP64, None, mf.params_from_dict(P))
    (2.0 * me).sum().backward()
    me_o, gx_o, gth_o = ograd.vjp(proc, P, x0, 2.0 * np.ones(n))
    assert np.abs(me.detach().cpu().numpy() / me_o - 1).max() < 1e-12
    assert _normwise(x.grad.cpu().numpy(), gx_o).max() < 1e-10
    assert abs(theta.grad[0].item() / gth_o[:, 0].sum() - 1) < 1e-10
    assert abs(theta.grad[1].item() / gth_o[:, 1].sum() - 1) < 1e-12


def test_precision_errors(h):
    ev = gpu_events(h, 'ee_mumu', 64, seed=1)
    with pytest.raises(mf.MFError) as ei:      # no colour to contract for e+e- -> mu+mu-
        mf.matrix_element(h, mf.MF_EE_MUMU, ev['p'], mf.MF_FP32_MFMA_F32)
    assert ei.value.status == -2
    with pytest.raises(mf.MFError) as ei:
        mf.matrix_element(h, mf.MF_EE_MUMU, ev['p'], 7)
    assert ei.value.status == -1


def test_oversized_request_rejected_before_launch(h):
    """A request above 2^36 events is refused by the argument check (nothing is launched: the
    buffers named here are far smaller than the request)."""
    import ctypes
    small = torch.empty(64, dtype=torch.float64, device='cuda')
    r = mf.mf_request(mf.MF_GG_TT, 0, (1 << 36) + 1, small.data_ptr(), small.data_ptr(), None, None, None, None)
    arr = (mf.mf_request * 1)(r)
    st = mf.lib().mf_matrix_element(h.h, arr, 1, mf.MF_FP64, ctypes.byref(mf.params()), None)
    assert st == -1 and b'2^36' in mf.lib().mf_last_error()


# ------------------------------------------------------------------ persistent batch, graphs, tuning
def _mixed_requests(h, spec, precision, seed0=200):
    reqs, outs, evs = [], [], []
    for i, (proc, n) in enumerate(spec):
        ev = gpu_events(h, proc, n, seed=seed0 + i)
        out = torch.empty(n, dtype=torch.float64 if precision == mf.MF_FP64 else torch.float32, device='cuda')
        reqs.append(mf.make_request(mf.PROCESS[proc], ev['p'], out))
        outs.append(out)
        evs.append(ev)
    return reqs, outs, evs


@pytest.mark.parametrize('prec', ['fp64', 'fp32_mfma_bf16'])
def test_persistent_batch_nan_event_stays_in_its_request(h, prec):
    """One persistent launch over mixed requests: NaN momenta in the ragged tail of one
    request give NaN there and leave every other result of every request bit-identical."""
    from paper_2211_14056_amd.workloads import mixed_batch
    spec = mixed_batch(12, seed=5, scale=0.004)
    spec[0] = ('gg_ttgg', 1)
    spec[1] = ('gg_tt', 65)
    say('persistent batch nan event', prec, spec)
    P_ = mf.PRECISION[prec]
    reqs, outs, evs = _mixed_requests(h, spec, P_)
    mf.mf_matrix_element(h, reqs, P_, mf.params())
    torch.cuda.synchronize()
    clean = [o.double().cpu().numpy() for o in outs]
    evs[1]['p'][2, :, 64] = float('nan')          # the request's buffers are the events' tensors
    torch.cuda.synchronize()
    mf.mf_matrix_element(h, reqs, P_, mf.params())
    torch.cuda.synchronize()
    got = [o.double().cpu().numpy() for o in outs]
    assert np.isnan(got[1][64])
    assert np.array_equal(got[1][:64], clean[1][:64])
    for i in range(len(spec)):
        if i != 1:
            assert np.array_equal(got[i], clean[i]), (i, spec[i])


@pytest.mark.parametrize('prec', ['fp64', 'fp32', 'fp32_mfma_f32', 'fp32_mfma_bf16'])
def test_persistent_batch_equals_separate_launches(h, prec):
    from paper_2211_14056_amd.workloads import mixed_batch
    spec = mixed_batch(12, seed=5, scale=0.004)
    spec[0] = ('gg_ttgg', 1)
    spec[1] = ('gg_tt', 65)
    say('persistent batch', prec, spec)
    P_ = mf.PRECISION[prec]
    reqs, outs, evs = _mixed_requests(h, spec, P_)
    h.set_launch(batch_persistent=1, batch_waves_per_cu=2)
    mf.mf_matrix_element(h, reqs, P_, mf.params())
    torch.cuda.synchronize()
    a = [o.clone() for o in outs]
    h.set_launch(batch_persistent=0)
    mf.mf_matrix_element(h, reqs, P_, mf.params())
    torch.cuda.synchronize()
    h.set_launch(batch_persistent=1, batch_waves_per_cu=4)
    # same generated body compiled into a different kernel: equal up to the
    # rounding of a different instruction order
    tol = 1e-13 if prec == 'fp64' else 1e-6
    for x, y in zip(a, outs):
        assert float(((x.double() - y.double()).abs() / y.double().abs()).max()) <= tol
    # other tiles of the work queue: the same kernel on the same events, bit for bit
    for t_tt, t_ttg in ((1, 1), (64, 16), (3, 5)):
        h.set_batch_tile(mf.MF_GG_TT, t_tt)
        h.set_batch_tile(mf.MF_GG_TTG, t_ttg)
        for o in outs:
            o.fill_(float('nan'))
        mf.mf_matrix_element(h, reqs, P_, mf.params())
        torch.cuda.synchronize()
        for x, y in zip(a, outs):
            assert torch.equal(x, y), (t_tt, t_ttg)
    h.set_batch_tile(mf.MF_GG_TT, 0)
    h.set_batch_tile(mf.MF_GG_TTG, 0)
    with pytest.raises(mf.MFError):
        h.set_batch_tile(mf.MF_GG_TTGG, 2)
    with pytest.raises(mf.MFError):
        h.set_batch_tile(mf.MF_GG_TT, 65)


def test_mixed_batch_full_size_one_launch(h):
    """The 64-request mixed workload at full size in one persistent launch, sampled against the oracle."""
    from paper_2211_14056_amd.workloads import mixed_batch
    spec = mixed_batch(64, seed=5)
    say('mixed batch full size', sum(n for _, n in spec), 'events')
    reqs, outs, evs = _mixed_requests(h, spec, mf.MF_FP32_MFMA_BF16)
    h.set_launch(batch_persistent=0)
    mf.mf_matrix_element(h, reqs, mf.MF_FP32_MFMA_BF16, mf.params())
    torch.cuda.synchronize()
    sep = [o.clone() for o in outs]
    h.set_launch(batch_persistent=1)
    mf.mf_matrix_element(h, reqs, mf.MF_FP32_MFMA_BF16, mf.params())
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for (proc, n), out, ev, ref in zip(spec, outs, evs, sep):
        assert bool(torch.isfinite(out).all())
        # every event equals the single-request launch (same generated body, other kernel)
        assert float(((out.double() - ref.double()).abs() / ref.double().abs()).max()) <= 1e-6
    for i in rng.choice(len(spec), 6, replace=False):
        proc, n = spec[i]
        idx = torch.tensor(rng.choice(n, min(n, 4), replace=False), device='cuda')
        ref = oracle_me(proc, evs[i]['p'][:, :, idx].cpu().numpy())
        got = outs[i][idx].double().cpu().numpy()
        ok = evs[i]['pass_'][idx].cpu().numpy().astype(bool)
        assert np.abs(got / ref - 1)[ok].max() < 1e-3 if ok.any() else True


def test_graph_replay_equals_eager(h):
    from paper_2211_14056_amd.integrator import VegasIntegrator
    say('graph replay gg_ttg')
    vi = VegasIntegrator('gg_ttg', precision=mf.MF_FP32, n=50_000, batches=2, seed=9, handle=h)
    eager = []
    for _ in range(4):
        vi.enqueue_iteration()
        eager.append((vi.acc.clone(), vi.edges.clone()))
        vi._record()
    vi.reset()
    vi.iterate(1)
    g = vi.capture()
    replayed = [(eager[0][0], eager[0][1])]
    for _ in range(3):
        g.launch()
        torch.cuda.synchronize()
        # unrelated eager work between replays
        junk = torch.randn(1000, device='cuda').sum()
        replayed.append((vi.acc.clone(), vi.edges.clone()))
        vi._record()
    for (a1, e1), (a2, e2) in zip(eager, replayed):
        assert torch.equal(a1, a2) and torch.equal(e1, e2)


def test_graph_vegas_gg_tt_cross_section(h):
    from paper_2211_14056_amd.integrator import VegasIntegrator
    say('graph vegas gg_tt')
    vi = VegasIntegrator('gg_tt', precision=mf.MF_FP64, n=1_000_000, batches=1, seed=2, handle=h)
    vi.iterate(1)
    vi.capture()
    vi.replay(4)
    I, sig, chi2 = vi.estimate()
    ref = closed_forms.gg_tt_sigma(P['sqrt_s'] ** 2, P['m_t'], P['alpha_s']) * closed_forms.GEV2_TO_PB
    say('  sigma', I, '+-', sig, 'closed form', ref)
    assert abs(I - ref) < 3 * sig


def test_vegas_gg_ttgg_fp32_matrix_core_matches_fp64(h):
    """The whole Vegas path for gg -> ttbar gg at the benchmark's scale (three iterations of 4 x 10^6
    events, the grid refined after each) with FP32 amplitudes and BF16x3 matrix-core colour, against the
    FP64 path on the same uniforms.  Per-event differences of about 1e-7 must leave every iteration's
    integral and the refined grid equal to far inside the Monte Carlo error (a cut decision that flips at
    rounding level moves one event, which that margin covers)."""
    from paper_2211_14056_amd.integrator import VegasIntegrator
    res = {}
    for prec in (mf.MF_FP64, mf.MF_FP32_MFMA_BF16):
        say('vegas gg_ttgg, precision', prec)
        vi = VegasIntegrator('gg_ttgg', precision=prec, n=1_000_000, batches=4, seed=9, handle=h)
        per_iter = vi.iterate(3)
        res[prec] = (per_iter, vi.estimate(), vi.edges.clone())
    (it64, (I64, s64, _), e64), (it32, (I32, s32, _), e32) = res[mf.MF_FP64], res[mf.MF_FP32_MFMA_BF16]
    say('  sigma fp64', I64, '+-', s64, ' fp32+mfma', I32, '+-', s32)
    assert I64 > 0 and s64 < 0.05 * I64
    for (a, va), (b, vb) in zip(it64, it32):
        assert abs(a - b) < 0.05 * math.sqrt(va)
        assert abs(vb / va - 1) < 1e-3
    assert abs(I32 - I64) < 0.05 * s64
    assert float((e32 - e64).abs().max()) < 1e-4


def test_autotune_report(h):
    """The sweep report (python -m paper_2211_14056_amd.autotune --report) measures every table and
    leaves the handle on its defaults, so later launches give the same numbers as before it."""
    from paper_2211_14056_amd import autotune
    say('autotune report')
    ev = gpu_events(h, 'gg_ttgg', 300, seed=8)
    before = mf.matrix_element(h, mf.MF_GG_TTGG, ev['p'], mf.MF_FP64)
    text = autotune.report(h, sizes=(1 << 12,))
    for head in ('## Block size', '## Event layout', '## Lanes per event', '## Block size, quark-initiated',
                 '## Persistent mixed batch', '## Tile of the persistent batch'):
        assert head in text
    assert text.count('| gg_tt | fp') == 3 and text.count('| gg_ttg | fp') == 3
    assert text.count('| qq_ttgg | fp') == 2 and text.count(' waves: ') == 6
    after = mf.matrix_element(h, mf.MF_GG_TTGG, ev['p'], mf.MF_FP64)
    torch.cuda.synchronize()
    assert torch.equal(before, after)


def test_autotuner(h, tmp_path, monkeypatch):
    from paper_2211_14056_amd import autotune
    monkeypatch.setenv('MF_TUNE_CACHE', str(tmp_path / 'tune.json'))
    say('autotune')
    t = autotune.sweep_block(h, 'gg_ttg', mf.MF_FP32, 1 << 16)
    assert set(t) == set(autotune.BLOCKS) and all(v > 0 for v in t.values())
    used = autotune.tune(h, procs=('gg_tt',), precisions=(mf.MF_FP32,), n=1 << 16,
                         batch=[('gg_tt', 3000), ('gg_ttg', 2000), ('gg_ttgg', 500)], mode='search')
    # block of gg_tt, the persistent grid, and the tiles of gg_tt and gg_ttg
    assert len(used) == 4 and sum('batch_tile' in k for k in used) == 2
    import json
    c = json.load(open(tmp_path / 'tune.json'))
    assert any('batch' in k for k in c)
    # tuned handle still gives the same numbers as the default one
    ev = gpu_events(h, 'gg_ttg', 1000, seed=3)
    h.set_launch(mf.MF_GG_TTG, mf.MF_FP32, 64)
    a = mf.matrix_element(h, mf.MF_GG_TTG, ev['p'], mf.MF_FP32)
    h.set_launch(mf.MF_GG_TTG, mf.MF_FP32, 0)
    b = mf.matrix_element(h, mf.MF_GG_TTG, ev['p'], mf.MF_FP32)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    h.set_launch(batch_persistent=1, batch_waves_per_cu=4)
    h.set_batch_tile(mf.MF_GG_TT, 0)
    h.set_batch_tile(mf.MF_GG_TTG, 0)
