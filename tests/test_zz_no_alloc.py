"""The allocation-free Vegas entry point against the handle-based one, through the C ABI.

mf_vegas_refine_noalloc keeps its block partials in the library's static device array
instead of a handle's workspace.  On the same inputs it must give the same sums, refined
grid, per-event F and counter advance as mf_vegas_refine, bit for bit: two calls in a row,
the second smaller than the first (so it reads only cells it wrote itself), each followed by
an accumulating call.
"""
import sys

import numpy as np
import pytest
import torch

import paper_2211_14056_amd as mf
from oracle import processes, vegas as ovegas

pytestmark = pytest.mark.gpu


def say(*a):
    print('[gpu-test]', *a, flush=True)
    sys.stdout.flush()


def _batch(h, proc, n, seed, edges):
    pid = mf.PROCESS[proc]
    d = processes.dims(proc)
    dev = torch.device('cuda', 0)
    ev = mf.mf_phase_space(h, pid, mf.params(), n, seed=seed, edges=edges, nb=50,
                           pass_=torch.empty(n, dtype=torch.uint8, device=dev),
                           bin_idx=torch.empty(d, n, dtype=torch.int16, device=dev),
                           jac=torch.empty(n, dtype=torch.float64, device=dev))
    ev['me'] = mf.matrix_element(h, pid, ev['p'], mf.MF_FP32_MFMA_BF16, mf.params())
    return ev


def _run(fn, h, ev, n, d, edges0, acc0, counter0, accumulate):
    edges, acc, counter = edges0.clone(), acc0.clone(), counter0.clone()
    F = torch.full((n,), -1.0, dtype=torch.float64, device=edges.device)
    args = (mf.params(), n, d, 50, 1.5, ev['w'], ev['jac'], ev['me'], ev['pass_'], ev['bin_idx'], acc, edges)
    kw = dict(F=F, update_edges=True, accumulate=accumulate, rng_counter=counter)
    if fn == 'noalloc':
        mf.mf_vegas_refine_noalloc(*args, **kw)
    else:
        mf.mf_vegas_refine(h, *args, **kw)
    torch.cuda.synchronize()
    return acc, edges, F, counter


def test_noalloc_vegas_equals_handle_vegas_on_two_calls():
    torch.cuda.init()
    h = mf.Handle(0)
    try:
        proc, d = 'gg_ttg', processes.dims('gg_ttg')
        dev = torch.device('cuda', 0)
        rng = np.random.default_rng(7)
        w_ = rng.uniform(0.5, 1.5, (d, 50))
        e0 = np.concatenate([np.zeros((d, 1)), np.cumsum(w_, 1) / w_.sum(1, keepdims=True)], 1)
        e0[:, -1] = 1.0
        edges0 = torch.tensor(e0, dtype=torch.float64, device=dev).contiguous()
        for n, seed in ((700_003, 11), (2_049, 12)):       # second call smaller: fewer blocks
            say('noalloc vegas', proc, n)
            ev = _batch(h, proc, n, seed, edges0)
            acc0 = torch.tensor(np.arange(2 + d * 50, dtype=np.float64), device=dev)
            counter0 = torch.tensor([5], dtype=torch.int64, device=dev)
            for accumulate in (False, True):
                ref = _run('handle', h, ev, n, d, edges0, acc0, counter0, accumulate)
                got = _run('noalloc', h, ev, n, d, edges0, acc0, counter0, accumulate)
                for name, a, b in zip(('acc', 'edges', 'F', 'counter'), ref, got):
                    assert torch.equal(a, b), (n, accumulate, name)
                assert int(got[3].item()) == 5 + n
                assert torch.isfinite(got[0]).all() and (torch.diff(got[1], dim=1) >= 0).all()
        # the sums are the oracle's accumulation of the same F (the last call)
        F = got[2].cpu().numpy()
        sf, sf2, hist = ovegas.accumulate(F, ev['bin_idx'].cpu().numpy().astype(np.int64), 50)
        a = got[0].cpu().numpy() - acc0.cpu().numpy()
        assert abs(a[0] / sf - 1) < 1e-12 and abs(a[1] / sf2 - 1) < 1e-12
        assert np.abs(a[2:].reshape(d, 50) - hist).max() <= 1e-12 * hist.max()
    finally:
        h.close()
