"""The benchmark's batch pipeline computes exactly what plain sequential calls compute.

With two streams the phase space of the next batch runs beside the matrix element
of the current one, into a second buffer, and events order the two streams.  A
missing wait, or a phase space enqueued too early, would let a batch read a grid
that is still being refined or momenta of another batch, so results would change.
The reference here is a plain loop of the same calls on one stream, one batch
after the other.  The Vegas reduction is deterministic, so both schedules must
match it bit for bit: on the last batch's momenta and |M|^2, on the accumulators
and on the refined grid, over a run that crosses a grid refinement.
"""
import os
import sys

import numpy as np
import pytest
import torch

import paper_2211_14056_amd as mf

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.fixture(scope='module')
def h():
    if not os.path.exists(mf.LIB_PATH):
        from paper_2211_14056_amd import build as _b
        _b.build()
    torch.cuda.init()
    return mf.Handle(0)


def sequential(h, prm, prec, last, seed):
    """Batches 0..last, each as phase space -> matrix element -> Vegas call, on one stream."""
    pid = mf.PROCESS[bench.PROC]
    d = mf.mf_process_dims(pid)
    n, nb, per_iter = bench.BATCH, bench.NB, bench.BATCHES_PER_ITER
    dev = torch.device('cuda', 0)
    f64 = dict(dtype=torch.float64, device=dev)
    edges = torch.tensor(np.tile(np.linspace(0, 1, nb + 1), (d, 1)), **f64).contiguous()
    acc = torch.zeros(2 + d * nb, **f64)
    p = torch.empty(6, 4, n, **f64)
    w, jac = torch.empty(n, **f64), torch.empty(n, **f64)
    pas = torch.empty(n, dtype=torch.uint8, device=dev)
    bins = torch.empty(d, n, dtype=torch.int16, device=dev)
    me = torch.empty(n, dtype=torch.float64 if prec == mf.MF_FP64 else torch.float32, device=dev)
    for i in range(last + 1):
        mf.mf_phase_space(h, pid, prm, n, seed=seed, offset=i * n, edges=edges, nb=nb, p=p, w=w,
                          pass_=pas, bin_idx=bins, jac=jac)
        mf.mf_matrix_element(h, [mf.make_request(pid, p, me)], prec, prm)
        mf.mf_vegas_refine(h, prm, n, d, nb, 1.5, w, jac, me, pas, bins, acc, edges,
                           update_edges=(i + 1) % per_iter == 0, accumulate=i % per_iter != 0)
    torch.cuda.synchronize()
    return dict(p=p, pas=pas, me=me, acc=acc, edges=edges)


@pytest.mark.parametrize('precision', ['fp32_mfma_bf16', 'fp64'])
def test_pipelined_schedules_match_sequential_calls(h, precision):
    prm = mf.params()
    prec = mf.PRECISION[precision]
    # warmup 1 + 18 timed batches: the grid is refined after batch 15 and batches
    # 16..18 start the next Vegas iteration on the refined grid
    steps, warmup = 18, 1
    print(f'[gpu-test] bench schedule {precision}: sequential reference', flush=True)
    ref = sequential(h, prm, prec, warmup + steps - 1, seed=7)
    for streams in (1, 2, 3):
        print(f'[gpu-test] bench schedule {precision}: streams {streams}', flush=True)
        got = bench.run_path(mf, h, prm, prec, steps, warmup, seed=7, streams=streams)
        torch.cuda.synchronize()
        for key in ('p', 'pas', 'me', 'acc', 'edges'):
            assert torch.equal(got[key], ref[key]), (streams, key)
    assert int(ref['pas'].sum()) > 0
