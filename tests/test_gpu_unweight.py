"""GPU unweighting (mf_unweight) against the oracle's hit-or-miss acceptance.

Integer and index work, so the bar is bit-exact: the kept indices (in increasing
order), their weight factors, the count and the reference maximum equal the
oracle's on the same seeded synthetic weights, with the acceptance decision
u * w_max < w taken in FP64 on both sides.  Covered: batch maximum and a given
maximum below it (overweight events), non-positive and NaN weights, a capacity
below the count (truncation with the full count reported), momenta gathered for
the kept events, empty and one-event batches, several block sizes' ragged tails,
and a full-size batch (2^24 + 5 events).  The weights come from numpy's seeded
generator, never from the GPU path.
"""
import sys

import numpy as np
import pytest
import torch

import paper_2211_14056_amd as mf
from oracle import unweight as ouw

pytestmark = pytest.mark.gpu


def say(*a):
    print('[gpu-test]', *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope='module')
def h():
    torch.cuda.init()
    return mf.Handle(0)


def _weights(n, seed):
    rng = np.random.default_rng(seed)
    w = rng.lognormal(0.0, 1.5, n)
    if n >= 10:
        w[rng.choice(n, n // 10, replace=False)] = 0.0            # events outside the cuts
        w[rng.choice(n, max(1, n // 100), replace=False)] = -1.0  # a negative weight
        w[rng.choice(n, max(1, n // 1000), replace=False)] = np.nan
    return w


def _gpu(h, w, w_max, seed, offset, cap=None, p=None):
    dev = torch.device('cuda', 0)
    wt = torch.tensor(w, dtype=torch.float64, device=dev)
    pt = None if p is None else torch.tensor(p, dtype=torch.float64, device=dev).contiguous()
    out = mf.mf_unweight(h, len(w), wt, w_max=w_max, seed=seed, offset=offset, p=pt, cap=cap)
    torch.cuda.synchronize()
    c = int(out['count'].item())
    k = min(c, len(w) if cap is None else cap)
    res = dict(count=c, idx=out['idx'][:k].cpu().numpy(), fac=out['fac'][:k].cpu().numpy(),
               w_max=float(out['w_max'].item()))
    if p is not None:
        res['p_out'] = out['p_out'][:, :, :k].cpu().numpy()
    return res


def _oracle(w, w_max, seed, offset):
    u = ouw.acceptance_uniforms(seed, len(w), offset)
    wm = w_max if w_max > 0 else ouw.batch_max(w)
    kept, fac = ouw.unweight(w, u, wm)
    return kept, fac, wm


@pytest.mark.parametrize('n', [1, 255, 256, 257, 100_003])
def test_unweight_bit_exact_vs_oracle(h, n):
    w = _weights(n, seed=n)
    for w_max in (0.0, 3.0):
        say('unweight', n, 'w_max', w_max)
        g = _gpu(h, w, w_max, seed=11, offset=1000)
        kept, fac, wm = _oracle(w, w_max, seed=11, offset=1000)
        assert g['w_max'] == wm
        assert g['count'] == kept.size
        assert np.array_equal(g['idx'], kept)
        assert np.array_equal(g['fac'], fac)


def test_unweight_truncation_and_momenta(h):
    n, n_ext = 70_001, 5
    w = _weights(n, seed=5)
    p = np.random.default_rng(6).normal(size=(n_ext, 4, n))
    kept, fac, wm = _oracle(w, 0.0, seed=2, offset=0)
    cap = kept.size // 2
    say('unweight truncation', n, 'cap', cap)
    g = _gpu(h, w, 0.0, seed=2, offset=0, cap=cap, p=p)
    assert g['count'] == kept.size
    assert np.array_equal(g['idx'], kept[:cap]) and np.array_equal(g['fac'], fac[:cap])
    assert np.array_equal(g['p_out'], p[:, :, kept[:cap]])
    g = _gpu(h, w, 0.0, seed=2, offset=0, p=p)
    assert np.array_equal(g['p_out'], p[:, :, kept])


def test_unweight_empty_and_degenerate(h):
    dev = torch.device('cuda', 0)
    out = mf.mf_unweight(h, 0, torch.empty(0, dtype=torch.float64, device=dev))
    torch.cuda.synchronize()
    assert int(out['count'].item()) == 0
    g = _gpu(h, np.zeros(1000), 0.0, seed=1, offset=0)              # nothing positive
    assert g['count'] == 0 and g['w_max'] == 0.0
    g = _gpu(h, np.full(1000, 2.0), 0.0, seed=1, offset=0)          # equal weights: all kept
    assert g['count'] == 1000 and np.array_equal(g['idx'], np.arange(1000))


def test_unweight_full_size(h):
    n = (1 << 24) + 5
    w = _weights(n, seed=77)
    say('unweight full size', n)
    g = _gpu(h, w, 0.0, seed=3, offset=5)
    kept, fac, wm = _oracle(w, 0.0, seed=3, offset=5)
    assert g['count'] == kept.size and g['w_max'] == wm
    assert np.array_equal(g['idx'], kept) and np.array_equal(g['fac'], fac)


def test_unweight_gg_ttg_events_end_to_end(h):
    """Phase space -> matrix element -> integrand -> unweighting on 10^6 gg -> ttbar g events:
    the kept momenta are the momenta of the kept events, every kept event has F > 0, and
    the number kept agrees with the expected sum of min(F / F_max, 1) within 5 binomial sigma."""
    proc, n = 'gg_ttg', 1_000_000
    pid = mf.PROCESS[proc]
    d = mf.mf_process_dims(pid)
    dev = torch.device('cuda', 0)
    prm = mf.params()
    say('unweight end to end', proc, n)
    ev = mf.mf_phase_space(h, pid, prm, n, seed=21, pass_=torch.empty(n, dtype=torch.uint8, device=dev),
                           bin_idx=torch.empty(d, n, dtype=torch.int16, device=dev),
                           jac=torch.empty(n, dtype=torch.float64, device=dev))
    me = mf.matrix_element(h, pid, ev['p'], mf.MF_FP32_MFMA_BF16, prm)
    F = torch.empty(n, dtype=torch.float64, device=dev)
    acc = torch.empty(2 + d * 50, dtype=torch.float64, device=dev)
    edges = torch.tensor(np.tile(np.linspace(0, 1, 51), (d, 1)), dtype=torch.float64, device=dev).contiguous()
    mf.mf_vegas_refine(h, prm, n, d, 50, 1.5, ev['w'], ev['jac'], me, ev['pass_'], ev['bin_idx'], acc, edges, F=F,
                       update_edges=False)
    out = mf.mf_unweight(h, n, F, seed=4, p=ev['p'])
    torch.cuda.synchronize()
    c = int(out['count'].item())
    idx = out['idx'][:c]
    assert torch.equal(out['p_out'][:, :, :c], ev['p'][:, :, idx])
    assert bool((F[idx] > 0).all())
    fm = float(out['w_max'].item())
    assert fm == float(F.max())
    prob = torch.clamp(F / fm, 0, 1).cpu().numpy()
    mean, var = prob.sum(), (prob * (1 - prob)).sum()
    say('  kept', c, 'expected', mean)
    assert abs(c - mean) < 5 * np.sqrt(var)


def test_event_file_round_trip(h, tmp_path):
    """The text writer puts every kept event, in order, with its momenta to full precision."""
    from paper_2211_14056_amd.events import write_events
    n, n_ext = 5000, 4
    w = _weights(n, seed=8)
    p = np.random.default_rng(9).normal(size=(n_ext, 4, n))
    dev = torch.device('cuda', 0)
    out = mf.mf_unweight(h, n, torch.tensor(w, dtype=torch.float64, device=dev), seed=5,
                         p=torch.tensor(p, dtype=torch.float64, device=dev).contiguous())
    torch.cuda.synchronize()
    path = tmp_path / 'events.txt'
    k = write_events(str(path), 'gg_tt', out, unit_weight_pb=1.0)
    kept, fac, wm = _oracle(w, 0.0, seed=5, offset=0)
    assert k == kept.size
    lines = path.read_text().splitlines()
    assert lines[0].startswith('# process gg_tt events %d' % k)
    body = lines[1:]
    assert len(body) == k * (1 + n_ext)
    for j in range(0, k, max(1, k // 50)):
        head = body[j * (1 + n_ext)].split()
        assert int(head[0]) == kept[j] and float(head[3]) == fac[j]
        for leg in range(n_ext):
            vals = np.array([float(v) for v in body[j * (1 + n_ext) + 1 + leg].split()])
            assert np.array_equal(vals, p[leg, :, kept[j]])
