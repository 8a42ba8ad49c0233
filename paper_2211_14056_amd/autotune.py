"""Launch-configuration autotuner.

The paper shows that the block size chosen for its custom kernels changes
the time of a fixed workload a lot, with a plateau of good choices (sect. 3,
Fig. 3).  Here the same question is answered by measurement on the device at
hand: for each (process, precision) the single-request matrix-element launch
is timed for every candidate block size, and the persistent mixed-batch
launches for every candidate grid (one-wave workgroups per compute unit, 0 =
as many as fit) against one launch per request; the
fastest is installed in the handle (mf_set_launch) and cached in a JSON file
keyed by (GPU architecture, process, precision, batch-size bucket).

Environment: MF_TUNE = off | use | search (default use: apply cached entries,
tune nothing); MF_TUNE_CACHE = path of the cache (default
~/.cache/mfhip/tuning.json).

`python -m paper_2211_14056_amd.autotune --report` prints the measured curves
(events/s against block size, event layout and persistent grid) as markdown.
"""
import json
import math
import os

import torch

from . import (MF_FP64, PRECISION, PROCESS, make_request, mf_matrix_element, mf_phase_space, mf_process_legs,
               params)

BLOCKS = (64, 128, 192, 256)
WAVES_PER_CU = (0, 1, 2, 4)     # 0 = as many as fit


def cache_path():
    return os.environ.get('MF_TUNE_CACHE', os.path.expanduser('~/.cache/mfhip/tuning.json'))


def arch():
    return torch.cuda.get_device_properties(0).gcnArchName.split(':')[0]


def bucket(n):
    return int(2 ** round(math.log2(max(n, 1))))


def _load():
    try:
        return json.load(open(cache_path()))
    except (OSError, ValueError):
        return {}


def _save(c):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + '.tmp'
    json.dump(c, open(tmp, 'w'), indent=1, sort_keys=True)
    os.replace(tmp, path)


def _events(h, pid, n, prm, seed=11):
    return mf_phase_space(h, pid, prm, n, seed=seed)['p']


def _time(fn, reps=3):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float('inf')
    for _ in range(reps):
        a.record()
        fn()
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def sweep_block(h, proc, precision, n, prm=None, blocks=BLOCKS):
    """Time of one launch over n events for each block size: {block: ms}."""
    prm = prm or params()
    pid = PROCESS[proc] if isinstance(proc, str) else proc
    p = _events(h, pid, n, prm)
    out = torch.empty(n, dtype=torch.float64 if precision == MF_FP64 else torch.float32, device=p.device)
    req = [make_request(pid, p, out)]
    res = {}
    for blk in blocks:
        h.set_launch(pid, precision, blk)
        res[blk] = _time(lambda: mf_matrix_element(h, req, precision, prm))
    return res


def sweep_batch(h, requests, precision, prm=None, waves=WAVES_PER_CU):
    """Time of one persistent launch over `requests` [(proc, n)] per grid size, and of per-request launches."""
    prm = prm or params()
    reqs = []
    for i, (proc, n) in enumerate(requests):
        pid = PROCESS[proc] if isinstance(proc, str) else proc
        p = _events(h, pid, n, prm, seed=100 + i)
        out = torch.empty(n, dtype=torch.float64 if precision == MF_FP64 else torch.float32, device=p.device)
        reqs.append(make_request(pid, p, out))
    res = {}
    for wv in waves:
        h.set_launch(batch_waves_per_cu=wv, batch_persistent=1)
        res[f'persistent_{wv}'] = _time(lambda: mf_matrix_element(h, reqs, precision, prm))
    h.set_launch(batch_persistent=0)
    res['per_request'] = _time(lambda: mf_matrix_element(h, reqs, precision, prm))
    h.set_launch(batch_persistent=1)
    return res


def tune(h, procs=('gg_tt', 'gg_ttg'), precisions=(MF_FP64,), n=1 << 18, batch=None, mode=None):
    """Apply cached settings, or measure and cache them (mode 'search').  Returns the settings used."""
    mode = mode or os.environ.get('MF_TUNE', 'use')
    if mode == 'off':
        return {}
    cache = _load()
    used = {}
    for proc in procs:
        for prec in precisions:
            key = f'{arch()}|{proc}|{prec}|{bucket(n)}'
            if key not in cache and mode == 'search':
                t = sweep_block(h, proc, prec, n)
                cache[key] = dict(block=min(t, key=t.get), times_ms=t)
            if key in cache:
                h.set_launch(PROCESS[proc], prec, int(cache[key]['block']))
                used[key] = cache[key]['block']
    if batch:
        for prec in precisions:
            key = f'{arch()}|batch|{prec}|{bucket(sum(n for _, n in batch))}'
            if key not in cache and mode == 'search':
                t = sweep_batch(h, batch, prec)
                best = min(t, key=t.get)
                cache[key] = dict(choice=best, times_ms=t)
            if key in cache:
                c = cache[key]['choice']
                if c == 'per_request':
                    h.set_launch(batch_persistent=0)
                else:
                    h.set_launch(batch_waves_per_cu=int(c.split('_')[1]), batch_persistent=1)
                used[key] = c
    if mode == 'search':
        _save(cache)
    return used


def report(h, sizes=(1 << 16, 1 << 20), precisions=('fp64', 'fp32', 'fp32_mfma_bf16')):
    """Markdown tables of the sweeps on this device; resets the handle to its defaults afterwards."""
    lines = [f'Device: {torch.cuda.get_device_name(0)} ({arch()}); best of 3 launches after one warm-up.', '',
             '## Block size (single-request launch, events/s in millions)', '',
             '| process | precision | events | ' + ' | '.join(f'block {b}' for b in BLOCKS) + ' | best |',
             '|---|---|---|' + '---|' * len(BLOCKS) + '---|']
    for proc in ('gg_tt', 'gg_ttg'):
        for pname in precisions:
            for n in sizes:
                t = sweep_block(h, proc, PRECISION[pname], n)
                best = min(t, key=t.get)
                lines.append(f'| {proc} | {pname} | {n} | ' + ' | '.join(f'{n / t[b] / 1e3:.1f}' for b in BLOCKS)
                             + f' | {best} |')
                h.set_launch(PROCESS[proc], PRECISION[pname], 0)
    n = 1 << 20
    t = sweep_block(h, 'gg_ttgg', MF_FP64, n, blocks=(64, 128, 256))
    h.set_launch(PROCESS['gg_ttgg'], MF_FP64, 0)
    lines += ['', '## Event layout, gg -> ttbar gg in FP64 (events/s in millions)', '',
              '| events | one lane per event | two lanes per event (default) | four lanes per event |',
              '|---|---|---|---|',
              f'| {n} | {n / t[64] / 1e3:.1f} | {n / t[128] / 1e3:.1f} | {n / t[256] / 1e3:.1f} |']
    from .workloads import mixed_batch
    spec = mixed_batch(64, seed=5)
    total = sum(k for _, k in spec)
    lines += ['', f'## Persistent mixed batch: 64 requests, {total} events, fp32_mfma_bf16 (ms per call)', '',
              '| grid | ms | events/s (millions) |', '|---|---|---|']
    t = sweep_batch(h, spec, PRECISION['fp32_mfma_bf16'])
    for k, v in t.items():
        label = 'one launch per request' if k == 'per_request' else \
            f"persistent, {k.split('_')[1]} one-wave blocks per CU" + (' (as many as fit)' if k.endswith('_0') else '')
        lines.append(f'| {label} | {v:.2f} | {total / v / 1e3:.0f} |')
    h.set_launch(batch_waves_per_cu=0, batch_persistent=1)
    return '\n'.join(lines)


if __name__ == '__main__':
    import argparse
    ap = argparse.ArgumentParser(description=__doc__.split('\n')[0])
    ap.add_argument('--report', action='store_true', help='print the measured sweep curves as markdown')
    args = ap.parse_args()
    if args.report:
        from . import Handle
        torch.cuda.init()
        print(report(Handle(0)), flush=True)
