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
"""
import json
import math
import os

import torch

from . import (MF_FP64, PROCESS, make_request, mf_matrix_element, mf_phase_space, mf_process_legs, params)

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
