"""Launch-configuration autotuner.

The paper shows that the block size chosen for its custom kernels changes
the time of a fixed workload a lot, with a plateau of good choices (sect. 3,
Fig. 3).  Here the same question is answered by measurement on the device at
hand: for each (process, precision) the single-request matrix-element launch
is timed for every candidate launch shape (block size; for gg -> ttbar gg in
FP64 the event layout, one, two or four lanes per event; for gg -> ttbar ggg
the lanes per event of its one-wavefront-per-event kernel, 16, 32 or 64); the
persistent mixed-batch launch for every candidate grid (one-wave workgroups per
compute unit, 0 = as many as fit) against one launch per request, and for every
candidate tile (64-event waves per work-queue pop, gg -> ttbar and gg -> ttbar g).
The fastest is installed in the handle (mf_set_launch, mf_set_batch_tile) and
cached in a JSON file keyed by (GPU architecture, process, precision, batch-size
bucket).

Environment: MF_TUNE = off | use | search (default use: apply cached entries,
tune nothing); MF_TUNE_CACHE = path of the cache (default
~/.cache/mfhip/tuning.json).

`python -m paper_2211_14056_amd.autotune --report` prints the measured curves
(events/s against block size, event layout, lanes per event, persistent grid and
tile) as markdown.
"""
import json
import math
import os

import torch

from . import (MF_FP64, PRECISION, PROCESS, make_request, mf_matrix_element, mf_phase_space, mf_process_legs,
               params)

BLOCKS = (64, 128, 192, 256)
WAVES_PER_CU = (0, 1, 2, 4)     # 0 = as many as fit
LANES_PER_EVENT = (16, 32, 64)  # gg -> ttbar ggg
TILES = {'gg_tt': (4, 16, 64), 'gg_ttg': (1, 4, 16)}   # 64-event waves per tile of the persistent batch
TTGG_LAYOUTS = (64, 128, 256)   # gg -> ttbar gg in FP64: one, two, four lanes per event


def candidates(proc, precision):
    """Launch shapes mf_set_launch accepts for (process, precision)."""
    if proc == 'gg_ttggg':
        return LANES_PER_EVENT
    if proc == 'gg_ttgg' and precision == MF_FP64:
        return TTGG_LAYOUTS
    return BLOCKS


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


def sweep_block(h, proc, precision, n, prm=None, blocks=None):
    """Time of one launch over n events for each launch shape: {block: ms}."""
    prm = prm or params()
    pid = PROCESS[proc] if isinstance(proc, str) else proc
    if blocks is None:
        name = proc if isinstance(proc, str) else [k for k, v in PROCESS.items() if v == proc][0]
        blocks = candidates(name, precision)
    p = _events(h, pid, n, prm)
    out = torch.empty(n, dtype=torch.float64 if precision == MF_FP64 else torch.float32, device=p.device)
    req = [make_request(pid, p, out)]
    res = {}
    for blk in blocks:
        h.set_launch(pid, precision, blk)
        res[blk] = _time(lambda: mf_matrix_element(h, req, precision, prm))
    h.set_launch(pid, precision, 0)
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


def sweep_tile(h, requests, precision, proc, prm=None, tiles=None):
    """Time of one persistent launch over `requests` for each tile size of process `proc`
    (64-event waves per queue pop), the other processes at their defaults."""
    prm = prm or params()
    pid = PROCESS[proc]
    reqs = []
    for i, (pr, n) in enumerate(requests):
        q = PROCESS[pr] if isinstance(pr, str) else pr
        p = _events(h, q, n, prm, seed=100 + i)
        out = torch.empty(n, dtype=torch.float64 if precision == MF_FP64 else torch.float32, device=p.device)
        reqs.append(make_request(q, p, out))
    h.set_launch(batch_persistent=1)
    res = {}
    for t in tiles or TILES[proc]:
        h.set_batch_tile(pid, t)
        res[t] = _time(lambda: mf_matrix_element(h, reqs, precision, prm))
    h.set_batch_tile(pid, 0)
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
            for proc in TILES:
                if not any(pr == proc for pr, _ in batch):
                    continue
                key = f'{arch()}|batch_tile|{proc}|{prec}|{bucket(sum(n for _, n in batch))}'
                if key not in cache and mode == 'search':
                    t = sweep_tile(h, batch, prec, proc)
                    cache[key] = dict(tile=min(t, key=t.get), times_ms=t)
                if key in cache:
                    h.set_batch_tile(PROCESS[proc], int(cache[key]['tile']))
                    used[key] = cache[key]['tile']
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
    t = sweep_block(h, 'gg_ttgg', MF_FP64, n)
    lines += ['', '## Event layout, gg -> ttbar gg in FP64 (events/s in millions)', '',
              '| events | one lane per event | two lanes per event (default) | four lanes per event |',
              '|---|---|---|---|',
              f'| {n} | {n / t[64] / 1e3:.1f} | {n / t[128] / 1e3:.1f} | {n / t[256] / 1e3:.1f} |']
    n5 = min(max(sizes), 1 << 18)
    lines += ['', '## Lanes per event, gg -> ttbar ggg (events/s in millions)', '',
              '| precision | events | ' + ' | '.join(f'{k} lanes' for k in LANES_PER_EVENT) + ' | best |',
              '|---|---|' + '---|' * len(LANES_PER_EVENT) + '---|']
    for pname in ('fp64', 'fp32'):
        t = sweep_block(h, 'gg_ttggg', PRECISION[pname], n5)
        best = min(t, key=t.get)
        lines.append(f'| {pname} | {n5} | ' + ' | '.join(f'{n5 / t[k] / 1e3:.2f}' for k in LANES_PER_EVENT)
                     + f' | {best} |')
    lines += ['', '## Block size, quark-initiated processes (events/s in millions)', '',
              '| process | precision | events | ' + ' | '.join(f'block {b}' for b in BLOCKS) + ' | best |',
              '|---|---|---|' + '---|' * len(BLOCKS) + '---|']
    nq = max(sizes)
    for proc in ('qq_ttg', 'qq_ttgg', 'qg_ttqg'):
        for pname in ('fp64', 'fp32'):
            t = sweep_block(h, proc, PRECISION[pname], nq)
            best = min(t, key=t.get)
            lines.append(f'| {proc} | {pname} | {nq} | ' + ' | '.join(f'{nq / t[b] / 1e3:.1f}' for b in BLOCKS)
                         + f' | {best} |')
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
    lines += ['', '## Tile of the persistent batch (same 64 requests, ms per call; other processes at their '
              'default tile)', '', '| process | ' + ' | '.join('tile' for _ in range(3)) + ' |', '|---|---|---|---|']
    for proc in TILES:
        t = sweep_tile(h, spec, PRECISION['fp32_mfma_bf16'], proc)
        lines.append(f'| {proc} | ' + ' | '.join(f'{k} waves: {v:.2f}' for k, v in t.items()) + ' |')
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
