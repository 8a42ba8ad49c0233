"""Benchmark: gg -> t tbar g g matrix-element events/s on one MI355X.

One step = one batch of 1e6 synthetic events through the whole forward hot
path: Philox uniforms -> Vegas map -> RAMBO-on-diet phase space + cuts ->
matrix element -> Vegas accumulation (the grid is refined after every 16th
batch, i.e. once per 16e6-event Vegas iteration).  The headline precision is
FP32 amplitudes with the colour contraction on matrix cores; the plain FP64
path is measured on the same batches and reported beside it, with the
per-event relative difference of the FP32 result from the FP64 one (the FP64
path matches the FP64 CPU oracle to 1e-12 in the parity tests).

By default the batches are pipelined over two HIP streams: the phase space of
batch i+1 runs beside the matrix element of batch i (`--streams 1` serialises
them; `--streams 3` also moves the Vegas calls to a third stream, which measured
no faster).  The matrix elements stay on one stream, one at a time, so the HIP
events around each matrix-element launch time that kernel alone; the roofline
figures come from those launch durations, the headline from the wall clock of
the steps.

The run publishes no throughput (exit status 3) unless the FP32 results meet their bars
(median 1e-5, max 1e-3 relative, no NaN) against FP64 on every event of the last batch that
passes the cuts and against the FP64 CPU oracle on the cpu_baseline sample, and FP64 meets
1e-12 against the oracle there.

Beside the headline the JSON line carries `extras`: the derivative (VJP) on the
gg -> ttbar g configuration (4e6 events, FP32 and FP64) and on gg -> ttbar gg
(2^18 events), the 64-request mixed batch (one persistent launch per process class
against one launch per request), the whole mixed Vegas iteration with the
derivative of its gg -> ttbar gg share, replayed as one library graph, and hadronic
gg -> ttbar gg events (parton densities from a toy grid, pp at 13 TeV).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32_mfma_f32] [--no-extras] [--streams 1|2|3]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = 'matrix-element events/sec, gg->ttbar gg, FP32-MFMA vs FP64, at stated rel. error'
PEAK = {'f64': 78.6e12, 'f32': 157.3e12}      # MI355X vector peaks (published), FLOP/s
PROC = 'gg_ttgg'
BATCH = 1_000_000
BATCHES_PER_ITER = 16
NB = 50
COPY_BYTES = 512 << 20


# sources of the two timed matrix-element kernels (the matrix-core-colour kernel
# and the FP64 kernel, two lanes per event), generated process code included
ME_SOURCES = ('me_kernels.hip', 'me_mfma.hip', 'me_mfma_colour.h', 'me_common.h', 'dual.h', 'internal.h',
              'me_ttgg_pair.hip', 'generated/me_gg_tt.inc', 'generated/me_gg_ttg.inc',
              'generated/me_gg_ttgg.inc', 'generated/me_gg_ttgg_pair.inc')


def source_hash():
    """Hash of the sources the timed matrix-element kernels are compiled from."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, 'paper_2211_14056_amd', 'csrc')
    for f in ME_SOURCES:
        h.update(f.encode())
        h.update(open(os.path.join(csrc, f), 'rb').read())
    return h.hexdigest()[:16]


def measured_traffic(precision_name):
    """HBM bytes per matrix-element launch from the committed counter summary, or None
    when the kernels have changed since the counters were taken."""
    path = os.path.join(ROOT, 'profiles', 'me_gg_ttgg_hbm_traffic.md')
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith('- ') and ':' in line:
            k, v = line[2:].split(':', 1)
            vals[k.strip()] = v.strip().strip('`')
    if vals.get('source-hash') != source_hash():
        return None
    v = vals.get(f'traffic-bytes-per-launch {precision_name}')
    return float(v) if v else None


def flops_per_event(proc, precision_name):
    """Flops per event of the form the kernel of that precision executes (generated-code
    count of the recursion and the colour form, FMA = 2)."""
    import ast
    key = {'fp64': 'per_event_f64', 'fp32': 'per_event_f32_valu'}.get(precision_name, 'per_event_f32')
    path = os.path.join(ROOT, 'paper_2211_14056_amd', 'csrc', 'generated', 'flops.txt')
    for line in open(path):
        name, rest = line.split(' ', 1)
        if name == proc:
            return ast.literal_eval(rest)[key]
    raise KeyError(proc)


def enqueue_order(first, count, streams):
    """[(op, batch)] in the order the batches first..first+count-1 are enqueued.

    op 'ps' is the phase space of the batch, 'me' its matrix element and 'vg' its
    Vegas call.  With two buffers (streams >= 2) the phase space of i+1 is enqueued
    before the matrix element of i, except where i+1 opens a Vegas iteration: its
    phase space needs the grid that batch i's refine writes, so it comes after that
    refine.  With one buffer it always comes after batch i, which still reads it."""
    order = [('ps', first)]
    for k in range(count):
        i = first + k
        nxt = k + 1 < count
        if nxt and streams > 1 and (i + 1) % BATCHES_PER_ITER != 0:
            order.append(('ps', i + 1))
            nxt = False
        order += [('me', i), ('vg', i)]
        if nxt:
            order.append(('ps', i + 1))
    return order


def run_path(mf, h, prm, precision, steps, warmup, seed, streams=2):
    """Time `steps` batches of the full forward path; returns timings and the last batch's ME.

    streams >= 2: the phase space of batch i+1 runs on a second HIP stream, into the second
    of two event buffers, while the matrix element of batch i runs.  Its waves take the
    compute units that batch i's last matrix-element waves leave idle: 1e6 events are 15.3
    waves per SIMD.  streams = 3: the Vegas calls run on a third stream, so the matrix
    element of batch i+1 need not wait for the Vegas call of batch i.  The matrix elements
    stay on one stream, in batch order, so no two matrix-element launches overlap and each
    launch's HIP events time that kernel alone; the Vegas calls, too, stay in batch order
    on one stream.  Events order the streams:
      * a matrix element starts only when its phase space is done;
      * a Vegas call starts only when its matrix element is done;
      * a buffer is refilled only after the Vegas call that last read it (and so after
        its matrix element), so a later matrix element cannot overwrite a result that
        is still to be read;
      * the first batch of a Vegas iteration waits for the grid refined by the previous one.
    streams = 1: everything on one stream.
    """
    pid = mf.PROCESS[PROC]
    d = mf.mf_process_dims(pid)
    dev = torch.device('cuda', 0)
    f64 = dict(dtype=torch.float64, device=dev)
    edges = torch.tensor(np.tile(np.linspace(0, 1, NB + 1), (d, 1)), **f64).contiguous()
    acc = torch.zeros(2 + d * NB, **f64)
    nbuf = 1 if streams == 1 else 2
    bufs = []
    for _ in range(nbuf):
        b = dict(p=torch.empty(6, 4, BATCH, **f64), w=torch.empty(BATCH, **f64), jac=torch.empty(BATCH, **f64),
                 pas=torch.empty(BATCH, dtype=torch.uint8, device=dev),
                 bins=torch.empty(d, BATCH, dtype=torch.int16, device=dev),
                 me=torch.empty(BATCH, dtype=torch.float64 if precision == mf.MF_FP64 else torch.float32,
                                device=dev))
        b['req'] = [mf.make_request(pid, b['p'], b['me'])]
        b['ready'] = torch.cuda.Event()       # recorded after the phase space that filled it
        b['computed'] = torch.cuda.Event()    # recorded after the matrix element that filled `me`
        b['free'] = torch.cuda.Event()        # recorded after the Vegas call that read the buffer
        bufs.append(b)
    main = torch.cuda.Stream()                # default priority (all three)
    side = torch.cuda.Stream() if streams >= 2 else main
    vstream = torch.cuda.Stream() if streams == 3 else main
    grid_done = torch.cuda.Event()
    # HIP events around every matrix-element launch of the timed region, recorded on
    # the stream the library launches it on; read after the end
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]

    def phase_space(i):
        b = bufs[i % nbuf]
        with torch.cuda.stream(side):
            side.wait_event(b['free'])
            if i % BATCHES_PER_ITER == 0:
                side.wait_event(grid_done)
            mf.mf_phase_space(h, pid, prm, BATCH, seed=seed, offset=i * BATCH, edges=edges, nb=NB, p=b['p'],
                              w=b['w'], pass_=b['pas'], bin_idx=b['bins'], jac=b['jac'])
            b['ready'].record(side)

    def matrix_element(i, ev=None):
        b = bufs[i % nbuf]
        with torch.cuda.stream(main):
            main.wait_event(b['ready'])
            if ev:
                ev[0].record(main)
            mf.mf_matrix_element(h, b['req'], precision, prm)
            if ev:
                ev[1].record(main)
            b['computed'].record(main)

    def vegas(i):
        b = bufs[i % nbuf]
        with torch.cuda.stream(vstream):
            vstream.wait_event(b['computed'])
            last = (i + 1) % BATCHES_PER_ITER == 0
            mf.mf_vegas_refine(h, prm, BATCH, d, NB, 1.5, b['w'], b['jac'], b['me'], b['pas'], b['bins'], acc,
                               edges, update_edges=last, accumulate=(i % BATCHES_PER_ITER) != 0)
            b['free'].record(vstream)
            if last:
                grid_done.record(vstream)

    def run(first, count, timed):
        for op, i in enqueue_order(first, count, streams):
            if op == 'ps':
                phase_space(i)
            elif op == 'me':
                matrix_element(i, evs[i - first] if timed else None)
            else:
                vegas(i)

    torch.cuda.synchronize()
    if warmup:
        run(0, warmup, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(warmup, steps, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    me_ms = [a.elapsed_time(b) for a, b in evs]
    lb = bufs[(warmup + steps - 1) % nbuf]
    return dict(seconds=t1 - t0, me_ms=float(np.mean(me_ms)), me=lb['me'], pas=lb['pas'], p=lb['p'], acc=acc,
                edges=edges)


def _best_ms(fn, reps=3):
    """Best of `reps` timed calls (HIP events on the current stream) after one warm-up call."""
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


def extras(mf, h, prm, seed):
    """The other rows of the path, timed beside the headline: the derivative on the
    gg -> ttbar g configuration (4e6 events) and on gg -> ttbar gg, the 64-request mixed
    batch in one persistent launch against one launch per request, hadronic events,
    gg -> ttbar ggg in its three layouts, the quark-initiated processes, and the mixed
    iteration as one graph."""
    from paper_2211_14056_amd.workloads import mixed_batch
    dev = torch.device('cuda', 0)
    f64 = dict(dtype=torch.float64, device=dev)
    out = {}
    pid, n = mf.MF_GG_TTG, 4_000_000
    d = mf.mf_process_dims(pid)
    x = torch.empty(d, n, **f64)
    mf.mf_phase_space(h, pid, prm, n, seed=seed, x_out=x)
    gx, gth = torch.empty(d, n, **f64), torch.empty(n, 2, **f64)
    gb = torch.ones(n, **f64)
    vjp = {}
    for name, prec in (('fp32', mf.MF_FP32), ('fp64', mf.MF_FP64)):
        me = torch.empty(n, dtype=torch.float32 if prec == mf.MF_FP32 else torch.float64, device=dev)
        req = mf.make_request(pid, None, me, x=x, grad_me=gb, grad_x=gx, grad_theta=gth, n=n)
        fwd = mf.make_request(pid, mf.mf_phase_space(h, pid, prm, n, seed=seed)['p'], me)
        t = _best_ms(lambda: mf.mf_matrix_element_vjp(h, [req], prec, prm))
        tf = _best_ms(lambda: mf.mf_matrix_element(h, [fwd], prec, prm))
        vjp[name] = {'ms': t, 'events_per_s': n / t * 1e3, 'forward_ms': tf, 'vjp_over_forward': t / tf}
    out['vjp_gg_ttg'] = {'events': n, 'inputs_per_event': d + 2, **vjp}
    del x, gx, gth, gb
    # the derivative on gg -> ttbar gg (the mixed batch's share), 2^18 events
    pid, n = mf.MF_GG_TTGG, 1 << 18
    d = mf.mf_process_dims(pid)
    x = torch.empty(d, n, **f64)
    ev = mf.mf_phase_space(h, pid, prm, n, seed=seed, x_out=x)
    gx, gth, gb = torch.empty(d, n, **f64), torch.empty(n, 2, **f64), torch.ones(n, **f64)
    vjp = {}
    for name, prec in (('fp32', mf.MF_FP32), ('fp64', mf.MF_FP64)):
        me = torch.empty(n, dtype=torch.float32 if prec == mf.MF_FP32 else torch.float64, device=dev)
        req = mf.make_request(pid, None, me, x=x, grad_me=gb, grad_x=gx, grad_theta=gth, n=n)
        fwd = mf.make_request(pid, ev['p'], me)
        fprec = mf.MF_FP32_MFMA_BF16 if prec == mf.MF_FP32 else prec
        t = _best_ms(lambda: mf.mf_matrix_element_vjp(h, [req], prec, prm))
        tf = _best_ms(lambda: mf.mf_matrix_element(h, [fwd], fprec, prm))
        vjp[name] = {'ms': t, 'events_per_s': n / t * 1e3, 'forward_ms': tf, 'vjp_over_forward': t / tf,
                     'forward_precision': [k for k, v in mf.PRECISION.items() if v == fprec][0]}
    out['vjp_gg_ttgg'] = {'events': n, 'inputs_per_event': d + 2, **vjp}
    del x, gx, gth, gb, ev
    spec = mixed_batch(64, seed=5)
    reqs, keep = [], []
    prec = mf.MF_FP32_MFMA_BF16
    for i, (proc, m) in enumerate(spec):
        q = mf.PROCESS[proc]
        p = mf.mf_phase_space(h, q, prm, m, seed=seed + 100 + i)['p']
        o = torch.empty(m, dtype=torch.float32, device=dev)
        keep += [p, o]
        reqs.append(mf.make_request(q, p, o))
    total = sum(m for _, m in spec)
    h.set_launch(batch_persistent=1)
    tp = _best_ms(lambda: mf.mf_matrix_element(h, reqs, prec, prm))
    h.set_launch(batch_persistent=0)
    ts = _best_ms(lambda: mf.mf_matrix_element(h, reqs, prec, prm))
    h.set_launch(batch_persistent=1)
    out['mixed_batch'] = {'requests': len(spec), 'events': total, 'precision': 'fp32_mfma_bf16',
                          'persistent_ms': tp, 'per_request_ms': ts, 'events_per_s': total / tp * 1e3}
    del reqs, keep
    # hadronic gg -> ttbar gg events (toy gluon density grid, pp at 13 TeV): density
    # interpolation + phase space, matrix element, Vegas step, 1e6 events
    from paper_2211_14056_amd.workloads import toy_pdf_grid
    grid = mf.PdfGrid(*toy_pdf_grid())
    pid, n = mf.MF_GG_TTGG, 1_000_000
    d = mf.mf_process_dims(pid) + 2
    sqS = 13000.0
    bufs = dict(p=torch.empty(6, 4, n, **f64), w=torch.empty(n, **f64), jac=torch.empty(n, **f64),
                pas=torch.empty(n, dtype=torch.uint8, device=dev), bins=torch.empty(d, n, dtype=torch.int16, device=dev),
                me=torch.empty(n, dtype=torch.float32, device=dev))
    ed = torch.tensor(np.tile(np.linspace(0, 1, NB + 1), (d, 1)), **f64).contiguous()
    acc = torch.zeros(2 + d * NB, **f64)
    vprm = mf.params(sqrt_s=sqS)
    req = [mf.make_request(pid, bufs['p'], bufs['me'])]

    def ps_pp():
        mf.mf_phase_space_pp(h, pid, prm, sqS, grid, n, seed=seed, edges=ed, nb=NB, p=bufs['p'], w=bufs['w'],
                             pass_=bufs['pas'], bin_idx=bufs['bins'], jac=bufs['jac'])

    def path_pp():
        ps_pp()
        mf.mf_matrix_element(h, req, mf.MF_FP32_MFMA_BF16, prm)
        mf.mf_vegas_refine(h, vprm, n, d, NB, 1.5, bufs['w'], bufs['jac'], bufs['me'], bufs['pas'], bufs['bins'],
                           acc, ed, update_edges=False)
    t_ps = _best_ms(ps_pp)
    t_all = _best_ms(path_pp)
    out['hadronic_gg_ttgg'] = {'events': n, 'sqrt_S_GeV': sqS, 'pdf': 'toy gluon grid 121 x 61 (ln x, ln Q^2)',
                               'precision': 'fp32_mfma_bf16', 'phase_space_and_pdf_ms': t_ps, 'path_ms': t_all,
                               'events_per_s': n / t_all * 1e3}
    del bufs, req
    # gg -> ttbar ggg: the table-driven recursion, one wavefront per event; 2^18 events per
    # launch for each precision and lanes-per-event layout
    pid, n = mf.MF_GG_TTGGG, 1 << 18
    p = mf.mf_phase_space(h, pid, prm, n, seed=seed)['p']
    layouts = {}
    for name, bprec in (('fp64', mf.MF_FP64), ('fp32', mf.MF_FP32)):
        fl = flops_per_event('gg_ttggg', name)
        me = torch.empty(n, dtype=torch.float64 if bprec == mf.MF_FP64 else torch.float32, device=dev)
        req = [mf.make_request(pid, p, me)]
        for lpe in (16, 32, 64):
            h.set_launch(proc=pid, precision=bprec, block=lpe)
            t = _best_ms(lambda: mf.mf_matrix_element(h, req, bprec, prm))
            layouts[f'{name}_lanes{lpe}'] = {'ms': t, 'events_per_s': n / t * 1e3, 'tflops': n * fl / t * 1e-9}
        h.set_launch(proc=pid, precision=bprec, block=0)
    out['me_gg_ttggg'] = {'events': n, 'flops_per_event': fl, 'layouts': layouts}
    del p, me, req
    # the quark-initiated processes (generated diagram code, one lane per event), 10^6 events
    quark = {}
    for name in ('qq_tt', 'qq_ttg', 'qq_ttgg', 'qg_ttq', 'qg_ttqg'):
        pid, n = mf.PROCESS[name], 1_000_000
        p = mf.mf_phase_space(h, pid, prm, n, seed=seed)['p']
        row = {}
        for pname, bprec in (('fp64', mf.MF_FP64), ('fp32', mf.MF_FP32)):
            fl = flops_per_event(name, pname)
            me = torch.empty(n, dtype=torch.float64 if bprec == mf.MF_FP64 else torch.float32, device=dev)
            req = [mf.make_request(pid, p, me)]
            t = _best_ms(lambda: mf.mf_matrix_element(h, req, bprec, prm))
            row[pname] = {'ms': t, 'events_per_s': n / t * 1e3, 'tflops': n * fl / t * 1e-9}
        quark[name] = {'events': n, 'flops_per_event': flops_per_event(name, 'fp64'), **row}
        del p, me, req
    out['me_quark_processes'] = quark
    # the whole mixed iteration (phase space, matrix elements, derivative of the gg -> ttbar gg
    # share, Vegas per request) as one library graph
    from paper_2211_14056_amd.mixed import MixedIteration
    it = MixedIteration(spec, precision=prec, handle=h)
    it.enqueue()
    it.capture()
    tg = _best_ms(it.launch)
    share = sum(r['n'] for r in it.reqs if 'x' in r)
    out['mixed_iteration_graph'] = {'requests': len(spec), 'events': total, 'vjp_events': share,
                                    'precision': 'fp32_mfma_bf16', 'ms': tg, 'events_per_s': total / tg * 1e3}
    it.graph.close()
    return out


def _cpu_model():
    try:
        for line in open('/proc/cpuinfo'):
            if line.startswith('model name'):
                return line.split(':', 1)[1].strip()
    except OSError:
        pass
    return 'unknown'


def _host_threads():
    """Threads the host share allows: the affinity mask, capped by OMP_NUM_THREADS when set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, 'sched_getaffinity') else (os.cpu_count() or 1)
    try:
        n = min(n, int(os.environ.get('OMP_NUM_THREADS', n)))
    except ValueError:
        pass
    return max(1, n)


def _oracle_pass(proc, par, x, edges):
    """One pass of the oracle over the uniforms x [d][n]: Vegas map, phase space, cuts,
    colour-ordered FP64 |M|^2, Vegas accumulation.  Returns (seconds, |M|^2, pass mask)."""
    from oracle import integrand, vegas as ovegas
    t0 = time.perf_counter()
    y, b, J = ovegas.vegas_map(x, edges)
    F, ok, me = integrand.integrand(proc, par, y)
    ovegas.accumulate(F * J, b, NB)
    return time.perf_counter() - t0, me, ok


def cpu_baseline(seed, run_s=7.0):
    """The FP64 oracle (colour-ordered mode) on the host cores, on bounded samples.

    gg -> ttbar gg: a warm-up pass, a pass of 2048 events that sizes the sample (about
    run_s seconds, at most 2e4 events), then the median of three timed passes with all
    threads of the host share, and one pass with a single thread on a sample sized the same
    way; gg -> ttbar and gg -> ttbar g: one pass each with all
    threads.  Every pass covers uniforms -> Vegas map -> phase space -> cuts -> |M|^2 ->
    Vegas accumulation.  Returns the record and the first timed sample's (x, |M|^2, pass)
    for the direct comparison of the GPU kernels with the oracle."""
    from oracle import philox, processes, vegas as ovegas
    par = processes.DEFAULT_PARAMS
    threads = _host_threads()
    torch.set_num_threads(threads)
    d = processes.dims(PROC)
    edges = ovegas.uniform_grid(d, NB)
    # warm-up (first-call costs), then size the sample from a pass of 2048 events
    _oracle_pass(PROC, par, philox.uniforms(seed, 512, d), edges)
    n0 = 2048
    dt0, _, _ = _oracle_pass(PROC, par, philox.uniforms(seed, n0, d), edges)
    n = int(max(n0, min(20000, n0 * run_s / max(dt0, 1e-3))))
    x = philox.uniforms(seed, n, d)
    times, keep = [], None
    for _ in range(3):
        dt, me, ok = _oracle_pass(PROC, par, x, edges)
        times.append(dt)
        keep = keep or (x, me, ok)
    t_med = float(np.median(times))
    torch.set_num_threads(1)
    m0 = 512
    dt1, _, _ = _oracle_pass(PROC, par, philox.uniforms(seed, m0, d), edges)
    n1 = int(max(m0, min(20000, m0 * run_s / max(dt1, 1e-3))))
    dt1, _, _ = _oracle_pass(PROC, par, philox.uniforms(seed + 1, n1, d), edges)
    torch.set_num_threads(threads)
    others = {}
    for proc, m in (('gg_tt', 100_000), ('gg_ttg', 20_000)):
        dp = processes.dims(proc)
        t, _, _ = _oracle_pass(proc, par, philox.uniforms(seed, m, dp), ovegas.uniform_grid(dp, NB))
        others[proc] = {'events': m, 'events_per_s': m / t, 'threads': threads}
    rec = dict(value=n / t_med, unit='events/s', cores=threads, kind='oracle',
               sample=f'{n} gg->ttbar gg events (uniforms, Vegas map, phase space, cuts, colour-ordered FP64 '
                      f'|M|^2, Vegas accumulation), median of 3 passes after a warm-up: '
                      f'{", ".join(f"{t:.2f}" for t in times)} s',
               cpu_model=_cpu_model(),
               one_thread={'events': n1, 'events_per_s': n1 / dt1, 'seconds': dt1},
               other_processes=others)
    return rec, keep


def oracle_check(mf, h, prm, sample):
    """Direct comparison of the GPU kernels with the oracle on the cpu_baseline sample:
    the same uniforms through the GPU phase space (identity Vegas map) and matrix element
    in both precisions, relative differences over the events that pass the cuts."""
    x, me_o, ok = sample
    pid = mf.PROCESS[PROC]
    dev = torch.device('cuda', 0)
    xt = torch.tensor(x, dtype=torch.float64, device=dev).contiguous()
    n = x.shape[1]
    ev = mf.mf_phase_space(h, pid, prm, n, x=xt)
    out = {'events': int(ok.sum())}
    for name, prec in (('fp32_mfma_bf16', mf.MF_FP32_MFMA_BF16), ('fp64', mf.MF_FP64)):
        m = mf.matrix_element(h, pid, ev['p'], prec, prm).double().cpu().numpy()
        rel = np.abs(m[ok] / me_o[ok] - 1.0)
        out[name] = {'median': float(np.median(rel)), 'max': float(rel.max())}
    return out


def accuracy_failures(rel_fp32_fp64, vs_oracle):
    """Reasons the run may not publish a throughput: the FP32 results off their bars (median
    1e-5, max 1e-3 relative, no NaN) against FP64 on the last batch or against the oracle,
    or FP64 off 1e-12 against the oracle."""
    bad = []
    r = rel_fp32_fp64
    if not (r['median'] <= 1e-5 and r['max'] <= 1e-3):
        bad.append(f'FP32 vs FP64 on the last batch: median {r["median"]}, max {r["max"]} '
                   f'(bars 1e-5, 1e-3; NaN fails)')
    if vs_oracle is not None:
        a, b = vs_oracle['fp32_mfma_bf16'], vs_oracle['fp64']
        if not (a['median'] <= 1e-5 and a['max'] <= 1e-3):
            bad.append(f'FP32 vs oracle: median {a["median"]}, max {a["max"]}')
        if not b['max'] <= 1e-12:
            bad.append(f'FP64 vs oracle: max {b["max"]} (bar 1e-12)')
    return bad


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=16)
    ap.add_argument('--warmup', type=int, default=2)
    ap.add_argument('--precision', default='auto')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--no-extras', action='store_true', help='skip the derivative and mixed-batch timings')
    ap.add_argument('--streams', type=int, default=2, choices=(1, 2, 3),
                    help='2: the next batch\'s phase space runs on a second stream beside the matrix element; '
                         '3: the Vegas calls run on a third stream')
    ap.add_argument('--seed', type=int, default=4)
    ap.add_argument('--copy-calibration', action='store_true',
                    help=f'also run one {COPY_BYTES >> 20} MiB device-to-device copy (counter calibration)')
    args = ap.parse_args()
    if args.gpus != 1:
        print(f'bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); '
              'the event axis would shard across GPUs with one all-reduce of the Vegas '
              'accumulators per iteration, which is not built here.', file=sys.stderr)
        sys.exit(2)
    import paper_2211_14056_amd as mf
    if not os.path.exists(mf.LIB_PATH):
        from paper_2211_14056_amd import build as _b
        _b.build()
    torch.cuda.init()
    h = mf.Handle(0)
    prm = mf.params()
    if args.copy_calibration:
        # a plain device copy of known size, so that HBM byte counters read for
        # the kernels of this run can be scaled by what they read for it
        src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device='cuda').fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    if args.precision == 'auto':
        prec = mf.MF_FP32_MFMA_BF16
    else:
        prec = mf.PRECISION[args.precision]
    head = run_path(mf, h, prm, prec, args.steps, args.warmup, args.seed, args.streams)
    ref = run_path(mf, h, prm, mf.MF_FP64, args.steps, args.warmup, args.seed, args.streams)
    # relative difference FP32 vs FP64 on the last batch (same events), events passing cuts
    ok = head['pas'].bool()
    rel = ((head['me'].double() - ref['me']) / ref['me']).abs()[ok]
    # NaN sorts last: a NaN anywhere makes the max NaN and fails the gate below
    rel_np = rel.cpu().numpy()
    nan = int(np.isnan(rel_np).sum())
    rel_stats = dict(median=float(np.median(rel_np)), p99=float(np.quantile(rel_np, 0.99)),
                     max=float('nan') if nan else float(rel_np.max()), events=int(ok.sum()), nan=nan)
    pname = [k for k, v in mf.PRECISION.items() if v == prec][0]
    fl = flops_per_event(PROC, pname)
    fl64 = flops_per_event(PROC, 'fp64')
    ev_s = args.steps * BATCH / head['seconds']
    ev_s64 = args.steps * BATCH / ref['seconds']
    me_ach = fl * BATCH / (head['me_ms'] * 1e-3)
    me_ach64 = fl64 * BATCH / (ref['me_ms'] * 1e-3)
    dt = 'f32'
    out = {
        'metric': METRIC,
        'value': ev_s,
        'unit': 'events/s',
        'n_gpus': 1,
        'steps': args.steps,
        'warmup': args.warmup,
        'ms_per_step': head['seconds'] / args.steps * 1e3,
        'higher_is_better': True,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': dt,
        'data': 'synthetic',
        'config': {'workload': 'gg->ttbar gg at sqrt(s_hat)=1 TeV, m_t=173 GeV, alpha_s=0.118, gluon pT>20 GeV, '
                               '|eta|<2.5, DeltaR>0.4; 1e6-event batches, Vegas refined every 16 batches',
                   'process': PROC, 'batch': BATCH, 'precision': pname, 'streams': args.streams},
        'me_events_per_s': BATCH / (head['me_ms'] * 1e-3),
        'rel_err_fp32_vs_fp64': rel_stats,
        'fp64': {'value': ev_s64, 'ms_per_step': ref['seconds'] / args.steps * 1e3,
                 'me_events_per_s': BATCH / (ref['me_ms'] * 1e-3),
                 'roofline': {'bound': 'alu', 'achieved': me_ach64 / 1e12, 'peak': PEAK['f64'] / 1e12,
                              'unit': 'TFLOP/s', 'frac': me_ach64 / PEAK['f64'],
                              'traffic': measured_traffic('fp64'), 'flops_per_event': fl64}},
        'roofline': {'bound': 'alu', 'achieved': me_ach / 1e12, 'peak': PEAK['f32'] / 1e12, 'unit': 'TFLOP/s',
                     'frac': me_ach / PEAK['f32'], 'traffic': measured_traffic(pname),
                     'kernel': 'matrix element', 'flops_per_event': fl},
    }
    if not args.no_extras:
        out['extras'] = extras(mf, h, prm, args.seed)
    vs_oracle = None
    if not args.no_cpu_baseline:
        out['cpu_baseline'], sample = cpu_baseline(args.seed)
        vs_oracle = oracle_check(mf, h, prm, sample)
        out['rel_err_vs_oracle'] = vs_oracle
    bad = accuracy_failures(rel_stats, vs_oracle)
    if bad:
        print('bench.py: results off their accuracy bars, no throughput published:\n  ' + '\n  '.join(bad),
              file=sys.stderr)
        sys.exit(3)
    print(json.dumps(out))


if __name__ == '__main__':
    main()
