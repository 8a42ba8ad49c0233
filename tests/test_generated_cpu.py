"""The generated matrix-element bodies, compiled for the host and run on the CPU.

The process compiler emits straight-line device code.  Its functions are plain
arithmetic, so they also compile as host C++ once the few GPU intrinsics are
stubbed (an empty-asm register barrier, a scheduling barrier, a lane
permutation the one-lane bodies do not use).  Evaluated in FP64 on events from
the oracle's phase space, every emitted form must reproduce the oracle's
|M|^2 to 1e-12.  The forms checked are the plain recursion, LDS parking and
shared quark-line products.  This pins the generator independently of any GPU.
"""
import os
import re
import shutil
import subprocess
import sys

import numpy as np
import pytest
import torch

from oracle import integrand, philox, processes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, 'paper_2211_14056_amd', 'csrc')
sys.path.insert(0, ROOT)
from paper_2211_14056_amd.gen import process_compiler as pc  # noqa: E402

P = processes.DEFAULT_PARAMS

HIP_STUB = """#pragma once
#include <cmath>
#include <cstdint>
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __constant__
#define __shared__
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
using std::sqrt; using std::fma; using std::fmax; using std::sin; using std::cos;
"""

DRIVER = r"""
#include <hip/hip_runtime.h>
#include <cstdio>
#include <vector>
#include "me_common.h"
#include "body.inc"
struct Sum { double acc = 0; void add(double a, double b) { acc += a + b; } };
int main()
{
    int n; double mt;
    if (scanf("%d %lf", &n, &mt) != 2) return 1;
    std::vector<double> lds(SLOTS * 64 + 64);
    for (int e = 0; e < n; ++e) {
        double pe[NEXT][4];
        for (int l = 0; l < NEXT; ++l) for (int c = 0; c < 4; ++c) if (scanf("%lf", &pe[l][c]) != 1) return 2;
        Sum s;
        BODY<double>(pe, mt, s LDSARG);
        printf("%.17g\n", s.acc * NORM());
    }
    return 0;
}
"""


def _host_headers(d):
    os.makedirs(os.path.join(d, 'hip'), exist_ok=True)
    open(os.path.join(d, 'hip', 'hip_runtime.h'), 'w').write(HIP_STUB)
    src = open(os.path.join(CSRC, 'me_common.h')).read()
    src = src.replace('asm volatile("" : "+v"(x));', '(void)x;')
    src = re.sub(r'return __builtin_amdgcn_update_dpp\([^;]*\);', 'return x;', src)
    open(os.path.join(d, 'me_common.h'), 'w').write(src)
    shutil.copy(os.path.join(CSRC, 'dual.h'), d)


def _events(proc, n, seed):
    x = philox.uniforms(seed, n, processes.dims(proc))
    p, _ = integrand.momenta(proc, P, torch.tensor(np.ascontiguousarray(x.T)))
    return p


CASES = [
    # (process, legs, variant options, events)
    ('gg_ttg', 5, dict(), 12),
    ('gg_ttg', 5, dict(share_products=True), 12),
    ('gg_ttgg', 6, dict(), 4),
    ('gg_ttgg', 6, dict(share_products=True), 4),
    ('gg_ttgg', 6, dict(share_products=True, lds_budget=152), 4),
    ('gg_ttgg', 6, dict(lds_budget=152), 4),
]


@pytest.mark.skipif(shutil.which('g++') is None, reason='needs a host C++ compiler')
@pytest.mark.parametrize('proc,legs,opts,n', CASES)
def test_generated_body_on_cpu_matches_oracle(tmp_path, proc, legs, opts, n):
    d = str(tmp_path)
    _host_headers(d)
    gp = pc.GGTTProcess(proc, legs)
    body, _ = pc.emit_qcd(gp, with_colour=True, **opts)
    open(os.path.join(d, 'body.inc'), 'w').write(body + '\n')
    open(os.path.join(d, 'driver.cpp'), 'w').write(DRIVER)
    slots = opts.get('lds_budget', 0)
    exe = os.path.join(d, 'me')
    cmd = ['g++', '-O1', '-std=c++17', f'-I{d}', f'-DSLOTS={max(slots, 1)}', f'-DNEXT={legs}',
           f'-DBODY=me_{proc}_body', f'-DNORM=me_{proc}_norm_noalpha',
           '-DLDSARG=' + (', lds.data()' if slots else ''), os.path.join(d, 'driver.cpp'), '-o', exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    p = _events(proc, n, seed=13)
    inp = f'{n} {P["m_t"]!r}\n' + '\n'.join(' '.join(repr(float(v)) for v in p[e].reshape(-1)) for e in range(n))
    out = subprocess.run([exe], input=inp + '\n', capture_output=True, text=True, check=True).stdout.split()
    g2 = 4 * np.pi * P['alpha_s']
    got = np.array([float(v) for v in out]) * g2 ** (legs - 2)
    ref = integrand.me(proc, p, P).numpy()
    assert np.abs(got / ref - 1).max() < 1e-12
