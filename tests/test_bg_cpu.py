"""The table-driven recursion (one wavefront per event on the GPU), compiled for the host.

csrc/me_bg.h walks the tables of gen/bg_tables.py; on the host it runs with one lane per
event (the lane loops then cover every node in order, and the workgroup barriers are
no-ops).  In FP64 it must reproduce the oracle's colour-ordered |M|^2 to 1e-12 for
gg -> ttbar g, gg -> ttbar gg and gg -> ttbar ggg, on events from the oracle's phase space.
This pins the tables, the vertex forms and the colour matrix of the 5-gluon process
independently of any GPU.
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
from paper_2211_14056_amd.gen import bg_tables  # noqa: E402

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
#define __launch_bounds__(...)
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
typedef int hipError_t;
typedef void* hipStream_t;
struct Dim3Stub { unsigned x = 0; };
static Dim3Stub threadIdx, blockIdx, blockDim;
inline void __syncthreads() {}
template <typename T> inline T __shfl_xor(T v, int) { return v; }
using std::sqrt; using std::fma; using std::fmax; using std::fmin; using std::sin; using std::cos;
"""

INTERNAL_STUB = """#pragma once
#include <cstdint>
"""

DRIVER = r'''
#include <hip/hip_runtime.h>
#include <cstdio>
#include <memory>
#include "me_common.h"
#include "tables.inc"
#include "me_bg.h"
int main()
{
    int n; double mt;
    if (scanf("%d %lf", &n, &mt) != 2) return 1;
    auto sh = std::make_unique<mf::BgShared<KG, double>>();
    for (int e = 0; e < n; ++e) {
        double pe[KG + 2][4];
        for (int l = 0; l < KG + 2; ++l) for (int c = 0; c < 4; ++c) if (scanf("%lf", &pe[l][c]) != 1) return 2;
        const double me = mf::bg_event<KG, double, 1>(pe, mt, *sh, 0);
        printf("%.17g\n", me * mf::bg_norm_noalpha<KG>());
    }
    return 0;
}
'''


def _host_headers(d):
    os.makedirs(os.path.join(d, 'hip'), exist_ok=True)
    open(os.path.join(d, 'hip', 'hip_runtime.h'), 'w').write(HIP_STUB)
    open(os.path.join(d, 'internal.h'), 'w').write(INTERNAL_STUB)
    src = open(os.path.join(CSRC, 'me_common.h')).read()
    src = src.replace('asm volatile("" : "+v"(x));', '(void)x;')
    src = re.sub(r'return __builtin_amdgcn_update_dpp\([^;]*\);', 'return x;', src)
    open(os.path.join(d, 'me_common.h'), 'w').write(src)
    for f in ('dual.h', 'me_bg.h'):
        shutil.copy(os.path.join(CSRC, f), d)


@pytest.mark.skipif(shutil.which('g++') is None, reason='needs a host C++ compiler')
@pytest.mark.parametrize('proc,n', [('gg_ttg', 12), ('gg_ttgg', 6), ('gg_ttggg', 3)])
def test_table_recursion_on_cpu_matches_oracle(tmp_path, proc, n):
    d = str(tmp_path)
    _host_headers(d)
    legs = processes.PROCESSES[proc]['n_ext']
    k = legs - 2
    src, _ = bg_tables.emit(k, f'bg{k}')
    open(os.path.join(d, 'tables.inc'), 'w').write(src)
    open(os.path.join(d, 'driver.cpp'), 'w').write(DRIVER)
    exe = os.path.join(d, 'bg')
    r = subprocess.run(['g++', '-O1', '-std=c++17', f'-I{d}', f'-DKG={k}', os.path.join(d, 'driver.cpp'), '-o', exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    x = philox.uniforms(13, n, processes.dims(proc))
    p, _ = integrand.momenta(proc, P, torch.tensor(np.ascontiguousarray(x.T)))
    inp = f'{n} {P["m_t"]!r}\n' + '\n'.join(' '.join(repr(float(v)) for v in p[e].reshape(-1)) for e in range(n))
    out = subprocess.run([exe], input=inp + '\n', capture_output=True, text=True, check=True).stdout.split()
    g2 = 4 * np.pi * P['alpha_s']
    got = np.array([float(v) for v in out]) * g2 ** k
    ref = integrand.me(proc, p, P).numpy()
    assert np.abs(got / ref - 1).max() < 1e-12
