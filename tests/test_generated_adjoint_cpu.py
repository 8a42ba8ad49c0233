"""The generated reverse-sweep derivative, compiled for the host and run on the CPU.

The process compiler emits, per process, the kinematic inputs of the recursion
(<proc>_kin, templated on an output policy) and the reverse sweep of the
helicity-summed, colour-contracted |M|^2 over them (<proc>_adjoint).  The
per-event derivative (me_vjp_event.h: FP64 kinematics, the adjoint, then
tangents of the kinematics contracted with its result) is the same header the
GPU kernel includes.  Compiled for the host (GPU intrinsics stubbed) and run in
FP64 and FP32 on uniforms through a non-uniform Vegas grid, it must reproduce
the oracle's reverse-mode gradient (torch autograd through the Vegas map, the
phase space and the colour-ordered matrix element): FP64 to 1e-10, FP32 to a
median of 1e-4 and a maximum of 1e-2 (normwise per event).  The tangent width
of the kinematic passes is varied, so a wrong direction bookkeeping fails too.
"""
import os
import re
import shutil
import subprocess
import sys

import numpy as np
import pytest

from oracle import grad as ograd, philox, processes

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
using std::sqrt; using std::fma; using std::fmax; using std::fmin; using std::sin; using std::cos;
using std::floor; using std::pow; using std::fabs;
"""

DRIVER = r"""
#include <hip/hip_runtime.h>
#include <cstdio>
#include "me_common.h"
#include "body.inc"
#include "me_vjp_event.h"
int main()
{
    int n, nb; double mt, rs;
    if (scanf("%d %d %lf %lf", &n, &nb, &mt, &rs) != 4) return 1;
    constexpr int D = 3 * KG - 4;
    double edges[D * 64];
    for (int i = 0; i < D * (nb + 1); ++i) if (scanf("%lf", &edges[i]) != 1) return 2;
    for (int e = 0; e < n; ++e) {
        double x[D];
        for (int k = 0; k < D; ++k) if (scanf("%lf", &x[k]) != 1) return 3;
        double me, g[D + 1];
        typedef mf::AdjProc<KG> A;
        RT zb[A::NZB > A::NZ ? A::NZB : A::NZ];
        mf::vjp_event<KG, RT, CHW, 1>(x, edges, nb, rs, mt, me, g, zb);
        printf("%.17g", me);
        for (int k = 0; k <= D; ++k) printf(" %.17g", g[k]);
        printf("\n");
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
    for f in ('dual.h', 'dualn.h', 'ps_core.h', 'me_vjp_event.h'):
        shutil.copy(os.path.join(CSRC, f), d)


def _edges(d, seed):
    rng = np.random.default_rng(seed)
    w_ = rng.uniform(0.5, 1.5, (d, 50))
    e = np.concatenate([np.zeros((d, 1)), np.cumsum(w_, 1) / w_.sum(1, keepdims=True)], 1)
    e[:, -1] = 1.0
    return e


def _norms(proc):
    gp = pc.GGTTProcess(proc, processes.PROCESSES[proc]['n_ext'])
    g2 = 4 * np.pi * P['alpha_s']
    return g2 ** gp.k * 2.0 / (gp.avg * gp.sym * gp.cden)


RG = dict(regroup=True)
ZB = dict(zb_mem=True, regroup=True)
CASES = [
    # (process, working type, tangent directions per kinematic pass, events, emitter options):
    # accumulators in registers or in the caller's memory (zb_mem; jb_mem: the current
    # adjoints too, all or the least read ones), quark line swept at once or by groups of
    # orderings sharing their first group_depth gluons (regroup), or with the gluon currents
    # recomputed per ordering too (recompute_currents).  gg -> ttbar gg compiles for a
    # minute, so it runs the register form and the library's form in both precisions only.
    ('gg_tt', 'double', 3, 16, {}),
    ('gg_ttg', 'double', 6, 16, {}),
    ('gg_ttg', 'double', 2, 6, {}),
    ('gg_ttg', 'float', 6, 16, {}),
    ('gg_ttgg', 'double', 3, 3, {}),
    ('gg_tt', 'double', 3, 8, RG),
    ('gg_ttg', 'double', 3, 16, RG),
    ('gg_ttg', 'float', 3, 16, RG),
    ('gg_tt', 'double', 1, 8, dict(ZB, group_depth=2)),
    ('gg_tt', 'float', 3, 8, dict(ZB, group_depth=2)),
    ('gg_ttg', 'double', 1, 16, dict(ZB, group_depth=3)),
    ('gg_ttg', 'float', 3, 16, dict(ZB, group_depth=3)),
    ('gg_ttg', 'double', 2, 8, dict(zb_mem=True, jb_mem=True)),
    ('gg_ttg', 'double', 1, 8, dict(ZB, group_depth=3, jb_mem=20)),
    ('gg_ttg', 'float', 3, 8, dict(ZB, group_depth=3, jb_mem=20)),
    ('gg_ttgg', 'double', 1, 3, dict(ZB, group_depth=4)),
    ('gg_ttgg', 'float', 3, 3, dict(ZB, group_depth=4)),
    ('gg_tt', 'double', 1, 8, dict(zb_mem=True, recompute_currents=True)),
    ('gg_ttg', 'double', 1, 16, dict(zb_mem=True, recompute_currents=True)),
    ('gg_ttg', 'float', 3, 16, dict(zb_mem=True, recompute_currents=True)),
]


@pytest.mark.skipif(shutil.which('g++') is None, reason='needs a host C++ compiler')
@pytest.mark.parametrize('proc,rtype,ch,n,opts', CASES)
def test_generated_adjoint_on_cpu_matches_oracle_gradient(tmp_path, proc, rtype, ch, n, opts):
    d_ = str(tmp_path)
    _host_headers(d_)
    legs = processes.PROCESSES[proc]['n_ext']
    gp = pc.GGTTProcess(proc, legs)
    body, _ = pc.emit_qcd_adjoint(gp, **opts)
    open(os.path.join(d_, 'body.inc'), 'w').write(body + '\n')
    open(os.path.join(d_, 'driver.cpp'), 'w').write(DRIVER)
    exe = os.path.join(d_, 'vjp')
    cmd = ['g++', '-O1', '-std=c++17', f'-I{d_}', f'-DKG={gp.k}', f'-DRT={rtype}', f'-DCHW={ch}',
           os.path.join(d_, 'driver.cpp'), '-o', exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    dim = processes.dims(proc)
    x = 0.02 + 0.96 * philox.uniforms(21, n, dim)
    ed = _edges(dim, 4)
    inp = [f'{n} 50 {P["m_t"]!r} {P["sqrt_s"]!r}', ' '.join(repr(float(v)) for v in ed.reshape(-1))]
    inp += [' '.join(repr(float(x[k, e])) for k in range(dim)) for e in range(n)]
    out = subprocess.run([exe], input='\n'.join(inp) + '\n', capture_output=True, text=True, check=True).stdout
    vals = np.array([[float(v) for v in line.split()] for line in out.strip().splitlines()])
    scale = _norms(proc)
    me = vals[:, 0] * scale
    g = vals[:, 1:].T * scale            # [d + 1][n]: x directions, then m_t
    me_o, gx_o, gth_o = ograd.vjp(proc, P, x, np.ones(n), edges=ed)
    ref = np.concatenate([gx_o, gth_o[:, :1].T], 0)
    rel_me = np.abs(me / me_o - 1)
    err = np.abs(g - ref).max(0) / np.abs(ref).max(0)
    if rtype == 'double':
        assert rel_me.max() < 1e-12
        assert err.max() < 1e-10, err
    else:
        assert np.median(rel_me) < 1e-5 and rel_me.max() < 1e-3
        assert np.median(err) < 1e-4 and err.max() < 1e-2, err


def test_the_library_forms_are_among_the_cases():
    """Each process's derivative form as the library builds it (ADJ_OPTS) runs above in both precisions."""
    for proc, opts in pc.ADJ_OPTS.items():
        for rtype in ('double', 'float'):
            assert any(c[0] == proc and c[1] == rtype and c[4] == opts for c in CASES), (proc, rtype, opts)
