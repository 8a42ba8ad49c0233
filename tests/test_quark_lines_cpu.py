"""The generated two-quark-line matrix elements (gen/quark_lines.py + csrc/me_quark.h),
compiled for the host, against the oracle's explicit-colour diagram sum.

The kernel code itself (external wavefunctions, per-event kinematics, the helicity loop over
the chirality-conserving half of the configurations, the generated diagram body and the
colour matrix) runs on the CPU with one event per call; FP64 must equal the oracle to 1e-12
on every event for q qbar -> t tbar (+g, +gg) and q g -> t tbar q (+g), also at m_t = 0.
The generator's own structure is checked too: diagram counts, the colour basis size, the
colour matrix (Hermitian, positive semi-definite), and every diagram's colour tensor exactly
reproduced by its decomposition.
"""
import math
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
from paper_2211_14056_amd.gen import quark_lines as ql  # noqa: E402

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
using std::sqrt; using std::fma; using std::fmax; using std::fmin; using std::sin; using std::cos;
using std::floor; using std::pow; using std::fabs;
"""

DRIVER = r'''
#include <hip/hip_runtime.h>
#include <cstdio>
#include "me_common.h"
#include "proc.inc"
#include "me_quark.h"
int main()
{
    int n; double mt;
    if (scanf("%d %lf", &n, &mt) != 2) return 1;
    typedef mf::QLPROC T;
    for (int e = 0; e < n; ++e) {
        double pe[T::NEXT][4];
        for (int l = 0; l < T::NEXT; ++l) for (int c = 0; c < 4; ++c) if (scanf("%lf", &pe[l][c]) != 1) return 2;
        printf("%.17g\n", mf::quark_event<T, double>(pe, mt));
    }
    return 0;
}
'''


def _host_dir(d, proc):
    os.makedirs(os.path.join(d, 'hip'), exist_ok=True)
    open(os.path.join(d, 'hip', 'hip_runtime.h'), 'w').write(HIP_STUB)
    src = open(os.path.join(CSRC, 'me_common.h')).read()
    src = src.replace('asm volatile("" : "+v"(x));', '(void)x;')
    src = re.sub(r'return __builtin_amdgcn_update_dpp\([^;]*\);', 'return x;', src)
    open(os.path.join(d, 'me_common.h'), 'w').write(src)
    for f in ('dual.h', 'me_quark.h'):
        shutil.copy(os.path.join(CSRC, f), d)
    text, _ = ql.emit(proc)
    open(os.path.join(d, 'proc.inc'), 'w').write(text)
    open(os.path.join(d, 'driver.cpp'), 'w').write(DRIVER.replace('QLPROC', f'QL_{proc}'))
    exe = os.path.join(d, 'me')
    r = subprocess.run(['g++', '-O1', '-std=c++17', f'-I{d}', os.path.join(d, 'driver.cpp'), '-o', exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


@pytest.mark.skipif(shutil.which('g++') is None, reason='needs a host C++ compiler')
@pytest.mark.parametrize('proc,n,mt', [('qq_tt', 40, 173.0), ('qq_ttg', 20, 173.0), ('qg_ttq', 20, 173.0),
                                       ('qq_ttgg', 6, 173.0), ('qg_ttqg', 6, 173.0), ('qq_ttg', 8, 0.0),
                                       ('qg_ttqg', 4, 0.0)])
def test_generated_code_on_cpu_matches_oracle(tmp_path, proc, n, mt):
    par = dict(P, m_t=mt)
    exe = _host_dir(str(tmp_path), proc)
    x = philox.uniforms(29, n, processes.dims(proc))
    p, _ = integrand.momenta(proc, par, torch.tensor(np.ascontiguousarray(x.T)))
    inp = f'{n} {mt!r}\n' + '\n'.join(' '.join(repr(float(v)) for v in p[e].reshape(-1)) for e in range(n))
    out = subprocess.run([exe], input=inp + '\n', capture_output=True, text=True, check=True).stdout.split()
    g2 = 4 * math.pi * P['alpha_s']
    got = np.array([float(v) for v in out]) * g2 ** (processes.PROCESSES[proc]['n_ext'] - 2)
    ref = integrand.me(proc, p, par).numpy()
    assert np.abs(got / ref - 1).max() < 1e-12


@pytest.mark.parametrize('proc,nd,nb', [('qq_tt', 1, 2), ('qq_ttg', 5, 4), ('qq_ttgg', 38, 12), ('qg_ttq', 5, 4),
                                        ('qg_ttqg', 38, 12)])
def test_diagrams_and_colour_decomposition(proc, nd, nb):
    legs, nodes, diagrams, labels, coeff, G = ql.decompose(proc)
    assert len(diagrams) == nd and len(labels) == nb
    Gm = np.array([[float(x) for x in row] for row in G])
    assert np.allclose(Gm, Gm.T) and np.linalg.eigvalsh(Gm).min() > -1e-12
    basis, blabels = ql.colour_basis(legs)
    B = {lab: t for lab, t in zip(blabels, basis)}
    for d, (r, g_) in enumerate(diagrams):
        T = ql.diagram_colour(r, g_, legs)
        rec = sum((float(coeff[d][i][0]) + 1j * float(coeff[d][i][1])) * B[lab] for i, lab in enumerate(labels))
        assert np.abs(rec - T).max() < 1e-13
