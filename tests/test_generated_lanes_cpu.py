"""The lane-split gg -> t tbar g g bodies (two and four lanes per event) run on the CPU.

These bodies are straight-line code in which the lanes that share an event
exchange currents and amplitudes by DPP.  On the host they are compiled with a
value type that holds all the lanes of one event at once: arithmetic acts lane
by lane, the pair exchange swaps the two lanes and the quad rotation rotates
the four, and branch decisions (kval) require every lane to agree, which holds
for the kinematics the lanes share.  The per-lane inputs (relabelled momenta,
polarisation bases, beam directions, helicity bits) are set as the kernels set
them.  The lanes' helicity sums, added, must reproduce the oracle's |M|^2 to
1e-12 in FP64.  This pins the lane relabelling, the current exchange and the
colour blocks of both layouts without a GPU.
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
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, 'tests'))
from paper_2211_14056_amd.gen import lane_split, process_compiler as pc  # noqa: E402
from test_generated_cpu import _host_headers  # noqa: E402

P = processes.DEFAULT_PARAMS

LANES_H = r"""
#pragma once
#include <cmath>
#include <cstdio>
#include <cstdlib>
template <int N> struct Lanes {
    double v[N];
    Lanes() { for (int i = 0; i < N; ++i) v[i] = 0.0; }
    Lanes(double x) { for (int i = 0; i < N; ++i) v[i] = x; }
};
#define LANES_BINOP(op) \
template <int N> Lanes<N> operator op(Lanes<N> a, Lanes<N> b) { Lanes<N> r; for (int i = 0; i < N; ++i) r.v[i] = a.v[i] op b.v[i]; return r; } \
template <int N> Lanes<N> operator op(double a, Lanes<N> b) { return Lanes<N>(a) op b; } \
template <int N> Lanes<N> operator op(Lanes<N> a, double b) { return a op Lanes<N>(b); } \
template <int N> Lanes<N>& operator op##=(Lanes<N>& a, Lanes<N> b) { a = a op b; return a; }
LANES_BINOP(+) LANES_BINOP(-) LANES_BINOP(*) LANES_BINOP(/)
template <int N> Lanes<N> operator-(Lanes<N> a) { for (int i = 0; i < N; ++i) a.v[i] = -a.v[i]; return a; }
template <int N> Lanes<N> fma(Lanes<N> a, Lanes<N> b, Lanes<N> c)
{ Lanes<N> r; for (int i = 0; i < N; ++i) r.v[i] = std::fma(a.v[i], b.v[i], c.v[i]); return r; }
template <int N> Lanes<N> sqrt(Lanes<N> a) { for (int i = 0; i < N; ++i) a.v[i] = std::sqrt(a.v[i]); return a; }
template <int N> double kval(Lanes<N> a)
{
    for (int i = 1; i < N; ++i)
        if (a.v[i] != a.v[0]) { fprintf(stderr, "lanes disagree on a branch\n"); abort(); }
    return a.v[0];
}
template <int N> void opaque(Lanes<N>&) {}
inline Lanes<2> pair_swap(Lanes<2> a) { Lanes<2> r; r.v[0] = a.v[1]; r.v[1] = a.v[0]; return r; }
template <int M> Lanes<4> quad_rot(Lanes<4> a) { Lanes<4> r; for (int i = 0; i < 4; ++i) r.v[i] = a.v[(i + M) & 3]; return r; }
template <int N> struct LaneInts { int v[N]; };
template <int N> Lanes<N> lamsel(int gconf, LaneInts<N> h)
{ Lanes<N> r; for (int i = 0; i < N; ++i) r.v[i] = ((gconf >> h.v[i]) & 1) ? 1.0 : -1.0; return r; }
"""

DRIVER = r"""
#include <hip/hip_runtime.h>
#include "lanes.h"
#include "me_common.h"
#include "body.inc"
#include <vector>
typedef Lanes<NL> L;
struct Sum { L acc; void add(L a, L b) { acc = acc + a + b; } };
int main()
{
    int n; double mt;
    if (scanf("%d %lf", &n, &mt) != 2) return 1;
    std::vector<L> lds((SLOTS > 0 ? SLOTS - 1 : 0) * 64 + 1);
    for (int e = 0; e < n; ++e) {
        double p[6][4];
        for (int l = 0; l < 6; ++l) for (int c = 0; c < 4; ++c) if (scanf("%lf", &p[l][c]) != 1) return 2;
        L kin[4][4], pt[4], ptb[4];
        LaneInts<NL> hb[4];
        for (int c = 0; c < 4; ++c) { pt[c] = L(p[2][c]); ptb[c] = L(p[3][c]); }
#if NL == 2
        L eu[2][3], ew[2][2], zs[2];
        for (int sub = 0; sub < 2; ++sub) {
            for (int j = 0; j < 4; ++j) {
                const int g = j ^ sub, leg = g < 2 ? g : g + 2;
                const double sgn = g < 2 ? 1.0 : -1.0;
                for (int c = 0; c < 4; ++c) kin[j][c].v[sub] = sgn * p[leg][c];
                hb[j].v[sub] = g;
                if (j >= 2) {
                    double u[3], w[2];
                    pol_basis<double, double>(p[leg], u, w);
                    for (int c = 0; c < 3; ++c) eu[j - 2][c].v[sub] = u[c];
                    for (int c = 0; c < 2; ++c) ew[j - 2][c].v[sub] = w[c];
                }
            }
            zs[0].v[sub] = sub ? -1.0 : 1.0;
            zs[1].v[sub] = -zs[0].v[sub];
        }
#else
        L eu[4][3], ew[4][2];
        for (int sub = 0; sub < 4; ++sub)
            for (int j = 0; j < 4; ++j) {
                const int g = (j + sub) & 3, leg = g < 2 ? g : g + 2;
                const double sgn = g < 2 ? 1.0 : -1.0;
                for (int c = 0; c < 4; ++c) kin[j][c].v[sub] = sgn * p[leg][c];
                hb[j].v[sub] = g;
                double u[3], w[2];
                pol_basis<double, double>(p[leg], u, w);
                for (int c = 0; c < 3; ++c) eu[j][c].v[sub] = u[c];
                for (int c = 0; c < 2; ++c) ew[j][c].v[sub] = -sgn * w[c];
            }
#endif
        for (auto& x : lds) x = L(NAN);
        Sum s;
        BODY<L, L>(kin, pt, ptb, eu, ew, EXTRA hb, L(mt), s, lds.data());
        double tot = 0.0;
        for (int i = 0; i < NL; ++i) tot += s.acc.v[i];
        printf("%.17g\n", tot * NORM);
    }
    return 0;
}
"""


def _events(n, seed):
    x = philox.uniforms(seed, n, processes.dims('gg_ttgg'))
    p, _ = integrand.momenta('gg_ttgg', P, torch.tensor(np.ascontiguousarray(x.T)))
    return p


@pytest.mark.skipif(shutil.which('g++') is None, reason='needs a host C++ compiler')
@pytest.mark.parametrize('layout', ['pair', 'quad'])
def test_lane_split_body_on_cpu_matches_oracle(tmp_path, layout):
    d = str(tmp_path)
    _host_headers(d)
    open(os.path.join(d, 'lanes.h'), 'w').write(LANES_H)
    proc = pc.GGTTProcess('gg_ttgg', 6)
    if layout == 'pair':
        src, info = lane_split.emit_pair(proc, pc.LDS_PAIR_F64, local_memo=True)
        nl, extra = 2, 'zs, '
    else:
        src, info = lane_split.emit_split(proc, pc.LDS_QUAD_F64, local_memo=True)
        nl, extra = 4, ''
    # per-lane helicity bits: the kernels pass an int per lane; here one value per lane of the event
    src = src.replace('const int (&hb)[4]', f'const LaneInts<{nl}> (&hb)[4]')
    src = re.sub(r'\(gconf >> hb\[(\d)\]\) & 1 \? R\(1\) : R\(-1\)', r'lamsel(gconf, hb[\1])', src)
    assert 'gconf >> hb' not in src
    open(os.path.join(d, 'body.inc'), 'w').write(src + '\n')
    open(os.path.join(d, 'driver.cpp'), 'w').write(DRIVER)
    norm = 2.0 / (proc.avg * float(proc.sym) * float(proc.cden))
    exe = os.path.join(d, 'me')
    cmd = ['g++', '-O1', '-std=c++17', f'-I{d}', f'-DNL={nl}', f'-DSLOTS={info["lds_slots"]}',
           f'-DBODY=me_gg_ttgg_{"pair" if layout == "pair" else "split"}', f'-DEXTRA={extra}',
           f'-DNORM={norm!r}', os.path.join(d, 'driver.cpp'), '-o', exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    n = 3
    p = _events(n, seed=17)
    inp = f'{n} {P["m_t"]!r}\n' + '\n'.join(' '.join(repr(float(v)) for v in p[e].reshape(-1)) for e in range(n))
    out = subprocess.run([exe], input=inp + '\n', capture_output=True, text=True, check=True).stdout.split()
    g2 = 4 * np.pi * P['alpha_s']
    got = np.array([float(v) for v in out]) * g2 ** 4
    ref = integrand.me('gg_ttgg', p, P).numpy()
    assert np.abs(got / ref - 1).max() < 1e-12, (got, ref)
