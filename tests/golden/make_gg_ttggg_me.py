"""Writes gg_ttggg_me.txt: the oracle's |M|^2 of g g -> t tbar g g g on seeded events.

The oracle at five gluons spends ~35 s per call (64 gluon helicity configurations, 120
orderings, one recursion per helicity over the whole batch), too slow for a GPU test to
recompute; the values are stored once, from the oracle alone:
  events   128 events, uniforms philox(seed 13, dims 11), the oracle's phase space at
           sqrt(s) = 1 TeV (no Vegas map);
  columns  |M|^2 with m_t = 173 GeV, |M|^2 with m_t = 0 (same momenta), the oracle's cut
           decision (pT > 20 GeV, |eta| < 2.5, Delta R > 0.4 over every gluon pair).
Run from the repository root:  PYTHONPATH=. python tests/golden/make_gg_ttggg_me.py
"""
import os

import numpy as np
import torch

from oracle import cuts, integrand, philox, processes

PROC, SEED, N = 'gg_ttggg', 13, 128
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), 'gg_ttggg_me.txt')


def events():
    P = processes.DEFAULT_PARAMS
    x = philox.uniforms(SEED, N, processes.dims(PROC))
    p, _ = integrand.momenta(PROC, P, torch.tensor(np.ascontiguousarray(x.T)))
    return p


def main():
    P = processes.DEFAULT_PARAMS
    p = events()
    me = integrand.me(PROC, p, P).numpy()
    me0 = integrand.me(PROC, p, dict(P, m_t=0.0)).numpy()
    ok = cuts.passes(p, P).numpy()
    with open(OUT, 'w') as f:
        f.write(f'# oracle |M|^2 of g g -> t tbar g g g: {N} events, philox seed {SEED}, sqrt(s) = '
                f'{P["sqrt_s"]} GeV, alpha_s = {P["alpha_s"]}\n')
        f.write('# written by tests/golden/make_gg_ttggg_me.py (oracle only)\n')
        f.write('# me(m_t = 173)  me(m_t = 0)  passes_cuts\n')
        for a, b, c in zip(me, me0, ok):
            f.write(f'{a:.17e} {b:.17e} {int(c)}\n')


if __name__ == '__main__':
    main()
