"""Process definitions and helicity tables.  Test infrastructure only.

Processes are the gg-initiated top-pair channels the paper benchmarks
(pp -> ttbar, ttbar g, ttbar gg; sect. 3, Table 1, Figs. 3-4) plus
e+e- -> mu+mu- as the simplest closed-form check.

Leg order in a momentum array p[N, n_ext, 4] (physical momenta):
  ee_mumu : e-(in), e+(in), mu-(out), mu+(out)
  gg_tt*  : g(in), g(in), t(out), tbar(out), g(out) ...
Helicity configurations are all of {-1,+1}^n_ext in lexicographic order over
legs 0..n_ext-1, -1 before +1.
"""
import itertools
import math

PROCESSES = {
    'ee_mumu': dict(n_ext=4, n_out_gluons=0, avg=4.0, sym=1.0, kind='ee'),
    'gg_tt': dict(n_ext=4, n_out_gluons=0, avg=256.0, sym=1.0, kind='qcd'),
    'gg_ttg': dict(n_ext=5, n_out_gluons=1, avg=256.0, sym=1.0, kind='qcd'),
    'gg_ttgg': dict(n_ext=6, n_out_gluons=2, avg=256.0, sym=2.0, kind='qcd'),
}

DEFAULT_PARAMS = dict(sqrt_s=1000.0, m_t=173.0, alpha_s=0.118, alpha=1.0 / 137.0,
                      pt_min=20.0, eta_max=2.5, dr_min=0.4)
EE_PARAMS = dict(DEFAULT_PARAMS, sqrt_s=100.0)


def n_out(proc):
    return PROCESSES[proc]['n_ext'] - 2


def dims(proc):
    """Number of uniforms per event: 3 n_out - 4."""
    return 3 * n_out(proc) - 4


def out_masses(proc, params):
    if PROCESSES[proc]['kind'] == 'ee':
        return [0.0, 0.0]
    return [params['m_t'], params['m_t']] + [0.0] * PROCESSES[proc]['n_out_gluons']


def helicities(proc):
    return list(itertools.product((-1, 1), repeat=PROCESSES[proc]['n_ext']))


def g_strong(params):
    return math.sqrt(4.0 * math.pi * params['alpha_s'])


def e_charge(params):
    return math.sqrt(4.0 * math.pi * params['alpha'])
