"""Process definitions and helicity tables.  Test infrastructure only.

Processes are the top-pair channels of the paper's benchmarks (pp -> ttbar, ttbar g,
ttbar gg; sect. 3, Table 1, Figs. 3-4): the gg-initiated ones, one more gluon
(gg -> ttbar ggg, where the growth with the number of diagrams the paper discusses
goes further), the quark-initiated ones with one massless light-quark flavour
(q qbar -> ttbar (+g, +gg), q g -> ttbar q (+g)), plus e+e- -> mu+mu- as the simplest
closed-form check.

Leg order in a momentum array p[N, n_ext, 4] (physical momenta):
  ee_mumu : e-(in), e+(in), mu-(out), mu+(out)
  gg_tt*  : g(in), g(in), t(out), tbar(out), g(out) ...
  qq_tt*  : q(in), qbar(in), t(out), tbar(out), g(out) ...
  qg_ttq* : q(in), g(in), t(out), tbar(out), q(out), g(out)
Legs 4, 5, ... are the massless final-state partons (gluons and the light quark).
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
    'gg_ttggg': dict(n_ext=7, n_out_gluons=3, avg=256.0, sym=6.0, kind='qcd'),
    # two quark lines; avg = spins x colours of the initial state (q qbar: 2 2 3 3, q g: 2 2 3 8)
    'qq_tt': dict(n_ext=4, n_out_gluons=0, avg=36.0, sym=1.0, kind='qcd4',
                  legs=[('q', True), ('qbar', True), ('t', False), ('tbar', False)]),
    'qq_ttg': dict(n_ext=5, n_out_gluons=1, avg=36.0, sym=1.0, kind='qcd4',
                   legs=[('q', True), ('qbar', True), ('t', False), ('tbar', False), ('g', False)]),
    'qq_ttgg': dict(n_ext=6, n_out_gluons=2, avg=36.0, sym=2.0, kind='qcd4',
                    legs=[('q', True), ('qbar', True), ('t', False), ('tbar', False), ('g', False),
                          ('g', False)]),
    'qg_ttq': dict(n_ext=5, n_out_gluons=0, avg=96.0, sym=1.0, kind='qcd4',
                   legs=[('q', True), ('g', True), ('t', False), ('tbar', False), ('q', False)]),
    'qg_ttqg': dict(n_ext=6, n_out_gluons=1, avg=96.0, sym=1.0, kind='qcd4',
                    legs=[('q', True), ('g', True), ('t', False), ('tbar', False), ('q', False),
                          ('g', False)]),
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
    return [params['m_t'], params['m_t']] + [0.0] * (PROCESSES[proc]['n_ext'] - 4)


def helicities(proc):
    return list(itertools.product((-1, 1), repeat=PROCESSES[proc]['n_ext']))


def g_strong(params):
    return math.sqrt(4.0 * math.pi * params['alpha_s'])


def e_charge(params):
    return math.sqrt(4.0 * math.pi * params['alpha'])
