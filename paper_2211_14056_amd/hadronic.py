"""pp -> t tbar (+ jet) cross sections: the sum over parton channels.

The paper's workload is hadronic (pp -> t tbar + jets, sect. 3, Table 1): each partonic
subprocess convoluted with the parton densities of the two beams.  With one light-quark
flavour q the tree-level channels are

  t tbar        g g -> t tbar;  q qbar and qbar q -> t tbar
  t tbar + jet  g g -> t tbar g;  q qbar and qbar q -> t tbar g;  q g and g q -> t tbar q;
                qbar g and g qbar -> t tbar qbar

Both beams are protons, so a channel and its beam-swapped partner give the same cross
section (x1 and x2 exchange, the rapidity range is symmetric): each pair is integrated once
and counted twice.  qbar g -> t tbar qbar is the charge conjugate of q g -> t tbar q with t and
tbar exchanged; the cross section does not distinguish t from tbar (equal masses, no cuts on
them), so it is q g -> t tbar q integrated with the antiquark density in place of the quark.
Every channel is one VegasIntegrator over mf_phase_space_pp; nothing here computes physics.
"""
from . import MF_FP64, PdfGrid, params
from .integrator import VegasIntegrator
from .workloads import toy_pdf_grid

# final state -> [(partonic process, density of parton 1, density of parton 2, multiplicity)]
CHANNELS = {
    'tt': [('gg_tt', 'g', 'g', 1), ('qq_tt', 'q', 'qbar', 2)],
    'ttj': [('gg_ttg', 'g', 'g', 1), ('qq_ttg', 'q', 'qbar', 2), ('qg_ttq', 'q', 'g', 2),
            ('qg_ttq', 'qbar', 'g', 2)],
}


def toy_grids():
    """The toy gluon, light-quark and antiquark densities as device grids."""
    return {k: PdfGrid(*toy_pdf_grid(kind=k)) for k in ('g', 'q', 'qbar')}


def sigma_pp(final='tt', sqrt_S=13000.0, grids=None, n=1_000_000, iters=4, warmup=1, precision=MF_FP64,
             prm=None, seed=1, handle=None):
    """sigma(pp -> final) in pb with its Monte Carlo error, and the per-channel results.

    Per channel: `warmup` Vegas iterations to adapt the grid (not counted), then `iters`
    iterations of n events combined with inverse-variance weights."""
    grids = grids or toy_grids()
    prm = prm or params()
    out = {}
    total, var = 0.0, 0.0
    for i, (proc, a, b, mult) in enumerate(CHANNELS[final]):
        vi = VegasIntegrator(proc, precision=precision, n=n, seed=seed + 101 * i, prm=prm, handle=handle,
                             pdf=dict(grid=grids[a], grid_b=grids[b], sqrt_S=sqrt_S))
        if warmup:
            vi.iterate(warmup)
            vi.results = []
        vi.iterate(iters)
        I, sig, chi2 = vi.estimate()
        out[f'{proc} ({a} {b})'] = dict(sigma_pb=mult * I, error_pb=mult * sig, multiplicity=mult, chi2=chi2)
        total += mult * I
        var += (mult * sig) ** 2
    return dict(final=final, sqrt_S=sqrt_S, sigma_pb=total, error_pb=var ** 0.5, channels=out)
