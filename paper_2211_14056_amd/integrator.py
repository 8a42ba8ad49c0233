"""Vegas integration driver over the library, with graph-captured iterations.

One Vegas iteration (Vegas iterations are the paper's integrator, sect. 1) is
`batches` launches of
    mf_phase_space -> mf_matrix_element -> mf_vegas_refine
on one stream.  The Philox counter offset lives in device memory: the phase
space reads it and the Vegas reduction advances it by the batch size, so a
captured HIP graph of one iteration (captured by the library, mf_graph_begin /
mf_graph_end) can be replayed iteration after iteration with no host work in
between except reading the two accumulated sums.

With `pdf` the events are hadronic (mf_phase_space_pp: one parton channel of pp at
sqrt_S, parton 1 with density `grid`, parton 2 with `grid_b`), d + 2 dimensions.
"""
import math

import numpy as np
import torch

from . import (Handle, MF_FP64, PROCESS, make_request, mf_graph_begin, mf_graph_end, mf_matrix_element,
               mf_phase_space, mf_phase_space_pp, mf_process_dims, mf_process_legs, mf_vegas_refine, params)


class VegasIntegrator:
    def __init__(self, proc, precision=MF_FP64, n=1_000_000, batches=1, nb=50, alpha=1.5, seed=1, prm=None,
                 handle=None, pdf=None):
        """pdf: None (partonic events at prm.sqrt_s) or dict(grid=PdfGrid, grid_b=PdfGrid or None,
        sqrt_S=collider energy) for hadronic events of one parton channel."""
        self.pid = PROCESS[proc] if isinstance(proc, str) else proc
        self.precision = precision
        self.n, self.batches, self.nb, self.alpha, self.seed = n, batches, nb, alpha, seed
        self.prm = prm or params()
        self.h = handle or Handle()
        self.pdf = pdf
        # the Vegas step forms the flux from sqrt(s): the collider's for hadronic events
        self.vprm = self.prm
        if pdf is not None:
            from . import mf_params
            v = mf_params()
            for f, _ in mf_params._fields_:
                setattr(v, f, getattr(self.prm, f))
            v.sqrt_s = float(pdf['sqrt_S'])
            self.vprm = v
        dev = torch.device('cuda', self.h.device)
        d = mf_process_dims(self.pid) + (2 if pdf is not None else 0)
        self.d = d
        f64 = dict(dtype=torch.float64, device=dev)
        self.p = torch.empty(mf_process_legs(self.pid), 4, n, **f64)
        self.w = torch.empty(n, **f64)
        self.jac = torch.empty(n, **f64)
        self.pass_ = torch.empty(n, dtype=torch.uint8, device=dev)
        self.bins = torch.empty(d, n, dtype=torch.int16, device=dev)
        self.me = torch.empty(n, dtype=torch.float64 if precision == MF_FP64 else torch.float32, device=dev)
        self.edges = torch.tensor(np.tile(np.linspace(0.0, 1.0, nb + 1), (d, 1)), **f64).contiguous()
        self.acc = torch.zeros(2 + d * nb, **f64)
        self.counter = torch.zeros(1, dtype=torch.int64, device=dev)     # Philox event offset
        self.req = [make_request(self.pid, self.p, self.me)]
        self.graph = None
        self.results = []

    def reset(self):
        self.edges.copy_(torch.tensor(np.tile(np.linspace(0.0, 1.0, self.nb + 1), (self.d, 1)),
                                      dtype=torch.float64))
        self.acc.zero_()
        self.counter.zero_()
        self.results = []

    def enqueue_iteration(self):
        """Enqueue one Vegas iteration on the current stream (capturable)."""
        for b in range(self.batches):
            if self.pdf is None:
                mf_phase_space(self.h, self.pid, self.prm, self.n, seed=self.seed, offset=0,
                               offset_dev=self.counter, edges=self.edges, nb=self.nb, p=self.p, w=self.w,
                               pass_=self.pass_, bin_idx=self.bins, jac=self.jac)
            else:
                mf_phase_space_pp(self.h, self.pid, self.prm, self.pdf['sqrt_S'], self.pdf['grid'], self.n,
                                  seed=self.seed, offset=0, offset_dev=self.counter, edges=self.edges, nb=self.nb,
                                  p=self.p, w=self.w, pass_=self.pass_, bin_idx=self.bins, jac=self.jac,
                                  grid_b=self.pdf.get('grid_b'))
            mf_matrix_element(self.h, self.req, self.precision, self.prm)
            mf_vegas_refine(self.h, self.vprm, self.n, self.d, self.nb, self.alpha, self.w, self.jac, self.me,
                            self.pass_, self.bins, self.acc, self.edges, update_edges=(b == self.batches - 1),
                            accumulate=(b > 0), rng_counter=self.counter)

    def _record(self):
        a = self.acc[:2].cpu().numpy()
        N = self.n * self.batches
        I = a[0] / N
        var = (a[1] / N - I * I) / (N - 1)
        self.results.append((I, var))
        return I, var

    def iterate(self, iters):
        """Eager iterations; returns the per-iteration (I, var)."""
        for _ in range(iters):
            self.enqueue_iteration()
            self._record()
        return self.results[-iters:]

    def capture(self):
        """Capture one iteration into a library-owned HIP graph (mf_graph_begin/end; run one
        eager iteration first so the first replay continues the integration)."""
        if not self.results:
            self.iterate(1)
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            mf_graph_begin(self.h, s)
            self.enqueue_iteration()
            self.graph = mf_graph_end(self.h, s)
        torch.cuda.synchronize()
        # capturing does not execute: the state is unchanged
        return self.graph

    def replay(self, iters):
        out = []
        for _ in range(iters):
            self.graph.launch()
            out.append(self._record())
        return out

    def estimate(self):
        Is = np.array([r[0] for r in self.results])
        w = 1.0 / np.array([r[1] for r in self.results])
        I = (Is * w).sum() / w.sum()
        sig = w.sum() ** -0.5
        chi2 = ((Is - I) ** 2 * w).sum() / max(len(Is) - 1, 1)
        return I, sig, chi2
