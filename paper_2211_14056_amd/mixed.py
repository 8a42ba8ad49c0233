"""The mixed persistent batch as one Vegas iteration, captured in one library graph.

A serving-style workload of the event-parallel generator (the paper's event
axis, sect. 1; block and grid choices, sect. 3, Fig. 3): 64 requests over
{gg -> ttbar, gg -> ttbar g, gg -> ttbar gg} with log-uniform event counts
(workloads.mixed_batch).  One iteration is

  * mf_phase_space for every request, on its process's Vegas grid, with Philox
    offsets (a per-process device counter plus the request's fixed position
    among the process's requests);
  * ONE mf_matrix_element call over all 64 requests (one persistent or grid
    launch per process class);
  * ONE mf_matrix_element_vjp call over the gg -> ttbar gg requests (one launch,
    a grid of 64-event tiles over them): d|M|^2/dx and d|M|^2/d(m_t, alpha_s),
    cotangent 1 per event;
  * mf_vegas_refine per request, accumulating into its process's sums; the last
    request of a process refines that process's grid and every call advances
    the process's counter.

capture() records the iteration with mf_graph_begin/mf_graph_end (the library
owns the graph); launch() replays it with no host work.
"""
import numpy as np
import torch

from . import (Handle, MF_FP32_MFMA_BF16, MF_FP64, PROCESS, make_request, mf_graph_begin, mf_graph_end,
               mf_matrix_element, mf_matrix_element_vjp, mf_phase_space, mf_process_dims, mf_process_legs,
               mf_vegas_refine, params)
from .workloads import mixed_batch

PROCS = ('gg_tt', 'gg_ttg', 'gg_ttgg')


class MixedIteration:
    def __init__(self, spec=None, precision=MF_FP32_MFMA_BF16, nb=50, alpha=1.5, seed=7, prm=None, handle=None,
                 vjp_proc='gg_ttgg'):
        self.spec = spec if spec is not None else mixed_batch(64, seed=5)
        self.precision = precision
        self.nb, self.alpha, self.seed = nb, alpha, seed
        self.prm = prm or params()
        self.h = handle or Handle()
        dev = torch.device('cuda', self.h.device)
        f64 = dict(dtype=torch.float64, device=dev)
        me_dt = torch.float64 if precision == MF_FP64 else torch.float32
        self.edges, self.acc, self.counter = {}, {}, {}
        for proc in PROCS:
            d = mf_process_dims(PROCESS[proc])
            self.edges[proc] = torch.tensor(np.tile(np.linspace(0.0, 1.0, nb + 1), (d, 1)), **f64).contiguous()
            self.acc[proc] = torch.zeros(2 + d * nb, **f64)
            self.counter[proc] = torch.zeros(1, dtype=torch.int64, device=dev)
        self.reqs = []
        placed = {p: 0 for p in PROCS}
        for i, (proc, n) in enumerate(self.spec):
            pid = PROCESS[proc]
            d = mf_process_dims(pid)
            r = dict(proc=proc, pid=pid, n=n, d=d, offset=placed[proc],
                     p=torch.empty(mf_process_legs(pid), 4, n, **f64), w=torch.empty(n, **f64),
                     jac=torch.empty(n, **f64), pass_=torch.empty(n, dtype=torch.uint8, device=dev),
                     bins=torch.empty(d, n, dtype=torch.int16, device=dev),
                     me=torch.empty(n, dtype=me_dt, device=dev))
            placed[proc] += n
            if proc == vjp_proc:
                r['x'] = torch.empty(d, n, **f64)
                r['gbar'] = torch.ones(n, **f64)
                r['gx'] = torch.empty(d, n, **f64)
                r['gth'] = torch.empty(n, 2, **f64)
            self.reqs.append(r)
        self.total = dict(placed)
        self.me_reqs = [make_request(r['pid'], r['p'], r['me']) for r in self.reqs]
        self.vjp_reqs = [make_request(r['pid'], None, None, x=r['x'], grad_me=r['gbar'], grad_x=r['gx'],
                                      grad_theta=r['gth'], n=r['n']) for r in self.reqs if 'x' in r]
        self.vjp_proc = vjp_proc
        self.last = {}
        for i, r in enumerate(self.reqs):
            self.last[r['proc']] = i
        self.graph = None

    def enqueue(self):
        """Enqueue one iteration on the current stream (capturable)."""
        for r in self.reqs:
            proc = r['proc']
            mf_phase_space(self.h, r['pid'], self.prm, r['n'], seed=self.seed + r['pid'], offset=r['offset'],
                           offset_dev=self.counter[proc], edges=self.edges[proc], nb=self.nb, p=r['p'], w=r['w'],
                           pass_=r['pass_'], bin_idx=r['bins'], jac=r['jac'], x_out=r.get('x'))
        mf_matrix_element(self.h, self.me_reqs, self.precision, self.prm)
        if self.vjp_reqs:
            mf_matrix_element_vjp(self.h, self.vjp_reqs, self.precision, self.prm, edges=self.edges[self.vjp_proc],
                                  nb=self.nb)
        first = set()
        for i, r in enumerate(self.reqs):
            proc = r['proc']
            mf_vegas_refine(self.h, self.prm, r['n'], r['d'], self.nb, self.alpha, r['w'], r['jac'], r['me'],
                            r['pass_'], r['bins'], self.acc[proc], self.edges[proc],
                            update_edges=(i == self.last[proc]), accumulate=(proc in first),
                            rng_counter=self.counter[proc])
            first.add(proc)

    def capture(self):
        """Record one iteration in a library-owned graph (nothing runs while capturing)."""
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            mf_graph_begin(self.h, s)
            self.enqueue()
            self.graph = mf_graph_end(self.h, s)
        torch.cuda.synchronize()
        return self.graph

    def launch(self):
        self.graph.launch()

    def state(self):
        """Copies of the per-process sums and grids and of the derivative outputs."""
        out = {f'acc_{p}': self.acc[p].clone() for p in PROCS}
        out.update({f'edges_{p}': self.edges[p].clone() for p in PROCS})
        for i, r in enumerate(self.reqs):
            if 'x' in r:
                out[f'gx_{i}'] = r['gx'].clone()
                out[f'gth_{i}'] = r['gth'].clone()
        return out

    def events(self):
        return sum(n for _, n in self.spec)
