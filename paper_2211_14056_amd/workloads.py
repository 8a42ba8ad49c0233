"""Seeded synthetic workload descriptions (no physics arithmetic here).

The mixed persistent batch: 64 requests, each a process drawn uniformly from
{gg -> ttbar, gg -> ttbar g, gg -> ttbar gg} and an event count drawn
log-uniformly from that process's range, from numpy's PCG64 generator.
"""
import math

import numpy as np

MIXED_RANGES = {'gg_tt': (1e3, 1e6), 'gg_ttg': (1e4, 4e6), 'gg_ttgg': (1e4, 1e6)}


def mixed_batch(n_requests=64, seed=5, scale=1.0):
    """[(process, n_events)]; `scale` shrinks the counts for small test runs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    procs = list(MIXED_RANGES)
    out = []
    for _ in range(n_requests):
        proc = procs[int(rng.integers(0, len(procs)))]
        lo, hi = MIXED_RANGES[proc]
        n = int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi))) * scale))
        out.append((proc, max(n, 1)))
    return out
