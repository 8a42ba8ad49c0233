"""Unweighting of weighted Monte Carlo events (hit-or-miss).  Test infrastructure only.

An event generator turns the weighted events of the integration into a sample
of unit-weight events (the generators the paper serves, sect. 1).  The paper
does not print the procedure; this is the standard acceptance-rejection
(von Neumann) step:

    event i is kept iff  u_i * w_max < w_i,

with u_i uniform in [0, 1) and w_max a reference maximum of the weights (the
largest weight of the batch unless one is given).  A kept event with
w_i > w_max (possible when w_max is given) carries the weight factor
w_i / w_max, every other kept event the factor 1.  Weights that are not
positive, or NaN, are never kept.  The kept events are listed in increasing
event order.

The acceptance uniform of global event e is drawn from Philox4x32-10 with
key = seed and counter = (e_lo, e_hi, 0, 1): the fourth counter word 1 keeps
this stream apart from the phase-space uniforms (which use 0 there); the first
64-bit output word r1:r0 gives u = (word >> 11) * 2^-53.
"""
import numpy as np

from .philox import MASK32, philox4x32_10


def acceptance_uniforms(seed, n, offset=0):
    """u[n] in [0, 1) for global events offset .. offset + n - 1."""
    ev = np.arange(n, dtype=np.uint64) + np.uint64(offset)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = (ev & MASK32).astype(np.uint32)
    ctr[:, 1] = (ev >> np.uint64(32)).astype(np.uint32)
    ctr[:, 3] = 1
    r = philox4x32_10(ctr, key)
    u0 = (r[:, 1].astype(np.uint64) << np.uint64(32)) | r[:, 0].astype(np.uint64)
    return (u0 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def batch_max(w):
    """Largest weight of the batch (NaN and non-positive weights ignored; 0 if none)."""
    w = np.asarray(w, dtype=np.float64)
    ok = w > 0
    return float(w[ok].max()) if ok.any() else 0.0


def unweight(w, u, w_max):
    """(kept event indices ascending, their weight factors) for weights w, uniforms u."""
    w = np.asarray(w, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    positive = w > 0                       # False for NaN
    kept = np.nonzero(positive & (u * w_max < w))[0].astype(np.int64)
    wk = w[kept]
    fac = np.where(wk > w_max, wk / w_max if w_max > 0 else np.inf, 1.0)
    return kept, fac
