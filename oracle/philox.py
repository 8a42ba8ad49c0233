"""Philox4x32-10 counter-based generator, written from its published definition.

Test infrastructure only (see ``oracle/__init__``).

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11, sect. 3.2 (Philox S-box: two
32x32->64 multiplications per round, xor with the key, key bumped by the Weyl
constants between rounds; 10 rounds for Philox4x32).

Stream layout used by the Monte Carlo (the paper only says that events are
independent and drawn in parallel, sect. 1):
    key     = (seed & 0xffffffff, seed >> 32)
    counter = (event & 0xffffffff, event >> 32, block, 0)
where ``event`` is the global event index (``offset`` + local index) and
``block`` = dimension // 2.  The four 32-bit outputs (r0, r1, r2, r3) give two
64-bit words u0 = r1<<32 | r0 and u1 = r3<<32 | r2; dimension 2*block uses u0
and 2*block+1 uses u1, each mapped to (u >> 11) * 2**-53 in [0, 1).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)


def _mulhilo(a, b):
    """32x32 -> (hi, lo) 32-bit halves of the 64-bit product."""
    prod = a.astype(np.uint64) * b
    return (prod >> np.uint64(32)).astype(np.uint32), (prod & MASK32).astype(np.uint32)


def philox4x32_10(counter, key):
    """Philox4x32 with 10 rounds.

    counter: uint32 array [..., 4]; key: uint32 array broadcastable to [..., 2].
    Returns uint32 array [..., 4].
    """
    c = np.asarray(counter, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    x0, x1, x2, x3 = (c[..., i].copy() for i in range(4))
    k0 = np.broadcast_to(k[..., 0], x0.shape).astype(np.uint32)
    k1 = np.broadcast_to(k[..., 1], x0.shape).astype(np.uint32)
    for r in range(10):
        if r > 0:
            k0 = (k0.astype(np.uint64) + np.uint64(W0)).astype(np.uint64) & MASK32
            k1 = (k1.astype(np.uint64) + np.uint64(W1)).astype(np.uint64) & MASK32
            k0 = k0.astype(np.uint32)
            k1 = k1.astype(np.uint32)
        hi0, lo0 = _mulhilo(x0, M0)
        hi1, lo1 = _mulhilo(x2, M1)
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return np.stack([x0, x1, x2, x3], axis=-1)


def uniforms(seed, n, d, offset=0):
    """x[d][n] in [0,1), float64, for global events offset .. offset+n-1."""
    ev = np.arange(n, dtype=np.uint64) + np.uint64(offset)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)
    out = np.empty((d, n), dtype=np.float64)
    for b in range((d + 1) // 2):
        ctr = np.zeros((n, 4), dtype=np.uint32)
        ctr[:, 0] = (ev & MASK32).astype(np.uint32)
        ctr[:, 1] = (ev >> np.uint64(32)).astype(np.uint32)
        ctr[:, 2] = b
        r = philox4x32_10(ctr, key)
        u0 = (r[:, 1].astype(np.uint64) << np.uint64(32)) | r[:, 0].astype(np.uint64)
        u1 = (r[:, 3].astype(np.uint64) << np.uint64(32)) | r[:, 2].astype(np.uint64)
        for j, u in enumerate((u0, u1)):
            dim = 2 * b + j
            if dim < d:
                out[dim] = (u >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return out
