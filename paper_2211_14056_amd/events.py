"""Event output: a unit-weight sample (mf_unweight) written as plain text.

One block per event:

    <event number> <process> <n legs> <weight factor>
    <E> <px> <py> <pz>        (one line per leg: incoming legs first, then outgoing)

preceded by a header line with the process, the number of events, the reference maximum and
the unit weight sigma/N (pb) the caller passes.  Pure host code: it reads the compacted
device buffers once and formats them.
"""


def write_events(path, proc, out, unit_weight_pb=None):
    """Write the kept events of an mf_unweight result dict (idx, fac, p_out, count, w_max)."""
    n = int(out['count'].item())
    cap = out['idx'].shape[0]
    k = min(n, cap)
    idx = out['idx'][:k].cpu().numpy()
    fac = out['fac'][:k].cpu().numpy()
    p = out['p_out'][:, :, :k].cpu().numpy() if out.get('p_out') is not None else None
    with open(path, 'w') as f:
        f.write(f'# process {proc} events {k} w_max {float(out["w_max"].item())!r} '
                f'unit_weight_pb {unit_weight_pb!r}\n')
        for j in range(k):
            legs = 0 if p is None else p.shape[0]
            f.write(f'{int(idx[j])} {proc} {legs} {float(fac[j])!r}\n')
            for leg in range(legs):
                f.write(' '.join(repr(float(v)) for v in p[leg, :, j]) + '\n')
    return k
