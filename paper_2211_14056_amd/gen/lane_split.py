"""Four-lanes-per-event form of the gg -> t tbar g g matrix element.

The one-lane-per-event body keeps all 24 colour-ordered partial amplitudes of
an event and every multi-gluon current they need live at once.  In FP64 that
working set is about twice the register file, so it spills.  Here the event is
shared by the four lanes of a quad.

* Lane ``sub`` takes the six orderings whose first gluon is gluon ``sub``.
* The lane relabels the gluons cyclically: its slot j holds gluon
  (j + sub) mod 4.  In slot labels every lane computes the same six orderings
  (0, x, y, z), so the code is the same for all four lanes.  Only the inputs
  (momenta, polarisation bases and helicity bit of each slot) depend on the
  lane.
* A lane needs 25 of the 34 gluon currents and 10 of the 40 quark-line
  prefixes, and holds 6 partial amplitudes per antitop helicity instead of 24.

Colour sum.  The colour matrix is invariant under a simultaneous relabelling
of the gluons, C(pi s, pi t) = C(s, t).  Lane k holds A(rho^k s) for the slot
orderings s, with rho the cyclic shift.  So the block of C between lane k and
lane k+m is C(s, rho^m t) for every k.  Each lane reads the amplitudes of the
lanes k+1 and k+2 of its quad by DPP and sums three pieces:

* its diagonal block (symmetric, upper triangle doubled);
* the block with k+1, doubled (it stands for the blocks k+1 and k-1);
* the block with k+2, once (lane k+2 computes the transposed block).

The four lanes together give exactly the full quadratic form.

Helicities.  As in the one-lane body, only the configurations in which gluon
k-1 (an actual gluon, not a slot) has helicity +1 are evaluated; their reverses
give the same colour-summed |M|^2 and are accounted for by a factor 2 in the
normalisation.
"""
import itertools
import math

from .ir import Block, C, S, ZERO, const, csum, cmat
from .process_compiler import SQRT1_2, GGTTProcess, Momentum, Recursion, assign_lds_slots, _sname


def rotate(t, m, k):
    """Relabel the ordering ``t`` by the cyclic shift g -> g + m (mod k)."""
    return tuple((x + m) % k for x in t)


def lane_orderings(proc):
    return [s for s in proc.orderings if s[0] == 0]


def needed_currents(orderings):
    """Canonical multi-gluon currents used by the quark lines of ``orderings`` (longest first)."""
    need = set()
    for s in orderings:
        for i in range(len(s)):
            for j in range(i + 2, len(s) + 1):
                need.add(Recursion.canon(s[i:j]))
    return sorted(need, key=lambda r: (-len(r), r))


def shared_currents(k, need):
    """Currents each lane computes itself when the quad shares the gluon currents.

    Lane k holds the actual current rho^k(c) under the slot label c, so the four
    lanes computing the slot current t produce the whole orbit {rho^m(t)}.  One
    representative per orbit of every multi-gluon current is therefore enough.
    Each lane computes the representatives, and reads every other current c as
    J(t) of the lane M places further in the quad, with
    canon(rho^m(c)) = t and M = -m mod k.
    Returns (own set, remote map c -> (t, M, sign))."""
    canon = Recursion.canon
    own, remote = set(), {}
    for r in range(2, k + 1):
        classes = sorted({canon(c) for S_ in itertools.combinations(range(k), r)
                          for c in itertools.permutations(S_)})
        seen = set()
        for c in sorted(classes, key=lambda c: (c not in need, c)):
            orbit = frozenset(canon(rotate(c, m, k)) for m in range(k))
            if orbit in seen:
                continue
            seen.add(orbit)
            own.add(c)
        for c in classes:
            if c in own:
                continue
            for m in range(1, k):
                t = rotate(c, m, k)
                if canon(t) in own:
                    sign = 1 if canon(t) == t else (-1) ** (len(c) + 1)
                    remote[c] = (canon(t), (-m) % k, sign)
                    break
    return own, remote


def emit_split(proc, lds_budget, opaque_inputs=True, group_barriers=True, stream=True, local_memo=False,
               share=True):
    """Source text and flop counts of me_<name>_split (four lanes per event)."""
    k = proc.k
    assert k == 4, 'the quad split is laid out for four gluons'
    fn = f'me_{proc.name}_split'
    mine = lane_orderings(proc)
    index = {s: i for i, s in enumerate(proc.orderings)}
    out = [f'// ---- {proc.name}, four lanes per event: lane sub takes the {len(mine)} orderings that start '
           f'with gluon sub; slot j holds gluon (j + sub) mod 4']
    out.append('template <typename R, typename KT, typename Sink>')
    out.append(f'__device__ __forceinline__ void {fn}(const KT (&kin)[4][4], const KT (&pt)[4], const KT (&ptb)[4], '
               'const R (&eu)[4][3], const R (&ew)[4][2], const int (&hb)[4], const KT mt, Sink& sink, '
               'R* __restrict__ lds)')
    out.append('{')
    pro = []
    pro.append('const KT mt2 = mt * mt;')
    for sub in proc.gluon_subsets():
        n = _sname(sub)
        terms = ' + '.join(f'kin[{i}][c]' for i in sub)
        pro.append(f'KT P{n}[4]; for (int c = 0; c < 4; ++c) P{n}[c] = {terms};')
        pro.append(f'const R ig{n} = cvt<R>(KT(1.0) / (P{n}[0] * P{n}[0] - P{n}[1] * P{n}[1] - '
                   f'P{n}[2] * P{n}[2] - P{n}[3] * P{n}[3]));')
    qsubs = sorted({tuple(sorted(s[:i])) for s in mine for i in range(1, k)}, key=lambda t: (len(t), t))
    for sub in qsubs:
        n = _sname(sub)
        terms = ' - '.join(['pt[c]'] + [f'kin[{i}][c]' for i in sub])
        pro.append(f'KT q{n}[4]; for (int c = 0; c < 4; ++c) q{n}[c] = {terms};')
        pro.append(f'const R iq{n} = cvt<R>(KT(1.0) / ((q{n}[0] - q{n}[3]) * (q{n}[0] + q{n}[3]) - '
                   f'q{n}[1] * q{n}[1] - q{n}[2] * q{n}[2] - mt2));')
    for j in range(k):
        pro.append(f'R K{j}[4] = {{cvt<R>(kin[{j}][0]), cvt<R>(kin[{j}][1]), cvt<R>(kin[{j}][2]), '
                   f'cvt<R>(kin[{j}][3])}};')
    pro.append('R PT[4] = {cvt<R>(pt[0]), cvt<R>(pt[1]), cvt<R>(pt[2]), cvt<R>(pt[3])};')
    pro.append('const R MT = cvt<R>(mt);')
    pro.append('cplx<R> ub[2][4], vs[2][4];')
    pro.append('ubar_spinor<R, KT>(pt, mt, -1, ub[0]); ubar_spinor<R, KT>(pt, mt, 1, ub[1]);')
    pro.append('v_spinor<R, KT>(ptb, mt, -1, vs[0]); v_spinor<R, KT>(ptb, mt, 1, vs[1]);')
    out += ['    ' + l for l in pro]

    # ---------------- gluon currents (per gluon-helicity configuration) ----------------
    b = Block('t')
    moms = [Momentum(b, [S(name=f'K{j}[{c}]') for c in range(4)]) for j in range(k)]
    eps = []
    for j in range(k):
        # every slot in the general form (-l u + i w); the caller flips w for incoming gluons
        ux, uy, uz = (S(name=f'eu[{j}][{c}]') for c in range(3))
        wx, wy = (S(name=f'ew[{j}][{c}]') for c in range(2))
        l = S(name=f'lam{j}')
        ez = b.mul(b.neg(l), uz)
        tr = b.sumprod([(l, b.neg(ux))], b.neg(wy))
        ti = b.sumprod([(l, b.neg(uy))], wx)
        tbr = b.sumprod([(l, b.neg(ux))], wy)
        tbi = b.sumprod([(l, uy)], wx)
        eps.append([C(ez), C(b.neg(ez)), C(tr, ti), C(tbr, tbi)])
    need = needed_currents(mine)
    lds_slot = assign_lds_slots(need, lds_budget)
    remote = None
    if share:
        own, far = shared_currents(k, set(need))
        remote = far.get
    rec = Recursion(b, moms, eps, lds_slot, stream=stream, local_memo=local_memo, remote=remote)
    for r in range(2, k + 1):
        for cur in need:
            if len(cur) == r:
                rec.J(cur)
    gluon_flops, gluon_lines = b.flops, b.lines

    # ---------------- quark line (per top helicity) ----------------
    q = Block('u')
    ub = [C(S(name=f'ubs[{j}].re'), S(name=f'ubs[{j}].im')) for j in range(4)]
    qmoms = [Momentum(q, [S(name=f'K{j}[{c}]') for c in range(4)]) for j in range(k)]
    rec.start_quark_line(q, qmoms, ub)
    vspin = [[C(S(name=f'vs[{h}][{j}].re'), S(name=f'vs[{h}][{j}].im')) for j in range(4)] for h in range(2)]
    amps = [[None] * len(mine) for _ in range(2)]
    prev = None
    for si, sigma in enumerate(mine):
        if group_barriers and prev is not None and sigma[1] != prev:
            q.lines.append('__builtin_amdgcn_sched_barrier(0);')
        prev = sigma[1]
        full = rec.closing(sigma)
        for h in range(2):
            amps[h][si] = cmat(q, csum(q, [(full[c], vspin[h][c]) for c in range(4)]))
    quark_flops = q.flops

    # ---------------- colour: own block, lane k+1 (doubled), lane k+2 ----------------
    cs = Block('w')
    n = len(mine)
    tot = []
    for h in range(2):
        A = amps[h]
        R1 = [C(cs.new(f'quad_rot<1>({cs.ref(a.re)})', 0), cs.new(f'quad_rot<1>({cs.ref(a.im)})', 0)) for a in A]
        R2 = [C(cs.new(f'quad_rot<2>({cs.ref(a.re)})', 0), cs.new(f'quad_rot<2>({cs.ref(a.im)})', 0)) for a in A]
        terms = []
        for i, s in enumerate(mine):
            row = []
            for j in range(i, n):
                c = proc.cnum[index[s]][index[mine[j]]]
                row.append((c if j == i else 2 * c, A[j]))
            for j, t in enumerate(mine):
                row.append((2 * proc.cnum[index[s]][index[rotate(t, 1, k)]], R1[j]))
                row.append((proc.cnum[index[s]][index[rotate(t, 2, k)]], R2[j]))
            y_r = cs.sumprod([(const(c), x.re) for c, x in row])
            y_i = cs.sumprod([(const(c), x.im) for c, x in row])
            terms += [(A[i].re, y_r), (A[i].im, y_i)]
        tot.append(cs.sumprod(terms))
    colour_flops = cs.flops

    body = []
    opq = []
    if opaque_inputs:
        opq = [f'opaque(K{j}[{c}]);' for j in range(k) for c in range(4)] + [f'opaque(PT[{c}]);' for c in range(4)]
    body.append('#pragma unroll 1')
    body.append(f'for (int gconf = {2 ** (k - 1)}; gconf < {2 ** k}; ++gconf) {{   // gluon {k - 1}: helicity +1')
    body += ['    ' + l for l in opq]
    for j in range(k):
        body.append(f'    const R lam{j} = (gconf >> hb[{j}]) & 1 ? R(1) : R(-1);')
    body += ['    ' + l for l in gluon_lines]
    body.append('    #pragma unroll 1')
    body.append('    for (int ht = 0; ht < 2; ++ht) {')
    body += ['        ' + l for l in opq]
    if group_barriers:
        body.append('        __builtin_amdgcn_sched_barrier(0);')
    body.append('        cplx<R> ubs[4];')
    body.append('        for (int j = 0; j < 4; ++j) ubs[j] = ht ? ub[1][j] : ub[0][j];')
    body += ['        ' + l for l in q.lines]
    body += ['        ' + l for l in cs.lines]
    body.append(f'        sink.add({cs.ref(tot[0])}, {cs.ref(tot[1])});')
    body.append('    }')
    body.append('}')
    out += ['    ' + l for l in body]
    out.append('}')
    per_lane = (2 ** (k - 1)) * (gluon_flops + 2 * (quark_flops + colour_flops))
    info = dict(lds_slots=8 * len(lds_slot), currents=len(need), gluon_per_gconf=gluon_flops,
                quark_per_top_hel=quark_flops, colour_per_top_hel=colour_flops,
                executed_per_event=4 * per_lane)
    return '\n'.join(out), info


# ---------------------------------------------------------------------------
# Two lanes per event.
#
# The relabelling is the involution sigma = (0 1)(2 3): it swaps the two beam
# gluons and the two final gluons, so in both lanes slots 0 and 1 hold beams
# (their momenta keep the zero x, y components) and slots 2 and 3 final
# gluons.  Lane sub holds gluon sigma^sub(j) in slot j.  sigma has no fixed
# ordering, so the 24 orderings fall into 12 pairs {s, sigma(s)}; each lane
# takes, in slot labels, the 12 orderings that start with gluon 0 or 2.
# Currents: lane sub needs J(sigma^sub(c)) under slot label c, which the other
# lane holds under the slot label sigma(c); one representative per orbit
# {c, sigma(c)} is computed and the other read from the partner by DPP.
# Colour: C(sigma s, sigma t) = C(s, t), so with A_own(s) and A_partner(t) in
# slot labels each lane adds its own 12 x 12 block and the cross block
# C(s, sigma t) once; over the two lanes that is the whole quadratic form.

def sigma(g):
    return g ^ 1


def pair_orderings(proc):
    return [s for s in proc.orderings if s[0] in (0, 2)]


def pair_shared_currents(k, need):
    """(own set, remote map c -> (t, 1, sign)) for the two-lane form (see above)."""
    canon = Recursion.canon
    own, remote = set(), {}
    for r in range(2, k + 1):
        classes = sorted({canon(c) for S_ in itertools.combinations(range(k), r)
                          for c in itertools.permutations(S_)})
        done = set()
        for c in sorted(classes, key=lambda c: (c not in need, c)):
            if c in done:
                continue
            t_raw = tuple(sigma(g) for g in c)
            t = canon(t_raw)
            done |= {c, t}
            own.add(c)
            if t != c:
                sign = 1 if t == t_raw else (-1) ** (len(c) + 1)
                remote[t] = (c, 1, sign)
    return own, remote


def emit_pair(proc, lds_budget, opaque_inputs=True, group_barriers=True, stream=True, local_memo=False,
              share_products=False):
    """Source text and flop counts of me_<name>_pair (two lanes per event)."""
    k = proc.k
    assert k == 4, 'the pair split is laid out for four gluons'
    fn = f'me_{proc.name}_pair'
    mine = pair_orderings(proc)
    index = {s: i for i, s in enumerate(proc.orderings)}
    out = [f'// ---- {proc.name}, two lanes per event: slot j of lane sub holds gluon j ^ sub; each lane '
           f'takes the {len(mine)} orderings that start with slot 0 or 2']
    out.append('template <typename R, typename KT, typename Sink>')
    out.append(f'__device__ __forceinline__ void {fn}(const KT (&kin)[4][4], const KT (&pt)[4], const KT (&ptb)[4], '
               'const R (&eu)[2][3], const R (&ew)[2][2], const R (&zs)[2], const int (&hb)[4], const KT mt, '
               'Sink& sink, R* __restrict__ lds)')
    out.append('{')
    pro = ['const KT mt2 = mt * mt;']
    for sub in proc.gluon_subsets():
        n = _sname(sub)
        terms = ' + '.join(f'kin[{i}][c]' for i in sub)
        pro.append(f'KT P{n}[4]; for (int c = 0; c < 4; ++c) P{n}[c] = {terms};')
        pro.append(f'const R ig{n} = cvt<R>(KT(1.0) / (P{n}[0] * P{n}[0] - P{n}[1] * P{n}[1] - '
                   f'P{n}[2] * P{n}[2] - P{n}[3] * P{n}[3]));')
    qsubs = sorted({tuple(sorted(s[:i])) for s in mine for i in range(1, k)}, key=lambda t: (len(t), t))
    for sub in qsubs:
        n = _sname(sub)
        terms = ' - '.join(['pt[c]'] + [f'kin[{i}][c]' for i in sub])
        pro.append(f'KT q{n}[4]; for (int c = 0; c < 4; ++c) q{n}[c] = {terms};')
        pro.append(f'const R iq{n} = cvt<R>(KT(1.0) / ((q{n}[0] - q{n}[3]) * (q{n}[0] + q{n}[3]) - '
                   f'q{n}[1] * q{n}[1] - q{n}[2] * q{n}[2] - mt2));')
    for j in range(k):
        pro.append(f'R K{j}[4] = {{cvt<R>(kin[{j}][0]), cvt<R>(kin[{j}][1]), cvt<R>(kin[{j}][2]), '
                   f'cvt<R>(kin[{j}][3])}};')
    pro.append('R PT[4] = {cvt<R>(pt[0]), cvt<R>(pt[1]), cvt<R>(pt[2]), cvt<R>(pt[3])};')
    pro.append('const R MT = cvt<R>(mt);')
    pro.append('cplx<R> ub[2][4], vs[2][4];')
    pro.append('ubar_spinor<R, KT>(pt, mt, -1, ub[0]); ubar_spinor<R, KT>(pt, mt, 1, ub[1]);')
    pro.append('v_spinor<R, KT>(ptb, mt, -1, vs[0]); v_spinor<R, KT>(ptb, mt, 1, vs[1]);')
    out += ['    ' + l for l in pro]

    # ---------------- gluon currents (per gluon-helicity configuration) ----------------
    b = Block('t')
    moms = []
    for j in range(k):
        if j < 2:
            # beam slot: k = (E, 0, 0, zs E), zs = +1 for gluon 0, -1 for gluon 1
            E = S(name=f'K{j}[0]')
            moms.append(Momentum(b, [E, ZERO, ZERO, S(name=f'K{j}[3]')]))
        else:
            moms.append(Momentum(b, [S(name=f'K{j}[{c}]') for c in range(4)]))
    eps = []
    for j in range(k):
        if j < 2:
            # eps of a beam along zs z with helicity l: t = (1 - zs l)/sqrt2, tb = -(1 + zs l)/sqrt2
            lz = S(name=f'lz{j}')
            t = b.sumprod([(lz, const(-SQRT1_2))], const(SQRT1_2))
            tb = b.sumprod([(lz, const(-SQRT1_2))], const(-SQRT1_2))
            eps.append([C(ZERO), C(ZERO), C(t), C(tb)])
        else:
            ux, uy, uz = (S(name=f'eu[{j - 2}][{c}]') for c in range(3))
            wx, wy = (S(name=f'ew[{j - 2}][{c}]') for c in range(2))
            l = S(name=f'lam{j}')
            ez = b.mul(b.neg(l), uz)
            tr = b.sumprod([(l, b.neg(ux))], b.neg(wy))
            ti = b.sumprod([(l, b.neg(uy))], wx)
            tbr = b.sumprod([(l, b.neg(ux))], wy)
            tbi = b.sumprod([(l, uy)], wx)
            eps.append([C(ez), C(b.neg(ez)), C(tr, ti), C(tbr, tbi)])
    need = needed_currents(mine)
    lds_slot = assign_lds_slots(need, lds_budget)
    own, far = pair_shared_currents(k, set(need))
    rec = Recursion(b, moms, eps, lds_slot, stream=stream, local_memo=local_memo, remote=far.get,
                    exchange='pair_swap')
    for r in range(2, k + 1):
        for cur in need:
            if len(cur) == r:
                rec.J(cur)
    gluon_flops, gluon_lines = b.flops, b.lines

    # ---------------- quark line (per top helicity) ----------------
    q = Block('u')
    ub = [C(S(name=f'ubs[{j}].re'), S(name=f'ubs[{j}].im')) for j in range(4)]
    qmoms = []
    for j in range(k):
        if j < 2:
            qmoms.append(Momentum(q, [S(name=f'K{j}[0]'), ZERO, ZERO, S(name=f'K{j}[3]')]))
        else:
            qmoms.append(Momentum(q, [S(name=f'K{j}[{c}]') for c in range(4)]))
    rec.start_quark_line(q, qmoms, ub, mine, share_products)
    vspin = [[C(S(name=f'vs[{h}][{j}].re'), S(name=f'vs[{h}][{j}].im')) for j in range(4)] for h in range(2)]
    amps = [[None] * len(mine) for _ in range(2)]
    prev = None
    for si, sg in enumerate(mine):
        if group_barriers and prev is not None and sg[0] != prev:
            q.lines.append('__builtin_amdgcn_sched_barrier(0);')
        prev = sg[0]
        full = rec.closing(sg)
        for h in range(2):
            amps[h][si] = cmat(q, csum(q, [(full[c], vspin[h][c]) for c in range(4)]))
    quark_flops = q.flops

    # ---------------- colour: own block + cross block with the partner ----------------
    cs = Block('w')
    n = len(mine)
    tot = []
    for h in range(2):
        A = amps[h]
        X = [C(cs.new(f'pair_swap({cs.ref(a.re)})', 0), cs.new(f'pair_swap({cs.ref(a.im)})', 0)) for a in A]
        terms = []
        for i, s_ in enumerate(mine):
            row = []
            for j in range(i, n):
                c = proc.cnum[index[s_]][index[mine[j]]]
                row.append((c if j == i else 2 * c, A[j]))
            for j, t in enumerate(mine):
                c = proc.cnum[index[s_]][index[tuple(sigma(g) for g in t)]]
                row.append((c, X[j]))
            y_r = cs.sumprod([(const(c), x.re) for c, x in row if c != 0])
            y_i = cs.sumprod([(const(c), x.im) for c, x in row if c != 0])
            terms += [(A[i].re, y_r), (A[i].im, y_i)]
        tot.append(cs.sumprod(terms))
    colour_flops = cs.flops

    body = []
    opq = []
    if opaque_inputs:
        opq = [f'opaque(K{j}[{c}]);' for j in range(k) for c in range(4)] + [f'opaque(PT[{c}]);' for c in range(4)]
    body.append('#pragma unroll 1')
    body.append(f'for (int gconf = {2 ** (k - 1)}; gconf < {2 ** k}; ++gconf) {{   // gluon {k - 1}: helicity +1')
    body += ['    ' + l for l in opq]
    for j in range(k):
        lam = f'((gconf >> hb[{j}]) & 1 ? R(1) : R(-1))'
        if j < 2:
            body.append(f'    const R lz{j} = zs[{j}] * {lam};')
        else:
            body.append(f'    const R lam{j} = {lam};')
    body += ['    ' + l for l in gluon_lines]
    body.append('    #pragma unroll 1')
    body.append('    for (int ht = 0; ht < 2; ++ht) {')
    body += ['        ' + l for l in opq]
    if group_barriers:
        body.append('        __builtin_amdgcn_sched_barrier(0);')
    body.append('        cplx<R> ubs[4];')
    body.append('        for (int j = 0; j < 4; ++j) ubs[j] = ht ? ub[1][j] : ub[0][j];')
    body += ['        ' + l for l in q.lines]
    body += ['        ' + l for l in cs.lines]
    body.append(f'        sink.add({cs.ref(tot[0])}, {cs.ref(tot[1])});')
    body.append('    }')
    body.append('}')
    out += ['    ' + l for l in body]
    out.append('}')
    per_lane = (2 ** (k - 1)) * (gluon_flops + 2 * (quark_flops + colour_flops))
    info = dict(lds_slots=8 * len(lds_slot), currents=len(need), own=len([c for c in need if c in own]),
                gluon_per_gconf=gluon_flops, quark_per_top_hel=quark_flops, colour_per_top_hel=colour_flops,
                executed_per_event=2 * per_lane)
    return '\n'.join(out), info
