"""Tables for the table-driven Berends-Giele kernel (processes too large for straight-line code).

For g g -> t tbar + (k-2) g with k gluons the colour-ordered recursion is the one of
``process_compiler`` (same vertex forms, same quark line, same colour matrix), but instead of
unrolling it per event into straight-line code, the kernel walks these tables with one
wavefront per event, the lanes of the wave taking the independent nodes of one level:

  currents   id 0..k-1 the external gluons; then every canonical ordered multi-gluon
             current, by length.  Each lists its three-vertex splits (a, b) and
             four-vertex splits (a, b, c) as current ids with reflection signs
             (J(reversed rho) = (-1)^(|rho|+1) J(rho)), and its gluon subset (mask) for the
             momentum sum and propagator.
  prefixes   id 0 is the bare spinor ubar(p_t); then every ordered sequence of distinct
             gluons shorter than k, by length.  Row spinor Q(prefix) = [sum over splits
             prefix = (pre, blk) of Q(pre) Jslash(blk)] S(p_t - P(prefix)).
  orderings  the k! orderings in the order of the colour matrix; the closing row spinor
             sum over splits sigma = (pre, blk) of Q(pre) Jslash(blk), contracted with v.

Everything is emitted as constant arrays for the kernel and returned as Python lists for
the host tests.
"""
import itertools

from . import colour_algebra


def canon(rho):
    return rho if rho[0] < rho[-1] or len(rho) == 1 else tuple(reversed(rho))


def build(k):
    gl = list(range(k))
    cur = {}                 # canonical rho -> id
    order = []
    for g in gl:
        cur[(g,)] = len(order)
        order.append((g,))
    levels = [(0, k)]
    for r in range(2, k + 1):
        start = len(order)
        for S in itertools.combinations(gl, r):
            for perm in itertools.permutations(S):
                if canon(perm) == perm:
                    cur[perm] = len(order)
                    order.append(perm)
        levels.append((start, len(order)))

    def jref(rho):
        c = canon(rho)
        return cur[c], (1 if c == rho else (-1) ** (len(rho) + 1))

    def mask(rho):
        m = 0
        for g in rho:
            m |= 1 << g
        return m

    currents = []
    for rho in order:
        s3, s4 = [], []
        if len(rho) > 1:
            for s in range(1, len(rho)):
                a, b = rho[:s], rho[s:]
                ia, sa = jref(a)
                ib, sb = jref(b)
                s3.append((ia, sa, ib, sb, mask(a), mask(b)))
            for s1 in range(1, len(rho) - 1):
                for s2 in range(s1 + 1, len(rho)):
                    a, b, c = rho[:s1], rho[s1:s2], rho[s2:]
                    ia, sa = jref(a)
                    ib, sb = jref(b)
                    ic, sc = jref(c)
                    s4.append((ia, sa, ib, sb, ic, sc))
        currents.append(dict(rho=rho, mask=mask(rho), s3=s3, s4=s4))

    pre = {(): 0}
    porder = [()]
    plevels = [(0, 1)]
    for L in range(1, k):
        start = len(porder)
        for seq in itertools.permutations(gl, L):
            pre[seq] = len(porder)
            porder.append(seq)
        plevels.append((start, len(porder)))
    prefixes = []
    for seq in porder:
        splits = []
        for s in range(len(seq)):
            jid, js = jref(seq[s:])
            splits.append((pre[seq[:s]], jid, js))
        prefixes.append(dict(seq=seq, mask=mask(seq), splits=splits))
    orderings = []
    for sigma in colour_algebra.orderings(k):
        splits = []
        for s in range(k):
            jid, js = jref(sigma[s:])
            splits.append((pre[sigma[:s]], jid, js))
        orderings.append(dict(sigma=sigma, splits=splits))
    C, den = colour_algebra.integer_form(colour_algebra.colour_matrix(k))
    return dict(k=k, currents=currents, levels=levels, prefixes=prefixes, plevels=plevels,
                orderings=orderings, cnum=C, cden=den)


def emit(k, name):
    """C++ constant tables for k gluons under the prefix ``name``."""
    t = build(k)
    cu, pr, od = t['currents'], t['prefixes'], t['orderings']
    n3 = max(len(c['s3']) for c in cu)
    n4 = max(max(len(c['s4']) for c in cu), 1)
    L = [f'// tables of the table-driven recursion, {k} gluons: {len(cu)} currents, {len(pr)} prefixes, '
         f'{len(od)} orderings',
         f'constexpr int {name}_k = {k};',
         f'constexpr int {name}_ncur = {len(cu)};',
         f'constexpr int {name}_npre = {len(pr)};',
         f'constexpr int {name}_nord = {len(od)};',
         f'constexpr int {name}_cden = {t["cden"]};',
         f'static __constant__ const short {name}_cur_levels[{k + 1}] = {{'
         + ', '.join(str(a) for a, _ in t['levels']) + f', {t["levels"][-1][1]}}};',
         f'static __constant__ const short {name}_pre_levels[{k + 1}] = {{'
         + ', '.join(str(a) for a, _ in t['plevels']) + f', {t["plevels"][-1][1]}}};']
    # current tables: mask, number of splits; splits packed as
    # s3: (ia, ib, maskA, maskB, signs) and s4: (ia, ib, ic, signs)
    L.append(f'static __constant__ const unsigned char {name}_cur_mask[{len(cu)}] = {{'
             + ', '.join(str(c['mask']) for c in cu) + '};')
    L.append(f'static __constant__ const unsigned char {name}_cur_n3[{len(cu)}] = {{'
             + ', '.join(str(len(c['s3'])) for c in cu) + '};')
    L.append(f'static __constant__ const unsigned char {name}_cur_n4[{len(cu)}] = {{'
             + ', '.join(str(len(c['s4'])) for c in cu) + '};')
    rows3, rows4 = [], []
    for c in cu:
        r3 = [(ia, ib, ma, mb, (1 if sa < 0 else 0) | (2 if sb < 0 else 0)) for ia, sa, ib, sb, ma, mb in c['s3']]
        r3 += [(0, 0, 0, 0, 0)] * (n3 - len(r3))
        rows3.append('{' + ', '.join('{' + ', '.join(str(v) for v in e) + '}' for e in r3) + '}')
        r4 = [(ia, ib, ic, (1 if sa < 0 else 0) | (2 if sb < 0 else 0) | (4 if sc < 0 else 0))
              for ia, sa, ib, sb, ic, sc in c['s4']]
        r4 += [(0, 0, 0, 0)] * (n4 - len(r4))
        rows4.append('{' + ', '.join('{' + ', '.join(str(v) for v in e) + '}' for e in r4) + '}')
    L.append(f'static __constant__ const short {name}_cur_s3[{len(cu)}][{n3}][5] = {{' + ', '.join(rows3) + '};')
    L.append(f'static __constant__ const short {name}_cur_s4[{len(cu)}][{n4}][4] = {{' + ', '.join(rows4) + '};')
    # prefix and ordering splits: (prefix id, current id, sign) ; prefix masks
    L.append(f'static __constant__ const unsigned char {name}_pre_mask[{len(pr)}] = {{'
             + ', '.join(str(p['mask']) for p in pr) + '};')
    np_ = k - 1
    rows = []
    for p in pr:
        r = [(a, b, 1 if s < 0 else 0) for a, b, s in p['splits']] + [(0, 0, 0)] * (np_ - len(p['splits']))
        rows.append('{' + ', '.join('{' + ', '.join(str(v) for v in e) + '}' for e in r) + '}')
    L.append(f'static __constant__ const short {name}_pre_split[{len(pr)}][{np_}][3] = {{' + ', '.join(rows) + '};')
    rows = []
    for o in od:
        rows.append('{' + ', '.join('{' + ', '.join(str(v) for v in (a, b, 1 if s < 0 else 0)) + '}'
                                     for a, b, s in o['splits']) + '}')
    L.append(f'static __constant__ const short {name}_ord_split[{len(od)}][{k}][3] = {{' + ', '.join(rows) + '};')
    n = len(od)
    # colour numerators as floats (integers, exact), each row padded with zeros to a multiple
    # of 64 columns: column i of row j is C'[j][i], and a lane reads the columns i = lane + r * LPE
    # of every row j, r < ceil(n / LPE), whatever the lanes per event
    cw = -(-n // 64) * 64
    L.append(f'static __constant__ const float {name}_cnumf[{n}][{cw}] = {{'
             + ', '.join('{' + ', '.join(f'{float(v)!r}f' for v in list(row) + [0] * (cw - n)) + '}'
                         for row in t['cnum']) + '};')
    L += ['namespace mf {',
          'template <int K> struct BgTab;',
          f'template <> struct BgTab<{k}> {{',
          f'    static constexpr int NCUR = {len(cu)}, NPRE = {len(pr)}, NORD = {len(od)}, CDEN = {t["cden"]};',
          f'    // prefixes shorter than k - 1 (the ones kept in LDS; each prefix of length k - 1 belongs',
          f'    // to one ordering and is formed by that ordering\'s lane)',
          f'    static constexpr int NPRE_STORED = {t["plevels"][k - 1][0]};',
          f'    __device__ static __forceinline__ int cur_levels(int i) {{ return {name}_cur_levels[i]; }}',
          f'    __device__ static __forceinline__ int pre_levels(int i) {{ return {name}_pre_levels[i]; }}',
          f'    __device__ static __forceinline__ int cur_mask(int c) {{ return {name}_cur_mask[c]; }}',
          f'    __device__ static __forceinline__ int cur_n3(int c) {{ return {name}_cur_n3[c]; }}',
          f'    __device__ static __forceinline__ int cur_n4(int c) {{ return {name}_cur_n4[c]; }}',
          f'    __device__ static __forceinline__ const short* cur_s3(int c, int s) {{ return {name}_cur_s3[c][s]; }}',
          f'    __device__ static __forceinline__ const short* cur_s4(int c, int s) {{ return {name}_cur_s4[c][s]; }}',
          f'    __device__ static __forceinline__ int pre_mask(int q) {{ return {name}_pre_mask[q]; }}',
          f'    __device__ static __forceinline__ const short* pre_split(int q, int s) {{ return {name}_pre_split[q][s]; }}',
          f'    __device__ static __forceinline__ const short* ord_split(int o, int s) {{ return {name}_ord_split[o][s]; }}',
          f'    __device__ static __forceinline__ float cnum(int j, int i) {{ return {name}_cnumf[j][i]; }}',
          '};',
          '}  // namespace mf']
    return '\n'.join(L) + '\n', t


def flops(k):
    """Flops per event of the table kernel as it executes (FMA = 2; complex multiply 6, complex
    FMA 8), by part: gluon currents per helicity configuration, quark line and colour sum per
    top helicity; and the total over the 2^(k-1) evaluated gluon configurations x 2 top
    helicities."""
    t = build(k)
    dot = 6 + 3 * 8                                  # 2 x.y in light-cone components
    cur = 0
    for c in t['currents']:
        if len(c['rho']) == 1:
            continue
        cur += len(c['s3']) * (3 * dot + 2 + 4 * (2 + 3 * 8))
        cur += len(c['s4']) * (3 * dot + 4 + 4 * 3 * 8)
        cur += 8                                     # times 1/P^2
    slash = 8 * 8                                    # row spinor times Jslash: 8 complex FMAs
    quark = 0
    for pf in t['prefixes'][1:]:
        quark += len(pf['splits']) * slash + 8 + slash
    n = len(t['orderings'])
    quark += n * (k * slash + 2 * 4 * 8)
    colour = 2 * 2 * n * n * 2 + 2 * 2 * n * 2
    per_event = 2 ** (k - 1) * (cur + 2 * (quark + colour))
    return dict(currents_per_gconf=cur, quark_per_top_hel=quark, colour_per_top_hel=colour, per_event=per_event,
                per_event_f64=per_event, per_event_f32=per_event, per_event_f32_valu=per_event)
