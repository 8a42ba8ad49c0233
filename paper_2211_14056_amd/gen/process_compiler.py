"""Process compiler: emits fused HIP device code for tree-level matrix elements.

The paper transpiles auto-generated per-process matrix-element code (external
wavefunctions, vertex and propagator routines, the process's diagram sequence)
into device code (sect. 2, Fig. 2), one kernel per vertex/spinor/propagator.
Here the process is compiled into ONE straight-line device function per event
whose intermediate currents live in registers, which is the footprint lever
the paper identifies (sect. 2, the discussion of Table 1).

Physics content.  For g g -> t tbar + (k-2) g, the amplitude is decomposed in
colour-ordered partial amplitudes A(sigma) over the k! gluon orderings with
colour factors (t^{a_sigma1}..t^{a_sigmak})_{i jbar}, and

    sum_{colour} |M|^2 = g^{2k} sum_{sigma,tau} Re(A_sigma^* C_{sigma tau} A_tau)

with the exact colour matrix from ``colour_algebra``.  Partial amplitudes are
built by the Berends-Giele off-shell recursion with colour-ordered vertices in
the normalisation where all couplings and phases are factored out:

  gluon current   J(rho) = 1/P_rho^2 [ sum_{rho = a b}  V3(J_a, P_a; J_b, P_b)
                                      + sum_{rho = a b c} V4(J_a, J_b, J_c) ]
      V3 = (J_a.J_b)(P_a - P_b) + 2 (P_b.J_a) J_b - 2 (P_a.J_b) J_a
      V4 = 2 J_b (J_a.J_c) - J_c (J_a.J_b) - J_a (J_b.J_c)
  quark line      A(sigma) = sum over splits of sigma into blocks b_1..b_r of
                  ubar(p_t) Jslash(b_1) S(q_1) Jslash(b_2) ... Jslash(b_r) v(p_tbar),
                  S(q) = (qslash + m)/(q^2 - m^2),  q_l = p_t - P(b_1..b_l)

(momenta P flow into the current: +p for incoming, -p for outgoing gluons;
external currents are eps(p) for incoming and eps*(p) for outgoing gluons).
V3 uses current conservation P_a.J_a = 0 of Berends-Giele currents with
physical external gluons.  Reflection J(reverse rho) = (-1)^(|rho|+1) J(rho)
halves the gluon currents.  Vectors are held in light-cone components
(v0+v3, v0-v3, v1+i v2, v1-i v2), in which gamma-matrix products need no
recombination.

Helicity recycling: gluon currents depend only on gluon helicities, so the
outer loop runs over the 2^k gluon helicity configurations and the quark
helicities are handled inside it (the top as a 2-trip loop, the antitop by
contracting the same open spinor with both v(+) and v(-)).

Kinematics (momenta, spinor and polarisation bases, all propagator
denominators) are evaluated once per event in FP64; the recursion and the
colour sum run in the kernel's working type R (double or float).
"""
import itertools
import math
import os

from . import colour_algebra
from .ir import Block, C, S, ZERO, ONE, const, csum, cadd, csub, cneg, cmat

SQRT1_2 = 1.0 / math.sqrt(2.0)


# ----------------------------------------------------------------- vectors
def lc_dot2(b, x, y):
    """2 x.y in light-cone components: x+ y- + x- y+ - xt ytb - xtb yt."""
    return csum(b, [(x[0], y[1]), (x[1], y[0]), (cneg(b, x[2]), y[3]), (cneg(b, x[3]), y[2])])


def real_lc(b, px, py, pp, pm):
    """Real four-vector (given by v+, v-, vx, vy) as a light-cone complex vector."""
    return [C(pp, ZERO), C(pm, ZERO), C(px, py), C(px, b.neg(py))]


class Momentum:
    """Real four-vector with named scalar components (E, x, y, z) and light-cone view."""

    def __init__(self, b, comps):
        self.E, self.x, self.y, self.z = comps
        self.b = b
        self._lc = None

    def lc(self):
        if self._lc is None:
            b = self.b
            pp = b.add(self.E, self.z)
            pm = b.sub(self.E, self.z)
            self._lc = real_lc(b, self.x, self.y, pp, pm)
        return self._lc


def msum(b, moms, signs):
    comps = []
    for c in range(4):
        acc = ZERO
        for m, s in zip(moms, signs):
            v = [m.E, m.x, m.y, m.z][c]
            acc = b.add(acc, v) if s > 0 else b.sub(acc, v)
        comps.append(acc)
    return Momentum(b, comps)


def assign_lds_slots(cands, budget):
    """LDS slots for the currents in ``cands`` (in order) within ``budget`` scalars:
    {current: {(mu, part): slot}}; every current has 4 complex light-cone components."""
    slots, nxt = {}, 0
    for perm in cands:
        if nxt + 8 > budget:
            break
        slots[perm] = {(mu, part): nxt + 2 * mu + part for mu in range(4) for part in range(2)}
        nxt += 8
    return slots


class Recursion:
    """Colour-ordered Berends-Giele recursion over the gluons, emitted into IR blocks.

    Gluon currents go to block ``b`` (outside the top-helicity loop) and the
    quark line to the block given to ``start_quark_line`` (inside it).  ``moms``
    are the gluon momenta (incoming convention) and ``eps`` the external
    currents, both indexed by gluon label; ``lds_slot`` maps the canonical
    currents parked in LDS to their slots.
    """

    def __init__(self, b, moms, eps, lds_slot, stream=False, local_memo=False, remote=None,
                 exchange='quad_rot<{m}>'):
        self.b, self.moms, self.eps, self.lds_slot = b, moms, eps, lds_slot
        self.stream = stream
        self.local_memo = local_memo
        # remote(rho) -> None, or (t, M, sign): J(rho) = sign * [J(t) of the lane M places
        # further in the group of lanes that share an event (see lane_split); `exchange`
        # is the device function that reads a value from that lane
        self.remote = remote
        self.exchange = exchange
        self.msum_memo, self.dot_memo, self.jmemo = {}, {}, {}

    @staticmethod
    def canon(rho):
        return rho if rho[0] < rho[-1] or len(rho) == 1 else tuple(reversed(rho))

    def orient(self, rho):
        """(canonical orientation, sign) with J(rho) = sign * J(canonical)."""
        c = self.canon(rho)
        return c, (1 if c == rho else (-1) ** (len(rho) + 1))

    def P(self, rho):
        """Momentum sum of a gluon subset (memoised)."""
        key = tuple(sorted(rho))
        if key not in self.msum_memo:
            if len(key) == 1:
                self.msum_memo[key] = self.moms[key[0]]
            else:
                self.msum_memo[key] = msum(self.b, [self.moms[i] for i in key], [1] * len(key))
        return self.msum_memo[key]

    def D(self, x, y):
        """2 J(x).J(y), memoised over canonical orientations."""
        b = self.b
        (cx, sx), (cy, sy) = self.orient(x), self.orient(y)
        key = (cx, cy) if cx <= cy else (cy, cx)
        if key not in self.dot_memo:
            self.dot_memo[key] = cmat(b, lc_dot2(b, self.J(cx), self.J(cy)))
        v = self.dot_memo[key]
        return v if sx * sy > 0 else cneg(b, v)

    def J(self, rho):
        """Off-shell gluon current of the ordered gluon sequence ``rho``."""
        b = self.b
        c = self.canon(rho)
        if c != rho:
            sgn = (-1) ** (len(rho) + 1)
            v = self.J(c)
            return v if sgn > 0 else [cneg(b, x) for x in v]
        if rho in self.jmemo:
            return self.jmemo[rho]
        if len(rho) == 1:
            self.jmemo[rho] = self.eps[rho[0]]
            return self.jmemo[rho]
        far = self.remote(rho) if self.remote else None
        vec = self._received(*far) if far else self._vertices(rho)
        self.jmemo[rho] = vec
        if rho in self.lds_slot:
            for (mu, part), slot in self.lds_slot[rho].items():
                v = vec[mu].re if part == 0 else vec[mu].im
                b.lines.append(f'lds[{slot * 64}] = {b.ref(v)};')
        return vec

    def _received(self, t, m, sign):
        """Current read from another lane sharing the event (DPP), with a reflection sign."""
        b = self.b
        own = self.J(t)
        fn = self.exchange.format(m=m)

        def rot(x):
            if x.is_const:
                return x
            v = b.new(f'{fn}({b.ref(x)})', 0)
            return v if sign > 0 else b.neg(v)
        return [C(rot(x.re), rot(x.im)) for x in own]

    def _vertices(self, rho):
        """Current from the three- and four-gluon vertex splits of rho."""
        b = self.b
        J, P, D = self.J, self.P, self.D
        if self.local_memo:
            # build the sub-currents first, then forget dot products and momentum sums
            # of earlier currents: recomputed here rather than kept live in between
            for s in range(1, len(rho)):
                J(rho[:s]), J(rho[s:])
            self.dot_memo, self.msum_memo = {}, {}
        terms = [[] for _ in range(4)]
        acc = [None] * 4

        def flush():
            # stream mode: fold the terms gathered so far into the running sums, so the
            # coefficients of one split die before the next split's are formed (same
            # operations in the same order as one chain over all terms)
            if self.stream:
                for mu in range(4):
                    acc[mu] = csum(b, terms[mu], acc[mu])
                    terms[mu] = []
        # three-vertex splits
        for s in range(1, len(rho)):
            a, bb = rho[:s], rho[s:]
            Ja, Jb = J(a), J(bb)
            Pa, Pb = P(a).lc(), P(bb).lc()
            dab = D(a, bb)
            hd = C(b.mul(dab.re, const(0.5)), b.mul(dab.im, const(0.5)))
            hd = cmat(b, hd)
            pbja = cmat(b, lc_dot2(b, Pb, Ja))        # 2 Pb.Ja
            pajb = cmat(b, lc_dot2(b, Pa, Jb))        # 2 Pa.Jb
            for mu in range(4):
                dP = csub(b, Pa[mu], Pb[mu])
                terms[mu].append((hd, dP))
                terms[mu].append((pbja, Jb[mu]))
                terms[mu].append((cneg(b, pajb), Ja[mu]))
            flush()
        # four-vertex splits
        for s1 in range(1, len(rho) - 1):
            for s2 in range(s1 + 1, len(rho)):
                a, bb, cc = rho[:s1], rho[s1:s2], rho[s2:]
                Ja, Jb, Jc = J(a), J(bb), J(cc)
                dac = D(a, cc)
                dab = D(a, bb)
                dbc = D(bb, cc)
                hab = cmat(b, C(b.mul(dab.re, const(-0.5)), b.mul(dab.im, const(-0.5))))
                hbc = cmat(b, C(b.mul(dbc.re, const(-0.5)), b.mul(dbc.im, const(-0.5))))
                for mu in range(4):
                    terms[mu].append((dac, Jb[mu]))
                    terms[mu].append((hab, Jc[mu]))
                    terms[mu].append((hbc, Ja[mu]))
                flush()
        ig = S(name=f'ig{_sname(sorted(rho))}')
        vec = []
        for mu in range(4):
            tot = acc[mu] if self.stream else csum(b, terms[mu])
            vec.append(cmat(b, C(b.mul(tot.re, ig), b.mul(tot.im, ig))))
        return vec

    # ------------------------------------------------------------ quark line
    def start_quark_line(self, q, qmoms, ub, orderings=(), share_products=False):
        """Quark-line block ``q``, the gluon momenta as seen there, and the row spinor ubar.
        share_products: form each product Q(prefix) Jslash(block) that the quark lines of
        ``orderings`` use more than once (a block and its reflection give the same product up
        to sign) once, and add it where it is used.  Left out: ubar Jslash(sigma) of a whole
        ordering, whose two uses (sigma and its reverse) are in the groups of different first
        gluons, so the shared value would stay live across most of the quark line."""
        self.q, self.qmoms = q, qmoms
        self.qsum_memo = {}
        self.qmemo = {(): ub}
        self.psimemo = {}
        self.pmemo = {}
        self.puses = {}
        if share_products:
            k = max((len(o) for o in orderings), default=0)
            self.puses = {key: v for key, v in self._count_products(orderings).items()
                          if not (key[0] == () and len(key[1]) == k)}

    def _count_products(self, orderings):
        """Occurrences of each product Q(prefix) Jslash(block), block up to reflection, on the
        quark lines of ``orderings`` (every memoised prefix counted once)."""
        uses, seen = {}, set()

        def add(pre, blk):
            key = (pre, self.canon(blk))
            uses[key] = uses.get(key, 0) + 1

        def prefix(p):
            if not p or p in seen:
                return
            seen.add(p)
            for s in range(len(p)):
                prefix(p[:s])
                add(p[:s], p[s:])
        for sigma in orderings:
            for s in range(len(sigma)):
                prefix(sigma[:s])
                add(sigma[:s], sigma[s:])
        return uses

    def _terms(self, pre, blk):
        """Terms of Q(pre) Jslash(blk), per spinor component."""
        key = (pre, self.canon(blk))
        if self.puses.get(key, 0) < 2:
            return self.slash_row(self.Q(pre), self.QJ(blk))
        c, sgn = self.orient(blk)
        if key not in self.pmemo:
            rows = self.slash_row(self.Q(pre), self.QJ(c))
            self.pmemo[key] = [cmat(self.q, csum(self.q, rows[i])) for i in range(4)]
        X = self.pmemo[key]
        return [[(X[i] if sgn > 0 else cneg(self.q, X[i]), C(ONE))] for i in range(4)]

    def QP(self, rho):
        key = tuple(sorted(rho))
        if key not in self.qsum_memo:
            self.qsum_memo[key] = (self.qmoms[key[0]] if len(key) == 1 else
                                   msum(self.q, [self.qmoms[i] for i in key], [1] * len(key)))
        return self.qsum_memo[key]

    def QJ(self, rho):
        """Gluon current as seen from the quark line (re-read from LDS if parked there)."""
        q = self.q
        c = self.canon(rho)
        if c not in self.lds_slot:
            return self.J(rho)
        sgn = 1 if c == rho else (-1) ** (len(rho) + 1)
        vec = []
        for mu in range(4):
            parts = []
            for part in range(2):
                v = q.new(f'lds[{self.lds_slot[c][(mu, part)] * 64}]', 0)
                parts.append(v if sgn > 0 else q.neg(v))
            vec.append(C(parts[0], parts[1]))
        return vec

    def slash_row(self, psi, Jv):
        """Terms of the row spinor psi * Jslash (light cone): list per component."""
        q = self.q
        Jp, Jm, Jt, Jtb = Jv
        return [
            [(psi[2], Jp), (psi[3], Jt)],
            [(psi[2], Jtb), (psi[3], Jm)],
            [(psi[0], Jm), (cneg(q, psi[1]), Jt)],
            [(cneg(q, psi[0]), Jtb), (psi[1], Jp)],
        ]

    def psi(self, prefix):
        """Row spinor ubar Jslash .. Jslash(last block of prefix), before the propagator of prefix."""
        if prefix in self.psimemo:
            return self.psimemo[prefix]
        q = self.q
        terms = [[] for _ in range(4)]
        for s in range(len(prefix)):
            rows = self._terms(prefix[:s], prefix[s:])
            for c in range(4):
                terms[c] += rows[c]
        self.psimemo[prefix] = [cmat(q, csum(q, terms[c])) for c in range(4)]
        return self.psimemo[prefix]

    def propagator(self, b, Pp, iq):
        """(q+, q-, qt, qtb) and m, each times 1/(q^2 - m^2), of q = p_t - Pp, emitted into ``b``."""
        qE = b.sub(S(name='PT[0]'), Pp.E)
        qx = b.sub(S(name='PT[1]'), Pp.x)
        qy = b.sub(S(name='PT[2]'), Pp.y)
        qz = b.sub(S(name='PT[3]'), Pp.z)
        qp = b.mul(b.add(qE, qz), iq)
        qm = b.mul(b.sub(qE, qz), iq)
        qxs = b.mul(qx, iq)
        qys = b.mul(qy, iq)
        ms = b.mul(S(name='MT'), iq)
        return [C(qp), C(qm), C(qxs, qys), C(qxs, b.neg(qys))], ms

    def Q(self, prefix):
        """Row spinor ubar Jslash .. S(q) after the gluons of ``prefix`` (propagator included)."""
        if prefix in self.qmemo:
            return self.qmemo[prefix]
        q = self.q
        psi = self.psi(prefix)
        # propagator: (psi qslash + m psi)/(q^2 - m^2), q = p_t - P(prefix)
        qlc, ms = self.propagator(q, self.QP(prefix), S(name=f'iq{_sname(sorted(prefix))}'))
        rows = self.slash_row(psi, qlc)
        out_ = []
        for c in range(4):
            out_.append(cmat(q, csum(q, rows[c] + [(psi[c], C(ms))])))
        self.qmemo[prefix] = out_
        return out_

    def closing(self, sigma):
        """Open row spinor of the full ordering: sum over the last block of Q(prefix) Jslash(block)."""
        q = self.q
        terms = [[] for _ in range(4)]
        for s in range(len(sigma)):
            rows = self._terms(sigma[:s], sigma[s:])
            for c in range(4):
                terms[c] += rows[c]
        return [cmat(q, csum(q, terms[c])) for c in range(4)]


# ----------------------------------------------------------------- process
class GGTTProcess:
    """g(0) g(1) -> t(2) tbar(3) g(4) ... g(n_ext-1)."""

    def __init__(self, name, n_ext):
        self.name = name
        self.n_ext = n_ext
        self.k = n_ext - 2                       # number of gluons
        self.gl_legs = [0, 1] + list(range(4, n_ext))
        self.sym = math.factorial(n_ext - 4)     # identical final gluons
        self.avg = 256.0
        C, den = colour_algebra.integer_form(colour_algebra.colour_matrix(self.k))
        self.cnum, self.cden = C, den
        self.orderings = colour_algebra.orderings(self.k)

    # subsets of gluons needing propagators
    def gluon_subsets(self):
        return [c for r in range(2, self.k + 1) for c in itertools.combinations(range(self.k), r)]

    def quark_subsets(self):
        return [c for r in range(1, self.k) for c in itertools.combinations(range(self.k), r)]


def _sname(sub):
    return ''.join(str(i) for i in sub)


class _IR:
    """The IR blocks of one process: gluon currents ``b`` (per gluon-helicity
    configuration), quark line ``q`` (per top helicity; amplitudes ``amps[h][sigma]`` for
    the two antitop helicities) and colour sums ``cs`` (``csq[h]``)."""


def _build_ir(proc, lds_budget=0, stream=False, share_products=False, group_barriers=True):
    k = proc.k
    # ---------------- loop body (working precision) ----------------
    b = Block('t')
    moms = [Momentum(b, [S(name=f'K{gi}[{c}]') for c in range(4)]) for gi in range(k)]
    # beams: gluon 0 along +z, gluon 1 along -z; known zero components
    for gi, leg in enumerate(proc.gl_legs):
        if leg < 2:
            E = S(name=f'K{gi}[0]')
            zsign = 1.0 if leg == 0 else -1.0
            mm = Momentum(b, [E, ZERO, ZERO, E if zsign > 0 else b.neg(E)])
            moms[gi] = mm
    lam = [S(name=f'lam{gi}') for gi in range(k)]
    # external gluon currents (light-cone components)
    eps = []
    for gi, leg in enumerate(proc.gl_legs):
        if leg == 0:
            # eps(+z, l) = (0, -l/sqrt2, -i/sqrt2, 0): t = (1-l)/sqrt2, tb = -(1+l)/sqrt2
            t = b.sumprod([(lam[gi], const(-SQRT1_2))], const(SQRT1_2))
            tb = b.sumprod([(lam[gi], const(-SQRT1_2))], const(-SQRT1_2))
            eps.append([C(ZERO), C(ZERO), C(t), C(tb)])
        elif leg == 1:
            # eps(-z, l) = (0, l/sqrt2, -i/sqrt2, 0): t = (1+l)/sqrt2, tb = (l-1)/sqrt2
            t = b.sumprod([(lam[gi], const(SQRT1_2))], const(SQRT1_2))
            tb = b.sumprod([(lam[gi], const(SQRT1_2))], const(-SQRT1_2))
            eps.append([C(ZERO), C(ZERO), C(t), C(tb)])
        else:
            # eps*(k, l) = (-l u + i w), u = eps1/sqrt2 (x,y,z), w = eps2/sqrt2 (x,y), w_z = 0
            ux, uy, uz = (S(name=f'e{gi}u[{c}]') for c in range(3))
            wx, wy = (S(name=f'e{gi}w[{c}]') for c in range(2))
            l = lam[gi]
            ez = b.mul(b.neg(l), uz)                       # eps^3 (real)
            # t = eps^1 + i eps^2 = (-l ux - wy) + i (wx - l uy)
            tr = b.sumprod([(l, b.neg(ux))], b.neg(wy))
            ti = b.sumprod([(l, b.neg(uy))], wx)
            # tb = eps^1 - i eps^2 = (-l ux + wy) + i (wx + l uy)
            tbr = b.sumprod([(l, b.neg(ux))], wy)
            tbi = b.sumprod([(l, uy)], wx)
            eps.append([C(ez), C(b.neg(ez)), C(tr, ti), C(tbr, tbi)])
    lds_slot = {}
    if lds_budget:
        cands = [perm for r in range(k, 1, -1) for S_ in itertools.combinations(range(k), r)
                 for perm in itertools.permutations(S_) if Recursion.canon(perm) == perm]
        lds_slot = assign_lds_slots(cands, lds_budget)
    rec = Recursion(b, moms, eps, lds_slot, stream=stream)
    # build every gluon current (canonical orientations), by length
    for r in range(2, k + 1):
        for S_ in itertools.combinations(range(k), r):
            for perm in itertools.permutations(S_):
                if Recursion.canon(perm) == perm:
                    rec.J(perm)
    gluon_flops = b.flops
    gluon_lines = b.lines
    # ---------------- quark line (inside the top-helicity loop) ----------------
    q = Block('u')
    ub = [C(S(name=f'ubs[{j}].re'), S(name=f'ubs[{j}].im')) for j in range(4)]
    qmoms = [Momentum(q, [S(name=f'K{gi}[{c}]') for c in range(4)]) for gi in range(k)]
    for gi, leg in enumerate(proc.gl_legs):
        if leg < 2:
            E = S(name=f'K{gi}[0]')
            qmoms[gi] = Momentum(q, [E, ZERO, ZERO, E if leg == 0 else q.neg(E)])
    rec.start_quark_line(q, qmoms, ub, proc.orderings, share_products)
    vspin = [[C(S(name=f'vs[{h}][{j}].re'), S(name=f'vs[{h}][{j}].im')) for j in range(4)] for h in range(2)]
    amps = [[None] * len(proc.orderings) for _ in range(2)]
    prev_first = None
    for si, sigma in enumerate(proc.orderings):
        if group_barriers and prev_first is not None and sigma[0] != prev_first:
            q.lines.append('__builtin_amdgcn_sched_barrier(0);')
        prev_first = sigma[0]
        full = rec.closing(sigma)
        for h in range(2):
            amps[h][si] = cmat(q, csum(q, [(full[c], vspin[h][c]) for c in range(4)]))
    quark_flops = q.flops
    # colour sums (one per antitop helicity)
    cs = Block('w')
    csq = []
    n_or = len(proc.orderings)
    for h in range(2):
        A = amps[h]
        tot_terms = []
        for i in range(n_or):
            yr = [(const(proc.cnum[i][i] if j == i else 2 * proc.cnum[i][j]), A[j].re) for j in range(i, n_or)]
            yi = [(const(proc.cnum[i][i] if j == i else 2 * proc.cnum[i][j]), A[j].im) for j in range(i, n_or)]
            y_r = cs.sumprod(yr)
            y_i = cs.sumprod(yi)
            tot_terms.append((A[i].re, y_r))
            tot_terms.append((A[i].im, y_i))
        csq.append(cs.sumprod(tot_terms))
    colour_flops = cs.flops
    ir = _IR()
    ir.b, ir.q, ir.cs, ir.csq, ir.amps, ir.rec, ir.lds_slot = b, q, cs, csq, amps, rec, lds_slot
    ir.gluon_flops, ir.gluon_lines, ir.quark_flops, ir.colour_flops = gluon_flops, gluon_lines, quark_flops, colour_flops
    ir.n_or = n_or
    return ir


def emit_qcd(proc, with_colour=True, opaque_inputs=True, group_barriers=True, lds_budget=0, constants=True,
             stream=False, share_products=False):
    """Return (source text, flop counts) of the device function for ``proc``.

    opaque_inputs: re-declare the momenta as opaque at the top of each helicity
      iteration, so that their sums are recomputed inside the loop instead of
      being hoisted and kept live across it (fewer registers, a few adds more).
    group_barriers: scheduling barriers between the gluon-current block and the
      quark line and between groups of orderings with the same first gluon, so
      that the scheduler cannot interleave them and widen the live set.
    lds_budget: number of working-type scalars per lane that may be parked in
      LDS.  Multi-gluon currents (longest first) are written to per-lane LDS
      slots when computed and re-read at each use on the quark line, so they do
      not occupy registers across the top-helicity loop.  The emitted body then
      takes an LDS pointer (this lane's column, stride 64) as extra argument.
    stream: fold each vertex split of a gluon current into running sums as soon
      as its coefficients are formed (fewer values live at once; same arithmetic).
    share_products: form a quark-line product Q(prefix) Jslash(block) used by several
      orderings once (see Recursion.start_quark_line).

    Helicity sum.  For real momenta, reversing every helicity turns each partial
    amplitude into its complex conjugate times one phase common to all orderings,
    so a configuration and its reverse have the same colour-summed |M|^2.  The body
    therefore runs only the gluon-helicity configurations in which the last gluon
    has helicity +1 (2^(k-1) of them; both top and antitop helicities each), and the
    normalisation constant carries the factor 2 for the reversed half.
    """
    k = proc.k
    out = []
    fn = f'me_{proc.name}'
    out.append(f'// ---- {proc.name}: {k} gluons, {math.factorial(k)} colour orderings, '
               f'{2 ** (k + 2)} helicities, {2 ** (k + 1)} evaluated (the rest by helicity reversal)')
    out.append(f'template <typename R, typename KT, typename Sink>')
    lds_arg = ', R* __restrict__ lds' if lds_budget else ''
    out.append(f'__device__ __forceinline__ void {fn}_body(const KT (&p)[{proc.n_ext}][4], '
               f'const KT mt, Sink& sink{lds_arg})')
    out.append('{')
    # ---------------- prologue (double precision kinematics) ----------------
    pro = []
    # incoming-convention momenta k_i of the gluons
    for gi, leg in enumerate(proc.gl_legs):
        sgn = '' if leg < 2 else '-'
        pro.append(f'const KT k{gi}[4] = {{{sgn}p[{leg}][0], {sgn}p[{leg}][1], '
                   f'{sgn}p[{leg}][2], {sgn}p[{leg}][3]}};')
    pro.append('const KT mt2 = mt * mt;')
    # gluon propagators 1/P_S^2
    for sub in proc.gluon_subsets():
        n = _sname(sub)
        terms = ' + '.join(f'k{i}[c]' for i in sub)
        pro.append(f'KT P{n}[4]; for (int c = 0; c < 4; ++c) P{n}[c] = {terms};')
        pro.append(f'const R ig{n} = cvt<R>(KT(1.0) / (P{n}[0] * P{n}[0] - P{n}[1] * P{n}[1] - '
                   f'P{n}[2] * P{n}[2] - P{n}[3] * P{n}[3]));')
    # quark propagators: q = p_t - P_S, 1/(q^2 - m^2)
    for sub in proc.quark_subsets():
        n = _sname(sub)
        terms = ' - '.join([f'p[2][c]'] + [f'k{i}[c]' for i in sub])
        pro.append(f'KT q{n}[4]; for (int c = 0; c < 4; ++c) q{n}[c] = {terms};')
        pro.append(f'const R iq{n} = cvt<R>(KT(1.0) / ((q{n}[0] - q{n}[3]) * (q{n}[0] + q{n}[3]) - '
                   f'q{n}[1] * q{n}[1] - q{n}[2] * q{n}[2] - mt2));')
    # momenta in working precision
    for gi in range(k):
        pro.append(f'R K{gi}[4] = {{cvt<R>(k{gi}[0]), cvt<R>(k{gi}[1]), cvt<R>(k{gi}[2]), '
                   f'cvt<R>(k{gi}[3])}};')
    pro.append('R PT[4] = {cvt<R>(p[2][0]), cvt<R>(p[2][1]), cvt<R>(p[2][2]), cvt<R>(p[2][3])};')
    pro.append('const R MT = cvt<R>(mt);')
    # outgoing-gluon polarisation bases (eps1/sqrt2, eps2/sqrt2)
    for gi, leg in enumerate(proc.gl_legs):
        if leg < 2:
            continue
        pro.append(f'R e{gi}u[3], e{gi}w[2]; pol_basis<R, KT>(p[{leg}], e{gi}u, e{gi}w);')
    # spinors for both helicities
    pro.append('cplx<R> ub[2][4], vs[2][4];')
    pro.append('ubar_spinor<R, KT>(p[2], mt, -1, ub[0]); ubar_spinor<R, KT>(p[2], mt, 1, ub[1]);')
    pro.append('v_spinor<R, KT>(p[3], mt, -1, vs[0]); v_spinor<R, KT>(p[3], mt, 1, vs[1]);')
    out += ['    ' + l for l in pro]

    # ---------------- loop body (working precision) ----------------
    ir = _build_ir(proc, lds_budget, stream, share_products, group_barriers)
    b, q, cs, csq, amps, lds_slot = ir.b, ir.q, ir.cs, ir.csq, ir.amps, ir.lds_slot
    gluon_flops, gluon_lines, quark_flops, colour_flops = ir.gluon_flops, ir.gluon_lines, ir.quark_flops, ir.colour_flops
    n_or = ir.n_or

    # ---------------- emit ----------------
    body = []
    opq = []
    if opaque_inputs:
        for gi, leg in enumerate(proc.gl_legs):
            comps = [0] if leg < 2 else [0, 1, 2, 3]
            opq += [f'opaque(K{gi}[{c}]);' for c in comps]
        opq += [f'opaque(PT[{c}]);' for c in range(4)]
    body.append('#pragma unroll 1')
    body.append(f'for (int gconf = {2 ** (k - 1)}; gconf < {2 ** k}; ++gconf) {{   // last gluon: helicity +1')
    body += ['    ' + l for l in opq]
    for gi in range(k):
        body.append(f'    const R lam{gi} = (gconf >> {gi}) & 1 ? R(1) : R(-1);')
    body += ['    ' + l for l in gluon_lines]
    body.append('    #pragma unroll 1')
    body.append('    for (int ht = 0; ht < 2; ++ht) {')
    body += ['        ' + l for l in opq]
    if group_barriers:
        body.append('        __builtin_amdgcn_sched_barrier(0);')
    body.append('        cplx<R> ubs[4];')
    body.append('        for (int j = 0; j < 4; ++j) ubs[j] = ht ? ub[1][j] : ub[0][j];')
    body += ['        ' + l for l in q.lines]
    if with_colour:
        body += ['        ' + l for l in cs.lines]
        body.append(f'        sink.add({cs.ref(csq[0])}, {cs.ref(csq[1])});')
    else:
        # hand the partial amplitudes to the sink (colour contraction done there)
        for h in range(2):
            for si in range(n_or):
                a = amps[h][si]
                body.append(f'        sink.a[{h}][{si}][0] = {q.ref(a.re)}; sink.a[{h}][{si}][1] = {q.ref(a.im)};')
        body.append('        sink.flush();')
    body.append('    }')
    body.append('}')
    out += ['    ' + l for l in body]
    out.append('}')
    nslots = 8 * len(lds_slot)
    if not with_colour or not constants:
        return '\n'.join(out), dict(lds_slots=nslots)
    out.append('')
    out.append(f'// normalisation: 2 (reversed helicities) / (avg * sym * colour denominator); times g^(2k)')
    out.append(f'__host__ __device__ constexpr double {fn}_norm_noalpha() '
               f'{{ return 2.0 / ({proc.avg!r} * {float(proc.sym)!r} * {float(proc.cden)!r}); }}')
    out.append(f'constexpr int {fn}_k = {k};')
    out.append(f'constexpr int {fn}_ncolour = {n_or};')
    helis = 2 ** (k + 2)
    flops = dict(gluon_per_gconf=gluon_flops, quark_per_top_hel=quark_flops,
                 colour_per_hel=colour_flops // 2,
                 per_event=(2 ** (k - 1)) * (gluon_flops + 2 * (quark_flops + colour_flops)),
                 helicities=helis, evaluated_helicities=helis // 2, lds_slots=nslots)
    out.append(f'// flops per event (generated count): {flops}')
    return '\n'.join(out), flops


# ----------------------------------------------------------------- adjoint
def _zname_key(n):
    order = ('K', 'PT', 'MT', 'ig', 'iq', 'e', 'ub', 'vs')
    for i, pfx in enumerate(order):
        if n.startswith(pfx):
            return (i, n)
    return (len(order), n)


def kin_slots(proc):
    """Names of the kinematic inputs the recursion reads (the vector z of the adjoint),
    in slot order.  The top-spinor row of the current top helicity, ubs, appears as the
    two rows ub[0] and ub[1]."""
    ir = _build_ir(proc)
    from .adjoint import operand_names, defined_names
    ops = ir.b.ops + ir.q.ops + ir.cs.ops
    names = operand_names(ops) - set(defined_names(ops))
    out = set()
    for n in names:
        if n.startswith('lam'):
            continue                      # helicity signs: no derivative
        if n.startswith('ubs['):
            j, part = n[4], n.split('.')[1]
            out.update({f'ub[0][{j}].{part}', f'ub[1][{j}].{part}'})
        else:
            out.add(n)
    return sorted(out, key=_zname_key)


def emit_kin(proc):
    """Kinematic inputs of the recursion from the momenta and m_t, in the kinematic type
    KT, each handed to out.put(slot, value): the same quantities, in the same
    arithmetic, as the prologue of the forward body (gluon and quark propagator
    denominators, momenta, polarisation bases, spinors)."""
    k = proc.k
    slots = kin_slots(proc)
    idx = {n: i for i, n in enumerate(slots)}
    fn = f'me_{proc.name}'
    L = [f'// kinematic inputs of the {proc.name} recursion: {len(slots)} slots',
         f'constexpr int {fn}_nkin = {len(slots)};',
         'template <typename KT, typename Out>',
         f'__device__ __forceinline__ void {fn}_kin(const KT (&p)[{proc.n_ext}][4], const KT mt, Out& out)',
         '{']
    B = []
    for gi, leg in enumerate(proc.gl_legs):
        sgn = '' if leg < 2 else '-'
        B.append(f'const KT k{gi}[4] = {{{sgn}p[{leg}][0], {sgn}p[{leg}][1], {sgn}p[{leg}][2], {sgn}p[{leg}][3]}};')
    B.append('const KT mt2 = mt * mt;')
    for sub in proc.gluon_subsets():
        n = _sname(sub)
        if f'ig{n}' not in idx:
            continue
        terms = ' + '.join(f'k{i}[c]' for i in sub)
        B.append(f'{{ KT P[4]; for (int c = 0; c < 4; ++c) P[c] = {terms};')
        B.append(f'  out.put({idx["ig" + n]}, KT(1.0) / (P[0] * P[0] - P[1] * P[1] - P[2] * P[2] - P[3] * P[3])); }}')
    for sub in proc.quark_subsets():
        n = _sname(sub)
        if f'iq{n}' not in idx:
            continue
        terms = ' - '.join(['p[2][c]'] + [f'k{i}[c]' for i in sub])
        B.append(f'{{ KT q[4]; for (int c = 0; c < 4; ++c) q[c] = {terms};')
        B.append(f'  out.put({idx["iq" + n]}, KT(1.0) / ((q[0] - q[3]) * (q[0] + q[3]) - q[1] * q[1] - q[2] * q[2] - mt2)); }}')
    for n in slots:
        if n.startswith('K'):
            gi, c = n[1:].split('[')
            B.append(f'out.put({idx[n]}, k{gi}[{c[:-1]}]);')
        elif n.startswith('PT'):
            B.append(f'out.put({idx[n]}, p[2][{n[3]}]);')
        elif n == 'MT':
            B.append(f'out.put({idx[n]}, mt);')
    for gi, leg in enumerate(proc.gl_legs):
        if leg < 2:
            continue
        B.append(f'{{ KT u[3], w[2]; pol_basis<KT, KT>(p[{leg}], u, w);')
        for c in range(3):
            if f'e{gi}u[{c}]' in idx:
                B.append(f'  out.put({idx[f"e{gi}u[{c}]"]}, u[{c}]);')
        for c in range(2):
            if f'e{gi}w[{c}]' in idx:
                B.append(f'  out.put({idx[f"e{gi}w[{c}]"]}, w[{c}]);')
        B.append('}')
    for arr, fnc, leg in (('ub', 'ubar_spinor', 2), ('vs', 'v_spinor', 3)):
        for h, lam in ((0, -1), (1, 1)):
            B.append(f'{{ cplx<KT> s[4]; {fnc}<KT, KT>(p[{leg}], mt, {lam}, s);')
            for j in range(4):
                for part in ('re', 'im'):
                    nm = f'{arr}[{h}][{j}].{part}'
                    if nm in idx:
                        B.append(f'  out.put({idx[nm]}, s[{j}].{part});')
            B.append('}')
    L += ['    ' + l for l in B]
    L.append('}')
    return '\n'.join(L), slots


def _adj_lvalue(n):
    """Accumulator of an input's adjoint: the input's name with _b after its identifier."""
    if n.startswith('lam'):
        return None
    i = 0
    while i < len(n) and (n[i].isalnum() or n[i] == '_'):
        i += 1
    return n[:i] + '_b' + n[i:]


def _regrouped_quark_sweeps(proc, ir, g_read, ext_adj, group_barriers, depth=1):
    """Reverse sweep of the quark line by groups of orderings with the same first `depth` gluons.

    The forward quark line and colour sums have run; the colour sums' sweep gives the
    adjoints of the amplitudes.  Per group, the statements its amplitudes depend on are
    emitted again under new names (recomputation) and swept backwards from those adjoints,
    so only one group's quark-line values are live during a sweep.  g_read: the gluon-current
    components whose adjoints are locals (any other input's goes through ext_adj).  Returns
    (lines, flops of the recomputation, flops of the sweeps)."""
    import re as _re
    from .adjoint import Adjoint, base_sign
    q = ir.q
    ops = {name: (kind, name, operands) for kind, name, operands in q.ops}
    order = [name for _, name, _ in q.ops]
    text = {}
    for l in q.lines:
        m = _re.match(r'const R (u\d+) = ', l)
        if m:
            text[m.group(1)] = l
    flops_of = {}
    for l in q.lines:
        m = _re.match(r'const R (u\d+) = (.*);', l)
        if m:
            e = m.group(2)
            flops_of[m.group(1)] = 2 if e.startswith('fma(') else (1 if (' + ' in e or ' * ' in e) else 0)
    lines, rec_flops, sweep_flops = [], 0, 0
    keys = []
    for sig in proc.orderings:
        if tuple(sig[:depth]) not in keys:
            keys.append(tuple(sig[:depth]))
    for gi, key in enumerate(keys):
        outs = [ir.amps[h][si] for h in range(2) for si, sig in enumerate(proc.orderings) if tuple(sig[:depth]) == key]
        need = set()
        stack = [base_sign(x)[0] for a in outs for x in (a.re, a.im) if not x.is_const]
        while stack:
            n = stack.pop()
            if n in need or n not in ops:
                continue
            need.add(n)
            for x in ops[n][2]:
                if not x.is_const:
                    stack.append(base_sign(x)[0])
        pfx = f'q{gi}_'
        ren = lambda n: pfx + n if n in need else n          # noqa: E731

        def rn(x):
            if x.is_const:
                return x
            b, sgn = base_sign(x)
            return S(name=ren(b) if sgn > 0 else f'(-{ren(b)})')
        sub = [n for n in order if n in need]
        if group_barriers:
            lines.append('__builtin_amdgcn_sched_barrier(0);')
        # the group's copy of the top spinor row, opaque to the compiler: every quark-line
        # value depends on it, so the recomputation cannot be merged with the forward pass
        # (which would keep the forward values live until the sweep instead)
        lines.append(f'cplx<R> {pfx}ubs[4];')
        for j in range(4):
            lines.append(f'{pfx}ubs[{j}] = ubs[{j}]; opaque({pfx}ubs[{j}].re); opaque({pfx}ubs[{j}].im);')
        for n in sub:
            l = _re.sub(r'\bu(\d+)\b', lambda m: ren('u' + m.group(1)), text[n])
            lines.append(_re.sub(r'\bubs\[', f'{pfx}ubs[', l))
            rec_flops += flops_of.get(n, 0)
        val = lambda n: pfx + n if n.startswith('ubs[') else n          # noqa: E731
        a = Adjoint({ren(n) for n in sub} | set(g_read), ext_adj, declared=g_read, val=val)
        for amp in outs:
            for x in (amp.re, amp.im):
                if not x.is_const:
                    b, sgn = base_sign(x)
                    a.seed(S(name=ren(b)), f'{b}_b' if sgn > 0 else f'(-{b}_b)')
        a.sweep([(kind, ren(name), tuple(rn(x) for x in operands)) for kind, name, operands in
                 (ops[n] for n in sub)])
        lines += a.lines
        sweep_flops += a.flops
    return lines, rec_flops, sweep_flops


def _ordering_sweeps_with_currents(proc, ir, ext_adj, group_barriers):
    """Reverse sweep of the quark line and the gluon currents, one colour ordering at a time.

    The forward pass (currents, quark line, colour sums) has run and the colour sums' sweep
    gives the adjoints of the amplitudes.  Per ordering, the gluon currents and quark-line
    values its two amplitudes depend on are emitted again under new names, from opaque copies
    of the helicity signs and of the top spinor (so the compiler can merge them neither with
    the forward pass nor with another ordering), and swept backwards into the adjoints of the
    kinematic inputs.  No current or current adjoint lives across orderings.  Returns (lines,
    flops of the recomputation, flops of the sweeps)."""
    import re as _re
    from .adjoint import Adjoint, base_sign
    allops = ir.b.ops + ir.q.ops
    ops = {name: (kind, name, operands) for kind, name, operands in allops}
    order = [name for _, name, _ in allops]
    text, flops_of = {}, {}
    for l in ir.gluon_lines + ir.q.lines:
        m = _re.match(r'const R ([tu]\d+) = (.*);', l)
        if m:
            text[m.group(1)] = l
            e = m.group(2)
            flops_of[m.group(1)] = 2 if e.startswith('fma(') else (1 if (' + ' in e or ' * ' in e) else 0)
    lines, rec_flops, sweep_flops = [], 0, 0
    for si in range(len(proc.orderings)):
        outs = [ir.amps[h][si] for h in range(2)]
        need = set()
        stack = [base_sign(x)[0] for a in outs for x in (a.re, a.im) if not x.is_const]
        while stack:
            n = stack.pop()
            if n in need or n not in ops:
                continue
            need.add(n)
            for x in ops[n][2]:
                if not x.is_const:
                    stack.append(base_sign(x)[0])
        pfx = f'o{si}_'
        ren = lambda n: pfx + n if n in need else n          # noqa: E731

        def rn(x):
            if x.is_const:
                return x
            b, sgn = base_sign(x)
            return S(name=ren(b) if sgn > 0 else f'(-{ren(b)})')
        sub = [n for n in order if n in need]
        if group_barriers:
            lines.append('__builtin_amdgcn_sched_barrier(0);')
        lines.append(f'cplx<R> {pfx}ubs[4];')
        for j in range(4):
            lines.append(f'{pfx}ubs[{j}] = ubs[{j}]; opaque({pfx}ubs[{j}].re); opaque({pfx}ubs[{j}].im);')
        for gi in range(proc.k):
            lines.append(f'R {pfx}lam{gi} = lam{gi}; opaque({pfx}lam{gi});')
        for n in sub:
            l = _re.sub(r'\b([tu]\d+)\b', lambda m: ren(m.group(1)), text[n])
            l = _re.sub(r'\bubs\[', f'{pfx}ubs[', l)
            lines.append(_re.sub(r'\blam(\d+)\b', lambda m: f'{pfx}lam{m.group(1)}', l))
            rec_flops += flops_of.get(n, 0)
        val = lambda n: pfx + n if n.startswith(('ubs[', 'lam')) else n          # noqa: E731
        a = Adjoint({ren(n) for n in sub}, ext_adj, val=val)
        for amp in outs:
            for x in (amp.re, amp.im):
                if not x.is_const:
                    b, sgn = base_sign(x)
                    a.seed(S(name=ren(b)), f'{b}_b' if sgn > 0 else f'(-{b}_b)')
        a.sweep([(kind, ren(name), tuple(rn(x) for x in operands)) for kind, name, operands in
                 (ops[n] for n in sub)])
        lines += a.lines
        sweep_flops += a.flops
    return lines, rec_flops, sweep_flops


def emit_qcd_adjoint(proc, opaque_inputs=True, group_barriers=True, regroup=False, zb_mem=False, jb_mem=False,
                     group_depth=1, recompute_currents=False):
    """Adjoint (reverse sweep) of the helicity-summed, colour-contracted |M|^2 with respect
    to the kinematic inputs z (emit_kin), recomputing every current per helicity.

    Per gluon-helicity configuration: the gluon currents forward; per top helicity the
    quark line and colour sums forward, then their reverse sweep seeded with 1 for both
    antitop helicities, which adds into the adjoints of the currents and of z; after the
    top-helicity loop the gluon currents are recomputed (no value of the first pass is
    kept across the loop except the currents the quark line reads) and swept backwards.
    No current is stored in memory.

    regroup: after the colour sums' sweep, the quark line is swept by groups of orderings
    sharing their first `group_depth` gluons, each group's values recomputed
    (_regrouped_quark_sweeps); otherwise the whole quark line is swept at once.
    zb_mem: the adjoints of z accumulate in place in the caller's array zb (slot i at
    zb[i * ZS]; ZS = 64 puts one lane's slots a wavefront apart in LDS) instead of in
    registers.  jb_mem (with zb_mem): the adjoints of the gluon currents the quark line
    reads accumulate there too, after the z slots, and are loaded back for the gluon
    sweep (True: all of them; a number: that many, the least read ones).
    recompute_currents: after the colour sums' sweep, each ordering recomputes its gluon
    currents as well as its quark line and sweeps both (_ordering_sweeps_with_currents), so
    no current adjoint accumulates across orderings and the gluon sweep after the loop goes.
    Returns (source, flop counts)."""
    from .adjoint import Adjoint, base_sign, operand_names, defined_names
    if jb_mem and not zb_mem:
        raise ValueError('jb_mem puts the current adjoints after the z slots of zb: it needs zb_mem')
    if recompute_currents and (regroup or jb_mem):
        raise ValueError('recompute_currents sweeps per ordering by itself: no regroup or jb_mem with it')
    k = proc.k
    ir = _build_ir(proc, 0, False, False, group_barriers)
    b, q, cs = ir.b, ir.q, ir.cs
    g_temps = defined_names(b.ops)
    qc_ops = q.ops + cs.ops
    qc_temps = defined_names(qc_ops)
    g_set = set(g_temps)
    g_read = sorted((operand_names(qc_ops) & g_set), key=lambda n: int(n[1:]))
    kin_src, slots = emit_kin(proc)
    fn = f'me_{proc.name}'
    out = [kin_src, '']
    out.append(f'// adjoint of {fn}: |M|^2 (no couplings, no normalisation) added to me, its gradient')
    out.append(f'// with respect to the kinematic inputs z written to zb')
    nz = len(slots)
    zidx = {n: i for i, n in enumerate(slots)}
    if jb_mem is True:
        jb_names = list(g_read)
    elif jb_mem:
        # the jb_mem current components the quark line reads least often
        from collections import Counter
        uses = Counter(base_sign(x)[0] for _, _, ops_ in qc_ops for x in ops_ if not x.is_const)
        jb_names = sorted(sorted(g_read, key=lambda n: (uses[n], int(n[1:])))[:int(jb_mem)], key=lambda n: int(n[1:]))
    else:
        jb_names = []
    jidx = {n: nz + j for j, n in enumerate(jb_names)}
    g_reg = [n for n in g_read if n not in jidx]          # current adjoints held as locals
    nzb = nz + len(jidx)
    if zb_mem:
        out.append(f'// (in place: slot i at zb[i * ZS], {nzb} slots: the {nz} inputs'
                   + (f', then the {len(jidx)} current components the quark line reads)' if jb_mem else ')'))
        out.append('template <typename R, int ZS>')
        out.append(f'__device__ __forceinline__ void {fn}_adjoint(const R (&z)[{nz}], R* zb, R& me)')
    else:
        out.append('template <typename R>')
        out.append(f'__device__ __forceinline__ void {fn}_adjoint(const R (&z)[{nz}], R (&zb)[{nz}], R& me)')
    out.append('{')
    body = []

    def zlv(n):
        """lvalue of the adjoint of input n (None: no derivative)"""
        if not zb_mem:
            return _adj_lvalue(n)
        if n.startswith('lam'):
            return None
        if n in zidx:
            return f'zb[{zidx[n]} * ZS]'
        if n in jidx:
            return f'zb[{jidx[n]} * ZS]'
        return _adj_lvalue(n)                 # ubs: the current top helicity's row, local
    if zb_mem:
        body += [f'zb[{i} * ZS] = R(0);' for i in range(nz)]
    # unpack z into the names the recursion reads; accumulators for their adjoints
    arrays = {}
    scalars = []
    for i, n in enumerate(slots):
        if '[' in n:
            base = n[:n.index('[')]
            arrays.setdefault(base, []).append((n, i))
        else:
            scalars.append((n, i))
    dims = {'ub': '[2][4]', 'vs': '[2][4]', 'PT': '[4]'}
    for base, items in arrays.items():
        if base in ('ub', 'vs'):
            body.append(f'cplx<R> {base}[2][4] = {{}};')
            if not zb_mem:
                body.append(f'cplx<R> {base}_b[2][4] = {{}};')
        else:
            size = max(int(n[len(base) + 1:].split(']')[0]) for n, _ in items) + 1
            body.append(f'R {base}[{size}] = {{}};')
            if not zb_mem:
                body.append(f'R {base}_b[{size}] = {{}};')
        for n, i in items:
            body.append(f'{n} = z[{i}];')
    for n, i in scalars:
        body.append(f'const R {n} = z[{i}];')
        if not zb_mem:
            body.append(f'R {n}_b = R(0);')
    opq = []
    if opaque_inputs:
        for gi, leg in enumerate(proc.gl_legs):
            comps = [0] if leg < 2 else [0, 1, 2, 3]
            opq += [f'opaque(K{gi}[{c}]);' for c in comps]
        opq += [f'opaque(PT[{c}]);' for c in range(4)]
    body.append('#pragma unroll 1')
    body.append(f'for (int gconf = {2 ** (k - 1)}; gconf < {2 ** k}; ++gconf) {{   // last gluon: helicity +1')
    body += ['    ' + l for l in opq]
    for gi in range(k):
        body.append(f'    const R lam{gi} = (gconf >> {gi}) & 1 ? R(1) : R(-1);')
    if not recompute_currents:
        body += ['    ' + l for l in ir.gluon_lines]
    body += [f'    zb[{jidx[n]} * ZS] = R(0);' for n in jb_names]
    if not recompute_currents:
        body += [f'    R {n}_b = R(0);' for n in g_reg]
    q_temps_extra = set(g_reg)
    q_declared = g_reg
    body.append('    #pragma unroll 1')
    body.append('    for (int ht = 0; ht < 2; ++ht) {')
    body += ['        ' + l for l in opq]
    if group_barriers:
        body.append('        __builtin_amdgcn_sched_barrier(0);')
    body.append('        cplx<R> ubs[4], ubs_b[4] = {};')
    body.append('        for (int j = 0; j < 4; ++j) ubs[j] = ht ? ub[1][j] : ub[0][j];')
    if recompute_currents:
        body += ['        ' + l for l in ir.gluon_lines]
    body += ['        ' + l for l in q.lines]
    body += ['        ' + l for l in cs.lines]
    body.append(f'        me += {cs.ref(ir.csq[0])} + {cs.ref(ir.csq[1])};')
    rec_q = 0
    if recompute_currents:
        # colour sums backwards to the amplitudes, then quark line and currents per ordering
        amp_names = {base_sign(x)[0] for row in ir.amps for a in row for x in (a.re, a.im) if not x.is_const}
        aq = Adjoint(set(defined_names(cs.ops)) | amp_names, zlv)
        for h in range(2):
            aq.seed(ir.csq[h], 'R(1)')
        aq.sweep(cs.ops)
        if group_barriers:
            body.append('        __builtin_amdgcn_sched_barrier(0);')
        body += ['        ' + l for l in aq.lines]
        glines, rec_q, sw = _ordering_sweeps_with_currents(proc, ir, zlv, group_barriers)
        body += ['        ' + l for l in glines]
        aq.flops += sw
    elif regroup:
        # colour sums backwards to the amplitudes, then the quark line group by group
        amp_names = {base_sign(x)[0] for row in ir.amps for a in row for x in (a.re, a.im) if not x.is_const}
        aq = Adjoint(set(defined_names(cs.ops)) | amp_names, zlv)
        for h in range(2):
            aq.seed(ir.csq[h], 'R(1)')
        aq.sweep(cs.ops)
        if group_barriers:
            body.append('        __builtin_amdgcn_sched_barrier(0);')
        body += ['        ' + l for l in aq.lines]
        glines, rec_q, sw = _regrouped_quark_sweeps(proc, ir, g_reg, zlv, group_barriers, depth=group_depth)
        body += ['        ' + l for l in glines]
        aq.flops += sw
    else:
        aq = Adjoint(set(qc_temps) | q_temps_extra, zlv, declared=q_declared)
        for h in range(2):
            aq.seed(ir.csq[h], 'R(1)')
        aq.sweep(qc_ops)
        if group_barriers:
            body.append('        __builtin_amdgcn_sched_barrier(0);')
        body += ['        ' + l for l in aq.lines]
    if zb_mem:
        for j in range(4):
            for part in ('re', 'im'):
                i0, i1 = zidx.get(f'ub[0][{j}].{part}'), zidx.get(f'ub[1][{j}].{part}')
                if i0 is not None:
                    body.append(f'        {{ R& t = zb[(ht ? {i1} : {i0}) * ZS]; t = t + ubs_b[{j}].{part}; }}')
    else:
        body.append('        for (int j = 0; j < 4; ++j) {')
        body.append('            cplx<R>& t = ht ? ub_b[1][j] : ub_b[0][j];')
        body.append('            t.re += ubs_b[j].re;')
        body.append('            t.im += ubs_b[j].im;')
        body.append('        }')
    body.append('    }')
    body += [f'    R {n}_b = zb[{jidx[n]} * ZS];' for n in jb_names]
    ag = Adjoint(g_set, zlv, declared=g_read)
    if not recompute_currents:
        # recompute the gluon currents (renamed), then sweep them backwards
        import re as _re
        ren = lambda n: 'tr' + n[1:] if n in g_set else n       # noqa: E731
        rec_lines = [_re.sub(r'\bt(\d+)\b', r'tr\1', l) for l in ir.gluon_lines]
        if group_barriers:
            body.append('    __builtin_amdgcn_sched_barrier(0);')
        body += ['    ' + l for l in rec_lines]
        ag = Adjoint(g_set, zlv, declared=g_read, val=ren)
        ag.sweep(b.ops)
        body += ['    ' + l for l in ag.lines]
    body.append('}')
    if not zb_mem:
        for i, n in enumerate(slots):
            if n.startswith(('ub[', 'vs[')):
                body.append(f'zb[{i}] = {n[:2]}_b{n[2:]};')
            else:
                body.append(f'zb[{i}] = {_adj_lvalue(n)};')
    out += ['    ' + l for l in body]
    out.append('}')
    if recompute_currents:
        per_gconf = 2 * (ir.gluon_flops + ir.quark_flops + rec_q + ir.colour_flops + 1 + aq.flops)
    else:
        per_gconf = 2 * ir.gluon_flops + ag.flops + 2 * (ir.quark_flops + rec_q + ir.colour_flops + 1 + aq.flops)
    flops = dict(adjoint_per_event=(2 ** (k - 1)) * per_gconf, kin_slots=len(slots),
                 adjoint_gluon_sweep=ag.flops, adjoint_quark_colour_sweep=aq.flops)
    out.append(f'// flops per event of the adjoint (generated count): {flops}')
    n = proc.n_ext
    out += ['',
            'namespace mf {',
            'template <int K> struct AdjProc;',
            f'template <> struct AdjProc<{k}> {{',
            f'    static constexpr int NZ = {len(slots)};',
            f'    static constexpr int NZB = {nzb if zb_mem else 0};        // slots of zb in memory (0: registers)',
            '    template <typename KT, typename Out>',
            f'    __device__ static __forceinline__ void kin(const KT (&p)[{n}][4], const KT mt, Out& o) '
            f'{{ {fn}_kin<KT>(p, mt, o); }}',
            '    template <typename R, int ZS>',
            f'    __device__ static __forceinline__ void adjoint(const R (&z)[NZ], R* zb, R& me) '
            + (f'{{ {fn}_adjoint<R, ZS>(z, zb, me); }}' if zb_mem else
               f'{{ {fn}_adjoint<R>(z, *reinterpret_cast<R (*)[NZ]>(zb), me); }}'),
            '    // 2 (reversed helicities) / (initial average * identical final gluons * colour denominator)',
            f'    static constexpr double norm = 2.0 / ({proc.avg!r} * {float(proc.sym)!r} * {float(proc.cden)!r});',
            '};',
            '}  // namespace mf']
    return '\n'.join(out), flops


def colour_table(proc):
    return proc.cnum, proc.cden


# Per-lane LDS budgets (working-type scalars) for the LDS-parking variants:
# at one wave per SIMD a wave may own 40 KB of the 160 KB LDS, i.e. 160 floats
# or 80 doubles per lane.
LDS_F32 = 152
LDS_F64 = 72
# The four-lanes-per-event FP64 kernel runs two waves per compute unit: 80 KB of
# LDS per wave, 160 doubles per lane.
LDS_QUAD_F64 = 152
# The two-lanes-per-event FP64 kernel runs one wave per SIMD with 80 doubles of
# LDS per lane: 4 x 40 KB, the whole 160 KB of a compute unit.
LDS_PAIR_F64 = 80
# Shared quark-line products (Recursion.start_quark_line): 13% fewer flops for
# gg -> ttbar gg.  The FP32 kernels run faster with them.  The FP64 kernel, whose
# working set already spills, runs slower (the shared values add to the spill), so it
# keeps the plain form.
SHARE_F32 = True
SHARE_F64 = False
# The FP32 body with the colour form on the VALU does not share products: its
# build with them (half helicity loop) returned wrong, run-to-run varying values
# on the GPU, while the same source is exact on the CPU.  Without them it has
# no spill and is deterministic; it costs 6%.
SHARE_F32_VALU = False


# The derivative kernels: the adjoints of z accumulate in LDS (zb_mem) and the quark
# line is swept one colour ordering at a time, each recomputed from an opaque copy of
# the top spinor (regroup, group_depth = number of gluons).  Measured against the
# register form with the whole quark line swept at once: gg -> ttbar g 9.81 -> 8.27 ms
# (FP32) and 47.3 -> 38.5 ms (FP64) on 4e6 events; gg -> ttbar gg 39.6 -> 28.6 ms
# (FP32) and 93.2 -> 82.5 ms (FP64) on 2^18 events.  For gg -> ttbar g, the 20 least
# read current adjoints in LDS too (jb_mem; 39.9 KB per wave in FP64, the most that
# leaves four waves per compute unit): FP64 38.6 -> 33.3 ms, FP32 unchanged (8.25 vs
# 8.36 ms).  For gg -> ttbar gg, 78 of them (40 KB per wave in FP32) was slower
# (28.5 -> 29.2 ms), and in FP64 its z slots alone take 42 KB.  Recomputing the gluon
# currents per ordering as well (recompute_currents: no current lives across orderings,
# 40% more flops for gg -> ttbar g) was slower for gg -> ttbar g (FP32 8.3 -> 10.9 ms, FP64
# 33.5 -> 49.0 ms), and gg -> ttbar gg in that form took over 30 minutes to compile.
ADJ_OPTS = {
    'gg_tt': dict(zb_mem=True, regroup=True, group_depth=2),
    'gg_ttg': dict(zb_mem=True, regroup=True, group_depth=3, jb_mem=20),
    'gg_ttgg': dict(zb_mem=True, regroup=True, group_depth=4),
}


def _variant(proc, name, suffix, **kw):
    src, info = emit_qcd(proc, **kw)
    return src.replace(f'me_{name}_body', f'me_{name}_{suffix}', 1) if suffix != 'body' else src, info


def emit_all(outdir, **opts):
    os.makedirs(outdir, exist_ok=True)
    summary = {}
    for name, n_ext in (('gg_tt', 4), ('gg_ttg', 5), ('gg_ttgg', 6)):
        proc = GGTTProcess(name, n_ext)
        src, flops = emit_qcd(proc, with_colour=True, **opts)
        # large process: LDS-parking variants for the FP32 (VALU and matrix-core colour) and FP64 kernels
        lds = n_ext >= 6
        src_a, ia = _variant(proc, name, 'amps', with_colour=False, lds_budget=LDS_F32 if lds else 0,
                             share_products=SHARE_F32, **opts)
        extra = []
        if lds:
            s32, i32 = _variant(proc, name, 'body_lds32', with_colour=True, lds_budget=LDS_F32, constants=False,
                                share_products=SHARE_F32_VALU, **opts)
            s64, i64 = _variant(proc, name, 'body_lds64', with_colour=True, lds_budget=LDS_F64, constants=False,
                                share_products=SHARE_F64, **opts)
            extra = [s32, s64,
                     f'constexpr int me_{name}_lds32_slots = {i32["lds_slots"]};',
                     f'constexpr int me_{name}_lds64_slots = {i64["lds_slots"]};',
                     f'constexpr int me_{name}_amps_slots = {ia["lds_slots"]};']
            flops['lds_slots_f32'] = i32['lds_slots']
            flops['lds_slots_f64'] = i64['lds_slots']
        # flops per event of the forms the kernels execute (colour form counted in both)
        flops['per_event_f64'] = emit_qcd(proc, share_products=SHARE_F64 and lds)[1]['per_event']
        flops['per_event_f32'] = emit_qcd(proc, share_products=SHARE_F32)[1]['per_event']
        flops['per_event_f32_valu'] = emit_qcd(proc, share_products=SHARE_F32_VALU and lds)[1]['per_event']
        cnum, cden = proc.cnum, proc.cden
        ctab = [f'// colour matrix numerators for {name} (denominator {cden})',
                f'static __constant__ const short me_{name}_cnum[{len(cnum)}][{len(cnum)}] = {{']
        for row in cnum:
            ctab.append('    {' + ', '.join(str(v) for v in row) + '},')
        ctab.append('};')
        ctab.append(f'constexpr int me_{name}_cden = {cden};')
        with open(os.path.join(outdir, f'me_{name}.inc'), 'w') as f:
            f.write('// Generated by paper_2211_14056_amd.gen.process_compiler -- do not edit.\n')
            f.write(src + '\n\n' + src_a + '\n\n' + '\n\n'.join(extra) + '\n\n' + '\n'.join(ctab) + '\n')
        if proc.k == 4:
            # four lanes per event (FP64 kernel), in a file of its own
            from . import lane_split
            src_q, info_q = lane_split.emit_split(proc, LDS_QUAD_F64, local_memo=True)
            with open(os.path.join(outdir, f'me_{name}_quad.inc'), 'w') as f:
                f.write('// Generated by paper_2211_14056_amd.gen.lane_split -- do not edit.\n')
                f.write(src_q + '\n\n' + f'constexpr int me_{name}_quad_slots = {info_q["lds_slots"]};\n')
                f.write(f'__host__ __device__ constexpr double me_{name}_quad_norm_noalpha() '
                        f'{{ return 2.0 / ({proc.avg!r} * {float(proc.sym)!r} * {float(proc.cden)!r}); }}\n')
            flops['quad_executed_per_event'] = info_q['executed_per_event']
            # two lanes per event (the default FP64 layout), in a file of its own
            src_p, info_p = lane_split.emit_pair(proc, LDS_PAIR_F64, local_memo=True)
            with open(os.path.join(outdir, f'me_{name}_pair.inc'), 'w') as f:
                f.write('// Generated by paper_2211_14056_amd.gen.lane_split -- do not edit.\n')
                f.write(src_p + '\n\n' + f'constexpr int me_{name}_pair_slots = {info_p["lds_slots"]};\n')
                f.write(f'__host__ __device__ constexpr double me_{name}_pair_norm_noalpha() '
                        f'{{ return 2.0 / ({proc.avg!r} * {float(proc.sym)!r} * {float(proc.cden)!r}); }}\n')
            flops['pair_executed_per_event'] = info_p['executed_per_event']
        # reverse-sweep derivative: kinematic inputs and the adjoint of the recursion
        src_adj, info_adj = emit_qcd_adjoint(proc, **ADJ_OPTS[name])
        with open(os.path.join(outdir, f'me_{name}_adj.inc'), 'w') as f:
            f.write('// Generated by paper_2211_14056_amd.gen.process_compiler -- do not edit.\n')
            f.write(src_adj + '\n')
        flops.update(info_adj)
        summary[name] = flops
    # gg -> ttbar ggg: tables of the table-driven recursion (one wavefront per event)
    from . import bg_tables
    src_bg, _ = bg_tables.emit(5, 'bg5')
    with open(os.path.join(outdir, 'me_bg_k5.inc'), 'w') as f:
        f.write('// Generated by paper_2211_14056_amd.gen.bg_tables -- do not edit.\n')
        f.write(src_bg)
    summary['gg_ttggg'] = bg_tables.flops(5)
    # the processes with two quark lines: generated diagram code (one lane per event)
    from . import quark_lines
    for qp in quark_lines.PROCESSES:
        src_q, info_q = quark_lines.emit(qp)
        with open(os.path.join(outdir, f'me_{qp}.inc'), 'w') as f:
            f.write('// Generated by paper_2211_14056_amd.gen.quark_lines -- do not edit.\n')
            f.write(src_q)
        info_q.update(per_event_f64=info_q['per_event'], per_event_f32=info_q['per_event'],
                      per_event_f32_valu=info_q['per_event'])
        summary[qp] = info_q
    with open(os.path.join(outdir, 'flops.txt'), 'w') as f:
        for name, fl in summary.items():
            f.write(f'{name} {fl}\n')
    return summary


if __name__ == '__main__':
    import sys
    print(emit_all(sys.argv[1] if len(sys.argv) > 1 else 'generated'))
