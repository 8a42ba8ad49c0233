"""Straight-line scalar IR with constant folding, emitted as HIP C++.

Every value is a real scalar: either a compile-time constant (a Python float)
or a named SSA variable of the generated code.  Complex numbers are pairs of
scalars and Lorentz vectors are lists of complex numbers, so zero components
known at generation time (polarisation time components, momenta of the beams
along the z axis, real parts of purely imaginary numbers) fold away and the
emitted code holds only the arithmetic that remains.

Each emitted statement is one multiply, add or fused multiply-add, so the
floating-point operation count of a block is known exactly (FMA = 2, add or
multiply = 1, negation and constant folding free).
"""


class S:
    """A real scalar: constant (val is not None) or variable (name)."""
    __slots__ = ('name', 'val')

    def __init__(self, name=None, val=None):
        self.name = name
        self.val = val

    @property
    def is_const(self):
        return self.val is not None

    def __repr__(self):
        return self.name if self.val is None else repr(self.val)


def const(x):
    return S(val=float(x))


ZERO = const(0.0)
ONE = const(1.0)


def _lit(x):
    if x == int(x) and abs(x) < 1e15:
        return f'R({int(x)})'
    return f'R({x!r})'


class Block:
    """Accumulates statements and counts flops."""

    def __init__(self, prefix, rtype='R'):
        self.prefix = prefix
        self.rtype = rtype
        self.lines = []
        self.count = 0
        self.flops = 0
        # structured record of every statement, in emission order, for the adjoint
        # emitter: (kind, name, operands) with kind 'add' (a + b), 'mul' (a * b),
        # 'fma' (a * b + c), 'copy' (a) or 'ext' (an expression the adjoint does not
        # differentiate through: an LDS read, a lane exchange)
        self.ops = []

    # ---------------------------------------------------------------- basics
    def ref(self, s):
        if s.is_const:
            return _lit(s.val)
        return s.name

    def new(self, expr, flops, op=None):
        name = f'{self.prefix}{self.count}'
        self.count += 1
        self.lines.append(f'const {self.rtype} {name} = {expr};')
        self.flops += flops
        kind, operands = op if op is not None else ('ext', (expr,))
        self.ops.append((kind, name, operands))
        return S(name=name)

    def var(self, name):
        return S(name=name)

    def neg(self, a):
        if a.is_const:
            return const(-a.val)
        if a.name.startswith('(-') and a.name.endswith(')'):
            return S(name=a.name[2:-1])
        return S(name=f'(-{a.name})')

    def add(self, a, b):
        if a.is_const and b.is_const:
            return const(a.val + b.val)
        if a.is_const and a.val == 0.0:
            return b
        if b.is_const and b.val == 0.0:
            return a
        if not a.is_const and not b.is_const and (b.name == f'(-{a.name})' or a.name == f'(-{b.name})'):
            return ZERO                          # x + (-x)
        return self.new(f'{self.ref(a)} + {self.ref(b)}', 1, ('add', (a, b)))

    def sub(self, a, b):
        return self.add(a, self.neg(b))

    def mul(self, a, b):
        if a.is_const and b.is_const:
            return const(a.val * b.val)
        if (a.is_const and a.val == 0.0) or (b.is_const and b.val == 0.0):
            return ZERO
        if a.is_const and a.val == 1.0:
            return b
        if b.is_const and b.val == 1.0:
            return a
        if a.is_const and a.val == -1.0:
            return self.neg(b)
        if b.is_const and b.val == -1.0:
            return self.neg(a)
        return self.new(f'{self.ref(a)} * {self.ref(b)}', 1, ('mul', (a, b)))

    def sumprod(self, terms, const_term=None):
        """sum_i a_i * b_i (+ c) as one fma chain; terms: list of (a, b)."""
        acc = const_term if const_term is not None else ZERO
        cval = 0.0
        live = []
        for a, b in terms:
            if a.is_const and b.is_const:
                cval += a.val * b.val
                continue
            if (a.is_const and a.val == 0.0) or (b.is_const and b.val == 0.0):
                continue
            live.append((a, b))
        if acc.is_const:
            cval += acc.val
            acc = None
        if not live:
            return const(cval) if acc is None else self.add(acc, const(cval))
        if acc is None and cval != 0.0:
            acc = const(cval)
        for a, b in live:
            if a.is_const and a.val in (1.0, -1.0):
                term = b if a.val == 1.0 else self.neg(b)
                acc = term if acc is None else self.add(acc, term)
                continue
            if b.is_const and b.val in (1.0, -1.0):
                term = a if b.val == 1.0 else self.neg(a)
                acc = term if acc is None else self.add(acc, term)
                continue
            if acc is None:
                acc = self.mul(a, b)
            else:
                acc = self.new(f'fma({self.ref(a)}, {self.ref(b)}, {self.ref(acc)})', 2, ('fma', (a, b, acc)))
        return acc

    def materialise(self, a):
        """Give a constant or negated reference a name of its own."""
        if a.is_const or a.name.startswith('('):
            return self.new(self.ref(a), 0, ('copy', (a,)))
        return a


class C:
    """Complex number as a pair of real scalars."""
    __slots__ = ('re', 'im')

    def __init__(self, re, im=ZERO):
        self.re = re
        self.im = im


CZERO = C(ZERO, ZERO)


def csum(b, pairs, const_c=None):
    """sum_i x_i * y_i for complex x_i, y_i as two fma chains."""
    re_t, im_t = [], []
    for x, y in pairs:
        re_t.append((x.re, y.re))
        re_t.append((x.im, b.neg(y.im)))
        im_t.append((x.re, y.im))
        im_t.append((x.im, y.re))
    cr = const_c.re if const_c is not None else None
    ci = const_c.im if const_c is not None else None
    return C(b.sumprod(re_t, cr), b.sumprod(im_t, ci))


def cmul(b, x, y):
    return csum(b, [(x, y)])


def cadd(b, x, y):
    return C(b.add(x.re, y.re), b.add(x.im, y.im))


def csub(b, x, y):
    return C(b.sub(x.re, y.re), b.sub(x.im, y.im))


def cneg(b, x):
    return C(b.neg(x.re), b.neg(x.im))


def creal(s):
    return C(s, ZERO)


def cmat(b, x):
    """Name both parts (for values reused many times)."""
    return C(b.materialise(x.re) if not x.re.is_const else x.re,
             b.materialise(x.im) if not x.im.is_const else x.im)
