"""Reverse-mode (adjoint) code for straight-line IR blocks.

Every statement of an IR block is one add, multiply, fused multiply-add or copy
of named scalars (``ir.Block.ops``).  The adjoint of a block walks its
statements backwards and propagates the adjoint of each result to its operands
with the exact first-order rules

    r = a + b        abar += rbar,        bbar += rbar
    r = a * b        abar += rbar * b,    bbar += rbar * a
    r = a * b + c    abar += rbar * b,    bbar += rbar * a,    cbar += rbar
    r = a            abar += rbar

(a negated operand takes the contribution with the opposite sign; constants
take none).  The forward values the rules read (the multiplicands) must be in
scope where the adjoint code runs: the caller emits the forward statements, or a
renamed recomputation of them, before it.

Adjoint variables are named after the forward temporaries with a ``_b``
suffix and are declared at their first contribution.  Operands that the block
does not define (its inputs) take their contributions through ``ext_adj``,
which maps an input name to the lvalue of its accumulator, or to None for an
input with no derivative (a helicity sign).
"""
from .ir import S


def base_sign(x):
    """(name, sign) of a variable operand, unwrapping a negated reference '(-name)'."""
    n = x.name
    sgn = 1
    while n.startswith('(-') and n.endswith(')'):
        n = n[2:-1]
        sgn = -sgn
    return n, sgn


class Adjoint:
    """Emits the reverse sweep of IR statements.

    declared: adjoint variables that already exist in scope (accumulated into with
      ``+=`` forms); every other temporary is declared at its first contribution.
    temps: the names defined by the blocks being differentiated (all others are inputs).
    ext_adj: input name -> accumulator lvalue, or None (no derivative).
    val: forward name -> name of the value to read (identity, or a renamed recomputation).
    """

    def __init__(self, temps, ext_adj, declared=(), val=None, rtype='R'):
        self.temps = set(temps)
        self.ext_adj = ext_adj
        self.declared = set(declared)
        self.val = val or (lambda n: n)
        self.rtype = rtype
        self.lines = []
        self.flops = 0

    def ref_val(self, x):
        if x.is_const:
            v = x.val
            return f'R({int(v)})' if v == int(v) and abs(v) < 1e15 else f'R({v!r})'
        n, sgn = base_sign(x)
        v = self.val(n)
        return v if sgn > 0 else f'(-{v})'

    def _contribute(self, target, rb, coeff, sign):
        """target_bar += sign * rb * coeff (coeff None = 1)."""
        if target.is_const:
            return
        n, s2 = base_sign(target)
        sign *= s2
        if coeff is not None and coeff.is_const:
            if coeff.val == 0.0:
                return
            if coeff.val in (1.0, -1.0):
                sign *= int(coeff.val)
                coeff = None
        if n in self.temps:
            lv = f'{n}_b'
            first = n not in self.declared
            self.declared.add(n)
        else:
            lv = self.ext_adj(n)
            if lv is None:
                return
            first = False
        src = rb if sign > 0 else f'(-{rb})'
        if coeff is None:
            if first:
                self.lines.append(f'{self.rtype} {lv} = {src};')
            else:
                self.lines.append(f'{lv} = {lv} + {src};')
                self.flops += 1
        else:
            c = self.ref_val(coeff)
            if first:
                self.lines.append(f'{self.rtype} {lv} = {src} * {c};')
                self.flops += 1
            else:
                self.lines.append(f'{lv} = fma({src}, {c}, {lv});')
                self.flops += 2

    def sweep(self, ops):
        """Reverse sweep over ``ops`` (a block's statements in forward order)."""
        for kind, name, operands in reversed(ops):
            if name not in self.declared:
                continue                         # adjoint is zero: nothing uses this value
            rb = f'{name}_b'
            if kind == 'add':
                a, b = operands
                self._contribute(a, rb, None, 1)
                self._contribute(b, rb, None, 1)
            elif kind == 'mul':
                a, b = operands
                self._contribute(a, rb, b, 1)
                self._contribute(b, rb, a, 1)
            elif kind == 'fma':
                a, b, c = operands
                self._contribute(a, rb, b, 1)
                self._contribute(b, rb, a, 1)
                self._contribute(c, rb, None, 1)
            elif kind == 'copy':
                self._contribute(operands[0], rb, None, 1)
            else:
                raise ValueError(f'cannot differentiate through {kind} statement {name}')

    def seed(self, x, expr):
        """Start the adjoint of result x at expr (declaring it)."""
        if x.is_const:
            return
        n, sgn = base_sign(x)
        src = expr if sgn > 0 else f'(-{expr})'
        if n in self.temps:
            if n in self.declared:
                self.lines.append(f'{n}_b = {n}_b + {src};')
                self.flops += 1
            else:
                self.lines.append(f'{self.rtype} {n}_b = {src};')
                self.declared.add(n)
        else:
            lv = self.ext_adj(n)
            if lv is not None:
                self.lines.append(f'{lv} = {lv} + {src};')
                self.flops += 1


def operand_names(ops):
    """Variable names (negation unwrapped) read by the statements ``ops``."""
    out = set()
    for _, _, operands in ops:
        for x in operands:
            if isinstance(x, S) and not x.is_const:
                out.add(base_sign(x)[0])
    return out


def defined_names(ops):
    return [name for _, name, _ in ops]
