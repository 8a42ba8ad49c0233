"""Machine-code hazard checks of every built device object (CPU only; reads our own gfx950 objects).

Some builds of the generated bodies computed wrong, launch-to-launch varying values on the GPU
while the same source is exact on the CPU. One cause was shown: a cross-shape MFMA accumulator
chain, which test_isa_mfma_chains.py now guards. This file checks the built code against further
issue rules of the CDNA3/CDNA4 instruction set. The compiler inserts wait states (s_nop or
independent instructions) or counter waits for these, and a miss would show up as exactly such
timing-dependent values:

  R1  a VALU writes a VGPR that a DPP instruction then reads as its source: 2 wait states;
  R2  a VALU writes EXEC (v_cmpx) ahead of a DPP instruction: 5 wait states;
  R3  a transcendental VALU result (rcp, rsq, sqrt, exp, log, sin, cos) read by the next
      non-transcendental VALU: 1 wait state;
  R4  a VALU writes an SGPR (or VCC) that a vector-memory instruction then reads: 5 wait states;
  R5  a VALU writes the SGPR that v_readlane / v_writelane then takes as lane select: 4;
  R6  a VALU writes VCC ahead of v_div_fmas: 4;
  R7  a register that an outstanding vector-memory or LDS load writes is read, or overwritten
      other than by a later load of the same counter, before an s_waitcnt that covers the load.  The model assumes that vmcnt retires in
      issue order, and that lgkmcnt does too while no scalar load is outstanding (otherwise
      only lgkmcnt(0) retires).  Code is scanned in program order, afresh after an
      unconditional jump.
  R8  a vector-memory store of more than 64 bits of data, then a VALU overwriting one of its
      data registers: 1 wait state.

Each rule is also run on a planted sequence that breaks it and must be flagged.
"""
import glob
import os
import re
import subprocess

import pytest

from test_isa_mfma_chains import BUILD, LLVM, disassemble, functions, regs

TRANS = re.compile(r'^v_(rcp|rsq|sqrt|exp|log|sin|cos|rcp_iflag)_')
SREG = re.compile(r'\bs\[(\d+):(\d+)\]|\bs(\d+)\b|\b(vcc|exec)\b')


def parse(ins):
    parts = ins.split(None, 1)
    rest = parts[1] if len(parts) > 1 else ''
    ops = [o.strip() for o in re.split(r',(?![^\[]*\])', rest)] if rest else []
    return parts[0], ops, rest


def sregs(text):
    out = set()
    for m in SREG.finditer(text):
        if m.group(1):
            out |= {('s', i) for i in range(int(m.group(1)), int(m.group(2)) + 1)}
        elif m.group(3):
            out.add(('s', int(m.group(3))))
        else:
            out.add((m.group(4), 0))
    return out


def is_valu(op):
    return op.startswith('v_')


def is_vmem(op):
    return op.split('_')[0] in ('buffer', 'global', 'scratch', 'flat')


def is_lds(op):
    return op.startswith('ds_')


def is_dpp(rest, op):
    return op.endswith('_dpp') or 'quad_perm' in rest or 'row_' in rest


def is_store(op):
    return 'store' in op or op.startswith('ds_write') or (op.startswith('ds_') and op[3:].split('_')[0] in
                                                          ('add', 'sub', 'min', 'max', 'and', 'or', 'xor')
                                                          and '_rtn' not in op)


def dst_src(ins):
    """(registers written, registers read) of one instruction, VGPR/AGPR/SGPR/VCC/EXEC."""
    op, ops, rest = parse(ins)
    if not ops:
        return set(), set()
    if is_vmem(op) or is_lds(op):
        returns = not ('atomic' in op and ' sc0' not in rest and ' glc' not in rest)
        if is_store(op) or not returns:
            return set(), regs(rest) | sregs(rest)
        tail = ', '.join(ops[1:])
        return regs(ops[0]), regs(tail) | sregs(tail)
    if is_valu(op):
        d = regs(ops[0]) | sregs(ops[0])
        src = ', '.join(ops[1:])
        if re.match(r'v_(add|sub|subrev|addc|subb|subbrev)_co|v_mad_[ui]64|v_div_scale', op) and len(ops) > 1:
            d |= sregs(ops[1])
            src = ', '.join(ops[2:])
        if '_e32' in op and re.match(r'v_(addc|subb|subbrev|cndmask)', op):
            src += ', vcc'
        return d, regs(src) | sregs(src)
    return sregs(ops[0]), sregs(', '.join(ops[1:]))


def wait_states(ins):
    op, ops, _ = parse(ins)
    return int(ops[0], 0) + 1 if op == 's_nop' else 1


def local_hazards(insts):
    """R1-R6 and R8 over straight-line windows (a window ends at a branch)."""
    found = []
    for i, x in enumerate(insts):
        op, ops, _ = parse(x)
        if not (is_valu(op) or is_vmem(op)):
            continue
        d, _ = dst_src(x)
        dv = {r for r in d if r[0] == 'v'}
        ds = {r for r in d if r[0] in ('s', 'vcc')}
        ws = 0
        for y in insts[i + 1:i + 9]:
            yop, yops, yrest = parse(y)
            if yop.startswith(('s_cbranch', 's_branch', 's_setpc', 's_endpgm')):
                break
            yd, ys = dst_src(y)
            if is_valu(op):
                if is_dpp(yrest, yop) and ws < 2 and len(yops) > 1 and dv & regs(yops[1]):
                    found.append(('R1', i, x, y))
                if op.startswith('v_cmpx') and is_dpp(yrest, yop) and ws < 5:
                    found.append(('R2', i, x, y))
                if TRANS.match(op) and is_valu(yop) and not TRANS.match(yop) and ws < 1 and dv & ys:
                    found.append(('R3', i, x, y))
                if is_vmem(yop) and ws < 5 and ds & sregs(yrest):
                    found.append(('R4', i, x, y))
                if yop in ('v_readlane_b32', 'v_writelane_b32') and ws < 4 and len(yops) > 2 and \
                        ds & sregs(yops[2]):
                    found.append(('R5', i, x, y))
                if yop.startswith('v_div_fmas') and ws < 4 and ('vcc', 0) in ds:
                    found.append(('R6', i, x, y))
            elif is_store(op) and re.search(r'x3|x4|b96|b128', op) and is_valu(yop) and ws < 1:
                data = regs(ops[1]) if op.startswith(('global', 'scratch', 'flat')) else regs(ops[0])
                if {r for r in yd if r[0] == 'v'} & data:
                    found.append(('R8', i, x, y))
            ws += wait_states(y)
    return found


def waitcnt_hazards(insts):
    """R7: accesses to the destination of a load whose counter wait has not been passed."""
    found = []
    vm, lg, smem = [], [], False
    for i, x in enumerate(insts):
        op, ops, rest = parse(x)
        if op in ('s_branch', 's_setpc_b64', 's_endpgm'):
            # the next instruction is reached by a jump only; the compiler waits for
            # everything outstanding where paths join, so the scan starts afresh there
            vm, lg, smem = [], [], False
            continue
        if op == 's_waitcnt':
            m = re.search(r'vmcnt\((\d+)\)', rest)
            if m and int(m.group(1)) < len(vm):
                vm = vm[len(vm) - int(m.group(1)):] if int(m.group(1)) else []
            m = re.search(r'lgkmcnt\((\d+)\)', rest)
            if m:
                k = int(m.group(1))
                if k == 0:
                    lg, smem = [], False
                elif not smem and k < len(lg):
                    lg = lg[len(lg) - k:]
            continue
        d, s = dst_src(x)
        pending = set().union(*vm, *lg)
        # a load may overwrite the target of an earlier load of its own counter: those
        # return in issue order, so the later value lands last
        same = set().union(*vm) if is_vmem(op) else set().union(*lg) if is_lds(op) and not smem else set()
        hit = (s & pending) | (d & (pending - same))
        if hit:
            found.append(('R7', i, x, sorted(hit)[:4]))
        if is_vmem(op):
            vm.append(d)
        elif is_lds(op):
            lg.append(d)
        elif op.startswith(('s_load', 's_buffer_load')):
            smem = True
            lg.append(d)
    return found


PLANTED = [
    ('R1', ['v_mov_b32_e32 v3, v4', 'v_mov_b32_dpp v1, v3 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf'],
     ['v_mov_b32_e32 v3, v4', 's_nop 1', 'v_mov_b32_dpp v1, v3 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf']),
    ('R2', ['v_cmpx_gt_f32_e32 vcc, v1, v2', 'v_mov_b32_dpp v1, v3 row_shl:1 row_mask:0xf bank_mask:0xf'],
     ['v_cmpx_gt_f32_e32 vcc, v1, v2', 's_nop 4', 'v_mov_b32_dpp v1, v3 row_shl:1 row_mask:0xf bank_mask:0xf']),
    ('R3', ['v_rcp_f32_e32 v8, v9', 'v_mul_f32_e32 v10, v8, v8'],
     ['v_rcp_f32_e32 v8, v9', 's_nop 0', 'v_mul_f32_e32 v10, v8, v8']),
    ('R4', ['v_readfirstlane_b32 s4, v1', 'global_load_dword v2, v3, s[4:5]'],
     ['v_readfirstlane_b32 s4, v1', 's_nop 4', 'global_load_dword v2, v3, s[4:5]']),
    ('R5', ['v_readfirstlane_b32 s4, v1', 'v_readlane_b32 s5, v2, s4'],
     ['v_readfirstlane_b32 s4, v1', 's_nop 3', 'v_readlane_b32 s5, v2, s4']),
    ('R6', ['v_div_scale_f32 v1, vcc, v2, v3, v2', 'v_div_fmas_f32 v4, v5, v6, v7'],
     ['v_div_scale_f32 v1, vcc, v2, v3, v2', 's_nop 3', 'v_div_fmas_f32 v4, v5, v6, v7']),
    ('R7', ['scratch_load_dword v5, off, s33 offset:16', 'v_add_f32_e32 v6, v5, v7'],
     ['scratch_load_dword v5, off, s33 offset:16', 's_waitcnt vmcnt(0)', 'v_add_f32_e32 v6, v5, v7']),
    ('R7', ['ds_read_b64 v[4:5], v1', 'ds_read_b32 v6, v1 offset:8', 's_waitcnt lgkmcnt(1)',
            'v_add_f32_e32 v7, v6, v6'],
     ['ds_read_b64 v[4:5], v1', 'ds_read_b32 v6, v1 offset:8', 's_waitcnt lgkmcnt(1)',
      'v_add_f32_e32 v7, v4, v5']),
    ('R8', ['global_store_dwordx4 v[0:1], v[4:7], off', 'v_mov_b32_e32 v5, 0'],
     ['global_store_dwordx4 v[0:1], v[4:7], off', 's_nop 0', 'v_mov_b32_e32 v5, 0']),
]


@pytest.mark.parametrize('rule,bad,good', PLANTED)
def test_checker_flags_planted_hazards(rule, bad, good):
    check = waitcnt_hazards if rule == 'R7' else local_hazards
    assert [f[0] for f in check(bad)] == [rule]
    assert check(good) == []


OBJECTS = sorted(os.path.basename(p) for p in glob.glob(os.path.join(BUILD, '*.o')) if not p.endswith('mf_api.o'))


@pytest.mark.skipif(not all(os.path.exists(f'{LLVM}/{t}') for t in ('llvm-objdump', 'llvm-objcopy',
                                                                   'clang-offload-bundler')),
                    reason='needs the ROCm LLVM tools')
@pytest.mark.skipif(not OBJECTS, reason='library not built')
@pytest.mark.parametrize('obj', OBJECTS)
def test_built_device_code_keeps_the_issue_rules(tmp_path, obj):
    try:
        funcs = functions(disassemble(os.path.join(BUILD, obj), str(tmp_path)))
    except subprocess.CalledProcessError:
        pytest.skip(f'{obj} holds no device code')
    assert funcs, 'no device function found'
    bad = {}
    for name, insts in funcs.items():
        f = local_hazards(insts) + waitcnt_hazards(insts)
        if f:
            bad[name] = f[:3]
    assert not bad, bad
