"""Machine-code check of the matrix-core kernels as built (CPU only; reads our own gfx950 objects).

An MFMA that takes as its accumulator (SrcC) the result of an MFMA of another shape
cannot use the accumulator forwarding of a same-shape chain and must wait for the
first one to finish.  With a 32x32x16 BF16 result read by a 32x32x8 BF16 MFMA, the
compiler asked for 16 wait states in a small kernel but left as few as 12 in the
large gg -> ttbar gg kernel, and that kernel returned wrong, timing-dependent colour
sums.  The colour sink therefore chains only MFMAs of one shape per accumulator.
This test disassembles the gfx950 code objects of the translation units that hold
matrix-core kernels and checks that invariant in every function.
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, 'paper_2211_14056_amd', '_build')
LLVM = '/opt/rocm/llvm/bin'
OBJECTS = ['me_mfma.o', 'me_batch_mfma.o']
TARGET = 'hipv4-amdgcn-amd-amdhsa--gfx950'

REG = re.compile(r'\b([va])\[(\d+):(\d+)\]|\b([va])(\d+)\b')


def regs(text):
    out = set()
    for m in REG.finditer(text):
        if m.group(1):
            out |= {(m.group(1), i) for i in range(int(m.group(2)), int(m.group(3)) + 1)}
        else:
            out.add((m.group(4), int(m.group(5))))
    return out


def disassemble(obj, tmp):
    fat = os.path.join(tmp, 'fatbin.bin')
    co = os.path.join(tmp, 'device.co')
    subprocess.run([f'{LLVM}/llvm-objcopy', f'--dump-section=.hip_fatbin={fat}', obj, os.path.join(tmp, 'x.o')],
                   check=True, capture_output=True)
    subprocess.run([f'{LLVM}/clang-offload-bundler', '--unbundle', '--type=o', f'--targets={TARGET}',
                    f'--input={fat}', f'--output={co}'], check=True, capture_output=True)
    r = subprocess.run([f'{LLVM}/llvm-objdump', '-d', '--mcpu=gfx950', co], check=True, capture_output=True,
                       text=True)
    return r.stdout


def functions(listing):
    """{name: [instruction text]} from an llvm-objdump listing."""
    out, cur = {}, None
    for line in listing.splitlines():
        m = re.match(r'^[0-9a-f]+ <(.+)>:$', line)
        if m:
            cur = out.setdefault(m.group(1), [])
            continue
        s = line.split('//')[0].strip()
        if cur is not None and s and not s.endswith(':'):
            cur.append(s)
    return out


def cross_shape_srcc(insts):
    """(writer, reader) opcode pairs where an MFMA reads as SrcC the result of an MFMA of
    another opcode, looking back to the most recent MFMA that wrote any of those registers."""
    found = []
    for i, s in enumerate(insts):
        op = s.split()[0]
        if not op.startswith('v_mfma'):
            continue
        ops = [o.strip() for o in s[len(op):].split(',')]
        srcc = regs(ops[3]) if len(ops) > 3 else set()
        if not srcc:
            continue
        for j in range(i - 1, -1, -1):
            pop = insts[j].split()[0]
            if pop.startswith('v_mfma') and regs(insts[j][len(pop):].split(',')[0]) & srcc:
                if pop != op:
                    found.append((pop, op, j, i))
                break
    return found


def test_cross_shape_checker_finds_a_planted_chain():
    insts = ['v_mfma_f32_32x32x16_bf16 a[0:15], a[104:107], v[94:97], 0',
             'v_perm_b32 v107, v88, v68, s16',
             'v_mfma_f32_32x32x8_bf16 a[0:15], a[68:69], v[106:107], a[0:15]',
             'v_mfma_f32_32x32x8_bf16 a[0:15], a[68:69], v[104:105], a[0:15]']
    assert [(w, r) for w, r, _, _ in cross_shape_srcc(insts)] == [('v_mfma_f32_32x32x16_bf16',
                                                                   'v_mfma_f32_32x32x8_bf16')]
    assert cross_shape_srcc(insts[:1] + insts[1:2] + [insts[0].replace(', 0', ', a[0:15]')]) == []


@pytest.mark.skipif(not all(os.path.exists(f'{LLVM}/{t}') for t in ('llvm-objdump', 'llvm-objcopy',
                                                                   'clang-offload-bundler')),
                    reason='needs the ROCm LLVM tools')
@pytest.mark.parametrize('obj', OBJECTS)
def test_no_mfma_reads_an_accumulator_of_another_shape(tmp_path, obj):
    path = os.path.join(BUILD, obj)
    if not os.path.exists(path):
        pytest.skip(f'{obj} not built')
    funcs = functions(disassemble(path, str(tmp_path)))
    kernels = {k: v for k, v in funcs.items() if any(s.startswith('v_mfma') for s in v)}
    assert kernels, 'no matrix-core kernel found'
    bad = {k: cross_shape_srcc(v) for k, v in kernels.items()}
    bad = {k: v for k, v in bad.items() if v}
    assert not bad, {k: v[:3] for k, v in bad.items()}
