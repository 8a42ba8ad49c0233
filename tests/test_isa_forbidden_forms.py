"""Machine-code check of every gfx950 code object the library is built from (CPU only).

Two instruction families stay out of the device code:

* packed FP32 arithmetic (the two-lane FP32 add, multiply and FMA): the build turns
  the target feature off, because some of these forms have returned wrong values,
  silently, on the hardware this library runs on; the compiler would otherwise form
  them from plain float code;
* writes through the scalar data cache (scalar stores and atomics, its write-back
  and discard): all device writes go through vector memory instructions.

The check disassembles our own objects and looks at every instruction of every
function.
"""
import os
import re
import subprocess
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_isa_mfma_chains import BUILD, LLVM, disassemble, functions  # noqa: E402

PACKED_F32 = re.compile(r'^v_pk_(fma|mul|add)_f32$')
SCALAR_WRITE = re.compile(r'^s_(store|buffer_store|scratch_store|atomic|buffer_atomic|dcache_wb|dcache_discard)')

TOOLS = all(os.path.exists(f'{LLVM}/{t}') for t in ('llvm-objdump', 'llvm-objcopy', 'clang-offload-bundler'))


def forbidden(insts):
    return sorted({s.split()[0] for s in insts
                   if PACKED_F32.match(s.split()[0]) or SCALAR_WRITE.match(s.split()[0])})


def test_checker_flags_planted_instructions():
    good = ['v_fma_f32 v1, v2, v3, v4', 'v_pk_fma_f16 v1, v2, v3, v4', 'global_store_dword v[0:1], v2, off',
            's_load_dwordx2 s[0:1], s[4:5], 0x0', 'v_pk_mov_b32 v[0:1], v[2:3], v[4:5]']
    assert forbidden(good) == []
    bad = good + ['v_pk_fma_f32 v[0:1], v[2:3], v[4:5], v[6:7]', 's_store_dword s0, s[2:3], 0x0',
                  's_dcache_wb']
    assert forbidden(bad) == ['s_dcache_wb', 's_store_dword', 'v_pk_fma_f32']


def _objects():
    if not os.path.isdir(BUILD):
        return []
    return sorted(o for o in os.listdir(BUILD) if o.endswith('.o'))


@pytest.mark.skipif(not TOOLS, reason='needs the ROCm LLVM tools')
def test_no_packed_fp32_and_no_scalar_writes(tmp_path):
    objs = _objects()
    if not objs:
        pytest.skip('library not built')
    seen, checked, bad = 0, set(), {}
    for o in objs:
        d = tmp_path / o
        d.mkdir()
        try:
            listing = disassemble(os.path.join(BUILD, o), str(d))
        except subprocess.CalledProcessError:
            continue                            # host-only translation unit: no device code object
        checked.add(o)
        for name, insts in functions(listing).items():
            seen += len(insts)
            f = forbidden(insts)
            if f:
                bad[f'{o}:{name}'] = f
    assert seen > 0, 'no device code found'
    kernels = {'me_mfma.o', 'me_batch_mfma.o', 'me_ttgg_pair.o', 'me_kernels.o', 'phase_space.o', 'vegas.o'}
    assert kernels <= checked, sorted(kernels - checked)
    assert not bad, bad
