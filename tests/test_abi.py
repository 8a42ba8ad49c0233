"""CPU-side checks of the C ABI: the library loads and exports every declared symbol.

No compute call is made here (no GPU in this environment)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, 'include', 'mf.h')
LIB = os.path.join(ROOT, 'paper_2211_14056_amd', 'libmfhip.so')


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r'/\*.*?\*/', '', src, flags=re.S)
    names = re.findall(r'\b(mf_[a-z_]+)\s*\(', src)
    return sorted(set(n for n in names if not n.endswith('_t')))


def test_header_declares_the_four_hot_path_entry_points():
    names = declared_functions()
    for n in ('mf_phase_space', 'mf_matrix_element', 'mf_matrix_element_vjp', 'mf_vegas_refine'):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason='library not built')
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(L, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason='library not built')
def test_host_only_helpers():
    L = ctypes.CDLL(LIB)
    assert [L.mf_process_legs(i) for i in range(10)] == [4, 4, 5, 6, 7, 4, 5, 6, 5, 6]
    assert [L.mf_process_dims(i) for i in range(10)] == [2, 2, 5, 8, 11, 2, 5, 8, 5, 8]
    assert L.mf_process_legs(10) == -1 and L.mf_process_dims(-1) == -1
    L.mf_last_error.restype = ctypes.c_char_p
    # argument validation happens before any device work
    L.mf_create.argtypes = [ctypes.c_int, ctypes.c_void_p]
    assert L.mf_create(0, None) == -1
    assert b'NULL' in L.mf_last_error()


def test_binding_has_same_names_as_header():
    import paper_2211_14056_amd as mf
    for n in ('mf_phase_space', 'mf_matrix_element', 'mf_matrix_element_vjp', 'mf_vegas_refine'):
        assert callable(getattr(mf, n))


def test_binding_process_ids_match_header():
    import paper_2211_14056_amd as mf
    text = open(os.path.join(ROOT, 'include', 'mf.h')).read()
    body = re.search(r'typedef enum \{([^}]*)\} mf_process;', text).group(1)
    ids = {k: int(v) for k, v in re.findall(r'(MF_[A-Z_]+) = (\d+)', body)}
    assert len(ids) == 10
    for name, v in ids.items():
        assert getattr(mf, name) == v, name
        assert mf.PROCESS[name[3:].lower()] == v


def test_generated_colour_matrices_match_oracle_brute_force():
    import numpy as np
    from oracle import colour
    from paper_2211_14056_amd.gen import colour_algebra
    for k in (2, 3, 4, 5):
        num, den = colour_algebra.integer_form(colour_algebra.colour_matrix(k))
        assert np.abs(np.array(num) / den - colour.colour_matrix(k)).max() < 1e-13


def test_process_compiler_flop_counts_are_stable():
    from paper_2211_14056_amd.gen import process_compiler as pc
    p = pc.GGTTProcess('gg_tt', 4)
    _, fl = pc.emit_qcd(p)
    assert fl['helicities'] == 16 and fl['per_event'] > 0


def test_vegas_binding_rejects_a_matrix_element_of_another_dtype():
    """The binding accepts only float32 or float64 |M|^2: a half-precision buffer would be
    read as 8 bytes per event by the kernel.  The check runs before any device call."""
    import torch
    import paper_2211_14056_amd as mf
    n, d, nb = 8, 2, 50
    me = torch.zeros(n, dtype=torch.float16)
    with pytest.raises(ValueError, match='me: dtype'):
        mf.mf_vegas_refine(None, mf.params(), n, d, nb, 1.5, torch.zeros(n, dtype=torch.float64), None, me, None,
                           torch.zeros(d, n, dtype=torch.int16), torch.zeros(2 + d * nb, dtype=torch.float64),
                           torch.zeros(d, nb + 1, dtype=torch.float64))


@pytest.mark.skipif(not os.path.exists(LIB), reason='library not built')
def test_noalloc_vegas_validates_arguments_before_any_device_work():
    """mf_vegas_refine_noalloc rejects bad sizes and NULL buffers on the host."""
    import paper_2211_14056_amd as mf
    L = mf.lib()
    prm = mf.params()
    for n, d, nb in ((10, 17, 50), (10, 2, 65), (10, 2, 1), (-1, 2, 50)):
        st = L.mf_vegas_refine_noalloc(ctypes.byref(prm), n, d, nb, 1.5, None, None, None, 0, None, None, None,
                                       None, None, 0, None, None)
        assert st == -1, (n, d, nb)
    assert b'mf_vegas_refine_noalloc' in L.mf_last_error()
