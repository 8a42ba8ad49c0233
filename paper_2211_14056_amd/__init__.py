"""MI355X-native event-parallel matrix-element library (Python binding).

Thin ctypes binding over the C ABI in include/mf.h (libmfhip.so built by
``python -m paper_2211_14056_amd.build``).  Functions keep the C names and only
marshal arguments: device buffers are torch tensors on the GPU, work is
enqueued on torch's current stream, and every step of the computation runs in
the library's HIP kernels.  There is no fallback: if the library is missing
or no GPU is present, the calls raise.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, 'libmfhip.so')

MF_EE_MUMU, MF_GG_TT, MF_GG_TTG, MF_GG_TTGG, MF_GG_TTGGG = 0, 1, 2, 3, 4
MF_QQ_TT, MF_QQ_TTG, MF_QQ_TTGG, MF_QG_TTQ, MF_QG_TTQG = 5, 6, 7, 8, 9
PROCESS = {'ee_mumu': MF_EE_MUMU, 'gg_tt': MF_GG_TT, 'gg_ttg': MF_GG_TTG, 'gg_ttgg': MF_GG_TTGG,
           'gg_ttggg': MF_GG_TTGGG, 'qq_tt': MF_QQ_TT, 'qq_ttg': MF_QQ_TTG, 'qq_ttgg': MF_QQ_TTGG,
           'qg_ttq': MF_QG_TTQ, 'qg_ttqg': MF_QG_TTQG}
MF_FP64, MF_FP32, MF_FP32_MFMA_BF16, MF_FP32_MFMA_F32 = 0, 1, 2, 3
PRECISION = {'fp64': MF_FP64, 'fp32': MF_FP32, 'fp32_mfma_bf16': MF_FP32_MFMA_BF16,
             'fp32_mfma_f32': MF_FP32_MFMA_F32}
STATUS = {0: 'MF_OK', -1: 'MF_ERR_INVALID_ARG', -2: 'MF_ERR_UNSUPPORTED', -3: 'MF_ERR_HIP',
          -4: 'MF_ERR_NO_MEMORY'}


class MFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f'{STATUS.get(status, status)}: {msg}')
        self.status = status


class mf_params(ctypes.Structure):
    _fields_ = [('sqrt_s', ctypes.c_double), ('m_t', ctypes.c_double), ('alpha_s', ctypes.c_double),
                ('alpha', ctypes.c_double), ('pt_min', ctypes.c_double), ('eta_max', ctypes.c_double),
                ('dr_min', ctypes.c_double)]


class mf_request(ctypes.Structure):
    _fields_ = [('proc', ctypes.c_int32), ('reserved', ctypes.c_int32), ('n', ctypes.c_int64),
                ('p', ctypes.c_void_p), ('me_out', ctypes.c_void_p), ('x', ctypes.c_void_p),
                ('grad_me', ctypes.c_void_p), ('grad_x', ctypes.c_void_p), ('grad_theta', ctypes.c_void_p)]


class mf_pdf_grid(ctypes.Structure):
    _fields_ = [('nx', ctypes.c_int32), ('nq', ctypes.c_int32), ('log_x', ctypes.c_void_p),
                ('log_q2', ctypes.c_void_p), ('xf', ctypes.c_void_p)]


_lib = None
VP, I64, U64, I32, DBL = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_double


def lib():
    """Load libmfhip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f'{LIB_PATH} not found: build it with `python -m paper_2211_14056_amd.build`')
    L = ctypes.CDLL(LIB_PATH)
    L.mf_last_error.restype = ctypes.c_char_p
    L.mf_create.argtypes = [I32, ctypes.POINTER(VP)]
    L.mf_destroy.argtypes = [VP]
    L.mf_failures.argtypes = [VP, ctypes.POINTER(U64)]
    L.mf_process_legs.argtypes = [I32]
    L.mf_process_dims.argtypes = [I32]
    L.mf_precision_available.argtypes = [I32]
    L.mf_set_launch.argtypes = [VP, I32, I32, I32, I32, I32]
    L.mf_set_launch.restype = I32
    L.mf_set_batch_tile.argtypes = [VP, I32, I32]
    L.mf_set_batch_tile.restype = I32
    L.mf_phase_space.argtypes = [VP, I32, ctypes.POINTER(mf_params), I64, VP, U64, U64, VP, VP, I32,
                                 VP, VP, VP, VP, VP, VP, VP]
    L.mf_matrix_element.argtypes = [VP, ctypes.POINTER(mf_request), I32, I32, ctypes.POINTER(mf_params), VP]
    L.mf_matrix_element_vjp.argtypes = [VP, ctypes.POINTER(mf_request), I32, I32, ctypes.POINTER(mf_params),
                                        VP, I32, VP]
    L.mf_vegas_refine.argtypes = [VP, ctypes.POINTER(mf_params), I64, I32, I32, DBL, VP, VP, VP, I32, VP, VP,
                                  VP, VP, VP, I32, VP, VP]
    L.mf_vegas_refine_noalloc.argtypes = [ctypes.POINTER(mf_params), I64, I32, I32, DBL, VP, VP, VP, I32, VP,
                                          VP, VP, VP, VP, I32, VP, VP]
    L.mf_unweight.argtypes = [VP, I64, VP, DBL, U64, U64, I32, VP, I64, VP, VP, VP, VP, VP, VP]
    L.mf_pdf_eval.argtypes = [VP, ctypes.POINTER(mf_pdf_grid), I64, VP, VP, VP, VP]
    L.mf_phase_space_pp.argtypes = [VP, I32, ctypes.POINTER(mf_params), DBL, ctypes.POINTER(mf_pdf_grid),
                                    ctypes.POINTER(mf_pdf_grid), I64, VP, U64, U64, VP, VP, I32, VP, VP, VP, VP,
                                    VP, VP, VP, VP]
    L.mf_graph_begin.argtypes = [VP, VP]
    L.mf_graph_end.argtypes = [VP, VP, ctypes.POINTER(VP)]
    L.mf_graph_launch.argtypes = [VP, VP]
    L.mf_graph_destroy.argtypes = [VP]
    for f in ('mf_create', 'mf_destroy', 'mf_failures', 'mf_phase_space', 'mf_matrix_element',
              'mf_matrix_element_vjp', 'mf_vegas_refine', 'mf_vegas_refine_noalloc', 'mf_graph_begin',
              'mf_graph_end', 'mf_graph_launch', 'mf_graph_destroy', 'mf_unweight', 'mf_pdf_eval',
              'mf_phase_space_pp'):
        getattr(L, f).restype = I32
    _lib = L
    return L


def _check(st):
    if st != 0:
        raise MFError(st, lib().mf_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError('device tensor expected')
    if not t.is_contiguous():
        raise ValueError('contiguous tensor expected')
    return t.data_ptr()


def _need(t, numel, name, dtype=None):
    """Host-side size check so a kernel never indexes past a caller's buffer."""
    if t is None:
        return
    if t.numel() < numel:
        raise ValueError(f'{name}: {t.numel()} elements, need {numel}')
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f'{name}: dtype {t.dtype}, need {dtype}')


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def params(sqrt_s=1000.0, m_t=173.0, alpha_s=0.118, alpha=1.0 / 137.0, pt_min=20.0, eta_max=2.5,
           dr_min=0.4):
    return mf_params(sqrt_s, m_t, alpha_s, alpha, pt_min, eta_max, dr_min)


def params_from_dict(d):
    return mf_params(*(float(d[k]) for k in ('sqrt_s', 'm_t', 'alpha_s', 'alpha', 'pt_min', 'eta_max',
                                              'dr_min')))


def mf_process_legs(proc):
    return lib().mf_process_legs(proc)


def mf_process_dims(proc):
    return lib().mf_process_dims(proc)


class Handle:
    """Owns an mf_handle on one device."""

    def __init__(self, device=None):
        if device is None:
            device = torch.cuda.current_device()
        h = VP()
        _check(lib().mf_create(int(device), ctypes.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().mf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_launch(self, proc=-1, precision=0, block=0, batch_waves_per_cu=-1, batch_persistent=-1):
        """mf_set_launch: per-(process, precision) block size and persistent-batch grid."""
        _check(lib().mf_set_launch(self.h, proc, precision, block, batch_waves_per_cu, batch_persistent))

    def set_batch_tile(self, proc, waves=0):
        """mf_set_batch_tile: 64-event waves per tile of the persistent batch (0 = default)."""
        _check(lib().mf_set_batch_tile(self.h, proc, waves))

    def failures(self):
        c = ctypes.c_uint64()
        _check(lib().mf_failures(self.h, ctypes.byref(c)))
        return c.value


def mf_phase_space(h, proc, prm, n, x=None, seed=0, offset=0, offset_dev=None, edges=None, nb=50,
                   p=None, w=None, pass_=None, bin_idx=None, jac=None, x_out=None, stream=None):
    """Uniforms, Vegas map, phase space and cuts; returns a dict of output tensors
    (allocated here when not given)."""
    dev = torch.device('cuda', h.device)
    n_ext = mf_process_legs(proc)
    d = mf_process_dims(proc)
    f64 = dict(dtype=torch.float64, device=dev)
    p = p if p is not None else torch.empty(n_ext, 4, n, **f64)
    w = w if w is not None else torch.empty(n, **f64)
    _need(p, n_ext * 4 * n, 'p', torch.float64)
    _need(w, n, 'w', torch.float64)
    _need(x, d * n, 'x', torch.float64)
    _need(edges, d * (nb + 1), 'edges', torch.float64)
    _need(pass_, n, 'pass', torch.uint8)
    _need(bin_idx, d * n, 'bin_idx', torch.int16)
    _need(jac, n, 'jac', torch.float64)
    _need(x_out, d * n, 'x_out', torch.float64)
    _need(offset_dev, 1, 'offset_dev', torch.int64)
    _check(lib().mf_phase_space(h.h, proc, ctypes.byref(prm), n, _ptr(x), seed, offset, _ptr(offset_dev),
                                _ptr(edges), nb, _ptr(p), _ptr(w), _ptr(pass_), _ptr(bin_idx), _ptr(jac),
                                _ptr(x_out), _stream(stream)))
    return dict(p=p, w=w, pass_=pass_, bin_idx=bin_idx, jac=jac, x=x_out if x_out is not None else x)


def make_request(proc, p, me_out, x=None, grad_me=None, grad_x=None, grad_theta=None, n=None):
    n = (p.shape[-1] if p is not None else x.shape[-1]) if n is None else n
    n_ext, d = mf_process_legs(proc), mf_process_dims(proc)
    if n_ext < 0:
        raise ValueError(f'unknown process {proc}')
    _need(p, n_ext * 4 * n, 'p', torch.float64)
    if me_out is not None and me_out.numel() < n:
        raise ValueError('me_out too small')
    _need(x, d * n, 'x', torch.float64)
    _need(grad_me, n, 'grad_me', torch.float64)
    _need(grad_x, d * n, 'grad_x', torch.float64)
    _need(grad_theta, 2 * n, 'grad_theta', torch.float64)
    r = mf_request(proc, 0, n, _ptr(p), _ptr(me_out), _ptr(x), _ptr(grad_me), _ptr(grad_x),
                   _ptr(grad_theta))
    r.me_dtype = None if me_out is None else me_out.dtype
    return r


def _check_out_dtypes(reqs, precision):
    want = torch.float64 if precision == MF_FP64 else torch.float32
    for r in reqs:
        dt = getattr(r, 'me_dtype', 'unknown')
        if dt == 'unknown':
            raise ValueError('requests must be built with make_request')
        if dt is not None and dt != want:
            raise ValueError(f'me_out dtype {dt} does not match precision {precision} ({want})')


def mf_matrix_element(h, reqs, precision, prm, stream=None):
    _check_out_dtypes(reqs, precision)
    arr = (mf_request * len(reqs))(*reqs)
    _check(lib().mf_matrix_element(h.h, arr, len(reqs), precision, ctypes.byref(prm), _stream(stream)))


def mf_matrix_element_vjp(h, reqs, precision, prm, edges=None, nb=50, stream=None):
    _check_out_dtypes(reqs, precision)
    if edges is not None:
        d = max(mf_process_dims(r.proc) for r in reqs)
        _need(edges, d * (nb + 1), 'edges', torch.float64)
    arr = (mf_request * len(reqs))(*reqs)
    _check(lib().mf_matrix_element_vjp(h.h, arr, len(reqs), precision, ctypes.byref(prm), _ptr(edges), nb,
                                       _stream(stream)))


MF_VEGAS_REFINE, MF_VEGAS_ACCUMULATE = 1, 2


def mf_precision_available(precision):
    return bool(lib().mf_precision_available(precision))


has_precision = mf_precision_available


def mf_vegas_refine(h, prm, n, d, nb, alpha, w, jac, me, pass_, bin_idx, acc, edges, F=None,
                    update_edges=True, accumulate=False, rng_counter=None, stream=None):
    if me.dtype not in (torch.float32, torch.float64):
        raise ValueError(f'me: dtype {me.dtype}, need torch.float32 or torch.float64')
    me_f32 = 1 if me.dtype == torch.float32 else 0
    _need(w, n, 'w', torch.float64)
    _need(jac, n, 'jac', torch.float64)
    _need(me, n, 'me')
    _need(pass_, n, 'pass', torch.uint8)
    _need(bin_idx, d * n, 'bin_idx', torch.int16)
    _need(acc, 2 + d * nb, 'acc', torch.float64)
    _need(edges, d * (nb + 1), 'edges', torch.float64)
    _need(F, n, 'F', torch.float64)
    _need(rng_counter, 1, 'rng_counter', torch.int64)
    _check(lib().mf_vegas_refine(h.h, ctypes.byref(prm), n, d, nb, alpha, _ptr(w), _ptr(jac), _ptr(me), me_f32,
                                 _ptr(pass_), _ptr(bin_idx), _ptr(F), _ptr(acc), _ptr(edges),
                                 (MF_VEGAS_REFINE if update_edges else 0)
                                 | (MF_VEGAS_ACCUMULATE if accumulate else 0),
                                 _ptr(rng_counter), _stream(stream)))


def mf_vegas_refine_noalloc(prm, n, d, nb, alpha, w, jac, me, pass_, bin_idx, acc, edges, F=None,
                            update_edges=True, accumulate=False, rng_counter=None, stream=None):
    """mf_vegas_refine without a handle and without allocation (static library workspace,
    current device)."""
    if me.dtype not in (torch.float32, torch.float64):
        raise ValueError(f'me: dtype {me.dtype}, need torch.float32 or torch.float64')
    me_f32 = 1 if me.dtype == torch.float32 else 0
    _need(w, n, 'w', torch.float64)
    _need(jac, n, 'jac', torch.float64)
    _need(me, n, 'me')
    _need(pass_, n, 'pass', torch.uint8)
    _need(bin_idx, d * n, 'bin_idx', torch.int16)
    _need(acc, 2 + d * nb, 'acc', torch.float64)
    _need(edges, d * (nb + 1), 'edges', torch.float64)
    _need(F, n, 'F', torch.float64)
    _need(rng_counter, 1, 'rng_counter', torch.int64)
    _check(lib().mf_vegas_refine_noalloc(ctypes.byref(prm), n, d, nb, alpha, _ptr(w), _ptr(jac), _ptr(me), me_f32,
                                         _ptr(pass_), _ptr(bin_idx), _ptr(F), _ptr(acc), _ptr(edges),
                                         (MF_VEGAS_REFINE if update_edges else 0)
                                         | (MF_VEGAS_ACCUMULATE if accumulate else 0),
                                         _ptr(rng_counter), _stream(stream)))


class PdfGrid:
    """A tabulated density on the device: ln x nodes [nx], ln Q^2 nodes [nq], x f [nq][nx]."""

    def __init__(self, log_x, log_q2, xf, device=None):
        dev = torch.device('cuda', torch.cuda.current_device() if device is None else device)
        self.log_x = torch.as_tensor(log_x, dtype=torch.float64).to(dev).contiguous()
        self.log_q2 = torch.as_tensor(log_q2, dtype=torch.float64).to(dev).contiguous()
        self.xf = torch.as_tensor(xf, dtype=torch.float64).to(dev).contiguous()
        nx, nq = self.log_x.numel(), self.log_q2.numel()
        if self.xf.numel() != nx * nq:
            raise ValueError(f'xf: {self.xf.numel()} values, need {nq} x {nx}')
        self.c = mf_pdf_grid(nx, nq, self.log_x.data_ptr(), self.log_q2.data_ptr(), self.xf.data_ptr())


def mf_pdf_eval(h, grid, x, q2, out=None, stream=None):
    """x f(x, Q^2) for the points x [n], q2 [n]."""
    n = x.numel()
    out = out if out is not None else torch.empty(n, dtype=torch.float64, device=x.device)
    _need(q2, n, 'q2', torch.float64)
    _need(out, n, 'out', torch.float64)
    if x.dtype != torch.float64:
        raise ValueError('x: need torch.float64')
    _check(lib().mf_pdf_eval(h.h, ctypes.byref(grid.c), n, _ptr(x), _ptr(q2), _ptr(out), _stream(stream)))
    return out


def mf_phase_space_pp(h, proc, prm, sqrt_S, grid, n, x=None, seed=0, offset=0, offset_dev=None, edges=None,
                      nb=50, p=None, w=None, pass_=None, bin_idx=None, jac=None, x_out=None, x12=None,
                      stream=None, grid_b=None):
    """Events of one parton channel of pp collisions (d + 2 uniforms per event): parton 1 with
    density `grid`, parton 2 with `grid_b` (None: `grid`); returns a dict of outputs."""
    dev = torch.device('cuda', h.device)
    n_ext = mf_process_legs(proc)
    d = mf_process_dims(proc) + 2
    f64 = dict(dtype=torch.float64, device=dev)
    p = p if p is not None else torch.empty(n_ext, 4, n, **f64)
    w = w if w is not None else torch.empty(n, **f64)
    _need(p, n_ext * 4 * n, 'p', torch.float64)
    _need(w, n, 'w', torch.float64)
    _need(x, d * n, 'x', torch.float64)
    _need(edges, d * (nb + 1), 'edges', torch.float64)
    _need(pass_, n, 'pass', torch.uint8)
    _need(bin_idx, d * n, 'bin_idx', torch.int16)
    _need(jac, n, 'jac', torch.float64)
    _need(x_out, d * n, 'x_out', torch.float64)
    _need(x12, 2 * n, 'x12', torch.float64)
    _need(offset_dev, 1, 'offset_dev', torch.int64)
    gb = ctypes.byref(grid_b.c) if grid_b is not None else None
    _check(lib().mf_phase_space_pp(h.h, proc, ctypes.byref(prm), float(sqrt_S), ctypes.byref(grid.c), gb, n, _ptr(x),
                                   seed, offset, _ptr(offset_dev), _ptr(edges), nb, _ptr(p), _ptr(w), _ptr(pass_),
                                   _ptr(bin_idx), _ptr(jac), _ptr(x_out), _ptr(x12), _stream(stream)))
    return dict(p=p, w=w, pass_=pass_, bin_idx=bin_idx, jac=jac, x=x_out if x_out is not None else x, x12=x12)


def mf_unweight(h, n, w, w_max=0.0, seed=0, offset=0, p=None, cap=None, idx=None, fac=None, p_out=None,
                count=None, w_max_out=None, stream=None):
    """Hit-or-miss unweighting of n weighted events; returns a dict with the output tensors
    (allocated here when not given; cap defaults to n).  The number kept is count[0]."""
    dev = torch.device('cuda', h.device)
    cap = n if cap is None else cap
    n_ext = 0 if p is None else p.shape[0]
    idx = idx if idx is not None else torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
    fac = fac if fac is not None else torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
    count = count if count is not None else torch.empty(1, dtype=torch.int64, device=dev)
    w_max_out = w_max_out if w_max_out is not None else torch.empty(1, dtype=torch.float64, device=dev)
    if p is not None and p_out is None:
        p_out = torch.empty(n_ext, 4, max(cap, 1), dtype=torch.float64, device=dev)
    _need(w, n, 'w', torch.float64)
    _need(p, n_ext * 4 * n, 'p', torch.float64)
    _need(idx, cap, 'idx', torch.int64)
    _need(fac, cap, 'fac', torch.float64)
    _need(p_out, n_ext * 4 * cap, 'p_out', torch.float64)
    _need(count, 1, 'count', torch.int64)
    _need(w_max_out, 1, 'w_max_out', torch.float64)
    if p_out is not None and cap > 0 and p_out.dim() == 3 and p_out.shape[2] != cap:
        raise ValueError(f'p_out: last dimension {p_out.shape[2]}, need the capacity {cap}')
    _check(lib().mf_unweight(h.h, n, _ptr(w), float(w_max), seed, offset, n_ext, _ptr(p), cap, _ptr(idx),
                             _ptr(fac), _ptr(p_out), _ptr(count), _ptr(w_max_out), _stream(stream)))
    return dict(idx=idx, fac=fac, p_out=p_out, count=count, w_max=w_max_out)


class Graph:
    """An executable graph of captured library calls (mf_graph_end), replayed by launch()."""

    def __init__(self, ptr, device):
        self.g = ptr
        self.device = device

    def launch(self, stream=None):
        _check(lib().mf_graph_launch(self.g, _stream(stream)))

    def close(self):
        if self.g:
            lib().mf_graph_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mf_graph_begin(h, stream=None):
    """Start capturing the library calls enqueued on `stream` (torch's current stream by
    default; not the default stream)."""
    _check(lib().mf_graph_begin(h.h, _stream(stream)))


def mf_graph_end(h, stream=None):
    """End the capture on `stream`; returns the executable Graph."""
    g = VP()
    _check(lib().mf_graph_end(h.h, _stream(stream), ctypes.byref(g)))
    return Graph(g, h.device)


def matrix_element(h, proc, p, precision=MF_FP64, prm=None, stream=None):
    """Convenience: |M|^2 for momenta p [n_ext][4][n] -> tensor [n]."""
    prm = prm or params()
    n = p.shape[-1]
    dt = torch.float64 if precision == MF_FP64 else torch.float32
    out = torch.empty(n, dtype=dt, device=p.device)
    mf_matrix_element(h, [make_request(proc, p, out)], precision, prm, stream)
    return out
