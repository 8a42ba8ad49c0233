"""torch.autograd binding of the matrix element as a function of the random inputs.

MatrixElementFn.apply(x, theta, ...) -> |M|^2 per event, where x [d][n] are the
uniforms that generate the events (through the Vegas map and the phase space)
and theta = (m_t, alpha_s).  The forward pass runs mf_phase_space +
mf_matrix_element; the backward pass runs mf_matrix_element_vjp, so gradients
with respect to x (per event) and theta (summed over events) come from the
library's derivative kernel.  Intended for flow-based importance sampling and
parameter fits.
"""
import torch

from . import (Handle, MF_FP64, PROCESS, make_request, mf_matrix_element, mf_matrix_element_vjp,
               mf_phase_space, mf_process_dims, params)


class MatrixElementFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, theta, handle, proc, precision, edges, base_params):
        pid = PROCESS[proc] if isinstance(proc, str) else proc
        d = mf_process_dims(pid)
        if x.dim() != 2 or x.shape[0] != d:
            raise ValueError(f'x must be [{d}][n]')
        x = x.detach().contiguous()
        n = x.shape[1]
        mt, als = (float(v) for v in theta.detach().cpu())
        bp = base_params or params()
        prm = params(bp.sqrt_s, mt, als, bp.alpha, bp.pt_min, bp.eta_max, bp.dr_min)
        nb = 0 if edges is None else edges.shape[1] - 1
        ev = mf_phase_space(handle, pid, prm, n, x=x, edges=edges, nb=nb if nb else 50)
        dt = torch.float64 if precision == MF_FP64 else torch.float32
        me = torch.empty(n, dtype=dt, device=x.device)
        mf_matrix_element(handle, [make_request(pid, ev['p'], me)], precision, prm)
        ctx.save_for_backward(x)
        ctx.cfg = (handle, pid, precision, edges, nb, prm, theta.dtype, theta.device)
        return me

    @staticmethod
    def backward(ctx, grad_me):
        (x,) = ctx.saved_tensors
        handle, pid, precision, edges, nb, prm, tdt, tdev = ctx.cfg
        n = x.shape[1]
        d = x.shape[0]
        gx = torch.empty(d, n, dtype=torch.float64, device=x.device)
        gth = torch.empty(n, 2, dtype=torch.float64, device=x.device)
        g = grad_me.detach().to(torch.float64).contiguous()
        req = make_request(pid, None, None, x=x, grad_me=g, grad_x=gx, grad_theta=gth, n=n)
        mf_matrix_element_vjp(handle, [req], precision, prm, edges=edges, nb=nb if nb else 50)
        return gx.to(x.dtype), gth.sum(0).to(tdt).to(tdev), None, None, None, None, None


def matrix_element_of_x(x, theta, handle=None, proc='gg_ttg', precision=MF_FP64, edges=None, base_params=None):
    """Differentiable |M|^2(x; m_t, alpha_s)."""
    handle = handle or Handle()
    return MatrixElementFn.apply(x, theta, handle, proc, precision, edges, base_params)
