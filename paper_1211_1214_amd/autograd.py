"""torch.autograd wrapper of the determinant-ratio exponents (argument marshalling only).

``exponents(ctx, kappa1, kappa2, links, eta)`` returns x_ij of Eq. (8) (two flavours) as a
float64 CPU tensor that is differentiable in ``kappa2`` (a 0-dim float64 tensor) and in
``links`` (the complex128 [4, V, 3, 3] device tensor the Context was created from).  The
backward pass calls ddwc_det_ratio_grad, which recomputes every solve of the forward pass
and runs the adjoint solves; nothing but the inputs is kept between the two passes.
``log_w_gl(x)`` is the log-domain combination of Eq. (8) computed by ddwc_log_w_combine
(value and d log W_gl / dx_ij on the host, in the library), wrapped so that the gradient
flows back through ``exponents``.

A Context holds its own copy of the links: to differentiate at other links, create a new
Context from them.
"""
from __future__ import annotations

import torch

from .binding import FP64, OP_SCHUR, log_w_combine


class _Exponents(torch.autograd.Function):
    @staticmethod
    def forward(fctx, kappa2, links, handle, kappa1, eta, op, tol, prec):
        res = handle.det_ratio_estimate(kappa1, float(kappa2), eta, op=op, tol=tol, prec=prec)
        fctx.args = (handle, kappa1, float(kappa2), eta, op, tol, prec)
        return torch.from_numpy(res["x"])

    @staticmethod
    def backward(fctx, gx):
        handle, kappa1, kappa2, eta, op, tol, prec = fctx.args
        want_k, want_u = fctx.needs_input_grad[0], fctx.needs_input_grad[1]
        if not (want_k or want_u):
            return (None,) * 8
        r = handle.det_ratio_grad(kappa1, kappa2, eta, gx.detach().cpu().numpy(), op=op, tol=tol, prec=prec,
                                  want_kappa2=want_k, want_links=want_u)
        dk = torch.tensor(r["dkappa2"], dtype=torch.float64) if want_k else None
        return dk, r["dU"], None, None, None, None, None, None


def exponents(handle, kappa1: float, kappa2: torch.Tensor, links: torch.Tensor, eta: torch.Tensor, op: int = OP_SCHUR,
              tol: float = 1e-12, prec: int = FP64) -> torch.Tensor:
    """x_ij [n_interp, n_hit], differentiable in kappa2 and links."""
    return _Exponents.apply(kappa2, links, handle, kappa1, eta, op, tol, prec)


class _LogWGl(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x):
        r = log_w_combine(x.detach().cpu().numpy(), n_f=2, grad=True)
        fctx.save_for_backward(torch.from_numpy(r["gx"]).to(x.device, x.dtype))
        return torch.tensor(r["log_w"], dtype=x.dtype, device=x.device)

    @staticmethod
    def backward(fctx, g):
        (gx,) = fctx.saved_tensors
        return g * gx


def log_w_gl(x: torch.Tensor) -> torch.Tensor:
    """sum_i [logsumexp_j(-x_ij) - ln n_hit] (Eq. 8), by ddwc_log_w_combine; differentiable in x."""
    return _LogWGl.apply(x)
