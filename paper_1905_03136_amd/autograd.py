"""Differentiation form: TSMTTSM as a torch.autograd.Function whose backward
runs on the library's TSMM kernels.

Forward C = op(A)^T B.  The backward follows PyTorch's convention for complex
inputs (the gradient with respect to z is the conjugate Wirtinger derivative
of the real loss, as torch's own matmul backward uses):

  real, op T:      dA = B dC^T          dB = A dC
  complex, op T:   dA = conj(B) dC^T    dB = conj(A) dC      (C = A^T B)
  complex, op C:   dA = B dC^H          dB = A dC            (C = A^H B)

Each gradient is one TSMM of a tall operand with the small dC; the transposed
or conjugated dC is read in that form while it is staged on chip
(tsg_tsmm_op), so no copy of it is made.
"""
import torch

from . import api


class TSMTTSM(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, op="T"):
        ctx.save_for_backward(A, B)
        ctx.op = op
        return api.tsmttsm(A, B, op=op)

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        dC = dC.contiguous()
        cplx = A.is_complex()
        dA = dB = None
        if ctx.needs_input_grad[0]:
            if not cplx:
                dA = api.tsmm(B, dC, opC="T")
            elif ctx.op == "T":
                dA = api.tsmm(B, dC, conjA=True, opC="T")
            else:
                dA = api.tsmm(B, dC, opC="C")
        if ctx.needs_input_grad[1]:
            dB = api.tsmm(A, dC, conjA=(cplx and ctx.op == "T"))
        return dA, dB, None


def tsmttsm(A, B, op="T"):
    """Differentiable C = op(A)^T B (see TSMTTSM)."""
    return TSMTTSM.apply(A, B, op)
