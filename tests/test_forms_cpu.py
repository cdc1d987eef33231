"""CPU checks of the production forms' host-side definitions.

The autograd backward formulas (complex: conjugate Wirtinger convention) are
checked here with the oracle's TSMM against torch's own CPU autograd of the
plain product, so the GPU form is compared to a convention fixed outside it.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_03136_amd import inputs


@pytest.mark.parametrize("cplx,op", [(False, "T"), (True, "T"), (True, "C")])
def test_backward_formulas_match_torch_convention(cplx, op):
    K, M, N = 300, 5, 7
    A = inputs.host_uniform(K, M, 40, inputs.STREAM_A, cplx)
    B = inputs.host_uniform(K, N, 40, inputs.STREAM_B, cplx)
    dC = inputs.host_uniform(M, N, 40, inputs.STREAM_DC, cplx)
    tA = torch.from_numpy(A.copy()).requires_grad_(True)
    tB = torch.from_numpy(B.copy()).requires_grad_(True)
    At = tA.conj().t() if op == "C" else tA.t()
    C = At @ tB
    gA, gB = torch.autograd.grad(C, (tA, tB), grad_outputs=torch.from_numpy(dC))
    # the formulas the GPU backward implements, evaluated with the oracle's TSMM
    if not cplx:
        dA = oracle.tsmm(B, np.ascontiguousarray(dC.T))
        dB = oracle.tsmm(A, dC)
    elif op == "T":
        dA = oracle.tsmm(B, np.ascontiguousarray(dC.T), conjA=True)
        dB = oracle.tsmm(A, dC, conjA=True)
    else:
        dA = oracle.tsmm(B, np.ascontiguousarray(dC.conj().T))
        dB = oracle.tsmm(A, dC)
    assert np.allclose(dA, gA.resolve_conj().numpy(), rtol=1e-13, atol=1e-13)
    assert np.allclose(dB, gB.resolve_conj().numpy(), rtol=1e-13, atol=1e-13)
