"""The reduction ablation hook of TSMTTSM (tsg_set_reduction): the global-
atomic reduction gives the oracle's result within the usual bound (its
order of additions varies, so not bit for bit), the fold (default) is
unchanged, and "none" leaves C unwritten.  Every mode is restored to the
fold before a test ends."""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_03136_amd import _lib, api, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("M,N", [(4, 4), (32, 32), (64, 64), (13, 7)])
@pytest.mark.parametrize("cplx", [False, True])
def test_atomic_reduction_within_bound(cplx, M, N):
    K = 200003
    A = inputs.host_uniform(K, M, 81, inputs.STREAM_A, cplx)
    B = inputs.host_uniform(K, N, 81, inputs.STREAM_B, cplx)
    ref = oracle.tsmttsm(A, B, compensated=True)
    bound = np.abs(A).T @ np.abs(B)
    dA, dB = dev(A), dev(B)
    fold = api.tsmttsm(dA, dB).cpu().numpy()
    assert _lib.tsg_set_reduction(_lib.TSG_REDUCE_ATOMIC) == 0
    try:
        C = torch.full((M, N), float("nan"), dtype=dA.dtype, device=DEV)
        got = api.tsmttsm(dA, dB, out=C).cpu().numpy()
    finally:
        _lib.tsg_set_reduction(_lib.TSG_REDUCE_FOLD)
    assert np.all(np.abs(got - ref) <= 1e-12 * bound)
    assert np.all(np.abs(fold - ref) <= 1e-12 * bound)
    # the default is back: bit for bit the fold's result
    assert np.array_equal(api.tsmttsm(dA, dB).cpu().numpy(), fold)


def test_no_reduction_leaves_c_unwritten():
    K, M, N = 1 << 20, 8, 8
    A = torch.ones((K, M), dtype=torch.float64, device=DEV)
    C = torch.full((M, N), 7.0, dtype=torch.float64, device=DEV)
    assert _lib.tsg_set_reduction(_lib.TSG_REDUCE_NONE) == 0
    try:
        api.tsmttsm(A, A, out=C)
        torch.cuda.synchronize()
    finally:
        _lib.tsg_set_reduction(_lib.TSG_REDUCE_FOLD)
    assert torch.all(C == 7.0).item()
    api.tsmttsm(A, A, out=C)
    assert torch.all(C == float(K)).item()
