"""The no-alloc TSMTTSM entry point (tsg_tsmttsm_noalloc) against the
allocating one (tsg_tsmttsm), through the C ABI: same kernels and grid, so
the same bits; integer inputs must also equal the oracle bit for bit and
uniform inputs meet the 1e-12 bounds.  Two calls in a row on one stream, the
second with a smaller input, so the second reuses the scratch the first left
behind."""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_03136_amd import _lib, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def call(fn, cplx, A, B):
    K, M = A.shape
    N = B.shape[1]
    C = torch.full((M, N), float("nan"), dtype=A.dtype, device=DEV)
    st = fn(_lib.TSG_C128 if cplx else _lib.TSG_R64, _lib.TSG_OP_T, K, M, N, A.data_ptr(), M,
            B.data_ptr(), N, C.data_ptr(), N, torch.cuda.current_stream().cuda_stream)
    assert st == _lib.TSG_OK, _lib.tsg_last_error()
    return C.cpu().numpy()


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("shapes", [((300007, 64, 64), (50021, 8, 8)),
                                    ((200003, 32, 8), (4099, 3, 5)),
                                    ((1 << 20, 16, 16), (1 << 20, 1, 1))])
def test_noalloc_matches_allocating_entry_point(cplx, shapes):
    assert _lib.tsg_init(0) == _lib.TSG_OK
    for i, (K, M, N) in enumerate(shapes):
        print("no-alloc case: %s K=%d M=%d N=%d call %d" % ("Z" if cplx else "D", K, M, N, i), flush=True)
        for kind in ("integer", "uniform"):
            if kind == "integer":
                A = inputs.host_integers(K, M, 70 + i, inputs.STREAM_A, cplx)
                B = inputs.host_integers(K, N, 70 + i, inputs.STREAM_B, cplx)
            else:
                A = inputs.host_uniform(K, M, 70 + i, inputs.STREAM_A, cplx)
                B = inputs.host_uniform(K, N, 70 + i, inputs.STREAM_B, cplx)
            dA, dB = dev(A), dev(B)
            got = call(_lib.tsg_tsmttsm_noalloc, cplx, dA, dB)
            want = call(_lib.tsg_tsmttsm, cplx, dA, dB)
            assert np.array_equal(got, want), "no-alloc and allocating results differ"
            if kind == "integer":
                assert np.array_equal(got, oracle.tsmttsm(A, B))
            else:
                ref = oracle.tsmttsm(A, B, compensated=True)
                bound = np.abs(A).T @ np.abs(B)
                assert np.all(np.abs(got - ref) <= 1e-12 * bound)
                assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_noalloc_validates_like_the_allocating_one():
    A = 1 << 12
    assert _lib.tsg_tsmttsm_noalloc(0, 0, -1, 4, 4, A, 4, A, 4, A, 4, None) == _lib.TSG_E_ARG
    assert _lib.tsg_tsmttsm_noalloc(0, 0, 10, 4, 65, A, 4, A, 65, A, 65, None) == _lib.TSG_E_UNSUPPORTED
