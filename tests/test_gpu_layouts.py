"""Layout gating of the kernels that need contiguous rows and 16-byte
alignment (the dot product for 1 x 1, the LDS-staged kernels in binary64 and
binary32 arithmetic, slab reads): with the layout they need the library
picks them, and with a leading dimension above the width or an 8-byte offset
it falls back to a kernel without the need.  Integer inputs make every
product and sum exact, so each result must equal the oracle bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_03136_amd import api, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
K = 4099

CASES = [  # (storage dtype, acc, M, N, kind of the layout-restricted kernel)
    ("r64", "f64", 1, 1, "dot"),
    ("c128", "f64", 64, 64, "lds"),
    ("r64", "f64", 56, 56, "lds"),
    ("c64", "f32", 64, 64, "lds"),
]
TORCH = {"r64": torch.float64, "c128": torch.complex128, "r32": torch.float32, "c64": torch.complex64}
NUMPY = {"r64": np.float64, "c128": np.complex128, "r32": np.float32, "c64": np.complex64}


def placed(x, dt, layout):
    """x (K x W) on the device as contiguous, strided (ld = W + 1) or offset by one element
    (8 bytes for binary64 and complex64: off the 16-byte alignment)."""
    x = x.astype(NUMPY[dt])
    k, w = x.shape
    if layout == "contiguous":
        return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    if layout == "strided":
        buf = torch.zeros((k, w + 1), dtype=TORCH[dt], device=DEV)
        buf[:, :w] = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
        return buf[:, :w]
    flat = torch.zeros(k * w + 1, dtype=TORCH[dt], device=DEV)
    flat[1:] = torch.from_numpy(np.ascontiguousarray(x).reshape(-1)).to(DEV)
    return flat[1:].view(k, w)


@pytest.mark.parametrize("dt,acc,M,N,kind", CASES)
@pytest.mark.parametrize("layout", ["contiguous", "strided", "offset"])
def test_layout_restricted_kernels_and_fallbacks(dt, acc, M, N, kind, layout):
    cplx = dt in ("c128", "c64")
    A = inputs.host_integers(K, M, 81, inputs.STREAM_A, cplx)
    B = inputs.host_integers(K, N, 81, inputs.STREAM_B, cplx)
    ref = oracle.tsmttsm(A, B)
    dA, dB = placed(A, dt, layout), placed(B, dt, layout)
    if layout == "strided":
        assert dA.stride(0) == M + 1
    if layout == "offset" and dA.element_size() < 16:
        # (complex128 elements are 16 bytes: an offset of one keeps the
        # alignment, and the restricted kernel runs at a non-zero offset)
        assert dA.data_ptr() % 16 != 0
    print("layout %s %s %dx%d %s" % (layout, dt, M, N, acc), flush=True)
    got = api.tsmttsm(dA, dB, acc=acc).cpu().numpy()
    assert np.array_equal(got.astype(ref.dtype), ref)
    if layout == "contiguous":
        name = api.kernel_name("tsmttsm", TORCH[dt], M, N, acc=acc)
        assert "_%s_" % kind in name, name
