"""GPU parity of the precision form: A and B stored in binary32 (real) or
complex64, C in binary64 / complex128, for the four storage/arithmetic types

  r32, c64     binary64 arithmetic on the exactly widened values;
  r32a, c64a   binary32 products summed in binary32 over stretches of 32 rows
               (TSMM: over the M terms of one output), binary64 beyond.

Every pre-generated width of the precision form (and two widths served by
run-time-width variants), both products:
  * integer-valued inputs: every product and partial sum is exact in binary32
    stretches and in binary64, so each type must equal the oracle bit for bit,
    on the full grid and on three blocks (every block then works through many
    tiles: register rings, reuse of staged operands, the binary32 flushes);
  * uniform inputs: against the compensated oracle on the widened binary32
    values, entry by entry, within the bound each type states.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_03136_amd import _lib, api, codegen, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
U32 = 2.0 ** -24
WIDTHS = codegen.PRECISION + [(5, 7), (17, 33)]
TYPES = [("r32", False, "f64"), ("c64", True, "f64"), ("r32a", False, "f32"), ("c64a", True, "f32")]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def f32(x):
    return x.astype(np.complex64 if np.iscomplexobj(x) else np.float32)


def widen(x):
    return x.astype(np.complex128 if np.iscomplexobj(x) else np.float64)


def run(op, A32, B, acc):
    if op == "tsmttsm":
        return api.tsmttsm(dev(A32), dev(B), acc=acc).cpu().numpy()
    return widen(api.tsmm(dev(A32), dev(B), acc=acc).cpu().numpy())


@pytest.mark.parametrize("M,N", WIDTHS)
@pytest.mark.parametrize("name,cplx,acc", TYPES)
@pytest.mark.parametrize("op", ["tsmttsm", "tsmm"])
def test_precision_integers_exact(op, name, cplx, acc, M, N):
    K = 30011
    A = inputs.host_integers(K, M, 60, inputs.STREAM_A, cplx)
    B = inputs.host_integers(K, N, 60, inputs.STREAM_B, cplx) if op == "tsmttsm" else \
        inputs.host_integers(M, N, 60, inputs.STREAM_C, cplx)
    ref = oracle.tsmttsm(A, B) if op == "tsmttsm" else oracle.tsmm(A, B)
    kname = api.kernel_name(op, torch.complex64 if cplx else torch.float32, M, N, acc=acc)
    assert np.array_equal(run(op, f32(A), B if op == "tsmm" else f32(B), acc), ref), kname
    assert _lib.tsg_set_grid_limit(3) == 0
    try:
        assert np.array_equal(run(op, f32(A), B if op == "tsmm" else f32(B), acc), ref), kname + " (3 blocks)"
    finally:
        _lib.tsg_set_grid_limit(0)


@pytest.mark.parametrize("M,N", WIDTHS)
@pytest.mark.parametrize("name,cplx,acc", TYPES)
@pytest.mark.parametrize("op", ["tsmttsm", "tsmm"])
def test_precision_uniform_within_stated_bound(op, name, cplx, acc, M, N):
    K = 100003
    A32 = f32(inputs.host_uniform(K, M, 61, inputs.STREAM_A, cplx))
    A = widen(A32)
    if op == "tsmttsm":
        B32 = f32(inputs.host_uniform(K, N, 61, inputs.STREAM_B, cplx))
        B = widen(B32)
        got = api.tsmttsm(dev(A32), dev(B32), acc=acc).cpu().numpy()
        ref = oracle.tsmttsm(A, B, compensated=True)
        absb = np.abs(A).T @ np.abs(B)
        # binary32 stretches of 32 rows (complex: 64 real products per part,
        # or the three-product form: 34 and 106 per part, sqrt(34^2 + 106^2)
        # < 112 on the modulus)
        tol = ((112 if cplx else 34) * U32 if acc == "f32" else 0.0) + 1e-12
        assert np.all(np.abs(got - ref) <= tol * absb), "max excess %g" % np.max(np.abs(got - ref) - tol * absb)
    else:
        X = inputs.host_uniform(M, N, 61, inputs.STREAM_C, cplx)
        got = widen(api.tsmm(dev(A32), dev(X), acc=acc).cpu().numpy())
        ref = oracle.tsmm(A, X, compensated=True)
        absb = np.abs(A) @ np.abs(X)
        # final rounding to binary32 per real part, plus (binary32 arithmetic)
        # C rounded to binary32 and M (complex 2M) products summed in binary32;
        # complex in the three-product form M + 3 and 3M + 13 per part, whose
        # modulus stays below 4M + 16
        terms = (4 * M + 16 if cplx else M + 3) if acc == "f32" else 0
        tol = np.sqrt(2) * U32 * np.abs(ref) + (terms * U32 + 1e-12) * absb
        assert np.all(np.abs(got - ref) <= tol), "max excess %g" % np.max(np.abs(got - ref) - tol)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print("precision %s %s %dx%d: normwise error vs the FP64 oracle on the stored values %.2e" %
          (op, name, M, N, err))
