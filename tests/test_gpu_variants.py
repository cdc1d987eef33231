"""Every generated configuration the autotuner may choose, checked against the
oracle: each candidate of the sweep widths is forced (through the C ABI's
tuning hook of the tuning library) and run on integer-valued inputs, whose
products and sums are exact in binary64, so each must equal the oracle bit
for bit; one float case per candidate checks the 1e-12 bounds."""
import ctypes
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1905_03136_amd import _lib, codegen, inputs
from paper_1905_03136_amd.tune import TUNE_LIB

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
# the widths whose candidates the tuning library holds (the build compiles
# every candidate of these widths; the product's own variant of every other
# width is checked in test_gpu_parity and test_gpu_exact_widths)
WIDTHS = codegen.TUNE_WIDTHS


@pytest.fixture(scope="module")
def tlib():
    if not os.path.exists(TUNE_LIB):
        pytest.skip("tuning library not built (python -m paper_1905_03136_amd.tune build)")
    return _lib.load(TUNE_LIB)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def run(tlib, op, cplx, A, B):
    """op(A)^T B (op='tsmttsm') or A B (op='tsmm') through the tuning library's C ABI."""
    dt = _lib.TSG_C128 if cplx else _lib.TSG_R64
    s = torch.cuda.current_stream().cuda_stream
    K, M = A.shape
    if op == "tsmttsm":
        N = B.shape[1]
        C = torch.empty((M, N), dtype=A.dtype, device=DEV)
        st = tlib.tsg_tsmttsm(dt, 0, K, M, N, A.data_ptr(), M, B.data_ptr(), N, C.data_ptr(), N, s)
    else:
        N = B.shape[1]
        C = torch.empty((K, N), dtype=A.dtype, device=DEV)
        st = tlib.tsg_tsmm(dt, 0, K, M, N, A.data_ptr(), M, B.data_ptr(), N, C.data_ptr(), N, 1.0, 0.0, s)
    assert st == 0, tlib.tsg_last_error().decode()
    return C.cpu().numpy()


@pytest.mark.parametrize("M,N", WIDTHS)
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("op", ["tsmttsm", "tsmm"])
def test_every_candidate_matches_oracle(tlib, op, cplx, M, N):
    dt = "c128" if cplx else "r64"
    names = {tlib.tsg_variant_name(i).decode() for i in range(tlib.tsg_variant_count())}
    cands = [codegen.variant_name(dict(op=op, dt=dt, M=M, N=N, maxM=M, maxN=N, cfg=c))
             for c in codegen.candidates(op, dt, M, N)]
    missing = [c for c in cands if c not in names]
    # a candidate absent from the library is one whose kernel spills (the
    # build leaves those out of the registry); every other one must be there
    cands = [c for c in cands if c in names]
    assert cands, "no candidate of this width is in the tuning library"
    assert len(missing) < len(cands), missing
    K = 4099
    A = inputs.host_integers(K, M, 31, inputs.STREAM_A, cplx)
    B = inputs.host_integers(K, N, 31, inputs.STREAM_B, cplx) if op == "tsmttsm" else \
        inputs.host_integers(M, N, 31, inputs.STREAM_C, cplx)
    ref = oracle.tsmttsm(A, B) if op == "tsmttsm" else oracle.tsmm(A, B)
    Af = inputs.host_uniform(K, M, 32, inputs.STREAM_A, cplx)
    Bf = inputs.host_uniform(K, N, 32, inputs.STREAM_B, cplx) if op == "tsmttsm" else \
        inputs.host_uniform(M, N, 32, inputs.STREAM_C, cplx)
    reff = oracle.tsmttsm(Af, Bf, compensated=True) if op == "tsmttsm" else oracle.tsmm(Af, Bf, compensated=True)
    bound = (np.abs(Af).T @ np.abs(Bf)) if op == "tsmttsm" else (np.abs(Af) @ np.abs(Bf))
    dA, dB, dAf, dBf = dev(A), dev(B), dev(Af), dev(Bf)
    bad = []
    try:
        for name in cands:
            assert tlib.tsg_force_variant(name.encode()) == 0
            got = run(tlib, op, cplx, dA, dB)
            if not np.array_equal(got, ref):
                bad.append(name + " (integer)")
            gotf = run(tlib, op, cplx, dAf, dBf)
            if not np.all(np.abs(gotf - reff) <= 1e-12 * bound):
                bad.append(name + " (float)")
            # three blocks: every block works through many tiles of the short
            # matrix (register rings, reuse of staged data), as at full size
            assert tlib.tsg_set_grid_limit(3) == 0
            try:
                if not np.array_equal(run(tlib, op, cplx, dA, dB), ref):
                    bad.append(name + " (integer, 3 blocks)")
            finally:
                tlib.tsg_set_grid_limit(0)
    finally:
        tlib.tsg_force_variant(None)
    assert not bad, bad
