"""GPU checks of the production forms: TSMM with a transposed small operand,
and the differentiable TSMTTSM (gradcheck by central differences, and the
full-size backward against the oracle on sampled rows)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_03136_amd import api, autograd, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("M,N", [(4, 4), (8, 32), (32, 8), (64, 64), (3, 5), (16, 16), (1, 1)])
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("opC", ["T", "C"])
def test_tsmm_transposed_small_operand(M, N, cplx, opC):
    K = 20011
    A = inputs.host_integers(K, M, 41, inputs.STREAM_A, cplx)
    Cs = inputs.host_integers(N, M, 41, inputs.STREAM_C, cplx)      # stored N x M
    Ce = Cs.T if opC == "T" else Cs.conj().T
    got = api.tsmm(dev(A), dev(Cs), opC=opC).cpu().numpy()
    assert np.array_equal(got, oracle.tsmm(A, np.ascontiguousarray(Ce)))
    # padded ldc and the update form
    Cp = np.zeros((N, M + 3), dtype=Cs.dtype)
    Cp[:, :M] = Cs
    B0 = inputs.host_integers(K, N, 42, inputs.STREAM_B, cplx)
    dB = dev(B0)
    api.tsmm(dev(A), dev(Cp)[:, :M], out=dB, alpha=-1.0, beta=1.0, opC=opC)
    assert np.array_equal(dB.cpu().numpy(), oracle.tsmm(A, np.ascontiguousarray(Ce), B0.copy(), -1.0, 1.0))


@pytest.mark.parametrize("cplx,op", [(False, "T"), (True, "T"), (True, "C")])
def test_gradcheck_central_differences(cplx, op):
    K, M, N = 256, 4, 4
    dt = torch.complex128 if cplx else torch.float64
    A = dev(inputs.host_uniform(K, M, 43, inputs.STREAM_A, cplx)).requires_grad_(True)
    B = dev(inputs.host_uniform(K, N, 43, inputs.STREAM_B, cplx)).requires_grad_(True)
    assert A.dtype == dt
    assert torch.autograd.gradcheck(lambda a, b: autograd.TSMTTSM.apply(a, b, op), (A, B), eps=1e-6,
                                    atol=1e-7, rtol=1e-6)


@pytest.mark.parametrize("cplx,op", [(False, "T"), (True, "T"), (True, "C")])
def test_backward_full_size_sampled(cplx, op):
    K, M, N = 1 << 22, 32, 32
    A = inputs.device_uniform(K, M, 44, inputs.STREAM_A, cplx, DEV).requires_grad_(True)
    B = inputs.device_uniform(K, N, 44, inputs.STREAM_B, cplx, DEV).requires_grad_(True)
    dC = inputs.host_uniform(M, N, 44, inputs.STREAM_DC, cplx)
    C = autograd.tsmttsm(A, B, op)
    C.backward(dev(dC))
    rows = np.unique(np.concatenate([np.random.default_rng(6).integers(0, K, 48), [0, K - 1]]))
    ridx = torch.from_numpy(rows).to(DEV)
    Ar, Br = A.detach()[ridx].cpu().numpy(), B.detach()[ridx].cpu().numpy()
    gA, gB = A.grad[ridx].cpu().numpy(), B.grad[ridx].cpu().numpy()
    if not cplx:
        rA, rB = oracle.tsmm(Br, np.ascontiguousarray(dC.T)), oracle.tsmm(Ar, dC)
    elif op == "T":
        rA, rB = oracle.tsmm(Br, np.ascontiguousarray(dC.T), conjA=True), oracle.tsmm(Ar, dC, conjA=True)
    else:
        rA, rB = oracle.tsmm(Br, np.ascontiguousarray(dC.conj().T)), oracle.tsmm(Ar, dC)
    bA = np.abs(Br) @ np.abs(dC.T)
    bB = np.abs(Ar) @ np.abs(dC)
    assert np.all(np.abs(gA - rA) <= 1e-12 * bA)
    assert np.all(np.abs(gB - rB) <= 1e-12 * bB)
    # forward against the oracle too (two sampled entries, each a length-K sum)
    for (m, n) in ((0, 0), (M - 1, 5)):
        a = A.detach()[:, m:m + 1].contiguous().cpu().numpy()
        b = B.detach()[:, n:n + 1].contiguous().cpu().numpy()
        ref = oracle.tsmttsm_entries(a, b, [(0, 0)], op=op)[0]
        assert abs(C.detach()[m, n].item() - ref) <= 1e-12 * float(np.sum(np.abs(a) * np.abs(b)))


# ------------------------------------------------------------ precision form
def _f32(x):
    return x.astype(np.complex64 if np.iscomplexobj(x) else np.float32)


def _widen(x):
    return x.astype(np.complex128 if np.iscomplexobj(x) else np.float64)


@pytest.mark.parametrize("M,N", [(8, 8), (32, 32), (64, 64), (5, 7), (17, 33), (1, 1), (32, 8)])
@pytest.mark.parametrize("cplx", [False, True])
def test_precision_form_integers_exact(M, N, cplx):
    K = 30011
    A = inputs.host_integers(K, M, 50, inputs.STREAM_A, cplx)
    B = inputs.host_integers(K, N, 50, inputs.STREAM_B, cplx)
    X = inputs.host_integers(M, N, 50, inputs.STREAM_C, cplx)
    dA, dB = dev(_f32(A)), dev(_f32(B))
    C = api.tsmttsm(dA, dB).cpu().numpy()
    assert C.dtype == (np.complex128 if cplx else np.float64)
    assert np.array_equal(C, oracle.tsmttsm(A, B))
    P = api.tsmm(dA, dev(X)).cpu().numpy()          # |entries| <= 64*64*... < 2^24: exact in binary32
    assert np.array_equal(_widen(P), oracle.tsmm(A, X))


@pytest.mark.parametrize("K", [1, 3, 17, 65, 257, 1027])
@pytest.mark.parametrize("M,N", [(8, 8), (16, 16), (64, 64)])
def test_precision_form_small_K(K, M, N):
    """Small and ragged row counts of the binary32-storage TSMM, whose kernels
    read A as one contiguous run per wave (clamped at the end of A)."""
    A = inputs.host_integers(K, M, 53, inputs.STREAM_A)
    X = inputs.host_integers(M, N, 53, inputs.STREAM_C)
    P = api.tsmm(dev(_f32(A)), dev(X)).cpu().numpy()
    assert np.array_equal(_widen(P), oracle.tsmm(A, X))


@pytest.mark.parametrize("M,N", [(8, 8), (32, 32), (64, 64), (13, 7)])
@pytest.mark.parametrize("cplx", [False, True])
def test_precision_form_uniform(M, N, cplx):
    """Arithmetic error: against the FP64 oracle on the binary32 values widened
    exactly; TSMTTSM must meet the FP64 bound (products exact, FP64 sums),
    TSMM must be within one binary32 rounding of the exact result."""
    K = 100003
    A32 = _f32(inputs.host_uniform(K, M, 51, inputs.STREAM_A, cplx))
    B32 = _f32(inputs.host_uniform(K, N, 51, inputs.STREAM_B, cplx))
    X = inputs.host_uniform(M, N, 51, inputs.STREAM_C, cplx)
    A, B = _widen(A32), _widen(B32)
    for op in (("T", "C") if cplx else ("T",)):
        C = api.tsmttsm(dev(A32), dev(B32), op=op).cpu().numpy()
        ref = oracle.tsmttsm(A, B, op=op, compensated=True)
        assert np.all(np.abs(C - ref) <= 1e-12 * (np.abs(A).T @ np.abs(B)))
    P = _widen(api.tsmm(dev(A32), dev(X)).cpu().numpy())
    ref = oracle.tsmm(A, X, compensated=True)
    # round-to-nearest binary32: |fl32(x) - x| <= 2^-24 |x| per real part
    tol = 2.0 ** -24 * (np.abs(ref.real) + (np.abs(ref.imag) if cplx else 0)) + 1e-12 * (np.abs(A) @ np.abs(X))
    assert np.all(np.abs(P - ref) <= tol * (np.sqrt(2) if cplx else 1))


@pytest.mark.parametrize("cplx", [False, True])
def test_precision_form_ill_conditioned_stated(cplx):
    """Near-parallel columns (j-th = base + 1e-4 noise_j): the Gram matrix
    A^T A cancels strongly.  The arithmetic error (vs the oracle on the stored
    binary32 values) stays at the FP64 level; the end-to-end error (vs the
    oracle on the original binary64 data) is the binary32 storage rounding
    amplified by the cancellation -- stated, not bounded by a target."""
    K, M = 1 << 18, 32
    A64 = inputs.near_parallel(K, M, 52, cplx)
    A32 = _f32(A64)
    C = api.tsmttsm(dev(A32), dev(A32), op="C" if cplx else "T").cpu().numpy()
    ref_arith = oracle.tsmttsm(_widen(A32), _widen(A32), op="C" if cplx else "T", compensated=True)
    ref_e2e = oracle.tsmttsm(A64, A64, op="C" if cplx else "T", compensated=True)
    arith = np.linalg.norm(C - ref_arith) / np.linalg.norm(ref_arith)
    e2e = np.linalg.norm(C - ref_e2e) / np.linalg.norm(ref_e2e)
    # the off-diagonal cancellation: error of C - mean(C) (the part that carries the noise)
    D = ref_e2e - ref_e2e.mean()
    e2e_dev = np.linalg.norm((C - C.mean()) - D) / np.linalg.norm(D)
    print("precision form, near-parallel Gram %s: arithmetic %.2e, end-to-end %.2e, on the deviation %.2e"
          % ("Z" if cplx else "D", arith, e2e, e2e_dev))
    assert arith <= 1e-12
    assert np.isfinite(e2e) and e2e < 1e-5
