"""GPU parity: the HIP kernels against the CPU oracle, element by element.

Tolerances (floating point): the kernels sum in a different order than the
oracle, so results agree only up to rounding.  Each entry must satisfy
    |C_gpu - C_ref| <= 1e-12 * (|A|^T |B|)_mn          (cancellation-free bound)
and the whole result the normwise bound
    ||C_gpu - C_ref||_F <= 1e-12 * ||C_ref||_F,
with C_ref from the compensated (Dot2) oracle, whose own error is far below
both.  A dropped, doubled or misplaced term changes an entry by about
|a_km b_kn| >> 1e-12 * sum_k |a_km b_kn|, so both bounds catch it.
Integer-valued inputs are exact in binary64 and must match bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_03136_amd import _lib, api, codegen, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-12


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def abs_bound_tsmttsm(A, B, op):
    Aa = np.abs(A)
    return Aa.T @ np.abs(B)


def check_close(got, ref, bound, tol=TOL):
    err = np.abs(got - ref)
    assert np.all(err <= tol * bound + 1e-300), "max elementwise excess %g" % np.max(err - tol * bound)
    nr = np.linalg.norm(ref)
    assert np.linalg.norm(got - ref) <= tol * max(nr, 1e-300)


WIDTHS = [(1, 1), (2, 2), (4, 4), (8, 8), (16, 16), (32, 32), (64, 64), (32, 8), (8, 32),
          (3, 5), (13, 7), (17, 33), (64, 1), (1, 64), (20, 20), (48, 48), (63, 63), (5, 64)]


@pytest.mark.parametrize("M,N", WIDTHS)
@pytest.mark.parametrize("cplx", [False, True])
def test_tsmttsm_parity(M, N, cplx):
    K = 100003                                      # several tiles and a ragged tail
    A = inputs.host_uniform(K, M, 20, inputs.STREAM_A, cplx)
    B = inputs.host_uniform(K, N, 20, inputs.STREAM_B, cplx)
    dA, dB = dev(A), dev(B)
    for op in (("T", "C") if cplx else ("T",)):
        C = host(api.tsmttsm(dA, dB, op=op))
        ref = oracle.tsmttsm(A, B, op=op, compensated=True)
        check_close(C, ref, abs_bound_tsmttsm(A, B, op))


@pytest.mark.parametrize("M,N", WIDTHS)
@pytest.mark.parametrize("cplx", [False, True])
def test_tsmm_parity(M, N, cplx):
    K = 100003
    A = inputs.host_uniform(K, M, 21, inputs.STREAM_A, cplx)
    X = inputs.host_uniform(M, N, 21, inputs.STREAM_C, cplx)
    B0 = inputs.host_uniform(K, N, 21, inputs.STREAM_B, cplx)
    dA, dX = dev(A), dev(X)
    bound = np.abs(A) @ np.abs(X)
    for conj in ((False, True) if cplx else (False,)):
        got = host(api.tsmm(dA, dX, conjA=conj))
        ref = oracle.tsmm(A, X, conjA=conj, compensated=True)
        check_close(got, ref, bound)
        # update form B <- B - A C (alpha = -1, beta = 1)
        dB = dev(B0)
        api.tsmm(dA, dX, out=dB, alpha=-1.0, beta=1.0, conjA=conj)
        ref2 = oracle.tsmm(A, X, B0.copy(), alpha=-1.0, beta=1.0, conjA=conj, compensated=True)
        check_close(host(dB), ref2, bound + np.abs(B0))


@pytest.mark.parametrize("M,N", [(1, 1), (4, 4), (8, 8), (16, 16), (32, 32), (64, 64), (32, 8), (7, 9),
                                 (24, 40), (8, 32)])
@pytest.mark.parametrize("cplx", [False, True])
def test_integer_inputs_bit_exact(M, N, cplx):
    K = 65537
    A = inputs.host_integers(K, M, 22, inputs.STREAM_A, cplx)
    B = inputs.host_integers(K, N, 22, inputs.STREAM_B, cplx)
    X = inputs.host_integers(M, N, 22, inputs.STREAM_C, cplx)
    dA, dB, dX = dev(A), dev(B), dev(X)
    assert np.array_equal(host(api.tsmttsm(dA, dB)), oracle.tsmttsm(A, B))
    assert np.array_equal(host(api.tsmm(dA, dX)), oracle.tsmm(A, X))
    if cplx:
        assert np.array_equal(host(api.tsmttsm(dA, dB, op="C")), oracle.tsmttsm(A, B, op="C"))
        assert np.array_equal(host(api.tsmm(dA, dX, conjA=True)), oracle.tsmm(A, X, conjA=True))


@pytest.mark.parametrize("w", range(1, 65))
@pytest.mark.parametrize("cplx", [False, True])
def test_every_square_width(w, cplx):
    """Each square width runs its own (tuned or default) variant: both products
    against the compensated oracle, integer inputs bit for bit."""
    check_width(w, w, cplx)


@pytest.mark.parametrize("M,N", codegen.NARROW)
@pytest.mark.parametrize("cplx", [False, True])
def test_every_narrow_pair(M, N, cplx):
    """The narrow non-square pairs (up to 8 x 8) run exact-width variants of
    their own, checked like the square widths."""
    dt = "c128" if cplx else "r64"
    for op in ("tsmttsm", "tsmm"):
        name = api.kernel_name(op, torch.complex128 if cplx else torch.float64, M, N)
        assert name.startswith("%s_%s_%dx%d_" % (op, dt, M, N)), name
    check_width(M, N, cplx)


def check_width(M, N, cplx):
    K = 20011                                       # several tiles and a ragged tail
    print("width %dx%d %s" % (M, N, "Z" if cplx else "D"), flush=True)
    A = inputs.host_uniform(K, M, 23, inputs.STREAM_A, cplx)
    B = inputs.host_uniform(K, N, 23, inputs.STREAM_B, cplx)
    X = inputs.host_uniform(M, N, 23, inputs.STREAM_C, cplx)
    dA, dB, dX = dev(A), dev(B), dev(X)
    check_close(host(api.tsmttsm(dA, dB)), oracle.tsmttsm(A, B, compensated=True), abs_bound_tsmttsm(A, B, "T"))
    check_close(host(api.tsmm(dA, dX)), oracle.tsmm(A, X, compensated=True), np.abs(A) @ np.abs(X))
    Ai = inputs.host_integers(K, M, 24, inputs.STREAM_A, cplx)
    Bi = inputs.host_integers(K, N, 24, inputs.STREAM_B, cplx)
    Xi = inputs.host_integers(M, N, 24, inputs.STREAM_C, cplx)
    Ci, Pi = oracle.tsmttsm(Ai, Bi), oracle.tsmm(Ai, Xi)
    Ui = oracle.tsmm(Ai, Xi, Bi.copy(), alpha=-1.0, beta=1.0)    # update form B - A C

    def update():
        dB = dev(Bi)
        api.tsmm(dev(Ai), dev(Xi), out=dB, alpha=-1.0, beta=1.0)
        return host(dB)
    assert np.array_equal(host(api.tsmttsm(dev(Ai), dev(Bi))), Ci)
    assert np.array_equal(host(api.tsmm(dev(Ai), dev(Xi))), Pi)
    assert np.array_equal(update(), Ui)
    # three blocks: each block works through many tiles (the multi-tile paths
    # that full-size calls take)
    assert _lib.tsg_set_grid_limit(3) == 0
    try:
        assert np.array_equal(host(api.tsmttsm(dev(Ai), dev(Bi))), Ci)
        assert np.array_equal(host(api.tsmm(dev(Ai), dev(Xi))), Pi)
        assert np.array_equal(update(), Ui)
    finally:
        _lib.tsg_set_grid_limit(0)


# (17, 17), (18, 18), (49, 49): the TSMM reads A as one contiguous run per wave
# (slab reads), whose last run is clamped at the end of A
@pytest.mark.parametrize("K", [0, 1, 3, 4, 63, 64, 65, 255, 257, 1023, 4097])
@pytest.mark.parametrize("M,N", [(1, 1), (4, 4), (8, 8), (32, 32), (64, 64), (3, 17), (17, 17), (18, 18),
                                 (49, 49)])
def test_small_and_ragged_K(K, M, N):
    for cplx in (False, True):
        A = inputs.host_integers(K, M, 23, inputs.STREAM_A, cplx)
        B = inputs.host_integers(K, N, 23, inputs.STREAM_B, cplx)
        X = inputs.host_integers(M, N, 23, inputs.STREAM_C, cplx)
        dA, dB = dev(A), dev(B)
        C = host(api.tsmttsm(dA, dB))
        assert np.array_equal(C, oracle.tsmttsm(A, B))
        if K:
            assert np.array_equal(host(api.tsmm(dA, dev(X))), oracle.tsmm(A, X))


@pytest.mark.parametrize("M,N", [(4, 4), (8, 8), (5, 3), (32, 32), (64, 64), (2, 2), (17, 17), (18, 18)])
@pytest.mark.parametrize("cplx", [False, True])
def test_leading_dimensions_and_canaries(M, N, cplx):
    """Padded rows (lda > M, odd lda that defeats paired loads, rows that are
    not one contiguous run) give the same result; padding of outputs and
    inputs is never written."""
    K = 20011
    dt = np.complex128 if cplx else np.float64
    A = inputs.host_uniform(K, M, 24, inputs.STREAM_A, cplx)
    B = inputs.host_uniform(K, N, 24, inputs.STREAM_B, cplx)
    X = inputs.host_uniform(M, N, 24, inputs.STREAM_C, cplx)
    for pad in (1, 3):
        Ap = np.full((K, M + pad), np.nan, dt)
        Ap[:, :M] = A
        Bp = np.full((K, N + pad), np.nan, dt)
        Bp[:, :N] = B
        dAp, dBp = dev(Ap), dev(Bp)
        Cp = torch.full((M, N + 2), float("nan"), dtype=dAp.dtype, device=DEV)
        api.tsmttsm(dAp[:, :M], dBp[:, :N], out=Cp[:, :N])
        ref = oracle.tsmttsm(A, B, compensated=True)
        Ch = host(Cp)
        check_close(Ch[:, :N], ref, abs_bound_tsmttsm(A, B, "T"))
        assert np.all(np.isnan(Ch[:, N:]))
        # TSMM into a padded output whose old values are NaN (beta = 0: never read)
        Op = torch.full((K, N + pad), float("nan"), dtype=dAp.dtype, device=DEV)
        api.tsmm(dAp[:, :M], dev(X), out=Op[:, :N])
        Oh = host(Op)
        check_close(Oh[:, :N], oracle.tsmm(A, X, compensated=True), np.abs(A) @ np.abs(X))
        assert np.all(np.isnan(Oh[:, N:]))


@pytest.mark.parametrize("M,N", [(1, 1), (4, 4), (16, 16), (64, 64), (32, 8), (11, 29)])
@pytest.mark.parametrize("cplx", [False, True])
def test_bitwise_reproducible(M, N, cplx):
    K = 1 << 20
    dA = inputs.device_uniform(K, M, 25, inputs.STREAM_A, cplx, DEV)
    dB = inputs.device_uniform(K, N, 25, inputs.STREAM_B, cplx, DEV)
    c1 = api.tsmttsm(dA, dB).clone()
    c2 = api.tsmttsm(dA, dB).clone()
    assert torch.equal(c1, c2)


def test_symmetry_and_linearity_on_gpu():
    K, M = 300007, 24
    A = inputs.host_uniform(K, M, 26, inputs.STREAM_A)
    dA = dev(A)
    G = host(api.tsmttsm(dA, dA))
    assert np.array_equal(G, G.T)                       # same rows, same order: bitwise symmetric
    C1 = host(api.tsmttsm(2.0 * dA, dA))
    assert np.array_equal(C1, 2.0 * G)                 # power-of-two scaling is exact


def test_non_default_stream_and_workspace_reuse():
    s = torch.cuda.Stream(device=DEV)
    K = 50001
    A = inputs.host_uniform(K, 8, 27, inputs.STREAM_A)
    B = inputs.host_uniform(K, 8, 27, inputs.STREAM_B)
    with torch.cuda.stream(s):
        dA, dB = dev(A), dev(B)
        outs = [api.tsmttsm(dA, dB) for _ in range(3)]
        big = api.tsmttsm(dev(inputs.host_uniform(K, 64, 27, 9)), dev(inputs.host_uniform(K, 64, 27, 10)))
        outs.append(api.tsmttsm(dA, dB))
    s.synchronize()
    ref = oracle.tsmttsm(A, B, compensated=True)
    for o in outs:
        check_close(host(o), ref, abs_bound_tsmttsm(A, B, "T"))
    assert big.shape == (64, 64)


# --------------------------------------------------------------- full size
@pytest.mark.parametrize("M,N", [(1, 1), (64, 64), (32, 8), (8, 32)])
@pytest.mark.parametrize("cplx", [False, True])
def test_full_size_sampled(M, N, cplx):
    """K = 2^24 (the sweep size), checked on sampled outputs the oracle
    computes one by one: entries of C (each a length-K sum) and rows of B."""
    K = 1 << 24
    dA = inputs.device_uniform(K, M, 28, inputs.STREAM_A, cplx, DEV)
    dB = inputs.device_uniform(K, N, 28, inputs.STREAM_B, cplx, DEV)
    C = host(api.tsmttsm(dA, dB))
    rng = np.random.default_rng(5)
    pairs = sorted({(int(rng.integers(M)), int(rng.integers(N))) for _ in range(3)} | {(M - 1, N - 1)})
    cols_a = {m: host(dA[:, m:m + 1].contiguous()) for m, _ in pairs}
    cols_b = {n: host(dB[:, n:n + 1].contiguous()) for _, n in pairs}
    for m, n in pairs:
        ref = oracle.tsmttsm_entries(cols_a[m], cols_b[n], [(0, 0)])[0]
        bound = float(np.sum(np.abs(cols_a[m]) * np.abs(cols_b[n])))
        assert abs(C[m, n] - ref) <= TOL * bound
    X = inputs.host_uniform(M, N, 28, inputs.STREAM_C, cplx)
    out = api.tsmm(dA, dev(X))
    rows = np.unique(np.concatenate([rng.integers(0, K, 64), [0, K - 1]]))
    ridx = torch.from_numpy(rows).to(DEV)
    got = host(out[ridx])
    Ar = host(dA[ridx])
    ref = oracle.tsmm_rows(Ar, X)
    check_close(got, ref, np.abs(Ar) @ np.abs(X))
    del dA, dB, out
    torch.cuda.empty_cache()
