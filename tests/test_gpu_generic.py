"""GPU parity of the run-time-width variants: the kernels that serve (M, N)
pairs without an exact-width kernel of their own (non-square pairs outside
the pre-generated set).  Each one is forced through the C ABI's tuning hook
and run on pairs it serves -- its maximum widths, a single row or column of
them, and odd pairs inside -- on a ragged K, also on a three-block grid so
that every block works through many tiles.  Integer-valued inputs make every
product and sum exact (binary64 accumulation; the binary32-storage results
stay below 2^24), so each result must equal the oracle bit for bit.  The
TSMM twins that read the old B with A run with beta = 1, the others with
beta = 0 and beta = 1."""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_03136_amd import _lib, api, codegen, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
K = 4099
F32 = {"r32": np.float32, "c64": np.complex64}

GENERIC = [(codegen.variant_name(v), v["op"], v["dt"], v["maxM"], v["maxN"], bool(v["cfg"].get("RB")))
           for v in codegen.generic_variants()]


def pairs_of(a, b):
    return sorted({(a, b), (1, b), (a, 1), (max(1, a - 1), max(1, b - 3)), (a // 2 + 1, b // 2 + 1)})


def dev(x, dt):
    x = np.ascontiguousarray(x)
    if dt in F32:
        x = x.astype(F32[dt])
    return torch.from_numpy(x).to(DEV)


def widen(x):
    return x.astype(np.complex128 if np.iscomplexobj(x) else np.float64)


def spilled_pairs_fall_through(name, op, dt, a, b, rb):
    cplx = dt in ("c128", "c64")
    tdt = {"r64": torch.float64, "c128": torch.complex128, "r32": torch.float32, "c64": torch.complex64}[dt]
    for M, N in pairs_of(a, b):
        print("%s (not registered) M=%d N=%d" % (name, M, N), flush=True)
        assert api.kernel_name(op, tdt, M, N) != name
        A = inputs.host_integers(K, M, 61, inputs.STREAM_A, cplx)
        dA = dev(A, dt)
        if op == "tsmttsm":
            B = inputs.host_integers(K, N, 61, inputs.STREAM_B, cplx)
            got = widen(api.tsmttsm(dA, dev(B, dt)).cpu().numpy())
            assert np.array_equal(got, oracle.tsmttsm(A, B)), (M, N)
        else:
            X = inputs.host_integers(M, N, 61, inputs.STREAM_C, cplx)
            B0 = inputs.host_integers(K, N, 62, inputs.STREAM_B, cplx)
            beta = 1.0 if rb else 0.0
            got = widen(api.tsmm(dA, torch.from_numpy(X).to(DEV), out=dev(B0, dt), beta=beta).cpu().numpy())
            assert np.array_equal(got, oracle.tsmm(A, X, B0.copy(), alpha=1.0, beta=beta)), (M, N)


@pytest.mark.parametrize("name,op,dt,a,b,rb", GENERIC, ids=[g[0] for g in GENERIC])
def test_generic_variant_matches_oracle(name, op, dt, a, b, rb):
    names = {_lib.tsg_variant_name(i) for i in range(_lib.tsg_variant_count())}
    if name not in names:
        # a kernel that spills registers is left out of the registry: the
        # runtime falls through to the next variant covering the pair, which
        # must give the exact result
        spilled_pairs_fall_through(name, op, dt, a, b, rb)
        return
    cplx = dt in ("c128", "c64")
    bad = []
    try:
        for M, N in pairs_of(a, b):
            print("%s M=%d N=%d" % (name, M, N), flush=True)
            A = inputs.host_integers(K, M, 61, inputs.STREAM_A, cplx)
            dA = dev(A, dt)
            if op == "tsmttsm":
                B = inputs.host_integers(K, N, 61, inputs.STREAM_B, cplx)
                dB = dev(B, dt)
                ref = oracle.tsmttsm(A, B)
                cases = [(lambda: api.tsmttsm(dA, dB), ref)]
            else:
                X = inputs.host_integers(M, N, 61, inputs.STREAM_C, cplx)
                B0 = inputs.host_integers(K, N, 62, inputs.STREAM_B, cplx)
                dX = torch.from_numpy(X).to(DEV)
                cases = []
                for beta in ((1.0,) if rb else (0.0, 1.0)):
                    ref = oracle.tsmm(A, X, B0.copy(), alpha=1.0, beta=beta)

                    def call(beta=beta):
                        out = dev(B0, dt)
                        return api.tsmm(dA, dX, out=out, beta=beta)
                    cases.append((call, ref))
            for fn, ref in cases:
                for grid in (0, 3):
                    assert _lib.tsg_force_variant(name) == 0
                    assert _lib.tsg_set_grid_limit(grid) == 0
                    try:
                        got = widen(fn().cpu().numpy())
                    finally:
                        _lib.tsg_set_grid_limit(0)
                        _lib.tsg_force_variant(None)
                    if not np.array_equal(got, ref):
                        bad.append("M=%d N=%d grid=%d" % (M, N, grid))
    finally:
        _lib.tsg_force_variant(None)
    assert not bad, bad


@pytest.mark.parametrize("M,N", [(1, 8), (3, 8), (8, 3), (2, 7), (7, 2), (1, 4), (4, 1), (5, 8), (3, 16),
                                 (6, 12), (12, 6), (16, 3)])
@pytest.mark.parametrize("cplx", [False, True])
def test_narrow_pairs_use_shallow_matrix_core_variants(M, N, cplx):
    """Narrow non-square TSMM pairs go to the matrix-core variants sized for
    their contraction depth (one or two 4-wide slices up to M = 8), not the
    vector kernel, and give the oracle's result."""
    dt = torch.complex128 if cplx else torch.float64
    name = api.kernel_name("tsmm", dt, M, N)
    if not name.startswith("tsmm_%s_%dx%d_" % ("c128" if cplx else "r64", M, N)):
        assert "_mfma_" in name, name
        if M <= 4:
            assert "_le4x16_" in name, name
        elif M <= 8:
            assert "_le8x16_" in name, name
    A = inputs.host_integers(K, M, 63, inputs.STREAM_A, cplx)
    X = inputs.host_integers(M, N, 63, inputs.STREAM_C, cplx)
    got = api.tsmm(torch.from_numpy(A).to(DEV), torch.from_numpy(X).to(DEV)).cpu().numpy()
    assert np.array_equal(got, oracle.tsmm(A, X))


@pytest.mark.parametrize("M,N", [(33, 40), (21, 9), (57, 50), (13, 60)])
def test_strided_rows_use_a_variant_without_slab_reads(M, N):
    """Run-time-width TSMM classes whose fastest kernel reads A in slabs
    (contiguous rows) keep a kernel without that need for a leading dimension
    above M; both give the oracle's result bit for bit."""
    A = inputs.host_integers(K, M, 64, inputs.STREAM_A, False)
    X = inputs.host_integers(M, N, 64, inputs.STREAM_C, False)
    ref = oracle.tsmm(A, X)
    wide = np.zeros((K, M + 3))
    wide[:, :M] = A
    dW = torch.from_numpy(wide).to(DEV)
    dA = dW[:, :M]
    assert dA.stride(0) == M + 3
    flat = torch.from_numpy(A).to(DEV)
    dX = torch.from_numpy(X).to(DEV)
    print("strided M=%d N=%d" % (M, N), flush=True)
    for a in (flat, dA):
        for grid in (0, 3):
            assert _lib.tsg_set_grid_limit(grid) == 0
            try:
                got = api.tsmm(a, dX).cpu().numpy()
            finally:
                _lib.tsg_set_grid_limit(0)
            assert np.array_equal(got, ref), (a.stride(0), grid)
