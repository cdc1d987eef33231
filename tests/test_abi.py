"""The C-ABI library loads, exports every entry point declared in
include/tsgemm.h, and validates arguments on the host before any HIP call.
No compute call is made here (no GPU in this environment)."""
import ctypes
import os
import re

import pytest

from paper_1905_03136_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsgemm.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tsg_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return _lib.lib()


def test_header_declares_expected_api():
    syms = declared_symbols()
    for s in ("tsg_tsmttsm", "tsg_tsmm", "tsg_init", "tsg_finalize", "tsg_status_string", "tsg_last_error",
              "tsg_workspace_size", "tsg_reserve", "tsg_kernel_name", "tsg_orth_batched", "tsg_orth_batched_check"):
        assert s in syms


def test_every_declared_symbol_is_exported(lib):
    for s in declared_symbols():
        assert hasattr(lib, s), s
        assert s in _lib.PROTOTYPES, "binding lacks a prototype for %s" % s


def test_status_strings(lib):
    for code, name in _lib.STATUS_NAMES.items():
        assert _lib.tsg_status_string(code).startswith(name)


A = 1 << 12   # fake, 16-byte aligned "device" addresses: validation fails before any use


@pytest.mark.parametrize("args,code", [
    ((0, 0, -1, 4, 4, A, 4, A, 4, A, 4), _lib.TSG_E_ARG),          # K < 0
    ((0, 0, 10, 0, 4, A, 4, A, 4, A, 4), _lib.TSG_E_ARG),          # M < 1
    ((0, 0, 10, 4, 65, A, 4, A, 65, A, 65), _lib.TSG_E_UNSUPPORTED),  # N > 64
    ((0, 0, 10, 4, 4, A, 3, A, 4, A, 4), _lib.TSG_E_ARG),          # lda < M
    ((0, 0, 10, 4, 4, A, 4, A, 3, A, 4), _lib.TSG_E_ARG),          # ldb < N
    ((0, 0, 10, 4, 4, A, 4, A, 4, A, 2), _lib.TSG_E_ARG),          # ldc < N
    ((0, 0, 10, 4, 4, None, 4, A, 4, A, 4), _lib.TSG_E_ARG),       # A NULL
    ((0, 0, 10, 4, 4, A, 4, A, 4, None, 4), _lib.TSG_E_ARG),       # C NULL
    ((0, 0, 10, 4, 4, A + 4, 4, A, 4, A, 4), _lib.TSG_E_ARG),      # misaligned double
    ((1, 0, 10, 4, 4, A + 8, 4, A, 4, A, 4), _lib.TSG_E_ARG),      # misaligned complex
    ((7, 0, 10, 4, 4, A, 4, A, 4, A, 4), _lib.TSG_E_ARG),          # unknown dtype
    ((0, 3, 10, 4, 4, A, 4, A, 4, A, 4), _lib.TSG_E_ARG),          # unknown op
])
def test_tsmttsm_validation(lib, args, code):
    assert _lib.tsg_tsmttsm(*args, None) == code
    assert _lib.tsg_last_error() != ""


@pytest.mark.parametrize("args,code", [
    ((0, 0, -5, 4, 4, A, 4, A, 4, A, 4), _lib.TSG_E_ARG),
    ((0, 0, 10, 65, 4, A, 65, A, 4, A, 4), _lib.TSG_E_UNSUPPORTED),
    ((0, 0, 10, 4, 4, A, 2, A, 4, A, 4), _lib.TSG_E_ARG),          # lda < M
    ((0, 0, 10, 4, 4, A, 4, A, 3, A, 4), _lib.TSG_E_ARG),          # ldc < N
    ((0, 0, 10, 4, 4, A, 4, A, 4, A, 3), _lib.TSG_E_ARG),          # ldb < N
    ((0, 0, 10, 4, 4, A, 4, None, 4, A, 4), _lib.TSG_E_ARG),       # C NULL
    ((1, 1, 10, 4, 4, A, 4, A, 4, A + 8, 4), _lib.TSG_E_ARG),      # misaligned complex B
])
def test_tsmm_validation(lib, args, code):
    assert _lib.tsg_tsmm(*args, 1.0, 0.0, None) == code


def test_tsmm_k_zero_is_a_no_op_without_device(lib):
    # K = 0 has nothing to do: valid arguments return OK without touching HIP
    assert _lib.tsg_tsmm(0, 0, 0, 4, 4, None, 4, A, 4, None, 4, 1.0, 0.0, None) == _lib.TSG_OK


def test_no_device_reports_hip_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert _lib.tsg_tsmttsm(0, 0, 100, 4, 4, A, 4, A, 4, A, 4, None) == _lib.TSG_E_HIP
    assert _lib.tsg_init(0) == _lib.TSG_E_HIP
    assert _lib.tsg_workspace_size(_lib.TSG_KIND_TSMTTSM, 0, 1 << 20, 4, 4, 1) == 0


def test_kernel_names_cover_all_widths(lib):
    for op in (0, 1):
        for dt in (_lib.TSG_R64, _lib.TSG_C128):
            for M in (1, 3, 16, 17, 33, 63, 64):
                for N in (1, 5, 16, 31, 64):
                    assert _lib.tsg_kernel_name(op, dt, 0, M, N) != ""
    assert _lib.tsg_kernel_name(0, 0, 0, 65, 1) == ""


def test_grid_limit_hook(lib):
    assert _lib.tsg_set_grid_limit(-1) == _lib.TSG_E_ARG
    assert "grid limit" in _lib.tsg_last_error()
    assert _lib.tsg_set_grid_limit(5) == _lib.TSG_OK
    assert _lib.tsg_set_grid_limit(0) == _lib.TSG_OK


def test_precision_dtypes_validated(lib):
    # binary32 storage: 4-byte (real) / 8-byte (complex) alignment of A and B, C stays binary64
    assert _lib.tsg_tsmttsm(_lib.TSG_R32, 0, 10, 4, 4, A + 4, 4, A, 4, A, 4, None) != _lib.TSG_E_ARG
    assert _lib.tsg_tsmttsm(_lib.TSG_R32, 0, 10, 4, 4, A + 2, 4, A, 4, A, 4, None) == _lib.TSG_E_ARG
    assert _lib.tsg_tsmttsm(_lib.TSG_C64, 0, 10, 4, 4, A + 4, 4, A, 4, A, 4, None) == _lib.TSG_E_ARG
    assert _lib.tsg_tsmttsm(_lib.TSG_R32, 0, 10, 4, 4, A, 4, A, 4, A + 4, 4, None) == _lib.TSG_E_ARG
    assert _lib.tsg_tsmm_op(_lib.TSG_R64, 0, 7, 10, 4, 4, A, 4, A, 4, A, 4, 1.0, 0.0, None) == _lib.TSG_E_ARG
    # a transposed small matrix is stored N x M: ldc >= M
    assert _lib.tsg_tsmm_op(_lib.TSG_R64, 0, _lib.TSG_OP_T, 10, 6, 4, A, 6, A, 5, A, 4, 1.0, 0.0, None) \
        == _lib.TSG_E_ARG


def _desc(K=100, M=8, N=4, V=A, ldv=None, W=A, ldw=None, C=A, ldc=None):
    return _lib.tsg_orth_desc(K, M, N, V, M if ldv is None else ldv, W, N if ldw is None else ldw,
                              C, N if ldc is None else ldc)


@pytest.mark.parametrize("desc,code", [
    (dict(K=-1), _lib.TSG_E_ARG),
    (dict(M=0), _lib.TSG_E_ARG),
    (dict(N=0), _lib.TSG_E_ARG),
    (dict(M=65), _lib.TSG_E_UNSUPPORTED),
    (dict(N=17), _lib.TSG_E_UNSUPPORTED),
    (dict(ldv=7), _lib.TSG_E_ARG),
    (dict(ldw=3), _lib.TSG_E_ARG),
    (dict(ldc=3), _lib.TSG_E_ARG),
    (dict(V=None), _lib.TSG_E_ARG),
    (dict(W=None), _lib.TSG_E_ARG),
    (dict(C=None), _lib.TSG_E_ARG),
    (dict(K=0, V=None, W=None, C=None), _lib.TSG_E_ARG),   # C is written even for K = 0
    (dict(V=A + 4), _lib.TSG_E_ARG),
    (dict(C=A + 2), _lib.TSG_E_ARG),
    (dict(ldv=1 << 28), _lib.TSG_E_UNSUPPORTED),            # slab offsets would pass 2^31 bytes
])
def test_orth_plan_validation(lib, desc, code):
    good = _desc()
    st, plan = _lib.tsg_orth_plan_create([good, _desc(**desc)], 0, None)
    assert st == code and plan is None
    assert "instance 1" in _lib.tsg_last_error()


def test_orth_plan_validation_misc(lib):
    assert _lib.tsg_orth_plan_create([], 0, None)[0] == _lib.TSG_E_ARG
    assert lib.tsg_orth_plan_create(None, 1, None, 0, None) == _lib.TSG_E_ARG
    # a fixed slab height beyond the offset bound of the leading dimension
    assert _lib.tsg_orth_plan_create([_desc(M=64, ldv=64)], 1 << 30, None)[0] == _lib.TSG_E_UNSUPPORTED
    for fn in (_lib.tsg_orth_plan_launch, _lib.tsg_orth_plan_run):
        assert fn(None, None) == _lib.TSG_E_ARG
    assert _lib.tsg_orth_plan_check(None) == _lib.TSG_E_ARG
    assert _lib.tsg_orth_plan_set_spin_limit(None, 0) == _lib.TSG_E_ARG
    _lib.tsg_orth_plan_destroy(None)                      # ignored


def test_orth_plan_no_device(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, plan = _lib.tsg_orth_plan_create([_desc(), _desc(K=0)], 0, None)
    assert st == _lib.TSG_E_HIP and plan is None


def test_orth_workspace_size_bounds_the_batch(lib):
    """The batched call's workspace size needs no device: it grows with the
    widths and the instance count and is 0 outside the supported range."""
    ws = lambda K, M, N, c: _lib.tsg_workspace_size(_lib.TSG_KIND_ORTH, _lib.TSG_R64, K, M, N, c)
    assert ws(1 << 22, 64, 16, 64) > 0
    assert ws(1 << 22, 64, 16, 64) > ws(1 << 22, 8, 4, 64)
    assert ws(1 << 22, 64, 16, 128) > ws(1 << 22, 64, 16, 64)
    # slabs of at most 256 per instance: the partial sums of 64 instances of 64 x 16
    assert ws(1 << 22, 64, 16, 64) >= 64 * 256 * 64 * 16 * 8
    assert ws(1 << 22, 65, 16, 64) == 0 and ws(1 << 22, 64, 17, 64) == 0
    assert ws(1 << 22, 64, 16, 0) == 0 and ws(1 << 22, 64, 16, 1025) == 0
    assert _lib.tsg_workspace_size(_lib.TSG_KIND_ORTH, _lib.TSG_C128, 1 << 20, 4, 4, 4) == 0
    assert _lib.tsg_workspace_size(_lib.TSG_KIND_TSMM, _lib.TSG_R64, 1 << 20, 4, 4, 1) == 0


def test_orth_batched_host_validation(lib):
    A = 1 << 12
    n = _lib.tsg_workspace_size(_lib.TSG_KIND_ORTH, _lib.TSG_R64, 1000, 8, 8, 2)
    assert _lib.tsg_orth_batched(None, 2, A, n, None) == _lib.TSG_E_ARG
    assert _lib.tsg_orth_batched(A, 2, None, n, None) == _lib.TSG_E_ARG
    assert _lib.tsg_orth_batched(A, 0, A, n, None) == _lib.TSG_E_ARG
    assert _lib.tsg_orth_batched(A, 1025, A, n, None) == _lib.TSG_E_UNSUPPORTED
    assert _lib.tsg_orth_batched(A + 8, 2, A + 8, n, None) == _lib.TSG_E_ARG   # workspace not 256-aligned
    assert _lib.tsg_orth_batched(A, 2, A, 64, None) == _lib.TSG_E_ARG          # below the queue's own size
    assert _lib.tsg_orth_batched_check(None) == _lib.TSG_E_ARG


def test_reduction_hook_rejects_unknown_modes(lib):
    """Host-side validation of the reduction ablation hook (no GPU needed)."""
    from paper_1905_03136_amd import _lib
    assert _lib.tsg_set_reduction(7) == _lib.TSG_E_ARG
    assert _lib.tsg_set_reduction(-1) == _lib.TSG_E_ARG
    assert _lib.tsg_set_reduction(_lib.TSG_REDUCE_FOLD) == _lib.TSG_OK
