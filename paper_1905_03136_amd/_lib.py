"""ctypes binding of libtsgemm (declared in include/tsgemm.h), same names.

Argument marshalling only: every step of the computation runs in the HIP
kernels of the shared library.  Importing this module fails loudly when the
library has not been built; there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TSG_LIBRARY", os.path.join(HERE, "libtsgemm.so"))

TSG_R64, TSG_C128, TSG_R32, TSG_C64, TSG_R32_ACC32, TSG_C64_ACC32 = 0, 1, 2, 3, 4, 5
TSG_OP_T, TSG_OP_C, TSG_OP_N = 0, 1, 2
TSG_KIND_TSMTTSM, TSG_KIND_TSMM, TSG_KIND_ORTH = 0, 1, 2
TSG_PEAK_MFMA_F64, TSG_PEAK_VALU_F64, TSG_PEAK_MFMA_F32, TSG_PEAK_MIXED_F64 = 0, 1, 2, 3
TSG_OK, TSG_E_ARG, TSG_E_UNSUPPORTED, TSG_E_NOMEM, TSG_E_HIP, TSG_E_CAPTURE = range(6)
STATUS_NAMES = {0: "TSG_OK", 1: "TSG_E_ARG", 2: "TSG_E_UNSUPPORTED", 3: "TSG_E_NOMEM", 4: "TSG_E_HIP",
                5: "TSG_E_CAPTURE"}

# exported symbols and their prototypes, in the order of include/tsgemm.h
_i32, _i64, _vp, _dbl, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_double, ctypes.c_size_t
PROTOTYPES = {
    "tsg_tsmttsm": (_i32, [_i32, _i32, _i64, _i32, _i32, _vp, _i64, _vp, _i64, _vp, _i64, _vp]),
    "tsg_tsmttsm_noalloc": (_i32, [_i32, _i32, _i64, _i32, _i32, _vp, _i64, _vp, _i64, _vp, _i64, _vp]),
    "tsg_tsmm": (_i32, [_i32, _i32, _i64, _i32, _i32, _vp, _i64, _vp, _i64, _vp, _i64, _dbl, _dbl, _vp]),
    "tsg_tsmm_op": (_i32, [_i32, _i32, _i32, _i64, _i32, _i32, _vp, _i64, _vp, _i64, _vp, _i64, _dbl, _dbl, _vp]),
    "tsg_orth_batched": (_i32, [_vp, _i32, _vp, _sz, _vp]),
    "tsg_orth_batched_check": (_i32, [_vp]),
    "tsg_orth_plan_create": (_i32, [_vp, _i32, _vp, _i64, _vp]),
    "tsg_orth_plan_launch": (_i32, [_vp, _vp]),
    "tsg_orth_plan_run": (_i32, [_vp, _vp]),
    "tsg_orth_plan_check": (_i32, [_vp]),
    "tsg_orth_plan_set_spin_limit": (_i32, [_vp, ctypes.c_uint32]),
    "tsg_orth_plan_destroy": (None, [_vp]),
    "tsg_reserve": (_i32, [_i32, _i64, _i32, _i32, _vp]),
    "tsg_workspace_size": (_sz, [_i32, _i32, _i64, _i32, _i32, _i32]),
    "tsg_init": (_i32, [_i32]),
    "tsg_finalize": (None, []),
    "tsg_status_string": (ctypes.c_char_p, [_i32]),
    "tsg_last_error": (ctypes.c_char_p, []),
    "tsg_kernel_name": (ctypes.c_char_p, [_i32, _i32, _i32, _i32, _i32]),
    "tsg_stream_read": (_i32, [_vp, _sz, _vp]),
    "tsg_stream_copy": (_i32, [_vp, _vp, _sz, _vp]),
    "tsg_stream_probe": (_i32, [_vp, _sz, _vp, _sz, _i32, _i32, _i32, ctypes.POINTER(_sz), _vp]),
    "tsg_peak_probe": (_i32, [_i32, _i32, _i64, ctypes.POINTER(_dbl), _vp]),
    "tsg_latency_probe": (_i32, [_vp, _i64, _vp, _vp]),
    "tsg_force_variant": (_i32, [ctypes.c_char_p]),
    "tsg_set_grid_limit": (_i32, [_i32]),
    "tsg_set_reduction": (_i32, [_i32]),
    "tsg_variant_count": (_i32, []),
    "tsg_variant_name": (ctypes.c_char_p, [_i32]),
}


class tsg_orth_desc(ctypes.Structure):
    """Instance descriptor of the batched orthogonalisation (layout of the C struct)."""
    _fields_ = [("K", _i64), ("M", _i32), ("N", _i32), ("V", _vp), ("ldv", _i64),
                ("W", _vp), ("ldw", _i64), ("C", _vp), ("ldc", _i64)]


class TsgError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), detail))


def load(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError("libtsgemm.so is not built (%s); run __graft_entry__.build() or "
                          "python -m paper_1905_03136_amd.build" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def check(status):
    if status != TSG_OK:
        raise TsgError(status, lib().tsg_last_error().decode())
    return status


def tsg_tsmttsm(dt, op, K, M, N, A, lda, B, ldb, C, ldc, stream):
    return lib().tsg_tsmttsm(dt, op, K, M, N, A, lda, B, ldb, C, ldc, stream)


def tsg_tsmttsm_noalloc(dt, op, K, M, N, A, lda, B, ldb, C, ldc, stream):
    return lib().tsg_tsmttsm_noalloc(dt, op, K, M, N, A, lda, B, ldb, C, ldc, stream)


def tsg_tsmm(dt, conjA, K, M, N, A, lda, C, ldc, B, ldb, alpha, beta, stream):
    return lib().tsg_tsmm(dt, conjA, K, M, N, A, lda, C, ldc, B, ldb, alpha, beta, stream)


def tsg_tsmm_op(dt, conjA, opC, K, M, N, A, lda, C, ldc, B, ldb, alpha, beta, stream):
    return lib().tsg_tsmm_op(dt, conjA, opC, K, M, N, A, lda, C, ldc, B, ldb, alpha, beta, stream)


def tsg_reserve(dt, K, M, N, stream):
    return lib().tsg_reserve(dt, K, M, N, stream)


def tsg_workspace_size(op_kind, dt, K, M, N, count):
    return lib().tsg_workspace_size(op_kind, dt, K, M, N, count)


def tsg_init(device):
    return lib().tsg_init(device)


def tsg_finalize():
    lib().tsg_finalize()


def tsg_status_string(s):
    return lib().tsg_status_string(s).decode()


def tsg_last_error():
    return lib().tsg_last_error().decode()


def tsg_kernel_name(op_kind, dt, conj, M, N):
    return lib().tsg_kernel_name(op_kind, dt, conj, M, N).decode()


def tsg_force_variant(name):
    return lib().tsg_force_variant(name.encode() if name else None)


def tsg_set_grid_limit(blocks):
    return lib().tsg_set_grid_limit(blocks)


TSG_REDUCE_FOLD, TSG_REDUCE_ATOMIC, TSG_REDUCE_NONE = 0, 1, 2


def tsg_set_reduction(mode):
    return lib().tsg_set_reduction(mode)


def tsg_variant_count():
    return lib().tsg_variant_count()


def tsg_variant_name(i):
    return lib().tsg_variant_name(i).decode()


def tsg_stream_read(x, nbytes, stream):
    return lib().tsg_stream_read(x, nbytes, stream)


def tsg_stream_copy(src, dst, nbytes, stream):
    return lib().tsg_stream_copy(src, dst, nbytes, stream)


def tsg_stream_probe(x, x_bytes, y, y_bytes, blocks_per_cu, loads_in_flight, stream_stores, stream):
    """Returns (status, bytes moved)."""
    moved = _sz(0)
    st = lib().tsg_stream_probe(x, x_bytes, y, y_bytes, blocks_per_cu, loads_in_flight, stream_stores,
                                ctypes.byref(moved), stream)
    return st, moved.value


def tsg_peak_probe(kind, blocks_per_cu, iters, stream):
    """Returns (status, flops of the launch)."""
    fl = _dbl(0.0)
    st = lib().tsg_peak_probe(kind, blocks_per_cu, iters, ctypes.byref(fl), stream)
    return st, fl.value


def tsg_latency_probe(next_ptr, steps, out_ptr, stream):
    return lib().tsg_latency_probe(next_ptr, steps, out_ptr, stream)


def tsg_orth_batched(d_descs, count, workspace, ws_bytes, stream):
    return lib().tsg_orth_batched(d_descs, count, workspace, ws_bytes, stream)


def tsg_orth_batched_check(workspace):
    return lib().tsg_orth_batched_check(workspace)


def tsg_orth_plan_create(descs, rows_per_item, stream):
    """descs: sequence of tsg_orth_desc.  Returns (status, plan handle or None)."""
    arr = (tsg_orth_desc * len(descs))(*descs)
    plan = ctypes.c_void_p()
    st = lib().tsg_orth_plan_create(ctypes.byref(plan), len(descs), arr if len(descs) else None,
                                    rows_per_item, stream)
    return st, (plan.value if st == TSG_OK else None)


def tsg_orth_plan_launch(plan, stream):
    return lib().tsg_orth_plan_launch(plan, stream)


def tsg_orth_plan_run(plan, stream):
    return lib().tsg_orth_plan_run(plan, stream)


def tsg_orth_plan_check(plan):
    return lib().tsg_orth_plan_check(plan)


def tsg_orth_plan_set_spin_limit(plan, limit):
    return lib().tsg_orth_plan_set_spin_limit(plan, limit)


def tsg_orth_plan_destroy(plan):
    lib().tsg_orth_plan_destroy(plan)
