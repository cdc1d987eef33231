"""torch-facing entry points.  torch supplies device memory and streams only;
the arithmetic runs in libtsgemm's HIP kernels (see ``_lib``)."""
import torch

from . import _lib

_DT = {torch.float64: _lib.TSG_R64, torch.complex128: _lib.TSG_C128,
       torch.float32: _lib.TSG_R32, torch.complex64: _lib.TSG_C64}
_SMALL = {torch.float64: torch.float64, torch.complex128: torch.complex128,
          torch.float32: torch.float64, torch.complex64: torch.complex128}


def _ld(X, name):
    if X.dim() != 2:
        raise ValueError("%s must be 2-D" % name)
    if X.numel() == 0:
        return max(1, X.size(1))
    if X.size(1) > 1 and X.stride(1) != 1:
        raise ValueError("%s must have unit column stride (row-major)" % name)
    if X.size(0) <= 1:
        return max(X.size(1), X.stride(0) if X.size(0) == 1 else X.size(1))
    return X.stride(0)


def _stream(dev):
    return torch.cuda.current_stream(dev).cuda_stream


def _dtype(t, acc):
    """ABI storage/arithmetic type of tensor dtype t; acc='f32' selects binary32
    arithmetic for binary32 storage (float32 / complex64)."""
    if acc not in ("f64", "f32"):
        raise ValueError("acc must be 'f64' or 'f32'")
    if acc == "f32":
        if t == torch.float32:
            return _lib.TSG_R32_ACC32
        if t == torch.complex64:
            return _lib.TSG_C64_ACC32
        raise TypeError("acc='f32' needs float32 or complex64 storage")
    return _DT[t]


def tsmttsm(A, B, op="T", out=None, acc="f64"):
    """C = op(A)^T B for tall row-major A (K x M) and B (K x N) on the GPU.

    op: 'T' (transpose) or 'C' (conjugate transpose, complex only).
    float32 / complex64 inputs are the precision form; C is always float64 /
    complex128.  acc='f32' (binary32 storage only) sums binary32 products in
    binary32 over stretches of 32 rows, binary64 beyond.  ``out`` may be an
    (M x N) row-major tensor to write into.
    """
    if A.dtype != B.dtype or A.dtype not in _DT:
        raise TypeError("A and B must share one of float64, complex128, float32, complex64")
    if A.device != B.device or A.device.type != "cuda":
        raise ValueError("A and B must be on the same GPU")
    K, M = A.shape
    if B.shape[0] != K:
        raise ValueError("A and B must have the same number of rows")
    N = B.shape[1]
    if out is None:
        out = torch.empty((M, N), dtype=_SMALL[A.dtype], device=A.device)
    elif out.shape != (M, N) or out.dtype != _SMALL[A.dtype] or out.device != A.device:
        raise ValueError("out must be an (M, N) %s tensor on %s" % (_SMALL[A.dtype], A.device))
    with torch.cuda.device(A.device):
        _lib.check(_lib.tsg_tsmttsm(_dtype(A.dtype, acc), _lib.TSG_OP_C if op == "C" else _lib.TSG_OP_T, K, M, N,
                                    A.data_ptr(), _ld(A, "A"), B.data_ptr(), _ld(B, "B"),
                                    out.data_ptr(), _ld(out, "out"), _stream(A.device)))
    return out


def tsmm(A, C, out=None, alpha=1.0, beta=0.0, conjA=False, opC="N", acc="f64"):
    """B = alpha * op(A) opC(C) + beta * out for tall A (K x M).

    opC: 'N' uses C (M x N); 'T' uses C^T and 'C' uses C^H of a stored
    (N x M) C -- the small matrix is transposed on chip, not copied.
    Writes into ``out`` (K x N, A's dtype) when given, else into a new tensor
    (beta must then be 0).  C is float64 / complex128 for every storage type.
    """
    if A.dtype not in _DT or C.dtype != _SMALL[A.dtype]:
        raise TypeError("unsupported dtype combination %s, %s" % (A.dtype, C.dtype))
    if A.device != C.device or A.device.type != "cuda":
        raise ValueError("A and C must be on the same GPU")
    if opC not in ("N", "T", "C"):
        raise ValueError("opC must be 'N', 'T' or 'C'")
    K, M = A.shape
    Mc, N = (C.shape[0], C.shape[1]) if opC == "N" else (C.shape[1], C.shape[0])
    if Mc != M:
        raise ValueError("op(C) must have M rows")
    if out is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs out")
        out = torch.empty((K, N), dtype=A.dtype, device=A.device)
    elif out.shape != (K, N) or out.dtype != A.dtype or out.device != A.device:
        raise ValueError("out must be a (K, N) %s tensor on %s" % (A.dtype, A.device))
    op = {"N": _lib.TSG_OP_N, "T": _lib.TSG_OP_T, "C": _lib.TSG_OP_C}[opC]
    with torch.cuda.device(A.device):
        _lib.check(_lib.tsg_tsmm_op(_dtype(A.dtype, acc), int(bool(conjA)), op, K, M, N, A.data_ptr(), _ld(A, "A"),
                                    C.data_ptr(), _ld(C, "C"), out.data_ptr(), _ld(out, "out"),
                                    float(alpha), float(beta), _stream(A.device)))
    return out


def kernel_name(op, dtype, M, N, conj=False, acc="f64"):
    """Name of the kernel variant the library launches for this problem."""
    return _lib.tsg_kernel_name(0 if op == "tsmttsm" else 1, _dtype(dtype, acc), int(conj), M, N)


class OrthPlan:
    """Batched block orthogonalisation: for every pair (V_i, W_i),
    C_i = V_i^T W_i and then W_i <- W_i - V_i C_i, all instances in one
    persistent kernel launch (replayed from a captured hipGraph).

    V_i (K_i x M_i, M_i <= 64) and W_i (K_i x N_i, N_i <= 16) are row-major
    float64 tensors on one GPU; W_i is updated in place and C_i (M_i x N_i)
    is written to ``self.C[i]``.  The tensors must stay alive and must not
    move while the plan exists.  Launches of one plan must not overlap.
    """

    def __init__(self, pairs, rows_per_item=0, C=None):
        if not pairs:
            raise ValueError("need at least one (V, W) pair")
        dev = pairs[0][0].device
        if dev.type != "cuda":
            raise ValueError("V and W must be on a GPU")
        self.device = dev
        self.pairs = list(pairs)
        self.C = []
        descs = []
        for i, (V, W) in enumerate(self.pairs):
            if V.dtype != torch.float64 or W.dtype != torch.float64:
                raise TypeError("instance %d: V and W must be float64" % i)
            if V.device != dev or W.device != dev:
                raise ValueError("instance %d: all tensors must be on %s" % (i, dev))
            if V.dim() != 2 or W.dim() != 2 or V.shape[0] != W.shape[0]:
                raise ValueError("instance %d: V (K x M) and W (K x N) must have the same rows" % i)
            K, M = V.shape
            N = W.shape[1]
            Ci = C[i] if C is not None else torch.empty((M, N), dtype=torch.float64, device=dev)
            if Ci.shape != (M, N) or Ci.dtype != torch.float64 or Ci.device != dev:
                raise ValueError("instance %d: C must be an (M, N) float64 tensor on %s" % (i, dev))
            self.C.append(Ci)
            descs.append(_lib.tsg_orth_desc(K, M, N, V.data_ptr(), _ld(V, "V"), W.data_ptr(), _ld(W, "W"),
                                            Ci.data_ptr(), _ld(Ci, "C")))
        with torch.cuda.device(dev):
            st, plan = _lib.tsg_orth_plan_create(descs, rows_per_item, _stream(dev))
        _lib.check(st)
        self._plan = plan

    def launch(self):
        """Replay the captured graph on the current stream (asynchronous)."""
        with torch.cuda.device(self.device):
            _lib.check(_lib.tsg_orth_plan_launch(self._plan, _stream(self.device)))
        return self.C

    def run(self):
        """Launch the persistent kernel directly on the current stream."""
        with torch.cuda.device(self.device):
            _lib.check(_lib.tsg_orth_plan_run(self._plan, _stream(self.device)))
        return self.C

    def check(self):
        """Wait for the device; raise if a wait inside a launch gave up."""
        with torch.cuda.device(self.device):
            _lib.check(_lib.tsg_orth_plan_check(self._plan))

    def set_spin_limit(self, limit):
        with torch.cuda.device(self.device):
            _lib.check(_lib.tsg_orth_plan_set_spin_limit(self._plan, int(limit)))

    def close(self):
        if getattr(self, "_plan", None):
            with torch.cuda.device(self.device):
                _lib.tsg_orth_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class OrthBatch:
    """The batched orthogonalisation through ``tsg_orth_batched``: the
    descriptors live in device memory and every ``run()`` is one call of two
    kernel launches on the current stream, with no allocation and no host
    synchronisation (it can be captured into a graph).  ``workspace`` may be
    a caller's uint8 tensor of at least ``workspace_bytes`` bytes (256-byte
    aligned); by default one is allocated here.  Same tensors and rules as
    ``OrthPlan``; calls sharing a workspace must not overlap."""

    def __init__(self, pairs, C=None, workspace=None):
        if not pairs:
            raise ValueError("need at least one (V, W) pair")
        dev = pairs[0][0].device
        self.device = dev
        self.pairs = list(pairs)
        self.C = []
        descs = []
        kmax = mmax = nmax = 1
        for i, (V, W) in enumerate(self.pairs):
            if V.dtype != torch.float64 or W.dtype != torch.float64:
                raise TypeError("instance %d: V and W must be float64" % i)
            if V.device != dev or W.device != dev or V.dim() != 2 or W.dim() != 2 or V.shape[0] != W.shape[0]:
                raise ValueError("instance %d: V (K x M) and W (K x N) on %s with the same rows" % (i, dev))
            K, M = V.shape
            N = W.shape[1]
            Ci = C[i] if C is not None else torch.empty((M, N), dtype=torch.float64, device=dev)
            self.C.append(Ci)
            descs.append(_lib.tsg_orth_desc(K, M, N, V.data_ptr(), _ld(V, "V"), W.data_ptr(), _ld(W, "W"),
                                            Ci.data_ptr(), _ld(Ci, "C")))
            kmax, mmax, nmax = max(kmax, K), max(mmax, M), max(nmax, N)
        raw = (_lib.tsg_orth_desc * len(descs))(*descs)
        host = torch.frombuffer(bytearray(bytes(raw)), dtype=torch.uint8)
        self.d_descs = host.to(dev)
        with torch.cuda.device(dev):
            self.workspace_bytes = _lib.tsg_workspace_size(_lib.TSG_KIND_ORTH, _lib.TSG_R64, kmax, mmax, nmax,
                                                           len(descs))
        if self.workspace_bytes == 0:
            raise ValueError("widths or instance count outside the supported range")
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=dev)
            off = (-workspace.data_ptr()) % 256
            workspace = workspace[off:off + self.workspace_bytes]
        self.workspace = workspace

    def run(self):
        with torch.cuda.device(self.device):
            _lib.check(_lib.tsg_orth_batched(self.d_descs.data_ptr(), len(self.pairs), self.workspace.data_ptr(),
                                             self.workspace.numel(), _stream(self.device)))
        return self.C

    def check(self):
        """Wait for the device; raise if the last call was rejected on the
        device or a wait inside it gave up."""
        with torch.cuda.device(self.device):
            _lib.check(_lib.tsg_orth_batched_check(self.workspace.data_ptr()))


def orth_batched(pairs, rows_per_item=0):
    """One batched orthogonalisation step over ``pairs`` [(V_i, W_i), ...]:
    W_i is updated in place, the list of C_i = V_i^T W_i (old W_i) returned."""
    plan = OrthPlan(pairs, rows_per_item)
    try:
        C = plan.launch()
        plan.check()
    finally:
        plan.close()
    return C
