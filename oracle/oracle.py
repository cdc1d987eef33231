"""ctypes wrapper around the C oracle in ``tso_oracle.c``.

TEST INFRASTRUCTURE ONLY: the plain CPU definition of the two products the GPU
library computes, used to check it.  It shares no code with the GPU library and
must never be called from the library's own code path.

Definitions (Section 1.1, problem statement; Section 2.2, Listing 1):
  TSMTTSM  C = op(A)^T B,  C[m][n] = sum_k op(A[k][m]) B[k][n]   (k ascending)
  TSMM     B = alpha * op(A) C + beta * B_old                      (m ascending)
with A (K x M), B (K x N) row-major tall & skinny, C (M x N) small.  op is the
identity or, for complex data, elementwise conjugation (the Hermitian product
A^H B that classical Gram-Schmidt needs, Section 1.2).

``compensated=True`` evaluates every sum with the Dot2 algorithm (Ogita, Rump,
Oishi 2005), which is as accurate as a sum in doubled precision.
"""
import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tso_oracle.c")
_LIB = os.path.join(_HERE, "libtso_oracle.so")
_lock = threading.Lock()
_lib = None

_CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11"]


def build(force=False, src=_SRC, out=_LIB):
    """Compile the oracle with gcc (no GPU toolchain involved)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_CFLAGS, src, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


def _bind(path):
    lib = ctypes.CDLL(path)
    i64, i32, dp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    lib.tso_tsmttsm.argtypes = [i32, i32, i32, i64, i32, i32, dp, i64, dp, i64, dp, i64, i32]
    lib.tso_tsmttsm.restype = i32
    lib.tso_tsmm.argtypes = [i32, i32, i32, i64, i32, i32, dp, i64, dp, i64, dp, i64,
                             ctypes.c_double, ctypes.c_double, i32]
    lib.tso_tsmm.restype = i32
    lib.tso_max_threads.argtypes = []
    lib.tso_max_threads.restype = i32
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            _lib = _bind(_LIB)
    return _lib


def _check2d(X, name):
    if not isinstance(X, np.ndarray) or X.ndim != 2:
        raise TypeError("%s must be a 2-D numpy array" % name)
    if X.dtype not in (np.float64, np.complex128):
        raise TypeError("%s must be float64 or complex128, got %s" % (name, X.dtype))
    it = X.itemsize
    if X.size == 0:
        return X.shape[1]
    if X.shape[1] > 1 and X.strides[1] != it:
        raise ValueError("%s must have unit column stride" % name)
    if X.shape[0] > 1 and (X.strides[0] % it or X.strides[0] < X.shape[1] * it):
        raise ValueError("%s has an unsupported row stride" % name)
    ld = X.strides[0] // it if X.shape[0] > 1 else X.shape[1]
    return max(ld, X.shape[1])


class Oracle:
    """The oracle bound to one compiled library (the default one, or a test
    build of the same source)."""

    def __init__(self, path=None):
        self._path = path
        self._handle = None

    def _lib(self):
        if self._path is None:
            return _load()
        if self._handle is None:
            self._handle = _bind(self._path)
        return self._handle

    def max_threads(self):
        """Number of OpenMP threads the oracle uses by default."""
        return int(self._lib().tso_max_threads())

    def tsmttsm(self, A, B, op="T", compensated=False, nthreads=0):
        """C = op(A)^T B as a new (M, N) array (float64 or complex128)."""
        ldA, ldB = _check2d(A, "A"), _check2d(B, "B")
        if A.dtype != B.dtype or A.shape[0] != B.shape[0]:
            raise ValueError("A and B must share dtype and row count")
        if op not in ("T", "C"):
            raise ValueError("op must be 'T' or 'C'")
        K, M = A.shape
        N = B.shape[1]
        cplx = A.dtype == np.complex128
        C = np.zeros((M, N), dtype=A.dtype)
        rc = self._lib().tso_tsmttsm(int(cplx), int(op == "C" and cplx), int(bool(compensated)), K, M, N,
                                     A.ctypes.data, ldA, B.ctypes.data, ldB, C.ctypes.data, N,
                                     int(nthreads))
        if rc:
            raise ValueError("oracle rejected the arguments")
        return C

    def tsmm(self, A, C, B=None, alpha=1.0, beta=0.0, conjA=False, compensated=False, nthreads=0):
        """B = alpha * op(A) C + beta * B (in place when B is given, else a new array)."""
        ldA, ldC = _check2d(A, "A"), _check2d(C, "C")
        K, M = A.shape
        if C.shape[0] != M or C.dtype != A.dtype:
            raise ValueError("C must be M x N with A's dtype")
        N = C.shape[1]
        if B is None:
            if beta != 0.0:
                raise ValueError("beta != 0 needs B")
            B = np.zeros((K, N), dtype=A.dtype)
        ldB = _check2d(B, "B")
        if B.shape != (K, N) or B.dtype != A.dtype:
            raise ValueError("B must be K x N with A's dtype")
        cplx = A.dtype == np.complex128
        rc = self._lib().tso_tsmm(int(cplx), int(bool(conjA) and cplx), int(bool(compensated)), K, M, N,
                                  A.ctypes.data, ldA, C.ctypes.data, ldC, B.ctypes.data, ldB,
                                  float(alpha), float(beta), int(nthreads))
        if rc:
            raise ValueError("oracle rejected the arguments")
        return B

    def tsmttsm_entries(self, A, B, pairs, op="T", compensated=True):
        """Selected entries C[m][n] of op(A)^T B, each a single length-K sum.

        Used to check full-size results one entry at a time: every entry is the
        1 x 1 TSMTTSM of column m of A and column n of B.
        """
        out = np.empty(len(pairs), dtype=A.dtype)
        for i, (m, n) in enumerate(pairs):
            out[i] = self.tsmttsm(A[:, m:m + 1], B[:, n:n + 1], op=op, compensated=compensated,
                                  nthreads=1)[0, 0]
        return out

    def tsmm_rows(self, A_rows, C, B_old_rows=None, alpha=1.0, beta=0.0, conjA=False):
        """Rows of alpha * op(A) C + beta * B_old for a sample of rows of A."""
        B = None if B_old_rows is None else np.array(B_old_rows, copy=True)
        return self.tsmm(np.ascontiguousarray(A_rows), np.ascontiguousarray(C), B, alpha, beta, conjA)

    def orth_step(self, V, W, compensated=False):
        """One block Gram-Schmidt projection step (Section 1.2).

        C = V^H W from the old W, then W_new = W - V C.  Returns (C, W_new); W is
        not modified.
        """
        op = "C" if V.dtype == np.complex128 else "T"
        C = self.tsmttsm(V, W, op=op, compensated=compensated)
        W_new = self.tsmm(V, C, np.array(W, copy=True), alpha=-1.0, beta=1.0)
        return C, W_new


_default = Oracle()
tsmttsm = _default.tsmttsm
tsmm = _default.tsmm
tsmttsm_entries = _default.tsmttsm_entries
tsmm_rows = _default.tsmm_rows
orth_step = _default.orth_step
max_threads = _default.max_threads
