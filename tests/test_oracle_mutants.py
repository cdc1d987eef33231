"""The oracle's pins have teeth: each planted mistake fails at least one pin.

A mutant is a copy of the oracle's C source with one plausible slip written
into it (a dropped term, a flipped sign, a transposed index, a wrong leading
dimension, an old output read when beta == 0, a lost conjugation, a lost
compensation).  It is built on the CPU into a temporary directory and run
through the pin tests of ``test_oracle``; the test passes only if some pin
rejects it.  The mutants never touch the real oracle.
"""
import os

import pytest

import oracle
from oracle.oracle import _SRC, Oracle
from tests import test_oracle as pins

MUTANTS = {
    "drop_last_k": ("for (int64_t k = 0; k < K; ++k) {\n            const double a = A[k * lda + m];",
                    "for (int64_t k = 0; k < K - 1; ++k) {\n            const double a = A[k * lda + m];"),
    "complex_sign": ("const double pr = ar * br - ai * bi;", "const double pr = ar * br + ai * bi;"),
    "tsmm_transposed_C": ("else      s = s + arow[m] * C[(int64_t)m * ldc + n];",
                          "else      s = s + arow[m] * C[(int64_t)n * ldc + m];"),
    "lda_as_M": ("const double a = A[k * lda + m];", "const double a = A[k * M + m];"),
    "beta_zero_reads_old": ("brow[n] = (beta == 0.0) ? alpha * s : alpha * s + beta * brow[n];",
                            "brow[n] = alpha * s + beta * brow[n];"),
    "lost_conjugation": ("const double ai = conjA ? -A[2 * (k * lda + m) + 1] : A[2 * (k * lda + m) + 1];",
                         "const double ai = A[2 * (k * lda + m) + 1];"),
    "tsmm_imag_sign": ("si = si + (ar * xi + ai * xr);", "si = si + (ar * xi - ai * xr);"),
    "lost_compensation": ("*c = *c + (et + ep);", "*c = *c + 0.0 * (et + ep);"),
    "alpha_dropped": ("brow[2 * n]     = alpha * sr;", "brow[2 * n]     = sr;"),
    "tsmm_lost_compensation": ("if (comp) s = s + c;", "if (comp) s = s + 0.0 * c;"),
    "tsmm_cplx_lost_compensation": ("if (comp) { sr = sr + cr; si = si + ci; }",
                                    "if (comp) { sr = sr + 0.0 * cr; si = si + ci; }"),
}

PIN_TESTS = [
    (pins.test_tsmttsm_exact_integers, [dict(M=5, N=7, cplx=False), dict(M=5, N=7, cplx=True),
                                        dict(M=1, N=13, cplx=True)]),
    (pins.test_tsmm_exact_integers, [dict(M=5, N=7, cplx=False), dict(M=5, N=7, cplx=True),
                                     dict(M=3, N=2, cplx=True)]),
    (pins.test_tsmttsm_error_bounds_vs_exact, [dict(cplx=False), dict(cplx=True)]),
    (pins.test_compensated_beats_plain_on_cancelling_sum, [dict()]),
    (pins.test_closed_forms, [dict(cplx=False), dict(cplx=True)]),
    (pins.test_symmetry_transpose_linearity, [dict(cplx=False), dict(cplx=True)]),
    (pins.test_complex_equals_real_expansion, [dict(conj=False), dict(conj=True)]),
    (pins.test_leading_dimensions_and_beta_zero, [dict(cplx=False), dict(cplx=True)]),
    (pins.test_numpy_blas_agreement, [dict(M=4, N=4, cplx=True)]),
    (pins.test_tsmm_compensated_error_bound_vs_exact, [dict(cplx=False), dict(cplx=True)]),
]


def _caught(orc):
    for fn, cases in PIN_TESTS:
        for kw in cases:
            try:
                fn(orc, **kw)
            except (AssertionError, ValueError):
                return fn.__name__
    return None


def test_unmutated_copy_passes_all_pins(tmp_path):
    with open(_SRC) as f:
        src = f.read()
    path = tmp_path / "same.c"
    path.write_text(src)
    lib = oracle.build(force=True, src=str(path), out=str(tmp_path / "libsame.so"))
    assert _caught(Oracle(lib)) is None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    with open(_SRC) as f:
        src = f.read()
    assert src.count(old) >= 1, "mutation site vanished from the oracle source"
    path = tmp_path / (name + ".c")
    path.write_text(src.replace(old, new, 1))
    lib = oracle.build(force=True, src=str(path), out=str(tmp_path / ("lib%s.so" % name)))
    assert os.path.exists(lib)
    assert _caught(Oracle(lib)) is not None, "mutant %s passed every pin" % name
