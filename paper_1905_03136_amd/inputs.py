"""Seeded synthetic inputs for the tall & skinny products.

This module only draws numbers.  It holds none of the products' arithmetic and
imports neither the GPU library nor the oracle, so that both sides can be fed
the very same inputs.

The paper does not state the value distribution of its matrices (it only fixes
the sweep size K = 2^29 / M in Section 5).  Inputs here are iid uniform(-1, 1)
entries (real and imaginary parts drawn independently for complex data), drawn
from numpy's PCG64 stream ``default_rng([seed, stream])`` so that every matrix
of a case has a stream of its own.  Complex data are interleaved (re, im).

Large matrices are generated on the GPU with torch's seeded Philox generator
(``device_uniform``); they are not bit-identical to the numpy draws, and parity
checks at such sizes copy the needed rows or columns back to the host.
"""
import numpy as np

# stream ids of the matrices of one case
STREAM_A, STREAM_B, STREAM_C, STREAM_DC, STREAM_BASE = 0, 1, 2, 3, 4
STREAM_NOISE0 = 5          # noise_j uses STREAM_NOISE0 + j
STREAM_KBATCH, STREAM_WIDTHS = 100, 101
STREAM_V0, STREAM_W0 = 1000, 2000


def rng(seed, stream):
    return np.random.default_rng([int(seed), int(stream)])


def host_uniform(rows, cols, seed=0, stream=STREAM_A, cplx=False, lo=-1.0, hi=1.0):
    """rows x cols float64 (or complex128) matrix of iid uniform(lo, hi) entries."""
    g = rng(seed, stream)
    if cplx:
        return g.uniform(lo, hi, (rows, 2 * cols)).view(np.complex128)
    return g.uniform(lo, hi, (rows, cols))


def host_integers(rows, cols, seed=0, stream=STREAM_A, cplx=False, lo=-8, hi=8):
    """Integer-valued doubles in [lo, hi]: sums of their products are exact in
    binary64 while K * max|a b| stays below 2^53."""
    g = rng(seed, stream)
    if cplx:
        return g.integers(lo, hi + 1, (rows, 2 * cols)).astype(np.float64).view(np.complex128)
    return g.integers(lo, hi + 1, (rows, cols)).astype(np.float64)


def near_parallel(rows, cols, seed=0, cplx=False, eps=1e-4):
    """Ill-conditioned block vector: column j = base + eps * noise_j, with base
    and noise_j iid uniform(-1, 1) columns."""
    base = host_uniform(rows, 1, seed, STREAM_BASE, cplx)
    out = np.empty((rows, cols), dtype=np.complex128 if cplx else np.float64)
    for j in range(cols):
        out[:, j:j + 1] = base + eps * host_uniform(rows, 1, seed, STREAM_NOISE0 + j, cplx)
    return out


def zero_column_sum(rows, cols, seed=0, stream=STREAM_C, cplx=False):
    """Small matrix whose columns sum to zero (the last row is minus the sum of
    the others), so that a product with near-parallel rows cancels strongly."""
    X = host_uniform(rows, cols, seed, stream, cplx)
    if rows > 1:
        X[-1, :] = -X[:-1, :].sum(axis=0)
    return X


def device_uniform(rows, cols, seed=0, stream=STREAM_A, cplx=False, device="cuda",
                   dtype=None, out=None):
    """Large uniform(-1, 1) matrix drawn directly in device memory.

    Returns a torch tensor (float64 or complex128 unless ``dtype`` asks for
    float32 / complex64).  ``out`` may be a preallocated tensor of that shape.
    """
    import torch
    g = torch.Generator(device=device)
    g.manual_seed((int(seed) << 20) + int(stream))
    real = {None: torch.float64, torch.float64: torch.float64, torch.complex128: torch.float64,
            torch.float32: torch.float32, torch.complex64: torch.float32}[dtype]
    width = 2 * cols if cplx else cols
    if out is None:
        flat = torch.empty((rows, width), dtype=real, device=device)
    else:
        flat = torch.view_as_real(out).reshape(rows, width) if cplx else out
    flat.uniform_(-1.0, 1.0, generator=g)
    if cplx:
        return torch.view_as_complex(flat.view(rows, cols, 2))
    return flat


def batched_instances(count=64, seed=0, kmin_log2=16, kmax_log2=22,
                      m_choices=(4, 8, 16, 32, 64), n_choices=(1, 4, 8, 16)):
    """Shapes of the batched block-orthogonalisation workload: K_i log-uniform
    in [2^kmin, 2^kmax], M_i and N_i uniform over the given choices."""
    g = rng(seed, STREAM_KBATCH)
    u = g.uniform(0.0, 1.0, count)
    Ks = np.rint(2.0 ** (kmin_log2 + (kmax_log2 - kmin_log2) * u)).astype(np.int64)
    gw = rng(seed, STREAM_WIDTHS)
    Ms = gw.choice(np.asarray(m_choices), count)
    Ns = gw.choice(np.asarray(n_choices), count)
    return [(int(k), int(m), int(n)) for k, m, n in zip(Ks, Ms, Ns)]


def orthonormal_block(rows, cols, seed=0, stream=STREAM_V0):
    """Tall block vector with orthonormal columns: the Q factor of a reduced
    CPU QR decomposition of a uniform(-1, 1) matrix."""
    X = host_uniform(rows, cols, seed, stream)
    Q, _ = np.linalg.qr(X, mode="reduced")
    return np.ascontiguousarray(Q)
