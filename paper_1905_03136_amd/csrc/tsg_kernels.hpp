// tsg_kernels.hpp -- gfx950 kernel templates for the two tall & skinny products
//   TSMTTSM  C = op(A)^T B   (Section 3 of the paper)
//   TSMM     B = alpha op(A) C + beta B   (Section 4)
// A (K x M), B (K x N) row-major with leading dimensions lda, ldb; C (M x N)
// row-major with ldc.  Complex data are interleaved (re, im) doubles.
//
// Template parameters MC / NC are the compile-time widths (0 = taken at run
// time, bounded by the tile extents).  The code generator instantiates one
// variant per (op, dtype, M, N) plus run-time-width fallbacks.
#pragma once
#include <type_traits>

#include "tsg_device.hpp"

namespace tsg {

template <bool CPLX>
using elem_t = typename std::conditional<CPLX, zd, double>::type;

template <class T>
__device__ __forceinline__ T zero_of();
template <>
__device__ __forceinline__ double zero_of<double>() { return 0.0; }
template <>
__device__ __forceinline__ zd zero_of<zd>() { return zd{0.0, 0.0}; }

// ============================================================================
// TSMTTSM on the matrix cores.
//
// The sum over the long dimension K is the contraction of
// v_mfma_f64_16x16x4f64: for four rows k0..k0+3 a wave multiplies the 16 x 4
// fragment A(k0..k0+3, m-block)^T by the 4 x 16 fragment B(k0..k0+3, n-block)
// and accumulates a 16 x 16 block of partial C.  Lane l supplies
// A(k0 + l/16, m0 + l%16) and B(k0 + l/16, n0 + l%16): sixteen lanes read 16
// consecutive elements of one row, so every fragment load is a fully used
// 128-byte (256-byte complex) segment, each element of A and B is read from
// HBM exactly once, and no lane needs another lane's data.  This is the
// paper's tiled K-loop mapping (Section 3, Listings 2-5) with the register
// tile replaced by matrix-core accumulators; the "next" fragment set is
// loaded while the current one is multiplied (leap frogging, Section 3.1).
//
// Complex data use four real products per complex block,
//   Cr += Ar Br - Ai Bi,   Ci += Ar Bi + Ai Br,
// with each lane holding the (re, im) pair of one element (one 16-byte load).
//
// Waves of a block are arranged as RG row groups x MW m-slices: the MW waves
// of a row group share the same rows and split the m-blocks of C between
// them (needed when the accumulators of a full C exceed the register file).
//
// Output layout of the 16x16 FP64 accumulator (checked on gfx950 with an
// in-bounds probe): lane l, element r holds D(l / 16 + 4 r, l % 16).
// ============================================================================
template <int MC, int NC, int MB, int NB, int MW, int U, bool CPLX, int WPB>
__global__ void __launch_bounds__(WPB * kWave)
tsmttsm_mfma(int64_t K, int Mr, int Nr, const void* __restrict__ Av, int64_t lda,
             const void* __restrict__ Bv, int64_t ldb, double* __restrict__ C, int64_t ldc,
             double* __restrict__ ws, unsigned* __restrict__ cnt, int conj)
{
    using T = elem_t<CPLX>;
    constexpr int CW = CPLX ? 2 : 1;
    constexpr int RG = WPB / MW;
    constexpr int RT = 4 * U * RG;
    constexpr int EMAX = (MC ? MC : MW * MB * 16) * (NC ? NC : NB * 16) * CW;
    static_assert(WPB % MW == 0, "waves must split evenly");
    __shared__ double part[EMAX];

    const T* __restrict__ A = static_cast<const T*>(Av);
    const T* __restrict__ B = static_cast<const T*>(Bv);
    const int M = MC ? MC : Mr;
    const int N = NC ? NC : Nr;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int mw = wave % MW;
    const int rg = wave / MW;
    const int lr = lane >> 4;
    const int lc = lane & 15;

    int moff[MB], noff[NB];
    bool mok[MB], nok[NB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int m = (mw * MB + i) * 16 + lc;
        mok[i] = m < M;
        moff[i] = mok[i] ? m : 0;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int n = j * 16 + lc;
        nok[j] = n < N;
        noff[j] = nok[j] ? n : 0;
    }

    dbl4 acc[MB][NB];
    dbl4 acci[CPLX ? MB : 1][CPLX ? NB : 1];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
            if constexpr (CPLX) acci[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
        }

    const int64_t ntiles = (K + RT - 1) / RT;
    T a[U][MB], b[U][NB], an[U][MB], bn[U][NB];

    auto load = [&](int64_t t, T (&xa)[U][MB], T (&xb)[U][NB]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = t * RT + (int64_t)(rg * U + u) * 4 + lr;
            const bool ok = row < K;
            const T* ar = A + row * lda;
            const T* br = B + row * ldb;
#pragma unroll
            for (int i = 0; i < MB; ++i) xa[u][i] = (ok && mok[i]) ? ld_stream(ar + moff[i]) : zero_of<T>();
#pragma unroll
            for (int j = 0; j < NB; ++j) xb[u][j] = (ok && nok[j]) ? ld_stream(br + noff[j]) : zero_of<T>();
        }
    };

    int64_t t = blockIdx.x;
    if (t < ntiles) load(t, a, b);
    for (; t < ntiles; t += gridDim.x) {
        const int64_t tn = t + gridDim.x;
        if (tn < ntiles) load(tn, an, bn);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (!CPLX) {
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][i], b[u][j], acc[i][j], 0, 0, 0);
            } else {
                double nbi[NB];
#pragma unroll
                for (int j = 0; j < NB; ++j) nbi[j] = -b[u][j].im;
#pragma unroll
                for (int i = 0; i < MB; ++i) {
                    const double ar = a[u][i].re;
                    const double ai = conj ? -a[u][i].im : a[u][i].im;
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, b[u][j].re, acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, nbi[j], acc[i][j], 0, 0, 0);
                        acci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, b[u][j].im, acci[i][j], 0, 0, 0);
                        acci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, b[u][j].re, acci[i][j], 0, 0, 0);
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int i = 0; i < MB; ++i) a[u][i] = an[u][i];
#pragma unroll
            for (int j = 0; j < NB; ++j) b[u][j] = bn[u][j];
        }
    }

    // Fold the row groups into the block partial, one group after the other.
    const int E = M * N * CW;
    for (int g = 0; g < RG; ++g) {
        if (rg == g) {
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int m = (mw * MB + i) * 16 + lr + 4 * r;
                        const int n = j * 16 + lc;
                        if (m < M && n < N) {
                            const int e = (m * N + n) * CW;
                            part[e] = (g == 0) ? acc[i][j][r] : part[e] + acc[i][j][r];
                            if constexpr (CPLX) part[e + 1] = (g == 0) ? acci[i][j][r] : part[e + 1] + acci[i][j][r];
                        }
                    }
        }
        __syncthreads();
    }
    grid_fold(part, E, ws, cnt, [&](int e, double v) {
        const int q = e / CW;
        const int m = q / N, n = q - (q / N) * N;
        C[((int64_t)m * ldc + n) * CW + (e - q * CW)] = v;
    });
}

// ============================================================================
// TSMTTSM on the vector ALUs for narrow widths.
//
// Parallelisation over K only (the paper's Fig. "genv1" mapping): every lane
// owns whole rows and keeps the full M x N partial C in registers, so a lane
// needs no data of any other lane and each FMA operand is a register.  A wave
// covers 64 consecutive rows per load instruction.  U rows per lane are in
// flight per iteration and the next iteration's rows are loaded while the
// current ones are multiplied (leap frogging).  After the K loop the lanes'
// partials are summed by a fixed butterfly (wave_sum), the waves of a block
// one after the other, and the blocks by grid_fold.
//
// MX x NX bound the register tile; MC / NC = 0 takes M, N at run time
// (entries beyond them are skipped by guards).  VA / VB load pairs of doubles
// with one 16-byte load (needs even widths, even leading dimensions and
// 16-byte aligned pointers; real data only).
// ============================================================================
template <int MC, int NC, int MX, int NX, int U, bool CPLX, bool VA, bool VB, int WPB>
__global__ void __launch_bounds__(WPB * kWave)
tsmttsm_valu(int64_t K, int Mr, int Nr, const void* __restrict__ Av, int64_t lda,
             const void* __restrict__ Bv, int64_t ldb, double* __restrict__ C, int64_t ldc,
             double* __restrict__ ws, unsigned* __restrict__ cnt, int conj)
{
    using T = elem_t<CPLX>;
    constexpr int CW = CPLX ? 2 : 1;
    constexpr int RT = kWave * U * WPB;
    constexpr int EMAX = MX * NX * CW;
    static_assert(!(CPLX && (VA || VB)), "complex elements are already 16-byte loads");
    static_assert(!VA || MX % 2 == 0, "paired loads need an even width");
    static_assert(!VB || NX % 2 == 0, "paired loads need an even width");
    __shared__ double part[EMAX];

    const T* __restrict__ A = static_cast<const T*>(Av);
    const T* __restrict__ B = static_cast<const T*>(Bv);
    const int M = MC ? MC : Mr;
    const int N = NC ? NC : Nr;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;

    T acc[MX][NX];
#pragma unroll
    for (int i = 0; i < MX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) acc[i][j] = zero_of<T>();

    const int64_t ntiles = (K + RT - 1) / RT;
    T a[U][MX], b[U][NX], an[U][MX], bn[U][NX];

    auto load = [&](int64_t t, T (&xa)[U][MX], T (&xb)[U][NX]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = t * RT + (int64_t)(wave * U + u) * kWave + lane;
            const bool ok = row < K;
            const T* ar = A + row * lda;
            const T* br = B + row * ldb;
            if constexpr (VA) {
                typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
                for (int i = 0; i < MX; i += 2) {
                    d2 v = d2{0.0, 0.0};
                    if (ok && (MC || i < M)) v = __builtin_nontemporal_load(reinterpret_cast<const d2*>(ar + i));
                    xa[u][i] = v.x;
                    xa[u][i + 1] = v.y;
                }
            } else {
#pragma unroll
                for (int i = 0; i < MX; ++i) xa[u][i] = (ok && (MC || i < M)) ? ld_stream(ar + i) : zero_of<T>();
            }
            if constexpr (VB) {
                typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
                for (int j = 0; j < NX; j += 2) {
                    d2 v = d2{0.0, 0.0};
                    if (ok && (NC || j < N)) v = __builtin_nontemporal_load(reinterpret_cast<const d2*>(br + j));
                    xb[u][j] = v.x;
                    xb[u][j + 1] = v.y;
                }
            } else {
#pragma unroll
                for (int j = 0; j < NX; ++j) xb[u][j] = (ok && (NC || j < N)) ? ld_stream(br + j) : zero_of<T>();
            }
        }
    };

    int64_t t = blockIdx.x;
    if (t < ntiles) load(t, a, b);
    for (; t < ntiles; t += gridDim.x) {
        const int64_t tn = t + gridDim.x;
        if (tn < ntiles) load(tn, an, bn);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < MX; ++i)
#pragma unroll
                for (int j = 0; j < NX; ++j) {
                    if constexpr (!CPLX) {
                        acc[i][j] = __builtin_fma(a[u][i], b[u][j], acc[i][j]);
                    } else {
                        const double ai = conj ? -a[u][i].im : a[u][i].im;
                        acc[i][j].re = __builtin_fma(a[u][i].re, b[u][j].re, acc[i][j].re);
                        acc[i][j].re = __builtin_fma(-ai, b[u][j].im, acc[i][j].re);
                        acc[i][j].im = __builtin_fma(a[u][i].re, b[u][j].im, acc[i][j].im);
                        acc[i][j].im = __builtin_fma(ai, b[u][j].re, acc[i][j].im);
                    }
                }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int i = 0; i < MX; ++i) a[u][i] = an[u][i];
#pragma unroll
            for (int j = 0; j < NX; ++j) b[u][j] = bn[u][j];
        }
    }

    // Wave sums (fixed butterfly), then the waves folded one after the other.
    const int E = M * N * CW;
#pragma unroll
    for (int i = 0; i < MX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            if ((MC || i < M) && (NC || j < N)) {
                if constexpr (CPLX) {
                    acc[i][j].re = wave_sum(acc[i][j].re);
                    acc[i][j].im = wave_sum(acc[i][j].im);
                } else {
                    acc[i][j] = wave_sum(acc[i][j]);
                }
            }
        }
    for (int w = 0; w < WPB; ++w) {
        if (wave == w) {
#pragma unroll
            for (int i = 0; i < MX; ++i)
#pragma unroll
                for (int j = 0; j < NX; ++j) {
                    if ((MC || i < M) && (NC || j < N) && lane == ((i * NX + j) & (kWave - 1))) {
                        const int e = (i * N + j) * CW;
                        if constexpr (CPLX) {
                            part[e] = (w == 0) ? acc[i][j].re : part[e] + acc[i][j].re;
                            part[e + 1] = (w == 0) ? acc[i][j].im : part[e + 1] + acc[i][j].im;
                        } else {
                            part[e] = (w == 0) ? acc[i][j] : part[e] + acc[i][j];
                        }
                    }
                }
        }
        __syncthreads();
    }
    grid_fold(part, E, ws, cnt, [&](int e, double v) {
        const int q = e / CW;
        const int m = q / N, n = q - (q / N) * N;
        C[((int64_t)m * ldc + n) * CW + (e - q * CW)] = v;
    });
}

// ============================================================================
// TSMM on the vector ALUs for narrow widths.
//
// Parallelisation over K only (the paper's Fig. "tsmm_mapping_1T" mapping):
// a lane computes whole rows of B.  All lanes of a wave use the same entry of
// C at the same time, so C is read through the scalar unit into SGPRs and
// broadcast to the FMAs: no LDS traffic and no per-lane C registers.  The
// rows of a wave are consecutive, so the wave's stores fill whole cache lines
// in L2 before they are written back (no write-allocate traffic on CDNA).
// ============================================================================
template <int MC, int NC, int MX, int NX, int U, bool CPLX, bool VA, bool VB, int WPB>
__global__ void __launch_bounds__(WPB * kWave)
tsmm_valu(int64_t K, int Mr, int Nr, const void* __restrict__ Av, int64_t lda,
          const double* __restrict__ Cm, int64_t ldc, void* __restrict__ Bv, int64_t ldb,
          double alpha, double beta, int conj)
{
    using T = elem_t<CPLX>;
    constexpr int RT = kWave * U * WPB;
    static_assert(!(CPLX && (VA || VB)), "complex elements are already 16-byte loads");
    const T* __restrict__ A = static_cast<const T*>(Av);
    T* __restrict__ B = static_cast<T*>(Bv);
    const T* __restrict__ Cz = reinterpret_cast<const T*>(Cm);
    const int M = MC ? MC : Mr;
    const int N = NC ? NC : Nr;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const bool read_b = beta != 0.0;
    const int64_t ntiles = (K + RT - 1) / RT;

    T a[U][MX], an[U][MX];
    auto load = [&](int64_t t, T (&xa)[U][MX]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = t * RT + (int64_t)(wave * U + u) * kWave + lane;
            const bool ok = row < K;
            const T* ar = A + row * lda;
            if constexpr (VA) {
                typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
                for (int i = 0; i < MX; i += 2) {
                    d2 v = d2{0.0, 0.0};
                    if (ok && (MC || i < M)) v = __builtin_nontemporal_load(reinterpret_cast<const d2*>(ar + i));
                    xa[u][i] = v.x;
                    xa[u][i + 1] = v.y;
                }
            } else {
#pragma unroll
                for (int i = 0; i < MX; ++i) xa[u][i] = (ok && (MC || i < M)) ? ld_stream(ar + i) : zero_of<T>();
            }
        }
    };

    int64_t t = blockIdx.x;
    if (t < ntiles) load(t, a);
    for (; t < ntiles; t += gridDim.x) {
        const int64_t tn = t + gridDim.x;
        if (tn < ntiles) load(tn, an);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = t * RT + (int64_t)(wave * U + u) * kWave + lane;
            if (row < K) {
                T* br = B + row * ldb;
                T out[NX];
#pragma unroll
                for (int j = 0; j < NX; ++j) {
                    T s = zero_of<T>();
#pragma unroll
                    for (int i = 0; i < MX; ++i) {
                        if ((MC || i < M) && (NC || j < N)) {
                            const T c = Cz[(int64_t)i * ldc + j];
                            if constexpr (!CPLX) {
                                s = __builtin_fma(a[u][i], c, s);
                            } else {
                                const double ai = conj ? -a[u][i].im : a[u][i].im;
                                s.re = __builtin_fma(a[u][i].re, c.re, s.re);
                                s.re = __builtin_fma(-ai, c.im, s.re);
                                s.im = __builtin_fma(a[u][i].re, c.im, s.im);
                                s.im = __builtin_fma(ai, c.re, s.im);
                            }
                        }
                    }
                    out[j] = s;
                }
                if constexpr (VB) {
                    typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
                    for (int j = 0; j < NX; j += 2) {
                        if (NC || j < N) {
                            d2 v = d2{alpha * out[j], alpha * out[j + 1]};
                            if (read_b) {
                                const d2 o = *reinterpret_cast<const d2*>(br + j);
                                v = d2{__builtin_fma(beta, o.x, v.x), __builtin_fma(beta, o.y, v.y)};
                            }
                            __builtin_nontemporal_store(v, reinterpret_cast<d2*>(br + j));
                        }
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < NX; ++j) {
                        if (NC || j < N) {
                            if constexpr (!CPLX) {
                                double v = alpha * out[j];
                                if (read_b) v = __builtin_fma(beta, br[j], v);
                                __builtin_nontemporal_store(v, br + j);
                            } else {
                                typedef double d2 __attribute__((ext_vector_type(2)));
                                d2 v = d2{alpha * out[j].re, alpha * out[j].im};
                                if (read_b) {
                                    const zd o = br[j];
                                    v = d2{__builtin_fma(beta, o.re, v.x), __builtin_fma(beta, o.im, v.y)};
                                }
                                __builtin_nontemporal_store(v, reinterpret_cast<d2*>(br + j));
                            }
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < MX; ++i) a[u][i] = an[u][i];
    }
}

// ============================================================================
// TSMM on the matrix cores for wider matrices.
//
// Sixteen rows of B at a time: B(k0..k0+15, n-block) = sum_s A(k0..k0+15,
// 4s..4s+3) C(4s..4s+3, n-block), one v_mfma_f64_16x16x4f64 per (s, n-block);
// the contraction runs over the short dimension M (the paper's Fig.
// "tsmm_cube": the TSMM cube reduces along M).  C is staged once per block in
// LDS in fragment order (Section 4.2: C in shared memory, loaded
// cooperatively and amortised over a grid-stride loop), so every lane reads
// its C operand with one conflict-free 8-byte LDS read, and each C operand
// feeds U row blocks (the paper's K-unrolling, Section 4.2).  A lane stores
// rows l/16 + 4r (r < 4) of column l%16 of each 16 x 16 output block: sixteen
// lanes write 128 consecutive bytes of a row.
// ============================================================================
template <int MC, int NC, int MS, int NB, int U, bool CPLX, int WPB>
__global__ void __launch_bounds__(WPB * kWave)
tsmm_mfma(int64_t K, int Mr, int Nr, const void* __restrict__ Av, int64_t lda,
          const double* __restrict__ Cm, int64_t ldc, void* __restrict__ Bv, int64_t ldb,
          double alpha, double beta, int conj)
{
    using T = elem_t<CPLX>;
    constexpr int CW = CPLX ? 2 : 1;
    constexpr int RT = 16 * U * WPB;
    constexpr int NFRAG = MS * NB * kWave;
    __shared__ double cf[NFRAG * CW];

    const T* __restrict__ A = static_cast<const T*>(Av);
    T* __restrict__ B = static_cast<T*>(Bv);
    const int M = MC ? MC : Mr;
    const int N = NC ? NC : Nr;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int lr = lane >> 4;
    const int lc = lane & 15;
    const bool read_b = beta != 0.0;

    // Stage C in fragment order: cf[(s * NB + j) * 64 + l] = C(4s + l/16, 16j + l%16).
    for (int idx = threadIdx.x; idx < NFRAG; idx += blockDim.x) {
        const int l = idx & (kWave - 1);
        const int sj = idx / kWave;
        const int s = sj / NB, j = sj - (sj / NB) * NB;
        const int m = 4 * s + (l >> 4), n = 16 * j + (l & 15);
        const bool ok = m < M && n < N;
        if constexpr (CPLX) {
            cf[idx] = ok ? Cm[2 * ((int64_t)m * ldc + n)] : 0.0;
            cf[NFRAG + idx] = ok ? Cm[2 * ((int64_t)m * ldc + n) + 1] : 0.0;
        } else {
            cf[idx] = ok ? Cm[(int64_t)m * ldc + n] : 0.0;
        }
    }
    __syncthreads();

    int koff[MS];
    bool kok[MS];
#pragma unroll
    for (int s = 0; s < MS; ++s) {
        const int m = 4 * s + lr;
        kok[s] = m < M;
        koff[s] = kok[s] ? m : 0;
    }

    const int64_t ntiles = (K + RT - 1) / RT;
    T a[U][MS], an[U][MS];
    auto load = [&](int64_t t, T (&xa)[U][MS]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = t * RT + (int64_t)(wave * U + u) * 16 + lc;
            const bool ok = row < K;
            const T* ar = A + row * lda;
#pragma unroll
            for (int s = 0; s < MS; ++s) xa[u][s] = (ok && kok[s]) ? ld_stream(ar + koff[s]) : zero_of<T>();
        }
    };

    int64_t t = blockIdx.x;
    if (t < ntiles) load(t, a);
    for (; t < ntiles; t += gridDim.x) {
        // Compiler-only barrier: keeps the loop-invariant C operands in LDS
        // instead of letting them be hoisted into (too many) registers.
        __asm__ volatile("" ::: "memory");
        const int64_t tn = t + gridDim.x;
        if (tn < ntiles) load(tn, an);
        dbl4 acc[U][NB];
        dbl4 acci[CPLX ? U : 1][CPLX ? NB : 1];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                acc[u][j] = dbl4{0.0, 0.0, 0.0, 0.0};
                if constexpr (CPLX) acci[u][j] = dbl4{0.0, 0.0, 0.0, 0.0};
            }
#pragma unroll
        for (int s = 0; s < MS; ++s)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const double cr = cf[(s * NB + j) * kWave + lane];
                if constexpr (!CPLX) {
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        acc[u][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][s], cr, acc[u][j], 0, 0, 0);
                } else {
                    const double ci = cf[NFRAG + (s * NB + j) * kWave + lane];
                    const double nci = -ci;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const double ar = a[u][s].re;
                        const double ai = conj ? -a[u][s].im : a[u][s].im;
                        acc[u][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, cr, acc[u][j], 0, 0, 0);
                        acc[u][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, nci, acc[u][j], 0, 0, 0);
                        acci[u][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, ci, acci[u][j], 0, 0, 0);
                        acci[u][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, cr, acci[u][j], 0, 0, 0);
                    }
                }
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t rbase = t * RT + (int64_t)(wave * U + u) * 16 + lr;
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int n = 16 * j + lc;
                if (n < N) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t row = rbase + 4 * r;
                        if (row < K) {
                            T* p = B + row * ldb + n;
                            if constexpr (!CPLX) {
                                double v = alpha * acc[u][j][r];
                                if (read_b) v = __builtin_fma(beta, *p, v);
                                __builtin_nontemporal_store(v, p);
                            } else {
                                typedef double d2 __attribute__((ext_vector_type(2)));
                                d2 v = d2{alpha * acc[u][j][r], alpha * acci[u][j][r]};
                                if (read_b) {
                                    const zd o = *p;
                                    v = d2{__builtin_fma(beta, o.re, v.x), __builtin_fma(beta, o.im, v.y)};
                                }
                                __builtin_nontemporal_store(v, reinterpret_cast<d2*>(p));
                            }
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int s = 0; s < MS; ++s) a[u][s] = an[u][s];
    }
}

}  // namespace tsg
