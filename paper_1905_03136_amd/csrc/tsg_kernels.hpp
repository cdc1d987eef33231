// tsg_kernels.hpp -- gfx950 kernel templates for the two tall & skinny products
//   TSMTTSM  C = op(A)^T B            (Section 3 of the paper)
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

__device__ __forceinline__ dbl4 mfma16(double a, double b, dbl4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Value of lane 16 (l / 16) + c for lane l: the DPP row broadcast
// (row_newbcast) of one lane of every row of 16 lanes, two 32-bit moves per
// double.  c must fold to a constant (the DPP control is an immediate).
template <int C_>
__device__ __forceinline__ double row_bcast_c(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x150 + C_, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x150 + C_, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row_bcast(double v, int c)
{
    switch (c) {
    case 0: return row_bcast_c<0>(v);
    case 1: return row_bcast_c<1>(v);
    case 2: return row_bcast_c<2>(v);
    case 3: return row_bcast_c<3>(v);
    case 4: return row_bcast_c<4>(v);
    case 5: return row_bcast_c<5>(v);
    case 6: return row_bcast_c<6>(v);
    case 7: return row_bcast_c<7>(v);
    case 8: return row_bcast_c<8>(v);
    case 9: return row_bcast_c<9>(v);
    case 10: return row_bcast_c<10>(v);
    case 11: return row_bcast_c<11>(v);
    case 12: return row_bcast_c<12>(v);
    case 13: return row_bcast_c<13>(v);
    case 14: return row_bcast_c<14>(v);
    default: return row_bcast_c<15>(v);
    }
}
__device__ __forceinline__ zd row_bcast(zd v, int c) { return zd{row_bcast(v.re, c), row_bcast(v.im, c)}; }

// acc += op(a) b for the VALU tail strips (op = conjugate when conj).
__device__ __forceinline__ void fma_tail(double& acc, double a, double b, int) { acc = __builtin_fma(a, b, acc); }
__device__ __forceinline__ void fma_tail(zd& acc, zd a, zd b, int conj)
{
    const double ai = conj ? -a.im : a.im;
    acc.re = __builtin_fma(a.re, b.re, __builtin_fma(-ai, b.im, acc.re));
    acc.im = __builtin_fma(a.re, b.im, __builtin_fma(ai, b.re, acc.im));
}

// Sum over the four k-slots (lanes l, l ^ 16, l ^ 32, l ^ 48), fixed order.
__device__ __forceinline__ double slot_sum(double v)
{
    v += __shfl_xor(v, 16, kWave);
    return v + __shfl_xor(v, 32, kWave);
}
__device__ __forceinline__ zd slot_sum(zd v) { return zd{slot_sum(v.re), slot_sum(v.im)}; }

// ---------------------------------------------------------- slab reads
// Where the rows of a tall matrix are contiguous (ld = width), the rows a wave
// consumes in one tile are one contiguous run; slab reads load that run with
// consecutive loads of FL storage elements per lane (one contiguous piece of
// up to 1 KB per load instruction, whatever the width), store it in the
// wave's own LDS region and read the matrix-core operands back from there.
// Registers of one tile: per-row fragments, or the lane's share of the run.
template <class T, int U, int MS>
struct row_regs {
    T a[U][MS];
};
template <class SV, int NL>
struct slab_regs {
    SV v[NL];
};
typedef float flt4 __attribute__((ext_vector_type(4)));
template <class S, int FL>
struct slab_vec;
template <>
struct slab_vec<double, 1> { typedef double type; };
template <>
struct slab_vec<double, 2> { typedef dbl2 type; };
template <>
struct slab_vec<float, 1> { typedef float type; };
template <>
struct slab_vec<float, 2> { typedef flt2 type; };
template <>
struct slab_vec<float, 4> { typedef flt4 type; };
// real type of a storage element (complex elements are two of them)
template <class S>
struct real_of { typedef S type; };
template <>
struct real_of<zd> { typedef double type; };
template <>
struct real_of<zf> { typedef float type; };
// element idx of a run staged in LDS, widened to binary64
__device__ __forceinline__ double lds_elem(const double* p, int idx, double) { return p[idx]; }
__device__ __forceinline__ double lds_elem(const float* p, int idx, double) { return (double)p[idx]; }
__device__ __forceinline__ zd lds_elem(const double* p, int idx, zd) { return zd{p[2 * idx], p[2 * idx + 1]}; }
__device__ __forceinline__ zd lds_elem(const float* p, int idx, zd)
{
    return zd{(double)p[2 * idx], (double)p[2 * idx + 1]};
}

// Load the lane's share of a run of n elements starting at element e0 of a
// matrix of `total` elements: load i covers elements e0 + (64 i + lane) FL ..;
// positions past the end are clamped to the last FL elements (total is a
// multiple of FL), their values are never used.
template <int FL, int NL, class SR, class SV>
__device__ __forceinline__ void slab_load(const SR* p, int64_t e0, int64_t total, int lane, SV (&v)[NL])
{
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int64_t e = e0 + (int64_t)(i * kWave + lane) * FL;
        const int64_t ec = e <= total - FL ? e : total - FL;
        v[i] = __builtin_nontemporal_load(reinterpret_cast<const SV*>(p + ec));
    }
}
// Store the lane's share (n elements of the run) into the wave's LDS region.
// The lanes then read each other's elements.  The hardware completes one
// wave's LDS accesses in order, so no barrier instruction is needed, but the
// compiler must see the exchange: without a memory barrier it may treat a
// lane's read as independent of the other lanes' writes, keep the value read
// for the previous tile, and move the read under the lane mask of the
// conditional write (observed: lanes past the run's end then used stale
// operands).  The empty asm with a memory clobber is that barrier.
template <int FL, int NL, int n, class SR, class SV>
__device__ __forceinline__ void slab_put(SR* lds, int lane, const SV (&v)[NL])
{
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int o = (i * kWave + lane) * FL;
        if (i + 1 < NL || o < n) *reinterpret_cast<SV*>(lds + o) = v[i];
    }
    __asm__ volatile("" ::: "memory");
}

// Run-time run length n (single-element loads, n at most 64 NL): load i of
// the lane is issued only where its element lies in the run; elements past
// the end of the matrix are clamped to its last one (their values are never
// used), and slab_put_n writes only the run's n elements.
template <int NL, class SR>
__device__ __forceinline__ void slab_load_n(const SR* p, int64_t e0, int64_t total, int lane, int n, SR (&v)[NL])
{
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int o = i * kWave + lane;
        if (o < n) {
            const int64_t e = e0 + o;
            v[i] = __builtin_nontemporal_load(p + (e < total ? e : total - 1));
        }
    }
}
template <int NL, class SR>
__device__ __forceinline__ void slab_put_n(SR* lds, int lane, int n, const SR (&v)[NL])
{
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int o = i * kWave + lane;
        if (o < n) lds[o] = v[i];
    }
    __asm__ volatile("" ::: "memory");
}

// Element (m, n) of TSMM's small operand op(C): opc 0 reads C(m, n) = C[m ldc + n];
// opc 1 (transpose) and 2 (conjugate transpose, the caller negates the
// imaginary part) read C[n ldc + m] of a stored N x M matrix.
__device__ __forceinline__ int64_t small_index(int m, int n, int64_t ldc, int opc)
{
    return opc ? (int64_t)n * ldc + m : (int64_t)m * ldc + n;
}

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
// tile replaced by matrix-core accumulators; the fragments of the next tile
// are loaded while the current ones are multiplied (leap frogging, Section 3.1).
//
// Complex data use four real products per complex block,
//   Cr += Ar Br - Ai Bi,   Ci += Ar Bi + Ai Br,
// with each lane holding the (re, im) pair of one element (one 16-byte load).
// With G3 they use three (Gauss's form of the complex product):
//   P1 += Ar Br,  P2 += Ai Bi,  P3 += (Ar + Ai)(Br + Bi),
//   Cr = P1 - P2,  Ci = P3 - P1 - P2,
// a quarter fewer matrix-core products for two vector additions per loaded
// element.  The sums are the same up to rounding; the error bound of Ci
// grows by a small constant factor (|Ar + Ai||Br + Bi| <= 2 |A||B|).
//
// Waves of a block are arranged as RG row groups x MW m-slices: the MW waves
// of a row group share the same rows and split the m-blocks of C between
// them (needed when the accumulators of a full C exceed the register file).
//
// Output layout of the 16x16 FP64 accumulator (checked on gfx950 with an
// in-bounds probe): lane l, element r holds D(l / 16 + 4 r, l % 16).
//
// TL (tails on the vector unit; compile-time widths, MW = 1): where M or N is
// not a multiple of 16, a padded 16-wide block would spend a whole row or
// column of matrix-core products on RM = M mod 16 (RN = N mod 16) useful
// rows, and these kernels are bound by the matrix cores there.  With TL only
// the full blocks go to the matrix cores; the column strip C(:, N - RN ..) and
// the row strip C(M - RM .., full columns) are vector FMAs: lane (q, i) of a
// k-slot q multiplies its A(k, 16 b + i) by B(k, N - RN + c), broadcast from
// lane c of its row of 16 lanes, and its B(k, 16 b + i) by A(k, M - RM + r)
// likewise, keeping (M_blocks RN + N_full RM) partial sums per lane, which
// the epilogue sums over the four k-slots.
//
// FL (slab reads; lda = M, ldb = N, compile-time widths whose rows are a
// multiple of FL real elements, MW = 1): the 4U rows of a wave are read as
// two contiguous runs (see slab_load), staged in the wave's LDS region, and
// the fragments above are read from there; at widths whose rows are not
// whole 128-byte lines the per-row fragment loads touch more lines per load.
// ============================================================================
template <int MC, int NC, int MB, int NB, int MW, int U, bool CPLX, int WPB, int NBUF, int OCC = 1,
          bool F32 = false, bool G3 = false, bool TL = false, int FL = 0>
__global__ void __launch_bounds__(WPB * kWave, OCC)
tsmttsm_mfma(int64_t K, int Mr, int Nr, const void* __restrict__ Av, int64_t lda,
             const void* __restrict__ Bv, int64_t ldb, double* __restrict__ C, int64_t ldc,
             double* __restrict__ ws, int conj)
{
    using T = elem_t<CPLX>;
    using S = typename storage<CPLX, F32>::type;  // storage type; loads widen S -> T
    constexpr int CW = CPLX ? 2 : 1;
    constexpr int RG = WPB / MW;
    constexpr int RT = 4 * U * RG;
    constexpr int EMAX = (MC ? MC : MW * MB * 16) * (NC ? NC : NB * 16) * CW;
    static_assert(WPB % MW == 0, "waves must split evenly");
    static_assert(!TL || (MC > 0 && NC > 0 && MW == 1 && MB == (MC + 15) / 16 && NB == (NC + 15) / 16),
                  "vector tails: compile-time widths, one wave per row group");
    static_assert(FL == 0 || (MW == 1 && MC > 0 && NC > 0 && (MC * CW) % FL == 0 && (NC * CW) % FL == 0),
                  "slab reads: compile-time widths whose rows are multiples of FL, one wave per row group");
    constexpr int RM = TL ? MC % 16 : 0;        // rows of C in the row strip
    constexpr int RN = TL ? NC % 16 : 0;        // columns of C in the column strip
    constexpr int MF = MB - (RM ? 1 : 0);       // m-blocks on the matrix cores
    constexpr int NF = NB - (RN ? 1 : 0);       // n-blocks on the matrix cores
    __shared__ double part[EMAX];

    const S* __restrict__ A = static_cast<const S*>(Av);
    const S* __restrict__ B = static_cast<const S*>(Bv);
    const int M = MC ? MC : Mr;
    const int N = NC ? NC : Nr;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int mw = wave % MW;
    const int rg = wave / MW;
    const int lr = lane >> 4;
    const int lc = lane & 15;

    // Column offsets.  A lane whose column lies past the width reads a valid
    // element of the same row instead (column 0); such values only reach
    // entries of C past M or N, which are never stored, so they need no
    // zeroing (rows past K are zeroed: they would reach every entry).  Where
    // a compile-time width covers every column a lane can address, the test
    // is the constant true and the offset is the plain column.
    int moff[MB], noff[NB];
    bool mok[MB], nok[NB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int m = (mw * MB + i) * 16 + lc;
        mok[i] = (MC && ((MW - 1) * MB + i + 1) * 16 <= MC) || m < M;
        moff[i] = mok[i] ? m : 0;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int n = j * 16 + lc;
        nok[j] = (NC && (j + 1) * 16 <= NC) || n < N;
        noff[j] = nok[j] ? n : 0;
    }

    static_assert(CPLX || !G3, "the three-product form is for complex data");
    dbl4 acc[MB][NB];
    dbl4 acci[CPLX ? MB : 1][CPLX ? NB : 1];
    dbl4 accs[G3 ? MB : 1][G3 ? NB : 1];  // G3: P1 in acc, P2 in acci, P3 in accs
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
            if constexpr (CPLX) acci[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
            if constexpr (G3) accs[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
        }
    // TL: tc[b][c] sums A(k, 16 b + lc) B(k, NF 16 + c), tr[b][r] sums A(k, MF 16 + r) B(k, 16 b + lc)
    static_assert(!TL || (MF >= 1 && NF >= 1), "vector tails serve widths above 16");
    T tc[RN ? MB : 1][RN ? RN : 1];
    T tr[RM ? NF : 1][RM ? RM : 1];
#pragma unroll
    for (int i = 0; i < (RN ? MB : 1); ++i)
#pragma unroll
        for (int c = 0; c < (RN ? RN : 1); ++c) tc[i][c] = zero_of<T>();
#pragma unroll
    for (int j = 0; j < (RM ? NF : 1); ++j)
#pragma unroll
        for (int r = 0; r < (RM ? RM : 1); ++r) tr[j][r] = zero_of<T>();

    // FL (slab reads, real data, lda = M and ldb = N): the 4U rows of a wave
    // are runs of 4U M elements of A and 4U N elements of B
    constexpr int SLA = FL ? 4 * U * MC * CW : 0, SLB = FL ? 4 * U * NC * CW : 0;  // real elements
    constexpr int NLA = FL ? (SLA + kWave * FL - 1) / (kWave * FL) : 1;
    constexpr int NLB = FL ? (SLB + kWave * FL - 1) / (kWave * FL) : 1;
    using SR = typename real_of<S>::type;                         // real storage type (slab reads)
    using SV = typename slab_vec<SR, FL ? FL : 1>::type;          // one slab load of a lane
    __shared__ __attribute__((aligned(16))) SR slab[FL ? WPB * (SLA + SLB) : 1];
    SR* const mya = slab + (FL ? wave * (SLA + SLB) : 0);
    SR* const myb = mya + SLA;

    struct RowFrag {
        T a[U][MB];
        T b[U][NB];
    };
    struct SlabFrag {
        SV a[NLA];
        SV b[NLB];
    };
    using Frag = typename std::conditional<FL != 0, SlabFrag, RowFrag>::type;
    Frag fr[NBUF];
    auto load = [&](int64_t t, Frag& f) {
        if constexpr (FL) {
            const int64_t r0 = t * RT + (int64_t)rg * U * 4;
            slab_load<FL, NLA>(reinterpret_cast<const SR*>(A), r0 * MC * CW, K * (int64_t)(MC * CW), lane, f.a);
            slab_load<FL, NLB>(reinterpret_cast<const SR*>(B), r0 * NC * CW, K * (int64_t)(NC * CW), lane, f.b);
        } else {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = t * RT + (int64_t)(rg * U + u) * 4 + lr;
            const bool ok = row < K;
            const int64_t rc = ok ? row : K - 1;
            const S* ar = A + rc * lda;
            const S* br = B + rc * ldb;
#pragma unroll
            for (int i = 0; i < MB; ++i) f.a[u][i] = keep(ok, ld_stream(ar + moff[i]));
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                // with MW > 1 the waves of a row group read the same B: keep it in cache
                if constexpr (MW > 1)
                    f.b[u][j] = keep(ok, ld_shared(br + noff[j]));
                else
                    f.b[u][j] = keep(ok, ld_stream(br + noff[j]));
            }
        }
        }
    };
    auto compute = [&](int64_t t, Frag& f) {
        // matrix-core operands of the tile (from LDS with slab reads; rows past K are zero)
        T av[U][MB], bv[U][NB];
        if constexpr (FL) {
            slab_put<FL, NLA, SLA>(mya, lane, f.a);
            slab_put<FL, NLB, SLB>(myb, lane, f.b);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool ok = t * RT + (int64_t)(rg * U + u) * 4 + lr < K;
#pragma unroll
                for (int i = 0; i < MB; ++i) av[u][i] = keep(ok, lds_elem(mya, (4 * u + lr) * MC + moff[i], T{}));
#pragma unroll
                for (int j = 0; j < NB; ++j) bv[u][j] = keep(ok, lds_elem(myb, (4 * u + lr) * NC + noff[j], T{}));
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int i = 0; i < MB; ++i) av[u][i] = f.a[u][i];
#pragma unroll
                for (int j = 0; j < NB; ++j) bv[u][j] = f.b[u][j];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // matrix cores: blocks i < MF, j < NF (all blocks without TL)
            if constexpr (!CPLX) {
#pragma unroll
                for (int i = 0; i < MF; ++i)
#pragma unroll
                    for (int j = 0; j < NF; ++j) acc[i][j] = mfma16(av[u][i], bv[u][j], acc[i][j]);
            } else if constexpr (G3) {
                // three passes over all blocks, so the updates of one
                // accumulator are MF NF instructions apart; the sums
                // Ar + Ai and Br + Bi are formed just before the pass that
                // uses them (fewer values live at once)
                double ai[MB];
#pragma unroll
                for (int i = 0; i < MF; ++i) ai[i] = conj ? -av[u][i].im : av[u][i].im;
#pragma unroll
                for (int i = 0; i < MF; ++i)
#pragma unroll
                    for (int j = 0; j < NF; ++j) acc[i][j] = mfma16(av[u][i].re, bv[u][j].re, acc[i][j]);
#pragma unroll
                for (int i = 0; i < MF; ++i)
#pragma unroll
                    for (int j = 0; j < NF; ++j) acci[i][j] = mfma16(ai[i], bv[u][j].im, acci[i][j]);
#pragma unroll
                for (int i = 0; i < MF; ++i) ai[i] += av[u][i].re;  // Ar + Ai
#pragma unroll
                for (int j = 0; j < NF; ++j) {
                    const double sb = bv[u][j].re + bv[u][j].im;
#pragma unroll
                    for (int i = 0; i < MF; ++i) accs[i][j] = mfma16(ai[i], sb, accs[i][j]);
                }
            } else {
                // All products with Re(a) first, then those with Im(a): the two
                // updates of one accumulator are 2 MF NF instructions apart
                // instead of back to back.
                double nbi[NB];
#pragma unroll
                for (int j = 0; j < NF; ++j) nbi[j] = -bv[u][j].im;
#pragma unroll
                for (int i = 0; i < MF; ++i)
#pragma unroll
                    for (int j = 0; j < NF; ++j) {
                        acc[i][j] = mfma16(av[u][i].re, bv[u][j].re, acc[i][j]);
                        acci[i][j] = mfma16(av[u][i].re, bv[u][j].im, acci[i][j]);
                    }
#pragma unroll
                for (int i = 0; i < MF; ++i) {
                    const double ai = conj ? -av[u][i].im : av[u][i].im;
#pragma unroll
                    for (int j = 0; j < NF; ++j) {
                        acc[i][j] = mfma16(ai, nbi[j], acc[i][j]);
                        acci[i][j] = mfma16(ai, bv[u][j].re, acci[i][j]);
                    }
                }
            }
            // vector unit: the column strip (all m-blocks, including the
            // partial one, times the broadcast tail columns of B) and the row
            // strip (broadcast tail rows of A times the full n-blocks of B)
            if constexpr (RN > 0) {
#pragma unroll
                for (int c = 0; c < RN; ++c) {
                    const T bc = row_bcast(bv[u][NB - 1], c);
#pragma unroll
                    for (int i = 0; i < MB; ++i) fma_tail(tc[i][c], av[u][i], bc, conj);
                }
            }
            if constexpr (RM > 0) {
#pragma unroll
                for (int r = 0; r < RM; ++r) {
                    const T ar = row_bcast(av[u][MB - 1], r);
#pragma unroll
                    for (int j = 0; j < NF; ++j) fma_tail(tr[j][r], ar, bv[u][j], conj);
                }
            }
        }
    };
    const int64_t ntiles = (K + RT - 1) / RT;
    pipeline<NBUF>(blockIdx.x, ntiles, (int64_t)gridDim.x, fr, load, compute);
    if constexpr (G3) {
        // Cr = P1 - P2, Ci = P3 - P1 - P2
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const dbl4 p1 = acc[i][j], p2 = acci[i][j];
                acc[i][j] = p1 - p2;
                acci[i][j] = accs[i][j] - p1 - p2;
            }
    }

    // TL: sum the tail strips over the four k-slots (every lane gets the sum)
#pragma unroll
    for (int i = 0; i < (RN ? MB : 0); ++i)
#pragma unroll
        for (int c = 0; c < RN; ++c) tc[i][c] = slot_sum(tc[i][c]);
#pragma unroll
    for (int j = 0; j < (RM ? NF : 0); ++j)
#pragma unroll
        for (int r = 0; r < RM; ++r) tr[j][r] = slot_sum(tr[j][r]);

    // Fold the row groups into the block partial, one group after the other.
    const int E = M * N * CW;
    auto put = [&](int g, int e, T v) {
        if constexpr (CPLX) {
            part[e] = (g == 0) ? v.re : part[e] + v.re;
            part[e + 1] = (g == 0) ? v.im : part[e + 1] + v.im;
        } else {
            part[e] = (g == 0) ? v : part[e] + v;
        }
    };
    for (int g = 0; g < RG; ++g) {
        if (rg == g) {
#pragma unroll
            for (int i = 0; i < MF; ++i)
#pragma unroll
                for (int j = 0; j < NF; ++j)
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
            if (lr == 0) {
#pragma unroll
                for (int i = 0; i < (RN ? MB : 0); ++i)
#pragma unroll
                    for (int c = 0; c < RN; ++c) {
                        const int m = i * 16 + lc;
                        if (m < M) put(g, (m * N + NF * 16 + c) * CW, tc[i][c]);
                    }
#pragma unroll
                for (int j = 0; j < (RM ? NF : 0); ++j)
#pragma unroll
                    for (int r = 0; r < RM; ++r) put(g, ((MF * 16 + r) * N + j * 16 + lc) * CW, tr[j][r]);
            }
        }
        __syncthreads();
    }
    block_out<CW>(part, E, N, ws, C, ldc);
}

// ============================================================================
// TSMTTSM on the matrix cores with the rows staged in LDS by direct loads.
//
// The register-ring kernels above hold the next tile's operands in VGPRs
// while the current tile is multiplied, so how far ahead they can load is
// set by the register file, and at the wide widths (complex 33..64, real
// 49..64) the rings that would hide the memory latency spill.  Here the rows
// travel from HBM straight into LDS (global_load_lds_dwordx4: each lane
// brings 16 bytes, a wave 1 KB of consecutive bytes, with no VGPR holding
// the data) in stages of RT rows shared by the whole block, two stages in
// turn: while the matrix cores work on stage t, stage t + 1 is in flight.
// Each wave reads the operands of its own blocks of C for the whole stage
// into registers (the matrix-core operand layout of tsmttsm_mfma) right after
// the barrier that publishes the stage, then issues the loads of the next
// stage into the other buffer and multiplies (with IL > 0 only the first IL
// steps are read up front, the rest IL steps ahead of their products).  A
// block of WM x WN waves covers C with MB x NB blocks of 16 x 16 per wave;
// every wave reads every row of the stage, each element of A and B crosses
// HBM once, and each lane writes its entries of the block partial straight
// from its accumulators (lds_out).
//
// Needs lda = M and ldb = N (a stage is one contiguous run of A and one of
// B), 16-byte aligned A and B, and an even number of doubles in each of A
// and B (complex data, or even real widths): lane addresses past the end of
// a matrix are clamped to its last 16 bytes, which then hold only elements
// of rows past K, zeroed when read from LDS.  (With an odd count the last
// element would share its 16 bytes with the end and be moved by the clamp.)
// ============================================================================

// Epilogue of the LDS-staged kernels, whose waves own disjoint blocks of C:
// lane (lr, lc) holds entry r of block (i, j) at row 16 (wm MB + i) + lr + 4 r
// (binary64 products) or + 4 lr + r (binary32 products, f32rows), column
// 16 (wn NB + j) + lc.  Each entry is written once, to slot blockIdx.x of the
// workspace in block_out's layout (E doubles per slot) or, for a grid of one
// block, to C.
template <int CW, int MB, int NB, class ACC, class ACCI>
__device__ __forceinline__ void lds_out(const ACC& acc, const ACCI& acci, int wm, int wn, int lr, int lc, int MC,
                                        int NC, int E, double* __restrict__ ws, double* __restrict__ C, int64_t ldc,
                                        bool f32rows)
{
    const bool direct = gridDim.x == 1;
    double* dst = ws + (direct ? 0 : (size_t)blockIdx.x * E);
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = (wm * MB + i) * 16 + (f32rows ? 4 * lr + r : lr + 4 * r);
                const int n = (wn * NB + j) * 16 + lc;
                if (m < MC && n < NC) {
                    double* p = direct ? C + ((int64_t)m * ldc + n) * CW : dst + (m * NC + n) * CW;
                    p[0] = acc[i][j][r];
                    if constexpr (CW == 2) p[1] = acci[i][j][r];
                }
            }
}

// One wave-wide direct load: 64 lanes x 16 bytes from src + 2 lane (doubles)
// into 1 KB of LDS at dst (the hardware places lane l at dst + 16 l).
__device__ __forceinline__ void dma16(const double* src, double* dst)
{
    __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
}

template <int MC, int NC, int MB, int NB, int WM, int WN, int RT, bool CPLX, bool G3 = false, int OCC = 1,
          int IL = 0>
__global__ void __launch_bounds__(WM * WN * kWave, OCC)
tsmttsm_lds(int64_t K, int Mr, int Nr, const void* __restrict__ Av, int64_t lda,
            const void* __restrict__ Bv, int64_t ldb, double* __restrict__ C, int64_t ldc,
            double* __restrict__ ws, int conj)
{
    using T = elem_t<CPLX>;
    constexpr int CW = CPLX ? 2 : 1;
    constexpr int WPB = WM * WN;
    constexpr int KS = RT / 4;                                   // 4-row steps of a stage
    static_assert(MC > 0 && NC > 0 && RT % 4 == 0 && RT % 2 == 0, "compile-time widths, stages of 4-row steps");
    static_assert(WM * MB * 16 >= MC && WN * NB * 16 >= NC, "the waves' blocks cover C");
    static_assert(CPLX || !G3, "the three-product form is for complex data");
    static_assert(CPLX || (MC % 2 == 0 && NC % 2 == 0), "an even number of doubles in A and B (see above)");
    constexpr int SA = ((RT * MC * CW + 127) / 128) * 128;       // doubles of A per stage (whole 1 KB loads)
    constexpr int SB = ((RT * NC * CW + 127) / 128) * 128;
    constexpr int SS = SA + SB;                                   // one stage
    constexpr int E = MC * NC * CW;
    constexpr int NLA = SA / 128, NLB = SB / 128;                 // wave loads per stage
    __shared__ __attribute__((aligned(16))) double lds[2 * SS];  // two stages

    const double* __restrict__ A = static_cast<const double*>(Av);
    const double* __restrict__ B = static_cast<const double*>(Bv);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int wm = wave % WM, wn = wave / WM;
    const int lr = lane >> 4;
    const int lc = lane & 15;
    const int64_t totA = K * (int64_t)(MC * CW), totB = K * (int64_t)(NC * CW);   // doubles
    const int64_t lastA = (totA - 2) & ~(int64_t)1, lastB = (totB - 2) & ~(int64_t)1;

    // the stage of tile t into buffer b: wave w issues loads w, w + WPB, ...
    auto stage = [&](int64_t t, int b) {
        double* dst = lds + b * SS;
        const int64_t ea = t * (int64_t)(RT * MC * CW), eb = t * (int64_t)(RT * NC * CW);
#pragma unroll
        for (int i = wave; i < NLA + NLB; i += WPB) {
            if (i < NLA) {
                const int64_t e = ea + (int64_t)i * 128 + 2 * lane;
                dma16(A + (e <= lastA ? e : lastA), dst + i * 128);
            } else {
                const int64_t e = eb + (int64_t)(i - NLA) * 128 + 2 * lane;
                dma16(B + (e <= lastB ? e : lastB), dst + SA + (i - NLA) * 128);
            }
        }
    };

    // columns of the wave's blocks; lanes past a width read column 0 of the
    // same row (those products reach only entries of C that are not stored)
    int moff[MB], noff[NB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int m = (wm * MB + i) * 16 + lc;
        moff[i] = m < MC ? m : 0;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int n = (wn * NB + j) * 16 + lc;
        noff[j] = n < NC ? n : 0;
    }

    dbl4 acc[MB][NB];
    dbl4 acci[CPLX ? MB : 1][CPLX ? NB : 1];
    dbl4 accs[G3 ? MB : 1][G3 ? NB : 1];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
            if constexpr (CPLX) acci[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
            if constexpr (G3) accs[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
        }

    const int64_t ntiles = (K + RT - 1) / RT;
    const int64_t G = gridDim.x;
    int64_t t = blockIdx.x;
    if (t < ntiles) stage(t, 0);
    for (int b = 0; t < ntiles; t += G, b ^= 1) {
        // every wave's loads of stage t have landed; every wave is done with
        // the other buffer (its reads completed before it reached here)
        __syncthreads();
        const double* sa = lds + b * SS;
        const double* sb = sa + SA;
        T av[KS][MB], bv[KS][NB];
        auto operands = [&](int s) {
            const bool ok = t * RT + 4 * s + lr < K;
            const int r = 4 * s + lr;
#pragma unroll
            for (int i = 0; i < MB; ++i) av[s][i] = keep(ok, lds_elem(sa, r * MC + moff[i], T{}));
#pragma unroll
            for (int j = 0; j < NB; ++j) bv[s][j] = keep(ok, lds_elem(sb, r * NC + noff[j], T{}));
        };
        // IL = 0: every operand of the stage is read right after the barrier
        // (all waves of the block then read LDS at once); IL > 0: the reads
        // of step s + IL are issued between the products of step s, so the
        // block's LDS reads spread over the whole stage (scheduling barriers
        // keep the compiler from hoisting them back to the top)
#pragma unroll
        for (int s = 0; s < (IL ? (IL < KS ? IL : KS) : KS); ++s) operands(s);
        if (t + G < ntiles) stage(t + G, b ^ 1);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if constexpr (IL > 0) {
                __builtin_amdgcn_sched_barrier(0);
                if (s + IL < KS) operands(s + IL);
            }
            if constexpr (!CPLX) {
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j) acc[i][j] = mfma16(av[s][i], bv[s][j], acc[i][j]);
            } else if constexpr (G3) {
                double ai[MB];
#pragma unroll
                for (int i = 0; i < MB; ++i) ai[i] = conj ? -av[s][i].im : av[s][i].im;
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j) acc[i][j] = mfma16(av[s][i].re, bv[s][j].re, acc[i][j]);
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j) acci[i][j] = mfma16(ai[i], bv[s][j].im, acci[i][j]);
#pragma unroll
                for (int i = 0; i < MB; ++i) ai[i] += av[s][i].re;  // Ar + Ai
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const double sbj = bv[s][j].re + bv[s][j].im;
#pragma unroll
                    for (int i = 0; i < MB; ++i) accs[i][j] = mfma16(ai[i], sbj, accs[i][j]);
                }
            } else {
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        acc[i][j] = mfma16(av[s][i].re, bv[s][j].re, acc[i][j]);
                        acci[i][j] = mfma16(av[s][i].re, bv[s][j].im, acci[i][j]);
                    }
#pragma unroll
                for (int i = 0; i < MB; ++i) {
                    const double ai = conj ? -av[s][i].im : av[s][i].im;
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        acc[i][j] = mfma16(ai, -bv[s][j].im, acc[i][j]);
                        acci[i][j] = mfma16(ai, bv[s][j].re, acci[i][j]);
                    }
                }
            }
        }
    }
    if constexpr (G3) {
        // Cr = P1 - P2, Ci = P3 - P1 - P2
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const dbl4 p1 = acc[i][j], p2 = acci[i][j];
                acc[i][j] = p1 - p2;
                acci[i][j] = accs[i][j] - p1 - p2;
            }
    }
    // the waves own disjoint blocks of C: every lane writes its entries of
    // the block partial (slot blockIdx.x of the workspace, as block_out
    // lays it out) or, for a grid of one block, of C itself
    lds_out<CW, MB, NB>(acc, acci, wm, wn, lr, lc, MC, NC, E, ws, C, ldc, false);
}

// ============================================================================
// TSMTTSM on the matrix cores for narrow widths (M, N <= 16): row packing.
//
// With M, N < 16 a plain 16 x 16 fragment would leave most lanes idle and
// make every load strided.  Instead, P = min(16 / M, 16 / N) consecutive rows
// are packed into one fragment: lane i (0..15) of k-slot q holds
// A(k0 + q P + i / M, i % M) and B(k0 + q P + i / N, i % N).  With lda = M the
// sixteen lanes of a slot read 16 consecutive elements, i.e. the wave reads
// 4 P complete rows as one contiguous run.  Of the 16 x 16 product only the
// entries whose row and column come from the same packed row (i / M == j / N)
// are partial sums of C; the others are discarded.  The packed blocks are
// summed in a fixed order in the epilogue.  The matrix cores have ample
// throughput for the low arithmetic intensity of these widths (Eq. 1: M/8
// flop per byte), so the unused products cost no time.
// ============================================================================
template <int MC, int NC, int U, bool CPLX, int WPB, int NBUF, bool F32 = false>
__global__ void __launch_bounds__(WPB * kWave)
tsmttsm_packed(int64_t K, int Mr, int Nr, const void* __restrict__ Av, int64_t lda,
               const void* __restrict__ Bv, int64_t ldb, double* __restrict__ C, int64_t ldc,
               double* __restrict__ ws, int conj)
{
    using T = elem_t<CPLX>;
    using S = typename storage<CPLX, F32>::type;  // storage type; loads widen S -> T
    constexpr int CW = CPLX ? 2 : 1;
    constexpr int MX = MC ? MC : 16;
    constexpr int NX = NC ? NC : 16;
    static_assert(MX <= 16 && NX <= 16, "row packing serves widths up to 16");
    const int M = MC ? MC : Mr;
    const int N = NC ? NC : Nr;
    const int P = MC && NC ? (16 / (MC > NC ? MC : NC)) : 16 / (M > N ? M : N);
    const int RS = 4 * P;          // rows per MFMA step of one wave
    const int64_t RT = (int64_t)RS * U * WPB;
    __shared__ double part[WPB * 16 * 16 * CW];
    __shared__ double fin[MX * NX * CW];

    const S* __restrict__ A = static_cast<const S*>(Av);
    const S* __restrict__ B = static_cast<const S*>(Bv);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int q = lane >> 4;
    const int i = lane & 15;
    const int ha = i / M, ca = i - ha * M;
    const int hb = i / N, cb = i - hb * N;
    const bool aok = ha < P, bok = hb < P;

    dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
    dbl4 acci = dbl4{0.0, 0.0, 0.0, 0.0};

    struct Frag {
        T a[U];
        T b[U];
    };
    Frag fr[NBUF];
    auto load = [&](int64_t t, Frag& f) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t r0 = t * RT + (int64_t)(wave * U + u) * RS + q * P;
            const int64_t ra = r0 + (aok ? ha : 0), rb = r0 + (bok ? hb : 0);
            const bool oka = aok & (ra < K), okb = bok & (rb < K);
            f.a[u] = keep(oka, ld_stream(A + (oka ? ra : K - 1) * lda + (aok ? ca : 0)));
            f.b[u] = keep(okb, ld_stream(B + (okb ? rb : K - 1) * ldb + (bok ? cb : 0)));
        }
    };
    auto compute = [&](int64_t, Frag& f) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (!CPLX) {
                acc = mfma16(f.a[u], f.b[u], acc);
            } else {
                const double ai = conj ? -f.a[u].im : f.a[u].im;
                acc = mfma16(f.a[u].re, f.b[u].re, acc);
                acci = mfma16(f.a[u].re, f.b[u].im, acci);
                acc = mfma16(ai, -f.b[u].im, acc);
                acci = mfma16(ai, f.b[u].re, acci);
            }
        }
    };
    const int64_t ntiles = (K + RT - 1) / RT;
    pipeline<NBUF>(blockIdx.x, ntiles, (int64_t)gridDim.x, fr, load, compute);

    // D(i, j) with i = lane / 16 + 4 r, j = lane % 16 -> LDS, then the diagonal
    // blocks (i / M == j / N) are summed over packed rows and waves in order.
    double* mine = part + wave * 256 * CW;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int e = ((lane >> 4) + 4 * r) * 16 + (lane & 15);
        mine[e * CW] = acc[r];
        if constexpr (CPLX) mine[e * CW + 1] = acci[r];
    }
    __syncthreads();
    const int E = M * N * CW;
    for (int e = threadIdx.x; e < E; e += blockDim.x) {
        const int qq = e / CW, c = e - qq * CW;
        const int m = qq / N, n = qq - m * N;
        double s = 0.0;
        for (int w = 0; w < WPB; ++w)
            for (int h = 0; h < P; ++h) s += part[(w * 256 + (h * M + m) * 16 + (h * N + n)) * CW + c];
        fin[e] = s;
    }
    __syncthreads();
    block_out<CW>(fin, E, N, ws, C, ldc);
}

// ============================================================================
// TSMTTSM on the vector ALUs for narrow widths.
//
// Parallelisation over K only (the paper's Fig. "genv1" mapping): every lane
// owns whole rows and keeps the full M x N partial C in registers, so a lane
// needs no data of any other lane and each FMA operand is a register.  A wave
// covers 64 consecutive rows per load instruction; U rows per lane are in
// flight per tile and the next tile is loaded while the current one is
// multiplied (leap frogging).  After the K loop the lanes' partials are summed
// by a fixed butterfly (wave_sum) and the waves of a block one after the
// other.
//
// MX x NX bound the register tile; MC / NC = 0 takes M, N at run time
// (entries beyond them are zero).  VA / VB load pairs of doubles with one
// 16-byte load (needs even widths, even leading dimensions and 16-byte
// aligned pointers; real data only).
// ============================================================================
template <int MC, int NC, int MX, int NX, int U, bool CPLX, bool VA, bool VB, int WPB>
__global__ void __launch_bounds__(WPB * kWave)
tsmttsm_valu(int64_t K, int Mr, int Nr, const void* __restrict__ Av, int64_t lda,
             const void* __restrict__ Bv, int64_t ldb, double* __restrict__ C, int64_t ldc,
             double* __restrict__ ws, int conj)
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

    struct Frag {
        T a[U][MX];
        T b[U][NX];
    };
    Frag x, y;
    auto load = [&](int64_t t, Frag& f) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = t * RT + (int64_t)(wave * U + u) * kWave + lane;
            const bool ok = row < K;
            const int64_t rc = ok ? row : K - 1;
            const T* ar = A + rc * lda;
            const T* br = B + rc * ldb;
            if constexpr (VA) {
#pragma unroll
                for (int i = 0; i < MX; i += 2) {
                    const dbl2 v = ld_stream2(ar + i);
                    f.a[u][i] = keep(ok, v.x);
                    f.a[u][i + 1] = keep(ok, v.y);
                }
            } else {
#pragma unroll
                for (int i = 0; i < MX; ++i) {
                    const bool in = MC || i < M;
                    f.a[u][i] = keep(ok & in, ld_stream(ar + (in ? i : 0)));
                }
            }
            if constexpr (VB) {
#pragma unroll
                for (int j = 0; j < NX; j += 2) {
                    const dbl2 v = ld_stream2(br + j);
                    f.b[u][j] = keep(ok, v.x);
                    f.b[u][j + 1] = keep(ok, v.y);
                }
            } else {
#pragma unroll
                for (int j = 0; j < NX; ++j) {
                    const bool in = NC || j < N;
                    f.b[u][j] = keep(ok & in, ld_stream(br + (in ? j : 0)));
                }
            }
        }
    };
    auto compute = [&](int64_t, Frag& f) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < MX; ++i)
#pragma unroll
                for (int j = 0; j < NX; ++j) {
                    if constexpr (!CPLX) {
                        acc[i][j] = __builtin_fma(f.a[u][i], f.b[u][j], acc[i][j]);
                    } else {
                        const double ai = conj ? -f.a[u][i].im : f.a[u][i].im;
                        acc[i][j].re = __builtin_fma(f.a[u][i].re, f.b[u][j].re, acc[i][j].re);
                        acc[i][j].re = __builtin_fma(-ai, f.b[u][j].im, acc[i][j].re);
                        acc[i][j].im = __builtin_fma(f.a[u][i].re, f.b[u][j].im, acc[i][j].im);
                        acc[i][j].im = __builtin_fma(ai, f.b[u][j].re, acc[i][j].im);
                    }
                }
    };
    const int64_t ntiles = (K + RT - 1) / RT;
    leapfrog(blockIdx.x, ntiles, gridDim.x, x, y, load, compute);

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
    block_out<CW>(part, E, N, ws, C, ldc);
}

// ============================================================================
// TSMTTSM for M = N = 1, real: the dot product of two contiguous vectors
// (lda = ldb = 1, 16-byte aligned).  A lane reads pairs of consecutive rows as
// one 16-byte load, so every wave load is one 1 KB run of A or B (the
// per-row kernels above read 512 bytes per wave load); U pairs per lane and
// matrix in each of the two register sets of the leap frog, two chains of
// fused multiply-adds per lane.  A pair that reaches past row K - 1 is read
// as its first element only (the clamped address keeps it inside the
// matrix) and zero.
// ============================================================================
template <int U, int WPB>
__global__ void __launch_bounds__(WPB * kWave)
tsmttsm_dot(int64_t K, int Mr, int Nr, const void* __restrict__ Av, int64_t lda,
            const void* __restrict__ Bv, int64_t ldb, double* __restrict__ C, int64_t ldc,
            double* __restrict__ ws, int conj)
{
    constexpr int RT = 2 * kWave * U * WPB;  // rows per tile
    __shared__ double part[WPB];
    const double* __restrict__ A = static_cast<const double*>(Av);
    const double* __restrict__ B = static_cast<const double*>(Bv);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;

    auto load2 = [&](const double* __restrict__ p, int64_t e) -> dbl2 {
        if (e + 1 < K) return ld_stream2(p + e);
        const int64_t c = e < K ? e : K - 1;
        dbl2 v;
        v.x = keep(e < K, ld_stream(p + c));
        v.y = 0.0;
        return v;
    };
    struct Frag {
        dbl2 a[U];
        dbl2 b[U];
    };
    Frag x, y;
    double acc0 = 0.0, acc1 = 0.0;
    auto load = [&](int64_t t, Frag& f) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = t * RT + 2 * ((int64_t)(wave * U + u) * kWave + lane);
            f.a[u] = load2(A, e);
            f.b[u] = load2(B, e);
        }
    };
    auto compute = [&](int64_t, Frag& f) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            acc0 = __builtin_fma(f.a[u].x, f.b[u].x, acc0);
            acc1 = __builtin_fma(f.a[u].y, f.b[u].y, acc1);
        }
    };
    const int64_t ntiles = (K + RT - 1) / RT;
    leapfrog(blockIdx.x, ntiles, gridDim.x, x, y, load, compute);

    // wave sums (fixed butterfly), then the waves' sums in wave order
    const double v = wave_sum(acc0 + acc1);
    if (lane == 0) part[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = part[0];
        for (int w = 1; w < WPB; ++w) sum += part[w];
        part[0] = sum;
    }
    __syncthreads();
    block_out<1>(part, 1, 1, ws, C, ldc);
}

// ============================================================================
// TSMM on the vector ALUs for narrow widths.
//
// Parallelisation over K only (the paper's Fig. "tsmm_mapping_1T" mapping):
// a lane computes whole rows of B.  All lanes of a wave use the same entry of
// C at the same time, so C is read through the scalar unit into SGPRs and
// broadcast to the FMAs: no LDS traffic and no per-lane copy of C.  The rows
// of a wave are consecutive, so the wave's stores fill whole cache lines in
// L2 before they are written back (no write-allocate traffic on CDNA).
// Full tiles store without guards; only the last, ragged tile is guarded.
// ============================================================================
template <int MC, int NC, int MX, int NX, int U, bool CPLX, bool VA, bool VB, int WPB>
__global__ void __launch_bounds__(WPB * kWave)
tsmm_valu(int64_t K, int Mr, int Nr, const void* __restrict__ Av, int64_t lda,
          const double* __restrict__ Cm, int64_t ldc, void* __restrict__ Bv, int64_t ldb,
          double alpha, double beta, int conj, int opc)
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

    struct Frag {
        T a[U][MX];
    };
    Frag x, y;
    auto load = [&](int64_t t, Frag& f) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = t * RT + (int64_t)(wave * U + u) * kWave + lane;
            const int64_t rc = row < K ? row : K - 1;
            const T* ar = A + rc * lda;
            if constexpr (VA) {
#pragma unroll
                for (int i = 0; i < MX; i += 2) {
                    const dbl2 v = ld_stream2(ar + i);
                    f.a[u][i] = v.x;
                    f.a[u][i + 1] = v.y;
                }
            } else {
#pragma unroll
                for (int i = 0; i < MX; ++i) {
                    const bool in = MC || i < M;
                    f.a[u][i] = keep(in, ld_stream(ar + (in ? i : 0)));
                }
            }
        }
    };
    auto row_out = [&](const T (&a)[MX], T (&out)[NX]) {
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            T s = zero_of<T>();
#pragma unroll
            for (int i = 0; i < MX; ++i) {
                if ((MC || i < M) && (NC || j < N)) {
                    T c = Cz[small_index(i, j, ldc, opc)];
                    if constexpr (CPLX) c.im = opc == 2 ? -c.im : c.im;
                    if constexpr (!CPLX) {
                        s = __builtin_fma(a[i], c, s);
                    } else {
                        const double ai = conj ? -a[i].im : a[i].im;
                        s.re = __builtin_fma(a[i].re, c.re, s.re);
                        s.re = __builtin_fma(-ai, c.im, s.re);
                        s.im = __builtin_fma(a[i].re, c.im, s.im);
                        s.im = __builtin_fma(ai, c.re, s.im);
                    }
                }
            }
            out[j] = s;
        }
    };
    auto store_row = [&](T* br, const T (&out)[NX]) {
        if constexpr (VB) {
#pragma unroll
            for (int j = 0; j < NX; j += 2) {
                dbl2 v = dbl2{alpha * out[j], alpha * out[j + 1]};
                if (read_b) {
                    const dbl2 o = *reinterpret_cast<const dbl2*>(br + j);
                    v = dbl2{__builtin_fma(beta, o.x, v.x), __builtin_fma(beta, o.y, v.y)};
                }
                __builtin_nontemporal_store(v, reinterpret_cast<dbl2*>(br + j));
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
                        dbl2 v = dbl2{alpha * out[j].re, alpha * out[j].im};
                        if (read_b) {
                            const zd o = br[j];
                            v = dbl2{__builtin_fma(beta, o.re, v.x), __builtin_fma(beta, o.im, v.y)};
                        }
                        __builtin_nontemporal_store(v, reinterpret_cast<dbl2*>(br + j));
                    }
                }
            }
        }
    };
    auto compute = [&](int64_t t, Frag& f) {
        const bool full = (t + 1) * RT <= K;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = t * RT + (int64_t)(wave * U + u) * kWave + lane;
            T out[NX];
            row_out(f.a[u], out);
            if (full || row < K) store_row(B + row * ldb, out);
        }
    };
    const int64_t ntiles = (K + RT - 1) / RT;
    leapfrog(blockIdx.x, ntiles, gridDim.x, x, y, load, compute);
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
template <int MC, int NC, int MS, int NB, int U, bool CPLX, int WPB, int NBUF, bool VA = false, int OCC = 1,
          bool F32 = false, bool G3 = false, int FL = 0, bool RB = false, bool CG = false>
__global__ void __launch_bounds__(WPB * kWave, OCC)
tsmm_mfma(int64_t K, int Mr, int Nr, const void* __restrict__ Av, int64_t lda,
          const double* __restrict__ Cm, int64_t ldc, void* __restrict__ Bv, int64_t ldb,
          double alpha, double beta, int conj, int opc)
{
    // VA: A is read with 16-byte loads, A(row, 8t + 2q .. 8t + 2q + 1) for the
    // lane of k-slot q, which serve the steps s = 2t (even column) and 2t + 1
    // (odd column); the contraction order over m is permuted accordingly,
    // m(s, q) = 8 (s / 2) + 2 q + s % 2, and C is staged in the same order.
    // G3 (complex): Gauss's three-product form, P1 = Ar Cr, P2 = Ai Ci,
    // P3 = (Ar + Ai)(Cr + Ci), Br = P1 - P2, Bi = P3 - P1 - P2; Cr + Ci is
    // staged beside Cr and Ci.
    // FL (real data with contiguous rows, lda == M): the 16 U rows of a wave
    // are one run of 16 U M elements, read as consecutive loads of FL
    // elements per lane (binary64: 8 or 16 bytes; binary32: 4, 8 or 16
    // bytes; M a multiple of FL, A 16-byte aligned), so every load
    // instruction of the wave covers one contiguous piece whatever M is.
    // The wave writes the run to its own LDS region and reads the
    // matrix-core operands A(row, 4s + l/16) back from there; only the wave
    // itself touches the region, and one wave's LDS accesses complete in
    // order, so no barrier is needed.
    static_assert(!VA || (!CPLX && !F32 && MS % 2 == 0), "paired A loads: binary64 real data, M a multiple of 8");
    static_assert(CPLX || !G3, "the three-product form is for complex data");
    static_assert(FL == 0 || (!CPLX && !VA && (MC > 0 ? MC % FL == 0 : FL == 1)),
                  "slab reads: real data, M a multiple of FL (run-time widths: single-element loads)");
    using T = elem_t<CPLX>;
    using S = typename storage<CPLX, F32>::type;  // storage type of A and B
    constexpr int CW = CPLX ? 2 : 1;
    constexpr int RT = 16 * U * WPB;
    constexpr int NFRAG = MS * NB * kWave;
    // slab reads with a run-time M (FL = 1): the region holds the widest run
    // the slices cover, 16 U rows of 4 MS elements; a tile's run is 16 U M
    constexpr int MCAP = MC ? MC : 4 * MS;
    constexpr int SLAB = FL ? 16 * U * MCAP : 0;             // elements of A per wave and tile
    constexpr int NL = FL ? (SLAB + kWave * FL - 1) / (kWave * FL) : 1;
    using SR = typename real_of<S>::type;                         // real storage type (slab reads)
    using SV = typename slab_vec<SR, FL ? FL : 1>::type;          // one slab load of a lane
    __shared__ double cf[CG ? 1 : NFRAG * (G3 ? 3 : CW)];
    __shared__ __attribute__((aligned(16))) SR slab[FL ? WPB * SLAB : 1];

    const S* __restrict__ A = static_cast<const S*>(Av);
    S* __restrict__ B = static_cast<S*>(Bv);
    const int M = MC ? MC : Mr;
    const int N = NC ? NC : Nr;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int lr = lane >> 4;
    const int lc = lane & 15;
    const bool read_b = beta != 0.0;

    // Stage C in fragment order: cf[(s * NB + j) * 64 + l] = C(m(s, l/16), 16j + l%16).
    // CG (an ablation of the C source): no copy; every tile reads the lane's C
    // operands from global memory through the caches instead.
    for (int idx = threadIdx.x; idx < (CG ? 0 : NFRAG); idx += blockDim.x) {
        const int l = idx & (kWave - 1);
        const int sj = idx / kWave;
        const int s = sj / NB, j = sj - (sj / NB) * NB;
        const int m = VA ? 8 * (s >> 1) + 2 * (l >> 4) + (s & 1) : 4 * s + (l >> 4);
        const int n = 16 * j + (l & 15);
        const bool ok = m < M && n < N;
        if constexpr (CPLX) {
            const int64_t ci = small_index(m, n, ldc, opc);
            const double re = ok ? Cm[2 * ci] : 0.0;
            const double im = ok ? (opc == 2 ? -Cm[2 * ci + 1] : Cm[2 * ci + 1]) : 0.0;
            cf[idx] = re;
            cf[NFRAG + idx] = im;
            if constexpr (G3) cf[2 * NFRAG + idx] = re + im;
        } else {
            cf[idx] = ok ? Cm[small_index(m, n, ldc, opc)] : 0.0;
        }
    }
    __syncthreads();

    // C operand `part` (0: real part, 1: imaginary, 2: their sum) of slice s
    // and column block j for this lane
    auto cfrag = [&](int part, int s, int j) -> double {
        if constexpr (!CG) {
            return cf[part * NFRAG + (s * NB + j) * kWave + lane];
        } else {
            const int m = VA ? 8 * (s >> 1) + 2 * lr + (s & 1) : 4 * s + lr;
            const int n = 16 * j + lc;
            if (m >= M || n >= N) return 0.0;
            const int64_t ci = small_index(m, n, ldc, opc);
            if constexpr (!CPLX) {
                return Cm[ci];
            } else {
                const double re = Cm[2 * ci];
                const double im = opc == 2 ? -Cm[2 * ci + 1] : Cm[2 * ci + 1];
                return part == 0 ? re : (part == 1 ? im : re + im);
            }
        }
    };

    int koff[MS];
    bool kok[MS];
#pragma unroll
    for (int s = 0; s < MS; ++s) {
        const int m = VA ? 8 * (s >> 1) + 2 * lr : 4 * s + lr;  // VA: first column of the pair
        const int mlast = VA ? 8 * (s >> 1) + 7 : 4 * s + 3;     // largest column any lane reads at s
        kok[s] = (MC && mlast < MC) || m < M;                     // constant true where MC covers it
        koff[s] = kok[s] ? m : 0;
    }

    // RB (calls with beta != 0): the old values of the tile's B are loaded with
    // its A, in the same register ring, so a store never waits for its own
    // read (the run-time beta path reads them one by one before each store).
    using ARegs = typename std::conditional<FL != 0, slab_regs<SV, NL>, row_regs<T, U, MS>>::type;
    struct Frag : ARegs {
        T ob[RB ? U : 1][RB ? NB : 1][4];
    };
    Frag fr[NBUF];
    const int64_t KM = K * (int64_t)M;  // slab reads: elements of A
    SR* const mine = slab + (FL ? wave * SLAB : 0);
    auto load = [&](int64_t t, Frag& f) {
        if constexpr (RB) {
            // old B at the positions this lane stores (clamped into B; values
            // of rows past K or columns past N are never used)
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t row = t * RT + (int64_t)(wave * U + u) * 16 + lr + 4 * r;
                        const int n = 16 * j + lc;
                        const int64_t rc = row < K ? row : K - 1;
                        const int nc = n < N ? n : N - 1;
                        f.ob[u][j][r] = ld_stream(B + rc * ldb + nc);
                    }
        }
        if constexpr (FL && MC > 0) {
            // the wave's run starts at row t RT + 16 U wave; positions past
            // the end of A are clamped to its last FL elements (K M is a
            // multiple of FL), their rows are never stored
            const int64_t base = (t * RT + (int64_t)wave * U * 16) * MC;
            slab_load<FL, NL>(reinterpret_cast<const SR*>(A), base, KM, lane, f.v);
            return;
        } else if constexpr (FL) {
            // run-time M: only the loads inside the run of 16 U M elements
            // are issued (single elements, clamped to the last element of A)
            const int64_t base = (t * RT + (int64_t)wave * U * 16) * M;
            slab_load_n<NL>(reinterpret_cast<const SR*>(A), base, KM, lane, 16 * U * M, f.v);
            return;
        } else {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = t * RT + (int64_t)(wave * U + u) * 16 + lc;
            const int64_t rc = row < K ? row : K - 1;
            const S* ar = A + rc * lda;
            if constexpr (VA) {
#pragma unroll
                for (int s = 0; s < MS; s += 2) {
                    const dbl2 v = ld_stream2(reinterpret_cast<const double*>(ar) + koff[s]);
                    f.a[u][s] = keep(kok[s], v.x);
                    f.a[u][s + 1] = keep(kok[s], v.y);
                }
            } else {
#pragma unroll
                for (int s = 0; s < MS; ++s) f.a[u][s] = keep(kok[s], ld_stream(ar + koff[s]));
            }
        }
        }
    };
    auto compute = [&](int64_t t, Frag& f) {
        // Compiler-only barrier: keeps the loop-invariant C operands in LDS
        // instead of letting them be hoisted into (too many) registers.
        __asm__ volatile("" ::: "memory");
        T av[U][MS];  // matrix-core A operands of the tile
        if constexpr (FL) {
            if constexpr (MC > 0)
                slab_put<FL, NL, SLAB>(mine, lane, f.v);
            else
                slab_put_n<NL>(mine, lane, 16 * U * M, f.v);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int s = 0; s < MS; ++s)
                    av[u][s] = keep(kok[s], (double)mine[(u * 16 + lc) * M + koff[s]]);
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int s = 0; s < MS; ++s) av[u][s] = f.a[u][s];
        }
        dbl4 acc[U][NB];
        dbl4 acci[CPLX ? U : 1][CPLX ? NB : 1];
        dbl4 accs[G3 ? U : 1][G3 ? NB : 1];  // G3: P1 in acc, P2 in acci, P3 in accs
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                acc[u][j] = dbl4{0.0, 0.0, 0.0, 0.0};
                if constexpr (CPLX) acci[u][j] = dbl4{0.0, 0.0, 0.0, 0.0};
                if constexpr (G3) accs[u][j] = dbl4{0.0, 0.0, 0.0, 0.0};
            }
#pragma unroll
        for (int s = 0; s < MS; ++s) {
            if constexpr (!CPLX) {
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const double cr = cfrag(0, s, j);
#pragma unroll
                    for (int u = 0; u < U; ++u) acc[u][j] = mfma16(av[u][s], cr, acc[u][j]);
                }
            } else if constexpr (G3) {
                double ai[U], sa[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    ai[u] = conj ? -av[u][s].im : av[u][s].im;
                    sa[u] = av[u][s].re + ai[u];
                }
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const double cr = cfrag(0, s, j);
#pragma unroll
                    for (int u = 0; u < U; ++u) acc[u][j] = mfma16(av[u][s].re, cr, acc[u][j]);
                }
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const double ci = cfrag(1, s, j);
#pragma unroll
                    for (int u = 0; u < U; ++u) acci[u][j] = mfma16(ai[u], ci, acci[u][j]);
                }
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const double cs = cfrag(2, s, j);
#pragma unroll
                    for (int u = 0; u < U; ++u) accs[u][j] = mfma16(sa[u], cs, accs[u][j]);
                }
            } else {
                // products with Re(a) for every block first, then those with
                // Im(a), so that dependent updates of one accumulator are apart
                double cr[NB], ci[NB];
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    cr[j] = cfrag(0, s, j);
                    ci[j] = cfrag(1, s, j);
                }
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        acc[u][j] = mfma16(av[u][s].re, cr[j], acc[u][j]);
                        acci[u][j] = mfma16(av[u][s].re, ci[j], acci[u][j]);
                    }
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const double ai = conj ? -av[u][s].im : av[u][s].im;
                        acc[u][j] = mfma16(ai, -ci[j], acc[u][j]);
                        acci[u][j] = mfma16(ai, cr[j], acci[u][j]);
                    }
            }
        }
        if constexpr (G3) {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const dbl4 p1 = acc[u][j], p2 = acci[u][j];
                    acc[u][j] = p1 - p2;
                    acci[u][j] = accs[u][j] - p1 - p2;
                }
        }
        const bool full = (t + 1) * RT <= K;
        // streaming stores where rows are whole lines or whole lines hold whole
        // rows; with several n-blocks per row, one store covers 16 elements of
        // each of four rows, which must be whole lines too (binary32: 64 bytes,
        // half a line, and the halves were written to memory separately: 26%
        // extra write traffic at 64 x 64), else the cache merges them
        constexpr bool kStream = stream_rows(NC * (int)sizeof(S)) && (NB == 1 || 16 * sizeof(S) >= 128);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t rbase = t * RT + (int64_t)(wave * U + u) * 16 + lr;
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int n = 16 * j + lc;
                if ((NC && (NC % 16 == 0)) || n < N) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t row = rbase + 4 * r;
                        if (full || row < K) {
                            S* p = B + row * ldb + n;
                            if constexpr (!CPLX) {
                                double v = alpha * acc[u][j][r];
                                if constexpr (RB)
                                    v = __builtin_fma(beta, f.ob[u][j][r], v);
                                else if (read_b)
                                    v = __builtin_fma(beta, ld_plain(p), v);
                                st_out<kStream>(p, v);
                            } else {
                                zd v = zd{alpha * acc[u][j][r], alpha * acci[u][j][r]};
                                if (RB || read_b) {
                                    zd o;
                                    if constexpr (RB)
                                        o = f.ob[u][j][r];
                                    else
                                        o = ld_plain(p);
                                    v = zd{__builtin_fma(beta, o.re, v.re), __builtin_fma(beta, o.im, v.im)};
                                }
                                st_out<kStream>(p, v);
                            }
                        }
                    }
                }
            }
        }
    };
    const int64_t ntiles = (K + RT - 1) / RT;
    pipeline<NBUF>(blockIdx.x, ntiles, (int64_t)gridDim.x, fr, load, compute);
}

// ============================================================================
// TSMM on the matrix cores for narrow widths (N <= 16): row packing.
//
// P = 16 / N rows of B are packed into the 16 columns of one output fragment:
// output column j = h N + n (h < P) of fragment row i is B(k0 + i P + h, n),
// so with ldb = N a lane's four outputs and the wave's 16 x 16 fragment are
// 512 contiguous bytes of B.  The contraction index runs over the pairs
// q = h M + m (h < P, m < M) in steps of four; the C operand of pair q and
// column j is C(m, n) when both belong to the same packed row h and zero
// otherwise (a block-diagonal copy of C, staged once per block in LDS in
// fragment order).  A lane's A operand for pair q is A(k0 + i P + h, m).
// ============================================================================
template <int MC, int NC, int U, bool CPLX, int WPB, int NBUF, bool F32 = false>
__global__ void __launch_bounds__(WPB * kWave)
tsmm_packed(int64_t K, int Mr, int Nr, const void* __restrict__ Av, int64_t lda,
            const double* __restrict__ Cm, int64_t ldc, void* __restrict__ Bv, int64_t ldb,
            double alpha, double beta, int conj, int opc)
{
    static_assert(MC > 0 && NC > 0 && NC <= 16, "row-packed TSMM needs compile-time widths, N <= 16");
    using T = elem_t<CPLX>;
    using ST = typename storage<CPLX, F32>::type;  // storage type of A and B
    constexpr int CW = CPLX ? 2 : 1;
    constexpr int P = 16 / NC;
    constexpr int QN = P * MC;             // contraction pairs (h, m)
    constexpr int S = (QN + 3) / 4;        // MFMA steps per fragment
    constexpr int RS = 16 * P;             // rows per fragment
    constexpr int RT = RS * U * WPB;       // rows per tile
    constexpr int NFRAG = S * kWave;
    __shared__ double cf[NFRAG * CW];

    const ST* __restrict__ A = static_cast<const ST*>(Av);
    ST* __restrict__ B = static_cast<ST*>(Bv);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int lr = lane >> 4;
    const int lc = lane & 15;
    const bool read_b = beta != 0.0;

    // C operand fragments: cf[s * 64 + l] = Cop(4s + l/16, l%16).
    for (int idx = threadIdx.x; idx < NFRAG; idx += blockDim.x) {
        const int l = idx & (kWave - 1);
        const int qq = 4 * (idx / kWave) + (l >> 4);
        const int j = l & 15;
        const int hq = qq / MC, m = qq - hq * MC;
        const int hj = j / NC, n = j - hj * NC;
        const bool ok = qq < QN && hj < P && hq == hj;
        if constexpr (CPLX) {
            const int64_t ci = small_index(m, n, ldc, opc);
            cf[idx] = ok ? Cm[2 * ci] : 0.0;
            cf[NFRAG + idx] = ok ? (opc == 2 ? -Cm[2 * ci + 1] : Cm[2 * ci + 1]) : 0.0;
        } else {
            cf[idx] = ok ? Cm[small_index(m, n, ldc, opc)] : 0.0;
        }
    }
    __syncthreads();

    // A operand of step s for this lane: row offset i P + h, column m.
    int aoff[S];
    bool aok[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int qq = 4 * s + lr;
        const int hq = qq / MC, m = qq - hq * MC;
        aok[s] = qq < QN;
        aoff[s] = aok[s] ? hq : 0;  // packed row h
        (void)m;
    }
    int acol[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int qq = 4 * s + lr;
        acol[s] = aok[s] ? qq - (qq / MC) * MC : 0;
    }
    const int hj = lc / NC, nj = lc - hj * NC;
    const bool jok = hj < P;

    struct Frag {
        T a[U][S];
    };
    Frag fr[NBUF];
    auto load = [&](int64_t t, Frag& f) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t r0 = t * RT + (int64_t)(wave * U + u) * RS + (int64_t)lc * P;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int64_t row = r0 + aoff[s];
                const bool ok = aok[s] & (row < K);
                f.a[u][s] = keep(ok, ld_stream(A + (ok ? row : K - 1) * lda + acol[s]));
            }
        }
    };
    auto compute = [&](int64_t t, Frag& f) {
        __asm__ volatile("" ::: "memory");
        dbl4 acc[U], acci[CPLX ? U : 1];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            acc[u] = dbl4{0.0, 0.0, 0.0, 0.0};
            if constexpr (CPLX) acci[u] = dbl4{0.0, 0.0, 0.0, 0.0};
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const double cr = cf[s * kWave + lane];
            if constexpr (!CPLX) {
#pragma unroll
                for (int u = 0; u < U; ++u) acc[u] = mfma16(f.a[u][s], cr, acc[u]);
            } else {
                const double ci = cf[NFRAG + s * kWave + lane];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const double ar = f.a[u][s].re;
                    const double ai = conj ? -f.a[u][s].im : f.a[u][s].im;
                    acc[u] = mfma16(ar, cr, acc[u]);
                    acc[u] = mfma16(ai, -ci, acc[u]);
                    acci[u] = mfma16(ar, ci, acci[u]);
                    acci[u] = mfma16(ai, cr, acci[u]);
                }
            }
        }
        const bool full = (t + 1) * (int64_t)RT <= K;
        constexpr bool kStream = stream_rows(NC * (int)sizeof(ST));  // whole lines per row (see st_plain)
        if (jok) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t r0 = t * RT + (int64_t)(wave * U + u) * RS + hj;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = r0 + (int64_t)(lr + 4 * r) * P;
                    if (full || row < K) {
                        ST* p = B + row * ldb + nj;
                        if constexpr (!CPLX) {
                            double v = alpha * acc[u][r];
                            if (read_b) v = __builtin_fma(beta, ld_plain(p), v);
                            st_out<kStream>(p, v);
                        } else {
                            zd v = zd{alpha * acc[u][r], alpha * acci[u][r]};
                            if (read_b) {
                                const zd o = ld_plain(p);
                                v = zd{__builtin_fma(beta, o.re, v.re), __builtin_fma(beta, o.im, v.im)};
                            }
                            st_out<kStream>(p, v);
                        }
                    }
                }
            }
        }
    };
    const int64_t ntiles = (K + RT - 1) / RT;
    pipeline<NBUF>(blockIdx.x, ntiles, (int64_t)gridDim.x, fr, load, compute);
}

// ============================================================================
// Binary32 arithmetic (precision form with binary32 accumulation).
//
// A and B are stored in binary32 and the products are formed and summed by
// v_mfma_f32_16x16x4f32 in binary32, at twice the matrix-core rate of the
// binary64 products on gfx950.  Sums in binary32 run over short stretches
// only: every RUN tiles (32 rows) the binary32 accumulators are added into
// binary64 accumulators and cleared, so each binary32 sum holds at most 32
// products, and every later addition (over the stretches, the waves, the
// blocks) is binary64.  Error per entry: at most about (32 + 2) 2^-24 times
// sum_k |a_k b_k|, against (K - 1) 2^-24 for one binary32 sum over all K
// rows.  The output layout of the binary32 16x16x4 product differs from the
// binary64 one: lane l, element r holds D(4 (l / 16) + r, l % 16) (checked
// with an in-bounds probe on gfx950).
// ============================================================================

__device__ __forceinline__ flt4 mfma16f(float a, float b, flt4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ dbl4 widen_add(dbl4 acc, flt4 v)
{
    return dbl4{acc[0] + (double)v[0], acc[1] + (double)v[1], acc[2] + (double)v[2], acc[3] + (double)v[3]};
}
template <bool CPLX>
using elem32_t = typename std::conditional<CPLX, zf, float>::type;
__device__ __forceinline__ float lds_elem32(const float* p, int idx, float) { return p[idx]; }
__device__ __forceinline__ zf lds_elem32(const float* p, int idx, zf) { return zf{p[2 * idx], p[2 * idx + 1]}; }

// TSMTTSM in binary32 arithmetic: the blocked mapping of tsmttsm_mfma (MB x NB
// blocks of 16 x 16 per wave, MW waves sharing a row group's rows, U groups of
// four rows per tile, NBUF register sets in flight, optional slab reads FL),
// with binary32 products and the binary64 flush every RUN tiles (4 U RUN = 32
// rows per binary32 sum).  Complex data use four real products per block,
// or with G3 Gauss's three: P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi)
// summed in binary32 over the stretch, then Cr += P1 - P2 and
// Ci += P3 - P1 - P2 formed in binary64 at the flush (so the binary64 sums
// stay two per block).
template <int MC, int NC, int MB, int NB, int MW, int U, bool CPLX, int WPB, int NBUF, int OCC = 1, int FL = 0,
          bool G3 = false>
__global__ void __launch_bounds__(WPB * kWave, OCC)
tsmttsm_a32(int64_t K, int Mr, int Nr, const void* __restrict__ Av, int64_t lda,
            const void* __restrict__ Bv, int64_t ldb, double* __restrict__ C, int64_t ldc,
            double* __restrict__ ws, int conj)
{
    using T = elem32_t<CPLX>;
    using S = T;  // storage = operand type
    constexpr int CW = CPLX ? 2 : 1;
    constexpr int RG = WPB / MW;
    constexpr int RT = 4 * U * RG;
    constexpr int RUN = 8 / U;  // tiles per binary32 stretch: 4 U RUN = 32 rows
    constexpr int EMAX = (MC ? MC : MW * MB * 16) * (NC ? NC : NB * 16) * CW;
    static_assert(WPB % MW == 0 && 8 % U == 0, "waves split evenly; U divides 8");
    static_assert(CPLX || !G3, "the three-product form is for complex data");
    static_assert(FL == 0 || (MW == 1 && MC > 0 && NC > 0 && (MC * CW) % FL == 0 && (NC * CW) % FL == 0),
                  "slab reads: compile-time widths whose rows are multiples of FL, one wave per row group");
    __shared__ double part[EMAX];

    const S* __restrict__ A = static_cast<const S*>(Av);
    const S* __restrict__ B = static_cast<const S*>(Bv);
    const int M = MC ? MC : Mr;
    const int N = NC ? NC : Nr;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int mw = wave % MW;
    const int rg = wave / MW;
    const int lr = lane >> 4;
    const int lc = lane & 15;

    // column offsets as in tsmttsm_mfma: lanes past the width read column 0
    // of the same row; their products reach only entries that are not stored
    int moff[MB], noff[NB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int m = (mw * MB + i) * 16 + lc;
        const bool ok = (MC && ((MW - 1) * MB + i + 1) * 16 <= MC) || m < M;
        moff[i] = ok ? m : 0;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int n = j * 16 + lc;
        const bool ok = (NC && (j + 1) * 16 <= NC) || n < N;
        noff[j] = ok ? n : 0;
    }

    dbl4 acc[MB][NB];                     // binary64 sums of the stretches
    dbl4 acci[CPLX ? MB : 1][CPLX ? NB : 1];
    flt4 s32[MB][NB];                     // binary32 sums of the current stretch (G3: P1)
    flt4 s32i[CPLX ? MB : 1][CPLX ? NB : 1];  // (G3: P2)
    flt4 s32s[G3 ? MB : 1][G3 ? NB : 1];      // G3: P3
    const flt4 fz = flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
            s32[i][j] = fz;
            if constexpr (CPLX) {
                acci[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
                s32i[i][j] = fz;
            }
            if constexpr (G3) s32s[i][j] = fz;
        }
    auto flush = [&]() {
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                if constexpr (G3) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double p1 = (double)s32[i][j][r], p2 = (double)s32i[i][j][r];
                        acc[i][j][r] += p1 - p2;
                        acci[i][j][r] += (double)s32s[i][j][r] - p1 - p2;
                    }
                    s32[i][j] = fz;
                    s32i[i][j] = fz;
                    s32s[i][j] = fz;
                } else {
                    acc[i][j] = widen_add(acc[i][j], s32[i][j]);
                    s32[i][j] = fz;
                    if constexpr (CPLX) {
                        acci[i][j] = widen_add(acci[i][j], s32i[i][j]);
                        s32i[i][j] = fz;
                    }
                }
            }
    };

    constexpr int SLA = FL ? 4 * U * MC * CW : 0, SLB = FL ? 4 * U * NC * CW : 0;  // real elements
    constexpr int NLA = FL ? (SLA + kWave * FL - 1) / (kWave * FL) : 1;
    constexpr int NLB = FL ? (SLB + kWave * FL - 1) / (kWave * FL) : 1;
    using SV = typename slab_vec<float, FL ? FL : 1>::type;
    __shared__ __attribute__((aligned(16))) float slab[FL ? WPB * (SLA + SLB) : 1];
    float* const mya = slab + (FL ? wave * (SLA + SLB) : 0);
    float* const myb = mya + SLA;

    struct RowFrag {
        T a[U][MB];
        T b[U][NB];
    };
    struct SlabFrag {
        SV a[NLA];
        SV b[NLB];
    };
    using Frag = typename std::conditional<FL != 0, SlabFrag, RowFrag>::type;
    Frag fr[NBUF];
    auto load = [&](int64_t t, Frag& f) {
        if constexpr (FL) {
            const int64_t r0 = t * RT + (int64_t)rg * U * 4;
            slab_load<FL, NLA>(reinterpret_cast<const float*>(A), r0 * MC * CW, K * (int64_t)(MC * CW), lane, f.a);
            slab_load<FL, NLB>(reinterpret_cast<const float*>(B), r0 * NC * CW, K * (int64_t)(NC * CW), lane, f.b);
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t row = t * RT + (int64_t)(rg * U + u) * 4 + lr;
                const bool ok = row < K;
                const int64_t rc = ok ? row : K - 1;
#pragma unroll
                for (int i = 0; i < MB; ++i) f.a[u][i] = keep(ok, ld_stream32(A + rc * lda + moff[i]));
#pragma unroll
                for (int j = 0; j < NB; ++j) f.b[u][j] = keep(ok, ld_stream32(B + rc * ldb + noff[j]));
            }
        }
    };
    int stretch = 0;
    auto compute = [&](int64_t t, Frag& f) {
        T av[U][MB], bv[U][NB];
        if constexpr (FL) {
            slab_put<FL, NLA, SLA>(mya, lane, f.a);
            slab_put<FL, NLB, SLB>(myb, lane, f.b);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool ok = t * RT + (int64_t)(rg * U + u) * 4 + lr < K;
#pragma unroll
                for (int i = 0; i < MB; ++i) av[u][i] = keep(ok, lds_elem32(mya, (4 * u + lr) * MC + moff[i], T{}));
#pragma unroll
                for (int j = 0; j < NB; ++j) bv[u][j] = keep(ok, lds_elem32(myb, (4 * u + lr) * NC + noff[j], T{}));
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int i = 0; i < MB; ++i) av[u][i] = f.a[u][i];
#pragma unroll
                for (int j = 0; j < NB; ++j) bv[u][j] = f.b[u][j];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (!CPLX) {
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j) s32[i][j] = mfma16f(av[u][i], bv[u][j], s32[i][j]);
            } else if constexpr (G3) {
                float ai[MB], sa[MB];
#pragma unroll
                for (int i = 0; i < MB; ++i) {
                    ai[i] = conj ? -av[u][i].im : av[u][i].im;
                    sa[i] = av[u][i].re + ai[i];
                }
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j) s32[i][j] = mfma16f(av[u][i].re, bv[u][j].re, s32[i][j]);
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j) s32i[i][j] = mfma16f(ai[i], bv[u][j].im, s32i[i][j]);
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const float sb = bv[u][j].re + bv[u][j].im;
#pragma unroll
                    for (int i = 0; i < MB; ++i) s32s[i][j] = mfma16f(sa[i], sb, s32s[i][j]);
                }
            } else {
                // Re(a) products of every block first, then Im(a): dependent
                // updates of one accumulator are 2 MB NB instructions apart
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        s32[i][j] = mfma16f(av[u][i].re, bv[u][j].re, s32[i][j]);
                        s32i[i][j] = mfma16f(av[u][i].re, bv[u][j].im, s32i[i][j]);
                    }
#pragma unroll
                for (int i = 0; i < MB; ++i) {
                    const float ai = conj ? -av[u][i].im : av[u][i].im;
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        s32[i][j] = mfma16f(ai, -bv[u][j].im, s32[i][j]);
                        s32i[i][j] = mfma16f(ai, bv[u][j].re, s32i[i][j]);
                    }
                }
            }
        }
        if (++stretch == RUN) {
            flush();
            stretch = 0;
        }
    };
    const int64_t ntiles = (K + RT - 1) / RT;
    pipeline<NBUF>(blockIdx.x, ntiles, (int64_t)gridDim.x, fr, load, compute);
    flush();

    // row groups folded into the block partial one after the other
    const int E = M * N * CW;
    for (int g = 0; g < RG; ++g) {
        if (rg == g) {
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int m = (mw * MB + i) * 16 + 4 * lr + r;
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
    block_out<CW>(part, E, N, ws, C, ldc);
}

// TSMTTSM in binary32 arithmetic with the rows staged in LDS (the scheme of
// tsmttsm_lds for binary32 storage): stages of RT rows brought by direct
// 16-byte loads, WM x WN waves of MB x NB blocks, binary32 products summed by
// the matrix cores over stretches of 32 rows and added into binary64 sums
// (complex: four products per block, or with G3 Gauss's three, combined in
// binary64 at each flush as in tsmttsm_a32).  Rows of A and B must hold a
// multiple of four binary32 values (whole 16-byte loads; lane addresses past
// the end are clamped to the last 16 bytes, which then hold only values of
// rows past K, zeroed when read).
template <int MC, int NC, int MB, int NB, int WM, int WN, int RT, bool CPLX, bool G3 = false, int OCC = 1,
          int IL = 0>
__global__ void __launch_bounds__(WM * WN * kWave, OCC)
tsmttsm_lds_a32(int64_t K, int Mr, int Nr, const void* __restrict__ Av, int64_t lda,
                const void* __restrict__ Bv, int64_t ldb, double* __restrict__ C, int64_t ldc,
                double* __restrict__ ws, int conj)
{
    using T = elem32_t<CPLX>;
    constexpr int CW = CPLX ? 2 : 1;
    constexpr int WPB = WM * WN;
    constexpr int KS = RT / 4;                                   // 4-row steps of a stage
    constexpr int FLUSH = 32 / RT;                               // stages per binary32 stretch
    static_assert(MC > 0 && NC > 0 && (RT == 16 || RT == 32), "compile-time widths; stages of 16 or 32 rows");
    static_assert(WM * MB * 16 >= MC && WN * NB * 16 >= NC, "the waves' blocks cover C");
    static_assert(CPLX || !G3, "the three-product form is for complex data");
    static_assert((MC * CW) % 4 == 0 && (NC * CW) % 4 == 0, "rows of whole 16-byte loads");
    constexpr int SA = ((RT * MC * CW + 255) / 256) * 256;       // floats of A per stage (whole 1 KB loads)
    constexpr int SB = ((RT * NC * CW + 255) / 256) * 256;
    constexpr int SS = SA + SB;                                   // one stage
    constexpr int E = MC * NC * CW;                               // doubles of the partial
    constexpr int NLA = SA / 256, NLB = SB / 256;                 // wave loads per stage
    __shared__ __attribute__((aligned(16))) float lds[2 * SS];   // two stages

    const float* __restrict__ A = static_cast<const float*>(Av);
    const float* __restrict__ B = static_cast<const float*>(Bv);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int wm = wave % WM, wn = wave / WM;
    const int lr = lane >> 4;
    const int lc = lane & 15;
    const int64_t totA = K * (int64_t)(MC * CW), totB = K * (int64_t)(NC * CW);   // floats
    const int64_t lastA = totA - 4, lastB = totB - 4;

    auto stage = [&](int64_t t, int b) {
        float* dst = lds + b * SS;
        const int64_t ea = t * (int64_t)(RT * MC * CW), eb = t * (int64_t)(RT * NC * CW);
#pragma unroll
        for (int i = wave; i < NLA + NLB; i += WPB) {
            if (i < NLA) {
                const int64_t e = ea + (int64_t)i * 256 + 4 * lane;
                __builtin_amdgcn_global_load_lds(A + (e <= lastA ? e : lastA), dst + i * 256, 16, 0, 0);
            } else {
                const int64_t e = eb + (int64_t)(i - NLA) * 256 + 4 * lane;
                __builtin_amdgcn_global_load_lds(B + (e <= lastB ? e : lastB), dst + SA + (i - NLA) * 256, 16, 0, 0);
            }
        }
    };

    int moff[MB], noff[NB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int m = (wm * MB + i) * 16 + lc;
        moff[i] = m < MC ? m : 0;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int n = (wn * NB + j) * 16 + lc;
        noff[j] = n < NC ? n : 0;
    }

    dbl4 acc[MB][NB];
    dbl4 acci[CPLX ? MB : 1][CPLX ? NB : 1];
    flt4 s32[MB][NB];                          // binary32 stretch sums (G3: P1)
    flt4 s32i[CPLX ? MB : 1][CPLX ? NB : 1];   // (G3: P2)
    flt4 s32s[G3 ? MB : 1][G3 ? NB : 1];       // G3: P3
    const flt4 fz = flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
            s32[i][j] = fz;
            if constexpr (CPLX) {
                acci[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
                s32i[i][j] = fz;
            }
            if constexpr (G3) s32s[i][j] = fz;
        }
    auto flush = [&]() {
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                if constexpr (G3) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double p1 = (double)s32[i][j][r], p2 = (double)s32i[i][j][r];
                        acc[i][j][r] += p1 - p2;
                        acci[i][j][r] += (double)s32s[i][j][r] - p1 - p2;
                    }
                    s32s[i][j] = fz;
                } else {
                    acc[i][j] = widen_add(acc[i][j], s32[i][j]);
                    if constexpr (CPLX) acci[i][j] = widen_add(acci[i][j], s32i[i][j]);
                }
                s32[i][j] = fz;
                if constexpr (CPLX) s32i[i][j] = fz;
            }
    };

    const int64_t ntiles = (K + RT - 1) / RT;
    const int64_t G = gridDim.x;
    int64_t t = blockIdx.x;
    int stretch = 0;
    if (t < ntiles) stage(t, 0);
    for (int b = 0; t < ntiles; t += G, b ^= 1) {
        __syncthreads();
        const float* sa = lds + b * SS;
        const float* sb = sa + SA;
        T av[KS][MB], bv[KS][NB];
        auto operands = [&](int s) {
            const bool ok = t * RT + 4 * s + lr < K;
            const int r = 4 * s + lr;
#pragma unroll
            for (int i = 0; i < MB; ++i) av[s][i] = keep(ok, lds_elem32(sa, r * MC + moff[i], T{}));
#pragma unroll
            for (int j = 0; j < NB; ++j) bv[s][j] = keep(ok, lds_elem32(sb, r * NC + noff[j], T{}));
        };
#pragma unroll
        for (int s = 0; s < (IL ? (IL < KS ? IL : KS) : KS); ++s) operands(s);
        if (t + G < ntiles) stage(t + G, b ^ 1);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if constexpr (IL > 0) {
                __builtin_amdgcn_sched_barrier(0);
                if (s + IL < KS) operands(s + IL);
            }
            if constexpr (!CPLX) {
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j) s32[i][j] = mfma16f(av[s][i], bv[s][j], s32[i][j]);
            } else if constexpr (G3) {
                float ai[MB], sum[MB];
#pragma unroll
                for (int i = 0; i < MB; ++i) {
                    ai[i] = conj ? -av[s][i].im : av[s][i].im;
                    sum[i] = av[s][i].re + ai[i];
                }
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j) s32[i][j] = mfma16f(av[s][i].re, bv[s][j].re, s32[i][j]);
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j) s32i[i][j] = mfma16f(ai[i], bv[s][j].im, s32i[i][j]);
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const float sbj = bv[s][j].re + bv[s][j].im;
#pragma unroll
                    for (int i = 0; i < MB; ++i) s32s[i][j] = mfma16f(sum[i], sbj, s32s[i][j]);
                }
            } else {
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        s32[i][j] = mfma16f(av[s][i].re, bv[s][j].re, s32[i][j]);
                        s32i[i][j] = mfma16f(av[s][i].re, bv[s][j].im, s32i[i][j]);
                    }
#pragma unroll
                for (int i = 0; i < MB; ++i) {
                    const float ai = conj ? -av[s][i].im : av[s][i].im;
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        s32[i][j] = mfma16f(ai, -bv[s][j].im, s32[i][j]);
                        s32i[i][j] = mfma16f(ai, bv[s][j].re, s32i[i][j]);
                    }
                }
            }
        }
        if (++stretch == FLUSH) {
            flush();
            stretch = 0;
        }
    }
    flush();
    // binary32 matrix-core output layout: lane l holds rows 4 (l/16) + r
    lds_out<CW, MB, NB>(acc, acci, wm, wn, lr, lc, MC, NC, E, ws, C, ldc, true);
}

// TSMM in binary32 arithmetic: the mapping of tsmm_mfma (sixteen rows per
// product chain, contraction over M in 4-wide slices, C staged once per block
// in LDS in fragment order, U row blocks per tile), with C rounded to binary32
// when it is staged and binary32 products summed by the matrix cores (at most
// 64 products per output).  alpha, beta and the old B are applied in
// binary64 and the result rounded once to binary32 when it is stored.  G3
// (complex): Gauss's three products P1 = Ar Cr, P2 = Ai Ci,
// P3 = (Ar + Ai)(Cr + Ci) summed in binary32, Br = P1 - P2 and
// Bi = P3 - P1 - P2 formed in binary64 (Cr + Ci staged in binary32 beside Cr
// and Ci).
template <int MC, int NC, int MS, int NB, int U, bool CPLX, int WPB, int NBUF, int FL = 0, bool RB = false,
          bool G3 = false>
__global__ void __launch_bounds__(WPB * kWave)
tsmm_a32(int64_t K, int Mr, int Nr, const void* __restrict__ Av, int64_t lda,
         const double* __restrict__ Cm, int64_t ldc, void* __restrict__ Bv, int64_t ldb,
         double alpha, double beta, int conj, int opc)
{
    static_assert(FL == 0 || (!CPLX && MC > 0 && MC % FL == 0), "slab reads: real data, M a multiple of FL");
    static_assert(CPLX || !G3, "the three-product form is for complex data");
    using T = elem32_t<CPLX>;
    using S = T;
    constexpr int CW = CPLX ? 2 : 1;
    constexpr int RT = 16 * U * WPB;
    constexpr int NFRAG = MS * NB * kWave;
    constexpr int SLAB = FL ? 16 * U * MC : 0;
    constexpr int NL = FL ? (SLAB + kWave * FL - 1) / (kWave * FL) : 1;
    using SV = typename slab_vec<float, FL ? FL : 1>::type;
    __shared__ float cf[NFRAG * (G3 ? 3 : CW)];
    __shared__ __attribute__((aligned(16))) float slab[FL ? WPB * SLAB : 1];

    const S* __restrict__ A = static_cast<const S*>(Av);
    S* __restrict__ B = static_cast<S*>(Bv);
    const int M = MC ? MC : Mr;
    const int N = NC ? NC : Nr;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int lr = lane >> 4;
    const int lc = lane & 15;
    const bool read_b = beta != 0.0;

    // C in fragment order: cf[(s NB + j) 64 + l] = C(4 s + l/16, 16 j + l%16), binary32
    for (int idx = threadIdx.x; idx < NFRAG; idx += blockDim.x) {
        const int l = idx & (kWave - 1);
        const int sj = idx / kWave;
        const int s = sj / NB, j = sj - (sj / NB) * NB;
        const int m = 4 * s + (l >> 4);
        const int n = 16 * j + (l & 15);
        const bool ok = m < M && n < N;
        if constexpr (CPLX) {
            const int64_t ci = small_index(m, n, ldc, opc);
            const double re = ok ? Cm[2 * ci] : 0.0;
            const double im = ok ? (opc == 2 ? -Cm[2 * ci + 1] : Cm[2 * ci + 1]) : 0.0;
            cf[idx] = (float)re;
            cf[NFRAG + idx] = (float)im;
            if constexpr (G3) cf[2 * NFRAG + idx] = (float)(re + im);
        } else {
            cf[idx] = ok ? (float)Cm[small_index(m, n, ldc, opc)] : 0.0f;
        }
    }
    __syncthreads();

    int koff[MS];
    bool kok[MS];
#pragma unroll
    for (int s = 0; s < MS; ++s) {
        const int m = 4 * s + lr;
        kok[s] = (MC && 4 * s + 3 < MC) || m < M;
        koff[s] = kok[s] ? m : 0;
    }

    using ARegs = typename std::conditional<FL != 0, slab_regs<SV, NL>, row_regs<T, U, MS>>::type;
    struct Frag : ARegs {
        T ob[RB ? U : 1][RB ? NB : 1][4];
    };
    Frag fr[NBUF];
    const int64_t KM = K * (int64_t)M;
    float* const mine = slab + (FL ? wave * SLAB : 0);
    auto load = [&](int64_t t, Frag& f) {
        if constexpr (RB) {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t row = t * RT + (int64_t)(wave * U + u) * 16 + 4 * lr + r;
                        const int n = 16 * j + lc;
                        const int64_t rc = row < K ? row : K - 1;
                        const int nc = n < N ? n : N - 1;
                        f.ob[u][j][r] = ld_stream32(B + rc * ldb + nc);
                    }
        }
        if constexpr (FL) {
            const int64_t base = (t * RT + (int64_t)wave * U * 16) * MC;
            slab_load<FL, NL>(reinterpret_cast<const float*>(A), base, KM, lane, f.v);
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t row = t * RT + (int64_t)(wave * U + u) * 16 + lc;
                const int64_t rc = row < K ? row : K - 1;
#pragma unroll
                for (int s = 0; s < MS; ++s) f.a[u][s] = keep(kok[s], ld_stream32(A + rc * lda + koff[s]));
            }
        }
    };
    auto compute = [&](int64_t t, Frag& f) {
        __asm__ volatile("" ::: "memory");  // C operands stay in LDS (not hoisted into registers)
        T av[U][MS];
        if constexpr (FL) {
            slab_put<FL, NL, SLAB>(mine, lane, f.v);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int s = 0; s < MS; ++s) av[u][s] = keep(kok[s], mine[(u * 16 + lc) * MC + koff[s]]);
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int s = 0; s < MS; ++s) av[u][s] = f.a[u][s];
        }
        flt4 acc[U][NB];
        flt4 acci[CPLX ? U : 1][CPLX ? NB : 1];
        flt4 accs[G3 ? U : 1][G3 ? NB : 1];  // G3: P1 in acc, P2 in acci, P3 in accs
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                acc[u][j] = flt4{0.f, 0.f, 0.f, 0.f};
                if constexpr (CPLX) acci[u][j] = flt4{0.f, 0.f, 0.f, 0.f};
                if constexpr (G3) accs[u][j] = flt4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
        for (int s = 0; s < MS; ++s) {
            if constexpr (!CPLX) {
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const float cr = cf[(s * NB + j) * kWave + lane];
#pragma unroll
                    for (int u = 0; u < U; ++u) acc[u][j] = mfma16f(av[u][s], cr, acc[u][j]);
                }
            } else if constexpr (G3) {
                float ai[U], sa[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    ai[u] = conj ? -av[u][s].im : av[u][s].im;
                    sa[u] = av[u][s].re + ai[u];
                }
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const float cr = cf[(s * NB + j) * kWave + lane];
#pragma unroll
                    for (int u = 0; u < U; ++u) acc[u][j] = mfma16f(av[u][s].re, cr, acc[u][j]);
                }
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const float ci = cf[NFRAG + (s * NB + j) * kWave + lane];
#pragma unroll
                    for (int u = 0; u < U; ++u) acci[u][j] = mfma16f(ai[u], ci, acci[u][j]);
                }
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const float cs = cf[2 * NFRAG + (s * NB + j) * kWave + lane];
#pragma unroll
                    for (int u = 0; u < U; ++u) accs[u][j] = mfma16f(sa[u], cs, accs[u][j]);
                }
            } else {
                float cr[NB], ci[NB];
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    cr[j] = cf[(s * NB + j) * kWave + lane];
                    ci[j] = cf[NFRAG + (s * NB + j) * kWave + lane];
                }
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        acc[u][j] = mfma16f(av[u][s].re, cr[j], acc[u][j]);
                        acci[u][j] = mfma16f(av[u][s].re, ci[j], acci[u][j]);
                    }
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const float ai = conj ? -av[u][s].im : av[u][s].im;
                        acc[u][j] = mfma16f(ai, -ci[j], acc[u][j]);
                        acci[u][j] = mfma16f(ai, cr[j], acci[u][j]);
                    }
            }
        }
        const bool full = (t + 1) * RT <= K;
        // a lane stores four consecutive rows of one column; sixteen lanes
        // cover 16 columns (64 bytes real, 128 complex) of each row
        constexpr bool kStream = stream_rows(NC * (int)sizeof(S)) && (NB == 1 || 16 * sizeof(S) >= 128);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t rbase = t * RT + (int64_t)(wave * U + u) * 16 + 4 * lr;
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int n = 16 * j + lc;
                if ((NC && (NC % 16 == 0)) || n < N) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t row = rbase + r;
                        if (full || row < K) {
                            S* p = B + row * ldb + n;
                            if constexpr (!CPLX) {
                                double v = alpha * (double)acc[u][j][r];
                                if constexpr (RB)
                                    v = __builtin_fma(beta, (double)f.ob[u][j][r], v);
                                else if (read_b)
                                    v = __builtin_fma(beta, ld_plain(p), v);
                                st_out<kStream>(p, v);
                            } else {
                                double br = (double)acc[u][j][r], bi = (double)acci[u][j][r];
                                if constexpr (G3) {
                                    const double p1 = br, p2 = bi;
                                    br = p1 - p2;
                                    bi = (double)accs[u][j][r] - p1 - p2;
                                }
                                zd v = zd{alpha * br, alpha * bi};
                                if (RB || read_b) {
                                    zd o;
                                    if constexpr (RB)
                                        o = zd{(double)f.ob[u][j][r].re, (double)f.ob[u][j][r].im};
                                    else
                                        o = ld_plain(p);
                                    v = zd{__builtin_fma(beta, o.re, v.re), __builtin_fma(beta, o.im, v.im)};
                                }
                                st_out<kStream>(p, v);
                            }
                        }
                    }
                }
            }
        }
    };
    const int64_t ntiles = (K + RT - 1) / RT;
    pipeline<NBUF>(blockIdx.x, ntiles, (int64_t)gridDim.x, fr, load, compute);
}

}  // namespace tsg
