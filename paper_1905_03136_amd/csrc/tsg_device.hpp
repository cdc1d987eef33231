// tsg_device.hpp -- device-side building blocks shared by the gfx950 kernels:
// element types, streaming loads, the leap-frog loop driver and wave sums.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsg {

constexpr int kWave = 64;  // CDNA wavefront width

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));

// Interleaved complex double (16 B).
struct zd {
    double re, im;
};

// ---------------------------------------------------------------- loads
// The tall operands are read exactly once: non-temporal loads.  Callers pass
// addresses that are always inside the matrix (out-of-range rows and columns
// are clamped to a valid element and the value is zeroed afterwards), so every
// load is issued unconditionally and the compiler can count the loads in
// flight and wait only for the ones it needs.
__device__ __forceinline__ double ld_stream(const double* p) { return __builtin_nontemporal_load(p); }

__device__ __forceinline__ zd ld_stream(const zd* p)
{
    dbl2 v = __builtin_nontemporal_load(reinterpret_cast<const dbl2*>(p));
    return zd{v.x, v.y};
}

__device__ __forceinline__ dbl2 ld_stream2(const double* p)
{
    return __builtin_nontemporal_load(reinterpret_cast<const dbl2*>(p));
}

// ---------------------------------------------------- binary32 storage
// The precision form stores the tall matrices in binary32 (complex: two
// binary32).  Loads widen to binary64 exactly; a product of two widened
// binary32 numbers has at most 48 significant bits, so it is exact in
// binary64 and the matrix cores accumulate it in binary64.  Stores round the
// binary64 result once to binary32.
struct zf {
    float re, im;
};
typedef float flt2 __attribute__((ext_vector_type(2)));

template <bool CPLX, bool F32>
struct storage;
template <>
struct storage<false, false> { typedef double type; };
template <>
struct storage<true, false> { typedef zd type; };
template <>
struct storage<false, true> { typedef float type; };
template <>
struct storage<true, true> { typedef zf type; };

__device__ __forceinline__ double ld_stream(const float* p) { return (double)__builtin_nontemporal_load(p); }
__device__ __forceinline__ zd ld_stream(const zf* p)
{
    const flt2 v = __builtin_nontemporal_load(reinterpret_cast<const flt2*>(p));
    return zd{(double)v.x, (double)v.y};
}

// Loads that keep binary32 values (the binary32-arithmetic kernels).
__device__ __forceinline__ float ld_stream32(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ zf ld_stream32(const zf* p)
{
    const flt2 v = __builtin_nontemporal_load(reinterpret_cast<const flt2*>(p));
    return zf{v.x, v.y};
}
__device__ __forceinline__ float keep(bool ok, float v) { return ok ? v : 0.0f; }
__device__ __forceinline__ zf keep(bool ok, zf v) { return zf{ok ? v.re : 0.0f, ok ? v.im : 0.0f}; }

// plain (cached) reads, e.g. of the old B when beta != 0
__device__ __forceinline__ double ld_plain(const double* p) { return *p; }
__device__ __forceinline__ double ld_plain(const float* p) { return (double)*p; }
__device__ __forceinline__ zd ld_plain(const zd* p)
{
    const dbl2 v = *reinterpret_cast<const dbl2*>(p);
    return zd{v.x, v.y};
}
__device__ __forceinline__ zd ld_plain(const zf* p)
{
    const flt2 v = *reinterpret_cast<const flt2*>(p);
    return zd{(double)v.x, (double)v.y};
}

// streaming stores of a binary64 result into the storage type
__device__ __forceinline__ void st_stream(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_stream(float* p, double v) { __builtin_nontemporal_store((float)v, p); }
__device__ __forceinline__ void st_stream(zd* p, zd v)
{
    __builtin_nontemporal_store(dbl2{v.re, v.im}, reinterpret_cast<dbl2*>(p));
}
__device__ __forceinline__ void st_stream(zf* p, zd v)
{
    __builtin_nontemporal_store(flt2{(float)v.re, (float)v.im}, reinterpret_cast<flt2*>(p));
}

// Cached stores.  Where the rows of the output are not whole cache lines (for
// example an odd number of binary64 columns), one line is completed by
// several store instructions; cached stores let the L2 merge them before the
// line is written back, while streaming stores can send the pieces to memory
// separately (measured up to 1.6x slower for 33 columns).
__device__ __forceinline__ void st_plain(double* p, double v) { *p = v; }
__device__ __forceinline__ void st_plain(float* p, double v) { *p = (float)v; }
__device__ __forceinline__ void st_plain(zd* p, zd v) { *reinterpret_cast<dbl2*>(p) = dbl2{v.re, v.im}; }
__device__ __forceinline__ void st_plain(zf* p, zd v) { *reinterpret_cast<flt2*>(p) = flt2{(float)v.re, (float)v.im}; }

// Store through the streaming or the cached path (compile-time choice).
template <bool STREAM, class S, class V>
__device__ __forceinline__ void st_out(S* p, V v)
{
    if constexpr (STREAM)
        st_stream(p, v);
    else
        st_plain(p, v);
}

// Streaming stores pay off where a row of the output fills whole 128-byte
// lines or whole lines hold whole rows: row_bytes % 128 == 0 or
// 128 % row_bytes == 0 (a run-time width, 0, stores through the cache).
constexpr bool stream_rows(int row_bytes) { return row_bytes > 0 && (row_bytes % 128 == 0 || 128 % row_bytes == 0); }

// Value or zero.  Component-wise selects, never a conditional on the whole
// struct: that one becomes a branch, the optimiser then sinks the load into
// it, and a conditionally issued load makes the loop wait for all loads in
// flight.
__device__ __forceinline__ double keep(bool ok, double v) { return ok ? v : 0.0; }
__device__ __forceinline__ zd keep(bool ok, zd v) { return zd{ok ? v.re : 0.0, ok ? v.im : 0.0}; }

// ------------------------------------------------------- leap-frog driver
// Grid-stride loop over tiles t = t0, t0 + G, ... < ntiles with two register
// sets used in turn: the loads of the next tile are issued before the current
// tile is computed (the paper's leap frogging, Section 3.1), without copying
// the "next" registers into the "current" ones.
template <class Buf, class Load, class Compute>
__device__ __forceinline__ void leapfrog(int64_t t, int64_t ntiles, int64_t G, Buf& x, Buf& y, Load load,
                                         Compute compute)
{
    if (t >= ntiles) return;
    load(t, x);
    while (true) {
        const int64_t t1 = t + G;
        if (t1 >= ntiles) {
            compute(t, x);
            return;
        }
        load(t1, y);
        compute(t, x);
        const int64_t t2 = t1 + G;
        if (t2 >= ntiles) {
            compute(t1, y);
            return;
        }
        load(t2, x);
        compute(t1, y);
        t = t2;
    }
}

// Deeper leap frogging: NBUF register sets in a ring, loads issued NBUF - 1
// tiles ahead of the multiplication.  Every pass of the (fully unrolled) ring
// issues the same loads, so the compiler waits only for the oldest set; near
// the end of a block's tiles the look-ahead index is clamped to the block's
// last tile (a repeated, cache-resident load instead of a conditional one).
template <int NBUF, class Buf, class Load, class Compute>
__device__ __forceinline__ void leapfrog_ring(int64_t t0, int64_t ntiles, int64_t G, Buf (&buf)[NBUF], Load load,
                                              Compute compute)
{
    static_assert(NBUF >= 2, "a ring needs two register sets at least");
    if (t0 >= ntiles) return;
    const int64_t last = ntiles - 1 - ((ntiles - 1 - t0) % G);
#pragma unroll
    for (int i = 0; i < NBUF - 1; ++i) {
        const int64_t ti = t0 + i * G;
        load(ti <= last ? ti : last, buf[i]);
    }
    int64_t t = t0;
    while (true) {
#pragma unroll
        for (int p = 0; p < NBUF; ++p) {
            const int64_t ta = t + (NBUF - 1) * G;
            load(ta <= last ? ta : last, buf[(p + NBUF - 1) % NBUF]);
            compute(t, buf[p]);
            t += G;
            if (t > last) return;
        }
    }
}

// Dispatch: two sets use the unclamped ping-pong loop, more use the ring.
template <int NBUF, class Buf, class Load, class Compute>
__device__ __forceinline__ void pipeline(int64_t t0, int64_t ntiles, int64_t G, Buf (&buf)[NBUF], Load load,
                                         Compute compute)
{
    if constexpr (NBUF == 2)
        leapfrog(t0, ntiles, G, buf[0], buf[1], load, compute);
    else
        leapfrog_ring<NBUF>(t0, ntiles, G, buf, load, compute);
}

// Cached load, for operands that several waves of a block read.
template <class S>
__device__ __forceinline__ auto ld_shared(const S* p)
{
    return ld_plain(p);
}

// -------------------------------------------------- wave reduction (fixed tree)
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// ------------------------------------------------------- block partial out
// Every block of a TSMTTSM launch ends with its partial C (E doubles) in LDS.
// A grid of one block writes C directly; otherwise the partial goes to slot
// blockIdx.x of the workspace and a second kernel (fold_partials) sums the
// slots in a fixed order.  The kernel boundary orders the two, so no
// device-scope fence or atomic is needed.
template <int CW>
__device__ __forceinline__ void block_out(const double* part, int E, int N, double* __restrict__ ws,
                                          double* __restrict__ C, int64_t ldc)
{
    if (gridDim.x == 1) {
        for (int e = threadIdx.x; e < E; e += blockDim.x) {
            const int q = e / CW;
            const int m = q / N, n = q - m * N;
            C[((int64_t)m * ldc + n) * CW + (e - q * CW)] = part[e];
        }
    } else {
        double* dst = ws + (size_t)blockIdx.x * E;
        for (int e = threadIdx.x; e < E; e += blockDim.x) dst[e] = part[e];
    }
}

}  // namespace tsg
