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

__device__ __forceinline__ double keep(bool ok, double v) { return ok ? v : 0.0; }
__device__ __forceinline__ zd keep(bool ok, zd v) { return ok ? v : zd{0.0, 0.0}; }

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
