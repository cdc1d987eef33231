// tsg_device.hpp -- device-side building blocks shared by the gfx950 kernels:
// element types, complex multiply-accumulate, wave reductions and the
// deterministic two-level grid reduction of the per-block partial C.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsg {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kGroup = 16;         // blocks folded by one first-level reducer

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Interleaved complex double (16 B).
struct zd {
    double re, im;
};

// ---------------------------------------------------------------- loads
// Plain loads through the vector memory path; the streaming operands are read
// exactly once, so they are marked non-temporal.
__device__ __forceinline__ double ld_stream(const double* p) { return __builtin_nontemporal_load(p); }

__device__ __forceinline__ zd ld_stream(const zd* p)
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2 v = __builtin_nontemporal_load(reinterpret_cast<const d2*>(p));
    return zd{v.x, v.y};
}

// -------------------------------------------------- wave reduction (fixed tree)
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// ------------------------------------------------- grid reduction of partials
// Every block holds its partial C (E doubles) in LDS.  Blocks write it to the
// workspace, the last block of each group of kGroup blocks folds its group in
// block order, and the last group folder folds the group sums in group order
// and writes C.  Each fold runs in a fixed order, so the result is
// bitwise reproducible.  Counters return to zero after use, so no memset is
// needed between launches.
//
// ws layout (doubles): level-1 partials [G][E], then level-2 partials [NG][E].
// cnt layout: NG first-level counters, then one second-level counter.
//
// `store(e, v)` writes the final value of partial entry e to C.
template <class Store>
__device__ void grid_fold(const double* lds_part, int E, double* __restrict__ ws,
                          unsigned* __restrict__ cnt, Store store)
{
    __shared__ int s_flag;
    const int G = gridDim.x;
    const int b = blockIdx.x;
    const int NG = (G + kGroup - 1) / kGroup;
    const int grp = b / kGroup;
    const int grp_size = min(kGroup, G - grp * kGroup);
    const int tid = threadIdx.x;
    const int nt = blockDim.x;

    if (G == 1) {
        for (int e = tid; e < E; e += nt) store(e, lds_part[e]);
        return;
    }
    double* l1 = ws;
    double* l2 = ws + (size_t)G * E;
    for (int e = tid; e < E; e += nt) l1[(size_t)b * E + e] = lds_part[e];
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        unsigned t = __hip_atomic_fetch_add(&cnt[grp], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_flag = (t == (unsigned)(grp_size - 1));
    }
    __syncthreads();
    if (!s_flag) return;
    __threadfence();
    if (tid == 0) __hip_atomic_store(&cnt[grp], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    const double* src = l1 + (size_t)grp * kGroup * E;
    if (NG == 1) {
        for (int e = tid; e < E; e += nt) {
            double s = 0.0;
            for (int j = 0; j < grp_size; ++j) s += src[(size_t)j * E + e];
            store(e, s);
        }
        return;
    }
    for (int e = tid; e < E; e += nt) {
        double s = 0.0;
        for (int j = 0; j < grp_size; ++j) s += src[(size_t)j * E + e];
        l2[(size_t)grp * E + e] = s;
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        unsigned t = __hip_atomic_fetch_add(&cnt[NG], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_flag = (t == (unsigned)(NG - 1));
    }
    __syncthreads();
    if (!s_flag) return;
    __threadfence();
    if (tid == 0) __hip_atomic_store(&cnt[NG], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int e = tid; e < E; e += nt) {
        double s = 0.0;
        for (int j = 0; j < NG; ++j) s += l2[(size_t)j * E + e];
        store(e, s);
    }
}

}  // namespace tsg
