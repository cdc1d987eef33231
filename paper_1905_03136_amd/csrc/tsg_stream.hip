// tsg_stream.hip -- memory bandwidth probes that define the achievable
// bandwidth b_s of the roofline (the paper measures b_s the same way: a
// read-only thread-local sum for TSMTTSM and a read + write stream for TSMM,
// Section 1.6 and Table 1).  Both stream 16-byte non-temporal accesses with a
// grid-stride loop over contiguous chunks and kUnroll loads in flight per lane.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tsgemm.h"

namespace {

typedef double d2 __attribute__((ext_vector_type(2)));
constexpr int kThreads = 256;
constexpr int kUnroll = 8;

// Each block streams contiguous chunks of kThreads * kUnroll 16-byte elements
// (32 KB), chunk c = blockIdx.x + i * gridDim.x; a wave's load instruction
// covers 1 KB of consecutive bytes.  The tail beyond whole chunks is handled
// element by element.
__global__ void __launch_bounds__(kThreads) stream_read(const d2* __restrict__ x, int64_t n, double* __restrict__ sink)
{
    constexpr int64_t CH = (int64_t)kThreads * kUnroll;
    double s = 0.0;
    const int64_t nch = n / CH;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const d2* p = x + c * CH + threadIdx.x;
        d2 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = __builtin_nontemporal_load(p + u * kThreads);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) s += v[u].x + v[u].y;
    }
    for (int64_t i = nch * CH + (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const d2 v = __builtin_nontemporal_load(x + i);
        s += v.x + v.y;
    }
    // keep the loads alive without a reduction: one store per block, value-dependent
    if (s == 1.2345e-300) sink[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) stream_copy(const d2* __restrict__ x, d2* __restrict__ y, int64_t n)
{
    constexpr int64_t CH = (int64_t)kThreads * kUnroll;
    const int64_t nch = n / CH;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const int64_t o = c * CH + threadIdx.x;
        d2 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = __builtin_nontemporal_load(x + o + u * kThreads);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) __builtin_nontemporal_store(v[u], y + o + u * kThreads);
    }
    for (int64_t i = nch * CH + (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        __builtin_nontemporal_store(__builtin_nontemporal_load(x + i), y + i);
}

int grid_of(int blocks_per_cu)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return cus * blocks_per_cu;
}

double* g_sink = nullptr;

}  // namespace

extern "C" tsg_status tsg_stream_read(const void* x, size_t bytes, void* stream)
{
    if (!x || bytes % 16 || reinterpret_cast<uintptr_t>(x) % 16) return TSG_E_ARG;
    const int grid = grid_of(8);
    if (!g_sink && hipMalloc(&g_sink, sizeof(double) * 65536) != hipSuccess) return TSG_E_NOMEM;
    hipLaunchKernelGGL(stream_read, dim3(grid), dim3(kThreads), 0, static_cast<hipStream_t>(stream),
                       static_cast<const d2*>(x), (int64_t)(bytes / 16), g_sink);
    return hipGetLastError() == hipSuccess ? TSG_OK : TSG_E_HIP;
}

extern "C" tsg_status tsg_stream_copy(const void* src, void* dst, size_t bytes, void* stream)
{
    if (!src || !dst || bytes % 16 || reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
        return TSG_E_ARG;
    hipLaunchKernelGGL(stream_copy, dim3(grid_of(8)), dim3(kThreads), 0, static_cast<hipStream_t>(stream),
                       static_cast<const d2*>(src), static_cast<d2*>(dst), (int64_t)(bytes / 16));
    return hipGetLastError() == hipSuccess ? TSG_OK : TSG_E_HIP;
}
