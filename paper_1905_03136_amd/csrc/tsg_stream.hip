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

// ---------------------------------------------- occupancy x loads in flight
// The paper's Table 1 measures the read bandwidth of a thread-local sum for
// a range of occupancies and loads in flight per thread (ILP); the same grid
// here, extended by a write stream: each of the nch chunks of x (256 threads
// x ILP 16-byte loads, issued together) is read, and a chunk of y of its
// share of y's size is written from the loaded values (streaming or cached
// stores), so that read:write ratios of the two products (K M : K N) can be
// probed.  With y empty it is the read-only sum.
template <int ILP, bool NT>
__global__ void __launch_bounds__(kThreads)
stream_mix(const d2* __restrict__ x, int64_t nch, d2* __restrict__ y, int64_t chy, double* __restrict__ sink)
{
    constexpr int64_t CH = (int64_t)kThreads * ILP;
    double s = 0.0;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const d2* p = x + c * CH + threadIdx.x;
        d2 v[ILP];
#pragma unroll
        for (int u = 0; u < ILP; ++u) v[u] = __builtin_nontemporal_load(p + u * kThreads);
        d2 t = {0.0, 0.0};
#pragma unroll
        for (int u = 0; u < ILP; ++u) t += v[u];
        s += t.x + t.y;
        // element i of the chunk of y takes v[(i / kThreads) % ILP]; the
        // register index is a compile-time constant (a run-time index would
        // put v in scratch memory)
        d2* q = y + c * chy;
        for (int64_t i0 = 0; i0 < chy; i0 += CH) {
#pragma unroll
            for (int u = 0; u < ILP; ++u) {
                const int64_t i = i0 + (int64_t)u * kThreads + threadIdx.x;
                if (i < chy) {
                    if constexpr (NT)
                        __builtin_nontemporal_store(v[u], q + i);
                    else
                        q[i] = v[u];
                }
            }
        }
    }
    if (s == 1.2345e-300) sink[blockIdx.x] = s;
}

template <int ILP, bool NT>
void launch_mix(int grid, hipStream_t st, const d2* x, int64_t nch, d2* y, int64_t chy, double* sink)
{
    hipLaunchKernelGGL((stream_mix<ILP, NT>), dim3(grid), dim3(kThreads), 0, st, x, nch, y, chy, sink);
}

// ---------------------------------------------- peak arithmetic rates
// Register-only loops with CH independent accumulator chains per lane, so
// that neither dependences nor memory limit the issue rate; the grid of
// blocks_per_cu blocks of 256 threads per compute unit sets the waves per
// SIMD.  Values stay small and normal (no denormal or overflow slow paths).
constexpr int kChains = 8;
typedef double dbl4p __attribute__((ext_vector_type(4)));
typedef float flt4p __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kThreads) peak_mfma_f64(int64_t iters, double a, double* __restrict__ sink)
{
    dbl4p acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = dbl4p{0.0, 0.0, 0.0, (double)c};
    const double b = a * 0.5 + threadIdx.x * 1e-9;
    for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) t += acc[c][0] + acc[c][3];
    if (t == 1.2345e-300) sink[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kThreads) peak_mfma_f32(int64_t iters, double a, double* __restrict__ sink)
{
    flt4p acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = flt4p{0.f, 0.f, 0.f, (float)c};
    const float af = (float)a, b = (float)(a * 0.5) + threadIdx.x * 1e-6f;
    for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, b, acc[c], 0, 0, 0);
    }
    float t = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) t += acc[c][0] + acc[c][3];
    if (t == 1.2345e-30f) sink[blockIdx.x] = t;
}

constexpr int kValuChains = 24;
__global__ void __launch_bounds__(kThreads) peak_valu_f64(int64_t iters, double a, double* __restrict__ sink)
{
    double acc[kValuChains];
#pragma unroll
    for (int c = 0; c < kValuChains; ++c) acc[c] = c * 1e-3 + threadIdx.x * 1e-9;
    const double b = a * 0.5;
    for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kValuChains; ++c) acc[c] = __builtin_fma(a, b, acc[c]);
    }
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < kValuChains; ++c) t += acc[c];
    if (t == 1.2345e-300) sink[blockIdx.x] = t;
}

// matrix cores and vector FMAs from the same waves: half the chains each
__global__ void __launch_bounds__(kThreads) peak_mixed_f64(int64_t iters, double a, double* __restrict__ sink)
{
    dbl4p acc[kChains / 2];
    double v[kValuChains / 2];
#pragma unroll
    for (int c = 0; c < kChains / 2; ++c) acc[c] = dbl4p{0.0, 0.0, 0.0, (double)c};
#pragma unroll
    for (int c = 0; c < kValuChains / 2; ++c) v[c] = c * 1e-3 + threadIdx.x * 1e-9;
    const double b = a * 0.5;
    for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains / 2; ++c) {
            acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
            v[2 * c] = __builtin_fma(a, b, v[2 * c]);
            v[2 * c + 1] = __builtin_fma(a, b, v[2 * c + 1]);
        }
    }
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < kChains / 2; ++c) t += acc[c][0] + acc[c][3];
#pragma unroll
    for (int c = 0; c < kValuChains / 2; ++c) t += v[c];
    if (t == 1.2345e-300) sink[blockIdx.x] = t;
}

// ---------------------------------------------- memory latency (pointer chase)
// One lane follows a chain of indices, each load waiting for the previous
// one; the elapsed shader clocks (s_memtime) and constant-rate clocks
// (s_memrealtime, 100 MHz) over `steps` loads give the latency of one load at
// the chain's working set (a few MB: caches; GBs: HBM).
__global__ void chase(const int64_t* __restrict__ next, int64_t steps, int64_t* __restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t i = 0;
    // one pass over the first loads (page-table and cache warm-up is excluded)
    for (int64_t k = 0; k < 64; ++k) i = next[i];
    const int64_t c0 = clock64(), w0 = wall_clock64();
    for (int64_t k = 0; k < steps; ++k) i = next[i];
    const int64_t c1 = clock64(), w1 = wall_clock64();
    out[0] = c1 - c0;
    out[1] = w1 - w0;
    out[2] = i;
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

extern "C" tsg_status tsg_stream_probe(const void* x, size_t x_bytes, void* y, size_t y_bytes, int32_t blocks_per_cu,
                                       int32_t loads_in_flight, int32_t stream_stores, size_t* moved, void* stream)
{
    const int ilp = loads_in_flight;
    if (!x || reinterpret_cast<uintptr_t>(x) % 16 || (y_bytes && (!y || reinterpret_cast<uintptr_t>(y) % 16)) ||
        blocks_per_cu < 1 || blocks_per_cu > 32 || !(ilp == 1 || ilp == 2 || ilp == 4 || ilp == 8 || ilp == 16))
        return TSG_E_ARG;
    const int64_t nch = (int64_t)(x_bytes / 16) / ((int64_t)kThreads * ilp);
    if (nch < 1) return TSG_E_ARG;
    const int64_t chy = (int64_t)(y_bytes / 16) / nch;
    if (moved) *moved = (size_t)(nch * kThreads * ilp + nch * chy) * 16;
    if (!g_sink && hipMalloc(&g_sink, sizeof(double) * 65536) != hipSuccess) return TSG_E_NOMEM;
    const int grid = grid_of(blocks_per_cu);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const d2* xs = static_cast<const d2*>(x);
    d2* ys = static_cast<d2*>(y);
    const bool nt = stream_stores != 0;
    switch (ilp * 2 + (nt ? 1 : 0)) {
    case 2: launch_mix<1, false>(grid, st, xs, nch, ys, chy, g_sink); break;
    case 3: launch_mix<1, true>(grid, st, xs, nch, ys, chy, g_sink); break;
    case 4: launch_mix<2, false>(grid, st, xs, nch, ys, chy, g_sink); break;
    case 5: launch_mix<2, true>(grid, st, xs, nch, ys, chy, g_sink); break;
    case 8: launch_mix<4, false>(grid, st, xs, nch, ys, chy, g_sink); break;
    case 9: launch_mix<4, true>(grid, st, xs, nch, ys, chy, g_sink); break;
    case 16: launch_mix<8, false>(grid, st, xs, nch, ys, chy, g_sink); break;
    case 17: launch_mix<8, true>(grid, st, xs, nch, ys, chy, g_sink); break;
    case 32: launch_mix<16, false>(grid, st, xs, nch, ys, chy, g_sink); break;
    default: launch_mix<16, true>(grid, st, xs, nch, ys, chy, g_sink); break;
    }
    return hipGetLastError() == hipSuccess ? TSG_OK : TSG_E_HIP;
}

extern "C" tsg_status tsg_peak_probe(int32_t kind, int32_t blocks_per_cu, int64_t iters, double* flops, void* stream)
{
    if (kind < 0 || kind > 3 || blocks_per_cu < 1 || blocks_per_cu > 32 || iters < 1) return TSG_E_ARG;
    if (!g_sink && hipMalloc(&g_sink, sizeof(double) * 65536) != hipSuccess) return TSG_E_NOMEM;
    const int grid = grid_of(blocks_per_cu);
    hipStream_t st = static_cast<hipStream_t>(stream);
    // flops per wave and iteration: a 16 x 16 x 4 product is 2048 flops
    double per_wave_iter = 0.0;
    switch (kind) {
    case TSG_PEAK_MFMA_F64:
        hipLaunchKernelGGL(peak_mfma_f64, dim3(grid), dim3(kThreads), 0, st, iters, 0.5, g_sink);
        per_wave_iter = 2048.0 * kChains;
        break;
    case TSG_PEAK_VALU_F64:
        hipLaunchKernelGGL(peak_valu_f64, dim3(grid), dim3(kThreads), 0, st, iters, 0.5, g_sink);
        per_wave_iter = 2.0 * 64 * kValuChains;
        break;
    case TSG_PEAK_MFMA_F32:
        hipLaunchKernelGGL(peak_mfma_f32, dim3(grid), dim3(kThreads), 0, st, iters, 0.5, g_sink);
        per_wave_iter = 2048.0 * kChains;
        break;
    default:
        hipLaunchKernelGGL(peak_mixed_f64, dim3(grid), dim3(kThreads), 0, st, iters, 0.5, g_sink);
        per_wave_iter = 2048.0 * (kChains / 2) + 2.0 * 64 * (kValuChains / 2);
        break;
    }
    if (flops) *flops = per_wave_iter * (double)iters * (double)grid * (kThreads / 64);
    return hipGetLastError() == hipSuccess ? TSG_OK : TSG_E_HIP;
}

extern "C" tsg_status tsg_latency_probe(const int64_t* next, int64_t steps, int64_t* out, void* stream)
{
    if (!next || !out || steps < 1) return TSG_E_ARG;
    hipLaunchKernelGGL(chase, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), next, steps, out);
    return hipGetLastError() == hipSuccess ? TSG_OK : TSG_E_HIP;
}
