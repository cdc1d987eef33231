// tsg_runtime.hip -- host side of libtsgemm: argument validation, choice of
// the kernel variant, per-(device, stream) workspace, grid sizing and launch.
// The C ABI is declared in include/tsgemm.h.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/tsgemm.h"
#include "tsg_registry.hpp"

namespace tsg {

// Sum of the G per-block partials of a TSMTTSM launch (slot b holds E doubles
// at ws + b * E) into C, in a fixed order: each block of kFoldThreads threads
// takes EB consecutive entries (EB a power of two <= 8) and S = kFoldThreads /
// EB slices; slice s sums slots s, s + S, s + 2S, ... in increasing order
// (loads issued eight at a time, the additions in slot order), and the slices
// are combined by a fixed pairwise tree.  The result is bitwise reproducible
// for a given grid.  Wide blocks keep the chain of dependent loads of a
// thread short (G <= 2048 slots: at most two batches of eight), which is what
// the fold's time is made of at small K.
constexpr int kFoldThreads = 1024;

template <int CW>
__global__ void __launch_bounds__(kFoldThreads)
fold_partials(const double* __restrict__ ws, int G, int E, int EB, int N, double* __restrict__ C, int64_t ldc)
{
    __shared__ double red[kFoldThreads];
    const int S = kFoldThreads / EB;
    const int el = threadIdx.x & (EB - 1);
    const int s = threadIdx.x / EB;
    const int e = blockIdx.x * EB + el;
    double v = 0.0;
    if (e < E) {
        int b = s;
        for (; b + 7 * S < G; b += 8 * S) {
            double x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = ws[(size_t)(b + u * S) * E + e];
#pragma unroll
            for (int u = 0; u < 8; ++u) v += x[u];
        }
        for (; b < G; b += S) v += ws[(size_t)b * E + e];
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = S / 2; h >= 1; h >>= 1) {
        if (s < h) red[threadIdx.x] += red[threadIdx.x + h * EB];
        __syncthreads();
    }
    if (s == 0 && e < E) {
        const int q = e / CW;
        const int m = q / N, n = q - m * N;
        C[((int64_t)m * ldc + n) * CW + (e - q * CW)] = red[el];
    }
}

// Reduction ablation only (never the default): every block's partial is
// added into C with global FP64 atomics, as the paper's global-atomic variant
// does (Section 3.2); C is cleared first.  Thread (b, e) adds slot b, entry e;
// the order of the additions, and so the rounding, varies from run to run.
template <int CW>
__global__ void __launch_bounds__(256)
atomic_partials(const double* __restrict__ ws, int G, int E, int N, double* __restrict__ C, int64_t ldc)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)G * E) return;
    const int b = (int)(i / E), e = (int)(i - (int64_t)b * E);
    const int q = e / CW;
    const int m = q / N, n = q - m * N;
    atomicAdd(C + ((int64_t)m * ldc + n) * CW + (e - q * CW), ws[(size_t)b * E + e]);
}

__global__ void __launch_bounds__(256) clear_small(double* __restrict__ C, int M, int N, int CW, int64_t ldc)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= M * N * CW) return;
    const int q = i / CW;
    const int m = q / N, n = q - m * N;
    C[((int64_t)m * ldc + n) * CW + (i - q * CW)] = 0.0;
}

// Fixed scratch of tsg_tsmttsm_noalloc: the per-block partial sums of one
// launch (a slot of M N (x2 complex) doubles per block).  Every device the
// library runs on holds its own copy for the life of the process.  In host
// code the array's name is only a stand-in; kernels and copies take the
// device address obtained once per device with hipGetSymbolAddress.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

}  // namespace tsg

namespace {

thread_local std::string g_err;
thread_local std::string g_force;  // variant forced by tsg_force_variant ("" = automatic choice)
thread_local int g_grid_cap = 0;   // block cap set by tsg_set_grid_limit (0 = none)
thread_local int g_reduction = 0;  // cross-block reduction set by tsg_set_reduction (0 = fixed-order fold)

tsg_status fail(tsg_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

constexpr int kMaxWidth = 64;

}  // namespace

namespace tsg {
size_t orth_workspace_size(int64_t K, int32_t M, int32_t N, int32_t count);  // tsg_batched.hip

// Error detail for tsg_last_error() from the library's other units.
tsg_status report(tsg_status s, const char* msg)
{
    g_err = msg;
    return s;
}
}  // namespace tsg

namespace {

struct DeviceInfo {
    int cus = 0;
    bool ok = false;
};

struct Workspace {
    void* data = nullptr;
    size_t bytes = 0;
};

std::mutex g_mu;
std::map<int, DeviceInfo> g_dev;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;
// Outgrown workspaces, kept until tsg_finalize: a graph captured earlier on
// the stream may still hold one of them and write its partial sums there.
std::vector<std::pair<int, void*>> g_retired;
std::map<std::pair<int, const tsg::Variant*>, int> g_occ;  // (device, variant) -> blocks per CU

std::map<int, double*> g_scratch;  // device -> device address of its no-alloc scratch

int is_complex(tsg_dtype dt) { return dt == TSG_C128 || dt == TSG_C64 || dt == TSG_C64_ACC32; }
size_t elem_bytes(tsg_dtype dt)
{
    switch (dt) {
    case TSG_R64: return 8;
    case TSG_C128: return 16;
    case TSG_R32: return 4;
    case TSG_C64: return 8;
    case TSG_R32_ACC32: return 4;
    case TSG_C64_ACC32: return 8;
    }
    return 0;
}
// Binary64-arithmetic type whose kernels also serve a binary32-arithmetic
// type (they are at least as accurate); -1 for the other types.
int twin_of(tsg_dtype dt)
{
    return dt == TSG_R32_ACC32 ? (int)TSG_R32 : dt == TSG_C64_ACC32 ? (int)TSG_C64 : -1;
}

tsg_status device_info(int dev, DeviceInfo* out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_dev.find(dev);
    if (it != g_dev.end() && it->second.ok) {
        *out = it->second;
        return TSG_OK;
    }
    DeviceInfo d;
    hipError_t e = hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return fail(TSG_E_HIP, "hipDeviceGetAttribute: %s", hipGetErrorString(e));
    d.ok = true;
    g_dev[dev] = d;
    *out = d;
    return TSG_OK;
}

tsg_status current_device(int* dev)
{
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return fail(TSG_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    return TSG_OK;
}

int occupancy(int dev, const tsg::Variant& v)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(dev, &v);
    auto it = g_occ.find(key);
    if (it != g_occ.end()) return it->second;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, v.kernel(), v.threads, 0) != hipSuccess || blocks < 1)
        blocks = 1;
    g_occ[key] = blocks;
    return blocks;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Device address of `dev`'s scratch array; `dev` must be the current device.
// Resolved on the first use per device (tsg_init or the first no-alloc call).
tsg_status scratch_of(int dev, double** out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
        *out = it->second;
        return TSG_OK;
    }
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(tsg::scratch));
    if (e != hipSuccess || !p)
        return fail(TSG_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch[dev] = static_cast<double*>(p);
    *out = static_cast<double*>(p);
    return TSG_OK;
}

// Choose the variant: the exact (op, dtype, M, N) one if its access
// requirements hold, else the first run-time-width variant covering (M, N).
const tsg::Variant* pick_for(int op, int dt, int M, int N, const void* A, int64_t lda, const void* X,
                             int64_t ldx, bool beta_nz);

// The variant of (op, dt): for a binary32-arithmetic type, its own exact-width
// variant if there is one, else what its binary64-arithmetic twin would run.
const tsg::Variant* pick(int op, tsg_dtype dt, int M, int N, const void* A, int64_t lda, const void* X,
                         int64_t ldx, bool beta_nz = false)
{
    const tsg::Variant* v = pick_for(op, (int)dt, M, N, A, lda, X, ldx, beta_nz);
    const int twin = twin_of(dt);
    if (twin >= 0 && (!v || v->M == 0)) {
        const tsg::Variant* w = pick_for(op, twin, M, N, A, lda, X, ldx, beta_nz);
        if (w) return w;
    }
    return v;
}

const tsg::Variant* pick_for(int op, int dt, int M, int N, const void* A, int64_t lda, const void* X,
                             int64_t ldx, bool beta_nz)
{
    const bool a_pairs = (lda % 2 == 0) && aligned(A, 16);
    const bool x_pairs = (ldx % 2 == 0) && aligned(X, 16);
    // slab reads: the rows of A (TSMTTSM: and of B) are one contiguous run
    const bool rows_contiguous = lda == M && (op != tsg::OP_TSMTTSM || ldx == N);
    const bool ax16 = aligned(A, 16) && aligned(X, 16);
    const tsg::Variant* best = nullptr;
    if (!g_force.empty()) {
        for (int i = 0; i < tsg::kNumVariants; ++i) {
            const tsg::Variant& v = tsg::kVariants[i];
            if (g_force != v.name) continue;
            const bool serves = (v.M == M && v.N == N) || (v.M == 0 && M <= v.maxM && N <= v.maxN);
            if (v.op == op && v.dt == dt && serves && (!v.pairA || a_pairs) && (!v.pairX || x_pairs) &&
                (!v.flatA || rows_contiguous) && (!v.readB || beta_nz) && (!v.align16 || ax16))
                return &v;
        }
        return nullptr;
    }
    for (int i = 0; i < tsg::kNumVariants; ++i) {
        const tsg::Variant& v = tsg::kVariants[i];
        if (v.op != op || v.dt != dt) continue;
        if (v.pairA && !a_pairs) continue;
        if (v.pairX && !x_pairs) continue;
        if (v.flatA && !rows_contiguous) continue;
        if (v.readB && !beta_nz) continue;
        if (v.align16 && !ax16) continue;
        if (v.M == M && v.N == N) return &v;
        if (v.M == 0 && !best && M <= v.maxM && N <= v.maxN && (!v.evenW || (M % 2 == 0 && N % 2 == 0)))
            best = &v;
    }
    return best;
}

tsg_status get_workspace(int dev, hipStream_t stream, size_t bytes, Workspace** out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    const char* lim = getenv("TSG_MAX_WORKSPACE");
    if (lim && bytes > (size_t)strtoull(lim, nullptr, 10))
        return fail(TSG_E_NOMEM, "workspace of %zu bytes exceeds TSG_MAX_WORKSPACE=%s", bytes, lim);
    Workspace& w = g_ws[std::make_pair(dev, stream)];
    if (w.data && w.bytes >= bytes) {
        *out = &w;
        return TSG_OK;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return fail(TSG_E_CAPTURE, "workspace must grow to %zu bytes while the stream is captured; "
                                   "run the call once before capture or use tsg_reserve", bytes);
    hipError_t e;
    // the outgrown buffer is retired, not freed (see g_retired)
    const size_t grow = bytes < (1u << 20) ? (1u << 20) : bytes;
    void* fresh = nullptr;
    e = hipMalloc(&fresh, grow);
    if (e != hipSuccess) return fail(TSG_E_NOMEM, "hipMalloc(%zu): %s", grow, hipGetErrorString(e));
    if (w.data) g_retired.emplace_back(dev, w.data);
    w.data = fresh;
    w.bytes = grow;
    *out = &w;
    return TSG_OK;
}

tsg_status validate(tsg_dtype dt, int64_t K, int32_t M, int32_t N, const void* A, int64_t lda, const void* X,
                    int64_t ldx, const void* Y, int64_t ldy, int op)
{
    if (elem_bytes(dt) == 0) return fail(TSG_E_ARG, "unknown dtype %d", (int)dt);
    if (K < 0) return fail(TSG_E_ARG, "K = %lld < 0", (long long)K);
    if (M < 1 || N < 1) return fail(TSG_E_ARG, "M = %d, N = %d: widths must be >= 1", M, N);
    if (M > kMaxWidth || N > kMaxWidth)
        return fail(TSG_E_UNSUPPORTED, "M = %d, N = %d: widths above %d are not supported", M, N, kMaxWidth);
    const size_t es = elem_bytes(dt);
    if (op == tsg::OP_TSMTTSM) {
        // A (K x M), X = B (K x N), Y = C (M x N)
        if (lda < M) return fail(TSG_E_ARG, "lda = %lld < M = %d", (long long)lda, M);
        if (ldx < N) return fail(TSG_E_ARG, "ldb = %lld < N = %d", (long long)ldx, N);
        if (ldy < N) return fail(TSG_E_ARG, "ldc = %lld < N = %d", (long long)ldy, N);
        if (!Y) return fail(TSG_E_ARG, "C is NULL");
        if (K > 0 && (!A || !X)) return fail(TSG_E_ARG, "A or B is NULL");
        if ((A && !aligned(A, es)) || (X && !aligned(X, es)))
            return fail(TSG_E_ARG, "A and B must be aligned to %zu bytes", es);
        if (!aligned(Y, is_complex(dt) ? 16 : 8)) return fail(TSG_E_ARG, "C must be aligned to its element size");
    } else {
        // A (K x M), X = C (M x N), Y = B (K x N)
        if (lda < M) return fail(TSG_E_ARG, "lda = %lld < M = %d", (long long)lda, M);
        if (ldx < N) return fail(TSG_E_ARG, "ldc = %lld < N = %d", (long long)ldx, N);
        if (ldy < N) return fail(TSG_E_ARG, "ldb = %lld < N = %d", (long long)ldy, N);
        if (K > 0 && (!A || !X || !Y)) return fail(TSG_E_ARG, "A, B or C is NULL");
        if ((A && !aligned(A, es)) || (Y && !aligned(Y, es)))
            return fail(TSG_E_ARG, "A and B must be aligned to %zu bytes", es);
        if (X && !aligned(X, is_complex(dt) ? 16 : 8)) return fail(TSG_E_ARG, "C must be aligned to its element size");
    }
    return TSG_OK;
}

int grid_for(int dev, const tsg::Variant& v, int64_t K, int M, int N, int cus)
{
    int64_t rows = v.rows_per_tile;
    if (v.pack == 1) rows *= 16 / (M > N ? M : N);
    if (v.pack == 2) rows *= 16 / N;
    const int64_t tiles = (K + rows - 1) / rows;
    const int64_t cap = (int64_t)cus * occupancy(dev, v);
    int64_t g = tiles < cap ? tiles : cap;
    if (v.op == tsg::OP_TSMTTSM) {
        // the per-block partial sums of a launch always fit the no-alloc
        // scratch, so both TSMTTSM entry points run the same grid (and give
        // the same bits) for every shape
        const int64_t E = (int64_t)M * N * (is_complex((tsg_dtype)v.dt) ? 2 : 1);
        const int64_t gmax = (int64_t)(tsg::kScratchBytes / (E * sizeof(double)));
        if (g > gmax) g = gmax;
    }
    if (g_grid_cap > 0 && g > g_grid_cap) g = g_grid_cap;
    return g < 1 ? 1 : (int)g;
}

size_t tsmttsm_ws_bytes(int grid, int M, int N, bool cplx)
{
    const size_t E = (size_t)M * N * (cplx ? 2 : 1);
    return grid > 1 ? (size_t)grid * E * sizeof(double) : 0;
}

// Launch the fold of the per-block partials (grid > 1) into C.
hipError_t launch_fold(const tsg::Launch& p, bool cplx)
{
    const int E = p.M * p.N * (cplx ? 2 : 1);
    int eb = 1;
    while (eb < E && eb < 8) eb <<= 1;
    const int blocks = (E + eb - 1) / eb;
    if (cplx)
        hipLaunchKernelGGL((tsg::fold_partials<2>), dim3(blocks), dim3(tsg::kFoldThreads), 0, p.stream, p.ws, p.grid,
                           E, eb, p.N, static_cast<double*>(p.Y), p.ldy);
    else
        hipLaunchKernelGGL((tsg::fold_partials<1>), dim3(blocks), dim3(tsg::kFoldThreads), 0, p.stream, p.ws, p.grid,
                           E, eb, p.N, static_cast<double*>(p.Y), p.ldy);
    return hipGetLastError();
}

// TSMTTSM launch shared by tsg_tsmttsm (per-stream workspace, allocated on
// first need) and tsg_tsmttsm_noalloc (the device's fixed scratch array).
tsg_status tsmttsm_call(tsg_dtype dt, tsg_op op, int64_t K, int32_t M, int32_t N, const void* A, int64_t lda,
                        const void* B, int64_t ldb, void* C, int64_t ldc, void* stream, bool noalloc)
{
    g_err.clear();
    if (op != TSG_OP_T && op != TSG_OP_C) return fail(TSG_E_ARG, "unknown op %d", (int)op);
    tsg_status s = validate(dt, K, M, N, A, lda, B, ldb, C, ldc, tsg::OP_TSMTTSM);
    if (s != TSG_OK) return s;
    int dev;
    if ((s = current_device(&dev)) != TSG_OK) return s;
    DeviceInfo di;
    if ((s = device_info(dev, &di)) != TSG_OK) return s;
    const tsg::Variant* v = pick(tsg::OP_TSMTTSM, dt, M, N, A, lda, B, ldb);
    if (!v) return fail(TSG_E_UNSUPPORTED, "no kernel variant for TSMTTSM %dx%d%s", M, N,
                        g_force.empty() ? "" : " (a forced variant does not apply)");
    tsg::Launch p{};
    p.stream = static_cast<hipStream_t>(stream);
    p.grid = grid_for(dev, *v, K, M, N, di.cus);
    p.K = K;
    p.M = M;
    p.N = N;
    p.conj = (op == TSG_OP_C && is_complex(dt)) ? 1 : 0;
    p.A = A;
    p.lda = lda;
    p.X = B;
    p.ldx = ldb;
    p.Y = C;
    p.ldy = ldc;
    const size_t need = tsmttsm_ws_bytes(p.grid, M, N, is_complex(dt));
    if (noalloc) {
        if (need > tsg::kScratchBytes)
            return fail(TSG_E_UNSUPPORTED, "TSMTTSM %dx%d on %d blocks needs %zu bytes of partial sums, more than "
                        "the %zu bytes of the no-alloc scratch", M, N, p.grid, need, tsg::kScratchBytes);
        if ((s = scratch_of(dev, &p.ws)) != TSG_OK) return s;
    } else {
        Workspace* w = nullptr;
        if ((s = get_workspace(dev, p.stream, need, &w)) != TSG_OK) return s;
        p.ws = static_cast<double*>(w->data);
    }
    v->launch(p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(TSG_E_HIP, "launch of %s: %s", v->name, hipGetErrorString(e));
    if (p.grid > 1 && g_reduction == TSG_REDUCE_ATOMIC) {
        const int cw = is_complex(dt) ? 2 : 1;
        const int E = M * N * cw;
        double* Cd = static_cast<double*>(C);
        hipLaunchKernelGGL(tsg::clear_small, dim3((E + 255) / 256), dim3(256), 0, p.stream, Cd, M, N, cw, ldc);
        const int64_t n = (int64_t)p.grid * E;
        if (cw == 2)
            hipLaunchKernelGGL((tsg::atomic_partials<2>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, p.stream,
                               p.ws, p.grid, E, N, Cd, ldc);
        else
            hipLaunchKernelGGL((tsg::atomic_partials<1>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, p.stream,
                               p.ws, p.grid, E, N, Cd, ldc);
        if ((e = hipGetLastError()) != hipSuccess)
            return fail(TSG_E_HIP, "launch of the atomic reduction: %s", hipGetErrorString(e));
        return TSG_OK;
    }
    if (p.grid > 1 && g_reduction == TSG_REDUCE_NONE) return TSG_OK;  // ablation: partials left in the workspace
    if (p.grid > 1 && (e = launch_fold(p, is_complex(dt))) != hipSuccess)
        return fail(TSG_E_HIP, "launch of the partial fold: %s", hipGetErrorString(e));
    return TSG_OK;
}

}  // namespace

extern "C" {

tsg_status tsg_tsmttsm(tsg_dtype dt, tsg_op op, int64_t K, int32_t M, int32_t N, const void* A, int64_t lda,
                       const void* B, int64_t ldb, void* C, int64_t ldc, void* stream)
{
    return tsmttsm_call(dt, op, K, M, N, A, lda, B, ldb, C, ldc, stream, false);
}

tsg_status tsg_tsmttsm_noalloc(tsg_dtype dt, tsg_op op, int64_t K, int32_t M, int32_t N, const void* A,
                               int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, void* stream)
{
    return tsmttsm_call(dt, op, K, M, N, A, lda, B, ldb, C, ldc, stream, true);
}

tsg_status tsg_tsmm_op(tsg_dtype dt, int32_t conjA, tsg_op opC, int64_t K, int32_t M, int32_t N, const void* A,
                       int64_t lda, const void* C, int64_t ldc, void* B, int64_t ldb, double alpha, double beta,
                       void* stream)
{
    g_err.clear();
    if (opC != TSG_OP_N && opC != TSG_OP_T && opC != TSG_OP_C) return fail(TSG_E_ARG, "unknown opC %d", (int)opC);
    if (opC != TSG_OP_N && M >= 1 && ldc < M)
        return fail(TSG_E_ARG, "ldc = %lld < M = %d for a transposed small matrix", (long long)ldc, M);
    const int64_t ldc_check = opC == TSG_OP_N ? ldc : (ldc > N ? ldc : (int64_t)N);
    tsg_status s = validate(dt, K, M, N, A, lda, C, ldc_check, B, ldb, tsg::OP_TSMM);
    if (s != TSG_OK) return s;
    if (K == 0) return TSG_OK;
    int dev;
    if ((s = current_device(&dev)) != TSG_OK) return s;
    DeviceInfo di;
    if ((s = device_info(dev, &di)) != TSG_OK) return s;
    const tsg::Variant* v = pick(tsg::OP_TSMM, dt, M, N, A, lda, B, ldb, beta != 0.0);
    if (!v) return fail(TSG_E_UNSUPPORTED, "no kernel variant for TSMM %dx%d%s", M, N,
                        g_force.empty() ? "" : " (a forced variant does not apply)");
    tsg::Launch p{};
    p.stream = static_cast<hipStream_t>(stream);
    p.grid = grid_for(dev, *v, K, M, N, di.cus);
    p.K = K;
    p.M = M;
    p.N = N;
    p.conj = (conjA && is_complex(dt)) ? 1 : 0;
    p.opc = opC == TSG_OP_N ? 0 : ((opC == TSG_OP_C && is_complex(dt)) ? 2 : 1);
    p.A = A;
    p.lda = lda;
    p.X = C;
    p.ldx = ldc;
    p.Y = B;
    p.ldy = ldb;
    p.alpha = alpha;
    p.beta = beta;
    v->launch(p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(TSG_E_HIP, "launch of %s: %s", v->name, hipGetErrorString(e));
    return TSG_OK;
}

tsg_status tsg_tsmm(tsg_dtype dt, int32_t conjA, int64_t K, int32_t M, int32_t N, const void* A, int64_t lda,
                    const void* C, int64_t ldc, void* B, int64_t ldb, double alpha, double beta, void* stream)
{
    return tsg_tsmm_op(dt, conjA, TSG_OP_N, K, M, N, A, lda, C, ldc, B, ldb, alpha, beta, stream);
}

size_t tsg_workspace_size(int32_t op_kind, tsg_dtype dt, int64_t K, int32_t M, int32_t N, int32_t count)
{
    if (op_kind == TSG_KIND_TSMM) return 0;
    if (op_kind == TSG_KIND_ORTH) return dt == TSG_R64 ? tsg::orth_workspace_size(K, M, N, count) : 0;
    if (op_kind != TSG_KIND_TSMTTSM) return 0;
    if (M < 1 || N < 1 || M > kMaxWidth || N > kMaxWidth || K < 0) return 0;
    int dev;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    DeviceInfo di;
    if (device_info(dev, &di) != TSG_OK) return 0;
    const tsg::Variant* v = pick(tsg::OP_TSMTTSM, dt, M, N, nullptr, M + (M & 1), nullptr, N + (N & 1));
    if (!v) return 0;
    return tsmttsm_ws_bytes(grid_for(dev, *v, K, M, N, di.cus), M, N, is_complex(dt));
}

tsg_status tsg_reserve(tsg_dtype dt, int64_t K, int32_t M, int32_t N, void* stream)
{
    g_err.clear();
    if (M < 1 || N < 1 || K < 0) return fail(TSG_E_ARG, "invalid shape");
    if (M > kMaxWidth || N > kMaxWidth) return fail(TSG_E_UNSUPPORTED, "widths above %d", kMaxWidth);
    int dev;
    tsg_status s = current_device(&dev);
    if (s != TSG_OK) return s;
    DeviceInfo di;
    if ((s = device_info(dev, &di)) != TSG_OK) return s;
    // the largest grid any TSMTTSM variant of this shape may use
    size_t need = 0;
    for (int i = 0; i < tsg::kNumVariants; ++i) {
        const tsg::Variant& v = tsg::kVariants[i];
        if (v.op != tsg::OP_TSMTTSM || v.dt != (int)dt) continue;
        if (!((v.M == M && v.N == N) || (v.M == 0 && M <= v.maxM && N <= v.maxN))) continue;
        size_t b = tsmttsm_ws_bytes(grid_for(dev, v, K, M, N, di.cus), M, N, is_complex(dt));
        if (b > need) need = b;
    }
    Workspace* w;
    return get_workspace(dev, static_cast<hipStream_t>(stream), need, &w);
}

tsg_status tsg_init(int32_t device)
{
    g_err.clear();
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(TSG_E_HIP, "no HIP device: %s", hipGetErrorString(e));
    if (device < 0 || device >= n) return fail(TSG_E_ARG, "device %d out of range [0, %d)", device, n);
    DeviceInfo di;
    tsg_status s = device_info(device, &di);
    if (s != TSG_OK) return s;
    // the no-alloc scratch address of `device`, resolved with it current
    int cur = -1;
    if ((e = hipGetDevice(&cur)) != hipSuccess) return fail(TSG_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess)
        return fail(TSG_E_HIP, "hipSetDevice(%d): %s", device, hipGetErrorString(e));
    double* ws = nullptr;
    s = scratch_of(device, &ws);
    if (cur != device) hipSetDevice(cur);
    return s;
}

void tsg_finalize(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = -1;
    hipGetDevice(&cur);
    for (auto& kv : g_ws) {
        hipSetDevice(kv.first.first);
        if (kv.second.data) hipFree(kv.second.data);
    }
    g_ws.clear();
    for (auto& r : g_retired) {
        hipSetDevice(r.first);
        hipFree(r.second);
    }
    g_retired.clear();
    g_occ.clear();
    if (cur >= 0) hipSetDevice(cur);
}

const char* tsg_status_string(tsg_status s)
{
    switch (s) {
    case TSG_OK: return "TSG_OK";
    case TSG_E_ARG: return "TSG_E_ARG: invalid argument";
    case TSG_E_UNSUPPORTED: return "TSG_E_UNSUPPORTED: outside the supported range";
    case TSG_E_NOMEM: return "TSG_E_NOMEM: workspace allocation failed";
    case TSG_E_HIP: return "TSG_E_HIP: HIP runtime error";
    case TSG_E_CAPTURE: return "TSG_E_CAPTURE: workspace cannot grow during stream capture";
    }
    return "unknown tsg_status";
}

const char* tsg_last_error(void) { return g_err.c_str(); }

tsg_status tsg_force_variant(const char* name)
{
    g_err.clear();
    if (!name || !*name) {
        g_force.clear();
        return TSG_OK;
    }
    for (int i = 0; i < tsg::kNumVariants; ++i)
        if (!strcmp(tsg::kVariants[i].name, name)) {
            g_force = name;
            return TSG_OK;
        }
    return fail(TSG_E_ARG, "no kernel variant named %s", name);
}

tsg_status tsg_set_grid_limit(int32_t blocks)
{
    g_err.clear();
    if (blocks < 0) return fail(TSG_E_ARG, "grid limit %d < 0", blocks);
    g_grid_cap = blocks;
    return TSG_OK;
}

tsg_status tsg_set_reduction(int32_t mode)
{
    if (mode != TSG_REDUCE_FOLD && mode != TSG_REDUCE_ATOMIC && mode != TSG_REDUCE_NONE)
        return fail(TSG_E_ARG, "unknown reduction mode %d", (int)mode);
    g_reduction = mode;
    return TSG_OK;
}

int32_t tsg_variant_count(void) { return tsg::kNumVariants; }

const char* tsg_variant_name(int32_t i) { return (i >= 0 && i < tsg::kNumVariants) ? tsg::kVariants[i].name : ""; }

const char* tsg_kernel_name(int32_t op_kind, tsg_dtype dt, int32_t conj, int32_t M, int32_t N)
{
    (void)conj;
    if (op_kind != 0 && op_kind != 1) return "";
    if (M < 1 || N < 1 || M > kMaxWidth || N > kMaxWidth) return "";
    alignas(16) static const char buf16[16] = {0};
    const void* al = static_cast<const void*>(buf16);
    // contiguous rows (lda = M, ldb = N), 16-byte aligned operands
    const tsg::Variant* v = pick(op_kind, dt, M, N, al, M, al, N);
    return v ? v->name : "";
}

}  // extern "C"
