// tsg_batched.hip -- batched block orthogonalisation in one persistent launch.
//
// For every instance i:  C_i = V_i^T W_i  (the paper's TSMTTSM, Section 3),
// then W_i <- W_i - V_i C_i (TSMM, Section 4, with alpha = -1 and beta = 1):
// the classical Gram-Schmidt projection that uses both products (Section 1.2).
//
// One kernel launch with a persistent grid consumes a device work queue:
//  * phase-1 items: a K-slab of one instance; its partial V^T W goes to the
//    slab's own slot; the last slab of an instance to finish (per-instance
//    arrival counter) sums the instance's slots in slab order into C_i and
//    raises ready[i];
//  * phase-2 items: a row slab of one instance; waits for ready[i], stages
//    -C_i on chip and updates its rows of W_i.
// Every phase-1 item precedes every phase-2 item in the queue and phase-1
// items never wait, so whatever an update waits for has already been taken by
// a running block: the waits cannot deadlock, whatever the grid.  They are
// bounded anyway (a spin limit raises an error word instead of hanging).  The
// last block to leave returns the queue head, counters and flags to zero, so
// the launch can be replayed from a captured graph without memset nodes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/tsgemm.h"
#include "tsg_device.hpp"
#include "tsg_registry.hpp"

namespace tsg {
tsg_status report(tsg_status s, const char* msg);  // sets the detail of tsg_last_error()
}

namespace {

using tsg::dbl4;
using tsg::kWave;

constexpr int kWPB = 4;  // waves per block
constexpr int kThreads = kWPB * kWave;
constexpr int kMaxM = 64, kMaxN = 16;
constexpr unsigned kDefaultSpin = 1u << 23;   // sleeps of ~0.2 us: about 2 s
constexpr int64_t kItemBytes = 4 << 20;       // input bytes of one slab (automatic sizing; 4 MB measured
                                              // 3% faster than 2 MB and 8 MB on the 64-instance workload)
constexpr int64_t kMaxSlabs = 256;            // slabs per instance (bounds the fold)

struct Item {
    int64_t row0;      // first row of the slab
    int64_t slot_off;  // phase 1: offset (doubles) of this slab's partial
    int32_t nrows;
    int32_t inst;
    int32_t phase;     // 1: slab of V^T W; 2: update of W rows
    int32_t pad;
};

struct DevDesc {
    int64_t K;
    const double* V;
    int64_t ldv;
    double* W;
    int64_t ldw;
    double* C;
    int64_t ldc;
    int64_t part0;  // offset (doubles) of the instance's first partial
    int32_t M, N;
    int32_t nparts;  // phase-1 slabs of the instance
    int32_t pad;
};

// Error bits of Ctrl::err.
constexpr unsigned kErrSpin = 1u;      // an update waited past the spin limit (results invalid)
constexpr unsigned kErrDesc = 2u;      // a descriptor failed the device-side checks (nothing was done)
constexpr unsigned kErrSpace = 4u;     // the queue or the partial sums do not fit the workspace (nothing was done)

struct Ctrl {
    unsigned head;   // next queue position
    unsigned done;   // blocks that have left the queue loop
    unsigned err;    // error bits (kErr*)
    unsigned spin;   // spin limit
    unsigned total;  // items in the queue, written by the set-up kernel
    unsigned pad[3];
};

__device__ __forceinline__ dbl4 mfma16(double a, double b, dbl4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// ------------------------------------------------------- slab addressing
// A slab (rows row0 .. row0 + nrows - 1 of a row-major matrix) is addressed
// through a raw buffer resource: base and extent live in scalar registers,
// every lane adds one 32-bit byte offset per row (columns go into the
// instruction's immediate offset).  The extent ends at the last element of
// the slab, so an access past it (a row beyond the slab, or a column past the
// end of the last row) returns zero and a store there is dropped: no address
// clamps are needed.  The plan keeps every offset below 2^31.
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format (CDNA)
constexpr int kNT = 2;                  // cache policy: streaming (last use)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t slab_rsrc(const double* base, int64_t row0, int32_t nrows,
                                                           int64_t ld, int cols)
{
    const int bytes = nrows > 0 ? (int)(((int64_t)(nrows - 1) * ld + cols) * 8) : 0;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base + row0 * ld), 0, bytes, kRsrcWord3);
}

template <int AUX>
__device__ __forceinline__ double ld_buf(__amdgpu_buffer_rsrc_t r, int off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX));
}

__device__ __forceinline__ void st_buf(__amdgpu_buffer_rsrc_t r, int off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                          off, 0, kNT);
}

// ------------------------------------------------------- one path per call
// Every (width class, phase) code path is a function of its own (not
// inlined), so that each gets its own register allocation: inlined into one
// loop, the paths' live ranges pile up and spill.  Call arguments arrive in
// vector registers, so each path re-reads its item and descriptor and makes
// the fields wave-uniform again (scalar registers, buffer descriptors
// without waterfall loops).
__shared__ double g_lds[kMaxM * kMaxN];  // C staging and the cross-wave sums

__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T* uni(T* p)
{
    return reinterpret_cast<T*>(uni(reinterpret_cast<int64_t>(p)));
}

__device__ __forceinline__ void fetch_item(const Item* items, const DevDesc* descs, int q, Item& it, DevDesc& d)
{
    it = uni(items)[uni(q)];
    it.row0 = uni(it.row0);
    it.slot_off = uni(it.slot_off);
    it.nrows = uni(it.nrows);
    it.inst = uni(it.inst);
    d = uni(descs)[it.inst];
    d.K = uni(d.K);
    d.V = uni(d.V);
    d.ldv = uni(d.ldv);
    d.W = uni(d.W);
    d.ldw = uni(d.ldw);
    d.C = uni(d.C);
    d.ldc = uni(d.ldc);
    d.part0 = uni(d.part0);
    d.M = uni(d.M);
    d.N = uni(d.N);
    d.nparts = uni(d.nparts);
}

// ---------------------------------------------------------------- phase 1
// V^T W over one slab, MB m-blocks of 16 (M <= 16 MB) and one n-block
// (N <= 16).  v_mfma_f64_16x16x4f64 takes lane l's A value as A(l%16, l/16)
// and its B value as B(l/16, l%16): lane (r = l/16, c = l%16) supplies
// V(k0 + r, 16 mb + c) and W(k0 + r, c), four rows per product; a step takes
// U such groups (4U rows).  The waves of the block take every fourth step,
// loading the rows of the next NBUF - 1 steps before the current ones are
// multiplied.  Rows past the slab read zero.  Lanes whose column is past M or
// N feed only output rows or columns that are never stored, so they need no
// guard.
template <int MB, int U, int NBUF>
__device__ __attribute__((noinline)) void slab_partial(const Item* items, const DevDesc* descs, int q, double* parts_)
{
    Item it;
    DevDesc d;
    fetch_item(items, descs, q, it, d);
    double* __restrict__ parts = uni(parts_);
    double* lds = g_lds;
    int lane = threadIdx.x & (kWave - 1);
    int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // uniform loop bounds
    // opaque per item: keeps lane-derived offsets of every code path from being
    // hoisted out of the queue loop (they would all stay live at once)
    __asm__ volatile("" : "+v"(lane), "+s"(wave));
    const int lr = lane >> 4, lc = lane & 15;
    const int M = d.M, N = d.N;
    const auto rv = slab_rsrc(d.V, it.row0, it.nrows, d.ldv, M);
    const auto rw = slab_rsrc(d.W, it.row0, it.nrows, d.ldw, N);
    const int sv = (int)(4 * d.ldv * 8), sw = (int)(4 * d.ldw * 8);  // bytes per four rows
    const int ov = (int)(lr * d.ldv + lc) * 8, ow = (int)(lr * d.ldw + lc) * 8;
    dbl4 acc[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) acc[i] = dbl4{0.0, 0.0, 0.0, 0.0};
    struct Frag {
        double a[U][MB];
        double b[U];
    };
    Frag fr[NBUF];  // register sets in flight (leap frogging)
    auto load = [&](int64_t g, Frag& f) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int grp = (int)(U * g + u);
#pragma unroll
            for (int i = 0; i < MB; ++i) f.a[u][i] = ld_buf<0>(rv, grp * sv + ov + 128 * i);
            f.b[u] = ld_buf<0>(rw, grp * sw + ow);
        }
    };
    auto compute = [&](int64_t, Frag& f) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < MB; ++i) acc[i] = mfma16(f.a[u][i], f.b[u], acc[i]);
    };
    const int64_t nsteps = (it.nrows + 4 * U - 1) / (4 * U);
    tsg::pipeline<NBUF>((int64_t)wave, nsteps, (int64_t)kWPB, fr, load, compute);

    // waves summed in wave order into lds[m * N + n]; lane holds D(l/16 + 4r, l%16)
    for (int w = 0; w < kWPB; ++w) {
        if (wave == w) {
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = 16 * i + lr + 4 * r;
                    if (m < M && lc < N) {
                        const int e = m * N + lc;
                        lds[e] = (w == 0) ? acc[i][r] : lds[e] + acc[i][r];
                    }
                }
        }
        __syncthreads();
    }
    double* part = parts + it.slot_off;
    for (int e = threadIdx.x; e < M * N; e += kThreads) part[e] = lds[e];
}

// Sum of the instance's partials in slab order, eight loads in flight.
__device__ void fold_instance(const DevDesc& d, const double* __restrict__ parts)
{
    const int E = d.M * d.N, P = d.nparts;
    for (int e = threadIdx.x; e < E; e += kThreads) {
        const double* p = parts + d.part0 + e;
        double s = 0.0;
        int j = 0;
        for (; j + 8 <= P; j += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(j + u) * E];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; j < P; ++j) s += p[(int64_t)j * E];
        const int m = e / d.N, n = e - m * d.N;
        d.C[(int64_t)m * d.ldc + n] = s;
    }
}

// ---------------------------------------------------------------- phase 2
// W(rows) <- W(rows) + V(rows) (-C), sixteen rows per MFMA chain: lane
// (r, c) supplies V(row0 + 16 b + c, 4 s + r) as the A value of contraction
// step s, and the B value -C(4 s + r, c) comes from LDS in fragment order
// (one conflict-free read per lane and step).  The accumulator starts from
// the W values the lane owns, W(row0 + 16 b + r + 4 q, c), q = 0..3, loaded
// with V NBUF - 1 steps ahead; a step takes U blocks of sixteen rows.  Only the
// last contraction step can reach past M (4 (MS - 1) < M); its lanes there
// are zeroed, since the staged C is zero but the loaded value need not be
// finite.  Rows past the slab read zero and their stores are dropped; lanes
// whose column is past N neither matter nor store.
template <int MS, int U, int NBUF>
__device__ __attribute__((noinline)) void slab_update(const Item* items, const DevDesc* descs, int q)
{
    Item it;
    DevDesc d;
    fetch_item(items, descs, q, it, d);
    const double* cf = g_lds;
    int lane = threadIdx.x & (kWave - 1);
    int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // uniform loop bounds
    // opaque per item: keeps lane-derived offsets of every code path from being
    // hoisted out of the queue loop (they would all stay live at once)
    __asm__ volatile("" : "+v"(lane), "+s"(wave));
    const int lr = lane >> 4, lc = lane & 15;
    const int M = d.M, N = d.N;
    const auto rv = slab_rsrc(d.V, it.row0, it.nrows, d.ldv, M);
    const auto rw = slab_rsrc(d.W, it.row0, it.nrows, d.ldw, N);
    const bool kok = 4 * (MS - 1) + lr < M;
    const bool nok = lc < N;
    const int sv = (int)(16 * d.ldv * 8), sw = (int)(16 * d.ldw * 8);  // bytes per sixteen rows
    const int ov = (int)(lc * d.ldv + lr) * 8;
    const int ow = (int)(lr * d.ldw + lc) * 8, qw = (int)(4 * d.ldw * 8);
    struct Frag {
        double a[U][MS];
        dbl4 w[U];
    };
    Frag fr[NBUF];  // register sets in flight (leap frogging)
    auto load = [&](int64_t g, Frag& f) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int blk = (int)(U * g + u);
#pragma unroll
            for (int s = 0; s < MS; ++s) f.a[u][s] = ld_buf<kNT>(rv, blk * sv + ov + 32 * s);
            f.a[u][MS - 1] = kok ? f.a[u][MS - 1] : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) f.w[u][q] = ld_buf<kNT>(rw, blk * sw + ow + q * qw);
        }
    };
    auto compute = [&](int64_t g, Frag& f) {
        __asm__ volatile("" ::: "memory");  // read C from LDS each time (no hoisting into registers)
#pragma unroll
        for (int u = 0; u < U; ++u) {
            dbl4 acc = f.w[u];
#pragma unroll
            for (int s = 0; s < MS; ++s) acc = mfma16(f.a[u][s], cf[s * kWave + lane], acc);
            const int blk = (int)(U * g + u);
            if (nok) {
#pragma unroll
                for (int q = 0; q < 4; ++q) st_buf(rw, blk * sw + ow + q * qw, acc[q]);
            }
        }
    };
    const int64_t nsteps = (it.nrows + 16 * U - 1) / (16 * U);
    tsg::pipeline<NBUF>((int64_t)wave, nsteps, (int64_t)kWPB, fr, load, compute);
}

// ------------------------------------------- slab reads (contiguous rows)
// With ldv = M and ldw = N the rows one wave takes in one step are one
// contiguous run of V and one of W.  Each run is read through a buffer
// resource that ends where the run (or the slab) ends, so loads past it
// return zero and cost no memory traffic: the wave issues consecutive 8-byte
// loads (512 contiguous bytes per instruction, whatever the widths), stages
// the runs in its own LDS region and reads the matrix-core operands back from
// there.  Phase 2 writes its results back into the staged W run and stores
// the run with consecutive 8-byte stores.  The lanes read each other's staged
// values: one wave's LDS accesses complete in order, and a compiler memory
// barrier on each side of the staging keeps the compiler from treating them
// as independent.
constexpr int kRunMax = 1280;  // doubles of staged runs per wave (largest path: 16 rows x (64 + 16))
__shared__ double g_run[kWPB * kRunMax];

__device__ __forceinline__ __amdgpu_buffer_rsrc_t run_rsrc(const double* base, int n)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), 0, n * 8, kRsrcWord3);
}
__device__ __forceinline__ void lds_barrier() { __asm__ volatile("" ::: "memory"); }

// Phase 1 on runs: steps of 4U rows; lane (r, c) takes V(k0 + r, 16 mb + c)
// and W(k0 + r, c) of each group of four rows from the staged runs (columns
// past M or N read the next row's values, which reach only outputs that are
// never stored).
template <int MB, int U, int NBUF>
__device__ __attribute__((noinline)) void run_partial(const Item* items, const DevDesc* descs, int q, double* parts_)
{
    Item it;
    DevDesc d;
    fetch_item(items, descs, q, it, d);
    double* __restrict__ parts = uni(parts_);
    double* lds = g_lds;
    int lane = threadIdx.x & (kWave - 1);
    int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    __asm__ volatile("" : "+v"(lane), "+s"(wave));
    const int lr = lane >> 4, lc = lane & 15;
    const int M = d.M, N = d.N;
    constexpr int NLV = U * MB, NLW = U;  // loads per lane: 4U rows x 16 MB (or 16) columns at most
    static_assert(kWave * (NLV + NLW) <= kRunMax, "staged runs exceed the wave's LDS region");
    double* run = g_run + wave * kRunMax;
    double* runw = run + kWave * NLV;
    dbl4 acc[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) acc[i] = dbl4{0.0, 0.0, 0.0, 0.0};
    struct Frag {
        double v[NLV];
        double w[NLW];
    };
    Frag fr[NBUF];
    auto load = [&](int64_t g, Frag& f) {
        const int64_t r0 = it.row0 + (int64_t)4 * U * g;
        const int rows = (int)min((int64_t)4 * U, (int64_t)it.nrows - 4 * U * g);
        const auto rv = run_rsrc(d.V + r0 * M, rows * M);
        const auto rw = run_rsrc(d.W + r0 * N, rows * N);
#pragma unroll
        for (int i = 0; i < NLV; ++i) f.v[i] = ld_buf<kNT>(rv, (i * kWave + lane) * 8);
#pragma unroll
        for (int i = 0; i < NLW; ++i) f.w[i] = ld_buf<kNT>(rw, (i * kWave + lane) * 8);
    };
    auto compute = [&](int64_t, Frag& f) {
        lds_barrier();
#pragma unroll
        for (int i = 0; i < NLV; ++i) run[i * kWave + lane] = f.v[i];
#pragma unroll
        for (int i = 0; i < NLW; ++i) runw[i * kWave + lane] = f.w[i];
        lds_barrier();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double b = runw[(4 * u + lr) * N + lc];
#pragma unroll
            for (int i = 0; i < MB; ++i) acc[i] = mfma16(run[(4 * u + lr) * M + 16 * i + lc], b, acc[i]);
        }
    };
    const int64_t nsteps = (it.nrows + 4 * U - 1) / (4 * U);
    tsg::pipeline<NBUF>((int64_t)wave, nsteps, (int64_t)kWPB, fr, load, compute);

    for (int w = 0; w < kWPB; ++w) {
        if (wave == w) {
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = 16 * i + lr + 4 * r;
                    if (m < M && lc < N) {
                        const int e = m * N + lc;
                        lds[e] = (w == 0) ? acc[i][r] : lds[e] + acc[i][r];
                    }
                }
        }
        __syncthreads();
    }
    double* part = parts + it.slot_off;
    for (int e = threadIdx.x; e < M * N; e += kThreads) part[e] = lds[e];
}

// Phase 1 on runs for M, N <= 16, with row packing: P = 16 / max(M, N) rows
// share one product (lane i of k-slot q takes V(k0 + q P + i / M, i % M) and
// W(k0 + q P + i / N, i % N), which in the staged runs are simply elements
// (4 P u + q P) M + i and (4 P u + q P) N + i); of the 16 x 16 product only
// the P diagonal blocks (row and column from the same packed row) are
// partial sums of C, and the epilogue adds them.  Lanes past P M or P N read
// neighbouring values that reach only the discarded blocks.  With P = 1 this
// is the plain mapping.  Narrow instances run P times fewer products, which
// bound them before (four rows per product).
template <int U, int NBUF>
__device__ __attribute__((noinline)) void run_partial_packed(const Item* items, const DevDesc* descs, int q,
                                                             double* parts_)
{
    Item it;
    DevDesc d;
    fetch_item(items, descs, q, it, d);
    double* __restrict__ parts = uni(parts_);
    int lane = threadIdx.x & (kWave - 1);
    int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    __asm__ volatile("" : "+v"(lane), "+s"(wave));
    const int lr = lane >> 4, lc = lane & 15;
    const int M = d.M, N = d.N;
    const int P = 16 / (M > N ? M : N);  // packed rows per fragment row
    const int RS = 4 * P;                // rows per product
    constexpr int NL = U;                // a run of 4 P U rows holds at most 64 U elements
    // the reads of lanes past P M or P N stay inside the wave's region
    static_assert(kWave * 2 * NL + 16 <= kRunMax, "staged runs exceed the wave's LDS region");
    double* run = g_run + wave * kRunMax;
    double* runw = run + kWave * NL;
    dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
    struct Frag {
        double v[NL];
        double w[NL];
    };
    Frag fr[NBUF];
    auto load = [&](int64_t g, Frag& f) {
        const int64_t r0 = it.row0 + (int64_t)RS * U * g;
        const int rows = (int)min((int64_t)RS * U, (int64_t)it.nrows - (int64_t)RS * U * g);
        const auto rv = run_rsrc(d.V + r0 * M, rows * M);
        const auto rw = run_rsrc(d.W + r0 * N, rows * N);
#pragma unroll
        for (int i = 0; i < NL; ++i) f.v[i] = ld_buf<kNT>(rv, (i * kWave + lane) * 8);
#pragma unroll
        for (int i = 0; i < NL; ++i) f.w[i] = ld_buf<kNT>(rw, (i * kWave + lane) * 8);
    };
    auto compute = [&](int64_t, Frag& f) {
        lds_barrier();
#pragma unroll
        for (int i = 0; i < NL; ++i) run[i * kWave + lane] = f.v[i];
#pragma unroll
        for (int i = 0; i < NL; ++i) runw[i * kWave + lane] = f.w[i];
        lds_barrier();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = RS * u + lr * P;  // first row of this k-slot's packed group
            acc = mfma16(run[r * M + lc], runw[r * N + lc], acc);
        }
    };
    const int64_t per = (int64_t)RS * U;
    const int64_t nsteps = (it.nrows + per - 1) / per;
    tsg::pipeline<NBUF>((int64_t)wave, nsteps, (int64_t)kWPB, fr, load, compute);

    // every wave's 16 x 16 product into its region; then the P diagonal
    // blocks of all waves are added in a fixed order (waves, then blocks)
    lds_barrier();
#pragma unroll
    for (int r = 0; r < 4; ++r) run[(lr + 4 * r) * 16 + lc] = acc[r];
    __syncthreads();
    double* part = parts + it.slot_off;
    for (int e = threadIdx.x; e < M * N; e += kThreads) {
        const int m = e / N, n = e - (e / N) * N;
        double s = 0.0;
        for (int w = 0; w < kWPB; ++w) {
            const double* Dw = g_run + w * kRunMax;
            for (int h = 0; h < P; ++h) s += Dw[(h * M + m) * 16 + h * N + n];
        }
        part[e] = s;
    }
}

// Phase 2 on runs: steps of 16U rows.  Lane (r, c) takes V(16 b + c, 4 s + r)
// from the staged V run (zeroed past M: the value there belongs to the next
// row, and although the staged C is zero there, a non-finite value times zero
// is not zero) and starts its accumulator from the staged old
// W(16 b + r + 4 q, c); the results go back to the same W positions (lanes
// with c < N only: a column past N addresses the next row) and the W run is
// stored.
template <int MS, int U, int NBUF>
__device__ __attribute__((noinline)) void run_update(const Item* items, const DevDesc* descs, int q)
{
    Item it;
    DevDesc d;
    fetch_item(items, descs, q, it, d);
    const double* cf = g_lds;
    int lane = threadIdx.x & (kWave - 1);
    int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    __asm__ volatile("" : "+v"(lane), "+s"(wave));
    const int lr = lane >> 4, lc = lane & 15;
    const int M = d.M, N = d.N;
    constexpr int NLV = U * MS, NLW = 4 * U;  // 16U rows x 4 MS (or 16) columns at most
    static_assert(kWave * (NLV + NLW) <= kRunMax, "staged runs exceed the wave's LDS region");
    double* run = g_run + wave * kRunMax;
    double* runw = run + kWave * NLV;
    const bool kok = 4 * (MS - 1) + lr < M;
    const bool nok = lc < N;
    struct Frag {
        double v[NLV];
        double w[NLW];
    };
    Frag fr[NBUF];
    auto load = [&](int64_t g, Frag& f) {
        const int64_t r0 = it.row0 + (int64_t)16 * U * g;
        const int rows = (int)min((int64_t)16 * U, (int64_t)it.nrows - 16 * U * g);
        const auto rv = run_rsrc(d.V + r0 * M, rows * M);
        const auto rw = run_rsrc(d.W + r0 * N, rows * N);
#pragma unroll
        for (int i = 0; i < NLV; ++i) f.v[i] = ld_buf<kNT>(rv, (i * kWave + lane) * 8);
#pragma unroll
        for (int i = 0; i < NLW; ++i) f.w[i] = ld_buf<kNT>(rw, (i * kWave + lane) * 8);
    };
    auto compute = [&](int64_t g, Frag& f) {
        lds_barrier();
#pragma unroll
        for (int i = 0; i < NLV; ++i) run[i * kWave + lane] = f.v[i];
#pragma unroll
        for (int i = 0; i < NLW; ++i) runw[i * kWave + lane] = f.w[i];
        lds_barrier();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            dbl4 acc;
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) acc[qq] = runw[(16 * u + lr + 4 * qq) * N + lc];
#pragma unroll
            for (int s = 0; s < MS; ++s) {
                double a = run[(16 * u + lc) * M + 4 * s + lr];
                if (s == MS - 1) a = kok ? a : 0.0;
                acc = mfma16(a, cf[s * kWave + lane], acc);
                // operands are read four steps at a time (the products keep
                // running meanwhile): all of them at once would not fit the
                // register budget of the wide paths
                if (s % 4 == 3) lds_barrier();
            }
            if (nok) {
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) runw[(16 * u + lr + 4 * qq) * N + lc] = acc[qq];
            }
        }
        lds_barrier();
        const int64_t r0 = it.row0 + (int64_t)16 * U * g;
        const int rows = (int)min((int64_t)16 * U, (int64_t)it.nrows - 16 * U * g);
        const auto rw = run_rsrc(d.W + r0 * N, rows * N);
#pragma unroll
        for (int i = 0; i < NLW; ++i) st_buf(rw, (i * kWave + lane) * 8, runw[i * kWave + lane]);
    };
    const int64_t nsteps = (it.nrows + 16 * U - 1) / (16 * U);
    tsg::pipeline<NBUF>((int64_t)wave, nsteps, (int64_t)kWPB, fr, load, compute);
}

// Two waves per SIMD: every path fits in 256 registers without spilling.
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2)))
orth_persistent(const DevDesc* __restrict__ descs, const Item* __restrict__ items,
                double* __restrict__ parts, unsigned* __restrict__ cnt, unsigned* __restrict__ ready,
                Ctrl* __restrict__ ctrl, int count)
{
    __shared__ int s_q, s_last;
    double* lds = g_lds;
    const int tid = threadIdx.x;
    // written by the set-up kernel earlier on the stream (0 when it rejected the batch)
    const int total = (int)__builtin_amdgcn_readfirstlane(ctrl->total);
    while (true) {
        if (tid == 0)
            s_q = (int)__hip_atomic_fetch_add(&ctrl->head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int q = __builtin_amdgcn_readfirstlane(s_q);  // uniform: item and descriptor go to SGPRs
        if (q >= total) break;
        const Item it = items[q];
        const DevDesc d = descs[it.inst];
        if (it.phase == 1) {
            // rows per step chosen so that a register set holds about 20 values;
            // contiguous instances read their rows as runs
            if (d.ldv == d.M && d.ldw == d.N) {
                switch ((d.M + 15) / 16) {
                case 1: run_partial_packed<8, 2>(items, descs, q, parts); break;
                case 2: run_partial<2, 4, 2>(items, descs, q, parts); break;
                case 3: run_partial<3, 2, 2>(items, descs, q, parts); break;
                default: run_partial<4, 1, 2>(items, descs, q, parts); break;
                }
            } else {
                switch ((d.M + 15) / 16) {
                case 1: slab_partial<1, 8, 2>(items, descs, q, parts); break;
                case 2: slab_partial<2, 4, 2>(items, descs, q, parts); break;
                case 3: slab_partial<3, 2, 2>(items, descs, q, parts); break;
                default: slab_partial<4, 2, 2>(items, descs, q, parts); break;
                }
            }
            fence_release();  // this wave's part of the partial, before the arrival is counted
            __syncthreads();
            if (tid == 0) {
                const unsigned old =
                    __hip_atomic_fetch_add(&cnt[it.inst], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                s_last = old == (unsigned)(d.nparts - 1);
            }
            __syncthreads();
            if (__builtin_amdgcn_readfirstlane(s_last)) {
                fence_acquire();  // every partial of the instance is visible
                fold_instance(d, parts);
                fence_release();
                __syncthreads();
                if (tid == 0) __hip_atomic_store(&ready[it.inst], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        } else {
            if (tid == 0) {
                const unsigned limit = __hip_atomic_load(&ctrl->spin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // bounded wait; the limit is checked first, so a limit of 0 always gives up
                for (unsigned spins = 0;; ++spins) {
                    if (spins >= limit) {
                        __hip_atomic_fetch_or(&ctrl->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    if (__hip_atomic_load(&ready[it.inst], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
                    __builtin_amdgcn_s_sleep(8);
                }
            }
            __syncthreads();
            fence_acquire();  // C_i as written by the fold
            // -C_i in MFMA operand order: lds[s * 64 + l] = -C(4 s + l/16, l%16)
            const int MS = (d.M + 3) / 4;
            for (int idx = tid; idx < MS * kWave; idx += kThreads) {
                const int l = idx & (kWave - 1), s = idx / kWave;
                const int m = 4 * s + (l >> 4), n = l & 15;
                lds[idx] = (m < d.M && n < d.N) ? -d.C[(int64_t)m * d.ldc + n] : 0.0;
            }
            __syncthreads();
            if (d.ldv == d.M && d.ldw == d.N) {
                switch (MS) {
                case 1: run_update<1, 2, 2>(items, descs, q); break;
                case 2: run_update<2, 2, 2>(items, descs, q); break;
                case 3: run_update<3, 2, 2>(items, descs, q); break;
                case 4: run_update<4, 2, 2>(items, descs, q); break;
                case 5: run_update<5, 1, 2>(items, descs, q); break;
                case 6: run_update<6, 1, 2>(items, descs, q); break;
                case 7: run_update<7, 1, 2>(items, descs, q); break;
                case 8: run_update<8, 1, 2>(items, descs, q); break;
                case 9: run_update<9, 1, 2>(items, descs, q); break;
                case 10: run_update<10, 1, 2>(items, descs, q); break;
                case 11: run_update<11, 1, 2>(items, descs, q); break;
                case 12: run_update<12, 1, 2>(items, descs, q); break;
                case 13: run_update<13, 1, 2>(items, descs, q); break;
                case 14: run_update<14, 1, 2>(items, descs, q); break;
                case 15: run_update<15, 1, 2>(items, descs, q); break;
                default: run_update<16, 1, 2>(items, descs, q); break;
                }
            } else switch (MS) {
            case 1: slab_update<1, 4, 2>(items, descs, q); break;
            case 2: slab_update<2, 2, 2>(items, descs, q); break;
            case 3: slab_update<3, 2, 2>(items, descs, q); break;
            case 4: slab_update<4, 2, 2>(items, descs, q); break;
            case 5: slab_update<5, 2, 2>(items, descs, q); break;
            case 6: slab_update<6, 1, 2>(items, descs, q); break;
            case 7: slab_update<7, 1, 2>(items, descs, q); break;
            case 8: slab_update<8, 1, 2>(items, descs, q); break;
            case 9: slab_update<9, 1, 2>(items, descs, q); break;
            case 10: slab_update<10, 1, 2>(items, descs, q); break;
            case 11: slab_update<11, 1, 2>(items, descs, q); break;
            case 12: slab_update<12, 1, 2>(items, descs, q); break;
            case 13: slab_update<13, 1, 2>(items, descs, q); break;
            case 14: slab_update<14, 1, 2>(items, descs, q); break;
            case 15: slab_update<15, 1, 2>(items, descs, q); break;
            default: slab_update<16, 1, 2>(items, descs, q); break;
            }
        }
        __syncthreads();  // LDS and s_q are reused by the next item
    }
    // the last block out resets the queue, counters and flags for the next launch
    if (tid == 0) {
        const unsigned old = __hip_atomic_fetch_add(&ctrl->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (old == gridDim.x - 1) {
            for (int i = 0; i < count; ++i) {
                __hip_atomic_store(&cnt[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&ready[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            __hip_atomic_store(&ctrl->head, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctrl->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ------------------------------------------------------------ work queue
// Slab height of an instance: rows_fixed if positive, else about item_bytes
// of input per slab and at most kMaxSlabs slabs; never more rows than keep
// the byte offsets inside a slab (plus one step past its end) below 2^31.
// Returns 0 if no height fits (leading dimensions too large).  Shared by the
// host (workspace sizes, plan checks) and the set-up kernel.
__host__ __device__ inline int64_t round16(int64_t x) { return (x + 15) / 16 * 16; }

__host__ __device__ inline int64_t slab_limit(int64_t ldv, int64_t ldw)
{
    const int64_t ld = ldv > ldw ? ldv : ldw;
    return ((((int64_t)1 << 31) / (8 * ld)) - 128) / 16 * 16;
}

__host__ __device__ inline int64_t slab_rows(int64_t K, int M, int N, int64_t ldv, int64_t ldw, int64_t rows_fixed,
                                             int64_t item_bytes)
{
    const int64_t lim = slab_limit(ldv, ldw);
    int64_t R = rows_fixed;
    if (R <= 0) {
        const int64_t want = round16(item_bytes / (8 * (int64_t)(M + N)));
        R = want > 16 ? want : 16;
        const int64_t few = round16((K + kMaxSlabs - 1) / kMaxSlabs);
        R = R > few ? R : few;
        R = R < lim ? R : lim;
    }
    return (R >= 1 && R <= lim) ? R : 0;
}

// Rows of one update item cut from a slab of nr rows into about f pieces
// (f = 1: the whole slab).
__host__ __device__ inline int64_t update_piece(int64_t nr, int f)
{
    if (f <= 1) return nr;
    const int64_t p = round16((nr + f - 1) / f);
    return p > 16 ? p : 16;
}

// Items per instance that a workspace sized by tsg_workspace_size holds:
// kMaxSlabs slab items and, at the end of the queue, up to four update
// pieces per slab.
constexpr int64_t kItemsPerInstance = 5 * kMaxSlabs;
constexpr int kMaxCount = 1024;  // instances per call (one set-up block, one thread each)

// Byte layout of a workspace: control words, descriptors, arrival counters
// and ready flags, the item queue, the partial sums.  Regions start at
// multiples of 256 bytes.
struct Layout {
    size_t ctrl, descs, flags, items, parts, bytes;
    int64_t max_items, max_parts;
};

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }

__host__ __device__ inline Layout make_layout(int count, int64_t max_items, int64_t max_parts)
{
    Layout L{};
    L.ctrl = 0;
    L.descs = align256(sizeof(Ctrl));
    L.flags = L.descs + align256(sizeof(DevDesc) * (size_t)count);
    L.items = L.flags + align256(sizeof(unsigned) * 2 * (size_t)count);
    L.parts = L.items + align256(sizeof(Item) * (size_t)max_items);
    L.bytes = L.parts + sizeof(double) * (size_t)(max_parts > 0 ? max_parts : 1);
    L.max_items = max_items;
    L.max_parts = max_parts;
    return L;
}

// Set-up kernel (one block of kMaxCount threads): checks the descriptors,
// orders the instances by decreasing input size K (M + N) (ties by index),
// cuts them into slabs, places the partial sums, writes the item queue and
// clears the counters, flags and queue head, all on the device, so a call
// with descriptors in device memory needs no host round trip and can be
// captured into a graph.  Queue order: the slab items of instance r (rank
// in size order) are followed by those of instance r + lag, then the update
// items of instance r (lag >= count: every slab item before any update
// item).  An update item waits only for slab items of its own instance, all
// of which precede it in the queue and never wait, so the persistent kernel
// cannot deadlock whatever the lag.  With automatic slab heights the updates
// at the end of the queue are cut finer (the instance whose later update
// items number fewer than `resident` into quarter slabs, fewer than three
// times that into half slabs), so the blocks still running after the queue
// drains hold short items.
__global__ void __launch_bounds__(kMaxCount)
orth_setup(const tsg_orth_desc* __restrict__ in, int count, int64_t rows_fixed, int64_t item_bytes, int lag,
           int resident, unsigned spin, Ctrl* __restrict__ ctrl, DevDesc* __restrict__ dd, unsigned* __restrict__ flags,
           Item* __restrict__ items, int64_t max_items, int64_t max_parts)
{
    // 56 KB: per instance its size key (then K), slab height, first partial
    // sum, slabs, rank order, queue positions, update pieces, pieces per full
    // slab, M N and its piece factor
    __shared__ int64_t s_key[kMaxCount], s_rows[kMaxCount], s_part0[kMaxCount];
    __shared__ int s_nsl[kMaxCount], s_ord[kMaxCount], s_pos1[kMaxCount], s_pos2[kMaxCount];
    __shared__ int s_pieces[kMaxCount], s_npf[kMaxCount], s_E[kMaxCount], s_f[kMaxCount];
    __shared__ unsigned s_err;
    __shared__ int s_total;
    const int tid = threadIdx.x;
    if (tid == 0) s_err = 0u;
    __syncthreads();
    tsg_orth_desc x{};
    if (tid < count) {
        x = in[tid];
        const uintptr_t al = reinterpret_cast<uintptr_t>(x.V) | reinterpret_cast<uintptr_t>(x.W) |
                             reinterpret_cast<uintptr_t>(x.C);
        bool ok = x.K >= 0 && x.M >= 1 && x.N >= 1 && x.M <= kMaxM && x.N <= kMaxN && x.ldv >= x.M &&
                  x.ldw >= x.N && x.ldc >= x.N && x.C && (x.K == 0 || (x.V && x.W)) && al % sizeof(double) == 0;
        const int64_t R = ok ? slab_rows(x.K, x.M, x.N, x.ldv, x.ldw, rows_fixed, item_bytes) : 0;
        const int64_t nsl = x.K > 0 && R > 0 ? (x.K + R - 1) / R : 1;  // K = 0: one empty slab sets C = 0
        ok = ok && R > 0 && nsl <= ((int64_t)1 << 24);
        if (!ok) atomicOr(&s_err, kErrDesc);
        s_key[tid] = x.K * (int64_t)(x.M + x.N);
        s_rows[tid] = ok ? R : 1;
        s_nsl[tid] = ok ? (int)nsl : 1;
        s_E[tid] = x.M * x.N;
        flags[tid] = 0u;           // arrival counter
        flags[count + tid] = 0u;   // ready flag
    }
    __syncthreads();
    // rank by decreasing size, ties by index
    if (tid < count) {
        int r = 0;
        for (int j = 0; j < count; ++j) r += (s_key[j] > s_key[tid]) || (s_key[j] == s_key[tid] && j < tid);
        s_ord[r] = tid;
    }
    __syncthreads();
    if (tid < count) s_key[tid] = x.K;  // the keys are no longer needed
    __syncthreads();
    if (tid == 0) {
        // update pieces per instance, from the end of the queue backwards
        int64_t made = 0;
        for (int r = count - 1; r >= 0; --r) {
            const int i = s_ord[r];
            const int64_t K = s_key[i], R = s_rows[i];
            const int n = s_nsl[i];
            int64_t pieces = 0, npf = 1;
            const int f = rows_fixed > 0 ? 1 : made < resident ? 4 : made < 3 * (int64_t)resident ? 2 : 1;
            if (K > 0) {
                const int64_t last = K - (int64_t)(n - 1) * R;
                const int64_t pf = update_piece(R, f), pl = update_piece(last, f);
                npf = (R + pf - 1) / pf;
                pieces = (int64_t)(n - 1) * npf + (last + pl - 1) / pl;
            }
            s_pieces[i] = (int)min(pieces, (int64_t)1 << 30);
            s_npf[i] = (int)npf;
            s_f[i] = f;
            made += pieces;
        }
        // queue positions and partial-sum offsets, largest instance first
        if (lag < 1) lag = 1;
        int64_t pos = 0, part = 0;
        for (int r = 0; r < count + lag; ++r) {
            if (r < count) {
                const int i = s_ord[r];
                s_part0[i] = part;
                part += (int64_t)s_nsl[i] * s_E[i];
                s_pos1[i] = (int)min(pos, (int64_t)1 << 30);
                pos += s_nsl[i];
            }
            if (r >= lag && r - lag < count) {
                const int i = s_ord[r - lag];
                s_pos2[i] = (int)min(pos, (int64_t)1 << 30);
                pos += s_pieces[i];
            }
        }
        if (pos > max_items || part > max_parts) s_err |= kErrSpace;
        s_total = s_err ? 0 : (int)pos;
    }
    __syncthreads();
    if (tid < count) {
        DevDesc d{};
        d.K = x.K;
        d.V = x.V;
        d.ldv = x.ldv;
        d.W = x.W;
        d.ldw = x.ldw;
        d.C = x.C;
        d.ldc = x.ldc;
        d.M = x.M;
        d.N = x.N;
        d.part0 = s_part0[tid];
        d.nparts = s_nsl[tid];
        dd[tid] = d;
    }
    if (s_total > 0) {
        for (int r = 0; r < count; ++r) {
            const int i = s_ord[r];
            const int64_t K = s_key[i], R = s_rows[i];
            const int n = s_nsl[i];
            const int64_t E = s_E[i];
            for (int j = tid; j < n; j += blockDim.x) {
                Item it{};
                it.row0 = (int64_t)j * R;
                it.nrows = (int32_t)min(R, K - it.row0);
                it.inst = i;
                it.phase = 1;
                it.slot_off = s_part0[i] + j * E;
                items[s_pos1[i] + j] = it;
            }
            const int npf = s_npf[i];
            const int64_t full = (int64_t)(n - 1) * npf;
            for (int p = tid; p < s_pieces[i]; p += blockDim.x) {
                const int j = p < full ? p / npf : n - 1;
                const int64_t k = p < full ? p - (int64_t)j * npf : p - full;
                const int64_t row0 = (int64_t)j * R, nr = min(R, K - row0);
                const int64_t piece = update_piece(nr, s_f[i]);
                Item it{};
                it.row0 = row0 + k * piece;
                it.nrows = (int32_t)min(piece, nr - k * piece);
                it.inst = i;
                it.phase = 2;
                items[s_pos2[i] + p] = it;
            }
        }
    }
    if (tid == 0) {
        ctrl->head = 0u;
        ctrl->done = 0u;
        ctrl->err = s_err;
        ctrl->spin = spin;
        ctrl->total = (unsigned)s_total;
    }
}

}  // namespace

// A plan owns a workspace laid out as above, filled once by the set-up
// kernel, and a graph holding one launch of the persistent kernel.
struct tsg_orth_plan_t {
    int dev = 0;
    int count = 0;
    int grid = 0;
    void* ws = nullptr;
    tsg_orth_desc* d_in = nullptr;  // the caller's descriptors, uploaded
    Layout L{};
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

template <class T>
T* at(void* ws, size_t off)
{
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

void free_plan(tsg_orth_plan p)
{
    if (!p) return;
    int cur = 0;
    const bool switched = hipGetDevice(&cur) == hipSuccess && cur != p->dev && hipSetDevice(p->dev) == hipSuccess;
    hipDeviceSynchronize();
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    if (p->cap) hipStreamDestroy(p->cap);
    hipFree(p->ws);
    hipFree(p->d_in);
    if (switched) hipSetDevice(cur);
    delete p;
}

// Resident blocks of the persistent kernel on the current device (0 on error).
int64_t resident_blocks(int* dev_out)
{
    int dev = 0, cus = 0, occ = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(&orth_persistent),
                                                         kThreads, 0);
    if (e != hipSuccess || cus < 1) return 0;
    if (dev_out) *dev_out = dev;
    return (int64_t)cus * std::max(occ, 1);
}

// Input bytes per slab under automatic sizing: the autotuner's choice
// (generated table), which TSG_ORTH_ITEM_BYTES overrides while tuning (values
// outside [64 KiB, 1 GiB] are ignored).
int64_t item_bytes()
{
    const char* v = getenv("TSG_ORTH_ITEM_BYTES");
    const long long b = v ? atoll(v) : 0;
    if (b >= (64 << 10) && b <= (1 << 30)) return (int64_t)b;
    return (tsg::kOrthItemBytes >= (64 << 10) && tsg::kOrthItemBytes <= (1 << 30)) ? tsg::kOrthItemBytes : kItemBytes;
}

hipError_t launch_setup(const tsg_orth_desc* d_in, int count, int64_t rows_fixed, int lag, int resident, void* ws,
                        const Layout& L, hipStream_t s)
{
    hipLaunchKernelGGL(orth_setup, dim3(1), dim3(kMaxCount), 0, s, d_in, count, rows_fixed, item_bytes(), lag,
                       resident, kDefaultSpin, at<Ctrl>(ws, L.ctrl), at<DevDesc>(ws, L.descs), at<unsigned>(ws, L.flags),
                       at<Item>(ws, L.items), L.max_items, L.max_parts);
    return hipGetLastError();
}

hipError_t launch_persistent(void* ws, const Layout& L, int count, int grid, hipStream_t s)
{
    unsigned* flags = at<unsigned>(ws, L.flags);
    hipLaunchKernelGGL(orth_persistent, dim3(grid), dim3(kThreads), 0, s, at<DevDesc>(ws, L.descs),
                       at<Item>(ws, L.items), at<double>(ws, L.parts), flags, flags + count, at<Ctrl>(ws, L.ctrl),
                       count);
    return hipGetLastError();
}

// Interleave lag of the queue (instances between an instance's slab items
// and its updates); TSG_ORTH_LAG overrides it for tuning.
int queue_lag(int count)
{
    const char* v = getenv("TSG_ORTH_LAG");
    const int lag = v ? atoi(v) : tsg::kOrthLag;
    return lag < 1 ? count : std::min(lag, count);
}

tsg_status fail(tsg_status st, const char* fmt, long long a = 0, long long b = 0)
{
    char buf[256];
    snprintf(buf, sizeof buf, fmt, a, b);
    return tsg::report(st, buf);
}

tsg_status read_error(Ctrl* d_ctrl)
{
    unsigned err = 0;
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(&err, &d_ctrl->err, sizeof(unsigned), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(TSG_E_HIP, "device synchronisation failed");
    if (!err) return TSG_OK;
    const unsigned zero = 0;
    if (hipMemcpy(&d_ctrl->err, &zero, sizeof(unsigned), hipMemcpyHostToDevice) != hipSuccess)
        return fail(TSG_E_HIP, "could not clear the error word");
    if (err & kErrDesc) return fail(TSG_E_ARG, "a descriptor failed the device-side checks: nothing was done");
    if (err & kErrSpace)
        return fail(TSG_E_NOMEM, "the batch does not fit the workspace (see tsg_workspace_size): nothing was done");
    return fail(TSG_E_HIP, "an update waited past the spin limit: results invalid");
}

}  // namespace

extern "C" {

tsg_status tsg_orth_plan_create(tsg_orth_plan* plan, int32_t count, const tsg_orth_desc* descs,
                                int64_t rows_per_item, void* stream)
{
    (void)stream;
    if (!plan) return fail(TSG_E_ARG, "plan is NULL");
    *plan = nullptr;
    if (!descs || count < 1) return fail(TSG_E_ARG, "need count >= 1 descriptors (count %lld)", count);
    if (count > kMaxCount) return fail(TSG_E_UNSUPPORTED, "at most %lld instances per plan", kMaxCount);
    int64_t slabs = 0, parts = 0;
    for (int i = 0; i < count; ++i) {
        const tsg_orth_desc& s = descs[i];
        if (s.K < 0 || s.M < 1 || s.N < 1) return fail(TSG_E_ARG, "instance %lld: K < 0, M < 1 or N < 1", i);
        if (s.M > kMaxM || s.N > kMaxN)
            return fail(TSG_E_UNSUPPORTED, "instance %lld: M <= 64 and N <= 16 are supported", i);
        if (s.ldv < s.M || s.ldw < s.N || s.ldc < s.N)
            return fail(TSG_E_ARG, "instance %lld: leading dimension below the width", i);
        if (!s.C || (s.K > 0 && (!s.V || !s.W))) return fail(TSG_E_ARG, "instance %lld: NULL pointer", i);
        if ((reinterpret_cast<uintptr_t>(s.V) | reinterpret_cast<uintptr_t>(s.W) |
             reinterpret_cast<uintptr_t>(s.C)) % sizeof(double))
            return fail(TSG_E_ARG, "instance %lld: pointer not aligned to 8 bytes", i);
        const int64_t R = slab_rows(s.K, s.M, s.N, s.ldv, s.ldw, rows_per_item, item_bytes());
        if (R < 1)
            return fail(TSG_E_UNSUPPORTED, "instance %lld: slab height must be in [1, %lld] for its leading dimensions",
                        i, slab_limit(s.ldv, s.ldw));
        const int64_t nslab = s.K > 0 ? (s.K + R - 1) / R : 1;
        if (nslab > ((int64_t)1 << 24)) return fail(TSG_E_UNSUPPORTED, "instance %lld: too many slabs", i);
        slabs += nslab;
        parts += nslab * s.M * s.N;
    }
    // at most four update pieces per slab
    if (5 * slabs > ((int64_t)1 << 30)) return fail(TSG_E_UNSUPPORTED, "too many work items");
    int dev = 0;
    const int64_t resident = resident_blocks(&dev);
    if (resident < 1) return fail(TSG_E_HIP, "no usable HIP device");

    tsg_orth_plan p = new (std::nothrow) tsg_orth_plan_t();
    if (!p) return fail(TSG_E_NOMEM, "host allocation failed");
    p->count = count;
    p->dev = dev;
    p->grid = (int)resident;
    p->L = make_layout(count, 5 * slabs, parts);
    if (hipMalloc(&p->ws, p->L.bytes) != hipSuccess || hipMalloc(&p->d_in, sizeof(tsg_orth_desc) * count) != hipSuccess) {
        free_plan(p);
        return fail(TSG_E_NOMEM, "device allocation of the plan failed");
    }
    const Ctrl ctrl0{0u, 0u, 0u, kDefaultSpin, 0u, {0u, 0u, 0u}};
    if (hipMemcpy(p->d_in, descs, sizeof(tsg_orth_desc) * count, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(at<Ctrl>(p->ws, p->L.ctrl), &ctrl0, sizeof(Ctrl), hipMemcpyHostToDevice) != hipSuccess ||
        launch_setup(p->d_in, count, rows_per_item, queue_lag(count), (int)resident, p->ws, p->L, nullptr) !=
            hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        free_plan(p);
        return fail(TSG_E_HIP, "upload of the plan failed");
    }
    const tsg_status st = read_error(at<Ctrl>(p->ws, p->L.ctrl));
    if (st != TSG_OK) {
        free_plan(p);
        return st;
    }
    // one launch of the persistent kernel captured on a private stream;
    // replays go to the caller's stream
    if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess ||
        hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        free_plan(p);
        return fail(TSG_E_HIP, "stream capture could not start");
    }
    const hipError_t e = launch_persistent(p->ws, p->L, count, p->grid, p->cap);
    const hipError_t e2 = hipStreamEndCapture(p->cap, &p->graph);
    if (e != hipSuccess || e2 != hipSuccess ||
        hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
        free_plan(p);
        return fail(TSG_E_HIP, "graph capture of the launch failed");
    }
    *plan = p;
    return TSG_OK;
}

tsg_status tsg_orth_plan_launch(tsg_orth_plan plan, void* stream)
{
    if (!plan) return fail(TSG_E_ARG, "plan is NULL");
    const hipError_t e = hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? TSG_OK : fail(TSG_E_HIP, "hipGraphLaunch failed (%lld)", (long long)e);
}

tsg_status tsg_orth_plan_run(tsg_orth_plan plan, void* stream)
{
    if (!plan) return fail(TSG_E_ARG, "plan is NULL");
    const hipError_t e = launch_persistent(plan->ws, plan->L, plan->count, plan->grid, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? TSG_OK : fail(TSG_E_HIP, "kernel launch failed (%lld)", (long long)e);
}

tsg_status tsg_orth_plan_check(tsg_orth_plan plan)
{
    if (!plan) return fail(TSG_E_ARG, "plan is NULL");
    return read_error(at<Ctrl>(plan->ws, plan->L.ctrl));
}

tsg_status tsg_orth_plan_set_spin_limit(tsg_orth_plan plan, uint32_t limit)
{
    if (!plan) return fail(TSG_E_ARG, "plan is NULL");
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(&at<Ctrl>(plan->ws, plan->L.ctrl)->spin, &limit, sizeof(unsigned), hipMemcpyHostToDevice) !=
            hipSuccess)
        return fail(TSG_E_HIP, "could not set the spin limit");
    return TSG_OK;
}

void tsg_orth_plan_destroy(tsg_orth_plan plan) { free_plan(plan); }

tsg_status tsg_orth_batched(const tsg_orth_desc* d_descs, int32_t count, void* workspace, size_t ws_bytes,
                            void* stream)
{
    if (!d_descs || !workspace) return fail(TSG_E_ARG, "descriptors and workspace must not be NULL");
    if (count < 1) return fail(TSG_E_ARG, "need count >= 1 descriptors (count %lld)", count);
    if (count > kMaxCount) return fail(TSG_E_UNSUPPORTED, "at most %lld instances per call", kMaxCount);
    if (reinterpret_cast<uintptr_t>(workspace) % 256 || reinterpret_cast<uintptr_t>(d_descs) % 8)
        return fail(TSG_E_ARG, "workspace must be 256-byte and descriptors 8-byte aligned");
    const Layout L0 = make_layout(count, kItemsPerInstance * count, 0);
    if (ws_bytes < L0.bytes)
        return fail(TSG_E_ARG, "workspace of %lld bytes is below the %lld this count needs", (long long)ws_bytes,
                    (long long)L0.bytes);
    const Layout L = make_layout(count, kItemsPerInstance * count, (int64_t)((ws_bytes - L0.parts) / sizeof(double)));
    const int64_t resident = resident_blocks(nullptr);
    if (resident < 1) return fail(TSG_E_HIP, "no usable HIP device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_setup(d_descs, count, 0, queue_lag(count), (int)resident, workspace, L, s);
    if (e == hipSuccess) e = launch_persistent(workspace, L, count, (int)resident, s);
    return e == hipSuccess ? TSG_OK : fail(TSG_E_HIP, "kernel launch failed (%lld)", (long long)e);
}

tsg_status tsg_orth_batched_check(void* workspace)
{
    if (!workspace) return fail(TSG_E_ARG, "workspace is NULL");
    return read_error(at<Ctrl>(workspace, 0));
}

}  // extern "C"

namespace tsg {
// Workspace bytes of tsg_orth_batched for `count` instances none of which
// exceeds K rows, M columns of V or N columns of W (contiguous rows; slabs as
// tsg_orth_batched cuts them).  0 if the shape is outside the supported range.
size_t orth_workspace_size(int64_t K, int32_t M, int32_t N, int32_t count)
{
    if (K < 0 || M < 1 || N < 1 || M > kMaxM || N > kMaxN || count < 1 || count > kMaxCount) return 0;
    const int64_t R = slab_rows(K, M, N, M, N, 0, item_bytes());
    const int64_t nslab = K > 0 && R > 0 ? (K + R - 1) / R : 1;
    return make_layout(count, kItemsPerInstance * count, (int64_t)count * nslab * M * N).bytes;
}
}  // namespace tsg
