// tsg_registry.hpp -- host-side description of the generated kernel variants.
// The code generator emits one Variant record (and one launcher) per
// instantiated kernel; the runtime picks a record for each call.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsg {

// Arguments of one launch.  For TSMTTSM, X/ldx is B and Y/ldy is C; for TSMM,
// X/ldx is C and Y/ldy is B.
struct Launch {
    hipStream_t stream;
    int grid;
    int64_t K;
    int M, N;
    int conj;
    int opc;  // TSMM small operand: 0 C, 1 C^T, 2 C^H
    const void* A;
    int64_t lda;
    const void* X;
    int64_t ldx;
    void* Y;
    int64_t ldy;
    double alpha, beta;
    double* ws;  // TSMTTSM: one slot of M*N (x2 complex) doubles per block
};

enum OpKind { OP_TSMTTSM = 0, OP_TSMM = 1 };

struct Variant {
    int op;             // OpKind
    int dt;             // tsg_dtype of the tall matrices
    int M, N;           // exact widths served, or 0 for a run-time-width variant
    int maxM, maxN;     // largest widths served (run-time-width variants)
    int pairA;          // needs 16-byte paired loads of A (even lda, aligned A)
    int pairX;          // TSMTTSM: paired loads of B; TSMM: paired stores of B
    int evenW;          // run-time-width variant that needs even widths (paired access)
    int threads;        // block size
    int rows_per_tile;  // rows consumed by one block per grid-stride iteration (for P = 1)
    int pack;           // row packing: 0 none, 1 P = 16 / max(M, N) (TSMTTSM), 2 P = 16 / N (TSMM)
    int flatA;          // reads the tall operands as runs of rows: needs lda == M (TSMTTSM: and ldb == N)
    int readB;          // TSMM reading the old B with A (serves only calls with beta != 0)
    int align16;        // needs A and X 16-byte aligned (direct 16-byte loads into LDS)
    const char* name;
    const void* (*kernel)(); // device function, for occupancy queries
    void (*launch)(const Launch&);
};

extern const Variant kVariants[];
extern const int kNumVariants;

// Batched orthogonalisation parameters chosen by the autotuner (generated):
// input bytes per slab under automatic sizing, and the queue interleave
// (instances between an instance's slab items and its update items; 0: every
// slab item before any update item).
extern const int64_t kOrthItemBytes;
extern const int kOrthLag;

}  // namespace tsg
