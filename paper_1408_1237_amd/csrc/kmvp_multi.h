// Arguments of the matrix-core multi-RHS product (kmvp_multi.hip), shared with
// the batched solver.
#pragma once

#include "krr_internal.h"

namespace krr {

struct MArgs {
    int64_t n, n_pad;
    int ntiles, nrowblocks, splits, tps, nrb;  // nrb: blocks of 16 right-hand sides
    const double *anchor;
    const double *tile_r2;
    const double *tile_nj;
    const float *tile_far;  // split-f16 exponent (FP32 / BF16): per-tile far threshold on |t|^2
    const void *slots;      // split-f16 exponent: source slot octets of the product's precision
    const void *off;
    const void *qwt;  // Q' as [nrb][n_pad][16]
    void *parts;      // [splits][nrb][n_pad][16]
};

// One work item of a batched product: (system, row tile, column chunk, RHS block).
struct MItem {
    int sys, bx, by, rbk;
};

// One system of a batched product: its product arguments, the offset of its
// block in the concatenated vectors, its weights and its two shifts (delta for
// the inner products, gamma for the outer ones).
struct MSysB {
    MArgs a;
    int64_t base;
    const void *w;
    double shift_in, shift_out;
    int col0;  // index of the system's first column in the solver's column arrays
};

// Which columns of a batched product are needed: column c is live when
// a[c] != 0 and b[c] != 0 (a null array counts as all ones).  A block of 16
// right-hand sides without a live column is skipped, and the outputs of dead
// columns are left as they were (their consumers skip them too).
struct ColGate {
    const int *a = nullptr;
    const int *b = nullptr;
};

// A batched product over the systems of one compiled dimension and one
// precision: device arrays of systems and work items, sizes for the grids.
struct BatchedProduct {
    int dpad = 0, prec = 0, nsys = 0, nrhs = 0, nitems = 0;
    MSysB *d_sys = nullptr;
    MItem *d_items = nullptr;
    int64_t max_elems = 0;  // max over systems of n_pad * 16 * nrb
    double pairs = 0.0;     // sum over systems of n^2
};

// Scratch of one system of a batched product whose work items cover at least
// min_tps column tiles each (partial sums of every column chunk, and Q').
size_t batched_product_scratch_bytes(const Prepared &P, int nrhs, int min_tps);
// The system's product arguments with tps column tiles per work item (tps >=
// the min_tps its scratch was sized for).
void fill_msys(MSysB &m, const Prepared &P, int prec, int nrhs, void *scratch, int64_t base, double shift_in,
               double shift_out, int tps);
// Y = K_hat Q + shift Q for every system of bp (inner != 0: shift_in), on the
// live columns of gate.
hipError_t batched_product(const BatchedProduct &bp, const void *Qall, void *Yall, int inner, ColGate gate,
                           hipStream_t s);

}  // namespace krr
