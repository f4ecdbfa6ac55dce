// batch_cg.hpp -- many independent CG solves advanced by one persistent
// kernel, one work-group per system.
#pragma once

#include "common.hpp"

namespace spx {

constexpr int kBatchThreads = 512;

enum SlotStatus : int32_t {
    kSlotRunning = 0,
    kSlotConverged = 1,
    kSlotBreakdown = 2,
    kSlotNonfinite = 3,
    kSlotMaxit = 4,
    kSlotEmpty = 5,
};

// Krylov method of a slot.
enum SlotSolver : int32_t {
    kSlotCg = 0,        // CG (symmetric positive definite systems)
    kSlotBicgstab = 1,  // BiCGSTAB (nonsymmetric systems)
};

// Device descriptor of one system (all pointers are device memory).
struct BatchSlot {
    const int32_t *rowptr;
    const int32_t *col;
    const double *val;
    const double *b;
    double *x, *r, *p, *q;  // BiCGSTAB: q holds v = A p
    double *rh, *t;         // BiCGSTAB only: shadow residual, t = A s
    int32_t n;
    int32_t sub;       // lanes per row in the product (power of two <= 64)
    int32_t status;    // SlotStatus
    int32_t started;   // 0 until r = b - A x0, p = r, rho are set up
    double tol2, bb, rho, rr;
    int32_t iters, maxit, budget, spmv;  // budget: iterations allowed in this launch
    double relres_true;
    int32_t solver;  // SlotSolver
    int32_t first;   // BiCGSTAB: the next step starts a (re)started recurrence (p = r)
    double rho0, alpha, omega;  // BiCGSTAB scalars carried between steps
};

// Lanes per row for a mean row length (smallest power of two >= mean, <= 16).
inline int32_t batch_sub_for(int64_t n, int64_t nnz)
{
    const double mean = n > 0 ? (double)nnz / (double)n : 1.0;
    int32_t s = 1;
    while (s < 16 && s < mean) s <<= 1;
    return s;
}

// Lanes per row in the one-group kernel: batch_sub_for divided by
// 2^kNarrowSubShift (more rows per pass, fewer dependent passes per product).
constexpr int kNarrowSubShift = 3;
inline int32_t narrow_sub_for(int64_t n, int64_t nnz)
{
    const int32_t s = batch_sub_for(n, nnz) >> kNarrowSubShift;
    return s > 0 ? s : 1;
}

// ---------------------------------------------------------------- wide systems
// Systems too large for one work-group are advanced together by a sequence of
// grid-wide phases. Each wide system is cut into virtual blocks of kWideRows
// rows; every phase launches a fixed grid that strides over the virtual
// blocks of all wide systems (vb_slot maps a virtual block to its system).
// A system's partition, partial sums and their fixed summation order depend
// only on its own n, so its iterates are bitwise the same alone or in any mix.
constexpr int kWideThreads = 256;  // vector phase
constexpr int kWideRows = 1024;    // rows per virtual block of the vector phase

enum WideMode : int32_t {
    kWideInit = 0,   // r = b (x0 = 0)
    kWideRun = 1,    // one CG step per product + vector phase pair
    kWideCheck = 2,  // true residual b - A x
    kWideDone = 3,
};

// Written by the host when the system is admitted. The product phase runs
// the load-balanced CSR tile kernel over the system's ntiles tiles (its
// partition in csr_part), one or two partials per tile in part_a (rows of
// ntiles); the vector phase works on nvb blocks of kWideRows rows, one or
// two partials each, into one half of part while it reads the other half
// (the halves alternate; each half holds two rows of nvb).
struct WideSlot {
    const int32_t *rowptr;
    const int32_t *col;
    const double *val;
    const double *b;
    double *x, *r, *p, *w, *s;  // CG: w = A r, s = A p; BiCGSTAB: w holds v = A p
    double *rh, *t;             // BiCGSTAB only: shadow residual, t = A s
    double *part;               // 4 * nvb partial sums of the vector phase
    double *part_a;             // 2 * ntiles partial sums of the product phase
    const int32_t *csr_part;    // tile partition of the product
    int64_t nnz;
    int32_t n, nvb, ntiles, maxit;
    double tol2;
    int32_t solver;  // SlotSolver
    int32_t pad;
};

// Written by the device (the vector phase's commit) and once at admission
// (zero but mode = kWideInit).
struct WideState {
    int32_t mode, status, iters, spmv;  // status: SlotStatus
    double rho, bb, rr, relres_true;    // CG: rho = r.r of the last step; BiCGSTAB: rho = r_hat.r
    double alpha;                       // the last step length
    int32_t restart;  // CG: 1 = the next step restarts the recurrences (p = r, s = w)
    int32_t truer;    // r.r about to be summed is of r = b (2), of a true residual (1), recursive (0)
    int32_t phase;    // which half of part the next vector phase reads
    int32_t bphase;   // BiCGSTAB: which part of a step the next product + vector pair runs
    double rho0, omega;  // BiCGSTAB: the previous r_hat.r, the last omega
};

// Header of the virtual-block maps, device memory: {total virtual row blocks,
// number of listed systems, total product tiles}.
struct WideMap {
    int32_t total_vb;
    int32_t nlisted;
    int32_t total_ta;
    int32_t pad;
};

inline int32_t wide_nvb(int64_t n) { return (int32_t)((n + kWideRows - 1) / kWideRows); }

// One iteration (two launches: the product with its r.w partials, then the
// vector phase with the scalar recurrences and the commit) for all listed
// wide systems, reading the systems' state from st and writing it to st_next
// (callers alternate two buffers, so an even number of iterations leaves the
// state in the first). grid: physical blocks of every phase. ta_slot /
// ta_local map product tiles, vb_slot / vb_local vector blocks to (system,
// local index).
spx_status wide_iteration_launch(const WideSlot *slots, const WideState *st, WideState *st_next,
                                 const WideMap *map, const int32_t *vb_slot, const int32_t *vb_local,
                                 const int32_t *ta_slot, const int32_t *ta_local, int grid, hipStream_t stream);

// Systems of at most kBatchSmallRows rows are advanced by their own kernel
// (batch_small_launch; one 512-thread work-group per system with p in LDS
// and x, r in registers while it runs), the others by batch_cg_launch. The
// split depends only on a system's own n, so its iterates stay bitwise the
// same alone or in any mix.
constexpr int kBatchSmallRows = 4096;
// Systems of at most kBatchLdsRows rows keep p in LDS in the general
// one-group kernel (128 KB).
constexpr int kBatchLdsRows = 16384;

// Advance slots[0..nslots) by at most slot.budget iterations each (or to
// convergence); work-groups take slots from *counter, which must be 0 at
// launch (batch_reset does that). grid: number of resident work-groups.
// batch_cg_launch runs every BiCGSTAB slot and the CG slots of more than
// kBatchSmallRows rows, and uses counter[0]; batch_small_launch takes the
// other CG slots and uses counter[1].
spx_status batch_cg_launch(BatchSlot *slots, int32_t nslots, int32_t *counter, int64_t grid, hipStream_t stream);
spx_status batch_small_launch(BatchSlot *slots, int32_t nslots, int32_t *counter, int64_t grid, hipStream_t stream);
// Zeroes counter[0] and counter[1].
spx_status batch_reset_launch(int32_t *counter, hipStream_t stream);
int64_t batch_resident_groups();
int64_t batch_small_resident_groups();

}  // namespace spx
