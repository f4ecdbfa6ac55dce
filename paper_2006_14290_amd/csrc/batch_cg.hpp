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

// Device descriptor of one system (all pointers are device memory).
struct BatchSlot {
    const int32_t *rowptr;
    const int32_t *col;
    const double *val;
    const double *b;
    double *x, *r, *p, *q;
    int32_t n;
    int32_t sub;       // lanes per row in the product (power of two <= 64)
    int32_t status;    // SlotStatus
    int32_t started;   // 0 until r = b - A x0, p = r, rho are set up
    double tol2, bb, rho, rr;
    int32_t iters, maxit, budget, spmv;  // budget: iterations allowed in this launch
    double relres_true;
};

// Lanes per row for a mean row length (smallest power of two >= mean, <= 16).
inline int32_t batch_sub_for(int64_t n, int64_t nnz)
{
    const double mean = n > 0 ? (double)nnz / (double)n : 1.0;
    int32_t s = 1;
    while (s < 16 && s < mean) s <<= 1;
    return s;
}

// Advance slots[0..nslots) by at most slot.budget CG iterations each (or to
// convergence); work-groups take slots from *counter, which must be 0 at
// launch (batch_reset does that). grid: number of resident work-groups.
spx_status batch_cg_launch(BatchSlot *slots, int32_t nslots, int32_t *counter, int64_t grid, hipStream_t stream);
spx_status batch_reset_launch(int32_t *counter, hipStream_t stream);
int64_t batch_resident_groups();

}  // namespace spx
