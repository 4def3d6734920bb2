// Internal declarations of the FGMRES driver.
#pragma once

#include <functional>

#include "kernels.hpp"

namespace fsi {

// A bound Jacobian apply y = J x (x, y in the call's precision) with its workspace.
struct JacobianCall {
    std::function<int(const void *x, void *y, void *ws, hipStream_t st)> apply;
    // optional: velocity rows of the operator on one input block, blk = 1: (x_u, 0), blk = 2:
    // (0, x_p) (the other block of x is not read; the pressure part of y is not written).  Empty
    // where not available: callers then apply the whole operator to a zero-padded input.
    std::function<int(int blk, const void *x, void *y, void *ws, hipStream_t st)> block;
};

// A bound preconditioner z = P^{-1} v: v is a [4][N] basis vector in the basis precision (FP64,
// or FP32 with opts.basis = FSI_F32), z is written in the inner precision; jws is the Jacobian
// workspace (free while the preconditioner runs).
struct Precond {
    std::function<int(const void *v, void *z, void *jws, hipStream_t st)> apply;
};

size_t fgmres_workspace_bytes(int64_t ndof, int restart, fsi_dtype inner, fsi_dtype basis, size_t jws_bytes);
// x_zero: the caller guarantees x = 0 on entry (the first cycle's residual is then b itself)
int fgmres_solve(const Geo &g, const JacobianCall &J64, const JacobianCall *J32, const Precond *pc,
                 const double *b, double *x, const fsi_solve_opts &o, fsi_solve_stats *stats,
                 void *ws, size_t jws_bytes, hipStream_t st, bool x_zero = false);

}  // namespace fsi
