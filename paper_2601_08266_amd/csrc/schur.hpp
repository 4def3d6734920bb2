// Internal declarations of the Schur-complement block preconditioner.
#pragma once

#include "fgmres.hpp"

namespace fsi {

constexpr int SC_MAX_LEVELS = 16;
constexpr int64_t SC_COARSE_MAX_NODES = 64;    // coarsen while a level holds more nodes
constexpr int64_t SC_DIRECT_MAX_NODES = 1000;  // largest coarsest level (dense inverse)

struct ScLevel {
    int nc[3];        // lattice cells per axis
    int nn[3];        // nodes per axis
    int64_t N, C;     // nodes, cells
    double l[3];      // lattice-cell sides
    double kc[8];     // box stiffness entry by axis-difference pattern (bit d: differs along d)
    size_t a64, a32, dm, x0, x1, b, r;   // byte offsets in the preconditioner object
};

struct ScPlan {
    int L;
    ScLevel lv[SC_MAX_LEVELS];
    size_t finv64, finv32, kinv64, kinv32, yt, mr_r, mr_x, mr_q, mr_part, cnt, total;
};

// Levels and layout of the preconditioner object for a grid (a pure function of the grid).
int sc_plan(const Geo &g, ScPlan &p);

// Builds the preconditioner object pc from the FP64 problem data and the nodal 4x4 blocks
// (the raw blocks of the block-Jacobi setup).  Synchronises the stream.
int schur_setup(const Geo &g, const fsi_vms_params &prm, const double *a, const double *s,
                const uint32_t *mask, const double *gram, const int32_t *occ_index,
                const double *blocks, void *pc, hipStream_t st);

// z = P^{-1} v ([4][N]); mode 1: block diagonal, 2: upper block triangular (uses J, in the
// precision `inner`, with workspace jws); vel_steps minimal-residual steps on the velocity block
// (0: the nodal block inverses alone; > 0 uses J).  z is in the precision `inner`; v is FP64
// when v_f64, else in `inner`.
int schur_apply(const Geo &g, fsi_dtype inner, bool v_f64, int mode, int vel_steps, void *pc, const void *v,
                void *z, const JacobianCall *J, void *jws, hipStream_t st);

}  // namespace fsi
