// Internal launcher declarations (host side), one namespace for the library.
#pragma once

#include "common.hpp"
#include "solid.hpp"

namespace fsi {

// Pre-computed constants of the Oseen-VMS operator in the compute precision.
template <typename T>
struct VmsConst {
    T c_m, nu, K1;     // K1 = C_T/dt^2 + C_I nu^2 G:G
    T ih[3];           // 1/h
    T ih2[3];          // 1/h^2
    T inv_trG;         // 1/tr G
    T detJ;            // hx hy hz
    T nu_hh[3][3];     // nu / (h_i h_k): viscous fluxes from reference-cell derivatives
    int32_t visc_strong;
    int32_t has_s;
};

template <typename T>
VmsConst<T> make_vms_const(const Geo &g, const fsi_vms_params &prm, bool has_s);

// ---- Q1 operator: brick partials + node gather ----
// one workgroup (4 wavefronts) per brick of 8x8x4 cells (one cell per lane)
constexpr int Q1_BX = 8, Q1_BY = 8, Q1_BZ = 4;
constexpr int Q1_NT = Q1_BX * Q1_BY * Q1_BZ;
constexpr int Q1_NL = (Q1_BX + 1) * (Q1_BY + 1) * (Q1_BZ + 1);

// ---- Q2 operator ----
constexpr int Q2_BX = 4, Q2_BY = 4, Q2_BZ = 4;
constexpr int Q2_NL = (2 * Q2_BX + 1) * (2 * Q2_BY + 1) * (2 * Q2_BZ + 1);

// How the node gather finishes each row.
template <typename T>
struct GatherOpts {
    const T *csum = nullptr;          // per-occupied-cell DLM corner sums (pointwise path)
    const int32_t *occ_index = nullptr;
    const T *sub3 = nullptr;          // [3][N] subtracted from the momentum rows
    const T *gD = nullptr;            // [3][N]: Dirichlet rows become x - gD instead of x
    int rows = 4;                     // 3: velocity rows only (three partial fields)
};

// Brick partial sums: bricks whose indices have equal parities (mod 2 per axis) share no
// node, so each of the 8 classes owns one [4][nn2][nn1][lx] array.  Along x a class only
// holds its own bricks' nodes, packed: brick b (span S = P * bricks cells) keeps its S + 1
// nodes at slot (b / 2) (S + 1) + (node x - S b), so the rows carry no holes.
struct PartIndex {
    int64_t lx, plane, field, cls;
    int span;   // nodes per brick along x minus one (P * BX)
    __host__ __device__ PartIndex(const int32_t nn[3], int nbx, int span_) : span(span_)
    {
        lx = (int64_t)(span_ + 1) * ((nbx + 1) / 2);
        plane = lx * nn[1];
        field = plane * nn[2];
        cls = 4 * field;
    }
    // offset of field 0 of node (gx, gy, gz) in the array of x-brick bxb's class (bxb holds gx)
    __host__ __device__ int64_t at(int cls_id, int bxb, int gx, int gy, int gz) const
    {
        return cls_id * cls + (int64_t)gz * plane + (int64_t)gy * lx + (int64_t)(bxb >> 1) * (span + 1) +
               (gx - span * bxb);
    }
};

struct BrickLayout {
    int bx, by, bz;   // cells per brick
    int nbx, nby, nbz;
    int64_t nb;
    int nl;           // local nodes per brick
};

BrickLayout brick_layout(const Geo &g);
size_t vms_workspace_bytes(const Geo &g, fsi_dtype dt);

// Point-table view used by the DLM kernels of the Jacobian.
struct DlmView {
    int64_t m;
    const int32_t *cell;
    const void *xi;
    const int32_t *perm;
    const int32_t *occ_cell;
    const int32_t *occ_start;
    int64_t n_occ;
    const int32_t *occ_index;   // [E] occupied index per cell or -1
    const void *kappa;
    const void *gram;           // [n_occ][nen][nen] or nullptr
    // hyperelastic solid block in place of the per-point kappa (kappa and gram unused):
    // the points are the solid's nodes, y += B^T (c_M M + c_K K(U) - c_V K_v(U)) B x_u
    const fsi_solid *solid = nullptr;
    const double *solid_U = nullptr;
    SolidCoefs solid_c{};
};

// y = A x (+ B^T kappa B x_u if dlm != nullptr), Dirichlet rows -> x.
int launch_vms_apply(const Geo &g, const fsi_vms_params &prm, fsi_dtype dt, const void *a,
                     const void *s, const uint32_t *mask, const void *x, void *y,
                     const DlmView *dlm, void *ws, size_t ws_bytes, hipStream_t st);

// Velocity rows of the same apply for one input block: blk = 1: y_u = [J (x_u, 0)]_u (x_p not
// read), blk = 2: y_u = [J (0, x_p)]_u (x_u not read, Dirichlet rows 0).  The pressure part of y
// is not written.  Q1 only: FSI_ERR_UNSUPPORTED, with nothing launched, for Q2.
int launch_vms_apply_block(const Geo &g, const fsi_vms_params &prm, fsi_dtype dt, int blk, const void *a,
                           const void *s, const uint32_t *mask, const void *x, void *y, const DlmView *dlm,
                           void *ws, hipStream_t st);

size_t dlm_csum_bytes(const Geo &g, int64_t n_occ, fsi_dtype dt);

template <typename T>
int launch_q1_cells(const Geo &g, const VmsConst<T> &k, const T *x, const T *a, const T *s,
                    const uint32_t *mask, const T *gram, const int32_t *occ_index, T *part,
                    const BrickLayout &bl, hipStream_t st, bool resid);
// Velocity rows of the Q1 apply on (x_u, 0) (blk = 1) or (0, x_p) (blk = 2): brick partials of
// the three momentum fields (gather with rows = 3).
template <typename T>
int launch_q1_block(const Geo &g, const VmsConst<T> &k, int blk, const T *x, const T *a, const T *s,
                    const uint32_t *mask, const T *gram, const int32_t *occ_index, T *part,
                    const BrickLayout &bl, hipStream_t st);
// Full-tangent correction (Q1): adds to the brick partials of a Picard apply with a = u the
// derivative terms that the Picard operator drops, for state x = (u, p), source f and
// velocity direction dv (Dirichlet entries of dv ignored).
template <typename T>
int launch_q1_tangent(const Geo &g, const VmsConst<T> &k, const T *x, const T *f, const T *s,
                      const uint32_t *mask, const T *dv, T *part, const BrickLayout &bl, hipStream_t st);
// The whole full Newton tangent (Q1) in one pass of cells: state x = (u, p), source f,
// direction v = (dv, dp) (Dirichlet entries of dv ignored), per-cell DLM blocks gram (or NULL).
template <typename T>
int launch_q1_tangent_fused(const Geo &g, const VmsConst<T> &k, const T *x, const T *f, const T *s,
                            const uint32_t *mask, const T *gram, const int32_t *occ_index, const T *v,
                            T *part, const BrickLayout &bl, hipStream_t st);
template <typename T>
int launch_q2_cells(const Geo &g, const VmsConst<T> &k, const T *x, const T *a, const T *s,
                    const uint32_t *mask, const T *gram, const int32_t *occ_index, T *part,
                    const BrickLayout &bl, hipStream_t st, bool resid = false);
template <typename T, int P, int BX, int BY, int BZ>
int launch_gather(const Geo &g, const T *part, const BrickLayout &bl, const T *x,
                  const uint32_t *mask, T *y, const GatherOpts<T> &o, hipStream_t st);

// Nonlinear residual of one implicit step (Q1 or Q2):
//   R = A(a = u) x - F(f) + B^T kappa B u - lamg,   Dirichlet rows R = u - gD
int launch_vms_residual(const Geo &g, const fsi_vms_params &prm, fsi_dtype dt, const void *s,
                        const uint32_t *mask, const void *gD, const void *x, const void *f,
                        const DlmView *dlm, const void *lamg, void *R, void *ws, hipStream_t st);

// Full Newton tangent of that residual times v (Q1): the Picard apply with a = u plus the
// correction above; Dirichlet rows y = v.  x: state [4][N], f: source [3][N], precision dt.
int launch_tangent_apply(const Geo &g, const fsi_vms_params &prm, fsi_dtype dt, const void *s,
                         const uint32_t *mask, const void *x, const void *f, const DlmView *dlm,
                         const void *v, void *y, void *ws, hipStream_t st);

}  // namespace fsi
