// C ABI entry points: argument validation, workspace layout and dispatch.
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "bjacobi.hpp"
#include "schur.hpp"
#include "dlm.hpp"
#include "fgmres.hpp"
#include "kernels.hpp"
#include "krylov.hpp"
#include "newton.hpp"
#include "nn.hpp"

namespace fsi {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

int check_grid(const fsi_grid *g)
{
    FSI_CHECK_ARG(g != nullptr, "grid is NULL");
    FSI_CHECK_ARG(g->order == 1 || g->order == 2, "order must be 1 or 2 (got %d)", g->order);
    int64_t N = 1, E = 1;
    for (int d = 0; d < 3; ++d) {
        FSI_CHECK_ARG(g->n[d] >= 1, "n[%d] must be >= 1", d);
        FSI_CHECK_ARG(std::isfinite(g->h[d]) && g->h[d] > 0.0, "h[%d] must be finite and > 0", d);
        FSI_CHECK_ARG(std::isfinite(g->x0[d]), "x0[%d] must be finite", d);
        N *= (int64_t)g->order * g->n[d] + 1;
        E *= g->n[d];
    }
    FSI_CHECK_ARG(E < ((int64_t)1 << 31) - 1, "too many cells (%lld)", (long long)E);
    FSI_CHECK_ARG(N < ((int64_t)1 << 40), "too many nodes");
    return FSI_OK;
}

static int check_params(const fsi_vms_params *p)
{
    FSI_CHECK_ARG(p != nullptr, "params are NULL");
    FSI_CHECK_ARG(std::isfinite(p->nu) && p->nu >= 0.0, "nu must be finite and >= 0");
    FSI_CHECK_ARG(std::isfinite(p->c_m) && p->c_m >= 0.0, "c_m must be finite and >= 0");
    FSI_CHECK_ARG(std::isfinite(p->dt) && p->dt > 0.0, "dt must be finite and > 0");
    FSI_CHECK_ARG(std::isfinite(p->C_T) && p->C_T >= 0.0, "C_T must be finite and >= 0");
    FSI_CHECK_ARG(std::isfinite(p->C_I) && p->C_I >= 0.0, "C_I must be finite and >= 0");
    return FSI_OK;
}

template <typename T>
VmsConst<T> make_vms_const(const Geo &g, const fsi_vms_params &prm, bool has_s)
{
    VmsConst<T> k;
    double GG = 0.0, trG = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double ih2 = 1.0 / (g.h[d] * g.h[d]);
        GG += ih2 * ih2;
        trG += ih2;
        k.ih[d] = (T)(1.0 / g.h[d]);
        k.ih2[d] = (T)ih2;
    }
    k.c_m = (T)prm.c_m;
    k.nu = (T)prm.nu;
    k.K1 = (T)(prm.C_T / (prm.dt * prm.dt) + prm.C_I * prm.nu * prm.nu * GG);
    k.inv_trG = (T)(1.0 / trG);
    k.detJ = (T)(g.h[0] * g.h[1] * g.h[2]);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) k.nu_hh[i][j] = (T)(prm.nu / (g.h[i] * g.h[j]));
    k.visc_strong = prm.visc_strong ? 1 : 0;
    k.has_s = has_s ? 1 : 0;
    return k;
}
template VmsConst<double> make_vms_const<double>(const Geo &, const fsi_vms_params &, bool);
template VmsConst<float> make_vms_const<float>(const Geo &, const fsi_vms_params &, bool);

BrickLayout brick_layout(const Geo &g)
{
    BrickLayout b;
    if (g.p == 1) {
        b.bx = Q1_BX; b.by = Q1_BY; b.bz = Q1_BZ; b.nl = Q1_NL;
    } else {
        b.bx = Q2_BX; b.by = Q2_BY; b.bz = Q2_BZ; b.nl = Q2_NL;
    }
    b.nbx = (g.n[0] + b.bx - 1) / b.bx;
    b.nby = (g.n[1] + b.by - 1) / b.by;
    b.nbz = (g.n[2] + b.bz - 1) / b.bz;
    b.nb = (int64_t)b.nbx * b.nby * b.nbz;
    return b;
}

size_t vms_workspace_bytes(const Geo &g, fsi_dtype dt)
{
    // brick partial sums: one [4][nn2][nn1][lx] array per brick parity class (8)
    const BrickLayout b = brick_layout(g);
    const PartIndex pi(g.nn, b.nbx, g.p * b.bx);
    return align_up((size_t)8 * (size_t)pi.cls * (dt == FSI_F64 ? 8 : 4));
}

// tstate / tsrc (Q1 only): apply the full Newton tangent at the state tstate = (u, p) with
// source tsrc instead (a must then be tstate's velocity): the Picard cells and the tangent
// correction (one merged pass in FP32, two passes into the same brick partials in FP64), then
// the node gather.
template <typename T>
static int vms_apply_t(const Geo &g, const fsi_vms_params &prm, const T *a, const T *s,
                       const uint32_t *mask, const T *x, T *y, const DlmView *dlm, void *ws,
                       hipStream_t st, const T *tstate = nullptr, const T *tsrc = nullptr, int blk = 0)
{
    // blk: 0 the whole apply; 1, 2 the velocity rows on (x_u, 0) / (0, x_p) (Q1, Picard form)
    if (blk != 0 && (g.p != 1 || tstate != nullptr)) return FSI_ERR_UNSUPPORTED;
    // on (0, x_p) the DLM block (a function of the velocity only) adds nothing
    if (blk == 2) dlm = nullptr;
    const BrickLayout bl = brick_layout(g);
    const VmsConst<T> k = make_vms_const<T>(g, prm, s != nullptr);
    T *part = reinterpret_cast<T *>(ws);
    const size_t vbytes = vms_workspace_bytes(g, sizeof(T) == 8 ? FSI_F64 : FSI_F32);
    T *csum = nullptr;
    // DLM block: per-cell blocks folded into the cell kernel when available
    const bool use_gram = dlm != nullptr && dlm->n_occ > 0 && dlm->gram != nullptr && dlm->solid == nullptr;
    const T *gram = use_gram ? reinterpret_cast<const T *>(dlm->gram) : nullptr;
    const int32_t *gidx = use_gram ? dlm->occ_index : nullptr;
    int rc = FSI_OK;
    if constexpr (sizeof(T) == 4) {
        // FP32: the Picard operator and the correction in one pass of cells (162 VGPRs, 3 waves
        // per SIMD); in FP64 the merged cell would need 388 registers (1 wave), so there the
        // correction is a second pass added to the Picard partials
        if (tstate != nullptr)
            rc = launch_q1_tangent_fused<T>(g, k, tstate, tsrc, s, mask, gram, gidx, x, part, bl, st);
    }
    if (blk != 0) {
        rc = launch_q1_block<T>(g, k, blk, x, a, s, mask, gram, gidx, part, bl, st);
    } else if (tstate == nullptr || sizeof(T) == 8) {
        if (g.p == 1)
            rc = launch_q1_cells<T>(g, k, x, a, s, mask, gram, gidx, part, bl, st, false);
        else
            rc = launch_q2_cells<T>(g, k, x, a, s, mask, gram, gidx, part, bl, st);
        if (rc) return rc;
        if (tstate != nullptr) rc = launch_q1_tangent<T>(g, k, tstate, tsrc, s, mask, x, part, bl, st);
    }
    if (rc) return rc;
    const fsi_dtype dt = sizeof(T) == 8 ? FSI_F64 : FSI_F32;
    if (dlm != nullptr && dlm->n_occ > 0 && dlm->solid != nullptr) {
        // solid block: u_s = B x (Dirichlet-masked), l_s = K_s u_s at the solid nodes, then the
        // corner sums of B^T l_s, added by the node gather before the Dirichlet rows
        char *w = reinterpret_cast<char *>(ws) + vbytes;
        csum = reinterpret_cast<T *>(w);
        w += dlm_csum_bytes(g, dlm->n_occ, dt);
        T *us = reinterpret_cast<T *>(w);
        w += align_up((size_t)3 * dlm->m * sizeof(T));
        T *ls = reinterpret_cast<T *>(w);
        w += align_up((size_t)3 * dlm->m * sizeof(T));
        rc = launch_dlm_B(g, dt, dlm->m, dlm->cell, dlm->xi, x, mask, us, st);
        if (rc) return rc;
        rc = launch_solid_apply(solid_view(*dlm->solid), dt, dlm->solid_U, dlm->solid_c, us, ls, w, st);
        if (rc) return rc;
        rc = launch_dlm_cell_reduce(g, dt, false, dlm->m, dlm->n_occ, dlm->occ_cell, dlm->occ_start,
                                    dlm->perm, dlm->xi, nullptr, ls, nullptr, csum, st);
        if (rc) return rc;
    } else if (dlm != nullptr && dlm->n_occ > 0 && !use_gram) {
        csum = reinterpret_cast<T *>(reinterpret_cast<char *>(ws) + vbytes);
        rc = launch_dlm_cell_reduce(g, dt, true, dlm->m, dlm->n_occ,
                                    dlm->occ_cell, dlm->occ_start, dlm->perm, dlm->xi, dlm->kappa, x,
                                    mask, csum, st);
        if (rc) return rc;
    }
    GatherOpts<T> o;
    o.csum = csum;
    o.occ_index = csum ? dlm->occ_index : nullptr;
    o.rows = blk != 0 ? 3 : 4;
    if (g.p == 1)
        return launch_gather<T, 1, Q1_BX, Q1_BY, Q1_BZ>(g, part, bl, blk == 2 ? nullptr : x, mask, y, o, st);
    return launch_gather<T, 2, Q2_BX, Q2_BY, Q2_BZ>(g, part, bl, x, mask, y, o, st);
}

template <typename T>
static int vms_residual_t(const Geo &g, const fsi_vms_params &prm, const T *s, const uint32_t *mask,
                          const T *gD, const T *x, const T *f, const DlmView *dlm, const T *lamg,
                          T *R, void *ws, hipStream_t st)
{
    const BrickLayout bl = brick_layout(g);
    const VmsConst<T> k = make_vms_const<T>(g, prm, s != nullptr);
    T *part = reinterpret_cast<T *>(ws);
    const bool use_gram = dlm != nullptr && dlm->n_occ > 0 && dlm->gram != nullptr;
    const T *gram = use_gram ? reinterpret_cast<const T *>(dlm->gram) : nullptr;
    const int32_t *gidx = use_gram ? dlm->occ_index : nullptr;
    int rc = g.p == 1 ? launch_q1_cells<T>(g, k, x, f, s, mask, gram, gidx, part, bl, st, true)
                      : launch_q2_cells<T>(g, k, x, f, s, mask, gram, gidx, part, bl, st, true);
    if (rc) return rc;
    GatherOpts<T> o;
    o.sub3 = lamg;
    o.gD = gD;
    if (o.gD == nullptr && mask != nullptr) {
        set_error("residual with a Dirichlet mask needs the Dirichlet values gD");
        return FSI_ERR_ARG;
    }
    if (g.p == 1) return launch_gather<T, 1, Q1_BX, Q1_BY, Q1_BZ>(g, part, bl, x, mask, R, o, st);
    return launch_gather<T, 2, Q2_BX, Q2_BY, Q2_BZ>(g, part, bl, x, mask, R, o, st);
}

int launch_vms_residual(const Geo &g, const fsi_vms_params &prm, fsi_dtype dt, const void *s,
                        const uint32_t *mask, const void *gD, const void *x, const void *f,
                        const DlmView *dlm, const void *lamg, void *R, void *ws, hipStream_t st)
{
    if (dt == FSI_F64)
        return vms_residual_t<double>(g, prm, (const double *)s, mask, (const double *)gD,
                                      (const double *)x, (const double *)f, dlm,
                                      (const double *)lamg, (double *)R, ws, st);
    return vms_residual_t<float>(g, prm, (const float *)s, mask, (const float *)gD, (const float *)x,
                                 (const float *)f, dlm, (const float *)lamg, (float *)R, ws, st);
}

int launch_tangent_apply(const Geo &g, const fsi_vms_params &prm, fsi_dtype dt, const void *s,
                         const uint32_t *mask, const void *x, const void *f, const DlmView *dlm,
                         const void *v, void *y, void *ws, hipStream_t st)
{
    if (g.p != 1) {
        set_error("the full Newton tangent is implemented for Q1 grids");
        return FSI_ERR_UNSUPPORTED;
    }
    if (dt == FSI_F64)
        return vms_apply_t<double>(g, prm, (const double *)x, (const double *)s, mask, (const double *)v,
                                   (double *)y, dlm, ws, st, (const double *)x, (const double *)f);
    return vms_apply_t<float>(g, prm, (const float *)x, (const float *)s, mask, (const float *)v, (float *)y,
                              dlm, ws, st, (const float *)x, (const float *)f);
}

int launch_vms_apply(const Geo &g, const fsi_vms_params &prm, fsi_dtype dt, const void *a,
                     const void *s, const uint32_t *mask, const void *x, void *y,
                     const DlmView *dlm, void *ws, size_t ws_bytes, hipStream_t st)
{
    (void)ws_bytes;
    if (dt == FSI_F64)
        return vms_apply_t<double>(g, prm, (const double *)a, (const double *)s, mask,
                                   (const double *)x, (double *)y, dlm, ws, st);
    return vms_apply_t<float>(g, prm, (const float *)a, (const float *)s, mask, (const float *)x,
                              (float *)y, dlm, ws, st);
}

int launch_vms_apply_block(const Geo &g, const fsi_vms_params &prm, fsi_dtype dt, int blk, const void *a,
                           const void *s, const uint32_t *mask, const void *x, void *y, const DlmView *dlm,
                           void *ws, hipStream_t st)
{
    if (blk != 1 && blk != 2) {
        set_error("operator block %d (1: velocity on (u, 0), 2: velocity rows on (0, p))", blk);
        return FSI_ERR_ARG;
    }
    if (g.p != 1) return FSI_ERR_UNSUPPORTED;
    if (dt == FSI_F64)
        return vms_apply_t<double>(g, prm, (const double *)a, (const double *)s, mask, (const double *)x,
                                   (double *)y, dlm, ws, st, nullptr, nullptr, blk);
    return vms_apply_t<float>(g, prm, (const float *)a, (const float *)s, mask, (const float *)x, (float *)y,
                              dlm, ws, st, nullptr, nullptr, blk);
}

}  // namespace fsi

using namespace fsi;

#define FSI_API extern "C" __attribute__((visibility("default")))

FSI_API const char *fsi_status_string(int status)
{
    switch (status) {
    case FSI_OK: return "ok";
    case FSI_ERR_ARG: return "invalid argument";
    case FSI_ERR_HIP: return "HIP runtime error";
    case FSI_ERR_WORKSPACE: return "workspace missing or too small";
    case FSI_ERR_NOT_CONVERGED: return "not converged";
    case FSI_ERR_BREAKDOWN: return "Krylov breakdown";
    case FSI_ERR_NAN: return "NaN or Inf detected";
    case FSI_ERR_UNSUPPORTED: return "unsupported combination";
    default: return "unknown status";
    }
}

FSI_API const char *fsi_last_error(void) { return g_err; }

FSI_API const char *fsi_version(void) { return "fsi-mi355x 0.1 (gfx950)"; }

static bool dtype_ok(fsi_dtype d) { return d == FSI_F64 || d == FSI_F32; }

FSI_API size_t fsi_vms_apply_workspace(const fsi_grid *grid, fsi_dtype dtype)
{
    if (check_grid(grid) != FSI_OK || !dtype_ok(dtype)) return 0;
    return vms_workspace_bytes(make_geo(*grid), dtype);
}

FSI_API int fsi_vms_apply(const fsi_grid *grid, const fsi_vms_params *prm, fsi_dtype dtype,
                          const void *a, const void *s, const uint32_t *dir_mask, const void *x,
                          void *y, void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    rc = check_params(prm);
    if (rc) return rc;
    FSI_CHECK_ARG(dtype_ok(dtype), "bad dtype %d", (int)dtype);
    FSI_CHECK_ARG(a && x && y, "a, x and y must be non-NULL");
    FSI_CHECK_ARG(x != y && a != y && s != y, "y must not alias x, a or s");
    const Geo g = make_geo(*grid);
    const size_t need = vms_workspace_bytes(g, dtype);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    return launch_vms_apply(g, *prm, dtype, a, s, dir_mask, x, y, nullptr, ws, ws_bytes,
                            as_stream(stream));
}

FSI_API size_t fsi_dlm_locate_workspace(const fsi_grid *grid, int64_t m)
{
    if (check_grid(grid) != FSI_OK || m < 0) return 0;
    return locate_workspace_bytes(make_geo(*grid), m);
}

FSI_API int fsi_dlm_locate(const fsi_grid *grid, int64_t m, const double *X, fsi_dtype dtype,
                           int32_t *cell, void *xi, int32_t *perm, int32_t *occ_cell,
                           int32_t *occ_start, int32_t *occ_index, void *s_out, double s_max,
                           int64_t *n_occ_host, int64_t *n_outside_host, void *ws,
                           size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    FSI_CHECK_ARG(dtype_ok(dtype), "bad dtype %d", (int)dtype);
    FSI_CHECK_ARG(m >= 0 && m < ((int64_t)1 << 31) - 1, "m out of range");
    FSI_CHECK_ARG(m == 0 || (X && cell && xi && perm), "X, cell, xi and perm must be non-NULL");
    FSI_CHECK_ARG(occ_cell && occ_start && occ_index, "occ_cell, occ_start and occ_index must be non-NULL");
    FSI_CHECK_ARG(std::isfinite(s_max), "s_max must be finite");
    const Geo g = make_geo(*grid);
    const size_t need = locate_workspace_bytes(g, m);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    return launch_locate(g, m, X, dtype, cell, xi, perm, occ_cell, occ_start, occ_index, s_out, s_max,
                         n_occ_host, n_outside_host, ws, as_stream(stream));
}

FSI_API int fsi_dlm_B(const fsi_grid *grid, fsi_dtype dtype, int64_t m, const int32_t *cell,
                      const void *xi, const void *u, void *Bu, void *stream)
{
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    FSI_CHECK_ARG(dtype_ok(dtype), "bad dtype %d", (int)dtype);
    FSI_CHECK_ARG(m >= 0 && m < ((int64_t)1 << 31) - 1, "m out of range");
    FSI_CHECK_ARG(m == 0 || (cell && xi && u && Bu), "cell, xi, u and Bu must be non-NULL");
    return launch_dlm_B(make_geo(*grid), dtype, m, cell, xi, u, nullptr, Bu, as_stream(stream));
}

FSI_API int fsi_dlm_B_located(const fsi_grid *grid, fsi_dtype dtype, int64_t m, const int32_t *occ_cell,
                              const int32_t *occ_start, int64_t n_occ, const void *xi_loc, const void *u,
                              void *Bu_loc, void *stream)
{
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    FSI_CHECK_ARG(dtype_ok(dtype), "bad dtype %d", (int)dtype);
    FSI_CHECK_ARG(m >= 0 && m < ((int64_t)1 << 31) - 1, "m out of range");
    const Geo g = make_geo(*grid);
    FSI_CHECK_ARG(n_occ >= 0 && n_occ <= g.E && n_occ <= m, "n_occ out of range");
    if (m == 0) return FSI_OK;
    FSI_CHECK_ARG(occ_cell && occ_start && xi_loc && u && Bu_loc, "point tables, u and Bu must be non-NULL");
    return launch_dlm_B_located(g, dtype, m, n_occ, occ_cell, occ_start, xi_loc, u, Bu_loc, as_stream(stream));
}

FSI_API int fsi_dlm_permute(fsi_dtype dtype, int64_t m, int32_t nf, const int32_t *perm, int32_t to_point,
                            const void *src, void *dst, void *stream)
{
    clear_error();
    FSI_CHECK_ARG(dtype_ok(dtype), "bad dtype %d", (int)dtype);
    FSI_CHECK_ARG(m >= 0 && m < ((int64_t)1 << 31) - 1, "m out of range");
    FSI_CHECK_ARG(nf >= 0 && nf <= 64, "nf out of range");
    if (m == 0 || nf == 0) return FSI_OK;
    FSI_CHECK_ARG(perm && src && dst && src != dst, "perm, src and dst must be non-NULL, dst not src");
    return launch_dlm_permute(dtype, m, nf, perm, to_point != 0, src, dst, as_stream(stream));
}

FSI_API size_t fsi_dlm_BT_workspace(const fsi_grid *grid, int64_t n_occ, fsi_dtype dtype)
{
    if (check_grid(grid) != FSI_OK || n_occ < 0 || !dtype_ok(dtype)) return 0;
    return dlm_csum_bytes(make_geo(*grid), n_occ, dtype);
}

FSI_API int fsi_dlm_BT(const fsi_grid *grid, fsi_dtype dtype, int64_t m, const int32_t *cell,
                       const void *xi, const int32_t *perm, const int32_t *occ_cell,
                       const int32_t *occ_start, const int32_t *occ_index, int64_t n_occ,
                       const void *lam, const void *kappa, void *y, void *ws, size_t ws_bytes,
                       void *stream)
{
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    FSI_CHECK_ARG(dtype_ok(dtype), "bad dtype %d", (int)dtype);
    FSI_CHECK_ARG(m >= 0 && m < ((int64_t)1 << 31) - 1, "m out of range");
    const Geo g = make_geo(*grid);
    FSI_CHECK_ARG(n_occ >= 0 && n_occ <= g.E && n_occ <= m, "n_occ out of range");
    FSI_CHECK_ARG(y != nullptr, "y must be non-NULL");
    (void)cell;
    if (n_occ == 0) return FSI_OK;
    FSI_CHECK_ARG(xi && occ_cell && occ_start && occ_index && lam, "point tables and lam must be non-NULL");
    const size_t need = dlm_csum_bytes(g, n_occ, dtype);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    hipStream_t st = as_stream(stream);
    // perm NULL: xi, lam and kappa are in located order (no indirection)
    rc = launch_dlm_cell_reduce(g, dtype, false, m, n_occ, occ_cell, occ_start, perm, xi, kappa, lam,
                                nullptr, ws, st);
    if (rc) return rc;
    return launch_dlm_node_gather(g, dtype, n_occ, occ_cell, ws, occ_index, y, st);
}

FSI_API int fsi_dlm_gram(const fsi_grid *grid, fsi_dtype dtype, int64_t m, const void *xi,
                         const int32_t *perm, const int32_t *occ_start, int64_t n_occ,
                         const void *kappa, void *gram, void *stream)
{
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    FSI_CHECK_ARG(dtype_ok(dtype), "bad dtype %d", (int)dtype);
    FSI_CHECK_ARG(m >= 0 && m < ((int64_t)1 << 31) - 1, "m out of range");
    const Geo g = make_geo(*grid);
    FSI_CHECK_ARG(n_occ >= 0 && n_occ <= g.E && n_occ <= m, "n_occ out of range");
    if (n_occ == 0) return FSI_OK;
    FSI_CHECK_ARG(xi && perm && occ_start && gram, "xi, perm, occ_start and gram must be non-NULL");
    return launch_dlm_gram(g, dtype, m, n_occ, occ_start, perm, xi, kappa, gram, as_stream(stream));
}

static int check_solid(const fsi_solid *S);
static DlmView view_of(const fsi_problem *p);

static int check_problem(const fsi_problem *p)
{
    FSI_CHECK_ARG(p != nullptr, "problem is NULL");
    int rc = check_grid(&p->grid);
    if (rc) return rc;
    rc = check_params(&p->prm);
    if (rc) return rc;
    FSI_CHECK_ARG(dtype_ok(p->dtype), "bad dtype %d", (int)p->dtype);
    FSI_CHECK_ARG(p->a != nullptr, "advection field a is NULL");
    FSI_CHECK_ARG(p->m >= 0 && p->m < ((int64_t)1 << 31) - 1, "m out of range");
    const Geo g = make_geo(p->grid);
    FSI_CHECK_ARG(p->n_occ >= 0 && p->n_occ <= g.E && p->n_occ <= p->m, "n_occ out of range");
    if (p->n_occ > 0)
        FSI_CHECK_ARG(p->xi && p->perm && p->occ_cell && p->occ_start && p->occ_index,
                      "point tables must be non-NULL when n_occ > 0");
    if (p->solid != nullptr) {
        rc = check_solid(p->solid);
        if (rc) return rc;
        FSI_CHECK_ARG(p->m == p->solid->n_nodes, "the problem's points (%lld) must be the solid's nodes (%lld)",
                      (long long)p->m, (long long)p->solid->n_nodes);
        FSI_CHECK_ARG(p->m == 0 || p->solid_U != nullptr, "solid_U must be non-NULL");
        FSI_CHECK_ARG(std::isfinite(p->solid_cM) && std::isfinite(p->solid_cK) && std::isfinite(p->solid_cV),
                      "solid coefficients must be finite");
        if (p->n_occ > 0) FSI_CHECK_ARG(p->cell != nullptr, "point cells must be non-NULL with a solid");
    }
    return FSI_OK;
}

// workspace of one Jacobian apply of problem p (with solid S in place of p->solid if given)
static size_t problem_ws(const fsi_problem *p, const fsi_solid *S = nullptr)
{
    const Geo g = make_geo(p->grid);
    if (S == nullptr) S = p->solid;
    size_t b = vms_workspace_bytes(g, p->dtype) + dlm_csum_bytes(g, p->n_occ, p->dtype);
    if (S != nullptr)
        b += 2 * align_up((size_t)3 * p->m * (p->dtype == FSI_F64 ? 8 : 4)) +
             solid_workspace_bytes(S->n_elem, p->dtype);
    return b;
}

FSI_API size_t fsi_jacobian_workspace(const fsi_problem *p)
{
    if (check_problem(p) != FSI_OK) return 0;
    return problem_ws(p);
}

FSI_API int fsi_jacobian_apply(const fsi_problem *p, const void *x, void *y, void *ws,
                               size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = check_problem(p);
    if (rc) return rc;
    FSI_CHECK_ARG(x && y, "x and y must be non-NULL");
    FSI_CHECK_ARG(x != y && p->a != y && p->s != y, "y must not alias x or the problem's a or s");
    const Geo g = make_geo(p->grid);
    const size_t need = problem_ws(p);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    const DlmView v = view_of(p);
    return launch_vms_apply(g, p->prm, p->dtype, p->a, p->s, p->dir_mask, x, y,
                            p->n_occ > 0 ? &v : nullptr, ws, ws_bytes, as_stream(stream));
}

FSI_API int fsi_jacobian_apply_block(const fsi_problem *p, int32_t block, const void *x, void *y, void *ws,
                                     size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = check_problem(p);
    if (rc) return rc;
    FSI_CHECK_ARG(block == FSI_BLOCK_F || block == FSI_BLOCK_G, "block must be FSI_BLOCK_F or FSI_BLOCK_G");
    FSI_CHECK_ARG(x && y, "x and y must be non-NULL");
    FSI_CHECK_ARG(x != y && p->a != y && p->s != y, "y must not alias x or the problem's a or s");
    const Geo g = make_geo(p->grid);
    if (g.p != 1) {
        set_error("the block products are implemented for Q1 grids");
        return FSI_ERR_UNSUPPORTED;
    }
    const size_t need = problem_ws(p);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    const DlmView v = view_of(p);
    return launch_vms_apply_block(g, p->prm, p->dtype, block, p->a, p->s, p->dir_mask, x, y,
                                  p->n_occ > 0 ? &v : nullptr, ws, as_stream(stream));
}

// ---- hyperelastic solid block ----

static int check_solid(const fsi_solid *S)
{
    FSI_CHECK_ARG(S != nullptr, "solid is NULL");
    FSI_CHECK_ARG(S->n_nodes >= 0 && S->n_nodes < ((int64_t)1 << 31) - 1, "solid n_nodes out of range");
    FSI_CHECK_ARG(S->n_elem >= 0 && S->n_elem < ((int64_t)1 << 28), "solid n_elem out of range");
    FSI_CHECK_ARG(S->n_nodes == 0 || (S->X0 && S->node_start), "solid X0 and node_start must be non-NULL");
    FSI_CHECK_ARG(S->n_elem == 0 || (S->conn && S->node_slot), "solid conn and node_slot must be non-NULL");
    FSI_CHECK_ARG(std::isfinite(S->C0) && std::isfinite(S->kappa_s) && std::isfinite(S->rho_s0) &&
                      std::isfinite(S->rho_f) && std::isfinite(S->mu_f),
                  "solid material parameters must be finite");
    return FSI_OK;
}

FSI_API int fsi_solid_setup(int64_t n_nodes, int64_t n_elem, const int32_t *conn, int32_t *node_start,
                            int32_t *node_slot, void *stream)
{
    clear_error();
    FSI_CHECK_ARG(n_nodes >= 0 && n_nodes < ((int64_t)1 << 31) - 1, "n_nodes out of range");
    FSI_CHECK_ARG(n_elem >= 0 && n_elem < ((int64_t)1 << 28), "n_elem out of range");
    FSI_CHECK_ARG(node_start != nullptr, "node_start must be non-NULL");
    FSI_CHECK_ARG(n_elem == 0 || (conn && node_slot), "conn and node_slot must be non-NULL");
    return solid_build_csr(n_nodes, n_elem, conn, node_start, node_slot, as_stream(stream));
}

FSI_API size_t fsi_solid_workspace(int64_t n_elem, fsi_dtype dtype)
{
    return solid_workspace_bytes(n_elem, dtype);
}

FSI_API int fsi_solid_apply(const fsi_solid *S, fsi_dtype dtype, const double *U, double cM, double cK,
                            double cV, const void *v, void *y, void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = check_solid(S);
    if (rc) return rc;
    FSI_CHECK_ARG(dtype_ok(dtype), "bad dtype %d", (int)dtype);
    FSI_CHECK_ARG(std::isfinite(cM) && std::isfinite(cK) && std::isfinite(cV), "coefficients must be finite");
    FSI_CHECK_ARG(S->n_nodes == 0 || (U && v && y), "U, v and y must be non-NULL");
    FSI_CHECK_ARG(v != y, "v and y must not alias");
    const size_t need = solid_workspace_bytes(S->n_elem, dtype);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    return launch_solid_apply(solid_view(*S), dtype, U, SolidCoefs{cM, cK, cV}, v, y, ws, as_stream(stream));
}

static size_t jacobian_solid_bytes(const fsi_problem *p, const fsi_solid *S) { return problem_ws(p, S); }

FSI_API size_t fsi_jacobian_solid_workspace(const fsi_problem *p, const fsi_solid *S)
{
    if (check_problem(p) != FSI_OK || check_solid(S) != FSI_OK) return 0;
    return jacobian_solid_bytes(p, S);
}

FSI_API int fsi_jacobian_solid_apply(const fsi_problem *p, const fsi_solid *S, const double *U, double cM,
                                     double cK, double cV, const void *x, void *y, void *ws,
                                     size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = check_problem(p);
    if (rc) return rc;
    rc = check_solid(S);
    if (rc) return rc;
    FSI_CHECK_ARG(p->m == S->n_nodes, "the problem's points (%lld) must be the solid's nodes (%lld)",
                  (long long)p->m, (long long)S->n_nodes);
    FSI_CHECK_ARG(std::isfinite(cM) && std::isfinite(cK) && std::isfinite(cV), "coefficients must be finite");
    FSI_CHECK_ARG(x && y, "x and y must be non-NULL");
    FSI_CHECK_ARG(x != y, "x and y must not alias");
    FSI_CHECK_ARG(S->n_nodes == 0 || U != nullptr, "U must be non-NULL");
    if (p->n_occ > 0)
        FSI_CHECK_ARG(p->cell != nullptr, "point cells must be non-NULL when n_occ > 0");
    const size_t need = jacobian_solid_bytes(p, S);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    DlmView v{p->m,     p->cell,      p->xi,   p->perm, p->occ_cell, p->occ_start,
              p->n_occ, p->occ_index, nullptr, nullptr};
    v.solid = S;
    v.solid_U = U;
    v.solid_c = SolidCoefs{cM, cK, cV};
    return launch_vms_apply(make_geo(p->grid), p->prm, p->dtype, p->a, p->s, p->dir_mask, x, y,
                            p->n_occ > 0 ? &v : nullptr, ws, ws_bytes, as_stream(stream));
}

// ---- the solid's nonlinear residual and the coupled step ----

FSI_API int fsi_solid_residual(const fsi_solid *S, const double *U, const double *V, const double *A, double *R,
                               void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = check_solid(S);
    if (rc) return rc;
    FSI_CHECK_ARG(S->n_nodes == 0 || (U && V && A && R), "U, V, A and R must be non-NULL");
    FSI_CHECK_ARG(R != U && R != V && R != A, "R must not alias the inputs");
    const size_t need = solid_workspace_bytes(S->n_elem, FSI_F64);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    return launch_solid_residual(solid_view(*S), U, V, A, R, ws, as_stream(stream));
}

int fsi::solid_step_residual(const Geo &g, const fsi_problem &P, const SolidStep &ss, const double *f,
                             const double *gD, const double *x, double *R, void *ws, hipStream_t st)
{
    // V = B u (the solid moves with the fluid), U = Ub + cU V, A = cA V - Ab, R^s at the solid
    // nodes, its B^T corner sums, then the fluid step residual whose node gather adds them before
    // the Dirichlet rows (u - gD)
    const int64_t m = P.m;
    const VmsConst<double> k = make_vms_const<double>(g, P.prm, P.s != nullptr);
    const BrickLayout bl = brick_layout(g);
    char *w = reinterpret_cast<char *>(ws);
    double *part = reinterpret_cast<double *>(w);
    w += vms_workspace_bytes(g, FSI_F64);
    double *csum = reinterpret_cast<double *>(w);
    w += dlm_csum_bytes(g, P.n_occ, FSI_F64);
    double *A = reinterpret_cast<double *>(w);
    w += align_up((size_t)3 * m * sizeof(double));
    double *Rs = reinterpret_cast<double *>(w);
    w += align_up((size_t)3 * m * sizeof(double));
    int rc = FSI_OK;
    const bool solid_on = P.n_occ > 0 && m > 0;
    if (m > 0) {
        rc = launch_dlm_B(g, FSI_F64, m, P.cell, P.xi, x, nullptr, ss.V, st);
        if (rc) return rc;
        rc = launch_solid_state(m, ss.cU, ss.cA, ss.Ub, ss.Ab, ss.V, ss.U, A, st);
        if (rc) return rc;
    }
    if (solid_on) {
        rc = launch_solid_residual(solid_view(*ss.S), ss.U, ss.V, A, Rs, w, st);
        if (rc) return rc;
        rc = launch_dlm_cell_reduce(g, FSI_F64, false, m, P.n_occ, P.occ_cell, P.occ_start, P.perm, P.xi, nullptr,
                                    Rs, nullptr, csum, st);
        if (rc) return rc;
    }
    rc = g.p == 1 ? launch_q1_cells<double>(g, k, (const double *)x, f, (const double *)P.s, P.dir_mask, nullptr,
                                            nullptr, part, bl, st, true)
                  : launch_q2_cells<double>(g, k, (const double *)x, f, (const double *)P.s, P.dir_mask, nullptr,
                                            nullptr, part, bl, st, true);
    if (rc) return rc;
    GatherOpts<double> o;
    o.csum = solid_on ? csum : nullptr;
    o.occ_index = solid_on ? P.occ_index : nullptr;
    o.gD = gD;
    if (g.p == 1) return launch_gather<double, 1, Q1_BX, Q1_BY, Q1_BZ>(g, part, bl, x, P.dir_mask, R, o, st);
    return launch_gather<double, 2, Q2_BX, Q2_BY, Q2_BZ>(g, part, bl, x, P.dir_mask, R, o, st);
}

static int check_solid_step(const fsi_problem *p, const fsi_solid *S, const double *Ub, const double *Ab,
                            double cU, double cA, const double *U, const double *V)
{
    int rc = check_problem(p);
    if (rc) return rc;
    rc = check_solid(S);
    if (rc) return rc;
    FSI_CHECK_ARG(p->dtype == FSI_F64, "the step residual takes the FP64 problem");
    FSI_CHECK_ARG(p->solid == nullptr, "pass the solid as the argument, not in the problem");
    FSI_CHECK_ARG(p->m == S->n_nodes, "the problem's points (%lld) must be the solid's nodes (%lld)",
                  (long long)p->m, (long long)S->n_nodes);
    FSI_CHECK_ARG(std::isfinite(cU) && std::isfinite(cA), "cU and cA must be finite");
    FSI_CHECK_ARG(p->m == 0 || (Ub && Ab && U && V && p->cell && p->xi), "solid state arrays must be non-NULL");
    FSI_CHECK_ARG(U != Ub && U != Ab && V != Ub && V != Ab && U != V,
                  "U, V must be distinct from U_base, A_base and each other");
    return FSI_OK;
}

FSI_API size_t fsi_solid_step_workspace(const fsi_problem *p, const fsi_solid *S)
{
    if (check_problem(p) != FSI_OK || check_solid(S) != FSI_OK) return 0;
    return problem_ws(p, S);
}

FSI_API int fsi_solid_step_residual(const fsi_problem *p, const fsi_solid *S, const double *U_base,
                                    const double *A_base, double cU, double cA, const double *f, const double *gD,
                                    const double *x, double *R, double *U, double *V, void *ws, size_t ws_bytes,
                                    void *stream)
{
    clear_error();
    int rc = check_solid_step(p, S, U_base, A_base, cU, cA, U, V);
    if (rc) return rc;
    FSI_CHECK_ARG(f && x && R && x != R, "f, x, R must be non-NULL and x != R");
    FSI_CHECK_ARG(p->dir_mask == nullptr || gD != nullptr, "gD required with a Dirichlet mask");
    const size_t need = problem_ws(p, S);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    const SolidStep ss{S, U_base, A_base, cU, cA, U, V};
    return solid_step_residual(make_geo(p->grid), *p, ss, f, gD, x, R, ws, as_stream(stream));
}

static DlmView view_of(const fsi_problem *p)
{
    DlmView v{p->m,     p->cell,      p->xi,    p->perm,     p->occ_cell, p->occ_start,
              p->n_occ, p->occ_index, p->kappa, p->dlm_gram};
    if (p->solid != nullptr) {
        v.solid = p->solid;
        v.solid_U = p->solid_U;
        v.solid_c = SolidCoefs{p->solid_cM, p->solid_cK, p->solid_cV};
    }
    return v;
}

FSI_API int fsi_vms_residual(const fsi_problem *p, const void *f, const void *lamg, const void *gD,
                             const void *x, void *R, void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    FSI_CHECK_ARG(p != nullptr, "problem is NULL");
    int rc = check_grid(&p->grid);
    if (rc) return rc;
    rc = check_params(&p->prm);
    if (rc) return rc;
    FSI_CHECK_ARG(dtype_ok(p->dtype), "bad dtype");
    FSI_CHECK_ARG(f && x && R && x != R, "f, x, R must be non-NULL and x != R");
    FSI_CHECK_ARG(p->dir_mask == nullptr || gD != nullptr, "gD required with a Dirichlet mask");
    if (p->n_occ > 0 && p->dlm_gram == nullptr) {
        set_error("the residual needs the per-cell DLM blocks (fsi_dlm_gram) when n_occ > 0");
        return FSI_ERR_UNSUPPORTED;
    }
    if (p->solid != nullptr) {
        set_error("a problem carrying the solid block: its step residual is fsi_solid_step_residual");
        return FSI_ERR_UNSUPPORTED;
    }
    const Geo g = make_geo(p->grid);
    const size_t need = vms_workspace_bytes(g, p->dtype) + dlm_csum_bytes(g, p->n_occ, p->dtype);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    DlmView v = view_of(p);
    return launch_vms_residual(g, p->prm, p->dtype, p->s, p->dir_mask, gD, x, f,
                               p->n_occ > 0 ? &v : nullptr, lamg, R, ws, as_stream(stream));
}

FSI_API size_t fsi_bjacobi_workspace(const fsi_grid *grid)
{
    if (check_grid(grid) != FSI_OK) return 0;
    return bjacobi_workspace_bytes(make_geo(*grid));
}

FSI_API int fsi_bjacobi_setup(const fsi_problem *p, double *pinv64, float *pinv32, double *blocks,
                              int64_t *n_singular_host, void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = check_problem(p);
    if (rc) return rc;
    FSI_CHECK_ARG(p->dtype == FSI_F64, "block-Jacobi setup takes the FP64 problem");
    FSI_CHECK_ARG(pinv64 || pinv32 || blocks, "no output requested");
    if (p->n_occ > 0 && p->dlm_gram == nullptr) {
        set_error("block-Jacobi setup needs the per-cell DLM blocks (fsi_dlm_gram) when n_occ > 0");
        return FSI_ERR_UNSUPPORTED;
    }
    const Geo g = make_geo(p->grid);
    const size_t need = bjacobi_workspace_bytes(g);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    return launch_bjacobi_setup(g, p->prm, (const double *)p->a, (const double *)p->s, p->dir_mask,
                                p->n_occ > 0 ? (const double *)p->dlm_gram : nullptr, p->occ_index,
                                blocks, pinv64, pinv32, n_singular_host, ws, as_stream(stream));
}

FSI_API int fsi_bjacobi_apply(const fsi_grid *grid, fsi_dtype dtype, const void *pinv, const void *v,
                              void *z, void *stream)
{
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    FSI_CHECK_ARG(dtype_ok(dtype), "bad dtype");
    FSI_CHECK_ARG(pinv && v && z, "pinv, v and z must be non-NULL");
    return launch_bjacobi_apply(make_geo(*grid).N, dtype, pinv, v, z, as_stream(stream));
}

// storage precision of the Krylov basis: FP64, or FP32 with an FP32 inner precision and a basis
// the fused Gram-Schmidt kernels hold
static int check_basis(fsi_dtype basis, fsi_dtype inner, int restart)
{
    FSI_CHECK_ARG(dtype_ok(basis), "bad basis dtype");
    if (basis == FSI_F32) {
        FSI_CHECK_ARG(inner == FSI_F32, "an FP32 Krylov basis needs the FP32 inner precision");
        FSI_CHECK_ARG(restart <= KRY_FUSED_MAXK, "an FP32 Krylov basis needs restart <= %d", KRY_FUSED_MAXK);
    }
    return FSI_OK;
}

static int check_solve(const fsi_problem *J64, const fsi_problem *J32, const fsi_solve_opts *o)
{
    int rc = check_problem(J64);
    if (rc) return rc;
    FSI_CHECK_ARG(J64->dtype == FSI_F64, "J64 must be an FP64 problem");
    FSI_CHECK_ARG(o != nullptr, "opts is NULL");
    FSI_CHECK_ARG(o->restart >= 1 && o->restart <= 400, "restart must be in [1, 400]");
    FSI_CHECK_ARG(o->max_iters >= 1, "max_iters must be >= 1");
    FSI_CHECK_ARG(std::isfinite(o->rtol) && o->rtol > 0.0 && o->rtol < 1.0, "rtol must be in (0,1)");
    FSI_CHECK_ARG(dtype_ok(o->inner), "bad inner dtype");
    FSI_CHECK_ARG(o->precond == FSI_PC_BJACOBI || o->precond == FSI_PC_SCHUR_DIAG ||
                      o->precond == FSI_PC_SCHUR_TRI,
                  "unknown preconditioner %d", (int)o->precond);
    FSI_CHECK_ARG(o->vel_steps >= 0 && o->vel_steps <= 16, "vel_steps must be in [0, 16]");
    if (o->inner == FSI_F32) {
        FSI_CHECK_ARG(J32 != nullptr, "inner FP32 needs the FP32 problem");
        rc = check_problem(J32);
        if (rc) return rc;
        FSI_CHECK_ARG(J32->dtype == FSI_F32, "J32 must be an FP32 problem");
        FSI_CHECK_ARG(std::memcmp(&J32->grid, &J64->grid, sizeof(fsi_grid)) == 0,
                      "J32 and J64 grids differ");
        FSI_CHECK_ARG(std::isfinite(o->inner_reduction) && o->inner_reduction > 0.0 &&
                          o->inner_reduction < 1.0,
                      "inner_reduction must be in (0,1)");
    }
    rc = check_basis(o->basis, o->inner, o->restart);
    if (rc) return rc;
    return FSI_OK;
}

static size_t jac_ws(const fsi_problem *p) { return problem_ws(p); }

FSI_API size_t fsi_fgmres_workspace(const fsi_problem *J64, const fsi_problem *J32,
                                    const fsi_solve_opts *o)
{
    if (check_solve(J64, J32, o) != FSI_OK) return 0;
    size_t jw = jac_ws(J64);
    if (o->inner == FSI_F32) jw = std::max(jw, jac_ws(J32));
    return fgmres_workspace_bytes(4 * make_geo(J64->grid).N, o->restart, o->inner, o->basis, jw);
}

FSI_API int fsi_fgmres_solve(const fsi_problem *J64, const fsi_problem *J32, const void *pinv,
                             const double *b, double *x, const fsi_solve_opts *o,
                             fsi_solve_stats *stats, void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = check_solve(J64, J32, o);
    if (rc) return rc;
    FSI_CHECK_ARG(b && x && b != x, "b and x must be non-NULL and distinct");
    size_t jw = jac_ws(J64);
    if (o->inner == FSI_F32) jw = std::max(jw, jac_ws(J32));
    const Geo g = make_geo(J64->grid);
    const size_t need = fgmres_workspace_bytes(4 * g.N, o->restart, o->inner, o->basis, jw);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    const DlmView v64 = view_of(J64);
    JacobianCall c64{[&](const void *xx, void *yy, void *w, hipStream_t s) {
        return launch_vms_apply(g, J64->prm, FSI_F64, J64->a, J64->s, J64->dir_mask, xx, yy,
                                J64->n_occ > 0 ? &v64 : nullptr, w, jw, s);
    }};
    if (g.p == 1)
        c64.block = [&](int blk, const void *xx, void *yy, void *w, hipStream_t s) {
            return launch_vms_apply_block(g, J64->prm, FSI_F64, blk, J64->a, J64->s, J64->dir_mask, xx, yy,
                                          J64->n_occ > 0 ? &v64 : nullptr, w, s);
        };
    DlmView v32{};
    JacobianCall c32;
    if (o->inner == FSI_F32) {
        v32 = view_of(J32);
        c32.apply = [&](const void *xx, void *yy, void *w, hipStream_t s) {
            return launch_vms_apply(g, J32->prm, FSI_F32, J32->a, J32->s, J32->dir_mask, xx, yy,
                                    J32->n_occ > 0 ? &v32 : nullptr, w, jw, s);
        };
        if (g.p == 1)
            c32.block = [&](int blk, const void *xx, void *yy, void *w, hipStream_t s) {
                return launch_vms_apply_block(g, J32->prm, FSI_F32, blk, J32->a, J32->s, J32->dir_mask, xx, yy,
                                              J32->n_occ > 0 ? &v32 : nullptr, w, s);
            };
    }
    Precond pc;
    const JacobianCall *Jin = o->inner == FSI_F32 ? &c32 : &c64;
    if (o->precond != FSI_PC_BJACOBI) {
        FSI_CHECK_ARG(pinv != nullptr, "the Schur preconditioner object (fsi_schur_setup) is required");
        void *obj = const_cast<void *>(pinv);
        const int mode = o->precond == FSI_PC_SCHUR_DIAG ? 1 : 2;
        const bool basis64 = o->basis != FSI_F32;
        pc.apply = [&, obj, mode, basis64](const void *v, void *z, void *w, hipStream_t s) {
            return schur_apply(g, o->inner, basis64, mode, o->vel_steps, obj, v, z, Jin, w, s);
        };
    } else if (pinv != nullptr) {
        pc.apply = [&](const void *v, void *z, void *, hipStream_t s) {
            if (o->basis == FSI_F32) return launch_bjacobi_apply(g.N, FSI_F32, pinv, v, z, s);
            if (o->inner == FSI_F32)
                return launch_bjacobi_apply_f64_to_f32(g.N, (const float *)pinv, (const double *)v, (float *)z, s);
            return launch_bjacobi_apply(g.N, FSI_F64, pinv, v, z, s);
        };
    }
    return fgmres_solve(g, c64, o->inner == FSI_F32 ? &c32 : nullptr, pc.apply ? &pc : nullptr, b, x, *o,
                        stats, ws, jw, as_stream(stream));
}

FSI_API size_t fsi_schur_size(const fsi_grid *grid)
{
    clear_error();
    if (check_grid(grid) != FSI_OK) return 0;
    ScPlan p;
    if (sc_plan(make_geo(*grid), p) != FSI_OK) return 0;
    return p.total;
}

FSI_API int fsi_schur_info(const fsi_grid *grid, int32_t *n_levels, int32_t *ncell, int64_t *alpha_offset)
{
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    ScPlan p;
    rc = sc_plan(make_geo(*grid), p);
    if (rc) return rc;
    if (n_levels) *n_levels = p.L;
    for (int l = 0; l < p.L; ++l) {
        if (ncell)
            for (int d = 0; d < 3; ++d) ncell[3 * l + d] = p.lv[l].nc[d];
        if (alpha_offset) alpha_offset[l] = (int64_t)p.lv[l].a64;
    }
    return FSI_OK;
}

FSI_API int fsi_schur_setup(const fsi_problem *p, const double *blocks, void *pc, size_t pc_bytes,
                            void *stream)
{
    clear_error();
    int rc = check_problem(p);
    if (rc) return rc;
    FSI_CHECK_ARG(p->dtype == FSI_F64, "the Schur preconditioner setup takes the FP64 problem");
    FSI_CHECK_ARG(blocks != nullptr && pc != nullptr, "blocks and pc must be non-NULL");
    if (p->n_occ > 0 && p->dlm_gram == nullptr) {
        set_error("the Schur preconditioner setup needs the per-cell DLM blocks (fsi_dlm_gram) when n_occ > 0");
        return FSI_ERR_UNSUPPORTED;
    }
    const Geo g = make_geo(p->grid);
    ScPlan plan;
    rc = sc_plan(g, plan);
    if (rc) return rc;
    if (pc_bytes < plan.total) {
        set_error("preconditioner object of %zu bytes needed (got %zu)", plan.total, pc_bytes);
        return FSI_ERR_WORKSPACE;
    }
    return schur_setup(g, p->prm, (const double *)p->a, (const double *)p->s, p->dir_mask,
                       p->n_occ > 0 ? (const double *)p->dlm_gram : nullptr, p->occ_index, blocks, pc,
                       as_stream(stream));
}

FSI_API int fsi_schur_apply(const fsi_problem *J, int32_t mode, int32_t vel_steps, void *pc, const void *v,
                            void *z, void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = check_problem(J);
    if (rc) return rc;
    FSI_CHECK_ARG(mode == FSI_PC_SCHUR_DIAG || mode == FSI_PC_SCHUR_TRI, "mode must be a Schur form");
    FSI_CHECK_ARG(pc && v && z && v != z, "pc, v and z must be non-NULL, v and z distinct");
    const Geo g = make_geo(J->grid);
    ScPlan plan;
    rc = sc_plan(g, plan);
    if (rc) return rc;
    const size_t jw = jac_ws(J);
    if ((mode == FSI_PC_SCHUR_TRI || vel_steps > 0) && (ws == nullptr || ws_bytes < jw)) {
        set_error("workspace of %zu bytes needed (got %zu)", jw, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    const DlmView dv = view_of(J);
    JacobianCall c{[&](const void *xx, void *yy, void *w, hipStream_t s) {
        return launch_vms_apply(g, J->prm, J->dtype, J->a, J->s, J->dir_mask, xx, yy,
                                J->n_occ > 0 ? &dv : nullptr, w, jw, s);
    }};
    if (g.p == 1)
        c.block = [&](int blk, const void *xx, void *yy, void *w, hipStream_t s) {
            return launch_vms_apply_block(g, J->prm, J->dtype, blk, J->a, J->s, J->dir_mask, xx, yy,
                                          J->n_occ > 0 ? &dv : nullptr, w, s);
        };
    return schur_apply(g, J->dtype, false, mode == FSI_PC_SCHUR_DIAG ? 1 : 2, vel_steps, pc, v, z, &c, ws,
                       as_stream(stream));
}

static int check_newton(const fsi_problem *P64, const fsi_problem *P32, const fsi_newton_opts *o)
{
    int rc = check_problem(P64);
    if (rc) return rc;
    FSI_CHECK_ARG(P64->dtype == FSI_F64, "P64 must be an FP64 problem");
    FSI_CHECK_ARG(o != nullptr, "opts is NULL");
    FSI_CHECK_ARG(o->max_newton >= 0 && o->max_newton <= 200, "max_newton out of range");
    FSI_CHECK_ARG(std::isfinite(o->tol_abs) && o->tol_abs >= 0.0, "tol_abs must be finite and >= 0");
    FSI_CHECK_ARG(std::isfinite(o->eta) && o->eta > 0.0 && o->eta < 1.0, "eta must be in (0,1)");
    FSI_CHECK_ARG(o->restart >= 1 && o->restart <= 400, "restart must be in [1, 400]");
    FSI_CHECK_ARG(o->max_krylov >= 1, "max_krylov must be >= 1");
    FSI_CHECK_ARG(dtype_ok(o->inner), "bad inner dtype");
    FSI_CHECK_ARG(o->precond == FSI_PC_BJACOBI || o->precond == FSI_PC_SCHUR_DIAG ||
                      o->precond == FSI_PC_SCHUR_TRI,
                  "unknown preconditioner %d", (int)o->precond);
    FSI_CHECK_ARG(o->vel_steps >= 0 && o->vel_steps <= 16, "vel_steps must be in [0, 16]");
    FSI_CHECK_ARG(o->tangent == 0 || o->tangent == 1, "tangent must be 0 (Picard) or 1 (full)");
    FSI_CHECK_ARG(o->pc_reuse == 0 || o->pc_reuse == 1, "pc_reuse must be 0 or 1");
    if (o->precond != FSI_PC_BJACOBI) {
        ScPlan sp;
        rc = sc_plan(make_geo(P64->grid), sp);
        if (rc) return rc;
    }
    if (P64->grid.order != 1 && o->tangent) {
        set_error("the full Newton tangent is implemented for Q1 grids");
        return FSI_ERR_UNSUPPORTED;
    }
    if (P64->solid != nullptr || (P32 != nullptr && P32->solid != nullptr)) {
        set_error("a problem carrying the solid block: its Newton step is fsi_newton_solid_solve (the solid passed "
                  "as its argument)");
        return FSI_ERR_UNSUPPORTED;
    }
    if (P64->n_occ > 0) FSI_CHECK_ARG(P64->dlm_gram != nullptr, "P64->dlm_gram required");
    if (o->inner == FSI_F32) {
        FSI_CHECK_ARG(P32 != nullptr, "inner FP32 needs the FP32 problem");
        rc = check_problem(P32);
        if (rc) return rc;
        FSI_CHECK_ARG(P32->dtype == FSI_F32, "P32 must be an FP32 problem");
        FSI_CHECK_ARG(std::memcmp(&P32->grid, &P64->grid, sizeof(fsi_grid)) == 0, "grids differ");
        if (P32->n_occ > 0) FSI_CHECK_ARG(P32->dlm_gram != nullptr, "P32->dlm_gram required");
        FSI_CHECK_ARG(std::isfinite(o->inner_reduction) && o->inner_reduction > 0.0 &&
                          o->inner_reduction < 1.0,
                      "inner_reduction must be in (0,1)");
    }
    rc = check_basis(o->basis, o->inner, o->restart);
    if (rc) return rc;
    return FSI_OK;
}

FSI_API size_t fsi_newton_workspace(const fsi_problem *P64, const fsi_problem *P32,
                                    const fsi_newton_opts *o)
{
    if (check_newton(P64, P32, o) != FSI_OK) return 0;
    size_t jw = jac_ws(P64);
    if (o->inner == FSI_F32) jw = std::max(jw, jac_ws(P32));
    return newton_workspace_bytes(make_geo(P64->grid), *o, jw);
}

FSI_API size_t fsi_tangent_workspace(const fsi_problem *P)
{
    clear_error();
    if (check_problem(P) != FSI_OK) return 0;
    return jac_ws(P);
}

FSI_API int fsi_tangent_apply(const fsi_problem *P, const void *x, const void *f, const void *v, void *y,
                              void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = check_problem(P);
    if (rc) return rc;
    if (P->grid.order != 1) {
        set_error("the full Newton tangent is implemented for Q1 grids");
        return FSI_ERR_UNSUPPORTED;
    }
    if (P->solid != nullptr) {
        set_error("a problem carrying the solid block: its step is fsi_newton_solid_solve (Picard only)");
        return FSI_ERR_UNSUPPORTED;
    }
    FSI_CHECK_ARG(x && f && v && y, "x, f, v and y must be non-NULL");
    FSI_CHECK_ARG(v != y && x != y && f != y, "y must not alias x, f or v");
    const Geo g = make_geo(P->grid);
    const size_t need = jac_ws(P);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    const DlmView dv = view_of(P);
    return launch_tangent_apply(g, P->prm, P->dtype, P->s, P->dir_mask, x, f, P->n_occ > 0 ? &dv : nullptr, v, y,
                                ws, as_stream(stream));
}

FSI_API int fsi_newton_solve(const fsi_problem *P64, const fsi_problem *P32, const double *f,
                             const double *lamg, const double *gD, double *x,
                             const fsi_newton_opts *o, fsi_newton_stats *stats, void *ws,
                             size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = check_newton(P64, P32, o);
    if (rc) return rc;
    FSI_CHECK_ARG(f && x, "f and x must be non-NULL");
    FSI_CHECK_ARG(P64->dir_mask == nullptr || gD != nullptr, "gD required with a Dirichlet mask");
    size_t jw = jac_ws(P64);
    if (o->inner == FSI_F32) jw = std::max(jw, jac_ws(P32));
    const Geo g = make_geo(P64->grid);
    const size_t need = newton_workspace_bytes(g, *o, jw);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    return newton_solve(g, *P64, o->inner == FSI_F32 ? P32 : nullptr, f, lamg, gD, x, *o, stats, ws, jw,
                        as_stream(stream));
}

FSI_API size_t fsi_newton_solid_workspace(const fsi_problem *P64, const fsi_problem *P32, const fsi_solid *S,
                                          const fsi_newton_opts *o)
{
    if (check_newton(P64, P32, o) != FSI_OK || check_solid(S) != FSI_OK) return 0;
    size_t jw = problem_ws(P64, S);
    if (o->inner == FSI_F32) jw = std::max(jw, problem_ws(P32, S));
    return newton_workspace_bytes(make_geo(P64->grid), *o, jw);
}

FSI_API int fsi_newton_solid_solve(const fsi_problem *P64, const fsi_problem *P32, const fsi_solid *S,
                                   const double *U_base, const double *A_base, double cU, double cA,
                                   const double *f, const double *gD, double *x, double *U, double *V,
                                   const fsi_newton_opts *o, fsi_newton_stats *stats, void *ws, size_t ws_bytes,
                                   void *stream)
{
    clear_error();
    int rc = check_newton(P64, P32, o);
    if (rc) return rc;
    rc = check_solid_step(P64, S, U_base, A_base, cU, cA, U, V);
    if (rc) return rc;
    if (o->inner == FSI_F32) FSI_CHECK_ARG(P32->m == S->n_nodes, "P32's points must be the solid's nodes");
    FSI_CHECK_ARG(o->tangent == 0, "the full tangent is not available with the solid block");
    FSI_CHECK_ARG(f && x, "f and x must be non-NULL");
    FSI_CHECK_ARG(P64->dir_mask == nullptr || gD != nullptr, "gD required with a Dirichlet mask");
    size_t jw = problem_ws(P64, S);
    if (o->inner == FSI_F32) jw = std::max(jw, problem_ws(P32, S));
    const Geo g = make_geo(P64->grid);
    const size_t need = newton_workspace_bytes(g, *o, jw);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    const SolidStep ss{S, U_base, A_base, cU, cA, U, V};
    return newton_solve(g, *P64, o->inner == FSI_F32 ? P32 : nullptr, f, nullptr, gD, x, *o, stats, ws, jw,
                        as_stream(stream), &ss);
}

// ---------------------------------------------------------------- warm-start network
static int check_dims(const int32_t *dims)
{
    FSI_CHECK_ARG(dims != nullptr, "dims is NULL");
    FSI_CHECK_ARG(dims[0] >= 1 && dims[1] >= 1 && dims[2] >= 1, "dims must be >= 1");
    FSI_CHECK_ARG((int64_t)dims[0] * dims[1] * dims[2] < ((int64_t)1 << 31), "lattice too large");
    return FSI_OK;
}

static bool chan_ok(int32_t c) { return c >= 32 && c % 32 == 0 && c <= 1024; }

FSI_API int fsi_conv3d_fwd(const int32_t *dims, int32_t cin, int32_t cout, const uint16_t *X,
                           const uint16_t *W, const float *bias, int32_t relu, const uint16_t *gate,
                           uint16_t *Y_bf16, float *Y_f32, void *stream)
{
    clear_error();
    int rc = check_dims(dims);
    if (rc) return rc;
    FSI_CHECK_ARG(chan_ok(cin) && chan_ok(cout), "cin and cout must be multiples of 32 in [32, 1024]");
    FSI_CHECK_ARG(X && W && (Y_bf16 || Y_f32), "X, W and an output must be non-NULL");
    return nn_conv_fwd(dims, cin, cout, X, W, bias, relu, gate, Y_bf16, Y_f32, as_stream(stream));
}

FSI_API size_t fsi_conv3d_wgrad_workspace(const int32_t *dims, int32_t cin, int32_t cout)
{
    if (check_dims(dims) != FSI_OK || !chan_ok(cin) || !chan_ok(cout)) return 0;
    return nn_wgrad_workspace(dims, cin, cout);
}

FSI_API int fsi_conv3d_wgrad(const int32_t *dims, int32_t cin, int32_t cout, const uint16_t *dY,
                             const uint16_t *X, float *dW, float *db, void *ws, size_t ws_bytes,
                             void *stream)
{
    clear_error();
    int rc = check_dims(dims);
    if (rc) return rc;
    FSI_CHECK_ARG(chan_ok(cin) && chan_ok(cout), "cin and cout must be multiples of 32 in [32, 1024]");
    FSI_CHECK_ARG(dY && X && dW, "dY, X and dW must be non-NULL");
    const size_t need = nn_wgrad_workspace(dims, cin, cout);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes needed (got %zu)", need, ws_bytes);
        return FSI_ERR_WORKSPACE;
    }
    return nn_conv_wgrad(dims, cin, cout, dY, X, dW, db, ws, as_stream(stream));
}

FSI_API int fsi_conv3d_flip_transpose(int32_t cin, int32_t cout, const uint16_t *W, uint16_t *Wd,
                                      void *stream)
{
    clear_error();
    FSI_CHECK_ARG(chan_ok(cin) && chan_ok(cout), "cin and cout must be multiples of 32 in [32, 1024]");
    FSI_CHECK_ARG(W && Wd && W != Wd, "W and Wd must be non-NULL and distinct");
    return nn_flip_transpose(cin, cout, W, Wd, as_stream(stream));
}

FSI_API size_t fsi_mse_workspace(void) { return nn_mse_workspace(); }

FSI_API int fsi_mse_loss(int64_t nvox, int32_t c, int32_t used, const float *pred, const float *target,
                         uint16_t *dpred, double *loss_host, void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    FSI_CHECK_ARG(nvox >= 1 && c >= 1 && used >= 1 && used <= c, "bad sizes");
    FSI_CHECK_ARG(pred && target, "pred and target must be non-NULL");
    if (ws == nullptr || ws_bytes < nn_mse_workspace()) {
        set_error("workspace of %zu bytes needed", nn_mse_workspace());
        return FSI_ERR_WORKSPACE;
    }
    return nn_mse(nvox, c, used, pred, target, dpred, loss_host, ws, as_stream(stream));
}

FSI_API int fsi_adam_step(int64_t n, float *w, const float *g, float *m, float *v, uint16_t *w_bf16,
                          int32_t t, float lr, float b1, float b2, float eps, void *stream)
{
    clear_error();
    FSI_CHECK_ARG(n >= 1 && w && g && m && v, "bad arguments");
    FSI_CHECK_ARG(t >= 1, "t counts from 1");
    FSI_CHECK_ARG(b1 >= 0.f && b1 < 1.f && b2 >= 0.f && b2 < 1.f && eps >= 0.f, "bad Adam constants");
    return nn_adam(n, w, g, m, v, w_bf16, t, lr, b1, b2, eps, as_stream(stream));
}

FSI_API int fsi_to_bf16(int64_t n, const float *in, uint16_t *out, void *stream)
{
    clear_error();
    FSI_CHECK_ARG(n >= 1 && in && out, "bad arguments");
    return nn_to_bf16(n, in, out, as_stream(stream));
}

FSI_API int fsi_nn_pack(int64_t nvox, int32_t c, const fsi_nn_pack_spec *p, float *out, void *stream)
{
    clear_error();
    FSI_CHECK_ARG(p && out && nvox >= 1, "bad arguments");
    FSI_CHECK_ARG(p->nch >= 0 && p->nch <= 32 && p->nch <= c && c >= 1, "bad channel counts");
    return nn_pack(nvox, c, *p, out, as_stream(stream));
}

FSI_API size_t fsi_nn_moments_workspace(int32_t c) { return c >= 1 ? nn_moments_workspace(c) : 0; }

FSI_API int fsi_nn_moments(int64_t nvox, int32_t c, const float *data, double *sums_host, void *ws,
                           size_t ws_bytes, void *stream)
{
    clear_error();
    FSI_CHECK_ARG(nvox >= 1 && c >= 1 && data && sums_host, "bad arguments");
    if (ws == nullptr || ws_bytes < nn_moments_workspace(c)) {
        set_error("workspace of %zu bytes needed", nn_moments_workspace(c));
        return FSI_ERR_WORKSPACE;
    }
    return nn_moments(nvox, c, data, sums_host, ws, as_stream(stream));
}

FSI_API int fsi_nn_unpack(int64_t nvox, int32_t c, const float *out, const double *base,
                          const fsi_nn_unpack_spec *u, const uint32_t *dir_mask, const double *gD,
                          double *x, void *stream)
{
    clear_error();
    FSI_CHECK_ARG(nvox >= 1 && c >= 4 && out && base && u && x, "bad arguments");
    return nn_unpack(nvox, c, out, base, *u, dir_mask, gD, x, as_stream(stream));
}

// ---------------------------------------------------------------- BLAS-1 helpers
FSI_API int fsi_axpby(int64_t n, double alpha, const double *x, double beta, double *y, void *stream)
{
    clear_error();
    FSI_CHECK_ARG(n >= 0 && (n == 0 || (x && y)), "bad arguments");
    if (n == 0) return FSI_OK;
    if (beta == 0.0) return kry_scale(n, alpha, x, y, as_stream(stream));
    return kry_axpby(n, alpha, x, beta, y, as_stream(stream));
}

FSI_API size_t fsi_dot_workspace(void) { return align_up((size_t)(KRY_NB + 8) * sizeof(double)); }

FSI_API int fsi_dot(int64_t n, const double *x, const double *y, double *out_host, void *ws,
                    size_t ws_bytes, void *stream)
{
    clear_error();
    FSI_CHECK_ARG(n >= 1 && x && y && out_host, "bad arguments");
    if (ws == nullptr || ws_bytes < fsi_dot_workspace()) {
        set_error("workspace of %zu bytes needed", fsi_dot_workspace());
        return FSI_ERR_WORKSPACE;
    }
    double *part = reinterpret_cast<double *>(ws);
    hipStream_t st = as_stream(stream);
    int rc = kry_multidot(n, 1, x, n, y, part, part + KRY_NB, st);
    if (rc) return rc;
    FSI_HIP(hipMemcpyAsync(out_host, part + KRY_NB, sizeof(double), hipMemcpyDeviceToHost, st));
    FSI_HIP(hipStreamSynchronize(st));
    return FSI_OK;
}
