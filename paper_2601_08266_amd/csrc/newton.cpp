// Newton's method for one implicit step (section 2.4), host-driven:
//   R_k = R(x_k)                      (residual kernel, FP64)
//   P_k = preconditioner of J(u_k)    (nodal block-Jacobi inverses, or the Schur-complement
//                                      block preconditioner built from the nodal blocks)
//   J(u_k) dx = -R_k                  (flexible GMRES, FP64 outer / inner precision); J is the
//                                      Picard/Oseen operator, or the full Newton tangent (the
//                                      Picard cells plus the tangent-correction cells, in the
//                                      inner precision)
//   x_{k+1} = x_k + dx
#include <algorithm>
#include <chrono>
#include <cmath>

#include "bjacobi.hpp"
#include "fgmres.hpp"
#include "krylov.hpp"
#include "newton.hpp"
#include "profile.hpp"
#include "schur.hpp"

namespace fsi {

namespace {

struct NLayout {
    size_t R, dx, pinv64, pinv32, blocks, pc, a32, f32, scratch, bjws, kws, total;
};

NLayout nlayout(const Geo &g, const fsi_newton_opts &o, size_t jws)
{
    NLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t r = off;
        off += align_up(bytes);
        return r;
    };
    L.R = take((size_t)4 * g.N * sizeof(double));
    L.dx = take((size_t)4 * g.N * sizeof(double));
    if (o.precond == FSI_PC_BJACOBI) {
        L.pinv64 = take((size_t)16 * g.N * sizeof(double));
        L.pinv32 = take((size_t)16 * g.N * sizeof(float));
    } else {
        ScPlan sp;
        const size_t pcb = sc_plan(g, sp) == FSI_OK ? sp.total : 0;
        L.blocks = take((size_t)16 * g.N * sizeof(double));
        L.pc = take(pcb);
    }
    // FP32 copy of the iterate (its velocity is the Picard advection field; the full tangent
    // also reads its pressure) and of the source (full tangent)
    L.a32 = take((size_t)4 * g.N * sizeof(float));
    L.f32 = o.tangent ? take((size_t)3 * g.N * sizeof(float)) : 0;
    L.scratch = take((size_t)(KRY_NB + 16) * sizeof(double));
    L.bjws = take(bjacobi_workspace_bytes(g));
    L.kws = take(fgmres_workspace_bytes(4 * g.N, o.restart, o.inner, o.basis, jws));
    L.total = off;
    return L;
}

double ms_since(std::chrono::steady_clock::time_point t)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
}

}  // namespace

size_t newton_workspace_bytes(const Geo &g, const fsi_newton_opts &o, size_t jws)
{
    return nlayout(g, o, jws).total;
}

int newton_solve(const Geo &g, const fsi_problem &P64, const fsi_problem *P32, const double *f,
                 const double *lamg, const double *gD, double *x, const fsi_newton_opts &o,
                 fsi_newton_stats *stats, void *ws, size_t jws, hipStream_t st, const SolidStep *ss)
{
    ProfileScope prof("newton_solve", st);
    const auto t0 = std::chrono::steady_clock::now();
    const NLayout L = nlayout(g, o, jws);
    char *base = reinterpret_cast<char *>(ws);
    double *R = reinterpret_cast<double *>(base + L.R);
    double *dx = reinterpret_cast<double *>(base + L.dx);
    double *pinv64 = reinterpret_cast<double *>(base + L.pinv64);
    float *pinv32 = reinterpret_cast<float *>(base + L.pinv32);
    double *blocks = reinterpret_cast<double *>(base + L.blocks);
    void *pcobj = base + L.pc;
    const bool schur = o.precond != FSI_PC_BJACOBI;
    float *a32 = reinterpret_cast<float *>(base + L.a32);
    float *f32 = o.tangent ? reinterpret_cast<float *>(base + L.f32) : nullptr;
    void *bjws = base + L.bjws;
    void *kws = base + L.kws;
    const int64_t n = 4 * g.N;

    fsi_newton_stats S{};
    int rc = FSI_OK;
    DlmView v64{P64.m,     P64.cell,      P64.xi,    P64.perm,     P64.occ_cell, P64.occ_start,
                P64.n_occ, P64.occ_index, P64.kappa, P64.dlm_gram};
    DlmView v32{};
    if (P32) v32 = DlmView{P32->m,     P32->cell,      P32->xi,    P32->perm,     P32->occ_cell,
                           P32->occ_start, P32->n_occ, P32->occ_index, P32->kappa, P32->dlm_gram};
    if (ss != nullptr) {
        // the operator's solid block at the current iterate (U is refreshed by every residual);
        // kappa and the per-cell blocks stay for the preconditioners
        for (DlmView *dv : {&v64, &v32}) {
            dv->solid = ss->S;
            dv->solid_U = ss->U;
            dv->solid_c = SolidCoefs{ss->cA, ss->cU, 1.0};
        }
    }
    double *scratch = reinterpret_cast<double *>(base + L.scratch);
    auto rnorm = [&](double &out) -> int {
        int r = kry_norm(n, R, scratch, scratch + KRY_NB, st);
        if (r) return r;
        FSI_HIP(hipMemcpyAsync(&out, scratch + KRY_NB, sizeof(double), hipMemcpyDeviceToHost, st));
        FSI_HIP(hipStreamSynchronize(st));
        return FSI_OK;
    };
    if (o.tangent && o.inner == FSI_F32) {
        rc = kry_cast_f64_f32(3 * g.N, f, f32, st);
        if (rc) {
            if (stats) *stats = S;
            return rc;
        }
    }
    for (int it = 0;; ++it) {
        auto tr = std::chrono::steady_clock::now();
        if (ss != nullptr)
            rc = solid_step_residual(g, P64, *ss, f, gD, x, R, kws, st);
        else
            rc = launch_vms_residual(g, P64.prm, FSI_F64, P64.s, P64.dir_mask, gD, x, f,
                                     P64.n_occ > 0 ? &v64 : nullptr, lamg, R, kws, st);
        if (rc) break;
        double rn = 0.0;
        rc = rnorm(rn);
        if (rc) break;
        S.t_residual_ms += ms_since(tr);
        if (it < 32) S.res_hist[it] = rn;
        if (!std::isfinite(rn)) {
            set_error("Newton residual is NaN/Inf");
            rc = FSI_ERR_NAN;
            break;
        }
        if (rn <= o.tol_abs) break;
        if (it >= o.max_newton) {
            set_error("Newton: no convergence in %d iterations (||R|| = %.3e, target %.3e)", it, rn,
                      o.tol_abs);
            rc = FSI_ERR_NOT_CONVERGED;
            break;
        }
        // J(u_k): advection field = current velocity (first 3N of x)
        auto ts = std::chrono::steady_clock::now();
        fsi_problem J64 = P64;
        J64.a = x;
        const double *gram64 = J64.n_occ > 0 ? (const double *)J64.dlm_gram : nullptr;
        // the preconditioner at u_k, or (pc_reuse) the one built at the call's first iterate
        const bool build_pc = it == 0 || !o.pc_reuse;
        if (build_pc && schur) {
            rc = launch_bjacobi_setup(g, J64.prm, x, (const double *)J64.s, J64.dir_mask, gram64, J64.occ_index,
                                      blocks, nullptr, nullptr, nullptr, bjws, st);
            if (rc) break;
            rc = schur_setup(g, J64.prm, x, (const double *)J64.s, J64.dir_mask, gram64, J64.occ_index, blocks,
                             pcobj, st);
        } else if (build_pc) {
            rc = launch_bjacobi_setup(g, J64.prm, x, (const double *)J64.s, J64.dir_mask, gram64, J64.occ_index,
                                      nullptr, pinv64, o.inner == FSI_F32 ? pinv32 : nullptr, nullptr, bjws,
                                      st);
        }
        if (rc) break;
        fsi_problem J32{};
        if (o.inner == FSI_F32) {
            rc = kry_cast_f64_f32((o.tangent ? 4 : 3) * g.N, x, a32, st);
            if (rc) break;
            J32 = *P32;
            J32.a = a32;
        }
        S.t_setup_ms += ms_since(ts);
        // b = -R, dx = 0
        auto tk = std::chrono::steady_clock::now();
        rc = kry_scale(n, -1.0, R, R, st);
        if (rc) break;
        FSI_HIP(hipMemsetAsync(dx, 0, (size_t)n * sizeof(double), st));
        fsi_solve_opts so{};
        so.restart = o.restart;
        so.max_iters = o.max_krylov;
        // forcing: eta, or what the last iteration needs (half the remaining reduction).  With
        // the full tangent (quadratic convergence) the first iteration solves to at most the
        // square root of that and the next ones to the final target, so that two iterations
        // reach it when the quadratic term is small
        const double last = 0.5 * o.tol_abs / rn;
        double eta = o.eta;
        if (o.tangent) eta = it == 0 ? std::min(o.eta, std::sqrt(last)) : last;
        so.rtol = std::max(eta, last);
        if (so.rtol >= 1.0) so.rtol = 0.5;
        so.inner = o.inner;
        so.inner_reduction = o.inner_reduction;
        so.basis = o.basis;
        JacobianCall c64{[&](const void *xx, void *yy, void *w, hipStream_t s2) {
            return launch_vms_apply(g, J64.prm, FSI_F64, J64.a, J64.s, J64.dir_mask, xx, yy,
                                    J64.n_occ > 0 ? &v64 : nullptr, w, jws, s2);
        }};
        JacobianCall c32{[&](const void *xx, void *yy, void *w, hipStream_t s2) {
            return launch_vms_apply(g, J32.prm, FSI_F32, J32.a, J32.s, J32.dir_mask, xx, yy,
                                    J32.n_occ > 0 ? &v32 : nullptr, w, jws, s2);
        }};
        if (g.p == 1) {
            // the Schur preconditioner's products with the velocity and pressure-gradient blocks
            c64.block = [&](int blk, const void *xx, void *yy, void *w, hipStream_t s2) {
                return launch_vms_apply_block(g, J64.prm, FSI_F64, blk, J64.a, J64.s, J64.dir_mask, xx, yy,
                                              J64.n_occ > 0 ? &v64 : nullptr, w, s2);
            };
            c32.block = [&](int blk, const void *xx, void *yy, void *w, hipStream_t s2) {
                return launch_vms_apply_block(g, J32.prm, FSI_F32, blk, J32.a, J32.s, J32.dir_mask, xx, yy,
                                              J32.n_occ > 0 ? &v32 : nullptr, w, s2);
            };
        }
        const JacobianCall *Jin = o.inner == FSI_F32 ? &c32 : &c64;
        const int mode = o.precond == FSI_PC_SCHUR_DIAG ? 1 : 2;
        Precond pc;
        const bool basis64 = o.basis != FSI_F32;   // the basis vectors the preconditioner reads
        if (schur)
            pc.apply = [&](const void *v, void *z, void *w, hipStream_t s2) {
                return schur_apply(g, o.inner, basis64, mode, o.vel_steps, pcobj, v, z, Jin, w, s2);
            };
        else
            pc.apply = [&](const void *v, void *z, void *, hipStream_t s2) {
                if (!basis64) return launch_bjacobi_apply(g.N, FSI_F32, pinv32, v, z, s2);
                if (o.inner == FSI_F32)
                    return launch_bjacobi_apply_f64_to_f32(g.N, pinv32, (const double *)v, (float *)z, s2);
                return launch_bjacobi_apply(g.N, FSI_F64, pinv64, v, z, s2);
            };
        so.precond = o.precond;
        so.vel_steps = o.vel_steps;
        so.host_ring = o.host_ring;
        so.host_ring_len = o.host_ring_len;
        fsi_solve_stats ks{};
        // operator of the linear solve: the Picard/Oseen J, or the full Newton tangent at x_k in
        // the same precision; the preconditioner keeps the Picard operator
        JacobianCall t64{[&](const void *xx, void *yy, void *w, hipStream_t s2) {
            return launch_tangent_apply(g, J64.prm, FSI_F64, J64.s, J64.dir_mask, x, f,
                                        J64.n_occ > 0 ? &v64 : nullptr, xx, yy, w, s2);
        }};
        JacobianCall t32{[&](const void *xx, void *yy, void *w, hipStream_t s2) {
            return launch_tangent_apply(g, J32.prm, FSI_F32, J32.s, J32.dir_mask, a32, f32,
                                        J32.n_occ > 0 ? &v32 : nullptr, xx, yy, w, s2);
        }};
        const JacobianCall &op64 = o.tangent ? t64 : c64;
        const JacobianCall &op32 = o.tangent ? t32 : c32;
        rc = fgmres_solve(g, op64, o.inner == FSI_F32 ? &op32 : nullptr, &pc, R, dx, so, &ks, kws, jws, st,
                          true);   // dx = 0 (cleared above)
        S.krylov_iters += ks.iters;
        S.t_krylov_ms += ms_since(tk);
        if (rc == FSI_ERR_NOT_CONVERGED) rc = FSI_OK;   // inexact Newton: take the step anyway
        if (rc) break;
        rc = kry_axpby(n, 1.0, dx, 1.0, x, st);
        if (rc) break;
        ++S.newton_iters;
    }
    S.status = rc;
    (void)hipStreamSynchronize(st);
    S.t_total_ms = ms_since(t0);
    if (stats) *stats = S;
    return rc;
}

}  // namespace fsi
