// Flexible GMRES with right preconditioning, restarted, host-driven.
//
// Precision split: the Krylov basis V, the CGS2 orthogonalisation, the
// Hessenberg/Givens recurrences, the solution x and the restart residual
// b - J x are FP64; the preconditioner and Jacobian applies inside a cycle
// run in the inner precision (FP32 or FP64) and the preconditioned vectors Z
// are stored in that precision.  Every restart begins from the true FP64
// residual, so the FP32 inner cycles act as iterative refinement steps.
// With an FP32 inner precision the basis may also be stored in FP32
// (opts.basis): the Gram-Schmidt passes then read half the bytes, while
// their products and sums, and the Gram matrix of the stored vectors that
// the second projection uses, stay FP64; a cycle already stops at the FP32
// level (inner_reduction), which such a basis resolves.
// Section 2.4 solves the reduced block system with block-preconditioned
// Krylov iterations; this is that loop, with the preconditioner passed in as a callable
// (nodal block-Jacobi or the Schur-complement block preconditioner).
#include <chrono>
#include <cmath>
#include <vector>

#include "fgmres.hpp"
#include "krylov.hpp"
#include "profile.hpp"
#include "stall.hpp"

namespace fsi {

namespace {

struct Layout {
    size_t V, Z, w64, t32b, partial, hdev, gram, jws, total;
};

Layout layout(int64_t n, int m, fsi_dtype inner, fsi_dtype basis, size_t jws_bytes)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return o;
    };
    L.V = take((size_t)(m + 1) * n * (basis == FSI_F32 ? sizeof(float) : sizeof(double)));
    L.Z = take((size_t)m * n * (inner == FSI_F64 ? sizeof(double) : sizeof(float)));
    L.w64 = take((size_t)n * sizeof(double));
    L.t32b = take((size_t)n * sizeof(float));
    L.partial = take((size_t)(2 * (m + 2)) * KRY_NB * sizeof(double));
    L.hdev = take((size_t)(4 * (m + 1) + 2) * sizeof(double));
    L.gram = take((size_t)(m + 1) * (m + 1) * sizeof(double));
    L.jws = take(jws_bytes);
    L.total = off;
    return L;
}

// The per-step events of one solve, created at its start and destroyed when it returns.
struct StepEvents {
    std::vector<hipEvent_t> ev;
    ~StepEvents()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    int create(int m)
    {
        while ((int)ev.size() < m) {
            hipEvent_t e = nullptr;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                set_error("hipEventCreate failed");
                return FSI_ERR_HIP;
            }
            ev.push_back(e);
        }
        return FSI_OK;
    }
};

}  // namespace

size_t fgmres_workspace_bytes(int64_t ndof, int restart, fsi_dtype inner, fsi_dtype basis, size_t jws_bytes)
{
    return layout(ndof, restart, inner, basis, jws_bytes).total;
}

int fgmres_solve(const Geo &g, const JacobianCall &J64, const JacobianCall *J32, const Precond *pc,
                 const double *b, double *x, const fsi_solve_opts &o, fsi_solve_stats *stats,
                 void *ws, size_t jws_bytes, hipStream_t st, bool x_zero)
{
    ProfileScope prof("fgmres_solve", st);
    const auto t_start = std::chrono::steady_clock::now();
    const int64_t n = 4 * g.N;
    const int m = o.restart;
    const fsi_dtype inner = o.inner;
    const bool b32 = o.basis == FSI_F32;   // basis stored in FP32 (the caller checked inner = FP32)
    const Layout L = layout(n, m, inner, o.basis, jws_bytes);
    char *base = reinterpret_cast<char *>(ws);
    double *V = reinterpret_cast<double *>(base + L.V);
    float *V32 = reinterpret_cast<float *>(base + L.V);
    void *Z = base + L.Z;
    double *w64 = reinterpret_cast<double *>(base + L.w64);
    float *t32b = reinterpret_cast<float *>(base + L.t32b);
    double *partial = reinterpret_cast<double *>(base + L.partial);
    double *hdev = reinterpret_cast<double *>(base + L.hdev);
    double *Gdev = reinterpret_cast<double *>(base + L.gram);
    void *jws = base + L.jws;
    const size_t zel = inner == FSI_F64 ? sizeof(double) : sizeof(float);

    fsi_solve_stats S{};
    int rc = FSI_OK;
    auto fetch = [&](double *host, const double *dev, int count) -> int {
        FSI_HIP(hipMemcpyAsync(host, dev, count * sizeof(double), hipMemcpyDeviceToHost, st));
        FSI_HIP(hipStreamSynchronize(st));
        return FSI_OK;
    };
#define TRY(expr)            \
    do {                     \
        rc = (expr);         \
        if (rc) goto done;   \
    } while (0)

    {
        double bnorm = 0.0;
        TRY(kry_norm(n, b, partial, hdev, st));
        TRY(fetch(&bnorm, hdev, 1));
        S.bnorm = bnorm;
        if (!std::isfinite(bnorm)) {
            set_error("right-hand side contains NaN/Inf");
            rc = FSI_ERR_NAN;
            goto done;
        }
        if (bnorm == 0.0) {
            FSI_HIP(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), st));
            S.res0 = S.res_final = 0.0;
            goto done;
        }
        const double target = o.rtol * bnorm;
        std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), y(m),
            hcopy(2 * (m + 1) + 1);
        (void)0;
        double prev_beta = -1.0;
        int stalls = 0;
        // host copies of the per-step coefficients: the caller's pinned ring (copies run behind
        // the device, see below) or, without one, host memory of this call with a wait per step
        const size_t ring_len = (size_t)m * (m + 2);
        const bool pinned = o.host_ring != nullptr;
        if (pinned && o.host_ring_len < (int64_t)ring_len) {
            set_error("host_ring holds %lld doubles, %zu needed", (long long)o.host_ring_len, ring_len);
            rc = FSI_ERR_ARG;
            goto done;
        }
        std::vector<double> own_ring(pinned ? 0 : ring_len);
        double *hring = pinned ? o.host_ring : own_ring.data();
        StepEvents events;
        TRY(events.create(m));
        std::vector<hipEvent_t> &ev = events.ev;
        for (;;) {
            // true residual r = b - J64 x in FP64 (stored in V[0]); b itself while x is still the
            // zero the caller guaranteed (then its norm is the one already computed)
            // (with an FP32 basis the residual is formed in w64 and rounded as it is scaled)
            double beta = 0.0;
            const double *r0 = b32 ? w64 : V;
            if (x_zero && S.cycles == 0) {
                // hdev[0] still holds ||b|| from the norm above, which the scaling below reads
                if (b32) r0 = b;
                else FSI_HIP(hipMemcpyAsync(V, b, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
                beta = bnorm;
            } else {
                {
                    ProfileScope pr("fgmres_residual", st);
                    TRY(J64.apply(x, w64, jws, st));
                    if (b32) {
                        TRY(kry_axpby(n, 1.0, b, -1.0, w64, st));
                    } else {
                        FSI_HIP(hipMemcpyAsync(V, b, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
                        TRY(kry_axpby(n, -1.0, w64, 1.0, V, st));
                    }
                }
                TRY(kry_norm(n, r0, partial, hdev, st));
                TRY(fetch(&beta, hdev, 1));
            }
            if (S.cycles == 0) S.res0 = beta;
            S.res_final = beta;
            if (!std::isfinite(beta)) {
                set_error("residual norm is NaN/Inf");
                rc = FSI_ERR_NAN;
                goto done;
            }
            if (beta <= target) break;
            if (S.iters >= o.max_iters) {
                set_error("no convergence in %d iterations (residual %.3e, target %.3e)", S.iters,
                          beta, target);
                rc = FSI_ERR_NOT_CONVERGED;
                goto done;
            }
            if (krylov_stagnated(prev_beta, beta, stalls)) {
                set_error("stagnation at residual %.3e (target %.3e)", beta, target);
                rc = FSI_ERR_NOT_CONVERGED;
                goto done;
            }
            prev_beta = beta;
            if (b32) TRY(kry_scale_inv_to_f32(n, r0, hdev, V32, st));
            else TRY(kry_scale_inv(n, V, hdev, V, st));
            std::fill(gv.begin(), gv.end(), 0.0);
            gv[0] = beta;
            // an FP32 inner cycle cannot resolve much below its own rounding level
            double cycle_target = target;
            if (inner == FSI_F32) cycle_target = std::max(target, o.inner_reduction * beta);
            // The Arnoldi steps are enqueued without waiting for the host: the coefficients stay
            // on the device, and each step's (h, ||w||) is copied to pinned host memory behind
            // it.  The host applies the Givens rotations one step behind the device, so the
            // convergence test lags by one step (at most one extra step per cycle is computed
            // and then ignored).
            int kk = 0, enq = 0;
            bool stop = false;
            auto process = [&](int j) -> int {
                // Givens update of Hessenberg column j from the host copy of its coefficients
                FSI_HIP(hipEventSynchronize(ev[j]));
                const double *hc = hring + (size_t)j * (m + 2);
                const double hn = hc[m + 1];
                for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hc[i];
                H[(size_t)(j + 1) * m + j] = hn;
                if (!std::isfinite(hn)) {
                    set_error("Arnoldi vector norm is NaN/Inf");
                    return FSI_ERR_NAN;
                }
                for (int i = 0; i < j; ++i) {
                    const double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
                    H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
                    H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
                }
                const double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
                const double den = std::hypot(a, c);
                if (den == 0.0) {
                    set_error("Krylov breakdown (zero Hessenberg column)");
                    return FSI_ERR_BREAKDOWN;
                }
                cs[j] = a / den;
                sn[j] = c / den;
                H[(size_t)j * m + j] = den;
                H[(size_t)(j + 1) * m + j] = 0.0;
                gv[j + 1] = -sn[j] * gv[j];
                gv[j] = cs[j] * gv[j];
                ++S.iters;
                kk = j + 1;
                if (std::fabs(gv[j + 1]) <= cycle_target || hn == 0.0) stop = true;
                return FSI_OK;
            };
            for (int j = 0; j < m && !stop && S.iters + (enq - kk) < o.max_iters; ++j) {
                double *Vj = V + (size_t)j * n;
                float *Vj32 = V32 + (size_t)j * n;
                char *Zj = reinterpret_cast<char *>(Z) + (size_t)j * n * zel;
                if (inner == FSI_F32) {
                    {
                        ProfileScope pp("fgmres_precond", st);
                        if (pc) TRY(pc->apply(b32 ? (const void *)Vj32 : (const void *)Vj, Zj, jws, st));
                        else if (b32)
                            FSI_HIP(hipMemcpyAsync(Zj, Vj32, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, st));
                        else TRY(kry_cast_f64_f32(n, Vj, reinterpret_cast<float *>(Zj), st));
                    }
                    ProfileScope pa("fgmres_apply", st);
                    TRY(J32->apply(Zj, t32b, jws, st));
                    // the fused Gram-Schmidt passes read the FP32 product and widen it as they
                    // go; the unfused ones take it widened
                    if (j + 1 > KRY_FUSED_MAXK && !b32) TRY(kry_cast_f32_f64(n, t32b, w64, st));
                } else {
                    {
                        ProfileScope pp("fgmres_precond", st);
                        if (pc) TRY(pc->apply(Vj, Zj, jws, st));
                        else FSI_HIP(hipMemcpyAsync(Zj, Vj, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
                    }
                    ProfileScope pa("fgmres_apply", st);
                    TRY(J64.apply(Zj, w64, jws, st));
                }
                // classical Gram-Schmidt with re-orthogonalisation through the Gram matrix
                // G = V^T V of the basis: one pass gives a = V^T w and the new Gram column
                // V^T V_j; the second projection V^T (w - V a) = a - G a needs no further pass,
                // so w -= V (a + (a - G a)) and ||w|| complete the step in a second pass.
                double *d_ab = hdev, *d_h = hdev + 2 * (m + 1), *d_hn = hdev + 3 * (m + 1);
                {
                    ProfileScope po("fgmres_orth", st);
                    if (b32) {
                        // w - V h goes straight into the next basis slot, rounded to FP32
                        TRY(kry_cgs_project_b32(n, j + 1, V32, n, t32b, Vj32, partial, d_ab, Gdev, m + 1, d_h, st));
                        TRY(kry_axpy_norm_b32(n, j + 1, V32, n, d_h, t32b, V32 + (size_t)(j + 1) * n, partial, d_hn,
                                              st));
                    } else if (j + 1 <= KRY_FUSED_MAXK && inner == FSI_F32) {
                        TRY(kry_cgs_project_f32w(n, j + 1, V, n, t32b, Vj, partial, d_ab, Gdev, m + 1, d_h, st));
                        TRY(kry_axpy_norm_f32w(n, j + 1, V, n, d_h, t32b, w64, partial, d_hn, st));
                    } else if (j + 1 <= KRY_FUSED_MAXK) {
                        TRY(kry_cgs_project(n, j + 1, V, n, w64, Vj, partial, d_ab, Gdev, m + 1, d_h, st));
                        TRY(kry_axpy_norm(n, j + 1, V, n, d_h, w64, partial, d_hn, st));
                    } else {
                        TRY(kry_multidot2(n, j + 1, V, n, w64, Vj, partial, d_ab, st));
                        TRY(kry_gram_coeffs(j + 1, d_ab, Gdev, m + 1, d_h, st));
                        TRY(kry_axpy_dot(n, j + 1, V, n, d_h, w64, 0, partial, d_hn, st));
                    }
                }
                FSI_HIP(hipMemcpyAsync(hring + (size_t)j * (m + 2), d_h, (size_t)(m + 2) * sizeof(double),
                                       hipMemcpyDeviceToHost, st));
                FSI_HIP(hipEventRecord(ev[j], st));
                if (!pinned) FSI_HIP(hipEventSynchronize(ev[j]));
                // next basis vector (if ||w|| = 0 the step ends the cycle and this vector is unused)
                if (b32) TRY(kry_scale_inv_f32(n, V32 + (size_t)(j + 1) * n, d_hn, V32 + (size_t)(j + 1) * n, st));
                else TRY(kry_scale_inv(n, w64, d_hn, V + (size_t)(j + 1) * n, st));
                ++enq;
                if (j >= 1) TRY(process(j - 1));
            }
            if (!stop && enq > kk) TRY(process(enq - 1));
            // y = H^{-1} g (upper triangular), x += Z y
            for (int i = kk - 1; i >= 0; --i) {
                double s = gv[i];
                for (int k2 = i + 1; k2 < kk; ++k2) s -= H[(size_t)i * m + k2] * y[k2];
                y[i] = s / H[(size_t)i * m + i];
            }
            FSI_HIP(hipMemcpyAsync(hdev, y.data(), kk * sizeof(double), hipMemcpyHostToDevice, st));
            TRY(kry_update(n, kk, inner, Z, n, hdev, x, st));
            FSI_HIP(hipStreamSynchronize(st));   // y lives on the host stack frame
            ++S.cycles;
        }
    }
done:
#undef TRY
    S.status = rc;
    (void)hipStreamSynchronize(st);
    S.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (stats) *stats = S;
    return rc;
}

}  // namespace fsi
