// Internal declarations of the Krylov vector kernels and the FGMRES driver.
#pragma once

#include "kernels.hpp"

namespace fsi {

constexpr int KRY_NB = 1024;   // blocks of the multi-dot (partials per vector)
constexpr int KRY_FUSED_MAXK = 52;   // basis size the fused CGS kernels support

int kry_cast_f64_f32(int64_t n, const double *in, float *out, hipStream_t st);
int kry_cast_f32_f64(int64_t n, const float *in, double *out, hipStream_t st);
int kry_axpby(int64_t n, double alpha, const double *x, double beta, double *y, hipStream_t st);
int kry_scale(int64_t n, double alpha, const double *x, double *y, hipStream_t st);
int kry_scale_inv(int64_t n, const double *x, const double *dev_scalar, double *out, hipStream_t st);
// the same scaling (FP64 arithmetic) into an FP32 vector, from FP64 or FP32 (out may be x)
int kry_scale_inv_to_f32(int64_t n, const double *x, const double *dev_scalar, float *out, hipStream_t st);
int kry_scale_inv_f32(int64_t n, const float *x, const double *dev_scalar, float *out, hipStream_t st);
int kry_multidot(int64_t n, int nk, const double *V, int64_t ldv, const double *w, double *partial,
                 double *out, hipStream_t st);
int kry_norm(int64_t n, const double *w, double *partial, double *out, hipStream_t st);
int kry_multi_axpy(int64_t n, int nk, const double *V, int64_t ldv, const double *h, double *w,
                   hipStream_t st);
// w -= V h (nk vectors); then out[k] = V[k] . w for k < nk_dot, or out[0] = ||w|| if nk_dot == 0
int kry_axpy_dot(int64_t n, int nk, const double *V, int64_t ldv, const double *h, double *w, int nk_dot,
                 double *partial, double *out, hipStream_t st);
// out[k] = V[k] . w, out[nk + k] = V[k] . u  (k < nk), one pass over V
int kry_multidot2(int64_t n, int nk, const double *V, int64_t ldv, const double *w, const double *u,
                  double *partial, double *out, hipStream_t st);
// Gram column update and twice-projected coefficients (see krylov.hip)
int kry_gram_coeffs(int nk, const double *ab, double *G, int ldg, double *h, hipStream_t st);
// CGS2 step kernels (16-byte loads, per-block partials reduced in a fixed order):
// ab = [V^T w; V^T u], Gram column j = nk - 1 from V^T u, h = a + (a - G a)  (nk <= 52)
int kry_cgs_project(int64_t n, int nk, const double *V, int64_t ldv, const double *w, const double *u,
                    double *partial, double *ab, double *G, int ldg, double *h, hipStream_t st);
// w -= V h and out[0] = ||w||
int kry_axpy_norm(int64_t n, int nk, const double *V, int64_t ldv, const double *h, double *w,
                  double *partial, double *out, hipStream_t st);
// the same two passes on a w given in FP32 (the inner-precision product, widened exactly as it
// is read): the projection reads it, the update writes w - V h to wout in FP64
int kry_cgs_project_f32w(int64_t n, int nk, const double *V, int64_t ldv, const float *w, const double *u,
                         double *partial, double *ab, double *G, int ldg, double *h, hipStream_t st);
int kry_axpy_norm_f32w(int64_t n, int nk, const double *V, int64_t ldv, const double *h, const float *w,
                       double *wout, double *partial, double *out, hipStream_t st);
// both passes with the basis stored in FP32 (V, u, w and the new vector wout in FP32; every
// product and sum in FP64)
int kry_cgs_project_b32(int64_t n, int nk, const float *V, int64_t ldv, const float *w, const float *u,
                        double *partial, double *ab, double *G, int ldg, double *h, hipStream_t st);
int kry_axpy_norm_b32(int64_t n, int nk, const float *V, int64_t ldv, const double *h, const float *w,
                      float *wout, double *partial, double *out, hipStream_t st);
int kry_update(int64_t n, int nk, fsi_dtype dz, const void *Z, int64_t ldz, const double *y, double *x,
               hipStream_t st);

}  // namespace fsi
