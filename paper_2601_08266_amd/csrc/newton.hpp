// Internal declarations of the Newton driver.
#pragma once

#include "kernels.hpp"

namespace fsi {

size_t newton_workspace_bytes(const Geo &g, const fsi_newton_opts &o, size_t jws);

// One time step with the hyperelastic solid (the problem's points are its nodes): V = B u,
// U = Ub + cU V, A = cA V - Ab; the step residual gains B^T R^s(U, V, A) and the Newton matrix
// B^T (c_M M + c_K K - c_V K_v) B with (cA, cU, 1); U and V receive the solid state of the last
// residual's iterate.
struct SolidStep {
    const fsi_solid *S;
    const double *Ub, *Ab;
    double cU, cA;
    double *U, *V;
};
// R = the step residual with the solid (FP64, Q1); ws: the Jacobian workspace of P64 with S
int solid_step_residual(const Geo &g, const fsi_problem &P64, const SolidStep &ss, const double *f,
                        const double *gD, const double *x, double *R, void *ws, hipStream_t st);
int newton_solve(const Geo &g, const fsi_problem &P64, const fsi_problem *P32, const double *f,
                 const double *lamg, const double *gD, double *x, const fsi_newton_opts &o,
                 fsi_newton_stats *stats, void *ws, size_t jws, hipStream_t st,
                 const SolidStep *ss = nullptr);

}  // namespace fsi
