// Internal declarations of the Newton driver.
#pragma once

#include "kernels.hpp"

namespace fsi {

size_t newton_workspace_bytes(const Geo &g, const fsi_newton_opts &o, size_t jws);
int newton_solve(const Geo &g, const fsi_problem &P64, const fsi_problem *P32, const double *f,
                 const double *lamg, const double *gD, double *x, const fsi_newton_opts &o,
                 fsi_newton_stats *stats, void *ws, size_t jws, hipStream_t st);

}  // namespace fsi
