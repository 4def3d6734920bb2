// Internal declarations of the block-Jacobi launchers.
#pragma once

#include "kernels.hpp"

namespace fsi {

size_t bjacobi_workspace_bytes(const Geo &g);
int launch_bjacobi_setup(const Geo &g, const fsi_vms_params &prm, const double *a, const double *s,
                         const uint32_t *mask, const double *gram, const int32_t *occ_index,
                         double *raw, double *pinv64, float *pinv32, int64_t *n_singular,
                         void *ws, hipStream_t st);
int launch_bjacobi_apply(int64_t N, fsi_dtype dt, const void *pinv, const void *v, void *z,
                         hipStream_t st);
// z = P^{-1} v with the FP32 inverse, v rounded from FP64 on the fly
int launch_bjacobi_apply_f64_to_f32(int64_t N, const float *pinv32, const double *v, float *z,
                                    hipStream_t st);

}  // namespace fsi
