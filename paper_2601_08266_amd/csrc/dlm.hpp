// Internal declarations of the DLM launchers.
#pragma once

#include "kernels.hpp"

namespace fsi {

size_t locate_workspace_bytes(const Geo &g, int64_t m);
int launch_locate(const Geo &g, int64_t m, const double *X, fsi_dtype dt, int32_t *cell, void *xi,
                  int32_t *perm, int32_t *occ_cell, int32_t *occ_start, int32_t *occ_index,
                  void *s_out, double s_max, int64_t *n_occ_host, int64_t *n_outside_host, void *ws,
                  hipStream_t st);
// Bu = B u; Dirichlet velocity entries of u (mask bits, or NULL) read as zero
int launch_dlm_B(const Geo &g, fsi_dtype dt, int64_t m, const int32_t *cell, const void *xi,
                 const void *u, const uint32_t *mask, void *Bu, hipStream_t st);
// B u with xi and Bu in located order (cell-sorted positions; outside points last, Bu = 0)
int launch_dlm_B_located(const Geo &g, fsi_dtype dt, int64_t m, int64_t n_occ, const int32_t *occ_cell,
                         const int32_t *occ_start, const void *xi, const void *u, void *Bu, hipStream_t st);
// nf fields of M points between point order and located order (back: located -> point)
int launch_dlm_permute(fsi_dtype dt, int64_t m, int nf, const int32_t *perm, bool back, const void *src, void *dst,
                       hipStream_t st);
// perm NULL: xi, kappa and src in located order
int launch_dlm_cell_reduce(const Geo &g, fsi_dtype dt, bool from_u, int64_t m, int64_t n_occ,
                           const int32_t *occ_cell, const int32_t *occ_start, const int32_t *perm,
                           const void *xi, const void *kappa, const void *src, const uint32_t *mask,
                           void *csum, hipStream_t st);
int launch_dlm_gram(const Geo &g, fsi_dtype dt, int64_t m, int64_t n_occ, const int32_t *occ_start,
                    const int32_t *perm, const void *xi, const void *kappa, void *gram, hipStream_t st);
int launch_dlm_node_gather(const Geo &g, fsi_dtype dt, int64_t n_occ, const int32_t *occ_cell, const void *csum,
                           const int32_t *occ_index, void *y, hipStream_t st);

}  // namespace fsi
