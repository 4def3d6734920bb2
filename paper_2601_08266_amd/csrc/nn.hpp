// Internal declarations of the warm-start network kernels.
#pragma once

#include <vector>

#include "kernels.hpp"

namespace fsi {

constexpr int NN_WG_RANGE = 4096;   // voxels per weight-gradient range (multiple of 64)
constexpr int NN_BG_RANGE = 512;    // voxels per bias-gradient range

typedef fsi_nn_pack_spec NnPack;
typedef fsi_nn_unpack_spec NnUnpack;

int nn_conv_fwd(const int32_t *dims, int cin, int cout, const uint16_t *X, const uint16_t *W,
                const float *bias, int relu, const uint16_t *gate, uint16_t *Ybf, float *Yf,
                hipStream_t st);
size_t nn_wgrad_workspace(const int32_t *dims, int cin, int cout);
int nn_conv_wgrad(const int32_t *dims, int cin, int cout, const uint16_t *dY, const uint16_t *X, float *dW,
                  float *db, void *ws, hipStream_t st);
int nn_flip_transpose(int cin, int cout, const uint16_t *W, uint16_t *Wd, hipStream_t st);
size_t nn_mse_workspace();
int nn_mse(int64_t V, int c, int used, const float *pred, const float *target, uint16_t *dpred,
           double *loss_host, void *ws, hipStream_t st);
int nn_adam(int64_t n, float *w, const float *g, float *m, float *v, uint16_t *wbf, int t, float lr, float b1,
            float b2, float eps, hipStream_t st);
int nn_to_bf16(int64_t n, const float *in, uint16_t *out, hipStream_t st);
int nn_pack(int64_t V, int c, const NnPack &p, float *out, hipStream_t st);
size_t nn_moments_workspace(int c);
int nn_moments(int64_t V, int c, const float *data, double *sums_host, void *ws, hipStream_t st);
int nn_unpack(int64_t V, int c, const float *out, const double *base, const NnUnpack &u,
              const uint32_t *mask, const double *gD, double *x, hipStream_t st);

}  // namespace fsi
