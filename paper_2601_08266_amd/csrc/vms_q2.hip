// Q2-Q2 Oseen-VMS operator (placeholder until the kernel lands).
#include "kernels.hpp"

namespace fsi {

template <typename T>
int launch_q2_cells(const Geo &, const VmsConst<T> &, const T *, const T *, const T *,
                    const uint32_t *, const T *, const int32_t *, T *, const BrickLayout &,
                    hipStream_t)
{
    set_error("Q2 operator not built yet");
    return FSI_ERR_UNSUPPORTED;
}

template int launch_q2_cells<double>(const Geo &, const VmsConst<double> &, const double *,
                                     const double *, const double *, const uint32_t *,
                                     const double *, const int32_t *, double *,
                                     const BrickLayout &, hipStream_t);
template int launch_q2_cells<float>(const Geo &, const VmsConst<float> &, const float *,
                                    const float *, const float *, const uint32_t *, const float *,
                                    const int32_t *, float *, const BrickLayout &, hipStream_t);

}  // namespace fsi
