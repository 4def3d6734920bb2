// Internal helpers shared by the library's translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/fsi.h"

namespace fsi {

// ---- error reporting -------------------------------------------------------
void set_error(const char *fmt, ...);
void clear_error();

#define FSI_CHECK_ARG(cond, ...)                 \
    do {                                         \
        if (!(cond)) {                           \
            ::fsi::set_error(__VA_ARGS__);       \
            return FSI_ERR_ARG;                  \
        }                                        \
    } while (0)

#define FSI_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                    \
            ::fsi::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                             __FILE__, __LINE__);                                  \
            return FSI_ERR_HIP;                                                    \
        }                                                                          \
    } while (0)

#define FSI_LAUNCH_CHECK()                                                                \
    do {                                                                                  \
        hipError_t e_ = hipGetLastError();                                                \
        if (e_ != hipSuccess) {                                                           \
            ::fsi::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_),   \
                             __FILE__, __LINE__);                                         \
            return FSI_ERR_HIP;                                                           \
        }                                                                                 \
    } while (0)

// ---- grid geometry in a form kernels take by value -------------------------
struct Geo {
    int32_t n[3];      // cells per axis
    int32_t nn[3];     // nodes per axis
    int32_t p;         // order
    int64_t N;         // nodes
    int64_t E;         // cells
    double x0[3], h[3];
};

inline Geo make_geo(const fsi_grid &g)
{
    Geo o;
    o.p = g.order;
    o.N = 1;
    o.E = 1;
    for (int d = 0; d < 3; ++d) {
        o.n[d] = g.n[d];
        o.nn[d] = g.order * g.n[d] + 1;
        o.x0[d] = g.x0[d];
        o.h[d] = g.h[d];
        o.N *= o.nn[d];
        o.E *= o.n[d];
    }
    return o;
}

// validates a grid; returns FSI_OK or FSI_ERR_ARG with a message
int check_grid(const fsi_grid *g);

inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Dirichlet bitmask test for flat velocity DOF index k (= f*N + node)
__device__ __forceinline__ bool mask_bit(const uint32_t *mask, int64_t k)
{
    return mask != nullptr && ((mask[k >> 5] >> (k & 31)) & 1u);
}

}  // namespace fsi
