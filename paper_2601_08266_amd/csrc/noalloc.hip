// fsi_dlm_BT_noalloc: y += B^T (kappa o lam) with the library's own scratch memory, for callers
// that cannot allocate device memory (code under HIP graph capture, serving loops that forbid
// hipMalloc).  The per-occupied-cell corner sums that fsi_dlm_BT keeps in the caller's workspace
// live here in one file-scope device array; the kernels are fsi_dlm_BT's.
#include <mutex>

#include "dlm.hpp"
#include "kernels.hpp"

namespace fsi {

namespace {

// FSI_NOALLOC_SCRATCH_BYTES of corner sums: n_occ (p+1)^3 3 values, so up to 174,762 occupied
// Q1 cells in FP64 (349,525 in FP32), 48,545 occupied Q2 cells in FP64.
constexpr size_t FSI_NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[FSI_NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` on each GPU (each holds its own copy of the array), looked up once
// per device with that device current.  The array's host-side name is not a device address.
std::mutex g_mu;
void *g_ptr[MAX_DEVICES];

int scratch_ptr(void **out)
{
    int dev = -1;
    FSI_HIP(hipGetDevice(&dev));
    FSI_CHECK_ARG(dev >= 0 && dev < MAX_DEVICES, "device index %d beyond %d", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[dev] == nullptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
            return FSI_ERR_HIP;
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return FSI_OK;
}

}  // namespace

}  // namespace fsi

using namespace fsi;

extern "C" __attribute__((visibility("default"))) size_t fsi_dlm_BT_noalloc_max_bytes(void)
{
    return FSI_NOALLOC_SCRATCH_BYTES;
}

extern "C" __attribute__((visibility("default"))) int
fsi_dlm_BT_noalloc(const fsi_grid *grid, fsi_dtype dtype, int64_t m, const int32_t *perm, const void *xi,
                   const int32_t *occ_cell, const int32_t *occ_start, const int32_t *occ_index, int64_t n_occ,
                   const void *lam, const void *kappa, void *y, void *stream)
{
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    FSI_CHECK_ARG(dtype == FSI_F64 || dtype == FSI_F32, "bad dtype %d", (int)dtype);
    FSI_CHECK_ARG(m >= 0 && m < ((int64_t)1 << 31) - 1, "m out of range");
    const Geo g = make_geo(*grid);
    FSI_CHECK_ARG(n_occ >= 0 && n_occ <= g.E && n_occ <= m, "n_occ out of range");
    const size_t need = dlm_csum_bytes(g, n_occ, dtype);
    if (need > FSI_NOALLOC_SCRATCH_BYTES) {
        set_error("%lld occupied cells need %zu bytes of corner sums, more than the %zu bytes of the "
                  "library's scratch array (use fsi_dlm_BT with a workspace)",
                  (long long)n_occ, need, FSI_NOALLOC_SCRATCH_BYTES);
        return FSI_ERR_WORKSPACE;
    }
    FSI_CHECK_ARG(y != nullptr, "y must be non-NULL");
    if (n_occ == 0) return FSI_OK;
    FSI_CHECK_ARG(xi && perm && occ_cell && occ_start && occ_index && lam,
                  "point tables and lam must be non-NULL");
    void *ws = nullptr;
    rc = scratch_ptr(&ws);
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    // every corner sum of the n_occ cells is written before it is read: nothing to clear
    rc = launch_dlm_cell_reduce(g, dtype, false, m, n_occ, occ_cell, occ_start, perm, xi, kappa, lam,
                                nullptr, ws, st);
    if (rc) return rc;
    return launch_dlm_node_gather(g, dtype, n_occ, occ_cell, ws, occ_index, y, st);
}
