// Vector kernels of the Krylov solver: casts, axpby, deterministic multi-dot
// (fixed-order block partials + fixed-order final sum), multi-axpy (CGS2
// projections, solution update from the preconditioned basis).
#include "krylov.hpp"

namespace fsi {

namespace {

constexpr int KT = 256;      // threads per block
constexpr int KG = 8;        // vectors per group in the multi-dot

template <typename TI, typename TO>
__global__ __launch_bounds__(KT) void cast_k(int64_t n, const TI *__restrict__ in, TO *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT)
        out[i] = (TO)in[i];
}

// y = alpha x + beta y
__global__ __launch_bounds__(KT) void axpby_k(int64_t n, double alpha, const double *__restrict__ x,
                                              double beta, double *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT)
        y[i] = alpha * x[i] + beta * y[i];
}

// y = alpha x
__global__ __launch_bounds__(KT) void scale_k(int64_t n, double alpha, const double *__restrict__ x,
                                              double *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT)
        y[i] = alpha * x[i];
}

// out = x * s, s = 1 / dev[0] computed on the device side in FP64 (out may be x)
template <typename TI, typename TO>
__global__ __launch_bounds__(KT) void scale_inv_k(int64_t n, const TI *x, const double *__restrict__ dev,
                                                  TO *out)
{
    const double s = 1.0 / dev[0];
    for (int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT)
        out[i] = (TO)((double)x[i] * s);
}

// partial[k][block] = sum over this block's contiguous chunk of V[k][i] * w[i], k < nk
__global__ __launch_bounds__(KT) void multidot_k(int64_t n, int nk, const double *__restrict__ V,
                                                 int64_t ldv, const double *__restrict__ w,
                                                 double *__restrict__ partial)
{
    __shared__ double red[KG][KT];
    const int t = threadIdx.x;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    for (int g0 = 0; g0 < nk; g0 += KG) {
        double acc[KG];
#pragma unroll
        for (int k = 0; k < KG; ++k) acc[k] = 0.0;
        for (int64_t i = lo + t; i < hi; i += KT) {
            const double wi = w[i];
#pragma unroll
            for (int k = 0; k < KG; ++k)
                if (g0 + k < nk) acc[k] += V[(int64_t)(g0 + k) * ldv + i] * wi;
        }
#pragma unroll
        for (int k = 0; k < KG; ++k) red[k][t] = acc[k];
        __syncthreads();
        for (int off = KT / 2; off > 0; off >>= 1) {
            if (t < off)
#pragma unroll
                for (int k = 0; k < KG; ++k) red[k][t] += red[k][t + off];
            __syncthreads();
        }
        if (t < KG && g0 + t < nk) partial[(int64_t)(g0 + t) * gridDim.x + blockIdx.x] = red[t][0];
        __syncthreads();
    }
}

// out[k] = sum_b partial[k][b] (sqrt of it if take_sqrt): one block per k; each thread sums a
// fixed set of partials (loads issued in groups of 4), then a fixed LDS tree
__global__ __launch_bounds__(KT) void reduce_partials_k(int nk, int nb, const double *__restrict__ partial,
                                                        double *__restrict__ out, int take_sqrt = 0)
{
    __shared__ double red[KT];
    const int k = blockIdx.x, t = threadIdx.x;
    const double *p = partial + (int64_t)k * nb;
    double s = 0.0;
    for (int b0 = 0; b0 < nb; b0 += 4 * KT) {
        double v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int b = b0 + q * KT + t;
            v[q] = b < nb ? p[b] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) s += v[q];
    }
    red[t] = s;
    __syncthreads();
    for (int off = KT / 2; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    if (t == 0) out[k] = take_sqrt ? sqrt(red[0]) : red[0];
}

// sqrt of a device scalar, in place
__global__ void sqrt_k(double *v) { v[0] = sqrt(v[0]); }

// w[i] -= sum_k h[k] V[k][i]
__global__ __launch_bounds__(KT) void multi_axpy_k(int64_t n, int nk, const double *__restrict__ V,
                                                   int64_t ldv, const double *__restrict__ h,
                                                   double *__restrict__ w)
{
    for (int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT) {
        double s = w[i];
        for (int k = 0; k < nk; ++k) s -= h[k] * V[(int64_t)k * ldv + i];
        w[i] = s;
    }
}

// fused CGS2 pass: w[i] -= sum_k h[k] V[k][i], then partial[k][block] of V[k] . w (new w);
// with nk_dot = 0 it only accumulates partial[0][block] = w . w (the norm pass)
__global__ __launch_bounds__(KT) void axpy_dot_k(int64_t n, int nk, const double *__restrict__ V, int64_t ldv,
                                                 const double *__restrict__ h, double *__restrict__ w,
                                                 int nk_dot, double *__restrict__ partial)
{
    __shared__ double red[KG][KT];
    const int t = threadIdx.x;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    // update the chunk of w
    for (int64_t i = lo + t; i < hi; i += KT) {
        double s = w[i];
        for (int k = 0; k < nk; ++k) s -= h[k] * V[(int64_t)k * ldv + i];
        w[i] = s;
    }
    // each thread re-reads only the elements it wrote, so no barrier is needed before the dots
    const int ngroups = nk_dot > 0 ? nk_dot : 1;
    for (int g0 = 0; g0 < ngroups; g0 += KG) {
        double acc[KG];
#pragma unroll
        for (int k = 0; k < KG; ++k) acc[k] = 0.0;
        for (int64_t i = lo + t; i < hi; i += KT) {
            const double wi = w[i];
            if (nk_dot == 0) {
                acc[0] += wi * wi;
            } else {
#pragma unroll
                for (int k = 0; k < KG; ++k)
                    if (g0 + k < nk_dot) acc[k] += V[(int64_t)(g0 + k) * ldv + i] * wi;
            }
        }
#pragma unroll
        for (int k = 0; k < KG; ++k) red[k][t] = acc[k];
        __syncthreads();
        for (int off = KT / 2; off > 0; off >>= 1) {
            if (t < off)
#pragma unroll
                for (int k = 0; k < KG; ++k) red[k][t] += red[k][t + off];
            __syncthreads();
        }
        if (t < KG && g0 + t < ngroups) partial[(int64_t)(g0 + t) * gridDim.x + blockIdx.x] = red[t][0];
        __syncthreads();
    }
}

// partial[k][block] = V[k] . w and partial[nk + k][block] = V[k] . u for k < nk (one read of V)
__global__ __launch_bounds__(KT) void multidot2_k(int64_t n, int nk, const double *__restrict__ V,
                                                  int64_t ldv, const double *__restrict__ w,
                                                  const double *__restrict__ u,
                                                  double *__restrict__ partial)
{
    __shared__ double red[2 * KG][KT];
    const int t = threadIdx.x;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    for (int g0 = 0; g0 < nk; g0 += KG) {
        double aw[KG], au[KG];
#pragma unroll
        for (int k = 0; k < KG; ++k) aw[k] = au[k] = 0.0;
        for (int64_t i = lo + t; i < hi; i += KT) {
            const double wi = w[i], ui = u[i];
#pragma unroll
            for (int k = 0; k < KG; ++k)
                if (g0 + k < nk) {
                    const double v = V[(int64_t)(g0 + k) * ldv + i];
                    aw[k] += v * wi;
                    au[k] += v * ui;
                }
        }
#pragma unroll
        for (int k = 0; k < KG; ++k) {
            red[k][t] = aw[k];
            red[KG + k][t] = au[k];
        }
        __syncthreads();
        for (int off = KT / 2; off > 0; off >>= 1) {
            if (t < off)
#pragma unroll
                for (int k = 0; k < 2 * KG; ++k) red[k][t] += red[k][t + off];
            __syncthreads();
        }
        if (t < KG && g0 + t < nk) {
            partial[(int64_t)(g0 + t) * gridDim.x + blockIdx.x] = red[t][0];
            partial[(int64_t)(nk + g0 + t) * gridDim.x + blockIdx.x] = red[KG + t][0];
        }
        __syncthreads();
    }
}

// Gram correction of classical Gram-Schmidt: with a = V^T w and b = V^T V_j (the new Gram
// column), store G[:, j] = G[j, :] = b and the twice-projected coefficients
// h = a + (a - G a) in h (one block, nk = j + 1 <= ldg).
__global__ __launch_bounds__(64) void gram_coeffs_k(int nk, const double *__restrict__ ab,
                                                    double *__restrict__ G, int ldg,
                                                    double *__restrict__ h)
{
    const int t = threadIdx.x;
    const int j = nk - 1;
    for (int k = t; k < nk; k += 64) {
        G[(int64_t)k * ldg + j] = ab[nk + k];
        G[(int64_t)j * ldg + k] = ab[nk + k];
    }
    __syncthreads();
    for (int k = t; k < nk; k += 64) {
        double ga = 0.0;
        for (int m = 0; m < nk; ++m) ga += G[(int64_t)k * ldg + m] * ab[m];
        h[k] = ab[k] + (ab[k] - ga);
    }
}

// x[i] += sum_k y[k] Z[k][i]   (Z in the inner precision)
template <typename TZ>
__global__ __launch_bounds__(KT) void update_k(int64_t n, int nk, const TZ *__restrict__ Z, int64_t ldz,
                                               const double *__restrict__ y, double *__restrict__ x)
{
    for (int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT) {
        double s = 0.0;
        for (int k = 0; k < nk; ++k) s += y[k] * (double)Z[(int64_t)k * ldz + i];
        x[i] += s;
    }
}

// ---- fused CGS2 step kernels: per-block partials, and the last block to finish reduces them
// in a fixed order (deterministic), so one launch replaces kernel + reduction + coefficients.

constexpr int CG_WAVES = KT / 64;           // waves per block
constexpr int CG_MAXK = 13;                 // vectors per wave: nk <= CG_WAVES * CG_MAXK
static_assert(CG_WAVES * CG_MAXK == KRY_FUSED_MAXK, "fused CGS size");

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// two consecutive entries as FP64 (FP64 vectors, or FP32 ones widened exactly: the inner
// precision's product, or a basis stored in FP32)
__device__ __forceinline__ double2 load2(const double *p) { return *reinterpret_cast<const double2 *>(p); }
__device__ __forceinline__ double2 load2(const float *p)
{
    const float2 v = *reinterpret_cast<const float2 *>(p);
    return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ void store2(double *p, double2 v) { *reinterpret_cast<double2 *>(p) = v; }
__device__ __forceinline__ void store2(float *p, double2 v)
{
    *reinterpret_cast<float2 *>(p) = make_float2((float)v.x, (float)v.y);
}

// E consecutive entries per lane as FP64: pairs (16-byte loads of FP64 data, 8-byte loads of
// FP32 data alongside an FP64 basis) or quadruples of FP32 data (16-byte loads, an FP32 basis)
template <int E>
struct DV {
    double v[E];
};
template <int E, typename T>
__device__ __forceinline__ DV<E> loadv(const T *p)
{
    DV<E> o;
    if constexpr (E == 2) {
        const double2 t = load2(p);
        o.v[0] = t.x;
        o.v[1] = t.y;
    } else {
        static_assert(E == 4 && sizeof(T) == 4, "quadruples are FP32 data");
        const float4 t = *reinterpret_cast<const float4 *>(p);
        o.v[0] = t.x;
        o.v[1] = t.y;
        o.v[2] = t.z;
        o.v[3] = t.w;
    }
    return o;
}
template <int E, typename T>
__device__ __forceinline__ void storev(T *p, const DV<E> &s)
{
    if constexpr (E == 2) {
        store2(p, make_double2(s.v[0], s.v[1]));
    } else {
        static_assert(E == 4 && sizeof(T) == 4, "quadruples are FP32 data");
        *reinterpret_cast<float4 *>(p) = make_float4((float)s.v[0], (float)s.v[1], (float)s.v[2], (float)s.v[3]);
    }
}

// Projection pass of classical Gram-Schmidt with re-orthogonalisation through the Gram matrix:
// per-block partials of V[k] . w and V[k] . u (u = V[nk-1], the newest basis vector), k < nk, in
// one read of V: wave wv of a block takes the vectors k = wv + 4q, q < KQ = ceil(nk / 4), and
// issues their loads together (past nk it loads nothing and accumulates nothing).  The
// basis (TV) and w (TW) are FP64 or FP32; products and sums are FP64.  Each lane moves E
// entries per vector and step (16-byte loads of the basis; E = 4 for an FP32 basis).
template <int KQ, typename TW, typename TV>
__global__ __launch_bounds__(KT) void cgs_project_k(int64_t n, int nk, const TV *__restrict__ V,
                                                    int64_t ldv, const TW *__restrict__ w,
                                                    const TV *__restrict__ u,
                                                    double *__restrict__ partial)
{
    constexpr int E = sizeof(TV) == 4 ? 4 : 2;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // chunks of a multiple of E elements (n, ldv and the vector bases are multiples of E /
    // 16-byte aligned, checked by the host wrappers)
    const int64_t chunk = ((n + gridDim.x - 1) / gridDim.x + E - 1) & ~(int64_t)(E - 1);
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    const TV *vk[KQ];
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
        const int k = wv + CG_WAVES * q;
        vk[q] = V + (int64_t)(k < nk ? k : nk - 1) * ldv;
    }
    double aw[KQ], au[KQ];
#pragma unroll
    for (int q = 0; q < KQ; ++q) aw[q] = au[q] = 0.0;
    for (int64_t i = lo + E * lane; i < hi; i += 64 * E) {
        const DV<E> wi = loadv<E>(w + i);
        const DV<E> ui = loadv<E>(u + i);
        DV<E> v[KQ];
#pragma unroll
        for (int q = 0; q < KQ; ++q)   // past nk (uniform over the wave) nothing is loaded
            v[q] = wv + CG_WAVES * q < nk ? loadv<E>(vk[q] + i) : DV<E>{};
        __builtin_amdgcn_sched_barrier(0);   // keep the loads in flight together
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                aw[q] += v[q].v[e] * wi.v[e];
                au[q] += v[q].v[e] * ui.v[e];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
        const int k = wv + CG_WAVES * q;
        const double sw = wave_sum(aw[q]), su = wave_sum(au[q]);
        if (k < nk && lane == 0) {
            partial[(int64_t)k * gridDim.x + blockIdx.x] = sw;
            partial[(int64_t)(nk + k) * gridDim.x + blockIdx.x] = su;
        }
    }
}

// out = w - V h (nk vectors, in groups of 8 whose loads are issued together) and per-block
// partials of ||out||^2 (of the FP64 sums, before out is rounded to TO); out may be w itself
// (TW = TO).  E entries per lane and step as in the projection.
template <typename TW, typename TV, typename TO>
__global__ __launch_bounds__(KT) void axpy_norm_k(int64_t n, int nk, const TV *__restrict__ V,
                                                  int64_t ldv, const double *__restrict__ h,
                                                  const TW *w, TO *out, double *__restrict__ partial)
{
    constexpr int KB = 8;
    constexpr int E = sizeof(TV) == 4 ? 4 : 2;
    __shared__ double red[CG_WAVES];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t chunk = ((n + gridDim.x - 1) / gridDim.x + E - 1) & ~(int64_t)(E - 1);
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    double acc = 0.0;
    for (int64_t i = lo + E * threadIdx.x; i < hi; i += E * KT) {
        DV<E> s = loadv<E>(w + i);
        for (int k0 = 0; k0 < nk; k0 += KB) {
            DV<E> v[KB];
            double hk[KB];
#pragma unroll
            for (int q = 0; q < KB; ++q) {
                // past nk (a condition uniform over the block) nothing is loaded and the term is 0
                const int k = k0 + q;
                v[q] = k < nk ? loadv<E>(V + (int64_t)k * ldv + i) : DV<E>{};
                hk[q] = k < nk ? h[k] : 0.0;
            }
            __builtin_amdgcn_sched_barrier(0);   // keep the loads in flight together
#pragma unroll
            for (int q = 0; q < KB; ++q) {
#pragma unroll
                for (int e = 0; e < E; ++e) s.v[e] -= hk[q] * v[q].v[e];
            }
        }
        storev<E>(out + i, s);
#pragma unroll
        for (int e = 0; e < E; ++e) acc += s.v[e] * s.v[e];
    }
    acc = wave_sum(acc);
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int q = 0; q < CG_WAVES; ++q) sum += red[q];
        partial[blockIdx.x] = sum;
    }
}

inline unsigned grid_for(int64_t n)
{
    int64_t b = (n + KT - 1) / KT;
    return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

int kry_cast_f64_f32(int64_t n, const double *in, float *out, hipStream_t st)
{
    hipLaunchKernelGGL((cast_k<double, float>), dim3(grid_for(n)), dim3(KT), 0, st, n, in, out);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int kry_cast_f32_f64(int64_t n, const float *in, double *out, hipStream_t st)
{
    hipLaunchKernelGGL((cast_k<float, double>), dim3(grid_for(n)), dim3(KT), 0, st, n, in, out);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int kry_axpby(int64_t n, double alpha, const double *x, double beta, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(axpby_k, dim3(grid_for(n)), dim3(KT), 0, st, n, alpha, x, beta, y);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int kry_scale(int64_t n, double alpha, const double *x, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(scale_k, dim3(grid_for(n)), dim3(KT), 0, st, n, alpha, x, y);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int kry_scale_inv(int64_t n, const double *x, const double *dev_scalar, double *out, hipStream_t st)
{
    hipLaunchKernelGGL((scale_inv_k<double, double>), dim3(grid_for(n)), dim3(KT), 0, st, n, x, dev_scalar, out);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int kry_scale_inv_to_f32(int64_t n, const double *x, const double *dev_scalar, float *out, hipStream_t st)
{
    hipLaunchKernelGGL((scale_inv_k<double, float>), dim3(grid_for(n)), dim3(KT), 0, st, n, x, dev_scalar, out);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int kry_scale_inv_f32(int64_t n, const float *x, const double *dev_scalar, float *out, hipStream_t st)
{
    hipLaunchKernelGGL((scale_inv_k<float, float>), dim3(grid_for(n)), dim3(KT), 0, st, n, x, dev_scalar, out);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int kry_multidot(int64_t n, int nk, const double *V, int64_t ldv, const double *w, double *partial,
                 double *out, hipStream_t st)
{
    hipLaunchKernelGGL(multidot_k, dim3(KRY_NB), dim3(KT), 0, st, n, nk, V, ldv, w, partial);
    FSI_LAUNCH_CHECK();
    hipLaunchKernelGGL(reduce_partials_k, dim3(nk), dim3(KT), 0, st, nk, KRY_NB, partial, out);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int kry_norm(int64_t n, const double *w, double *partial, double *out, hipStream_t st)
{
    int rc = kry_multidot(n, 1, w, n, w, partial, out, st);
    if (rc) return rc;
    hipLaunchKernelGGL(sqrt_k, dim3(1), dim3(1), 0, st, out);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int kry_multi_axpy(int64_t n, int nk, const double *V, int64_t ldv, const double *h, double *w,
                   hipStream_t st)
{
    hipLaunchKernelGGL(multi_axpy_k, dim3(grid_for(n)), dim3(KT), 0, st, n, nk, V, ldv, h, w);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int kry_axpy_dot(int64_t n, int nk, const double *V, int64_t ldv, const double *h, double *w, int nk_dot,
                 double *partial, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(axpy_dot_k, dim3(KRY_NB), dim3(KT), 0, st, n, nk, V, ldv, h, w, nk_dot, partial);
    FSI_LAUNCH_CHECK();
    const int nr = nk_dot > 0 ? nk_dot : 1;
    hipLaunchKernelGGL(reduce_partials_k, dim3(nr), dim3(KT), 0, st, nr, KRY_NB, partial, out);
    FSI_LAUNCH_CHECK();
    if (nk_dot == 0) {
        hipLaunchKernelGGL(sqrt_k, dim3(1), dim3(1), 0, st, out);
        FSI_LAUNCH_CHECK();
    }
    return FSI_OK;
}

int kry_multidot2(int64_t n, int nk, const double *V, int64_t ldv, const double *w, const double *u,
                  double *partial, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(multidot2_k, dim3(KRY_NB), dim3(KT), 0, st, n, nk, V, ldv, w, u, partial);
    FSI_LAUNCH_CHECK();
    hipLaunchKernelGGL(reduce_partials_k, dim3(2 * nk), dim3(KT), 0, st, 2 * nk, KRY_NB, partial, out);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

template <typename TW, typename TV>
static int cgs_project_t(int64_t n, int nk, const TV *V, int64_t ldv, const TW *w, const TV *u,
                         double *partial, double *ab, double *G, int ldg, double *h, hipStream_t st)
{
    constexpr int64_t E = sizeof(TV) == 4 ? 4 : 2;
    if ((n | ldv) & (E - 1) || ((uintptr_t)V | (uintptr_t)u) & 15 || (uintptr_t)w & (E * sizeof(TW) - 1)) {
        set_error("CGS projection needs lengths divisible by its entries per lane and aligned vectors");
        return FSI_ERR_ARG;
    }
    switch ((nk + CG_WAVES - 1) / CG_WAVES) {
#define FSI_CGS_CASE(KQ)                                                                           \
    case KQ:                                                                                       \
        hipLaunchKernelGGL((cgs_project_k<KQ, TW, TV>), dim3(KRY_NB), dim3(KT), 0, st, n, nk, V, ldv, w, \
                           u, partial);                                                            \
        break;
        FSI_CGS_CASE(1) FSI_CGS_CASE(2) FSI_CGS_CASE(3) FSI_CGS_CASE(4) FSI_CGS_CASE(5)
        FSI_CGS_CASE(6) FSI_CGS_CASE(7) FSI_CGS_CASE(8) FSI_CGS_CASE(9) FSI_CGS_CASE(10)
        FSI_CGS_CASE(11) FSI_CGS_CASE(12) FSI_CGS_CASE(13)
#undef FSI_CGS_CASE
    default:
        set_error("CGS projection supports at most %d basis vectors (got %d)", KRY_FUSED_MAXK, nk);
        return FSI_ERR_ARG;
    }
    FSI_LAUNCH_CHECK();
    hipLaunchKernelGGL(reduce_partials_k, dim3(2 * nk), dim3(KT), 0, st, 2 * nk, KRY_NB, partial, ab, 0);
    FSI_LAUNCH_CHECK();
    hipLaunchKernelGGL(gram_coeffs_k, dim3(1), dim3(64), 0, st, nk, ab, G, ldg, h);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int kry_cgs_project(int64_t n, int nk, const double *V, int64_t ldv, const double *w, const double *u,
                    double *partial, double *ab, double *G, int ldg, double *h, hipStream_t st)
{
    return cgs_project_t<double, double>(n, nk, V, ldv, w, u, partial, ab, G, ldg, h, st);
}

int kry_cgs_project_f32w(int64_t n, int nk, const double *V, int64_t ldv, const float *w, const double *u,
                         double *partial, double *ab, double *G, int ldg, double *h, hipStream_t st)
{
    return cgs_project_t<float, double>(n, nk, V, ldv, w, u, partial, ab, G, ldg, h, st);
}

int kry_cgs_project_b32(int64_t n, int nk, const float *V, int64_t ldv, const float *w, const float *u,
                        double *partial, double *ab, double *G, int ldg, double *h, hipStream_t st)
{
    return cgs_project_t<float, float>(n, nk, V, ldv, w, u, partial, ab, G, ldg, h, st);
}

template <typename TW, typename TV, typename TO>
static int axpy_norm_t(int64_t n, int nk, const TV *V, int64_t ldv, const double *h, const TW *w,
                       TO *wout, double *partial, double *out, hipStream_t st)
{
    constexpr int64_t E = sizeof(TV) == 4 ? 4 : 2;
    if ((n | ldv) & (E - 1) || (uintptr_t)V & 15 || (uintptr_t)wout & (E * sizeof(TO) - 1) ||
        (uintptr_t)w & (E * sizeof(TW) - 1)) {
        set_error("CGS update needs lengths divisible by its entries per lane and aligned vectors");
        return FSI_ERR_ARG;
    }
    hipLaunchKernelGGL((axpy_norm_k<TW, TV, TO>), dim3(KRY_NB), dim3(KT), 0, st, n, nk, V, ldv, h, w, wout,
                       partial);
    FSI_LAUNCH_CHECK();
    hipLaunchKernelGGL(reduce_partials_k, dim3(1), dim3(KT), 0, st, 1, KRY_NB, partial, out, 1);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int kry_axpy_norm(int64_t n, int nk, const double *V, int64_t ldv, const double *h, double *w,
                  double *partial, double *out, hipStream_t st)
{
    return axpy_norm_t<double, double, double>(n, nk, V, ldv, h, w, w, partial, out, st);
}

int kry_axpy_norm_f32w(int64_t n, int nk, const double *V, int64_t ldv, const double *h, const float *w,
                       double *wout, double *partial, double *out, hipStream_t st)
{
    return axpy_norm_t<float, double, double>(n, nk, V, ldv, h, w, wout, partial, out, st);
}

int kry_axpy_norm_b32(int64_t n, int nk, const float *V, int64_t ldv, const double *h, const float *w,
                      float *wout, double *partial, double *out, hipStream_t st)
{
    return axpy_norm_t<float, float, float>(n, nk, V, ldv, h, w, wout, partial, out, st);
}

int kry_gram_coeffs(int nk, const double *ab, double *G, int ldg, double *h, hipStream_t st)
{
    hipLaunchKernelGGL(gram_coeffs_k, dim3(1), dim3(64), 0, st, nk, ab, G, ldg, h);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int kry_update(int64_t n, int nk, fsi_dtype dz, const void *Z, int64_t ldz, const double *y, double *x,
               hipStream_t st)
{
    if (dz == FSI_F64)
        hipLaunchKernelGGL(update_k<double>, dim3(grid_for(n)), dim3(KT), 0, st, n, nk,
                           (const double *)Z, ldz, y, x);
    else
        hipLaunchKernelGGL(update_k<float>, dim3(grid_for(n)), dim3(KT), 0, st, n, nk,
                           (const float *)Z, ldz, y, x);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

}  // namespace fsi
