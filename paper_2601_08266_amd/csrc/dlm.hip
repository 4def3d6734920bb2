// DLM coupling on gfx950 (section 2.3, eqs. nodal_solid_velo and
// fsi_constraint_matrix; appendix A's per-point steps).
//
//  locate   one lane per point: floor guess + exact breakpoint correction,
//           parametric position xi in FP64, sort key = cell (E for outside).
//  sort     stable LSD radix sort of (key, point) with 8-bit digits; within a
//           wave the stable rank of equal digits comes from 8 ballots (match
//           mask) and a popcount, across waves and tiles from LDS prefix sums
//           and a global digit-major exclusive scan.
//  CSR      occupied cells from the sorted keys (flag + scan), the inverse map
//           cell -> occupied index, and the interface band of s.
//  B        one lane per point: (p+1)^3 shape values, gather of the cell nodes.
//  B^T      8 lanes (Q1) or a wavefront (Q2) per occupied cell reduce its points' N_A kappa lambda
//           (or N_A kappa (B u) when fused into the Jacobian) into per-cell
//           corner sums with a fixed butterfly order; a gather over the
//           occupied cells' corners (the corner of a node's first occupied
//           cell owns the node) adds the corner sums of the occupied cells
//           around each node in a fixed order.  No floating-point atomics
//           anywhere, so results are bitwise reproducible.
#include <algorithm>
#include <utility>

#include "dlm.hpp"
#include "profile.hpp"

namespace fsi {

namespace {

constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 8;
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ __forceinline__ double bp(double x0, int64_t k, double h)
{
    // breakpoint x0 + k h rounded as written: the product is rounded before the sum
    // (the _rn helpers alone do not stop the compiler from forming an fma)
#pragma clang fp contract(off)
    const double kh = (double)k * h;
    return x0 + kh;
}

template <typename T>
__global__ __launch_bounds__(256) void locate_kernel(Geo g, int64_t m, const double *__restrict__ X,
                                                     int32_t *__restrict__ cell, T *__restrict__ xi,
                                                     int32_t *__restrict__ keys,
                                                     int32_t *__restrict__ vals,
                                                     int32_t *__restrict__ n_outside)
{
#pragma clang fp contract(off)
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= m) return;
    int idx[3];
    bool inside = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double Xd = X[d * m + b];
        const int n = g.n[d];
        const double x0 = g.x0[d], h = g.h[d];
        if (!(Xd >= bp(x0, 0, h) && Xd <= bp(x0, n, h))) {   // also rejects NaN
            inside = false;
            idx[d] = 0;
            continue;
        }
        double guess = floor(__ddiv_rn(__dsub_rn(Xd, x0), h));
        int64_t k = guess < 0.0 ? 0 : (guess > (double)n ? (int64_t)n : (int64_t)guess);
        // largest k in [0,n] with b_k <= X (k moves monotonically; bounded by n steps)
        while (k > 0 && bp(x0, k, h) > Xd) --k;
        while (k < n && bp(x0, k + 1, h) <= Xd) ++k;
        idx[d] = (int)(k < n - 1 ? k : n - 1);
    }
    if (inside) {
        const int32_t c = idx[0] + g.n[0] * (idx[1] + g.n[1] * idx[2]);
        cell[b] = c;
        keys[b] = c;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double lo = bp(g.x0[d], idx[d], g.h[d]);
            xi[d * m + b] = (T)__ddiv_rn(__dsub_rn(X[d * m + b], lo), g.h[d]);
        }
    } else {
        cell[b] = -1;
        keys[b] = (int32_t)g.E;
#pragma unroll
        for (int d = 0; d < 3; ++d) xi[d * m + b] = T(0);
        atomicAdd(n_outside, 1);
    }
    vals[b] = (int32_t)b;
}

// ---- stable LSD radix sort ------------------------------------------------
__global__ __launch_bounds__(SORT_THREADS) void radix_hist(const int32_t *__restrict__ keys,
                                                           int64_t m, int shift, int nblocks,
                                                           int32_t *__restrict__ hist)
{
    __shared__ int32_t cnt[RADIX];
    const int t = threadIdx.x;
    cnt[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int64_t i = base + (int64_t)r * SORT_THREADS + t;
        if (i < m) atomicAdd(&cnt[(keys[i] >> shift) & (RADIX - 1)], 1);
    }
    __syncthreads();
    hist[(int64_t)t * nblocks + blockIdx.x] = cnt[t];   // digit-major
}

__global__ __launch_bounds__(SORT_THREADS) void radix_scatter(
    const int32_t *__restrict__ keys_in, const int32_t *__restrict__ vals_in, int64_t m, int shift,
    int nblocks, const int32_t *__restrict__ offs, int32_t *__restrict__ keys_out,
    int32_t *__restrict__ vals_out)
{
    constexpr int NW = SORT_THREADS / 64;
    __shared__ int32_t running[RADIX];
    __shared__ int32_t wcnt[NW][RADIX];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    running[t] = offs[(int64_t)t * nblocks + blockIdx.x];
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_ITEMS; ++r) {
        for (int j = 0; j < NW; ++j) wcnt[j][t] = 0;
        __syncthreads();
        const int64_t i = base + (int64_t)r * SORT_THREADS + t;
        const bool valid = i < m;
        int32_t key = 0, val = 0;
        int digit = 0;
        if (valid) {
            key = keys_in[i];
            val = vals_in[i];
            digit = (key >> shift) & (RADIX - 1);
        }
        // lanes of this wave holding the same digit (match mask from 8 ballots)
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < RADIX_BITS; ++bit) {
            const uint64_t bal = __ballot((digit >> bit) & 1);
            peers &= ((digit >> bit) & 1) ? bal : ~bal;
        }
        const int rank = __popcll(peers & lt);
        const int total = __popcll(peers);
        if (valid && rank == 0) wcnt[w][digit] = total;   // lowest lane of each digit group
        __syncthreads();
        if (valid) {
            int pos = running[digit] + rank;
            for (int j = 0; j < w; ++j) pos += wcnt[j][digit];
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        int add = 0;
        for (int j = 0; j < NW; ++j) add += wcnt[j][t];
        running[t] += add;
        __syncthreads();
    }
}

// ---- exclusive scan of int32 (reduce / scan of partials / downsweep) ------
__global__ __launch_bounds__(SCAN_THREADS) void scan_reduce(const int32_t *__restrict__ in, int64_t n,
                                                            int32_t *__restrict__ part)
{
    __shared__ int32_t sm[SCAN_THREADS];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int32_t s = 0;
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        const int64_t i = base + (int64_t)r * SCAN_THREADS + t;
        if (i < n) s += in[i];
    }
    sm[t] = s;
    __syncthreads();
    for (int off = SCAN_THREADS / 2; off > 0; off >>= 1) {
        if (t < off) sm[t] += sm[t + off];
        __syncthreads();
    }
    if (t == 0) part[blockIdx.x] = sm[0];
}

// single block: exclusive scan of the block partials in place, total at part[nparts]
__global__ __launch_bounds__(1024) void scan_partials(int32_t *__restrict__ part, int64_t nparts)
{
    __shared__ int32_t sm[1024];
    const int t = threadIdx.x;
    const int64_t per = (nparts + 1023) / 1024;
    const int64_t lo = t * per, hi = lo + per < nparts ? lo + per : nparts;
    int32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += part[i];
    sm[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int32_t v = t >= off ? sm[t - off] : 0;
        __syncthreads();
        sm[t] += v;
        __syncthreads();
    }
    int32_t run = t > 0 ? sm[t - 1] : 0;
    for (int64_t i = lo; i < hi; ++i) {
        const int32_t v = part[i];
        part[i] = run;
        run += v;
    }
    if (t == 1023) part[nparts] = sm[1023];
}

__global__ __launch_bounds__(SCAN_THREADS) void scan_down(const int32_t *__restrict__ in, int64_t n,
                                                          const int32_t *__restrict__ part,
                                                          int32_t *__restrict__ out)
{
    __shared__ int32_t sm[SCAN_THREADS];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)t * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int32_t s = 0;
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        const int64_t i = base + r;
        v[r] = i < n ? in[i] : 0;
        s += v[r];
    }
    sm[t] = s;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        int32_t u = t >= off ? sm[t - off] : 0;
        __syncthreads();
        sm[t] += u;
        __syncthreads();
    }
    int32_t run = part[blockIdx.x] + (t > 0 ? sm[t - 1] : 0);
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        const int64_t i = base + r;
        if (i < n) out[i] = run;
        run += v[r];
    }
}

// ---- occupied-cell CSR from the sorted keys --------------------------------
__global__ __launch_bounds__(256) void occ_flags(const int32_t *__restrict__ skeys, int64_t m, int64_t E,
                                                 int32_t *__restrict__ flags)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const int32_t k = skeys[j];
    flags[j] = (k < E && (j == 0 || skeys[j - 1] != k)) ? 1 : 0;
}

__global__ __launch_bounds__(256) void occ_emit(const int32_t *__restrict__ skeys, int64_t m, int64_t E,
                                                const int32_t *__restrict__ flags,
                                                const int32_t *__restrict__ pos,
                                                int32_t *__restrict__ occ_cell,
                                                int32_t *__restrict__ occ_start,
                                                int32_t *__restrict__ occ_index)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const int32_t k = skeys[j];
    if (flags[j]) {
        const int32_t o = pos[j];
        occ_cell[o] = k;
        occ_start[o] = (int32_t)j;
        occ_index[k] = o;
    }
}

__global__ __launch_bounds__(256) void fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void fill_t(T *__restrict__ p, int64_t n, T v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void mark_s(Geo g, const int32_t *__restrict__ occ_cell,
                                              const int32_t *__restrict__ n_occ_dev, T *__restrict__ s,
                                              T s_max)
{
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= *n_occ_dev) return;
    const int32_t c = occ_cell[o];
    const int cx = c % g.n[0], cy = (c / g.n[0]) % g.n[1], cz = c / (g.n[0] * g.n[1]);
    const int q = g.p + 1;
    for (int az = 0; az < q; ++az)
        for (int ay = 0; ay < q; ++ay)
            for (int ax = 0; ax < q; ++ax) {
                const int64_t node = (int64_t)(g.p * cx + ax) +
                                     (int64_t)g.nn[0] * ((g.p * cy + ay) + (int64_t)g.nn[1] * (g.p * cz + az));
                s[node] = s_max;   // same value from every writer
            }
}

template <typename T, int P>
__device__ __forceinline__ void lagrange(T t, T N[P + 1])
{
    if constexpr (P == 1) {
        N[0] = T(1) - t;
        N[1] = t;
    } else {
        N[0] = T(2) * (t - T(0.5)) * (t - T(1));
        N[1] = T(-4) * t * (t - T(1));
        N[2] = T(2) * t * (t - T(0.5));
    }
}

// MASKED: Dirichlet velocity entries of u (mask bits) read as zero; the unmasked variant keeps
// its loads unconditional, so they issue as one batch
template <typename T, int P, bool MASKED>
__global__ __launch_bounds__(256) void dlm_B_kernel(Geo g, int64_t m, const int32_t *__restrict__ cell,
                                                    const T *__restrict__ xi, const T *__restrict__ u,
                                                    const uint32_t *__restrict__ mask,
                                                    T *__restrict__ Bu)
{
    constexpr int Q = P + 1;
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= m) return;
    const int32_t c = cell[b];
    T acc[3] = {T(0), T(0), T(0)};
    if (c >= 0) {
        T Nx[Q], Ny[Q], Nz[Q];
        lagrange<T, P>(xi[b], Nx);
        lagrange<T, P>(xi[m + b], Ny);
        lagrange<T, P>(xi[2 * m + b], Nz);
        const int cx = c % g.n[0], cy = (c / g.n[0]) % g.n[1], cz = c / (g.n[0] * g.n[1]);
#pragma unroll
        for (int az = 0; az < Q; ++az)
#pragma unroll
            for (int ay = 0; ay < Q; ++ay)
#pragma unroll
                for (int ax = 0; ax < Q; ++ax) {
                    const int64_t node = (int64_t)(P * cx + ax) +
                                         (int64_t)g.nn[0] * ((P * cy + ay) + (int64_t)g.nn[1] * (P * cz + az));
                    const T w = Nx[ax] * Ny[ay] * Nz[az];
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        const T uf = u[f * g.N + node];
                        if constexpr (MASKED)
                            acc[f] += ((mask[(f * g.N + node) >> 5] >> ((f * g.N + node) & 31)) & 1u) ? T(0) : w * uf;
                        else
                            acc[f] += w * uf;
                    }
                }
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) Bu[f * m + b] = acc[f];
}

// Corner sums  csum[o][A][f] = sum_{B in cell} N_A(xi_B) kappa_B mu_B,f  with mu = lam (FROM_U =
// false) or mu = B u restricted to the cell, Dirichlet-masked (FROM_U = true).  LPC lanes per
// occupied cell (64 / LPC cells per wavefront): lane r takes the cell's points r, r + LPC, ...
// in sorted order, then an xor butterfly over the LPC lanes gives every lane the sums and lane
// r stores the entries e = r, r + LPC, ... (fixed order: deterministic).  The sums run in FP64
// for both precisions (a cell can hold hundreds of points; an FP32 product is rounded once
// per term and the total once when stored).
// B u for per-point arrays in located order (position j of the cell-sorted point list, the
// points of occupied cell k at occ_start[k] .. occ_start[k+1]): LPC lanes per occupied cell
// load its nodes once, then take its points in turn, so xi and Bu are read and written
// contiguously.  Per point the same products in the same order as dlm_B_kernel (bitwise equal).
template <typename T, int P, int LPC>
__global__ __launch_bounds__(256) void dlm_B_located(Geo g, int64_t m, int64_t n_occ,
                                                     const int32_t *__restrict__ occ_cell,
                                                     const int32_t *__restrict__ occ_start,
                                                     const T *__restrict__ xi, const T *__restrict__ u,
                                                     T *__restrict__ Bu)
{
    constexpr int Q = P + 1, NEN = Q * Q * Q;
    const int64_t o = ((int64_t)blockIdx.x * 256 + threadIdx.x) / LPC;
    const int lane = threadIdx.x % LPC;
    if (o >= n_occ) return;
    const int32_t c = occ_cell[o];
    const int cx = c % g.n[0], cy = (c / g.n[0]) % g.n[1], cz = c / (g.n[0] * g.n[1]);
    T un[3][NEN];
#pragma unroll
    for (int A = 0; A < NEN; ++A) {
        const int ax = A % Q, ay = (A / Q) % Q, az = A / (Q * Q);
        const int64_t node = (int64_t)(P * cx + ax) + (int64_t)g.nn[0] * ((P * cy + ay) + (int64_t)g.nn[1] * (P * cz + az));
#pragma unroll
        for (int f = 0; f < 3; ++f) un[f][A] = u[f * g.N + node];
    }
    const int32_t j0 = occ_start[o], j1 = occ_start[o + 1];
    for (int32_t j = j0 + lane; j < j1; j += LPC) {
        T Nx[Q], Ny[Q], Nz[Q];
        lagrange<T, P>(xi[j], Nx);
        lagrange<T, P>(xi[m + j], Ny);
        lagrange<T, P>(xi[2 * m + j], Nz);
        T acc[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int A = 0; A < NEN; ++A) {
            const T w = Nx[A % Q] * Ny[(A / Q) % Q] * Nz[A / (Q * Q)];
#pragma unroll
            for (int f = 0; f < 3; ++f) acc[f] += w * un[f][A];
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) Bu[f * m + j] = acc[f];
    }
}

// Bu = 0 at the located positions of the points outside the grid (occ_start[n_occ] .. m - 1)
template <typename T>
__global__ __launch_bounds__(256) void dlm_zero_tail(int64_t m, int64_t n_occ, const int32_t *__restrict__ occ_start,
                                                     T *__restrict__ Bu)
{
    const int64_t first = occ_start[n_occ];
    for (int64_t j = first + (int64_t)blockIdx.x * 256 + threadIdx.x; j < m; j += (int64_t)gridDim.x * 256)
#pragma unroll
        for (int f = 0; f < 3; ++f) Bu[f * m + j] = T(0);
}

// dst[f][j] = src[f][perm[j]] (to located order) or dst[f][perm[j]] = src[f][j] (back)
template <typename T, bool BACK>
__global__ __launch_bounds__(256) void dlm_permute_k(int64_t m, int nf, const int32_t *__restrict__ perm,
                                                     const T *__restrict__ src, T *__restrict__ dst)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const int64_t p = perm[j];
    for (int f = 0; f < nf; ++f) {
        if (BACK)
            dst[f * m + p] = src[f * m + j];
        else
            dst[f * m + j] = src[f * m + p];
    }
}

template <typename T, int P, bool FROM_U, int LPC>
__global__ __launch_bounds__(256) void dlm_cell_reduce(Geo g, int64_t m, int64_t n_occ,
                                                       const int32_t *__restrict__ occ_cell,
                                                       const int32_t *__restrict__ occ_start,
                                                       const int32_t *__restrict__ perm,
                                                       const T *__restrict__ xi,
                                                       const T *__restrict__ kappa,
                                                       const T *__restrict__ src,
                                                       const uint32_t *__restrict__ mask,
                                                       T *__restrict__ csum)
{
    constexpr int Q = P + 1, NEN = Q * Q * Q;
    static_assert(LPC == 8 || LPC == 64, "lanes per cell");
    const int64_t o = ((int64_t)blockIdx.x * 256 + threadIdx.x) / LPC;
    const int lane = threadIdx.x % LPC;
    if (o >= n_occ) return;   // the LPC lanes of a cell leave together
    const int32_t c = occ_cell[o];
    const int cx = c % g.n[0], cy = (c / g.n[0]) % g.n[1], cz = c / (g.n[0] * g.n[1]);
    T un[FROM_U ? 3 : 1][FROM_U ? NEN : 1];
    if constexpr (FROM_U) {
#pragma unroll
        for (int A = 0; A < NEN; ++A) {
            const int ax = A % Q, ay = (A / Q) % Q, az = A / (Q * Q);
            const int64_t node = (int64_t)(P * cx + ax) +
                                 (int64_t)g.nn[0] * ((P * cy + ay) + (int64_t)g.nn[1] * (P * cz + az));
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                T v = src[f * g.N + node];
                if (mask_bit(mask, f * g.N + node)) v = T(0);
                un[f][A] = v;
            }
        }
    }
    double acc[NEN][3];
#pragma unroll
    for (int A = 0; A < NEN; ++A)
#pragma unroll
        for (int f = 0; f < 3; ++f) acc[A][f] = 0.0;
    const int32_t j0 = occ_start[o], j1 = occ_start[o + 1];
    // FP32: UB points per lane and round, their sorted positions' point indices loaded together,
    // then their xi / kappa / src, then accumulated in ascending order (the loads of a round in
    // flight together instead of one dependent chain per point).  FP64 keeps one point per round:
    // the extra registers cost it a wave per SIMD, which measured slower.
    constexpr int UB = sizeof(T) == 4 ? (P == 1 ? 4 : 2) : 1;
    for (int32_t j = j0 + lane; j < j1; j += LPC * UB) {
        int32_t bs[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int32_t ju = j + u * LPC;
            const int32_t jc = ju < j1 ? ju : j;
            bs[u] = perm != nullptr ? perm[jc] : jc;   // NULL: per-point arrays in located order
        }
        T xs[UB][3], kbs[UB], ms[UB][3];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int32_t b = bs[u];
#pragma unroll
            for (int d = 0; d < 3; ++d) xs[u][d] = xi[d * m + b];
            kbs[u] = kappa ? kappa[b] : T(1);
            if constexpr (!FROM_U) {
#pragma unroll
                for (int f = 0; f < 3; ++f) ms[u][f] = src[f * m + b];
            }
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            if (j + u * LPC >= j1) break;
            T Nx[Q], Ny[Q], Nz[Q];
            lagrange<T, P>(xs[u][0], Nx);
            lagrange<T, P>(xs[u][1], Ny);
            lagrange<T, P>(xs[u][2], Nz);
            const T kb = kbs[u];
            T mu[3];
            if constexpr (FROM_U) {
                T bu[3] = {T(0), T(0), T(0)};
#pragma unroll
                for (int A = 0; A < NEN; ++A) {
                    const T w = Nx[A % Q] * Ny[(A / Q) % Q] * Nz[A / (Q * Q)];
#pragma unroll
                    for (int f = 0; f < 3; ++f) bu[f] += w * un[f][A];
                }
#pragma unroll
                for (int f = 0; f < 3; ++f) mu[f] = kb * bu[f];
            } else {
#pragma unroll
                for (int f = 0; f < 3; ++f) mu[f] = kb * ms[u][f];
            }
#pragma unroll
            for (int A = 0; A < NEN; ++A) {
                const T w = Nx[A % Q] * Ny[(A / Q) % Q] * Nz[A / (Q * Q)];
#pragma unroll
                for (int f = 0; f < 3; ++f) acc[A][f] += (double)(w * mu[f]);
            }
        }
    }
#pragma unroll
    for (int A = 0; A < NEN; ++A)
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            double v = acc[A][f];
#pragma unroll
            for (int off = 1; off < LPC; off <<= 1) v += __shfl_xor(v, off, 64);
            if ((A * 3 + f) % LPC == lane) csum[(o * NEN + A) * 3 + f] = (T)v;
        }
}

// Per occupied cell o, the (p+1)^3 x (p+1)^3 block of B^T diag(kappa) B restricted to the
// cell's nodes: gram[o][A][C] = sum_{B in cell} kappa_B N_A(xi_B) N_C(xi_B).  One wave per cell:
// lanes stage 64 points' shape values in LDS, then each lane sums its entries over the staged
// points in point order (deterministic; the two triangles are bitwise equal).
template <typename T, int P>
__global__ __launch_bounds__(64) void dlm_gram_kernel(int64_t m, const int32_t *__restrict__ occ_start,
                                                      const int32_t *__restrict__ perm,
                                                      const T *__restrict__ xi,
                                                      const T *__restrict__ kappa,
                                                      T *__restrict__ gram)
{
    constexpr int Q = P + 1, NEN = Q * Q * Q, NE = NEN * NEN;
    constexpr int PER = (NE + 63) / 64;
    __shared__ T sN[NEN][64];
    __shared__ T sK[64];
    const int64_t o = blockIdx.x;
    const int lane = threadIdx.x;
    const int32_t j0 = occ_start[o], j1 = occ_start[o + 1];
    T acc[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) acc[r] = T(0);
    for (int32_t base = j0; base < j1; base += 64) {
        const int32_t j = base + lane;
        if (j < j1) {
            const int32_t b = perm[j];
            T Nx[Q], Ny[Q], Nz[Q];
            lagrange<T, P>(xi[b], Nx);
            lagrange<T, P>(xi[m + b], Ny);
            lagrange<T, P>(xi[2 * m + b], Nz);
#pragma unroll
            for (int A = 0; A < NEN; ++A) sN[A][lane] = Nx[A % Q] * Ny[(A / Q) % Q] * Nz[A / (Q * Q)];
            sK[lane] = kappa ? kappa[b] : T(1);
        }
        __syncthreads();
        const int cnt = (j1 - base) < 64 ? (j1 - base) : 64;
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int e = lane + 64 * r;
            if (e < NE) {
                const int A = e / NEN, C = e % NEN;
                T v = acc[r];
                for (int k = 0; k < cnt; ++k) {
                    // the product kappa N_A N_C is formed symmetrically in A and C
                    const T na = sN[A][k], nc = sN[C][k];
                    const T w = (A <= C) ? (sK[k] * na) * nc : (sK[k] * nc) * na;
                    v += w;
                }
                acc[r] = v;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int e = lane + 64 * r;
        if (e < NE) gram[o * NE + e] = acc[r];
    }
}

// y[3][N] += corner sums of the occupied neighbour cells (standalone B^T)
// y += (B^T kappa lam) at the nodes of occupied cells.  One lane per (occupied cell, corner):
// the lane whose cell is the node's first occupied cell in the fixed loop order below sums the
// corner sums of every occupied cell holding the node, in that order, and writes the node once
// (no atomics, deterministic; nodes away from the solid are not visited)
template <typename T, int P>
__global__ __launch_bounds__(256) void dlm_node_gather(Geo g, int64_t n_occ, const int32_t *__restrict__ occ_cell,
                                                       const T *__restrict__ csum,
                                                       const int32_t *__restrict__ occ_index,
                                                       T *__restrict__ y)
{
    constexpr int Q = P + 1, NEN = Q * Q * Q;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_occ * NEN) return;
    const int64_t o = t / NEN;
    const int corner = (int)(t - o * NEN);
    const int32_t c0 = occ_cell[o];
    const int gv[3] = {P * (c0 % g.n[0]) + corner % Q, P * ((c0 / g.n[0]) % g.n[1]) + (corner / Q) % Q,
                       P * (c0 / (g.n[0] * g.n[1])) + corner / (Q * Q)};
    const int64_t node = gv[0] + (int64_t)g.nn[0] * (gv[1] + (int64_t)g.nn[1] * gv[2]);
    int cs[3][2], as[3][2], nc[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        nc[d] = 0;
        if (gv[d] >= P && gv[d] % P == 0) { cs[d][nc[d]] = gv[d] / P - 1; as[d][nc[d]++] = P; }
        const int c = gv[d] / P;
        if (c < g.n[d]) { cs[d][nc[d]] = c; as[d][nc[d]++] = gv[d] - P * c; }
    }
    T acc[3] = {T(0), T(0), T(0)};
    bool first = true;
    for (int iz = 0; iz < nc[2]; ++iz)
        for (int iy = 0; iy < nc[1]; ++iy)
            for (int ix = 0; ix < nc[0]; ++ix) {
                const int64_t c = cs[0][ix] + (int64_t)g.n[0] * (cs[1][iy] + (int64_t)g.n[1] * cs[2][iz]);
                const int32_t ko = occ_index[c];
                if (ko >= 0) {
                    if (first && ko != o) return;   // another lane owns this node
                    first = false;
                    const int A = as[0][ix] + Q * (as[1][iy] + Q * as[2][iz]);
#pragma unroll
                    for (int f = 0; f < 3; ++f) acc[f] += csum[((int64_t)ko * NEN + A) * 3 + f];
                }
            }
#pragma unroll
    for (int f = 0; f < 3; ++f) y[f * g.N + node] += acc[f];
}

inline unsigned nblk(int64_t n, int per = 256) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int scan_exclusive(const int32_t *in, int64_t n, int32_t *out, int32_t *part,
                          hipStream_t st)
{
    const int64_t nparts = (n + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(scan_reduce, dim3((unsigned)nparts), dim3(SCAN_THREADS), 0, st, in, n, part);
    FSI_LAUNCH_CHECK();
    hipLaunchKernelGGL(scan_partials, dim3(1), dim3(1024), 0, st, part, nparts);
    FSI_LAUNCH_CHECK();
    hipLaunchKernelGGL(scan_down, dim3((unsigned)nparts), dim3(SCAN_THREADS), 0, st, in, n, part, out);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

struct LocateWs {
    int32_t *keys_a, *keys_b, *vals_a, *vals_b, *hist, *flags, *pos, *part, *counters;
    size_t bytes;
};

static LocateWs locate_ws_layout(const Geo &g, int64_t m, char *base)
{
    LocateWs w{};
    const int64_t nb = (m + SORT_TILE - 1) / SORT_TILE;
    const int64_t nhist = (int64_t)RADIX * (nb > 0 ? nb : 1);
    const int64_t nscan = m > nhist ? m : nhist;
    const int64_t nparts = (nscan + SCAN_TILE - 1) / SCAN_TILE + 1;
    size_t off = 0;
    auto take = [&](int64_t count) {
        int32_t *p = base ? reinterpret_cast<int32_t *>(base + off) : nullptr;
        off += align_up((size_t)count * sizeof(int32_t));
        return p;
    };
    w.keys_a = take(m > 0 ? m : 1);
    w.keys_b = take(m > 0 ? m : 1);
    w.vals_a = take(m > 0 ? m : 1);
    w.vals_b = take(m > 0 ? m : 1);
    w.hist = take(nhist);
    w.flags = take(m > 0 ? m : 1);
    w.pos = take(nhist > m ? nhist : (m > 0 ? m : 1));
    w.part = take(nparts + 1);
    w.counters = take(4);
    w.bytes = off;
    (void)g;
    return w;
}

size_t locate_workspace_bytes(const Geo &g, int64_t m) { return locate_ws_layout(g, m, nullptr).bytes; }

int launch_locate(const Geo &g, int64_t m, const double *X, fsi_dtype dt, int32_t *cell, void *xi,
                  int32_t *perm, int32_t *occ_cell, int32_t *occ_start, int32_t *occ_index,
                  void *s_out, double s_max, int64_t *n_occ_host, int64_t *n_outside_host, void *ws,
                  hipStream_t st)
{
    LocateWs w = locate_ws_layout(g, m, reinterpret_cast<char *>(ws));
    ProfileScope prof("dlm_locate", st);
    FSI_HIP(hipMemsetAsync(w.counters, 0, 4 * sizeof(int32_t), st));
    // occ_index = -1 everywhere
    hipLaunchKernelGGL(fill_i32, dim3(nblk(g.E)), dim3(256), 0, st, occ_index, g.E, -1);
    FSI_LAUNCH_CHECK();
    if (m > 0) {
        if (dt == FSI_F64)
            hipLaunchKernelGGL(locate_kernel<double>, dim3(nblk(m)), dim3(256), 0, st, g, m, X, cell,
                               (double *)xi, w.keys_a, w.vals_a, w.counters);
        else
            hipLaunchKernelGGL(locate_kernel<float>, dim3(nblk(m)), dim3(256), 0, st, g, m, X, cell,
                               (float *)xi, w.keys_a, w.vals_a, w.counters);
        FSI_LAUNCH_CHECK();
        // stable radix sort over the bits needed for keys in [0, E]
        int bits = 0;
        while (bits < 31 && ((int64_t)1 << bits) <= g.E) ++bits;
        const int nb = (int)((m + SORT_TILE - 1) / SORT_TILE);
        int32_t *kin = w.keys_a, *vin = w.vals_a, *kout = w.keys_b, *vout = w.vals_b;
        for (int shift = 0; shift < bits; shift += RADIX_BITS) {
            hipLaunchKernelGGL(radix_hist, dim3(nb), dim3(SORT_THREADS), 0, st, kin, m, shift, nb, w.hist);
            FSI_LAUNCH_CHECK();
            int rc = scan_exclusive(w.hist, (int64_t)RADIX * nb, w.pos, w.part, st);
            if (rc) return rc;
            hipLaunchKernelGGL(radix_scatter, dim3(nb), dim3(SORT_THREADS), 0, st, kin, vin, m, shift, nb,
                               w.pos, kout, vout);
            FSI_LAUNCH_CHECK();
            std::swap(kin, kout);
            std::swap(vin, vout);
        }
        FSI_HIP(hipMemcpyAsync(perm, vin, (size_t)m * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
        // occupied cells: flags at the first point of each inside run, positions by scan
        hipLaunchKernelGGL(occ_flags, dim3(nblk(m)), dim3(256), 0, st, kin, m, g.E, w.flags);
        FSI_LAUNCH_CHECK();
        int rc = scan_exclusive(w.flags, m, w.pos, w.part, st);
        if (rc) return rc;
        hipLaunchKernelGGL(occ_emit, dim3(nblk(m)), dim3(256), 0, st, kin, m, g.E, w.flags, w.pos,
                           occ_cell, occ_start, occ_index);
        FSI_LAUNCH_CHECK();
    }
    // n_occ = total of flags (part[nparts] after the scan), n_inside = m - n_outside
    int32_t host[2] = {0, 0};
    const int64_t nparts = (m + SCAN_TILE - 1) / SCAN_TILE;
    if (m > 0) FSI_HIP(hipMemcpyAsync(&host[0], w.part + nparts, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FSI_HIP(hipMemcpyAsync(&host[1], w.counters, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FSI_HIP(hipStreamSynchronize(st));
    const int64_t n_occ = host[0];
    const int64_t n_inside = m - host[1];
    // close the CSR: occ_start[n_occ] = number of inside points
    const int32_t last = (int32_t)n_inside;
    FSI_HIP(hipMemcpyAsync(occ_start + n_occ, &last, sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (s_out) {
        FSI_HIP(hipMemcpyAsync(w.counters + 2, &host[0], sizeof(int32_t), hipMemcpyHostToDevice, st));
        if (dt == FSI_F64) {
            hipLaunchKernelGGL(fill_t<double>, dim3(nblk(g.N)), dim3(256), 0, st, (double *)s_out, g.N, 1.0);
            FSI_LAUNCH_CHECK();
            if (n_occ > 0)
                hipLaunchKernelGGL(mark_s<double>, dim3(nblk(n_occ)), dim3(256), 0, st, g, occ_cell,
                                   w.counters + 2, (double *)s_out, s_max);
        } else {
            hipLaunchKernelGGL(fill_t<float>, dim3(nblk(g.N)), dim3(256), 0, st, (float *)s_out, g.N, 1.0f);
            FSI_LAUNCH_CHECK();
            if (n_occ > 0)
                hipLaunchKernelGGL(mark_s<float>, dim3(nblk(n_occ)), dim3(256), 0, st, g, occ_cell,
                                   w.counters + 2, (float *)s_out, (float)s_max);
        }
        FSI_LAUNCH_CHECK();
    }
    // the host copy of `last` must stay alive until the copy ran
    FSI_HIP(hipStreamSynchronize(st));
    if (n_occ_host) *n_occ_host = n_occ;
    if (n_outside_host) *n_outside_host = host[1];
    return FSI_OK;
}

template <typename T>
static int launch_B_t(const Geo &g, int64_t m, const int32_t *cell, const T *xi, const T *u,
                      const uint32_t *mask, T *Bu, hipStream_t st)
{
    if (m == 0) return FSI_OK;
    if (g.p == 1) {
        if (mask != nullptr)
            hipLaunchKernelGGL((dlm_B_kernel<T, 1, true>), dim3(nblk(m)), dim3(256), 0, st, g, m, cell, xi, u, mask, Bu);
        else
            hipLaunchKernelGGL((dlm_B_kernel<T, 1, false>), dim3(nblk(m)), dim3(256), 0, st, g, m, cell, xi, u, mask, Bu);
    } else {
        if (mask != nullptr)
            hipLaunchKernelGGL((dlm_B_kernel<T, 2, true>), dim3(nblk(m)), dim3(256), 0, st, g, m, cell, xi, u, mask, Bu);
        else
            hipLaunchKernelGGL((dlm_B_kernel<T, 2, false>), dim3(nblk(m)), dim3(256), 0, st, g, m, cell, xi, u, mask, Bu);
    }
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int launch_dlm_B(const Geo &g, fsi_dtype dt, int64_t m, const int32_t *cell, const void *xi,
                 const void *u, const uint32_t *mask, void *Bu, hipStream_t st)
{
    if (dt == FSI_F64)
        return launch_B_t<double>(g, m, cell, (const double *)xi, (const double *)u, mask, (double *)Bu, st);
    return launch_B_t<float>(g, m, cell, (const float *)xi, (const float *)u, mask, (float *)Bu, st);
}

template <typename T>
static int launch_B_located_t(const Geo &g, int64_t m, int64_t n_occ, const int32_t *occ_cell,
                              const int32_t *occ_start, const T *xi, const T *u, T *Bu, hipStream_t st)
{
    if (m == 0) return FSI_OK;
    if (n_occ > 0) {
        if (g.p == 1)
            hipLaunchKernelGGL((dlm_B_located<T, 1, 8>), dim3((unsigned)((n_occ + 31) / 32)), dim3(256), 0, st, g, m,
                               n_occ, occ_cell, occ_start, xi, u, Bu);
        else
            hipLaunchKernelGGL((dlm_B_located<T, 2, 64>), dim3((unsigned)((n_occ + 3) / 4)), dim3(256), 0, st, g,
                               m, n_occ, occ_cell, occ_start, xi, u, Bu);
        FSI_LAUNCH_CHECK();
    }
    const unsigned tb = (unsigned)std::min<int64_t>(nblk(m), 1024);
    hipLaunchKernelGGL(dlm_zero_tail<T>, dim3(tb), dim3(256), 0, st, m, n_occ, occ_start, Bu);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int launch_dlm_B_located(const Geo &g, fsi_dtype dt, int64_t m, int64_t n_occ, const int32_t *occ_cell,
                         const int32_t *occ_start, const void *xi, const void *u, void *Bu, hipStream_t st)
{
    if (dt == FSI_F64)
        return launch_B_located_t<double>(g, m, n_occ, occ_cell, occ_start, (const double *)xi, (const double *)u,
                                          (double *)Bu, st);
    return launch_B_located_t<float>(g, m, n_occ, occ_cell, occ_start, (const float *)xi, (const float *)u,
                                     (float *)Bu, st);
}

int launch_dlm_permute(fsi_dtype dt, int64_t m, int nf, const int32_t *perm, bool back, const void *src, void *dst,
                       hipStream_t st)
{
    if (m == 0 || nf == 0) return FSI_OK;
    const dim3 grid(nblk(m));
    if (dt == FSI_F64) {
        if (back)
            hipLaunchKernelGGL((dlm_permute_k<double, true>), grid, dim3(256), 0, st, m, nf, perm,
                               (const double *)src, (double *)dst);
        else
            hipLaunchKernelGGL((dlm_permute_k<double, false>), grid, dim3(256), 0, st, m, nf, perm,
                               (const double *)src, (double *)dst);
    } else {
        if (back)
            hipLaunchKernelGGL((dlm_permute_k<float, true>), grid, dim3(256), 0, st, m, nf, perm,
                               (const float *)src, (float *)dst);
        else
            hipLaunchKernelGGL((dlm_permute_k<float, false>), grid, dim3(256), 0, st, m, nf, perm,
                               (const float *)src, (float *)dst);
    }
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

size_t dlm_csum_bytes(const Geo &g, int64_t n_occ, fsi_dtype dt)
{
    const int nen = (g.p + 1) * (g.p + 1) * (g.p + 1);
    const size_t es = dt == FSI_F64 ? 8 : 4;
    return align_up((size_t)(n_occ > 0 ? n_occ : 1) * nen * 3 * es);
}

template <typename T>
static int launch_reduce_t(const Geo &g, bool from_u, int64_t m, int64_t n_occ, const int32_t *occ_cell,
                           const int32_t *occ_start, const int32_t *perm, const T *xi, const T *kappa,
                           const T *src, const uint32_t *mask, T *csum, hipStream_t st)
{
    if (n_occ == 0) return FSI_OK;
    ProfileScope prof("dlm_cell_reduce", st);
    if (g.p == 1) {
        // Q1: 8 lanes per cell (24 corner sums, ~tens of points per cell)
        const unsigned blocks = (unsigned)((n_occ + 31) / 32);
        if (from_u)
            hipLaunchKernelGGL((dlm_cell_reduce<T, 1, true, 8>), dim3(blocks), dim3(256), 0, st, g, m, n_occ,
                               occ_cell, occ_start, perm, xi, kappa, src, mask, csum);
        else
            hipLaunchKernelGGL((dlm_cell_reduce<T, 1, false, 8>), dim3(blocks), dim3(256), 0, st, g, m, n_occ,
                               occ_cell, occ_start, perm, xi, kappa, src, mask, csum);
    } else {
        // Q2: a wavefront per cell (81 corner sums)
        const unsigned blocks = (unsigned)((n_occ + 3) / 4);
        if (from_u)
            hipLaunchKernelGGL((dlm_cell_reduce<T, 2, true, 64>), dim3(blocks), dim3(256), 0, st, g, m, n_occ,
                               occ_cell, occ_start, perm, xi, kappa, src, mask, csum);
        else
            hipLaunchKernelGGL((dlm_cell_reduce<T, 2, false, 64>), dim3(blocks), dim3(256), 0, st, g, m, n_occ,
                               occ_cell, occ_start, perm, xi, kappa, src, mask, csum);
    }
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int launch_dlm_cell_reduce(const Geo &g, fsi_dtype dt, bool from_u, int64_t m, int64_t n_occ,
                           const int32_t *occ_cell, const int32_t *occ_start, const int32_t *perm,
                           const void *xi, const void *kappa, const void *src, const uint32_t *mask,
                           void *csum, hipStream_t st)
{
    if (dt == FSI_F64)
        return launch_reduce_t<double>(g, from_u, m, n_occ, occ_cell, occ_start, perm, (const double *)xi,
                                       (const double *)kappa, (const double *)src, mask, (double *)csum, st);
    return launch_reduce_t<float>(g, from_u, m, n_occ, occ_cell, occ_start, perm, (const float *)xi,
                                  (const float *)kappa, (const float *)src, mask, (float *)csum, st);
}

int launch_dlm_gram(const Geo &g, fsi_dtype dt, int64_t m, int64_t n_occ, const int32_t *occ_start,
                    const int32_t *perm, const void *xi, const void *kappa, void *gram, hipStream_t st)
{
    if (n_occ == 0) return FSI_OK;
    ProfileScope prof("dlm_gram", st);
    if (dt == FSI_F64) {
        if (g.p == 1)
            hipLaunchKernelGGL((dlm_gram_kernel<double, 1>), dim3((unsigned)n_occ), dim3(64), 0, st, m,
                               occ_start, perm, (const double *)xi, (const double *)kappa, (double *)gram);
        else
            hipLaunchKernelGGL((dlm_gram_kernel<double, 2>), dim3((unsigned)n_occ), dim3(64), 0, st, m,
                               occ_start, perm, (const double *)xi, (const double *)kappa, (double *)gram);
    } else {
        if (g.p == 1)
            hipLaunchKernelGGL((dlm_gram_kernel<float, 1>), dim3((unsigned)n_occ), dim3(64), 0, st, m,
                               occ_start, perm, (const float *)xi, (const float *)kappa, (float *)gram);
        else
            hipLaunchKernelGGL((dlm_gram_kernel<float, 2>), dim3((unsigned)n_occ), dim3(64), 0, st, m,
                               occ_start, perm, (const float *)xi, (const float *)kappa, (float *)gram);
    }
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int launch_dlm_node_gather(const Geo &g, fsi_dtype dt, int64_t n_occ, const int32_t *occ_cell, const void *csum,
                           const int32_t *occ_index, void *y, hipStream_t st)
{
    if (n_occ == 0) return FSI_OK;
    const unsigned blocks = nblk(n_occ * (g.p == 1 ? 8 : 27));
    if (dt == FSI_F64) {
        if (g.p == 1)
            hipLaunchKernelGGL((dlm_node_gather<double, 1>), dim3(blocks), dim3(256), 0, st, g, n_occ, occ_cell,
                               (const double *)csum, occ_index, (double *)y);
        else
            hipLaunchKernelGGL((dlm_node_gather<double, 2>), dim3(blocks), dim3(256), 0, st, g, n_occ, occ_cell,
                               (const double *)csum, occ_index, (double *)y);
    } else {
        if (g.p == 1)
            hipLaunchKernelGGL((dlm_node_gather<float, 1>), dim3(blocks), dim3(256), 0, st, g, n_occ, occ_cell,
                               (const float *)csum, occ_index, (float *)y);
        else
            hipLaunchKernelGGL((dlm_node_gather<float, 2>), dim3(blocks), dim3(256), 0, st, g, n_occ, occ_cell,
                               (const float *)csum, occ_index, (float *)y);
    }
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

}  // namespace fsi
