// Schur-complement block preconditioner of the reduced 2x2 system (section 2.4: the
// block system is solved by Krylov iterations with block preconditioners built from
// its sub-matrices).
//
// With J = [[F, G], [D, C]] (velocity rows, pressure rows), P = [[F_hat, G], [0, S_hat]]
// (or its block diagonal): F_hat = the nodal 3x3 velocity blocks of J; S_hat = the
// variable-coefficient pressure Laplacian -div(alpha grad p) on the node lattice
// (trilinear elements, lattice spacing h/p), alpha = tau_m + 1/(c_m + DLM density),
// which is what S = C - D F^{-1} G looks like for this operator (PSPG gives C =
// tau_m Laplacian; D = -G^T and F ~ c_m M + the DLM block give G^T F^{-1} G ~ a
// Laplacian scaled by 1/(c_m + DLM density)).  S_hat^{-1} is one geometric-multigrid
// V(2,2) cycle: weighted Jacobi (8/9) smoothing, trilinear prolongation,
// restriction = its transpose, coefficients averaged 2x2x2 onto coarser levels,
// coarsest level solved by a dense inverse.  The Laplacian has Dirichlet rows at
// boundary nodes whose velocity is not fully prescribed (traction-free boundaries fix
// the pressure level); their rows are solved by the diagonal.
//
// Kernels (one lane per node or lattice cell, no atomics except a per-block flag count):
//   sc_node_beta   beta_A = 1/(c_m + max(d_A,0)/v_A), d_A = DLM row sums from the per-cell
//                  Gram blocks (partition of unity: sum_A' G_AA' = sum_B kappa_B N_A(xi_B))
//   sc_cell_alpha  alpha per lattice cell from corner means of a, s, beta
//   sc_dmask0      Dirichlet flags of the Laplacian (level 0)
//   sc_coarsen_*   coarse alpha (mean of 8 children), coarse flags by injection
//   sc_vel_inverse 3x3 velocity block inverses (FP64, FP32 copy)
//   sc_first/sc_sweep/sc_restrict/sc_prolong/sc_coarse: the V-cycle (sc_sweep: Jacobi sweep or
//                  residual with the 27-point variable-coefficient stencil)
//   sc_vel_apply   z_u = F_hat^{-1} (v_u - [J (0, z_p)]_u) with the nodal block inverses, or
//   sc_vel_resid, sc_mr_dots, sc_mr_alpha, sc_mr_update: minimal-residual steps on F (the velocity
//                  rows of J [u; 0]) preconditioned by them; the step length stays on the device
// Every vector of the V-cycle keeps zeros at Dirichlet nodes, so the 27-point stencil
// needs no mask on its neighbours.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "profile.hpp"
#include "schur.hpp"

namespace fsi {

namespace {

constexpr int SC_TX = 32, SC_TY = 8;

template <typename T>
struct Lv {
    int nn[3], nc[3];
    T kc[8];
};

template <typename T>
Lv<T> lv_of(const ScLevel &L)
{
    Lv<T> o;
    for (int d = 0; d < 3; ++d) {
        o.nn[d] = L.nn[d];
        o.nc[d] = L.nc[d];
    }
    for (int i = 0; i < 8; ++i) o.kc[i] = (T)L.kc[i];
    return o;
}

dim3 node_grid(const ScLevel &L)
{
    return dim3((unsigned)((L.nn[0] + SC_TX - 1) / SC_TX), (unsigned)((L.nn[1] + SC_TY - 1) / SC_TY),
                (unsigned)L.nn[2]);
}

// alpha of the 8 lattice cells around node (i, j, k), zero where a cell does not exist;
// al[oz][oy][ox] is the cell (i - 1 + ox, j - 1 + oy, k - 1 + oz)
template <typename T>
__device__ __forceinline__ void cell_alphas(const Lv<T> &L, const T *__restrict__ alpha, int i, int j,
                                            int k, T al[2][2][2])
{
#pragma unroll
    for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int oy = 0; oy < 2; ++oy)
#pragma unroll
            for (int ox = 0; ox < 2; ++ox) {
                const int cx = i - 1 + ox, cy = j - 1 + oy, cz = k - 1 + oz;
                const bool ok = cx >= 0 && cx < L.nc[0] && cy >= 0 && cy < L.nc[1] && cz >= 0 && cz < L.nc[2];
                const int qx = ok ? cx : 0, qy = ok ? cy : 0, qz = ok ? cz : 0;
                const T v = alpha[qx + L.nc[0] * (qy + L.nc[1] * qz)];
                al[oz][oy][ox] = ok ? v : T(0);
            }
}

template <typename T>
__device__ __forceinline__ T diag_only(const Lv<T> &L, const T *__restrict__ alpha, int i, int j, int k)
{
    T al[2][2][2];
    cell_alphas(L, alpha, i, j, k, al);
    T s = T(0);
#pragma unroll
    for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int oy = 0; oy < 2; ++oy)
#pragma unroll
            for (int ox = 0; ox < 2; ++ox) s += al[oz][oy][ox];
    return L.kc[0] * s;
}

#define SC_NODE_INDEX(L)                                                   \
    const int i = blockIdx.x * SC_TX + threadIdx.x;                        \
    const int j = blockIdx.y * SC_TY + threadIdx.y;                        \
    const int k = blockIdx.z;                                              \
    if (i >= (L).nn[0] || j >= (L).nn[1]) return;                          \
    const int id = i + (L).nn[0] * (j + (L).nn[1] * k)

// level 0, first sweep from a zero guess: b = v_p (all nodes), x = w b / diag (0 at Dirichlet)
template <typename T, typename TV>
__global__ __launch_bounds__(256) void sc_first(Lv<T> L, const T *__restrict__ alpha,
                                                const uint8_t *__restrict__ dm, const TV *__restrict__ vp,
                                                T *__restrict__ b, T *__restrict__ x, T omega)
{
    SC_NODE_INDEX(L);
    const T bv = (T)vp[id];
    b[id] = bv;
    x[id] = dm[id] ? T(0) : omega * bv / diag_only(L, alpha, i, j, k);
}

// One stencil sweep over a level, one lane per node (32 x 8 nodes per block, one plane per
// block, 32-bit offsets: every level holds fewer than 2^31 nodes).  The coefficient of
// neighbour A + delta is kc[pattern(delta)] times the sum of alpha over the cells holding both
// nodes: along an axis with delta = -1 only the lower cell, +1 the upper one, 0 both.
//   MODE 0: xo = x + w (b - K x) / diag     (0 at Dirichlet nodes)
//   MODE 1: xo = b - K x                    (0 at Dirichlet nodes)
//   MODE 2: zp = x + w (b - K x) / diag, b / diag at Dirichlet nodes (output precision TZ)
constexpr int SW_TX = 32, SW_TY = 8;

template <typename T, typename TZ, int MODE>
__global__ __launch_bounds__(256) void sc_sweep(Lv<T> L, const T *__restrict__ alpha,
                                                const uint8_t *__restrict__ dm, const T *__restrict__ b,
                                                const T *__restrict__ x, T *__restrict__ xo,
                                                TZ *__restrict__ zp, T omega)
{
    const int i = blockIdx.x * SW_TX + threadIdx.x, j = blockIdx.y * SW_TY + threadIdx.y, k = blockIdx.z;
    const int nx = L.nn[0], ny = L.nn[1], nz = L.nn[2];
    if (i >= nx || j >= ny) return;
    const int cnx = L.nc[0], cnxy = L.nc[0] * L.nc[1];
    T al[2][2][2];
#pragma unroll
    for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int oy = 0; oy < 2; ++oy)
#pragma unroll
            for (int ox = 0; ox < 2; ++ox) {
                const int cx = i - 1 + ox, cy = j - 1 + oy, cz = k - 1 + oz;
                const bool ok = cx >= 0 && cx < L.nc[0] && cy >= 0 && cy < L.nc[1] && cz >= 0 && cz < L.nc[2];
                const T v = alpha[ok ? cx + cnx * cy + cnxy * cz : 0];
                al[oz][oy][ox] = ok ? v : T(0);
            }
    T sx[2][2][3];
#pragma unroll
    for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int oy = 0; oy < 2; ++oy) {
            sx[oz][oy][0] = al[oz][oy][0];
            sx[oz][oy][2] = al[oz][oy][1];
            sx[oz][oy][1] = al[oz][oy][0] + al[oz][oy][1];
        }
    T sy[2][3][3];
#pragma unroll
    for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            sy[oz][0][dx] = sx[oz][0][dx];
            sy[oz][2][dx] = sx[oz][1][dx];
            sy[oz][1][dx] = sx[oz][0][dx] + sx[oz][1][dx];
        }
    const int nxy = nx * ny;
    T y = T(0), d = T(1);
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) {
        const int kk = min(max(k + dz - 1, 0), nz - 1);
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int row = min(max(j + dy - 1, 0), ny - 1) * nx + kk * nxy;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int ii = min(max(i + dx - 1, 0), nx - 1);
                const T S = dz == 0 ? sy[0][dy][dx] : (dz == 2 ? sy[1][dy][dx] : sy[0][dy][dx] + sy[1][dy][dx]);
                const int pat = (dx != 1) + 2 * (dy != 1) + 4 * (dz != 1);
                y += (L.kc[pat] * S) * x[row + ii];
                if (pat == 0) d = L.kc[0] * S;
            }
        }
    }
    const int id = i + nx * j + nxy * k;
    const bool dir = dm[id] != 0;
    const T bv = b[id];
    if (MODE == 0) xo[id] = dir ? T(0) : x[id] + omega * (bv - y) / d;
    if (MODE == 1) xo[id] = dir ? T(0) : bv - y;
    if (MODE == 2) zp[id] = (TZ)(dir ? bv / d : x[id] + omega * (bv - y) / d);
}

dim3 sweep_grid(const ScLevel &L)
{
    return dim3((unsigned)((L.nn[0] + SW_TX - 1) / SW_TX), (unsigned)((L.nn[1] + SW_TY - 1) / SW_TY),
                (unsigned)L.nn[2]);
}

// coarse node (i, j, k): b_c = sum of fine residuals at (2i + di, ...) with weights 1 (di = 0)
// or 1/2 (di = +-1) per axis; first coarse sweep x_c = w b_c / diag_c
template <typename T>
__global__ __launch_bounds__(256) void sc_restrict(Lv<T> L, Lv<T> F, const T *__restrict__ alpha,
                                                   const uint8_t *__restrict__ dm, const T *__restrict__ rf,
                                                   T *__restrict__ b, T *__restrict__ x, T omega)
{
    SC_NODE_INDEX(L);
    if (dm[id]) {
        b[id] = T(0);
        x[id] = T(0);
        return;
    }
    const int fnx = F.nn[0], fnxy = F.nn[0] * F.nn[1];
    T s = T(0);
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
        const int fz = 2 * k + dz;
        if (fz < 0 || fz >= F.nn[2]) continue;
        T sz = T(0);
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            const int fy = 2 * j + dy;
            if (fy < 0 || fy >= F.nn[1]) continue;
            const T *row = rf + fy * fnx + fz * fnxy;
            const int fx = 2 * i;
            T sx = row[fx];
            if (fx > 0) sx += T(0.5) * row[fx - 1];
            if (fx + 1 < F.nn[0]) sx += T(0.5) * row[fx + 1];
            sz += dy == 0 ? sx : T(0.5) * sx;
        }
        s += dz == 0 ? sz : T(0.5) * sz;
    }
    b[id] = s;
    x[id] = omega * s / diag_only(L, alpha, i, j, k);
}

// fine node: x_f += trilinear interpolation of the coarse correction (skipped at Dirichlet
// nodes; coarse Dirichlet nodes hold zero)
template <typename T>
__global__ __launch_bounds__(256) void sc_prolong(Lv<T> L, Lv<T> C, const uint8_t *__restrict__ dm,
                                                  const T *__restrict__ xc, T *__restrict__ x)
{
    SC_NODE_INDEX(L);
    if (dm[id]) return;
    const int ci[2] = {i >> 1, (i >> 1) + (i & 1)}, cj[2] = {j >> 1, (j >> 1) + (j & 1)},
              ck[2] = {k >> 1, (k >> 1) + (k & 1)};
    const T wx = (i & 1) ? T(0.5) : T(1), wy = (j & 1) ? T(0.5) : T(1), wz = (k & 1) ? T(0.5) : T(1);
    const int nx = (i & 1) ? 2 : 1, ny = (j & 1) ? 2 : 1, nz = (k & 1) ? 2 : 1;
    T s = T(0);
    for (int c = 0; c < nz; ++c) {
        T sy = T(0);
        for (int bb = 0; bb < ny; ++bb) {
            const T *row = xc + cj[bb] * C.nn[0] + ck[c] * C.nn[0] * C.nn[1];
            T sx = T(0);
            for (int a = 0; a < nx; ++a) sx += row[ci[a]];
            sy += wx * sx;
        }
        s += wy * sy;
    }
    x[id] += wz * s;
}

// coarsest level: x = Kinv b (Kinv symmetric, zero rows/columns at Dirichlet nodes); one
// wavefront per row, lanes stride the row, then a butterfly sum across the wavefront
template <typename T>
__global__ __launch_bounds__(64) void sc_coarse(int n, const T *__restrict__ kinv, const T *__restrict__ b,
                                                T *__restrict__ x)
{
    const int r = blockIdx.x, lane = threadIdx.x;
    const T *row = kinv + (int64_t)r * n;
    T s = T(0);
    for (int c = lane; c < n; c += 64) s += row[c] * b[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) x[r] = s;
}

// single-level case: z_p = b / diag at Dirichlet nodes, the coarse solution elsewhere
template <typename T, typename TZ>
__global__ __launch_bounds__(256) void sc_finish(Lv<T> L, const T *__restrict__ alpha,
                                                 const uint8_t *__restrict__ dm, const T *__restrict__ b,
                                                 const T *__restrict__ x, TZ *__restrict__ zp)
{
    SC_NODE_INDEX(L);
    zp[id] = (TZ)(dm[id] ? b[id] / diag_only(L, alpha, i, j, k) : x[id]);
}

// z_u = F_hat^{-1} (v_u - yt_u)   (yt = J (0, z_p) or nullptr)
template <typename T, typename TV, typename TZ>
__global__ __launch_bounds__(256) void sc_vel_apply(int64_t N, const T *__restrict__ finv,
                                                    const TV *__restrict__ v, const T *__restrict__ yt,
                                                    TZ *__restrict__ z)
{
    const int64_t node = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (node >= N) return;
    T t[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        t[f] = (T)v[f * N + node];
        if (yt != nullptr) t[f] -= yt[f * N + node];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        T s = T(0);
#pragma unroll
        for (int c = 0; c < 3; ++c) s += finv[(int64_t)(3 * r + c) * N + node] * t[c];
        z[r * N + node] = (TZ)s;
    }
}

// ---- minimal-residual steps on the velocity block ----
constexpr int MR_NB = 2048;  // blocks of the dot-product pass (8 waves per SIMD)

// r = v_u - yt_u (yt = J (0, z_p) in the block-triangular form, or nullptr)
template <typename T, typename TV>
__global__ __launch_bounds__(256) void sc_vel_resid(int64_t n3, const TV *__restrict__ v, const T *__restrict__ yt,
                                                    T *__restrict__ r)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (int64_t)gridDim.x * 256) {
        T t = (T)v[i];
        if (yt != nullptr) t -= yt[i];
        r[i] = t;
    }
}

// per-block partial sums of q.r and q.q (FP64 accumulation, fixed tree order)
template <typename T>
__global__ __launch_bounds__(256) void sc_mr_dots(int64_t n3, const T *__restrict__ q, const T *__restrict__ r,
                                                  double *__restrict__ part)
{
    __shared__ double sh[2][256];
    double qr = 0.0, qq = 0.0;
    // 16-byte loads (the vectors are 16-byte aligned workspace slices), then the tail
    typedef T T16 __attribute__((ext_vector_type(16 / sizeof(T))));
    constexpr int L = 16 / sizeof(T);
    const int64_t nv = n3 / L, stride = (int64_t)gridDim.x * 256;
    const int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (int64_t i = i0; i < nv; i += stride) {
        const T16 a = reinterpret_cast<const T16 *>(q)[i], b = reinterpret_cast<const T16 *>(r)[i];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const double av = (double)a[l];
            qr += av * (double)b[l];
            qq += av * av;
        }
    }
    for (int64_t i = nv * L + i0; i < n3; i += stride) {
        const double a = (double)q[i];
        qr += a * (double)r[i];
        qq += a * a;
    }
    sh[0][threadIdx.x] = qr;
    sh[1][threadIdx.x] = qq;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sh[0][0];
        part[2 * blockIdx.x + 1] = sh[1][0];
    }
}

// alpha = (q.r) / (q.q) from the partials (0 if q = 0), kept on the device
__global__ __launch_bounds__(256) void sc_mr_alpha(int nb, const double *__restrict__ part, double *__restrict__ alpha)
{
    __shared__ double sh[2][256];
    double qr = 0.0, qq = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) {
        qr += part[2 * b];
        qq += part[2 * b + 1];
    }
    sh[0][threadIdx.x] = qr;
    sh[1][threadIdx.x] = qq;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) alpha[0] = sh[1][0] > 0.0 ? sh[0][0] / sh[1][0] : 0.0;
}

// z = (first ? 0 : z) + alpha p;  r -= alpha q
template <typename T>
__global__ __launch_bounds__(256) void sc_mr_update(int64_t n3, const double *__restrict__ alpha,
                                                    const T *__restrict__ p, const T *__restrict__ q,
                                                    T *__restrict__ z, T *__restrict__ r, int first)
{
    const T a = (T)alpha[0];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (int64_t)gridDim.x * 256) {
        z[i] = (first ? T(0) : z[i]) + a * p[i];
        r[i] -= a * q[i];
    }
}

// ---- setup kernels (FP64) ----

// node weight beta_A; the DLM row sum of node A is the sum over the occupied grid cells that
// hold A of row A of their Gram block (shape functions sum to one at every point)
template <int P>
__global__ __launch_bounds__(256) void sc_node_beta(Geo g, const double *__restrict__ gram,
                                                    const int32_t *__restrict__ occ_index, double c_m,
                                                    double v8, double *__restrict__ beta)
{
    constexpr int Q = P + 1, NEN = Q * Q * Q;
    const int64_t node = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (node >= g.N) return;
    const int gv[3] = {(int)(node % g.nn[0]), (int)((node / g.nn[0]) % g.nn[1]),
                       (int)(node / ((int64_t)g.nn[0] * g.nn[1]))};
    double d = 0.0;
    if (gram != nullptr) {
        int cs[3][2], as[3][2], nc[3];
        for (int dd = 0; dd < 3; ++dd) {
            nc[dd] = 0;
            if (gv[dd] >= P && gv[dd] % P == 0) { cs[dd][nc[dd]] = gv[dd] / P - 1; as[dd][nc[dd]++] = P; }
            const int c = gv[dd] / P;
            if (c < g.n[dd]) { cs[dd][nc[dd]] = c; as[dd][nc[dd]++] = gv[dd] - P * c; }
        }
        for (int iz = 0; iz < nc[2]; ++iz)
            for (int iy = 0; iy < nc[1]; ++iy)
                for (int ix = 0; ix < nc[0]; ++ix) {
                    const int64_t cell = cs[0][ix] + (int64_t)g.n[0] * (cs[1][iy] + (int64_t)g.n[1] * cs[2][iz]);
                    const int32_t ko = occ_index[cell];
                    if (ko < 0) continue;
                    const int A = as[0][ix] + Q * (as[1][iy] + Q * as[2][iz]);
                    const double *row = gram + ((int64_t)ko * NEN + A) * NEN;
                    for (int B = 0; B < NEN; ++B) d += row[B];
                }
    }
    double cnt = 1.0;
    for (int dd = 0; dd < 3; ++dd) cnt *= (gv[dd] == 0 || gv[dd] == g.nn[dd] - 1) ? 1.0 : 2.0;
    const double vA = cnt * v8;
    beta[node] = 1.0 / (c_m + (d > 0.0 ? d : 0.0) / vA);
}

// alpha per lattice cell: tau_m from the corner means of a and s, plus the corner mean of beta
__global__ __launch_bounds__(256) void sc_cell_alpha(Geo g, VmsConst<double> k, int ncx, int ncy, int ncz,
                                                     const double *__restrict__ a, const double *__restrict__ s,
                                                     const double *__restrict__ beta, double *__restrict__ a64,
                                                     float *__restrict__ a32)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t C = (int64_t)ncx * ncy * ncz;
    if (c >= C) return;
    const int cx = (int)(c % ncx), cy = (int)((c / ncx) % ncy), cz = (int)(c / ((int64_t)ncx * ncy));
    double am[3] = {0.0, 0.0, 0.0}, sm = 0.0, bm = 0.0;
    for (int o = 0; o < 8; ++o) {
        const int64_t node = (cx + (o & 1)) + (int64_t)g.nn[0] * ((cy + ((o >> 1) & 1)) +
                                                                  (int64_t)g.nn[1] * (cz + (o >> 2)));
        for (int d = 0; d < 3; ++d) am[d] += a[d * g.N + node];
        if (s != nullptr) sm += s[node];
        bm += beta[node];
    }
    for (int d = 0; d < 3; ++d) am[d] *= 0.125;
    sm = s != nullptr ? 0.125 * sm : 1.0;
    const double tb = sm * (k.K1 + am[0] * am[0] * k.ih2[0] + am[1] * am[1] * k.ih2[1] + am[2] * am[2] * k.ih2[2]);
    const double al = 1.0 / sqrt(tb) + 0.125 * bm;
    a64[c] = al;
    a32[c] = (float)al;
}

// Dirichlet flags of the Laplacian: boundary nodes whose velocity is not fully prescribed;
// per block, one count if the block flagged any node
__global__ __launch_bounds__(256) void sc_dmask0(Geo g, const uint32_t *__restrict__ mask,
                                                 uint8_t *__restrict__ dm, int32_t *__restrict__ cnt)
{
    const int64_t node = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int flag = 0;
    if (node < g.N) {
        const int64_t row = node / g.nn[0];   // one 64-bit division, the rest in 32 bits
        const int gv[3] = {(int)(node - row * g.nn[0]), (int)((uint32_t)row % (uint32_t)g.nn[1]),
                           (int)((uint32_t)row / (uint32_t)g.nn[1])};
        bool bnd = false;
        for (int d = 0; d < 3; ++d) bnd = bnd || gv[d] == 0 || gv[d] == g.nn[d] - 1;
        const bool all = mask_bit(mask, node) && mask_bit(mask, g.N + node) && mask_bit(mask, 2 * g.N + node);
        flag = bnd && !all;
        dm[node] = (uint8_t)flag;
    }
    if (__syncthreads_or(flag) && threadIdx.x == 0) atomicAdd(cnt, 1);
}

__global__ __launch_bounds__(256) void sc_coarsen_alpha(int fx, int fy, int cx_, int cy_, int cz_,
                                                        const double *__restrict__ af, double *__restrict__ ac64,
                                                        float *__restrict__ ac32)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= (int64_t)cx_ * cy_ * cz_) return;
    const int x = (int)(c % cx_), y = (int)((c / cx_) % cy_), z = (int)(c / ((int64_t)cx_ * cy_));
    double s = 0.0;
    for (int o = 0; o < 8; ++o)
        s += af[(2 * x + (o & 1)) + (int64_t)fx * ((2 * y + ((o >> 1) & 1)) + (int64_t)fy * (2 * z + (o >> 2)))];
    ac64[c] = 0.125 * s;
    ac32[c] = (float)(0.125 * s);
}

__global__ __launch_bounds__(256) void sc_coarsen_mask(int fnx, int fny, int cnx, int cny, int cnz,
                                                       const uint8_t *__restrict__ dmf, uint8_t *__restrict__ dmc)
{
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= (int64_t)cnx * cny * cnz) return;
    const int x = (int)(n % cnx), y = (int)((n / cnx) % cny), z = (int)(n / ((int64_t)cnx * cny));
    dmc[n] = dmf[2 * x + (int64_t)fnx * (2 * y + (int64_t)fny * 2 * z)];
}

// inverse of the 3x3 velocity part of each nodal 4x4 block (adjugate / determinant)
__global__ __launch_bounds__(256) void sc_vel_inverse(int64_t N, const double *__restrict__ raw,
                                                      double *__restrict__ f64, float *__restrict__ f32)
{
    const int64_t node = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (node >= N) return;
    double m[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) m[i][j] = raw[(int64_t)(4 * i + j) * N + node];
    double r[3][3];
    r[0][0] = m[1][1] * m[2][2] - m[1][2] * m[2][1];
    r[0][1] = m[0][2] * m[2][1] - m[0][1] * m[2][2];
    r[0][2] = m[0][1] * m[1][2] - m[0][2] * m[1][1];
    r[1][0] = m[1][2] * m[2][0] - m[1][0] * m[2][2];
    r[1][1] = m[0][0] * m[2][2] - m[0][2] * m[2][0];
    r[1][2] = m[0][2] * m[1][0] - m[0][0] * m[1][2];
    r[2][0] = m[1][0] * m[2][1] - m[1][1] * m[2][0];
    r[2][1] = m[0][1] * m[2][0] - m[0][0] * m[2][1];
    r[2][2] = m[0][0] * m[1][1] - m[0][1] * m[1][0];
    const double det = m[0][0] * r[0][0] + m[0][1] * r[1][0] + m[0][2] * r[2][0];
    const bool ok = det != 0.0 && std::isfinite(det);
    const double id = ok ? 1.0 / det : 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double v = ok ? r[i][j] * id : (i == j ? 1.0 : 0.0);
            f64[(int64_t)(3 * i + j) * N + node] = v;
            f32[(int64_t)(3 * i + j) * N + node] = (float)v;
        }
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// dense inverse of the coarsest operator on its non-Dirichlet nodes (host, FP64): Cholesky
// A = L L^T row by row, U = L^{-T} (upper), A^{-1} = U U^T; every inner loop is a contiguous
// dot product
int coarse_inverse(const ScLevel &L, const std::vector<double> &alpha, const std::vector<uint8_t> &dm,
                   std::vector<double> &kinv)
{
    const int64_t n = L.N;
    std::vector<int64_t> pos((size_t)n, -1), keep;
    for (int64_t i = 0; i < n; ++i)
        if (!dm[(size_t)i]) {
            pos[(size_t)i] = (int64_t)keep.size();
            keep.push_back(i);
        }
    const int64_t m = (int64_t)keep.size();
    std::vector<double> A((size_t)(m * m), 0.0);
    for (int cz = 0; cz < L.nc[2]; ++cz)
        for (int cy = 0; cy < L.nc[1]; ++cy)
            for (int cx = 0; cx < L.nc[0]; ++cx) {
                const double al = alpha[(size_t)(cx + L.nc[0] * (cy + L.nc[1] * cz))];
                int64_t ids[8];
                for (int o = 0; o < 8; ++o)
                    ids[o] = pos[(size_t)((cx + (o & 1)) +
                                          (int64_t)L.nn[0] * ((cy + ((o >> 1) & 1)) + (int64_t)L.nn[1] * (cz + (o >> 2))))];
                for (int a = 0; a < 8; ++a)
                    for (int b = 0; b < 8; ++b)
                        if (ids[a] >= 0 && ids[b] >= 0) A[(size_t)(ids[a] * m + ids[b])] += al * L.kc[a ^ b];
            }
    // Cholesky-Banachiewicz: row i of L from rows j < i
    std::vector<double> Lm((size_t)(m * m), 0.0);
    for (int64_t i = 0; i < m; ++i) {
        double *li = &Lm[(size_t)(i * m)];
        for (int64_t j = 0; j <= i; ++j) {
            const double *lj = &Lm[(size_t)(j * m)];
            double s = A[(size_t)(i * m + j)];
            for (int64_t k = 0; k < j; ++k) s -= li[k] * lj[k];
            if (j == i) {
                if (!(s > 0.0)) {
                    set_error("coarsest pressure Laplacian is not positive definite");
                    return FSI_ERR_BREAKDOWN;
                }
                li[i] = std::sqrt(s);
            } else {
                li[j] = s / lj[j];
            }
        }
    }
    // U = L^{-T}: row r of U^T = L^{-1}; solve L y = e_c for each column c, store U[c][.] = y
    // transposed as U^T rows so that A^{-1}[i][j] = sum_k W[i][k] W[j][k] with W = L^{-T} rows
    std::vector<double> W((size_t)(m * m), 0.0);   // W[c][k] = (L^{-1})[k][c], k >= c
    std::vector<double> y((size_t)m);
    for (int64_t c = 0; c < m; ++c) {
        for (int64_t k = 0; k < c; ++k) y[(size_t)k] = 0.0;
        for (int64_t k = c; k < m; ++k) {
            const double *lk = &Lm[(size_t)(k * m)];
            double s = (k == c) ? 1.0 : 0.0;
            for (int64_t t = c; t < k; ++t) s -= lk[t] * y[(size_t)t];
            y[(size_t)k] = s / lk[k];
        }
        for (int64_t k = 0; k < m; ++k) W[(size_t)(c * m + k)] = y[(size_t)k];
    }
    // A^{-1} = L^{-T} L^{-1}: entry (i, j) = sum_k (L^{-1})[k][i] (L^{-1})[k][j] = W[i] . W[j]
    kinv.assign((size_t)(n * n), 0.0);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            const double *wi = &W[(size_t)(i * m)], *wj = &W[(size_t)(j * m)];
            double s = 0.0;
            for (int64_t k = i; k < m; ++k) s += wi[k] * wj[k];
            kinv[(size_t)(keep[i] * n + keep[j])] = s;
            kinv[(size_t)(keep[j] * n + keep[i])] = s;
        }
    return FSI_OK;
}

template <typename T, typename TV, typename TZ>
int vcycle(const ScPlan &p, char *base, const TV *vp, TZ *zp, hipStream_t st)
{
    const T omega = T(8.0 / 9.0);
    auto A = [&](int l) { return reinterpret_cast<const T *>(base + (sizeof(T) == 8 ? p.lv[l].a64 : p.lv[l].a32)); };
    auto D = [&](int l) { return reinterpret_cast<const uint8_t *>(base + p.lv[l].dm); };
    auto V = [&](int l, size_t off) { return reinterpret_cast<T *>(base + off); };
    const dim3 blk(SC_TX, SC_TY, 1), sblk(SW_TX, SW_TY, 1);
    const int Lc = p.L - 1;
    const ScLevel &L0 = p.lv[0];
    hipLaunchKernelGGL((sc_first<T, TV>), node_grid(L0), blk, 0, st, lv_of<T>(L0), A(0), D(0), vp,
                       V(0, L0.b), V(0, L0.x0), omega);
    FSI_LAUNCH_CHECK();
    for (int l = 0; l < Lc; ++l) {
        const ScLevel &F = p.lv[l], &C = p.lv[l + 1];
        hipLaunchKernelGGL((sc_sweep<T, T, 0>), sweep_grid(F), sblk, 0, st, lv_of<T>(F), A(l), D(l),
                           V(l, F.b), V(l, F.x0), V(l, F.x1), (T *)nullptr, omega);
        FSI_LAUNCH_CHECK();
        hipLaunchKernelGGL((sc_sweep<T, T, 1>), sweep_grid(F), sblk, 0, st, lv_of<T>(F), A(l), D(l),
                           V(l, F.b), V(l, F.x1), V(l, F.r), (T *)nullptr, omega);
        FSI_LAUNCH_CHECK();
        hipLaunchKernelGGL((sc_restrict<T>), node_grid(C), blk, 0, st, lv_of<T>(C), lv_of<T>(F), A(l + 1),
                           D(l + 1), V(l, F.r), V(l + 1, C.b), V(l + 1, C.x0), omega);
        FSI_LAUNCH_CHECK();
    }
    {
        const ScLevel &C = p.lv[Lc];
        const T *kinv = reinterpret_cast<const T *>(base + (sizeof(T) == 8 ? p.kinv64 : p.kinv32));
        hipLaunchKernelGGL((sc_coarse<T>), dim3((unsigned)C.N), dim3(64), 0, st, (int)C.N, kinv,
                           V(Lc, C.b), V(Lc, C.x1));
        FSI_LAUNCH_CHECK();
        if (Lc == 0) {
            hipLaunchKernelGGL((sc_finish<T, TZ>), node_grid(C), blk, 0, st, lv_of<T>(C), A(0), D(0),
                               V(0, C.b), V(0, C.x1), zp);
            FSI_LAUNCH_CHECK();
            return FSI_OK;
        }
    }
    for (int l = Lc - 1; l >= 0; --l) {
        const ScLevel &F = p.lv[l], &C = p.lv[l + 1];
        hipLaunchKernelGGL((sc_prolong<T>), node_grid(F), blk, 0, st, lv_of<T>(F), lv_of<T>(C), D(l),
                           V(l + 1, C.x1), V(l, F.x1));
        FSI_LAUNCH_CHECK();
        hipLaunchKernelGGL((sc_sweep<T, T, 0>), sweep_grid(F), sblk, 0, st, lv_of<T>(F), A(l), D(l),
                           V(l, F.b), V(l, F.x1), V(l, F.x0), (T *)nullptr, omega);
        FSI_LAUNCH_CHECK();
        if (l == 0)
            hipLaunchKernelGGL((sc_sweep<T, TZ, 2>), sweep_grid(F), sblk, 0, st, lv_of<T>(F), A(l), D(l),
                               V(l, F.b), V(l, F.x0), (T *)nullptr, zp, omega);
        else
            hipLaunchKernelGGL((sc_sweep<T, T, 0>), sweep_grid(F), sblk, 0, st, lv_of<T>(F), A(l), D(l),
                               V(l, F.b), V(l, F.x0), V(l, F.x1), (T *)nullptr, omega);
        FSI_LAUNCH_CHECK();
    }
    return FSI_OK;
}

template <typename T, typename TV, typename TZ>
int apply_t(const Geo &g, const ScPlan &p, int mode, int vel_steps, char *base, const TV *v, TZ *z,
            const JacobianCall *J, void *jws, hipStream_t st)
{
    static_assert(sizeof(T) == sizeof(TZ), "the preconditioned vector is in the compute precision");
    const int64_t N = g.N;
    int rc = vcycle<T, TV, TZ>(p, base, v + 3 * N, z + 3 * N, st);
    if (rc) return rc;
    const T *yt = nullptr;
    if (mode == 2) {
        // yt = velocity rows of J (0, z_p): the pressure-gradient block where the operator has
        // one, else the whole operator on z with its velocity part cleared (z_u is written
        // below without being read)
        T *y = reinterpret_cast<T *>(base + p.yt);
        if (J->block) {
            rc = J->block(2, z, y, jws, st);
        } else {
            FSI_HIP(hipMemsetAsync(z, 0, (size_t)3 * N * sizeof(TZ), st));
            rc = J->apply(z, y, jws, st);
        }
        if (rc) return rc;
        yt = y;
    }
    const T *finv = reinterpret_cast<const T *>(base + (sizeof(T) == 8 ? p.finv64 : p.finv32));
    if (vel_steps == 0) {
        hipLaunchKernelGGL((sc_vel_apply<T, TV, TZ>), dim3(blocks_for(N)), dim3(256), 0, st, N, finv, v, yt, z);
        FSI_LAUNCH_CHECK();
        return FSI_OK;
    }
    // minimal-residual steps on F = velocity rows of J [u; 0], preconditioned by the block inverses
    T *r = reinterpret_cast<T *>(base + p.mr_r);
    T *xin = reinterpret_cast<T *>(base + p.mr_x);
    T *q = reinterpret_cast<T *>(base + p.mr_q);
    double *part = reinterpret_cast<double *>(base + p.mr_part);
    double *alpha = part + 2 * MR_NB;
    TZ *zu = z;   // the velocity part of z accumulates the steps (TZ = T)
    const int64_t n3 = 3 * N;
    const unsigned ub = (unsigned)std::min<int64_t>(blocks_for(n3), 4096);
    hipLaunchKernelGGL((sc_vel_resid<T, TV>), dim3(ub), dim3(256), 0, st, n3, v, yt, r);
    FSI_LAUNCH_CHECK();
    // F xin = velocity rows of J (xin_u, 0): the velocity block where the operator has one, else
    // the whole operator on xin with a zero pressure part
    if (!J->block) FSI_HIP(hipMemsetAsync(xin + n3, 0, (size_t)N * sizeof(T), st));
    for (int it = 0; it < vel_steps; ++it) {
        hipLaunchKernelGGL((sc_vel_apply<T, T, T>), dim3(blocks_for(N)), dim3(256), 0, st, N, finv, r, (const T *)nullptr,
                           xin);
        FSI_LAUNCH_CHECK();
        rc = J->block ? J->block(1, xin, q, jws, st) : J->apply(xin, q, jws, st);
        if (rc) return rc;
        hipLaunchKernelGGL((sc_mr_dots<T>), dim3(MR_NB), dim3(256), 0, st, n3, q, r, part);
        FSI_LAUNCH_CHECK();
        hipLaunchKernelGGL(sc_mr_alpha, dim3(1), dim3(256), 0, st, MR_NB, part, alpha);
        FSI_LAUNCH_CHECK();
        hipLaunchKernelGGL((sc_mr_update<T>), dim3(ub), dim3(256), 0, st, n3, alpha, xin, q,
                           reinterpret_cast<T *>(zu), r, it == 0 ? 1 : 0);
        FSI_LAUNCH_CHECK();
    }
    return FSI_OK;
}

}  // namespace

int sc_plan(const Geo &g, ScPlan &p)
{
    std::memset(&p, 0, sizeof(p));
    int nc[3] = {g.p * g.n[0], g.p * g.n[1], g.p * g.n[2]};
    double l[3] = {g.h[0] / g.p, g.h[1] / g.p, g.h[2] / g.p};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    for (int L = 0;; ++L) {
        if (L >= SC_MAX_LEVELS) {
            set_error("too many multigrid levels");
            return FSI_ERR_ARG;
        }
        ScLevel &v = p.lv[L];
        v.N = 1;
        v.C = 1;
        for (int d = 0; d < 3; ++d) {
            v.nc[d] = nc[d];
            v.nn[d] = nc[d] + 1;
            v.l[d] = l[d];
            v.N *= v.nn[d];
            v.C *= v.nc[d];
        }
        const double vol = l[0] * l[1] * l[2];
        for (int pat = 0; pat < 8; ++pat) {
            double s = 0.0;
            for (int d = 0; d < 3; ++d) {
                double t = (((pat >> d) & 1) ? -1.0 : 1.0) / (l[d] * l[d]);
                for (int e = 0; e < 3; ++e)
                    if (e != d) t *= ((pat >> e) & 1) ? 1.0 / 6.0 : 1.0 / 3.0;
                s += t;
            }
            v.kc[pat] = vol * s;
        }
        v.a64 = take((size_t)v.C * sizeof(double));
        v.a32 = take((size_t)v.C * sizeof(float));
        v.dm = take((size_t)v.N);
        v.x0 = take((size_t)v.N * sizeof(double));
        v.x1 = take((size_t)v.N * sizeof(double));
        v.b = take((size_t)v.N * sizeof(double));
        v.r = take((size_t)v.N * sizeof(double));
        p.L = L + 1;
        const bool even = nc[0] % 2 == 0 && nc[1] % 2 == 0 && nc[2] % 2 == 0;
        if (!even || v.N <= SC_COARSE_MAX_NODES) break;
        for (int d = 0; d < 3; ++d) {
            nc[d] /= 2;
            l[d] *= 2.0;
        }
    }
    if (p.lv[0].N >= ((int64_t)1 << 31)) {
        set_error("the pressure lattice has %lld nodes; at most 2^31 - 1 are supported",
                  (long long)p.lv[0].N);
        return FSI_ERR_ARG;
    }
    const int64_t nco = p.lv[p.L - 1].N;
    if (nco > SC_DIRECT_MAX_NODES) {
        set_error("the pressure lattice (%d x %d x %d cells) cannot be coarsened to at most %lld nodes; "
                  "use cell counts with more factors of two",
                  p.lv[0].nc[0], p.lv[0].nc[1], p.lv[0].nc[2], (long long)SC_DIRECT_MAX_NODES);
        return FSI_ERR_ARG;
    }
    p.finv64 = take((size_t)9 * g.N * sizeof(double));
    p.finv32 = take((size_t)9 * g.N * sizeof(float));
    p.kinv64 = take((size_t)(nco * nco) * sizeof(double));
    p.kinv32 = take((size_t)(nco * nco) * sizeof(float));
    p.yt = take((size_t)4 * g.N * sizeof(double));
    p.mr_r = take((size_t)3 * g.N * sizeof(double));
    p.mr_x = take((size_t)4 * g.N * sizeof(double));
    p.mr_q = take((size_t)4 * g.N * sizeof(double));
    p.mr_part = take((size_t)(2 * MR_NB + 8) * sizeof(double));
    p.cnt = take(256);
    p.total = off;
    return FSI_OK;
}

int schur_setup(const Geo &g, const fsi_vms_params &prm, const double *a, const double *s,
                const uint32_t *mask, const double *gram, const int32_t *occ_index,
                const double *blocks, void *pc, hipStream_t st)
{
    ProfileScope prof("schur_setup", st);
    ScPlan p;
    int rc = sc_plan(g, p);
    if (rc) return rc;
    char *base = reinterpret_cast<char *>(pc);
    const ScLevel &L0 = p.lv[0];
    int32_t *cnt = reinterpret_cast<int32_t *>(base + p.cnt);
    FSI_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t), st));
    double *beta = reinterpret_cast<double *>(base + L0.x0);
    const double v8 = L0.l[0] * L0.l[1] * L0.l[2] / 8.0;
    if (g.p == 1)
        hipLaunchKernelGGL(sc_node_beta<1>, dim3(blocks_for(g.N)), dim3(256), 0, st, g, gram, occ_index,
                           prm.c_m, v8, beta);
    else
        hipLaunchKernelGGL(sc_node_beta<2>, dim3(blocks_for(g.N)), dim3(256), 0, st, g, gram, occ_index,
                           prm.c_m, v8, beta);
    FSI_LAUNCH_CHECK();
    const VmsConst<double> k = make_vms_const<double>(g, prm, s != nullptr);
    hipLaunchKernelGGL(sc_cell_alpha, dim3(blocks_for(L0.C)), dim3(256), 0, st, g, k, L0.nc[0], L0.nc[1],
                       L0.nc[2], a, s, beta, reinterpret_cast<double *>(base + L0.a64),
                       reinterpret_cast<float *>(base + L0.a32));
    FSI_LAUNCH_CHECK();
    hipLaunchKernelGGL(sc_dmask0, dim3(blocks_for(g.N)), dim3(256), 0, st, g, mask,
                       reinterpret_cast<uint8_t *>(base + L0.dm), cnt);
    FSI_LAUNCH_CHECK();
    for (int l = 1; l < p.L; ++l) {
        const ScLevel &F = p.lv[l - 1], &C = p.lv[l];
        hipLaunchKernelGGL(sc_coarsen_alpha, dim3(blocks_for(C.C)), dim3(256), 0, st, F.nc[0], F.nc[1], C.nc[0],
                           C.nc[1], C.nc[2], reinterpret_cast<const double *>(base + F.a64),
                           reinterpret_cast<double *>(base + C.a64), reinterpret_cast<float *>(base + C.a32));
        FSI_LAUNCH_CHECK();
        hipLaunchKernelGGL(sc_coarsen_mask, dim3(blocks_for(C.N)), dim3(256), 0, st, F.nn[0], F.nn[1], C.nn[0],
                           C.nn[1], C.nn[2], reinterpret_cast<const uint8_t *>(base + F.dm),
                           reinterpret_cast<uint8_t *>(base + C.dm));
        FSI_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(sc_vel_inverse, dim3(blocks_for(g.N)), dim3(256), 0, st, g.N, blocks,
                       reinterpret_cast<double *>(base + p.finv64), reinterpret_cast<float *>(base + p.finv32));
    FSI_LAUNCH_CHECK();
    // coarsest level: operator on the host, inverted by Cholesky
    const ScLevel &C = p.lv[p.L - 1];
    std::vector<double> ac((size_t)C.C);
    std::vector<uint8_t> dc((size_t)C.N);
    int32_t hcnt = 0;
    FSI_HIP(hipMemcpyAsync(&hcnt, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FSI_HIP(hipMemcpyAsync(ac.data(), base + C.a64, ac.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    FSI_HIP(hipMemcpyAsync(dc.data(), base + C.dm, dc.size(), hipMemcpyDeviceToHost, st));
    FSI_HIP(hipStreamSynchronize(st));
    if (hcnt == 0) {
        // no node fixes the pressure level (an enclosed flow): node 0 of every level does
        static const uint8_t one = 1;
        for (int l = 0; l < p.L; ++l)
            FSI_HIP(hipMemcpyAsync(base + p.lv[l].dm, &one, 1, hipMemcpyHostToDevice, st));
        dc[0] = 1;
    }
    std::vector<double> kinv;
    rc = coarse_inverse(C, ac, dc, kinv);
    if (rc) return rc;
    std::vector<float> kinv32(kinv.size());
    for (size_t i = 0; i < kinv.size(); ++i) kinv32[i] = (float)kinv[i];
    FSI_HIP(hipMemcpyAsync(base + p.kinv64, kinv.data(), kinv.size() * sizeof(double), hipMemcpyHostToDevice, st));
    FSI_HIP(hipMemcpyAsync(base + p.kinv32, kinv32.data(), kinv32.size() * sizeof(float), hipMemcpyHostToDevice, st));
    FSI_HIP(hipStreamSynchronize(st));
    return FSI_OK;
}

int schur_apply(const Geo &g, fsi_dtype inner, bool v_f64, int mode, int vel_steps, void *pc, const void *v,
                void *z, const JacobianCall *J, void *jws, hipStream_t st)
{
    ProfileScope prof("schur_apply", st);
    ScPlan p;
    int rc = sc_plan(g, p);
    if (rc) return rc;
    if (mode != 1 && mode != 2) {
        set_error("unknown Schur preconditioner mode %d", mode);
        return FSI_ERR_ARG;
    }
    if ((mode == 2 || vel_steps > 0) && J == nullptr) {
        set_error("the block-triangular form and the velocity steps need the Jacobian");
        return FSI_ERR_ARG;
    }
    if (vel_steps < 0 || vel_steps > 16) {
        set_error("velocity minimal-residual steps must be in [0, 16] (got %d)", vel_steps);
        return FSI_ERR_ARG;
    }
    char *base = reinterpret_cast<char *>(pc);
    if (inner == FSI_F64)
        return apply_t<double, double, double>(g, p, mode, vel_steps, base, (const double *)v, (double *)z, J, jws,
                                               st);
    if (v_f64)
        return apply_t<float, double, float>(g, p, mode, vel_steps, base, (const double *)v, (float *)z, J, jws, st);
    return apply_t<float, float, float>(g, p, mode, vel_steps, base, (const float *)v, (float *)z, J, jws, st);
}

}  // namespace fsi
