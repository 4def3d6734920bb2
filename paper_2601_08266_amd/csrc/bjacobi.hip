// Nodal 4x4 block-Jacobi preconditioner of the reduced system (section 2.4:
// block preconditioners assembled from sub-matrices of the 2x2 block system;
// the nodal (u,v,w,p) diagonal blocks are the simplest such choice).
//
//  bj_qp    one lane per (cell, quadrature point): advection, s (clamped), tau_m
//           and tau_c at the point -> a small per-point table, stored value- and
//           point-major ([5][nq][E]) so that lanes on consecutive cells read and write
//           consecutive entries.
//  bj_node  one lane per node: sums, over the (up to 8) cells holding the node and
//           their quadrature points, the node's own 4x4 entries of the element
//           matrix (same terms as the operator), adds the diagonal of the DLM block
//           (gram[o][A][A] kappa N_A^2 sums) of occupied neighbour cells, replaces
//           Dirichlet rows/columns by the identity, and inverts the block in FP64
//           (Gauss-Jordan with partial pivoting) when an inverse is asked for.  No
//           atomics in the sums: deterministic.
//  bj_apply z = P^{-1} v, one lane per node, blocks stored [16][N].
#include "bjacobi.hpp"
#include "profile.hpp"

namespace fsi {

namespace {

template <int P>
struct Rule;
template <>
struct Rule<1> {
    static constexpr int NQ = 2;
    __device__ static double pt(int q) { return q == 0 ? 0.21132486540518711775 : 0.78867513459481288225; }
    __device__ static double wt(int) { return 0.5; }
};
template <>
struct Rule<2> {
    static constexpr int NQ = 3;
    __device__ static double pt(int q)
    {
        return q == 0 ? 0.11270166537925831148 : (q == 1 ? 0.5 : 0.88729833462074168852);
    }
    __device__ static double wt(int q) { return q == 1 ? 0.44444444444444444444 : 0.27777777777777777778; }
};

template <int P>
__device__ __forceinline__ void basis1d(int a, double t, double &n, double &d, double &d2)
{
    if (P == 1) {
        n = a == 0 ? 1.0 - t : t;
        d = a == 0 ? -1.0 : 1.0;
        d2 = 0.0;
    } else {
        if (a == 0) {
            n = 2.0 * (t - 0.5) * (t - 1.0); d = 4.0 * t - 3.0; d2 = 4.0;
        } else if (a == 1) {
            n = -4.0 * t * (t - 1.0); d = -8.0 * t + 4.0; d2 = -8.0;
        } else {
            n = 2.0 * t * (t - 0.5); d = 4.0 * t - 1.0; d2 = 4.0;
        }
    }
}

// Block index -> position in the lattice: blocks are dealt to the 8 XCDs round-robin, and each
// XCD is given a contiguous range of positions, so the neighbouring rows and planes that one
// block's lanes and the next blocks share are read under the same L2.
__device__ __forceinline__ uint32_t xcd_range(uint32_t bid, uint32_t nb)
{
    const uint32_t q = nb >> 3, r = nb & 7u, xcd = bid & 7u, idx = bid >> 3;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// per-point table: a0 a1 a2 tau_m tau_c; entry f of point q of cell e at tab[(f NQ3 + q) E + e]
template <int P>
__global__ __launch_bounds__(256) void bj_qp(Geo g, VmsConst<double> k, const double *__restrict__ a,
                                             const double *__restrict__ s, double *__restrict__ tab)
{
    constexpr int Q = P + 1, NQ = Rule<P>::NQ, NQ3 = NQ * NQ * NQ;
    const int64_t id = (int64_t)xcd_range(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (id >= g.E * NQ3) return;
    const int q = (int)(id / g.E);
    const int64_t e = id - (int64_t)q * g.E;
    const int64_t row = e / g.n[0];   // one 64-bit division, the rest in 32 bits
    const int cx = (int)(e - row * g.n[0]), cy = (int)((uint32_t)row % (uint32_t)g.n[1]),
              cz = (int)((uint32_t)row / (uint32_t)g.n[1]);
    const double t[3] = {Rule<P>::pt(q % NQ), Rule<P>::pt((q / NQ) % NQ), Rule<P>::pt(q / (NQ * NQ))};
    double A[3] = {0.0, 0.0, 0.0}, S = 0.0, smin = 0.0;
    bool first = true;
    for (int c = 0; c < Q; ++c)
        for (int b = 0; b < Q; ++b)
            for (int aa = 0; aa < Q; ++aa) {
                double nx, ny, nz, d, d2;
                basis1d<P>(aa, t[0], nx, d, d2);
                basis1d<P>(b, t[1], ny, d, d2);
                basis1d<P>(c, t[2], nz, d, d2);
                const double w = nx * ny * nz;
                const int64_t node = (int64_t)(P * cx + aa) +
                                     (int64_t)g.nn[0] * ((P * cy + b) + (int64_t)g.nn[1] * (P * cz + c));
                for (int dd = 0; dd < 3; ++dd) A[dd] += w * a[dd * g.N + node];
                const double sv = s ? s[node] : 1.0;
                S += w * sv;
                smin = first ? sv : (sv < smin ? sv : smin);
                first = false;
            }
    if (s == nullptr) S = 1.0;
    else S = S < smin ? smin : S;
    const double tb = S * (k.K1 + A[0] * A[0] * k.ih2[0] + A[1] * A[1] * k.ih2[1] + A[2] * A[2] * k.ih2[2]);
    const double sq = sqrt(tb);
    const int64_t fs = (int64_t)NQ3 * g.E;   // stride between the table's values
    tab[id] = A[0];
    tab[id + fs] = A[1];
    tab[id + 2 * fs] = A[2];
    tab[id + 3 * fs] = 1.0 / sq;
    tab[id + 4 * fs] = sq * k.inv_trG;
}

// 4x4 inverse, Gauss-Jordan with partial pivoting; returns false if singular
__device__ __forceinline__ bool inv4(double M[4][4], double R[4][4])
{
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) R[i][j] = (i == j) ? 1.0 : 0.0;
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        double best = fabs(M[c][c]);
        for (int r = c + 1; r < 4; ++r)
            if (fabs(M[r][c]) > best) {
                best = fabs(M[r][c]);
                piv = r;
            }
        if (!(best > 0.0)) return false;
        if (piv != c)
            for (int j = 0; j < 4; ++j) {
                double t = M[c][j]; M[c][j] = M[piv][j]; M[piv][j] = t;
                t = R[c][j]; R[c][j] = R[piv][j]; R[piv][j] = t;
            }
        const double inv = 1.0 / M[c][c];
        for (int j = 0; j < 4; ++j) {
            M[c][j] *= inv;
            R[c][j] *= inv;
        }
        for (int r = 0; r < 4; ++r)
            if (r != c) {
                const double f = M[r][c];
                for (int j = 0; j < 4; ++j) {
                    M[r][j] -= f * M[c][j];
                    R[r][j] -= f * R[c][j];
                }
            }
    }
    return true;
}

// One Gauss point's contribution to a node's 4x4 block on a trilinear cell (the general
// formulas below with what vanishes for trilinear shape functions taken out: no second
// derivative along a single axis, so the Laplacian of the shape function is zero and its
// Hessian is the symmetric off-diagonal mixed derivatives; the velocity-velocity part is then
// symmetric off the diagonal).  la: the node's corner in the cell, q: the point.
__device__ __forceinline__ void node_q1_point(const VmsConst<double> &k, const double *__restrict__ tab,
                                              int64_t E, int64_t cell, int q, const int la[3], double Bk[4][4])
{
    double n1[3], d1[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double t = Rule<1>::pt((q >> d) & 1);
        n1[d] = la[d] == 0 ? 1.0 - t : t;
        d1[d] = (la[d] == 0 ? -1.0 : 1.0) * k.ih[d];   // physical derivative of the 1D factor
    }
    const double W = k.detJ * 0.125;
    const double N = n1[0] * n1[1] * n1[2];
    const double dN[3] = {d1[0] * n1[1] * n1[2], n1[0] * d1[1] * n1[2], n1[0] * n1[1] * d1[2]};
    const double H01 = d1[0] * d1[1] * n1[2], H02 = d1[0] * d1[2] * n1[1], H12 = d1[1] * d1[2] * n1[0];
    const int64_t fs = 8 * E;
    const double *tq = tab + (int64_t)q * E + cell;
    const double A0 = tq[0], A1 = tq[fs], A2 = tq[2 * fs];
    const double tau_m = tq[3 * fs], tau_c = tq[4 * fs];
    const double nu = k.nu, c_m = k.c_m;
    const double adN = A0 * dN[0] + A1 * dN[1] + A2 * dN[2];
    const double gg = dN[0] * dN[0] + dN[1] * dN[1] + dN[2] * dN[2];
    const double nt = nu + tau_c, tma = tau_m * adN, rr = c_m * N + adN;
    const double D = c_m * N * N + N * adN + nu * gg + tma * rr;
#pragma unroll
    for (int i = 0; i < 3; ++i) Bk[i][i] += W * (nt * dN[i] * dN[i] + D);
    // off the diagonal: nu and tau_c grad-grad terms, the SUPG-weighted strong viscous term
    const double vs = k.visc_strong ? nu : 0.0;
    const double o01 = W * (nt * dN[0] * dN[1] - tma * vs * H01);
    const double o02 = W * (nt * dN[0] * dN[2] - tma * vs * H02);
    const double o12 = W * (nt * dN[1] * dN[2] - tma * vs * H12);
    Bk[0][1] += o01; Bk[1][0] += o01;
    Bk[0][2] += o02; Bk[2][0] += o02;
    Bk[1][2] += o12; Bk[2][1] += o12;
    // pressure column (Galerkin -div w p, SUPG) and row (continuity, PSPG)
    const double hv[3] = {dN[1] * H01 + dN[2] * H02, dN[0] * H01 + dN[2] * H12, dN[0] * H02 + dN[1] * H12};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        Bk[i][3] += W * (dN[i] * (tma - N));
        Bk[3][i] += W * (N * dN[i] + tau_m * (dN[i] * rr - vs * hv[i]));
    }
    Bk[3][3] += W * tau_m * gg;
}

template <int P>
__global__ __launch_bounds__(256) void bj_node(Geo g, VmsConst<double> k, const double *__restrict__ tab,
                                               const uint32_t *__restrict__ mask,
                                               const double *__restrict__ gram,
                                               const int32_t *__restrict__ occ_index,
                                               double *__restrict__ raw, double *__restrict__ pinv64,
                                               float *__restrict__ pinv32, int32_t *__restrict__ nsing)
{
    constexpr int Q = P + 1, NQ = Rule<P>::NQ, NQ3 = NQ * NQ * NQ, NEN = Q * Q * Q;
    const int64_t node = (int64_t)xcd_range(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (node >= g.N) return;
    const int gv[3] = {(int)(node % g.nn[0]), (int)((node / g.nn[0]) % g.nn[1]),
                       (int)(node / ((int64_t)g.nn[0] * g.nn[1]))};
    int cs[3][2], as[3][2], nc[3];
    for (int d = 0; d < 3; ++d) {
        nc[d] = 0;
        if (gv[d] >= P && gv[d] % P == 0) { cs[d][nc[d]] = gv[d] / P - 1; as[d][nc[d]++] = P; }
        const int c = gv[d] / P;
        if (c < g.n[d]) { cs[d][nc[d]] = c; as[d][nc[d]++] = gv[d] - P * c; }
    }
    const double ih[3] = {k.ih[0], k.ih[1], k.ih[2]};
    const double nu = k.nu, c_m = k.c_m;
    double Bk[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) Bk[i][j] = 0.0;
    double dlm = 0.0;
    for (int iz = 0; iz < nc[2]; ++iz)
        for (int iy = 0; iy < nc[1]; ++iy)
            for (int ix = 0; ix < nc[0]; ++ix) {
                const int64_t cell = cs[0][ix] + (int64_t)g.n[0] * (cs[1][iy] + (int64_t)g.n[1] * cs[2][iz]);
                const int la[3] = {as[0][ix], as[1][iy], as[2][iz]};
                // points not unrolled: unrolled, the trilinear case needs 262 registers (1 wave)
#pragma unroll 1
                for (int q = 0; q < NQ3; ++q) {
                    if constexpr (P == 1) {
                        node_q1_point(k, tab, g.E, cell, q, la, Bk);
                        continue;
                    }
                    const int qi[3] = {q % NQ, (q / NQ) % NQ, q / (NQ * NQ)};
                    double n1[3], d1[3], dd1[3];
                    double W = k.detJ;
                    for (int d = 0; d < 3; ++d) {
                        basis1d<P>(la[d], Rule<P>::pt(qi[d]), n1[d], d1[d], dd1[d]);
                        W *= Rule<P>::wt(qi[d]);
                    }
                    const double N = n1[0] * n1[1] * n1[2];
                    double dN[3], H[3][3];
                    dN[0] = d1[0] * n1[1] * n1[2] * ih[0];
                    dN[1] = n1[0] * d1[1] * n1[2] * ih[1];
                    dN[2] = n1[0] * n1[1] * d1[2] * ih[2];
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) {
                            double v = 1.0;
                            for (int d = 0; d < 3; ++d) {
                                const int ord = (d == i) + (d == j);
                                v *= ord == 0 ? n1[d] : (ord == 1 ? d1[d] * ih[d] : dd1[d] * ih[d] * ih[d]);
                            }
                            H[i][j] = v;
                        }
                    const int64_t fs = (int64_t)NQ3 * g.E;
                    const double *tq = tab + (int64_t)q * g.E + cell;
                    const double A[3] = {tq[0], tq[fs], tq[2 * fs]};
                    const double tau_m = tq[3 * fs], tau_c = tq[4 * fs];
                    const double adN = A[0] * dN[0] + A[1] * dN[1] + A[2] * dN[2];
                    const double lap = H[0][0] + H[1][1] + H[2][2];
                    const double gg = dN[0] * dN[0] + dN[1] * dN[1] + dN[2] * dN[2];
                    for (int i = 0; i < 3; ++i) {
                        for (int j = 0; j < 3; ++j) {
                            double v = nu * dN[j] * dN[i] + tau_c * dN[i] * dN[j];
                            double r = 0.0;
                            if (i == j) {
                                v += c_m * N * N + N * adN + nu * gg;
                                r = c_m * N + adN;
                            }
                            if (k.visc_strong) r -= nu * (((i == j) ? lap : 0.0) + H[i][j]);
                            v += tau_m * adN * r;
                            Bk[i][j] += W * v;
                        }
                        Bk[i][3] += W * (-dN[i] * N + tau_m * adN * dN[i]);
                        double r = dN[i] * (c_m * N + adN);
                        if (k.visc_strong) {
                            double t2 = dN[i] * lap;
                            for (int m = 0; m < 3; ++m) t2 += dN[m] * H[m][i];
                            r -= nu * t2;
                        }
                        Bk[3][i] += W * (N * dN[i] + tau_m * r);
                    }
                    Bk[3][3] += W * tau_m * gg;
                }
                if (gram != nullptr) {
                    const int32_t ko = occ_index[cell];
                    if (ko >= 0) {
                        const int A = la[0] + Q * (la[1] + Q * la[2]);
                        dlm += gram[((int64_t)ko * NEN + A) * NEN + A];
                    }
                }
            }
    for (int i = 0; i < 3; ++i) Bk[i][i] += dlm;
    for (int f = 0; f < 3; ++f)
        if (mask_bit(mask, f * g.N + node))
            for (int m = 0; m < 4; ++m) {
                Bk[f][m] = (m == f) ? 1.0 : 0.0;
                Bk[m][f] = (m == f) ? 1.0 : 0.0;
            }
    if (raw != nullptr)
        for (int i = 0; i < 16; ++i) raw[(int64_t)i * g.N + node] = Bk[i / 4][i % 4];
    if (pinv64 == nullptr && pinv32 == nullptr && nsing == nullptr) return;   // the blocks only
    double R[4][4];
    if (!inv4(Bk, R)) {
        if (nsing != nullptr) atomicAdd(nsing, 1);
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) R[i][j] = (i == j) ? 1.0 : 0.0;
    }
    for (int i = 0; i < 16; ++i) {
        if (pinv64) pinv64[(int64_t)i * g.N + node] = R[i / 4][i % 4];
        if (pinv32) pinv32[(int64_t)i * g.N + node] = (float)R[i / 4][i % 4];
    }
}

template <typename T, typename TV, typename TZ>
__global__ __launch_bounds__(256) void bj_apply(int64_t N, const T *__restrict__ pinv,
                                                const TV *__restrict__ v, TZ *__restrict__ z)
{
    const int64_t node = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (node >= N) return;
    T vin[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) vin[f] = (T)v[f * N + node];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc += pinv[(int64_t)(i * 4 + j) * N + node] * vin[j];
        z[i * N + node] = (TZ)acc;
    }
}

}  // namespace

size_t bjacobi_workspace_bytes(const Geo &g)
{
    const int nq = g.p == 1 ? 8 : 27;
    return align_up((size_t)g.E * nq * 5 * sizeof(double)) + align_up(sizeof(int32_t) * 4);
}

int launch_bjacobi_setup(const Geo &g, const fsi_vms_params &prm, const double *a, const double *s,
                         const uint32_t *mask, const double *gram, const int32_t *occ_index,
                         double *raw, double *pinv64, float *pinv32, int64_t *n_singular,
                         void *ws, hipStream_t st)
{
    ProfileScope prof("bjacobi_setup", st);
    const VmsConst<double> k = make_vms_const<double>(g, prm, s != nullptr);
    const int nq = g.p == 1 ? 8 : 27;
    double *tab = reinterpret_cast<double *>(ws);
    int32_t *cnt = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(ws) +
                                               align_up((size_t)g.E * nq * 5 * sizeof(double)));
    // the singular-block count is kept only when it is asked for (or an inverse is)
    if (n_singular != nullptr || pinv64 != nullptr || pinv32 != nullptr)
        FSI_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t), st));
    else
        cnt = nullptr;
    const unsigned b1 = (unsigned)((g.E * nq + 255) / 256);
    const unsigned b2 = (unsigned)((g.N + 255) / 256);
    if (g.p == 1) {
        hipLaunchKernelGGL(bj_qp<1>, dim3(b1), dim3(256), 0, st, g, k, a, s, tab);
        FSI_LAUNCH_CHECK();
        hipLaunchKernelGGL(bj_node<1>, dim3(b2), dim3(256), 0, st, g, k, tab, mask, gram, occ_index, raw,
                           pinv64, pinv32, cnt);
    } else {
        hipLaunchKernelGGL(bj_qp<2>, dim3(b1), dim3(256), 0, st, g, k, a, s, tab);
        FSI_LAUNCH_CHECK();
        hipLaunchKernelGGL(bj_node<2>, dim3(b2), dim3(256), 0, st, g, k, tab, mask, gram, occ_index, raw,
                           pinv64, pinv32, cnt);
    }
    FSI_LAUNCH_CHECK();
    if (n_singular) {
        int32_t h = 0;
        FSI_HIP(hipMemcpyAsync(&h, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        FSI_HIP(hipStreamSynchronize(st));
        *n_singular = h;
    }
    return FSI_OK;
}

int launch_bjacobi_apply(int64_t N, fsi_dtype dt, const void *pinv, const void *v, void *z,
                         hipStream_t st)
{
    const unsigned b = (unsigned)((N + 255) / 256);
    if (dt == FSI_F64)
        hipLaunchKernelGGL((bj_apply<double, double, double>), dim3(b), dim3(256), 0, st, N,
                           (const double *)pinv, (const double *)v, (double *)z);
    else
        hipLaunchKernelGGL((bj_apply<float, float, float>), dim3(b), dim3(256), 0, st, N,
                           (const float *)pinv, (const float *)v, (float *)z);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int launch_bjacobi_apply_f64_to_f32(int64_t N, const float *pinv32, const double *v, float *z,
                                    hipStream_t st)
{
    const unsigned b = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL((bj_apply<float, double, float>), dim3(b), dim3(256), 0, st, N, pinv32, v, z);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

}  // namespace fsi
