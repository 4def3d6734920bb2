// Matrix-free Q1-Q1 Oseen-VMS operator on gfx950 (section 2.1: Galerkin weak
// form + residual-based SUPG/PSPG/LSIC with the paper's tau_m, tau_c, G).
//
// Design
//  * One workgroup = a brick of 8x8x4 cells, one cell per lane (4 waves).
//  * Per cell, each nodal field is turned into the 8 coefficients of its
//    trilinear monomial expansion c_m xi^a eta^b zeta^c (three rounds of
//    differences); values and derivatives at the 2x2x2 Gauss points are
//    then short polynomials in compile-time constants.
//  * The test side accumulates the same 8 monomial moments per output field
//    and maps them back to the 8 nodes with the transposed difference rounds.
//  * Element -> node accumulation inside the brick goes through LDS in 8
//    ordered passes (one per cell corner: no two lanes hit the same node in a
//    pass), so the result is deterministic without atomics.  Brick-face
//    nodes are completed by a second, node-parallel gather kernel that sums
//    the partials of the (up to 8) bricks holding each node in a fixed order,
//    adds the DLM corner sums of occupied neighbour cells if requested, and
//    applies the Dirichlet rows.
#include "kernels.hpp"
#include "profile.hpp"

namespace fsi {

namespace {

// 2-point Gauss-Legendre on [0,1]
constexpr double GQ0 = 0.21132486540518711775;   // 1/2 - 1/(2 sqrt 3)
constexpr double GQ1 = 0.78867513459481288225;   // 1/2 + 1/(2 sqrt 3)

// nodal values (index a + 2b + 4c) -> monomial coefficients (same indexing, xi^a eta^b zeta^c)
template <typename T>
__device__ __forceinline__ void to_monomial(T v[8])
{
    v[1] -= v[0]; v[3] -= v[2]; v[5] -= v[4]; v[7] -= v[6];
    v[2] -= v[0]; v[3] -= v[1]; v[6] -= v[4]; v[7] -= v[5];
    v[4] -= v[0]; v[5] -= v[1]; v[6] -= v[2]; v[7] -= v[3];
}

// transpose of to_monomial: monomial moments -> nodal values
template <typename T>
__device__ __forceinline__ void from_moments(T v[8])
{
    v[0] -= v[4]; v[1] -= v[5]; v[2] -= v[6]; v[3] -= v[7];
    v[0] -= v[2]; v[1] -= v[3]; v[4] -= v[6]; v[5] -= v[7];
    v[0] -= v[1]; v[2] -= v[3]; v[4] -= v[5]; v[6] -= v[7];
}

// inverse of from_moments: a nodal vector -> the moments that from_moments maps back onto it
template <typename T>
__device__ __forceinline__ void to_moments(T v[8])
{
    v[0] += v[1]; v[2] += v[3]; v[4] += v[5]; v[6] += v[7];
    v[0] += v[2]; v[1] += v[3]; v[4] += v[6]; v[5] += v[7];
    v[0] += v[4]; v[1] += v[5]; v[2] += v[6]; v[3] += v[7];
}

template <typename T>
struct QP {
    T x, y, z, xy, xz, yz, xyz;
};

template <typename T>
__device__ __forceinline__ T mval(const T c[8], const QP<T> &q)
{
    return c[0] + c[1] * q.x + c[2] * q.y + c[3] * q.xy + c[4] * q.z + c[5] * q.xz + c[6] * q.yz +
           c[7] * q.xyz;
}
template <typename T>
__device__ __forceinline__ T mdx(const T c[8], const QP<T> &q)
{
    return c[1] + c[3] * q.y + c[5] * q.z + c[7] * q.yz;
}
template <typename T>
__device__ __forceinline__ T mdy(const T c[8], const QP<T> &q)
{
    return c[2] + c[3] * q.x + c[6] * q.z + c[7] * q.xz;
}
template <typename T>
__device__ __forceinline__ T mdz(const T c[8], const QP<T> &q)
{
    return c[4] + c[5] * q.x + c[6] * q.y + c[7] * q.xy;
}

// accumulate monomial moments of the test side: F0 * phi_m + grad_ref(phi_m) . G
template <typename T>
__device__ __forceinline__ void moments(T m[8], T F0, T G0, T G1, T G2, const QP<T> &q)
{
    m[0] += F0;
    m[1] += F0 * q.x + G0;
    m[2] += F0 * q.y + G1;
    m[3] += F0 * q.xy + G0 * q.y + G1 * q.x;
    m[4] += F0 * q.z + G2;
    m[5] += F0 * q.xz + G0 * q.z + G2 * q.x;
    m[6] += F0 * q.yz + G1 * q.z + G2 * q.y;
    m[7] += F0 * q.xyz + G0 * q.yz + G1 * q.xz + G2 * q.xy;
}

// Full element computation for one Q1 cell: in[f][A] nodal x (masked), a, s; out[f][A].
// If dlm != nullptr, the cell's 8x8 block of B^T diag(kappa) B is applied to the
// velocity and added to the momentum outputs.
// RESID = true: nonlinear residual of a time step instead of the linear apply: the
// advection field is the velocity itself (a = u) and ca holds the nodal source
// f = c_m u_old + body force, whose Galerkin/SUPG/PSPG weighting is subtracted.
template <typename T, bool RESID>
__device__ __forceinline__ void q1_cell(const VmsConst<T> &k, T cu[4][8], T ca[3][8], T cs[8],
                                        T smin, const T *__restrict__ dlm, T out[4][8])
{
    T mom[4][8];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int i = 0; i < 8; ++i) mom[f][i] = T(0);
    if (dlm != nullptr) {
        // DLM block on the nodal (Dirichlet-masked) velocity, carried in moment form
#pragma unroll
        for (int A = 0; A < 8; ++A) {
            T r0 = T(0), r1 = T(0), r2 = T(0);
#pragma unroll
            for (int C = 0; C < 8; ++C) {
                const T gAC = dlm[A * 8 + C];
                r0 += gAC * cu[0][C];
                r1 += gAC * cu[1][C];
                r2 += gAC * cu[2][C];
            }
            mom[0][A] = r0;
            mom[1][A] = r1;
            mom[2][A] = r2;
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) to_moments(mom[f]);
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) to_monomial(cu[f]);
#pragma unroll
    for (int d = 0; d < 3; ++d) to_monomial(ca[d]);
    if (k.has_s) to_monomial(cs);

    const T W = k.detJ * T(0.125);
    const T Wh0 = W * k.ih[0], Wh1 = W * k.ih[1], Wh2 = W * k.ih[2];
    const T h01 = k.ih[0] * k.ih[1], h02 = k.ih[0] * k.ih[2], h12 = k.ih[1] * k.ih[2];

#pragma unroll
    for (int qi = 0; qi < 8; ++qi) {
        QP<T> q;
        q.x = (qi & 1) ? T(GQ1) : T(GQ0);
        q.y = (qi & 2) ? T(GQ1) : T(GQ0);
        q.z = (qi & 4) ? T(GQ1) : T(GQ0);
        q.xy = q.x * q.y;
        q.xz = q.x * q.z;
        q.yz = q.y * q.z;
        q.xyz = q.xy * q.z;

        T U[3], dU[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            U[i] = mval(cu[i], q);
            dU[i][0] = mdx(cu[i], q) * k.ih[0];
            dU[i][1] = mdy(cu[i], q) * k.ih[1];
            dU[i][2] = mdz(cu[i], q) * k.ih[2];
        }
        const T P = mval(cu[3], q);
        const T dP0 = mdx(cu[3], q) * k.ih[0];
        const T dP1 = mdy(cu[3], q) * k.ih[1];
        const T dP2 = mdz(cu[3], q) * k.ih[2];
        T A0, A1, A2, Fs[3] = {T(0), T(0), T(0)};
        if constexpr (RESID) {
            A0 = U[0];
            A1 = U[1];
            A2 = U[2];
            Fs[0] = mval(ca[0], q);
            Fs[1] = mval(ca[1], q);
            Fs[2] = mval(ca[2], q);
        } else {
            A0 = mval(ca[0], q);
            A1 = mval(ca[1], q);
            A2 = mval(ca[2], q);
        }
        T S = T(1);
        if (k.has_s) {
            S = mval(cs, q);
            S = S < smin ? smin : S;
        }
        // tau_m = (s (C_T/dt^2 + a.Ga + C_I nu^2 G:G))^{-1/2},  tau_c = (tau_m tr G)^{-1}
        const T tb = S * (k.K1 + A0 * A0 * k.ih2[0] + A1 * A1 * k.ih2[1] + A2 * A2 * k.ih2[2]);
        const T sq = sqrt(tb);
        const T tau_m = T(1) / sq;
        const T tau_c = sq * k.inv_trG;

        const T div = dU[0][0] + dU[1][1] + dU[2][2];
        // grad(div u) for trilinear fields on Cartesian cells (pure second derivatives vanish)
        T gd[3] = {T(0), T(0), T(0)};
        if (k.visc_strong) {
            const T u1xy = (cu[1][3] + cu[1][7] * q.z) * h01;
            const T u2xz = (cu[2][5] + cu[2][7] * q.y) * h02;
            const T u0xy = (cu[0][3] + cu[0][7] * q.z) * h01;
            const T u2yz = (cu[2][6] + cu[2][7] * q.x) * h12;
            const T u0xz = (cu[0][5] + cu[0][7] * q.y) * h02;
            const T u1yz = (cu[1][6] + cu[1][7] * q.x) * h12;
            gd[0] = u1xy + u2xz;
            gd[1] = u0xy + u2yz;
            gd[2] = u0xz + u1yz;
        }
        const T dP[3] = {dP0, dP1, dP2};
        const T Aq[3] = {A0, A1, A2};
        T tr[3];
        T F0[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            T g = k.c_m * U[i] + (A0 * dU[i][0] + A1 * dU[i][1] + A2 * dU[i][2]);
            if constexpr (RESID) g -= Fs[i];
            F0[i] = g;
            const T r = g + dP[i] - k.nu * gd[i];
            tr[i] = tau_m * r;
        }
        const T diag = tau_c * div - P;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            T G[3];
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) {
                T fl = k.nu * (dU[i][kk] + dU[kk][i]) + Aq[kk] * tr[i];
                if (kk == i) fl += diag;
                G[kk] = fl;
            }
            moments(mom[i], W * F0[i], Wh0 * G[0], Wh1 * G[1], Wh2 * G[2], q);
        }
        moments(mom[3], W * div, Wh0 * tr[0], Wh1 * tr[1], Wh2 * tr[2], q);
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        from_moments(mom[f]);
#pragma unroll
        for (int i = 0; i < 8; ++i) out[f][i] = mom[f][i];
    }
}

template <typename T, bool RESID>
__global__ __launch_bounds__(256) void vms_q1_cells(Geo g, VmsConst<T> k, const T *__restrict__ x,
                                                    const T *__restrict__ a,
                                                    const T *__restrict__ s,
                                                    const uint32_t *__restrict__ mask,
                                                    const T *__restrict__ gram,
                                                    const int32_t *__restrict__ occ_index,
                                                    T *__restrict__ part, int nbx, int nby)
{
    __shared__ T acc[4 * Q1_NL];
    const int t = threadIdx.x;
    const int64_t bid = blockIdx.x;
    const int bx = (int)(bid % nbx), by = (int)((bid / nbx) % nby), bz = (int)(bid / ((int64_t)nbx * nby));
    const int tx = t & 7, ty = (t >> 3) & 7, tz = t >> 6;
    const int cx = bx * Q1_BX + tx, cy = by * Q1_BY + ty, cz = bz * Q1_BZ + tz;
    const bool valid = cx < g.n[0] && cy < g.n[1] && cz < g.n[2];
    for (int i = t; i < 4 * Q1_NL; i += 256) acc[i] = T(0);

    T out[4][8];
    if (valid) {
        T cu[4][8], ca[3][8], cs[8];
        T smin = T(1);
        const int64_t N = g.N;
#pragma unroll
        for (int A = 0; A < 8; ++A) {
            const int64_t node = (int64_t)(cx + (A & 1)) +
                                 (int64_t)g.nn[0] * ((cy + ((A >> 1) & 1)) + (int64_t)g.nn[1] * (cz + (A >> 2)));
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                T v = x[f * N + node];
                if (!RESID && mask_bit(mask, f * N + node)) v = T(0);
                cu[f][A] = v;
                ca[f][A] = a[f * N + node];
            }
            cu[3][A] = x[3 * N + node];
            cs[A] = k.has_s ? s[node] : T(1);
        }
        if (k.has_s) {
            smin = cs[0];
#pragma unroll
            for (int A = 1; A < 8; ++A) smin = cs[A] < smin ? cs[A] : smin;
        }
        const T *dlm = nullptr;
        if (gram != nullptr) {
            const int32_t ko = occ_index[cx + (int64_t)g.n[0] * (cy + (int64_t)g.n[1] * cz)];
            if (ko >= 0) dlm = gram + (int64_t)ko * 64;
        }
        q1_cell<T, RESID>(k, cu, ca, cs, smin, dlm, out);
    }
    __syncthreads();
#pragma unroll
    for (int A = 0; A < 8; ++A) {
        if (valid) {
            const int l = (tx + (A & 1)) + (Q1_BX + 1) * ((ty + ((A >> 1) & 1)) + (Q1_BY + 1) * (tz + (A >> 2)));
#pragma unroll
            for (int f = 0; f < 4; ++f) acc[f * Q1_NL + l] += out[f][A];
        }
        __syncthreads();
    }
    for (int l = t; l < Q1_NL; l += 256) {
        const int lx = l % (Q1_BX + 1), ly = (l / (Q1_BX + 1)) % (Q1_BY + 1), lz = l / ((Q1_BX + 1) * (Q1_BY + 1));
        const int gx = bx * Q1_BX + lx, gy = by * Q1_BY + ly, gz = bz * Q1_BZ + lz;
        if (gx < g.nn[0] && gy < g.nn[1] && gz < g.nn[2]) {
#pragma unroll
            for (int f = 0; f < 4; ++f) part[(bid * 4 + f) * Q1_NL + l] = acc[f * Q1_NL + l];
        }
    }
}

}  // namespace

// Node gather shared by all orders: sums brick partials (bricks of BXxBYxBZ cells, order P)
// and, optionally, DLM corner sums of occupied neighbour cells; then Dirichlet rows.
template <typename T, int P, int BX, int BY, int BZ>
__global__ __launch_bounds__(256) void vms_gather(Geo g, const T *__restrict__ part, int nbx,
                                                  int nby, int nbz, const T *__restrict__ x,
                                                  const uint32_t *__restrict__ mask,
                                                  T *__restrict__ y, GatherOpts<T> o)
{
    const T *__restrict__ csum = o.csum;
    const int32_t *__restrict__ occ_index = o.occ_index;
    constexpr int LX = P * BX + 1, LY = P * BY + 1, LZ = P * BZ + 1, NL = LX * LY * LZ;
    constexpr int NEN = (P + 1) * (P + 1) * (P + 1);
    const int64_t node = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (node >= g.N) return;
    const int gx = (int)(node % g.nn[0]);
    const int gy = (int)((node / g.nn[0]) % g.nn[1]);
    const int gz = (int)(node / ((int64_t)g.nn[0] * g.nn[1]));
    // bricks holding the node along each axis (lower brick first)
    int bxs[2], lxs[2], nxb = 0;
    int bys[2], lys[2], nyb = 0;
    int bzs[2], lzs[2], nzb = 0;
    {
        const int sx = P * BX, sy = P * BY, sz = P * BZ;
        int b = gx / sx, l = gx % sx;
        if (l == 0 && b > 0) { bxs[nxb] = b - 1; lxs[nxb++] = sx; }
        if (b < nbx) { bxs[nxb] = b; lxs[nxb++] = l; }
        b = gy / sy; l = gy % sy;
        if (l == 0 && b > 0) { bys[nyb] = b - 1; lys[nyb++] = sy; }
        if (b < nby) { bys[nyb] = b; lys[nyb++] = l; }
        b = gz / sz; l = gz % sz;
        if (l == 0 && b > 0) { bzs[nzb] = b - 1; lzs[nzb++] = sz; }
        if (b < nbz) { bzs[nzb] = b; lzs[nzb++] = l; }
    }
    T acc[4] = {T(0), T(0), T(0), T(0)};
    for (int iz = 0; iz < nzb; ++iz)
        for (int iy = 0; iy < nyb; ++iy)
            for (int ix = 0; ix < nxb; ++ix) {
                const int64_t bid = bxs[ix] + (int64_t)nbx * (bys[iy] + (int64_t)nby * bzs[iz]);
                const int l = lxs[ix] + LX * (lys[iy] + LY * lzs[iz]);
#pragma unroll
                for (int f = 0; f < 4; ++f) acc[f] += part[(bid * 4 + f) * NL + l];
            }
    if (csum != nullptr) {
        // cells containing the node along each axis: c with P c <= g <= P c + P
        int cxs[2], axs[2], ncx = 0, cys[2], ays[2], ncy = 0, czs[2], azs[2], ncz = 0;
        {
            if (gx >= P && gx % P == 0) { cxs[ncx] = gx / P - 1; axs[ncx++] = P; }
            int c = gx / P;
            if (c < g.n[0]) { cxs[ncx] = c; axs[ncx++] = gx - P * c; }
            if (gy >= P && gy % P == 0) { cys[ncy] = gy / P - 1; ays[ncy++] = P; }
            c = gy / P;
            if (c < g.n[1]) { cys[ncy] = c; ays[ncy++] = gy - P * c; }
            if (gz >= P && gz % P == 0) { czs[ncz] = gz / P - 1; azs[ncz++] = P; }
            c = gz / P;
            if (c < g.n[2]) { czs[ncz] = c; azs[ncz++] = gz - P * c; }
        }
        for (int iz = 0; iz < ncz; ++iz)
            for (int iy = 0; iy < ncy; ++iy)
                for (int ix = 0; ix < ncx; ++ix) {
                    const int64_t cell = cxs[ix] + (int64_t)g.n[0] * (cys[iy] + (int64_t)g.n[1] * czs[iz]);
                    const int32_t ko = occ_index[cell];
                    if (ko >= 0) {
                        const int corner = axs[ix] + (P + 1) * (ays[iy] + (P + 1) * azs[iz]);
#pragma unroll
                        for (int f = 0; f < 3; ++f) acc[f] += csum[((int64_t)ko * NEN + corner) * 3 + f];
                    }
                }
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        T v = acc[f];
        if (f < 3 && o.sub3 != nullptr) v -= o.sub3[f * g.N + node];
        if (f < 3 && mask_bit(mask, f * g.N + node)) {
            // Dirichlet rows: identity (apply) or u - g_D (residual)
            v = x[f * g.N + node];
            if (o.gD != nullptr) v -= o.gD[f * g.N + node];
        }
        y[f * g.N + node] = v;
    }
}

template <typename T>
int launch_q1_cells(const Geo &g, const VmsConst<T> &k, const T *x, const T *a, const T *s,
                    const uint32_t *mask, const T *gram, const int32_t *occ_index, T *part,
                    const BrickLayout &bl, hipStream_t st, bool resid)
{
    ProfileScope prof(resid ? "vms_q1_residual" : "vms_q1_cells", st);
    if (resid)
        hipLaunchKernelGGL((vms_q1_cells<T, true>), dim3((unsigned)bl.nb), dim3(256), 0, st, g, k, x, a,
                           s, mask, gram, occ_index, part, bl.nbx, bl.nby);
    else
        hipLaunchKernelGGL((vms_q1_cells<T, false>), dim3((unsigned)bl.nb), dim3(256), 0, st, g, k, x,
                           a, s, mask, gram, occ_index, part, bl.nbx, bl.nby);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

template <typename T, int P, int BX, int BY, int BZ>
int launch_gather(const Geo &g, const T *part, const BrickLayout &bl, const T *x,
                  const uint32_t *mask, T *y, const GatherOpts<T> &o, hipStream_t st)
{
    const unsigned blocks = (unsigned)((g.N + 255) / 256);
    ProfileScope prof("vms_gather", st);
    hipLaunchKernelGGL((vms_gather<T, P, BX, BY, BZ>), dim3(blocks), dim3(256), 0, st, g, part,
                       bl.nbx, bl.nby, bl.nbz, x, mask, y, o);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

template int launch_q1_cells<double>(const Geo &, const VmsConst<double> &, const double *,
                                     const double *, const double *, const uint32_t *,
                                     const double *, const int32_t *, double *,
                                     const BrickLayout &, hipStream_t, bool);
template int launch_q1_cells<float>(const Geo &, const VmsConst<float> &, const float *,
                                    const float *, const float *, const uint32_t *, const float *,
                                    const int32_t *, float *, const BrickLayout &, hipStream_t, bool);
#define FSI_GATHER_INST(T, P, BX, BY, BZ)                                                           \
    template int launch_gather<T, P, BX, BY, BZ>(const Geo &, const T *, const BrickLayout &,     \
                                                 const T *, const uint32_t *, T *,                \
                                                 const GatherOpts<T> &, hipStream_t);
FSI_GATHER_INST(double, 1, Q1_BX, Q1_BY, Q1_BZ)
FSI_GATHER_INST(float, 1, Q1_BX, Q1_BY, Q1_BZ)
FSI_GATHER_INST(double, 2, Q2_BX, Q2_BY, Q2_BZ)
FSI_GATHER_INST(float, 2, Q2_BX, Q2_BY, Q2_BZ)

}  // namespace fsi
