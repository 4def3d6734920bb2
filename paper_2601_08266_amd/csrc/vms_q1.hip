// Matrix-free Q1-Q1 Oseen-VMS operator on gfx950 (section 2.1: Galerkin weak
// form + residual-based SUPG/PSPG/LSIC with the paper's tau_m, tau_c, G).
//
// Design
//  * One workgroup = a brick of 8x8x4 cells, one cell per lane (4 waves).  Bricks
//    are dealt to the XCDs in contiguous ranges so neighbouring bricks share L2.
//  * The brick's 9x9x5 nodes of every field (x, a or f, s) are staged in LDS
//    with one batch of buffer loads (two nodes per lane per field); the
//    Dirichlet mask is applied while staging.
//  * Per cell, the velocity/pressure fields are turned into the 8 coefficients
//    of their trilinear monomial expansion (three rounds of differences).
//  * Phase 1 evaluates what depends only on the advection field and s at the 8
//    Gauss points (a/h, tau_m, tau_c) by one interpolation pass per axis into a
//    per-lane LDS table.  Phase 2 walks the points in x-pairs (not unrolled: the
//    live set is the coefficients and the moment accumulators, which keeps FP64
//    at two waves per SIMD); along a pair a field is E + x O with O its
//    x-derivative.  Derivatives stay on the reference cell, the 1/h factors sit
//    in the table and the constants, and the equal Gauss weight is applied once
//    at the end.
//  * The test side accumulates 8 monomial moments per output field and maps
//    them back to the 8 nodes with the transposed difference rounds.
//  * Element -> node accumulation: each lane parks its 32 nodal outputs in LDS
//    and each brick node sums the corners of its (up to 8) cells in a fixed
//    order, so the result is deterministic without atomics.  Bricks of one
//    parity class (bx, by, bz mod 2) share no node, so each class writes a
//    grid-shaped partial array; a node-parallel gather kernel sums the classes
//    holding each node in a fixed order, adds the DLM corner sums of occupied
//    neighbour cells if requested, and applies the Dirichlet rows.
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

// inverse of to_monomial
template <typename T>
__device__ __forceinline__ void from_monomial(T v[8])
{
    v[4] += v[0]; v[5] += v[1]; v[6] += v[2]; v[7] += v[3];
    v[2] += v[0]; v[3] += v[1]; v[6] += v[4]; v[7] += v[5];
    v[1] += v[0]; v[3] += v[2]; v[5] += v[4]; v[7] += v[6];
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
    // each product is fused into the running moment (20 operations per point and field
    // instead of 28 with separately formed sums)
    m[0] += F0;
    m[1] = fma(F0, q.x, m[1]) + G0;
    m[2] = fma(F0, q.y, m[2]) + G1;
    m[3] = fma(G1, q.x, fma(G0, q.y, fma(F0, q.xy, m[3])));
    m[4] = fma(F0, q.z, m[4]) + G2;
    m[5] = fma(G2, q.x, fma(G0, q.z, fma(F0, q.xz, m[5])));
    m[6] = fma(G2, q.y, fma(G1, q.z, fma(F0, q.yz, m[6])));
    m[7] = fma(G2, q.xy, fma(G1, q.xz, fma(G0, q.yz, fma(F0, q.xyz, m[7]))));
}

// the same with F0 = 0 (a test side that carries only gradient terms)
template <typename T>
__device__ __forceinline__ void moments_grad(T m[8], T G0, T G1, T G2, const QP<T> &q)
{
    m[1] += G0;
    m[2] += G1;
    m[3] = fma(G1, q.x, fma(G0, q.y, m[3]));
    m[4] += G2;
    m[5] = fma(G2, q.x, fma(G0, q.z, m[5]));
    m[6] = fma(G2, q.y, fma(G1, q.z, m[6]));
    m[7] = fma(G2, q.xy, fma(G1, q.xz, fma(G0, q.yz, m[7])));
}

// Buffer loads: one resource per field and block (base = the brick's first node), the
// lane's node offset in a VGPR and the cell-corner offset, uniform, in an SGPR.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t field_rsrc(const void *base, int64_t bytes)
{
    const int32_t n = bytes > (int64_t)0x7fffffff ? 0x7fffffff : (int32_t)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, n, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// 1/sqrt(x) for x > 0: hardware estimate refined by Newton steps y <- y + y (1 - x y^2) / 2
// (two in FP64, one in FP32: both end within a few ulp of the correctly rounded value).
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double e = fma(-(x * y), y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}
__device__ __forceinline__ float rsqrt_nr(float x)
{
    float y = __builtin_amdgcn_rsqf(x);
    const float e = fmaf(-(x * y), y, 1.0f);
    return fmaf(0.5f * y, e, y);
}

// Values at the 8 Gauss points (index ix + 2 iy + 4 iz) of a trilinear field given by its
// nodal values (index a + 2 b + 4 c): one linear-interpolation pass per axis.
template <typename T>
__device__ __forceinline__ void gauss_values(const T v[8], T q[8])
{
#pragma unroll
    for (int i = 0; i < 8; ++i) q[i] = v[i];
#pragma unroll
    for (int st = 1; st < 8; st <<= 1) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (i & st) continue;
            const T v0 = q[i], d = q[i + st] - v0;
            q[i] = v0 + T(GQ0) * d;
            q[i + st] = v0 + T(GQ1) * d;
        }
    }
}

// Per-Gauss-point quantities that depend only on the advection field and s, computed
// before the element loop and kept in LDS (slot j of point q at lq[(5 q + j) * Q1_NT]).
// Apply: the advection velocity scaled by 1/h (a_k / h_k); residual: the source f.
// Then tau_m and tau_c.
constexpr int Q1_NQV = 5;

// Phase 1.  cu: nodal x (Dirichlet-masked in apply mode), turned into monomial form in
// place; ca: nodal advection field (apply) or source (residual); cs: nodal s.
// tau_m = (s (C_T/dt^2 + a.Ga + C_I nu^2 G:G))^{-1/2},  tau_c = (tau_m tr G)^{-1}.
template <typename T, bool RESID>
__device__ __forceinline__ void q1_point_table(const VmsConst<T> &k, T cu[4][8], T ca[3][8], T cs[8],
                                               T *lq)
{
    T Sq[8];
    if (k.has_s) {
        T smin = cs[0];
#pragma unroll
        for (int A = 1; A < 8; ++A) smin = cs[A] < smin ? cs[A] : smin;
        gauss_values(cs, Sq);
#pragma unroll
        for (int q = 0; q < 8; ++q) Sq[q] = Sq[q] < smin ? smin : Sq[q];
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) Sq[q] = T(1);
    }
    // a.G a at the points (advection by the velocity itself in the residual)
    T aGa[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) aGa[q] = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T vq[8], aq[8];
        gauss_values(ca[d], vq);
        if constexpr (RESID) {
            gauss_values(cu[d], aq);
#pragma unroll
            for (int q = 0; q < 8; ++q) lq[(Q1_NQV * q + d) * Q1_NT] = vq[q];
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                aq[q] = vq[q] * k.ih[d];
                lq[(Q1_NQV * q + d) * Q1_NT] = aq[q];
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const T ah = RESID ? aq[q] * k.ih[d] : aq[q];
            aGa[q] += ah * ah;
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const T tb = Sq[q] * (k.K1 + aGa[q]);
        const T tau_m = rsqrt_nr(tb);
        lq[(Q1_NQV * q + 3) * Q1_NT] = tau_m;
        lq[(Q1_NQV * q + 4) * Q1_NT] = (tb * tau_m) * k.inv_trG;
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) to_monomial(cu[f]);
}

// Gauss point coordinates on [0,1]^3 and their products, point q = ix + 2 iy + 4 iz
template <typename T>
struct Q1Points {
    T v[8][8];   // x, y, z, xy, xz, yz, xyz, 0
};
#define FSI_QP_ROW(q)                                                                              \
    {(q & 1) ? GQ1 : GQ0, (q & 2) ? GQ1 : GQ0, (q & 4) ? GQ1 : GQ0,                               \
     ((q & 1) ? GQ1 : GQ0) * ((q & 2) ? GQ1 : GQ0), ((q & 1) ? GQ1 : GQ0) * ((q & 4) ? GQ1 : GQ0), \
     ((q & 2) ? GQ1 : GQ0) * ((q & 4) ? GQ1 : GQ0),                                              \
     ((q & 1) ? GQ1 : GQ0) * ((q & 2) ? GQ1 : GQ0) * ((q & 4) ? GQ1 : GQ0), 0.0}
__constant__ Q1Points<double> q1_points_f64 = {{FSI_QP_ROW(0), FSI_QP_ROW(1), FSI_QP_ROW(2),
                                                FSI_QP_ROW(3), FSI_QP_ROW(4), FSI_QP_ROW(5),
                                                FSI_QP_ROW(6), FSI_QP_ROW(7)}};
#undef FSI_QP_ROW
#define FSI_QP_ROW(q)                                                                              \
    {(float)((q & 1) ? GQ1 : GQ0), (float)((q & 2) ? GQ1 : GQ0), (float)((q & 4) ? GQ1 : GQ0),    \
     (float)(((q & 1) ? GQ1 : GQ0) * ((q & 2) ? GQ1 : GQ0)),                                      \
     (float)(((q & 1) ? GQ1 : GQ0) * ((q & 4) ? GQ1 : GQ0)),                                      \
     (float)(((q & 2) ? GQ1 : GQ0) * ((q & 4) ? GQ1 : GQ0)),                                      \
     (float)(((q & 1) ? GQ1 : GQ0) * ((q & 2) ? GQ1 : GQ0) * ((q & 4) ? GQ1 : GQ0)), 0.0f}
__constant__ Q1Points<float> q1_points_f32 = {{FSI_QP_ROW(0), FSI_QP_ROW(1), FSI_QP_ROW(2),
                                               FSI_QP_ROW(3), FSI_QP_ROW(4), FSI_QP_ROW(5),
                                               FSI_QP_ROW(6), FSI_QP_ROW(7)}};
#undef FSI_QP_ROW
template <typename T>
__device__ __forceinline__ QP<T> q1_point(int q)
{
    const T *r;
    if constexpr (sizeof(T) == 8)
        r = q1_points_f64.v[q];
    else
        r = q1_points_f32.v[q];
    QP<T> o;
    o.x = r[0]; o.y = r[1]; o.z = r[2]; o.xy = r[3]; o.xz = r[4]; o.yz = r[5]; o.xyz = r[6];
    return o;
}

// The same values selected by the point's index bits (uniform: scalar selects instead of a
// memory load whose wait would share the LDS counter); used by the apply and residual cells
template <typename T>
__device__ __forceinline__ QP<T> q1_point_sel(int q)
{
    const bool bx = q & 1, by = (q >> 1) & 1, bz = (q >> 2) & 1;
    const double x = bx ? GQ1 : GQ0, y = by ? GQ1 : GQ0, z = bz ? GQ1 : GQ0;
    const double xy = bx ? (by ? GQ1 * GQ1 : GQ1 * GQ0) : (by ? GQ0 * GQ1 : GQ0 * GQ0);
    const double xz = bx ? (bz ? GQ1 * GQ1 : GQ1 * GQ0) : (bz ? GQ0 * GQ1 : GQ0 * GQ0);
    const double yz = by ? (bz ? GQ1 * GQ1 : GQ1 * GQ0) : (bz ? GQ0 * GQ1 : GQ0 * GQ0);
    const double xyz = bz ? (by ? (bx ? GQ1 * GQ1 * GQ1 : GQ0 * GQ1 * GQ1) : (bx ? GQ1 * GQ0 * GQ1 : GQ0 * GQ0 * GQ1))
                          : (by ? (bx ? GQ1 * GQ1 * GQ0 : GQ0 * GQ1 * GQ0) : (bx ? GQ1 * GQ0 * GQ0 : GQ0 * GQ0 * GQ0));
    QP<T> o;
    o.x = T(x); o.y = T(y); o.z = T(z); o.xy = T(xy); o.xz = T(xz); o.yz = T(yz); o.xyz = T(xyz);
    return o;
}

// Phase 2: Galerkin + SUPG/PSPG/LSIC weighting at the 8 Gauss points from the monomial
// coefficients cu and the point table lq; output out[f][A] (nodal).  Derivatives are
// taken on the reference cell and the 1/h factors folded into the table and the
// constants.  The points are visited in x-pairs sharing (y, z): a field's value along the
// pair is E + x O with O its x-derivative, so E and O are formed once per pair.
// If dlm != nullptr, the cell's 8x8 block of B^T diag(kappa) B is applied to the nodal
// velocity and added to the momentum rows.  RESID = true: nonlinear residual of a time
// step instead of the linear apply: the advection field is the velocity itself (a = u)
// and the table holds the source f = c_m u_old + body force, whose Galerkin/SUPG/PSPG
// weighting is subtracted.  VB = true (apply only): the velocity rows of the operator applied
// to (u, 0): the pressure coefficients are not read and the continuity row is not formed.
template <typename T, bool RESID, bool VS, bool VB = false>
__device__ __forceinline__ void q1_cell(const VmsConst<T> &k, T cu[4][8], const T *lq,
                                        const T *__restrict__ dlm, T out[4][8])
{
    static_assert(!(RESID && VB), "the velocity block is a part of the linear apply");
    constexpr int NI = VB ? 3 : 4;   // input fields used, output rows formed
    T mom[4][8];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int i = 0; i < 8; ++i) mom[f][i] = T(0);

#pragma unroll 1
    for (int pr = 0; pr < 4; ++pr) {
        const QP<T> q0 = q1_point_sel<T>(2 * pr);
        T E[4], O[4];
#pragma unroll
        for (int f = 0; f < NI; ++f) {
            const T *c = cu[f];
            E[f] = c[0] + c[2] * q0.y + c[4] * q0.z + c[6] * q0.yz;
            O[f] = c[1] + c[3] * q0.y + c[5] * q0.z + c[7] * q0.yz;
        }
#pragma unroll
        for (int ix = 0; ix < 2; ++ix) {
            const int qi = 2 * pr + ix;
            const QP<T> q = q1_point_sel<T>(qi);
            const T *lp = lq + Q1_NQV * qi * Q1_NT;
            T Ah[3] = {lp[0], lp[Q1_NT], lp[2 * Q1_NT]};
            const T tau_m = lp[3 * Q1_NT], tau_c = lp[4 * Q1_NT];

            // values and reference derivatives (d/dxi_k)
            T U[3], dU[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                U[i] = E[i] + q.x * O[i];
                dU[i][0] = O[i];
                dU[i][1] = mdy(cu[i], q);
                dU[i][2] = mdz(cu[i], q);
            }
            T P = T(0), dP[3] = {T(0), T(0), T(0)};
            if constexpr (!VB) {
                P = E[3] + q.x * O[3];
                dP[0] = O[3];
                dP[1] = mdy(cu[3], q);
                dP[2] = mdz(cu[3], q);
            }
            T Fs[3] = {T(0), T(0), T(0)};
            if constexpr (RESID) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    Fs[d] = Ah[d];
                    Ah[d] = U[d] * k.ih[d];
                }
            }
            const T div = dU[0][0] * k.ih[0] + dU[1][1] * k.ih[1] + dU[2][2] * k.ih[2];
            // nu grad(div u) for trilinear fields on Cartesian cells (only mixed second
            // derivatives survive)
            T ngd[3] = {T(0), T(0), T(0)};
            if constexpr (VS) {
                const T u1xy = (cu[1][3] + cu[1][7] * q.z) * k.nu_hh[0][1];
                const T u2xz = (cu[2][5] + cu[2][7] * q.y) * k.nu_hh[0][2];
                const T u0xy = (cu[0][3] + cu[0][7] * q.z) * k.nu_hh[0][1];
                const T u2yz = (cu[2][6] + cu[2][7] * q.x) * k.nu_hh[1][2];
                const T u0xz = (cu[0][5] + cu[0][7] * q.y) * k.nu_hh[0][2];
                const T u1yz = (cu[1][6] + cu[1][7] * q.x) * k.nu_hh[1][2];
                ngd[0] = u1xy + u2xz;
                ngd[1] = u0xy + u2yz;
                ngd[2] = u0xz + u1yz;
            }
            T tr[3], F0[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                T gm = k.c_m * U[i] + (Ah[0] * dU[i][0] + Ah[1] * dU[i][1] + Ah[2] * dU[i][2]);
                if constexpr (RESID) gm -= Fs[i];
                F0[i] = gm;
                T r;
                if constexpr (VB)
                    r = gm - ngd[i];
                else
                    r = (gm + dP[i] * k.ih[i]) - ngd[i];
                tr[i] = tau_m * r;
            }
            T diag;
            if constexpr (VB)
                diag = tau_c * div;
            else
                diag = tau_c * div - P;
            // test-side fluxes, already multiplied by 1/h_k:
            //   nu (d_k u_i + d_i u_k) + a_k tau_m r_i + delta_ik (tau_c div u - p)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                T G[3];
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    T fl;
                    if (kk == i)
                        fl = T(2) * k.nu_hh[i][i] * dU[i][i] + diag * k.ih[i];
                    else
                        fl = k.nu_hh[kk][kk] * dU[i][kk] + k.nu_hh[kk][i] * dU[kk][i];
                    G[kk] = fl + Ah[kk] * tr[i];
                }
                moments(mom[i], F0[i], G[0], G[1], G[2], q);
            }
            if constexpr (!VB) moments(mom[3], div, tr[0] * k.ih[0], tr[1] * k.ih[1], tr[2] * k.ih[2], q);
        }
    }
    const T W = k.detJ * T(0.125);
#pragma unroll
    for (int f = 0; f < NI; ++f) {
#pragma unroll
        for (int i = 0; i < 8; ++i) mom[f][i] *= W;
        from_moments(mom[f]);
#pragma unroll
        for (int i = 0; i < 8; ++i) out[f][i] = mom[f][i];
    }
    if (dlm != nullptr) {
        // DLM block on the nodal (Dirichlet-masked) velocity
#pragma unroll
        for (int f = 0; f < 3; ++f) from_monomial(cu[f]);
#pragma unroll
        for (int A = 0; A < 8; ++A) {
#pragma unroll
            for (int C = 0; C < 8; ++C) {
                const T gAC = dlm[A * 8 + C];
                out[0][A] += gAC * cu[0][C];
                out[1][A] += gAC * cu[1][C];
                out[2][A] += gAC * cu[2][C];
            }
        }
    }
}

// Velocity rows of the operator applied to (0, p): with u = 0 the momentum residual is the
// pressure gradient, div u = 0, and the Galerkin, viscous and DLM terms vanish, so per Gauss
// point the momentum test w carries -p div w + ((a.grad) w) . tau_m grad p.  cp: the pressure in
// monomial form; lq: the apply's point table (a/h, tau_m, tau_c).
template <typename T>
__device__ __forceinline__ void q1_cell_grad_p(const VmsConst<T> &k, const T cp[8], const T *lq, T out[3][8])
{
    T mom[3][8];
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int i = 0; i < 8; ++i) mom[f][i] = T(0);

#pragma unroll 1
    for (int pr = 0; pr < 4; ++pr) {
        const QP<T> q0 = q1_point_sel<T>(2 * pr);
        const T E = cp[0] + cp[2] * q0.y + cp[4] * q0.z + cp[6] * q0.yz;
        const T O = cp[1] + cp[3] * q0.y + cp[5] * q0.z + cp[7] * q0.yz;
#pragma unroll
        for (int ix = 0; ix < 2; ++ix) {
            const int qi = 2 * pr + ix;
            const QP<T> q = q1_point_sel<T>(qi);
            const T *lp = lq + Q1_NQV * qi * Q1_NT;
            const T Ah[3] = {lp[0], lp[Q1_NT], lp[2 * Q1_NT]};
            const T tau_m = lp[3 * Q1_NT];
            const T P = E + q.x * O;
            const T dP[3] = {O, mdy(cp, q), mdz(cp, q)};
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const T tr = tau_m * (dP[i] * k.ih[i]);
                T G[3];
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) G[kk] = kk == i ? -P * k.ih[i] + Ah[kk] * tr : Ah[kk] * tr;
                moments_grad(mom[i], G[0], G[1], G[2], q);
            }
        }
    }
    const T W = k.detJ * T(0.125);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
#pragma unroll
        for (int i = 0; i < 8; ++i) mom[f][i] *= W;
        from_moments(mom[f]);
#pragma unroll
        for (int i = 0; i < 8; ++i) out[f][i] = mom[f][i];
    }
}

// Phase 2 of the full Newton tangent (section 2.4: Newton on the monolithic system): what the
// Picard/Oseen operator with a = u leaves out of the derivative of the step residual, applied
// to the velocity direction dv.  With rho = r_m(u, p) - f the strong momentum residual of the
// state and c = (dv.grad)u, per Gauss point
//   momentum test w:   w.c + ((u.grad)w).(tau_m c + sigma rho) + tau_m ((dv.grad)w).rho
//                      + dtau_c (div w)(div u)
//   continuity test q: grad q.(tau_m c + sigma rho)
// with sigma = d tau_m = -tau_m^3 s (u.G dv) = -(tau_m / B)(u.G dv), B = K1 + u.G u, and
// dtau_c = -(tau_c / tau_m) sigma.  cu: state (u, p) in monomial form; cd: dv in monomial form;
// lq: the residual's point table (f, tau_m, tau_c).
template <typename T>
__device__ __forceinline__ void q1_tangent_cell(const VmsConst<T> &k, const T cu[4][8], const T cd[3][8],
                                                const T *lq, T out[4][8])
{
    T mom[4][8];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int i = 0; i < 8; ++i) mom[f][i] = T(0);

    // the points in x-pairs sharing (y, z): along a pair a field is E + x O (O its x-derivative)
#pragma unroll 1
    for (int pr = 0; pr < 4; ++pr) {
        const QP<T> q0 = q1_point<T>(2 * pr);
        T Eu[3], Ou[3], Ed[3], Od[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            Eu[i] = cu[i][0] + cu[i][2] * q0.y + cu[i][4] * q0.z + cu[i][6] * q0.yz;
            Ou[i] = cu[i][1] + cu[i][3] * q0.y + cu[i][5] * q0.z + cu[i][7] * q0.yz;
            Ed[i] = cd[i][0] + cd[i][2] * q0.y + cd[i][4] * q0.z + cd[i][6] * q0.yz;
            Od[i] = cd[i][1] + cd[i][3] * q0.y + cd[i][5] * q0.z + cd[i][7] * q0.yz;
        }
#pragma unroll
        for (int ix = 0; ix < 2; ++ix) {
            const int qi = 2 * pr + ix;
            const QP<T> q = q1_point<T>(qi);
            const T *lp = lq + Q1_NQV * qi * Q1_NT;
            const T tau_m = lp[3 * Q1_NT], tau_c = lp[4 * Q1_NT];
            T U[3], dU[3][3], Ah[3], D[3], Dh[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                U[i] = Eu[i] + q.x * Ou[i];
                dU[i][0] = Ou[i];
                dU[i][1] = mdy(cu[i], q);
                dU[i][2] = mdz(cu[i], q);
                Ah[i] = U[i] * k.ih[i];
                D[i] = Ed[i] + q.x * Od[i];
                Dh[i] = D[i] * k.ih[i];
            }
            const T dP[3] = {mdx(cu[3], q), mdy(cu[3], q), mdz(cu[3], q)};
            const T div = dU[0][0] * k.ih[0] + dU[1][1] * k.ih[1] + dU[2][2] * k.ih[2];
            T ngd[3] = {T(0), T(0), T(0)};
            if (k.visc_strong) {
                const T u1xy = (cu[1][3] + cu[1][7] * q.z) * k.nu_hh[0][1];
                const T u2xz = (cu[2][5] + cu[2][7] * q.y) * k.nu_hh[0][2];
                const T u0xy = (cu[0][3] + cu[0][7] * q.z) * k.nu_hh[0][1];
                const T u2yz = (cu[2][6] + cu[2][7] * q.x) * k.nu_hh[1][2];
                const T u0xz = (cu[0][5] + cu[0][7] * q.y) * k.nu_hh[0][2];
                const T u1yz = (cu[1][6] + cu[1][7] * q.x) * k.nu_hh[1][2];
                ngd[0] = u1xy + u2xz;
                ngd[1] = u0xy + u2yz;
                ngd[2] = u0xz + u1yz;
            }
            // rho_i and c_i = dv_j d_j u_i (physical derivatives: reference ones times 1/h)
            T rho[3], c[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const T conv = Ah[0] * dU[i][0] + Ah[1] * dU[i][1] + Ah[2] * dU[i][2];
                rho[i] = ((k.c_m * U[i] + conv - lp[i * Q1_NT]) + dP[i] * k.ih[i]) - ngd[i];
                c[i] = Dh[0] * dU[i][0] + Dh[1] * dU[i][1] + Dh[2] * dU[i][2];
            }
            const T B = k.K1 + (Ah[0] * Ah[0] + Ah[1] * Ah[1] + Ah[2] * Ah[2]);
            const T sigma = -(tau_m / B) * (Ah[0] * Dh[0] + Ah[1] * Dh[1] + Ah[2] * Dh[2]);
            const T dtc_div = -(tau_c / tau_m) * sigma * div;
            T e[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) e[i] = tau_m * c[i] + sigma * rho[i];
            // test-side fluxes multiplied by 1/h_k (reference derivatives of the test functions)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const T tr = tau_m * rho[i];
                T G[3];
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) G[kk] = Ah[kk] * e[i] + Dh[kk] * tr;
                G[i] += dtc_div * k.ih[i];
                moments(mom[i], c[i], G[0], G[1], G[2], q);
            }
            moments(mom[3], T(0), e[0] * k.ih[0], e[1] * k.ih[1], e[2] * k.ih[2], q);
        }
    }
    const T W = k.detJ * T(0.125);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
#pragma unroll
        for (int i = 0; i < 8; ++i) mom[f][i] *= W;
        from_moments(mom[f]);
#pragma unroll
        for (int i = 0; i < 8; ++i) out[f][i] = mom[f][i];
    }
}

// The whole full-Newton-tangent contribution of one cell in one pass: the Picard operator with
// a = u applied to the direction (dv, dp) plus the correction of q1_tangent_cell, whose test
// fluxes are merged so that each field's moments are accumulated once per point.  cu: state
// (u, p), cd: direction (dv masked, dp), both in monomial form; lq: the residual's point table
// (f, tau_m, tau_c); dlm: the cell's DLM block (applied to the nodal direction) or nullptr.
template <typename T>
__device__ __forceinline__ void q1_fused_tangent_cell(const VmsConst<T> &k, const T cu[4][8], T cd[4][8],
                                                      const T *lq, const T *__restrict__ dlm, T out[4][8])
{
    T mom[4][8];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int i = 0; i < 8; ++i) mom[f][i] = T(0);

#pragma unroll 1
    for (int pr = 0; pr < 4; ++pr) {
        const QP<T> q0 = q1_point<T>(2 * pr);
        T Es[4], Os[4], Ed[4], Od[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            Es[f] = cu[f][0] + cu[f][2] * q0.y + cu[f][4] * q0.z + cu[f][6] * q0.yz;
            Os[f] = cu[f][1] + cu[f][3] * q0.y + cu[f][5] * q0.z + cu[f][7] * q0.yz;
            Ed[f] = cd[f][0] + cd[f][2] * q0.y + cd[f][4] * q0.z + cd[f][6] * q0.yz;
            Od[f] = cd[f][1] + cd[f][3] * q0.y + cd[f][5] * q0.z + cd[f][7] * q0.yz;
        }
#pragma unroll
        for (int ix = 0; ix < 2; ++ix) {
            const int qi = 2 * pr + ix;
            const QP<T> q = q1_point<T>(qi);
            const T *lp = lq + Q1_NQV * qi * Q1_NT;
            const T tau_m = lp[3 * Q1_NT], tau_c = lp[4 * Q1_NT];
            // state (s) and direction (d): values and reference derivatives
            T Us[3], dUs[3][3], Ah[3], D[3], dD[3][3], Dh[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                Us[i] = Es[i] + q.x * Os[i];
                dUs[i][0] = Os[i];
                dUs[i][1] = mdy(cu[i], q);
                dUs[i][2] = mdz(cu[i], q);
                Ah[i] = Us[i] * k.ih[i];
                D[i] = Ed[i] + q.x * Od[i];
                dD[i][0] = Od[i];
                dD[i][1] = mdy(cd[i], q);
                dD[i][2] = mdz(cd[i], q);
                Dh[i] = D[i] * k.ih[i];
            }
            const T dPs[3] = {Os[3], mdy(cu[3], q), mdz(cu[3], q)};
            const T Pd = Ed[3] + q.x * Od[3];
            const T dPd[3] = {Od[3], mdy(cd[3], q), mdz(cd[3], q)};
            const T divs = dUs[0][0] * k.ih[0] + dUs[1][1] * k.ih[1] + dUs[2][2] * k.ih[2];
            const T divd = dD[0][0] * k.ih[0] + dD[1][1] * k.ih[1] + dD[2][2] * k.ih[2];
            // nu grad(div) of the state and of the direction (mixed second derivatives only)
            T ngs[3] = {T(0), T(0), T(0)}, ngdd[3] = {T(0), T(0), T(0)};
            if (k.visc_strong) {
                ngs[0] = (cu[1][3] + cu[1][7] * q.z) * k.nu_hh[0][1] + (cu[2][5] + cu[2][7] * q.y) * k.nu_hh[0][2];
                ngs[1] = (cu[0][3] + cu[0][7] * q.z) * k.nu_hh[0][1] + (cu[2][6] + cu[2][7] * q.x) * k.nu_hh[1][2];
                ngs[2] = (cu[0][5] + cu[0][7] * q.y) * k.nu_hh[0][2] + (cu[1][6] + cu[1][7] * q.x) * k.nu_hh[1][2];
                ngdd[0] = (cd[1][3] + cd[1][7] * q.z) * k.nu_hh[0][1] + (cd[2][5] + cd[2][7] * q.y) * k.nu_hh[0][2];
                ngdd[1] = (cd[0][3] + cd[0][7] * q.z) * k.nu_hh[0][1] + (cd[2][6] + cd[2][7] * q.x) * k.nu_hh[1][2];
                ngdd[2] = (cd[0][5] + cd[0][7] * q.y) * k.nu_hh[0][2] + (cd[1][6] + cd[1][7] * q.x) * k.nu_hh[1][2];
            }
            // Picard part on the direction: gm = c_m dv + (u.grad) dv, tr = tau_m r_m(dv, dp)
            // correction: rho = r_m(u, p) - f, c = (dv.grad)u, sigma = d tau_m, e = tau_m c + sigma rho
            T gm[3], tr[3], rho[3], c[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                gm[i] = k.c_m * D[i] + (Ah[0] * dD[i][0] + Ah[1] * dD[i][1] + Ah[2] * dD[i][2]);
                tr[i] = tau_m * ((gm[i] + dPd[i] * k.ih[i]) - ngdd[i]);
                const T conv = Ah[0] * dUs[i][0] + Ah[1] * dUs[i][1] + Ah[2] * dUs[i][2];
                rho[i] = ((k.c_m * Us[i] + conv - lp[i * Q1_NT]) + dPs[i] * k.ih[i]) - ngs[i];
                c[i] = Dh[0] * dUs[i][0] + Dh[1] * dUs[i][1] + Dh[2] * dUs[i][2];
            }
            const T B = k.K1 + (Ah[0] * Ah[0] + Ah[1] * Ah[1] + Ah[2] * Ah[2]);
            const T sigma = -(tau_m / B) * (Ah[0] * Dh[0] + Ah[1] * Dh[1] + Ah[2] * Dh[2]);
            const T dtc_div = -(tau_c / tau_m) * sigma * divs;
            const T diag = tau_c * divd - Pd;
            T e[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) e[i] = tau_m * c[i] + sigma * rho[i];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const T te = tr[i] + e[i], trho = tau_m * rho[i];
                T G[3];
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    T fl;
                    if (kk == i)
                        fl = T(2) * k.nu_hh[i][i] * dD[i][i] + (diag + dtc_div) * k.ih[i];
                    else
                        fl = k.nu_hh[kk][kk] * dD[i][kk] + k.nu_hh[kk][i] * dD[kk][i];
                    G[kk] = fl + Ah[kk] * te + Dh[kk] * trho;
                }
                moments(mom[i], gm[i] + c[i], G[0], G[1], G[2], q);
            }
            moments(mom[3], divd, (tr[0] + e[0]) * k.ih[0], (tr[1] + e[1]) * k.ih[1], (tr[2] + e[2]) * k.ih[2], q);
        }
    }
    const T W = k.detJ * T(0.125);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
#pragma unroll
        for (int i = 0; i < 8; ++i) mom[f][i] *= W;
        from_moments(mom[f]);
#pragma unroll
        for (int i = 0; i < 8; ++i) out[f][i] = mom[f][i];
    }
    if (dlm != nullptr) {
        // DLM block on the nodal (Dirichlet-masked) direction
#pragma unroll
        for (int f = 0; f < 3; ++f) from_monomial(cd[f]);
#pragma unroll
        for (int A = 0; A < 8; ++A) {
#pragma unroll
            for (int C = 0; C < 8; ++C) {
                const T gAC = dlm[A * 8 + C];
                out[0][A] += gAC * cd[0][C];
                out[1][A] += gAC * cd[1][C];
                out[2][A] += gAC * cd[2][C];
            }
        }
    }
}

// Brick handled by block bid.  Blocks are dealt to the 8 XCDs round-robin; each XCD is
// given a contiguous range of bricks (x fastest), so bricks that share face nodes (and
// the cache lines holding them) mostly run under the same L2.
// (32-bit: a launch has fewer than 2^32 blocks, and 64-bit divisions are long scalar sequences)
__device__ __forceinline__ uint32_t xcd_brick(uint32_t bid, uint32_t nb)
{
    const uint32_t q = nb >> 3, r = nb & 7u, xcd = bid & 7u, idx = bid >> 3;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// MODE 0: linear apply (advection field a); 1: step residual (a = u, source f in `a`);
// 2: full-tangent correction: x = state (u, p), `a` = source f, dv = velocity direction; the
// result is added to the brick partials that the Picard apply (MODE 0 with a = u) wrote;
// 3: the whole full-Newton tangent in one pass: x = state, `a` = source f, dv = direction
// (velocity and pressure), gram = the per-cell DLM blocks; the partials are overwritten;
// 4: velocity rows of the apply on (x_u, 0) (x_p is not read); 5: velocity rows of the apply on
// (0, x_p) (x_u is not read, no DLM block).  Modes 4 and 5 write three partial fields.
template <typename T, int MODE, bool VS = true>
__global__ __launch_bounds__(Q1_NT) void vms_q1_cells(Geo g, VmsConst<T> k, const T *__restrict__ x,
                                                    const T *__restrict__ a,
                                                    const T *__restrict__ s,
                                                    const uint32_t *__restrict__ mask,
                                                    const T *__restrict__ gram,
                                                    const int32_t *__restrict__ occ_index,
                                                    T *__restrict__ part, int nbx, int nby,
                                                    const T *__restrict__ dv)
{
    constexpr bool RESID = MODE >= 1 && MODE <= 3;
    constexpr bool DIR = MODE == 2 || MODE == 3;   // a direction next to the state
    constexpr bool XU = MODE != 5, XP = MODE != 4;   // velocity / pressure of x read
    constexpr int NO = MODE >= 4 ? 3 : 4;            // output rows
    // LDS, one region used three ways: the brick's nodal fields (staged with coalesced
    // loads), then the lanes' Gauss-point tables, then the lanes' nodal outputs.
    constexpr int NF = MODE == 3 ? 12 : (MODE == 2 ? 11 : 8);   // x (4), a or f (3), s (, dv (3 or 4))
    constexpr int NJ = (Q1_NL + Q1_NT - 1) / Q1_NT;   // staged nodes per lane
    static_assert(8 * Q1_NQV >= 32 && 8 * Q1_NQV * Q1_NT >= NF * Q1_NL, "LDS too small");
    __shared__ T lds[8 * Q1_NQV * Q1_NT];
    const int t = threadIdx.x;
    const uint32_t bid = xcd_brick(blockIdx.x, gridDim.x);
    const uint32_t bxy = bid / (uint32_t)nbx;
    const int bx = (int)(bid - bxy * (uint32_t)nbx), by = (int)(bxy % (uint32_t)nby), bz = (int)(bxy / (uint32_t)nby);
    const int tx = t % Q1_BX, ty = (t / Q1_BX) % Q1_BY, tz = t / (Q1_BX * Q1_BY);
    const int cx = bx * Q1_BX + tx, cy = by * Q1_BY + ty, cz = bz * Q1_BZ + tz;
    const bool valid = cx < g.n[0] && cy < g.n[1] && cz < g.n[2];
    const int64_t N = g.N;
    const int64_t nn01 = (int64_t)g.nn[0] * g.nn[1];
    constexpr int LX = Q1_BX + 1, LY = Q1_BY + 1;

    // stage the brick's (LX x LY x (BZ+1)) nodes of every field: 2 nodes per lane
    {
        const int64_t base = (int64_t)bx * Q1_BX + (int64_t)g.nn[0] * (by * Q1_BY) + nn01 * (bz * Q1_BZ);
        const int64_t rem = (N - base) * (int64_t)sizeof(T);
        uint32_t voff[NJ];
        bool inb[NJ];
        int64_t node[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int l = t + Q1_NT * j;
            const int lx = l % LX, ly = (l / LX) % LY, lz = l / (LX * LY);
            inb[j] = l < Q1_NL && bx * Q1_BX + lx < g.nn[0] && by * Q1_BY + ly < g.nn[1] &&
                     bz * Q1_BZ + lz < g.nn[2];
            const int64_t o = lx + (int64_t)g.nn[0] * ly + nn01 * lz;
            voff[j] = (uint32_t)(o * (int64_t)sizeof(T));
            node[j] = base + o;
        }
        // all loads first (one batch in flight; the buffer range check makes the ones past
        // the grid harmless), then the Dirichlet mask, then the LDS stores
        T v[NF][NJ];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if ((f < 3 && !XU) || (f == 3 && !XP)) continue;
            if (f == 7 && !k.has_s) {
#pragma unroll
                for (int j = 0; j < NJ; ++j) v[f][j] = T(1);
                continue;
            }
            const T *src = f < 4 ? x + f * N : (f < 7 ? a + (f - 4) * N : (f == 7 ? s : dv + (f - 8) * N));
            const __amdgpu_buffer_rsrc_t r = field_rsrc(src + base, rem);
#pragma unroll
            for (int j = 0; j < NJ; ++j) v[f][j] = buf_load<T>(r, voff[j], 0u);
        }
        if (MODE != 1 && MODE != 5 && mask != nullptr) {
            // Dirichlet columns: the apply's x, the tangent's direction
            constexpr int F0 = DIR ? 8 : 0;
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int j = 0; j < NJ; ++j)
                    if (inb[j] && mask_bit(mask, f * N + node[j])) v[F0 + f][j] = T(0);
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if ((f < 3 && !XU) || (f == 3 && !XP)) continue;
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                if (t + Q1_NT * j < Q1_NL) lds[f * Q1_NL + t + Q1_NT * j] = inb[j] ? v[f][j] : T(0);
        }
    }
    __syncthreads();

    T cu[4][8];
    T ca[3][8], cs[8];
    T cd[MODE == 3 ? 4 : (MODE == 2 ? 3 : 1)][8];
    if (valid) {
#pragma unroll
        for (int A = 0; A < 8; ++A) {
            const int l = (tx + (A & 1)) + LX * ((ty + ((A >> 1) & 1)) + LY * (tz + (A >> 2)));
#pragma unroll
            for (int f = 0; f < 4; ++f) cu[f][A] = (f < 3 ? XU : XP) ? lds[f * Q1_NL + l] : T(0);
#pragma unroll
            for (int d = 0; d < 3; ++d) ca[d][A] = lds[(4 + d) * Q1_NL + l];
            cs[A] = k.has_s ? lds[7 * Q1_NL + l] : T(1);
            if constexpr (DIR) {
#pragma unroll
                for (int d = 0; d < NF - 8; ++d) cd[d][A] = lds[(8 + d) * Q1_NL + l];
            }
        }
    }
    __syncthreads();
    T out[4][8];
    if (valid) {
        q1_point_table<T, RESID>(k, cu, ca, cs, lds + t);
        const T *dlm = nullptr;
        if (MODE != 5 && gram != nullptr) {
            const int32_t ko = occ_index[cx + (int64_t)g.n[0] * (cy + (int64_t)g.n[1] * cz)];
            if (ko >= 0) dlm = gram + (int64_t)ko * 64;
        }
        if constexpr (DIR) {
#pragma unroll
            for (int d = 0; d < NF - 8; ++d) to_monomial(cd[d]);
            if constexpr (MODE == 3)
                q1_fused_tangent_cell<T>(k, cu, cd, lds + t, dlm, out);
            else
                q1_tangent_cell<T>(k, cu, cd, lds + t, out);
        } else if constexpr (MODE == 5) {
            q1_cell_grad_p<T>(k, cu[3], lds + t, out);
        } else {
            q1_cell<T, RESID, VS, MODE == 4>(k, cu, lds + t, dlm, out);
        }
    }
    // element -> node accumulation: every lane parks its 32 nodal outputs in LDS, then each
    // brick node sums the corners of the (up to 8) cells around it in a fixed order
    __syncthreads();
#pragma unroll
    for (int f = 0; f < NO; ++f)
#pragma unroll
        for (int A = 0; A < 8; ++A) lds[(f * 8 + A) * Q1_NT + t] = valid ? out[f][A] : T(0);
    __syncthreads();
    for (int l = t; l < Q1_NL; l += Q1_NT) {
        const int lx = l % LX, ly = (l / LX) % LY, lz = l / (LX * LY);
        const int gx = bx * Q1_BX + lx, gy = by * Q1_BY + ly, gz = bz * Q1_BZ + lz;
        if (gx < g.nn[0] && gy < g.nn[1] && gz < g.nn[2]) {
            T sum[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const int czl = lz - 1 + kk;
                if (czl < 0 || czl >= Q1_BZ) continue;
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int cyl = ly - 1 + j;
                    if (cyl < 0 || cyl >= Q1_BY) continue;
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        const int cxl = lx - 1 + i;
                        if (cxl < 0 || cxl >= Q1_BX) continue;
                        const int A = (1 - i) + 2 * (1 - j) + 4 * (1 - kk);
                        const int lane = cxl + Q1_BX * (cyl + Q1_BY * czl);
#pragma unroll
                        for (int f = 0; f < NO; ++f) sum[f] += lds[(f * 8 + A) * Q1_NT + lane];
                    }
                }
            }
            // bricks of one parity class never share a node: one array per class
            const PartIndex pi(g.nn, nbx, Q1_BX);
            T *pc = part + pi.at((bx & 1) + 2 * (by & 1) + 4 * (bz & 1), bx, gx, gy, gz);
            if constexpr (MODE == 2) {
                // added to what the Picard apply of the same brick wrote (stream order)
#pragma unroll
                for (int f = 0; f < 4; ++f) pc[f * pi.field] += sum[f];
            } else {
#pragma unroll
                for (int f = 0; f < NO; ++f) pc[f * pi.field] = sum[f];
            }
        }
    }
}

}  // namespace

// Node gather shared by all orders: sums the brick partials (bricks of BXxBYxBZ cells of
// order P; part holds one x-packed [4][nn2][nn1][lx] array per brick parity class, so the
// reads are coalesced and dense) and, optionally, DLM corner sums of occupied neighbour
// cells; then Dirichlet rows.  NR = 3: only the velocity rows (partials of three fields; the
// pressure part of y is not written).
template <typename T, int P, int BX, int BY, int BZ, int NR = 4>
__global__ __launch_bounds__(256) void vms_gather(Geo g, const T *__restrict__ part, int nbx,
                                                  int nby, int nbz, const T *__restrict__ x,
                                                  const uint32_t *__restrict__ mask,
                                                  T *__restrict__ y, GatherOpts<T> o)
{
    const T *__restrict__ csum = o.csum;
    const int32_t *__restrict__ occ_index = o.occ_index;
    constexpr int NEN = (P + 1) * (P + 1) * (P + 1);
    // grid: x over the nodes of one z-plane, y over the planes (32-bit index math)
    const uint32_t plane = (uint32_t)g.nn[0] * (uint32_t)g.nn[1];
    const uint32_t pidx = blockIdx.x * 256u + threadIdx.x;
    if (pidx >= plane) return;
    const int gy = (int)(pidx / (uint32_t)g.nn[0]);
    const int gx = (int)pidx - gy * g.nn[0];
    const int gz = (int)blockIdx.y;
    const int64_t node = (int64_t)gz * plane + pidx;
    // bricks holding the node along each axis (lower brick first)
    int bxs[2], nxb = 0, bys[2], nyb = 0, bzs[2], nzb = 0;
    {
        constexpr int sx = P * BX, sy = P * BY, sz = P * BZ;
        int b = gx / sx;
        if (gx % sx == 0 && b > 0) bxs[nxb++] = b - 1;
        if (b < nbx) bxs[nxb++] = b;
        b = gy / sy;
        if (gy % sy == 0 && b > 0) bys[nyb++] = b - 1;
        if (b < nby) bys[nyb++] = b;
        b = gz / sz;
        if (gz % sz == 0 && b > 0) bzs[nzb++] = b - 1;
        if (b < nbz) bzs[nzb++] = b;
    }
    T acc[4] = {T(0), T(0), T(0), T(0)};
    const PartIndex pi(g.nn, nbx, P * BX);
    // the up to 8 bricks' partials are all loaded before any is added (a node on a brick face
    // would otherwise wait for one load round per brick), then summed in the fixed order z, y, x
    T pv[2][2][2][4];
#pragma unroll
    for (int iz = 0; iz < 2; ++iz)
#pragma unroll
        for (int iy = 0; iy < 2; ++iy)
#pragma unroll
            for (int ix = 0; ix < 2; ++ix)
                if (iz < nzb && iy < nyb && ix < nxb) {
                    const int cls = (bxs[ix] & 1) + 2 * (bys[iy] & 1) + 4 * (bzs[iz] & 1);
                    const T *pc = part + pi.at(cls, bxs[ix], gx, gy, gz);
#pragma unroll
                    for (int f = 0; f < NR; ++f) pv[iz][iy][ix][f] = pc[f * pi.field];
                }
#pragma unroll
    for (int iz = 0; iz < 2; ++iz)
#pragma unroll
        for (int iy = 0; iy < 2; ++iy)
#pragma unroll
            for (int ix = 0; ix < 2; ++ix)
                if (iz < nzb && iy < nyb && ix < nxb) {
#pragma unroll
                    for (int f = 0; f < NR; ++f) acc[f] += pv[iz][iy][ix][f];
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
    for (int f = 0; f < NR; ++f) {
        T v = acc[f];
        if (f < 3 && o.sub3 != nullptr) v -= o.sub3[f * g.N + node];
        if (f < 3 && mask_bit(mask, f * g.N + node)) {
            // Dirichlet rows: identity (apply; on a zero velocity when x is NULL) or u - g_D
            // (residual)
            v = x != nullptr ? x[f * g.N + node] : T(0);
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
    // buffer offsets of a brick's nodes are 32-bit: (nodes per plane) x (brick height + 1)
    FSI_CHECK_ARG((int64_t)g.nn[0] * g.nn[1] * (Q1_BZ + 1) * (int64_t)sizeof(T) < ((int64_t)1 << 31),
                  "Q1 grid planes too large (%d x %d nodes)", g.nn[0], g.nn[1]);
    ProfileScope prof(resid ? "vms_q1_residual" : "vms_q1_cells", st);
    // the strong viscous term as a compile-time switch: no branch inside the Gauss loop
    const dim3 grid((unsigned)bl.nb), block(Q1_NT);
    const T *nod = nullptr;
    if (resid) {
        if (k.visc_strong)
            hipLaunchKernelGGL((vms_q1_cells<T, 1, true>), grid, block, 0, st, g, k, x, a, s, mask, gram, occ_index,
                               part, bl.nbx, bl.nby, nod);
        else
            hipLaunchKernelGGL((vms_q1_cells<T, 1, false>), grid, block, 0, st, g, k, x, a, s, mask, gram,
                               occ_index, part, bl.nbx, bl.nby, nod);
    } else {
        if (k.visc_strong)
            hipLaunchKernelGGL((vms_q1_cells<T, 0, true>), grid, block, 0, st, g, k, x, a, s, mask, gram, occ_index,
                               part, bl.nbx, bl.nby, nod);
        else
            hipLaunchKernelGGL((vms_q1_cells<T, 0, false>), grid, block, 0, st, g, k, x, a, s, mask, gram,
                               occ_index, part, bl.nbx, bl.nby, nod);
    }
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

// Velocity rows of the apply on (x_u, 0) (blk = 1) or on (0, x_p) (blk = 2): brick partials of
// the three momentum fields.
template <typename T>
int launch_q1_block(const Geo &g, const VmsConst<T> &k, int blk, const T *x, const T *a, const T *s,
                    const uint32_t *mask, const T *gram, const int32_t *occ_index, T *part,
                    const BrickLayout &bl, hipStream_t st)
{
    FSI_CHECK_ARG((int64_t)g.nn[0] * g.nn[1] * (Q1_BZ + 1) * (int64_t)sizeof(T) < ((int64_t)1 << 31),
                  "Q1 grid planes too large (%d x %d nodes)", g.nn[0], g.nn[1]);
    FSI_CHECK_ARG(blk == 1 || blk == 2, "operator block %d (1: velocity, 2: pressure gradient)", blk);
    ProfileScope prof(blk == 1 ? "vms_q1_block_u" : "vms_q1_block_p", st);
    const dim3 grid((unsigned)bl.nb), block(Q1_NT);
    const T *nod = nullptr;
    if (blk == 2)
        hipLaunchKernelGGL((vms_q1_cells<T, 5>), grid, block, 0, st, g, k, x, a, s, mask, gram, occ_index, part,
                           bl.nbx, bl.nby, nod);
    else if (k.visc_strong)
        hipLaunchKernelGGL((vms_q1_cells<T, 4, true>), grid, block, 0, st, g, k, x, a, s, mask, gram, occ_index,
                           part, bl.nbx, bl.nby, nod);
    else
        hipLaunchKernelGGL((vms_q1_cells<T, 4, false>), grid, block, 0, st, g, k, x, a, s, mask, gram, occ_index,
                           part, bl.nbx, bl.nby, nod);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}
template int launch_q1_block<double>(const Geo &, const VmsConst<double> &, int, const double *, const double *,
                                     const double *, const uint32_t *, const double *, const int32_t *, double *,
                                     const BrickLayout &, hipStream_t);
template int launch_q1_block<float>(const Geo &, const VmsConst<float> &, int, const float *, const float *,
                                    const float *, const uint32_t *, const float *, const int32_t *, float *,
                                    const BrickLayout &, hipStream_t);

template <typename T>
int launch_q1_tangent(const Geo &g, const VmsConst<T> &k, const T *x, const T *f, const T *s,
                      const uint32_t *mask, const T *dv, T *part, const BrickLayout &bl, hipStream_t st)
{
    FSI_CHECK_ARG((int64_t)g.nn[0] * g.nn[1] * (Q1_BZ + 1) * (int64_t)sizeof(T) < ((int64_t)1 << 31),
                  "Q1 grid planes too large (%d x %d nodes)", g.nn[0], g.nn[1]);
    ProfileScope prof("vms_q1_tangent", st);
    hipLaunchKernelGGL((vms_q1_cells<T, 2>), dim3((unsigned)bl.nb), dim3(Q1_NT), 0, st, g, k, x, f, s, mask,
                       (const T *)nullptr, (const int32_t *)nullptr, part, bl.nbx, bl.nby, dv);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}
// The whole full Newton tangent at state x = (u, p), source f, on direction v = (dv, dp), with
// the per-cell DLM blocks (gram, or NULL): one pass of cells writing the brick partials.
template <typename T>
int launch_q1_tangent_fused(const Geo &g, const VmsConst<T> &k, const T *x, const T *f, const T *s,
                            const uint32_t *mask, const T *gram, const int32_t *occ_index, const T *v,
                            T *part, const BrickLayout &bl, hipStream_t st)
{
    FSI_CHECK_ARG((int64_t)g.nn[0] * g.nn[1] * (Q1_BZ + 1) * (int64_t)sizeof(T) < ((int64_t)1 << 31),
                  "Q1 grid planes too large (%d x %d nodes)", g.nn[0], g.nn[1]);
    ProfileScope prof("vms_q1_tangent_fused", st);
    hipLaunchKernelGGL((vms_q1_cells<T, 3>), dim3((unsigned)bl.nb), dim3(Q1_NT), 0, st, g, k, x, f, s, mask,
                       gram, occ_index, part, bl.nbx, bl.nby, v);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}
template int launch_q1_tangent_fused<float>(const Geo &, const VmsConst<float> &, const float *,
                                            const float *, const float *, const uint32_t *, const float *,
                                            const int32_t *, const float *, float *, const BrickLayout &,
                                            hipStream_t);
template int launch_q1_tangent<double>(const Geo &, const VmsConst<double> &, const double *, const double *,
                                       const double *, const uint32_t *, const double *, double *,
                                       const BrickLayout &, hipStream_t);
template int launch_q1_tangent<float>(const Geo &, const VmsConst<float> &, const float *, const float *,
                                      const float *, const uint32_t *, const float *, float *,
                                      const BrickLayout &, hipStream_t);

template <typename T, int P, int BX, int BY, int BZ>
int launch_gather(const Geo &g, const T *part, const BrickLayout &bl, const T *x,
                  const uint32_t *mask, T *y, const GatherOpts<T> &o, hipStream_t st)
{
    FSI_CHECK_ARG(g.nn[2] <= 65535 && (int64_t)g.nn[0] * g.nn[1] < ((int64_t)1 << 31),
                  "grid too large for the node gather (%d x %d x %d nodes)", g.nn[0], g.nn[1], g.nn[2]);
    const unsigned blocks = (unsigned)(((int64_t)g.nn[0] * g.nn[1] + 255) / 256);
    ProfileScope prof("vms_gather", st);
    if (o.rows == 3)
        hipLaunchKernelGGL((vms_gather<T, P, BX, BY, BZ, 3>), dim3(blocks, (unsigned)g.nn[2]), dim3(256), 0, st, g,
                           part, bl.nbx, bl.nby, bl.nbz, x, mask, y, o);
    else
        hipLaunchKernelGGL((vms_gather<T, P, BX, BY, BZ>), dim3(blocks, (unsigned)g.nn[2]), dim3(256), 0, st, g,
                           part, bl.nbx, bl.nby, bl.nbz, x, mask, y, o);
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
