// Hyperelastic solid block of the reduced system on gfx950 (section 2.4's
// C^lambda dR^s/dU (C^lambda)^T with the solid weak form of section 2.2, eq.
// solid_weak_form, and the nearly-incompressible neo-Hookean energy of eq. inc_neoHk:
// psi = C0/2 (tr Cbar - 3) + kappa_s/2 ((J^2 - 1)/2 - ln J), Fbar = J^{-1/3} F).
//
// The solid is a mesh of trilinear hexahedra whose nodes are the multiplier points
// (section 2.3), so the fluid sees the block through the same B / B^T kernels as the
// point stand-in.  Applied to solid-node velocities v it is
//   y = c_M M v + c_K K(U) v - c_V K_v(U) v
//   M   = int (rho_s0 - rho_f J) N_A N_B dOmega_0           (inertia, current J)
//   K   = int grad_0 N_A . dP/dF(F) . grad_0 N_B dOmega_0     (material tangent)
//   K_v = 2 mu_f int eps(N_A) : eps(N_B) dOmega_t             (subtracted viscous work)
// with F = I + grad_0 U on the reference mesh X0 and 2x2x2 Gauss points on [0,1]^3.
//
// Design
//  * Eight lanes per element, one per Gauss point (a wavefront holds 8 elements).
//    Corner positions and displacements are taken relative to corner 0 and differenced
//    in FP64, so the FP32 variant keeps its accuracy on small elements far from the
//    origin; in FP32 lane q loads corner q's values and the 8 lanes exchange them by
//    cross-lane permutes (fewer memory instructions), in FP64 each lane loads all 8
//    corners (a permute per FP64 value costs two, on a VALU-bound kernel).  A lane forms dX/dxi, F and dF = grad_0 v at its point by a loop over
//    the 8 corners, then the stress increment Q = c_K dP - c_V J sigma_v F^{-T} and the
//    inertia c_M (rho_s0 - rho_f J) v(x_q), and finally its weighted share of the 24
//    nodal forces, summed over the 8 lanes by an xor butterfly (the same bits in every lane,
//    independent of scheduling).  Lane c stores corner c's 3 sums.
//  * Element -> node: a node-parallel gather sums the corner slots of the elements
//    around each node in ascending order (CSR built once per mesh), so the result
//    is deterministic without atomics.
#include "profile.hpp"
#include "solid.hpp"

#include <vector>

namespace fsi {

namespace {

constexpr double SQ0 = 0.21132486540518711775;   // 1/2 - 1/(2 sqrt 3)
constexpr double SQ1 = 0.78867513459481288225;   // 1/2 + 1/(2 sqrt 3)

template <typename T>
struct SolidK {
    T cM, cK, cV;
    T C0, kap, rho_s0, rho_f, mu_f;
};

template <typename T>
__device__ __forceinline__ T sum8(T v)
{
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    return v;
}

// trilinear shape function of corner c (offsets (c & 1, c >> 1 & 1, c >> 2)) at xi and its
// xi-derivatives
template <typename T>
__device__ __forceinline__ void corner_shape(int c, const T xi[3], T &N, T dN[3])
{
    T f[3], df[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const bool hi = (c >> d) & 1;
        f[d] = hi ? xi[d] : T(1) - xi[d];
        df[d] = hi ? T(1) : T(-1);
    }
    N = f[0] * f[1] * f[2];
    dN[0] = df[0] * f[1] * f[2];
    dN[1] = f[0] * df[1] * f[2];
    dN[2] = f[0] * f[1] * df[2];
}

template <typename T>
__device__ __forceinline__ T det3(const T A[3][3])
{
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
           A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

// cofactor matrix: cof[i][j] = d det / d A[i][j]  (A^{-T} = cof / det)
template <typename T>
__device__ __forceinline__ void cofactor3(const T A[3][3], T C[3][3])
{
    C[0][0] = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    C[0][1] = A[1][2] * A[2][0] - A[1][0] * A[2][2];
    C[0][2] = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    C[1][0] = A[0][2] * A[2][1] - A[0][1] * A[2][2];
    C[1][1] = A[0][0] * A[2][2] - A[0][2] * A[2][0];
    C[1][2] = A[0][1] * A[2][0] - A[0][0] * A[2][1];
    C[2][0] = A[0][1] * A[1][2] - A[0][2] * A[1][1];
    C[2][1] = A[0][2] * A[1][0] - A[0][0] * A[1][2];
    C[2][2] = A[0][0] * A[1][1] - A[0][1] * A[1][0];
}

template <typename T>
__device__ __forceinline__ T cbrt_t(T x);
template <>
__device__ __forceinline__ double cbrt_t<double>(double x) { return cbrt(x); }
template <>
__device__ __forceinline__ float cbrt_t<float>(float x) { return cbrtf(x); }

// RESID = false: the tangent block applied to v.  RESID = true (FP64): the solid's nonlinear
// residual R^s = M_rho(U) A + f_int(U) - K_v(U) V with v = V and acc = A; the same element walk
// with P(F) in place of c_K dP, c_V = 1 and the inertia of A instead of c_M v.
template <typename T, bool RESID>
__global__ __launch_bounds__(256) void solid_elem_k(int64_t ne, int64_t m, const int32_t *__restrict__ conn,
                                                    const double *__restrict__ X0,
                                                    const double *__restrict__ U,
                                                    const T *__restrict__ v, const T *__restrict__ acc,
                                                    SolidK<T> k, T *__restrict__ ef)
{
    static_assert(!RESID || sizeof(T) == 8, "the residual is FP64");
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool valid = (gid >> 3) < ne;
    // lanes past the last element repeat it (their sums are not stored)
    const int64_t e = valid ? (gid >> 3) : ne - 1;
    const int q = (int)(gid & 7);
    const int lane0 = (int)(threadIdx.x & 63) & ~7;
    // FP32: lane q loads corner q's position, displacement and v (relative to corner 0, in
    // FP64) and the element's 8 lanes exchange them by cross-lane permutes.  FP64 (two
    // permutes per value on a VALU-bound kernel): every lane loads the corners itself.
    constexpr bool XCH = sizeof(T) == 4;
    const int32_t mine = conn[e * 8 + q];
    T dxm[3], dum[3], vm[3];
    int32_t nd[8];
    double xr[3], ur[3];
    if constexpr (XCH) {
        double xm[3], um[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            xm[d] = X0[d * m + mine];
            um[d] = U[d * m + mine];
            vm[d] = v[d * m + mine];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            dxm[d] = (T)(xm[d] - __shfl(xm[d], lane0, 64));
            dum[d] = (T)(um[d] - __shfl(um[d], lane0, 64));
        }
    } else {
#pragma unroll
        for (int c = 0; c < 8; ++c) nd[c] = __shfl(mine, lane0 + c, 64);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            xr[d] = X0[d * m + nd[0]];
            ur[d] = U[d * m + nd[0]];
        }
    }
    // corner c's position / displacement relative to corner 0, and its v
    auto dx_at = [&](int c, int i) -> T {
        if constexpr (XCH) return __shfl(dxm[i], lane0 + c, 64);
        else return (T)(X0[i * m + nd[c]] - xr[i]);
    };
    auto du_at = [&](int c, int i) -> T {
        if constexpr (XCH) return __shfl(dum[i], lane0 + c, 64);
        else return (T)(U[i * m + nd[c]] - ur[i]);
    };
    auto v_at = [&](int c, int i) -> T {
        if constexpr (XCH) return __shfl(vm[i], lane0 + c, 64);
        else return v[i * m + nd[c]];
    };

    const T xi[3] = {T((q & 1) ? SQ1 : SQ0), T((q & 2) ? SQ1 : SQ0), T((q & 4) ? SQ1 : SQ0)};
    // dX/dxi at the point
    T J0[3][3] = {};
#pragma unroll
    for (int c = 1; c < 8; ++c) {
        T Nc, dN[3];
        corner_shape<T>(c, xi, Nc, dN);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const T dx = dx_at(c, i);
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) J0[i][kk] += dx * dN[kk];
        }
    }
    T Ji[3][3];   // (dX/dxi)^{-1}: Ji[k][K] = dxi_k / dX_K
    const T det0 = det3(J0);
    {
        T C[3][3];
        cofactor3(J0, C);
        const T r = T(1) / det0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) Ji[a][b] = C[b][a] * r;
    }
    // F - I, dF = grad_0 v and v at the point (and A at the point for the residual)
    T F[3][3] = {}, dF[3][3] = {}, vq[3] = {}, aq[3] = {};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        T Nc, dN[3], G[3];
        corner_shape<T>(c, xi, Nc, dN);
#pragma unroll
        for (int K = 0; K < 3; ++K) G[K] = dN[0] * Ji[0][K] + dN[1] * Ji[1][K] + dN[2] * Ji[2][K];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const T du = du_at(c, i);
            const T vc = v_at(c, i);
            vq[i] += Nc * vc;
            if constexpr (RESID) aq[i] += Nc * acc[i * m + nd[c]];
#pragma unroll
            for (int K = 0; K < 3; ++K) {
                F[i][K] += du * G[K];
                dF[i][K] += vc * G[K];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) F[i][i] += T(1);
    const T J = det3(F);
    T Fit[3][3];   // F^{-T}
    {
        cofactor3(F, Fit);
        const T r = T(1) / J;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) Fit[a][b] *= r;
    }
    T I1 = T(0), tr = T(0), FdF = T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            I1 += F[a][b] * F[a][b];
            tr += Fit[a][b] * dF[a][b];
            FdF += F[a][b] * dF[a][b];
        }
    // d(F^{-T}) = -F^{-T} dF^T F^{-T}
    T dFit[3][3];
    {
        T t[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                t[i][b] = Fit[i][0] * dF[b][0] + Fit[i][1] * dF[b][1] + Fit[i][2] * dF[b][2];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int K = 0; K < 3; ++K)
                dFit[i][K] = -(t[i][0] * Fit[0][K] + t[i][1] * Fit[1][K] + t[i][2] * Fit[2][K]);
    }
    // stress increment of eq. inc_neoHk: isochoric and volumetric parts of dP (the residual:
    // P = C0 J^{-2/3} (F - I1/3 F^{-T}) + kap/2 (J^2 - 1) F^{-T})
    const T cb = cbrt_t<T>(J);
    const T a23 = T(1) / (cb * cb);           // J^{-2/3}
    const T J2 = J * J;
    const T ci = (RESID ? T(1) : k.cK) * k.C0 * a23;
    const T vol_t = RESID ? T(0) : k.cK * k.kap * J2 * tr;
    const T vol_d = (RESID ? T(1) : k.cK) * T(0.5) * k.kap * (J2 - T(1));
    // viscous stress of the velocity gradient on the current configuration:
    // grad_x v = dF F^{-1}, sigma = mu_f (grad_x v + grad_x v^T), pulled back: J sigma F^{-T}
    T L[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
            L[i][kk] = dF[i][0] * Fit[kk][0] + dF[i][1] * Fit[kk][1] + dF[i][2] * Fit[kk][2];
    T Q[3][3];
    const T cvJ = (RESID ? T(1) : k.cV) * k.mu_f * J;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int K = 0; K < 3; ++K) {
            T sv = T(0);
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) sv += (L[i][kk] + L[kk][i]) * Fit[kk][K];
            if constexpr (RESID) {
                Q[i][K] = ci * (F[i][K] - I1 * T(1.0 / 3.0) * Fit[i][K]) + vol_d * Fit[i][K] - cvJ * sv;
            } else {
                const T iso = T(-2.0 / 3.0) * tr * (F[i][K] - I1 * T(1.0 / 3.0) * Fit[i][K]) + dF[i][K] -
                              T(2.0 / 3.0) * FdF * Fit[i][K] - I1 * T(1.0 / 3.0) * dFit[i][K];
                Q[i][K] = ci * iso + vol_t * Fit[i][K] + vol_d * dFit[i][K] - cvJ * sv;
            }
        }
    const T mq = (RESID ? T(1) : k.cM) * (k.rho_s0 - k.rho_f * J);
    if constexpr (RESID) {
#pragma unroll
        for (int i = 0; i < 3; ++i) vq[i] = aq[i];   // the inertia acts on A
    }
    const T w = det0 * T(0.125);
    // nodal forces: f_c = w (Q grad_0 N_c + mq v(x_q) N_c), summed over the 8 points
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        T Nc, dN[3], G[3];
        corner_shape<T>(c, xi, Nc, dN);
#pragma unroll
        for (int K = 0; K < 3; ++K) G[K] = dN[0] * Ji[0][K] + dN[1] * Ji[1][K] + dN[2] * Ji[2][K];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const T f = w * (Q[i][0] * G[0] + Q[i][1] * G[1] + Q[i][2] * G[2] + mq * vq[i] * Nc);
            const T s = sum8(f);
            if (valid && q == c) ef[(e * 8 + c) * 3 + i] = s;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void solid_gather_k(int64_t m, const int32_t *__restrict__ start,
                                                      const int32_t *__restrict__ slot,
                                                      const T *__restrict__ ef, T *__restrict__ y)
{
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= m) return;
    T s0 = T(0), s1 = T(0), s2 = T(0);
    for (int32_t j = start[n]; j < start[n + 1]; ++j) {
        const int64_t b = (int64_t)slot[j] * 3;
        s0 += ef[b];
        s1 += ef[b + 1];
        s2 += ef[b + 2];
    }
    y[n] = s0;
    y[m + n] = s1;
    y[2 * m + n] = s2;
}

template <typename T>
int solid_apply_t(const SolidView &s, const double *U, const SolidCoefs &c, const T *v, T *y, void *ws,
                  hipStream_t st)
{
    const int64_t m = s.n_nodes, ne = s.n_elem;
    if (m == 0) return FSI_OK;
    T *ef = reinterpret_cast<T *>(ws);
    if (ne > 0) {
        SolidK<T> k;
        k.cM = (T)c.cM; k.cK = (T)c.cK; k.cV = (T)c.cV;
        k.C0 = (T)s.C0; k.kap = (T)s.kappa_s; k.rho_s0 = (T)s.rho_s0; k.rho_f = (T)s.rho_f;
        k.mu_f = (T)s.mu_f;
        ProfileScope prof("solid_elem", st);
        const unsigned blocks = (unsigned)((ne * 8 + 255) / 256);
        hipLaunchKernelGGL((solid_elem_k<T, false>), dim3(blocks), dim3(256), 0, st, ne, m, s.conn, s.X0, U, v,
                           (const T *)nullptr, k, ef);
        FSI_LAUNCH_CHECK();
    }
    ProfileScope prof("solid_gather", st);
    hipLaunchKernelGGL(solid_gather_k<T>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, m,
                       s.node_start, s.node_slot, ef, y);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

// solid state from the solid velocity V: U = Ub + cU V, A = cA V - Ab (backward Euler:
// Ub = U_n, cU = dt, Ab = V_n / dt, cA = 1 / dt)
__global__ __launch_bounds__(256) void solid_state_k(int64_t n, double cU, double cA, const double *__restrict__ Ub,
                                                     const double *__restrict__ Ab, const double *__restrict__ V,
                                                     double *__restrict__ U, double *__restrict__ A)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double vi = V[i];
    U[i] = Ub[i] + cU * vi;
    A[i] = cA * vi - Ab[i];
}

}  // namespace

int launch_solid_residual(const SolidView &s, const double *U, const double *V, const double *A, double *R,
                          void *ws, hipStream_t st)
{
    const int64_t m = s.n_nodes, ne = s.n_elem;
    if (m == 0) return FSI_OK;
    double *ef = reinterpret_cast<double *>(ws);
    if (ne > 0) {
        SolidK<double> k{};
        k.C0 = s.C0; k.kap = s.kappa_s; k.rho_s0 = s.rho_s0; k.rho_f = s.rho_f; k.mu_f = s.mu_f;
        ProfileScope prof("solid_resid", st);
        const unsigned blocks = (unsigned)((ne * 8 + 255) / 256);
        hipLaunchKernelGGL((solid_elem_k<double, true>), dim3(blocks), dim3(256), 0, st, ne, m, s.conn, s.X0, U, V,
                           A, k, ef);
        FSI_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(solid_gather_k<double>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, m,
                       s.node_start, s.node_slot, (const double *)ef, R);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int launch_solid_state(int64_t m, double cU, double cA, const double *Ub, const double *Ab, const double *V,
                       double *U, double *A, hipStream_t st)
{
    if (m == 0) return FSI_OK;
    const int64_t n = 3 * m;
    hipLaunchKernelGGL(solid_state_k, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, cU, cA, Ub, Ab, V, U,
                       A);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

size_t solid_workspace_bytes(int64_t n_elem, fsi_dtype dt)
{
    return align_up((size_t)(n_elem > 0 ? n_elem : 1) * 24 * (dt == FSI_F64 ? 8 : 4));
}

// Node -> (element, corner) table: for every node, the slots e*8 + c of the element
// corners on it, in ascending order.  Mesh set-up, once per mesh, on the host; the
// connectivity is validated here, so the kernels never see an index out of range.
int solid_build_csr(int64_t n_nodes, int64_t n_elem, const int32_t *conn, int32_t *node_start,
                    int32_t *node_slot, hipStream_t st)
{
    std::vector<int32_t> h((size_t)n_elem * 8);
    if (n_elem > 0) {
        FSI_HIP(hipMemcpyAsync(h.data(), conn, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        FSI_HIP(hipStreamSynchronize(st));
    }
    std::vector<int32_t> start((size_t)n_nodes + 1, 0), slot(h.size());
    for (size_t j = 0; j < h.size(); ++j) {
        if (h[j] < 0 || h[j] >= n_nodes) {
            set_error("connectivity entry %zu (element %zu, corner %zu) = %d is not a node index in [0, %lld)",
                      j, j / 8, j % 8, h[j], (long long)n_nodes);
            return FSI_ERR_ARG;
        }
        ++start[(size_t)h[j] + 1];
    }
    for (size_t n = 0; n < (size_t)n_nodes; ++n) start[n + 1] += start[n];
    std::vector<int32_t> fill(start.begin(), start.end() - 1);
    for (size_t j = 0; j < h.size(); ++j) slot[(size_t)fill[(size_t)h[j]]++] = (int32_t)j;
    FSI_HIP(hipMemcpyAsync(node_start, start.data(), start.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (!slot.empty())
        FSI_HIP(hipMemcpyAsync(node_slot, slot.data(), slot.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    FSI_HIP(hipStreamSynchronize(st));
    return FSI_OK;
}

int launch_solid_apply(const SolidView &s, fsi_dtype dt, const double *U, const SolidCoefs &k,
                       const void *v, void *y, void *ws, hipStream_t st)
{
    if (dt == FSI_F64)
        return solid_apply_t<double>(s, U, k, (const double *)v, (double *)y, ws, st);
    return solid_apply_t<float>(s, U, k, (const float *)v, (float *)y, ws, st);
}

}  // namespace fsi
