// Matrix-free Q2-Q2 Oseen-VMS operator on gfx950 (section 2.1: Galerkin weak
// form + residual-based SUPG/PSPG/LSIC with the paper's tau_m, tau_c, G).
//
// Design
//  * One workgroup = a brick of 4x4x4 cells (9x9x9 nodes), processed in 8
//    rounds of a 2x2x2 group of cells.  In a round, each half-wavefront (32
//    lanes) holds one cell: lane j < 27 of it owns index j, read as a node
//    (a,b,c), an intermediate (q,b,c) / (q,q',c) or a quadrature point
//    (q,q',q'') depending on the pass.  A cell's passes exchange values only
//    among its own lanes (per-cell LDS slices, one wavefront), so they are
//    ordered by wavefront-level fences instead of workgroup barriers.
//  * Interpolation is sum-factorised through LDS: nodal values -> x-line
//    values (N, N', N'') -> xy-plane values -> quadrature-point values,
//    value/gradient/second derivatives as each field needs them (velocity:
//    all 10, pressure: 4, advection and s: values).  3 FMAs per output per
//    pass instead of 27 per output for direct evaluation.
//  * The test side is the transposed contraction: per quadrature point the
//    4 weighted flux components (value, d/dx, d/dy, d/dz) of each output
//    field go through z, y, x passes back to the 27 nodes.
//  * The 8 cells of a round park their nodal outputs in LDS; after one
//    workgroup barrier each of the round's 5x5x5 nodes adds the outputs of
//    the cells holding it in a fixed cell order to the brick's LDS node
//    accumulator (deterministic); brick faces are finished by the shared
//    node-gather kernel.
#include "kernels.hpp"
#include "profile.hpp"

namespace fsi {

namespace {

constexpr int CPR = 8;           // cells per round (one per 32-lane half-wavefront)
constexpr int BN = 2 * Q2_BX + 1;

// Orders one wavefront's LDS accesses: the stores before it are seen by the loads after it
// (lanes of one wavefront; no workgroup barrier).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 3-point Gauss-Legendre on [0,1]
constexpr double G3_0 = 0.11270166537925831148;
constexpr double G3_1 = 0.5;
constexpr double G3_2 = 0.88729833462074168852;
constexpr double W3_0 = 0.27777777777777777778;   // 5/18
constexpr double W3_1 = 0.44444444444444444444;   // 8/18

template <typename T>
struct Tab {
    T N[3][3], D[3][3], D2[3][3];   // [node a][point q]: value, first, second reference derivative
    T w[3];
};

template <typename T>
__device__ __forceinline__ void fill_tab(Tab<T> &tb, int t)
{
    if (t < 9) {
        const int a = t / 3, q = t % 3;
        const T x = q == 0 ? T(G3_0) : (q == 1 ? T(G3_1) : T(G3_2));
        T n, d, d2;
        if (a == 0) {
            n = T(2) * (x - T(0.5)) * (x - T(1)); d = T(4) * x - T(3); d2 = T(4);
        } else if (a == 1) {
            n = T(-4) * x * (x - T(1)); d = T(-8) * x + T(4); d2 = T(-8);
        } else {
            n = T(2) * x * (x - T(0.5)); d = T(4) * x - T(1); d2 = T(4);
        }
        tb.N[a][q] = n;
        tb.D[a][q] = d;
        tb.D2[a][q] = d2;
    }
    if (t == 9) {
        tb.w[0] = T(W3_0);
        tb.w[1] = T(W3_1);
        tb.w[2] = T(W3_0);
    }
}

// Interpolate one nodal field (this lane's node value v) to this lane's quadrature point.
// nder: 0 = value only, 1 = value + gradient, 2 = value + gradient + second derivatives.
// Outputs (reference derivatives): out[0] value, out[1..3] d/dxi_k, out[4..6] d2/dxi_k^2,
// out[7] d2/dxi0 dxi1, out[8] d2/dxi0 dxi2, out[9] d2/dxi1 dxi2.
template <typename T, int NDER>
__device__ __forceinline__ void interp(const Tab<T> &tb, T (*nod)[27], T (*bx)[3][27],
                                       T (*by)[6][27], int lc, int j, bool act, T v, T out[10])
{
    const int i0 = j % 3, i1 = (j / 3) % 3, i2 = j / 9;
    if (act) nod[lc][j] = v;
    wave_sync();
    // pass x: (q, b, c) <- nodes (a, b, c)
    if (act) {
        T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const T nv = nod[lc][a + 3 * i1 + 9 * i2];
            s0 += tb.N[a][i0] * nv;
            if (NDER >= 1) s1 += tb.D[a][i0] * nv;
            if (NDER >= 2) s2 += tb.D2[a][i0] * nv;
        }
        bx[lc][0][j] = s0;
        if (NDER >= 1) bx[lc][1][j] = s1;
        if (NDER >= 2) bx[lc][2][j] = s2;
    }
    wave_sync();
    // pass y: (q, q', c) <- (q, b, c); derivative orders (x, y):
    // 0:(0,0) 1:(1,0) 2:(0,1) 3:(2,0) 4:(1,1) 5:(0,2)
    if (act) {
        T r[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int src = i0 + 3 * b + 9 * i2;
            const T n = tb.N[b][i1];
            const T v0 = bx[lc][0][src];
            r[0] += n * v0;
            if (NDER >= 1) {
                const T d = tb.D[b][i1];
                const T v1 = bx[lc][1][src];
                r[1] += n * v1;
                r[2] += d * v0;
                if (NDER >= 2) {
                    r[3] += n * bx[lc][2][src];
                    r[4] += d * v1;
                    r[5] += tb.D2[b][i1] * v0;
                }
            }
        }
        by[lc][0][j] = r[0];
        if (NDER >= 1) {
            by[lc][1][j] = r[1];
            by[lc][2][j] = r[2];
        }
        if (NDER >= 2) {
            by[lc][3][j] = r[3];
            by[lc][4][j] = r[4];
            by[lc][5][j] = r[5];
        }
    }
    wave_sync();
    // pass z: (q, q', q'') <- (q, q', c)
#pragma unroll
    for (int k = 0; k < 10; ++k) out[k] = T(0);
    if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int src = i0 + 3 * i1 + 9 * c;
            const T n = tb.N[c][i2];
            out[0] += n * by[lc][0][src];
            if (NDER >= 1) {
                const T d = tb.D[c][i2];
                out[1] += n * by[lc][1][src];
                out[2] += n * by[lc][2][src];
                out[3] += d * by[lc][0][src];
                if (NDER >= 2) {
                    out[4] += n * by[lc][3][src];
                    out[5] += n * by[lc][5][src];
                    out[6] += tb.D2[c][i2] * by[lc][0][src];
                    out[7] += n * by[lc][4][src];
                    out[8] += d * by[lc][1][src];
                    out[9] += d * by[lc][2][src];
                }
            }
        }
    }
    wave_sync();
}

// Transposed contraction of one output field: this lane holds the weighted flux
// components at its quadrature point (f0 for the test value, g0..g2 for the reference
// test derivatives); returns the contribution to this lane's node.
template <typename T>
__device__ __forceinline__ T project(const Tab<T> &tb, T (*fl)[4][27], T (*bx)[3][27],
                                     T (*by)[6][27], int lc, int j, bool act, T f0, T g0, T g1,
                                     T g2)
{
    const int i0 = j % 3, i1 = (j / 3) % 3, i2 = j / 9;
    if (act) {
        fl[lc][0][j] = f0;
        fl[lc][1][j] = g0;
        fl[lc][2][j] = g1;
        fl[lc][3][j] = g2;
    }
    wave_sync();
    // z^T: (q, q', c) <- points (q, q', q'')
    if (act) {
        T p0 = T(0), p1 = T(0), p2 = T(0);
#pragma unroll
        for (int qz = 0; qz < 3; ++qz) {
            const int src = i0 + 3 * i1 + 9 * qz;
            const T n = tb.N[i2][qz];
            p0 += n * fl[lc][0][src] + tb.D[i2][qz] * fl[lc][3][src];
            p1 += n * fl[lc][1][src];
            p2 += n * fl[lc][2][src];
        }
        bx[lc][0][j] = p0;
        bx[lc][1][j] = p1;
        bx[lc][2][j] = p2;
    }
    wave_sync();
    // y^T: (q, b, c) <- (q, q', c)
    if (act) {
        T r0 = T(0), r1 = T(0);
#pragma unroll
        for (int qy = 0; qy < 3; ++qy) {
            const int src = i0 + 3 * qy + 9 * i2;
            const T n = tb.N[i1][qy];
            r0 += n * bx[lc][0][src] + tb.D[i1][qy] * bx[lc][2][src];
            r1 += n * bx[lc][1][src];
        }
        by[lc][0][j] = r0;
        by[lc][1][j] = r1;
    }
    wave_sync();
    // x^T: node (a, b, c) <- (q, b, c)
    T y = T(0);
    if (act) {
#pragma unroll
        for (int qx = 0; qx < 3; ++qx) {
            const int src = qx + 3 * i1 + 9 * i2;
            y += tb.N[i0][qx] * by[lc][0][src] + tb.D[i0][qx] * by[lc][1][src];
        }
    }
    wave_sync();
    return y;
}

// RESID = false: the linear apply with advection field a (x Dirichlet-masked); RESID = true:
// the nonlinear residual of a time step, advection by the velocity itself (a = u), `a` holds
// the source f = c_m u_old + body force, whose Galerkin/SUPG/PSPG weighting is subtracted
// (x unmasked: the gather sets the Dirichlet rows to u - g_D).
template <typename T, bool RESID>
__global__ __launch_bounds__(256, 3) void vms_q2_cells(Geo g, VmsConst<T> k, const T *__restrict__ x,
                                                    const T *__restrict__ a,
                                                    const T *__restrict__ s,
                                                    const uint32_t *__restrict__ mask,
                                                    const T *__restrict__ gram,
                                                    const int32_t *__restrict__ occ_index,
                                                    T *__restrict__ part, int nbx, int nby)
{
    __shared__ T acc[4 * Q2_NL];
    __shared__ T nod[CPR][27];
    __shared__ T nodu[CPR][3][27];
    __shared__ T bx[CPR][3][27];
    __shared__ T by[CPR][6][27];
    __shared__ T fl[CPR][4][27];   // the projections' fluxes, then the round's nodal outputs
    __shared__ T smin_s[CPR];
    __shared__ Tab<T> tb;

    const int t = threadIdx.x;
    const int64_t bid = blockIdx.x;
    const int bxi = (int)(bid % nbx), byi = (int)((bid / nbx) % nby), bzi = (int)(bid / ((int64_t)nbx * nby));
    const int lc = t / 32, j = t % 32;
    const bool lane_on = j < 27;
    fill_tab(tb, t);
    for (int i = t; i < 4 * Q2_NL; i += 256) acc[i] = T(0);
    __syncthreads();

    const int64_t N = g.N;
    const int na = j % 3, nb = (j / 3) % 3, nc = j / 9;   // this lane's node in its cell
    // this lane's node values of round r (x with the Dirichlet mask applied later, a, s), loaded
    // one round ahead so their latency hides behind the previous round's arithmetic
    auto load_round = [&](int r, T v[8]) {
        const int cxl = 2 * (r & 1) + (lc & 1), cyl = 2 * ((r >> 1) & 1) + ((lc >> 1) & 1),
                  czl = 2 * (r >> 2) + (lc >> 2);
        const int cx = bxi * Q2_BX + cxl, cy = byi * Q2_BY + cyl, cz = bzi * Q2_BZ + czl;
#pragma unroll
        for (int f = 0; f < 7; ++f) v[f] = T(0);
        v[7] = T(1);
        if (lane_on && cx < g.n[0] && cy < g.n[1] && cz < g.n[2]) {
            const int64_t node = (int64_t)(2 * cx + na) +
                                 (int64_t)g.nn[0] * ((2 * cy + nb) + (int64_t)g.nn[1] * (2 * cz + nc));
#pragma unroll
            for (int f = 0; f < 4; ++f) v[f] = x[f * N + node];
#pragma unroll
            for (int f = 0; f < 3; ++f) v[4 + f] = a[f * N + node];
            if (k.has_s) v[7] = s[node];
        }
    };
    T vnext[8];
    load_round(0, vnext);
    for (int r = 0; r < 8; ++r) {
        const int cxl = 2 * (r & 1) + (lc & 1), cyl = 2 * ((r >> 1) & 1) + ((lc >> 1) & 1),
                  czl = 2 * (r >> 2) + (lc >> 2);
        const int cx = bxi * Q2_BX + cxl, cy = byi * Q2_BY + cyl, cz = bzi * Q2_BZ + czl;
        const bool act = lane_on && cx < g.n[0] && cy < g.n[1] && cz < g.n[2];
        T v[8];
#pragma unroll
        for (int f = 0; f < 8; ++f) v[f] = vnext[f];
        if (r + 1 < 8) load_round(r + 1, vnext);
        if (act) {
            const int64_t node = (int64_t)(2 * cx + na) +
                                 (int64_t)g.nn[0] * ((2 * cy + nb) + (int64_t)g.nn[1] * (2 * cz + nc));
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                if (!RESID && mask_bit(mask, f * N + node)) v[f] = T(0);
                nodu[lc][f][j] = v[f];
            }
        }
        // quadrature-point values
        T qu[3][10], qp[10], qa[3][10], qs[10];
        interp<T, 2>(tb, nod, bx, by, lc, j, act, v[0], qu[0]);
        interp<T, 2>(tb, nod, bx, by, lc, j, act, v[1], qu[1]);
        interp<T, 2>(tb, nod, bx, by, lc, j, act, v[2], qu[2]);
        interp<T, 1>(tb, nod, bx, by, lc, j, act, v[3], qp);
        interp<T, 0>(tb, nod, bx, by, lc, j, act, v[4], qa[0]);
        interp<T, 0>(tb, nod, bx, by, lc, j, act, v[5], qa[1]);
        interp<T, 0>(tb, nod, bx, by, lc, j, act, v[6], qa[2]);
        T S = T(1);
        if (k.has_s) {
            if (act) nod[lc][j] = v[7];
            wave_sync();
            if (act && j == 0) {
                T m = nod[lc][0];
                for (int i = 1; i < 27; ++i) m = nod[lc][i] < m ? nod[lc][i] : m;
                smin_s[lc] = m;
            }
            wave_sync();
            interp<T, 0>(tb, nod, bx, by, lc, j, act, v[7], qs);
            if (act) S = qs[0] < smin_s[lc] ? smin_s[lc] : qs[0];
        }

        // pointwise quantities at quadrature point (i0, i1, i2) = (j%3, (j/3)%3, j/9)
        T F0[4], G[4][3];
        {
            const T ih[3] = {k.ih[0], k.ih[1], k.ih[2]};
            T U[3], dU[3][3], lap[3], hes[3][3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                U[i] = qu[i][0];
#pragma unroll
                for (int d = 0; d < 3; ++d) dU[i][d] = qu[i][1 + d] * ih[d];
                hes[i][0][0] = qu[i][4] * k.ih2[0];
                hes[i][1][1] = qu[i][5] * k.ih2[1];
                hes[i][2][2] = qu[i][6] * k.ih2[2];
                hes[i][0][1] = hes[i][1][0] = qu[i][7] * (ih[0] * ih[1]);
                hes[i][0][2] = hes[i][2][0] = qu[i][8] * (ih[0] * ih[2]);
                hes[i][1][2] = hes[i][2][1] = qu[i][9] * (ih[1] * ih[2]);
                lap[i] = hes[i][0][0] + hes[i][1][1] + hes[i][2][2];
            }
            const T P = qp[0];
            const T dP[3] = {qp[1] * ih[0], qp[2] * ih[1], qp[3] * ih[2]};
            // advection: the field a, or (residual) the velocity itself with the source f
            const T Aq[3] = {RESID ? U[0] : qa[0][0], RESID ? U[1] : qa[1][0], RESID ? U[2] : qa[2][0]};
            const T Fs[3] = {RESID ? qa[0][0] : T(0), RESID ? qa[1][0] : T(0), RESID ? qa[2][0] : T(0)};
            const T tbk = S * (k.K1 + Aq[0] * Aq[0] * k.ih2[0] + Aq[1] * Aq[1] * k.ih2[1] +
                               Aq[2] * Aq[2] * k.ih2[2]);
            const T sq = sqrt(tbk);
            const T tau_m = T(1) / sq;
            const T tau_c = sq * k.inv_trG;
            const T div = dU[0][0] + dU[1][1] + dU[2][2];
            T tr[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                T gi = k.c_m * U[i] + (Aq[0] * dU[i][0] + Aq[1] * dU[i][1] + Aq[2] * dU[i][2]);
                if constexpr (RESID) gi -= Fs[i];
                F0[i] = gi;
                T visc = T(0);
                if (k.visc_strong) visc = lap[i] + (hes[0][i][0] + hes[1][i][1] + hes[2][i][2]);
                tr[i] = tau_m * (gi + dP[i] - k.nu * visc);
            }
            const T diag = tau_c * div - P;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    T fl2 = k.nu * (dU[i][d] + dU[d][i]) + Aq[d] * tr[i];
                    if (d == i) fl2 += diag;
                    G[i][d] = fl2;
                }
            F0[3] = div;
            G[3][0] = tr[0];
            G[3][1] = tr[1];
            G[3][2] = tr[2];
        }
        const int q0 = j % 3, q1 = (j / 3) % 3, q2 = j / 9;
        const T W = act ? tb.w[q0] * tb.w[q1] * tb.w[q2] * k.detJ : T(0);
        T out[4];
#pragma unroll
        for (int f = 0; f < 4; ++f)
            out[f] = project(tb, fl, bx, by, lc, j, act, W * F0[f], W * k.ih[0] * G[f][0],
                             W * k.ih[1] * G[f][1], W * k.ih[2] * G[f][2]);
        // DLM block of an occupied cell on its nodal (masked) velocity
        if (act && gram != nullptr) {
            const int32_t ko = occ_index[cx + (int64_t)g.n[0] * (cy + (int64_t)g.n[1] * cz)];
            if (ko >= 0) {
                const T *gr = gram + ((int64_t)ko * 27 + j) * 27;
                T r0 = T(0), r1 = T(0), r2 = T(0);
                for (int C = 0; C < 27; ++C) {
                    const T gv = gr[C];
                    r0 += gv * nodu[lc][0][C];
                    r1 += gv * nodu[lc][1][C];
                    r2 += gv * nodu[lc][2][C];
                }
                out[0] += r0;
                out[1] += r1;
                out[2] += r2;
            }
        }
        // ordered accumulation of the round's 8 cells into the brick's nodes: each node of the
        // round's 5x5x5 group adds the outputs of the cells holding it in cell order
        // (the last projection ended with this wavefront's fence, so its cell's slice of fl is free)
        if (lane_on) {
#pragma unroll
            for (int f = 0; f < 4; ++f) fl[lc][f][j] = act ? out[f] : T(0);
        }
        __syncthreads();
        if (t < 125) {
            const int gx = t % 5, gy = (t / 5) % 5, gz = t / 25;
            T sum[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int ck = 0; ck < 2; ++ck) {
                const int lz = gz - 2 * ck;
                if (lz < 0 || lz > 2) continue;
#pragma unroll
                for (int cj = 0; cj < 2; ++cj) {
                    const int ly = gy - 2 * cj;
                    if (ly < 0 || ly > 2) continue;
#pragma unroll
                    for (int ci = 0; ci < 2; ++ci) {
                        const int lx = gx - 2 * ci;
                        if (lx < 0 || lx > 2) continue;
                        const int cell = ci + 2 * cj + 4 * ck;
                        const int jn = lx + 3 * ly + 9 * lz;
#pragma unroll
                        for (int f = 0; f < 4; ++f) sum[f] += fl[cell][f][jn];
                    }
                }
            }
            const int l = (4 * (r & 1) + gx) + BN * ((4 * ((r >> 1) & 1) + gy) + BN * (4 * (r >> 2) + gz));
#pragma unroll
            for (int f = 0; f < 4; ++f) acc[f * Q2_NL + l] += sum[f];
        }
        __syncthreads();
    }
    for (int l = t; l < Q2_NL; l += 256) {
        const int lx = l % BN, ly = (l / BN) % BN, lz = l / (BN * BN);
        const int gx = 2 * bxi * Q2_BX + lx, gy = 2 * byi * Q2_BY + ly, gz = 2 * bzi * Q2_BZ + lz;
        if (gx < g.nn[0] && gy < g.nn[1] && gz < g.nn[2]) {
            // bricks of one parity class never share a node: one array per class
            const PartIndex pi(g.nn, nbx, 2 * Q2_BX);
            T *pc = part + pi.at((bxi & 1) + 2 * (byi & 1) + 4 * (bzi & 1), bxi, gx, gy, gz);
#pragma unroll
            for (int f = 0; f < 4; ++f) pc[f * pi.field] = acc[f * Q2_NL + l];
        }
    }
}

}  // namespace

template <typename T>
int launch_q2_cells(const Geo &g, const VmsConst<T> &k, const T *x, const T *a, const T *s,
                    const uint32_t *mask, const T *gram, const int32_t *occ_index, T *part,
                    const BrickLayout &bl, hipStream_t st, bool resid)
{
    ProfileScope prof(resid ? "vms_q2_residual" : "vms_q2_cells", st);
    if (resid)
        hipLaunchKernelGGL((vms_q2_cells<T, true>), dim3((unsigned)bl.nb), dim3(256), 0, st, g, k, x, a, s, mask,
                           gram, occ_index, part, bl.nbx, bl.nby);
    else
        hipLaunchKernelGGL((vms_q2_cells<T, false>), dim3((unsigned)bl.nb), dim3(256), 0, st, g, k, x, a, s, mask,
                           gram, occ_index, part, bl.nbx, bl.nby);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

template int launch_q2_cells<double>(const Geo &, const VmsConst<double> &, const double *,
                                     const double *, const double *, const uint32_t *,
                                     const double *, const int32_t *, double *,
                                     const BrickLayout &, hipStream_t, bool);
template int launch_q2_cells<float>(const Geo &, const VmsConst<float> &, const float *,
                                    const float *, const float *, const uint32_t *, const float *,
                                    const int32_t *, float *, const BrickLayout &, hipStream_t, bool);

}  // namespace fsi
