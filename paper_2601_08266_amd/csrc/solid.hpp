// Internal declarations of the hyperelastic solid block.
#pragma once

#include "common.hpp"

namespace fsi {

// Material and mesh of the immersed solid (all device pointers).
struct SolidView {
    int64_t n_nodes, n_elem;
    const double *X0;            // [3][n_nodes] reference positions
    const int32_t *conn;         // [n_elem][8]
    const int32_t *node_start;   // [n_nodes + 1]
    const int32_t *node_slot;    // [8 n_elem]: element corners e*8 + c around each node, ascending
    double C0, kappa_s, rho_s0, rho_f, mu_f;
};

// Time-integration coefficients of the block c_M M + c_K K(U) - c_V K_v(U).
struct SolidCoefs {
    double cM, cK, cV;
};

inline SolidView solid_view(const fsi_solid &S)
{
    return SolidView{S.n_nodes, S.n_elem,  S.X0,     S.conn,  S.node_start, S.node_slot,
                     S.C0,      S.kappa_s, S.rho_s0, S.rho_f, S.mu_f};
}

size_t solid_workspace_bytes(int64_t n_elem, fsi_dtype dt);
int solid_build_csr(int64_t n_nodes, int64_t n_elem, const int32_t *conn, int32_t *node_start,
                    int32_t *node_slot, hipStream_t st);
// y [3][n_nodes] = (c_M M + c_K K(U) - c_V K_v(U)) v, v [3][n_nodes] in precision dt
int launch_solid_apply(const SolidView &s, fsi_dtype dt, const double *U, const SolidCoefs &k,
                       const void *v, void *y, void *ws, hipStream_t st);
// R [3][n_nodes] = M_rho(U) A + f_int(U) - K_v(U) V (FP64; ws: solid_workspace_bytes(n_elem, F64))
int launch_solid_residual(const SolidView &s, const double *U, const double *V, const double *A, double *R,
                          void *ws, hipStream_t st);
// U = Ub + cU V, A = cA V - Ab over [3][m]
int launch_solid_state(int64_t m, double cU, double cA, const double *Ub, const double *Ab, const double *V,
                       double *U, double *A, hipStream_t st);

}  // namespace fsi
