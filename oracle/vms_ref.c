/*
 * CPU reference ("oracle") of the VMS-stabilised Oseen operator used by the
 * immersed FD/DLM method.  TEST INFRASTRUCTURE ONLY: it is called by the test
 * suite, by the smoke check and by the CPU-baseline leg of the benchmark, and
 * never by the product path.  It shares no code with the HIP library.
 *
 * What it computes, written the slow and obvious way (plain FP64, explicit
 * dense element matrices, y = sum_e P_e^T K_e P_e x):
 *
 *  Galerkin part: the incompressible Navier-Stokes weak form of section 2.1
 *  (eq. fluid_weak_form) per unit density, linearised about a given advection
 *  field a (Oseen) and discretised in time with a mass coefficient c_m:
 *      c_m w.u + w.(a.grad)u + 2 nu eps(w):eps(u) - (div w) p + q div u
 *  VMS part (the paper omits the weak form; the residual-based SUPG/PSPG/LSIC
 *  reading of the cited VMS method is used):
 *      + tau_m ((a.grad)w + grad q) . r_m(u,p) + tau_c (div w)(div u),
 *      r_m = c_m u + (a.grad)u + grad p - nu (lap u + grad div u)
 *  with tau_m, tau_c and G exactly as the stabilisation-parameter equations of
 *  section 2.1 (s multiplies the whole bracket, rho = 1 so mu/rho = nu).
 *
 * Discretisation: uniform hex cells, reference element [0,1]^3, map
 * x = x_cell + h xi, equispaced Lagrange basis of order p (1 or 2), tensor
 * Gauss-Legendre quadrature, a and s interpolated with the same basis.
 *
 * Local numbering: node A = ax + (p+1)(ay + (p+1) az); local DOF = f*nen + A
 * with f = 0,1,2 (velocity components) and 3 (pressure).
 * Global numbering: node id = i + Nx (j + Ny k), vectors stored field-major
 * [4][N] (velocity [3][N] for a and the mask).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MASS 1u
#define OR_CONV 2u
#define OR_VISC 4u
#define OR_PDIV 8u
#define OR_CONT 16u
#define OR_SUPG 32u
#define OR_PSPG 64u
#define OR_LSIC 128u
#define OR_ALL 255u

/* Gauss-Legendre rule with nq points mapped from [-1,1] to [0,1]. */
static int gauss01(int nq, double *pt, double *wt)
{
    double x[4], w[4];
    if (nq == 1) {
        x[0] = 0.0; w[0] = 2.0;
    } else if (nq == 2) {
        x[0] = -1.0 / sqrt(3.0); x[1] = -x[0];
        w[0] = w[1] = 1.0;
    } else if (nq == 3) {
        x[0] = -sqrt(3.0 / 5.0); x[1] = 0.0; x[2] = -x[0];
        w[0] = w[2] = 5.0 / 9.0; w[1] = 8.0 / 9.0;
    } else if (nq == 4) {
        double a = sqrt(3.0 / 7.0 - 2.0 / 7.0 * sqrt(6.0 / 5.0));
        double b = sqrt(3.0 / 7.0 + 2.0 / 7.0 * sqrt(6.0 / 5.0));
        x[0] = -b; x[1] = -a; x[2] = a; x[3] = b;
        w[1] = w[2] = (18.0 + sqrt(30.0)) / 36.0;
        w[0] = w[3] = (18.0 - sqrt(30.0)) / 36.0;
    } else {
        return -1;
    }
    for (int i = 0; i < nq; ++i) {
        pt[i] = 0.5 * (x[i] + 1.0);
        wt[i] = 0.5 * w[i];
    }
    return 0;
}

/* 1D Lagrange basis on equispaced nodes k/p of [0,1]: values, first and second derivatives. */
static void lagrange1d(int p, double t, double *N, double *dN, double *d2N)
{
    if (p == 1) {
        N[0] = 1.0 - t;  dN[0] = -1.0; d2N[0] = 0.0;
        N[1] = t;        dN[1] = 1.0;  d2N[1] = 0.0;
    } else {
        N[0] = 2.0 * (t - 0.5) * (t - 1.0); dN[0] = 4.0 * t - 3.0;  d2N[0] = 4.0;
        N[1] = -4.0 * t * (t - 1.0);        dN[1] = -8.0 * t + 4.0; d2N[1] = -8.0;
        N[2] = 2.0 * t * (t - 0.5);         dN[2] = 4.0 * t - 1.0;  d2N[2] = 4.0;
    }
}

typedef struct {
    double N[27];
    double dN[27][3];       /* physical first derivatives */
    double d2N[27][3][3];   /* physical second derivatives */
} shape_t;

/* Shape functions of the (p+1)^3 element nodes at reference point xi. */
static void shape3d(int p, const double *h, const double *xi, shape_t *S)
{
    double n[3][3], d[3][3], dd[3][3];
    for (int k = 0; k < 3; ++k) lagrange1d(p, xi[k], n[k], d[k], dd[k]);
    int q = p + 1;
    for (int az = 0; az < q; ++az)
        for (int ay = 0; ay < q; ++ay)
            for (int ax = 0; ax < q; ++ax) {
                int A = ax + q * (ay + q * az);
                int idx[3] = {ax, ay, az};
                S->N[A] = n[0][ax] * n[1][ay] * n[2][az];
                for (int i = 0; i < 3; ++i) {
                    double v = 1.0;
                    for (int k = 0; k < 3; ++k) v *= (k == i) ? d[k][idx[k]] / h[k] : n[k][idx[k]];
                    S->dN[A][i] = v;
                }
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        double v = 1.0;
                        for (int k = 0; k < 3; ++k) {
                            int order = (k == i) + (k == j);
                            double f = order == 0 ? n[k][idx[k]]
                                     : order == 1 ? d[k][idx[k]] / h[k]
                                                  : dd[k][idx[k]] / (h[k] * h[k]);
                            v *= f;
                        }
                        S->d2N[A][i][j] = v;
                    }
            }
}

/*
 * s at a quadrature point: interpolated with the element basis (section 2.1
 * interpolates s with the pressure space) and clamped below by the smallest
 * nodal s of the cell.  For Q1 the interpolant is a convex combination and the
 * clamp is inactive; for Q2 the basis has negative lobes, so a jump in the
 * nodal s (1 next to s_max) would otherwise produce s <= 0 and no real tau_m.
 */
static double clamp_s(double sq, const double *s_e, int nen)
{
    if (!s_e) return sq;
    double lo = s_e[0];
    for (int A = 1; A < nen; ++A) lo = s_e[A] < lo ? s_e[A] : lo;
    return sq < lo ? lo : sq;
}

/* tau_m and tau_c of section 2.1 for a uniform Cartesian cell: G = diag(1/h^2). */
static void stab_params(const double *h, const double *prm, const double *aq, double sq,
                        double *tau_m, double *tau_c)
{
    const double nu = prm[0], dt = prm[2], C_T = prm[3], C_I = prm[4];
    double G[3][3] = {{0}};
    for (int i = 0; i < 3; ++i) G[i][i] = 1.0 / (h[i] * h[i]);
    double aGa = 0.0, GG = 0.0, trG = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            aGa += aq[i] * G[i][j] * aq[j];
            GG += G[i][j] * G[i][j];
        }
    for (int i = 0; i < 3; ++i) trG += G[i][i];
    double bracket = C_T / (dt * dt) + aGa + C_I * nu * nu * GG;
    *tau_m = 1.0 / sqrt(sq * bracket);
    *tau_c = 1.0 / (*tau_m * trG);
}

/*
 * Dense element matrix K (row-major, (4 nen)^2), rows = test DOFs, columns =
 * trial DOFs.  prm = {nu, c_m, dt, C_T, C_I}.  a_e = [3][nen] nodal advection,
 * s_e = [nen] nodal interface scaling or NULL (s = 1).  terms selects which
 * groups of the bilinear form are included (OR_* flags); visc_strong != 0
 * keeps the viscous second-derivative term in the strong residual.
 * nq = Gauss points per direction (0 means p+1).
 */
int oracle_element_matrix(int p, const double *h, const double *prm, int visc_strong, int nq,
                          const double *a_e, const double *s_e, unsigned terms, double *K)
{
    if (p != 1 && p != 2) return -1;
    if (nq == 0) nq = p + 1;
    const int q = p + 1, nen = q * q * q, nd = 4 * nen;
    const double nu = prm[0], c_m = prm[1];
    double pt[4], wt[4];
    if (gauss01(nq, pt, wt)) return -1;
    memset(K, 0, sizeof(double) * (size_t)nd * nd);
    const double detJ = h[0] * h[1] * h[2];
    shape_t S;
    for (int qz = 0; qz < nq; ++qz)
        for (int qy = 0; qy < nq; ++qy)
            for (int qx = 0; qx < nq; ++qx) {
                double xi[3] = {pt[qx], pt[qy], pt[qz]};
                double W = wt[qx] * wt[qy] * wt[qz] * detJ;
                shape3d(p, h, xi, &S);
                double aq[3] = {0, 0, 0}, sq = 0.0;
                for (int A = 0; A < nen; ++A) {
                    for (int d = 0; d < 3; ++d) aq[d] += S.N[A] * a_e[d * nen + A];
                    sq += S.N[A] * (s_e ? s_e[A] : 1.0);
                }
                sq = clamp_s(sq, s_e, nen);
                double tau_m, tau_c;
                stab_params(h, prm, aq, sq, &tau_m, &tau_c);
                double adN[27], lapN[27];
                for (int A = 0; A < nen; ++A) {
                    adN[A] = aq[0] * S.dN[A][0] + aq[1] * S.dN[A][1] + aq[2] * S.dN[A][2];
                    lapN[A] = S.d2N[A][0][0] + S.d2N[A][1][1] + S.d2N[A][2][2];
                }
                for (int A = 0; A < nen; ++A)
                    for (int B = 0; B < nen; ++B) {
                        double gAgB = S.dN[A][0] * S.dN[B][0] + S.dN[A][1] * S.dN[B][1]
                                    + S.dN[A][2] * S.dN[B][2];
                        /* velocity test (A,i) x velocity trial (B,j) */
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j) {
                                double v = 0.0;
                                if (i == j) {
                                    if (terms & OR_MASS) v += c_m * S.N[A] * S.N[B];
                                    if (terms & OR_CONV) v += S.N[A] * adN[B];
                                    if (terms & OR_VISC) v += nu * gAgB;
                                }
                                if (terms & OR_VISC) v += nu * S.dN[A][j] * S.dN[B][i];
                                if (terms & OR_LSIC) v += tau_c * S.dN[A][i] * S.dN[B][j];
                                if (terms & OR_SUPG) {
                                    double r = (i == j) ? c_m * S.N[B] + adN[B] : 0.0;
                                    if (visc_strong)
                                        r -= nu * (((i == j) ? lapN[B] : 0.0) + S.d2N[B][i][j]);
                                    v += tau_m * adN[A] * r;
                                }
                                K[(size_t)(i * nen + A) * nd + (j * nen + B)] += W * v;
                            }
                        /* velocity test (A,i) x pressure trial B */
                        for (int i = 0; i < 3; ++i) {
                            double v = 0.0;
                            if (terms & OR_PDIV) v -= S.dN[A][i] * S.N[B];
                            if (terms & OR_SUPG) v += tau_m * adN[A] * S.dN[B][i];
                            K[(size_t)(i * nen + A) * nd + (3 * nen + B)] += W * v;
                        }
                        /* pressure test A x velocity trial (B,j) */
                        for (int j = 0; j < 3; ++j) {
                            double v = 0.0;
                            if (terms & OR_CONT) v += S.N[A] * S.dN[B][j];
                            if (terms & OR_PSPG) {
                                double r = S.dN[A][j] * (c_m * S.N[B] + adN[B]);
                                if (visc_strong) {
                                    double t = S.dN[A][j] * lapN[B];
                                    for (int i = 0; i < 3; ++i) t += S.dN[A][i] * S.d2N[B][i][j];
                                    r -= nu * t;
                                }
                                v += tau_m * r;
                            }
                            K[(size_t)(3 * nen + A) * nd + (j * nen + B)] += W * v;
                        }
                        /* pressure test A x pressure trial B */
                        if (terms & OR_PSPG)
                            K[(size_t)(3 * nen + A) * nd + (3 * nen + B)] += W * tau_m * gAgB;
                    }
            }
    return 0;
}

/*
 * Source weighting matrix L ((4 nen) x (3 nen), row-major): the Galerkin,
 * SUPG and PSPG test functions applied to a nodal body-force-like field f
 * (f = c_m u_old + body force in a time step), i.e. the load
 *   int w.f + tau_m ((a.grad)w + grad q).f.
 * terms selects the test functions (OR_SRC_* flags; OR_SRC_ALL for the load
 * of the method).
 */
#define OR_SRC_GAL 1u
#define OR_SRC_SUPG 2u
#define OR_SRC_PSPG 4u
#define OR_SRC_ALL 7u
int oracle_source_matrix(int p, const double *h, const double *prm, int nq,
                         const double *a_e, const double *s_e, unsigned terms, double *L)
{
    if (p != 1 && p != 2) return -1;
    if (nq == 0) nq = p + 1;
    const int q = p + 1, nen = q * q * q, nr = 4 * nen, nc = 3 * nen;
    double pt[4], wt[4];
    if (gauss01(nq, pt, wt)) return -1;
    memset(L, 0, sizeof(double) * (size_t)nr * nc);
    const double detJ = h[0] * h[1] * h[2];
    shape_t S;
    for (int qz = 0; qz < nq; ++qz)
        for (int qy = 0; qy < nq; ++qy)
            for (int qx = 0; qx < nq; ++qx) {
                double xi[3] = {pt[qx], pt[qy], pt[qz]};
                double W = wt[qx] * wt[qy] * wt[qz] * detJ;
                shape3d(p, h, xi, &S);
                double aq[3] = {0, 0, 0}, sq = 0.0;
                for (int A = 0; A < nen; ++A) {
                    for (int d = 0; d < 3; ++d) aq[d] += S.N[A] * a_e[d * nen + A];
                    sq += S.N[A] * (s_e ? s_e[A] : 1.0);
                }
                sq = clamp_s(sq, s_e, nen);
                double tau_m, tau_c;
                stab_params(h, prm, aq, sq, &tau_m, &tau_c);
                for (int A = 0; A < nen; ++A) {
                    double adNA = aq[0] * S.dN[A][0] + aq[1] * S.dN[A][1] + aq[2] * S.dN[A][2];
                    const double gal = (terms & OR_SRC_GAL) ? S.N[A] : 0.0;
                    const double supg = (terms & OR_SRC_SUPG) ? tau_m * adNA : 0.0;
                    const double pspg = (terms & OR_SRC_PSPG) ? tau_m : 0.0;
                    for (int B = 0; B < nen; ++B) {
                        for (int i = 0; i < 3; ++i)
                            L[(size_t)(i * nen + A) * nc + (i * nen + B)] +=
                                W * (gal * S.N[B] + supg * S.N[B]);
                        for (int j = 0; j < 3; ++j)
                            L[(size_t)(3 * nen + A) * nc + (j * nen + B)] +=
                                W * pspg * S.dN[A][j] * S.N[B];
                    }
                }
            }
    return 0;
}

/* Global node ids of cell (cx,cy,cz). */
static void cell_nodes(const int *n, int p, int64_t cx, int64_t cy, int64_t cz, int64_t *ids)
{
    const int q = p + 1;
    const int64_t Nx = (int64_t)p * n[0] + 1, Ny = (int64_t)p * n[1] + 1;
    for (int az = 0; az < q; ++az)
        for (int ay = 0; ay < q; ++ay)
            for (int ax = 0; ax < q; ++ax)
                ids[ax + q * (ay + q * az)] = (p * cx + ax) + Nx * ((p * cy + ay) + Ny * (p * cz + az));
}

static void gather_cell(int p, int64_t N, const int64_t *ids, const double *a, const double *s,
                        const uint8_t *dmask, const double *x, double *a_e, double *s_e,
                        double *x_e)
{
    const int q = p + 1, nen = q * q * q;
    for (int A = 0; A < nen; ++A) {
        int64_t g = ids[A];
        for (int d = 0; d < 3; ++d) a_e[d * nen + A] = a[d * N + g];
        if (s) s_e[A] = s[g];
        if (x) {
            for (int f = 0; f < 4; ++f) {
                double v = x[f * N + g];
                if (f < 3 && dmask && dmask[f * N + g]) v = 0.0;   /* Dirichlet columns */
                x_e[f * nen + A] = v;
            }
        }
    }
}

/*
 * y = A x over the whole grid (n cells per axis, order p, cell size h).
 * dmask (bytes, [3][N], nonzero = Dirichlet velocity DOF) or NULL: masked
 * columns are zeroed before the apply and masked rows return x.
 */
int oracle_vms_apply(const int *n, int p, const double *h, const double *prm, int visc_strong,
                     const double *a, const double *s, const uint8_t *dmask, const double *x,
                     double *y)
{
    if (p != 1 && p != 2) return -1;
    const int q = p + 1, nen = q * q * q, nd = 4 * nen;
    const int64_t Nx = (int64_t)p * n[0] + 1, Ny = (int64_t)p * n[1] + 1, Nz = (int64_t)p * n[2] + 1;
    const int64_t N = Nx * Ny * Nz;
    const int64_t E = (int64_t)n[0] * n[1] * n[2];
    double *ye = (double *)malloc(sizeof(double) * (size_t)E * nd);
    if (!ye) return -2;
    int err = 0;
#pragma omp parallel
    {
        double *K = (double *)malloc(sizeof(double) * (size_t)nd * nd);
        double a_e[81], s_e[27], x_e[108];
        int64_t ids[27];
        if (!K) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(static)
        for (int64_t e = 0; e < E; ++e) {
            if (!K) continue;
            int64_t cx = e % n[0], cy = (e / n[0]) % n[1], cz = e / ((int64_t)n[0] * n[1]);
            cell_nodes(n, p, cx, cy, cz, ids);
            gather_cell(p, N, ids, a, s, dmask, x, a_e, s_e, x_e);
            oracle_element_matrix(p, h, prm, visc_strong, 0, a_e, s ? s_e : NULL, OR_ALL, K);
            for (int r = 0; r < nd; ++r) {
                double acc = 0.0;
                for (int c = 0; c < nd; ++c) acc += K[(size_t)r * nd + c] * x_e[c];
                ye[(size_t)e * nd + r] = acc;
            }
        }
        free(K);
    }
    if (err) {
        free(ye);
        return err;
    }
    memset(y, 0, sizeof(double) * (size_t)(4 * N));
    int64_t ids[27];
    for (int64_t e = 0; e < E; ++e) {
        int64_t cx = e % n[0], cy = (e / n[0]) % n[1], cz = e / ((int64_t)n[0] * n[1]);
        cell_nodes(n, p, cx, cy, cz, ids);
        for (int f = 0; f < 4; ++f)
            for (int A = 0; A < nen; ++A) y[f * N + ids[A]] += ye[(size_t)e * nd + f * nen + A];
    }
    if (dmask)
        for (int64_t i = 0; i < 3 * N; ++i)
            if (dmask[i]) y[i] = x[i];
    free(ye);
    return 0;
}

/*
 * Selected entries of y = A x: rows[r] = f*N + node.  Each row is the sum over
 * the cells containing the node of (K_e x_e)[f*nen + A].  Used to check a
 * full-size apply at sampled outputs.
 */
int oracle_vms_rows(const int *n, int p, const double *h, const double *prm, int visc_strong,
                    const double *a, const double *s, const uint8_t *dmask, const double *x,
                    const int64_t *rows, int64_t nrows, double *out)
{
    if (p != 1 && p != 2) return -1;
    const int q = p + 1, nen = q * q * q, nd = 4 * nen;
    const int64_t Nx = (int64_t)p * n[0] + 1, Ny = (int64_t)p * n[1] + 1, Nz = (int64_t)p * n[2] + 1;
    const int64_t N = Nx * Ny * Nz;
    int err = 0;
#pragma omp parallel
    {
        double *K = (double *)malloc(sizeof(double) * (size_t)nd * nd);
        double a_e[81], s_e[27], x_e[108];
        int64_t ids[27];
        if (!K) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < nrows; ++r) {
            if (!K) continue;
            int64_t row = rows[r];
            int f = (int)(row / N);
            int64_t g = row % N;
            int64_t gi[3] = {g % Nx, (g / Nx) % Ny, g / (Nx * Ny)};
            if (f < 3 && dmask && dmask[row]) {
                out[r] = x[row];
                continue;
            }
            double acc = 0.0;
            int64_t lo[3], hi[3];
            for (int d = 0; d < 3; ++d) {
                lo[d] = (gi[d] - p + p - 1) / p;   /* ceil((g - p) / p) for g >= 0 */
                if (gi[d] - p < 0) lo[d] = 0;
                hi[d] = gi[d] / p;
                if (hi[d] > n[d] - 1) hi[d] = n[d] - 1;
            }
            for (int64_t cz = lo[2]; cz <= hi[2]; ++cz)
                for (int64_t cy = lo[1]; cy <= hi[1]; ++cy)
                    for (int64_t cx = lo[0]; cx <= hi[0]; ++cx) {
                        int A = (int)((gi[0] - p * cx) + q * ((gi[1] - p * cy) + q * (gi[2] - p * cz)));
                        cell_nodes(n, p, cx, cy, cz, ids);
                        gather_cell(p, N, ids, a, s, dmask, x, a_e, s_e, x_e);
                        oracle_element_matrix(p, h, prm, visc_strong, 0, a_e, s ? s_e : NULL,
                                              OR_ALL, K);
                        const double *Kr = K + (size_t)(f * nen + A) * nd;
                        for (int c = 0; c < nd; ++c) acc += Kr[c] * x_e[c];
                    }
            out[r] = acc;
        }
        free(K);
    }
    return err;
}

/*
 * Nodal 4x4 diagonal blocks of A: blocks[node][4][4] (row = test field,
 * column = trial field), summed over the cells containing the node.  Dirichlet
 * velocity rows/columns are replaced by identity rows/columns.
 */
int oracle_vms_diag_blocks(const int *n, int p, const double *h, const double *prm,
                           int visc_strong, const double *a, const double *s,
                           const uint8_t *dmask, double *blocks)
{
    if (p != 1 && p != 2) return -1;
    const int q = p + 1, nen = q * q * q, nd = 4 * nen;
    const int64_t Nx = (int64_t)p * n[0] + 1, Ny = (int64_t)p * n[1] + 1, Nz = (int64_t)p * n[2] + 1;
    const int64_t N = Nx * Ny * Nz;
    const int64_t E = (int64_t)n[0] * n[1] * n[2];
    double *be = (double *)malloc(sizeof(double) * (size_t)E * nen * 16);
    if (!be) return -2;
#pragma omp parallel
    {
        double *K = (double *)malloc(sizeof(double) * (size_t)nd * nd);
        double a_e[81], s_e[27];
        int64_t ids[27];
#pragma omp for schedule(static)
        for (int64_t e = 0; e < E; ++e) {
            if (!K) continue;
            int64_t cx = e % n[0], cy = (e / n[0]) % n[1], cz = e / ((int64_t)n[0] * n[1]);
            cell_nodes(n, p, cx, cy, cz, ids);
            gather_cell(p, N, ids, a, s, NULL, NULL, a_e, s_e, NULL);
            oracle_element_matrix(p, h, prm, visc_strong, 0, a_e, s ? s_e : NULL, OR_ALL, K);
            for (int A = 0; A < nen; ++A)
                for (int f = 0; f < 4; ++f)
                    for (int g = 0; g < 4; ++g)
                        be[((size_t)e * nen + A) * 16 + f * 4 + g] =
                            K[(size_t)(f * nen + A) * nd + (g * nen + A)];
        }
        free(K);
    }
    memset(blocks, 0, sizeof(double) * (size_t)N * 16);
    int64_t ids[27];
    for (int64_t e = 0; e < E; ++e) {
        int64_t cx = e % n[0], cy = (e / n[0]) % n[1], cz = e / ((int64_t)n[0] * n[1]);
        cell_nodes(n, p, cx, cy, cz, ids);
        for (int A = 0; A < nen; ++A)
            for (int k = 0; k < 16; ++k) blocks[ids[A] * 16 + k] += be[((size_t)e * nen + A) * 16 + k];
    }
    free(be);
    if (dmask)
        for (int64_t g = 0; g < N; ++g)
            for (int f = 0; f < 3; ++f)
                if (dmask[f * N + g])
                    for (int k = 0; k < 4; ++k) {
                        blocks[g * 16 + f * 4 + k] = (k == f) ? 1.0 : 0.0;
                        blocks[g * 16 + k * 4 + f] = (k == f) ? 1.0 : 0.0;
                    }
    return 0;
}

/*
 * Element-level nonlinear residual contributions for the time step: for each
 * cell, r_e = K_e(a = u) x_e - L_e(a = u) f_e with f = c_m u_old + body force
 * (nodal, [3][N]).  The sum over cells is written to R ([4][N]); Dirichlet rows
 * are left to the caller.  x is NOT masked here.
 */
int oracle_vms_residual(const int *n, int p, const double *h, const double *prm, int visc_strong,
                        const double *s, const double *x, const double *f, double *R)
{
    if (p != 1 && p != 2) return -1;
    const int q = p + 1, nen = q * q * q, nd = 4 * nen, nc = 3 * nen;
    const int64_t Nx = (int64_t)p * n[0] + 1, Ny = (int64_t)p * n[1] + 1, Nz = (int64_t)p * n[2] + 1;
    const int64_t N = Nx * Ny * Nz;
    const int64_t E = (int64_t)n[0] * n[1] * n[2];
    double *re = (double *)malloc(sizeof(double) * (size_t)E * nd);
    if (!re) return -2;
#pragma omp parallel
    {
        double *K = (double *)malloc(sizeof(double) * (size_t)nd * nd);
        double *L = (double *)malloc(sizeof(double) * (size_t)nd * nc);
        double a_e[81], s_e[27], x_e[108], f_e[81];
        int64_t ids[27];
#pragma omp for schedule(static)
        for (int64_t e = 0; e < E; ++e) {
            if (!K || !L) continue;
            int64_t cx = e % n[0], cy = (e / n[0]) % n[1], cz = e / ((int64_t)n[0] * n[1]);
            cell_nodes(n, p, cx, cy, cz, ids);
            for (int A = 0; A < nen; ++A) {
                int64_t g = ids[A];
                for (int d = 0; d < 3; ++d) {
                    a_e[d * nen + A] = x[d * N + g];
                    f_e[d * nen + A] = f[d * N + g];
                }
                for (int d = 0; d < 4; ++d) x_e[d * nen + A] = x[d * N + g];
                if (s) s_e[A] = s[g];
            }
            oracle_element_matrix(p, h, prm, visc_strong, 0, a_e, s ? s_e : NULL, OR_ALL, K);
            oracle_source_matrix(p, h, prm, 0, a_e, s ? s_e : NULL, OR_SRC_ALL, L);
            for (int r = 0; r < nd; ++r) {
                double acc = 0.0;
                for (int c = 0; c < nd; ++c) acc += K[(size_t)r * nd + c] * x_e[c];
                for (int c = 0; c < nc; ++c) acc -= L[(size_t)r * nc + c] * f_e[c];
                re[(size_t)e * nd + r] = acc;
            }
        }
        free(K);
        free(L);
    }
    memset(R, 0, sizeof(double) * (size_t)(4 * N));
    int64_t ids[27];
    for (int64_t e = 0; e < E; ++e) {
        int64_t cx = e % n[0], cy = (e / n[0]) % n[1], cz = e / ((int64_t)n[0] * n[1]);
        cell_nodes(n, p, cx, cy, cz, ids);
        for (int f2 = 0; f2 < 4; ++f2)
            for (int A = 0; A < nen; ++A) R[f2 * N + ids[A]] += re[(size_t)e * nd + f2 * nen + A];
    }
    free(re);
    return 0;
}

/*
 * Full Newton tangent of the element residual (section 2.4: Newton's method on
 * the monolithic system).  The element residual of a time step is
 *   r_e(x) = K_e(a = u, tau(u)) x - L_e(a = u, tau(u)) f,
 * i.e. per quadrature point, with rho = r_m(u, p) - f the strong momentum
 * residual including the source,
 *   momentum test w:  w.(c_m u + (u.grad)u - f) + 2 nu eps(w):eps(u) - (div w) p
 *                     + tau_m ((u.grad)w).rho + tau_c (div w)(div u)
 *   continuity test q: q div u + tau_m grad q . rho.
 * T = d r_e / d x ((4 nen) x (4 nen), row-major), written out term by term:
 * besides the Picard/Oseen entries it has the reactive convection
 * (du.grad)u in the Galerkin, SUPG and PSPG terms, the derivative of the SUPG
 * test function (du.grad)w . rho, and the derivatives of tau_m and tau_c
 * with respect to the advecting velocity,
 *   d tau_m = -tau_m^3 s (u . G du),   d tau_c = -(tau_c / tau_m) d tau_m.
 * x_e = [4][nen] state (u, p), f_e = [3][nen] nodal source, s_e as above.
 */
int oracle_element_tangent(int p, const double *h, const double *prm, int visc_strong, int nq,
                           const double *x_e, const double *f_e, const double *s_e, double *T)
{
    if (p != 1 && p != 2) return -1;
    if (nq == 0) nq = p + 1;
    const int q = p + 1, nen = q * q * q, nd = 4 * nen;
    const double nu = prm[0], c_m = prm[1];
    const double vs = visc_strong ? nu : 0.0;
    double pt[4], wt[4];
    if (gauss01(nq, pt, wt)) return -1;
    memset(T, 0, sizeof(double) * (size_t)nd * nd);
    const double detJ = h[0] * h[1] * h[2];
    double Gd[3];
    for (int k = 0; k < 3; ++k) Gd[k] = 1.0 / (h[k] * h[k]);
    shape_t S;
    for (int qz = 0; qz < nq; ++qz)
        for (int qy = 0; qy < nq; ++qy)
            for (int qx = 0; qx < nq; ++qx) {
                double xi[3] = {pt[qx], pt[qy], pt[qz]};
                double W = wt[qx] * wt[qy] * wt[qz] * detJ;
                shape3d(p, h, xi, &S);
                /* state at the point */
                double u[3] = {0, 0, 0}, gu[3][3] = {{0}}, gp[3] = {0, 0, 0}, f[3] = {0, 0, 0};
                double lapu[3] = {0, 0, 0}, gdiv[3] = {0, 0, 0}, sq = 0.0;
                for (int B = 0; B < nen; ++B) {
                    for (int i = 0; i < 3; ++i) {
                        const double ui = x_e[i * nen + B];
                        u[i] += S.N[B] * ui;
                        f[i] += S.N[B] * f_e[i * nen + B];
                        for (int k = 0; k < 3; ++k) gu[i][k] += S.dN[B][k] * ui;
                        lapu[i] += (S.d2N[B][0][0] + S.d2N[B][1][1] + S.d2N[B][2][2]) * ui;
                        /* d_k (div u) collects d_k d_i u_i */
                        for (int k = 0; k < 3; ++k) gdiv[k] += S.d2N[B][k][i] * ui;
                    }
                    for (int k = 0; k < 3; ++k) gp[k] += S.dN[B][k] * x_e[3 * nen + B];
                    sq += S.N[B] * (s_e ? s_e[B] : 1.0);
                }
                sq = clamp_s(sq, s_e, nen);
                double tau_m, tau_c;
                stab_params(h, prm, u, sq, &tau_m, &tau_c);
                double divu = gu[0][0] + gu[1][1] + gu[2][2];
                double rho[3];
                for (int i = 0; i < 3; ++i) {
                    double conv = u[0] * gu[i][0] + u[1] * gu[i][1] + u[2] * gu[i][2];
                    rho[i] = c_m * u[i] + conv + gp[i] - vs * (lapu[i] + gdiv[i]) - f[i];
                }
                /* derivatives of tau_m, tau_c along the trial velocity component j (per N_B) */
                double dtm[3], dtc[3];
                for (int j = 0; j < 3; ++j) {
                    dtm[j] = -tau_m * tau_m * tau_m * sq * u[j] * Gd[j];
                    dtc[j] = -(tau_c / tau_m) * dtm[j];
                }
                double adN[27], lapN[27], gNrho[27];
                for (int A = 0; A < nen; ++A) {
                    adN[A] = u[0] * S.dN[A][0] + u[1] * S.dN[A][1] + u[2] * S.dN[A][2];
                    lapN[A] = S.d2N[A][0][0] + S.d2N[A][1][1] + S.d2N[A][2][2];
                    gNrho[A] = S.dN[A][0] * rho[0] + S.dN[A][1] * rho[1] + S.dN[A][2] * rho[2];
                }
                for (int A = 0; A < nen; ++A)
                    for (int B = 0; B < nen; ++B) {
                        const double NA = S.N[A], NB = S.N[B];
                        const double gAgB = S.dN[A][0] * S.dN[B][0] + S.dN[A][1] * S.dN[B][1]
                                          + S.dN[A][2] * S.dN[B][2];
                        /* d rho_i / d u_{B,j} */
                        double drho[3][3];
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j)
                                drho[i][j] = (i == j ? c_m * NB + adN[B] - vs * lapN[B] : 0.0)
                                           + NB * gu[i][j] - vs * S.d2N[B][i][j];
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j) {
                                double v = 0.0;
                                /* Galerkin: mass, convection (both factors), viscous */
                                if (i == j) v += c_m * NA * NB + NA * adN[B] + nu * gAgB;
                                v += NA * NB * gu[i][j];
                                v += nu * S.dN[A][j] * S.dN[B][i];
                                /* SUPG: tau_m (u.grad N_A) rho_i, all three factors varied */
                                v += tau_m * adN[A] * drho[i][j];
                                v += tau_m * NB * S.dN[A][j] * rho[i];
                                v += dtm[j] * NB * adN[A] * rho[i];
                                /* LSIC: tau_c d_i N_A div u */
                                v += tau_c * S.dN[A][i] * S.dN[B][j];
                                v += dtc[j] * NB * S.dN[A][i] * divu;
                                T[(size_t)(i * nen + A) * nd + (j * nen + B)] += W * v;
                            }
                        for (int i = 0; i < 3; ++i) {
                            double v = -S.dN[A][i] * NB + tau_m * adN[A] * S.dN[B][i];
                            T[(size_t)(i * nen + A) * nd + (3 * nen + B)] += W * v;
                        }
                        for (int j = 0; j < 3; ++j) {
                            double v = NA * S.dN[B][j];
                            double t = 0.0;
                            for (int i = 0; i < 3; ++i) t += S.dN[A][i] * drho[i][j];
                            v += tau_m * t + dtm[j] * NB * gNrho[A];
                            T[(size_t)(3 * nen + A) * nd + (j * nen + B)] += W * v;
                        }
                        T[(size_t)(3 * nen + A) * nd + (3 * nen + B)] += W * tau_m * gAgB;
                    }
            }
    return 0;
}

/*
 * y = T(x) v over the whole grid: the fluid part of the full Newton tangent of
 * the step residual at the state x ([4][N]) with nodal source f ([3][N]).
 * dmask (bytes, [3][N]) or NULL: masked entries of v are zeroed before the
 * apply (Dirichlet columns) and masked rows return v (the derivative of
 * u_D - g_D).
 */
int oracle_vms_tangent_apply(const int *n, int p, const double *h, const double *prm,
                             int visc_strong, const double *s, const uint8_t *dmask,
                             const double *x, const double *f, const double *v, double *y)
{
    if (p != 1 && p != 2) return -1;
    const int q = p + 1, nen = q * q * q, nd = 4 * nen;
    const int64_t Nx = (int64_t)p * n[0] + 1, Ny = (int64_t)p * n[1] + 1, Nz = (int64_t)p * n[2] + 1;
    const int64_t N = Nx * Ny * Nz;
    const int64_t E = (int64_t)n[0] * n[1] * n[2];
    double *ye = (double *)malloc(sizeof(double) * (size_t)E * nd);
    if (!ye) return -2;
    int err = 0;
#pragma omp parallel
    {
        double *T = (double *)malloc(sizeof(double) * (size_t)nd * nd);
        double x_e[108], f_e[81], s_e[27], v_e[108];
        int64_t ids[27];
        if (!T) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(static)
        for (int64_t e = 0; e < E; ++e) {
            if (!T) continue;
            int64_t cx = e % n[0], cy = (e / n[0]) % n[1], cz = e / ((int64_t)n[0] * n[1]);
            cell_nodes(n, p, cx, cy, cz, ids);
            for (int A = 0; A < nen; ++A) {
                int64_t g = ids[A];
                for (int d = 0; d < 4; ++d) {
                    x_e[d * nen + A] = x[d * N + g];
                    double vv = v[d * N + g];
                    if (d < 3 && dmask && dmask[d * N + g]) vv = 0.0;
                    v_e[d * nen + A] = vv;
                }
                for (int d = 0; d < 3; ++d) f_e[d * nen + A] = f[d * N + g];
                if (s) s_e[A] = s[g];
            }
            oracle_element_tangent(p, h, prm, visc_strong, 0, x_e, f_e, s ? s_e : NULL, T);
            for (int r = 0; r < nd; ++r) {
                double acc = 0.0;
                for (int c = 0; c < nd; ++c) acc += T[(size_t)r * nd + c] * v_e[c];
                ye[(size_t)e * nd + r] = acc;
            }
        }
        free(T);
    }
    if (err) {
        free(ye);
        return err;
    }
    memset(y, 0, sizeof(double) * (size_t)(4 * N));
    int64_t ids[27];
    for (int64_t e = 0; e < E; ++e) {
        int64_t cx = e % n[0], cy = (e / n[0]) % n[1], cz = e / ((int64_t)n[0] * n[1]);
        cell_nodes(n, p, cx, cy, cz, ids);
        for (int f2 = 0; f2 < 4; ++f2)
            for (int A = 0; A < nen; ++A) y[f2 * N + ids[A]] += ye[(size_t)e * nd + f2 * nen + A];
    }
    if (dmask)
        for (int64_t i = 0; i < 3 * N; ++i)
            if (dmask[i]) y[i] = v[i];
    free(ye);
    return 0;
}

/*
 * Selected rows (rows[r] = f*N + node) of the step residual's fluid part
 * (mode 1: sum_e K_e(a=u) x_e - L_e(a=u) f_e, no Dirichlet handling, as
 * oracle_vms_residual) or of the full tangent times v (mode 2: as
 * oracle_vms_tangent_apply, Dirichlet columns of v zeroed and rows = v).
 * Each row sums the contributions of the cells containing the node.
 */
int oracle_vms_step_rows(const int *n, int p, const double *h, const double *prm, int visc_strong,
                         const double *s, const uint8_t *dmask, const double *x, const double *f,
                         const double *v, int mode, const int64_t *rows, int64_t nrows, double *out)
{
    if ((p != 1 && p != 2) || (mode != 1 && mode != 2)) return -1;
    const int q = p + 1, nen = q * q * q, nd = 4 * nen, nc = 3 * nen;
    const int64_t Nx = (int64_t)p * n[0] + 1, Ny = (int64_t)p * n[1] + 1, Nz = (int64_t)p * n[2] + 1;
    const int64_t N = Nx * Ny * Nz;
    int err = 0;
#pragma omp parallel
    {
        double *K = (double *)malloc(sizeof(double) * (size_t)nd * nd);
        double *L = (double *)malloc(sizeof(double) * (size_t)nd * nc);
        double x_e[108], f_e[81], s_e[27], v_e[108];
        int64_t ids[27];
        if (!K || !L) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < nrows; ++r) {
            if (!K || !L) continue;
            int64_t row = rows[r];
            int fr = (int)(row / N);
            int64_t g = row % N;
            if (mode == 2 && fr < 3 && dmask && dmask[row]) {
                out[r] = v[row];
                continue;
            }
            int64_t gi[3] = {g % Nx, (g / Nx) % Ny, g / (Nx * Ny)};
            int64_t lo[3], hi[3];
            for (int d = 0; d < 3; ++d) {
                lo[d] = gi[d] - p < 0 ? 0 : (gi[d] - 1) / p;
                hi[d] = gi[d] / p;
                if (hi[d] > n[d] - 1) hi[d] = n[d] - 1;
            }
            double acc = 0.0;
            for (int64_t cz = lo[2]; cz <= hi[2]; ++cz)
                for (int64_t cy = lo[1]; cy <= hi[1]; ++cy)
                    for (int64_t cx = lo[0]; cx <= hi[0]; ++cx) {
                        int A = (int)((gi[0] - p * cx) + q * ((gi[1] - p * cy) + q * (gi[2] - p * cz)));
                        cell_nodes(n, p, cx, cy, cz, ids);
                        for (int B = 0; B < nen; ++B) {
                            int64_t gg = ids[B];
                            for (int d = 0; d < 4; ++d) {
                                x_e[d * nen + B] = x[d * N + gg];
                                if (mode == 2) {
                                    double vv = v[d * N + gg];
                                    if (d < 3 && dmask && dmask[d * N + gg]) vv = 0.0;
                                    v_e[d * nen + B] = vv;
                                }
                            }
                            for (int d = 0; d < 3; ++d) f_e[d * nen + B] = f[d * N + gg];
                            if (s) s_e[B] = s[gg];
                        }
                        const int rr = fr * nen + A;
                        if (mode == 1) {
                            oracle_element_matrix(p, h, prm, visc_strong, 0, x_e, s ? s_e : NULL, OR_ALL, K);
                            oracle_source_matrix(p, h, prm, 0, x_e, s ? s_e : NULL, OR_SRC_ALL, L);
                            for (int c = 0; c < nd; ++c) acc += K[(size_t)rr * nd + c] * x_e[c];
                            for (int c = 0; c < nc; ++c) acc -= L[(size_t)rr * nc + c] * f_e[c];
                        } else {
                            oracle_element_tangent(p, h, prm, visc_strong, 0, x_e, f_e, s ? s_e : NULL, K);
                            for (int c = 0; c < nd; ++c) acc += K[(size_t)rr * nd + c] * v_e[c];
                        }
                    }
            out[r] = acc;
        }
        free(K);
        free(L);
    }
    return err;
}
