/*
 * fr_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, serial, double-precision CPU reference for the flux-reconstruction
 * (FR) right-hand side of the artificial compressibility method with
 * hyperbolised diffusion (ACM-HD) on constant-Jacobian tensor-product
 * hexahedra, and for the time integrators built on it.  It exists to check the
 * GPU library; nothing in the product path may link, load or call it.  Only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark use it.
 * It shares no source with the GPU library.
 *
 * Paper: Trojak, Watson, Witherden, "Hyperbolic Diffusion in Flux
 * Reconstruction: Optimisation through Kernel Fusion within Tensor-Product
 * Elements" (arXiv:2107.14027).
 *
 *   - governing system: Sec. 2.2, eq. (acmhd_nd) (3D ACM-HD, 13 unknowns);
 *   - FR divergence with correction functions: Sec. 2.1, 1D FR equation;
 *   - algorithmic stages 1..6: Sec. 3, Table 1 (this file follows them in that
 *     order, unfused and unoptimised: no partially-corrected operator);
 *   - interface flux: Sec. 5 (Rusanov on the hyperbolic ACM part, plain mean
 *     of the left/right fluxes for the auxiliary equations);
 *   - physical time: Sec. 5 (BDF2 dual time stepping; the pseudo-time solver
 *     here is classical RK4 with a fixed pseudo step).
 *
 * Readings taken where the paper is silent:
 *   - correction functions: the DG (right/left Radau) member,
 *       h_l = ((-1)^p / 2) (P_p - P_{p+1}),   h_r = (1/2)(P_p + P_{p+1}),
 *     which satisfies the endpoint conditions the paper states in Sec. 2.1;
 *   - Rusanov wave speed: lambda = max over both sides of |V.n| + sqrt((V.n)^2 + zeta);
 *     dissipation acts on P, u, v, w only;
 *   - residual sign: R = -div F + S (Table 1, stage 6), so dU/dtau = R.
 *
 * Layout: U[e][v][k][j][i], i (xi_1) fastest, e = ex + nx*(ey + ny*ez),
 * v in [P, u, v, w, q_x, q_y, q_z, r_x, r_y, r_z, s_x, s_y, s_z] where
 * q = grad u, r = grad v, s = grad w.
 *
 * Every function is pinned by tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NV 13

/* ------------------------------------------------------------------------ */
/* 1D operators (Sec. 2.1)                                                   */
/* ------------------------------------------------------------------------ */

/* Legendre polynomial P_n(x) and its derivative by the three-term recurrence
 * (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}, P'_{n+1} = P'_{n-1} + (2n+1) P_n. */
static void legendre(int n, double x, double *Pn, double *dPn)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (n == 0) { *Pn = 1.0; *dPn = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        double d2 = d0 + (2.0 * k + 1.0) * p1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *Pn = p1; *dPn = d1;
}

/* Gauss-Legendre nodes (ascending) and weights for m points: Newton on P_m. */
int orc_gauss_legendre(int m, double *x, double *w)
{
    if (m < 1 || m > 32) return -1;
    for (int i = 0; i < m; ++i) {
        /* Chebyshev-like first guess, descending in i, mapped to ascending slot. */
        double t = cos(M_PI * (i + 0.75) / (m + 0.5));
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(m, t, &P, &dP);
            double dt = P / dP;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        double P, dP;
        legendre(m, t, &P, &dP);
        x[m - 1 - i] = t;
        w[m - 1 - i] = 2.0 / ((1.0 - t * t) * dP * dP);
    }
    return 0;
}

/* Lagrange basis l_k(t) on nodes x (plain product formula). */
void orc_lagrange_eval(int m, const double *x, double t, double *l)
{
    for (int k = 0; k < m; ++k) {
        double v = 1.0;
        for (int j = 0; j < m; ++j)
            if (j != k) v *= (t - x[j]) / (x[k] - x[j]);
        l[k] = v;
    }
}

/* D[i*m + k] = l_k'(x_i), from the product rule written out term by term. */
void orc_lagrange_deriv(int m, const double *x, double *D)
{
    for (int i = 0; i < m; ++i)
        for (int k = 0; k < m; ++k) {
            double s = 0.0;
            for (int a = 0; a < m; ++a) {
                if (a == k) continue;
                double term = 1.0 / (x[k] - x[a]);
                for (int j = 0; j < m; ++j)
                    if (j != k && j != a) term *= (x[i] - x[j]) / (x[k] - x[j]);
                s += term;
            }
            D[i * m + k] = s;
        }
}

/* Derivatives of the DG correction functions at the nodes:
 *   h_l = ((-1)^p/2)(P_p - P_{p+1}),  h_r = (1/2)(P_p + P_{p+1}). */
void orc_correction_deriv(int p, const double *x, double *dhl, double *dhr)
{
    int m = p + 1;
    double sgn = (p % 2 == 0) ? 1.0 : -1.0;
    for (int i = 0; i < m; ++i) {
        double Pa, dPa, Pb, dPb;
        legendre(p, x[i], &Pa, &dPa);
        legendre(p + 1, x[i], &Pb, &dPb);
        dhl[i] = 0.5 * sgn * (dPa - dPb);
        dhr[i] = 0.5 * (dPa + dPb);
    }
}

/* ------------------------------------------------------------------------ */
/* Physics: eq. (acmhd_nd)                                                   */
/* ------------------------------------------------------------------------ */

/* Physical flux F[j*NV + v] (direction j = x, y, z) of the 13-variable system:
 *   P      : zeta * V
 *   V      : V (x) V + P I - nu S^T      (momentum i, direction j:
 *                                         u_i u_j + P delta_ij - nu dU_i/dx_j)
 *   q,r,s  : -(1/T) V (x) I               (aux (i,k), direction j: -u_i delta_jk / T)
 * where S_ik = d u_i / d x_k is held in U[4 + 3 i + k]. */
void orc_phys_flux(const double *U, double zeta, double nu, double T, double *F)
{
    double P = U[0];
    const double *V = U + 1;
    const double *S = U + 4;
    for (int j = 0; j < 3; ++j) {
        double *Fj = F + j * NV;
        Fj[0] = zeta * V[j];
        for (int i = 0; i < 3; ++i)
            Fj[1 + i] = V[i] * V[j] + (i == j ? P : 0.0) - nu * S[3 * i + j];
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k)
                Fj[4 + 3 * i + k] = (j == k) ? -V[i] / T : 0.0;
    }
}

/* Source S(U) = -(1/T) [0; 0; q; r; s]. */
void orc_source(const double *U, double T, double *S)
{
    for (int v = 0; v < 4; ++v) S[v] = 0.0;
    for (int v = 4; v < NV; ++v) S[v] = -U[v] / T;
}

/* Common interface flux F^I . nh between the state UL (element on the side the
 * unit normal nh points away from) and UR.  Rusanov on the ACM part (P, V),
 * plain mean of the two normal fluxes for the nine auxiliary variables. */
void orc_common_flux(const double *UL, const double *UR, const double *nh,
                     double zeta, double nu, double T, double *Fn)
{
    double FL[3 * NV], FR[3 * NV];
    orc_phys_flux(UL, zeta, nu, T, FL);
    orc_phys_flux(UR, zeta, nu, T, FR);
    double vnl = UL[1] * nh[0] + UL[2] * nh[1] + UL[3] * nh[2];
    double vnr = UR[1] * nh[0] + UR[2] * nh[1] + UR[3] * nh[2];
    double al = fabs(vnl) + sqrt(vnl * vnl + zeta);
    double ar = fabs(vnr) + sqrt(vnr * vnr + zeta);
    double lam = al > ar ? al : ar;
    for (int v = 0; v < NV; ++v) {
        double fl = 0.0, fr = 0.0;
        for (int j = 0; j < 3; ++j) {
            fl += FL[j * NV + v] * nh[j];
            fr += FR[j * NV + v] * nh[j];
        }
        Fn[v] = 0.5 * (fl + fr);
        if (v < 4) Fn[v] -= 0.5 * lam * (UR[v] - UL[v]);
    }
}

/* ------------------------------------------------------------------------ */
/* Geometry of a constant-Jacobian hexahedral lattice                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int p, m, nx, ny, nz;
    double zeta, nu, T;
    double J[9], Jinv[9], detJ;
    double nvec[3][3];   /* n_d = detJ * J^{-T} e_d: scaled reference-face normal */
    double nmag[3], nhat[3][3];
    double x[8], w[8];   /* Gauss nodes, weights */
    double D[64];        /* D[i*m+k] = l_k'(x_i) */
    double lm[8], lp[8]; /* l_k(-1), l_k(+1) */
    double dhl[8], dhr[8];
} orc_geom;

static int geom_init(orc_geom *g, int p, int nx, int ny, int nz, const double *jac,
                     double zeta, double nu, double T)
{
    if (p < 1 || p > 7 || nx < 1 || ny < 1 || nz < 1) return -1;
    g->p = p; g->m = p + 1; g->nx = nx; g->ny = ny; g->nz = nz;
    g->zeta = zeta; g->nu = nu; g->T = T;
    if (jac) {
        memcpy(g->J, jac, sizeof g->J);
    } else { /* periodic box [0, 2 pi]^3: element width 2 pi / n, dx/dxi = pi / n */
        memset(g->J, 0, sizeof g->J);
        g->J[0] = M_PI / nx; g->J[4] = M_PI / ny; g->J[8] = M_PI / nz;
    }
    const double *A = g->J;
    double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6])
               + A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(det > 0.0)) return -1;
    g->detJ = det;
    /* inverse by the adjugate */
    double *B = g->Jinv;
    B[0] = (A[4] * A[8] - A[5] * A[7]) / det; B[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    B[2] = (A[1] * A[5] - A[2] * A[4]) / det; B[3] = (A[5] * A[6] - A[3] * A[8]) / det;
    B[4] = (A[0] * A[8] - A[2] * A[6]) / det; B[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    B[6] = (A[3] * A[7] - A[4] * A[6]) / det; B[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    B[8] = (A[0] * A[4] - A[1] * A[3]) / det;
    for (int d = 0; d < 3; ++d) {
        double s = 0.0;
        for (int j = 0; j < 3; ++j) {
            /* (J^{-T} e_d)_j = (J^{-1})_{d j} */
            g->nvec[d][j] = det * B[3 * d + j];
            s += g->nvec[d][j] * g->nvec[d][j];
        }
        g->nmag[d] = sqrt(s);
        for (int j = 0; j < 3; ++j) g->nhat[d][j] = g->nvec[d][j] / g->nmag[d];
    }
    orc_gauss_legendre(g->m, g->x, g->w);
    orc_lagrange_deriv(g->m, g->x, g->D);
    orc_lagrange_eval(g->m, g->x, -1.0, g->lm);
    orc_lagrange_eval(g->m, g->x, +1.0, g->lp);
    orc_correction_deriv(p, g->x, g->dhl, g->dhr);
    return 0;
}

static inline int64_t elem_index(const orc_geom *g, int ex, int ey, int ez)
{
    ex = (ex % g->nx + g->nx) % g->nx;
    ey = (ey % g->ny + g->ny) % g->ny;
    ez = (ez % g->nz + g->nz) % g->nz;
    return (int64_t)ex + (int64_t)g->nx * ((int64_t)ey + (int64_t)g->ny * ez);
}

/* point index of (i, j, k) within an element */
static inline int pidx(int m, int i, int j, int k) { return i + m * (j + m * k); }

/* index of the point at position l along the direction-d line through the face
 * point (a, b); (a, b) are the two tangential indices in increasing direction. */
static inline int line_point(int m, int d, int a, int b, int l)
{
    if (d == 0) return pidx(m, l, a, b);
    if (d == 1) return pidx(m, a, l, b);
    return pidx(m, a, b, l);
}

/* ------------------------------------------------------------------------ */
/* Residual of one element, stages 1..6 of Table 1, in that order.           */
/* ------------------------------------------------------------------------ */

static void element_residual(const orc_geom *g, const double *U, int ex, int ey, int ez,
                             double *Re /* [NV][m^3] */)
{
    const int m = g->m, ns = m * m * m, nfp = m * m;
    const int64_t stride = (int64_t)NV * ns;
    int64_t e = elem_index(g, ex, ey, ez);
    const double *Ue = U + e * stride;

    double *Fs = malloc(sizeof(double) * 3 * NV * ns);      /* transformed flux F_hat_d */
    double *div = calloc((size_t)NV * ns, sizeof(double));
    double uf_own[NV], uf_nb[NV], fI[NV], fdelta[NV], upt[NV], fphys[3 * NV];

    /* Stage 2: transformed flux at the solution points, F_hat_d = F . n_d */
    for (int q = 0; q < ns; ++q) {
        for (int v = 0; v < NV; ++v) upt[v] = Ue[v * ns + q];
        orc_phys_flux(upt, g->zeta, g->nu, g->T, fphys);
        for (int d = 0; d < 3; ++d)
            for (int v = 0; v < NV; ++v) {
                double s = 0.0;
                for (int j = 0; j < 3; ++j) s += fphys[j * NV + v] * g->nvec[d][j];
                Fs[(d * NV + v) * ns + q] = s;
            }
    }

    /* Stage 3 (uncorrected): derivative of the flux interpolant along each line */
    for (int k = 0; k < m; ++k)
        for (int j = 0; j < m; ++j)
            for (int i = 0; i < m; ++i) {
                int q = pidx(m, i, j, k);
                for (int v = 0; v < NV; ++v) {
                    double s = 0.0;
                    for (int l = 0; l < m; ++l) {
                        s += g->D[i * m + l] * Fs[(0 * NV + v) * ns + pidx(m, l, j, k)];
                        s += g->D[j * m + l] * Fs[(1 * NV + v) * ns + pidx(m, i, l, k)];
                        s += g->D[k * m + l] * Fs[(2 * NV + v) * ns + pidx(m, i, j, l)];
                    }
                    div[v * ns + q] = s;
                }
            }

    /* Stages 1, 4, 5 per face: project U to the face (own and neighbour side),
     * common flux, correction (f^I - f^delta) h' along the normal line. */
    for (int d = 0; d < 3; ++d)
        for (int side = 0; side < 2; ++side) {
            int dx = (d == 0) ? (side ? 1 : -1) : 0;
            int dy = (d == 1) ? (side ? 1 : -1) : 0;
            int dz = (d == 2) ? (side ? 1 : -1) : 0;
            const double *Un = U + elem_index(g, ex + dx, ey + dy, ez + dz) * stride;
            const double *lown = side ? g->lp : g->lm;  /* own face at xi = +-1  */
            const double *lnb = side ? g->lm : g->lp;   /* neighbour's opposite face */
            const double *dh = side ? g->dhr : g->dhl;
            for (int b = 0; b < m; ++b)
                for (int a = 0; a < m; ++a) {
                    /* Stage 1: solution projected to the face point */
                    for (int v = 0; v < NV; ++v) {
                        double so = 0.0, sn = 0.0, sf = 0.0;
                        for (int l = 0; l < m; ++l) {
                            int q = line_point(m, d, a, b, l);
                            so += lown[l] * Ue[v * ns + q];
                            sn += lnb[l] * Un[v * ns + q];
                            sf += lown[l] * Fs[(d * NV + v) * ns + q];
                        }
                        uf_own[v] = so; uf_nb[v] = sn;
                        fdelta[v] = sf;  /* f^delta: flux interpolant at the face */
                    }
                    /* Stage 4: common flux; the left state is the element on the
                     * minus side of the face, the normal points along +xi_d. */
                    if (side)
                        orc_common_flux(uf_own, uf_nb, g->nhat[d], g->zeta, g->nu, g->T, fI);
                    else
                        orc_common_flux(uf_nb, uf_own, g->nhat[d], g->zeta, g->nu, g->T, fI);
                    /* Stage 5: correction along the normal line */
                    for (int l = 0; l < m; ++l) {
                        int q = line_point(m, d, a, b, l);
                        for (int v = 0; v < NV; ++v)
                            div[v * ns + q] += dh[l] * (g->nmag[d] * fI[v] - fdelta[v]);
                    }
                }
            (void)nfp;
        }

    /* Stage 6: negate, divide by the Jacobian determinant, add the source */
    for (int q = 0; q < ns; ++q) {
        double src[NV];
        for (int v = 0; v < NV; ++v) upt[v] = Ue[v * ns + q];
        orc_source(upt, g->T, src);
        for (int v = 0; v < NV; ++v)
            Re[v * ns + q] = -div[v * ns + q] / g->detJ + src[v];
    }
    free(Fs);
    free(div);
}

/* Full residual R = -div F + S over a periodic nx*ny*nz lattice.
 * jac: constant dx/dxi (row-major 3x3), NULL for the periodic box [0,2pi]^3. */
int orc_residual(int p, int nx, int ny, int nz, const double *jac, double zeta, double nu,
                 double T, const double *U, double *R)
{
    orc_geom g;
    if (geom_init(&g, p, nx, ny, nz, jac, zeta, nu, T)) return -1;
    const int64_t stride = (int64_t)NV * g.m * g.m * g.m;
    for (int ez = 0; ez < nz; ++ez)
        for (int ey = 0; ey < ny; ++ey)
            for (int ex = 0; ex < nx; ++ex)
                element_residual(&g, U, ex, ey, ez, R + elem_index(&g, ex, ey, ez) * stride);
    return 0;
}

/* Residual of the listed elements only (R_sel[n][NV][m^3]); the residual of an
 * element depends on its own state and its six face neighbours only. */
int orc_residual_elems(int p, int nx, int ny, int nz, const double *jac, double zeta,
                       double nu, double T, const double *U, int64_t nsel,
                       const int64_t *sel, double *Rsel)
{
    orc_geom g;
    if (geom_init(&g, p, nx, ny, nz, jac, zeta, nu, T)) return -1;
    const int64_t stride = (int64_t)NV * g.m * g.m * g.m;
    const int64_t ne = (int64_t)nx * ny * nz;
    for (int64_t s = 0; s < nsel; ++s) {
        int64_t e = sel[s];
        if (e < 0 || e >= ne) return -1;
        int ex = (int)(e % nx), ey = (int)((e / nx) % ny), ez = (int)(e / ((int64_t)nx * ny));
        element_residual(&g, U, ex, ey, ez, Rsel + s * stride);
    }
    return 0;
}

/* Geometry query for tests: detJ, n_d (3x3, row d), |n_d|. */
int orc_geometry(int nx, int ny, int nz, const double *jac, double *detJ, double *nvec,
                 double *nmag)
{
    orc_geom g;
    if (geom_init(&g, 1, nx, ny, nz, jac, 1.0, 0.0, 1.0)) return -1;
    *detJ = g.detJ;
    for (int d = 0; d < 3; ++d) {
        nmag[d] = g.nmag[d];
        for (int j = 0; j < 3; ++j) nvec[3 * d + j] = g.nvec[d][j];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Time integration                                                          */
/* ------------------------------------------------------------------------ */

/* Classical four-stage Runge-Kutta on dU/dt = R(U), all 13 variables, nsteps
 * steps of size dt (weights 1/6, 1/3, 1/3, 1/6). */
int orc_rk4(int p, int nx, int ny, int nz, const double *jac, double zeta, double nu,
            double T, double *U, double dt, int nsteps)
{
    const int64_t n = (int64_t)nx * ny * nz * NV * (p + 1) * (p + 1) * (p + 1);
    double *k = malloc(sizeof(double) * n), *Us = malloc(sizeof(double) * n);
    double *acc = malloc(sizeof(double) * n);
    const double c[4] = {0.0, 0.5, 0.5, 1.0};
    const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    int rc = 0;
    for (int step = 0; step < nsteps && !rc; ++step) {
        for (int64_t i = 0; i < n; ++i) acc[i] = 0.0;
        for (int s = 0; s < 4 && !rc; ++s) {
            /* stage state U + c_s dt k_{s-1} */
            if (s == 0) memcpy(Us, U, sizeof(double) * n);
            else for (int64_t i = 0; i < n; ++i) Us[i] = U[i] + c[s] * dt * k[i];
            rc = orc_residual(p, nx, ny, nz, jac, zeta, nu, T, Us, k);
            for (int64_t i = 0; i < n; ++i) acc[i] += b[s] * k[i];
        }
        for (int64_t i = 0; i < n; ++i) U[i] += dt * acc[i];
    }
    free(k); free(Us); free(acc);
    return rc;
}

/* Pseudo-time residual of one BDF physical step (Sec. 2.2 time-derivative masks:
 * the physical time derivative acts on V only):
 *   R*(U) = R(U) - M_V * (3U - 4U^n + U^{n-1}) / (2 dt)     (order 2)
 *   R*(U) = R(U) - M_V * (U - U^n) / dt                     (order 1)      */
static int pseudo_residual(int p, int nx, int ny, int nz, const double *jac, double zeta,
                           double nu, double T, const double *U, const double *Un,
                           const double *Unm1, double dt, int order, double *Rs)
{
    int rc = orc_residual(p, nx, ny, nz, jac, zeta, nu, T, U, Rs);
    if (rc) return rc;
    const int ns = (p + 1) * (p + 1) * (p + 1);
    const int64_t ne = (int64_t)nx * ny * nz;
    for (int64_t e = 0; e < ne; ++e)
        for (int v = 1; v <= 3; ++v)
            for (int q = 0; q < ns; ++q) {
                int64_t i = (e * NV + v) * ns + q;
                double dudt = (order == 2) ? (3.0 * U[i] - 4.0 * Un[i] + Unm1[i]) / (2.0 * dt)
                                           : (U[i] - Un[i]) / dt;
                Rs[i] -= dudt;
            }
    return 0;
}

/* Root mean square of the velocity components of R* over all points. */
static double velocity_rms(int p, int64_t ne, const double *Rs)
{
    const int ns = (p + 1) * (p + 1) * (p + 1);
    double s = 0.0;
    for (int64_t e = 0; e < ne; ++e)
        for (int v = 1; v <= 3; ++v)
            for (int q = 0; q < ns; ++q) {
                double r = Rs[(e * NV + v) * ns + q];
                s += r * r;
            }
    return sqrt(s / (3.0 * (double)ne * ns));
}

/* One physical BDF step by dual time stepping: classical RK4 pseudo-steps of
 * size dtau on dU/dtau = R*(U) until RMS(R*_V) < tol, tested on the first
 * stage residual of each pseudo-step.  U holds the initial guess on entry and
 * the last iterate on exit.  Returns 0 on convergence, -5 if max_iters
 * pseudo-steps completed without it; *iters = completed pseudo-steps,
 * *resid = the last RMS computed. */
int orc_dual_step(int p, int nx, int ny, int nz, const double *jac, double zeta, double nu,
                  double T, double *U, const double *Un, const double *Unm1, int order,
                  double dt, double dtau, double tol, int max_iters, int *iters, double *resid)
{
    const int64_t ne = (int64_t)nx * ny * nz;
    const int64_t n = ne * NV * (p + 1) * (p + 1) * (p + 1);
    double *k = malloc(sizeof(double) * n), *Us = malloc(sizeof(double) * n);
    double *acc = malloc(sizeof(double) * n);
    const double c[4] = {0.0, 0.5, 0.5, 1.0};
    const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    int rc = -5, it = 0;
    double res = 0.0;
    for (;;) {
        int r = pseudo_residual(p, nx, ny, nz, jac, zeta, nu, T, U, Un, Unm1, dt, order, k);
        if (r) { rc = r; break; }
        res = velocity_rms(p, ne, k);
        if (!(res == res)) { rc = -4; break; }  /* non-finite */
        if (res < tol) { rc = 0; break; }
        if (it >= max_iters) { rc = -5; break; }
        for (int64_t i = 0; i < n; ++i) acc[i] = b[0] * k[i];
        for (int s = 1; s < 4; ++s) {
            for (int64_t i = 0; i < n; ++i) Us[i] = U[i] + c[s] * dtau * k[i];
            pseudo_residual(p, nx, ny, nz, jac, zeta, nu, T, Us, Un, Unm1, dt, order, k);
            for (int64_t i = 0; i < n; ++i) acc[i] += b[s] * k[i];
        }
        for (int64_t i = 0; i < n; ++i) U[i] += dtau * acc[i];
        ++it;
    }
    *iters = it;
    *resid = res;
    free(k); free(Us); free(acc);
    return rc;
}

/* Polynomial extrapolation in time of the past states to the next step:
 * order 1: 2 U^n - U^{n-1};  order 2: 3 U^n - 3 U^{n-1} + U^{n-2}. */
int orc_extrap(int64_t n, const double *Un, const double *Unm1, const double *Unm2, int order,
               double *G)
{
    if (order == 1) {
        for (int64_t i = 0; i < n; ++i) G[i] = 2.0 * Un[i] - Unm1[i];
    } else if (order == 2) {
        for (int64_t i = 0; i < n; ++i) G[i] = 3.0 * Un[i] - 3.0 * Unm1[i] + Unm2[i];
    } else {
        return -1;
    }
    return 0;
}
