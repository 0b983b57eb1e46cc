/*
 * mf_oracle.c -- plain FP64 CPU reference for the Q2 heat and linearized
 * momentum operators of the diffuse-interface two-phase model.
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the
 * benchmark's CPU-baseline leg are the only users of this file.  It shares no
 * source, header, table or helper with the GPU library, and the GPU library
 * never calls it.
 *
 * Everything is computed from its definition, not for speed:
 *   - 1D Lagrange basis of degree 2 on the nodes {0, 1/2, 1} and its
 *     derivative by the product formula; 3-point Gauss-Legendre rule
 *     ((k+1) points per direction for k = 2, App. B "Numerical framework");
 *   - every cell is mapped by a general trilinear map from its 8 vertices;
 *     J, det J and J^{-1} are computed at every quadrature point;
 *   - every basis function and every physical gradient is evaluated
 *     explicitly at every quadrature point (no sum factorization);
 *   - per-cell dense matrices by full 3x3x3 Gauss quadrature, assembled into
 *     a global CSR matrix by summation.
 * OpenMP is used only across cells that share no node (8-colouring by cell
 * parity) and across matrix rows, which changes nothing but rounding order.
 *
 * Node numbering: Q2 node grid (2nx+1)(2ny+1)(2nz+1), id = i + NX*(j + NY*k).
 * Vector unknowns are component-major: dof = comp * n_nodes + node.
 * Quadrature points in a cell: q = qx + 3 qy + 9 qz; local nodes a + 3b + 9c.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    int32_t n[3];      /* cells per direction */
    int32_t dirichlet; /* bit f: homogeneous Dirichlet on face f (x-,x+,y-,y+,z-,z+) */
    double lo[3];
    double hi[3];
} orc_mesh;

typedef struct {
    int32_t heaviside; /* 0: H = clamp((1+phi)/2, 0, 1); 1: sine form of eq. heaviside */
    int32_t pad_;
    double eps;        /* interface thickness parameter (sine form) */
    double alpha_m;    /* mass factor (1/dt for backward Euler) */
    double alpha_k;    /* conduction factor (heat) */
    double alpha_c;    /* convection factor (momentum) */
    double alpha_v;    /* viscous factor (momentum) */
    double k_l, k_g, rc_l, rc_g, rho_l, rho_g, mu_l, mu_g;
    /* three-phase coefficients (used when a nodal temperature Tc is given) */
    double k_s, rc_s, rho_s, mu_s; /* solid properties */
    double T_sol, T_liq;           /* solidus and liquidus temperatures */
    double darcy_C, darcy_b;       /* Darcy damping of the solid (momentum) */
    double penalty;                /* Tanasawa penalty beta (heat), 0: off */
} orc_coeffs;

/* ------------------------------------------------------------------------ */
/* Reference element                                                         */
/* ------------------------------------------------------------------------ */

static const double NODE1D[3] = {0.0, 0.5, 1.0};

/* l_a(xi) = prod_{b != a} (xi - x_b) / (x_a - x_b) */
static double lag1(int a, double xi)
{
    double v = 1.0;
    for (int b = 0; b < 3; ++b)
        if (b != a) v *= (xi - NODE1D[b]) / (NODE1D[a] - NODE1D[b]);
    return v;
}

/* d l_a / d xi = sum_{m != a} 1/(x_a - x_m) prod_{b != a, m} (xi - x_b)/(x_a - x_b) */
static double dlag1(int a, double xi)
{
    double s = 0.0;
    for (int m = 0; m < 3; ++m) {
        if (m == a) continue;
        double t = 1.0 / (NODE1D[a] - NODE1D[m]);
        for (int b = 0; b < 3; ++b)
            if (b != a && b != m) t *= (xi - NODE1D[b]) / (NODE1D[a] - NODE1D[b]);
        s += t;
    }
    return s;
}

/* 3-point Gauss-Legendre rule on [-1,1] (roots 0, +-sqrt(3/5) of P3, weights
 * 8/9 and 5/9) mapped affinely to [0,1]. */
static void gauss3(double xi[3], double w[3])
{
    const double r = sqrt(0.6);
    const double t[3] = {-r, 0.0, r};
    const double wt[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
    for (int i = 0; i < 3; ++i) {
        xi[i] = 0.5 * (1.0 + t[i]);
        w[i] = 0.5 * wt[i];
    }
}

void orc_gauss3(double *xi, double *w) { gauss3(xi, w); }

void orc_basis1d(double xi, double *val, double *der)
{
    for (int a = 0; a < 3; ++a) {
        val[a] = lag1(a, xi);
        der[a] = dlag1(a, xi);
    }
}

/* ------------------------------------------------------------------------ */
/* Geometry and per-quadrature-point data                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    double N[27];     /* basis values */
    double G[27][3];  /* physical gradients */
    double W;         /* quadrature weight times |det J| */
    double x[3];      /* physical position */
} qp_data;

/* Local shape data at reference point xi (3 coords) through the trilinear map
 * defined by the 8 vertices X[v], v = vx + 2 vy + 4 vz. */
static void eval_point(const double X[8][3], const double xi[3], qp_data *out, double wref)
{
    double J[3][3] = {{0}};
    double pos[3] = {0, 0, 0};
    for (int v = 0; v < 8; ++v) {
        const int b[3] = {v & 1, (v >> 1) & 1, (v >> 2) & 1};
        double L[3], dL[3];
        for (int d = 0; d < 3; ++d) {
            L[d] = b[d] ? xi[d] : 1.0 - xi[d];
            dL[d] = b[d] ? 1.0 : -1.0;
        }
        const double Lv = L[0] * L[1] * L[2];
        const double dLv[3] = {dL[0] * L[1] * L[2], L[0] * dL[1] * L[2], L[0] * L[1] * dL[2]};
        for (int d = 0; d < 3; ++d) {
            pos[d] += X[v][d] * Lv;
            for (int k = 0; k < 3; ++k) J[d][k] += X[v][d] * dLv[k];
        }
    }
    /* inverse by cofactors */
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                     - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                     + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    double Ji[3][3];
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;

    double l[3][3], dl[3][3];
    for (int d = 0; d < 3; ++d)
        for (int a = 0; a < 3; ++a) {
            l[d][a] = lag1(a, xi[d]);
            dl[d][a] = dlag1(a, xi[d]);
        }
    for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                const int i = a + 3 * b + 9 * c;
                out->N[i] = l[0][a] * l[1][b] * l[2][c];
                const double gref[3] = {dl[0][a] * l[1][b] * l[2][c],
                                        l[0][a] * dl[1][b] * l[2][c],
                                        l[0][a] * l[1][b] * dl[2][c]};
                /* grad N = J^{-T} grad_ref N : (grad N)_d = sum_k Ji[k][d] gref[k] */
                for (int d = 0; d < 3; ++d)
                    out->G[i][d] = Ji[0][d] * gref[0] + Ji[1][d] * gref[1] + Ji[2][d] * gref[2];
            }
    out->W = wref * fabs(det);
    for (int d = 0; d < 3; ++d) out->x[d] = pos[d];
}

static void cell_qp(const double X[8][3], int q, qp_data *out)
{
    double xg[3], wg[3];
    gauss3(xg, wg);
    const int qi[3] = {q % 3, (q / 3) % 3, q / 9};
    const double xi[3] = {xg[qi[0]], xg[qi[1]], xg[qi[2]]};
    eval_point(X, xi, out, wg[qi[0]] * wg[qi[1]] * wg[qi[2]]);
}

/* ------------------------------------------------------------------------ */
/* Mesh helpers                                                              */
/* ------------------------------------------------------------------------ */

static inline int64_t nnodes(const orc_mesh *m)
{
    return (int64_t)(2 * m->n[0] + 1) * (2 * m->n[1] + 1) * (2 * m->n[2] + 1);
}

static inline int64_t node_id(const orc_mesh *m, int i, int j, int k)
{
    return (int64_t)i + (int64_t)(2 * m->n[0] + 1) * ((int64_t)j + (int64_t)(2 * m->n[1] + 1) * k);
}

static void cell_vertices(const orc_mesh *m, int cx, int cy, int cz, double X[8][3])
{
    const int c[3] = {cx, cy, cz};
    for (int v = 0; v < 8; ++v)
        for (int d = 0; d < 3; ++d) {
            const int b = (v >> d) & 1;
            const double h = (m->hi[d] - m->lo[d]) / m->n[d];
            X[v][d] = m->lo[d] + h * (c[d] + b);
        }
}

static void cell_nodes(const orc_mesh *m, int cx, int cy, int cz, int64_t idx[27])
{
    for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a)
                idx[a + 3 * b + 9 * c] = node_id(m, 2 * cx + a, 2 * cy + b, 2 * cz + c);
}

static int node_constrained(const orc_mesh *m, int64_t id)
{
    const int NX = 2 * m->n[0] + 1, NY = 2 * m->n[1] + 1;
    const int i = (int)(id % NX), j = (int)((id / NX) % NY), k = (int)(id / ((int64_t)NX * NY));
    const int f = m->dirichlet;
    return ((f & 1) && i == 0) || ((f & 2) && i == 2 * m->n[0]) ||
           ((f & 4) && j == 0) || ((f & 8) && j == 2 * m->n[1]) ||
           ((f & 16) && k == 0) || ((f & 32) && k == 2 * m->n[2]);
}

void orc_constrained_mask(const orc_mesh *m, uint8_t *mask)
{
    const int64_t n = nnodes(m);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) mask[i] = (uint8_t)node_constrained(m, i);
}

/* ------------------------------------------------------------------------ */
/* Coefficients (Sec. 2.3)                                                   */
/* ------------------------------------------------------------------------ */

/* Smoothed Heaviside.  kind 0: H = clamp((1+phi)/2, 0, 1).  kind 1: eq.
 * heaviside with the signed distance recovered from the tanh profile of eq.
 * initial_phi, d = 2 eps artanh(phi).  Returns H and writes dH/dphi. */
static double heaviside(int kind, double eps, double phi, double *dH)
{
    if (kind == 0) {
        if (phi <= -1.0) { *dH = 0.0; return 0.0; }
        if (phi >= 1.0) { *dH = 0.0; return 1.0; }
        *dH = 0.5;
        return 0.5 * (1.0 + phi);
    }
    const double lim = 1.0 - 1e-15;
    const double p = phi < -lim ? -lim : (phi > lim ? lim : phi);
    const double d = 2.0 * eps * atanh(p);
    if (d <= -3.0 * eps) { *dH = 0.0; return 0.0; }
    if (d >= 3.0 * eps) { *dH = 0.0; return 1.0; }
    const double dH_dd = 1.0 / (6.0 * eps) + cos(M_PI * d / (3.0 * eps)) / (6.0 * eps);
    const double dd_dphi = 2.0 * eps / (1.0 - p * p);
    *dH = dH_dd * dd_dphi;
    return 0.5 + d / (6.0 * eps) + sin(M_PI * d / (3.0 * eps)) / (2.0 * M_PI);
}

void orc_heaviside(int32_t kind, double eps, const double *phi, double *H, double *dH, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) H[i] = heaviside(kind, eps, phi[i], &dH[i]);
}

/* eq. muEff: arithmetic phase-fraction weighted average */
static inline double blend_arith(double H, double a_l, double a_g) { return H * a_l + (1.0 - H) * a_g; }
/* eq. rhoEff: reciprocal interpolation of the density */
static inline double blend_recip(double H, double r_l, double r_g) { return 1.0 / (H / r_l + (1.0 - H) / r_g); }

/* Solid fraction from the temperature (eq. solid_fraction): 1 below the
 * solidus, 0 above the liquidus, linear in between. */
static double solid_fraction(double T, double Ts, double Tl)
{
    if (T < Ts) return 1.0;
    if (T > Tl) return 0.0;
    return (Tl - T) / (Tl - Ts);
}

/* Smooth solid indicator (eq. heaviside_sl), zero slope at both ends. */
static inline double heaviside_sl(double fs) { return 3.0 * fs * fs - 2.0 * fs * fs * fs; }

/* Three-phase arithmetic blend (eqs. phase_fractions, solid_liquid_gas_property):
 * a = H_phi (H_s a_s + (1 - H_s) a_l) + (1 - H_phi) a_g. */
static inline double blend3(double Hp, double Hs, double a_s, double a_l, double a_g)
{
    return Hp * (Hs * a_s + (1.0 - Hs) * a_l) + (1.0 - Hp) * a_g;
}

/* Three-phase density (eq. solid_liquid_gas_density): reciprocal between the
 * dense mixture H_s rho_s + (1 - H_s) rho_l and the gas. */
static inline double density3(double Hp, double Hs, const orc_coeffs *cf)
{
    return blend_recip(Hp, Hs * cf->rho_s + (1.0 - Hs) * cf->rho_l, cf->rho_g);
}

/* Coefficient of the Darcy damping (eq. darcy_damping_force): the force is
 * K u with K = -C fs^2 / ((1 - fs)^3 + b); on the left-hand side of the
 * momentum balance it is the reaction term +C fs^2 / ((1 - fs)^3 + b) u. */
static inline double darcy(double fs, const orc_coeffs *cf)
{
    return cf->darcy_C * fs * fs / ((1.0 - fs) * (1.0 - fs) * (1.0 - fs) + cf->darcy_b);
}

/* ------------------------------------------------------------------------ */
/* Cell matrices                                                             */
/* ------------------------------------------------------------------------ */

/* Heat cell matrix, from the weak form of eq. heat_transfer after one
 * backward-Euler step:
 *   A_e[i][j] = sum_q W_q ( alpha_m rc_q N_i N_j + alpha_k k_q grad N_i . grad N_j
 *                         + alpha_c rc_q N_i (u_q . grad N_j) ),
 * the last (convective) term only when a nodal velocity u0_27x3 (component
 * major, 3 x 27) is given, u_q = sum_j N_j(x_q) u_j.  Coefficients: from
 * nodal phi (phi27 != NULL) through H and eq. muEff, or given per
 * quadrature point (kq27, rcq27). */
static void heat_cell_matrix(const double X[8][3], const orc_coeffs *cf, const double *phi27,
                             const double *kq27, const double *rcq27, const double *u0_27x3, const double *Tc27,
                             double *Ae)
{
    memset(Ae, 0, sizeof(double) * 27 * 27);
    qp_data Q;
    for (int q = 0; q < 27; ++q) {
        cell_qp(X, q, &Q);
        double k, rc, react = 0.0;
        if (phi27) {
            double phiq = 0.0, dH, g[3] = {0.0, 0.0, 0.0};
            for (int j = 0; j < 27; ++j) {
                phiq += Q.N[j] * phi27[j];
                for (int d = 0; d < 3; ++d) g[d] += Q.G[j][d] * phi27[j];
            }
            const double H = heaviside(cf->heaviside, cf->eps, phiq, &dH);
            if (Tc27) { /* three phases at the frozen temperature */
                double Tq = 0.0;
                for (int j = 0; j < 27; ++j) Tq += Q.N[j] * Tc27[j];
                const double Hs = heaviside_sl(solid_fraction(Tq, cf->T_sol, cf->T_liq));
                k = blend3(H, Hs, cf->k_s, cf->k_l, cf->k_g);
                rc = blend3(H, Hs, cf->rc_s, cf->rc_l, cf->rc_g);
            } else {
                k = blend_arith(H, cf->k_l, cf->k_g);
                rc = blend_arith(H, cf->rc_l, cf->rc_g);
            }
            if (cf->penalty != 0.0) {
                /* Tanasawa penalty beta delta_rcp T (App. C, eq. penalty_virtual_work), with
                 * delta_rcp of eq. deltaRhoCp: the liquid-gas blend of rc */
                const double c_rcp = 3.0 / (cf->rc_g * cf->rc_g + cf->rc_l * cf->rc_g + cf->rc_l * cf->rc_l);
                react = cf->penalty * dH * sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) *
                        blend_arith(H, cf->rc_l, cf->rc_g) * c_rcp;
            }
        } else {
            k = kq27[q];
            rc = rcq27[q];
        }
        const double cm = Q.W * (cf->alpha_m * rc + react), ck = Q.W * cf->alpha_k * k;
        for (int i = 0; i < 27; ++i)
            for (int j = 0; j < 27; ++j)
                Ae[i * 27 + j] += cm * Q.N[i] * Q.N[j] +
                                  ck * (Q.G[i][0] * Q.G[j][0] + Q.G[i][1] * Q.G[j][1] + Q.G[i][2] * Q.G[j][2]);
        if (u0_27x3) {
            double uq[3] = {0.0, 0.0, 0.0};
            for (int j = 0; j < 27; ++j)
                for (int c = 0; c < 3; ++c) uq[c] += Q.N[j] * u0_27x3[c * 27 + j];
            const double cc = Q.W * cf->alpha_c * rc;
            for (int i = 0; i < 27; ++i)
                for (int j = 0; j < 27; ++j)
                    Ae[i * 27 + j] += cc * Q.N[i] * (uq[0] * Q.G[j][0] + uq[1] * Q.G[j][1] + uq[2] * Q.G[j][2]);
        }
    }
}

void orc_heat_cell_matrix(const double *X24, const orc_coeffs *cf, const double *phi27,
                          const double *kq27, const double *rcq27, const double *u0_27x3, const double *Tc27,
                          double *Ae)
{
    double X[8][3];
    memcpy(X, X24, sizeof(X));
    heat_cell_matrix(X, cf, phi27, kq27, rcq27, u0_27x3, Tc27, Ae);
}

/* The 27 nodal values of a cell of the nodal velocity u0 ([3][n_nodes]), 3 x 27. */
static void cell_velocity(const orc_mesh *m, const double *u0, const int64_t idx[27], double *u27)
{
    const int64_t nn = nnodes(m);
    for (int a = 0; a < 27; ++a)
        for (int c = 0; c < 3; ++c) u27[c * 27 + a] = u0[c * nn + idx[a]];
}

/* Linearized momentum cell matrix from eq. momentum_balance with the viscous
 * stress 2 mu eps(u) (Sec. 2.1), backward Euler and the convective velocity
 * frozen at u0 (Oseen form).  Local dof index c*27 + i:
 *   A_e[(i,c),(j,c')] = sum_q W_q [ alpha_m rho N_i N_j d_cc'
 *                                 + alpha_c rho N_i (u0_q . grad N_j) d_cc'
 *                                 + alpha_v mu (grad N_i . grad N_j d_cc' + d_c' N_i d_c N_j) ]
 * rho by the reciprocal blend of eq. rhoEff, mu by eq. muEff. */
static void oseen_cell_matrix(const double X[8][3], const orc_coeffs *cf, const double *phi27,
                              const double *u0_27x3, const double *Tc27, double *Ae)
{
    memset(Ae, 0, sizeof(double) * 81 * 81);
    qp_data Q;
    for (int q = 0; q < 27; ++q) {
        cell_qp(X, q, &Q);
        double phiq = 0.0, dH, u0q[3] = {0, 0, 0};
        for (int j = 0; j < 27; ++j) {
            phiq += Q.N[j] * phi27[j];
            for (int c = 0; c < 3; ++c) u0q[c] += Q.N[j] * u0_27x3[c * 27 + j];
        }
        const double H = heaviside(cf->heaviside, cf->eps, phiq, &dH);
        double rho = blend_recip(H, cf->rho_l, cf->rho_g);
        double mu = blend_arith(H, cf->mu_l, cf->mu_g), react = 0.0;
        if (Tc27) { /* three phases at the frozen temperature, Darcy damping of the solid */
            double Tq = 0.0;
            for (int j = 0; j < 27; ++j) Tq += Q.N[j] * Tc27[j];
            const double fs = solid_fraction(Tq, cf->T_sol, cf->T_liq), Hs = heaviside_sl(fs);
            rho = density3(H, Hs, cf);
            mu = blend3(H, Hs, cf->mu_s, cf->mu_l, cf->mu_g);
            react = darcy(fs, cf);
        }
        for (int i = 0; i < 27; ++i)
            for (int j = 0; j < 27; ++j) {
                const double mass = Q.N[i] * Q.N[j];
                const double conv = Q.N[i] * (u0q[0] * Q.G[j][0] + u0q[1] * Q.G[j][1] + u0q[2] * Q.G[j][2]);
                const double lap = Q.G[i][0] * Q.G[j][0] + Q.G[i][1] * Q.G[j][1] + Q.G[i][2] * Q.G[j][2];
                const double diag = Q.W * ((cf->alpha_m * rho + react) * mass + cf->alpha_c * rho * conv +
                                           cf->alpha_v * mu * lap);
                for (int c = 0; c < 3; ++c)
                    for (int cp = 0; cp < 3; ++cp) {
                        double v = Q.W * cf->alpha_v * mu * Q.G[i][cp] * Q.G[j][c];
                        if (c == cp) v += diag;
                        Ae[(c * 27 + i) * 81 + cp * 27 + j] += v;
                    }
            }
    }
}

void orc_oseen_cell_matrix(const double *X24, const orc_coeffs *cf, const double *phi27,
                           const double *u0_27x3, const double *Tc27, double *Ae)
{
    double X[8][3];
    memcpy(X, X24, sizeof(X));
    oseen_cell_matrix(X, cf, phi27, u0_27x3, Tc27, Ae);
}

/* ------------------------------------------------------------------------ */
/* Global CSR pattern: row (c, i) couples to (c', j) for all components c'   */
/* and all nodes j sharing a cell with node i.                               */
/* ------------------------------------------------------------------------ */

/* Range of node indices, along one direction, of the cells containing node t:
 * cells c with 2c <= t <= 2c+2, clipped to [0, n-1]. */
static void neighbor_range(int t, int n, int *lo, int *hi)
{
    int cmin = (t - 1) / 2; /* ceil((t-2)/2) for t >= 0 */
    if (t < 2) cmin = 0;
    int cmax = t / 2;
    if (cmax > n - 1) cmax = n - 1;
    *lo = 2 * cmin;
    *hi = 2 * cmax + 2;
}

int64_t orc_csr_rowptr(const orc_mesh *m, int32_t ncomp, int64_t *rowptr)
{
    const int64_t nn = nnodes(m);
    const int NX = 2 * m->n[0] + 1, NY = 2 * m->n[1] + 1;
    rowptr[0] = 0;
    for (int64_t r = 0; r < ncomp * nn; ++r) {
        const int64_t id = r % nn;
        const int i = (int)(id % NX), j = (int)((id / NX) % NY), k = (int)(id / ((int64_t)NX * NY));
        int lo[3], hi[3];
        neighbor_range(i, m->n[0], &lo[0], &hi[0]);
        neighbor_range(j, m->n[1], &lo[1], &hi[1]);
        neighbor_range(k, m->n[2], &lo[2], &hi[2]);
        const int64_t len = (int64_t)(hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
        rowptr[r + 1] = rowptr[r] + ncomp * len;
    }
    return rowptr[ncomp * nn];
}

void orc_csr_cols(const orc_mesh *m, int32_t ncomp, const int64_t *rowptr, int32_t *cols)
{
    const int64_t nn = nnodes(m);
    const int NX = 2 * m->n[0] + 1, NY = 2 * m->n[1] + 1;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < ncomp * nn; ++r) {
        const int64_t id = r % nn;
        const int i = (int)(id % NX), j = (int)((id / NX) % NY), k = (int)(id / ((int64_t)NX * NY));
        int lo[3], hi[3];
        neighbor_range(i, m->n[0], &lo[0], &hi[0]);
        neighbor_range(j, m->n[1], &lo[1], &hi[1]);
        neighbor_range(k, m->n[2], &lo[2], &hi[2]);
        int64_t p = rowptr[r];
        for (int c = 0; c < ncomp; ++c)
            for (int kk = lo[2]; kk <= hi[2]; ++kk)
                for (int jj = lo[1]; jj <= hi[1]; ++jj)
                    for (int ii = lo[0]; ii <= hi[0]; ++ii)
                        cols[p++] = (int32_t)(c * nn + node_id(m, ii, jj, kk));
    }
}

static int64_t find_col(const int64_t *rowptr, const int32_t *cols, int64_t row, int32_t col)
{
    int64_t a = rowptr[row], b = rowptr[row + 1] - 1;
    while (a <= b) {
        const int64_t mid = (a + b) / 2;
        if (cols[mid] == col) return mid;
        if (cols[mid] < col) a = mid + 1; else b = mid - 1;
    }
    return -1;
}

/* Identity rows and removed columns for constrained dofs. */
static void apply_dirichlet(const orc_mesh *m, int ncomp, const int64_t *rowptr, const int32_t *cols, double *vals)
{
    const int64_t nn = nnodes(m);
    if (!m->dirichlet) return;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < ncomp * nn; ++r) {
        const int rc = node_constrained(m, r % nn);
        for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
            if (rc) vals[p] = (cols[p] == r) ? 1.0 : 0.0;
            else if (node_constrained(m, cols[p] % nn)) vals[p] = 0.0;
        }
    }
}

/* Assembly of the heat operator.  phi (nodal) or kq/rcq (per quadrature point,
 * cell-major, 27 per cell) select how the coefficients are formed; a non-NULL
 * nodal velocity u0 ([3][n_nodes]) adds the convective term. */
void orc_assemble_heat(const orc_mesh *m, const orc_coeffs *cf, const double *phi,
                       const double *kq, const double *rcq, const double *u0, const double *Tc,
                       const int64_t *rowptr, const int32_t *cols, double *vals)
{
    const int64_t nnz = rowptr[nnodes(m)];
    memset(vals, 0, sizeof(double) * nnz);
    for (int color = 0; color < 8; ++color) {
        const int px = color & 1, py = (color >> 1) & 1, pz = (color >> 2) & 1;
#pragma omp parallel for collapse(3) schedule(dynamic, 16)
        for (int cz = pz; cz < m->n[2]; cz += 2)
            for (int cy = py; cy < m->n[1]; cy += 2)
                for (int cx = px; cx < m->n[0]; cx += 2) {
                    double X[8][3], Ae[27 * 27], phi27[27], u27[81];
                    int64_t idx[27];
                    cell_vertices(m, cx, cy, cz, X);
                    cell_nodes(m, cx, cy, cz, idx);
                    const int64_t cell = cx + (int64_t)m->n[0] * (cy + (int64_t)m->n[1] * cz);
                    double Tc27[27];
                    if (u0) cell_velocity(m, u0, idx, u27);
                    if (Tc)
                        for (int a = 0; a < 27; ++a) Tc27[a] = Tc[idx[a]];
                    if (phi) {
                        for (int a = 0; a < 27; ++a) phi27[a] = phi[idx[a]];
                        heat_cell_matrix(X, cf, phi27, NULL, NULL, u0 ? u27 : NULL, Tc ? Tc27 : NULL, Ae);
                    } else {
                        heat_cell_matrix(X, cf, NULL, kq + 27 * cell, rcq + 27 * cell, u0 ? u27 : NULL, NULL, Ae);
                    }
                    for (int i = 0; i < 27; ++i)
                        for (int j = 0; j < 27; ++j) {
                            const int64_t p = find_col(rowptr, cols, idx[i], (int32_t)idx[j]);
                            vals[p] += Ae[i * 27 + j];
                        }
                }
    }
    apply_dirichlet(m, 1, rowptr, cols, vals);
}

void orc_assemble_oseen(const orc_mesh *m, const orc_coeffs *cf, const double *phi, const double *u0,
                        const double *Tc, const int64_t *rowptr, const int32_t *cols, double *vals)
{
    const int64_t nn = nnodes(m);
    const int64_t nnz = rowptr[3 * nn];
    memset(vals, 0, sizeof(double) * nnz);
    for (int color = 0; color < 8; ++color) {
        const int px = color & 1, py = (color >> 1) & 1, pz = (color >> 2) & 1;
#pragma omp parallel for collapse(3) schedule(dynamic, 4)
        for (int cz = pz; cz < m->n[2]; cz += 2)
            for (int cy = py; cy < m->n[1]; cy += 2)
                for (int cx = px; cx < m->n[0]; cx += 2) {
                    double X[8][3], phi27[27], u27[81], Tc27[27];
                    double *Ae = (double *)malloc(sizeof(double) * 81 * 81);
                    int64_t idx[27];
                    cell_vertices(m, cx, cy, cz, X);
                    cell_nodes(m, cx, cy, cz, idx);
                    for (int a = 0; a < 27; ++a) {
                        phi27[a] = phi[idx[a]];
                        if (Tc) Tc27[a] = Tc[idx[a]];
                        for (int c = 0; c < 3; ++c) u27[c * 27 + a] = u0[c * nn + idx[a]];
                    }
                    oseen_cell_matrix(X, cf, phi27, u27, Tc ? Tc27 : NULL, Ae);
                    for (int c = 0; c < 3; ++c)
                        for (int i = 0; i < 27; ++i)
                            for (int cp = 0; cp < 3; ++cp)
                                for (int j = 0; j < 27; ++j) {
                                    const int64_t p = find_col(rowptr, cols, c * nn + idx[i], (int32_t)(cp * nn + idx[j]));
                                    vals[p] += Ae[(c * 27 + i) * 81 + cp * 27 + j];
                                }
                    free(Ae);
                }
    }
    apply_dirichlet(m, 3, rowptr, cols, vals);
}

/* y = A x */
void orc_spmv(int64_t nrows, const int64_t *rowptr, const int32_t *cols, const double *vals,
              const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        double s = 0.0;
        for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) s += vals[p] * x[cols[p]];
        y[r] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Selected rows of y = A x, from cell matrices, without assembling A        */
/* (for spot checks at sizes where the global matrix is too large).          */
/* ------------------------------------------------------------------------ */

static void cells_of_node(const orc_mesh *m, int64_t id, int clo[3], int chi[3])
{
    const int NX = 2 * m->n[0] + 1, NY = 2 * m->n[1] + 1;
    const int t[3] = {(int)(id % NX), (int)((id / NX) % NY), (int)(id / ((int64_t)NX * NY))};
    for (int d = 0; d < 3; ++d) {
        int lo, hi;
        neighbor_range(t[d], m->n[d], &lo, &hi);
        clo[d] = lo / 2;
        chi[d] = (hi - 2) / 2;
    }
}

/* Rows of y = A x (transpose != 0: of y = A^T x) of the heat operator, with
 * the convective term when u0 is given. */
void orc_heat_rows(const orc_mesh *m, const orc_coeffs *cf, const double *phi, const double *kq,
                   const double *rcq, const double *u0, const double *Tc, const double *x, int32_t transpose,
                   int64_t nrows, const int64_t *rows, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < nrows; ++s) {
        const int64_t r = rows[s];
        if (node_constrained(m, r)) { out[s] = x[r]; continue; }
        int clo[3], chi[3];
        cells_of_node(m, r, clo, chi);
        double acc = 0.0;
        for (int cz = clo[2]; cz <= chi[2]; ++cz)
            for (int cy = clo[1]; cy <= chi[1]; ++cy)
                for (int cx = clo[0]; cx <= chi[0]; ++cx) {
                    double X[8][3], Ae[27 * 27], phi27[27], u27[81];
                    int64_t idx[27];
                    cell_vertices(m, cx, cy, cz, X);
                    cell_nodes(m, cx, cy, cz, idx);
                    const int64_t cell = cx + (int64_t)m->n[0] * (cy + (int64_t)m->n[1] * cz);
                    double Tc27[27];
                    if (u0) cell_velocity(m, u0, idx, u27);
                    if (Tc)
                        for (int a = 0; a < 27; ++a) Tc27[a] = Tc[idx[a]];
                    if (phi) {
                        for (int a = 0; a < 27; ++a) phi27[a] = phi[idx[a]];
                        heat_cell_matrix(X, cf, phi27, NULL, NULL, u0 ? u27 : NULL, Tc ? Tc27 : NULL, Ae);
                    } else {
                        heat_cell_matrix(X, cf, NULL, kq + 27 * cell, rcq + 27 * cell, u0 ? u27 : NULL, NULL, Ae);
                    }
                    int il = -1;
                    for (int a = 0; a < 27; ++a) if (idx[a] == r) il = a;
                    for (int j = 0; j < 27; ++j) {
                        const double e = transpose ? Ae[j * 27 + il] : Ae[il * 27 + j];
                        if (!node_constrained(m, idx[j])) acc += e * x[idx[j]];
                    }
                }
        out[s] = acc;
    }
}

/* rows are dof indices comp * n_nodes + node; transpose != 0 gives rows of A^T x. */
void orc_oseen_rows(const orc_mesh *m, const orc_coeffs *cf, const double *phi, const double *u0,
                    const double *Tc, const double *x, int32_t transpose, int64_t nrows, const int64_t *rows,
                    double *out)
{
    const int64_t nn = nnodes(m);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < nrows; ++s) {
        const int64_t r = rows[s];
        const int64_t node = r % nn;
        const int comp = (int)(r / nn);
        if (node_constrained(m, node)) { out[s] = x[r]; continue; }
        int clo[3], chi[3];
        cells_of_node(m, node, clo, chi);
        double acc = 0.0;
        double *Ae = (double *)malloc(sizeof(double) * 81 * 81);
        for (int cz = clo[2]; cz <= chi[2]; ++cz)
            for (int cy = clo[1]; cy <= chi[1]; ++cy)
                for (int cx = clo[0]; cx <= chi[0]; ++cx) {
                    double X[8][3], phi27[27], u27[81], Tc27[27];
                    int64_t idx[27];
                    cell_vertices(m, cx, cy, cz, X);
                    cell_nodes(m, cx, cy, cz, idx);
                    for (int a = 0; a < 27; ++a) {
                        phi27[a] = phi[idx[a]];
                        if (Tc) Tc27[a] = Tc[idx[a]];
                        for (int c = 0; c < 3; ++c) u27[c * 27 + a] = u0[c * nn + idx[a]];
                    }
                    oseen_cell_matrix(X, cf, phi27, u27, Tc ? Tc27 : NULL, Ae);
                    int il = -1;
                    for (int a = 0; a < 27; ++a) if (idx[a] == node) il = a;
                    const int li = comp * 27 + il;
                    for (int cp = 0; cp < 3; ++cp)
                        for (int j = 0; j < 27; ++j) {
                            if (node_constrained(m, idx[j])) continue;
                            const int lj = cp * 27 + j;
                            const double a = transpose ? Ae[lj * 81 + li] : Ae[li * 81 + lj];
                            acc += a * x[cp * nn + idx[j]];
                        }
                }
        free(Ae);
        out[s] = acc;
    }
}

/* ------------------------------------------------------------------------ */
/* Quadrature-point fields                                                   */
/* ------------------------------------------------------------------------ */

/* Physical coordinates of all quadrature points, [n_cells*27][3]. */
void orc_quad_points(const orc_mesh *m, double *xq)
{
    const int64_t nc = (int64_t)m->n[0] * m->n[1] * m->n[2];
#pragma omp parallel for schedule(static)
    for (int64_t cell = 0; cell < nc; ++cell) {
        const int cx = (int)(cell % m->n[0]), cy = (int)((cell / m->n[0]) % m->n[1]),
                  cz = (int)(cell / ((int64_t)m->n[0] * m->n[1]));
        double X[8][3];
        cell_vertices(m, cx, cy, cz, X);
        qp_data Q;
        for (int q = 0; q < 27; ++q) {
            cell_qp(X, q, &Q);
            for (int d = 0; d < 3; ++d) xq[(cell * 27 + q) * 3 + d] = Q.x[d];
        }
    }
}

/* k and rho*cp at all quadrature points from nodal phi (eqs. heaviside, muEff). */
void orc_heat_qp_coeffs(const orc_mesh *m, const orc_coeffs *cf, const double *phi, double *kq, double *rcq)
{
    const int64_t nc = (int64_t)m->n[0] * m->n[1] * m->n[2];
#pragma omp parallel for schedule(static)
    for (int64_t cell = 0; cell < nc; ++cell) {
        const int cx = (int)(cell % m->n[0]), cy = (int)((cell / m->n[0]) % m->n[1]),
                  cz = (int)(cell / ((int64_t)m->n[0] * m->n[1]));
        double X[8][3];
        int64_t idx[27];
        cell_vertices(m, cx, cy, cz, X);
        cell_nodes(m, cx, cy, cz, idx);
        qp_data Q;
        for (int q = 0; q < 27; ++q) {
            cell_qp(X, q, &Q);
            double phiq = 0.0, dH;
            for (int j = 0; j < 27; ++j) phiq += Q.N[j] * phi[idx[j]];
            const double H = heaviside(cf->heaviside, cf->eps, phiq, &dH);
            kq[cell * 27 + q] = blend_arith(H, cf->k_l, cf->k_g);
            rcq[cell * 27 + q] = blend_arith(H, cf->rc_l, cf->rc_g);
        }
    }
}

/* Gradient of L(T) through one implicit heat step A(k, rc) T = alpha_m M(rc) T_old,
 * given the adjoint state lam (A^T lam = dL/dT):
 *   dL/dk_q  = -alpha_k W_q grad lam(x_q) . grad T(x_q)
 *   dL/drc_q = -alpha_m W_q lam(x_q) (T - T_old)(x_q)
 * and, when phi != NULL (coefficients formed from phi through H),
 *   dL/dphi_j = sum_{cells, q} N_j(x_q) H'(phi_q) [(k_l - k_g) dL/dk_q + (rc_l - rc_g) dL/drc_q].
 * T - T_old is taken from dTin when given (the step solved in delta form),
 * which avoids the cancellation of forming it from T and T_old.
 * The formulas hold for lam = 0 on Dirichlet nodes (adjoint right-hand side
 * zeroed there, since T is fixed on them) and T, T_old = 0 on Dirichlet nodes.
 * dphi is accumulated cell by cell (8-colouring) over all nodes. */
void orc_heat_grad(const orc_mesh *m, const orc_coeffs *cf, const double *phi, const double *T,
                   const double *Told, const double *dTin, const double *lam, double *dk, double *drc, double *dphi)
{
    const int64_t nn = nnodes(m);
    if (dphi) memset(dphi, 0, sizeof(double) * nn);
    for (int color = 0; color < 8; ++color) {
        const int px = color & 1, py = (color >> 1) & 1, pz = (color >> 2) & 1;
#pragma omp parallel for collapse(3) schedule(dynamic, 16)
        for (int cz = pz; cz < m->n[2]; cz += 2)
            for (int cy = py; cy < m->n[1]; cy += 2)
                for (int cx = px; cx < m->n[0]; cx += 2) {
                    double X[8][3];
                    int64_t idx[27];
                    cell_vertices(m, cx, cy, cz, X);
                    cell_nodes(m, cx, cy, cz, idx);
                    const int64_t cell = cx + (int64_t)m->n[0] * (cy + (int64_t)m->n[1] * cz);
                    qp_data Q;
                    for (int q = 0; q < 27; ++q) {
                        cell_qp(X, q, &Q);
                        double l = 0, dT = 0, gl[3] = {0, 0, 0}, gT[3] = {0, 0, 0}, phiq = 0;
                        for (int j = 0; j < 27; ++j) {
                            const int64_t g = idx[j];
                            l += Q.N[j] * lam[g];
                            dT += Q.N[j] * (dTin ? dTin[g] : T[g] - Told[g]);
                            for (int d = 0; d < 3; ++d) {
                                gl[d] += Q.G[j][d] * lam[g];
                                gT[d] += Q.G[j][d] * T[g];
                            }
                            if (phi) phiq += Q.N[j] * phi[g];
                        }
                        const double gk = -cf->alpha_k * Q.W * (gl[0] * gT[0] + gl[1] * gT[1] + gl[2] * gT[2]);
                        const double grc = -cf->alpha_m * Q.W * l * dT;
                        if (dk) dk[cell * 27 + q] = gk;
                        if (drc) drc[cell * 27 + q] = grc;
                        if (phi && dphi) {
                            double dH;
                            (void)heaviside(cf->heaviside, cf->eps, phiq, &dH);
                            const double s = dH * ((cf->k_l - cf->k_g) * gk + (cf->rc_l - cf->rc_g) * grc);
                            for (int j = 0; j < 27; ++j) dphi[idx[j]] += Q.N[j] * s;
                        }
                    }
                }
    }
}

/* ------------------------------------------------------------------------ */
/* Multigrid transfer: P[i][j] = N_j^coarse(x_i^fine) (Q2 embedding)         */
/* ------------------------------------------------------------------------ */

/* Count (pass cols == NULL) or fill the CSR of the prolongation from the
 * coarse mesh mc (n cells) to the fine mesh with 2n cells on the same box.
 * Entries whose value is exactly zero are dropped. */
int64_t orc_prolongation(const orc_mesh *mc, int64_t *rowptr, int32_t *cols, double *vals)
{
    const int nf[3] = {2 * mc->n[0], 2 * mc->n[1], 2 * mc->n[2]};
    const int NXf = 2 * nf[0] + 1, NYf = 2 * nf[1] + 1, NZf = 2 * nf[2] + 1;
    int64_t p = 0;
    if (!cols) rowptr[0] = 0;
    for (int k = 0; k < NZf; ++k)
        for (int j = 0; j < NYf; ++j)
            for (int i = 0; i < NXf; ++i) {
                const int64_t row = i + (int64_t)NXf * (j + (int64_t)NYf * k);
                /* fine node position in coarse-cell units: t/4 cells */
                const int t[3] = {i, j, k};
                int c[3];
                double xi[3];
                for (int d = 0; d < 3; ++d) {
                    c[d] = t[d] / 4;
                    if (c[d] > mc->n[d] - 1) c[d] = mc->n[d] - 1;
                    xi[d] = (t[d] - 4.0 * c[d]) / 4.0;
                }
                int64_t start = cols ? rowptr[row] : p;
                int64_t q = start;
                /* columns in increasing global coarse index: c outer, b, a inner */
                for (int cc = 0; cc < 3; ++cc)
                    for (int b = 0; b < 3; ++b)
                        for (int a = 0; a < 3; ++a) {
                            const double v = lag1(a, xi[0]) * lag1(b, xi[1]) * lag1(cc, xi[2]);
                            if (v == 0.0) continue;
                            if (cols) {
                                cols[q] = (int32_t)node_id(mc, 2 * c[0] + a, 2 * c[1] + b, 2 * c[2] + cc);
                                vals[q] = v;
                            }
                            ++q;
                        }
                if (!cols) {
                    p = q;
                    rowptr[row + 1] = p;
                }
            }
    return cols ? rowptr[(int64_t)NXf * NYf * NZf] : p;
}

/* Load vector b_i = int f N_i, by the same Gauss rule, from values of f at the
 * quadrature points (cell-major, 27 per cell).  No Dirichlet treatment. */
void orc_load_vector(const orc_mesh *m, const double *fq, double *b)
{
    const int64_t nn = nnodes(m);
    memset(b, 0, sizeof(double) * nn);
    for (int color = 0; color < 8; ++color) {
        const int px = color & 1, py = (color >> 1) & 1, pz = (color >> 2) & 1;
#pragma omp parallel for collapse(3) schedule(dynamic, 16)
        for (int cz = pz; cz < m->n[2]; cz += 2)
            for (int cy = py; cy < m->n[1]; cy += 2)
                for (int cx = px; cx < m->n[0]; cx += 2) {
                    double X[8][3];
                    int64_t idx[27];
                    cell_vertices(m, cx, cy, cz, X);
                    cell_nodes(m, cx, cy, cz, idx);
                    const int64_t cell = cx + (int64_t)m->n[0] * (cy + (int64_t)m->n[1] * cz);
                    qp_data Q;
                    for (int q = 0; q < 27; ++q) {
                        cell_qp(X, q, &Q);
                        for (int i = 0; i < 27; ++i) b[idx[i]] += Q.W * fq[cell * 27 + q] * Q.N[i];
                    }
                }
    }
}

/* ------------------------------------------------------------------------ */
/* Interface heat sources (Sec. 2.4, Sec. 4)                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t terms;        /* bit 0: evaporative cooling, bit 1: laser heat flux,
                             bit 2: right-hand side of the Tanasawa penalty, beta T_v delta_rcp */
    int32_t pad_;
    double evap_coeff;    /* evaporation coefficient of the Tanasawa model, 0 < . <= 1 */
    double molar_mass;    /* M, kg/mol; specific gas constant R/M */
    double vapor_density; /* vapor density in the Tanasawa coefficient */
    double T_boil;        /* boiling temperature T_v */
    double h_v;           /* latent heat of evaporation */
    double power, absorptivity, radius; /* laser P_L, chi_L, r_L */
    double focus[3];      /* a point of the beam axis */
    double dir[3];        /* unit beam direction e_L */
} orc_sources;

/* Right-hand side of the heat equation from the interface fluxes,
 *   b_i = sum_cells sum_q W_q N_i(x_q) [ s_evap(x_q) + q_laser(x_q) ],
 * with, at each quadrature point (phi, grad phi and T interpolated from the
 * nodes):
 *   delta     = |grad H(phi)| = H'(phi) |grad phi|                 (eq. delta)
 *   delta_rcp = delta rc(phi) c_rcp, c_rcp = 3 / (rc_g^2 + rc_l rc_g + rc_l^2)
 *                                                                (eq. deltaRhoCp)
 *   mdot      = alpha_v (T - T_v),                              (eq. mDotTanasawa)
 *   alpha_v   = 2 gamma / (2 - gamma) h_v / sqrt(2 pi R/M) rho_v / T_v^{3/2}
 *   s_evap    = -mdot h_v delta_rcp                          (eq. vapor_heat_loss)
 *   n         = -grad phi / |grad phi| (from the liquid, phi > 0, into the gas)
 *   q_laser   = 2 chi P / (pi r^2) <-n . e_L> exp(-2 d_L^2 / r^2) delta_rcp
 *                                                                (eq. laser_gauss)
 * d_L the distance of x_q from the beam axis.  Dirichlet nodes get 0.  The
 * temperature enters at the quadrature point itself (local temperature). */
void orc_heat_sources(const orc_mesh *m, const orc_coeffs *cf, const orc_sources *src, const double *phi,
                      const double *T, double *b)
{
    const int64_t nn = nnodes(m);
    memset(b, 0, sizeof(double) * nn);
    const double Rgas = 8.314;
    const double gam = src->evap_coeff;
    const double alpha_v = 2.0 * gam / (2.0 - gam) * src->h_v / sqrt(2.0 * M_PI * Rgas / src->molar_mass) *
                           src->vapor_density / pow(src->T_boil, 1.5);
    const double c_rcp = 3.0 / (cf->rc_g * cf->rc_g + cf->rc_l * cf->rc_g + cf->rc_l * cf->rc_l);
    const double peak = 2.0 * src->absorptivity * src->power / (M_PI * src->radius * src->radius);
    for (int color = 0; color < 8; ++color) {
        const int px = color & 1, py = (color >> 1) & 1, pz = (color >> 2) & 1;
#pragma omp parallel for collapse(3) schedule(dynamic, 16)
        for (int cz = pz; cz < m->n[2]; cz += 2)
            for (int cy = py; cy < m->n[1]; cy += 2)
                for (int cx = px; cx < m->n[0]; cx += 2) {
                    double X[8][3];
                    int64_t idx[27];
                    cell_vertices(m, cx, cy, cz, X);
                    cell_nodes(m, cx, cy, cz, idx);
                    qp_data Q;
                    for (int q = 0; q < 27; ++q) {
                        cell_qp(X, q, &Q);
                        double ph = 0.0, Tq = 0.0, g[3] = {0.0, 0.0, 0.0};
                        for (int j = 0; j < 27; ++j) {
                            ph += Q.N[j] * phi[idx[j]];
                            Tq += Q.N[j] * T[idx[j]];
                            for (int d = 0; d < 3; ++d) g[d] += Q.G[j][d] * phi[idx[j]];
                        }
                        double dH;
                        const double H = heaviside(cf->heaviside, cf->eps, ph, &dH);
                        const double gnorm = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
                        const double delta = dH * gnorm;
                        const double delta_rcp = delta * blend_arith(H, cf->rc_l, cf->rc_g) * c_rcp;
                        double s = 0.0;
                        if (src->terms & 1) s += -alpha_v * (Tq - src->T_boil) * src->h_v * delta_rcp;
                        if (src->terms & 4) s += cf->penalty * src->T_boil * delta_rcp;
                        if ((src->terms & 2) && gnorm > 0.0) {
                            double n_dot_e = 0.0, r[3], t = 0.0;
                            for (int d = 0; d < 3; ++d) {
                                n_dot_e += -g[d] / gnorm * src->dir[d];
                                r[d] = Q.x[d] - src->focus[d];
                                t += r[d] * src->dir[d];
                            }
                            double dl2 = 0.0;
                            for (int d = 0; d < 3; ++d) {
                                const double p = r[d] - t * src->dir[d];
                                dl2 += p * p;
                            }
                            const double mac = -n_dot_e > 0.0 ? -n_dot_e : 0.0;
                            s += peak * mac * exp(-2.0 * dl2 / (src->radius * src->radius)) * delta_rcp;
                        }
                        for (int i = 0; i < 27; ++i) b[idx[i]] += Q.W * Q.N[i] * s;
                    }
                }
    }
    for (int64_t i = 0; i < nn; ++i)
        if (node_constrained(m, i)) b[i] = 0.0;
}

/* ------------------------------------------------------------------------ */
/* Level-set transport velocity (Sec. 2.5, App. A)                           */
/* ------------------------------------------------------------------------ */

/* Signed distance recovered from the tanh profile of eq. initial_phi,
 * phi = tanh(d / (2 eps)):  d = 2 eps artanh(phi), phi clamped to
 * +-(1 - 1e-15) (the same reading as the sine Heaviside). */
static double distance_from_phi(double eps, double phi)
{
    const double lim = 1.0 - 1e-15;
    const double p = phi < -lim ? -lim : (phi > lim ? lim : phi);
    return eps * log((1.0 + p) / (1.0 - p));
}

/* Gradient of the Q2 interpolant of the nodal field f at every node,
 * averaged over the cells that contain the node: for each cell, the physical
 * basis gradients (general trilinear map) are evaluated at the reference
 * position (a/2, b/2, c/2) of each of its 27 nodes.  g: component-major [3][n]. */
void orc_nodal_gradient(const orc_mesh *m, const double *f, double *g)
{
    const int64_t nn = nnodes(m);
    int *cnt = (int *)calloc((size_t)nn, sizeof(int));
    memset(g, 0, sizeof(double) * 3 * nn);
    for (int cz = 0; cz < m->n[2]; ++cz)
        for (int cy = 0; cy < m->n[1]; ++cy)
            for (int cx = 0; cx < m->n[0]; ++cx) {
                double X[8][3];
                int64_t idx[27];
                cell_vertices(m, cx, cy, cz, X);
                cell_nodes(m, cx, cy, cz, idx);
                for (int i = 0; i < 27; ++i) {
                    const double xi[3] = {NODE1D[i % 3], NODE1D[(i / 3) % 3], NODE1D[i / 9]};
                    qp_data P;
                    eval_point(X, xi, &P, 1.0);
                    for (int d = 0; d < 3; ++d) {
                        double s = 0.0;
                        for (int j = 0; j < 27; ++j) s += P.G[j][d] * f[idx[j]];
                        g[d * nn + idx[i]] += s;
                    }
                    cnt[idx[i]] += 1;
                }
            }
    for (int64_t i = 0; i < nn; ++i)
        for (int d = 0; d < 3; ++d) g[d * nn + i] /= cnt[i];
    free(cnt);
}

/* Value at the physical point x of the Q2 interpolant of the nodal field f:
 * x is first moved to the nearest point of the box, then located in its
 * cell (the uniform mesh's affine map inverted), and the 27 basis functions
 * are evaluated there explicitly. */
static double point_value(const orc_mesh *m, const double *f, const double x[3])
{
    int c[3];
    double xi[3];
    for (int d = 0; d < 3; ++d) {
        const double h = (m->hi[d] - m->lo[d]) / m->n[d];
        double p = x[d] < m->lo[d] ? m->lo[d] : (x[d] > m->hi[d] ? m->hi[d] : x[d]);
        int k = (int)floor((p - m->lo[d]) / h);
        if (k < 0) k = 0;
        if (k > m->n[d] - 1) k = m->n[d] - 1;
        c[d] = k;
        xi[d] = (p - (m->lo[d] + h * k)) / h;
    }
    int64_t idx[27];
    cell_nodes(m, c[0], c[1], c[2], idx);
    double v = 0.0;
    for (int i = 0; i < 27; ++i)
        v += f[idx[i]] * lag1(i % 3, xi[0]) * lag1((i / 3) % 3, xi[1]) * lag1(i / 9, xi[2]);
    return v;
}

void orc_point_values(const orc_mesh *m, const double *f, int64_t np, const double *x, double *out)
{
    for (int64_t p = 0; p < np; ++p) out[p] = point_value(m, f, x + 3 * p);
}

/* Level-set transport velocity at every node (u, u_gamma component-major):
 *   n      = grad d / |grad d| (0 where |grad d| <= 1e-8: no normal), with
 *            d_j = d(phi_j) the recovered signed distance: the unit normal
 *            pointing into the liquid (phi > 0);
 *   mdot   = alpha_v (T - T_v)                                 (eq. mDotTanasawa)
 *   variant 1 (eq. transport_vel_local_continuous):
 *            u_gamma = u_j + mdot(T_j) / rho(phi_j) n_j, rho by eq. rhoEff;
 *   variant 2 (eq. transport_vel_extension_liquid):
 *            x_G = x_j - d_j n_j          (projection along n to phi = 0),
 *            x_l = x_j + (3 eps - d_j) n_j (to the contour d = 3 eps, H = 1),
 *            u_gamma = u(x_l) + mdot(T(x_G)) / rho_l n_j,
 *            u(x_l), T(x_G) values of the Q2 interpolants.
 * Optional outputs (component-major [3][n]): nrm, xg, xl (variant 2). */
void orc_transport_velocity(const orc_mesh *m, const orc_coeffs *cf, const orc_sources *src, int32_t variant,
                            const double *phi, const double *u, const double *T, double *ug, double *nrm,
                            double *xg, double *xl)
{
    const int64_t nn = nnodes(m);
    const double gam = src->evap_coeff;
    const double alpha_v = 2.0 * gam / (2.0 - gam) * src->h_v / sqrt(2.0 * M_PI * 8.314 / src->molar_mass) *
                           src->vapor_density / pow(src->T_boil, 1.5);
    double *d = (double *)calloc((size_t)nn, sizeof(double));
    double *g = (double *)calloc((size_t)(3 * nn), sizeof(double));
    for (int64_t i = 0; i < nn; ++i) d[i] = distance_from_phi(cf->eps, phi[i]);
    orc_nodal_gradient(m, d, g);
    const int NX = 2 * m->n[0] + 1, NY = 2 * m->n[1] + 1;
    for (int64_t i = 0; i < nn; ++i) {
        const int ijk[3] = {(int)(i % NX), (int)((i / NX) % NY), (int)(i / ((int64_t)NX * NY))};
        double x[3], n[3];
        for (int k = 0; k < 3; ++k) x[k] = m->lo[k] + ijk[k] * 0.5 * (m->hi[k] - m->lo[k]) / m->n[k];
        const double gn = sqrt(g[i] * g[i] + g[nn + i] * g[nn + i] + g[2 * nn + i] * g[2 * nn + i]);
        /* |grad d| is 1 for a signed distance; where it is (numerically) zero,
         * at a point of symmetry or where phi saturates, there is no normal */
        for (int k = 0; k < 3; ++k) n[k] = gn > 1e-8 ? g[k * nn + i] / gn : 0.0;
        if (nrm)
            for (int k = 0; k < 3; ++k) nrm[k * nn + i] = n[k];
        if (variant == 1) {
            double dH;
            const double H = heaviside(cf->heaviside, cf->eps, phi[i], &dH);
            const double mdot = alpha_v * (T[i] - src->T_boil);
            const double rho = blend_recip(H, cf->rho_l, cf->rho_g);
            for (int k = 0; k < 3; ++k) ug[k * nn + i] = u[k * nn + i] + mdot / rho * n[k];
        } else {
            double pg[3], pl[3];
            for (int k = 0; k < 3; ++k) {
                pg[k] = x[k] - d[i] * n[k];
                pl[k] = x[k] + (3.0 * cf->eps - d[i]) * n[k];
                if (xg) xg[k * nn + i] = pg[k];
                if (xl) xl[k * nn + i] = pl[k];
            }
            const double mdot = alpha_v * (point_value(m, T, pg) - src->T_boil);
            for (int k = 0; k < 3; ++k) ug[k * nn + i] = point_value(m, u + k * nn, pl) + mdot / cf->rho_l * n[k];
        }
    }
    free(d);
    free(g);
}
