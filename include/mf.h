/*
 * mf.h -- C ABI of the matrix-free Q2 operator and solver library for one
 * MI355X (gfx950) GPU.
 *
 * The library applies, on uniform hexahedral meshes with continuous
 * Lagrange Q2 elements and 3x3x3 Gauss quadrature (App. B "Numerical
 * framework"), the two implicit operators of the diffuse-interface
 * two-phase model:
 *
 *   heat  (Sec. 2.1, eq. heat_transfer without convection, one backward-Euler
 *         step):  A = alpha_m M(rho c_p) + alpha_k K(k)
 *   Oseen (Sec. 2.1, eq. momentum_balance linearized about a frozen velocity
 *         u0, viscous stress 2 mu eps(u)):
 *         A = alpha_m M(rho) + alpha_c C(rho, u0) + alpha_v V(mu)
 *
 * with k, rho c_p and mu blended arithmetically (Sec. 2.3, eq. muEff) and rho
 * reciprocally (eq. rhoEff) through a smoothed Heaviside H(phi) of a nodal
 * level-set field (eq. heaviside, or the linear form H = (1+phi)/2), and
 * solves them with CG (symmetric) or GMRES (non-symmetric) as in App. B.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Mesh      n[d] cells per direction on the box [lo, hi]; Q2 nodes
 *           (2n0+1)(2n1+1)(2n2+1) numbered i + NX*(j + NY*k), x fastest.
 * Vectors   scalar fields: n_nodes entries; velocity: component-major
 *           [3][n_nodes].  Quadrature-point fields: cell-major, 27 per cell,
 *           q = qx + 3 qy + 9 qz, cell = cx + n0 (cy + n1 cz).
 * Dirichlet faces flagged in mesh.dirichlet carry homogeneous conditions:
 *           those dofs are identity rows of A with their columns removed.
 * Pointers  every array argument is DEVICE memory on the device that was
 *           current when the context was created, owned by the caller,
 *           contiguous, of the element type given by the operator precision
 *           (double for MF_FP64, float for MF_FP32).  Host pointers are only
 *           the descriptor structs and the mf_solve_info output.
 * Streams   work is enqueued on the given stream (0 = default stream).
 *           Applies return without synchronizing; solvers synchronize the
 *           stream to read convergence state.
 * Errors    functions return an mf_status; nothing aborts.  On error a
 *           message is available from mf_last_error(ctx).
 * Threads   a context must not be used by two host threads at once; calls
 *           on one context that overlap on the GPU race on its workspace.
 */
#ifndef MF_H
#define MF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *mf_stream; /* a hipStream_t */

typedef enum {
    MF_OK = 0,
    MF_NOT_CONVERGED = 1, /* solver reached maxit; x and info are still written */
    MF_BREAKDOWN = 2,     /* Krylov breakdown (p.Ap <= 0, NaN/Inf); x holds the last iterate */
    MF_ERR_ARG = -1,      /* invalid argument (null pointer, size, enum value) */
    MF_ERR_HIP = -2,      /* a HIP runtime call failed */
    MF_ERR_OOM = -3,      /* device allocation failed */
    MF_ERR_STATE = -4     /* object used in a state that does not allow the call */
} mf_status;

enum { MF_HEAT = 0, MF_OSEEN = 1 };
enum { MF_FP64 = 0, MF_FP32 = 1 };
enum { MF_COEFF_LEVELSET = 0, MF_COEFF_QUAD = 1 };
enum { MF_H_LINEAR = 0, MF_H_SINE = 1 };
enum { MF_PC_NONE = 0, MF_PC_JACOBI = 1, MF_PC_BLOCK_JACOBI = 2 };

/* Face bits of mf_mesh.dirichlet. */
enum { MF_FACE_XLO = 1, MF_FACE_XHI = 2, MF_FACE_YLO = 4, MF_FACE_YHI = 8, MF_FACE_ZLO = 16, MF_FACE_ZHI = 32 };

typedef struct {
    int32_t n[3];       /* cells per direction, each >= 1; total nodes < 2^31 */
    uint32_t dirichlet; /* MF_FACE_* bits with homogeneous Dirichlet conditions */
    double lo[3];       /* box corner */
    double hi[3];       /* opposite corner, hi[d] > lo[d] */
} mf_mesh;

/* Operator descriptor (host struct; the arrays it points to are device memory). */
typedef struct {
    int32_t kind;       /* MF_HEAT or MF_OSEEN */
    int32_t precision;  /* MF_FP64 or MF_FP32: element type of every array */
    int32_t coeff_mode; /* MF_COEFF_LEVELSET: coefficients from nodal phi;
                           MF_COEFF_QUAD: heat k and rho c_p given per quadrature point */
    int32_t heaviside;  /* MF_H_LINEAR: H = clamp((1+phi)/2, 0, 1);
                           MF_H_SINE: eq. heaviside with d = 2 eps artanh(phi) */
    double eps;         /* interface thickness parameter (MF_H_SINE only) */
    double alpha_m;     /* mass factor, 1/dt */
    double alpha_k;     /* heat conduction factor */
    double alpha_c;     /* Oseen convection factor */
    double alpha_v;     /* Oseen viscous factor */
    double k_l, k_g;    /* conductivity, liquid / gas */
    double rc_l, rc_g;  /* volumetric heat capacity rho c_p, liquid / gas */
    double rho_l, rho_g;/* density, liquid / gas (reciprocal blend) */
    double mu_l, mu_g;  /* dynamic viscosity, liquid / gas */
    const void *phi;    /* nodal level set [n_nodes] (LEVELSET mode, and Oseen) */
    const void *k_q;    /* conductivity per quadrature point [n_cells*27] (QUAD mode) */
    const void *rc_q;   /* rho c_p per quadrature point [n_cells*27] (QUAD mode) */
    const void *u0;     /* Oseen convective velocity, nodal [3][n_nodes]; for heat, optional:
                           the convective term alpha_c C(rc, u0) (FP64, LEVELSET mode) */
    /* Three phases (Sec. 4.1-4.3, FP64, LEVELSET mode): if T_coef is given the
     * coefficients are evaluated at that frozen nodal temperature with the
     * solid fraction f_s(T) (eq. solid_fraction, solidus T_sol < liquidus
     * T_liq), H_s = 3 f_s^2 - 2 f_s^3 (eq. heaviside_sl) and the blends
     * a = H (H_s a_s + (1 - H_s) a_l) + (1 - H) a_g (k, rc_p, mu), rho
     * reciprocal between H_s rho_s + (1 - H_s) rho_l and rho_g; the Oseen
     * operator then gains the Darcy damping of the solid
     * + darcy_C f_s^2 / ((1 - f_s)^3 + darcy_b) u (eq. darcy_damping_force). */
    double k_s, rc_s, rho_s, mu_s; /* solid properties */
    double T_sol, T_liq;
    double darcy_C, darcy_b;
    double penalty;     /* heat, LEVELSET mode: Tanasawa penalty beta delta_rcp T on the left-hand
                           side (App. C, eq. penalty_virtual_work; 0: off) */
    const void *T_coef; /* nodal temperature of the coefficients [n_nodes], or NULL */
} mf_operator;

typedef struct {
    int32_t iters;      /* operator applications in the Krylov iteration */
    int32_t converged;  /* 1 if the stopping test was met */
    double rel_res;     /* true ||b - A x|| / ||b|| recomputed at exit */
    double rel_res_est; /* the residual estimate the stopping test used */
} mf_solve_info;

typedef struct mf_ctx mf_ctx;
typedef struct mf_mg mf_mg;

/* ---- context ---------------------------------------------------------------- */

/* Create a context for `mesh` on the current HIP device.  The context owns
 * its workspace (Krylov vectors, reduction buffers), allocated on first use
 * and freed by mf_destroy.  Returns MF_ERR_ARG for n[d] < 1, hi <= lo or
 * meshes with 2^31 or more nodes. */
mf_status mf_create(const mf_mesh *mesh, mf_ctx **ctx);
void mf_destroy(mf_ctx *ctx);
/* Last error message of the context; with ctx NULL, of the last failed call
 * without a context on this host thread. */
const char *mf_last_error(const mf_ctx *ctx);
int64_t mf_n_nodes(const mf_ctx *ctx);
int64_t mf_n_cells(const mf_ctx *ctx);

/* ---- kernel timing (profiling aid) ------------------------------------------- */

/* While enabled, every operator apply records HIP events on the caller's
 * stream immediately around its main kernel (not around the clearing of the
 * output).  mf_timing_read waits for the last recorded event and returns the
 * summed kernel time in milliseconds and the number of timed launches since
 * the last reset (reset != 0 starts a new count).  Events are owned by the
 * context. */
mf_status mf_timing_enable(mf_ctx *ctx, int32_t on);
mf_status mf_timing_read(mf_ctx *ctx, double *ms, int64_t *launches, int32_t reset);

/* ---- operator application (Sec. 2.1, 2.3; App. B matrix-free products) ------ */

/* y = A x.  x and y: n_dofs entries (n_nodes for heat, 3 n_nodes for Oseen),
 * distinct buffers.  Dirichlet dofs: y_i = x_i; x is read as zero there in
 * the products of the other rows.  FP32 operators are supported for heat. */
mf_status mf_operator_apply(mf_ctx *ctx, const mf_operator *op, const void *x, void *y, mf_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): y = A x as
 * mf_operator_apply, without a context and without any allocation.  The
 * brick kernels' shared-face scratch lives in a fixed device array of 64 MiB
 * per GPU (held until the process ends), enough for
 *   n_bricks * 891 * comps * sizeof(element) bytes,
 * n_bricks = ceil(n0/4) ceil(n1/4) ceil(n2/4), comps 1 (heat) or 3 (Oseen):
 * e.g. heat FP64 up to 64^3 cells and beyond (64^3 needs 29.2 MB), Oseen
 * FP64 at 48^3 (37 MB).  A larger mesh returns MF_ERR_ARG with a message.
 * Calls on one GPU share that array and keep no state between calls;
 * calls that overlap on one GPU (other streams or host threads) race on it.
 * mesh: as mf_create; op, x, y: as mf_operator_apply (FP32 heat included).
 * Errors are reported by mf_last_error(NULL) of the calling host thread. */
mf_status mf_operator_apply_noalloc(const mf_mesh *mesh, const mf_operator *op, const void *x, void *y,
                                    mf_stream stream);

/* y = A^T x (the adjoint operator).  For the heat operator A^T = A; for the
 * Oseen operator the convective term acts on the test function. */
mf_status mf_operator_apply_transpose(mf_ctx *ctx, const mf_operator *op, const void *x, void *y,
                                      mf_stream stream);

/* Diagonal of A (heat; n_nodes entries) or the 3x3 nodal diagonal blocks of
 * A (Oseen; [n_nodes][3][3] row-major, entry (c, c') couples component c'
 * into row c).  Dirichlet dofs give 1 (identity block). */
mf_status mf_operator_diagonal(mf_ctx *ctx, const mf_operator *op, void *diag, mf_stream stream);

/* ---- Krylov solvers (App. B), FP64 operators only ---------------------------- */

/* Preconditioned CG for the symmetric heat operator, x0 = 0.  precond:
 * MF_PC_NONE or MF_PC_JACOBI (inverse diagonal).  Stops when the recursively
 * updated residual satisfies ||r|| <= rtol ||b||; info->iters counts
 * products with A.  b and x are device arrays of n_nodes doubles. */
mf_status mf_cg_solve(mf_ctx *ctx, const mf_operator *op, int32_t precond, const double *b, double *x,
                      double rtol, int32_t maxit, mf_solve_info *info, mf_stream stream);

/* Right-preconditioned restarted GMRES(restart), x0 = 0, with classical
 * Gram-Schmidt and one re-orthogonalization pass (taken one Arnoldi step
 * late, two passes over the basis per step) and Givens rotations.
 * precond: MF_PC_NONE, MF_PC_JACOBI, or MF_PC_BLOCK_JACOBI (inverse 3x3 nodal
 * blocks, Oseen).  transpose != 0 solves A^T x = b.  Stops when the residual
 * estimate is <= rtol ||b|| and the true residual confirms it.  restart is
 * 1..31 (MF_ERR_ARG otherwise).  The context keeps the Krylov basis (restart
 * + 1 columns of 3 n_nodes doubles, each rounded up to a multiple of 64)
 * until it is destroyed; a later call with a larger restart reallocates it. */
mf_status mf_gmres_solve(mf_ctx *ctx, const mf_operator *op, int32_t precond, int32_t restart, int32_t transpose,
                         const double *b, double *x, double rtol, int32_t maxit, mf_solve_info *info,
                         mf_stream stream);

/* ---- FP32 geometric multigrid preconditioner (heat) ----------------------------- */

typedef struct {
    int32_t coarse_cells;     /* coarsest level: cells per direction (the fine n must be this times 2^L) */
    int32_t degree;           /* Chebyshev smoother degree (pre and post) */
    double smoothing_range;   /* lambda_min = lambda_max / smoothing_range */
    int32_t eig_steps;        /* Lanczos steps for lambda_max of D^{-1} A per level */
    double eig_safety;        /* lambda_max = eig_safety * Lanczos estimate */
    const double *lambda_max; /* optional host array, one per level (coarsest first), overriding the estimate */
    double coarse_rtol;       /* FP64 CG tolerance of the coarse solve (a coarsest level of at most 4 cells
                                 per direction: of the columns of its inverse, formed at setup) */
    int32_t coarse_maxit;
    int32_t auto_levels;      /* 0: levels down to coarse_cells.  1: level rule -- the first level, from the
                                 finest down, on which the mass term dominates the diagonal,
                                   beta = 17.5 (hx^-2 + hy^-2 + hz^-2) max(alpha_k k / (alpha_m rc)) <= beta_stop
                                 (max over the liquid and gas values), becomes the coarsest and is treated by
                                 Chebyshev smoothing (degree smooth_degree, bounds [lambda_min / eig_safety,
                                 eig_safety lambda_max] from the Lanczos Ritz values) instead of a coarse
                                 solve; without such a level the hierarchy goes down to coarse_cells */
    int32_t smooth_degree;    /* Chebyshev degree on a smoothed coarsest level (auto_levels) */
    double beta_stop;         /* threshold of the rule (auto_levels), e.g. 1 */
    const double *lambda_min; /* optional host array, one per level (coarsest first), overriding the lower bound */
} mf_mg_params;

/* Build the level hierarchy of a heat operator in LEVELSET mode: levels are
 * rediscretized in FP32 with the level set injected to the coarse nodes; the
 * coarsest level is kept in FP64 for its CG solve.  op->precision must be
 * MF_FP64 (the fine-level operator of the outer solve). */
mf_status mf_mg_create(mf_ctx *ctx, const mf_operator *op, const mf_mg_params *params, mf_mg **mg, mf_stream stream);
void mf_mg_destroy(mf_mg *mg);
int32_t mf_mg_n_levels(const mf_mg *mg);
/* Chebyshev bounds in use, one per level, coarsest first (host array of n_levels). */
mf_status mf_mg_lambda_max(const mf_mg *mg, double *out);
/* Per level, coarsest first (host arrays of n_levels entries, each may be
 * NULL): cells per direction, Chebyshev degree (0 for a coarsest level solved
 * by CG), and the smoother's bounds. */
mf_status mf_mg_levels(const mf_mg *mg, int32_t *cells, int32_t *degree, double *lambda_min, double *lambda_max);

/* z = V(r): one V-cycle (Chebyshev pre-smoothing from zero, residual,
 * restriction R = P^T, coarse correction, prolongation P = Q2 embedding,
 * Chebyshev post-smoothing) computed in FP32 with the coarsest level solved
 * by FP64 CG.  r and z are FP64 device arrays of n_nodes. */
mf_status mf_mg_vcycle(mf_mg *mg, const double *r, double *z, mf_stream stream);

/* Flexible CG (Polak-Ribiere beta) in FP64 preconditioned by mf_mg_vcycle,
 * x0 = 0; same stopping test and info as mf_cg_solve. */
mf_status mf_mg_cg_solve(mf_mg *mg, const double *b, double *x, double rtol, int32_t maxit, mf_solve_info *info,
                         mf_stream stream);

/* ---- quadrature-point fields and the adjoint gradient (heat, FP64) --------------- */

/* Physical coordinates of all quadrature points, [n_cells*27][3] doubles. */
mf_status mf_quad_points(mf_ctx *ctx, double *xq, mf_stream stream);

/* k and rho c_p at all quadrature points from the operator's nodal phi
 * (eqs. heaviside, muEff); n_cells*27 doubles each. */
mf_status mf_heat_qp_coeffs(mf_ctx *ctx, const mf_operator *op, double *k_q, double *rc_q, mf_stream stream);

/* ---- interface heat sources (heat right-hand side) ----------------------------- */

enum { MF_SRC_EVAPORATION = 1, MF_SRC_LASER = 2, MF_SRC_PENALTY = 4 };

typedef struct {
    int32_t terms;                   /* MF_SRC_* bits */
    double evaporation_coefficient;  /* gamma of the Tanasawa model, 0 < gamma <= 1 */
    double molar_mass;               /* M, kg/mol (specific gas constant 8.314/M) */
    double vapor_density;            /* vapor density in the Tanasawa coefficient, kg/m^3 */
    double boiling_temperature;      /* T_v, K */
    double latent_heat;              /* h_v, J/kg */
    double laser_power;              /* P_L, W */
    double absorptivity;             /* chi_L */
    double laser_radius;             /* r_L, > 0 */
    double focus[3];                 /* a point of the beam axis */
    double direction[3];             /* e_L, unit length (within 1e-9) */
} mf_heat_sources;

/* Right-hand side of the heat equation from the interface fluxes (Sec. 2.4,
 * Sec. 4), integrated against the Q2 basis by the Gauss rule:
 *   b_i = sum_cells sum_q W_q N_i(x_q) s(x_q),  s = s_evap + q_laser,
 *   s_evap  = -mdot(T) h_v delta_rcp                                     (eq. vapor_heat_loss)
 *   mdot    = alpha_v (T - T_v),
 *   alpha_v = 2 gamma/(2 - gamma) h_v / sqrt(2 pi R/M) rho_v / T_v^{3/2}  (eq. mDotTanasawa)
 *   q_laser = 2 chi P/(pi r^2) <-n . e_L> exp(-2 d_L^2/r^2) delta_rcp  (eq. laser_gauss)
 *   delta_rcp = |grad H(phi)| rc(phi) 3/(rc_g^2 + rc_l rc_g + rc_l^2)  (eqs. delta, deltaRhoCp)
 * where rc(phi) is the liquid-gas blend of rc_l and rc_g, also when the
 * operator carries a frozen temperature for three-phase coefficients.
 * with phi, grad phi and T interpolated at each quadrature point (the local
 * temperature), n = -grad phi/|grad phi| the interface normal pointing from
 * the liquid (phi > 0) into the gas, and d_L the distance from the beam axis.
 * MF_SRC_PENALTY adds the right-hand side of the Tanasawa penalty, beta T_v
 * delta_rcp with beta = op->penalty and T_v = boiling_temperature (the
 * penalty form of the evaporative cooling, App. C).
 * op: FP64 heat operator in LEVELSET mode (phi, Heaviside form, rc_l, rc_g).
 * T: nodal temperature (n_nodes doubles; may be NULL without evaporation).
 * b: n_nodes doubles, overwritten; 0 on Dirichlet nodes. */
mf_status mf_heat_source_rhs(mf_ctx *ctx, const mf_operator *op, const mf_heat_sources *src, const double *T,
                             double *b, mf_stream stream);

/* ---- level-set transport velocity (Sec. 2.5, App. A) ------------------------- */

enum { MF_TRANSPORT_LOCAL = 1, MF_TRANSPORT_LIQUID_EXTENSION = 2 };

typedef struct {
    int32_t variant;                /* MF_TRANSPORT_LOCAL or MF_TRANSPORT_LIQUID_EXTENSION */
    int32_t heaviside;              /* H of rho(phi) (local variant); the extension needs MF_H_SINE */
    double eps;                     /* interface thickness parameter, > 0 */
    double rho_l, rho_g;            /* densities, liquid / gas */
    double evaporation_coefficient; /* Tanasawa model (eq. mDotTanasawa), as in mf_heat_sources */
    double molar_mass;
    double vapor_density;
    double boiling_temperature;
    double latent_heat;
} mf_transport_params;

/* Level-set transport velocity at every node of the nodal level set:
 *   MF_TRANSPORT_LOCAL (eq. transport_vel_local_continuous):
 *       u_G = u + mdot(T) / rho(phi) n,        rho by eq. rhoEff;
 *   MF_TRANSPORT_LIQUID_EXTENSION (eq. transport_vel_extension_liquid):
 *       u_G = u(x_l) + mdot(T(x_G)) / rho_l n,
 * with mdot = alpha_v (T - T_v) (eq. mDotTanasawa), the recovered signed
 * distance d = 2 eps artanh(phi) (phi clamped to +-(1 - 1e-15)), the unit
 * normal n = grad d / |grad d| pointing into the liquid (phi > 0; n = 0 where
 * |grad d| <= 1e-8, e.g. at a sphere's centre), grad d the gradient of the Q2 interpolant of the
 * nodal d averaged over the cells that contain the node, the projections
 * x_G = x - d n onto phi = 0 and x_l = x + (3 eps - d) n onto d = 3 eps (where
 * the sine Heaviside reaches 1), and u(x_l), T(x_G) the values of the Q2
 * interpolants at those points, each moved to the nearest point of the box.
 * phi, T: n_nodes doubles; u, u_gamma: [3][n_nodes] doubles (u_gamma != u).
 * Uses one workspace vector of the context.  Meshes with more than 65535
 * nodes along z or 2^23 along y are rejected (MF_ERR_ARG). */
mf_status mf_transport_velocity(mf_ctx *ctx, const mf_transport_params *params, const double *phi, const double *u,
                                const double *T, double *u_gamma, mf_stream stream);

/* Gradient of a loss L(T) through one implicit heat step
 * A(k, rc) T = alpha_m M(rc) T_old, given the adjoint state lambda
 * (A^T lambda = dL/dT with zeros on Dirichlet nodes):
 *   dk_q  = -alpha_k W_q grad(lambda).grad(T) at quadrature point q
 *   drc_q = -alpha_m W_q lambda (T - T_old)    at q
 * and, if dphi != NULL (LEVELSET mode), the chain rule through H:
 *   dphi_j = sum_q N_j(x_q) H'(phi_q) [(k_l - k_g) dk_q + (rc_l - rc_g) drc_q].
 * dT = T - T_old is passed directly (the step is solved in delta form).
 * dk_q, drc_q may be NULL.  All arrays FP64. */
mf_status mf_heat_coeff_grad(mf_ctx *ctx, const mf_operator *op, const double *T, const double *dT,
                             const double *lambda, double *dk_q, double *drc_q, double *dphi, mf_stream stream);

/* ---- whole implicit heat steps (Sec. 2.1 eq. heat_transfer, backward Euler; App. B) ---- */

/* Boundary values.  In the step functions below a Dirichlet face holds the
 * values of T_old: T = T_old on Dirichlet nodes, and the free rows see those
 * values (the operator's columns at Dirichlet nodes are present when it acts
 * on T_old), i.e. on the free rows
 *     alpha_m M(rc) (T - T_old) + alpha_k K(k) T (+ R T) = b.
 * With T_old = 0 on Dirichlet nodes this is the homogeneous problem. */

/* One backward-Euler step of the two-phase heat equation in delta form:
 * dT = T - T_old solves A dT = -alpha_k K T_old on the free rows (dT = 0 on
 * Dirichlet nodes) by Jacobi-CG (x0 = 0, stopping test and info as
 * mf_cg_solve), then T = T_old + dT.  Forming T - T_old from T would cancel
 * about eight digits at small time steps, so dT is returned as well.
 * op: FP64 heat operator, LEVELSET or QUAD coefficients, no convection, no
 * T_coef, no penalty.  T_old, T, dT: distinct device arrays of n_nodes
 * doubles; T and dT are written.  Returns the CG status (MF_NOT_CONVERGED
 * and MF_BREAKDOWN still write T and dT). */
mf_status mf_heat_step(mf_ctx *ctx, const mf_operator *op, const double *T_old, double *T, double *dT, double rtol,
                       int32_t maxit, mf_solve_info *info, mf_stream stream);

/* Adjoint of mf_heat_step for a loss L(T, dT) with gradients gT = dL/dT and
 * gdT = dL/d(dT) (either may be NULL: zero).  Solves A lam = gT + gdT on
 * the free rows (A is symmetric; lam = 0 on Dirichlet nodes) by Jacobi-CG,
 * then writes, for every output that is not NULL:
 *   dk_q, drc_q, dphi   the gradients of mf_heat_coeff_grad at (T, dT, lam)
 *                       (dphi needs LEVELSET mode);
 *   gT_old = dL/dT_old = gT - alpha_k K lam, the operator's columns at
 *                       Dirichlet nodes present (on free rows this equals
 *                       alpha_m M lam - gdT; on Dirichlet rows gT - alpha_k (K lam)).
 * T and dT are those returned by mf_heat_step.  All arrays FP64 device
 * memory (quadrature-point arrays n_cells*27, nodal ones n_nodes). */
mf_status mf_heat_step_adjoint(mf_ctx *ctx, const mf_operator *op, const double *T, const double *dT, const double *gT,
                               const double *gdT, double rtol, int32_t maxit, double *dk_q, double *drc_q,
                               double *dphi, double *gT_old, mf_solve_info *info, mf_stream stream);

typedef struct {
    int32_t iterations;    /* Picard iterations done */
    int32_t converged;     /* 1 if the update test was met */
    int32_t cg_iterations; /* CG iterations summed over the Picard iterations */
    int32_t pad;
    double update;         /* ||T^{k+1} - T^k|| / ||T^{k+1}|| of the last iteration */
} mf_picard_info;

/* One implicit heat step with temperature-dependent three-phase coefficients
 * (Sec. 4.1-4.3), the Tanasawa penalty of op (App. C) and the interface
 * sources of src (Sec. 2.4, Sec. 4; NULL: none), by Picard iteration:
 * T^0 = T_old; with the coefficients and b frozen at T^k, solve
 *     A(T^k) dT = b(T^k) - (K(T^k) + R(T^k)) T_old   (free rows; dT = 0 on Dirichlet nodes)
 * by Jacobi-CG to cg_rtol, set T^{k+1} = T_old + dT, and stop when
 * ||T^{k+1} - T^k|| <= tol ||T^{k+1}||.  A = alpha_m M + K + R is symmetric.
 * op: FP64 heat operator in LEVELSET mode with the three-phase data (k_s,
 * rc_s, T_sol < T_liq), no convection and T_coef = NULL (the iterate is
 * used).  T: n_nodes doubles, written (the last iterate on any status).
 * updates, cg_iters: optional host arrays of maxit entries, per iteration.
 * Returns MF_NOT_CONVERGED after maxit iterations, MF_BREAKDOWN on a CG
 * breakdown or a non-finite iterate. */
mf_status mf_heat_picard_step(mf_ctx *ctx, const mf_operator *op, const mf_heat_sources *src, const double *T_old,
                              double *T, double tol, int32_t maxit, double cg_rtol, int32_t cg_maxit,
                              mf_picard_info *info, double *updates, int32_t *cg_iters, mf_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* MF_H */
