// kernels.hpp -- internal launcher interface between the C ABI (api.hip) and
// the kernel translation units.  Not part of the public boundary.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mf_common.hpp"

namespace mf {

// Coefficients of the heat operator as the kernels take them.
struct HeatArgs {
    int mode;        // 0: from nodal phi, 1: per quadrature point
    int hkind;       // Heaviside form
    double eps;
    double am, ak;   // alpha_m, alpha_k
    double k_l, k_g, rc_l, rc_g;
    const void *phi, *kq, *rcq;
    int conv;        // convective term: 0 none, 1 A, 2 A^T (FP64, mode 0)
    double ac;       // alpha_c
    const double *u0; // nodal velocity [3][n_nodes] (conv != 0)
    // mode 2: three phases at the frozen nodal temperature tc, and/or the
    // Tanasawa penalty (FP64)
    double k_s, rc_s, T_sol, T_liq, penalty;
    const double *tc;
};

// Interface heat sources as the kernel takes them (scalars formed on the host).
struct SourceArgs {
    int terms;                 // bit 0 evaporative cooling, bit 1 laser heat flux, bit 2 penalty right-hand side
    double alpha_v, T_boil, h_v; // Tanasawa coefficient, boiling temperature, latent heat
    double penalty;            // Tanasawa penalty beta (bit 2: beta T_v delta_rcp)
    double peak, inv_r2;       // 2 chi P / (pi r^2), 1 / r^2
    double focus[3], dir[3];   // beam axis point and unit direction
    double c_rcp;              // 3 / (rc_g^2 + rc_l rc_g + rc_l^2)
};

// Level-set transport velocity (transport.hip).
struct TransportArgs {
    int variant;     // 1: local (eq. transport_vel_local_continuous), 2: liquid extension
    int hkind;       // Heaviside form of rho(phi) in variant 1
    double eps;      // interface thickness parameter: d = 2 eps artanh(phi), H = 1 at d = 3 eps
    double rho_l, rho_g;
    double alpha_v;  // Tanasawa coefficient: mdot = alpha_v (T - T_v)
    double T_boil;
};

// Coefficients of the Oseen operator.
struct OseenArgs {
    int hkind;
    double eps;
    double am, ac, av;
    double rho_l, rho_g, mu_l, mu_g;
    const double *phi, *u0;
    // three phases at the frozen nodal temperature tc (null: two phases)
    double rho_s, mu_s, T_sol, T_liq, darcy_C, darcy_b;
    const double *tc;
};

// Device state of a CG solve; scalars never leave the device during the
// iteration except for the periodic convergence check.  rz_old is a copy of
// rz taken one launch before rz is overwritten, so that no kernel reads a
// field that another workgroup of the same launch writes.
struct CGState {
    double rz, rz_old, pAp, rr, bb, alpha, beta, thresh2;
    double rzprev; // flexible CG: r_{k+1} . z_k
    int iter, maxit, done, breakdown, flexible;
    int run;   // set by the CG residual kernel: whether it ran this iteration
    int xpend; // flexible CG: x still lacks the last alpha p
};

// Partial sums of one reduction: NV sets of nblocks doubles, reduced by a
// later launch.
struct RedWS {
    double *partials;
    unsigned capacity; // max partial entries
};

// Optional events recorded immediately around a launcher's main kernel.
struct KTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};

// ---- heat (heat.hip) ----
// y = A x in two launches (bricks, then the shared-face combine); `face` is
// a workspace of face_buffer_elems(m) elements of the operator's type.  With
// cg != nullptr (FP64 only) the apply also forms p.Ap from per-brick
// partials and a third, single-workgroup launch sets alpha = rz / p.Ap.
hipError_t heat_apply(const KMesh &m, const HeatArgs &a, int fp32, const void *x, void *y, void *face, CGState *cg,
                      const RedWS *red, hipStream_t s, const KTiming *t = nullptr);
int64_t face_buffer_elems(const KMesh &m);
hipError_t heat_qp_coeffs(const KMesh &m, const HeatArgs &a, double *kq, double *rcq, hipStream_t s);
// Whole FP64 Jacobi-CG solve (x0 = 0) in one single-workgroup launch, for a
// LEVELSET-mode operator on a mesh of at most 4 cells per direction; b and x
// are FP32 (the coarsest multigrid level).
bool heat_fits_one_brick(const KMesh &m);
hipError_t heat_cg_one_brick(const KMesh &m, const HeatArgs &a, const float *b32, float *x32, double rtol, int maxit,
                             hipStream_t s);
// A^-1 of a one-brick heat operator (the coarsest multigrid level): column c
// solved by the same CG from e_c, all columns in one launch; inv is FP64,
// n_nodes x n_nodes, column-major.
hipError_t heat_inverse_one_brick(const KMesh &m, const HeatArgs &a, double *inv, double rtol, int maxit,
                                  hipStream_t s);
hipError_t quad_points(const KMesh &m, double *xq, hipStream_t s);
// diag(A) (Dirichlet rows 1); with invert its reciprocals (the Jacobi preconditioner).
hipError_t heat_diagonal(const KMesh &m, const HeatArgs &a, int fp32, void *diag, void *face, hipStream_t s,
                         bool invert = false);
hipError_t heat_grad(const KMesh &m, const HeatArgs &a, const double *T, const double *dT, const double *lam,
                     double *dk, double *drc, double *dphi, void *face, hipStream_t s);

// ---- interface heat sources (sources.hip) ----
// b = right-hand side of the interface fluxes from nodal phi (in a) and T;
// level-set mode, FP64; 0 on Dirichlet nodes.
hipError_t heat_sources(const KMesh &m, const HeatArgs &a, const SourceArgs &sa, const double *T, double *b,
                        void *face, hipStream_t s);

// ---- level-set transport velocity (transport.hip) ----
// ug ([3][n_nodes]) from phi, u ([3][n_nodes]) and T; dwork: n_nodes doubles
// of workspace (the recovered signed distance).
hipError_t transport_velocity(const KMesh &m, const TransportArgs &a, const double *phi, const double *u,
                              const double *T, double *ug, double *dwork, hipStream_t s);

// ---- Oseen (oseen.hip) ----
// y = A x or A^T x; `face` holds 3 face_buffer_elems(m) doubles.
hipError_t oseen_apply(const KMesh &m, const OseenArgs &a, int transpose, const double *x, double *y, void *face,
                       hipStream_t s, const KTiming *t = nullptr);
// The 3x3 nodal blocks of A ([n_nodes][3][3]); `face` holds 6 face_buffer_elems(m) doubles.
hipError_t oseen_block_diagonal(const KMesh &m, const OseenArgs &a, double *blocks, void *face, hipStream_t s);

// ---- vectors and Krylov steps (vec.hip) ----
hipError_t vfill(void *y, double v, int64_t n, int fp32, hipStream_t s);
hipError_t vcopy(const double *x, double *y, int64_t n, hipStream_t s);
hipError_t vaxpby(double a, const double *x, double b, double *y, int64_t n, hipStream_t s); // y = a x + b y
hipError_t vaxpbyz(double a, const double *x, double b, const double *y, double *z, int64_t n,
                   hipStream_t s); // z = a x + b y
// z = a x + b y on free dofs, 0 on Dirichlet dofs (comps components of the
// mesh's nodes); a null x or y reads as zero.
hipError_t vmask_axpby(const KMesh &m, int comps, double a, const double *x, double b, const double *y, double *z,
                       hipStream_t s);
// T = T_old + dT; out[0] = ||T_new - T_prev||^2, out[1] = ||T_new||^2 (device)
hipError_t picard_update(const double *T_old, const double *dT, double *T, int64_t n, double *out, const RedWS *red,
                         hipStream_t s);
hipError_t vscale_copy(const double *scale_dev, int invert, const double *x, double *y, int64_t n,
                       hipStream_t s); // y = x * (*s) or x / (*s)
hipError_t vmul(const double *d, const double *x, double *y, int64_t n, hipStream_t s); // y = d .* x
hipError_t vinv(double *d, int64_t n, hipStream_t s);                                   // d = 1 / d
hipError_t vcvt_d2f(const double *x, float *y, int64_t n, hipStream_t s);
hipError_t vcvt_f2d(const float *x, double *y, int64_t n, hipStream_t s);
hipError_t vmulf(const float *d, const float *x, float *y, int64_t n, hipStream_t s);
// out[0] = ||b - t||^2 (device scalar), the partials in red.
hipError_t vdiffnorm2(const double *b, const double *t, int64_t n, double *out, const RedWS *red, hipStream_t s);
// out[k] = sum_i V_k[i] w[i] for k < nv (V columns of length n, leading dim ld);
// nv = 1 with V = x gives a plain dot product.  out is device memory.
hipError_t vmultidot(const double *V, int64_t ld, int nv, const double *w, int64_t n, double *out,
                     const RedWS *red, hipStream_t s);
// y = sum_k V_k h[k] (h device)
hipError_t vcombine(const double *V, int64_t ld, int nv, const double *h, double *y, int64_t n, hipStream_t s);
// Arnoldi step j with delayed re-orthogonalization (vec.hip).  V holds the
// final q_0 .. q_{j-1}; u = column j (once orthogonalized), w = column j + 1
// (A M^-1 u on entry when full).  Completes column j - 1 of the unrotated
// Hessenberg matrix H (device, row stride DGS_LDH) and copies it to col;
// when full, also writes q_j into u, the next candidate into w, and column
// j's first projection into H.  j <= DGS_MAXJ (a closing step: full = false).
constexpr int DGS_MAXJ = 31, DGS_LDH = 32, DGS_INV = 32, DGS_C = 33;
hipError_t dgs_step(const double *V, int64_t ld, int j, bool full, double *u, double *w, int64_t n, double *H,
                    double *coef, double *col, const RedWS *red, hipStream_t s);
hipError_t block3_invert(double *blocks, int64_t nn, hipStream_t s);
hipError_t block3_apply(const double *binv, const double *x, double *y, int64_t nn, hipStream_t s);

// x = 0, p = D^-1 b and r = D^-1 b (the z of cg_resid; flexible: r = b, p = 0), rz and |b|^2 into st.
hipError_t cg_init(CGState *st, const double *b, const double *dinv, double *x, double *r, double *p, int64_t n,
                   double rtol, int maxit, int flexible, const RedWS *red, hipStream_t s);
// alpha = rz / p.Ap from the nb per-brick partials of a CG-mode apply.
hipError_t cg_alpha(CGState *st, const RedWS *red, unsigned nb, hipStream_t s);
// With the diagonal preconditioner (dinv non-null) the vector r holds
// z = D^-1 r: z -= alpha D^-1 q and the partials of r.z and r.r with
// r = z / D^-1; without one, r -= alpha q and the partials of r.r (twice).
hipError_t cg_resid(CGState *st, const double *dinv, double *r, const double *q, int64_t n, const RedWS *red,
                    hipStream_t s);
// beta and the convergence test from cg_resid's partials; x += alpha p, p = z + beta p
hipError_t cg_step(CGState *st, double *x, const double *z, double *p, int64_t n, const RedWS *red, hipStream_t s);
// Flexible-CG pieces (FP32 preconditioner output z, supplied by the caller):
// r -= alpha q, r32 = fl32(r), r.r and r.z_old, convergence test;
hipError_t fcg_resid(CGState *st, double *r, const double *q, const float *zold, float *r32, int64_t n,
                     const RedWS *red, hipStream_t s);
// beta from r.z, x += alpha p (deferred from fcg_resid), p = z + beta p;
hipError_t fcg_direction(CGState *st, const double *r, const float *z, double *p, double *x, int64_t n,
                         const RedWS *red, hipStream_t s);
// after the last poll: x += alpha p if still pending.
hipError_t fcg_finish(const CGState *st, const double *p, double *x, int64_t n, hipStream_t s);

// ---- multigrid (mg.hip) ----
// Separable transfers, one direction per pass; w1 (NXf NYc NZc floats) and w2
// (NXf NYf NZc floats) are work arrays.
hipError_t mg_restrict(const KMesh &fine, const KMesh &coarse, const float *rf, float *rc, float *w1, float *w2,
                       hipStream_t s);
hipError_t mg_prolong_add(const KMesh &coarse, const KMesh &fine, const float *ec, float *xf, float *w1, float *w2,
                          hipStream_t s);
hipError_t mg_inject(const KMesh &fine, const KMesh &coarse, const void *phif, void *phic, int fp32,
                     hipStream_t s);
// Chebyshev pieces in FP32 (see mg.hip)
// Chebyshev smoother vector steps (FP32); see mg.hip.
hipError_t cheb_first(const float *dinv, const float *b, const float *t, float *r, float *d, float *x, float inv_theta,
                      bool more, int64_t n, hipStream_t s);
hipError_t cheb_step(const float *dinv, const float *rin, const float *Ad, float *r, float *d, float *x, float c1,
                     float c2, bool xprev_d, bool last, int64_t n, hipStream_t s);
hipError_t vsub_f(const float *b, const float *Ax, float *r, int64_t n, hipStream_t s); // r = b - Ax

} // namespace mf
