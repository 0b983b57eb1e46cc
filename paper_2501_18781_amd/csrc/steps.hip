// steps.hip -- whole implicit heat steps behind the C ABI: the delta-form
// backward-Euler step and its adjoint (the differentiable step), and the
// Picard iteration of a step with temperature-dependent coefficients.
//
// Dirichlet faces hold the nodal values of T_old: the step's unknown is
// dT = T - T_old with dT = 0 on Dirichlet nodes, and the free rows see the
// boundary values of T_old through the operator applied on the same mesh
// without Dirichlet faces (every column present), masked to the free rows.
// On the free rows this is exactly
//   alpha_m M (T - T_old) + K T = b,  T = T_old on Dirichlet nodes,
// and for T_old = 0 on those nodes it is the homogeneous problem.
#include <math.h>

#include "ctx.hpp"

using namespace mf;

// y = (A - alpha_m M) x, every column present: the heat operator without
// its mass term on the context's mesh with its Dirichlet faces removed.
// The three-phase penalty term (not scaled by alpha_m) stays in.
static hipError_t apply_without_mass(mf_ctx *c, const mf_operator *op, const double *x, double *y, hipStream_t s)
{
    mf_operator o = *op;
    o.alpha_m = 0.0;
    KMesh m = c->km;
    m.dirichlet = 0u;
    return heat_apply(m, heat_args(&o), 0, x, y, c->face, nullptr, nullptr, s);
}

static mf_status check_step_op(mf_ctx *c, const mf_operator *op, const char *who)
{
    mf_status st = check_op(c, op);
    if (st) return st;
    if (op->kind != MF_HEAT || op->precision != MF_FP64 || op->u0 || op->T_coef || op->penalty != 0.0)
        return fail(c, MF_ERR_ARG, "%s needs an FP64 two-phase heat operator without convection", who);
    return MF_OK;
}

extern "C" mf_status mf_heat_step(mf_ctx *c, const mf_operator *op, const double *T_old, double *T, double *dT,
                                  double rtol, int32_t maxit, mf_solve_info *info, mf_stream stream)
{
    mf_status st = check_step_op(c, op, "mf_heat_step");
    if (st) return st;
    if (!T_old || !T || !dT || !info) return fail(c, MF_ERR_ARG, "null argument");
    if (T == T_old || dT == T_old || dT == T) return fail(c, MF_ERR_ARG, "T_old, T and dT must be distinct arrays");
    if (!(rtol >= 0.0) || maxit < 0) return fail(c, MF_ERR_ARG, "invalid rtol or maxit");
    hipStream_t s = (hipStream_t)stream;
    double *rhs;
    if ((st = ws_vec(c, 6, &rhs)) || (st = ensure_face(c, 1))) return st;
    // rhs = -(K T_old) on the free rows, 0 on the Dirichlet rows
    HIPCHK(c, apply_without_mass(c, op, T_old, rhs, s));
    HIPCHK(c, vmask_axpby(c->km, 1, -1.0, rhs, 0.0, nullptr, rhs, s));
    st = cg_solve(c, op, MF_PC_JACOBI, rhs, dT, rtol, maxit, info, s);
    if (st < 0) return st;
    HIPCHK(c, vaxpbyz(1.0, T_old, 1.0, dT, T, c->nn, s));
    return st;
}

extern "C" mf_status mf_heat_step_adjoint(mf_ctx *c, const mf_operator *op, const double *T, const double *dT,
                                          const double *gT, const double *gdT, double rtol, int32_t maxit,
                                          double *dk_q, double *drc_q, double *dphi, double *gT_old,
                                          mf_solve_info *info, mf_stream stream)
{
    mf_status st = check_step_op(c, op, "mf_heat_step_adjoint");
    if (st) return st;
    if (!T || !dT || !info) return fail(c, MF_ERR_ARG, "null argument");
    if (dphi && op->coeff_mode != MF_COEFF_LEVELSET)
        return fail(c, MF_ERR_ARG, "dphi needs the LEVELSET coefficient mode");
    if (!(rtol >= 0.0) || maxit < 0) return fail(c, MF_ERR_ARG, "invalid rtol or maxit");
    hipStream_t s = (hipStream_t)stream;
    double *g, *lam;
    if ((st = ws_vec(c, 6, &g)) || (st = ws_vec(c, 7, &lam)) || (st = ensure_face(c, 1))) return st;
    // A lam = gT + gdT on the free rows (A is symmetric), lam = 0 on Dirichlet nodes
    HIPCHK(c, vmask_axpby(c->km, 1, 1.0, gT, 1.0, gdT, g, s));
    st = cg_solve(c, op, MF_PC_JACOBI, g, lam, rtol, maxit, info, s);
    if (st < 0) return st;
    if (dk_q || drc_q || dphi) HIPCHK(c, heat_grad(c->km, heat_args(op), T, dT, lam, dk_q, drc_q, dphi, c->face, s));
    if (gT_old) {
        // dL/dT_old = gT - (K lam) with every column: T = T_old + dT, and
        // T_old enters dT through the right-hand side -(K T_old) of the free rows
        HIPCHK(c, apply_without_mass(c, op, lam, g, s));
        if (gT) HIPCHK(c, vaxpbyz(1.0, gT, -1.0, g, gT_old, c->nn, s));
        else HIPCHK(c, vaxpbyz(0.0, g, -1.0, g, gT_old, c->nn, s));
    }
    return st;
}

extern "C" mf_status mf_heat_picard_step(mf_ctx *c, const mf_operator *op, const mf_heat_sources *src,
                                         const double *T_old, double *T, double tol, int32_t maxit, double cg_rtol,
                                         int32_t cg_maxit, mf_picard_info *info, double *updates, int32_t *cg_iters,
                                         mf_stream stream)
{
    mf_status st = check_op(c, op);
    if (st) return st;
    if (op->kind != MF_HEAT || op->precision != MF_FP64 || op->coeff_mode != MF_COEFF_LEVELSET || op->u0 ||
        op->T_coef)
        return fail(c, MF_ERR_ARG,
                    "mf_heat_picard_step needs an FP64 heat operator in LEVELSET mode without convection and "
                    "without T_coef (the coefficients follow the iterate)");
    if (!(op->T_liq > op->T_sol)) return fail(c, MF_ERR_ARG, "need T_sol < T_liq");
    if (!T_old || !T || !info || T == T_old) return fail(c, MF_ERR_ARG, "null or aliased argument");
    if (!(tol >= 0.0) || maxit < 1 || !(cg_rtol >= 0.0) || cg_maxit < 0)
        return fail(c, MF_ERR_ARG, "invalid tolerances or iteration limits");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = c->nn;
    double *rhs, *dT, *b = nullptr;
    if ((st = ws_vec(c, 6, &rhs)) || (st = ws_vec(c, 7, &dT)) || (st = ensure_face(c, 1))) return st;
    SourceArgs sa{};
    if (src) {
        if ((st = ws_vec(c, 8, &b))) return st;
        if ((st = source_args(c, op, src, T, &sa))) return st;
    }
    info->iterations = 0;
    info->converged = 0;
    info->cg_iterations = 0;
    info->update = 0.0;
    HIPCHK(c, vcopy(T_old, T, n, s));
    RedWS red = redws(c);
    for (int k = 0; k < maxit; ++k) {
        mf_operator o = *op; // coefficients frozen at the iterate T^k
        o.T_coef = T;
        const HeatArgs ha = heat_args(&o);
        if (b) {
            HeatArgs hs = ha;
            hs.conv = 0;
            HIPCHK(c, heat_sources(c->km, hs, sa, T, b, c->face, s));
        }
        // rhs = b(T^k) - (K(T^k) + R(T^k)) T_old on the free rows, 0 on Dirichlet rows
        HIPCHK(c, apply_without_mass(c, &o, T_old, rhs, s));
        HIPCHK(c, vmask_axpby(c->km, 1, 1.0, b, -1.0, rhs, rhs, s));
        mf_solve_info ci{};
        st = cg_solve(c, &o, MF_PC_JACOBI, rhs, dT, cg_rtol, cg_maxit, &ci, s);
        if (st < 0 || st == MF_BREAKDOWN) return st;
        info->cg_iterations += ci.iters;
        if (cg_iters) cg_iters[k] = ci.iters;
        // T^{k+1} = T_old + dT, with ||T^{k+1} - T^k||^2 and ||T^{k+1}||^2
        HIPCHK(c, picard_update(T_old, dT, T, n, c->scal, &red, s));
        HIPCHK(c, hipMemcpyAsync(c->h_scal, c->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        const double d2 = c->h_scal[0], n2 = c->h_scal[1];
        const double upd = n2 > 0.0 ? sqrt(d2 / n2) : (d2 > 0.0 ? INFINITY : 0.0);
        info->iterations = k + 1;
        info->update = upd;
        if (updates) updates[k] = upd;
        if (!isfinite(upd)) return fail(c, MF_BREAKDOWN, "Picard iterate is not finite at iteration %d", k + 1);
        if (upd <= tol) {
            info->converged = 1;
            return MF_OK;
        }
    }
    return fail(c, MF_NOT_CONVERGED, "Picard iteration reached maxit = %d (update %g)", maxit, info->update);
}
