// api.hip -- the C ABI declared in include/mf.h: contexts, argument
// checking, and the host loops of the Krylov solvers (App. B: CG for
// symmetric, GMRES for non-symmetric systems).  All arithmetic on vectors
// runs in the kernels of heat.hip, oseen.hip, vec.hip and mg.hip; the host
// only orchestrates, reads convergence scalars and runs the GMRES
// Hessenberg least-squares update on at most 31 numbers.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "ctx.hpp"

using namespace mf;

// Message of the last failed call that had no context, per host thread (a
// fixed buffer: recording it allocates nothing).
static thread_local char g_noctx_err[512] = "no context";

mf_status fail(mf_ctx *c, mf_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c ? buf : g_noctx_err, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return st;
}

// Validate a mesh descriptor and fill the kernels' mesh description.
mf_status mesh_to_kmesh(mf_ctx *c, const mf_mesh *mesh, KMesh *out, int64_t *n_nodes, int64_t *n_cells)
{
    if (!mesh) return fail(c, MF_ERR_ARG, "null mesh");
    int64_t nn = 1, nc = 1;
    for (int d = 0; d < 3; ++d) {
        if (mesh->n[d] < 1 || !(mesh->hi[d] > mesh->lo[d]))
            return fail(c, MF_ERR_ARG, "mesh needs n[d] >= 1 and hi[d] > lo[d]");
        nn *= 2 * (int64_t)mesh->n[d] + 1;
        nc *= mesh->n[d];
    }
    if (3 * nn >= (int64_t)1 << 31) return fail(c, MF_ERR_ARG, "mesh too large: 3 n_nodes must stay below 2^31");
    if (mesh->dirichlet > 63u) return fail(c, MF_ERR_ARG, "unknown Dirichlet face bits");
    KMesh k;
    k.nx = mesh->n[0];
    k.ny = mesh->n[1];
    k.nz = mesh->n[2];
    k.NX = 2 * k.nx + 1;
    k.NY = 2 * k.ny + 1;
    k.NZ = 2 * k.nz + 1;
    k.dirichlet = mesh->dirichlet;
    k.hx = (mesh->hi[0] - mesh->lo[0]) / mesh->n[0];
    k.hy = (mesh->hi[1] - mesh->lo[1]) / mesh->n[1];
    k.hz = (mesh->hi[2] - mesh->lo[2]) / mesh->n[2];
    k.lox = mesh->lo[0];
    k.loy = mesh->lo[1];
    k.loz = mesh->lo[2];
    *out = k;
    if (n_nodes) *n_nodes = nn;
    if (n_cells) *n_cells = nc;
    return MF_OK;
}

RedWS redws(mf_ctx *c) { return RedWS{c->partials, c->cap}; }

// Workspace vector i (3 * n_nodes doubles), allocated on first use.
mf_status ensure_face(mf_ctx *c, int comps)
{
    const int64_t need = comps * face_buffer_elems(c->km);
    if (c->face_elems >= need) return MF_OK;
    if (c->face) (void)hipFree(c->face); // synchronizes with work that may still use it
    c->face = nullptr;
    c->face_elems = 0;
    if (hipMalloc((void **)&c->face, sizeof(double) * need) != hipSuccess)
        return fail(c, MF_ERR_OOM, "face buffer allocation of %lld doubles failed", (long long)need);
    c->face_elems = need;
    return MF_OK;
}

mf_status ws_vec(mf_ctx *c, int i, double **out)
{
    while ((int)c->vec.size() <= i) c->vec.push_back(nullptr);
    if (!c->vec[i]) {
        if (hipMalloc((void **)&c->vec[i], sizeof(double) * 3 * c->nn) != hipSuccess)
            return fail(c, MF_ERR_OOM, "workspace allocation of %lld doubles failed", (long long)(3 * c->nn));
    }
    *out = c->vec[i];
    return MF_OK;
}

extern "C" {

int64_t mf_n_nodes(const mf_ctx *c) { return c ? c->nn : 0; }
int64_t mf_n_cells(const mf_ctx *c) { return c ? c->nc : 0; }

const char *mf_last_error(const mf_ctx *c) { return c ? c->err.c_str() : g_noctx_err; }

mf_status mf_create(const mf_mesh *mesh, mf_ctx **out)
{
    if (!mesh || !out) return MF_ERR_ARG;
    *out = nullptr;
    KMesh km;
    int64_t nn, nc;
    if (mesh_to_kmesh(nullptr, mesh, &km, &nn, &nc)) return MF_ERR_ARG;
    mf_ctx *c = new mf_ctx();
    c->mesh = *mesh;
    c->nn = nn;
    c->nc = nc;
    c->km = km;
    const KMesh &k = c->km;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return MF_ERR_HIP;
    }
    // reduction workspace: enough for one partial per heat brick and 64 sets of 1024 blocks
    const int64_t nbricks = ((k.nx + 3) / 4) * (int64_t)((k.ny + 3) / 4) * ((k.nz + 3) / 4);
    int64_t cap = nbricks > 64 * 1024 ? nbricks : 64 * 1024;
    c->cap = (unsigned)cap;
    bool ok = hipMalloc((void **)&c->partials, sizeof(double) * cap) == hipSuccess &&
              hipMalloc((void **)&c->cg, sizeof(CGState)) == hipSuccess &&
              hipMalloc((void **)&c->scal, sizeof(double) * 2048) == hipSuccess &&
              hipHostMalloc((void **)&c->h_state, sizeof(CGState), hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void **)&c->h_scal, sizeof(double) * 256, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        mf_destroy(c);
        return MF_ERR_OOM;
    }
    *out = c;
    return MF_OK;
}

void mf_destroy(mf_ctx *c)
{
    if (!c) return;
    for (double *p : c->vec)
        if (p) (void)hipFree(p);
    if (c->partials) (void)hipFree(c->partials);
    if (c->cg) (void)hipFree(c->cg);
    if (c->scal) (void)hipFree(c->scal);
    if (c->V) (void)hipFree(c->V);
    if (c->blocks) (void)hipFree(c->blocks);
    if (c->face) (void)hipFree(c->face);
    if (c->h_state) (void)hipHostFree(c->h_state);
    if (c->h_scal) (void)hipHostFree(c->h_scal);
    for (KTiming &t : c->events) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    for (hipEvent_t &e : c->poll_ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

mf_status mf_timing_enable(mf_ctx *c, int32_t on)
{
    if (!c) return MF_ERR_ARG;
    c->timing = on != 0;
    return MF_OK;
}

mf_status mf_timing_read(mf_ctx *c, double *ms, int64_t *launches, int32_t reset)
{
    if (!c || !ms || !launches) return MF_ERR_ARG;
    double tot = 0.0;
    for (size_t i = 0; i < c->events_used; ++i) {
        float f = 0.0f;
        HIPCHK(c, hipEventSynchronize(c->events[i].stop));
        HIPCHK(c, hipEventElapsedTime(&f, c->events[i].start, c->events[i].stop));
        tot += f;
    }
    *ms = tot;
    *launches = (int64_t)c->events_used;
    if (reset) c->events_used = 0;
    return MF_OK;
}

} // extern "C"

// ---------------------------------------------------------------------------
// Operator descriptors
// ---------------------------------------------------------------------------
mf_status check_op(mf_ctx *c, const mf_operator *op)
{
    if (!c) return MF_ERR_ARG;
    return check_op_desc(c, op);
}

mf_status check_op_desc(mf_ctx *c, const mf_operator *op)
{
    if (!op) return fail(c, MF_ERR_ARG, "null operator");
    if (op->kind != MF_HEAT && op->kind != MF_OSEEN) return fail(c, MF_ERR_ARG, "unknown operator kind %d", op->kind);
    if (op->precision != MF_FP64 && op->precision != MF_FP32)
        return fail(c, MF_ERR_ARG, "unknown precision %d", op->precision);
    if (op->heaviside != MF_H_LINEAR && op->heaviside != MF_H_SINE)
        return fail(c, MF_ERR_ARG, "unknown Heaviside form %d", op->heaviside);
    if (op->heaviside == MF_H_SINE && !(op->eps > 0.0)) return fail(c, MF_ERR_ARG, "sine Heaviside needs eps > 0");
    if (op->T_coef || op->penalty != 0.0) {
        if (op->precision != MF_FP64 || op->coeff_mode != MF_COEFF_LEVELSET)
            return fail(c, MF_ERR_ARG, "three-phase coefficients and the penalty need FP64 and LEVELSET mode");
        if (op->T_coef && !(op->T_liq > op->T_sol)) return fail(c, MF_ERR_ARG, "need T_sol < T_liq");
        if (op->kind == MF_HEAT && op->u0)
            return fail(c, MF_ERR_ARG, "convection with three-phase coefficients or the penalty is not provided");
        if (op->kind == MF_OSEEN && op->penalty != 0.0) return fail(c, MF_ERR_ARG, "the penalty is a heat term");
    }
    if (op->kind == MF_OSEEN && op->T_coef && op->darcy_C != 0.0 && !(op->darcy_b > 0.0))
        return fail(c, MF_ERR_ARG, "Darcy damping needs darcy_b > 0");
    if (op->kind == MF_HEAT) {
        if (op->u0 && (op->precision != MF_FP64 || op->coeff_mode != MF_COEFF_LEVELSET))
            return fail(c, MF_ERR_ARG, "the convective heat operator (u0 given) is FP64 in LEVELSET mode only");
        if (op->coeff_mode == MF_COEFF_LEVELSET) {
            if (!op->phi) return fail(c, MF_ERR_ARG, "heat operator in LEVELSET mode needs phi");
        } else if (op->coeff_mode == MF_COEFF_QUAD) {
            if (!op->k_q || !op->rc_q) return fail(c, MF_ERR_ARG, "heat operator in QUAD mode needs k_q and rc_q");
        } else {
            return fail(c, MF_ERR_ARG, "unknown coefficient mode %d", op->coeff_mode);
        }
    } else {
        if (op->precision != MF_FP64) return fail(c, MF_ERR_ARG, "the Oseen operator is FP64 only");
        if (!op->phi || !op->u0) return fail(c, MF_ERR_ARG, "the Oseen operator needs phi and u0");
        if (!(op->rho_l > 0.0) || !(op->rho_g > 0.0)) return fail(c, MF_ERR_ARG, "densities must be positive");
    }
    return MF_OK;
}

HeatArgs heat_args(const mf_operator *op)
{
    HeatArgs a;
    a.mode = op->coeff_mode == MF_COEFF_QUAD ? 1 : 0;
    a.hkind = op->heaviside;
    a.eps = op->eps;
    a.am = op->alpha_m;
    a.ak = op->alpha_k;
    a.k_l = op->k_l;
    a.k_g = op->k_g;
    a.rc_l = op->rc_l;
    a.rc_g = op->rc_g;
    a.phi = op->phi;
    a.kq = op->k_q;
    a.rcq = op->rc_q;
    a.conv = op->u0 ? 1 : 0;
    a.ac = op->alpha_c;
    a.u0 = (const double *)op->u0;
    a.k_s = op->k_s;
    a.rc_s = op->rc_s;
    a.T_sol = op->T_sol;
    a.T_liq = op->T_liq;
    a.penalty = op->penalty;
    a.tc = (const double *)op->T_coef;
    if (a.mode == 0 && (a.tc || a.penalty != 0.0)) a.mode = 2;
    return a;
}

OseenArgs oseen_args(const mf_operator *op)
{
    OseenArgs a;
    a.hkind = op->heaviside;
    a.eps = op->eps;
    a.am = op->alpha_m;
    a.ac = op->alpha_c;
    a.av = op->alpha_v;
    a.rho_l = op->rho_l;
    a.rho_g = op->rho_g;
    a.mu_l = op->mu_l;
    a.mu_g = op->mu_g;
    a.phi = (const double *)op->phi;
    a.u0 = (const double *)op->u0;
    a.rho_s = op->rho_s;
    a.mu_s = op->mu_s;
    a.T_sol = op->T_sol;
    a.T_liq = op->T_liq;
    a.darcy_C = op->darcy_C;
    a.darcy_b = op->darcy_b;
    a.tc = (const double *)op->T_coef;
    return a;
}

int64_t ndofs(const mf_ctx *c, const mf_operator *op) { return op->kind == MF_OSEEN ? 3 * c->nn : c->nn; }

// Next event pair for a timed launch (nullptr when timing is off).
static const KTiming *next_timing(mf_ctx *c)
{
    if (!c->timing) return nullptr;
    if (c->events_used == c->events.size()) {
        KTiming t;
        if (hipEventCreate(&t.start) != hipSuccess || hipEventCreate(&t.stop) != hipSuccess) return nullptr;
        c->events.push_back(t);
    }
    return &c->events[c->events_used++];
}

// y = A x or A^T x, FP64 or FP32 (heat)
hipError_t apply_any(mf_ctx *c, const mf_operator *op, int transpose, const void *x, void *y, hipStream_t s,
                     bool timed)
{
    if (ensure_face(c, op->kind == MF_OSEEN ? 3 : 1) != MF_OK) return hipErrorOutOfMemory;
    const KTiming *t = timed ? next_timing(c) : nullptr;
    if (op->kind == MF_HEAT) {
        HeatArgs ha = heat_args(op);
        if (transpose && ha.conv) ha.conv = 2; // without convection A^T = A
        return heat_apply(c->km, ha, op->precision == MF_FP32, x, y, c->face, nullptr, nullptr, s, t);
    }
    return oseen_apply(c->km, oseen_args(op), transpose, (const double *)x, (double *)y, c->face, s, t);
}

// Kernel arguments of the interface heat sources (scalars formed on the host).
mf_status source_args(mf_ctx *c, const mf_operator *op, const mf_heat_sources *src, const double *T,
                      SourceArgs *out)
{
    if (src->terms & ~(MF_SRC_EVAPORATION | MF_SRC_LASER | MF_SRC_PENALTY))
        return fail(c, MF_ERR_ARG, "unknown source terms");
    SourceArgs sa{};
    sa.terms = src->terms;
    if (src->terms & MF_SRC_PENALTY) {
        if (!(src->boiling_temperature > 0.0)) return fail(c, MF_ERR_ARG, "invalid boiling temperature");
        sa.penalty = op->penalty;
        sa.T_boil = src->boiling_temperature;
    }
    if (src->terms & MF_SRC_EVAPORATION) {
        const double gam = src->evaporation_coefficient;
        if (!T) return fail(c, MF_ERR_ARG, "evaporative cooling needs the temperature");
        if (!(gam > 0.0 && gam <= 1.0) || !(src->molar_mass > 0.0) || !(src->boiling_temperature > 0.0))
            return fail(c, MF_ERR_ARG, "invalid evaporation parameters");
        sa.alpha_v = tanasawa_coefficient(gam, src->molar_mass, src->vapor_density, src->boiling_temperature,
                                          src->latent_heat);
        sa.T_boil = src->boiling_temperature;
        sa.h_v = src->latent_heat;
    }
    if (src->terms & MF_SRC_LASER) {
        const double *e = src->direction;
        const double len = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        if (!(src->laser_radius > 0.0)) return fail(c, MF_ERR_ARG, "laser radius must be positive");
        if (!(fabs(len - 1.0) <= 1e-9)) return fail(c, MF_ERR_ARG, "laser direction must be a unit vector");
        sa.peak = 2.0 * src->absorptivity * src->laser_power / (M_PI * src->laser_radius * src->laser_radius);
        sa.inv_r2 = 1.0 / (src->laser_radius * src->laser_radius);
        for (int d = 0; d < 3; ++d) {
            sa.focus[d] = src->focus[d];
            sa.dir[d] = e[d];
        }
    }
    sa.c_rcp = 3.0 / (op->rc_g * op->rc_g + op->rc_l * op->rc_g + op->rc_l * op->rc_l);
    *out = sa;
    return MF_OK;
}

// Tanasawa: alpha_v = 2 gamma/(2 - gamma) h_v / sqrt(2 pi R_s) rho_v / T_v^{3/2}, R_s = R/M
// (eq. mDotTanasawa, mdot = alpha_v (T - T_v)).
double tanasawa_coefficient(double gamma, double molar_mass, double vapor_density, double T_v, double h_v)
{
    const double Rs = 8.314 / molar_mass;
    return 2.0 * gamma / (2.0 - gamma) * h_v / sqrt(2.0 * M_PI * Rs) * vapor_density / (T_v * sqrt(T_v));
}

extern "C" {

mf_status mf_operator_apply(mf_ctx *c, const mf_operator *op, const void *x, void *y, mf_stream stream)
{
    mf_status st = check_op(c, op);
    if (st) return st;
    if (!x || !y || x == y) return fail(c, MF_ERR_ARG, "x and y must be distinct non-null device arrays");
    HIPCHK(c, apply_any(c, op, 0, x, y, (hipStream_t)stream, true));
    return MF_OK;
}

mf_status mf_operator_apply_transpose(mf_ctx *c, const mf_operator *op, const void *x, void *y, mf_stream stream)
{
    mf_status st = check_op(c, op);
    if (st) return st;
    if (!x || !y || x == y) return fail(c, MF_ERR_ARG, "x and y must be distinct non-null device arrays");
    HIPCHK(c, apply_any(c, op, 1, x, y, (hipStream_t)stream, true));
    return MF_OK;
}

mf_status mf_operator_diagonal(mf_ctx *c, const mf_operator *op, void *diag, mf_stream stream)
{
    mf_status st = check_op(c, op);
    if (st) return st;
    if (!diag) return fail(c, MF_ERR_ARG, "null diag");
    if (op->kind == MF_HEAT) {
        if ((st = ensure_face(c, 1))) return st;
        HIPCHK(c, heat_diagonal(c->km, heat_args(op), op->precision == MF_FP32, diag, c->face, (hipStream_t)stream));
    } else {
        if ((st = ensure_face(c, 6))) return st;
        HIPCHK(c, oseen_block_diagonal(c->km, oseen_args(op), (double *)diag, c->face, (hipStream_t)stream));
    }
    return MF_OK;
}

mf_status mf_quad_points(mf_ctx *c, double *xq, mf_stream stream)
{
    if (!c) return MF_ERR_ARG;
    if (!xq) return fail(c, MF_ERR_ARG, "null xq");
    HIPCHK(c, quad_points(c->km, xq, (hipStream_t)stream));
    return MF_OK;
}

mf_status mf_heat_qp_coeffs(mf_ctx *c, const mf_operator *op, double *kq, double *rcq, mf_stream stream)
{
    mf_status st = check_op(c, op);
    if (st) return st;
    if (op->kind != MF_HEAT || op->coeff_mode != MF_COEFF_LEVELSET || op->precision != MF_FP64 || op->T_coef)
        return fail(c, MF_ERR_ARG, "mf_heat_qp_coeffs needs an FP64 two-phase heat operator in LEVELSET mode");
    if (!kq || !rcq) return fail(c, MF_ERR_ARG, "null output");
    HIPCHK(c, heat_qp_coeffs(c->km, heat_args(op), kq, rcq, (hipStream_t)stream));
    return MF_OK;
}

mf_status mf_heat_source_rhs(mf_ctx *c, const mf_operator *op, const mf_heat_sources *src, const double *T,
                             double *b, mf_stream stream)
{
    mf_status st = check_op(c, op);
    if (st) return st;
    if (op->kind != MF_HEAT || op->precision != MF_FP64 || op->coeff_mode != MF_COEFF_LEVELSET)
        return fail(c, MF_ERR_ARG, "mf_heat_source_rhs needs an FP64 heat operator in LEVELSET mode");
    if (!src || !b) return fail(c, MF_ERR_ARG, "null argument");
    SourceArgs sa{};
    if ((st = source_args(c, op, src, T, &sa))) return st;
    if ((st = ensure_face(c, 1))) return st;
    // the sources use the level set and rho c_p of the operator only (no convection)
    HeatArgs ha = heat_args(op);
    ha.conv = 0;
    HIPCHK(c, heat_sources(c->km, ha, sa, T ? T : (const double *)op->phi, b, c->face, (hipStream_t)stream));
    return MF_OK;
}

mf_status mf_transport_velocity(mf_ctx *c, const mf_transport_params *p, const double *phi, const double *u,
                                const double *T, double *u_gamma, mf_stream stream)
{
    if (!c) return MF_ERR_ARG;
    if (!p || !phi || !u || !T || !u_gamma) return fail(c, MF_ERR_ARG, "null argument");
    if (u_gamma == u) return fail(c, MF_ERR_ARG, "u_gamma must not alias u");
    if (p->variant != MF_TRANSPORT_LOCAL && p->variant != MF_TRANSPORT_LIQUID_EXTENSION)
        return fail(c, MF_ERR_ARG, "unknown transport-velocity variant %d", p->variant);
    if (p->heaviside != MF_H_LINEAR && p->heaviside != MF_H_SINE)
        return fail(c, MF_ERR_ARG, "unknown Heaviside form %d", p->heaviside);
    if (p->variant == MF_TRANSPORT_LIQUID_EXTENSION && p->heaviside != MF_H_SINE)
        return fail(c, MF_ERR_ARG, "the liquid-extension variant needs the sine Heaviside (H = 1 at d = 3 eps)");
    if (!(p->eps > 0.0)) return fail(c, MF_ERR_ARG, "eps must be positive");
    if (!(p->rho_l > 0.0) || !(p->rho_g > 0.0)) return fail(c, MF_ERR_ARG, "densities must be positive");
    if (c->km.NZ > 65535 || c->km.NY >= (1 << 23))
        return fail(c, MF_ERR_ARG, "the transport velocity takes at most 65535 nodes along z and 2^23 along y");
    const double gam = p->evaporation_coefficient;
    if (!(gam > 0.0 && gam <= 1.0) || !(p->molar_mass > 0.0) || !(p->boiling_temperature > 0.0))
        return fail(c, MF_ERR_ARG, "invalid evaporation parameters");
    TransportArgs a;
    a.variant = p->variant;
    a.hkind = p->heaviside;
    a.eps = p->eps;
    a.rho_l = p->rho_l;
    a.rho_g = p->rho_g;
    a.alpha_v = tanasawa_coefficient(gam, p->molar_mass, p->vapor_density, p->boiling_temperature, p->latent_heat);
    a.T_boil = p->boiling_temperature;
    double *dwork;
    mf_status st = ws_vec(c, 6, &dwork);
    if (st) return st;
    HIPCHK(c, transport_velocity(c->km, a, phi, u, T, u_gamma, dwork, (hipStream_t)stream));
    return MF_OK;
}

mf_status mf_heat_coeff_grad(mf_ctx *c, const mf_operator *op, const double *T, const double *dT,
                             const double *lambda, double *dk, double *drc, double *dphi, mf_stream stream)
{
    mf_status st = check_op(c, op);
    if (st) return st;
    if (op->kind != MF_HEAT || op->precision != MF_FP64 || op->u0 || op->T_coef || op->penalty != 0.0)
        return fail(c, MF_ERR_ARG, "mf_heat_coeff_grad needs an FP64 two-phase heat operator without convection");
    if (!T || !dT || !lambda) return fail(c, MF_ERR_ARG, "null input");
    if (dphi && op->coeff_mode != MF_COEFF_LEVELSET)
        return fail(c, MF_ERR_ARG, "dphi needs the LEVELSET coefficient mode");
    if (dphi && (st = ensure_face(c, 1))) return st;
    HIPCHK(c, heat_grad(c->km, heat_args(op), T, dT, lambda, dk, drc, dphi, c->face, (hipStream_t)stream));
    return MF_OK;
}

} // extern "C"

// ---------------------------------------------------------------------------
// Helpers for the solvers
// ---------------------------------------------------------------------------
hipError_t poll_events(mf_ctx *c)
{
    for (hipEvent_t &e : c->poll_ev)
        if (!e) {
            hipError_t err = hipEventCreateWithFlags(&e, hipEventDisableTiming);
            if (err != hipSuccess) return err;
        }
    return hipSuccess;
}

// a.b read back to the host (synchronizes the stream)
mf_status host_dot(mf_ctx *c, const double *a, const double *b, int64_t n, double *out, hipStream_t s)
{
    RedWS r = redws(c);
    HIPCHK(c, vmultidot(a, n, 1, b, n, c->scal, &r, s));
    HIPCHK(c, hipMemcpyAsync(c->h_scal, c->scal, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    *out = c->h_scal[0];
    return MF_OK;
}

// true relative residual ||b - A x|| / ||b||, using workspace vector `tmp`
mf_status true_residual(mf_ctx *c, const mf_operator *op, int transpose, const double *b, const double *x,
                               double *tmp, double bnorm, double *out, hipStream_t s)
{
    const int64_t n = ndofs(c, op);
    HIPCHK(c, apply_any(c, op, transpose, x, tmp, s));
    RedWS r = redws(c);
    HIPCHK(c, vdiffnorm2(b, tmp, n, c->scal, &r, s));
    HIPCHK(c, hipMemcpyAsync(c->h_scal, c->scal, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const double rr = c->h_scal[0];
    *out = bnorm > 0.0 ? sqrt(rr) / bnorm : 0.0;
    return MF_OK;
}

extern "C" mf_status mf_cg_solve(mf_ctx *c, const mf_operator *op, int32_t precond, const double *b, double *x,
                                 double rtol, int32_t maxit, mf_solve_info *info, mf_stream stream)
{
    mf_status st = check_op(c, op);
    if (st) return st;
    if (op->kind != MF_HEAT || op->precision != MF_FP64 || op->u0)
        return fail(c, MF_ERR_ARG, "mf_cg_solve needs a symmetric operator: FP64 heat without convection");
    if (precond != MF_PC_NONE && precond != MF_PC_JACOBI)
        return fail(c, MF_ERR_ARG, "mf_cg_solve supports MF_PC_NONE and MF_PC_JACOBI");
    if (!b || !x || !info) return fail(c, MF_ERR_ARG, "null argument");
    if (!(rtol >= 0.0) || maxit < 0) return fail(c, MF_ERR_ARG, "invalid rtol or maxit");
    return cg_solve(c, op, precond, b, x, rtol, maxit, info, (hipStream_t)stream);
}

// The CG iteration of mf_cg_solve on a checked symmetric heat operator;
// uses workspace vectors 0, 2, 3 and 4.
mf_status cg_solve(mf_ctx *c, const mf_operator *op, int precond, const double *b, double *x, double rtol, int maxit,
                   mf_solve_info *info, hipStream_t s)
{
    mf_status st;
    const int64_t n = c->nn;
    double *r, *p, *q, *dinv = nullptr;
    if ((st = ws_vec(c, 0, &r)) || (st = ws_vec(c, 2, &p)) || (st = ws_vec(c, 3, &q))) return st;
    const HeatArgs ha = heat_args(op);
    if ((st = ensure_face(c, 1))) return st;
    if (precond == MF_PC_JACOBI) {
        if ((st = ws_vec(c, 4, &dinv))) return st;
        HIPCHK(c, heat_diagonal(c->km, ha, 0, dinv, c->face, s, true));
    }
    RedWS red = redws(c);
    HIPCHK(c, cg_init(c->cg, b, dinv, x, r, p, n, rtol, maxit, 0, &red, s));
    // Iterations are launched in batches, each followed by a copy of the
    // state that the host polls.  While the host waits for that copy and
    // decides, the GPU already runs one more iteration (launched before the
    // wait), so it does not idle through the poll; an iteration launched
    // after convergence is a chain of no-op launches.  After the first batch
    // the next one is sized from the residual's decay so far (geometric
    // extrapolation to the threshold): that only sets how often the host
    // polls, never what is computed.
    HIPCHK(c, poll_events(c));
    auto iterate = [&](int k) -> hipError_t {
        for (int i = 0; i < k; ++i) {
            hipError_t e = heat_apply(c->km, ha, 0, p, q, c->face, c->cg, &red, s);
            if (e == hipSuccess) e = cg_resid(c->cg, dinv, r, q, n, &red, s);
            if (e == hipSuccess) e = cg_step(c->cg, x, r, p, n, &red, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    int batch = 8, launched = 8;
    double rr_prev = -1.0;
    int iters_prev = 0;
    HIPCHK(c, iterate(batch));
    for (;;) {
        HIPCHK(c, hipMemcpyAsync(c->h_state, c->cg, sizeof(CGState), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipEventRecord(c->poll_ev[0], s));
        HIPCHK(c, iterate(1)); // runs while the host polls
        launched += 1;
        HIPCHK(c, hipEventSynchronize(c->poll_ev[0]));
        const CGState &h = *c->h_state;
        if (h.done || launched >= maxit + 8) break;
        const double rr0 = rr_prev > 0.0 ? rr_prev : h.bb;
        const int dk = h.iter - iters_prev;
        batch = 8;
        if (dk > 0 && h.rr > 0.0 && rr0 > h.rr && h.thresh2 > 0.0) {
            const double rate = log(h.rr / rr0) / dk; // per iteration, < 0
            const double need = ceil(log(h.thresh2 / h.rr) / rate);
            batch = need < 1.0 ? 1 : (need > 16.0 ? 16 : (int)need);
        }
        batch = batch > 1 ? batch - 1 : 1; // one iteration is already queued
        rr_prev = h.rr;
        iters_prev = h.iter;
        HIPCHK(c, iterate(batch));
        launched += batch;
    }
    // The state copied at the last poll is final when it says done: the
    // iteration queued behind it only sets `run`.  Otherwise (the iteration
    // limit guard) read the state again.
    if (!c->h_state->done) {
        HIPCHK(c, hipMemcpyAsync(c->h_state, c->cg, sizeof(CGState), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    const CGState hs = *c->h_state;
    const double bnorm = sqrt(hs.bb);
    info->iters = hs.iter;
    info->rel_res_est = bnorm > 0.0 ? sqrt(hs.rr) / bnorm : 0.0;
    info->converged = !hs.breakdown && hs.rr <= hs.thresh2;
    if ((st = true_residual(c, op, 0, b, x, q, bnorm, &info->rel_res, s))) return st;
    if (hs.breakdown) return fail(c, MF_BREAKDOWN, "CG breakdown at iteration %d (p.Ap = %g)", hs.iter, hs.pAp);
    if (!info->converged) return fail(c, MF_NOT_CONVERGED, "CG reached maxit = %d", maxit);
    return MF_OK;
}

// ---------------------------------------------------------------------------
// GMRES(m), right preconditioned, Arnoldi by classical Gram-Schmidt applied twice
// (the second pass delayed by one step), Givens rotations (Saad Alg. 9.5)
// ---------------------------------------------------------------------------
extern "C" mf_status mf_gmres_solve(mf_ctx *c, const mf_operator *op, int32_t precond, int32_t restart,
                                    int32_t transpose, const double *b, double *x, double rtol, int32_t maxit,
                                    mf_solve_info *info, mf_stream stream)
{
    mf_status st = check_op(c, op);
    if (st) return st;
    if (op->precision != MF_FP64) return fail(c, MF_ERR_ARG, "mf_gmres_solve needs an FP64 operator");
    if (restart < 1 || restart > 31) return fail(c, MF_ERR_ARG, "restart must be in [1, 31]");
    if (!b || !x || !info) return fail(c, MF_ERR_ARG, "null argument");
    if (!(rtol >= 0.0) || maxit < 0) return fail(c, MF_ERR_ARG, "invalid rtol or maxit");
    if (precond == MF_PC_BLOCK_JACOBI && op->kind != MF_OSEEN)
        return fail(c, MF_ERR_ARG, "block Jacobi is defined for the 3-component Oseen operator");
    if (precond != MF_PC_NONE && precond != MF_PC_JACOBI && precond != MF_PC_BLOCK_JACOBI)
        return fail(c, MF_ERR_ARG, "unknown preconditioner %d", precond);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = ndofs(c, op);
    const int m = restart;
    // basis columns start on 512-byte boundaries (every wavefront's loads of
    // a column cover whole 128-byte lines)
    const int64_t ld = (3 * c->nn + 63) / 64 * 64;
    if (!c->V || c->V_cols < m + 1) {
        if (c->V) (void)hipFree(c->V);
        c->V = nullptr;
        if (hipMalloc((void **)&c->V, sizeof(double) * (int64_t)(m + 1) * ld) != hipSuccess)
            return fail(c, MF_ERR_OOM, "GMRES basis allocation failed");
        c->V_cols = m + 1;
    }
    double *V = c->V;
    double *tmp, *pc = nullptr;
    if ((st = ws_vec(c, 0, &tmp))) return st;
    // preconditioner setup
    if (precond == MF_PC_JACOBI) {
        if ((st = ws_vec(c, 1, &pc))) return st;
        if (op->kind == MF_HEAT) {
            if ((st = ensure_face(c, 1))) return st;
            HIPCHK(c, heat_diagonal(c->km, heat_args(op), 0, pc, c->face, s));
        } else {
            // diagonal of the 3x3 blocks
            if (!c->blocks && hipMalloc((void **)&c->blocks, sizeof(double) * 9 * c->nn) != hipSuccess)
                return fail(c, MF_ERR_OOM, "block allocation failed");
            if ((st = ensure_face(c, 6))) return st;
            HIPCHK(c, oseen_block_diagonal(c->km, oseen_args(op), c->blocks, c->face, s));
            for (int comp = 0; comp < 3; ++comp)
                HIPCHK(c, hipMemcpy2DAsync(pc + comp * c->nn, sizeof(double), c->blocks + 4 * comp, 9 * sizeof(double),
                                           sizeof(double), c->nn, hipMemcpyDeviceToDevice, s));
        }
        HIPCHK(c, vinv(pc, n, s));
    } else if (precond == MF_PC_BLOCK_JACOBI) {
        if (!c->blocks && hipMalloc((void **)&c->blocks, sizeof(double) * 9 * c->nn) != hipSuccess)
            return fail(c, MF_ERR_OOM, "block allocation failed");
        if ((st = ensure_face(c, 6))) return st;
        HIPCHK(c, oseen_block_diagonal(c->km, oseen_args(op), c->blocks, c->face, s));
        HIPCHK(c, block3_invert(c->blocks, c->nn, s));
    }
    double *zt;
    if ((st = ws_vec(c, 2, &zt))) return st;
    auto prec = [&](const double *in, double *out) -> hipError_t {
        if (precond == MF_PC_JACOBI) return vmul(pc, in, out, n, s);
        if (precond == MF_PC_BLOCK_JACOBI) {
            if (transpose) return hipErrorInvalidValue; // handled below by not allowing it
            return block3_apply(c->blocks, in, out, c->nn, s);
        }
        return vcopy(in, out, n, s);
    };
    if (precond == MF_PC_BLOCK_JACOBI && transpose)
        return fail(c, MF_ERR_ARG, "block Jacobi for the transposed system is not provided");

    RedWS red = redws(c);
    double bnorm2;
    if ((st = host_dot(c, b, b, n, &bnorm2, s))) return st;
    const double bnorm = sqrt(bnorm2);
    HIPCHK(c, vfill(x, 0.0, n, 0, s));
    info->iters = 0;
    info->converged = 0;
    info->rel_res = 1.0;
    info->rel_res_est = 1.0;
    if (bnorm == 0.0) {
        info->converged = 1;
        info->rel_res = info->rel_res_est = 0.0;
        return MF_OK;
    }
    std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), h(m + 1);
    int total = 0;
    bool conv = false;
    while (total < maxit) {
        // r = b - A x into V_0
        HIPCHK(c, apply_any(c, op, transpose, x, tmp, s));
        HIPCHK(c, vcopy(b, V, n, s));
        HIPCHK(c, vaxpby(-1.0, tmp, 1.0, V, n, s));
        double beta2;
        if ((st = host_dot(c, V, V, n, &beta2, s))) return st;
        const double beta = sqrt(beta2);
        info->rel_res = beta / bnorm;
        if (beta / bnorm <= rtol) {
            conv = true;
            break;
        }
        HIPCHK(c, vaxpby(1.0 / beta, V, 0.0, V, n, s));
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jdone = 0;
        // Arnoldi with delayed re-orthogonalization on the device: step j
        // forms w = A M^-1 u_j from the once-orthogonalized candidate u_j,
        // completes column j - 1 of the Hessenberg matrix with one pass
        // over the basis, and with a second pass writes q_j and the next
        // candidate (two passes per step).  The closing step of a cycle
        // only completes the last column.  Column j - 1 is copied to slot
        // j mod 2 of the host scalars; while the host applies the Givens
        // rotations to it, the GPU already runs step j + 1 (a step launched
        // past the end of the cycle is not used).
        const int mc = std::min(m, maxit - total); // columns of this cycle at most
        double *Hd = c->scal + 512;
        HIPCHK(c, vfill(Hd, 0.0, DGS_LDH * DGS_LDH, 0, s));
        auto step = [&](int j) -> hipError_t {
            const bool full = j < mc;
            double *u = V + (int64_t)j * ld, *w = full ? V + (int64_t)(j + 1) * ld : u;
            double *coef = c->scal + 1536 + (j & 1) * 128, *col = c->scal + 1792 + (j & 1) * 64;
            hipError_t e = hipSuccess;
            if (full) {
                e = prec(u, zt);
                if (e == hipSuccess) e = apply_any(c, op, transpose, zt, w, s);
            }
            if (e == hipSuccess) e = dgs_step(V, ld, j, full, u, w, n, Hd, coef, col, &red, s);
            if (e == hipSuccess && j > 0)
                e = hipMemcpyAsync(c->h_scal + (j & 1) * 64, col, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipEventRecord(c->poll_ev[j & 1], s);
            return e;
        };
        HIPCHK(c, poll_events(c));
        HIPCHK(c, step(0));
        HIPCHK(c, step(1));
        for (int j = 0; j < mc; ++j) {
            // column j is completed by step j + 1, launched already; queue step j + 2
            if (j + 2 <= mc) HIPCHK(c, step(j + 2));
            HIPCHK(c, hipEventSynchronize(c->poll_ev[(j + 1) & 1]));
            ++total;
            const double *hh = c->h_scal + ((j + 1) & 1) * 64;
            for (int i = 0; i <= j + 1; ++i) H[i * m + j] = hh[i];
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
                H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
                H[i * m + j] = t;
            }
            const double den = hypot(H[j * m + j], H[(j + 1) * m + j]);
            if (!(den > 0.0) || !isfinite(den)) {
                info->iters = total;
                HIPCHK(c, hipStreamSynchronize(s)); // a step launched ahead may still use the host copies
                return fail(c, MF_BREAKDOWN, "GMRES breakdown at step %d", total);
            }
            cs[j] = H[j * m + j] / den;
            sn[j] = H[(j + 1) * m + j] / den;
            H[j * m + j] = den;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            jdone = j + 1;
            info->rel_res_est = fabs(g[j + 1]) / bnorm;
            if (info->rel_res_est <= rtol || total >= maxit) break;
        }
        // y = H^{-1} g (upper triangular), x += M^{-1} V y
        for (int i = jdone - 1; i >= 0; --i) {
            double v = g[i];
            for (int k = i + 1; k < jdone; ++k) v -= H[i * m + k] * h[k];
            h[i] = v / H[i * m + i];
        }
        HIPCHK(c, hipMemcpyAsync(c->scal, h.data(), sizeof(double) * jdone, hipMemcpyHostToDevice, s));
        HIPCHK(c, vcombine(V, ld, jdone, c->scal, tmp, n, s));
        HIPCHK(c, prec(tmp, zt));
        HIPCHK(c, vaxpby(1.0, zt, 1.0, x, n, s));
        HIPCHK(c, hipStreamSynchronize(s)); // h is a host vector reused by the next cycle
    }
    info->iters = total;
    double tr;
    if ((st = true_residual(c, op, transpose, b, x, tmp, bnorm, &tr, s))) return st;
    info->rel_res = tr;
    info->converged = tr <= rtol;
    if (!info->converged) return fail(c, MF_NOT_CONVERGED, "GMRES reached maxit = %d (rel. res. %g)", maxit, tr);
    (void)conv;
    return MF_OK;
}
