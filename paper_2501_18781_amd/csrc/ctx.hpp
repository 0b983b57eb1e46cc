// ctx.hpp -- internal definition of the library context and the host
// helpers shared by api.hip (operators, CG, GMRES) and mg.hip (multigrid).
// Not part of the public boundary (include/mf.h).
#pragma once

#include <string>
#include <vector>

#include "mf.h"
#include "kernels.hpp"

struct mf_ctx {
    mf_mesh mesh;
    mf::KMesh km;
    int device = 0;
    int64_t nn = 0, nc = 0;
    std::string err;
    // workspace: vectors of 3 * n_nodes doubles each
    std::vector<double *> vec;
    double *partials = nullptr;
    unsigned cap = 0;
    mf::CGState *cg = nullptr;
    double *scal = nullptr;      // device scalars
    mf::CGState *h_state = nullptr;  // pinned host copy
    double *h_scal = nullptr;    // pinned host scalars
    double *V = nullptr;         // GMRES basis
    int V_cols = 0;
    double *blocks = nullptr;    // Oseen block-Jacobi inverse
    double *face = nullptr;      // shared-face partial sums of the brick kernels
    int64_t face_elems = 0;      // its capacity in doubles
    // mark the state copies a solve loop polls (created on first use; GMRES
    // alternates between the two)
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
    // kernel timing
    bool timing = false;
    std::vector<mf::KTiming> events;
    size_t events_used = 0;
};


#define HIPCHK(c, expr)                                                                             \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail((c), MF_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Record an error message on the context and return the status.
mf_status fail(mf_ctx *c, mf_status st, const char *fmt, ...);
mf::RedWS redws(mf_ctx *c);
// Face buffer for operators with `comps` components (allocated on demand).
mf_status ensure_face(mf_ctx *c, int comps);
// Workspace vector i of the context (3 * n_nodes doubles), allocated on first use.
mf_status ws_vec(mf_ctx *c, int i, double **out);
mf_status check_op(mf_ctx *c, const mf_operator *op);
// The descriptor checks of check_op; c may be null (messages then go to the
// calling thread's context-free error buffer, read by mf_last_error(NULL)).
mf_status check_op_desc(mf_ctx *c, const mf_operator *op);
// Validate a mesh descriptor and fill the kernels' mesh description (c may be null).
mf_status mesh_to_kmesh(mf_ctx *c, const mf_mesh *mesh, mf::KMesh *out, int64_t *n_nodes, int64_t *n_cells);
mf::HeatArgs heat_args(const mf_operator *op);
mf::OseenArgs oseen_args(const mf_operator *op);
int64_t ndofs(const mf_ctx *c, const mf_operator *op);
// y = A x or A^T x for any operator kind / precision; timed: record kernel events.
hipError_t apply_any(mf_ctx *c, const mf_operator *op, int transpose, const void *x, void *y, hipStream_t s,
                     bool timed = false);
// The two poll events of the context, created on first use.
hipError_t poll_events(mf_ctx *c);
// a.b read back to the host (synchronizes the stream).
mf_status host_dot(mf_ctx *c, const double *a, const double *b, int64_t n, double *out, hipStream_t s);
// ||b - A x|| / bnorm using workspace vector tmp.
mf_status true_residual(mf_ctx *c, const mf_operator *op, int transpose, const double *b, const double *x,
                        double *tmp, double bnorm, double *out, hipStream_t s);
// Jacobi-preconditioned (or plain) CG on a checked FP64 heat operator without
// convection, x0 = 0; workspace vectors 0-4.  Status and info as mf_cg_solve.
mf_status cg_solve(mf_ctx *c, const mf_operator *op, int precond, const double *b, double *x, double rtol, int maxit,
                   mf_solve_info *info, hipStream_t s);
// Kernel arguments of the interface heat sources of mf_heat_source_rhs.
mf_status source_args(mf_ctx *c, const mf_operator *op, const mf_heat_sources *src, const double *T,
                      mf::SourceArgs *out);
// Tanasawa coefficient alpha_v of mdot = alpha_v (T - T_v) (eq. mDotTanasawa)
// from the evaporation coefficient, molar mass, vapor density, boiling
// temperature and latent heat.
double tanasawa_coefficient(double gamma, double molar_mass, double vapor_density, double T_v, double h_v);
