// mg.hip -- FP32 geometric multigrid preconditioner for the heat operator,
// and flexible CG in FP64 preconditioned by it.
//
// Levels: the fine mesh and its uniform coarsenings (cells halved per
// direction) down to `coarse_cells` cells.  Every level is rediscretized
// with the level set injected to the coarse nodes; all levels but the
// coarsest apply the operator in FP32, the coarsest is solved by FP64 CG
// (App. B: CG for symmetric systems) with a Jacobi preconditioner.
//
// Level rule (auto_levels): coarsening stops at the first level, from the
// finest down, on which the mass term dominates the diagonal of A at every
// node:
//   beta_l = 17.5 (1/hx^2 + 1/hy^2 + 1/hz^2) max_phase alpha_k k / (alpha_m rc) <= beta_stop,
// 17.5 being the largest ratio of the 1D Q2 stiffness to mass diagonal
// entries (a vertex node: (14/3) / (8/30), against 10 at a midpoint), and the
// arithmetic blends of k and rc never exceeding the larger phase ratio.  Then
// D^{-1} A is within the factor (1 + beta) of the Jacobi-scaled mass matrix
// from below, its spectrum is in the smoother's reach and a coarse-grid
// correction would only add work: the level becomes the coarsest and is
// treated by Chebyshev smoothing (degree smooth_degree) over the Lanczos
// estimate [lambda_min / safety, safety lambda_max] of its spectrum, which
// converges fast for such a well-conditioned operator.  In the
// mass-dominated regime (small time steps) this is already the finest level.
//
// Transfer: P is the embedding of the coarse Q2 space into the fine one
// (coarse Q2 functions are fine Q2 functions): in 1D a fine node at a coarse
// node takes its value, the fine nodes at the quarter points of a coarse
// cell take (3/8, 3/4, -1/8) and (-1/8, 3/4, 3/8) of the cell's three coarse
// nodes; in 3D the tensor product.  Restriction R = P^T.  Rows of P at
// Dirichlet fine nodes and columns at Dirichlet coarse nodes are zero.
//
// Smoother: Chebyshev iteration of degree k on D^{-1} A over
// [lambda_max / range, lambda_max] (Saad, Iterative Methods, Alg. 12.1, with
// the residual updated recursively); lambda_max = safety x the largest
// eigenvalue of the Lanczos tridiagonal matrix of D^{-1/2} A D^{-1/2} after
// a fixed number of steps from a deterministic start vector (Knuth's
// multiplicative hash).  The V-cycle: pre-smoothing from zero, residual,
// restriction, coarse correction, prolongation, post-smoothing.
#include <math.h>
#include <stdint.h>

#include <vector>

#include "ctx.hpp"

using namespace mf;

namespace mf {

#define GSTRIDE(i, n) for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

static unsigned grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 65535 * 16) b = 65535 * 16;
    return (unsigned)(b < 1 ? 1 : b);
}

// 1D transfer taps.  Prolongation, fine node t from coarse nodes s0..s0+2:
// t even: the coincident coarse node t/2; t = 4c+1 and t = 4c+3: the quarter
// points of coarse cell c, weights (3/8, 3/4, -1/8) and (-1/8, 3/4, 3/8).
// Unused taps get weight 0 and a valid index.  A tap on a Dirichlet face of
// the coarse mesh (direction bits lo/hi) gets weight 0 (column zeroed).
__device__ __forceinline__ void prolong_taps(int t, int NC, bool dlo, bool dhi, int &s0, float *w)
{
    if ((t & 1) == 0) {
        const int sc = t >> 1;
        s0 = sc < NC - 3 ? sc : NC - 3; // NC >= 3: three valid indices
        const int k = sc - s0;
        w[0] = k == 0 ? 1.0f : 0.0f;
        w[1] = k == 1 ? 1.0f : 0.0f;
        w[2] = k == 2 ? 1.0f : 0.0f;
    } else {
        s0 = 2 * (t >> 2);
        const bool first = (t & 3) == 1;
        w[0] = first ? 0.375f : -0.125f;
        w[1] = 0.75f;
        w[2] = first ? -0.125f : 0.375f;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int sk = s0 + k;
        if ((dlo && sk == 0) || (dhi && sk == NC - 1)) w[k] = 0.0f;
    }
}

// Restriction (transpose), coarse node s from fine nodes: s even:
// 2s-3, 2s-1, 2s, 2s+1, 2s+3 with (-1/8, 3/8, 1, 3/8, -1/8); s odd: 2s-1,
// 2s, 2s+1 with (3/4, 1, 3/4), padded to five taps.  Taps outside the fine
// mesh or on its Dirichlet faces get weight 0 (rows of P zeroed).
__device__ __forceinline__ void restrict_taps(int s, int NF, bool dlo, bool dhi, int *t, float *w)
{
    if ((s & 1) == 0) {
        const int tt[5] = {2 * s - 3, 2 * s - 1, 2 * s, 2 * s + 1, 2 * s + 3};
        const float ww[5] = {-0.125f, 0.375f, 1.0f, 0.375f, -0.125f};
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            t[k] = tt[k];
            w[k] = ww[k];
        }
    } else {
        const int tt[5] = {2 * s - 1, 2 * s, 2 * s + 1, 2 * s, 2 * s};
        const float ww[5] = {0.75f, 1.0f, 0.75f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            t[k] = tt[k];
            w[k] = ww[k];
        }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const bool out = t[k] < 0 || t[k] > NF - 1;
        if (out || (dlo && t[k] == 0) || (dhi && t[k] == NF - 1)) w[k] = 0.0f;
        if (out) t[k] = 2 * s;
    }
}

// The transfers are separable, P = P_z P_y P_x with the 1D operators above,
// and are applied one direction at a time, each pass a streaming kernel over
// its output with the 1D taps of one line (coalesced along x; the y and z
// passes read whole rows).  Prolongation: x, y, then z (adding into the fine
// vector); restriction: z, y, then x.  The Dirichlet zeroing is per
// direction (a tap on a Dirichlet face has weight 0), so it factors too.
// The intermediate arrays are two fine-level work vectors.
constexpr int XNT = 256; // threads per transfer workgroup

// Position of the thread in an (NX x NY) plane of a 3D array: grid
// (ceil(NX NY / XNT), NZ); the row is split by a single-precision estimate
// and one correction (exact for NY < 2^23).
struct PlanePos {
    int x, y, z;
    bool ok;
    __device__ __forceinline__ PlanePos(int NX, int NY)
    {
        const unsigned p = blockIdx.x * XNT + threadIdx.x, nx = (unsigned)NX;
        ok = p < nx * (unsigned)NY;
        unsigned q = (unsigned)((float)p * (1.0f / (float)nx));
        if (q * nx > p) --q;
        else if ((q + 1) * nx <= p) ++q;
        x = (int)(p - q * nx);
        y = (int)q;
        z = blockIdx.y;
    }
};

// Prolongation pass along direction DIR: out(.., t, ..) = sum_k w_k in(.., s0 + k, ..)
// with t the fine index along DIR; in has NC nodes along DIR, out NF.
// (nx, ny, nz): out's extents; the in extent along DIR is NC.
template <int DIR, bool ADD>
__global__ void __launch_bounds__(XNT) prolong_pass_kernel(const float *__restrict__ in, float *__restrict__ out,
                                                           int nx, int ny, int nz, int NC, unsigned dmask,
                                                           KMesh f)
{
    const PlanePos P(nx, ny);
    if (!P.ok) return;
    const int t = DIR == 0 ? P.x : (DIR == 1 ? P.y : P.z);
    if (ADD && node_constrained(f, P.x, P.y, P.z)) return; // rows of P at Dirichlet fine nodes
    int s0;
    float w[3];
    prolong_taps(t, NC, dmask & 1u, dmask & 2u, s0, w);
    const int inx = DIR == 0 ? NC : nx, iny = DIR == 1 ? NC : ny;
    const int64_t sd = DIR == 0 ? 1 : (DIR == 1 ? (int64_t)inx : (int64_t)inx * iny);
    const int ix = DIR == 0 ? s0 : P.x, iy = DIR == 1 ? s0 : P.y, iz = DIR == 2 ? s0 : P.z;
    const float *src = in + (int64_t)ix + (int64_t)inx * ((int64_t)iy + (int64_t)iny * iz);
    const float v = w[0] * src[0] + w[1] * src[sd] + w[2] * src[2 * sd];
    float *dst = out + (int64_t)P.x + (int64_t)nx * ((int64_t)P.y + (int64_t)ny * P.z);
    if (ADD) *dst += v;
    else *dst = v;
}

// Restriction pass along DIR: out(.., s, ..) = sum_k w_k in(.., t_k, ..), s the
// coarse index along DIR; in has NF nodes along DIR.  The last pass (x)
// writes 0 at the coarse Dirichlet nodes.
template <int DIR, bool LAST>
__global__ void __launch_bounds__(XNT) restrict_pass_kernel(const float *__restrict__ in, float *__restrict__ out,
                                                            int nx, int ny, int nz, int NF, unsigned dmask,
                                                            KMesh c)
{
    const PlanePos P(nx, ny);
    if (!P.ok) return;
    float *dst = out + (int64_t)P.x + (int64_t)nx * ((int64_t)P.y + (int64_t)ny * P.z);
    if (LAST && node_constrained(c, P.x, P.y, P.z)) {
        *dst = 0.0f;
        return;
    }
    const int sc = DIR == 0 ? P.x : (DIR == 1 ? P.y : P.z);
    int t[5];
    float w[5];
    restrict_taps(sc, NF, dmask & 1u, dmask & 2u, t, w);
    const int inx = DIR == 0 ? NF : nx, iny = DIR == 1 ? NF : ny;
    const int64_t sd = DIR == 0 ? 1 : (DIR == 1 ? (int64_t)inx : (int64_t)inx * iny);
    const int64_t base = (DIR == 0 ? 0 : P.x) + (int64_t)inx * ((DIR == 1 ? 0 : P.y) + (int64_t)iny * (DIR == 2 ? 0 : P.z));
    float v = 0.0f;
#pragma unroll
    for (int k = 0; k < 5; ++k) v += w[k] * in[base + sd * t[k]];
    *dst = v;
}

template <typename T> __global__ void inject_kernel(KMesh f, KMesh c, const T *__restrict__ pf, T *__restrict__ pc)
{
    const int64_t ncn = (int64_t)c.NX * c.NY * c.NZ;
    GSTRIDE(i, ncn)
    {
        const int sx = (int)(i % c.NX), sy = (int)((i / c.NX) % c.NY), sz = (int)(i / ((int64_t)c.NX * c.NY));
        pc[i] = pf[node_index(f, 2 * sx, 2 * sy, 2 * sz)];
    }
}

// First Chebyshev step on the residual r = b - t (t null: x starts from zero
// and r = b): d = D^{-1} r / theta, then x = d or x += d.  With MORE steps to
// follow, r and d are stored; from zero neither r (the next step reads b)
// nor x (the next step forms x = d + d') is written.
template <bool XZERO, bool MORE>
__global__ void cheb_first_kernel(const float *__restrict__ dinv, const float *__restrict__ b,
                                  const float *__restrict__ t, float *__restrict__ r, float *__restrict__ d,
                                  float *__restrict__ x, float inv_theta, int64_t n)
{
    GSTRIDE(i, n)
    {
        const float ri = XZERO ? b[i] : b[i] - t[i];
        if (MORE && !XZERO) r[i] = ri;
        const float di = dinv[i] * ri * inv_theta;
        if (MORE) d[i] = di;
        if (!XZERO) x[i] += di;
        else if (!MORE) x[i] = di;
    }
}

// Chebyshev step: r = rin - A d, d = c1 d + c2 D^{-1} r, x += d (x = d_old + d
// right after a first step from zero).  The last step stores x only.  rin and
// r may be the same vector.
template <bool XPREV_D, bool LAST>
__global__ void cheb_step_kernel(const float *__restrict__ dinv, const float *rin, const float *__restrict__ Ad,
                                 float *r, float *__restrict__ d, float *__restrict__ x, float c1, float c2, int64_t n)
{
    GSTRIDE(i, n)
    {
        const float ri = rin[i] - Ad[i];
        if (!LAST) r[i] = ri;
        const float dold = d[i];
        const float di = c1 * dold + c2 * dinv[i] * ri;
        if (!LAST) d[i] = di;
        x[i] = (XPREV_D ? dold : x[i]) + di;
    }
}

__global__ void sub_f_kernel(const float *__restrict__ b, const float *__restrict__ Ax, float *__restrict__ r, int64_t n)
{
    GSTRIDE(i, n) r[i] = b[i] - Ax[i];
}

__global__ void knuth_kernel(double *__restrict__ v, int64_t n)
{
    GSTRIDE(i, n)
    {
        const uint32_t h = (uint32_t)i * 2654435761u; // wraps modulo 2^32
        v[i] = (double)h / 4294967296.0 - 0.5;
    }
}

__global__ void sqrt_kernel(const double *__restrict__ d, double *__restrict__ s, int64_t n) { GSTRIDE(i, n) s[i] = sqrt(d[i]); }

static dim3 plane_grid(int nx, int ny, int nz)
{
    return dim3((unsigned)(((int64_t)nx * ny + XNT - 1) / XNT), (unsigned)nz);
}

hipError_t mg_restrict(const KMesh &fine, const KMesh &coarse, const float *rf, float *rc, float *w1, float *w2,
                       hipStream_t s)
{
    const unsigned D = fine.dirichlet;
    // z: (NXf, NYf, NZc) <- rf;  y: (NXf, NYc, NZc);  x: (NXc, NYc, NZc) = rc
    restrict_pass_kernel<2, false><<<plane_grid(fine.NX, fine.NY, coarse.NZ), XNT, 0, s>>>(
        rf, w2, fine.NX, fine.NY, coarse.NZ, fine.NZ, (D >> 4) & 3u, coarse);
    restrict_pass_kernel<1, false><<<plane_grid(fine.NX, coarse.NY, coarse.NZ), XNT, 0, s>>>(
        w2, w1, fine.NX, coarse.NY, coarse.NZ, fine.NY, (D >> 2) & 3u, coarse);
    restrict_pass_kernel<0, true><<<plane_grid(coarse.NX, coarse.NY, coarse.NZ), XNT, 0, s>>>(
        w1, rc, coarse.NX, coarse.NY, coarse.NZ, fine.NX, D & 3u, coarse);
    return hipGetLastError();
}

hipError_t mg_prolong_add(const KMesh &coarse, const KMesh &fine, const float *ec, float *xf, float *w1, float *w2,
                          hipStream_t s)
{
    const unsigned D = coarse.dirichlet;
    // x: (NXf, NYc, NZc) <- ec;  y: (NXf, NYf, NZc);  z: xf (NXf, NYf, NZf) +=
    prolong_pass_kernel<0, false><<<plane_grid(fine.NX, coarse.NY, coarse.NZ), XNT, 0, s>>>(
        ec, w1, fine.NX, coarse.NY, coarse.NZ, coarse.NX, D & 3u, fine);
    prolong_pass_kernel<1, false><<<plane_grid(fine.NX, fine.NY, coarse.NZ), XNT, 0, s>>>(
        w1, w2, fine.NX, fine.NY, coarse.NZ, coarse.NY, (D >> 2) & 3u, fine);
    prolong_pass_kernel<2, true><<<plane_grid(fine.NX, fine.NY, fine.NZ), XNT, 0, s>>>(
        w2, xf, fine.NX, fine.NY, fine.NZ, coarse.NZ, (D >> 4) & 3u, fine);
    return hipGetLastError();
}

hipError_t mg_inject(const KMesh &fine, const KMesh &coarse, const void *phif, void *phic, int fp32, hipStream_t s)
{
    const unsigned g = grid_for((int64_t)coarse.NX * coarse.NY * coarse.NZ);
    if (fp32) inject_kernel<float><<<g, 256, 0, s>>>(fine, coarse, (const float *)phif, (float *)phic);
    else inject_kernel<double><<<g, 256, 0, s>>>(fine, coarse, (const double *)phif, (double *)phic);
    return hipGetLastError();
}

hipError_t cheb_first(const float *dinv, const float *b, const float *t, float *r, float *d, float *x, float inv_theta,
                      bool more, int64_t n, hipStream_t s)
{
    const unsigned g = grid_for(n);
    if (!t) {
        if (more) cheb_first_kernel<true, true><<<g, 256, 0, s>>>(dinv, b, t, r, d, x, inv_theta, n);
        else cheb_first_kernel<true, false><<<g, 256, 0, s>>>(dinv, b, t, r, d, x, inv_theta, n);
    } else {
        if (more) cheb_first_kernel<false, true><<<g, 256, 0, s>>>(dinv, b, t, r, d, x, inv_theta, n);
        else cheb_first_kernel<false, false><<<g, 256, 0, s>>>(dinv, b, t, r, d, x, inv_theta, n);
    }
    return hipGetLastError();
}

hipError_t cheb_step(const float *dinv, const float *rin, const float *Ad, float *r, float *d, float *x, float c1,
                     float c2, bool xprev_d, bool last, int64_t n, hipStream_t s)
{
    const unsigned g = grid_for(n);
    if (xprev_d) {
        if (last) cheb_step_kernel<true, true><<<g, 256, 0, s>>>(dinv, rin, Ad, r, d, x, c1, c2, n);
        else cheb_step_kernel<true, false><<<g, 256, 0, s>>>(dinv, rin, Ad, r, d, x, c1, c2, n);
    } else {
        if (last) cheb_step_kernel<false, true><<<g, 256, 0, s>>>(dinv, rin, Ad, r, d, x, c1, c2, n);
        else cheb_step_kernel<false, false><<<g, 256, 0, s>>>(dinv, rin, Ad, r, d, x, c1, c2, n);
    }
    return hipGetLastError();
}

hipError_t vsub_f(const float *b, const float *Ax, float *r, int64_t n, hipStream_t s)
{
    sub_f_kernel<<<grid_for(n), 256, 0, s>>>(b, Ax, r, n);
    return hipGetLastError();
}

hipError_t vknuth(double *v, int64_t n, hipStream_t s)
{
    knuth_kernel<<<grid_for(n), 256, 0, s>>>(v, n);
    return hipGetLastError();
}

hipError_t vsqrt(const double *d, double *out, int64_t n, hipStream_t s)
{
    sqrt_kernel<<<grid_for(n), 256, 0, s>>>(d, out, n);
    return hipGetLastError();
}

} // namespace mf

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// Largest (or smallest) eigenvalue of the symmetric tridiagonal matrix
// (a, b) by bisection on the Sturm count of the LDL^T pivots.
static double tridiag_extreme_eig(const std::vector<double> &a, const std::vector<double> &b, bool largest)
{
    const int n = (int)a.size();
    double lo = a[0], hi = a[0];
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i < n - 1 ? fabs(b[i]) : 0.0);
        lo = fmin(lo, a[i] - r);
        hi = fmax(hi, a[i] + r);
    }
    auto count_below = [&](double x) {
        int cnt = 0;
        double d = 1.0;
        for (int i = 0; i < n; ++i) {
            d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0.0) ++cnt;
        }
        return cnt;
    };
    const int target = largest ? n : 1; // eigenvalues below x: all of them, or at least one
    for (int it = 0; it < 200 && hi - lo > 1e-15 * fmax(fabs(lo), fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (count_below(mid) >= target) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

struct MGLevel {
    mf_ctx *ctx = nullptr;     // mesh context of the level (workspace, face buffer)
    mf_mesh mesh;
    int64_t nn = 0;
    double *phi64 = nullptr;   // level set, FP64 (owned except on the finest level)
    bool own_phi64 = false;
    float *phi32 = nullptr;
    float *dinv = nullptr;     // FP32 inverse diagonal
    float *b = nullptr, *x = nullptr, *r = nullptr, *d = nullptr, *t = nullptr;
    double lmax = 0.0, lmin = 0.0;
    double est_max = 0.0, est_min = 0.0; // Lanczos Ritz extremes of D^{-1} A (0: not estimated)
    int degree = 0;                      // Chebyshev degree (0: the level is solved by CG)
    mf_operator op32, op64;
};

struct mf_mg {
    mf_ctx *parent = nullptr;
    mf_operator fine_op;
    mf_mg_params prm;
    std::vector<MGLevel> L; // 0 = coarsest
    bool smooth_coarsest = false;          // the coarsest level is smoothed, not solved (level rule)
    double *b64 = nullptr, *x64 = nullptr; // coarse FP64 right-hand side and solution
    double *cinv = nullptr;                // A^-1 of a one-brick coarsest level (FP64, column-major)
};

static mf_status mg_fail(mf_mg *mg, mf_status st, const char *msg)
{
    return fail(mg ? mg->parent : nullptr, st, "%s", msg);
}

#define MGCHK(mg, expr)                                                                                   \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess) return fail((mg)->parent, MF_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

static void level_free(MGLevel &l)
{
    if (l.own_phi64 && l.phi64) (void)hipFree(l.phi64);
    for (void *p : {(void *)l.phi32, (void *)l.dinv, (void *)l.b, (void *)l.x, (void *)l.r, (void *)l.d, (void *)l.t})
        if (p) (void)hipFree(p);
    if (l.ctx) mf_destroy(l.ctx);
    l = MGLevel();
}

// x = A^-1 b on a one-brick coarsest level (n <= 729 nodes): workgroup r0
// takes rows r0 .. r0 + 63; its 16 wavefronts split the columns (every
// 16th), each reading 64 consecutive entries of a column per load and
// keeping four loads in flight.
constexpr int CINV_MAXN = 729, CINV_WAVES = 16;
__global__ void __launch_bounds__(64 * CINV_WAVES) coarse_inverse_apply_kernel(const double *__restrict__ inv, int n,
                                                                               const float *__restrict__ b,
                                                                               float *__restrict__ x)
{
    constexpr int S = CINV_WAVES;
    __shared__ double bs[CINV_MAXN];
    __shared__ double part[S][64];
    for (int c = threadIdx.x; c < n; c += 64 * S) bs[c] = (double)b[c];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r = blockIdx.x * 64 + lane;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (r < n) {
        const double *col = inv + r;
        int c = w;
        for (; c + 3 * S < n; c += 4 * S) {
            a0 += col[(int64_t)c * n] * bs[c];
            a1 += col[(int64_t)(c + S) * n] * bs[c + S];
            a2 += col[(int64_t)(c + 2 * S) * n] * bs[c + 2 * S];
            a3 += col[(int64_t)(c + 3 * S) * n] * bs[c + 3 * S];
        }
        for (; c < n; c += S) a0 += col[(int64_t)c * n] * bs[c];
    }
    part[w][lane] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (w == 0 && r < n) {
        double v = 0.0;
        for (int k = 0; k < S; ++k) v += part[k][lane];
        x[r] = (float)v;
    }
}

static void mg_free(mf_mg *mg)
{
    if (!mg) return;
    for (MGLevel &l : mg->L) level_free(l);
    if (mg->b64) (void)hipFree(mg->b64);
    if (mg->x64) (void)hipFree(mg->x64);
    if (mg->cinv) (void)hipFree(mg->cinv);
    delete mg;
}

// Extreme Ritz values of D^{-1} A on a level: Lanczos on D^{-1/2} A D^{-1/2}
// in FP64 (the largest converges from below to lambda_max, the smallest from
// above to lambda_min).
static mf_status lanczos_bounds(mf_mg *mg, MGLevel &l, int steps, double *out_max, double *out_min, hipStream_t s)
{
    mf_ctx *c = l.ctx;
    const int64_t n = l.nn;
    double *sv, *q, *qp, *w, *tmp;
    mf_status st;
    if ((st = ws_vec(c, 0, &sv)) || (st = ws_vec(c, 1, &q)) || (st = ws_vec(c, 2, &qp)) || (st = ws_vec(c, 3, &w)) ||
        (st = ws_vec(c, 4, &tmp)))
        return st;
    MGCHK(mg, heat_diagonal(c->km, heat_args(&l.op64), 0, tmp, c->face, s, true));
    MGCHK(mg, vsqrt(tmp, sv, n, s));
    MGCHK(mg, vknuth(q, n, s));
    double nq2;
    if ((st = host_dot(c, q, q, n, &nq2, s))) return st;
    MGCHK(mg, vaxpby(1.0 / sqrt(nq2), q, 0.0, q, n, s));
    MGCHK(mg, vfill(qp, 0.0, n, 0, s));
    std::vector<double> al, be;
    double beta = 0.0;
    for (int k = 0; k < steps; ++k) {
        MGCHK(mg, vmul(sv, q, tmp, n, s));
        MGCHK(mg, heat_apply(c->km, heat_args(&l.op64), 0, tmp, w, c->face, nullptr, nullptr, s));
        MGCHK(mg, vmul(sv, w, w, n, s));
        double a;
        if ((st = host_dot(c, w, q, n, &a, s))) return st;
        MGCHK(mg, vaxpby(-a, q, 1.0, w, n, s));
        MGCHK(mg, vaxpby(-beta, qp, 1.0, w, n, s));
        al.push_back(a);
        double b2;
        if ((st = host_dot(c, w, w, n, &b2, s))) return st;
        beta = sqrt(b2);
        if (k == steps - 1 || beta == 0.0) break;
        be.push_back(beta);
        MGCHK(mg, vcopy(q, qp, n, s));
        MGCHK(mg, vaxpby(1.0 / beta, w, 0.0, q, n, s));
    }
    be.resize(al.size() > 0 ? al.size() - 1 : 0);
    *out_max = tridiag_extreme_eig(al, be, true);
    *out_min = tridiag_extreme_eig(al, be, false);
    return MF_OK;
}

extern "C" {

mf_status mf_mg_create(mf_ctx *c, const mf_operator *op, const mf_mg_params *prm, mf_mg **out, mf_stream stream)
{
    if (!out) return MF_ERR_ARG;
    *out = nullptr;
    mf_status st = check_op(c, op);
    if (st) return st;
    if (!prm) return fail(c, MF_ERR_ARG, "null multigrid parameters");
    if (op->kind != MF_HEAT || op->precision != MF_FP64 || op->coeff_mode != MF_COEFF_LEVELSET || op->u0 ||
        op->T_coef || op->penalty != 0.0)
        return fail(c, MF_ERR_ARG, "multigrid needs an FP64 two-phase heat operator in LEVELSET mode without convection");
    if (prm->coarse_cells < 1 || prm->degree < 1 || !(prm->smoothing_range > 1.0) || prm->eig_steps < 1 ||
        !(prm->eig_safety >= 1.0) || !(prm->coarse_rtol > 0.0) || prm->coarse_maxit < 1)
        return fail(c, MF_ERR_ARG, "invalid multigrid parameters");
    if (prm->auto_levels && (prm->smooth_degree < 1 || !(prm->beta_stop > 0.0)))
        return fail(c, MF_ERR_ARG, "the level rule needs smooth_degree >= 1 and beta_stop > 0");
    hipStream_t s = (hipStream_t)stream;
    // level meshes: halve every direction while n[0] > coarse_cells
    std::vector<mf_mesh> meshes{c->mesh};
    while (meshes.back().n[0] > prm->coarse_cells) {
        mf_mesh m = meshes.back();
        for (int d = 0; d < 3; ++d) {
            if (m.n[d] % 2) return fail(c, MF_ERR_ARG, "cells per direction must halve evenly down to the coarse level");
            m.n[d] /= 2;
        }
        meshes.push_back(m);
    }

    mf_mg *mg = new mf_mg();
    mg->parent = c;
    mg->fine_op = *op;
    mg->prm = *prm;
    const int nl = (int)meshes.size();
    mg->L.resize(nl);
    for (int i = 0; i < nl; ++i) {
        MGLevel &l = mg->L[nl - 1 - i]; // index 0 = coarsest
        l.mesh = meshes[i];
        if ((st = mf_create(&l.mesh, &l.ctx)) != MF_OK) {
            mg_free(mg);
            return fail(c, st, "level context creation failed");
        }
        l.nn = l.ctx->nn;
    }
    // level sets: finest borrowed (FP64), the others injected
    MGLevel &top = mg->L[nl - 1];
    top.phi64 = (double *)op->phi;
    for (int li = nl - 2; li >= 0; --li) {
        MGLevel &l = mg->L[li], &f = mg->L[li + 1];
        bool ok = hipMalloc((void **)&l.phi64, sizeof(double) * l.nn) == hipSuccess;
        l.own_phi64 = ok;
        if (!ok) {
            mg_free(mg);
            return fail(c, MF_ERR_OOM, "multigrid allocation failed");
        }
        MGCHK(mg, mg_inject(f.ctx->km, l.ctx->km, f.phi64, l.phi64, 0, s));
    }
    for (int li = 0; li < nl; ++li) {
        MGLevel &l = mg->L[li];
        l.op64 = *op;
        l.op64.phi = l.phi64;
        l.op32 = l.op64;
        l.op32.precision = MF_FP32;
    }
    // Level rule: from the finest level down, the first level with a
    // well-conditioned Jacobi-scaled operator becomes the (smoothed) coarsest.
    int first = 0;
    if (prm->auto_levels) {
        const double diff = fmax(op->alpha_k * op->k_l / (op->alpha_m * op->rc_l),
                                 op->alpha_k * op->k_g / (op->alpha_m * op->rc_g));
        for (int li = nl - 1; li >= 0; --li) {
            const KMesh &k = mg->L[li].ctx->km;
            const double beta = 17.5 * (1.0 / (k.hx * k.hx) + 1.0 / (k.hy * k.hy) + 1.0 / (k.hz * k.hz)) * diff;
            if (beta <= prm->beta_stop) {
                first = li;
                mg->smooth_coarsest = true;
                break;
            }
        }
        for (int li = 0; li < first; ++li) level_free(mg->L[li]);
        mg->L.erase(mg->L.begin(), mg->L.begin() + first);
    }
    if (mg->L.size() < 2 && !mg->smooth_coarsest) {
        mg_free(mg);
        return fail(c, MF_ERR_ARG, "the mesh is already at the coarse size");
    }
    const int nk = (int)mg->L.size();
    for (int li = 0; li < nk; ++li) {
        MGLevel &l = mg->L[li];
        const bool smoothed = li > 0 || mg->smooth_coarsest;
        const size_t fb = sizeof(float) * l.nn;
        bool ok = hipMalloc((void **)&l.b, fb) == hipSuccess && hipMalloc((void **)&l.x, fb) == hipSuccess;
        if (ok && smoothed) // a solved coarsest level only needs its right-hand side and solution
            ok = hipMalloc((void **)&l.phi32, fb) == hipSuccess && hipMalloc((void **)&l.dinv, fb) == hipSuccess &&
                 hipMalloc((void **)&l.r, fb) == hipSuccess && hipMalloc((void **)&l.d, fb) == hipSuccess &&
                 hipMalloc((void **)&l.t, fb) == hipSuccess;
        if (!ok) {
            mg_free(mg);
            return fail(c, MF_ERR_OOM, "multigrid allocation failed");
        }
        if (!smoothed) continue; // coarsest: FP64 CG only
        MGCHK(mg, vcvt_d2f(l.phi64, l.phi32, l.nn, s));
        l.op32.phi = l.phi32;
        if ((st = ensure_face(l.ctx, 1))) {
            mg_free(mg);
            return st;
        }
        MGCHK(mg, heat_diagonal(l.ctx->km, heat_args(&l.op32), 1, l.dinv, l.ctx->face, s, true));
        const bool coarsest_smoothed = li == 0 && mg->smooth_coarsest;
        const bool need_est = !prm->lambda_max || (coarsest_smoothed && !prm->lambda_min);
        if (need_est && (st = lanczos_bounds(mg, l, prm->eig_steps, &l.est_max, &l.est_min, s))) {
            mg_free(mg);
            return st;
        }
        l.degree = coarsest_smoothed ? prm->smooth_degree : prm->degree;
        l.lmax = prm->lambda_max ? prm->lambda_max[li] : prm->eig_safety * l.est_max;
        if (prm->lambda_min) l.lmin = prm->lambda_min[li];
        else l.lmin = coarsest_smoothed ? l.est_min / prm->eig_safety : l.lmax / prm->smoothing_range;
    }
    MGLevel &co = mg->L[0];
    if (hipMalloc((void **)&mg->b64, sizeof(double) * co.nn) != hipSuccess ||
        hipMalloc((void **)&mg->x64, sizeof(double) * co.nn) != hipSuccess) {
        mg_free(mg);
        return fail(c, MF_ERR_OOM, "multigrid allocation failed");
    }
    // A one-brick coarsest level that is solved, not smoothed, keeps A^-1:
    // its columns are solved once here by the coarse CG to coarse_rtol, and
    // every coarse solve is then one dense product (a few microseconds
    // instead of a CG of tens of iterations in one workgroup).
    if (!mg->smooth_coarsest && heat_fits_one_brick(co.ctx->km) && co.nn <= CINV_MAXN) {
        if (hipMalloc((void **)&mg->cinv, sizeof(double) * co.nn * co.nn) != hipSuccess) {
            mg_free(mg);
            return fail(c, MF_ERR_OOM, "multigrid allocation failed");
        }
        const hipError_t e = heat_inverse_one_brick(co.ctx->km, heat_args(&co.op64), mg->cinv, prm->coarse_rtol,
                                                    prm->coarse_maxit, s);
        if (e != hipSuccess) {
            mg_free(mg);
            return fail(c, MF_ERR_HIP, "coarse inverse: %s", hipGetErrorString(e));
        }
    }
    if (hipStreamSynchronize(s) != hipSuccess) {
        mg_free(mg);
        return fail(c, MF_ERR_HIP, "multigrid setup failed");
    }
    *out = mg;
    return MF_OK;
}

void mf_mg_destroy(mf_mg *mg) { mg_free(mg); }

int32_t mf_mg_n_levels(const mf_mg *mg) { return mg ? (int32_t)mg->L.size() : 0; }

mf_status mf_mg_lambda_max(const mf_mg *mg, double *out)
{
    if (!mg || !out) return MF_ERR_ARG;
    for (size_t i = 0; i < mg->L.size(); ++i) out[i] = mg->L[i].lmax;
    return MF_OK;
}

mf_status mf_mg_levels(const mf_mg *mg, int32_t *cells, int32_t *degree, double *lambda_min, double *lambda_max)
{
    if (!mg) return MF_ERR_ARG;
    for (size_t i = 0; i < mg->L.size(); ++i) {
        const MGLevel &l = mg->L[i];
        if (cells) cells[i] = l.mesh.n[0];
        if (degree) degree[i] = l.degree;
        if (lambda_min) lambda_min[i] = l.lmin;
        if (lambda_max) lambda_max[i] = l.lmax;
    }
    return MF_OK;
}

} // extern "C"

// Chebyshev smoothing of A_l x = b on level l (FP32); x from zero if x_zero.
// Residual and direction are kept in l.r and l.d; the first step fuses the
// initial residual, the last one updates x only.
static mf_status cheb_smooth(mf_mg *mg, MGLevel &l, const float *b, float *x, bool x_zero, hipStream_t s)
{
    mf_ctx *c = l.ctx;
    const int64_t n = l.nn;
    const int deg = l.degree;
    const double theta = 0.5 * (l.lmax + l.lmin), delta = 0.5 * (l.lmax - l.lmin), sigma = theta / delta;
    if (!x_zero) MGCHK(mg, heat_apply(c->km, heat_args(&l.op32), 1, x, l.t, c->face, nullptr, nullptr, s));
    MGCHK(mg, cheb_first(l.dinv, b, x_zero ? nullptr : l.t, l.r, l.d, x, (float)(1.0 / theta), deg > 1, n, s));
    double rho = 1.0 / sigma;
    for (int k = 1; k < deg; ++k) {
        MGCHK(mg, heat_apply(c->km, heat_args(&l.op32), 1, l.d, l.t, c->face, nullptr, nullptr, s));
        const double rho_new = 1.0 / (2.0 * sigma - rho);
        const bool from_zero = x_zero && k == 1; // x is still d, r is still b
        MGCHK(mg, cheb_step(l.dinv, from_zero ? b : l.r, l.t, l.r, l.d, x, (float)(rho_new * rho),
                            (float)(2.0 * rho_new / delta), from_zero, k == deg - 1, n, s));
        rho = rho_new;
    }
    return MF_OK;
}

// x_l = V_l(b_l): recursive V-cycle, level 0 solved by FP64 CG (a one-brick
// level by its inverse, formed by that CG at setup).
static mf_status vcycle(mf_mg *mg, int li, hipStream_t s)
{
    MGLevel &l = mg->L[li];
    mf_status st;
    if (li == 0 && mg->smooth_coarsest) return cheb_smooth(mg, l, l.b, l.x, true, s);
    if (li == 0) {
        if (mg->cinv) {
            coarse_inverse_apply_kernel<<<(unsigned)((l.nn + 63) / 64), 64 * CINV_WAVES, 0, s>>>(mg->cinv, (int)l.nn,
                                                                                            l.b, l.x);
            MGCHK(mg, hipGetLastError());
            return MF_OK;
        }
        if (heat_fits_one_brick(l.ctx->km)) {
            MGCHK(mg, heat_cg_one_brick(l.ctx->km, heat_args(&l.op64), l.b, l.x, mg->prm.coarse_rtol,
                                        mg->prm.coarse_maxit, s));
            return MF_OK;
        }
        MGCHK(mg, vcvt_f2d(l.b, mg->b64, l.nn, s));
        mf_solve_info info;
        st = mf_cg_solve(l.ctx, &l.op64, MF_PC_JACOBI, mg->b64, mg->x64, mg->prm.coarse_rtol, mg->prm.coarse_maxit,
                         &info, (mf_stream)s);
        if (st < 0) return fail(mg->parent, st, "coarse solve: %s", mf_last_error(l.ctx));
        MGCHK(mg, vcvt_d2f(mg->x64, l.x, l.nn, s));
        return MF_OK;
    }
    MGLevel &cl = mg->L[li - 1];
    if ((st = cheb_smooth(mg, l, l.b, l.x, true, s))) return st;
    MGCHK(mg, heat_apply(l.ctx->km, heat_args(&l.op32), 1, l.x, l.t, l.ctx->face, nullptr, nullptr, s));
    MGCHK(mg, vsub_f(l.b, l.t, l.r, l.nn, s));
    MGCHK(mg, mg_restrict(l.ctx->km, cl.ctx->km, l.r, cl.b, l.d, l.t, s)); // l.d, l.t: free work vectors here
    if ((st = vcycle(mg, li - 1, s))) return st;
    MGCHK(mg, mg_prolong_add(cl.ctx->km, l.ctx->km, cl.x, l.x, l.d, l.t, s)); // l.d, l.t: free until smoothing
    return cheb_smooth(mg, l, l.b, l.x, false, s);
}

extern "C" mf_status mf_mg_vcycle(mf_mg *mg, const double *r, double *z, mf_stream stream)
{
    if (!mg) return MF_ERR_ARG;
    if (!r || !z) return mg_fail(mg, MF_ERR_ARG, "null vector");
    hipStream_t s = (hipStream_t)stream;
    MGLevel &top = mg->L.back();
    MGCHK(mg, vcvt_d2f(r, top.b, top.nn, s));
    mf_status st = vcycle(mg, (int)mg->L.size() - 1, s);
    if (st) return st;
    MGCHK(mg, vcvt_f2d(top.x, z, top.nn, s));
    return MF_OK;
}

// Flexible CG (Notay; Polak-Ribiere beta) in FP64 preconditioned by the
// V-cycle.  The V-cycle's FP32 input (the residual, rounded by the update
// kernel that forms it) and output (z, used as stored: its conversion to
// FP64 is exact) stay in FP32 on the finest level.
extern "C" mf_status mf_mg_cg_solve(mf_mg *mg, const double *b, double *x, double rtol, int32_t maxit,
                                    mf_solve_info *info, mf_stream stream)
{
    if (!mg) return MF_ERR_ARG;
    mf_ctx *c = mg->parent;
    if (!b || !x || !info) return fail(c, MF_ERR_ARG, "null argument");
    if (!(rtol >= 0.0) || maxit < 0) return fail(c, MF_ERR_ARG, "invalid rtol or maxit");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = c->nn;
    double *r, *p, *q;
    mf_status st;
    if ((st = ws_vec(c, 0, &r)) || (st = ws_vec(c, 2, &p)) || (st = ws_vec(c, 3, &q))) return st;
    RedWS red = redws(c);
    if ((st = ensure_face(c, 1))) return st;
    const HeatArgs ha = heat_args(&mg->fine_op);
    MGLevel &top = mg->L.back();
    const int ltop = (int)mg->L.size() - 1;
    // the flexible CG of vec.hip: z = V(r) is top.x (FP32), its input r32 is top.b
    // No poll before the first V-cycle: when the initial residual already
    // meets the threshold (b = 0, maxit = 0) the state says done, the
    // direction, apply and residual kernels are no-ops and the V-cycle's
    // output is unused.  The state read at the last poll is final: the
    // finishing kernel only adds the pending alpha p to x.
    HIPCHK(c, cg_init(c->cg, b, nullptr, x, r, p, n, rtol, maxit, 1, &red, s));
    HIPCHK(c, vcvt_d2f(b, top.b, n, s)); // r = b
    if ((st = vcycle(mg, ltop, s))) return st;
    HIPCHK(c, fcg_direction(c->cg, r, top.x, p, x, n, &red, s));
    for (;;) {
        HIPCHK(c, heat_apply(c->km, ha, 0, p, q, c->face, c->cg, &red, s));
        HIPCHK(c, fcg_resid(c->cg, r, q, top.x, top.b, n, &red, s));
        HIPCHK(c, hipMemcpyAsync(c->h_state, c->cg, sizeof(CGState), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        if (c->h_state->done) break;
        if ((st = vcycle(mg, ltop, s))) return st;
        HIPCHK(c, fcg_direction(c->cg, r, top.x, p, x, n, &red, s));
    }
    HIPCHK(c, fcg_finish(c->cg, p, x, n, s));
    const CGState hs = *c->h_state;
    const double bnorm = sqrt(hs.bb);
    info->iters = hs.iter;
    info->rel_res_est = bnorm > 0.0 ? sqrt(hs.rr) / bnorm : 0.0;
    info->converged = !hs.breakdown && hs.rr <= hs.thresh2;
    if ((st = true_residual(c, &mg->fine_op, 0, b, x, q, bnorm, &info->rel_res, s))) return st;
    if (hs.breakdown) return fail(c, MF_BREAKDOWN, "flexible CG breakdown at iteration %d", hs.iter);
    if (!info->converged) return fail(c, MF_NOT_CONVERGED, "flexible CG reached maxit = %d", maxit);
    return MF_OK;
}
