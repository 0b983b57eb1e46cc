// oseen.hip -- matrix-free Q2 linearized momentum (Oseen) operator on gfx950.
//
// Operator (Sec. 2.1, eq. momentum_balance with the viscous stress
// 2 mu eps(u), linearized about a frozen velocity u0 and one backward-Euler
// step; rho by the reciprocal blend of eq. rhoEff, mu by eq. muEff):
//   a(u, v) = int alpha_m rho u.v + alpha_c rho ((u0.grad) u).v
//           + alpha_v mu (grad u + grad u^T) : grad v
// (the last term equals 2 mu eps(u):eps(v)).  The transpose moves the
// convective term onto the test function: alpha_c rho u_c (u0.grad) v_c.
//
// Work decomposition: one workgroup of three wavefronts per brick of 4x4x4
// cells (brick.hpp); wavefront c takes velocity component c, one thread per
// cell.  Nodal x (3 components), u0 (3 components) and phi are staged in LDS
// once for the three.  Per cell and component:
//   acc = alpha_m rho W u_c                                  (Gauss values)
//       + alpha_c rho W sum_d u0_d d_d u_c                   (forward)
//   acc += sum_d D_d^T [ W mu alpha_v (d_d u_c + d_c u_d)    (viscous)
//                        + alpha_c rho W u0_d u_c ]          (transpose only)
//   y_c = S^T acc
// where d_c u_d is formed by interpolating u_d and differentiating along c,
// so no gradient fields are exchanged between threads.
#include <type_traits>

#include "brick.hpp"

namespace mf {

constexpr int ONT = 3 * BNT; // threads per Oseen brick
constexpr int NB = lds_field<double>(); // LDS entries of one staged nodal field

// Heaviside of the interpolated level set at the 27 Gauss points (in place).
template <int HK> __device__ __forceinline__ void heaviside27(const OseenArgs &a, double *ph)
{
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        if (HK == 0) {
            ph[q] = heaviside_linear<double>(ph[q]);
        } else {
            ph[q] = heaviside_sine_value(a.eps, ph[q]);
        }
    }
}

__device__ __forceinline__ double gauss_weight(int q)
{
    return Q2<double>::weight(q % 3) * Q2<double>::weight((q / 3) % 3) * Q2<double>::weight(q / 9);
}

// d_c applied line by line to the Gauss values v (in place), scaled by s.
template <int DIR> __device__ __forceinline__ void deriv_inplace(double *v, double s)
{
#pragma unroll
    for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int i0 = lidx<DIR>(0, m, n), i1 = lidx<DIR>(1, m, n), i2 = lidx<DIR>(2, m, n);
            double t0, t1, t2;
            Q2<double>::deriv(v[i0], v[i1], v[i2], t0, t1, t2);
            v[i0] = s * t0;
            v[i1] = s * t1;
            v[i2] = s * t2;
        }
}

// Viscous part along DIR: g = nu .* (s d_DIR u + e), acc += s D_DIR^T g, line
// by line (e = d_c u_d already scaled, or null for the d = c term with factor 2).
template <int DIR, bool TWICE>
__device__ __forceinline__ void visc_dir(const double *u, const double *nu, const double *e, double s, double *acc)
{
#pragma unroll
    for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int i0 = lidx<DIR>(0, m, n), i1 = lidx<DIR>(1, m, n), i2 = lidx<DIR>(2, m, n);
            double t0, t1, t2;
            Q2<double>::deriv(u[i0], u[i1], u[i2], t0, t1, t2);
            double g0, g1, g2;
            if (TWICE) {
                g0 = 2.0 * s * nu[i0] * t0;
                g1 = 2.0 * s * nu[i1] * t1;
                g2 = 2.0 * s * nu[i2] * t2;
            } else {
                g0 = nu[i0] * (s * t0 + e[i0]);
                g1 = nu[i1] * (s * t1 + e[i1]);
                g2 = nu[i2] * (s * t2 + e[i2]);
            }
            Q2<double>::derivT_acc(s * g0, s * g1, s * g2, acc[i0], acc[i1], acc[i2]);
        }
}

// Solid fraction (eq. solid_fraction) and smooth indicator H_s (eq. heaviside_sl).
__device__ __forceinline__ double solid_fraction(const OseenArgs &a, double T)
{
    return fmin(fmax((a.T_liq - T) / (a.T_liq - a.T_sol), 0.0), 1.0);
}
__device__ __forceinline__ double solid_indicator(double fs) { return fs * fs * (3.0 - 2.0 * fs); }

// Gauss-point fields shared by the brick's three wavefronts are kept in LDS
// as [q][cell] (27 x 64 doubles each): a lane reads its own cell's column,
// consecutive lanes in consecutive banks.
constexpr int GQ = 27 * BNT; // doubles of one shared Gauss-point field

// Phase 1 of component C on one cell (every wavefront of the brick runs it
// for its own C, on the staged nodal fields):
//   u   = S x_C at the Gauss points (returned in u);
//   w0  = S u0_C at the Gauss points (returned in w0, shared after a barrier);
//   the coefficients rho W and alpha_v mu W at the nine Gauss points
//   9C .. 9C + 8 (the three wavefronts split the 27 points), written to the
//   shared fields rwl and nul;
//   acc = Darcy weight * u with three phases (TP), untouched otherwise.
template <int C, int HK, bool TP>
__device__ __forceinline__ void oseen_phase1(const Brick &br, const OseenArgs &a, const KMesh &m, const double *stage,
                                             double *rwl, double *nul, double *u, double *w0, double *acc)
{
    const double *ps = stage, *us = stage + NB, *u0s = stage + 4 * NB, *tcs = stage + 7 * NB;
    const double vol = m.hx * m.hy * m.hz;
    const int t = br.t;
    double h[27];
    br.gather27(ps, h);
    interp3(h);
    if constexpr (TP) {
        double tq[27];
        br.gather27(tcs, tq);
        interp3(tq);
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const int q = 9 * C + j;
            const double H = HK == 0 ? heaviside_linear<double>(h[q]) : heaviside_sine_value(a.eps, h[q]);
            const double Hs = solid_indicator(solid_fraction(a, tq[q]));
            const double W = vol * gauss_weight(q);
            rwl[q * BNT + t] = W / (H / (Hs * a.rho_s + (1.0 - Hs) * a.rho_l) + (1.0 - H) / a.rho_g);
            nul[q * BNT + t] = a.av * W * (H * (Hs * a.mu_s + (1.0 - Hs) * a.mu_l) + (1.0 - H) * a.mu_g);
        }
        // Darcy weight W C fs^2 / ((1 - fs)^3 + b), held in acc until u is known
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            const double fs = solid_fraction(a, tq[q]);
            acc[q] = vol * gauss_weight(q) * a.darcy_C * fs * fs / ((1.0 - fs) * (1.0 - fs) * (1.0 - fs) + a.darcy_b);
        }
        pin27(acc);
    } else {
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const int q = 9 * C + j;
            const double H = HK == 0 ? heaviside_linear<double>(h[q]) : heaviside_sine_value(a.eps, h[q]);
            const double W = vol * gauss_weight(q);
            rwl[q * BNT + t] = W / (H / a.rho_l + (1.0 - H) / a.rho_g);
            nul[q * BNT + t] = a.av * W * (a.mu_g + H * (a.mu_l - a.mu_g));
        }
    }
    if constexpr (TP) pin27(acc);
    br.gather27(us + C * NB, u);
    interp3(u);
    if constexpr (TP) {
#pragma unroll
        for (int q = 0; q < 27; ++q) acc[q] *= u[q];
        pin27(acc);
    }
    pin27(u);
    br.gather27(u0s + C * NB, w0);
    interp3(w0);
}

// Phase 2 of component C: mass and convection with rho W from rwl and the
// Gauss-point u0 of all three components from the shared fields w0l[d]:
//   acc (+)= alpha_m rho W u                                   (mass)
//   forward:   acc += alpha_c rho W sum_d u0_d d_d u
//   transpose: acc += sum_d D_d^T (alpha_c rho W u0_d u)
template <int C, bool TR, bool TP>
__device__ __forceinline__ void oseen_phase2(const Brick &br, const OseenArgs &a, const KMesh &m, const double *rwl,
                                             const double *w0l, const double *u, double *acc)
{
    const int t = br.t;
    const double sdir[3] = {1.0 / (kR * m.hx), 1.0 / (kR * m.hy), 1.0 / (kR * m.hz)};
    double rw[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) rw[q] = rwl[q * BNT + t];
#pragma unroll
    for (int q = 0; q < 27; ++q) acc[q] = (TP ? acc[q] : 0.0) + a.am * rw[q] * u[q];
    auto dir = [&](auto D) {
        constexpr int d = decltype(D)::value;
        // one direction at a time: its 27 reads are not hoisted above the
        // previous direction's arithmetic
        pin27(acc);
        pin27(rw);
        pin27((double *)u);
        const double *w = w0l + d * GQ + t;
        const double s = a.ac * sdir[d];
#pragma unroll
        for (int n = 0; n < 3; ++n)
#pragma unroll
            for (int mm = 0; mm < 3; ++mm) {
                const int i0 = lidx<d>(0, mm, n), i1 = lidx<d>(1, mm, n), i2 = lidx<d>(2, mm, n);
                if constexpr (TR) {
                    Q2<double>::derivT_acc(s * rw[i0] * w[i0 * BNT] * u[i0], s * rw[i1] * w[i1 * BNT] * u[i1],
                                           s * rw[i2] * w[i2 * BNT] * u[i2], acc[i0], acc[i1], acc[i2]);
                } else {
                    double t0, t1, t2;
                    Q2<double>::deriv(u[i0], u[i1], u[i2], t0, t1, t2);
                    acc[i0] += s * rw[i0] * w[i0 * BNT] * t0;
                    acc[i1] += s * rw[i1] * w[i1 * BNT] * t1;
                    acc[i2] += s * rw[i2] * w[i2 * BNT] * t2;
                }
            }
    };
    dir(std::integral_constant<int, 0>{});
    dir(std::integral_constant<int, 1>{});
    dir(std::integral_constant<int, 2>{});
}

// Phase 3 of component C: viscosity with nu = alpha_v mu W from nul and the
// Gauss-point values of the other two components from the shared fields ul[d]:
//   acc += D_C^T (2 nu d_C u_C) + sum_{d != C} D_d^T (nu (d_d u_C + d_C u_d)),
// then y_C = S^T acc (in acc).
template <int C>
__device__ __forceinline__ void oseen_phase3(const Brick &br, const KMesh &m, const double *nul, const double *ul,
                                             const double *u, double *acc)
{
    const int t = br.t;
    const double sdir[3] = {1.0 / (kR * m.hx), 1.0 / (kR * m.hy), 1.0 / (kR * m.hz)};
    double nu[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) nu[q] = nul[q * BNT + t];
    double e[27];
    auto cross = [&](auto D) {
        constexpr int d = decltype(D)::value;
        pin27(acc);
        pin27(nu);
        pin27((double *)u);
        if constexpr (d == C) {
            visc_dir<d, true>(u, nu, nullptr, sdir[d], acc);
        } else {
#pragma unroll
            for (int q = 0; q < 27; ++q) e[q] = ul[d * GQ + q * BNT + t];
            deriv_inplace<C>(e, sdir[C]); // d_C u_d
            visc_dir<d, false>(u, nu, e, sdir[d], acc);
        }
    };
    cross(std::integral_constant<int, 0>{});
    cross(std::integral_constant<int, 1>{});
    cross(std::integral_constant<int, 2>{});
    interp3T(acc);
}

// One workgroup of three wavefronts per brick; wavefront c computes velocity
// component c of every cell.  The nodal fields (phi, x and u0, three
// components each, and with three phases the frozen temperature) are staged
// once; each wavefront interpolates its own components of x and u0 and the
// coefficients at a third of the Gauss points, and the brick's Gauss-point
// fields are exchanged through LDS:
//   region A: staging, then u0 at the Gauss points (3 fields), then x at the
//             Gauss points (3 fields); region C: rho W and nu.
template <int HK, bool TR, bool TP>
__global__ void __launch_bounds__(ONT) oseen_apply_kernel(KMesh m, OseenArgs a, const double *__restrict__ x,
                                                          double *__restrict__ y, double *__restrict__ face)
{
    constexpr int STAGE = (TP ? 8 : 7) * NB, GAUSS3 = 3 * GQ;
    constexpr int AREG = STAGE > GAUSS3 ? STAGE : GAUSS3;
    __shared__ double lds[AREG + 2 * GQ];
    double *A = lds, *rwl = lds + AREG, *nul = rwl + GQ;
    const int comp = threadIdx.x / BNT; // uniform over a wavefront
    const Brick br(m, threadIdx.x % BNT);
    const int64_t nn = (int64_t)m.NX * m.NY * m.NZ;
    double *ps = A, *us = A + NB, *u0s = A + 4 * NB, *tcs = A + 7 * NB;
    if constexpr (TP) {
        const double *src[8] = {a.phi, x, x + nn, x + 2 * nn, a.u0, a.u0 + nn, a.u0 + 2 * nn, a.tc};
        double *const dst[8] = {ps, us, us + NB, us + 2 * NB, u0s, u0s + NB, u0s + 2 * NB, tcs};
        br.stage_nodes_wg<ONT, 8>(m, threadIdx.x, src, dst, 0xEu);
    } else {
        const double *src[7] = {a.phi, x, x + nn, x + 2 * nn, a.u0, a.u0 + nn, a.u0 + 2 * nn};
        double *const dst[7] = {ps, us, us + NB, us + 2 * NB, u0s, u0s + NB, u0s + 2 * NB};
        br.stage_nodes_wg<ONT, 7>(m, threadIdx.x, src, dst, 0xEu);
    }
    __syncthreads();
    double u[27], acc[27];
    {
        double w0[27];
        if (comp == 0) oseen_phase1<0, HK, TP>(br, a, m, A, rwl, nul, u, w0, acc);
        else if (comp == 1) oseen_phase1<1, HK, TP>(br, a, m, A, rwl, nul, u, w0, acc);
        else oseen_phase1<2, HK, TP>(br, a, m, A, rwl, nul, u, w0, acc);
        __syncthreads(); // staging no longer read: region A takes u0 at the Gauss points
#pragma unroll
        for (int q = 0; q < 27; ++q) A[comp * GQ + q * BNT + br.t] = w0[q];
    }
    __syncthreads();
    if (comp == 0) oseen_phase2<0, TR, TP>(br, a, m, rwl, A, u, acc);
    else if (comp == 1) oseen_phase2<1, TR, TP>(br, a, m, rwl, A, u, acc);
    else oseen_phase2<2, TR, TP>(br, a, m, rwl, A, u, acc);
    __syncthreads(); // u0 no longer read: region A takes x at the Gauss points
#pragma unroll
    for (int q = 0; q < 27; ++q) A[comp * GQ + q * BNT + br.t] = u[q];
    __syncthreads();
    if (comp == 0) oseen_phase3<0>(br, m, nul, A, u, acc);
    else if (comp == 1) oseen_phase3<1>(br, m, nul, A, u, acc);
    else oseen_phase3<2>(br, m, nul, A, u, acc);
    __syncthreads(); // region A no longer read: it takes the node-sum exchange
    br.assemble27(acc, lds + comp * 9 * BNT);
    double *fb = face + ((int64_t)comp * n_bricks(m) + br.brick) * BFACE;
    double *yc = y + comp * nn;
    const double *xc = x + comp * nn;
    br.for_owned_nodes(m, [&](int ai, int bi, int ci, int l, int64_t g, bool, int sh) {
        const double s = acc[ai + 3 * bi + 9 * ci];
        double *dst = sh ? fb + br.fslot(ai, bi, ci) : yc + g;
        *dst = s;
    });
    if (br.touches_dirichlet(m)) {
        br.for_owned_nodes(m, [&](int, int, int, int, int64_t g, bool constrained, int sh) {
            if (constrained && !sh) yc[g] = xc[g];
        });
    }
}

// Shared nodes of component blockIdx.y, brick by brick (combine_brick).
__global__ void __launch_bounds__(BNT * CBW) oseen_combine_kernel(KMesh m, const double *__restrict__ face,
                                                                  const double *__restrict__ x, double *__restrict__ y)
{
    const int comp = blockIdx.y;
    const int64_t nn = (int64_t)m.NX * m.NY * m.NZ, nb = n_bricks(m);
    combine_brick<double, 1>(m, face + comp * nb * BFACE, x + comp * nn, y + comp * nn);
}

hipError_t oseen_apply(const KMesh &m, const OseenArgs &a, int transpose, const double *x, double *y, void *face,
                       hipStream_t s, const KTiming *t)
{
    const unsigned nb = (unsigned)n_bricks(m);
    if (!face) return hipErrorInvalidValue;
    if (t && t->start) {
        hipError_t e = hipEventRecord(t->start, s);
        if (e != hipSuccess) return e;
    }
    double *fb = (double *)face;
    const int key = (a.tc ? 4 : 0) | (a.hkind ? 2 : 0) | (transpose ? 1 : 0);
    switch (key) {
    case 0: oseen_apply_kernel<0, false, false><<<nb, ONT, 0, s>>>(m, a, x, y, fb); break;
    case 1: oseen_apply_kernel<0, true, false><<<nb, ONT, 0, s>>>(m, a, x, y, fb); break;
    case 2: oseen_apply_kernel<1, false, false><<<nb, ONT, 0, s>>>(m, a, x, y, fb); break;
    case 3: oseen_apply_kernel<1, true, false><<<nb, ONT, 0, s>>>(m, a, x, y, fb); break;
    case 4: oseen_apply_kernel<0, false, true><<<nb, ONT, 0, s>>>(m, a, x, y, fb); break;
    case 5: oseen_apply_kernel<0, true, true><<<nb, ONT, 0, s>>>(m, a, x, y, fb); break;
    case 6: oseen_apply_kernel<1, false, true><<<nb, ONT, 0, s>>>(m, a, x, y, fb); break;
    case 7: oseen_apply_kernel<1, true, true><<<nb, ONT, 0, s>>>(m, a, x, y, fb); break;
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && t && t->stop) e = hipEventRecord(t->stop, s);
    if (e != hipSuccess) return e;
    if (nb > 1) oseen_combine_kernel<<<dim3((nb + CBW - 1) / CBW, 3), BNT * CBW, 0, s>>>(m, fb, x, y);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 3x3 nodal diagonal blocks: for each cell node i and component pair (c, c'),
//   B_i[c][c'] = sum_q W [ (alpha_m rho N_i^2 + alpha_c rho N_i (u0.grad N_i)
//                           + alpha_v mu |grad N_i|^2) delta_cc'
//                         + alpha_v mu d_c' N_i d_c N_i ]
// (+ the Darcy weight in the mass term with three phases) by direct loops
// over the Gauss points (setup only), one pass per entry.  Shared nodes go
// through the face buffer, one sheet per entry, and the combine pass, like
// the applies: every entry is written once and the result is reproducible.
// ---------------------------------------------------------------------------
template <int HK, bool TP>
__global__ void __launch_bounds__(BNT) oseen_block_kernel(KMesh m, OseenArgs a, double *__restrict__ blocks,
                                                          double *__restrict__ face)
{
    constexpr int STAGE = (TP ? 5 : 4) * NB, CONTRIB = 27 * BNT;
    __shared__ double lds[STAGE > CONTRIB ? STAGE : CONTRIB];
    __shared__ double E[27 * BNT];
    const Brick br(m, threadIdx.x);
    const int64_t nn = (int64_t)m.NX * m.NY * m.NZ;
    double *ps = lds, *u0s = lds + NB, *tcs = lds + 4 * NB;
    if constexpr (TP) {
        const double *src[5] = {a.phi, a.u0, a.u0 + nn, a.u0 + 2 * nn, a.tc};
        double *const dst[5] = {ps, u0s, u0s + NB, u0s + 2 * NB, tcs};
        br.stage_nodes_wg<BNT, 5>(m, threadIdx.x, src, dst, 0u);
    } else {
        const double *src[4] = {a.phi, a.u0, a.u0 + nn, a.u0 + 2 * nn};
        double *const dst[4] = {ps, u0s, u0s + NB, u0s + 2 * NB};
        br.stage_nodes_wg<BNT, 4>(m, threadIdx.x, src, dst, 0u);
    }
    __syncthreads();
    const double vol = m.hx * m.hy * m.hz;
    const double ih[3] = {1.0 / m.hx, 1.0 / m.hy, 1.0 / m.hz};
    double rw[27], nu[27], w0[27], dw[27]; // rho W, alpha_v mu W, scratch (velocity), Darcy W
    br.gather27(ps, rw);
    interp3(rw);
    heaviside27<HK>(a, rw);
    if (TP) {
        br.gather27(tcs, dw);
        interp3(dw);
    }
    // unrolled (a loop over q would index the arrays at run time and put them
    // in scratch memory), one point at a time
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        const double H = rw[q];
        const double W = vol * gauss_weight(q);
        if (TP) {
            const double fs = solid_fraction(a, dw[q]), Hs = solid_indicator(fs);
            const double rho_sl = Hs * a.rho_s + (1.0 - Hs) * a.rho_l;
            rw[q] = W / (H / rho_sl + (1.0 - H) / a.rho_g);
            nu[q] = a.av * W * (H * (Hs * a.mu_s + (1.0 - Hs) * a.mu_l) + (1.0 - H) * a.mu_g);
            dw[q] = W * a.darcy_C * fs * fs / ((1.0 - fs) * (1.0 - fs) * (1.0 - fs) + a.darcy_b);
        } else {
            rw[q] = W / (H / a.rho_l + (1.0 - H) / a.rho_g);
            nu[q] = a.av * W * (a.mu_g + H * (a.mu_l - a.mu_g));
            dw[q] = 0.0;
        }
        asm volatile("" : "+v"(rw[q]), "+v"(nu[q]), "+v"(dw[q]));
    }
    // Every term is a product of 1D factors along x, y, z, so its sum over the
    // Gauss points is a contraction of a Gauss-point weight with 1D tables
    // (as the heat diagonal): N_i^2 -> S^2 along all three directions;
    // N_i d_d N_i -> S.G / h_d along d; (d_d N_i)^2 -> G^2 / h_d^2 along d;
    // d_c N_i d_c' N_i -> S.G / h along c and along c'.
    constexpr double s0 = Q2<double>::s0, s1 = Q2<double>::s1, s2 = Q2<double>::s2;
    constexpr double g0 = Q2<double>::g0, g1 = Q2<double>::g1, g2 = Q2<double>::g2;
    const double S2[3][3] = {{s0 * s0, s1 * s1, s2 * s2}, {0.0, 1.0, 0.0}, {s2 * s2, s1 * s1, s0 * s0}};
    const double G2[3][3] = {{g0 * g0, g1 * g1, g2 * g2}, {1.0, 0.0, 1.0}, {g2 * g2, g1 * g1, g0 * g0}};
    const double SG[3][3] = {{s0 * g0, s1 * g1, s2 * g2}, {0.0, 0.0, 0.0}, {-s2 * g2, -s1 * g1, -s0 * g0}};
    auto contract3 = [&](const double *f, const double(&Tx)[3][3], const double(&Ty)[3][3],
                         const double(&Tz)[3][3], double *out) {
        double t[27], u[27];
        contract1d<2>(f, t, Tz);
        contract1d<1>(t, u, Ty);
        contract1d<0>(u, out, Tx);
    };
    // base = mass (with Darcy) + convection + the viscous |grad N_i|^2 part,
    // common to the three diagonal entries
    double base[27], t[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) w0[q] = a.am * rw[q] + dw[q];
    contract3(w0, S2, S2, S2, base);
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
        br.gather27(u0s + dir * NB, w0);
        interp3(w0);
#pragma unroll
        for (int q = 0; q < 27; ++q) w0[q] *= a.ac * rw[q] * ih[dir];
        contract3(w0, dir == 0 ? SG : S2, dir == 1 ? SG : S2, dir == 2 ? SG : S2, t);
#pragma unroll
        for (int i = 0; i < 27; ++i) base[i] += t[i];
        contract3(nu, dir == 0 ? G2 : S2, dir == 1 ? G2 : S2, dir == 2 ? G2 : S2, t);
#pragma unroll
        for (int i = 0; i < 27; ++i) base[i] += ih[dir] * ih[dir] * t[i];
    }
    // entries (0,0) (1,1) (2,2) (0,1) (0,2) (1,2); the block is symmetric but
    // for the convective term, which only enters the diagonal
    for (int e = 0; e < 6; ++e) {
        const int c = e < 3 ? e : (e == 5 ? 1 : 0);
        const int cp = e < 3 ? e : (e == 3 ? 1 : 2);
        double d[27];
        if (e < 3) { // base + nu (d_c N_i)^2
            contract3(nu, c == 0 ? G2 : S2, c == 1 ? G2 : S2, c == 2 ? G2 : S2, d);
#pragma unroll
            for (int i = 0; i < 27; ++i) d[i] = base[i] + ih[c] * ih[c] * d[i];
        } else { // nu d_c N_i d_c' N_i
            const bool x = c == 0 || cp == 0, y = c == 1 || cp == 1, z = c == 2 || cp == 2;
            contract3(nu, x ? SG : S2, y ? SG : S2, z ? SG : S2, d);
#pragma unroll
            for (int i = 0; i < 27; ++i) d[i] *= ih[c] * ih[cp];
        }
        __syncthreads();
        br.store_cell(E, d);
        __syncthreads();
        // entry e of a shared node goes to face sheet e; the combine sums it
        double *fb = face + ((int64_t)e * n_bricks(m) + br.brick) * BFACE;
        br.for_owned_nodes(m, [&](int ai, int bi, int ci, int l, int64_t g, bool constrained, int sh) {
            double *B = blocks + 9 * g;
            if (sh) {
                fb[br.fslot(ai, bi, ci)] = br.node_sum(E, ai, bi, ci); // Dirichlet ones: identity in the combine
            } else if (constrained) {
                B[3 * c + cp] = (c == cp) ? 1.0 : 0.0;
                B[3 * cp + c] = (c == cp) ? 1.0 : 0.0;
            } else {
                const double s = br.node_sum(E, ai, bi, ci);
                B[3 * c + cp] = s;
                B[3 * cp + c] = s;
            }
        });
    }
}

// Shared nodes of the 3x3 blocks: entry e = blockIdx.y of the face sheets,
// summed in the fixed order brick by brick (combine_brick_visit), written to
// both symmetric positions; Dirichlet nodes get the identity.
__global__ void __launch_bounds__(BNT * CBW) oseen_block_combine_kernel(KMesh m, const double *__restrict__ face,
                                                                        double *__restrict__ blocks)
{
    const int e = blockIdx.y;
    const int c = e < 3 ? e : (e == 5 ? 1 : 0), cp = e < 3 ? e : (e == 3 ? 1 : 2);
    const int64_t nb = n_bricks(m);
    const int brick = Brick::xcd_index() * CBW + (int)threadIdx.x / BNT;
    if (brick >= nb) return; // a whole wavefront; no barrier follows in it
    combine_brick_visit<double, true>(m, brick, (int)threadIdx.x % BNT, face + (int64_t)e * nb * BFACE,
                                      [&](int64_t g, bool constrained, double v) {
                                          double *B = blocks + 9 * g;
                                          const double s = constrained ? (c == cp ? 1.0 : 0.0) : v;
                                          B[3 * c + cp] = s;
                                          B[3 * cp + c] = s;
                                      });
}

hipError_t oseen_block_diagonal(const KMesh &m, const OseenArgs &a, double *blocks, void *face, hipStream_t s)
{
    const unsigned nb = (unsigned)n_bricks(m);
    if (!face) return hipErrorInvalidValue;
    double *fc = (double *)face;
    if (a.tc) {
        if (a.hkind == 0) oseen_block_kernel<0, true><<<nb, BNT, 0, s>>>(m, a, blocks, fc);
        else oseen_block_kernel<1, true><<<nb, BNT, 0, s>>>(m, a, blocks, fc);
    } else {
        if (a.hkind == 0) oseen_block_kernel<0, false><<<nb, BNT, 0, s>>>(m, a, blocks, fc);
        else oseen_block_kernel<1, false><<<nb, BNT, 0, s>>>(m, a, blocks, fc);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nb == 1) return hipSuccess; // single brick: nothing shared
    oseen_block_combine_kernel<<<dim3((nb + CBW - 1) / CBW, 6), BNT * CBW, 0, s>>>(m, fc, blocks);
    return hipGetLastError();
}

} // namespace mf
