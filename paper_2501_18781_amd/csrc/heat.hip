// heat.hip -- matrix-free Q2 heat operator on gfx950.
//
// Operator (Sec. 2.1, eq. heat_transfer, one backward Euler step;
// coefficients by eqs. heaviside and muEff of Sec. 2.3):
//   (A x)_i = sum_cells sum_q W_q ( alpha_m rc_q N_i x_q + alpha_k k_q grad N_i . grad x_q
//                                 [+ alpha_c rc_q N_i u_q . grad x_q] )
// applied without assembling A (App. B: matrix-free products).  The
// bracketed convective term, with a frozen nodal velocity u, is optional
// (FP64, level-set coefficients); its transpose moves the derivative onto
// the test function: alpha_c rc_q x_q u_q . grad N_i.
//
// Work decomposition (brick.hpp): one 64-thread workgroup (one wavefront)
// per brick of 4x4x4 cells, one thread per cell (the FP32 applies: bricks
// of 4x4x8 cells, two wavefronts).
//   1. the brick's nodal x and phi are staged in LDS (FP64: each node read
//      once, node-parallel over the wavefront; FP32: each cell reads its 27
//      nodes); Dirichlet columns read as zero when x is gathered;
//   2. each thread evaluates its cell entirely in registers by sum
//      factorization (3x3 contractions along one direction at a time,
//      collocation derivatives at the Gauss points, one 3-point line at a
//      time);
//   3. each owned node sums the (at most 8) cells of the brick that share it
//      in a fixed order, in registers (cross-lane shifts in x and y, an LDS
//      exchange in z);
//   4. nodes complete within the brick are stored; nodes on a face shared
//      with a neighbouring brick go to a face buffer, and a second kernel
//      adds the partials of the bricks sharing each such node in a fixed
//      order, brick by brick.  Every output entry is written once, without
//      atomics, and the result is bitwise reproducible.  Dirichlet nodes get
//      y_i = x_i.
#include <hip/hip_ext.h>

#include <type_traits>

#include "brick.hpp"

namespace mf {

// ---------------------------------------------------------------------------
// Per-cell coefficient factors at the 27 Gauss points:
//   cm_q = alpha_m |J| w_q rc_q,   ck_q = alpha_k |J| w_q k_q / r^2
// MODE 0: from the level set through H (HK 0 linear, HK 1 sine form);
// MODE 1: k and rc given per quadrature point.
// ---------------------------------------------------------------------------
template <typename T, int MODE, int HK>
__device__ __forceinline__ void heat_cell_coeffs(const HeatArgs &a, T *phq, const T *kq, const T *rcq, T am_w,
                                                 T ak_w, T *cm, T *ck)
{
    if (MODE == 0 && HK == 1) {
        // out of line and not unrolled: one transcendental evaluation per point
        for (int q = 0; q < 27; ++q) phq[q] = T(heaviside_sine_value(a.eps, (double)phq[q]));
    }
    // The Gauss weight of point q is w[q%3] w[q/3%3] w[q/9], one of four
    // products w0^3, w0^2 w1, w0 w1^2, w1^3 (class = number of middle-point
    // indices).  cm_q = A[class] + B[class] H_q, ck_q likewise: one FMA each.
    T Am[4], Bm[4], Ak[4], Bk[4];
    if (MODE == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            T w = T(1);
#pragma unroll
            for (int i = 0; i < 3; ++i) w *= i < j ? Q2<T>::w1 : Q2<T>::w0;
            Am[j] = am_w * w * T(a.rc_g);
            Bm[j] = am_w * w * (T(a.rc_l) - T(a.rc_g));
            Ak[j] = ak_w * w * T(a.k_g);
            Bk[j] = ak_w * w * (T(a.k_l) - T(a.k_g));
        }
    }
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        const int j = (q % 3 == 1) + ((q / 3) % 3 == 1) + (q / 9 == 1);
        if (MODE == 0) {
            const T H = HK == 0 ? heaviside_linear<T>(phq[q]) : phq[q];
            cm[q] = Am[j] + Bm[j] * H;
            ck[q] = Ak[j] + Bk[j] * H;
        } else {
            const T wq = Q2<T>::weight(q % 3) * Q2<T>::weight((q / 3) % 3) * Q2<T>::weight(q / 9);
            cm[q] = am_w * wq * rcq[q];
            ck[q] = ak_w * wq * kq[q];
        }
    }
}

// Mode 2 coefficients (FP64): three phases at the frozen nodal temperature
// (staged at ts, if a.tc) and/or the Tanasawa penalty.  At each Gauss point
//   H = H(phi), H_s = 3 f_s^2 - 2 f_s^3 with f_s = clamp((T_liq - T)/(T_liq - T_sol), 0, 1),
//   k, rc = H (H_s a_s + (1 - H_s) a_l) + (1 - H) a_g         (H_s = 0 without a.tc)
//   cm_q = |J| w_q (alpha_m rc + beta H' |grad phi| rc_lg c_rcp),  ck_q = alpha_k |J| w_q k / r^2
// with rc_lg the liquid-gas blend of eq. deltaRhoCp.
template <int HK, typename BR>
__device__ __forceinline__ void heat_cell_coeffs3(const BR &br, const KMesh &m, const HeatArgs &a,
                                                  const double *ps, const double *ts, double *cm, double *ck,
                                                  double ck_scale = 1.0)
{
    double ph[27], gn[27], Tq[27];
    br.gather27(ps, ph);
    interp3(ph);
#pragma unroll
    for (int q = 0; q < 27; ++q) gn[q] = 0.0;
    if (a.penalty != 0.0) { // |grad phi|^2 at the Gauss points
        const double h[3] = {m.hx, m.hy, m.hz};
        auto dir = [&](auto D) {
            constexpr int d = decltype(D)::value;
#pragma unroll
            for (int n = 0; n < 3; ++n)
#pragma unroll
                for (int mm = 0; mm < 3; ++mm) {
                    const int i0 = lidx<d>(0, mm, n), i1 = lidx<d>(1, mm, n), i2 = lidx<d>(2, mm, n);
                    double t0, t1, t2;
                    Q2<double>::deriv_scaled(ph[i0], ph[i1], ph[i2], 1.0 / (kR * h[d]), t0, t1, t2);
                    gn[i0] += t0 * t0;
                    gn[i1] += t1 * t1;
                    gn[i2] += t2 * t2;
                }
        };
        dir(std::integral_constant<int, 0>{});
        dir(std::integral_constant<int, 1>{});
        dir(std::integral_constant<int, 2>{});
    }
    if (a.tc) {
        br.gather27(ts, Tq);
        interp3(Tq);
    }
    const double vol = m.hx * m.hy * m.hz;
    const double c_rcp = 3.0 / (a.rc_g * a.rc_g + a.rc_l * a.rc_g + a.rc_l * a.rc_l);
    const double inv_range = 1.0 / (a.T_liq - a.T_sol);
    const double ak_r2 = a.ak * ck_scale / (kR * kR); // ck_scale: 1, or 1/(4 h^2) for the equal-edge form
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        double dH;
        const double H = heaviside<double>(HK, a.eps, ph[q], &dH);
        double Hs = 0.0;
        if (a.tc) {
            const double fs = fmin(fmax((a.T_liq - Tq[q]) * inv_range, 0.0), 1.0);
            Hs = fs * fs * (3.0 - 2.0 * fs);
        }
        const double k = H * (Hs * a.k_s + (1.0 - Hs) * a.k_l) + (1.0 - H) * a.k_g;
        const double rc = H * (Hs * a.rc_s + (1.0 - Hs) * a.rc_l) + (1.0 - H) * a.rc_g;
        const double react = a.penalty * dH * sqrt(gn[q]) * (a.rc_g + H * (a.rc_l - a.rc_g)) * c_rcp;
        const double w = vol * Q2<double>::weight(q % 3) * Q2<double>::weight((q / 3) % 3) * Q2<double>::weight(q / 9);
        cm[q] = w * (a.am * rc + react);
        ck[q] = w * ak_r2 * k;
        asm volatile("" : "+v"(cm[q]), "+v"(ck[q])); // one point at a time
    }
}

// y_e = A_e x_e on one cell, in place on u (27 nodal values in, 27 out).
template <typename T>
__device__ __forceinline__ void heat_cell_apply(T *u, const T *cm, const T *ck, T ihx, T ihy, T ihz)
{
    interp3(u);
    T acc[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) acc[q] = cm[q] * u[q];
    grad_line_apply<T, 0>(u, ck, ihx, acc);
    grad_line_apply<T, 1>(u, ck, ihy, acc);
    grad_line_apply<T, 2>(u, ck, ihz, acc);
    interp3T(acc);
#pragma unroll
    for (int q = 0; q < 27; ++q) u[q] = acc[q];
}

// The same on a mesh with equal cell edges: ck4 = ck / (4 h^2) (1/h^2 and
// the 1/4 of D'' = 2 D' folded into the stiffness weights), so the
// derivative passes need no scaling.
template <typename T> __device__ __forceinline__ void heat_cell_apply_iso(T *u, const T *cm, const T *ck4)
{
    interp3(u);
    T acc[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) acc[q] = cm[q] * u[q];
    grad2_line_apply<T, 0>(u, ck4, acc);
    grad2_line_apply<T, 1>(u, ck4, acc);
    grad2_line_apply<T, 2>(u, ck4, acc);
    interp3T(acc);
#pragma unroll
    for (int q = 0; q < 27; ++q) u[q] = acc[q];
}

// A coefficient at the 27 Gauss points from H_q: A[class] + B[class] H_q,
// class = number of middle-point indices of q (the Gauss weight's class).
struct ClassCoef {
    const double *H;
    double A[4], B[4];
    __device__ __forceinline__ ClassCoef(const double *h, double scale, double c_g, double c_l) : H(h)
    {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double w = 1.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) w *= i < j ? kW1 : kW0;
            A[j] = scale * w * c_g;
            B[j] = scale * w * (c_l - c_g);
        }
    }
    __device__ __forceinline__ double operator[](int q) const
    {
        const int j = (q % 3 == 1) + ((q / 3) % 3 == 1) + (q / 9 == 1);
        return A[j] + B[j] * H[q];
    }
};

// H(phi) at the Gauss points of this thread's cell, phi from the LDS brick.
template <int HK>
__device__ __forceinline__ void cell_heaviside(const Brick &br, const HeatArgs &a, const double *ps, double *H)
{
    br.gather27(ps, H);
    interp3(H);
    if (HK == 1) {
        for (int q = 0; q < 27; ++q) // out of line, not unrolled (as in heat_cell_coeffs)
            H[q] = heaviside_sine_value(a.eps, H[q]);
    } else {
#pragma unroll
        for (int q = 0; q < 27; ++q) H[q] = heaviside_linear<double>(H[q]);
    }
}

// The convective heat operator on one cell (or its transpose, TR), in place
// on u (nodal x in, nodal y out); ps is the brick's staged phi, us its
// staged velocity components.  The coefficients rc W and k W are evaluated
// from H(phi) where they are used, and the passes are ordered so that at
// most three 27-vectors are live besides the one being formed:
//   A:   cv = u0 . grad u;  H;  acc = rc W (alpha_m u + alpha_c cv);  acc += conduction
//   A^T: H;  acc = conduction;  z = rc W u;  acc += alpha_m z + alpha_c sum_d D_d^T (u0_d z)
// The velocity components are staged in LDS one at a time, in the region
// vs, just before the pass that uses them (all threads of the brick call
// this function: the staging barriers are uniform).
template <bool TR, int HK, bool ISO = false>
__device__ __forceinline__ void heat_conv_cell_apply(const Brick &br, const KMesh &m, const HeatArgs &a,
                                                     const double *ps, double *vs, double *u)
{
    const double vol = m.hx * m.hy * m.hz;
    const double h[3] = {m.hx, m.hy, m.hz};
    const int64_t nn = (int64_t)m.NX * m.NY * m.NZ;
    interp3(u);
    double acc[27], v[27]; // v: a velocity component, then H
    auto velocity = [&](int d) {
        // read and interpolate each component where it is used, and keep the
        // derivatives of u from being formed ahead of it
        pin27(acc);
        pin27(u);
        __syncthreads(); // every thread is done with the previous component
        br.stage_nodes<1, double>(m, a.u0 + d * nn, vs, nullptr, nullptr);
        __syncthreads();
        br.gather27(vs, v);
        interp3(v);
    };
    // with equal cell edges (ISO) 1/(4 h^2) is in the stiffness weights and
    // the passes take the integer derivative form
    const double kscale = ISO ? a.ak * vol / (kR * kR) * 0.25 / (h[0] * h[0]) : a.ak * vol / (kR * kR);
    auto conduction = [&](const ClassCoef &ckw) {
        if constexpr (ISO) {
            grad2_line_apply<double, 0>(u, ckw, acc);
            grad2_line_apply<double, 1>(u, ckw, acc);
            grad2_line_apply<double, 2>(u, ckw, acc);
        } else {
            grad_line_apply<double, 0>(u, ckw, 1.0 / (h[0] * h[0]), acc);
            grad_line_apply<double, 1>(u, ckw, 1.0 / (h[1] * h[1]), acc);
            grad_line_apply<double, 2>(u, ckw, 1.0 / (h[2] * h[2]), acc);
        }
    };
#pragma unroll
    for (int q = 0; q < 27; ++q) acc[q] = 0.0;
    if (!TR) {
        velocity(0);
        vel_grad_acc<double, 0>(u, v, 1.0 / (kR * h[0]), acc);
        velocity(1);
        vel_grad_acc<double, 1>(u, v, 1.0 / (kR * h[1]), acc);
        velocity(2);
        vel_grad_acc<double, 2>(u, v, 1.0 / (kR * h[2]), acc);
        pin27(acc);
        cell_heaviside<HK>(br, a, ps, v);
        const ClassCoef rcw(v, vol, a.rc_g, a.rc_l);
#pragma unroll
        for (int q = 0; q < 27; ++q) acc[q] = rcw[q] * (a.am * u[q] + a.ac * acc[q]);
        const ClassCoef ckw(v, kscale, a.k_g, a.k_l);
#pragma unroll
        for (int q = 0; q < 27; ++q) v[q] = ckw[q]; // H -> k W, in place
        pin27(v);
        pin27(u);
        pin27(acc);
        if constexpr (ISO) {
            grad2_line_apply<double, 0>(u, v, acc);
            grad2_line_apply<double, 1>(u, v, acc);
            grad2_line_apply<double, 2>(u, v, acc);
        } else {
            grad_line_apply<double, 0>(u, v, 1.0 / (h[0] * h[0]), acc);
            grad_line_apply<double, 1>(u, v, 1.0 / (h[1] * h[1]), acc);
            grad_line_apply<double, 2>(u, v, 1.0 / (h[2] * h[2]), acc);
        }
    } else {
        cell_heaviside<HK>(br, a, ps, v);
        conduction(ClassCoef(v, kscale, a.k_g, a.k_l));
        const ClassCoef rcw(v, vol, a.rc_g, a.rc_l);
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            u[q] *= rcw[q];
            acc[q] += a.am * u[q];
        }
        velocity(0);
        vel_gradT_acc<double, 0>(u, v, a.ac / (kR * h[0]), acc);
        velocity(1);
        vel_gradT_acc<double, 1>(u, v, a.ac / (kR * h[1]), acc);
        velocity(2);
        vel_gradT_acc<double, 2>(u, v, a.ac / (kR * h[2]), acc);
    }
    interp3T(acc);
#pragma unroll
    for (int q = 0; q < 27; ++q) u[q] = acc[q];
}

// CONV: 0 plain heat operator; 1 with the convective term; 2 its transpose
// (FP64, level-set coefficients, no CG epilogue).  Bricks of 4 x 4 x BZ
// cells, one thread per cell (BZ = 8: two wavefronts per brick).
template <typename T, int MODE, int HK, bool CG, int CONV = 0, bool ISO = false, int BZ = BB>
__global__ void __launch_bounds__(BrickDims<BZ>::NT) heat_apply_kernel(KMesh m, HeatArgs a, const T *__restrict__ x,
                                                                       T *__restrict__ y, T *__restrict__ face,
                                                                       CGState *cg, RedWS red)
{
    static_assert(CONV == 0 || (std::is_same<T, double>::value && MODE == 0 && !CG), "convective form: FP64 only");
    static_assert(MODE != 2 || std::is_same<T, double>::value, "three-phase coefficients: FP64 only");
    static_assert(CONV == 0 || BZ == BB, "convective form: 4x4x4 bricks (its velocity staging)");
    using BR = BrickT<BZ>;
    constexpr int NT = BR::NT;
    // x stays resident (Dirichlet rows y = x and the CG epilogue read it);
    // the second region takes phi (with one velocity component at a time, or
    // the frozen temperature), then the z exchange of the node sums (for the
    // transposed convective form, the cell results).
    constexpr int NB = lds_field<T, BZ>(); // one staged field
    constexpr int STAGE = CONV == 2 ? 27 * NT : ((CONV || MODE == 2) ? 2 * NB : NB);
    static_assert(STAGE >= 9 * NT, "the second region takes the z exchange of the node sums");
    constexpr int LDS_T = NB + STAGE;
    __shared__ T lds[LDS_T];
    __shared__ double red_lds[NT];
    if (CG) {
        if (cg->done) return; // converged or broken down: the rest of the batch is a no-op
    }
    const BR br(m, threadIdx.x);
    T *xs = lds;
    T *ps = lds + NB;
    if constexpr (MODE == 2) {
        if (a.tc) {
            const double *src[3] = {(const double *)x, (const double *)a.phi, (const double *)a.tc};
            double *const dst[3] = {(double *)xs, (double *)ps, (double *)ps + NB};
            br.template stage_nodes_wg<NT, 3>(m, threadIdx.x, src, dst, 0u);
        } else {
            br.template stage_nodes<2, T>(m, x, xs, (const T *)a.phi, ps);
        }
    } else if constexpr (sizeof(T) == 8) {
        if (MODE != 1) br.template stage_nodes<2, T>(m, x, xs, (const T *)a.phi, ps);
        else br.template stage_nodes<1, T>(m, x, xs, nullptr, nullptr);
    } else {
        if (MODE != 1) br.load_fields(m, x, xs, (const T *)a.phi, ps);
        else br.load_fields(m, x, xs);
    }
    __syncthreads();

    const T vol = T(m.hx * m.hy * m.hz);
    const T am_w = T(a.am) * vol;
    const T ak_w = T(a.ak) * vol / T(kR * kR);
    const T ihx = T(1.0 / (m.hx * m.hx)), ihy = T(1.0 / (m.hy * m.hy)), ihz = T(1.0 / (m.hz * m.hz));
    T u[27];
    if constexpr (CONV != 0) {
        br.gather27_dirichlet(m, xs, u);
        heat_conv_cell_apply<CONV == 2, HK, ISO>(br, m, a, ps, ps + NB, u);
    } else {
        // With equal cell edges (ISO) 1/h^2 and the 1/4 of D'' = 2 D' go into
        // the stiffness weights, and the derivative passes take the integer
        // form (5 operations per line instead of 7).
        const T akw = ISO ? ak_w * ihx * T(0.25) : ak_w;
        T cm[27], ck[27];
        if constexpr (MODE == 2) {
            heat_cell_coeffs3<HK>(br, m, a, (const double *)ps, (const double *)ps + NB, cm, ck,
                                  ISO ? double(ihx) * 0.25 : 1.0);
        } else if (MODE == 0) {
            T ph[27];
            br.gather27(ps, ph);
            interp3(ph);
            heat_cell_coeffs<T, 0, HK>(a, ph, nullptr, nullptr, am_w, akw, cm, ck);
        } else {
            const int64_t cell = br.valid ? br.cell_index(m) : 0;
            heat_cell_coeffs<T, 1, 0>(a, nullptr, (const T *)a.kq + 27 * cell, (const T *)a.rcq + 27 * cell, am_w,
                                      akw, cm, ck);
        }
        br.gather27_dirichlet(m, xs, u);
        if constexpr (ISO) heat_cell_apply_iso<T>(u, cm, ck);
        else heat_cell_apply<T>(u, cm, ck, ihx, ihy, ihz);
    }
    __syncthreads(); // the phi region is now reused for the node sums
    if constexpr (CONV == 2) {
        // through LDS: the transposed convective form has no registers to
        // spare for the register exchange
        T *E = ps;
        br.store_cell(E, u);
        __syncthreads();
        br.template for_owned_nodes<T>(m, [&](int ai, int bi, int ci, int, int64_t, bool, int) {
            u[ai + 3 * bi + 9 * ci] = br.node_sum(E, ai, bi, ci);
        });
    } else {
        br.assemble27(u, ps);
    }

    // Owned nodes: complete nodes go to y, shared ones to the face buffer;
    // Dirichlet rows get y_i = x_i (shared ones in the combine pass).
    // x.Ax = sum over bricks of x_i times the brick's partial sum at node i,
    // with x_i^2 for a Dirichlet node counted once, by the brick that
    // finishes it.
    double energy = 0.0;
    T *fb = face + (int64_t)br.brick * BR::NFACE;
    br.template for_owned_nodes<T>(m, [&](int ai, int bi, int ci, int l, int64_t g, bool constrained, int sh) {
        const T xv = xs[l], s = u[ai + 3 * bi + 9 * ci];
        if (CG) energy += constrained ? ((sh & 2) ? 0.0 : (double)xv * (double)xv) : (double)xv * (double)s;
        T *dst = sh ? fb + br.fslot(ai, bi, ci) : y + g;
        *dst = constrained ? xv : s;
    });
    if (CG) {
        // one partial per brick; the alpha kernel sums them in brick order
        const double tot = block_sum<NT>(energy, red_lds);
        write_partials<1>(&tot, red.partials, gridDim.x, (unsigned)br.brick);
    }
}

// Second pass of an apply, a diagonal or a gradient: the shared nodes, each
// the sum of the bricks' face partials in a fixed order, finished brick by
// brick (combine_brick in brick.hpp).  In CG mode the first workgroup first
// sums the bricks' partials of p.Ap (complete once the brick kernel has
// finished) and sets alpha = rz / p.Ap, which saves a launch per
// iteration.  A breakdown sets done here; a workgroup of this launch that
// then skips its nodes leaves q incomplete, which no later step of the
// solve reads.
template <typename T, bool CG, int DMODE = 1, int BZ = BB>
__global__ void __launch_bounds__(BNT * CBW) face_combine_brick_kernel(KMesh m, const T *__restrict__ face,
                                                                 const T *__restrict__ x, T *__restrict__ y,
                                                                 CGState *cg, const double *__restrict__ partials,
                                                                 unsigned nbricks)
{
    if (CG) {
        if (cg->done) return;
    }
    if (CG && blockIdx.x == 0) {
        // before the combine, which lets wavefronts without a brick leave
        __shared__ double red[BNT * CBW];
        const double pAp = sum_partials<BNT * CBW>(partials, nbricks, 0, red);
        if (threadIdx.x == 0) {
            cg->pAp = pAp;
            if (!(pAp > 0.0) || !isfinite(pAp)) {
                cg->breakdown = 1;
                cg->done = 1;
                cg->alpha = 0.0;
            } else {
                cg->alpha = cg->rz / pAp;
            }
        }
    }
    combine_brick<T, DMODE, BZ>(m, face, x, y);
}

// Brick depth of the FP32 applies (the multigrid levels): 4x4x8 cells, two
// wavefronts per brick.  Against 4x4x4 bricks this halves the internal z
// planes of the brick grid, and with them the face-buffer partials and the
// combine pass's z-shared nodes (128^3 FP32 whole apply about 5 % faster).
// The FP64 applies keep 4x4x4 bricks: there the deeper brick made the brick
// kernel slower by as much as it made the combine faster.
constexpr int HEAT_BZ32 = 8;

int64_t face_buffer_elems(const KMesh &m)
{
    const int64_t b4 = n_bricks<BB>(m) * BrickDims<BB>::NFACE;
    const int64_t b8 = n_bricks<HEAT_BZ32>(m) * BrickDims<HEAT_BZ32>::NFACE;
    return b4 > b8 ? b4 : b8;
}

// One apply: the brick kernel, then the combine pass of its shared nodes
// (with CG, alpha from the bricks' partials of p.Ap).  With timing on, the
// events are attached to the brick kernel's own dispatch (they record its
// start and end, not the neighbouring queue packets).
template <typename T, int MODE, int HK, bool CGF, int CV, bool ISO>
static hipError_t heat_apply_launch(const KMesh &m, const HeatArgs &a, const void *x, void *y, void *face,
                                    CGState *cg, const RedWS &r, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    constexpr int BZ = sizeof(T) == 4 ? HEAT_BZ32 : BB;
    constexpr int NT = BrickDims<BZ>::NT;
    const unsigned nb = (unsigned)n_bricks<BZ>(m);
    if (ev0)
        hipExtLaunchKernelGGL(heat_apply_kernel<T, MODE, HK, CGF, CV, ISO, BZ>, dim3(nb), dim3(NT), 0, s, ev0, ev1, 0,
                              m, a, (const T *)x, (T *)y, (T *)face, cg, r);
    else
        heat_apply_kernel<T, MODE, HK, CGF, CV, ISO, BZ><<<nb, NT, 0, s>>>(m, a, (const T *)x, (T *)y, (T *)face, cg, r);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // a single brick shares nothing; alpha from its partial
    if (nb == 1) return CGF ? cg_alpha(cg, &r, nb, s) : hipSuccess;
    constexpr int BPW = BNT * CBW / CombineLanes<BZ>::value; // bricks per combine workgroup
    face_combine_brick_kernel<T, CGF, 1, BZ><<<(nb + BPW - 1) / BPW, BNT * CBW, 0, s>>>(
        m, (const T *)face, (const T *)x, (T *)y, CGF ? cg : nullptr, CGF ? r.partials : nullptr, CGF ? nb : 0u);
    return hipGetLastError();
}

hipError_t heat_apply(const KMesh &m, const HeatArgs &a, int fp32, const void *x, void *y, void *face, CGState *cg,
                      const RedWS *red, hipStream_t s, const KTiming *t)
{
    const unsigned nb = (unsigned)n_bricks(m); // the most bricks of any layout
    RedWS r = red ? *red : RedWS{nullptr, 0};
    if (!face) return hipErrorInvalidValue;
    if (cg && (!red || red->capacity < nb)) return hipErrorInvalidValue;
    if (fp32 && cg) return hipErrorInvalidValue;
    hipEvent_t ev0 = t ? t->start : nullptr, ev1 = t ? t->stop : nullptr;
    if (a.conv && (fp32 || cg || a.mode != 0 || !a.u0)) return hipErrorInvalidValue;
    if (a.mode == 2 && fp32) return hipErrorInvalidValue;
    // (convective form, precision, coefficient mode, Heaviside form, CG epilogue)
    const int hk = a.mode == 1 ? 0 : (a.hkind ? 1 : 0);
    // equal cell edges (a cube's cells): the scale-free derivative form
    const bool iso = m.hx == m.hy && m.hy == m.hz;
    const int key = (iso ? 128 : 0) | (a.conv << 5) | (fp32 ? 16 : 0) | (a.mode << 2) | (hk << 1) | (cg ? 1 : 0);
    switch (key) {
#define HEAT_CASE(K, T, MODE, HK, CGF, CV, ISO)                                                               \
    case K:                                                                                                   \
        return heat_apply_launch<T, MODE, HK, CGF, CV, ISO>(m, a, x, y, face, cg, r, s, ev0, ev1);
        HEAT_CASE(0, double, 0, 0, false, 0, false)
        HEAT_CASE(1, double, 0, 0, true, 0, false)
        HEAT_CASE(2, double, 0, 1, false, 0, false)
        HEAT_CASE(3, double, 0, 1, true, 0, false)
        HEAT_CASE(4, double, 1, 0, false, 0, false)
        HEAT_CASE(5, double, 1, 0, true, 0, false)
        HEAT_CASE(8, double, 2, 0, false, 0, false)
        HEAT_CASE(9, double, 2, 0, true, 0, false)
        HEAT_CASE(10, double, 2, 1, false, 0, false)
        HEAT_CASE(11, double, 2, 1, true, 0, false)
        HEAT_CASE(16, float, 0, 0, false, 0, false)
        HEAT_CASE(18, float, 0, 1, false, 0, false)
        HEAT_CASE(20, float, 1, 0, false, 0, false)
        HEAT_CASE(32, double, 0, 0, false, 1, false)
        HEAT_CASE(34, double, 0, 1, false, 1, false)
        HEAT_CASE(64, double, 0, 0, false, 2, false)
        HEAT_CASE(66, double, 0, 1, false, 2, false)
        HEAT_CASE(128, double, 0, 0, false, 0, true)
        HEAT_CASE(129, double, 0, 0, true, 0, true)
        HEAT_CASE(130, double, 0, 1, false, 0, true)
        HEAT_CASE(131, double, 0, 1, true, 0, true)
        HEAT_CASE(132, double, 1, 0, false, 0, true)
        HEAT_CASE(133, double, 1, 0, true, 0, true)
        HEAT_CASE(136, double, 2, 0, false, 0, true)
        HEAT_CASE(137, double, 2, 0, true, 0, true)
        HEAT_CASE(138, double, 2, 1, false, 0, true)
        HEAT_CASE(139, double, 2, 1, true, 0, true)
        HEAT_CASE(160, double, 0, 0, false, 1, true)
        HEAT_CASE(162, double, 0, 1, false, 1, true)
        HEAT_CASE(192, double, 0, 0, false, 2, true)
        HEAT_CASE(194, double, 0, 1, false, 2, true)
        HEAT_CASE(144, float, 0, 0, false, 0, true)
        HEAT_CASE(146, float, 0, 1, false, 0, true)
        HEAT_CASE(148, float, 1, 0, false, 0, true)
#undef HEAT_CASE
    default:
        return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Diagonal: diag_i = sum_cells sum_q cm_q N_i(q)^2 + ck_q sum_d ih_d (d_d N_i(q))^2.
// N_i(q) and its derivatives are products of 1D factors, so the sum over q
// factorizes like the apply: contractions with the elementwise squares of
// the 1D value and derivative tables S and G along z, y, x.  Node sums and
// shared faces as in the apply; Dirichlet nodes get 1.
// ---------------------------------------------------------------------------

// Cell diagonal from cm_q and ck_q (ck_q for the true 1D derivatives G).
template <typename T>
__device__ __forceinline__ void heat_cell_diag(const T *cm, const T *ck, T ihx, T ihy, T ihz, T *d)
{
    // squares of S[q][a] = l_a(xi_q) and G[q][a] = l_a'(xi_q)
    constexpr T s0 = Q2<T>::s0, s1 = Q2<T>::s1, s2 = Q2<T>::s2;
    constexpr T g0 = Q2<T>::g0, g1 = Q2<T>::g1, g2 = Q2<T>::g2;
    const T S2[3][3] = {{s0 * s0, s1 * s1, s2 * s2}, {T(0), T(1), T(0)}, {s2 * s2, s1 * s1, s0 * s0}};
    const T G2[3][3] = {{g0 * g0, g1 * g1, g2 * g2}, {T(1), T(0), T(1)}, {g2 * g2, g1 * g1, g0 * g0}};
    T t[27], u[27], w[27];
    contract1d<2>(cm, t, S2);
    contract1d<1>(t, w, S2);          // mass, contracted along z and y
    contract1d<2>(ck, t, S2);
    contract1d<1>(t, u, G2);          // y-derivative part
#pragma unroll
    for (int i = 0; i < 27; ++i) w[i] += ihy * u[i];
    contract1d<1>(t, u, S2);          // x-derivative part, before x
    contract1d<0>(u, d, G2);
    contract1d<2>(ck, t, G2);
    contract1d<1>(t, u, S2);          // z-derivative part
#pragma unroll
    for (int i = 0; i < 27; ++i) w[i] += ihz * u[i];
    contract1d<0>(w, t, S2);
#pragma unroll
    for (int i = 0; i < 27; ++i) d[i] = t[i] + ihx * d[i];
}

// Convective part of the cell diagonal: sum_q c_q N_i(q) u_q . grad N_i(q)
// with c_q = alpha_c |J| w_q rc_q (rcw_q times alpha_c).  Along direction d,
// N_i d_d N_i is (1/h_d) l_a l_a' along d times l^2 along the other two, so
// each velocity component is contracted with S.G along d and S^2 elsewhere.
__device__ __forceinline__ void heat_cell_conv_diag(const Brick &br, const KMesh &m, const double *us,
                                                    const double *rcw, double ac, double *d)
{
    constexpr double s0 = Q2<double>::s0, s1 = Q2<double>::s1, s2 = Q2<double>::s2;
    constexpr double g0 = Q2<double>::g0, g1 = Q2<double>::g1, g2 = Q2<double>::g2;
    const double S2[3][3] = {{s0 * s0, s1 * s1, s2 * s2}, {0.0, 1.0, 0.0}, {s2 * s2, s1 * s1, s0 * s0}};
    const double SG[3][3] = {{s0 * g0, s1 * g1, s2 * g2}, {0.0, 0.0, 0.0}, {-s2 * g2, -s1 * g1, -s0 * g0}};
    const double h[3] = {m.hx, m.hy, m.hz};
    double w[27], t[27], v[27];
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
        br.gather27(us + dir * lds_field<double>(), w);
        interp3(w);
        const double sc = ac / h[dir];
#pragma unroll
        for (int q = 0; q < 27; ++q) w[q] *= sc * rcw[q];
        contract1d<2>(w, t, dir == 2 ? SG : S2);
        contract1d<1>(t, v, dir == 1 ? SG : S2);
        contract1d<0>(v, t, dir == 0 ? SG : S2);
#pragma unroll
        for (int i = 0; i < 27; ++i) d[i] += t[i];
    }
}

// INV: store 1 / diag (the Jacobi preconditioner) instead of diag.
template <typename T, int MODE, int HK, bool CONV = false, bool INV = false>
__global__ void __launch_bounds__(BNT) heat_diag_kernel(KMesh m, HeatArgs a, T *__restrict__ diag, T *__restrict__ face)
{
    static_assert(!CONV || (std::is_same<T, double>::value && MODE == 0), "convective form: FP64 only");
    constexpr int NB = lds_field<T>(); // one staged field
    constexpr int STAGE = CONV ? 4 * NB : NB;
    constexpr int LDS_T = (STAGE > 27 * BNT ? STAGE : 27 * BNT);
    __shared__ T lds[LDS_T];
    const Brick br(m, threadIdx.x);
    if constexpr (CONV) {
        const int64_t nn = (int64_t)m.NX * m.NY * m.NZ;
        const double *u0 = (const double *)a.u0;
        const double *src[4] = {(const double *)a.phi, u0, u0 + nn, u0 + 2 * nn};
        double *const dst[4] = {(double *)lds, (double *)lds + NB, (double *)lds + 2 * NB, (double *)lds + 3 * NB};
        br.stage_nodes_wg<BNT, 4>(m, threadIdx.x, src, dst, 0u);
    } else if constexpr (MODE == 2) {
        if (a.tc) br.template stage_nodes<2, T>(m, (const T *)a.phi, lds, (const T *)a.tc, lds + NB);
        else br.template stage_nodes<1, T>(m, (const T *)a.phi, lds, nullptr, nullptr);
    } else if constexpr (MODE != 1) {
        if constexpr (sizeof(T) == 8) br.template stage_nodes<1, T>(m, (const T *)a.phi, lds, nullptr, nullptr);
        else br.load(m, (const T *)a.phi, lds, false);
    }
    __syncthreads();
    const T vol = T(m.hx * m.hy * m.hz);
    const T am_w = CONV ? vol : T(a.am) * vol, ak_w = T(a.ak) * vol;
    const T ihx = T(1.0 / (m.hx * m.hx)), ihy = T(1.0 / (m.hy * m.hy)), ihz = T(1.0 / (m.hz * m.hz));
    T cm[27], ck[27];
    if constexpr (MODE == 2) {
        heat_cell_coeffs3<HK>(br, m, a, (const double *)lds, (const double *)lds + NB, cm, ck);
        // heat_cell_diag takes the stiffness factor for the true derivatives (no 1/r^2)
#pragma unroll
        for (int q = 0; q < 27; ++q) ck[q] *= kR * kR;
    } else if (MODE == 0) {
        T ph[27];
        br.gather27(lds, ph);
        interp3(ph);
        heat_cell_coeffs<T, 0, HK>(a, ph, nullptr, nullptr, am_w, ak_w, cm, ck);
    } else {
        const int64_t cell = br.valid ? br.cell_index(m) : 0;
        heat_cell_coeffs<T, 1, 0>(a, nullptr, (const T *)a.kq + 27 * cell, (const T *)a.rcq + 27 * cell, am_w, ak_w,
                                  cm, ck);
    }
    T d[27];
    if constexpr (CONV) {
        // cm holds |J| w_q rc_q here
        T md[27];
#pragma unroll
        for (int q = 0; q < 27; ++q) md[q] = T(a.am) * cm[q];
        heat_cell_diag<T>(md, ck, ihx, ihy, ihz, d);
        heat_cell_conv_diag(br, m, (const double *)lds + NB, (const double *)cm, a.ac, (double *)d);
    } else {
        heat_cell_diag<T>(cm, ck, ihx, ihy, ihz, d);
    }
    __syncthreads();
    br.store_cell(lds, d);
    __syncthreads();
    T *fb = face + (int64_t)br.brick * BFACE;
    br.template for_owned_nodes<T>(m, [&](int ai, int bi, int ci, int, int64_t g, bool constrained, int sh) {
        const T v = br.node_sum(lds, ai, bi, ci);
        if (sh) fb[br.fslot(ai, bi, ci)] = v; // constrained ones: 1 in the combine
        else diag[g] = constrained ? T(1) : (INV ? T(1) / v : v);
    });
}

template <bool INV>
static hipError_t heat_diagonal_launch(const KMesh &m, const HeatArgs &a, int fp32, void *diag, void *face,
                                       hipStream_t s)
{
    const unsigned nb = (unsigned)n_bricks(m);
    if (!face) return hipErrorInvalidValue;
    float *df = (float *)diag, *ff = (float *)face;
    double *dd = (double *)diag, *fd = (double *)face;
    if (fp32) {
        if (a.mode == 1) heat_diag_kernel<float, 1, 0, false, INV><<<nb, BNT, 0, s>>>(m, a, df, ff);
        else if (a.hkind == 1) heat_diag_kernel<float, 0, 1, false, INV><<<nb, BNT, 0, s>>>(m, a, df, ff);
        else heat_diag_kernel<float, 0, 0, false, INV><<<nb, BNT, 0, s>>>(m, a, df, ff);
    } else if (a.conv) {
        if (a.mode != 0 || !a.u0) return hipErrorInvalidValue;
        if (a.hkind == 1) heat_diag_kernel<double, 0, 1, true, INV><<<nb, BNT, 0, s>>>(m, a, dd, fd);
        else heat_diag_kernel<double, 0, 0, true, INV><<<nb, BNT, 0, s>>>(m, a, dd, fd);
    } else {
        if (a.mode == 2) {
            if (a.hkind == 1) heat_diag_kernel<double, 2, 1, false, INV><<<nb, BNT, 0, s>>>(m, a, dd, fd);
            else heat_diag_kernel<double, 2, 0, false, INV><<<nb, BNT, 0, s>>>(m, a, dd, fd);
        } else if (a.mode == 1)
            heat_diag_kernel<double, 1, 0, false, INV><<<nb, BNT, 0, s>>>(m, a, dd, fd);
        else if (a.hkind == 1) heat_diag_kernel<double, 0, 1, false, INV><<<nb, BNT, 0, s>>>(m, a, dd, fd);
        else heat_diag_kernel<double, 0, 0, false, INV><<<nb, BNT, 0, s>>>(m, a, dd, fd);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nb == 1) return hipSuccess; // a single brick shares nothing
    // DMODE 2: Dirichlet rows 1; 4: the same, and the reciprocals of the others
    constexpr int DM = INV ? 4 : 2;
    const unsigned wg = (nb + CBW - 1) / CBW;
    if (fp32) face_combine_brick_kernel<float, false, DM><<<wg, BNT * CBW, 0, s>>>(m, ff, nullptr, df, nullptr, nullptr, 0);
    else face_combine_brick_kernel<double, false, DM><<<wg, BNT * CBW, 0, s>>>(m, fd, nullptr, dd, nullptr, nullptr, 0);
    return hipGetLastError();
}

hipError_t heat_diagonal(const KMesh &m, const HeatArgs &a, int fp32, void *diag, void *face, hipStream_t s,
                         bool invert)
{
    return invert ? heat_diagonal_launch<true>(m, a, fp32, diag, face, s)
                  : heat_diagonal_launch<false>(m, a, fp32, diag, face, s);
}

// ---------------------------------------------------------------------------
// Whole Jacobi-preconditioned CG solve (x0 = 0) of an FP64 heat operator on a
// mesh that is a single brick (at most 4 cells per direction), in one
// workgroup launch: all vectors live in LDS, the cell coefficients stay in
// registers across iterations, reductions are one wavefront's shuffles.
// Serves the coarsest multigrid level, whose right-hand side and solution
// are FP32.  Stops when ||r|| <= rtol ||b||, at maxit, or on breakdown.
// ---------------------------------------------------------------------------
// Sum over the wavefront, identical in every lane.
__device__ __forceinline__ double wave_total(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return __shfl(v, 0, 64);
}

// INV: workgroup c solves A x = e_c and writes x as column c of inv (FP64,
// column-major, n_nodes rows): the columns of A^-1, all solved at once.
template <int HK, bool INV = false>
__global__ void __launch_bounds__(BNT) heat_cg_brick_kernel(KMesh m, HeatArgs a, const float *__restrict__ b32,
                                                            float *__restrict__ x32, double rtol, int maxit,
                                                            double *__restrict__ inv)
{
    constexpr int NB = lds_field<double>();
    __shared__ double X[NB], R[NB], P[NB], Q[NB], S[NB], Dv[NB];
    __shared__ double E[27 * BNT];
    const Brick br(m, threadIdx.x, 0); // the mesh is one brick, whatever the workgroup (INV: one per column)
    br.stage_nodes<1, double>(m, (const double *)a.phi, S, nullptr, nullptr);
    __syncthreads();
    const double vol = m.hx * m.hy * m.hz;
    const double am_w = a.am * vol, ak_w = a.ak * vol / (kR * kR);
    const double ihx = 1.0 / (m.hx * m.hx), ihy = 1.0 / (m.hy * m.hy), ihz = 1.0 / (m.hz * m.hz);
    double cm[27], ck[27];
    {
        double ph[27];
        br.gather27(S, ph);
        interp3(ph);
        heat_cell_coeffs<double, 0, HK>(a, ph, nullptr, nullptr, am_w, ak_w, cm, ck);
        double ckd[27], d[27];
#pragma unroll
        for (int q = 0; q < 27; ++q) ckd[q] = ck[q] * (kR * kR);
        heat_cell_diag<double>(cm, ckd, ihx, ihy, ihz, d);
        br.store_cell(E, d);
    }
    __syncthreads();
    double rz = 0.0, bb = 0.0;
    br.for_owned_nodes(m, [&](int ai, int bi, int ci, int l, int64_t g, bool constrained, int) {
        const double dv = br.node_sum(E, ai, bi, ci);
        const double di = constrained ? 1.0 : 1.0 / dv;
        const double bv = INV ? (g == (int64_t)blockIdx.x ? 1.0 : 0.0) : (double)b32[g];
        Dv[l] = di;
        X[l] = 0.0;
        R[l] = bv;
        const double z = di * bv;
        P[l] = z;
        rz += bv * z;
        bb += bv * bv;
    });
    rz = wave_total(rz);
    bb = wave_total(bb);
    const double thresh2 = rtol * rtol * bb;
    for (int it = 0; it < maxit && bb > 0.0; ++it) {
        br.for_owned_nodes(m, [&](int, int, int, int l, int64_t, bool constrained, int) {
            S[l] = constrained ? 0.0 : P[l];
        });
        __syncthreads(); // S complete; E no longer read
        double u[27];
        br.gather27(S, u);
        heat_cell_apply<double>(u, cm, ck, ihx, ihy, ihz);
        br.store_cell(E, u);
        __syncthreads();
        double pq = 0.0;
        br.for_owned_nodes(m, [&](int ai, int bi, int ci, int l, int64_t, bool constrained, int) {
            const double qv = constrained ? P[l] : br.node_sum(E, ai, bi, ci);
            Q[l] = qv;
            pq += P[l] * qv;
        });
        pq = wave_total(pq);
        if (!(pq > 0.0) || !isfinite(pq)) break;
        const double alpha = rz / pq;
        double rzn = 0.0, rr = 0.0;
        br.for_owned_nodes(m, [&](int, int, int, int l, int64_t, bool, int) {
            X[l] += alpha * P[l];
            const double r = R[l] - alpha * Q[l];
            R[l] = r;
            const double z = Dv[l] * r;
            Q[l] = z;
            rzn += r * z;
            rr += r * r;
        });
        rzn = wave_total(rzn);
        rr = wave_total(rr);
        if (rr <= thresh2 || !isfinite(rr)) break;
        const double beta = rzn / rz;
        rz = rzn;
        br.for_owned_nodes(m, [&](int, int, int, int l, int64_t, bool, int) { P[l] = Q[l] + beta * P[l]; });
    }
    br.for_owned_nodes(m, [&](int, int, int, int l, int64_t g, bool, int) {
        if constexpr (INV) inv[(int64_t)blockIdx.x * m.NX * m.NY * m.NZ + g] = X[l];
        else x32[g] = (float)X[l];
    });
}

bool heat_fits_one_brick(const KMesh &m) { return m.nx <= BB && m.ny <= BB && m.nz <= BB; }

hipError_t heat_cg_one_brick(const KMesh &m, const HeatArgs &a, const float *b32, float *x32, double rtol, int maxit,
                             hipStream_t s)
{
    if (!heat_fits_one_brick(m) || a.mode != 0) return hipErrorInvalidValue;
    if (a.hkind == 1) heat_cg_brick_kernel<1><<<1, BNT, 0, s>>>(m, a, b32, x32, rtol, maxit, nullptr);
    else heat_cg_brick_kernel<0><<<1, BNT, 0, s>>>(m, a, b32, x32, rtol, maxit, nullptr);
    return hipGetLastError();
}

hipError_t heat_inverse_one_brick(const KMesh &m, const HeatArgs &a, double *inv, double rtol, int maxit, hipStream_t s)
{
    if (!heat_fits_one_brick(m) || a.mode != 0) return hipErrorInvalidValue;
    const unsigned nn = (unsigned)(m.NX * m.NY * m.NZ);
    if (a.hkind == 1) heat_cg_brick_kernel<1, true><<<nn, BNT, 0, s>>>(m, a, nullptr, nullptr, rtol, maxit, inv);
    else heat_cg_brick_kernel<0, true><<<nn, BNT, 0, s>>>(m, a, nullptr, nullptr, rtol, maxit, inv);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Quadrature-point fields: coordinates and coefficients (one thread per cell,
// nodal values read straight from global memory).
// ---------------------------------------------------------------------------
__global__ void quad_points_kernel(KMesh m, double *__restrict__ xq)
{
    const int64_t nc = (int64_t)m.nx * m.ny * m.nz;
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= nc) return;
    const int cx = (int)(cell % m.nx), cy = (int)((cell / m.nx) % m.ny), cz = (int)(cell / ((int64_t)m.nx * m.ny));
    const double xi[3] = {0.5 - kR, 0.5, 0.5 + kR};
    for (int q = 0; q < 27; ++q) {
        double *o = xq + (cell * 27 + q) * 3;
        o[0] = m.lox + m.hx * (cx + xi[q % 3]);
        o[1] = m.loy + m.hy * (cy + xi[(q / 3) % 3]);
        o[2] = m.loz + m.hz * (cz + xi[q / 9]);
    }
}

hipError_t quad_points(const KMesh &m, double *xq, hipStream_t s)
{
    const int64_t nc = (int64_t)m.nx * m.ny * m.nz;
    quad_points_kernel<<<(unsigned)((nc + 255) / 256), 256, 0, s>>>(m, xq);
    return hipGetLastError();
}

constexpr int QPT = 256; // threads per workgroup of the quadrature-point coefficient pass

__global__ void __launch_bounds__(QPT) heat_qp_kernel(KMesh m, HeatArgs a, double *__restrict__ kq,
                                                     double *__restrict__ rcq)
{
    const int64_t nc = (int64_t)m.nx * m.ny * m.nz;
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= nc) return;
    const int cx = (int)(cell % m.nx), cy = (int)((cell / m.nx) % m.ny), cz = (int)(cell / ((int64_t)m.nx * m.ny));
    double ph[27];
    const double *phi = (const double *)a.phi;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int i = 0; i < 3; ++i) ph[i + 3 * b + 9 * c] = phi[node_index(m, 2 * cx + i, 2 * cy + b, 2 * cz + c)];
    interp3(ph);
    // unrolled: a loop over q would index ph at run time and put it in
    // scratch memory
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        const double H = heaviside<double>(a.hkind, a.eps, ph[q], nullptr);
        kq[cell * 27 + q] = a.k_g + H * (a.k_l - a.k_g);
        rcq[cell * 27 + q] = a.rc_g + H * (a.rc_l - a.rc_g);
    }
}

hipError_t heat_qp_coeffs(const KMesh &m, const HeatArgs &a, double *kq, double *rcq, hipStream_t s)
{
    const int64_t nc = (int64_t)m.nx * m.ny * m.nz;
    heat_qp_kernel<<<(unsigned)((nc + QPT - 1) / QPT), QPT, 0, s>>>(m, a, kq, rcq);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adjoint gradient of one implicit heat step (FP64):
//   dk_q  = -alpha_k W_q grad(lam) . grad(T)
//   drc_q = -alpha_m W_q lam dT
//   dphi_j = sum_q N_j(x_q) H'(phi_q) [(k_l - k_g) dk_q + (rc_l - rc_g) drc_q]
// ---------------------------------------------------------------------------
template <int HK>
__global__ void __launch_bounds__(BNT) heat_grad_kernel(KMesh m, HeatArgs a, const double *__restrict__ T,
                                                        const double *__restrict__ dT, const double *__restrict__ lam,
                                                        double *__restrict__ dk, double *__restrict__ drc,
                                                        double *__restrict__ dphi, double *__restrict__ face)
{
    constexpr int NF = 4;
    constexpr int NB = lds_field<double>();
    constexpr int LDS_T = (NF * NB > 27 * BNT ? NF * NB : 27 * BNT);
    __shared__ double lds[LDS_T];
    const Brick br(m, threadIdx.x);
    double *Ts = lds, *dTs = lds + NB, *ls = lds + 2 * NB, *ps = lds + 3 * NB;
    const bool with_phi = (a.mode == 0) && dphi != nullptr;
    if (with_phi) {
        const double *src[4] = {T, dT, lam, (const double *)a.phi};
        double *const dst[4] = {Ts, dTs, ls, ps};
        br.stage_nodes_wg<BNT, 4>(m, threadIdx.x, src, dst, 0u);
    } else {
        const double *src[3] = {T, dT, lam};
        double *const dst[3] = {Ts, dTs, ls};
        br.stage_nodes_wg<BNT, 3>(m, threadIdx.x, src, dst, 0u);
    }
    __syncthreads();
    const int64_t cell = br.valid ? br.cell_index(m) : 0;
    const double vol = m.hx * m.hy * m.hz;
    const double ih[3] = {1.0 / (m.hx * m.hx * kR * kR), 1.0 / (m.hy * m.hy * kR * kR), 1.0 / (m.hz * m.hz * kR * kR)};
    double lq[27], Tq[27], gk[27];
    br.gather27(ls, lq);
    br.gather27(Ts, Tq);
    interp3(lq);
    interp3(Tq);
    for (int q = 0; q < 27; ++q) gk[q] = 0.0;
    grad_dot_acc<double, 0>(lq, Tq, ih[0], gk);
    grad_dot_acc<double, 1>(lq, Tq, ih[1], gk);
    grad_dot_acc<double, 2>(lq, Tq, ih[2], gk);
    pin27(gk);
    pin27(lq);
    double s[27]; // T - T_old at the Gauss points, then drc_q, then the phi-gradient weights
    br.gather27(dTs, s);
    interp3(s);
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        const double wq = vol * Q2<double>::weight(q % 3) * Q2<double>::weight((q / 3) % 3) * Q2<double>::weight(q / 9);
        const double gkq = -a.ak * wq * gk[q];
        const double grq = -a.am * wq * lq[q] * s[q];
        if (br.valid) {
            if (dk) dk[cell * 27 + q] = gkq;
            if (drc) drc[cell * 27 + q] = grq;
        }
        gk[q] = gkq;
        s[q] = grq;
        asm volatile("" : "+v"(gk[q]), "+v"(s[q])::"memory"); // one point at a time
    }
    if (!with_phi) return; // uniform over the launch
    pin27(gk);
    pin27(s);
    double ph[27];
    br.gather27(ps, ph);
    interp3(ph);
    if constexpr (HK == 0) {
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            double dH;
            (void)heaviside<double>(0, a.eps, ph[q], &dH);
            s[q] = dH * ((a.k_l - a.k_g) * gk[q] + (a.rc_l - a.rc_g) * s[q]);
            asm volatile("" : "+v"(s[q])); // one point at a time
        }
    } else {
        for (int q = 0; q < 27; ++q) { // out of line and not unrolled: one transcendental evaluation per point
            double dH;
            (void)heaviside<double>(1, a.eps, ph[q], &dH);
            s[q] = dH * ((a.k_l - a.k_g) * gk[q] + (a.rc_l - a.rc_g) * s[q]);
        }
    }
    interp3T(s);
    __syncthreads();
    br.store_cell(lds, s);
    __syncthreads();
    double *fb = face + (int64_t)br.brick * BFACE;
    br.for_owned_nodes(m, [&](int ai, int bi, int ci, int l, int64_t g, bool, int sh) {
        const double v = br.node_sum(lds, ai, bi, ci);
        if (sh) fb[br.fslot(ai, bi, ci)] = v;
        else dphi[g] = v;
    });
}

hipError_t heat_grad(const KMesh &m, const HeatArgs &a, const double *T, const double *dT, const double *lam,
                     double *dk, double *drc, double *dphi, void *face, hipStream_t s)
{
    const unsigned nb = (unsigned)n_bricks(m);
    if (dphi && !face) return hipErrorInvalidValue;
    if (a.mode == 0 && a.hkind)
        heat_grad_kernel<1><<<nb, BNT, 0, s>>>(m, a, T, dT, lam, dk, drc, dphi, (double *)face);
    else
        heat_grad_kernel<0><<<nb, BNT, 0, s>>>(m, a, T, dT, lam, dk, drc, dphi, (double *)face);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !dphi || a.mode != 0) return e;
    // the level-set gradient sums over Dirichlet nodes too (DMODE 0)
    if (nb == 1) return hipSuccess;
    face_combine_brick_kernel<double, false, 0><<<(nb + CBW - 1) / CBW, BNT * CBW, 0, s>>>(
        m, (const double *)face, nullptr, dphi, nullptr, nullptr, 0);
    return hipGetLastError();
}

} // namespace mf
