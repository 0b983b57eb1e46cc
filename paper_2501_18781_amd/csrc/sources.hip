// sources.hip -- right-hand side of the heat equation from the interface
// fluxes on gfx950 (Sec. 2.4: regularized delta, eq. delta; its rho c_p
// scaled form, eq. deltaRhoCp; evaporative cooling, eq. vapor_heat_loss,
// with the Tanasawa mass flux, eq. mDotTanasawa; Sec. 4: the Gaussian laser
// heat flux, eq. laser_gauss):
//   b_i = sum_cells sum_q W_q N_i(x_q) s(x_q),
//   s   = [ -alpha_v (T - T_v) h_v |grad phi| + beta T_v |grad phi|
//           + peak <grad phi . e_L> exp(-2 d_L^2 / r^2) ] H'(phi) rc(phi) c_rcp
// (the second term, the right-hand side of the Tanasawa penalty of App. C,
// only on request)
// (the laser factor <-n . e_L> |grad H| with n = -grad phi/|grad phi| is
// H' <grad phi . e_L>, so no division by |grad phi| is needed).
//
// Same brick scheme as the operators (brick.hpp): phi and T staged in LDS,
// one thread per cell, values and gradients at the Gauss points by sum
// factorization, S^T integration, node sums, shared nodes through the face
// buffer; Dirichlet nodes get 0.
#include "brick.hpp"

namespace mf {

constexpr int NB = lds_field<double>(); // LDS entries of one staged nodal field

template <int HK>
__global__ void __launch_bounds__(BNT) heat_source_kernel(KMesh m, HeatArgs a, SourceArgs sa,
                                                          const double *__restrict__ T, double *__restrict__ b,
                                                          double *__restrict__ face)
{
    constexpr int LDS_T = 2 * NB > 9 * BNT ? 2 * NB : 9 * BNT; // phi and T; then the node-sum exchange
    __shared__ double lds[LDS_T];
    const Brick br(m, threadIdx.x);
    double *ps = lds, *ts = lds + NB;
    br.stage_nodes<2, double>(m, (const double *)a.phi, ps, T, ts);
    __syncthreads();

    const double h[3] = {m.hx, m.hy, m.hz};
    double ph[27], ge[27], gn[27]; // phi, grad phi . e_L, |grad phi|^2 at the Gauss points
    br.gather27(ps, ph);
    interp3(ph);
#pragma unroll
    for (int q = 0; q < 27; ++q) ge[q] = gn[q] = 0.0;
    auto grad_dir = [&](auto D) {
        constexpr int d = decltype(D)::value;
        const double sc = 1.0 / (kR * h[d]), e = sa.dir[d];
#pragma unroll
        for (int n = 0; n < 3; ++n)
#pragma unroll
            for (int mm = 0; mm < 3; ++mm) {
                const int i0 = lidx<d>(0, mm, n), i1 = lidx<d>(1, mm, n), i2 = lidx<d>(2, mm, n);
                double t0, t1, t2;
                Q2<double>::deriv_scaled(ph[i0], ph[i1], ph[i2], sc, t0, t1, t2);
                ge[i0] += e * t0;
                ge[i1] += e * t1;
                ge[i2] += e * t2;
                gn[i0] += t0 * t0;
                gn[i1] += t1 * t1;
                gn[i2] += t2 * t2;
            }
    };
    grad_dir(std::integral_constant<int, 0>{});
    grad_dir(std::integral_constant<int, 1>{});
    grad_dir(std::integral_constant<int, 2>{});
    // Pointwise, phi's last use: the laser term times delta_rcp in place of
    // grad phi . e_L, and delta_rcp = |grad phi| H' rc c_rcp in place of
    // |grad phi|^2, so that phi is dead before the temperature is gathered
    // (three 27-vectors live at a time).
    const bool evap = sa.terms & 1, laser = sa.terms & 2, pen = sa.terms & 4;
    const double xc[3] = {m.lox + m.hx * (br.c0x + br.tx), m.loy + m.hy * (br.c0y + br.ty),
                          m.loz + m.hz * (br.c0z + br.tz)};
    const double xi[3] = {0.5 - kR, 0.5, 0.5 + kR};
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        const int qi[3] = {q % 3, (q / 3) % 3, q / 9};
        double dH;
        const double H = heaviside<double>(HK, a.eps, ph[q], &dH);
        const double drc = dH * (a.rc_g + H * (a.rc_l - a.rc_g)) * sa.c_rcp; // delta_rcp / |grad phi|
        double lq = 0.0;
        if (laser && ge[q] > 0.0) {
            double r[3], t = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                r[d] = xc[d] + h[d] * xi[qi[d]] - sa.focus[d];
                t += r[d] * sa.dir[d];
            }
            double d2 = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double p = r[d] - t * sa.dir[d];
                d2 += p * p;
            }
            lq = sa.peak * ge[q] * exp(-2.0 * d2 * sa.inv_r2) * drc;
        }
        ge[q] = lq;
        gn[q] = sqrt(gn[q]) * drc; // delta_rcp
        // one point at a time: interleaving the 27 exponentials would take
        // more registers than the three live vectors
        asm volatile("" : "+v"(ge[q]), "+v"(gn[q]));
    }
    pin27(ge);
    pin27(gn);
    // evaporative part, -alpha_v (T - T_v) h_v delta_rcp, and the penalty
    // right-hand side, beta T_v delta_rcp; the weighted source in place of T
    const double vol = m.hx * m.hy * m.hz;
    double *sq = ph;
    br.gather27(ts, sq);
    interp3(sq);
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        const double f = (evap ? -sa.alpha_v * (sq[q] - sa.T_boil) * sa.h_v : 0.0) + (pen ? sa.penalty * sa.T_boil : 0.0);
        const double w = Q2<double>::weight(q % 3) * Q2<double>::weight((q / 3) % 3) * Q2<double>::weight(q / 9);
        sq[q] = vol * w * (f * gn[q] + ge[q]);
    }
    interp3T(ph);

    __syncthreads(); // staging no longer read
    br.assemble27(ph, lds);
    double *fb = face + (int64_t)br.brick * BFACE;
    br.for_owned_nodes(m, [&](int ai, int bi, int ci, int l, int64_t g, bool constrained, int sh) {
        const double v = ph[ai + 3 * bi + 9 * ci];
        if (sh) fb[br.fslot(ai, bi, ci)] = v; // constrained ones: 0 in the combine
        else b[g] = constrained ? 0.0 : v;
    });
}

// Shared nodes, brick by brick (combine_brick); Dirichlet ones get 0.
__global__ void __launch_bounds__(BNT * CBW) source_combine_kernel(KMesh m, const double *__restrict__ face,
                                                                   double *__restrict__ b)
{
    combine_brick<double, 3>(m, face, nullptr, b);
}

hipError_t heat_sources(const KMesh &m, const HeatArgs &a, const SourceArgs &sa, const double *T, double *b,
                        void *face, hipStream_t s)
{
    const unsigned nb = (unsigned)n_bricks(m);
    if (!face || !T || !b || a.mode == 1) return hipErrorInvalidValue;
    if (a.hkind == 1) heat_source_kernel<1><<<nb, BNT, 0, s>>>(m, a, sa, T, b, (double *)face);
    else heat_source_kernel<0><<<nb, BNT, 0, s>>>(m, a, sa, T, b, (double *)face);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nb == 1) return hipSuccess; // a single brick shares nothing
    source_combine_kernel<<<(nb + CBW - 1) / CBW, BNT * CBW, 0, s>>>(m, (const double *)face, b);
    return hipGetLastError();
}

} // namespace mf
