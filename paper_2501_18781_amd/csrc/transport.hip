// transport.hip -- level-set transport velocity (Sec. 2.5, App. A) at every
// node of the Q2 level-set grid, in two variants:
//   1 (eq. transport_vel_local_continuous):  u_G = u + mdot(T) / rho(phi) n
//   2 (eq. transport_vel_extension_liquid):  u_G = u(x_l) + mdot(T(x_G)) / rho_l n
// with mdot = alpha_v (T - T_v) (eq. mDotTanasawa), rho by eq. rhoEff, and
//   d   = 2 eps artanh(phi)        the signed distance of the tanh profile,
//   n   = grad d / |grad d|        unit normal into the liquid (phi > 0), 0 where
//                                  |grad d| <= 1e-8 (no normal),
//   x_G = x - d n                  projection along n onto phi = 0,
//   x_l = x + (3 eps - d) n        projection onto d = 3 eps, where H = 1.
//
// grad d at a node is the gradient of the Q2 interpolant of the nodal d,
// averaged over the cells that contain the node.  Inside a cell the
// derivative along one axis at a node depends only on the three nodes of
// that cell on the axis line through it (the other directions' basis
// functions are 1 at the node and 0 at the others), so the average over up
// to 8 cells reduces to an average over the (one or two) cells along each
// axis, one 1D stencil per axis.  In reference coordinates the derivative of
// the quadratic through nodes (0, 1/2, 1) is (-3, 4, -1) at 0, (-1, 0, 1) at
// 1/2 and (1, -4, 3) at 1, divided by the cell edge h.
//
// Values of the interpolants at x_G and x_l: the point is moved to the
// nearest point of the box, located in its cell, and the 27 nodal values
// are contracted with the 1D Lagrange weights along x, y, z in turn.
#include "kernels.hpp"

namespace mf {

constexpr int TNT = 256; // threads per workgroup

__global__ void __launch_bounds__(TNT) distance_kernel(const double *__restrict__ phi, double *__restrict__ d,
                                                       double eps, int64_t n)
{
    const double lim = 1.0 - 1e-15;
    for (int64_t i = (int64_t)blockIdx.x * TNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * TNT) {
        const double p = fmin(fmax(phi[i], -lim), lim);
        d[i] = 2.0 * eps * atanh(p);
    }
}

// Averaged derivative along one axis at node index g (N nodes on the axis,
// stride s in the nodal array, cell edge h).
__device__ __forceinline__ double axis_derivative(const double *__restrict__ d, int64_t c, int g, int N, int64_t s,
                                                  double ih)
{
    if (g & 1) return (d[c + s] - d[c - s]) * ih; // cell midpoint
    double acc = 0.0;
    int cells = 0;
    if (g > 0) { // the cell below: the node is its end point
        acc += d[c - 2 * s] - 4.0 * d[c - s] + 3.0 * d[c];
        ++cells;
    }
    if (g < N - 1) { // the cell above: the node is its start point
        acc += -3.0 * d[c] + 4.0 * d[c + s] - d[c + 2 * s];
        ++cells;
    }
    return cells == 2 ? 0.5 * acc * ih : acc * ih;
}

// 1D Lagrange weights of the nodes (0, 1/2, 1) at xi.
__device__ __forceinline__ void lagrange3(double xi, double w[3])
{
    w[0] = (2.0 * xi - 1.0) * (xi - 1.0);
    w[1] = 4.0 * xi * (1.0 - xi);
    w[2] = xi * (2.0 * xi - 1.0);
}

// Cell base index and 1D weights of a physical point (moved into the box).
struct PointLoc {
    int64_t base;
    double wx[3], wy[3], wz[3];
};

__device__ __forceinline__ PointLoc locate(const KMesh &m, const double p[3], const double ih[3])
{
    const double lo[3] = {m.lox, m.loy, m.loz}, h[3] = {m.hx, m.hy, m.hz};
    const int n[3] = {m.nx, m.ny, m.nz};
    int c[3];
    double xi[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double hi = lo[k] + h[k] * n[k];
        const double q = fmin(fmax(p[k], lo[k]), hi);
        int ck = (int)floor((q - lo[k]) * ih[k]);
        ck = min(max(ck, 0), n[k] - 1);
        c[k] = ck;
        xi[k] = (q - (lo[k] + h[k] * ck)) * ih[k];
    }
    PointLoc L;
    L.base = node_index(m, 2 * c[0], 2 * c[1], 2 * c[2]);
    lagrange3(xi[0], L.wx);
    lagrange3(xi[1], L.wy);
    lagrange3(xi[2], L.wz);
    return L;
}

// Value of the Q2 interpolant of f at the located point.
__device__ __forceinline__ double point_value(const KMesh &m, const PointLoc &L, const double *__restrict__ f)
{
    const int64_t sy = m.NX, sz = (int64_t)m.NX * m.NY;
    double vz = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double vy = 0.0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double *r = f + L.base + b * sy + c * sz;
            vy += L.wy[b] * (L.wx[0] * r[0] + L.wx[1] * r[1] + L.wx[2] * r[2]);
        }
        vz += L.wz[c] * vy;
    }
    return vz;
}

// H of the sine form from the signed distance d (heaviside_sine recovers
// the same d from phi first; the distance kernel has stored it).
__device__ __forceinline__ double heaviside_sine_of_d(double eps, double d)
{
    if (d <= -3.0 * eps) return 0.0;
    if (d >= 3.0 * eps) return 1.0;
    const double a = M_PI * d / (3.0 * eps);
    return 0.5 + d / (6.0 * eps) + sin(a) / (2.0 * M_PI);
}

// One thread per node: blockIdx.y is the z plane, the plane's nodes run
// along blockIdx.x * TNT + threadIdx.x (row = j, split without an integer
// division: a single-precision estimate, corrected by one step).
template <int VARIANT, int HK>
__global__ void __launch_bounds__(TNT) transport_velocity_kernel(KMesh m, TransportArgs a,
                                                                 const double *__restrict__ phi,
                                                                 const double *__restrict__ d,
                                                                 const double *__restrict__ u,
                                                                 const double *__restrict__ T,
                                                                 double *__restrict__ ug)
{
    const int64_t nn = (int64_t)m.NX * m.NY * m.NZ;
    const unsigned NX = m.NX, NP = NX * (unsigned)m.NY;
    const unsigned pidx = blockIdx.x * TNT + threadIdx.x, k = blockIdx.y;
    if (pidx >= NP) return;
    unsigned j = (unsigned)((float)pidx * (1.0f / (float)NX));
    if (j * NX > pidx) --j;
    else if ((j + 1) * NX <= pidx) ++j;
    const int i = (int)(pidx - j * NX);
    const int64_t g = (int64_t)k * NP + pidx;
    const double ih[3] = {1.0 / m.hx, 1.0 / m.hy, 1.0 / m.hz};
    const double gx = axis_derivative(d, g, i, m.NX, 1, ih[0]);
    const double gy = axis_derivative(d, g, (int)j, m.NY, m.NX, ih[1]);
    const double gz = axis_derivative(d, g, (int)k, m.NZ, (int64_t)NP, ih[2]);
    const double gn = sqrt(gx * gx + gy * gy + gz * gz);
    // |grad d| is 1 for a signed distance; at a point of symmetry (a
    // sphere's centre) or where phi saturates it vanishes: no normal there
    const double inv = gn > 1e-8 ? 1.0 / gn : 0.0;
    const double n[3] = {gx * inv, gy * inv, gz * inv};
    double base[3], mdot, irho;
    if constexpr (VARIANT == 1) {
        const double H = HK == 1 ? heaviside_sine_of_d(a.eps, d[g]) : heaviside_linear<double>(phi[g]);
        irho = H / a.rho_l + (1.0 - H) / a.rho_g; // 1 / rho_eff
        mdot = a.alpha_v * (T[g] - a.T_boil);
#pragma unroll
        for (int c = 0; c < 3; ++c) base[c] = u[c * nn + g];
    } else {
        const double x[3] = {m.lox + i * 0.5 * m.hx, m.loy + j * 0.5 * m.hy, m.loz + k * 0.5 * m.hz};
        const double dg = d[g], dl = 3.0 * a.eps - dg;
        const double pg[3] = {x[0] - dg * n[0], x[1] - dg * n[1], x[2] - dg * n[2]};
        const double pl[3] = {x[0] + dl * n[0], x[1] + dl * n[1], x[2] + dl * n[2]};
        const PointLoc Lg = locate(m, pg, ih);
        mdot = a.alpha_v * (point_value(m, Lg, T) - a.T_boil);
        irho = 1.0 / a.rho_l;
        const PointLoc Ll = locate(m, pl, ih);
#pragma unroll
        for (int c = 0; c < 3; ++c) base[c] = point_value(m, Ll, u + c * nn);
    }
    const double s = mdot * irho;
#pragma unroll
    for (int c = 0; c < 3; ++c) ug[c * nn + g] = base[c] + s * n[c];
}

static unsigned grid_for(int64_t n)
{
    int64_t b = (n + TNT - 1) / TNT;
    if (b > 1 << 20) b = 1 << 20;
    return (unsigned)(b < 1 ? 1 : b);
}

hipError_t transport_velocity(const KMesh &m, const TransportArgs &a, const double *phi, const double *u,
                              const double *T, double *ug, double *dwork, hipStream_t s)
{
    const int64_t nn = (int64_t)m.NX * m.NY * m.NZ;
    distance_kernel<<<grid_for(nn), TNT, 0, s>>>(phi, dwork, a.eps, nn);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t np = (int64_t)m.NX * m.NY;
    // the row split's single-precision estimate is within one row for NY < 2^23
    if (np > 0xFFFFFFFFll || m.NZ > 65535 || m.NY >= (1 << 23)) return hipErrorInvalidValue;
    const dim3 g((unsigned)((np + TNT - 1) / TNT), (unsigned)m.NZ);
    const int key = a.variant * 2 + (a.hkind ? 1 : 0);
    switch (key) {
    case 2: transport_velocity_kernel<1, 0><<<g, TNT, 0, s>>>(m, a, phi, dwork, u, T, ug); break;
    case 3: transport_velocity_kernel<1, 1><<<g, TNT, 0, s>>>(m, a, phi, dwork, u, T, ug); break;
    case 5: transport_velocity_kernel<2, 1><<<g, TNT, 0, s>>>(m, a, phi, dwork, u, T, ug); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace mf
