// mf_common.hpp -- shared device definitions of the gfx950 matrix-free library.
//
// Q2 Lagrange elements on uniform hexahedra with 3x3x3 Gauss quadrature
// (App. B "Numerical framework": degree-2 elements, (k+1)^dim Gauss points).
// Everything a cell needs is expressed through three 3x3 matrices acting
// along one direction at a time (sum factorization):
//   S[q][a]  = l_a(xi_q)     value of node basis a at Gauss point q
//   D[q][p]  = L_p'(xi_q)    derivative of the Lagrange polynomial through
//                            the Gauss points (collocation derivative):
//                            exact for the quadratic restriction of a Q2
//                            function to a line
//   G[q][a]  = l_a'(xi_q)    = (D S)[q][a]
// With r = sqrt(15)/10 and xi = (1/2 - r, 1/2, 1/2 + r) these are
//   S = [[.3+r, .4, .3-r], [0, 1, 0], [.3-r, .4, .3+r]]
//   D = (1/r) [[-3/2, 2, -1/2], [-1/2, 0, 1/2], [1/2, -2, 3/2]]
//   G = [[-1-4r, 8r, 1-4r], [-1, 0, 1], [-1+4r, -8r, 1+4r]]
// and the weights are (5/18, 4/9, 5/18).  The 1/r of D is folded into the
// stiffness factors (it enters squared), so the kernels use D' = r D.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mf {

constexpr double kR = 0.38729833462074168851792653997823996;  // sqrt(15)/10
constexpr double kW0 = 5.0 / 18.0, kW1 = 4.0 / 9.0;

// Device mesh description (uniform box).
struct KMesh {
    int nx, ny, nz;     // cells
    int NX, NY, NZ;     // nodes per direction (2n+1)
    unsigned dirichlet; // face bits
    double hx, hy, hz;  // cell edges
    double lox, loy, loz;
};

__device__ __forceinline__ bool node_constrained(const KMesh &m, int i, int j, int k)
{
    const unsigned f = m.dirichlet;
    return ((f & 1u) && i == 0) || ((f & 2u) && i == m.NX - 1) || ((f & 4u) && j == 0) ||
           ((f & 8u) && j == m.NY - 1) || ((f & 16u) && k == 0) || ((f & 32u) && k == m.NZ - 1);
}

__device__ __forceinline__ int64_t node_index(const KMesh &m, int i, int j, int k)
{
    return (int64_t)i + (int64_t)m.NX * ((int64_t)j + (int64_t)m.NY * k);
}

// ---------------------------------------------------------------------------
// 1D line operators on 3 values (in -> out), templated on the real type.
// ---------------------------------------------------------------------------

template <typename T> struct Q2 {
    static constexpr T s0 = T(0.3 + kR), s1 = T(0.4), s2 = T(0.3 - kR);
    static constexpr T g0 = T(-1.0 - 4.0 * kR), g1 = T(8.0 * kR), g2 = T(1.0 - 4.0 * kR);
    static constexpr T w0 = T(kW0), w1 = T(kW1);

    // values at Gauss points: out = S in
    static __device__ __forceinline__ void interp(T i0, T i1, T i2, T &o0, T &o1, T &o2)
    {
        o0 = s0 * i0 + s1 * i1 + s2 * i2;
        o1 = i1;
        o2 = s2 * i0 + s1 * i1 + s0 * i2;
    }
    // integration against node basis: out = S^T in
    static __device__ __forceinline__ void interpT(T i0, T i1, T i2, T &o0, T &o1, T &o2)
    {
        o0 = s0 * i0 + s2 * i2;
        o1 = s1 * (i0 + i2) + i1;
        o2 = s2 * i0 + s0 * i2;
    }
    // collocation derivative (scaled by r): out = D' in, in even/odd form:
    // with h = (i2 - i0) / 2 and w = 2 i1 - (i0 + i2), out = (h + w, h, h - w)
    // (6 operations instead of 8).
    static __device__ __forceinline__ void deriv(T i0, T i1, T i2, T &o0, T &o1, T &o2)
    {
        const T h = T(0.5) * (i2 - i0);
        const T w = T(2) * i1 - (i0 + i2);
        o0 = h + w;
        o1 = h;
        o2 = h - w;
    }
    // out = s D' in for a uniform scale s, in even/odd form:
    // with e = i0 + i2, h = s (i2 - i0) / 2, w = s (2 i1 - e):
    // o0 = w + h, o1 = h, o2 = h - w  (7 operations instead of 8 + 3).
    static __device__ __forceinline__ void deriv_scaled(T i0, T i1, T i2, T s, T &o0, T &o1, T &o2)
    {
        const T e = i0 + i2;
        const T h = (T(0.5) * s) * (i2 - i0);
        const T w = s * (T(2) * i1 - e);
        o0 = w + h;
        o1 = h;
        o2 = h - w;
    }
    // transposed collocation derivative accumulated: out += D'^T in
    static __device__ __forceinline__ void derivT_acc(T i0, T i1, T i2, T &o0, T &o1, T &o2)
    {
        o0 += T(-1.5) * i0 - T(0.5) * i1 + T(0.5) * i2;
        o1 += T(2) * (i0 - i2);
        o2 += T(-0.5) * i0 + T(0.5) * i1 + T(1.5) * i2;
    }
    // D'' = 2 D' = [[-3, 4, -1], [-1, 0, 1], [1, -4, 3]] (integer entries):
    // with d = i2 - i0 and w = 2 i1 - (i0 + i2), out = (d + 2w, d, d - 2w),
    // 5 operations.
    static __device__ __forceinline__ void deriv2(T i0, T i1, T i2, T &o0, T &o1, T &o2)
    {
        const T d = i2 - i0;
        const T w = T(2) * i1 - (i0 + i2);
        o0 = T(2) * w + d;
        o1 = d;
        o2 = T(-2) * w + d;
    }
    // out += D''^T in
    static __device__ __forceinline__ void deriv2T_acc(T i0, T i1, T i2, T &o0, T &o1, T &o2)
    {
        o0 += T(-3) * i0 - i1 + i2;
        o1 += T(4) * (i0 - i2);
        o2 += T(3) * i2 + (i1 - i0);
    }
    static __device__ __forceinline__ T weight(int q) { return q == 1 ? w1 : w0; }
};

// Apply a line operator along direction DIR of a 3x3x3 register array
// (index a + 3b + 9c).
template <int DIR> __device__ __forceinline__ constexpr int lidx(int l, int m, int n)
{
    // l runs along DIR; (m, n) enumerate the other two directions
    return DIR == 0 ? l + 3 * m + 9 * n : (DIR == 1 ? m + 3 * l + 9 * n : m + 3 * n + 9 * l);
}

template <typename T, int DIR, typename F>
__device__ __forceinline__ void line_apply(const T *in, T *out, F f)
{
#pragma unroll
    for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            T o0, o1, o2;
            f(in[lidx<DIR>(0, m, n)], in[lidx<DIR>(1, m, n)], in[lidx<DIR>(2, m, n)], o0, o1, o2);
            out[lidx<DIR>(0, m, n)] = o0;
            out[lidx<DIR>(1, m, n)] = o1;
            out[lidx<DIR>(2, m, n)] = o2;
        }
}

// in-place S along all three directions: nodal -> Gauss point values
template <typename T> __device__ __forceinline__ void interp3(T *v)
{
    auto f = [](T a, T b, T c, T &x, T &y, T &z) { Q2<T>::interp(a, b, c, x, y, z); };
    line_apply<T, 0>(v, v, f);
    line_apply<T, 1>(v, v, f);
    line_apply<T, 2>(v, v, f);
}

// in-place S^T along all three directions: Gauss point values -> nodal integrals
template <typename T> __device__ __forceinline__ void interp3T(T *v)
{
    auto f = [](T a, T b, T c, T &x, T &y, T &z) { Q2<T>::interpT(a, b, c, x, y, z); };
    line_apply<T, 0>(v, v, f);
    line_apply<T, 1>(v, v, f);
    line_apply<T, 2>(v, v, f);
}

template <typename T, int DIR> __device__ __forceinline__ void deriv_dir(const T *in, T *out)
{
    auto f = [](T a, T b, T c, T &x, T &y, T &z) { Q2<T>::deriv(a, b, c, x, y, z); };
    line_apply<T, DIR>(in, out, f);
}

template <typename T, int DIR> __device__ __forceinline__ void derivT_acc_dir(const T *in, T *acc)
{
#pragma unroll
    for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int m = 0; m < 3; ++m)
            Q2<T>::derivT_acc(in[lidx<DIR>(0, m, n)], in[lidx<DIR>(1, m, n)], in[lidx<DIR>(2, m, n)],
                              acc[lidx<DIR>(0, m, n)], acc[lidx<DIR>(1, m, n)], acc[lidx<DIR>(2, m, n)]);
}

// Along direction DIR, line by line: t = ih D' u, g = c .* t, acc += D'^T g.
// Working on one 3-point line at a time keeps only 3 temporaries live.
template <typename T, int DIR, typename C>
__device__ __forceinline__ void grad_line_apply(const T *u, const C &c, T ih, T *acc)
{
#pragma unroll
    for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int i0 = lidx<DIR>(0, m, n), i1 = lidx<DIR>(1, m, n), i2 = lidx<DIR>(2, m, n);
            T t0, t1, t2;
            Q2<T>::deriv_scaled(u[i0], u[i1], u[i2], ih, t0, t1, t2);
            Q2<T>::derivT_acc(c[i0] * t0, c[i1] * t1, c[i2] * t2, acc[i0], acc[i1], acc[i2]);
        }
}

// The same with D'' and no scale (the scale is in c): acc += D''^T (c .* D'' u).
template <typename T, int DIR, typename C> __device__ __forceinline__ void grad2_line_apply(const T *u, const C &c, T *acc)
{
#pragma unroll
    for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int i0 = lidx<DIR>(0, m, n), i1 = lidx<DIR>(1, m, n), i2 = lidx<DIR>(2, m, n);
            T t0, t1, t2;
            Q2<T>::deriv2(u[i0], u[i1], u[i2], t0, t1, t2);
            Q2<T>::deriv2T_acc(c[i0] * t0, c[i1] * t1, c[i2] * t2, acc[i0], acc[i1], acc[i2]);
        }
}

// out = in contracted along direction DIR with M: out[.., a, ..] = sum_q M[q][a] in[.., q, ..]
// (M a 3x3 table over Gauss points q and nodes a; the diagonals and nodal
// blocks contract Gauss-point weights with squares and products of S and G).
template <int DIR, typename T> __device__ __forceinline__ void contract1d(const T *in, T *out, const T (&M)[3][3])
{
    constexpr int st = DIR == 0 ? 1 : (DIR == 1 ? 3 : 9);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int a = (i / st) % 3, base = i - a * st;
        out[i] = M[0][a] * in[base] + M[1][a] * in[base + st] + M[2][a] * in[base + 2 * st];
    }
}

// Ordering point: all 27 values of v are computed before it and no memory
// access moves across it.  Placed at the phase boundaries of a cell's
// computation, it keeps the compiler from forming later passes early and
// merging them into one long live range.
__device__ __forceinline__ void pin27(double *v)
{
#pragma unroll
    for (int i = 0; i < 27; ++i) asm volatile("" : "+v"(v[i])::"memory");
}

// Convection along DIR, line by line, with t = D'_DIR u the collocation derivative:
// forward, acc += s rw .* w .* t; transposed, acc += D'_DIR^T (s rw .* w .* u).
// (rw: coefficient times quadrature weight, w: velocity component DIR at the
// Gauss points, s = alpha / (r h_DIR).)
template <typename T, int DIR>
__device__ __forceinline__ void conv_forward(const T *u, const T *rw, const T *w, T s, T *acc)
{
#pragma unroll
    for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int i0 = lidx<DIR>(0, m, n), i1 = lidx<DIR>(1, m, n), i2 = lidx<DIR>(2, m, n);
            T t0, t1, t2;
            Q2<T>::deriv(u[i0], u[i1], u[i2], t0, t1, t2);
            acc[i0] += s * rw[i0] * w[i0] * t0;
            acc[i1] += s * rw[i1] * w[i1] * t1;
            acc[i2] += s * rw[i2] * w[i2] * t2;
        }
}

// Velocity component DIR times the derivative along DIR, accumulated:
// cv += s w .* (D'_DIR u), line by line.
template <typename T, int DIR>
__device__ __forceinline__ void vel_grad_acc(const T *u, const T *w, T s, T *cv)
{
#pragma unroll
    for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int i0 = lidx<DIR>(0, m, n), i1 = lidx<DIR>(1, m, n), i2 = lidx<DIR>(2, m, n);
            T t0, t1, t2;
            Q2<T>::deriv(u[i0], u[i1], u[i2], t0, t1, t2);
            cv[i0] += s * w[i0] * t0;
            cv[i1] += s * w[i1] * t1;
            cv[i2] += s * w[i2] * t2;
        }
}

// Its transpose: acc += D'_DIR^T (s w .* z), line by line.
template <typename T, int DIR>
__device__ __forceinline__ void vel_gradT_acc(const T *z, const T *w, T s, T *acc)
{
#pragma unroll
    for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int i0 = lidx<DIR>(0, m, n), i1 = lidx<DIR>(1, m, n), i2 = lidx<DIR>(2, m, n);
            Q2<T>::derivT_acc(s * w[i0] * z[i0], s * w[i1] * z[i1], s * w[i2] * z[i2], acc[i0], acc[i1], acc[i2]);
        }
}

template <typename T, int DIR>
__device__ __forceinline__ void conv_transpose(const T *u, const T *rw, const T *w, T s, T *acc)
{
#pragma unroll
    for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int i0 = lidx<DIR>(0, m, n), i1 = lidx<DIR>(1, m, n), i2 = lidx<DIR>(2, m, n);
            Q2<T>::derivT_acc(s * rw[i0] * w[i0] * u[i0], s * rw[i1] * w[i1] * u[i1], s * rw[i2] * w[i2] * u[i2],
                              acc[i0], acc[i1], acc[i2]);
        }
}

// Along direction DIR: out += ih * (D' a) .* (D' b), line by line.
template <typename T, int DIR>
__device__ __forceinline__ void grad_dot_acc(const T *a, const T *b, T ih, T *out)
{
#pragma unroll
    for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int i0 = lidx<DIR>(0, m, n), i1 = lidx<DIR>(1, m, n), i2 = lidx<DIR>(2, m, n);
            T a0, a1, a2, b0, b1, b2;
            Q2<T>::deriv(a[i0], a[i1], a[i2], a0, a1, a2);
            Q2<T>::deriv(b[i0], b[i1], b[i2], b0, b1, b2);
            out[i0] += ih * a0 * b0;
            out[i1] += ih * a1 * b1;
            out[i2] += ih * a2 * b2;
        }
}

// ---------------------------------------------------------------------------
// Smoothed Heaviside (Sec. 2.3, eq. heaviside) and its derivative.
// kind 0: H = clamp((1+phi)/2, 0, 1).  kind 1: sine form with the signed
// distance d = 2 eps artanh(phi) recovered from the tanh profile.
// ---------------------------------------------------------------------------

// Linear form, branch free.
template <typename T> __device__ __forceinline__ T heaviside_linear(T phi)
{
    return fmin(fmax(T(0.5) + T(0.5) * phi, T(0)), T(1));
}

// Sine form in FP64, kept out of line: its transcendental functions would
// otherwise be replicated at every unrolled Gauss point.
__device__ __noinline__ inline double heaviside_sine(double eps, double phi, double *dH)
{
    const double lim = 1.0 - 1e-15;
    const double p = phi < -lim ? -lim : (phi > lim ? lim : phi);
    const double d = 2.0 * eps * atanh(p);
    if (d <= -3.0 * eps) { *dH = 0.0; return 0.0; }
    if (d >= 3.0 * eps) { *dH = 0.0; return 1.0; }
    const double a = M_PI * d / (3.0 * eps);
    *dH = (1.0 + cos(a)) / (6.0 * eps) * (2.0 * eps / (1.0 - p * p));
    return 0.5 + d / (6.0 * eps) + sin(a) / (2.0 * M_PI);
}

// The sine form's value alone: the same expression as heaviside_sine without
// its derivative (one transcendental fewer per point).
__device__ __noinline__ inline double heaviside_sine_value(double eps, double phi)
{
    const double lim = 1.0 - 1e-15;
    const double p = phi < -lim ? -lim : (phi > lim ? lim : phi);
    const double d = 2.0 * eps * atanh(p);
    if (d <= -3.0 * eps) return 0.0;
    if (d >= 3.0 * eps) return 1.0;
    const double a = M_PI * d / (3.0 * eps);
    return 0.5 + d / (6.0 * eps) + sin(a) / (2.0 * M_PI);
}

template <typename T> __device__ __forceinline__ T heaviside(int kind, T eps, T phi, T *dH)
{
    if (kind == 0) {
        if (dH) *dH = (phi > T(-1) && phi < T(1)) ? T(0.5) : T(0);
        return heaviside_linear<T>(phi);
    }
    if (!dH) return T(heaviside_sine_value((double)eps, (double)phi));
    double d;
    const double H = heaviside_sine((double)eps, (double)phi, &d);
    *dH = T(d);
    return T(H);
}

// ---------------------------------------------------------------------------
// Deterministic reductions without atomics.  A block sums its threads' values
// in a fixed tree order and stores one partial per set with a plain store
// (layout [NV][nblocks]).  A later launch, whose start makes those stores
// visible, sums the partials in a fixed order: every reader of a partial set
// obtains bitwise the same total, and no workgroup waits on another.
// (A last-block-arrives scheme needs one device-scope acquire-release atomic
// per workgroup on a single address; with thousands of workgroups these
// serialize across the XCDs and cost more than the kernel's own work.)
// ---------------------------------------------------------------------------

template <int NT> __device__ __forceinline__ double block_sum(double v, double *red)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Store NV block sums (valid in thread 0) as partial `block` of each set.
template <int NV>
__device__ __forceinline__ void write_partials(const double *v, double *partials, unsigned nblocks, unsigned block)
{
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) partials[(size_t)i * nblocks + block] = v[i];
    }
}

// Total of partial set i (nblocks entries written by an earlier launch),
// returned to every thread of an NT-thread block.  Thread t sums entries
// t, t + NT, ... with four interleaved accumulators (combined in a fixed
// order), then the block sums the threads in a fixed tree.
template <int NT>
__device__ __forceinline__ double sum_partials(const double *partials, unsigned nblocks, int i, double *red)
{
    const double *p = partials + (size_t)i * nblocks;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    unsigned b = threadIdx.x;
    for (; b + 3 * NT < nblocks; b += 4 * NT) {
        s0 += p[b];
        s1 += p[b + NT];
        s2 += p[b + 2 * NT];
        s3 += p[b + 3 * NT];
    }
    for (; b < nblocks; b += NT) s0 += p[b];
    return block_sum<NT>((s0 + s1) + (s2 + s3), red);
}

} // namespace mf
