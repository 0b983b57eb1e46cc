// vec.hip -- vector kernels and the fused Krylov steps (App. B: CG and GMRES).
//
// Reductions are deterministic and use no atomics: every thread accumulates
// a fixed grid-stride subsequence, wavefronts reduce with shuffles in a fixed
// order, the waves of a block through LDS, and each block stores its partial;
// the next launch sums the partials in a fixed order (a single-workgroup
// finalize kernel, or every workgroup of the consuming kernel when the
// partials are few).  Solver scalars (alpha, beta, residual norms, iteration
// count, convergence flag) live in device memory; kernels read them directly
// and become no-ops once the solve is done, so the host only synchronizes to
// poll convergence.
#include <algorithm>
#include <atomic>
#include <cstdint>

#include "kernels.hpp"

namespace mf {

constexpr int VNT = 256;   // threads per block of the vector kernels
constexpr int VMAXB = 1024; // max blocks of a reduction kernel
constexpr int MAXV = 32;   // max vectors in a multi-dot
constexpr int FNT = 1024;  // threads of the single-workgroup finalize kernels
constexpr unsigned CG_RESID_BLOCKS = 512; // partials the CG step kernels reduce in every workgroup
constexpr int64_t CG_STEP_BLOCKS = 1024;

static unsigned vec_blocks(int64_t n)
{
    int64_t b = (n + VNT * 4 - 1) / (VNT * 4);
    if (b < 1) b = 1;
    if (b > VMAXB) b = VMAXB;
    return (unsigned)b;
}

static unsigned ew_blocks(int64_t n)
{
    int64_t b = (n + VNT - 1) / VNT;
    if (b > 65535 * 16) b = 65535 * 16;
    if (b < 1) b = 1;
    return (unsigned)b;
}

#define GRID_STRIDE(i, n) for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v; // valid in lane 0
}

// Sum NV per-thread values over the block; results valid in thread 0 (out[]).
// One lane's share of a set of nb partials: entries lane, lane + 64, ...,
// in four interleaved sums so that four loads are in flight at a time.
__device__ __forceinline__ double lane_partial_sum(const double *p, unsigned nb, int lane)
{
    double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
    unsigned b = lane;
    for (; b + 192 < nb; b += 256) {
        v0 += p[b];
        v1 += p[b + 64];
        v2 += p[b + 128];
        v3 += p[b + 192];
    }
    for (; b < nb; b += 64) v0 += p[b];
    return (v0 + v1) + (v2 + v3);
}

template <int NV> __device__ __forceinline__ void block_sum_n(double *v, double *lds /*[NV][VNT/64]*/)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == 0) lds[k * (VNT / 64) + wid] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < VNT / 64; ++w) s += lds[k * (VNT / 64) + w];
            v[k] = s;
        }
    }
    __syncthreads();
}

// Block sums of NV values, stored as this block's partials.
template <int NV> __device__ __forceinline__ void grid_partials(double *v, const RedWS &red, double *lds)
{
    block_sum_n<NV>(v, lds);
    write_partials<NV>(v, red.partials, gridDim.x, blockIdx.x);
}

// Totals of NV <= blockDim/64 partial sets of nb entries: wavefront k sums
// set k (lane-strided, then shuffles) and publishes it in out_lds[k].
template <int NV>
__device__ __forceinline__ void wave_set_sums(const double *partials, unsigned nb, double *out_lds)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (w < NV) {
        const double s = wave_sum(lane_partial_sum(partials + (size_t)w * nb, nb, lane));
        if (lane == 0) out_lds[w] = s;
    }
    __syncthreads();
}

// out[k] = total of partial set k, k < nv.
__global__ void __launch_bounds__(FNT) sum_finalize_kernel(const double *__restrict__ partials, unsigned nb, int nv,
                                                           double *__restrict__ out)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = w; k < nv; k += FNT / 64) {
        const double s = wave_sum(lane_partial_sum(partials + (size_t)k * nb, nb, lane));
        if (lane == 0) out[k] = s;
    }
}

static hipError_t sum_finalize(const RedWS &red, unsigned nb, int nv, double *out, hipStream_t s)
{
    sum_finalize_kernel<<<1, FNT, 0, s>>>(red.partials, nb, nv, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Elementwise kernels
// ---------------------------------------------------------------------------
template <typename T> __global__ void fill_kernel(T *y, T v, int64_t n)
{
    GRID_STRIDE(i, n) y[i] = v;
}

hipError_t vfill(void *y, double v, int64_t n, int fp32, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (fp32) fill_kernel<float><<<ew_blocks(n), VNT, 0, s>>>((float *)y, (float)v, n);
    else fill_kernel<double><<<ew_blocks(n), VNT, 0, s>>>((double *)y, v, n);
    return hipGetLastError();
}

__global__ void copy_kernel(const double *x, double *y, int64_t n) { GRID_STRIDE(i, n) y[i] = x[i]; }
hipError_t vcopy(const double *x, double *y, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    copy_kernel<<<ew_blocks(n), VNT, 0, s>>>(x, y, n);
    return hipGetLastError();
}

__global__ void axpby_kernel(double a, const double *x, double b, double *y, int64_t n)
{
    GRID_STRIDE(i, n) y[i] = a * x[i] + b * y[i];
}
hipError_t vaxpby(double a, const double *x, double b, double *y, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    axpby_kernel<<<ew_blocks(n), VNT, 0, s>>>(a, x, b, y, n);
    return hipGetLastError();
}

__global__ void scale_copy_kernel(const double *sc, int invert, const double *x, double *y, int64_t n)
{
    const double f = invert ? 1.0 / sc[0] : sc[0];
    GRID_STRIDE(i, n) y[i] = x[i] * f;
}
hipError_t vscale_copy(const double *sc, int invert, const double *x, double *y, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    scale_copy_kernel<<<ew_blocks(n), VNT, 0, s>>>(sc, invert, x, y, n);
    return hipGetLastError();
}

template <typename T> __global__ void mul_kernel(const T *d, const T *x, T *y, int64_t n)
{
    GRID_STRIDE(i, n) y[i] = d[i] * x[i];
}
template <typename T> __global__ void inv_kernel(T *d, int64_t n) { GRID_STRIDE(i, n) d[i] = T(1) / d[i]; }

hipError_t vmul(const double *d, const double *x, double *y, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    mul_kernel<double><<<ew_blocks(n), VNT, 0, s>>>(d, x, y, n);
    return hipGetLastError();
}
hipError_t vmulf(const float *d, const float *x, float *y, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    mul_kernel<float><<<ew_blocks(n), VNT, 0, s>>>(d, x, y, n);
    return hipGetLastError();
}
hipError_t vinv(double *d, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    inv_kernel<double><<<ew_blocks(n), VNT, 0, s>>>(d, n);
    return hipGetLastError();
}

__global__ void d2f_kernel(const double *x, float *y, int64_t n) { GRID_STRIDE(i, n) y[i] = (float)x[i]; }
__global__ void f2d_kernel(const float *x, double *y, int64_t n) { GRID_STRIDE(i, n) y[i] = (double)x[i]; }
hipError_t vcvt_d2f(const double *x, float *y, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    d2f_kernel<<<ew_blocks(n), VNT, 0, s>>>(x, y, n);
    return hipGetLastError();
}
hipError_t vcvt_f2d(const float *x, double *y, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    f2d_kernel<<<ew_blocks(n), VNT, 0, s>>>(x, y, n);
    return hipGetLastError();
}

// z = a x + b y out of place (z may alias x or y).
__global__ void axpbyz_kernel(double a, const double *x, double b, const double *y, double *z, int64_t n)
{
    GRID_STRIDE(i, n) z[i] = a * x[i] + b * y[i];
}
hipError_t vaxpbyz(double a, const double *x, double b, const double *y, double *z, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    axpbyz_kernel<<<ew_blocks(n), VNT, 0, s>>>(a, x, b, y, z, n);
    return hipGetLastError();
}

// z = a x + b y on the free dofs and 0 on the Dirichlet dofs of the mesh; a
// null x or y reads as zero.  The grid runs over the comps * NY * NZ node
// rows (y, z and the component from the workgroup index), x across threads,
// so the Dirichlet test needs no division.
__global__ void mask_axpby_kernel(KMesh m, double a, const double *__restrict__ x, double b,
                                  const double *__restrict__ y, double *__restrict__ z)
{
    const int row = blockIdx.y, k = blockIdx.z % m.NZ;
    const int64_t base = (int64_t)m.NX * m.NY * m.NZ * (blockIdx.z / m.NZ) + (int64_t)m.NX * (row + (int64_t)m.NY * k);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m.NX; i += gridDim.x * blockDim.x) {
        const int64_t g = base + i;
        double v = 0.0;
        if (!node_constrained(m, i, row, k)) v = (x ? a * x[g] : 0.0) + (y ? b * y[g] : 0.0);
        z[g] = v;
    }
}
hipError_t vmask_axpby(const KMesh &m, int comps, double a, const double *x, double b, const double *y, double *z,
                       hipStream_t s)
{
    const unsigned bx = (unsigned)((m.NX + VNT - 1) / VNT);
    mask_axpby_kernel<<<dim3(bx, m.NY, m.NZ * comps), VNT, 0, s>>>(m, a, x, b, y, z);
    return hipGetLastError();
}

// Picard update: T = T_old + dT, with the partials of ||T_new - T||^2 and
// ||T_new||^2 (T holds the previous iterate on entry); out[0], out[1] are
// their totals (device).
__global__ void __launch_bounds__(VNT) picard_update_kernel(const double *__restrict__ T_old,
                                                            const double *__restrict__ dT, double *__restrict__ T,
                                                            int64_t n, RedWS red)
{
    __shared__ double lds[2 * (VNT / 64)];
    double acc[2] = {0.0, 0.0};
    GRID_STRIDE(i, n)
    {
        const double tn = T_old[i] + dT[i];
        const double d = tn - T[i];
        T[i] = tn;
        acc[0] += d * d;
        acc[1] += tn * tn;
    }
    grid_partials<2>(acc, red, lds);
}
hipError_t picard_update(const double *T_old, const double *dT, double *T, int64_t n, double *out, const RedWS *red,
                         hipStream_t s)
{
    const unsigned nb = vec_blocks(n);
    if (red->capacity < 2 * nb) return hipErrorInvalidValue;
    picard_update_kernel<<<nb, VNT, 0, s>>>(T_old, dT, T, n, *red);
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : sum_finalize(*red, nb, 2, out, s);
}

// ---------------------------------------------------------------------------
// Multi-dot and combination of basis vectors.  The number of vectors NV is
// a template parameter (1..32, chosen by a switch), so that every loop over
// the vectors is unrolled without conditions and all NV loads of an element
// are in flight together.
// ---------------------------------------------------------------------------

#define MF_NV_CASES(X)                                                                                      \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) \
        X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)

// Block partials of NV sums: set k of the partials holds block b at k * gridDim.x + b.
template <int NV> __device__ __forceinline__ void store_block_partials(double *acc, double *lds, const RedWS &red)
{
    block_sum_n<NV>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red.partials[(size_t)k * gridDim.x + blockIdx.x] = acc[k];
    }
}

// out_k = V_k . w
template <int NV>
__global__ void __launch_bounds__(VNT) multidot_kernel(const double *__restrict__ V, int64_t ld,
                                                       const double *__restrict__ w, int64_t n, RedWS red)
{
    __shared__ double lds[NV * (VNT / 64)];
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    GRID_STRIDE(i, n)
    {
        const double wi = w[i];
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] += V[(int64_t)k * ld + i] * wi;
    }
    store_block_partials<NV>(acc, lds, red);
}

hipError_t vmultidot(const double *V, int64_t ld, int nv, const double *w, int64_t n, double *out, const RedWS *red,
                     hipStream_t s)
{
    if (nv < 1 || nv > MAXV) return hipErrorInvalidValue;
    const unsigned nb = vec_blocks(n);
    if (red->capacity < nb * MAXV) return hipErrorInvalidValue;
    switch (nv) {
#define MF_CASE(N)                                                                                            \
    case N: multidot_kernel<N><<<nb, VNT, 0, s>>>(V, ld, w, n, *red); break;
        MF_NV_CASES(MF_CASE)
#undef MF_CASE
    }
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : sum_finalize(*red, nb, nv, out, s);
}

// Partials of ||b - t||^2 (the true residual of a solve, without storing it).
__global__ void __launch_bounds__(VNT) diffnorm2_kernel(const double *__restrict__ b, const double *__restrict__ t,
                                                        int64_t n, RedWS red)
{
    __shared__ double lds[VNT / 64];
    double acc = 0.0;
    GRID_STRIDE(i, n)
    {
        const double d = b[i] - t[i];
        acc += d * d;
    }
    grid_partials<1>(&acc, red, lds);
}

hipError_t vdiffnorm2(const double *b, const double *t, int64_t n, double *out, const RedWS *red, hipStream_t s)
{
    const unsigned nb = vec_blocks(n);
    if (red->capacity < nb) return hipErrorInvalidValue;
    diffnorm2_kernel<<<nb, VNT, 0, s>>>(b, t, n, *red);
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : sum_finalize(*red, nb, 1, out, s);
}

// y = V h
template <int NV>
__global__ void combine_kernel(const double *__restrict__ V, int64_t ld, const double *__restrict__ h,
                               double *__restrict__ y, int64_t n)
{
    __shared__ double hs[NV];
    if (threadIdx.x < NV) hs[threadIdx.x] = h[threadIdx.x];
    __syncthreads();
    GRID_STRIDE(i, n)
    {
        double vk[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) vk[k] = V[(int64_t)k * ld + i];
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < NV; ++k) v += vk[k] * hs[k];
        y[i] = v;
    }
}

hipError_t vcombine(const double *V, int64_t ld, int nv, const double *h, double *y, int64_t n, hipStream_t s)
{
    if (nv < 1 || nv > MAXV) return hipErrorInvalidValue;
    const unsigned g = ew_blocks(n);
    switch (nv) {
#define MF_CASE(N)                                                                                            \
    case N: combine_kernel<N><<<g, VNT, 0, s>>>(V, ld, h, y, n); break;
        MF_NV_CASES(MF_CASE)
#undef MF_CASE
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Arnoldi with delayed re-orthogonalization (classical Gram-Schmidt applied
// twice, the second pass of a vector taken one step later; the low-synchro-
// nization form of Swirydowicz, Langou, Ananthan, Yang and Thomas, 2020).
// Step j of a cycle starts from the final q_0 .. q_{j-1} and u_j, the j-th
// candidate orthogonalized once, and from w = A M^-1 u_j.  One pass over the
// basis forms a = Q^T u_j, b = Q^T w, u_j.u_j and u_j.w.  Then
//   s = a, nu = sqrt(u_j.u_j - s.s), q_j = (u_j - Q s) / nu
// completes column j-1 of the Hessenberg matrix (the first projection of
// the previous step plus s, and nu).  Since A M^-1 Q = Q_j H (Arnoldi), the
// product with q_j is (w - Q_j H s) / nu: with t = H s its first projection
// is h = ((Q^T w, q_j.w) - t) / nu, where q_j.w = (u_j.w - s.b) / nu, and
//   u_{j+1} = w / nu - Q_j (t / nu + h)
// is the next candidate.  A second pass over the basis writes q_j and
// u_{j+1}: two passes per step instead of three, and the normalization is
// part of the second.  The device keeps the (unrotated) Hessenberg matrix.
// ---------------------------------------------------------------------------
#define MF_NV0_CASES(X)                                                                                     \
    X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) \
        X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31)

// partial sets: 0..NV-1 q_k.u, NV..2NV-1 q_k.w, 2NV u.u, 2NV+1 u.w
template <int NV>
__global__ void __launch_bounds__(VNT) dgs_dot_kernel(const double *__restrict__ V, int64_t ld,
                                                      const double *__restrict__ u, const double *__restrict__ w,
                                                      int64_t n, RedWS red)
{
    constexpr int NS = 2 * NV + 2;
    __shared__ double lds[NS * (VNT / 64)];
    double acc[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] = 0.0;
    GRID_STRIDE(i, n)
    {
        const double ui = u[i], wi = w[i];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const double v = V[(int64_t)k * ld + i];
            acc[k] += v * ui;
            acc[NV + k] += v * wi;
        }
        acc[2 * NV] += ui * ui;
        acc[2 * NV + 1] += ui * wi;
    }
    store_block_partials<NS>(acc, lds, red);
}

// The same over element pairs (2i, 2i + 1) with 16-byte loads; V, u and w
// 16-byte aligned and ld even.  The last element of an odd n goes to thread
// 0 of block 0.
template <int NV>
__global__ void __launch_bounds__(VNT) dgs_dot_pair_kernel(const double *__restrict__ V, int64_t ld,
                                                           const double *__restrict__ u,
                                                           const double *__restrict__ w, int64_t n, RedWS red)
{
    constexpr int NS = 2 * NV + 2;
    __shared__ double lds[NS * (VNT / 64)];
    double acc[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] = 0.0;
    GRID_STRIDE(i, n / 2)
    {
        const double2 ui = ((const double2 *)u)[i], wi = ((const double2 *)w)[i];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const double2 v = ((const double2 *)(V + (int64_t)k * ld))[i];
            acc[k] += v.x * ui.x + v.y * ui.y;
            acc[NV + k] += v.x * wi.x + v.y * wi.y;
        }
        acc[2 * NV] += ui.x * ui.x + ui.y * ui.y;
        acc[2 * NV + 1] += ui.x * wi.x + ui.y * wi.y;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const double ui = u[n - 1], wi = w[n - 1];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const double v = V[(int64_t)k * ld + n - 1];
            acc[k] += v * ui;
            acc[NV + k] += v * wi;
        }
        acc[2 * NV] += ui * ui;
        acc[2 * NV + 1] += ui * wi;
    }
    store_block_partials<NS>(acc, lds, red);
}

// One workgroup: totals of the dot pass, then the scalars of step j.
// H: unrotated Hessenberg matrix, row i at i * DGS_LDH; column j-1 holds the
// first projection of the previous step until this kernel completes it.
// coef: s at 0..j-1, 1 / nu at DGS_INV, t / nu + h at DGS_C + 0..j.
// col: the completed column j-1 (rows 0..j), for the host.
__global__ void __launch_bounds__(FNT) dgs_scalars_kernel(const double *__restrict__ partials, unsigned nb, int j,
                                                          int full, double *__restrict__ H,
                                                          double *__restrict__ coef, double *__restrict__ col)
{
    __shared__ double sums[2 * DGS_MAXJ + 2];
    __shared__ double cprev[DGS_MAXJ + 1];
    __shared__ double sh[3];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, t = threadIdx.x;
    const int ns = 2 * j + 2;
    for (int k = wv; k < ns; k += FNT / 64) {
        const double v = wave_sum(lane_partial_sum(partials + (size_t)k * nb, nb, lane));
        if (lane == 0) sums[k] = v;
    }
    __syncthreads();
    if (wv == 0) {
        double ss = 0.0, sb = 0.0;
        if (lane < j) {
            ss = sums[lane] * sums[lane];
            sb = sums[lane] * sums[j + lane];
        }
        ss = wave_sum(ss);
        sb = wave_sum(sb);
        if (lane == 0) {
            // q_0 is r / ||r||: it is final as it stands
            const double nu = j == 0 ? 1.0 : sqrt(fmax(sums[2 * j] - ss, 0.0));
            sh[0] = nu;
            sh[1] = 1.0 / nu;
            sh[2] = sb;
        }
    }
    __syncthreads();
    const double inv = sh[1];
    if (j > 0 && t <= j) {
        const double v = t < j ? H[t * DGS_LDH + (j - 1)] + sums[t] : sh[0];
        cprev[t] = v;
        H[t * DGS_LDH + (j - 1)] = v;
        col[t] = v;
    }
    __syncthreads();
    if (full && t <= j) {
        // t_i = (H s)_i over the completed columns 0 .. j-1 (zero below the subdiagonal)
        double tt = 0.0;
        for (int k = 0; k + 1 < j; ++k) tt += H[t * DGS_LDH + k] * sums[k];
        if (j > 0) tt += cprev[t] * sums[j - 1];
        const double qw = t < j ? sums[j + t] : (sums[2 * j + 1] - sh[2]) * inv;
        const double h = (qw - tt) * inv;
        H[t * DGS_LDH + j] = h;
        coef[DGS_C + t] = tt * inv + h;
        if (t < j) coef[t] = sums[t];
    }
    if (t == 0) coef[DGS_INV] = inv;
}

// q_j = (u - Q s) / nu into u, u_{j+1} = w / nu - Q c - q_j c_j into w
template <int NV>
__global__ void __launch_bounds__(VNT) dgs_update_kernel(const double *__restrict__ V, int64_t ld,
                                                         double *__restrict__ u, double *__restrict__ w, int64_t n,
                                                         const double *__restrict__ coef)
{
    __shared__ double cs[2 * NV + 2];
    if (threadIdx.x < NV) cs[threadIdx.x] = coef[threadIdx.x];
    if (threadIdx.x <= NV) cs[NV + threadIdx.x] = coef[DGS_C + threadIdx.x];
    if (threadIdx.x == 0) cs[2 * NV + 1] = coef[DGS_INV];
    __syncthreads();
    const double inv = cs[2 * NV + 1];
    GRID_STRIDE(i, n)
    {
        double vk[NV > 0 ? NV : 1];
#pragma unroll
        for (int k = 0; k < NV; ++k) vk[k] = V[(int64_t)k * ld + i];
        double q = u[i], y = w[i] * inv;
#pragma unroll
        for (int k = 0; k < NV; ++k) q -= vk[k] * cs[k];
        q *= inv;
#pragma unroll
        for (int k = 0; k < NV; ++k) y -= vk[k] * cs[NV + k];
        y -= q * cs[2 * NV];
        u[i] = q;
        w[i] = y;
    }
}

// the same over element pairs (see dgs_dot_pair_kernel)
template <int NV>
__global__ void __launch_bounds__(VNT) dgs_update_pair_kernel(const double *__restrict__ V, int64_t ld,
                                                              double *__restrict__ u, double *__restrict__ w,
                                                              int64_t n, const double *__restrict__ coef)
{
    __shared__ double cs[2 * NV + 2];
    if (threadIdx.x < NV) cs[threadIdx.x] = coef[threadIdx.x];
    if (threadIdx.x <= NV) cs[NV + threadIdx.x] = coef[DGS_C + threadIdx.x];
    if (threadIdx.x == 0) cs[2 * NV + 1] = coef[DGS_INV];
    __syncthreads();
    const double inv = cs[2 * NV + 1];
    GRID_STRIDE(i, n / 2)
    {
        double2 vk[NV > 0 ? NV : 1];
#pragma unroll
        for (int k = 0; k < NV; ++k) vk[k] = ((const double2 *)(V + (int64_t)k * ld))[i];
        double2 q = ((const double2 *)u)[i], y = ((const double2 *)w)[i];
        y.x *= inv;
        y.y *= inv;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            q.x -= vk[k].x * cs[k];
            q.y -= vk[k].y * cs[k];
        }
        q.x *= inv;
        q.y *= inv;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            y.x -= vk[k].x * cs[NV + k];
            y.y -= vk[k].y * cs[NV + k];
        }
        y.x -= q.x * cs[2 * NV];
        y.y -= q.y * cs[2 * NV];
        ((double2 *)u)[i] = q;
        ((double2 *)w)[i] = y;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t i = n - 1;
        double q = u[i], y = w[i] * inv;
#pragma unroll
        for (int k = 0; k < NV; ++k) q -= V[(int64_t)k * ld + i] * cs[k];
        q *= inv;
#pragma unroll
        for (int k = 0; k < NV; ++k) y -= V[(int64_t)k * ld + i] * cs[NV + k];
        y -= q * cs[2 * NV];
        u[i] = q;
        w[i] = y;
    }
}

constexpr int DGS_PAIR_MIN = 10; // basis widths from which the passes take element pairs

// Workgroups of VNT threads of `kernel` that the device holds at once (its
// occupancy times the compute units), cached by the caller per kernel.  The
// wide passes use 60-170 VGPRs: a grid of exactly one resident round avoids
// a second, partly filled round that runs alone.
static int compute_units()
{
    static std::atomic<int> cus{0};
    int v = cus.load(std::memory_order_relaxed);
    if (v <= 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        cus.store(v, std::memory_order_relaxed);
    }
    return v;
}

template <typename K> static unsigned resident_blocks(K kernel, std::atomic<int> *cache)
{
    int b = cache->load(std::memory_order_relaxed);
    if (b <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, VNT, 0) != hipSuccess || b < 1) b = 1;
        cache->store(b, std::memory_order_relaxed);
    }
    return (unsigned)(b * compute_units());
}


hipError_t dgs_step(const double *V, int64_t ld, int j, bool full, double *u, double *w, int64_t n, double *H,
                    double *coef, double *col, const RedWS *red, hipStream_t s)
{
    if (j < 0 || j > DGS_MAXJ || (full && j >= DGS_MAXJ)) return hipErrorInvalidValue;
    const int ns = 2 * j + 2;
    unsigned nb = vec_blocks(n);
    if (nb * (unsigned)ns > red->capacity) nb = (unsigned)(red->capacity / (unsigned)ns);
    if (nb < 1) return hipErrorInvalidValue;
    const double *wd = full ? w : u; // a closing step has no new product
    const bool pair = j >= DGS_PAIR_MIN && (ld & 1) == 0 && ((uintptr_t)V & 15) == 0 && ((uintptr_t)u & 15) == 0 &&
                      ((uintptr_t)w & 15) == 0;
    static std::atomic<int> occ[4][DGS_MAXJ + 1]; // resident workgroups per CU: dot, dot pairs, update, update pairs
    switch (j) {
#define MF_CASE(N)                                                                                            \
    case N:                                                                                                   \
        if (pair) nb = std::min(nb, resident_blocks(dgs_dot_pair_kernel<N>, &occ[1][N]));                      \
        else nb = std::min(nb, resident_blocks(dgs_dot_kernel<N>, &occ[0][N]));                                \
        if (pair) dgs_dot_pair_kernel<N><<<nb, VNT, 0, s>>>(V, ld, u, wd, n, *red);                           \
        else dgs_dot_kernel<N><<<nb, VNT, 0, s>>>(V, ld, u, wd, n, *red);                                     \
        break;
        MF_NV0_CASES(MF_CASE)
#undef MF_CASE
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dgs_scalars_kernel<<<1, FNT, 0, s>>>(red->partials, nb, j, full ? 1 : 0, H, coef, col);
    e = hipGetLastError();
    if (e != hipSuccess || !full) return e;
    const unsigned g = ew_blocks(n) < VMAXB ? ew_blocks(n) : VMAXB;
    switch (j) {
#define MF_CASE(N)                                                                                            \
    case N:                                                                                                   \
        if (pair)                                                                                             \
            dgs_update_pair_kernel<N><<<std::min(g, resident_blocks(dgs_update_pair_kernel<N>, &occ[3][N])), VNT, \
                                        0, s>>>(V, ld, u, w, n, coef);                                        \
        else                                                                                                  \
            dgs_update_kernel<N><<<std::min(g, resident_blocks(dgs_update_kernel<N>, &occ[2][N])), VNT, 0, s>>>( \
                V, ld, u, w, n, coef);                                                                        \
        break;
        MF_NV0_CASES(MF_CASE)
#undef MF_CASE
    }
    return hipGetLastError();
}

#undef MF_NV0_CASES
#undef MF_NV_CASES

// ---------------------------------------------------------------------------
// 3x3 nodal blocks ([node][3][3], row-major): inversion by cofactors and
// application to component-major vectors.
// ---------------------------------------------------------------------------
__global__ void block3_invert_kernel(double *B, int64_t nn)
{
    GRID_STRIDE(i, nn)
    {
        double *a = B + 9 * i;
        const double c00 = a[4] * a[8] - a[5] * a[7], c01 = a[5] * a[6] - a[3] * a[8], c02 = a[3] * a[7] - a[4] * a[6];
        const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
        const double id = 1.0 / det;
        const double r[9] = {c00 * id, (a[2] * a[7] - a[1] * a[8]) * id, (a[1] * a[5] - a[2] * a[4]) * id,
                             c01 * id, (a[0] * a[8] - a[2] * a[6]) * id, (a[2] * a[3] - a[0] * a[5]) * id,
                             c02 * id, (a[1] * a[6] - a[0] * a[7]) * id, (a[0] * a[4] - a[1] * a[3]) * id};
        for (int k = 0; k < 9; ++k) a[k] = r[k];
    }
}
hipError_t block3_invert(double *B, int64_t nn, hipStream_t s)
{
    block3_invert_kernel<<<ew_blocks(nn), VNT, 0, s>>>(B, nn);
    return hipGetLastError();
}

__global__ void block3_apply_kernel(const double *__restrict__ B, const double *__restrict__ x, double *__restrict__ y,
                                    int64_t nn)
{
    GRID_STRIDE(i, nn)
    {
        const double *a = B + 9 * i;
        const double x0 = x[i], x1 = x[nn + i], x2 = x[2 * nn + i];
        y[i] = a[0] * x0 + a[1] * x1 + a[2] * x2;
        y[nn + i] = a[3] * x0 + a[4] * x1 + a[5] * x2;
        y[2 * nn + i] = a[6] * x0 + a[7] * x1 + a[8] * x2;
    }
}
hipError_t block3_apply(const double *B, const double *x, double *y, int64_t nn, hipStream_t s)
{
    block3_apply_kernel<<<ew_blocks(nn), VNT, 0, s>>>(B, x, y, nn);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CG (preconditioned with a diagonal, Saad Alg. 9.1).  With the diagonal
// preconditioner the solver keeps z = D^-1 r in place of r (r = z / D^-1
// where a dot product needs it), so that the direction update needs no
// D^-1.  One iteration is
//   apply   q = A p, per-brick partials of p.q     (heat.hip, CG mode)
//   alpha   alpha = rz / p.q                        (one workgroup)
//   resid   z -= alpha D^-1 q; partials of r.z and r.r; iteration count,
//           rz_old = rz                              (reads z, q, D^-1; writes z)
//   step    every workgroup sums the residual partials in the same order:
//           beta = rz / rz_old and the convergence test; then
//           x += alpha p and (unless converged) p = z + beta p
//                                                    (reads x, p, z; writes x, p)
// Nine vector passes per iteration (without a preconditioner z = r).
// Each thread keeps CG_UNROLL elements of its grid-stride sequence in flight.
//
// The done flag: a kernel that reads it at entry must not write it (another
// workgroup of the same launch could start after the write).  The step
// kernel writes it, so it tests `run` instead, which the residual kernel
// (an earlier launch, that only reads done) sets to whether it ran.
// ---------------------------------------------------------------------------
constexpr int CG_UNROLL = 4;

__global__ void __launch_bounds__(VNT) cg_init_kernel(const double *__restrict__ b, const double *__restrict__ dinv,
                                                      double *__restrict__ x, double *__restrict__ r,
                                                      double *__restrict__ p, int64_t n, int flexible, RedWS red)
{
    __shared__ double lds[2 * (VNT / 64)];
    double acc[2] = {0.0, 0.0};
    GRID_STRIDE(i, n)
    {
        const double bi = b[i];
        x[i] = 0.0;
        if (!flexible) {
            const double zi = dinv ? dinv[i] * bi : bi;
            r[i] = zi; // the preconditioned CG keeps z = D^-1 r in place of r
            p[i] = zi;
            acc[0] += bi * zi;
        } else {
            r[i] = bi;
            p[i] = 0.0;
        }
        acc[1] += bi * bi;
    }
    grid_partials<2>(acc, red, lds);
}

__global__ void __launch_bounds__(FNT) cg_init_finalize_kernel(CGState *st, const double *__restrict__ partials,
                                                               unsigned nb, double rtol, int maxit, int flexible)
{
    __shared__ double tot[2];
    wave_set_sums<2>(partials, nb, tot);
    if (threadIdx.x == 0) {
        st->rz = tot[0];
        st->rz_old = 0.0;
        st->rr = tot[1];
        st->bb = tot[1];
        st->thresh2 = rtol * rtol * tot[1];
        st->iter = 0;
        st->maxit = maxit;
        st->breakdown = 0;
        st->flexible = flexible;
        st->run = (tot[1] == 0.0 || maxit <= 0) ? 0 : 1; // the flexible CG's first direction step runs
        st->xpend = 0;
        st->rzprev = 0.0;
        st->alpha = 0.0;
        st->beta = 0.0;
        st->pAp = 0.0;
        st->done = (tot[1] == 0.0 || maxit <= 0) ? 1 : 0;
    }
}

hipError_t cg_init(CGState *st, const double *b, const double *dinv, double *x, double *r, double *p, int64_t n,
                   double rtol, int maxit, int flexible, const RedWS *red, hipStream_t s)
{
    const unsigned nb = vec_blocks(n);
    if (red->capacity < 2 * nb) return hipErrorInvalidValue;
    cg_init_kernel<<<nb, VNT, 0, s>>>(b, dinv, x, r, p, n, flexible, *red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    cg_init_finalize_kernel<<<1, FNT, 0, s>>>(st, red->partials, nb, rtol, maxit, flexible);
    return hipGetLastError();
}

__global__ void __launch_bounds__(FNT) cg_alpha_kernel(CGState *st, const double *__restrict__ partials, unsigned nb)
{
    __shared__ double lds[FNT];
    if (st->done) return; // the apply was skipped; its partials are stale
    const double pAp = sum_partials<FNT>(partials, nb, 0, lds);
    if (threadIdx.x == 0) {
        st->pAp = pAp;
        if (!(pAp > 0.0) || !isfinite(pAp)) {
            st->breakdown = 1;
            st->done = 1;
            st->alpha = 0.0;
        } else {
            st->alpha = st->rz / pAp;
        }
    }
}

hipError_t cg_alpha(CGState *st, const RedWS *red, unsigned nb, hipStream_t s)
{
    if (red->capacity < nb) return hipErrorInvalidValue;
    cg_alpha_kernel<<<1, FNT, 0, s>>>(st, red->partials, nb);
    return hipGetLastError();
}

static unsigned cg_resid_blocks(int64_t n)
{
    int64_t b = (n + (int64_t)VNT * CG_UNROLL - 1) / ((int64_t)VNT * CG_UNROLL);
    if (b < 1) b = 1;
    return (unsigned)(b < CG_RESID_BLOCKS ? b : CG_RESID_BLOCKS);
}

// Grid-stride visit of [0, n) with CG_UNROLL elements per step: load(k, i)
// for all k first, then use(k, i) in order k = 0, 1, ...
template <typename L, typename U> __device__ __forceinline__ void grid_stride_unrolled(int64_t n, L load, U use)
{
    const int64_t S = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (CG_UNROLL - 1) * S < n; i += CG_UNROLL * S) {
#pragma unroll
        for (int k = 0; k < CG_UNROLL; ++k) load(k, i + k * S);
#pragma unroll
        for (int k = 0; k < CG_UNROLL; ++k) use(k, i + k * S);
    }
    for (; i < n; i += S) {
        load(0, i);
        use(0, i);
    }
}

// The same visit, with the first step's loads issued before mid(), which
// every thread calls once (a workgroup reduction with a barrier): the loads
// are in flight while the workgroup sums the partials that use() needs.
template <typename L, typename M, typename U>
__device__ __forceinline__ void grid_stride_early(int64_t n, L load, M mid, U use)
{
    const int64_t S = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool full = i + (CG_UNROLL - 1) * S < n;
    if (full) {
#pragma unroll
        for (int k = 0; k < CG_UNROLL; ++k) load(k, i + k * S);
    }
    mid();
    while (full) {
#pragma unroll
        for (int k = 0; k < CG_UNROLL; ++k) use(k, i + k * S);
        i += CG_UNROLL * S;
        full = i + (CG_UNROLL - 1) * S < n;
        if (full) {
#pragma unroll
            for (int k = 0; k < CG_UNROLL; ++k) load(k, i + k * S);
        }
    }
    for (; i < n; i += S) {
        load(0, i);
        use(0, i);
    }
}

template <bool PC>
__global__ void __launch_bounds__(VNT) cg_resid_kernel(CGState *st, const double *__restrict__ dinv,
                                                       double *__restrict__ r, const double *__restrict__ q,
                                                       int64_t n, RedWS red)
{
    __shared__ double lds[2 * (VNT / 64)];
    const int skip = st->done;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->run = !skip; // read by the step kernel only
    if (skip) return;
    const double alpha = st->alpha;
    double acc[2] = {0.0, 0.0};
    double rv[CG_UNROLL], qv[CG_UNROLL], dv[CG_UNROLL];
    grid_stride_unrolled(
        n,
        [&](int k, int64_t i) {
            rv[k] = r[i];
            qv[k] = q[i];
            if (PC) dv[k] = dinv[i];
        },
        [&](int k, int64_t i) {
            if (PC) {
                // the vector holds z = D^-1 r: z -= alpha D^-1 q, r = z / D^-1
                const double zi = rv[k] - alpha * (dv[k] * qv[k]);
                r[i] = zi;
                const double ri = zi / dv[k];
                acc[0] += ri * zi;
                acc[1] += ri * ri;
            } else {
                const double ri = rv[k] - alpha * qv[k];
                r[i] = ri;
                acc[0] += ri * ri;
                acc[1] += ri * ri;
            }
        });
    grid_partials<2>(acc, red, lds);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // no other workgroup of this launch reads these two fields
        st->iter += 1;
        st->rz_old = st->rz;
    }
}

hipError_t cg_resid(CGState *st, const double *dinv, double *r, const double *q, int64_t n, const RedWS *red,
                    hipStream_t s)
{
    const unsigned nb = cg_resid_blocks(n);
    if (red->capacity < 2 * nb) return hipErrorInvalidValue;
    if (dinv) cg_resid_kernel<true><<<nb, VNT, 0, s>>>(st, dinv, r, q, n, *red);
    else cg_resid_kernel<false><<<nb, VNT, 0, s>>>(st, dinv, r, q, n, *red);
    return hipGetLastError();
}

__global__ void __launch_bounds__(VNT) cg_step_kernel(CGState *st, const double *__restrict__ partials, unsigned nb,
                                                      double *__restrict__ x, const double *__restrict__ z,
                                                      double *__restrict__ p, int64_t n)
{
    __shared__ double tot[2];
    if (!st->run) return; // this iteration's residual update was skipped (written by an earlier launch)
    double xv[CG_UNROLL], pv[CG_UNROLL], zv[CG_UNROLL];
    double alpha = 0.0, beta = 0.0;
    bool stop = false;
    grid_stride_early(
        n,
        [&](int k, int64_t i) {
            xv[k] = x[i];
            pv[k] = p[i];
            zv[k] = z[i];
        },
        [&] {
            wave_set_sums<2>(partials, nb, tot);
            const double rz = tot[0], rr = tot[1];
            const bool bad = !isfinite(rz) || !isfinite(rr);
            stop = bad || rr <= st->thresh2 || st->iter >= st->maxit;
            beta = rz / st->rz_old;
            alpha = st->alpha;
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                st->rr = rr;
                st->rz = rz;
                st->beta = beta;
                if (bad) st->breakdown = 1;
                if (stop) st->done = 1;
            }
        },
        [&](int k, int64_t i) {
            x[i] = xv[k] + alpha * pv[k];
            if (!stop) p[i] = zv[k] + beta * pv[k]; // the last iteration updates x only
        });
}

hipError_t cg_step(CGState *st, double *x, const double *z, double *p, int64_t n, const RedWS *red, hipStream_t s)
{
    unsigned nb = (unsigned)std::min<int64_t>(((n + (int64_t)VNT * CG_UNROLL - 1) / ((int64_t)VNT * CG_UNROLL)),
                                              CG_STEP_BLOCKS);
    if (nb < 1) nb = 1;
    cg_step_kernel<<<nb, VNT, 0, s>>>(st, red->partials, cg_resid_blocks(n), x, z, p, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Flexible CG (Notay) with an FP32 preconditioner z = V(r).  One iteration:
//   apply     q = A p, alpha = rz / p.Ap             (CG-mode apply)
//   resid     r -= alpha q, r32 = fl32(r); partials of r.r and r.z_old,
//             z_old (FP32) being the last preconditioner output, still in
//             place                                  (reads r, q, z_old;
//                                                     writes r, r32)
//   finalize  iteration count, r.r, r.z_old, convergence; the host polls
//   z = V(r32)                                       (the caller)
//   dir       partials of r.z                        (reads r, z)
//   step      every workgroup sums dir's partials in the same order:
//             rz_new, Polak-Ribiere beta = (rz_new - r.z_old) / rz (0 for
//             the first direction); x += alpha p, the update the residual
//             step deferred, and p = z + beta p      (reads z, p, x;
//                                                     writes p, x)
// After the last poll fcg_finish adds a still pending alpha p to x.  The
// step kernel writes done (on breakdown), so it tests `run` (set by the
// residual kernel or the initialization) instead.  `xpend` records whether
// x still lacks the last alpha p.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(VNT) fcg_resid_kernel(CGState *st, double *__restrict__ r,
                                                        const double *__restrict__ q,
                                                        const float *__restrict__ zold, float *__restrict__ r32,
                                                        int64_t n, RedWS red)
{
    __shared__ double lds[2 * (VNT / 64)];
    const int skip = st->done;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->run = !skip; // read by the step kernel only
        if (!skip) st->xpend = 1;
    }
    if (skip) return;
    const double alpha = st->alpha;
    double acc[2] = {0.0, 0.0};
    double rv[CG_UNROLL], qv[CG_UNROLL];
    float zv[CG_UNROLL];
    grid_stride_unrolled(
        n,
        [&](int k, int64_t i) {
            rv[k] = r[i];
            qv[k] = q[i];
            zv[k] = zold[i];
        },
        [&](int k, int64_t i) {
            const double ri = rv[k] - alpha * qv[k];
            r[i] = ri;
            r32[i] = (float)ri; // the FP32 preconditioner's input
            acc[0] += ri * ri;
            acc[1] += ri * (double)zv[k];
        });
    grid_partials<2>(acc, red, lds);
}

__global__ void __launch_bounds__(FNT) fcg_resid_finalize_kernel(CGState *st, const double *__restrict__ partials,
                                                                 unsigned nb)
{
    __shared__ double tot[2];
    if (st->done) return;
    wave_set_sums<2>(partials, nb, tot);
    if (threadIdx.x == 0) {
        const double rr = tot[0];
        st->iter += 1;
        st->rr = rr;
        st->rzprev = tot[1];
        st->rz_old = st->rz; // read by the step kernel, which writes rz
        if (!isfinite(rr)) {
            st->breakdown = 1;
            st->done = 1;
        } else if (rr <= st->thresh2 || st->iter >= st->maxit) {
            st->done = 1;
        }
    }
}

hipError_t fcg_resid(CGState *st, double *r, const double *q, const float *zold, float *r32, int64_t n,
                     const RedWS *red, hipStream_t s)
{
    const unsigned nb = vec_blocks(n);
    if (red->capacity < 2 * nb) return hipErrorInvalidValue;
    fcg_resid_kernel<<<nb, VNT, 0, s>>>(st, r, q, zold, r32, n, *red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    fcg_resid_finalize_kernel<<<1, FNT, 0, s>>>(st, red->partials, nb);
    return hipGetLastError();
}

__global__ void __launch_bounds__(VNT) fcg_dir_kernel(const CGState *st, const double *__restrict__ r,
                                                      const float *__restrict__ z, int64_t n, RedWS red)
{
    __shared__ double lds[VNT / 64];
    if (!st->run) return;
    double acc = 0.0;
    double rv[CG_UNROLL];
    float zv[CG_UNROLL];
    grid_stride_unrolled(
        n,
        [&](int k, int64_t i) {
            rv[k] = r[i];
            zv[k] = z[i];
        },
        [&](int k, int64_t) { acc += rv[k] * (double)zv[k]; });
    grid_partials<1>(&acc, red, lds);
}

static unsigned stream_blocks(int64_t n)
{
    const int64_t b = (n + (int64_t)VNT * CG_UNROLL - 1) / ((int64_t)VNT * CG_UNROLL);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, CG_STEP_BLOCKS));
}

__global__ void __launch_bounds__(VNT) fcg_step_kernel(CGState *st, const double *__restrict__ partials, unsigned nb,
                                                       const float *__restrict__ z, double *__restrict__ p,
                                                       double *__restrict__ x, int64_t n)
{
    __shared__ double tot[1];
    if (!st->run) return; // written by an earlier launch; this kernel may write done
    float zv[CG_UNROLL];
    double pv[CG_UNROLL], xv[CG_UNROLL];
    double alpha = 0.0, beta = 0.0;
    bool bad = false;
    grid_stride_early(
        n,
        [&](int k, int64_t i) {
            zv[k] = z[i];
            pv[k] = p[i];
            xv[k] = x[i];
        },
        [&] {
            wave_set_sums<1>(partials, nb, tot);
            // fields read here are written by earlier launches only (rz_old by
            // the residual step's finalize; rz, written below, is not read)
            const double rz = tot[0], rz_old = st->rz_old;
            alpha = st->alpha;
            bad = !isfinite(rz) || !(rz > 0.0);
            // first direction: rz_old == 0 marks "no previous direction"
            beta = (!bad && rz_old != 0.0) ? (rz - st->rzprev) / rz_old : 0.0;
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                st->beta = beta;
                st->xpend = 0;
                if (bad) {
                    st->breakdown = 1;
                    st->done = 1;
                } else {
                    st->rz = rz;
                }
            }
        },
        [&](int k, int64_t i) {
            x[i] = xv[k] + alpha * pv[k];
            // on a breakdown x still takes the deferred update; p is not needed any more
            if (!bad) p[i] = (double)zv[k] + beta * pv[k];
        });
}

hipError_t fcg_direction(CGState *st, const double *r, const float *z, double *p, double *x, int64_t n,
                         const RedWS *red, hipStream_t s)
{
    const unsigned nb = cg_resid_blocks(n);
    if (red->capacity < nb) return hipErrorInvalidValue;
    fcg_dir_kernel<<<nb, VNT, 0, s>>>(st, r, z, n, *red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    fcg_step_kernel<<<stream_blocks(n), VNT, 0, s>>>(st, red->partials, nb, z, p, x, n);
    return hipGetLastError();
}

__global__ void __launch_bounds__(VNT) fcg_finish_kernel(const CGState *st, const double *__restrict__ p,
                                                         double *__restrict__ x, int64_t n)
{
    if (!st->xpend) return;
    const double alpha = st->alpha;
    double pv[CG_UNROLL], xv[CG_UNROLL];
    grid_stride_unrolled(
        n, [&](int k, int64_t i) { pv[k] = p[i]; xv[k] = x[i]; },
        [&](int k, int64_t i) { x[i] = xv[k] + alpha * pv[k]; });
}

hipError_t fcg_finish(const CGState *st, const double *p, double *x, int64_t n, hipStream_t s)
{
    fcg_finish_kernel<<<stream_blocks(n), VNT, 0, s>>>(st, p, x, n);
    return hipGetLastError();
}

} // namespace mf
