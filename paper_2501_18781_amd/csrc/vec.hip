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
        const double *p = partials + (size_t)w * nb;
        double s = 0.0;
        for (unsigned b = lane; b < nb; b += 64) s += p[b];
        s = wave_sum(s);
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
        const double *p = partials + (size_t)k * nb;
        double s = 0.0;
        for (unsigned b = lane; b < nb; b += 64) s += p[b];
        s = wave_sum(s);
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
// Multi-dot, multi-axpy, combination (GMRES Gram-Schmidt).  The number of
// vectors NV is a template parameter (1..32, chosen by a switch), so that
// every loop over the vectors is unrolled without conditions and all NV
// loads of an element are in flight together.  From PAIR_MIN vectors on,
// the multi-dot and the multi-update take two consecutive elements per
// thread (16-byte loads) when the stride and the pointers allow it: with
// one element the compiler's batching of 20 or more loads dropped these
// passes to about 4 TB/s at some widths, with pairs they stream at about
// 5.5 TB/s for every width.
// ---------------------------------------------------------------------------
constexpr int PAIR_MIN = 20;

static bool pairable(const double *V, int64_t ld, const double *w)
{
    return (ld & 1) == 0 && ((uintptr_t)V & 15) == 0 && ((uintptr_t)w & 15) == 0;
}
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

// The same sums over element pairs (2i, 2i + 1); ld even, V and w 16-byte
// aligned.  The last element of an odd n goes to thread 0 of block 0.
template <int NV>
__global__ void __launch_bounds__(VNT) multidot_pair_kernel(const double *__restrict__ V, int64_t ld,
                                                            const double *__restrict__ w, int64_t n, RedWS red)
{
    __shared__ double lds[NV * (VNT / 64)];
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    GRID_STRIDE(i, n / 2)
    {
        const double2 wi = ((const double2 *)w)[i];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const double2 v = ((const double2 *)(V + (int64_t)k * ld))[i];
            acc[k] += v.x * wi.x + v.y * wi.y;
        }
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] += V[(int64_t)k * ld + n - 1] * w[n - 1];
    }
    store_block_partials<NV>(acc, lds, red);
}

template <int NV> static void launch_multidot(bool pair, unsigned nb, const double *V, int64_t ld, const double *w,
                                              int64_t n, const RedWS &red, hipStream_t s)
{
    if constexpr (NV >= PAIR_MIN) {
        if (pair) {
            multidot_pair_kernel<NV><<<nb, VNT, 0, s>>>(V, ld, w, n, red);
            return;
        }
    }
    multidot_kernel<NV><<<nb, VNT, 0, s>>>(V, ld, w, n, red);
}

hipError_t vmultidot(const double *V, int64_t ld, int nv, const double *w, int64_t n, double *out, const RedWS *red,
                     hipStream_t s)
{
    if (nv < 1 || nv > MAXV) return hipErrorInvalidValue;
    const unsigned nb = vec_blocks(n);
    if (red->capacity < nb * MAXV) return hipErrorInvalidValue;
    const bool pair = pairable(V, ld, w);
    switch (nv) {
#define MF_CASE(N)                                                                                            \
    case N: launch_multidot<N>(pair, nb, V, ld, w, n, *red, s); break;
        MF_NV_CASES(MF_CASE)
#undef MF_CASE
    }
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : sum_finalize(*red, nb, nv, out, s);
}

__global__ void scale_inv_norm_kernel(double *__restrict__ w, int64_t n, const double *__restrict__ n2)
{
    const double hn = sqrt(n2[0]);
    if (!(hn > 0.0)) return;
    const double a = 1.0 / hn;
    GRID_STRIDE(i, n) w[i] = a * w[i];
}

hipError_t vscale_inv_norm(double *w, int64_t n, const double *n2, hipStream_t s)
{
    scale_inv_norm_kernel<<<ew_blocks(n), VNT, 0, s>>>(w, n, n2);
    return hipGetLastError();
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

// w -= V h; optionally ||w||^2 of the result
template <int NV>
__global__ void __launch_bounds__(VNT) multiaxpy_kernel(const double *__restrict__ V, int64_t ld,
                                                        const double *__restrict__ h, double *__restrict__ w,
                                                        int64_t n, bool norm, RedWS red)
{
    __shared__ double lds[VNT / 64];
    __shared__ double hs[NV];
    if (threadIdx.x < NV) hs[threadIdx.x] = h[threadIdx.x];
    __syncthreads();
    double acc = 0.0;
    GRID_STRIDE(i, n)
    {
        double vk[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) vk[k] = V[(int64_t)k * ld + i];
        double v = w[i];
#pragma unroll
        for (int k = 0; k < NV; ++k) v -= vk[k] * hs[k];
        w[i] = v;
        acc += v * v;
    }
    if (norm) grid_partials<1>(&acc, red, lds);
}

// The same update over element pairs (2i, 2i + 1); ld even, V and w 16-byte
// aligned.  Each element takes the same operations in the same order as in
// the one-element kernel; only the norm's partial sums are grouped
// differently.
template <int NV>
__global__ void __launch_bounds__(VNT) multiaxpy_pair_kernel(const double *__restrict__ V, int64_t ld,
                                                             const double *__restrict__ h, double *__restrict__ w,
                                                             int64_t n, bool norm, RedWS red)
{
    __shared__ double lds[VNT / 64];
    __shared__ double hs[NV];
    if (threadIdx.x < NV) hs[threadIdx.x] = h[threadIdx.x];
    __syncthreads();
    double acc = 0.0;
    GRID_STRIDE(i, n / 2)
    {
        double2 vk[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) vk[k] = ((const double2 *)(V + (int64_t)k * ld))[i];
        double2 v = ((double2 *)w)[i];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            v.x -= vk[k].x * hs[k];
            v.y -= vk[k].y * hs[k];
        }
        ((double2 *)w)[i] = v;
        acc += v.x * v.x + v.y * v.y;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        double v = w[n - 1];
#pragma unroll
        for (int k = 0; k < NV; ++k) v -= V[(int64_t)k * ld + n - 1] * hs[k];
        w[n - 1] = v;
        acc += v * v;
    }
    if (norm) grid_partials<1>(&acc, red, lds);
}

template <int NV> static void launch_multiaxpy(bool pair, unsigned nb, const double *V, int64_t ld, const double *h,
                                               double *w, int64_t n, bool norm, const RedWS &red, hipStream_t s)
{
    if constexpr (NV >= PAIR_MIN) {
        if (pair) {
            multiaxpy_pair_kernel<NV><<<nb, VNT, 0, s>>>(V, ld, h, w, n, norm, red);
            return;
        }
    }
    multiaxpy_kernel<NV><<<nb, VNT, 0, s>>>(V, ld, h, w, n, norm, red);
}

hipError_t vmultiaxpy(const double *V, int64_t ld, int nv, const double *h, double *w, int64_t n, double *out_norm2,
                      const RedWS *red, hipStream_t s)
{
    if (nv < 1 || nv > MAXV) return hipErrorInvalidValue;
    const unsigned nb = vec_blocks(n);
    if (out_norm2 && red->capacity < nb) return hipErrorInvalidValue;
    const RedWS r = red ? *red : RedWS{nullptr, 0};
    const bool norm = out_norm2 != nullptr;
    const bool pair = pairable(V, ld, w);
    switch (nv) {
#define MF_CASE(N)                                                                                            \
    case N: launch_multiaxpy<N>(pair, nb, V, ld, h, w, n, norm, r, s); break;
        MF_NV_CASES(MF_CASE)
#undef MF_CASE
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !norm) return e;
    return sum_finalize(*red, nb, 1, out_norm2, s);
}

// w -= V h and, in the same pass, g = V^T w (the new w): the first update
// and the second projection of classical Gram-Schmidt applied twice share
// one read of V.
template <int NV>
__global__ void __launch_bounds__(VNT) multiaxpy_dot_kernel(const double *__restrict__ V, int64_t ld,
                                                            const double *__restrict__ h, double *__restrict__ w,
                                                            int64_t n, RedWS red)
{
    __shared__ double lds[NV * (VNT / 64)];
    __shared__ double hs[NV];
    if (threadIdx.x < NV) hs[threadIdx.x] = h[threadIdx.x];
    __syncthreads();
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    GRID_STRIDE(i, n)
    {
        double vk[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) vk[k] = V[(int64_t)k * ld + i];
        double v = w[i];
#pragma unroll
        for (int k = 0; k < NV; ++k) v -= vk[k] * hs[k];
        w[i] = v;
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] += vk[k] * v;
    }
    store_block_partials<NV>(acc, lds, red);
}

hipError_t vmultiaxpy_dot(const double *V, int64_t ld, int nv, const double *h, double *w, int64_t n, double *out,
                          const RedWS *red, hipStream_t s)
{
    if (nv < 1 || nv > MAXV) return hipErrorInvalidValue;
    const unsigned nb = vec_blocks(n);
    if (red->capacity < nb * MAXV) return hipErrorInvalidValue;
    switch (nv) {
#define MF_CASE(N)                                                                                            \
    case N: multiaxpy_dot_kernel<N><<<nb, VNT, 0, s>>>(V, ld, h, w, n, *red); break;
        MF_NV_CASES(MF_CASE)
#undef MF_CASE
    }
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : sum_finalize(*red, nb, nv, out, s);
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
