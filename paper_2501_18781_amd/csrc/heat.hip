// heat.hip -- matrix-free Q2 heat operator on gfx950.
//
// Operator (Sec. 2.1, eq. heat_transfer without convection, one backward
// Euler step; coefficients by eqs. heaviside and muEff of Sec. 2.3):
//   (A x)_i = sum_cells sum_q W_q ( alpha_m rc_q N_i x_q + alpha_k k_q grad N_i . grad x_q )
// applied without assembling A (App. B: matrix-free products).
//
// Work decomposition: one workgroup per brick of BX x BY x BZ cells, one
// thread per cell.
//   1. the brick's nodal values of x (Dirichlet nodes read as zero) and of
//      phi are staged in LDS with contiguous row loads;
//   2. each thread gathers its cell's 27 values from LDS and evaluates the
//      cell operator entirely in registers by sum factorization (3x3
//      contractions along one direction at a time, collocation derivatives
//      at the Gauss points);
//   3. the 27 cell results go to a cell-major LDS array; one thread per
//      brick node sums the contributions of the cells that share it in a
//      fixed order;
//   4. nodes interior to the brick are written with plain stores; nodes on a
//      face shared with a neighbouring brick are added with hardware FP64
//      atomics into an output the caller zeroed.
// Dirichlet nodes are written as y_i = x_i.
#include "kernels.hpp"

namespace mf {

template <int BX, int BY, int BZ> struct BrickGeo {
    static constexpr int PX = 2 * BX + 1, PY = 2 * BY + 1, PZ = 2 * BZ + 1;
    static constexpr int NB = PX * PY * PZ;
    static constexpr int NC = BX * BY * BZ;
    int c0x, c0y, c0z; // first cell
    int ncx, ncy, ncz; // valid cells in the brick (clipped at the mesh end)

    __device__ __forceinline__ BrickGeo(const KMesh &m, int brick)
    {
        const int nbx = (m.nx + BX - 1) / BX, nby = (m.ny + BY - 1) / BY;
        const int bx = brick % nbx, by = (brick / nbx) % nby, bz = brick / (nbx * nby);
        c0x = bx * BX;
        c0y = by * BY;
        c0z = bz * BZ;
        ncx = min(BX, m.nx - c0x);
        ncy = min(BY, m.ny - c0y);
        ncz = min(BZ, m.nz - c0z);
    }
    static __device__ __forceinline__ int lds_index(int lx, int ly, int lz) { return lx + PX * (ly + PY * lz); }

    // Cooperative load of a nodal field into LDS; zero outside the mesh and,
    // if mask, on Dirichlet nodes.
    template <int NT, typename T>
    __device__ __forceinline__ void load(const KMesh &m, const T *__restrict__ g, T *lds, bool mask) const
    {
        for (int i = threadIdx.x; i < NB; i += NT) {
            const int lx = i % PX, ly = (i / PX) % PY, lz = i / (PX * PY);
            const int gx = 2 * c0x + lx, gy = 2 * c0y + ly, gz = 2 * c0z + lz;
            T v = T(0);
            if (gx < m.NX && gy < m.NY && gz < m.NZ && !(mask && node_constrained(m, gx, gy, gz)))
                v = g[node_index(m, gx, gy, gz)];
            lds[i] = v;
        }
    }

    __device__ __forceinline__ void cell_of_thread(int t, int &tx, int &ty, int &tz, bool &valid) const
    {
        tx = t % BX;
        ty = (t / BX) % BY;
        tz = t / (BX * BY);
        valid = tx < ncx && ty < ncy && tz < ncz;
    }

    template <typename T> __device__ __forceinline__ void gather27(const T *lds, int tx, int ty, int tz, T *v) const
    {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int a = 0; a < 3; ++a) v[a + 3 * b + 9 * c] = lds[lds_index(2 * tx + a, 2 * ty + b, 2 * tz + c)];
    }

    // Sum of the cell-major contributions E[cell*27 + local] at brick node
    // (lx, ly, lz), cells in fixed (z, y, x) order.
    template <typename T> __device__ __forceinline__ T node_sum(const T *E, int lx, int ly, int lz) const
    {
        const int xlo = max(0, (lx - 1) >> 1), xhi = min(ncx - 1, lx >> 1);
        const int ylo = max(0, (ly - 1) >> 1), yhi = min(ncy - 1, ly >> 1);
        const int zlo = max(0, (lz - 1) >> 1), zhi = min(ncz - 1, lz >> 1);
        T s = T(0);
        for (int cz = zlo; cz <= zhi; ++cz)
            for (int cy = ylo; cy <= yhi; ++cy)
                for (int cx = xlo; cx <= xhi; ++cx) {
                    const int cell = cx + BX * (cy + BY * cz);
                    const int loc = (lx - 2 * cx) + 3 * (ly - 2 * cy) + 9 * (lz - 2 * cz);
                    s += E[cell * 27 + loc];
                }
        return s;
    }

    // Whether brick node (lx,ly,lz) at global (gx,gy,gz) also belongs to a
    // neighbouring brick.
    __device__ __forceinline__ bool shared(const KMesh &m, int lx, int ly, int lz, int gx, int gy, int gz) const
    {
        return (lx == 0 && gx > 0) || (lx == 2 * ncx && gx < m.NX - 1) || (ly == 0 && gy > 0) ||
               (ly == 2 * ncy && gy < m.NY - 1) || (lz == 0 && gz > 0) || (lz == 2 * ncz && gz < m.NZ - 1);
    }
    // The brick that writes y = x on a Dirichlet node (the one whose half-open
    // node range holds it; the last brick also holds the closing node).
    __device__ __forceinline__ bool owns(const KMesh &m, int lx, int ly, int lz, int gx, int gy, int gz) const
    {
        return (lx < 2 * ncx || gx == m.NX - 1) && (ly < 2 * ncy || gy == m.NY - 1) &&
               (lz < 2 * ncz || gz == m.NZ - 1);
    }
};

// ---------------------------------------------------------------------------
// Per-cell coefficient factors at the 27 Gauss points:
//   cm_q = alpha_m |J| w_q rc_q,   ck_q = alpha_k |J| w_q k_q / r^2
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__device__ __forceinline__ void heat_cell_coeffs(const HeatArgs &a, const T *phq, const T *kq, const T *rcq, T am_w,
                                                 T ak_w, T *cm, T *ck)
{
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        const T wq = Q2<T>::weight(q % 3) * Q2<T>::weight((q / 3) % 3) * Q2<T>::weight(q / 9);
        T k, rc;
        if (MODE == 0) {
            const T H = heaviside<T>(a.hkind, T(a.eps), phq[q], nullptr);
            k = T(a.k_g) + H * (T(a.k_l) - T(a.k_g));
            rc = T(a.rc_g) + H * (T(a.rc_l) - T(a.rc_g));
        } else {
            k = kq[q];
            rc = rcq[q];
        }
        cm[q] = am_w * wq * rc;
        ck[q] = ak_w * wq * k;
    }
}

// y_e = A_e x_e on one cell, returned in u (27 nodal values); energy += x_e.A_e x_e.
template <typename T>
__device__ __forceinline__ void heat_cell_apply(T *u, const T *cm, const T *ck, T ihx, T ihy, T ihz, double &energy)
{
    interp3(u);
    T acc[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        acc[q] = cm[q] * u[q];
        energy += (double)(u[q] * acc[q]);
    }
    grad_line_apply<T, 0>(u, ck, ihx, acc, energy);
    grad_line_apply<T, 1>(u, ck, ihy, acc, energy);
    grad_line_apply<T, 2>(u, ck, ihz, acc, energy);
    interp3T(acc);
#pragma unroll
    for (int q = 0; q < 27; ++q) u[q] = acc[q];
}

constexpr int HB_X = 8, HB_Y = 8, HB_Z = 4;
constexpr int HB_NT = HB_X * HB_Y * HB_Z;

template <typename T, int MODE, bool CG>
__global__ void __launch_bounds__(HB_NT) heat_apply_kernel(KMesh m, HeatArgs a, const T *__restrict__ x,
                                                           T *__restrict__ y, CGState *cg, RedWS red)
{
    using G = BrickGeo<HB_X, HB_Y, HB_Z>;
    // x stays resident for the energy; phi and then the cell contributions share the rest
    constexpr int LDS_T = G::NB + (G::NB > 27 * G::NC ? G::NB : 27 * G::NC);
    __shared__ T lds[LDS_T];
    __shared__ double red_lds[HB_NT];
    __shared__ int flag_lds;
    if (CG) {
        if (cg->done) return; // converged or broken down: the rest of the batch is a no-op
    }
    const G br(m, blockIdx.x);
    T *xs = lds;
    T *ps = lds + G::NB;
    br.template load<HB_NT>(m, x, xs, true);
    if (MODE == 0) br.template load<HB_NT>(m, (const T *)a.phi, ps, false);
    __syncthreads();

    int tx, ty, tz;
    bool valid;
    br.cell_of_thread(threadIdx.x, tx, ty, tz, valid);
    const T vol = T(m.hx * m.hy * m.hz);
    const T am_w = T(a.am) * vol;
    const T ak_w = T(a.ak) * vol / T(kR * kR);
    const T ihx = T(1.0 / (m.hx * m.hx)), ihy = T(1.0 / (m.hy * m.hy)), ihz = T(1.0 / (m.hz * m.hz));
    T u[27];
    double energy_unused = 0.0;
    {
        T cm[27], ck[27];
        if (MODE == 0) {
            T ph[27];
            br.gather27(ps, tx, ty, tz, ph);
            interp3(ph);
            heat_cell_coeffs<T, 0>(a, ph, nullptr, nullptr, am_w, ak_w, cm, ck);
        } else {
            const int64_t cell = valid ? (int64_t)(br.c0x + tx) + (int64_t)m.nx * ((br.c0y + ty) + (int64_t)m.ny * (br.c0z + tz)) : 0;
            heat_cell_coeffs<T, 1>(a, nullptr, (const T *)a.kq + 27 * cell, (const T *)a.rcq + 27 * cell, am_w, ak_w,
                                   cm, ck);
        }
        br.gather27(xs, tx, ty, tz, u);
        heat_cell_apply<T>(u, cm, ck, ihx, ihy, ihz, energy_unused);
    }
    __syncthreads(); // the phi region is now reused for the cell-major contributions
    T *E = ps;
#pragma unroll
    for (int i = 0; i < 27; ++i) E[threadIdx.x * 27 + i] = valid ? u[i] : T(0);
    __syncthreads();

    // x.Ax = sum over bricks of x_i times the brick's partial sum at node i
    double energy = 0.0;
    for (int i = threadIdx.x; i < G::NB; i += HB_NT) {
        const int lx = i % G::PX, ly = (i / G::PX) % G::PY, lz = i / (G::PX * G::PY);
        if (lx > 2 * br.ncx || ly > 2 * br.ncy || lz > 2 * br.ncz) continue;
        const int gx = 2 * br.c0x + lx, gy = 2 * br.c0y + ly, gz = 2 * br.c0z + lz;
        const int64_t g = node_index(m, gx, gy, gz);
        if (node_constrained(m, gx, gy, gz)) {
            if (br.owns(m, lx, ly, lz, gx, gy, gz)) {
                const T xv = x[g];
                y[g] = xv;
                if (CG) energy += (double)xv * (double)xv;
            }
            continue;
        }
        const T s = br.node_sum(E, lx, ly, lz);
        if (CG) energy += (double)xs[i] * (double)s;
        if (br.shared(m, lx, ly, lz, gx, gy, gz))
            atomicAdd(&y[g], s);
        else
            y[g] = s;
    }
    if (CG) {
        const double tot = block_sum<HB_NT>(energy, red_lds);
        if (publish_partials<1>(&tot, red.partials, red.counter, gridDim.x, &flag_lds)) {
            const double pAp = sum_partials<HB_NT>(red.partials, gridDim.x, 0, red_lds);
            if (threadIdx.x == 0) {
                cg->pAp = pAp;
                if (!(pAp > 0.0) || !isfinite(pAp)) {
                    cg->breakdown = 1;
                    cg->done = 1;
                    cg->alpha = 0.0;
                } else {
                    cg->alpha = cg->rz / pAp;
                }
                __hip_atomic_store(red.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

hipError_t heat_apply(const KMesh &m, const HeatArgs &a, int fp32, const void *x, void *y, CGState *cg,
                      const RedWS *red, hipStream_t s)
{
    const int nbx = (m.nx + HB_X - 1) / HB_X, nby = (m.ny + HB_Y - 1) / HB_Y, nbz = (m.nz + HB_Z - 1) / HB_Z;
    const unsigned nb = (unsigned)(nbx * nby * nbz);
    const int64_t nn = (int64_t)m.NX * m.NY * m.NZ;
    RedWS r = red ? *red : RedWS{nullptr, nullptr, 0};
    if (cg && (!red || red->capacity < nb)) return hipErrorInvalidValue;
    if (!cg) {
        hipError_t e = vfill(y, 0.0, nn, fp32, s);
        if (e != hipSuccess) return e;
    }
    if (fp32) {
        if (cg) return hipErrorInvalidValue;
        if (a.mode == 0)
            heat_apply_kernel<float, 0, false><<<nb, HB_NT, 0, s>>>(m, a, (const float *)x, (float *)y, nullptr, r);
        else
            heat_apply_kernel<float, 1, false><<<nb, HB_NT, 0, s>>>(m, a, (const float *)x, (float *)y, nullptr, r);
    } else if (cg) {
        if (a.mode == 0)
            heat_apply_kernel<double, 0, true><<<nb, HB_NT, 0, s>>>(m, a, (const double *)x, (double *)y, cg, r);
        else
            heat_apply_kernel<double, 1, true><<<nb, HB_NT, 0, s>>>(m, a, (const double *)x, (double *)y, cg, r);
    } else {
        if (a.mode == 0)
            heat_apply_kernel<double, 0, false><<<nb, HB_NT, 0, s>>>(m, a, (const double *)x, (double *)y, nullptr, r);
        else
            heat_apply_kernel<double, 1, false><<<nb, HB_NT, 0, s>>>(m, a, (const double *)x, (double *)y, nullptr, r);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Diagonal: diag_i = sum_cells sum_q cm_q N_i(q)^2 + ck_q sum_d (D'_d N_i(q))^2 / h_d^2,
// evaluated per cell node by a direct loop over the Gauss points (setup only).
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ void __launch_bounds__(HB_NT) heat_diag_kernel(KMesh m, HeatArgs a, T *__restrict__ diag)
{
    using G = BrickGeo<HB_X, HB_Y, HB_Z>;
    constexpr int LDS_T = (G::NB > 27 * G::NC ? G::NB : 27 * G::NC);
    __shared__ T lds[LDS_T];
    const G br(m, blockIdx.x);
    if (MODE == 0) br.template load<HB_NT>(m, (const T *)a.phi, lds, false);
    __syncthreads();
    int tx, ty, tz;
    bool valid;
    br.cell_of_thread(threadIdx.x, tx, ty, tz, valid);
    const T vol = T(m.hx * m.hy * m.hz);
    const T am_w = T(a.am) * vol, ak_w = T(a.ak) * vol;
    const T ih[3] = {T(1.0 / (m.hx * m.hx)), T(1.0 / (m.hy * m.hy)), T(1.0 / (m.hz * m.hz))};
    T cm[27], ck[27];
    if (MODE == 0) {
        T ph[27];
        br.gather27(lds, tx, ty, tz, ph);
        interp3(ph);
        heat_cell_coeffs<T, 0>(a, ph, nullptr, nullptr, am_w, ak_w, cm, ck);
    } else {
        const int64_t cell = valid ? (int64_t)(br.c0x + tx) + (int64_t)m.nx * ((br.c0y + ty) + (int64_t)m.ny * (br.c0z + tz)) : 0;
        heat_cell_coeffs<T, 1>(a, nullptr, (const T *)a.kq + 27 * cell, (const T *)a.rcq + 27 * cell, am_w, ak_w, cm, ck);
    }
    // 1D tables: S[q][a] and G[q][a] = l_a'(xi_q)
    const T S[3][3] = {{Q2<T>::s0, Q2<T>::s1, Q2<T>::s2}, {T(0), T(1), T(0)}, {Q2<T>::s2, Q2<T>::s1, Q2<T>::s0}};
    const T Gd[3][3] = {{Q2<T>::g0, Q2<T>::g1, Q2<T>::g2}, {T(-1), T(0), T(1)}, {-Q2<T>::g2, -Q2<T>::g1, -Q2<T>::g0}};
    T d[27];
    for (int i = 0; i < 27; ++i) {
        const int ia = i % 3, ib = (i / 3) % 3, ic = i / 9;
        T s = T(0);
        for (int q = 0; q < 27; ++q) {
            const int qa = q % 3, qb = (q / 3) % 3, qc = q / 9;
            const T nx = S[qa][ia], ny = S[qb][ib], nz = S[qc][ic];
            const T n = nx * ny * nz;
            const T gx = Gd[qa][ia] * ny * nz, gy = nx * Gd[qb][ib] * nz, gz = nx * ny * Gd[qc][ic];
            s += cm[q] * n * n + ck[q] * (gx * gx * ih[0] + gy * gy * ih[1] + gz * gz * ih[2]);
        }
        d[i] = s;
    }
    __syncthreads();
    T *E = lds;
    for (int i = 0; i < 27; ++i) E[threadIdx.x * 27 + i] = valid ? d[i] : T(0);
    __syncthreads();
    for (int i = threadIdx.x; i < G::NB; i += HB_NT) {
        const int lx = i % G::PX, ly = (i / G::PX) % G::PY, lz = i / (G::PX * G::PY);
        if (lx > 2 * br.ncx || ly > 2 * br.ncy || lz > 2 * br.ncz) continue;
        const int gx = 2 * br.c0x + lx, gy = 2 * br.c0y + ly, gz = 2 * br.c0z + lz;
        const int64_t g = node_index(m, gx, gy, gz);
        if (node_constrained(m, gx, gy, gz)) {
            if (br.owns(m, lx, ly, lz, gx, gy, gz)) diag[g] = T(1);
            continue;
        }
        const T s = br.node_sum(E, lx, ly, lz);
        if (br.shared(m, lx, ly, lz, gx, gy, gz))
            atomicAdd(&diag[g], s);
        else
            diag[g] = s;
    }
}

hipError_t heat_diagonal(const KMesh &m, const HeatArgs &a, int fp32, void *diag, hipStream_t s)
{
    const int nbx = (m.nx + HB_X - 1) / HB_X, nby = (m.ny + HB_Y - 1) / HB_Y, nbz = (m.nz + HB_Z - 1) / HB_Z;
    const unsigned nb = (unsigned)(nbx * nby * nbz);
    const int64_t nn = (int64_t)m.NX * m.NY * m.NZ;
    hipError_t e = vfill(diag, 0.0, nn, fp32, s);
    if (e != hipSuccess) return e;
    if (fp32) {
        if (a.mode == 0) heat_diag_kernel<float, 0><<<nb, HB_NT, 0, s>>>(m, a, (float *)diag);
        else heat_diag_kernel<float, 1><<<nb, HB_NT, 0, s>>>(m, a, (float *)diag);
    } else {
        if (a.mode == 0) heat_diag_kernel<double, 0><<<nb, HB_NT, 0, s>>>(m, a, (double *)diag);
        else heat_diag_kernel<double, 1><<<nb, HB_NT, 0, s>>>(m, a, (double *)diag);
    }
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

__device__ __forceinline__ void gather_global27(const KMesh &m, const double *__restrict__ g, int cx, int cy, int cz,
                                                double *v)
{
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) v[a + 3 * b + 9 * c] = g[node_index(m, 2 * cx + a, 2 * cy + b, 2 * cz + c)];
}

__global__ void heat_qp_kernel(KMesh m, HeatArgs a, double *__restrict__ kq, double *__restrict__ rcq)
{
    const int64_t nc = (int64_t)m.nx * m.ny * m.nz;
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= nc) return;
    const int cx = (int)(cell % m.nx), cy = (int)((cell / m.nx) % m.ny), cz = (int)(cell / ((int64_t)m.nx * m.ny));
    double ph[27];
    gather_global27(m, (const double *)a.phi, cx, cy, cz, ph);
    interp3(ph);
    for (int q = 0; q < 27; ++q) {
        const double H = heaviside<double>(a.hkind, a.eps, ph[q], nullptr);
        kq[cell * 27 + q] = a.k_g + H * (a.k_l - a.k_g);
        rcq[cell * 27 + q] = a.rc_g + H * (a.rc_l - a.rc_g);
    }
}

hipError_t heat_qp_coeffs(const KMesh &m, const HeatArgs &a, double *kq, double *rcq, hipStream_t s)
{
    const int64_t nc = (int64_t)m.nx * m.ny * m.nz;
    heat_qp_kernel<<<(unsigned)((nc + 255) / 256), 256, 0, s>>>(m, a, kq, rcq);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adjoint gradient of one implicit heat step (FP64):
//   dk_q  = -alpha_k W_q grad(lam) . grad(T)
//   drc_q = -alpha_m W_q lam dT
//   dphi_j = sum_q N_j(x_q) H'(phi_q) [(k_l - k_g) dk_q + (rc_l - rc_g) drc_q]
// Brick of 4x4x4 cells, one thread per cell; dphi gathered like the apply.
// ---------------------------------------------------------------------------
constexpr int GB = 4, GB_NT = GB * GB * GB;

__global__ void __launch_bounds__(GB_NT) heat_grad_kernel(KMesh m, HeatArgs a, const double *__restrict__ T,
                                                          const double *__restrict__ dT, const double *__restrict__ lam,
                                                          double *__restrict__ dk, double *__restrict__ drc,
                                                          double *__restrict__ dphi)
{
    using G = BrickGeo<GB, GB, GB>;
    constexpr int NF = 4;
    constexpr int LDS_T = (NF * G::NB > 27 * G::NC ? NF * G::NB : 27 * G::NC);
    __shared__ double lds[LDS_T];
    const G br(m, blockIdx.x);
    double *Ts = lds, *dTs = lds + G::NB, *ls = lds + 2 * G::NB, *ps = lds + 3 * G::NB;
    br.load<GB_NT>(m, T, Ts, false);
    br.load<GB_NT>(m, dT, dTs, false);
    br.load<GB_NT>(m, lam, ls, false);
    const bool with_phi = (a.mode == 0) && dphi != nullptr;
    if (with_phi) br.load<GB_NT>(m, (const double *)a.phi, ps, false);
    __syncthreads();
    int tx, ty, tz;
    bool valid;
    br.cell_of_thread(threadIdx.x, tx, ty, tz, valid);
    const int64_t cell = (int64_t)(br.c0x + tx) + (int64_t)m.nx * ((br.c0y + ty) + (int64_t)m.ny * (br.c0z + tz));
    const double vol = m.hx * m.hy * m.hz;
    const double ih[3] = {1.0 / (m.hx * m.hx * kR * kR), 1.0 / (m.hy * m.hy * kR * kR), 1.0 / (m.hz * m.hz * kR * kR)};
    double lq[27], Tq[27], gk[27];
    br.gather27(ls, tx, ty, tz, lq);
    br.gather27(Ts, tx, ty, tz, Tq);
    interp3(lq);
    interp3(Tq);
    for (int q = 0; q < 27; ++q) gk[q] = 0.0;
    grad_dot_acc<double, 0>(lq, Tq, ih[0], gk);
    grad_dot_acc<double, 1>(lq, Tq, ih[1], gk);
    grad_dot_acc<double, 2>(lq, Tq, ih[2], gk);
    double dtq[27];
    br.gather27(dTs, tx, ty, tz, dtq);
    interp3(dtq);
    double s[27];
    for (int q = 0; q < 27; ++q) {
        const double wq = vol * Q2<double>::weight(q % 3) * Q2<double>::weight((q / 3) % 3) * Q2<double>::weight(q / 9);
        const double gkq = -a.ak * wq * gk[q];
        const double grq = -a.am * wq * lq[q] * dtq[q];
        if (valid) {
            if (dk) dk[cell * 27 + q] = gkq;
            if (drc) drc[cell * 27 + q] = grq;
        }
        gk[q] = gkq;
        s[q] = grq;
    }
    if (!with_phi) return; // uniform over the launch
    double ph[27];
    br.gather27(ps, tx, ty, tz, ph);
    interp3(ph);
    for (int q = 0; q < 27; ++q) {
        double dH;
        (void)heaviside<double>(a.hkind, a.eps, ph[q], &dH);
        s[q] = dH * ((a.k_l - a.k_g) * gk[q] + (a.rc_l - a.rc_g) * s[q]);
    }
    interp3T(s);
    __syncthreads();
    double *E = lds;
    for (int i = 0; i < 27; ++i) E[threadIdx.x * 27 + i] = valid ? s[i] : 0.0;
    __syncthreads();
    for (int i = threadIdx.x; i < G::NB; i += GB_NT) {
        const int lx = i % G::PX, ly = (i / G::PX) % G::PY, lz = i / (G::PX * G::PY);
        if (lx > 2 * br.ncx || ly > 2 * br.ncy || lz > 2 * br.ncz) continue;
        const int gx = 2 * br.c0x + lx, gy = 2 * br.c0y + ly, gz = 2 * br.c0z + lz;
        const int64_t g = node_index(m, gx, gy, gz);
        const double v = br.node_sum(E, lx, ly, lz);
        if (br.shared(m, lx, ly, lz, gx, gy, gz))
            atomicAdd(&dphi[g], v);
        else
            dphi[g] = v;
    }
}

hipError_t heat_grad(const KMesh &m, const HeatArgs &a, const double *T, const double *dT, const double *lam,
                     double *dk, double *drc, double *dphi, hipStream_t s)
{
    const int nbx = (m.nx + GB - 1) / GB, nby = (m.ny + GB - 1) / GB, nbz = (m.nz + GB - 1) / GB;
    const unsigned nb = (unsigned)(nbx * nby * nbz);
    if (dphi) {
        hipError_t e = vfill(dphi, 0.0, (int64_t)m.NX * m.NY * m.NZ, 0, s);
        if (e != hipSuccess) return e;
    }
    heat_grad_kernel<<<nb, GB_NT, 0, s>>>(m, a, T, dT, lam, dk, drc, dphi);
    return hipGetLastError();
}

} // namespace mf
