// brick.hpp -- the cell-brick work unit shared by the operator kernels.
//
// A 64-thread workgroup (one wavefront) owns a brick of 4x4x4 cells, one
// thread per cell; the brick's 9x9x9 Q2 nodes are staged in LDS.
//
// Node ownership is static: a cell owns its local nodes (a, b, c) with
// a, b, c in {0, 1}, and the last valid cell of the brick in a direction
// also owns the local nodes with index 2 in that direction.  Every brick
// node is therefore loaded and finished by exactly one thread, with fully
// unrolled code, no index division and no per-node branches.  A node's sum
// runs over the cells of the brick that contain it (at most 8) in a fixed
// order.
//
// A node on a face that a neighbouring brick also touches ("shared") is not
// written to the output: its partial sum goes to the brick's slot in a face
// buffer (386 slots per brick: the 9x9x9 surface), and a second kernel adds
// the partials of the (2, 4 or 8) bricks that share it, in a fixed order.
// Every output entry is therefore written exactly once, without atomics and
// without clearing the output first, and the result is bitwise reproducible.
//
// Bricks are numbered so that each XCD receives a contiguous range of them
// (workgroups are dispatched to the 8 XCDs round robin), which keeps the
// neighbours that share faces, and their halo loads, in one L2.
#pragma once

#include <type_traits>

#include "kernels.hpp"

namespace mf {

constexpr int BB = 4;               // cells per brick edge
constexpr int BNT = BB * BB * BB;   // threads (cells) per brick
constexpr int BP = 2 * BB + 1;      // nodes per brick edge
constexpr int BNB = BP * BP * BP;   // nodes per brick
constexpr int BFACE = BNB - (BP - 2) * (BP - 2) * (BP - 2); // 386 surface nodes
constexpr int NXCD = 8;

__host__ __device__ inline int64_t n_bricks(const KMesh &m)
{
    return (int64_t)((m.nx + BB - 1) / BB) * ((m.ny + BB - 1) / BB) * ((m.nz + BB - 1) / BB);
}

// Slot of a surface node (at least one local coordinate 0 or 8) of a brick:
// the z faces first, then the y faces without the z rows, then the x faces.
__device__ __forceinline__ int face_slot(int lx, int ly, int lz)
{
    if (lz == 0) return lx + BP * ly;
    if (lz == BP - 1) return BP * BP + lx + BP * ly;
    if (ly == 0) return 2 * BP * BP + lx + BP * (lz - 1);
    if (ly == BP - 1) return 2 * BP * BP + BP * (BP - 2) + lx + BP * (lz - 1);
    if (lx == 0) return 2 * BP * BP + 2 * BP * (BP - 2) + (ly - 1) + (BP - 2) * (lz - 1);
    return 2 * BP * BP + 2 * BP * (BP - 2) + (BP - 2) * (BP - 2) + (ly - 1) + (BP - 2) * (lz - 1);
}

struct Brick {
    int brick;         // natural brick index (x fastest)
    int bx, by, bz;    // brick coordinates
    int c0x, c0y, c0z; // first cell of the brick
    int ncx, ncy, ncz; // valid cells per direction (clipped at the mesh end)
    int tx, ty, tz;    // this thread's cell within the brick
    bool valid;
    bool lastx, lasty, lastz;

    __device__ __forceinline__ Brick(const KMesh &m, int t)
    {
        // XCD-contiguous numbering: workgroup b runs on XCD b % 8; XCD k gets
        // bricks [start_k, start_k + count_k).
        const int G = gridDim.x, q = G / NXCD, r = G % NXCD;
        const int k = blockIdx.x % NXCD, j = blockIdx.x / NXCD;
        brick = k * q + min(k, r) + j;
        const int nbx = (m.nx + BB - 1) / BB, nby = (m.ny + BB - 1) / BB;
        bx = brick % nbx;
        by = (brick / nbx) % nby;
        bz = brick / (nbx * nby);
        c0x = bx * BB;
        c0y = by * BB;
        c0z = bz * BB;
        ncx = min(BB, m.nx - c0x);
        ncy = min(BB, m.ny - c0y);
        ncz = min(BB, m.nz - c0z);
        tx = t & (BB - 1);
        ty = (t / BB) & (BB - 1);
        tz = t / (BB * BB);
        valid = tx < ncx && ty < ncy && tz < ncz;
        lastx = valid && tx == ncx - 1;
        lasty = valid && ty == ncy - 1;
        lastz = valid && tz == ncz - 1;
    }

    static __device__ __forceinline__ constexpr int lds_index(int lx, int ly, int lz) { return lx + BP * (ly + BP * lz); }

    __device__ __forceinline__ int64_t cell_index(const KMesh &m) const
    {
        return (int64_t)(c0x + tx) + (int64_t)m.nx * ((c0y + ty) + (int64_t)m.ny * (c0z + tz));
    }

    // Whether the brick has a node on a Dirichlet face (uniform over the brick).
    __device__ __forceinline__ bool touches_dirichlet(const KMesh &m) const
    {
        const unsigned f = m.dirichlet;
        return ((f & 1u) && c0x == 0) || ((f & 2u) && c0x + ncx == m.nx) || ((f & 4u) && c0y == 0) ||
               ((f & 8u) && c0y + ncy == m.ny) || ((f & 16u) && c0z == 0) || ((f & 32u) && c0z + ncz == m.nz);
    }

    // Visit the nodes this thread owns: f(a, b, c, lds_index, global_index,
    // constrained, shared), with a, b, c compile-time constants.  `shared` is
    // an int: bit 0 set if a neighbouring brick also touches the node, bit 1
    // if that happens through one of this brick's high faces (the node is
    // then finished by another brick's combine pass).  The eight
    // low nodes of every valid cell come first; the high faces, owned by the
    // last cells, follow in seven groups that each test one uniform flag.
    template <typename F> __device__ __forceinline__ void for_owned_nodes(const KMesh &m, F f) const
    {
        if (!valid) return;
        const int gx0 = 2 * (c0x + tx), gy0 = 2 * (c0y + ty), gz0 = 2 * (c0z + tz);
        const int64_t g0 = node_index(m, gx0, gy0, gz0);
        const int64_t sy = m.NX, sz = (int64_t)m.NX * m.NY;
        const int l0 = lds_index(2 * tx, 2 * ty, 2 * tz);
        // Per direction, for local index 0 and 2 (index 1 is never on a
        // boundary or a brick face): Dirichlet flag and shared-face flag.
        const unsigned f6 = m.dirichlet;
        const bool dx0 = (f6 & 1u) && gx0 == 0, dx2 = (f6 & 2u) && gx0 + 2 == m.NX - 1;
        const bool dy0 = (f6 & 4u) && gy0 == 0, dy2 = (f6 & 8u) && gy0 + 2 == m.NY - 1;
        const bool dz0 = (f6 & 16u) && gz0 == 0, dz2 = (f6 & 32u) && gz0 + 2 == m.NZ - 1;
        const bool sx0 = tx == 0 && gx0 > 0, sx2 = gx0 + 2 < m.NX - 1;
        const bool sy0 = ty == 0 && gy0 > 0, sy2 = gy0 + 2 < m.NY - 1;
        const bool sz0 = tz == 0 && gz0 > 0, sz2 = gz0 + 2 < m.NZ - 1;
        auto node = [&](auto A, auto B, auto C) {
            constexpr int a = decltype(A)::value, b = decltype(B)::value, c = decltype(C)::value;
            const bool constrained = (a == 0 && dx0) || (a == 2 && dx2) || (b == 0 && dy0) || (b == 2 && dy2) ||
                                     (c == 0 && dz0) || (c == 2 && dz2);
            const bool shared_hi = (a == 2 && sx2) || (b == 2 && sy2) || (c == 2 && sz2);
            const bool shared = shared_hi || (a == 0 && sx0) || (b == 0 && sy0) || (c == 0 && sz0);
            f(a, b, c, l0 + a + BP * b + BP * BP * c, g0 + a + sy * b + sz * c, constrained,
              (shared ? 1 : 0) | (shared_hi ? 2 : 0));
        };
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        node(I0{}, I0{}, I0{}); node(I1{}, I0{}, I0{}); node(I0{}, I1{}, I0{}); node(I1{}, I1{}, I0{});
        node(I0{}, I0{}, I1{}); node(I1{}, I0{}, I1{}); node(I0{}, I1{}, I1{}); node(I1{}, I1{}, I1{});
        if (lastx) { node(I2{}, I0{}, I0{}); node(I2{}, I1{}, I0{}); node(I2{}, I0{}, I1{}); node(I2{}, I1{}, I1{}); }
        if (lasty) { node(I0{}, I2{}, I0{}); node(I1{}, I2{}, I0{}); node(I0{}, I2{}, I1{}); node(I1{}, I2{}, I1{}); }
        if (lastz) { node(I0{}, I0{}, I2{}); node(I1{}, I0{}, I2{}); node(I0{}, I1{}, I2{}); node(I1{}, I1{}, I2{}); }
        if (lastx && lasty) { node(I2{}, I2{}, I0{}); node(I2{}, I2{}, I1{}); }
        if (lastx && lastz) { node(I2{}, I0{}, I2{}); node(I2{}, I1{}, I2{}); }
        if (lasty && lastz) { node(I0{}, I2{}, I2{}); node(I1{}, I2{}, I2{}); }
        if (lastx && lasty && lastz) node(I2{}, I2{}, I2{});
    }

    // Stage a nodal field into LDS; Dirichlet nodes read as zero if mask.
    template <typename T>
    __device__ __forceinline__ void load(const KMesh &m, const T *__restrict__ g, T *lds, bool mask) const
    {
        for_owned_nodes(m, [&](int, int, int, int l, int64_t gi, bool constrained, bool) {
            const T v = g[gi];
            lds[l] = (mask && constrained) ? T(0) : v;
        });
    }

    // The cell's 27 nodal values from LDS (zero for threads without a cell).
    template <typename T> __device__ __forceinline__ void gather27(const T *lds, T *v) const
    {
        const int l0 = valid ? lds_index(2 * tx, 2 * ty, 2 * tz) : 0;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int a = 0; a < 3; ++a) v[a + 3 * b + 9 * c] = lds[l0 + a + BP * b + BP * BP * c];
    }

    // Cell results, node-major: E[local * BNT + thread]; zero without a cell.
    template <typename T> __device__ __forceinline__ void store_cell(T *E, const T *v) const
    {
        const int t = threadIdx.x;
#pragma unroll
        for (int i = 0; i < 27; ++i) E[i * BNT + t] = valid ? v[i] : T(0);
    }

    // Sum over the brick's cells containing local node (a, b, c) of this
    // thread's cell: the cell itself and, for index 0 in a direction, the
    // neighbour on the low side (local index 2 there).  Branch free: a
    // missing neighbour (brick edge) reads this cell's slot, weighted by 0.
    template <typename T> __device__ __forceinline__ T node_sum(const T *E, int a, int b, int c) const
    {
        const int t = threadIdx.x;
        T s = E[(a + 3 * b + 9 * c) * BNT + t];
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx) {
                    if (dx + dy + dz == 0) continue;
                    if ((dx && a != 0) || (dy && b != 0) || (dz && c != 0)) continue;
                    const bool ok = !((dx && tx == 0) || (dy && ty == 0) || (dz && tz == 0));
                    const int loc = (a + 2 * dx) + 3 * (b + 2 * dy) + 9 * (c + 2 * dz);
                    const int nb = ok ? t - dx - BB * dy - BB * BB * dz : t;
                    s += (ok ? T(1) : T(0)) * E[loc * BNT + nb];
                }
        return s;
    }
};

// Add the face partials of the bricks sharing each shared node.  One
// workgroup per brick handles the shared nodes on its low faces (their
// global index g has g = 8 b in a shared direction); every shared node is
// finished by exactly one brick.  Partials are summed over the contributing
// bricks in a fixed order (own brick first, then x, y, z neighbours).
// Shared Dirichlet nodes: DMODE 1 writes y = x (identity rows of an
// operator), DMODE 2 writes y = 1 (its diagonal), DMODE 0 sums them like
// every other node (a plain nodal field such as a gradient).
template <typename T, int DMODE = 1>
__device__ __forceinline__ void combine_faces(const KMesh &m, const T *__restrict__ face, const T *__restrict__ x,
                                              T *__restrict__ y, int brick, int lane)
{
    const int nbx = (m.nx + BB - 1) / BB, nby = (m.ny + BB - 1) / BB;
    const int bx = brick % nbx, by = (brick / nbx) % nby, bz = brick / (nbx * nby);
    const int ncx = min(BB, m.nx - bx * BB), ncy = min(BB, m.ny - by * BB), ncz = min(BB, m.nz - bz * BB);
    const bool shx = bx > 0, shy = by > 0, shz = bz > 0;
    // candidates: plane z = 0 (81), plane y = 0 without the z = 0 row (72),
    // plane x = 0 without the y = 0 and z = 0 rows (64)
    for (int i = lane; i < BP * BP + BP * (BP - 1) + (BP - 1) * (BP - 1); i += BNT) {
        int lx, ly, lz;
        if (i < BP * BP) {
            lx = i % BP; ly = i / BP; lz = 0;
        } else if (i < BP * BP + BP * (BP - 1)) {
            const int j = i - BP * BP;
            lx = j % BP; ly = 0; lz = 1 + j / BP;
        } else {
            const int j = i - BP * BP - BP * (BP - 1);
            lx = 0; ly = 1 + j % (BP - 1); lz = 1 + j / (BP - 1);
        }
        if (lx > 2 * ncx || ly > 2 * ncy || lz > 2 * ncz) continue;
        // nodes on the high faces belong to the next brick unless the mesh ends
        if ((lx == BP - 1 && 2 * ncx == BP - 1 && bx * BB + ncx < m.nx) ||
            (ly == BP - 1 && 2 * ncy == BP - 1 && by * BB + ncy < m.ny) ||
            (lz == BP - 1 && 2 * ncz == BP - 1 && bz * BB + ncz < m.nz))
            continue;
        const bool sx = lx == 0 && shx, sy = ly == 0 && shy, sz = lz == 0 && shz;
        if (!(sx || sy || sz)) continue;
        const int gx = 2 * bx * BB + lx, gy = 2 * by * BB + ly, gz = 2 * bz * BB + lz;
        const int64_t g = node_index(m, gx, gy, gz);
        if (DMODE != 0 && node_constrained(m, gx, gy, gz)) {
            y[g] = DMODE == 1 ? x[g] : T(1);
            continue;
        }
        T s = T(0);
        for (int dz = 0; dz <= (sz ? 1 : 0); ++dz)
            for (int dy = 0; dy <= (sy ? 1 : 0); ++dy)
                for (int dx = 0; dx <= (sx ? 1 : 0); ++dx) {
                    const int nb = brick - dx - nbx * (dy + nby * dz);
                    s += face[(int64_t)nb * BFACE + face_slot(lx + (BP - 1) * dx, ly + (BP - 1) * dy, lz + (BP - 1) * dz)];
                }
        y[g] = s;
    }
}

} // namespace mf
