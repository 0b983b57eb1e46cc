// brick.hpp -- the cell-brick work unit shared by the operator kernels.
//
// A 64-thread workgroup (one wavefront) owns a brick of 4x4x4 cells, one
// thread per cell; the brick's 9x9x9 Q2 nodes are staged in LDS.  The brick
// code is templated on the brick's depth along z (BrickT<BZ>): the FP32
// heat applies take 4x4x8 cells, two wavefronts per workgroup and 9x9x17
// nodes.
//
// Staging is per cell (each thread reads the 27 nodes of its cell and
// writes them to LDS; nodes shared by cells of the brick are written with
// the same value by each) or per node (the lanes stage whole 9-node rows of
// the brick; used by the FP64 kernels).  Finishing is by ownership: a cell owns its
// local nodes (a, b, c) with a, b, c in {0, 1}, and the last valid cell of
// the brick in a direction also owns the local nodes with index 2 in that
// direction, so every brick node is finished by exactly one thread, with
// fully unrolled code and no index division.  A node's sum runs over the
// cells of the brick that contain it (at most 8) in a fixed order.
//
// A node on a face that a neighbouring brick also touches ("shared") is not
// written to the output: its partial sum goes to the brick's slot in a face
// buffer (one slot per brick node), and a second kernel adds
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
constexpr int NXCD = 8;

// LDS layout of a staged brick field: node (lx, ly, lz) at lx + R ly + R BP lz.
// For 8-byte entries the rows are padded to R = 10: a wavefront's gather of
// node (2tx + a, 2ty + b, 2tz + c) then spreads its stride-2 accesses over
// more LDS banks than with R = 9 (FP64 apply kernel 30.0 -> 27.7 us at 64^3,
// Oseen 72.6 -> 68.4 us at 48^3); 4-byte entries keep R = 9 (padding
// measured no faster there).
template <typename T> __host__ __device__ constexpr int lds_row() { return sizeof(T) == 8 ? BP + 1 : BP; }
template <typename T> __host__ __device__ constexpr int lds_plane() { return lds_row<T>() * BP; }
// LDS entries of one staged field of a brick BZ cells deep in z
template <typename T, int BZ = BB> __host__ __device__ constexpr int lds_field() { return lds_plane<T>() * (2 * BZ + 1); }

// Bricks are BB x BB x BZ cells; BZ = BB unless a kernel says otherwise.
// Per brick: threads (cells), node planes along z, nodes, face-buffer slots.
template <int BZ> struct BrickDims {
    static constexpr int NT = BB * BB * BZ;
    static constexpr int PZ = 2 * BZ + 1;
    static constexpr int NNODES = BP * BP * PZ;
    static constexpr int NFACE = NNODES + 2 * BP * PZ; // see face_slot
};
constexpr int BNB = BrickDims<BB>::NNODES;  // nodes per 4x4x4 brick
constexpr int BFACE = BrickDims<BB>::NFACE; // its face-buffer slots

template <int BZ = BB> __host__ __device__ inline int64_t n_bricks(const KMesh &m)
{
    return (int64_t)((m.nx + BB - 1) / BB) * ((m.ny + BB - 1) / BB) * ((m.nz + BZ - 1) / BZ);
}

// Face-buffer slot of a brick node (only the slots of shared surface nodes
// are ever written or read).  Nodes on the brick's two x faces get a region
// of their own, (side, ly, lz) with ly fastest, so that the combine pass
// reads them in runs along y; every other node keeps its lexicographic brick
// index, so that runs along x stay contiguous.
template <int BZ = BB> __host__ __device__ __forceinline__ constexpr int face_slot(int lx, int ly, int lz)
{
    return (lx == 0 || lx == 2 * BB) ? BrickDims<BZ>::NNODES + (lx ? BP * (2 * BZ + 1) : 0) + ly + BP * lz
                                     : lx + BP * (ly + BP * lz);
}

template <int BZ> struct BrickT {
    static constexpr int NT = BrickDims<BZ>::NT, PZ = BrickDims<BZ>::PZ;
    static constexpr int NNODES = BrickDims<BZ>::NNODES, NFACE = BrickDims<BZ>::NFACE;

    int brick;         // natural brick index (x fastest)
    int bx, by, bz;    // brick coordinates
    int c0x, c0y, c0z; // first cell of the brick
    int ncx, ncy, ncz; // valid cells per direction (clipped at the mesh end)
    int t;             // this thread's cell slot within the brick (0..63)
    int tx, ty, tz;    // this thread's cell within the brick
    bool valid;
    bool lastx, lasty, lastz;

    __device__ __forceinline__ BrickT(const KMesh &m, int slot) : BrickT(m, slot, xcd_index()) {}

    // XCD-contiguous numbering: workgroup b runs on XCD b % 8; XCD k gets
    // the workgroup indices [start_k, start_k + count_k).
    static __device__ __forceinline__ int xcd_index()
    {
        const int G = gridDim.x, q = G / NXCD, r = G % NXCD;
        const int k = blockIdx.x % NXCD, j = blockIdx.x / NXCD;
        return k * q + min(k, r) + j;
    }

    // The brick of natural index b.
    __device__ __forceinline__ BrickT(const KMesh &m, int slot, int b) : t(slot)
    {
        brick = b;
        const int nbx = (m.nx + BB - 1) / BB, nby = (m.ny + BB - 1) / BB;
        bx = brick % nbx;
        by = (brick / nbx) % nby;
        bz = brick / (nbx * nby);
        c0x = bx * BB;
        c0y = by * BB;
        c0z = bz * BZ;
        ncx = min(BB, m.nx - c0x);
        ncy = min(BB, m.ny - c0y);
        ncz = min(BZ, m.nz - c0z);
        tx = t & (BB - 1);
        ty = (t / BB) & (BB - 1);
        tz = t / (BB * BB);
        valid = tx < ncx && ty < ncy && tz < ncz;
        lastx = valid && tx == ncx - 1;
        lasty = valid && ty == ncy - 1;
        lastz = valid && tz == ncz - 1;
    }

    template <typename T> static __device__ __forceinline__ constexpr int lds_index(int lx, int ly, int lz)
    {
        return lx + lds_row<T>() * ly + lds_plane<T>() * lz;
    }

    // face_slot of this thread's cell node (a, b, c).
    __device__ __forceinline__ int fslot(int a, int b, int c) const
    {
        const int lex = (2 * tx + a) + BP * ((2 * ty + b) + BP * (2 * tz + c));
        if (a == 1) return lex;
        const bool xface = a == 0 ? tx == 0 : tx == BB - 1;
        return xface ? NNODES + (a ? BP * PZ : 0) + (2 * ty + b) + BP * (2 * tz + c) : lex;
    }

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
    // constrained, shared), with a, b, c compile-time constants and
    // lds_index in the layout of a staged field of T.  `shared` is
    // an int: bit 0 set if a neighbouring brick also touches the node, bit 1
    // if that happens through one of this brick's high faces (the node is
    // then finished by another brick's combine pass).  The eight
    // low nodes of every valid cell come first; the high faces, owned by the
    // last cells, follow in seven groups that each test one uniform flag.
    template <typename T = double, typename F> __device__ __forceinline__ void for_owned_nodes(const KMesh &m, F f) const
    {
        constexpr int R = lds_row<T>(), P = lds_plane<T>();
        if (!valid) return;
        const int gx0 = 2 * (c0x + tx), gy0 = 2 * (c0y + ty), gz0 = 2 * (c0z + tz);
        const int64_t g0 = node_index(m, gx0, gy0, gz0);
        const int64_t sy = m.NX, sz = (int64_t)m.NX * m.NY;
        const int l0 = lds_index<T>(2 * tx, 2 * ty, 2 * tz);
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
            f(a, b, c, l0 + a + R * b + P * c, g0 + a + sy * b + sz * c, constrained,
              (shared ? 1 : 0) | (shared_hi ? 2 : 0));
        };
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        // A brick with neighbours on all six sides and no Dirichlet face:
        // nothing is constrained, a low node is shared exactly on the
        // brick's low faces and every high node is shared.  Such bricks take
        // a copy of the visits with these flags folded in (a uniform branch;
        // 26.1 -> 25.6 us for the FP64 apply kernel at 64^3).
        const int nbx = (m.nx + BB - 1) / BB, nby = (m.ny + BB - 1) / BB, nbz = (m.nz + BZ - 1) / BZ;
        const bool inner = bx > 0 && by > 0 && bz > 0 && bx < nbx - 1 && by < nby - 1 && bz < nbz - 1 &&
                           !touches_dirichlet(m);
        auto inode = [&](auto A, auto B, auto C) {
            constexpr int a = decltype(A)::value, b = decltype(B)::value, c = decltype(C)::value;
            constexpr bool hi = a == 2 || b == 2 || c == 2;
            const bool shared = hi || (a == 0 && tx == 0) || (b == 0 && ty == 0) || (c == 0 && tz == 0);
            f(a, b, c, l0 + a + R * b + P * c, g0 + a + sy * b + sz * c, false, (shared ? 1 : 0) | (hi ? 2 : 0));
        };
        if (inner) {
            inode(I0{}, I0{}, I0{}); inode(I1{}, I0{}, I0{}); inode(I0{}, I1{}, I0{}); inode(I1{}, I1{}, I0{});
            inode(I0{}, I0{}, I1{}); inode(I1{}, I0{}, I1{}); inode(I0{}, I1{}, I1{}); inode(I1{}, I1{}, I1{});
            if (lastx) { inode(I2{}, I0{}, I0{}); inode(I2{}, I1{}, I0{}); inode(I2{}, I0{}, I1{}); inode(I2{}, I1{}, I1{}); }
            if (lasty) { inode(I0{}, I2{}, I0{}); inode(I1{}, I2{}, I0{}); inode(I0{}, I2{}, I1{}); inode(I1{}, I2{}, I1{}); }
            if (lastz) { inode(I0{}, I0{}, I2{}); inode(I1{}, I0{}, I2{}); inode(I0{}, I1{}, I2{}); inode(I1{}, I1{}, I2{}); }
            if (lastx && lasty) { inode(I2{}, I2{}, I0{}); inode(I2{}, I2{}, I1{}); }
            if (lastx && lastz) { inode(I2{}, I0{}, I2{}); inode(I2{}, I1{}, I2{}); }
            if (lasty && lastz) { inode(I0{}, I2{}, I2{}); inode(I1{}, I2{}, I2{}); }
            if (lastx && lasty && lastz) inode(I2{}, I2{}, I2{});
            return;
        }
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


    // Nodal fields are read through buffer resources based at the brick's
    // first node (uniform over the workgroup): node (2tx + a, 2ty + b,
    // 2tz + c) of the thread's cell lies at byte offset vo + a sizeof(T)
    // (per thread, immediate) plus b sy + c sz (uniform), so the loads need
    // no per-node 64-bit address arithmetic.  The brick's nodes span less
    // than 2^32 bytes from its first node; the records limit is the rest of
    // the array.  nodal_rsrc is the resource, nodal_vo the per-thread offset.
    template <typename T>
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t nodal_rsrc(const KMesh &m, const T *g) const
    {
        static_assert(sizeof(T) == 8 || sizeof(T) == 4, "FP64 or FP32 nodal arrays");
        const int64_t o = node_index(m, 2 * c0x, 2 * c0y, 2 * c0z);
        const int64_t rem = ((int64_t)m.NX * m.NY * m.NZ - o) * (int64_t)sizeof(T);
        const int nrec = (int)(unsigned)(rem > 0xFFFFFFFFll ? 0xFFFFFFFFll : rem);
        constexpr int kFormat = 0x00020000; // buffer descriptor word 3 for the gfx9 family
        return __builtin_amdgcn_make_buffer_rsrc((void *)(g + o), 0, nrec, kFormat);
    }
    template <typename T> __device__ __forceinline__ unsigned nodal_vo(const KMesh &m) const
    {
        return (unsigned)sizeof(T) * (unsigned)(2 * tx + m.NX * (2 * ty + m.NY * 2 * tz));
    }
    template <typename T>
    static __device__ __forceinline__ T nodal_load(__amdgpu_buffer_rsrc_t r, unsigned vofs, unsigned sofs)
    {
        if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, vofs, sofs, 0));
        else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, vofs, sofs, 0));
    }

    // Staging reads all 27 nodes of the thread's cell (of the brick's first
    // cell for a thread without one) and writes them to LDS.  A node that
    // several cells of the brick share is written by each of them with the
    // same value, so the staging needs no ownership test and no branches;
    // every read lies inside the mesh.
    template <typename T> __device__ __forceinline__ unsigned stage_vo(const KMesh &m) const
    {
        return valid ? nodal_vo<T>(m) : 0u;
    }
    template <typename T> __device__ __forceinline__ int stage_l0() const
    {
        return valid ? lds_index<T>(2 * tx, 2 * ty, 2 * tz) : 0;
    }

    // Stage a nodal field into LDS; Dirichlet nodes read as zero if mask.
    template <typename T>
    __device__ __forceinline__ void load(const KMesh &m, const T *__restrict__ g, T *lds, bool mask) const
    {
        const __amdgpu_buffer_rsrc_t r = nodal_rsrc(m, g);
        const unsigned vo = stage_vo<T>(m), sy = (unsigned)sizeof(T) * (unsigned)m.NX, sz = sy * (unsigned)m.NY;
        const int l0 = stage_l0<T>();
        constexpr int R = lds_row<T>(), P = lds_plane<T>();
        const unsigned f6 = mask ? m.dirichlet : 0u;
        const int gx0 = 2 * (c0x + (valid ? tx : 0)), gy0 = 2 * (c0y + (valid ? ty : 0)),
                  gz0 = 2 * (c0z + (valid ? tz : 0));
        const bool dx0 = (f6 & 1u) && gx0 == 0, dx2 = (f6 & 2u) && gx0 + 2 == m.NX - 1;
        const bool dy0 = (f6 & 4u) && gy0 == 0, dy2 = (f6 & 8u) && gy0 + 2 == m.NY - 1;
        const bool dz0 = (f6 & 16u) && gz0 == 0, dz2 = (f6 & 32u) && gz0 + 2 == m.NZ - 1;
        T v[27];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    v[a + 3 * b + 9 * c] = nodal_load<T>(r, vo + (unsigned)(a * sizeof(T)), b * sy + c * sz);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const bool k = (a == 0 && dx0) || (a == 2 && dx2) || (b == 0 && dy0) || (b == 2 && dy2) ||
                                   (c == 0 && dz0) || (c == 2 && dz2);
                    lds[l0 + a + R * b + P * c] = k ? T(0) : v[a + 3 * b + 9 * c];
                }
    }

    // Stage NF (1 or 2) nodal fields into LDS, unmasked, every read issued
    // before the first LDS write.
    template <int NF, typename T>
    __device__ __forceinline__ void stage_fields(const KMesh &m, const T *__restrict__ g0, T *l0s,
                                                 const T *__restrict__ g1, T *l1s) const
    {
        const __amdgpu_buffer_rsrc_t r0 = nodal_rsrc(m, g0), r1 = nodal_rsrc(m, NF == 2 ? g1 : g0);
        const unsigned vo = stage_vo<T>(m), sy = (unsigned)sizeof(T) * (unsigned)m.NX, sz = sy * (unsigned)m.NY;
        const int l0 = stage_l0<T>();
        constexpr int R = lds_row<T>(), P = lds_plane<T>();
        T v0[27], v1[27];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const unsigned vofs = vo + (unsigned)(a * sizeof(T)), sofs = b * sy + c * sz;
                    v0[a + 3 * b + 9 * c] = nodal_load<T>(r0, vofs, sofs);
                    if constexpr (NF == 2) v1[a + 3 * b + 9 * c] = nodal_load<T>(r1, vofs, sofs);
                }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int l = l0 + a + R * b + P * c;
                    l0s[l] = v0[a + 3 * b + 9 * c];
                    if constexpr (NF == 2) l1s[l] = v1[a + 3 * b + 9 * c];
                }
    }
    // Node-parallel staging over a workgroup of WG threads (tid = the
    // thread's index in it) of NF fields of 8-byte entries: field f is read
    // from src[f] into the LDS region dst[f]; with MASK, a field with bit f
    // of maskbits set reads its Dirichlet nodes as zero.  Thread tid takes
    // the node column l_x = tid mod 9 of the rows (l_y, l_z) = row0 + RPI k,
    // row0 = tid div 9 and RPI = WG div 9 rows per step (the WG mod 9 threads
    // left over idle), so each step reads RPI whole 9-node rows, contiguous
    // along x, and the row index advances by constant steps (no per-node
    // division or multiply).  Every brick node is read once; all reads are
    // issued before the first LDS write.  Nodes beyond a clipped brick's valid
    // range are staged too: their reads stay inside the array or fall beyond
    // the buffer resource's range and read as zero, and no valid cell reads
    // their LDS slots.  Steps past the last row write to the row padding
    // (slot 9 of row 0), which nothing reads.
    template <int WG, int NF, bool MASK, typename T>
    __device__ __forceinline__ void stage_rows(const KMesh &m, int tid, const T *const (&src)[NF],
                                               T *const (&dst)[NF], unsigned maskbits) const
    {
        static_assert(sizeof(T) == 8, "8-byte entries (padded LDS rows)");
        constexpr int R = lds_row<T>(), P = lds_plane<T>();
        static_assert(R > BP, "the padding slot of row 0 takes the writes of the idle steps");
        constexpr int RPI = WG / BP, K = (BP * PZ + RPI - 1) / RPI;
        constexpr int DLY = RPI % BP, DLZ = RPI / BP;
        __amdgpu_buffer_rsrc_t rs[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) rs[f] = nodal_rsrc(m, src[f]);
        const unsigned NX = m.NX, NXY = (unsigned)m.NX * m.NY;
        asm volatile("" : "+v"(tid)); // set up per call: nothing kept live across stagings
        const int lx = tid % BP, row0 = tid / BP;
        const bool active = tid < RPI * BP;
        int ly = row0 % BP, lz = row0 / BP;
        unsigned vofs = 8u * ((unsigned)lx + NX * (unsigned)ly + NXY * (unsigned)lz);
        int lo = lx + R * ly + P * lz;
        const unsigned vstep = 8u * (DLY * NX + DLZ * NXY), vcarry = 8u * (NXY - BP * NX);
        T v[K][NF];
        int slot[K];
        bool con[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (k > 0) {
                ly += DLY;
                lz += DLZ;
                vofs += vstep;
                lo += DLY * R + DLZ * P;
                if (ly >= BP) {
                    ly -= BP;
                    lz += 1;
                    vofs += vcarry;
                    lo += P - BP * R;
                }
            }
            const bool ok = active && lz < PZ;
            slot[k] = ok ? lo : BP; // padding slot of row 0
            con[k] = MASK && ok && node_constrained(m, 2 * c0x + lx, 2 * c0y + ly, 2 * c0z + lz);
#pragma unroll
            for (int f = 0; f < NF; ++f) v[k][f] = nodal_load<T>(rs[f], ok ? vofs : 0u, 0);
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int f = 0; f < NF; ++f) dst[f][slot[k]] = (MASK && ((maskbits >> f) & 1u) && con[k]) ? T(0) : v[k][f];
    }

    // The brick's NF (1 or 2) unmasked 8-byte fields, staged by its NT lanes.
    template <int NF, typename T>
    __device__ __forceinline__ void stage_nodes(const KMesh &m, const T *__restrict__ g0, T *l0s,
                                                const T *__restrict__ g1, T *l1s) const
    {
        if constexpr (NF == 1) {
            const T *src[1] = {g0};
            T *const dst[1] = {l0s};
            stage_rows<NT, 1, false, T>(m, t, src, dst, 0u);
        } else {
            const T *src[2] = {g0, g1};
            T *const dst[2] = {l0s, l1s};
            stage_rows<NT, 2, false, T>(m, t, src, dst, 0u);
        }
    }

    // NF FP64 fields over a workgroup of WG threads; bit f of maskbits: field f
    // reads its Dirichlet nodes as zero.
    template <int WG, int NF>
    __device__ __forceinline__ void stage_nodes_wg(const KMesh &m, int tid, const double *const (&src)[NF],
                                                   double *const (&dst)[NF], unsigned maskbits) const
    {
        if (maskbits) stage_rows<WG, NF, true, double>(m, tid, src, dst, maskbits);
        else stage_rows<WG, NF, false, double>(m, tid, src, dst, 0u);
    }

    template <typename T> __device__ __forceinline__ void load_fields(const KMesh &m, const T *g0, T *l0s) const
    {
        stage_fields<1, T>(m, g0, l0s, nullptr, nullptr);
    }
    template <typename T>
    __device__ __forceinline__ void load_fields(const KMesh &m, const T *g0, T *l0s, const T *g1, T *l1s) const
    {
        stage_fields<2, T>(m, g0, l0s, g1, l1s);
    }

    // The cell's 27 nodal values with its Dirichlet nodes read as zero (the
    // constrained columns are removed); bricks away from Dirichlet faces
    // skip the test (uniform branch).
    template <typename T> __device__ __forceinline__ void gather27_dirichlet(const KMesh &m, const T *lds, T *v) const
    {
        gather27(lds, v);
        if (!touches_dirichlet(m)) return;
        const unsigned f6 = m.dirichlet;
        const int gx0 = 2 * (c0x + tx), gy0 = 2 * (c0y + ty), gz0 = 2 * (c0z + tz);
        const bool dx0 = (f6 & 1u) && gx0 == 0, dx2 = (f6 & 2u) && gx0 + 2 == m.NX - 1;
        const bool dy0 = (f6 & 4u) && gy0 == 0, dy2 = (f6 & 8u) && gy0 + 2 == m.NY - 1;
        const bool dz0 = (f6 & 16u) && gz0 == 0, dz2 = (f6 & 32u) && gz0 + 2 == m.NZ - 1;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const bool k = (a == 0 && dx0) || (a == 2 && dx2) || (b == 0 && dy0) || (b == 2 && dy2) ||
                                   (c == 0 && dz0) || (c == 2 && dz2);
                    v[a + 3 * b + 9 * c] = k ? T(0) : v[a + 3 * b + 9 * c];
                }
    }

    // The cell's 27 nodal values from LDS (zero for threads without a cell).
    template <typename T> __device__ __forceinline__ void gather27(const T *lds, T *v) const
    {
        const int l0 = valid ? lds_index<T>(2 * tx, 2 * ty, 2 * tz) : 0;
        constexpr int R = lds_row<T>(), P = lds_plane<T>();
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int a = 0; a < 3; ++a) v[a + 3 * b + 9 * c] = lds[l0 + a + R * b + P * c];
    }

    // Cell results, node-major: E[local * NT + thread].  A thread without a
    // cell stores whatever it computed: node_sum reads only the lower
    // neighbours of a valid cell within the brick, and those are valid too.
    template <typename T> __device__ __forceinline__ void store_cell(T *E, const T *v) const
    {
#pragma unroll
        for (int i = 0; i < 27; ++i) E[i * NT + t] = v[i];
    }

    // Lane shift within the 16-lane rows of the wavefront (DPP row_shr:S):
    // lane i takes lane i - S of its row, the first S lanes of a row take 0.
    template <int S, typename T> static __device__ __forceinline__ T row_shr(T v)
    {
        static_assert(S >= 1 && S <= 15, "row shift");
        constexpr int ctrl = 0x110 + S;
        if constexpr (sizeof(T) == 8) {
            const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
            const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, ctrl, 0xF, 0xF, true);
            const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), ctrl, 0xF, 0xF, true);
            return __builtin_bit_cast(T, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
        } else {
            return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), ctrl, 0xF, 0xF, true));
        }
    }

    // Node sums in registers.  On entry u holds this cell's 27 contributions;
    // on exit u[a + 3b + 9c] is the sum over the brick's cells containing
    // that node for every node the cell owns (the entries of index 2 of a
    // cell that is not the last in that direction are partial).  Cells are
    // lanes t = tx + 4 ty + 16 tz, so the low neighbour in x is lane t - 1
    // and in y lane t - 4, both in the same 16-lane row (a DPP row shift;
    // the first cell of an x line is masked, the first of a y line is at a
    // row's start and takes zero), and in z lane t - 16, exchanged through
    // LDS (xch, 9 NT values; with two wavefronts per brick the exchange
    // between tz = 3 and tz = 4 crosses them).  The sums run x, then y, then z: a fixed order.
    // All lanes of the wavefront must call it.
    template <typename T> __device__ __forceinline__ void assemble27(T *u, T *xch) const
    {
#pragma unroll
        for (int i = 0; i < 9; ++i) { // x: (b, c) = (i % 3, i / 3)
            const T nb = row_shr<1>(u[2 + 3 * i]);
            u[3 * i] += tx > 0 ? nb : T(0);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int a = 0; a < 3; ++a) u[a + 9 * c] += row_shr<4>(u[a + 6 + 9 * c]);
#pragma unroll
        for (int i = 0; i < 9; ++i) xch[i * NT + t] = u[18 + i];
        __syncthreads();
        const int src = tz > 0 ? t - BB * BB : t;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const T nb = xch[i * NT + src];
            u[i] += tz > 0 ? nb : T(0);
        }
    }

    // Sum over the brick's cells containing local node (a, b, c) of this
    // thread's cell: the cell itself and, for index 0 in a direction, the
    // neighbour on the low side (local index 2 there).  Branch free: a
    // missing neighbour (brick edge) reads this cell's slot, weighted by 0.
    template <typename T> __device__ __forceinline__ T node_sum(const T *E, int a, int b, int c) const
    {
        T s = E[(a + 3 * b + 9 * c) * NT + t];
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
                    s += (ok ? T(1) : T(0)) * E[loc * NT + nb];
                }
        return s;
    }
};

using Brick = BrickT<BB>;

// ---------------------------------------------------------------------------
// Shared-node combine.  The nodes that several bricks touch lie on the
// internal brick planes of some direction.  A node's value is the sum of the
// face partials of the 2, 4 or 8 bricks containing it, in a fixed order (z
// outer, then y, then x; lower brick first).  Shared Dirichlet nodes: DMODE 1
// writes y = x (identity rows of an operator), DMODE 2 writes y = 1 (its
// diagonal), DMODE 3 writes 0 (a right-hand side), DMODE 0 sums them like
// every other node (a plain nodal field such as a gradient).  DMODE 4 is
// DMODE 2 with the reciprocal of every other sum stored (the inverse
// diagonal).
// ---------------------------------------------------------------------------

// Brick-owned combine: a wavefront per 4 cells of brick depth (numbered
// like the brick kernels, XCD-contiguously).  Each shared node is finished
// by the one brick that holds it at local index 0 in every direction in
// which it is shared: the brick's nodes on its low faces that lie on
// internal brick planes, without its shared high faces (the next brick's
// low faces).  For a 4x4x4 brick with lower neighbours in x, y and z that is
// up to 64 + 56 + 49 nodes (217 for a brick at the far end of the mesh in
// every direction), at most four per lane; a 4x4x8 brick has up to
// 81 + 144 + 128 = 353 over two wavefronts, three per lane.  They are
// enumerated in three slabs: l_z = 0 (runs along x); l_y = 0 (runs along x);
// l_x = 0 (runs along y, where the x-face slots are contiguous).  The
// partials are summed in the fixed order above (the same order as a pass
// that enumerates the shared nodes flat, which this pass replaced with
// bitwise the same results); all loads of a lane's nodes are issued before
// the sums.
// Lanes that finish one brick's shared nodes: a wavefront per 4 cells of
// brick depth.
template <int BZ> struct CombineLanes {
    static constexpr int value = BNT * BZ / BB;
};

// The visit for one brick; INNER: a brick with neighbours on all six sides
// and no Dirichlet face, for which the ranges, the sharing flags and the
// slab divisions are compile-time constants and nothing is constrained.
template <typename T, bool SKIP_CONSTRAINED, int BZ, bool INNER, typename F>
__device__ __forceinline__ void combine_brick_nodes(const KMesh &m, const BrickT<BZ> &br, int nbx, int nby, int nbz,
                                                    int lane, const T *__restrict__ face, F f)
{
    using BD = BrickDims<BZ>;
    // lower neighbour: the low face is shared
    const bool fx = INNER || br.bx > 0, fy = INNER || br.by > 0, fz = INNER || br.bz > 0;
    // local range without a shared high face
    const int ex = INNER ? 2 * BB : 2 * br.ncx + (br.bx == nbx - 1 ? 1 : 0);
    const int ey = INNER ? 2 * BB : 2 * br.ncy + (br.by == nby - 1 ? 1 : 0);
    const int ez = INNER ? 2 * BZ : 2 * br.ncz + (br.bz == nbz - 1 ? 1 : 0);
    const int z0 = fz ? 1 : 0, y0 = fy ? 1 : 0;
    const int nzs = fz ? ex * ey : 0, nys = fy ? ex * (ez - z0) : 0, nxs = fx ? (ey - y0) * (ez - z0) : 0;
    const int tot = nzs + nys + nxs;
    // small exact divisions: floor((j + 1/2) / w) for j < 512, w <= 9
    const float iex = 1.0f / (float)ex, iw = 1.0f / (float)(ey - y0);
    auto div = [&](int j, int w, float iw_) { return INNER ? j / w : (int)(((float)j + 0.5f) * iw_); };
    // nodes per lane: BP^2 + 2 BP (PZ - 1) at most over the brick's lanes
    constexpr int L = CombineLanes<BZ>::value;
    constexpr int K = (BP * BP + 2 * BP * (BD::PZ - 1) + L - 1) / L;
    bool has[K], con[K];
    int64_t g[K];
    T v[K][8];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int j = lane + L * k;
        has[k] = j < tot;
        int lx = 0, ly = 0, lz = 0;
        if (j < nzs) {
            ly = div(j, ex, iex);
            lx = j - ly * ex;
        } else if ((j -= nzs) < nys) {
            const int q = div(j, ex, iex);
            lz = z0 + q;
            lx = j - q * ex;
        } else {
            j -= nys;
            const int w = ey - y0, q = div(j, w, iw);
            lz = z0 + q;
            ly = y0 + j - q * w;
        }
        if (!has[k]) lx = ly = lz = 0;
        const int gx = 2 * br.c0x + lx, gy = 2 * br.c0y + ly, gz = 2 * br.c0z + lz;
        con[k] = !INNER && has[k] && node_constrained(m, gx, gy, gz);
        g[k] = node_index(m, gx, gy, gz);
        const bool read = has[k] && !(SKIP_CONSTRAINED && con[k]);
        const bool sx = lx == 0 && fx, sy = ly == 0 && fy, sz = lz == 0 && fz;
        const int kx0 = sx ? br.bx - 1 : br.bx, lx0 = sx ? 2 * BB : lx;
        const int ky0 = sy ? br.by - 1 : br.by, ly0 = sy ? 2 * BB : ly;
        const int kz0 = sz ? br.bz - 1 : br.bz, lz0 = sz ? 2 * BZ : lz;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int ex_ = e & 1, ey_ = (e >> 1) & 1, ez_ = e >> 2;
            v[k][e] = T(0);
            if (read && (!ex_ || sx) && (!ey_ || sy) && (!ez_ || sz)) {
                const int b = (kx0 + ex_) + nbx * ((ky0 + ey_) + nby * (kz0 + ez_));
                v[k][e] = face[(int64_t)b * BD::NFACE + face_slot<BZ>(ex_ ? 0 : lx0, ey_ ? 0 : ly0, ez_ ? 0 : lz0)];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (!has[k]) continue;
        T s = v[k][0];
#pragma unroll
        for (int e = 1; e < 8; ++e) s += v[k][e];
        f(g[k], con[k], (SKIP_CONSTRAINED && con[k]) ? T(0) : s);
    }
}

template <typename T, bool SKIP_CONSTRAINED, int BZ = BB, typename F>
__device__ __forceinline__ void combine_brick_visit(const KMesh &m, int brick, int lane, const T *__restrict__ face,
                                                    F f)
{
    const BrickT<BZ> br(m, lane, brick);
    const int nbx = (m.nx + BB - 1) / BB, nby = (m.ny + BB - 1) / BB, nbz = (m.nz + BZ - 1) / BZ;
    const bool inner = br.bx > 0 && br.by > 0 && br.bz > 0 && br.bx < nbx - 1 && br.by < nby - 1 &&
                       br.bz < nbz - 1 && !br.touches_dirichlet(m);
    if (inner) combine_brick_nodes<T, SKIP_CONSTRAINED, BZ, true>(m, br, nbx, nby, nbz, lane, face, f);
    else combine_brick_nodes<T, SKIP_CONSTRAINED, BZ, false>(m, br, nbx, nby, nbz, lane, face, f);
}

// Threads of a brick-combine workgroup: 4 bricks of 4x4x4 cells, 2 of 4x4x8.
constexpr int CBW = 4;

template <typename T, int DMODE, int BZ = BB>
__device__ __forceinline__ void combine_brick(const KMesh &m, const T *__restrict__ face, const T *__restrict__ x,
                                              T *__restrict__ y)
{
    constexpr int L = CombineLanes<BZ>::value, BPW = BNT * CBW / L; // bricks per workgroup
    const int brick = Brick::xcd_index() * BPW + (int)threadIdx.x / L;
    if (brick >= n_bricks<BZ>(m)) return; // whole wavefronts; no barrier follows in them
    combine_brick_visit<T, DMODE != 0, BZ>(m, brick, (int)threadIdx.x % L, face,
                                           [&](int64_t g, bool constrained, T s) {
        if (DMODE != 0 && constrained) y[g] = DMODE == 1 ? x[g] : ((DMODE == 2 || DMODE == 4) ? T(1) : T(0));
        else y[g] = DMODE == 4 ? T(1) / s : s;
    });
}

} // namespace mf
