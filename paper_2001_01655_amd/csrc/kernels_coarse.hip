// Geometric coarse levels.
//
// Galerkin operators A^{l+1} = P^T A^l P (Sec. 3.2) are formed element by
// element: every coarse element E holds the dense matrix
//     K_E = sum_{children c} Q~_c^T K_c Q~_c,
// where Q_c interpolates E's corner values to child c's corners with the
// coarse shape functions (the restriction of P to one element, exact because
// a fine element's corners only interpolate from its parent's corners) and
// Q~_c drops supported fine dofs on the finest level.  The level operator is
// then stored as a structured stencil: node I keeps, for each of its 3^dim
// neighbour offsets, the dense dim x dim block (zero outside the grid), laid
// out [offset][entry][node] so consecutive threads read consecutive words.
#include "tm_device.h"

namespace tmi {

// --------------------------------------------------------------- Galerkin
// Coarse element E: K_E = sum over its children c of Q_c^T K_c Q_c (masked
// rows/columns of supported fine dofs dropped).  Per axis a coarse element has
// two children (fine elements 2X, 2X+1), or one (the last coarse element of an
// odd count, which is the fine element 2X itself); Q_c is the tensor product of
// the per-axis weights of the child's two fine nodes on the coarse element's
// two nodes.
__device__ __forceinline__ double axis_w(int kind, int a, int b) {
    // kind 0 / 1: first / second half (fine node 2X + kind + a); kind 2: whole
    if (kind == 2) return a == b ? 1.0 : 0.0;
    const int d = kind + a - 2 * b;
    return d == 0 ? 1.0 : (d == 1 || d == -1) ? 0.5 : 0.0;
}

// corner a's coordinate bit on axis ax (local order loc2 / loc3)
__device__ __forceinline__ int gal_bit(int a, int ax) {
    return ax == 0 ? (a == 1 || a == 2 || a == 5 || a == 6) : ax == 1 ? (a == 2 || a == 3 || a == 6 || a == 7) : a >= 4;
}

// Unit Galerkin products G_k = Q_k^T KE Q_k for every child kind triple
// k = kx + 3 ky (+ 9 kz), kind per axis 0 / 1 (first / second half) or 2
// (whole): a first coarse level whose children touch no supported dof is
// sum_c E_c G_k(c), since a fine element's matrix there is E_e KE.
template <int DIM>
__global__ void k_galerkin_unit(const double* __restrict__ KE, double* __restrict__ G) {
    constexpr int NPE = 1 << DIM, ND = DIM * NPE;
    const int k = blockIdx.x, t = threadIdx.x;
    const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
    const int rp = t / ND, sp = t % ND;
    const int b = rp / DIM, i = rp % DIM, bq = sp / DIM, j = sp % DIM;
    auto w = [&](int a, int c) {
        return axis_w(kx, gal_bit(a, 0), gal_bit(c, 0)) * axis_w(ky, gal_bit(a, 1), gal_bit(c, 1)) *
               (DIM == 3 ? axis_w(kz, gal_bit(a, 2), gal_bit(c, 2)) : 1.0);
    };
    double v = 0.0;
    for (int a = 0; a < NPE; ++a) {
        const double wa = w(a, b);
        if (wa == 0.0) continue;
        double u = 0.0;
        for (int a2 = 0; a2 < NPE; ++a2) u += KE[(DIM * a + i) * ND + DIM * a2 + j] * w(a2, bq);
        v += wa * u;
    }
    G[(int64_t)k * ND * ND + t] = v;
}

void launch_galerkin_unit(int dim, const double* KE, double* G, hipStream_t s) {
    if (dim == 3)
        hipLaunchKernelGGL(k_galerkin_unit<3>, dim3(27), dim3(576), 0, s, KE, G);
    else
        hipLaunchKernelGGL(k_galerkin_unit<2>, dim3(9), dim3(64), 0, s, KE, G);
}

template <int DIM>
__global__ void k_galerkin(const double* __restrict__ child, const double* __restrict__ E,
                           const double* __restrict__ KE, const double* __restrict__ G,
                           const uint8_t* __restrict__ nm, int fnx, int fny, int fnz, int cnx, int cny,
                           int cnz, double* __restrict__ parent) {
    constexpr int NPE = 1 << DIM, ND = DIM * NPE;
    __shared__ double Kc[ND * ND];
    __shared__ double Tm[ND * ND];
    __shared__ double q[NPE * NPE];
    __shared__ double msk[NPE * DIM];
    const int64_t pe = blockIdx.x;
    const int X = (int)(pe % cnx);
    const int Y = (int)((pe / cnx) % cny);
    const int Z = DIM == 3 ? (int)(pe / ((int64_t)cnx * cny)) : 0;
    const int t = threadIdx.x;
    const int r = t / ND, s = t % ND;
    // children per axis: 2, or 1 (whole) for the last element of an odd count
    const bool wx = 2 * X + 1 == fnx, wy = 2 * Y + 1 == fny, wz = DIM == 3 && 2 * Z + 1 == fnz;
    if (!child) {
        // first coarse level: children are E_e KE; without supported dofs among
        // the parent's fine nodes the product is sum_c E_c G_k(c)
        int touched = 0;
        if (nm && t < (DIM == 3 ? 27 : 9)) {
            const int nx_ = 2 * X + t % 3, ny_ = 2 * Y + (t / 3) % 3, nz_ = 2 * Z + t / 9;
            if (nx_ <= fnx && ny_ <= fny && (DIM == 2 || nz_ <= fnz)) {
                const int64_t fnode = DIM == 3 ? ((int64_t)nz_ * (fny + 1) + ny_) * (fnx + 1) + nx_
                                               : (int64_t)ny_ * (fnx + 1) + nx_;
                touched = nm[fnode] != 0;
            }
        }
        if (!__syncthreads_or(touched)) {
            double acc = 0.0;
            for (int c = 0; c < NPE; ++c) {
                const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
                if ((wx && cx) || (wy && cy) || (wz && cz)) continue;
                const int kx = wx ? 2 : cx, ky = wy ? 2 : cy, kz = wz ? 2 : cz;
                const int gx = 2 * X + cx, gy = 2 * Y + cy, gz = 2 * Z + cz;
                const int64_t ce = DIM == 3 ? ((int64_t)gz * fny + gy) * fnx + gx : (int64_t)gy * fnx + gx;
                acc += E[ce] * G[(int64_t)(kx + 3 * ky + 9 * kz) * ND * ND + t];
            }
            parent[pe * ND * ND + t] = acc;
            return;
        }
    }
    double acc = 0.0;
    for (int c = 0; c < NPE; ++c) {
        const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;   // child position bits
        if ((wx && cx) || (wy && cy) || (wz && cz)) continue;         // block-uniform
        const int kx = wx ? 2 : cx, ky = wy ? 2 : cy, kz = wz ? 2 : cz;
        const int gx = 2 * X + cx, gy = 2 * Y + cy, gz = 2 * Z + cz;
        const int64_t ce = DIM == 3 ? ((int64_t)gz * fny + gy) * fnx + gx : (int64_t)gy * fnx + gx;
        if (child) {
            Kc[t] = child[ce * ND * ND + t];
        } else {
            Kc[t] = E[ce] * KE[t];
        }
        if (t < NPE * NPE) {
            // q[a][b]: weight of the child's local corner a on the coarse corner b
            const int a = t / NPE, b = t % NPE;
            const int ax = (a == 1 || a == 2 || a == 5 || a == 6) ? 1 : 0;
            const int ay = (a == 2 || a == 3 || a == 6 || a == 7) ? 1 : 0;
            const int az = a >= 4 ? 1 : 0;
            const int bx = (b == 1 || b == 2 || b == 5 || b == 6) ? 1 : 0;
            const int by = (b == 2 || b == 3 || b == 6 || b == 7) ? 1 : 0;
            const int bz = b >= 4 ? 1 : 0;
            q[t] = axis_w(kx, ax, bx) * axis_w(ky, ay, by) * (DIM == 3 ? axis_w(kz, az, bz) : 1.0);
        }
        if (t < NPE * DIM) {
            const int a = t / DIM, comp = t % DIM;
            double m = 1.0;
            if (nm) {
                // child-local corner a -> fine node
                const int ax = (a == 1 || a == 2 || a == 5 || a == 6) ? 1 : 0;
                const int ay = (a == 2 || a == 3 || a == 6 || a == 7) ? 1 : 0;
                const int az = a >= 4 ? 1 : 0;
                const int64_t fnode = DIM == 3
                    ? ((int64_t)(gz + az) * (fny + 1) + (gy + ay)) * (fnx + 1) + gx + ax
                    : (int64_t)(gy + ay) * (fnx + 1) + gx + ax;
                if (nm[fnode] & (1u << comp)) m = 0.0;
            }
            msk[t] = m;
        }
        __syncthreads();
        {   // T[r][s] = sum_a' Kc[r][DIM a' + j] m[a'][j] q[a'][b'],  s = DIM b' + j
            const int bp = s / DIM, j = s % DIM;
            double v = 0.0;
#pragma unroll
            for (int ap = 0; ap < NPE; ++ap)
                v += Kc[r * ND + DIM * ap + j] * (msk[ap * DIM + j] * q[ap * NPE + bp]);
            Tm[r * ND + s] = v;
        }
        __syncthreads();
        {   // K_E[r'][s] += sum_a q[a][b] m[a][i] T[DIM a + i][s],  r' = DIM b + i
            const int b = r / DIM, i = r % DIM;
            double v = 0.0;
#pragma unroll
            for (int a = 0; a < NPE; ++a) v += (q[a * NPE + b] * msk[a * DIM + i]) * Tm[(DIM * a + i) * ND + s];
            acc += v;
        }
        __syncthreads();
    }
    parent[pe * ND * ND + t] = acc;
}

void launch_galerkin_elems(const tm_hierarchy* h, int fine_level, const double* child,
                           double* parent, hipStream_t s) {
    const Level& F = h->lv[fine_level];
    const Level& C = h->lv[fine_level + 1];
    const int64_t n_par = (int64_t)C.nel[0] * C.nel[1] * (h->dim == 3 ? C.nel[2] : 1);
    const uint8_t* nm = fine_level == 0 ? F.nmask : nullptr;
    if (h->dim == 3)
        hipLaunchKernelGGL(k_galerkin<3>, dim3((unsigned)n_par), dim3(576), 0, s, child, F.E64,
                           h->KE64, h->galG, nm, F.nel[0], F.nel[1], F.nel[2], C.nel[0], C.nel[1], C.nel[2],
                           parent);
    else
        hipLaunchKernelGGL(k_galerkin<2>, dim3((unsigned)n_par), dim3(64), 0, s, child, F.E64,
                           h->KE64, h->galG, nm, F.nel[0], F.nel[1], 1, C.nel[0], C.nel[1], 1, parent);
}

// --------------------------------------------------------------- stencil assembly
// thread per (node I, neighbour offset o): block (I, I+o) = sum over the elements
// holding both nodes, in a fixed order.
template <int DIM>
__global__ void k_stencil_assemble(const double* __restrict__ elem, int nx, int ny, int nz,
                                   int64_t N, double* __restrict__ st64) {
    constexpr int NPE = 1 << DIM, ND = DIM * NPE, NST = DIM == 3 ? 27 : 9;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= N * NST) return;
    const int o = (int)(tid / N);
    const int64_t node = tid % N;
    const int NX = nx + 1, NY = ny + 1;
    const int i = (int)(node % NX);
    const int j = (int)((node / NX) % NY);
    const int k = DIM == 3 ? (int)(node / ((int64_t)NX * NY)) : 0;
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = DIM == 3 ? o / 9 - 1 : 0;
    double blk[DIM * DIM] = {};
#pragma unroll
    for (int ez = 0; ez < (DIM == 3 ? 2 : 1); ++ez)
#pragma unroll
        for (int ey = 0; ey < 2; ++ey)
#pragma unroll
            for (int ex = 0; ex < 2; ++ex) {
                // element with lower corner (i-1+ex, ...): our corner (1-ex, ...), neighbour (1-ex+ox, ...)
                const int lx = 1 - ex, ly = 1 - ey, lz = DIM == 3 ? 1 - ez : 0;
                const int mx = lx + ox, my = ly + oy, mz = lz + oz;
                if (mx < 0 || mx > 1 || my < 0 || my > 1 || mz < 0 || mz > 1) continue;
                const int gx = i - 1 + ex, gy = j - 1 + ey, gz = k - 1 + ez;
                if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) continue;
                if (DIM == 3 && (gz < 0 || gz >= nz)) continue;
                const int64_t e = DIM == 3 ? ((int64_t)gz * ny + gy) * nx + gx : (int64_t)gy * nx + gx;
                const int a = DIM == 3 ? loc3(lx, ly, lz) : loc2(lx, ly);
                const int bb = DIM == 3 ? loc3(mx, my, mz) : loc2(mx, my);
                const double* Ke = elem + e * ND * ND;
#pragma unroll
                for (int r = 0; r < DIM; ++r)
#pragma unroll
                    for (int c = 0; c < DIM; ++c) blk[r * DIM + c] += Ke[(DIM * a + r) * ND + DIM * bb + c];
            }
    if (o == (NST - 1) / 2) {
        // a dof with no coupling at all (exactly zero diagonal) gets a unit diagonal
#pragma unroll
        for (int r = 0; r < DIM; ++r)
            if (blk[r * DIM + r] == 0.0) blk[r * DIM + r] = 1.0;
    }
#pragma unroll
    for (int q = 0; q < DIM * DIM; ++q) {
        st64[((int64_t)o * DIM * DIM + q) * N + node] = blk[q];
    }
}

void launch_stencil_assemble(const Level& L, const double* elem, hipStream_t s) {
    const int64_t nt = L.n_nodes * L.nst;
    if (L.dim == 3)
        hipLaunchKernelGGL(k_stencil_assemble<3>, dim3(grid_for(nt)), dim3(WG), 0, s, elem, L.nel[0],
                           L.nel[1], L.nel[2], L.n_nodes, L.st64);
    else
        hipLaunchKernelGGL(k_stencil_assemble<2>, dim3(grid_for(nt)), dim3(WG), 0, s, elem, L.nel[0],
                           L.nel[1], 1, L.n_nodes, L.st64);
}

// --------------------------------------------------------------- symmetric form
// Compact V-cycle copy: q < NU*BB holds entry e of the block towards upper
// neighbour u (grid offset index (NST+1)/2 + u); the last DIM(DIM+1)/2 hold the
// diagonal block's upper triangle, row by row.
template <int DIM>
__global__ void k_stencil_compact(const double* __restrict__ st64, int64_t N, double* __restrict__ c64,
                                  float* __restrict__ c32) {
    constexpr int NST = DIM == 3 ? 27 : 9, BB = DIM * DIM, NU = (NST - 1) / 2;
    constexpr int NQ = NU * BB + DIM * (DIM + 1) / 2;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= N * NQ) return;
    const int q = (int)(tid / N);
    const int64_t node = tid % N;
    int src;
    if (q < NU * BB) {
        src = (NU + 1 + q / BB) * BB + q % BB;
    } else {
        int t = q - NU * BB, r = 0;
        while (t >= DIM - r) {
            t -= DIM - r;
            ++r;
        }
        src = NU * BB + r * DIM + r + t;  // centre block, row r, column r + t
    }
    const double v = st64[(int64_t)src * N + node];
    c64[(int64_t)q * N + node] = v;
    c32[(int64_t)q * N + node] = (float)v;
}

void launch_stencil_compact(const Level& L, hipStream_t s) {
    const int64_t nt = L.n_nodes * L.nq;
    if (L.dim == 3)
        hipLaunchKernelGGL(k_stencil_compact<3>, dim3(grid_for(nt)), dim3(WG), 0, s, L.st64, L.n_nodes, L.stc64,
                           L.stc32);
    else
        hipLaunchKernelGGL(k_stencil_compact<2>, dim3(grid_for(nt)), dim3(WG), 0, s, L.st64, L.n_nodes, L.stc64,
                           L.stc32);
}

// --------------------------------------------------------------- stencil diagonal
template <int DIM>
__global__ void k_stencil_dinv(const double* __restrict__ st, int64_t N, int point,
                               double* __restrict__ d64, float* __restrict__ d32, int* flags) {
    constexpr int SELF = DIM == 3 ? 13 : 4;
    const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= N) return;
    double D[DIM][DIM];
#pragma unroll
    for (int r = 0; r < DIM; ++r)
#pragma unroll
        for (int c = 0; c < DIM; ++c) D[r][c] = st[((int64_t)SELF * DIM * DIM + r * DIM + c) * N + node];
    // a dof whose diagonal is exactly zero (no coarse coupling at all) gets a unit row
#pragma unroll
    for (int r = 0; r < DIM; ++r)
        if (D[r][r] == 0.0) D[r][r] = 1.0;
    store_dinv<DIM>(D, point, node, N, d64, d32, flags);
}

void launch_stencil_dinv(const Level& L, int point_jacobi, int* flags, hipStream_t s) {
    if (L.dim == 3)
        hipLaunchKernelGGL(k_stencil_dinv<3>, dim3(grid_for(L.n_nodes)), dim3(WG), 0, s, L.st64,
                           L.n_nodes, point_jacobi, L.dinv64, L.dinv32, flags);
    else
        hipLaunchKernelGGL(k_stencil_dinv<2>, dim3(grid_for(L.n_nodes)), dim3(WG), 0, s, L.st64,
                           L.n_nodes, point_jacobi, L.dinv64, L.dinv32, flags);
}

// --------------------------------------------------------------- stencil operator
// y = A x from the symmetric form: the diagonal block, the stored blocks towards
// the upper neighbours, and for each lower neighbour m the transpose of m's
// stored block towards this node (A is symmetric).  Neighbours outside the grid
// have zero stored blocks (upper) or have their x masked to zero (lower); all
// loads use clamped, in-bounds indices, with no branches.
// Offset visited at step t of the neighbour loop: the mirror pair
// (NU-1-q, NU+1+q) for t = 2q, 2q+1 (both read stored row group q of the
// symmetric form: the upper offset as the node's own block, the lower one as
// the neighbour's block, transposed), the centre NU last.
template <int NU>
__host__ __device__ constexpr int pair_order(int t) {
    return t >= 2 * NU ? NU : ((t & 1) ? NU + 1 + t / 2 : NU - 1 - t / 2);
}
// every offset once, and the two offsets of a pair read the same row group:
// the lower one reads row NU-1-o, the upper one row o-NU-1
template <int NU>
constexpr bool pair_order_ok() {
    bool seen[2 * NU + 1] = {};
    for (int t = 0; t <= 2 * NU; ++t) {
        const int o = pair_order<NU>(t);
        if (o < 0 || o > 2 * NU || seen[o]) return false;
        seen[o] = true;
    }
    for (int q = 0; q < NU; ++q)
        if (NU - 1 - pair_order<NU>(2 * q) != q || pair_order<NU>(2 * q + 1) - NU - 1 != q) return false;
    return true;
}
static_assert(pair_order_ok<13>() && pair_order_ok<4>(), "stencil visiting order");

template <typename T, int DIM, int OP, int G, int NB>
__global__ __launch_bounds__(WG) void k_stencil_op(const Pack<OpA<T>, NB> pk, int nx, int ny, int nz, int64_t N,
                                                   T omega, double c1, double c2) {
    const OpA<T>& A_ = lane_of(pk);
    const T* __restrict__ st = A_.E;
    const T* __restrict__ x = A_.x;
    const T* __restrict__ b = A_.b;
    T* __restrict__ y = A_.y;
    const T* __restrict__ dinv = A_.dinv;
    const int* __restrict__ done = A_.done;
    ChebArgs ch;
    ch.din = A_.din;
    ch.dout = A_.dout;
    ch.c1 = c1;
    ch.c2 = c2;
    if (done && *done) return;
    const int64_t node = xcd_block() * WG + threadIdx.x;
    if (node >= N) return;
    constexpr int BB = DIM * DIM, NST = DIM == 3 ? 27 : 9, NU = (NST - 1) / 2;
    constexpr int NQ = NU * BB + DIM * (DIM + 1) / 2;
    const int NX = nx + 1, NY = ny + 1, NZ = nz + 1;
    const int i = (int)(node % NX);
    const int j = (int)((node / NX) % NY);
    const int k = DIM == 3 ? (int)(node / ((int64_t)NX * NY)) : 0;
    // 32-bit byte offsets through buffer descriptors (level sizes < 2 GB)
    const auto sr = buf_rsrc(st, (int64_t)N * NQ * sizeof(T));
    const auto xr = buf_rsrc(x, (int64_t)N * DIM * sizeof(T));
    const uint32_t un = (uint32_t)node, uN = (uint32_t)N;
    uint32_t ci[3], cj[3], ck[3];
    bool ii[3], ij[3], ik[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ci[d] = (uint32_t)min(max(i + d - 1, 0), NX - 1);
        cj[d] = (uint32_t)min(max(j + d - 1, 0), NY - 1);
        ck[d] = DIM == 3 ? (uint32_t)min(max(k + d - 1, 0), NZ - 1) : 0u;
        ii[d] = i + d - 1 >= 0 && i + d - 1 < NX;
        ij[d] = j + d - 1 >= 0 && j + d - 1 < NY;
        ik[d] = DIM == 2 || (k + d - 1 >= 0 && k + d - 1 < NZ);
    }
    T acc[DIM] = {};
    T xo[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) xo[c] = bld<T>(xr, (DIM * un + c) * (uint32_t)sizeof(T));
    // diagonal block (upper triangle stored)
    {
        int q = NU * BB;
#pragma unroll
        for (int r = 0; r < DIM; ++r)
#pragma unroll
            for (int c = r; c < DIM; ++c, ++q) {
                const T a = bld<T>(sr, ((uint32_t)q * uN + un) * (uint32_t)sizeof(T));
                acc[r] += a * xo[c];
                if (c != r) acc[c] += a * xo[r];
            }
    }
    // neighbours in groups of G: all loads of a group are issued before its
    // arithmetic (the scheduling barrier keeps them batched), so G * (BB + DIM)
    // loads are in flight per wave (small levels: larger groups, fewer round
    // trips, since occupancy no longer hides the latency).  Offsets are visited
    // in mirror pairs (pair_order), so a stored row is read as an own block and
    // as a neighbour's transposed block at about the same time.
#pragma unroll
    for (int g0 = 0; g0 < NST; g0 += G) {
        T xv[G][DIM], blk[G][BB];
#pragma unroll
        for (int gg = 0; gg < G; ++gg) {
            if (g0 + gg >= NST) continue;
            const int o = pair_order<NU>(g0 + gg);
            if (o == NU) continue;
            const int dx = o % 3, dy = (o / 3) % 3, dz = DIM == 3 ? o / 9 : 1;
            const uint32_t J = (ck[dz] * (uint32_t)NY + cj[dy]) * (uint32_t)NX + ci[dx];
#pragma unroll
            for (int c = 0; c < DIM; ++c) xv[gg][c] = bld<T>(xr, (DIM * J + c) * (uint32_t)sizeof(T));
            if (o > NU) {
                // own block towards upper neighbour o - NU - 1 (zero if outside)
                const uint32_t q0 = (uint32_t)(o - NU - 1) * BB;
#pragma unroll
                for (int e = 0; e < BB; ++e) blk[gg][e] = bld<T>(sr, ((q0 + e) * uN + un) * (uint32_t)sizeof(T));
            } else {
                // neighbour J's block towards this node (its upper neighbour NST-1-o), transposed
                const uint32_t q0 = (uint32_t)(NST - 1 - o - NU - 1) * BB;
#pragma unroll
                for (int r = 0; r < DIM; ++r)
#pragma unroll
                    for (int c = 0; c < DIM; ++c)
                        blk[gg][r * DIM + c] = bld<T>(sr, ((q0 + c * DIM + r) * uN + J) * (uint32_t)sizeof(T));
                const bool in = ii[dx] && ij[dy] && ik[dz];
#pragma unroll
                for (int c = 0; c < DIM; ++c) xv[gg][c] = in ? xv[gg][c] : T(0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int gg = 0; gg < G; ++gg) {
            if (g0 + gg >= NST) continue;
            const int o = pair_order<NU>(g0 + gg);
            if (o == NU) continue;
#pragma unroll
            for (int r = 0; r < DIM; ++r)
#pragma unroll
                for (int c = 0; c < DIM; ++c) acc[r] += blk[gg][r * DIM + c] * xv[gg][c];
        }
    }
    double dots[2];
    finish_node<T, DIM, OP>(node, N, acc, xo, 0, b, y, dinv, omega, dots, ch);
}

// The same operator for R right-hand sides of ONE hierarchy per thread (the
// load cases of one solve): the stored stencil and the block inverse are read
// once for all of them, the vectors per right-hand side.  Lanes R*blockIdx.y ..
// +R-1 of the pack; a lane index at or past n_lanes repeats the last lane's
// reads and stores nothing, a lane whose solve has stopped stores nothing.
// Each lane's sums run in the order of k_stencil_op, so every right-hand side
// gets bitwise the result of its own launch.
template <typename T, int DIM, int OP, int G, int R>
__global__ __launch_bounds__(WG) void k_stencil_opm(const Pack<OpA<T>, MAXB> pk, int n_lanes, int nx, int ny,
                                                    int nz, int64_t N, T omega, double c1, double c2) {
    const int l0 = (int)blockIdx.y * R;
    const T* __restrict__ st = pk.a[l0].E;
    const T* __restrict__ dinv = pk.a[l0].dinv;
    // the lanes' pointers, copied out of the argument block once
    const T* xs[R];
    const T* bs[R];
    T* ys[R];
    const T* dis[R];
    T* dos[R];
    bool act[R];
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int lr = min(l0 + r, n_lanes - 1);
        xs[r] = pk.a[lr].x;
        bs[r] = pk.a[lr].b;
        ys[r] = pk.a[lr].y;
        dis[r] = pk.a[lr].din;
        dos[r] = pk.a[lr].dout;
        const int* dn = pk.a[lr].done;
        act[r] = l0 + r < n_lanes && !(dn && *dn);
        any = any || act[r];
    }
    if (!any) return;
    const int64_t node = xcd_block() * WG + threadIdx.x;
    if (node >= N) return;
    constexpr int BB = DIM * DIM, NST = DIM == 3 ? 27 : 9, NU = (NST - 1) / 2;
    constexpr int NQ = NU * BB + DIM * (DIM + 1) / 2;
    const int NX = nx + 1, NY = ny + 1, NZ = nz + 1;
    const int i = (int)(node % NX);
    const int j = (int)((node / NX) % NY);
    const int k = DIM == 3 ? (int)(node / ((int64_t)NX * NY)) : 0;
    const auto sr = buf_rsrc(st, (int64_t)N * NQ * sizeof(T));
    decltype(buf_rsrc(st, 0)) xr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) xr[r] = buf_rsrc(xs[r], (int64_t)N * DIM * sizeof(T));
    const uint32_t un = (uint32_t)node, uN = (uint32_t)N;
    uint32_t ci[3], cj[3], ck[3];
    bool ii[3], ij[3], ik[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ci[d] = (uint32_t)min(max(i + d - 1, 0), NX - 1);
        cj[d] = (uint32_t)min(max(j + d - 1, 0), NY - 1);
        ck[d] = DIM == 3 ? (uint32_t)min(max(k + d - 1, 0), NZ - 1) : 0u;
        ii[d] = i + d - 1 >= 0 && i + d - 1 < NX;
        ij[d] = j + d - 1 >= 0 && j + d - 1 < NY;
        ik[d] = DIM == 2 || (k + d - 1 >= 0 && k + d - 1 < NZ);
    }
    T acc[R][DIM] = {};
    T xo[R][DIM];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < DIM; ++c) xo[r][c] = bld<T>(xr[r], (DIM * un + c) * (uint32_t)sizeof(T));
    {
        int q = NU * BB;
#pragma unroll
        for (int rr = 0; rr < DIM; ++rr)
#pragma unroll
            for (int c = rr; c < DIM; ++c, ++q) {
                const T a = bld<T>(sr, ((uint32_t)q * uN + un) * (uint32_t)sizeof(T));
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    acc[r][rr] += a * xo[r][c];
                    if (c != rr) acc[r][c] += a * xo[r][rr];
                }
            }
    }
#pragma unroll
    for (int g0 = 0; g0 < NST; g0 += G) {
        T xv[G][R][DIM], blk[G][BB];
#pragma unroll
        for (int gg = 0; gg < G; ++gg) {
            if (g0 + gg >= NST) continue;
            const int o = pair_order<NU>(g0 + gg);
            if (o == NU) continue;
            const int dx = o % 3, dy = (o / 3) % 3, dz = DIM == 3 ? o / 9 : 1;
            const uint32_t J = (ck[dz] * (uint32_t)NY + cj[dy]) * (uint32_t)NX + ci[dx];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int c = 0; c < DIM; ++c) xv[gg][r][c] = bld<T>(xr[r], (DIM * J + c) * (uint32_t)sizeof(T));
            if (o > NU) {
                const uint32_t q0 = (uint32_t)(o - NU - 1) * BB;
#pragma unroll
                for (int e = 0; e < BB; ++e) blk[gg][e] = bld<T>(sr, ((q0 + e) * uN + un) * (uint32_t)sizeof(T));
            } else {
                const uint32_t q0 = (uint32_t)(NST - 1 - o - NU - 1) * BB;
#pragma unroll
                for (int rr = 0; rr < DIM; ++rr)
#pragma unroll
                    for (int c = 0; c < DIM; ++c)
                        blk[gg][rr * DIM + c] = bld<T>(sr, ((q0 + c * DIM + rr) * uN + J) * (uint32_t)sizeof(T));
                const bool in = ii[dx] && ij[dy] && ik[dz];
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int c = 0; c < DIM; ++c) xv[gg][r][c] = in ? xv[gg][r][c] : T(0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int gg = 0; gg < G; ++gg) {
            if (g0 + gg >= NST) continue;
            const int o = pair_order<NU>(g0 + gg);
            if (o == NU) continue;
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int rr = 0; rr < DIM; ++rr)
#pragma unroll
                    for (int c = 0; c < DIM; ++c) acc[r][rr] += blk[gg][rr * DIM + c] * xv[gg][r][c];
        }
    }
    // pin the sums here: used only under the per-lane condition below, they
    // would otherwise be sunk into it, past every group's scheduling barrier
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < DIM; ++c) asm volatile("" : "+v"(acc[r][c]));
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!act[r]) continue;
        ChebArgs ch;
        ch.din = dis[r];
        ch.dout = dos[r];
        ch.c1 = c1;
        ch.c2 = c2;
        double dots[2];
        finish_node<T, DIM, OP>(node, N, acc[r], xo[r], 0, bs[r], ys[r], dinv, omega, dots, ch);
    }
}

template <typename T>
static const T* st_of(const Level& L);
template <>
const double* st_of<double>(const Level& L) { return L.stc64; }
template <>
const float* st_of<float>(const Level& L) { return L.stc32; }
template <typename T>
static const T* dinv_of(const Level& L);
template <>
const double* dinv_of<double>(const Level& L) { return L.dinv64; }
template <>
const float* dinv_of<float>(const Level& L) { return L.dinv32; }

// The same operator with P lanes per node (small levels, where a launch is
// one latency chain): lane p takes the neighbours p, p + P, ... in one batch of
// loads with uniform control flow (the slot's kind, upper / lower / diagonal,
// only selects addresses) that also carries the finishing step's operands,
// then the P partial sums meet in a butterfly and the node's first lane finishes.
template <typename T, int DIM, int OP, int P, int NB>
__global__ __launch_bounds__(WG) void k_stencil_split(const Pack<OpA<T>, NB> pk, int nx, int ny, int nz,
                                                      int64_t N, T omega, double c1, double c2) {
    const OpA<T>& A_ = lane_of(pk);
    const T* __restrict__ st = A_.E;
    const T* __restrict__ x = A_.x;
    const T* __restrict__ b = A_.b;
    T* __restrict__ y = A_.y;
    const T* __restrict__ dinv = A_.dinv;
    const int* __restrict__ done = A_.done;
    ChebArgs ch;
    ch.din = A_.din;
    ch.dout = A_.dout;
    ch.c1 = c1;
    ch.c2 = c2;
    if (done && *done) return;
    const int64_t gid = xcd_block() * WG + threadIdx.x;
    const int64_t node = gid / P;
    const int p = (int)(gid & (P - 1));
    if (node >= N) return;      // all P lanes of a node leave together
    constexpr int BB = DIM * DIM, NST = DIM == 3 ? 27 : 9, NU = (NST - 1) / 2;
    constexpr int NQ = NU * BB + DIM * (DIM + 1) / 2;
    constexpr int NS = (NST + P - 1) / P;
    const int NX = nx + 1, NY = ny + 1, NZ = nz + 1;
    const int i = (int)(node % NX);
    const int j = (int)((node / NX) % NY);
    const int k = DIM == 3 ? (int)(node / ((int64_t)NX * NY)) : 0;
    const auto sr = buf_rsrc(st, (int64_t)N * NQ * sizeof(T));
    const auto xr = buf_rsrc(x, (int64_t)N * DIM * sizeof(T));
    const uint32_t un = (uint32_t)node, uN = (uint32_t)N;
    uint32_t ci[3], cj[3], ck[3];
    bool ii[3], ij[3], ik[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ci[d] = (uint32_t)min(max(i + d - 1, 0), NX - 1);
        cj[d] = (uint32_t)min(max(j + d - 1, 0), NY - 1);
        ck[d] = DIM == 3 ? (uint32_t)min(max(k + d - 1, 0), NZ - 1) : 0u;
        ii[d] = i + d - 1 >= 0 && i + d - 1 < NX;
        ij[d] = j + d - 1 >= 0 && j + d - 1 < NY;
        ik[d] = DIM == 2 || (k + d - 1 >= 0 && k + d - 1 < NZ);
    }
    T xo[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) xo[c] = bld<T>(xr, (DIM * un + c) * (uint32_t)sizeof(T));
    FinIn<T, DIM> fin;
    finish_load<T, DIM, OP>(node, N, b, dinv, ch, fin);
    T xv[NS][DIM], blk[NS][BB];
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
        const int o = sl * P + p;
        const bool valid = o < NST;
        const int oc = valid ? o : NST - 1;    // spare slot: any in-bounds block, x zeroed below
        const int dx = oc % 3, dy = (oc / 3) % 3, dz = DIM == 3 ? oc / 9 : 1;
        const uint32_t J = (ck[dz] * (uint32_t)NY + cj[dy]) * (uint32_t)NX + ci[dx];
#pragma unroll
        for (int c = 0; c < DIM; ++c) xv[sl][c] = bld<T>(xr, (DIM * J + c) * (uint32_t)sizeof(T));
        const bool up = oc > NU, lo = oc < NU;
        // upper: own block towards neighbour oc; lower: neighbour J's block
        // towards this node, transposed; diagonal: own upper triangle
        const uint32_t qU = (uint32_t)(oc - NU - 1) * BB, qL = (uint32_t)(NST - 1 - oc - NU - 1) * BB;
        const uint32_t at = lo ? J : un;
#pragma unroll
        for (int r = 0; r < DIM; ++r)
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const int lr = r < c ? r : c, hc = r < c ? c : r;
                const uint32_t qd = (uint32_t)(NU * BB + lr * DIM - lr * (lr - 1) / 2 + (hc - lr));
                const uint32_t q = up ? qU + (uint32_t)(r * DIM + c) : (lo ? qL + (uint32_t)(c * DIM + r) : qd);
                blk[sl][r * DIM + c] = bld<T>(sr, (q * uN + at) * (uint32_t)sizeof(T));
            }
        const bool keep = valid && (!lo || (ii[dx] && ij[dy] && ik[dz]));
#pragma unroll
        for (int c = 0; c < DIM; ++c) xv[sl][c] = keep ? xv[sl][c] : T(0);
    }
    __builtin_amdgcn_sched_barrier(0);
    T acc[DIM] = {};
#pragma unroll
    for (int sl = 0; sl < NS; ++sl)
#pragma unroll
        for (int r = 0; r < DIM; ++r)
#pragma unroll
            for (int c = 0; c < DIM; ++c) acc[r] += blk[sl][r * DIM + c] * xv[sl][c];
#pragma unroll
    for (int m = 1; m < P; m <<= 1)
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[c] += __shfl_xor(acc[c], m, 64);
    if (p == 0) {
        double dots[2];
        finish_store<T, DIM, OP>(node, acc, xo, 0, fin, y, omega, dots, ch);
    }
}

template <typename T, int NB>
static Pack<OpA<T>, NB> stencil_pack(int level, const LaneIO* L, int n) {
    Pack<OpA<T>, NB> pk{};
    for (int q = 0; q < n; ++q) {
        const Level& Lq = L[q].h->lv[level];
        OpA<T>& a = pk.a[q];
        a.E = st_of<T>(Lq);
        a.x = (const T*)L[q].x;
        a.b = (const T*)L[q].b;
        a.y = (T*)L[q].y;
        a.dinv = dinv_of<T>(Lq);
        a.done = L[q].done;
        a.din = (const T*)L[q].din;
        a.dout = (T*)L[q].dout;
    }
    return pk;
}

// one launch for lanes L[0..n), n <= NB: the small-level form (P lanes per
// node) or the large-level form (groups of G neighbours)
template <typename T, int DIM, int NB>
static void stencil_launch(int level, const LaneIO* L, int n, int op, T omega, double c1, double c2,
                           hipStream_t s) {
    const Level& V = L[0].h->lv[level];
    const auto pk = stencil_pack<T, NB>(level, L, n);
    const int nz = DIM == 3 ? V.nel[2] : 0;
    // fewer workgroups than compute units: latency-bound; 3D splits each
    // node over 4 lanes, 2D batches all nine neighbours (the level's
    // op_kernel can pin either form, whatever the size)
    const bool small = V.op_kernel == 0 ? grid_for(V.n_nodes) < 256 : V.op_kernel == 2;
    const dim3 blk(WG);
    if (small && DIM == 3) {
        constexpr int P = 4;
        const dim3 g(grid_for(V.n_nodes * P), n);
#define TM_SL(OPV)                                                                                   \
    hipLaunchKernelGGL((k_stencil_split<T, DIM, OPV, P, NB>), g, blk, 0, s, pk, V.nel[0], V.nel[1], nz, V.n_nodes, \
                       omega, c1, c2)
        switch (op) {
            case OP_APPLY: TM_SL(OP_APPLY); break;
            case OP_RESID: TM_SL(OP_RESID); break;
            case OP_CHEB: TM_SL(OP_CHEB); break;
            default: TM_SL(OP_SMOOTH); break;
        }
#undef TM_SL
        return;
    }
    const dim3 g(grid_for(V.n_nodes), n);
#define TM_SO(OPV, G)                                                                                \
    hipLaunchKernelGGL((k_stencil_op<T, DIM, OPV, G, NB>), g, blk, 0, s, pk, V.nel[0], V.nel[1], nz, V.n_nodes, \
                       omega, c1, c2)
#define TM_SOG(G)                                                                                    \
    switch (op) {                                                                                    \
        case OP_APPLY: TM_SO(OP_APPLY, G); break;                                                    \
        case OP_RESID: TM_SO(OP_RESID, G); break;                                                    \
        case OP_CHEB: TM_SO(OP_CHEB, G); break;                                                      \
        default: TM_SO(OP_SMOOTH, G); break;                                                         \
    }
    if (small) {
        TM_SOG(9)
    } else {
        TM_SOG(4)
    }
#undef TM_SOG
#undef TM_SO
}

// Several right-hand sides of one hierarchy on a large level: R per thread
// (the operator read once for R of them), ceil(n / 4) groups of lanes.
template <typename T, int DIM, int R>
static void stencil_launch_shared(int level, const LaneIO* L, int n, int op, T omega, double c1, double c2,
                                  hipStream_t s) {
    const Level& V = L[0].h->lv[level];
    const auto pk = stencil_pack<T, MAXB>(level, L, n);
    const int nz = DIM == 3 ? V.nel[2] : 0;
    const dim3 g(grid_for(V.n_nodes), (unsigned)ceil_div(n, R)), blk(WG);
#define TM_SM(OPV)                                                                                   \
    hipLaunchKernelGGL((k_stencil_opm<T, DIM, OPV, 4, R>), g, blk, 0, s, pk, n, V.nel[0], V.nel[1], nz,   \
                       V.n_nodes, omega, c1, c2)
    switch (op) {
        case OP_APPLY: TM_SM(OP_APPLY); break;
        case OP_RESID: TM_SM(OP_RESID); break;
        case OP_CHEB: TM_SM(OP_CHEB); break;
        default: TM_SM(OP_SMOOTH); break;
    }
#undef TM_SM
}

template <typename T, int DIM>
static bool try_shared(int level, const LaneIO* L, int n, int op, T omega, double c1, double c2, hipStream_t s) {
    const Level& V = L[0].h->lv[level];
    const bool small = V.op_kernel == 0 ? grid_for(V.n_nodes) < 256 : V.op_kernel == 2;
    if (n < 2 || small) return false;
    for (int q = 1; q < n; ++q)
        if (L[q].h != L[0].h) return false;
    const int groups = (int)ceil_div(n, 4), R = (int)ceil_div(n, groups);
    switch (R) {
        case 2: stencil_launch_shared<T, DIM, 2>(level, L, n, op, omega, c1, c2, s); break;
        case 3: stencil_launch_shared<T, DIM, 3>(level, L, n, op, omega, c1, c2, s); break;
        default: stencil_launch_shared<T, DIM, 4>(level, L, n, op, omega, c1, c2, s); break;
    }
    return true;
}

template <typename T>
void launch_stencil_op_b(int level, int op, const LaneIO* L, int n, T omega, double c1, double c2,
                         hipStream_t s) {
    if (n < 1) return;
    if constexpr (std::is_same<T, float>::value) {
        if (level == 1 && L[0].h->lv[1].subf) {
            launch_coarse1_tensor_b<T>(op, L, n, omega, c1, c2, s);
            return;
        }
    }
    const int dim = L[0].h->lv[level].dim;
    for (int q0 = 0; q0 < n; q0 += MAXB) {
        const int m = std::min(MAXB, n - q0);
        if (dim == 3 ? try_shared<T, 3>(level, L + q0, m, op, omega, c1, c2, s)
                     : try_shared<T, 2>(level, L + q0, m, op, omega, c1, c2, s))
            continue;
        if (dim == 3) {
            if (m == 1) stencil_launch<T, 3, 1>(level, L + q0, 1, op, omega, c1, c2, s);
            else stencil_launch<T, 3, MAXB>(level, L + q0, m, op, omega, c1, c2, s);
        } else {
            if (m == 1) stencil_launch<T, 2, 1>(level, L + q0, 1, op, omega, c1, c2, s);
            else stencil_launch<T, 2, MAXB>(level, L + q0, m, op, omega, c1, c2, s);
        }
    }
}
template void launch_stencil_op_b<double>(int, int, const LaneIO*, int, double, double, double, hipStream_t);
template void launch_stencil_op_b<float>(int, int, const LaneIO*, int, float, double, double, hipStream_t);

// --------------------------------------------------------------- transfers
// Per axis with nf fine elements and ceil(nf/2) coarse ones, coarse node I sits
// on fine node min(2I, nf): for an odd nf the last coarse node sits on the last
// fine node, and the last coarse element is a single fine element.
__device__ __forceinline__ int coarse_pos(int I, int nf) { return min(2 * I, nf); }

// weight of the fine node at offset d in {-1, 0, 1} from coarse node I's position
template <typename T>
__device__ __forceinline__ T restrict_w(int I, int d, int nf) {
    if (2 * I > nf) return d == 0 ? T(1) : T(0);
    const int j = 2 * I + d;
    if (j < 0 || j > nf) return T(0);
    if (d == 0) return T(1);
    return ((nf & 1) && j == nf) ? T(0) : T(0.5);      // the last fine node of an odd count is coarse
}

// the (one or two) coarse parents of fine node i and their weights
template <typename T>
__device__ __forceinline__ void prolong_parents(int i, int nf, int (&ia)[2], T (&w)[2]) {
    const int nc1 = (nf + 1) / 2;                       // last coarse node
    if ((nf & 1) && i == nf) {
        ia[0] = ia[1] = nc1;
        w[0] = T(1);
        w[1] = T(0);
    } else {
        ia[0] = i >> 1;
        ia[1] = min((i >> 1) + 1, nc1);
        w[0] = (i & 1) ? T(0.5) : T(1);
        w[1] = (i & 1) ? T(0.5) : T(0);
    }
}


// restriction b_c = P~^T r_f: coarse node I gathers the fine nodes at offsets d in
// {-1,0,1}^dim from its position, with weight prod restrict_w (1 on it, 1/2 on a
// fine midpoint, 0 otherwise); supported fine dofs contribute 0.
// Optionally also x_c = omega D_c^-1 b_c (the first sweep of the coarse level from zero).
template <typename T, int DIM, bool FIRST, bool MASK, int NB>
__global__ __launch_bounds__(WG) void k_restrict(const Pack<RestrictA<T>, NB> pk, int fnx, int fny, int fnz,
                                                 int cnx, int cny, int cnz, T omega) {
    const RestrictA<T>& A_ = lane_of(pk);
    const T* __restrict__ rf = A_.rf;
    const uint8_t* __restrict__ nm = A_.nm;
    T* __restrict__ bc = A_.bc;
    T* __restrict__ xc = A_.xc;
    const T* __restrict__ dinv = A_.dinv;
    const int* __restrict__ done = A_.done;
    if (done && *done) return;
    const int CX = cnx + 1, CY = cny + 1, CZ = cnz + 1;
    const int64_t Nc = (int64_t)CX * CY * (DIM == 3 ? CZ : 1);
    const int64_t node = xcd_block() * WG + threadIdx.x;
    if (node >= Nc) return;
    const int FX = fnx + 1, FY = fny + 1, FZ = fnz + 1;
    const int I = (int)(node % CX);
    const int J = (int)((node / CX) % CY);
    const int K = DIM == 3 ? (int)(node / ((int64_t)CX * CY)) : 0;
    const int64_t Nf = (int64_t)FX * FY * (DIM == 3 ? FZ : 1);
    const auto rr = buf_rsrc(rf, Nf * DIM * sizeof(T));
    // every load is unconditional (clamped, in-bounds index) and issued before
    // the arithmetic; weights and masks zero what lies outside or is supported
    constexpr int NS = DIM == 3 ? 27 : 9;
    T v[NS][DIM], w[NS];
    uint8_t m[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = DIM == 3 ? q / 9 - 1 : 0;
        const int fi = coarse_pos(I, fnx) + dx, fj = coarse_pos(J, fny) + dy;
        const int fk = DIM == 3 ? coarse_pos(K, fnz) + dz : 0;
        const int gi = min(max(fi, 0), FX - 1), gj = min(max(fj, 0), FY - 1);
        const int gk = DIM == 3 ? min(max(fk, 0), FZ - 1) : 0;
        const uint32_t f = (uint32_t)(DIM == 3 ? (gk * FY + gj) * FX + gi : gj * FX + gi);
        w[q] = restrict_w<T>(I, dx, fnx) * restrict_w<T>(J, dy, fny) * (DIM == 3 ? restrict_w<T>(K, dz, fnz) : T(1));
        if constexpr (DIM == 3) {
            bld3(rr, f * (uint32_t)(3 * sizeof(T)), v[q]);
        } else {
#pragma unroll
            for (int c = 0; c < DIM; ++c) v[q][c] = bld<T>(rr, (DIM * f + c) * (uint32_t)sizeof(T));
        }
        m[q] = MASK ? nm[f] : (uint8_t)0;
    }
    T dv[sym_n(DIM)];
    if (FIRST) {
#pragma unroll
        for (int e = 0; e < sym_n(DIM); ++e) dv[e] = dinv[(int64_t)e * Nc + node];
    }
    T acc[DIM] = {};
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[c] += ((m[q] >> c) & 1u) ? T(0) : w[q] * v[q][c];
#pragma unroll
    for (int c = 0; c < DIM; ++c) bc[DIM * node + c] = acc[c];
    if (FIRST) {
#pragma unroll
        for (int r = 0; r < DIM; ++r) {
            T t = 0;
#pragma unroll
            for (int c = 0; c < DIM; ++c) t += dv[sym_at(r, c, DIM)] * acc[c];
            xc[DIM * node + r] = omega * t;
        }
    }
}

template <typename T, int DIM, bool FIRST, int NB>
static void restrict_launch(int fl, const LaneIO* L, int n, T omega, hipStream_t s) {
    const Level& fine = L[0].h->lv[fl];
    const Level& coarse = L[0].h->lv[fl + 1];
    Pack<RestrictA<T>, NB> pk{};
    for (int q = 0; q < n; ++q) {
        RestrictA<T>& a = pk.a[q];
        a.rf = (const T*)L[q].x;
        a.nm = fine.kind == TM_LEVEL_FINE ? L[q].h->lv[fl].nmask : nullptr;
        a.bc = (T*)L[q].y;
        a.xc = (T*)L[q].y2;
        a.dinv = dinv_of<T>(L[q].h->lv[fl + 1]);
        a.done = L[q].done;
    }
    const dim3 g(grid_for(coarse.n_nodes), n), blk(WG);
    const int fz = DIM == 3 ? fine.nel[2] : 0, cz = DIM == 3 ? coarse.nel[2] : 0;
    if (fine.kind == TM_LEVEL_FINE)
        hipLaunchKernelGGL((k_restrict<T, DIM, FIRST, true, NB>), g, blk, 0, s, pk, fine.nel[0], fine.nel[1], fz,
                           coarse.nel[0], coarse.nel[1], cz, omega);
    else
        hipLaunchKernelGGL((k_restrict<T, DIM, FIRST, false, NB>), g, blk, 0, s, pk, fine.nel[0], fine.nel[1], fz,
                           coarse.nel[0], coarse.nel[1], cz, omega);
}

// b_c = P~^T r_f (lane x -> y) and, if the lanes give y2, the coarse level's
// first sweep into y2 (all lanes alike)
template <typename T>
void launch_restrict_b(int fl, const LaneIO* L, int n, T omega, hipStream_t s) {
    if (n < 1) return;
    const int dim = L[0].h->lv[fl].dim;
    const bool first = L[0].y2 != nullptr;
    for (int q0 = 0; q0 < n; q0 += MAXB) {
        const int m = std::min(MAXB, n - q0);
#define TM_RL(D, F)                                                        \
    if (m == 1) restrict_launch<T, D, F, 1>(fl, L + q0, 1, omega, s);      \
    else restrict_launch<T, D, F, MAXB>(fl, L + q0, m, omega, s);
        if (dim == 3) {
            if (first) { TM_RL(3, true) } else { TM_RL(3, false) }
        } else {
            if (first) { TM_RL(2, true) } else { TM_RL(2, false) }
        }
#undef TM_RL
    }
}
template void launch_restrict_b<double>(int, const LaneIO*, int, double, hipStream_t);
template void launch_restrict_b<float>(int, const LaneIO*, int, float, hipStream_t);

// The last restriction and the coarsest solve in one launch: every workgroup
// forms the whole coarsest right-hand side b_c = P~^T r_f (the gather of
// k_restrict, per coarse node) in LDS, then four rows of x_c = A_c^-1 b_c,
// one wave per row in the coarsest solve's summation order.
template <typename T>
struct RsolveA {
    const T* rf;
    const uint8_t* nm;
    const double* Ainv;
    T* x;
    const int* done;
};

constexpr int RS_MAX = 4096;     // coarsest dofs (the dense factorisation's limit)

template <typename T, int DIM, bool MASK, int NB>
__global__ __launch_bounds__(WG) void k_restrict_solve(const Pack<RsolveA<T>, NB> pk, int fnx, int fny, int fnz,
                                                       int cnx, int cny, int cnz, int nc) {
    const RsolveA<T>& A_ = lane_of(pk);
    if (A_.done && *A_.done) return;
    __shared__ double bsh[RS_MAX];
    const int CX = cnx + 1, CY = cny + 1, CZ = cnz + 1;
    const int Nc = CX * CY * (DIM == 3 ? CZ : 1);
    const int FX = fnx + 1, FY = fny + 1, FZ = fnz + 1;
    const int64_t Nf = (int64_t)FX * FY * (DIM == 3 ? FZ : 1);
    const auto rr = buf_rsrc(A_.rf, Nf * DIM * sizeof(T));
    constexpr int NS = DIM == 3 ? 27 : 9;
    for (int node = threadIdx.x; node < Nc; node += WG) {
        const int I = node % CX, J = (node / CX) % CY, K = DIM == 3 ? node / (CX * CY) : 0;
        T v[NS][DIM], w[NS];
        uint8_t m[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = DIM == 3 ? q / 9 - 1 : 0;
            const int gi = min(max(coarse_pos(I, fnx) + dx, 0), FX - 1);
            const int gj = min(max(coarse_pos(J, fny) + dy, 0), FY - 1);
            const int gk = DIM == 3 ? min(max(coarse_pos(K, fnz) + dz, 0), FZ - 1) : 0;
            const uint32_t f = (uint32_t)(DIM == 3 ? (gk * FY + gj) * FX + gi : gj * FX + gi);
            w[q] = restrict_w<T>(I, dx, fnx) * restrict_w<T>(J, dy, fny) * (DIM == 3 ? restrict_w<T>(K, dz, fnz) : T(1));
            if constexpr (DIM == 3) {
                bld3(rr, f * (uint32_t)(3 * sizeof(T)), v[q]);
            } else {
#pragma unroll
                for (int c = 0; c < DIM; ++c) v[q][c] = bld<T>(rr, (DIM * f + c) * (uint32_t)sizeof(T));
            }
            m[q] = MASK ? A_.nm[f] : (uint8_t)0;
        }
        T acc[DIM] = {};
#pragma unroll
        for (int q = 0; q < NS; ++q)
#pragma unroll
            for (int c = 0; c < DIM; ++c) acc[c] += ((m[q] >> c) & 1u) ? T(0) : w[q] * v[q][c];
#pragma unroll
        for (int c = 0; c < DIM; ++c) bsh[DIM * node + c] = (double)acc[c];
    }
    __syncthreads();
    const int row = (int)blockIdx.x * (WG / 64) + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nc) return;
    const double* Ar = A_.Ainv + (int64_t)row * nc;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int c = lane;
    for (; c + 192 < nc; c += 256) {
        a0 += Ar[c] * bsh[c];
        a1 += Ar[c + 64] * bsh[c + 64];
        a2 += Ar[c + 128] * bsh[c + 128];
        a3 += Ar[c + 192] * bsh[c + 192];
    }
    if (c < nc) a0 += Ar[c] * bsh[c];
    if (c + 64 < nc) a1 += Ar[c + 64] * bsh[c + 64];
    if (c + 128 < nc) a2 += Ar[c + 128] * bsh[c + 128];
    double a = (a0 + a1) + (a2 + a3);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o, 64);
    if (lane == 0) A_.x[row] = (T)a;
}

bool restrict_solve_ok(const tm_hierarchy* h) {
    const int L = (int)h->lv.size();
    if (L < 2 || h->lv[L - 2].xfer_bsr || h->nc > RS_MAX) return false;
    const Level& c = h->lv[L - 1];
    return (c.kind == TM_LEVEL_GEOMETRIC) && c.n == h->nc;
}

template <typename T, int DIM, bool MASK, int NB>
static void restrict_solve_launch(const LaneIO* L, int n, hipStream_t s) {
    const tm_hierarchy* h = L[0].h;
    const int nl = (int)h->lv.size();
    const Level& fine = h->lv[nl - 2];
    const Level& coarse = h->lv[nl - 1];
    Pack<RsolveA<T>, NB> pk{};
    for (int q = 0; q < n; ++q) {
        RsolveA<T>& a = pk.a[q];
        a.rf = (const T*)L[q].x;
        a.nm = MASK ? L[q].h->lv[nl - 2].nmask : nullptr;
        a.Ainv = L[q].h->ainv;
        a.x = (T*)L[q].y;
        a.done = L[q].done;
    }
    const int nc = (int)h->nc;
    const int fz = DIM == 3 ? fine.nel[2] : 0, cz = DIM == 3 ? coarse.nel[2] : 0;
    hipLaunchKernelGGL((k_restrict_solve<T, DIM, MASK, NB>), dim3((unsigned)ceil_div(nc, WG / 64), n), dim3(WG), 0, s,
                       pk, fine.nel[0], fine.nel[1], fz, coarse.nel[0], coarse.nel[1], cz, nc);
}

// x_c = A_c^-1 P~^T r_f for lanes L (x: the residual of the level above the
// coarsest, y: the coarsest correction), where restrict_solve_ok holds
template <typename T>
void launch_restrict_solve_b(const LaneIO* L, int n, hipStream_t s) {
    if (n < 1) return;
    const tm_hierarchy* h = L[0].h;
    if (!restrict_solve_ok(h)) fail(TM_ERR_ARG, "fused coarsest restriction: not a geometric coarsest transfer");
    const int nl = (int)h->lv.size();
    const int dim = h->lv[nl - 2].dim;
    const bool mask = h->lv[nl - 2].kind == TM_LEVEL_FINE;
    for (int q0 = 0; q0 < n; q0 += MAXB) {
        const int m = std::min(MAXB, n - q0);
#define TM_RS(D, M)                                                   \
    if (m == 1) restrict_solve_launch<T, D, M, 1>(L + q0, 1, s);      \
    else restrict_solve_launch<T, D, M, MAXB>(L + q0, m, s);
        if (dim == 3) {
            if (mask) { TM_RS(3, true) } else { TM_RS(3, false) }
        } else {
            if (mask) { TM_RS(2, true) } else { TM_RS(2, false) }
        }
#undef TM_RS
    }
}
template void launch_restrict_solve_b<double>(const LaneIO*, int, hipStream_t);
template void launch_restrict_solve_b<float>(const LaneIO*, int, hipStream_t);

// prolongation x_f += M P x_c: fine node i interpolates from the coarse nodes
// around it (1, 2, 4 or 8 of them), weights 1 or 1/2 per axis.
template <typename T, int DIM, int NB>
__global__ __launch_bounds__(WG) void k_prolong(const Pack<ProlongA<T>, NB> pk, int fnx, int fny, int fnz) {
    const ProlongA<T>& A_ = lane_of(pk);
    const T* __restrict__ xc = A_.xc;
    const uint8_t* __restrict__ nm = A_.nm;
    T* __restrict__ xf = A_.xf;
    const int* __restrict__ done = A_.done;
    if (done && *done) return;
    const int FX = fnx + 1, FY = fny + 1, FZ = fnz + 1;
    const int64_t Nf = (int64_t)FX * FY * (DIM == 3 ? FZ : 1);
    const int64_t node = xcd_block() * WG + threadIdx.x;
    if (node >= Nf) return;
    const int CX = (fnx + 1) / 2 + 1, CY = (fny + 1) / 2 + 1;     // ceil(n/2) + 1 coarse nodes
    const int i = (int)(node % FX);
    const int j = (int)((node / FX) % FY);
    const int k = DIM == 3 ? (int)(node / ((int64_t)FX * FY)) : 0;
    const int CZ = (fnz + 1) / 2 + 1;
    // per axis: the coarse parents (one with weight 1, or two with 1/2 each)
    int ia[2], ja[2], ka[2] = {0, 0};
    T wi[2], wj[2], wk[2] = {T(1), T(0)};
    prolong_parents<T>(i, fnx, ia, wi);
    prolong_parents<T>(j, fny, ja, wj);
    if (DIM == 3) prolong_parents<T>(k, fnz, ka, wk);
    // all loads (the coarse corners, this node's value and mask) before the
    // arithmetic; the store is unconditional (supported dofs keep their value)
    const int64_t Nc = (int64_t)CX * CY * (DIM == 3 ? CZ : 1);
    const auto cr = buf_rsrc(xc, Nc * DIM * sizeof(T));
    const auto fr = buf_rsrc(xf, Nf * DIM * sizeof(T));
    constexpr int NC = DIM == 3 ? 8 : 4;
    T v[NC][DIM], xo[DIM];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        const int a2 = q & 1, b2 = (q >> 1) & 1, c2 = q >> 2;
        const uint32_t C = (uint32_t)(DIM == 3 ? (ka[c2] * CY + ja[b2]) * CX + ia[a2] : ja[b2] * CX + ia[a2]);
        if constexpr (DIM == 3) {
            bld3(cr, C * (uint32_t)(3 * sizeof(T)), v[q]);
        } else {
#pragma unroll
            for (int c = 0; c < DIM; ++c) v[q][c] = bld<T>(cr, (DIM * C + c) * (uint32_t)sizeof(T));
        }
    }
    if constexpr (DIM == 3) {
        bld3(fr, (uint32_t)node * (uint32_t)(3 * sizeof(T)), xo);
    } else {
#pragma unroll
        for (int c = 0; c < DIM; ++c) xo[c] = bld<T>(fr, (DIM * (uint32_t)node + c) * (uint32_t)sizeof(T));
    }
    const uint8_t m = nm ? nm[node] : 0;
    T acc[DIM] = {};
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        const int a2 = q & 1, b2 = (q >> 1) & 1, c2 = q >> 2;
        const T w = wi[a2] * wj[b2] * (DIM == 3 ? wk[c2] : T(1));
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[c] += w * v[q][c];
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) xf[DIM * node + c] = ((m >> c) & 1u) ? xo[c] : xo[c] + acc[c];
}

// The prolongation x_l + P x_{l+1} fused into the first post-smoothing step of
// a small geometric level (coarse level geometric too): the step reads the
// prolonged iterate of the node and of its neighbours, formed on the fly
// exactly as k_prolong forms it (same parents, weights and order), so the
// prolongation launch and its store are saved.  The coarse values a node needs
// lie in a 3^DIM block of coarse nodes (per axis: the parents of fine nodes
// i-1 .. i+1); the P lanes of a node load that block into LDS together, then
// (after the barrier) each lane loads its neighbour slots as k_stencil_split
// does and forms their prolonged values.  Neighbour slots, blocks and sums are
// those of k_stencil_split with P lanes per node (used in 2D with P = 1).
// Nodes past the end compute on a clamped node and store nothing (every
// thread reaches the barrier).
template <typename T, int DIM, int OP, int P, int NB>
__global__ __launch_bounds__(WG) void k_stencil_pro(const Pack<OpA<T>, NB> pk, int nx, int ny, int nz,
                                                    int64_t N, T omega, double c1, double c2) {
    constexpr int NCB = DIM == 3 ? 27 : 9;          // coarse block
    __shared__ T cblk[WG / P][NCB][DIM];
    const OpA<T>& A_ = lane_of(pk);
    const T* __restrict__ st = A_.E;
    const T* __restrict__ x = A_.x;
    const T* __restrict__ xc = A_.xc;
    const T* __restrict__ b = A_.b;
    T* __restrict__ y = A_.y;
    const T* __restrict__ dinv = A_.dinv;
    const int* __restrict__ done = A_.done;
    if (done && *done) return;                       // uniform over the workgroup (one lane per grid row)
    const int64_t gid = xcd_block() * WG + threadIdx.x;
    const bool live = gid / P < N;
    const int64_t node = live ? gid / P : N - 1;
    const int p = (int)(gid & (P - 1));
    const int nl = (int)threadIdx.x / P;
    constexpr int BB = DIM * DIM, NST = DIM == 3 ? 27 : 9, NU = (NST - 1) / 2;
    constexpr int NQ = NU * BB + DIM * (DIM + 1) / 2;
    constexpr int NS = (NST + P - 1) / P;
    const int NX = nx + 1, NY = ny + 1, NZ = nz + 1;
    const int i = (int)(node % NX);
    const int j = (int)((node / NX) % NY);
    const int k = DIM == 3 ? (int)(node / ((int64_t)NX * NY)) : 0;
    const int CX = (nx + 1) / 2 + 1, CY = (ny + 1) / 2 + 1, CZ = DIM == 3 ? (nz + 1) / 2 + 1 : 1;
    const int64_t Nc = (int64_t)CX * CY * CZ;
    const auto sr = buf_rsrc(st, (int64_t)N * NQ * sizeof(T));
    const auto xr = buf_rsrc(x, (int64_t)N * DIM * sizeof(T));
    const auto cr = buf_rsrc(xc, Nc * DIM * sizeof(T));
    const uint32_t un = (uint32_t)node, uN = (uint32_t)N;
    uint32_t ci[3], cj[3], ck[3];
    bool ii[3], ij[3], ik[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ci[d] = (uint32_t)min(max(i + d - 1, 0), NX - 1);
        cj[d] = (uint32_t)min(max(j + d - 1, 0), NY - 1);
        ck[d] = DIM == 3 ? (uint32_t)min(max(k + d - 1, 0), NZ - 1) : 0u;
        ii[d] = i + d - 1 >= 0 && i + d - 1 < NX;
        ij[d] = j + d - 1 >= 0 && j + d - 1 < NY;
        ik[d] = DIM == 2 || (k + d - 1 >= 0 && k + d - 1 < NZ);
    }
    // the block starts at the first parent of fine node i - 1 (clamped) per axis
    const int lx = (int)ci[0] >> 1, ly = (int)cj[0] >> 1, lz = DIM == 3 ? (int)ck[0] >> 1 : 0;
    // the coarse block [lx, lx+2] x [ly, ly+2] (x [lz, lz+2]), indices clamped
#pragma unroll
    for (int sb = p; sb < NCB; sb += P) {
        const int sx = sb % 3, sy = (sb / 3) % 3, sz = sb / 9;
        const uint32_t C = (uint32_t)((DIM == 3 ? min(lz + sz, CZ - 1) * CY : 0) + min(ly + sy, CY - 1)) *
                               (uint32_t)CX + (uint32_t)min(lx + sx, CX - 1);
#pragma unroll
        for (int c = 0; c < DIM; ++c) cblk[nl][sb][c] = bld<T>(cr, (DIM * C + c) * (uint32_t)sizeof(T));
    }
    __syncthreads();
    // this node's value and the finishing operands, then the slots' loads
    // (after the barrier, so that it waits for the coarse block only)
    T xraw[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) xraw[c] = bld<T>(xr, (DIM * un + c) * (uint32_t)sizeof(T));
    ChebArgs ch;
    ch.din = nullptr;
    ch.dout = A_.dout;
    ch.c1 = c1;
    ch.c2 = c2;
    FinIn<T, DIM> fin;
    finish_load<T, DIM, OP == OP_CHEB ? OP_SMOOTH : OP>(node, N, b, dinv, ch, fin);
    T xv[NS][DIM], blk[NS][BB];
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
        const int o = sl * P + p;
        const bool valid = o < NST;
        const int oc = valid ? o : NST - 1;
        const int dx = oc % 3, dy = (oc / 3) % 3, dz = DIM == 3 ? oc / 9 : 1;
        const uint32_t J = (ck[dz] * (uint32_t)NY + cj[dy]) * (uint32_t)NX + ci[dx];
#pragma unroll
        for (int c = 0; c < DIM; ++c) xv[sl][c] = bld<T>(xr, (DIM * J + c) * (uint32_t)sizeof(T));
        const bool up = oc > NU, lo = oc < NU;
        const uint32_t qU = (uint32_t)(oc - NU - 1) * BB, qL = (uint32_t)(NST - 1 - oc - NU - 1) * BB;
        const uint32_t at = lo ? J : un;
#pragma unroll
        for (int r = 0; r < DIM; ++r)
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const int lr = r < c ? r : c, hc = r < c ? c : r;
                const uint32_t qd = (uint32_t)(NU * BB + lr * DIM - lr * (lr - 1) / 2 + (hc - lr));
                const uint32_t q = up ? qU + (uint32_t)(r * DIM + c) : (lo ? qL + (uint32_t)(c * DIM + r) : qd);
                blk[sl][r * DIM + c] = bld<T>(sr, (q * uN + at) * (uint32_t)sizeof(T));
            }
    }
    __builtin_amdgcn_sched_barrier(0);
    // prolonged value of fine node (fi, fj, fk): x + sum of the corners, as in k_prolong
    auto pro = [&](int fi, int fj, int fk, const T (&xin)[DIM], T (&out)[DIM]) {
        int pa[2], pb[2], pc[2] = {lz, lz};
        T wa[2], wb[2], wc[2] = {T(1), T(0)};
        prolong_parents<T>(fi, nx, pa, wa);
        prolong_parents<T>(fj, ny, pb, wb);
        if (DIM == 3) prolong_parents<T>(fk, nz, pc, wc);
        T acc[DIM] = {};
#pragma unroll
        for (int q = 0; q < (DIM == 3 ? 8 : 4); ++q) {
            const int a2 = q & 1, b2 = (q >> 1) & 1, c2 = q >> 2;
            const T w = wa[a2] * wb[b2] * (DIM == 3 ? wc[c2] : T(1));
            const int sb = (pa[a2] - lx) + 3 * ((pb[b2] - ly) + (DIM == 3 ? 3 * (pc[c2] - lz) : 0));
#pragma unroll
            for (int c = 0; c < DIM; ++c) acc[c] += w * cblk[nl][sb][c];
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) out[c] = xin[c] + acc[c];
    };
    T xo[DIM];
    pro((int)ci[1], (int)cj[1], (int)ck[1], xraw, xo);
    // slot by slot (the sums in the order of k_stencil_split), so that only one
    // slot's prolonged values are live
    T acc[DIM] = {};
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
        const int oc = min(sl * P + p, NST - 1);
        const int dx = oc % 3, dy = (oc / 3) % 3, dz = DIM == 3 ? oc / 9 : 1;
        T xp[DIM];
        pro((int)ci[dx], (int)cj[dy], (int)ck[dz], xv[sl], xp);
        const bool lo = oc < NU;
        const bool keep = sl * P + p < NST && (!lo || (ii[dx] && ij[dy] && ik[dz]));
#pragma unroll
        for (int c = 0; c < DIM; ++c) xp[c] = keep ? xp[c] : T(0);
#pragma unroll
        for (int r = 0; r < DIM; ++r)
#pragma unroll
            for (int c = 0; c < DIM; ++c) acc[r] += blk[sl][r * DIM + c] * xp[c];
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int m = 1; m < P; m <<= 1)
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[c] += __shfl_xor(acc[c], m, 64);
    if (p == 0 && live) {
        // the step starts from the prolonged iterate, which is also the first
        // Chebyshev step's direction input (its coefficient is zero)
#pragma unroll
        for (int c = 0; c < DIM; ++c) fin.din[c] = xo[c];
        double dots[2];
        finish_store<T, DIM, OP>(node, acc, xo, 0, fin, y, omega, dots, ch);
    }
}

template <typename T, int DIM, int NB>
static void prolong_launch(int fl, const LaneIO* L, int n, hipStream_t s) {
    const Level& fine = L[0].h->lv[fl];
    Pack<ProlongA<T>, NB> pk{};
    for (int q = 0; q < n; ++q) {
        ProlongA<T>& a = pk.a[q];
        a.xc = (const T*)L[q].x;
        a.nm = fine.kind == TM_LEVEL_FINE ? L[q].h->lv[fl].nmask : nullptr;
        a.xf = (T*)L[q].y;
        a.done = L[q].done;
    }
    const dim3 g(grid_for(fine.n_nodes), n), blk(WG);
    hipLaunchKernelGGL((k_prolong<T, DIM, NB>), g, blk, 0, s, pk, fine.nel[0], fine.nel[1],
                       DIM == 3 ? fine.nel[2] : 0);
}

// x_f += M P x_c (lane x = coarse, y = fine)
// a small 2D geometric level (the small-level operator form) below a geometric
// level.  In 3D the fused step needs every register of a lane for its seven
// neighbour slots' prolonged values and was slower than the two launches, so
// 3D levels keep the separate prolongation.
bool stencil_pro_ok(const tm_hierarchy* h, int level) {
    if (level < 1 || level + 1 >= (int)h->lv.size() || h->dim != 2) return false;
    const Level& V = h->lv[level];
    if (V.kind != TM_LEVEL_GEOMETRIC || h->lv[level + 1].kind != TM_LEVEL_GEOMETRIC || V.xfer_bsr) return false;
    return V.op_kernel == 0 ? grid_for(V.n_nodes) < 256 : V.op_kernel == 2;
}

template <typename T, int DIM, int NB>
static void stencil_pro_launch(int level, const LaneIO* L, int n, int op, T omega, double c1, double c2,
                               hipStream_t s) {
    const Level& V = L[0].h->lv[level];
    auto pk = stencil_pack<T, NB>(level, L, n);
    for (int q = 0; q < n; ++q) pk.a[q].xc = (const T*)L[q].xc;
    const int nz = DIM == 3 ? V.nel[2] : 0;
    constexpr int P = DIM == 3 ? 4 : 1;
    const dim3 g(grid_for(V.n_nodes * P), n), blk(WG);
#define TM_SP(OPV)                                                                                   \
    hipLaunchKernelGGL((k_stencil_pro<T, DIM, OPV, P, NB>), g, blk, 0, s, pk, V.nel[0], V.nel[1], nz, V.n_nodes, \
                       omega, c1, c2)
    if (op == OP_CHEB)
        TM_SP(OP_CHEB);
    else
        TM_SP(OP_SMOOTH);
#undef TM_SP
}

template <typename T>
void launch_stencil_pro_b(int level, int op, const LaneIO* L, int n, T omega, double c1, double c2,
                          hipStream_t s) {
    if (n < 1) return;
    if (op != OP_CHEB && op != OP_SMOOTH) fail(TM_ERR_ARG, "fused prolongation takes a smoothing step");
    if (L[0].h->lv[level].dim != 2) fail(TM_ERR_ARG, "fused prolongation is for 2D levels");
    for (int q0 = 0; q0 < n; q0 += MAXB) {
        const int m = std::min(MAXB, n - q0);
        if (m == 1) stencil_pro_launch<T, 2, 1>(level, L + q0, 1, op, omega, c1, c2, s);
        else stencil_pro_launch<T, 2, MAXB>(level, L + q0, m, op, omega, c1, c2, s);
    }
}
template void launch_stencil_pro_b<double>(int, int, const LaneIO*, int, double, double, double, hipStream_t);
template void launch_stencil_pro_b<float>(int, int, const LaneIO*, int, float, double, double, hipStream_t);

template <typename T>
void launch_prolong_b(int fl, const LaneIO* L, int n, hipStream_t s) {
    if (n < 1) return;
    const int dim = L[0].h->lv[fl].dim;
    for (int q0 = 0; q0 < n; q0 += MAXB) {
        const int m = std::min(MAXB, n - q0);
        if (dim == 3) {
            if (m == 1) prolong_launch<T, 3, 1>(fl, L + q0, 1, s);
            else prolong_launch<T, 3, MAXB>(fl, L + q0, m, s);
        } else {
            if (m == 1) prolong_launch<T, 2, 1>(fl, L + q0, 1, s);
            else prolong_launch<T, 2, MAXB>(fl, L + q0, m, s);
        }
    }
}
template void launch_prolong_b<double>(int, const LaneIO*, int, hipStream_t);
template void launch_prolong_b<float>(int, const LaneIO*, int, hipStream_t);

// first smoothing sweep from x = 0:  x = omega D^-1 b  (block per node)
template <typename T, int BS, int NB>
__global__ __launch_bounds__(WG) void k_first_smooth(const Pack<FirstA<T>, NB> pk, int64_t N, T omega) {
    const FirstA<T>& A_ = lane_of(pk);
    const T* __restrict__ b = A_.b;
    const T* __restrict__ dinv = A_.dinv;
    T* __restrict__ x = A_.x;
    const int* __restrict__ done = A_.done;
    if (done && *done) return;
    const int64_t node = xcd_block() * WG + threadIdx.x;
    if (node >= N) return;
    T bv[BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) bv[c] = b[(int64_t)BS * node + c];
#pragma unroll
    for (int r = 0; r < BS; ++r) {
        T t = 0;
#pragma unroll
        for (int c = 0; c < BS; ++c) t += dinv[(int64_t)sym_at(r, c, BS) * N + node] * bv[c];
        x[(int64_t)BS * node + r] = omega * t;
    }
}

template <typename T, int BS, int NB>
static void first_launch(int l, const LaneIO* L, int n, T omega, hipStream_t s) {
    const Level& V = L[0].h->lv[l];
    Pack<FirstA<T>, NB> pk{};
    for (int q = 0; q < n; ++q) {
        FirstA<T>& a = pk.a[q];
        a.b = (const T*)L[q].b;
        a.dinv = dinv_of<T>(L[q].h->lv[l]);
        a.x = (T*)L[q].y;
        a.done = L[q].done;
    }
    hipLaunchKernelGGL((k_first_smooth<T, BS, NB>), dim3(grid_for(V.n_nodes), n), dim3(WG), 0, s, pk, V.n_nodes,
                       omega);
}

// first sweep from zero on level l: y = omega D^-1 b
template <typename T>
void launch_first_smooth_b(int l, const LaneIO* L, int n, T omega, hipStream_t s) {
    if (n < 1) return;
    const int bs = L[0].h->lv[l].bs;
    for (int q0 = 0; q0 < n; q0 += MAXB) {
        const int m = std::min(MAXB, n - q0);
#define TM_FS(BS)                                                         \
    if (m == 1) first_launch<T, BS, 1>(l, L + q0, 1, omega, s);           \
    else first_launch<T, BS, MAXB>(l, L + q0, m, omega, s);
        switch (bs) {
            case 2: TM_FS(2) break;
            case 3: TM_FS(3) break;
            case 6: TM_FS(6) break;
            default: fail(TM_ERR_ARG, "unsupported block size");
        }
#undef TM_FS
    }
}
template void launch_first_smooth_b<double>(int, const LaneIO*, int, double, hipStream_t);
template void launch_first_smooth_b<float>(int, const LaneIO*, int, float, hipStream_t);

}  // namespace tmi
