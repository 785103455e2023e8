// Fine-level kernels: SIMP moduli, point-block diagonal and the matrix-free
// operator K~ = M K M + (I - M), K = sum_e E_e L_e^T KE L_e (Sec. 2), applied
// node by node so that every output is summed in a fixed order (deterministic,
// no atomics): node i gathers its 3^dim neighbours once and accumulates
// E_e * KE[rows of i's local corner] * U_e over the 2^dim elements around it.
// KE is read through uniform (scalar) loads; the work is one 2^dim*dim-row
// slice of an element product per element per node, i.e. exactly the flops
// of the element-by-element product, without redundancy.
#include <type_traits>
#include <utility>

#include "tm_device.h"

namespace tmi {

// ------------------------------------------------------------ SIMP
__global__ void k_simp(const double* __restrict__ rho, int64_t n, double p, double E0, double Emin,
                       double* __restrict__ E64, float* __restrict__ E32, double* __restrict__ rho64,
                       int* flags) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double r = rho[e];
    if (!(r >= 0.0 && r <= 1.0)) {          // also catches NaN
        atomicOr(flags, FLAG_BAD_RHO);
        r = 0.0;
    }
    double E = Emin + (E0 - Emin) * pow(r, p);
    E64[e] = E;
    E32[e] = (float)E;
    rho64[e] = r;
}

void launch_simp(const double* rho, int64_t n_el, double p, double E0, double Emin, double* E64,
                 float* E32, double* rho64, int* flags, hipStream_t s) {
    hipLaunchKernelGGL(k_simp, dim3(grid_for(n_el)), dim3(WG), 0, s, rho, n_el, p, E0, Emin, E64,
                       E32, rho64, flags);
}

// ------------------------------------------------------------ sensitivities
// dc_e = -p rho_e^(p-1) (E0 - Emin) sum_k u_k,e^T KE u_k,e: the derivative of
// the summed compliances for the modified SIMP law (compliance is
// self-adjoint, Sec. 2).  One thread per element; KE enters as its class
// values with compile-time signs, u_e is gathered from the element's corners.
template <int DIM, int R, int S>
__device__ __forceinline__ double ke_entry(const KeVals<double>& kc) {
    constexpr int sg = DIM == 3 ? KE_CLS3.sgn[R][S] : KE_CLS2.sgn[R][S];
    constexpr int cl = DIM == 3 ? KE_CLS3.cls[R][S] : KE_CLS2.cls[R][S];
    if constexpr (sg > 0) return kc.k[cl];
    else if constexpr (sg < 0) return -kc.k[cl];
    else return 0.0;
}
template <int DIM, int R, int... S>
__device__ __forceinline__ double ke_row_dot(const KeVals<double>& kc, const double* ue,
                                             std::integer_sequence<int, S...>) {
    double t = 0.0;
    ((t += ke_entry<DIM, R, S>(kc) * ue[S]), ...);
    return t;
}
template <int DIM, int... R>
__device__ __forceinline__ double ke_quad(const KeVals<double>& kc, const double* ue,
                                          std::integer_sequence<int, R...>) {
    constexpr int ND = DIM << DIM;
    double q = 0.0;
    ((q += ue[R] * ke_row_dot<DIM, R>(kc, ue, std::make_integer_sequence<int, ND>{})), ...);
    return q;
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_sensitivity(const double* __restrict__ rho, const KeVals<double> kc,
                                                    int nx, int ny, int nz, int64_t n_el, int n_rhs,
                                                    const double* __restrict__ u, int64_t n_dof, double p,
                                                    double dE, double* __restrict__ dc) {
    constexpr int NPE = 1 << DIM, ND = DIM * NPE;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_el) return;
    const int ex = (int)(e % nx), ey = (int)((e / nx) % ny), ez = DIM == 3 ? (int)(e / ((int64_t)nx * ny)) : 0;
    const int64_t NX = nx + 1, NY = ny + 1;
    int64_t nd[NPE];
#pragma unroll
    for (int a = 0; a < NPE; ++a)
        nd[a] = (ex + corner_coord(a, 0)) + NX * ((ey + corner_coord(a, 1)) + (DIM == 3 ? NY * (ez + corner_coord(a, 2)) : 0));
    double q = 0.0;
    for (int k = 0; k < n_rhs; ++k) {
        const double* uk = u + (int64_t)k * n_dof;
        double ue[ND];
#pragma unroll
        for (int a = 0; a < NPE; ++a)
#pragma unroll
            for (int c = 0; c < DIM; ++c) ue[DIM * a + c] = uk[DIM * nd[a] + c];
        q += ke_quad<DIM>(kc, ue, std::make_integer_sequence<int, ND>{});
    }
    const double r = rho[e];
    dc[e] = -p * (p == 1.0 ? 1.0 : pow(r, p - 1.0)) * dE * q;
}

void launch_sensitivity(const tm_hierarchy* h, int n_rhs, const double* u, double* dc, hipStream_t s) {
    const Level& L = h->lv[0];
    const double dE = h->mat.E0 - h->mat.Emin;
    if (L.dim == 3)
        hipLaunchKernelGGL(k_sensitivity<3>, dim3(grid_for(h->n_el)), dim3(WG), 0, s, h->rho64, h->kc64, L.nel[0],
                           L.nel[1], L.nel[2], h->n_el, n_rhs, u, h->n_dof, h->mat.p, dE, dc);
    else
        hipLaunchKernelGGL(k_sensitivity<2>, dim3(grid_for(h->n_el)), dim3(WG), 0, s, h->rho64, h->kc64, L.nel[0],
                           L.nel[1], 1, h->n_el, n_rhs, u, h->n_dof, h->mat.p, dE, dc);
}

// ------------------------------------------------------------ fine diagonal
template <int DIM>
__global__ void k_fine_dinv(const double* __restrict__ E, const double* __restrict__ KE,
                            const uint8_t* __restrict__ nm, int nx, int ny, int nz, int64_t N,
                            int point, double* __restrict__ d64, float* __restrict__ d32,
                            int* flags) {
    constexpr int NPE = 1 << DIM, ND = DIM * NPE;
    int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= N) return;
    const int NX = nx + 1, NY = ny + 1;
    const int i = (int)(node % NX);
    const int j = (int)((node / NX) % NY);
    const int k = DIM == 3 ? (int)(node / ((int64_t)NX * NY)) : 0;
    double D[DIM][DIM] = {};
#pragma unroll
    for (int ez = 0; ez < (DIM == 3 ? 2 : 1); ++ez)
#pragma unroll
        for (int ey = 0; ey < 2; ++ey)
#pragma unroll
            for (int ex = 0; ex < 2; ++ex) {
                const int gx = i - 1 + ex, gy = j - 1 + ey, gz = k - 1 + ez;
                const bool ok = gx >= 0 && gx < nx && gy >= 0 && gy < ny &&
                                (DIM == 2 || (gz >= 0 && gz < nz));
                if (!ok) continue;
                const int64_t e = DIM == 3 ? ((int64_t)gz * ny + gy) * nx + gx : (int64_t)gy * nx + gx;
                const int a = DIM == 3 ? loc3(1 - ex, 1 - ey, 1 - ez) : loc2(1 - ex, 1 - ey);
                const double Ee = E[e];
#pragma unroll
                for (int r = 0; r < DIM; ++r)
#pragma unroll
                    for (int c = 0; c < DIM; ++c) D[r][c] += Ee * KE[(DIM * a + r) * ND + DIM * a + c];
            }
    const uint8_t m = nm[node];
#pragma unroll
    for (int r = 0; r < DIM; ++r)
        if (m & (1u << r)) {
#pragma unroll
            for (int c = 0; c < DIM; ++c) D[r][c] = D[c][r] = 0.0;
            D[r][r] = 1.0;
        }
    store_dinv<DIM>(D, point, node, N, d64, d32, flags);
}

void launch_fine_dinv(const Level& L, const double* KE64, int point_jacobi, int* flags,
                      hipStream_t s) {
    const dim3 g(grid_for(L.n_nodes)), b(WG);
    if (L.dim == 3)
        hipLaunchKernelGGL(k_fine_dinv<3>, g, b, 0, s, L.E64, KE64, L.nmask, L.nel[0], L.nel[1],
                           L.nel[2], L.n_nodes, point_jacobi, L.dinv64, L.dinv32, flags);
    else
        hipLaunchKernelGGL(k_fine_dinv<2>, g, b, 0, s, L.E64, KE64, L.nmask, L.nel[0], L.nel[1], 1,
                           L.n_nodes, point_jacobi, L.dinv64, L.dinv32, flags);
}

// 3D: 27 neighbour nodes, 8 elements, 24x24 KE.  Indices are 32-bit (dofs <
// 2^31 is checked at setup).  Neighbour loads use clamped coordinates and are
// unconditional; an element outside the grid gets modulus 0, so the values
// loaded for it (from a clamped, in-bounds node) contribute nothing.
//
// KE enters as its 12 symmetry-class values (kernel arguments, so they sit in
// scalar registers for the whole kernel); each entry is a class value with a
// compile-time sign.  The 27 neighbours are streamed one z-plane (9 nodes) at
// a time: plane dz holds corner layer bz = dz - ez of the elements of layer
// ez, so each (element, plane) pair gives a partial KE-row product that is
// scaled by the element's modulus and added to the node's accumulator at
// once, and only one plane of values is live.
template <int R, int S, typename T>
__device__ __forceinline__ void ke_fma3(const KeVals<T>& kc, T& t, T v) {
    constexpr int sg = KE_CLS3.sgn[R][S];
    constexpr int cl = KE_CLS3.cls[R][S];
    if constexpr (sg > 0) t += kc.k[cl] * v;
    else if constexpr (sg < 0) t -= kc.k[cl] * v;
}

template <int A, int BZ, int EY, int EX, typename T>
__device__ __forceinline__ void elem_plane3(const KeVals<T>& kc, const T (&w)[9][3], T (&t)[3]) {
    // corners (bx, by, BZ) of the element sit at plane offsets (EX+bx, EY+by)
#define TM_CORNER(BX, BY)                                                                         \
    {                                                                                              \
        constexpr int bb = loc3(BX, BY, BZ);                                                       \
        const T* vn = w[(EY + BY) * 3 + EX + BX];                                                  \
        ke_fma3<3 * A + 0, 3 * bb + 0>(kc, t[0], vn[0]);                                            \
        ke_fma3<3 * A + 0, 3 * bb + 1>(kc, t[0], vn[1]);                                            \
        ke_fma3<3 * A + 0, 3 * bb + 2>(kc, t[0], vn[2]);                                            \
        ke_fma3<3 * A + 1, 3 * bb + 0>(kc, t[1], vn[0]);                                            \
        ke_fma3<3 * A + 1, 3 * bb + 1>(kc, t[1], vn[1]);                                            \
        ke_fma3<3 * A + 1, 3 * bb + 2>(kc, t[1], vn[2]);                                            \
        ke_fma3<3 * A + 2, 3 * bb + 0>(kc, t[2], vn[0]);                                            \
        ke_fma3<3 * A + 2, 3 * bb + 1>(kc, t[2], vn[1]);                                            \
        ke_fma3<3 * A + 2, 3 * bb + 2>(kc, t[2], vn[2]);                                            \
    }
    TM_CORNER(0, 0)
    TM_CORNER(1, 0)
    TM_CORNER(0, 1)
    TM_CORNER(1, 1)
#undef TM_CORNER
}

// all elements of layer EZ that have corners in plane DZ
template <int DZ, int EZ, typename T>
__device__ __forceinline__ void layer_plane3(const KeVals<T>& kc, const T (&w)[9][3], const T (&Ee)[2][2][2],
                                             T (&acc)[3]) {
    constexpr int BZ = DZ - EZ;
    if constexpr (BZ >= 0 && BZ <= 1) {
#define TM_ELEM(EY, EX)                                                                           \
        {                                                                                          \
            T t[3] = {0, 0, 0};                                                                    \
            elem_plane3<loc3(1 - EX, 1 - EY, 1 - EZ), BZ, EY, EX>(kc, w, t);                       \
            acc[0] += Ee[EZ][EY][EX] * t[0];                                                       \
            acc[1] += Ee[EZ][EY][EX] * t[1];                                                       \
            acc[2] += Ee[EZ][EY][EX] * t[2];                                                       \
        }
        TM_ELEM(0, 0)
        TM_ELEM(0, 1)
        TM_ELEM(1, 0)
        TM_ELEM(1, 1)
#undef TM_ELEM
    }
}

template <typename T, int OP, bool MASK_IN, int NB>
__global__ __launch_bounds__(WG) void k_fine3(const Pack<OpA<T>, NB> pk, const KeVals<T> kc, int nx, int ny,
                                              int nz, int64_t N64, T omega, double c1, double c2) {
    const OpA<T>& A_ = lane_of(pk);
    const T* __restrict__ E = A_.E;
    const uint8_t* __restrict__ nm = A_.nm;
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
    double* partials = A_.partials;
    if (done && *done) return;
    const uint32_t N = (uint32_t)N64;
    const uint32_t node = (uint32_t)xcd_block() * WG + threadIdx.x;
    const bool live = node < N;
    const uint32_t NX = nx + 1, NY = ny + 1, NZ = nz + 1;
    const uint32_t nd = live ? node : 0u;
    const uint32_t i = nd % NX, tq = nd / NX, j = tq % NY, k = tq / NY;
    // neighbour node = node + ox[dx] + oy[dy] + oz[dz], clamped to the grid
    // (the operator zeroes what lies outside): additions only, no per-neighbour
    // integer multiplies (quarter rate)
    const uint32_t PL = NX * NY;
    const uint32_t ox[3] = {i ? 0u - 1u : 0u, 0u, i + 1 < NX ? 1u : 0u};
    const uint32_t oy[3] = {j ? 0u - NX : 0u, 0u, j + 1 < NY ? NX : 0u};
    const uint32_t oz[3] = {k ? 0u - PL : 0u, 0u, k + 1 < NZ ? PL : 0u};
    constexpr uint32_t NBY = 3u * sizeof(T);     // bytes per node
    // byte offsets of the neighbours, as sums; the empty asm keeps the
    // compiler from folding them back into one multiply per neighbour
    uint32_t nb0 = nd * NBY;
    asm volatile("" : "+v"(nb0));
    const uint32_t bx[3] = {i ? 0u - NBY : 0u, 0u, i + 1 < NX ? NBY : 0u};
    const uint32_t by[3] = {j ? 0u - NX * NBY : 0u, 0u, j + 1 < NY ? NX * NBY : 0u};
    const uint32_t bz[3] = {k ? 0u - PL * NBY : 0u, 0u, k + 1 < NZ ? PL * NBY : 0u};
    const auto xr = buf_rsrc(x, (int64_t)N * 3 * sizeof(T));
    const auto er = buf_rsrc(E, (int64_t)nx * ny * nz * sizeof(T));
    // moduli of the 8 elements around the node, [ez][ey][ex]: element with
    // lower corner (i-1+ex, j-1+ey, k-1+ez), index clamped, value zero outside
    const uint32_t EX = (uint32_t)nx, EP = EX * (uint32_t)ny;
    const uint32_t jE = j * EX, kE = k * EP;
    const uint32_t gx[2] = {i ? i - 1 : 0u, i < EX ? i : i - 1};
    const uint32_t gy[2] = {j ? jE - EX : 0u, j < (uint32_t)ny ? jE : jE - EX};
    const uint32_t gz[2] = {k ? kE - EP : 0u, k < (uint32_t)nz ? kE : kE - EP};
    T Ee[2][2][2];
#pragma unroll
    for (int ez = 0; ez < 2; ++ez)
#pragma unroll
        for (int ey = 0; ey < 2; ++ey)
#pragma unroll
            for (int ex = 0; ex < 2; ++ex) {
                const bool in = (ex || i) && (ex == 0 || i < (uint32_t)nx) && (ey || j) &&
                                (ey == 0 || j < (uint32_t)ny) && (ez || k) && (ez == 0 || k < (uint32_t)nz);
                Ee[ez][ey][ex] = in ? bld<T>(er, (gz[ez] + gy[ey] + gx[ex]) * (uint32_t)sizeof(T)) : T(0);
            }
    T acc[3] = {0, 0, 0};
    T w[9][3];
    auto load_plane = [&](int dz) {
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const uint32_t row = nd + oz[dz] + oy[dy];
            const uint32_t rowb = nb0 + bz[dz] + by[dy];
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const uint32_t id = row + ox[dx];
                T a[3];
                bld3(xr, rowb + bx[dx], a);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (MASK_IN) a[c] = ((nm[id] >> c) & 1u) ? T(0) : a[c];
                    w[dy * 3 + dx][c] = a[c];
                }
            }
        }
    };
    // the finishing step's operands (b, block inverse, direction, mask) are
    // requested first, so that they arrive while the neighbours are gathered
    FinIn<T, 3> fin;
    finish_load<T, 3, OP>(nd, N, b, dinv, ch, fin);
    const uint8_t mo = nm[nd];
    load_plane(0);
    layer_plane3<0, 0>(kc, w, Ee, acc);
    load_plane(1);
    T xo[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) xo[c] = w[4][c];     // this node's own value
    if (MASK_IN) {
#pragma unroll
        for (int c = 0; c < 3; ++c) xo[c] = x[3u * nd + c];
    }
    layer_plane3<1, 0>(kc, w, Ee, acc);
    layer_plane3<1, 1>(kc, w, Ee, acc);
    load_plane(2);
    layer_plane3<2, 1>(kc, w, Ee, acc);
    double dots[2] = {0.0, 0.0};
    if (live) finish_store<T, 3, OP>(node, acc, xo, mo, fin, y, omega, dots, ch);
    if (OP == OP_QDOT) block_reduce_store<2>(dots, partials);
}

// The same operator for two nodes stacked in z per thread (k even, k + 1):
// their neighbourhoods share two of the four planes k-1 .. k+2, so a thread
// gathers 36 neighbour values and 12 moduli for two nodes instead of 54 and 16.
// Each node's terms are summed in the order of k_fine3 (layer 0 of plane 0,
// layers 0 and 1 of plane 1, layer 1 of plane 2), so the results are bitwise
// those of k_fine3.  Used for the V-cycle's operators (no partial sums).
template <typename T, int OP, int NB>
__global__ __launch_bounds__(WG) void k_fine3z2(const Pack<OpA<T>, NB> pk, const KeVals<T> kc, int nx, int ny,
                                                int nz, int64_t N64, T omega, double c1, double c2) {
    static_assert(OP != OP_QDOT, "no partial sums in the two-node operator");
    const OpA<T>& A_ = lane_of(pk);
    const T* __restrict__ E = A_.E;
    const uint8_t* __restrict__ nm = A_.nm;
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
    const uint32_t N = (uint32_t)N64;
    const uint32_t NX = nx + 1, NY = ny + 1, NZ = nz + 1, PL = NX * NY;
    const uint32_t NT = PL * ((NZ + 1) / 2);           // threads: z pairs
    const uint32_t p = (uint32_t)xcd_block() * WG + threadIdx.x;
    const bool live = p < NT;
    const uint32_t pp = live ? p : 0u;
    const uint32_t i = pp % NX, tq = pp / NX, j = tq % NY, k = 2u * (tq / NY);
    const bool two = k + 1 < NZ;                        // the upper node exists
    const uint32_t nd0 = k * PL + j * NX + i;
    const uint32_t nd1 = two ? nd0 + PL : nd0;
    constexpr uint32_t NBY = 3u * sizeof(T);
    uint32_t nb0 = nd0 * NBY;
    asm volatile("" : "+v"(nb0));
    const uint32_t bx[3] = {i ? 0u - NBY : 0u, 0u, i + 1 < NX ? NBY : 0u};
    const uint32_t by[3] = {j ? 0u - NX * NBY : 0u, 0u, j + 1 < NY ? NX * NBY : 0u};
    // planes k-1 .. k+2 relative to node k, clamped into the grid (what lies
    // outside only meets elements of modulus zero)
    const uint32_t bz[4] = {k ? 0u - PL * NBY : 0u, 0u, k + 1 < NZ ? PL * NBY : 0u,
                            k + 2 < NZ ? 2u * PL * NBY : (k + 1 < NZ ? PL * NBY : 0u)};
    const auto xr = buf_rsrc(x, (int64_t)N * 3 * sizeof(T));
    const auto er = buf_rsrc(E, (int64_t)nx * ny * nz * sizeof(T));
    // moduli of element layers k-1, k, k+1 (index clamped, zero outside)
    const uint32_t EX = (uint32_t)nx, EP = EX * (uint32_t)ny;
    const uint32_t jE = j * EX;
    const uint32_t gx[2] = {i ? i - 1 : 0u, i < EX ? i : i - 1};
    const uint32_t gy[2] = {j ? jE - EX : 0u, j < (uint32_t)ny ? jE : jE - EX};
    T El[3][2][2];
#pragma unroll
    for (int lz = 0; lz < 3; ++lz) {
        const int layer = (int)k - 1 + lz;
        const bool zin = layer >= 0 && layer < nz;
        const uint32_t gz = zin ? (uint32_t)layer * EP : 0u;
#pragma unroll
        for (int ey = 0; ey < 2; ++ey)
#pragma unroll
            for (int ex = 0; ex < 2; ++ex) {
                const bool in = zin && (ex || i) && (ex == 0 || i < (uint32_t)nx) && (ey || j) &&
                                (ey == 0 || j < (uint32_t)ny);
                El[lz][ey][ex] = in ? bld<T>(er, (gz + gy[ey] + gx[ex]) * (uint32_t)sizeof(T)) : T(0);
            }
    }
    T E0[2][2][2], E1[2][2][2];
#pragma unroll
    for (int ez = 0; ez < 2; ++ez)
#pragma unroll
        for (int ey = 0; ey < 2; ++ey)
#pragma unroll
            for (int ex = 0; ex < 2; ++ex) {
                E0[ez][ey][ex] = El[ez][ey][ex];
                E1[ez][ey][ex] = El[ez + 1][ey][ex];
            }
    T acc0[3] = {0, 0, 0}, acc1[3] = {0, 0, 0};
    T w[9][3];
    auto load_plane = [&](int P) {
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const uint32_t rowb = nb0 + bz[P] + by[dy];
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) bld3(xr, rowb + bx[dx], w[dy * 3 + dx]);
        }
    };
    FinIn<T, 3> fin0, fin1;
    finish_load<T, 3, OP>(nd0, N, b, dinv, ch, fin0);
    finish_load<T, 3, OP>(nd1, N, b, dinv, ch, fin1);
    const uint8_t m0 = nm[nd0], m1 = nm[nd1];
    load_plane(0);
    layer_plane3<0, 0>(kc, w, E0, acc0);
    load_plane(1);
    T xo0[3], xo1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) xo0[c] = w[4][c];
    layer_plane3<1, 0>(kc, w, E0, acc0);
    layer_plane3<1, 1>(kc, w, E0, acc0);
    layer_plane3<0, 0>(kc, w, E1, acc1);
    load_plane(2);
#pragma unroll
    for (int c = 0; c < 3; ++c) xo1[c] = w[4][c];
    layer_plane3<2, 1>(kc, w, E0, acc0);
    layer_plane3<1, 0>(kc, w, E1, acc1);
    layer_plane3<1, 1>(kc, w, E1, acc1);
    load_plane(3);
    layer_plane3<2, 1>(kc, w, E1, acc1);
    double dots[2] = {0.0, 0.0};
    if (live) finish_store<T, 3, OP>(nd0, acc0, xo0, m0, fin0, y, omega, dots, ch);
    if (live && two) finish_store<T, 3, OP>(nd1, acc1, xo1, m1, fin1, y, omega, dots, ch);
}

// 3D fine operator in the tensor-product form (SfSlots), FP32 for the V-cycle
// and FP64 for the outer q = K~p (with its partial sums) and the FP64 V-cycle.
// A workgroup owns a tile of
// SF_NX x SF_NY node columns and a range of node planes; its SF_TX x SF_TY threads
// are the element columns around the tile (one ring beyond it, so every owned
// node has all of its elements), each marching up its column one element
// layer at a time.  Per layer, a thread:
//   loads the four corner values of the layer's top face and forms their face
//   modes (sums and differences in x and y; the bottom face's modes are the
//   previous layer's top),
//   forms the element's eight modes per component (z sum and difference),
//   scales them by the element's modulus and applies the 45 couplings,
//   splits the result back into bottom- and top-face modes, adds the bottom
//   ones to the previous layer's top ones (both belong to the bottom face's
//   node plane) and turns them into the face's four corner values,
//   which go to LDS; after one barrier each owned node adds the corner values
//   of its four element columns (own column first, then +x, +y, +x+y) and
//   finishes as the node-gather form does.
// An element outside the grid has modulus zero; the corner loads of such
// columns read clamped in-grid nodes, so every value stays finite.  The tile
// is 32 x 8 columns: wider rows coalesce better, narrower tiles repeat more
// columns in their halo ring.
constexpr int SF_TX = 32, SF_TY = 8;                // element columns per tile
constexpr int SF_NX = SF_TX - 1, SF_NY = SF_TY - 1;  // owned node columns per tile

template <int I, typename T>
__device__ __forceinline__ void sf_couple(const SfCoef<T>& cf, const T (&md)[8][3], T (&o)[8][3]) {
    if constexpr (I < 72) {
        constexpr int c = I / 24, d = (I / 8) % 3, m = I % 8;
        constexpr int sl = SF_SLOTS.s[c][d][m];
        if constexpr (sl >= 0) {
            constexpr int mo = sf_out_mode(c, d, m);
            o[mo][c] = fma_of(cf.k[sl], md[m][d], o[mo][c]);
        }
        sf_couple<I + 1, T>(cf, md, o);
    }
}

// face modes of corner values v[2 ly + lx][c]: [0] sum, [1] x difference,
// [2] y difference, [3] both
template <typename T>
__device__ __forceinline__ void sf_face_modes(const T (&v)[4][3], T (&m)[4][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T s0 = v[0][c] + v[1][c], d0 = v[1][c] - v[0][c];
        const T s1 = v[2][c] + v[3][c], d1 = v[3][c] - v[2][c];
        m[0][c] = s0 + s1;
        m[1][c] = d0 + d1;
        m[2][c] = s1 - s0;
        m[3][c] = d1 - d0;
    }
}

// three consecutive values stored at byte offset off (one 12-byte store in
// FP32, a 16- and an 8-byte store in FP64); an offset past the descriptor's
// end drops the store
__device__ __forceinline__ void bst3(__amdgpu_buffer_rsrc_t r, uint32_t off, const float (&v)[3]) {
    typedef float f3 __attribute__((ext_vector_type(3)));
    __builtin_amdgcn_raw_buffer_store_b96(f3{v[0], v[1], v[2]}, r, off, 0, 0);
}
__device__ __forceinline__ void bst3(__amdgpu_buffer_rsrc_t r, uint32_t off, const double (&v)[3]) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, d2{v[0], v[1]}), r, off, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v[2]), r, off + 16, 0, 0);
}

// Level 1 in the tensor form.  With every fine element count even, each
// level-1 element holds 2 x 2 x 2 fine elements, and the Galerkin product is
// the sum over them of P_k^T (E_k M_k KE M_k) P_k (P_k the trilinear
// interpolation from the element's corners to sub-element k's, M_k the
// supports).  Per axis, in sum / difference modes, P_k maps (sigma, delta) to
// (sigma -+ delta / 2, delta / 2) for the lower / upper half, and its
// transpose maps output modes back as (sigma, (delta -+ sigma) / 2); the
// sub-element's modes then take the 45 couplings like a fine element.
template <int A, typename T>
__device__ __forceinline__ void sf_half(T (&m)[8][3], int h) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
        if (!((i >> A) & 1)) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T d = m[i | (1 << A)][c] * T(0.5);
                m[i][c] = h ? m[i][c] + d : m[i][c] - d;
                m[i | (1 << A)][c] = d;
            }
        }
}
template <int A, typename T>
__device__ __forceinline__ void sf_half_t(T (&m)[8][3], int h) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
        if (!((i >> A) & 1)) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T sg = m[i][c], dl = m[i | (1 << A)][c];
                m[i | (1 << A)][c] = (h ? dl + sg : dl - sg) * T(0.5);
            }
        }
}
// a sub-element with supported dofs: modes to corner values (corner index
// lx | ly << 1 | lz << 2), supported components zeroed, back to modes; IN
// selects the input side (values = F^-1 modes, modes = F values) or the output
// side (values = F^T modes, modes = F^-T values)
template <bool IN, typename T>
__device__ __forceinline__ void sf_mask(T (&m)[8][3], const uint32_t (&mk)[8]) {
#pragma unroll
    for (int A = 0; A < 3; ++A)
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (!((i >> A) & 1)) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T a = m[i][c], b = m[i | (1 << A)][c];
                    m[i][c] = IN ? (a - b) * T(0.5) : a - b;
                    m[i | (1 << A)][c] = IN ? (a + b) * T(0.5) : a + b;
                }
            }
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if ((mk[i] >> c) & 1u) m[i][c] = T(0);
#pragma unroll
    for (int A = 0; A < 3; ++A)
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (!((i >> A) & 1)) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T a = m[i][c], b = m[i | (1 << A)][c];
                    m[i][c] = IN ? a + b : (a + b) * T(0.5);
                    m[i | (1 << A)][c] = IN ? b - a : (b - a) * T(0.5);
                }
            }
}

// cv: the plane's corner values per element column, two buffers (LDS)
// GAL: level 1 in the tensor form (nx, ny, nz its element counts; E, nm the
// fine level's moduli and supports; no supports on level 1 itself).
// PRO: the iterate is x + P~ xc (xc the level-1 correction, P~ the trilinear
// prolongation with the supported dofs left out, fine counts even), formed
// as each face is loaded: the first post-smoothing step with the prolongation
// in it (nothing stores x + P~ xc itself)
template <typename T, int OP, int NB, bool GAL = false, bool PRO = false>
__device__ __forceinline__ void fine3sf_body(const Pack<OpA<T>, NB>& pk, const SfCoef<T>& cf, int nx, int ny,
                                             int nz, int tiles_x, int tiles_y, int zlen, T omega, double c1,
                                             double c2, T (&cv)[2][4][3][SF_TX * SF_TY]) {
    static_assert(OP != OP_QDOT || std::is_same<T, double>::value, "partial sums in the FP64 form only");
    const OpA<T>& A_ = lane_of(pk);
    const int* __restrict__ done = A_.done;
    if (done && *done) return;
    const uint32_t NX = nx + 1, NY = ny + 1, NZ = nz + 1, PL = NX * NY, N = PL * NZ;
    const uint32_t blk = (uint32_t)xcd_block();
    const uint32_t bx = blk % (uint32_t)tiles_x, br = blk / (uint32_t)tiles_x;
    const uint32_t by = br % (uint32_t)tiles_y, bz = br / (uint32_t)tiles_y;
    const int t = threadIdx.x;
    const int tx = t % SF_TX, ty = t / SF_TX;
    const int ex = (int)bx * SF_NX - 1 + tx, ey = (int)by * SF_NY - 1 + ty;
    const bool ecol = ex >= 0 && ex < nx && ey >= 0 && ey < ny;
    const uint32_t ix0 = (uint32_t)min(max(ex, 0), (int)NX - 1), ix1 = (uint32_t)min(max(ex + 1, 0), (int)NX - 1);
    const uint32_t iy0 = (uint32_t)min(max(ey, 0), (int)NY - 1), iy1 = (uint32_t)min(max(ey + 1, 0), (int)NY - 1);
    constexpr uint32_t NBY = 3u * sizeof(T);
    const uint32_t fo[4] = {(iy0 * NX + ix0) * NBY, (iy0 * NX + ix1) * NBY, (iy1 * NX + ix0) * NBY,
                            (iy1 * NX + ix1) * NBY};
    // owned node: the column's upper corner in x and y
    const uint32_t own_col = iy1 * NX + ix1;
    const bool own = tx < SF_NX && ty < SF_NY && ex + 1 < (int)NX && ey + 1 < (int)NY;
    const uint32_t EP = (uint32_t)nx * (uint32_t)ny;
    const uint32_t ecix = ecol ? (uint32_t)ey * (uint32_t)nx + (uint32_t)ex : 0u;
    const int k0 = (int)bz * zlen;
    const int k1 = min(k0 + zlen, (int)NZ);
    // Every access goes through a buffer descriptor with a clamped offset, and
    // the loop body has no branch besides its barrier, so the compiler can
    // wait for exactly the loads a step reads while later ones stay in
    // flight.  A store of a node the thread does not own (or of a plane past
    // the range) gets an offset past the descriptor's end, which the hardware
    // drops; with no direction output the direction descriptor is empty.
    const auto xr = buf_rsrc(A_.x, (int64_t)N * NBY);
    const auto er = buf_rsrc(A_.E, (int64_t)EP * nz * (GAL ? 8 : 1) * sizeof(T));
    const auto mr = buf_rsrc(A_.nm, GAL ? (int64_t)(2 * nx + 1) * (2 * ny + 1) * (2 * nz + 1) : (int64_t)N);
    const auto fr = buf_rsrc(A_.sub, GAL ? (int64_t)EP * nz : 0);
    // GAL: the clamped element column (every index stays in bounds)
    const uint32_t exc = (uint32_t)min(max(ex, 0), nx - 1), eyc = (uint32_t)min(max(ey, 0), ny - 1);
    const auto brs = buf_rsrc(A_.b, OP == OP_APPLY ? 0 : (int64_t)N * NBY);
    const auto dr = buf_rsrc(A_.dinv, OP == OP_SMOOTH || OP == OP_CHEB ? (int64_t)6 * N * sizeof(T) : 0);
    const auto inr = buf_rsrc(A_.din, OP == OP_CHEB && A_.din ? (int64_t)N * NBY : 0);
    const auto yr = buf_rsrc(A_.y, (int64_t)N * NBY);
    const auto dor = buf_rsrc(A_.dout, OP == OP_CHEB && A_.dout ? (int64_t)N * NBY : 0);
    const T fc1 = (T)c1, fc2 = (T)c2;
    // PRO: the level-1 nodes around the column (two per axis, clamped)
    const uint32_t CX = (uint32_t)nx / 2u + 1u, CY = (uint32_t)ny / 2u + 1u, CZ = (uint32_t)nz / 2u + 1u;
    const auto cr = buf_rsrc(A_.xc, PRO ? (int64_t)CX * CY * CZ * NBY : 0);
    const uint32_t ax = ix0 >> 1, ay = iy0 >> 1;
    const uint32_t cxo[2] = {ax, (uint32_t)min(ax + 1u, CX - 1u)}, cyo[2] = {ay, (uint32_t)min(ay + 1u, CY - 1u)};
    // weight of the lower level-1 node per axis at the column's two node
    // positions (the upper one takes the rest): odd positions lie halfway,
    // even ones on a level-1 node
    T ux[2], uy[2];
#pragma unroll
    for (int lq = 0; lq < 2; ++lq) {
        const uint32_t i = lq ? ix1 : ix0, j = lq ? iy1 : iy0;
        ux[lq] = (i & 1u) ? T(0.5) : ((i >> 1) == ax ? T(1) : T(0));
        uy[lq] = (j & 1u) ? T(0.5) : ((j >> 1) == ay ? T(1) : T(0));
    }
    // the four level-1 nodes of the column in level-1 plane a (clamped), and
    // their interpolation to the face's corners in x and y
    auto pro_plane = [&](int a, T (&cc)[2][2][3]) {
        const uint32_t az = (uint32_t)min(a, (int)CZ - 1);
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int x = 0; x < 2; ++x) bld3(cr, ((az * CY + cyo[y]) * CX + cxo[x]) * NBY, cc[y][x]);
    };
    auto pro_xy = [&](const T (&cc)[2][2][3], T (&s)[4][3]) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T u = ux[q & 1];
                const T r0 = cc[0][1][c] + u * (cc[0][0][c] - cc[0][1][c]);
                const T r1 = cc[1][1][c] + u * (cc[1][0][c] - cc[1][1][c]);
                s[q][c] = r1 + uy[q >> 1] * (r0 - r1);
            }
    };
    // PRO: the correction at the face's corners on level-1 plane za, and the
    // level-1 values of plane za + 1
    T sa[4][3], cb[2][2][3];
    int za = -2;
    auto load_face = [&](int p, T (&v)[4][3]) {
        const uint32_t pc = (uint32_t)min(max(p, 0), (int)NZ - 1);
        const uint32_t pb = pc * PL * NBY;
#pragma unroll
        for (int q = 0; q < 4; ++q) bld3(xr, pb + fo[q], v[q]);
        if constexpr (PRO) {
            // the march takes the planes in order, so each level-1 plane is
            // loaded once: plane a + 1 as soon as the march reaches plane a
            const int az = (int)(pc >> 1);
            if (az != za) {
                if (az == za + 1) {
                    pro_xy(cb, sa);
                } else {
                    T c0[2][2][3];
                    pro_plane(az, c0);
                    pro_xy(c0, sa);
                }
                pro_plane(az + 1, cb);
                za = az;
            }
            T sb[4][3];
            pro_xy(cb, sb);
            const T hz = (pc & 1u) ? T(0.5) : T(0);
            uint32_t mk[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) mk[q] = __builtin_amdgcn_raw_buffer_load_b8(mr, pc * PL + fo[q] / NBY, 0, 0);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T a = sa[q][c] + hz * (sb[q][c] - sa[q][c]);
                    v[q][c] += ((mk[q] >> c) & 1u) ? T(0) : a;
                }
        }
    };
    // operands of element layer l: its top face's corners and its modulus
    // (with weight 0 for an element outside the grid, applied where the
    // layer is used, so that nothing waits for the load when it is issued)
    struct Face {
        T v[4][3];
        T E[GAL ? 8 : 1], w;
        uint32_t f;     // GAL: sub-element support flags
    };
    auto fetch_face = [&](int l, Face& F) {
        load_face(l + 1, F.v);
        const uint32_t lz = (uint32_t)min(max(l, 0), nz - 1);
        if constexpr (GAL) {
            // the eight fine moduli, two consecutive ones per (z, y) pair
            const uint32_t FX = 2u * (uint32_t)nx, FP = FX * 2u * (uint32_t)ny;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                T e2[2];
                bld2(er, (((2u * lz + (q >> 1)) * FP) + (2u * eyc + (q & 1)) * FX + 2u * exc) * (uint32_t)sizeof(T), e2);
                F.E[2 * q] = e2[0];
                F.E[2 * q + 1] = e2[1];
            }
            F.f = __builtin_amdgcn_raw_buffer_load_b8(fr, lz * EP + eyc * (uint32_t)nx + exc, 0, 0);
        } else {
            F.E[0] = bld<T>(er, (lz * EP + ecix) * (uint32_t)sizeof(T));
        }
        F.w = (ecol && l >= 0 && l < nz) ? T(1) : T(0);
    };
    // finishing operands of the owned node in plane l
    struct Fin {
        T b[3], dv[6], din[3];
        uint32_t m;
    };
    auto node_of = [&](int l) { return (uint32_t)min(max(l, 0), (int)NZ - 1) * PL + own_col; };
    auto fetch_fin = [&](int l, Fin& f) {
        const uint32_t nd = node_of(l);
        if (OP != OP_APPLY) bld3(brs, nd * NBY, f.b);
        if (OP == OP_SMOOTH || OP == OP_CHEB) {
#pragma unroll
            for (int e = 0; e < 6; ++e) f.dv[e] = bld<T>(dr, ((uint32_t)e * N + nd) * (uint32_t)sizeof(T));
        }
        if (OP == OP_CHEB) bld3(inr, nd * NBY, f.din);
        f.m = GAL ? 0u : __builtin_amdgcn_raw_buffer_load_b8(mr, nd, 0, 0);
    };
    // element layer l from its top face S and the bottom face's modes fb:
    // the plane-l face modes pm (this layer's bottom plus the layer below's
    // top, st), and st, fb for the next layer
    T fb[4][3], st[4][3];
    // GAL: the supports of sub-element k's corners (fine nodes, clamped)
    auto sub_masks = [&](int l, int k, uint32_t (&mk)[8]) {
        const uint32_t FNX = 2u * (uint32_t)nx + 1u, FPL = FNX * (2u * (uint32_t)ny + 1u);
        const uint32_t lz = (uint32_t)min(max(l, 0), nz - 1);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint32_t fx = 2u * exc + (k & 1) + (c & 1), fy = 2u * eyc + ((k >> 1) & 1) + ((c >> 1) & 1);
            const uint32_t fz = 2u * lz + (k >> 2) + (c >> 2);
            mk[c] = __builtin_amdgcn_raw_buffer_load_b8(mr, fz * FPL + fy * FNX + fx, 0, 0);
        }
    };
    auto layer = [&](int l, const T (&v)[4][3], const Face& F, T (&pm)[4][3]) {
        T ft[4][3];
        sf_face_modes(v, ft);
        T md[8][3], o[8][3];
        const T Ee = F.E[0] * F.w;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                md[q][c] = GAL ? ft[q][c] + fb[q][c] : Ee * (ft[q][c] + fb[q][c]);
                md[q + 4][c] = GAL ? ft[q][c] - fb[q][c] : Ee * (ft[q][c] - fb[q][c]);
                o[q][c] = T(0);
                o[q + 4][c] = T(0);
            }
        if constexpr (GAL) {
            // the eight sub-elements, in a fixed order (x fastest), one at a
            // time (unrolled, their registers would not fit)
#pragma unroll 1
            for (int k = 0; k < 8; ++k) {
                T mf[8][3], of[8][3];
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        mf[i][c] = md[i][c];
                        of[i][c] = T(0);
                    }
                sf_half<0>(mf, k & 1);
                sf_half<1>(mf, (k >> 1) & 1);
                sf_half<2>(mf, k >> 2);
                const bool msk = (F.f >> k) & 1u;
                uint32_t mk[8];
                if (msk) {
                    sub_masks(l, k, mk);
                    sf_mask<true>(mf, mk);
                }
                T ek = F.E[0];
#pragma unroll
                for (int q = 1; q < 8; ++q) ek = k == q ? F.E[q] : ek;
                ek *= F.w;
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int c = 0; c < 3; ++c) mf[i][c] *= ek;
                sf_couple<0, T>(cf, mf, of);
                if (msk) sf_mask<false>(of, mk);
                sf_half_t<0>(of, k & 1);
                sf_half_t<1>(of, (k >> 1) & 1);
                sf_half_t<2>(of, k >> 2);
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int c = 0; c < 3; ++c) o[i][c] += of[i][c];
            }
        } else {
            sf_couple<0, T>(cf, md, o);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                pm[q][c] = st[q][c] + (o[q][c] - o[q + 4][c]);
                st[q][c] = o[q][c] + o[q + 4][c];
                fb[q][c] = ft[q][c];
            }
    };
    T xo[3];            // the owned node's value in the plane being finished
    // the operands of one step: layer l's top face and modulus, and the
    // finishing operands of node plane l
    struct Ops {
        Face f;
        Fin n;
    };
    auto fetch = [&](int l, Ops& o) {
        fetch_fin(l, o.n);
        fetch_face(l, o.f);
    };
    Ops OA, OB;
    {
        // layer k0 - 1: only its top-face outputs (plane k0) are kept
        T v0[4][3];
        load_face(k0 - 1, v0);
        Face F0;
        fetch_face(k0 - 1, F0);
        if (!GAL && !PRO) fetch(k0, OA);
        sf_face_modes(v0, fb);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) st[q][c] = T(0);
        T pm[4][3];
        layer(k0 - 1, F0.v, F0, pm);
#pragma unroll
        for (int c = 0; c < 3; ++c) xo[c] = F0.v[3][c];
    }
    // plane l from the operands C, fetched during the previous step while the
    // next ones go to the other set (two sets alternate, the march being
    // unrolled by two, so no set is copied while its loads are in flight and
    // every load has a whole step to arrive)
    double dots[2] = {0.0, 0.0};
    auto step = [&](int l, const Ops& C) {
        const Fin& fin = C.n;
        T pm[4][3];
        layer(l, C.f.v, C.f, pm);
        __builtin_amdgcn_sched_barrier(0);          // the finishing operands are read below
        const int buf = (l - k0) & 1;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T P = pm[0][c] + pm[2][c], Q = pm[0][c] - pm[2][c];
            const T R = pm[1][c] + pm[3][c], U = pm[1][c] - pm[3][c];
            cv[buf][0][c][t] = Q - U;
            cv[buf][1][c][t] = Q + U;
            cv[buf][2][c][t] = P - R;
            cv[buf][3][c][t] = P + R;
        }
        __syncthreads();
        // the four columns' corner values at the owned node (threads that own
        // none read their own slots instead, and store nothing)
        const int t1 = own ? t + 1 : t, t16 = own ? t + SF_TX : t, t17 = own ? t + SF_TX + 1 : t;
        T kx[3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            kx[c] = ((cv[buf][3][c][t] + cv[buf][2][c][t1]) + cv[buf][1][c][t16]) + cv[buf][0][c][t17];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (fin.m & (1u << c)) kx[c] = xo[c];           // unit row of a supported dof
        const bool live = own && l < k1;
        T yv[3], dn[3] = {T(0), T(0), T(0)};
        if (OP == OP_APPLY || OP == OP_QDOT) {
#pragma unroll
            for (int c = 0; c < 3; ++c) yv[c] = kx[c];
        } else if (OP == OP_RESID) {
#pragma unroll
            for (int c = 0; c < 3; ++c) yv[c] = fin.b[c] - kx[c];
        } else {
            T rr[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) rr[c] = fin.b[c] - kx[c];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                T s = T(0);
#pragma unroll
                for (int c = 0; c < 3; ++c) s += fin.dv[sym_at(r, c, 3)] * rr[c];
                if (OP == OP_SMOOTH) {
                    yv[r] = xo[r] + omega * s;
                } else {
                    dn[r] = fma_of(s, fc2, fc1 * fin.din[r]);
                    yv[r] = xo[r] + dn[r];
                }
            }
        }
        if (OP == OP_QDOT) {
            // p^T q and p^T r (b holds r) over the owned nodes of the range
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                dots[0] += live ? (double)xo[c] * (double)kx[c] : 0.0;
                dots[1] += live ? (double)xo[c] * (double)fin.b[c] : 0.0;
            }
        }
        // the dropped stores' offset stays past any descriptor's end (at most
        // 2^31 - 1 bytes) also after the 16 bytes the FP64 form adds for its
        // third value, without wrapping around 2^32
        const uint32_t so = live ? node_of(l) * NBY : 0xfffff000u;
        bst3(yr, so, yv);
        if (OP == OP_CHEB) bst3(dor, so, dn);
#pragma unroll
        for (int c = 0; c < 3; ++c) xo[c] = C.f.v[3][c];
    };
    if constexpr (GAL || PRO) {
        // level 1 is bound by its arithmetic, and the prolonged iterate needs
        // its loads at once: each step fetches its own operands
        for (int l = k0; l < k1; ++l) {
            Ops C;
            fetch(l, C);
            step(l, C);
        }
    } else {
        // an even number of steps (a last one past the range stores nothing)
        for (int l = k0; l < k1; l += 2) {
            fetch(l + 1, OB);
            __builtin_amdgcn_sched_barrier(0);      // keep the next step's loads first
            step(l, OA);
            fetch(l + 2, OA);
            __builtin_amdgcn_sched_barrier(0);
            step(l + 1, OB);
        }
    }
    if (OP == OP_QDOT) block_reduce_store<2>(dots, A_.partials);
}

template <int OP, int NB>
__global__ __launch_bounds__(SF_TX * SF_TY) __attribute__((amdgpu_waves_per_eu(4))) void k_fine3sf(
    const Pack<OpA<float>, NB> pk, const SfCoef<float> cf, int nx, int ny, int nz, int tiles_x, int tiles_y,
    int zlen, float omega, double c1, double c2) {
    __shared__ float cv[2][4][3][SF_TX * SF_TY];
    fine3sf_body<float, OP, NB>(pk, cf, nx, ny, nz, tiles_x, tiles_y, zlen, omega, c1, c2, cv);
}

template <int OP, int NB>
__global__ __launch_bounds__(SF_TX * SF_TY) __attribute__((amdgpu_waves_per_eu(4))) void k_fine3sf_pro(const Pack<OpA<float>, NB> pk, const SfCoef<float> cf,
                                                               int nx, int ny, int nz, int tiles_x, int tiles_y,
                                                               int zlen, float omega, double c1, double c2) {
    __shared__ float cv[2][4][3][SF_TX * SF_TY];
    fine3sf_body<float, OP, NB, false, true>(pk, cf, nx, ny, nz, tiles_x, tiles_y, zlen, omega, c1, c2, cv);
}

template <typename T, int OP, int NB>
__global__ __launch_bounds__(SF_TX * SF_TY) void k_coarse1sf(const Pack<OpA<T>, NB> pk, const SfCoef<T> cf, int nx,
                                                             int ny, int nz, int tiles_x, int tiles_y, int zlen,
                                                             T omega, double c1, double c2) {
    __shared__ T cv[2][4][3][SF_TX * SF_TY];
    fine3sf_body<T, OP, NB, true>(pk, cf, nx, ny, nz, tiles_x, tiles_y, zlen, omega, c1, c2, cv);
}

template <int OP, int NB>
__global__ __launch_bounds__(SF_TX * SF_TY) void k_fine3sf64(const Pack<OpA<double>, NB> pk, const SfCoef<double> cf,
                                                             int nx, int ny, int nz, int tiles_x, int tiles_y,
                                                             int zlen, double omega, double c1, double c2) {
    __shared__ double cv[2][4][3][SF_TX * SF_TY];
    fine3sf_body<double, OP, NB>(pk, cf, nx, ny, nz, tiles_x, tiles_y, zlen, omega, c1, c2, cv);
}

static int sf_tiles(int nn, int per) { return (nn + per - 1) / per; }

// node planes per workgroup.  The grid runs in rounds of `slots` resident
// workgroups (four per compute unit in FP32, two in FP64 for its registers);
// each workgroup also recomputes one element layer below its range.  Take the
// number of plane ranges whose grid fills its last round best, weighed by that
// extra layer (fill x planes / (planes + 1)), the fewest ranges on a tie.
static int sf_zlen(int tiles, int nz_nodes, int slots) {
    tiles = std::max(1, tiles);
    int best_c = 1;
    double best = -1.0;
    const int cmax = std::max(1, std::min(nz_nodes, 8 * slots / tiles));
    for (int c = 1; c <= cmax; ++c) {
        const int zl = (int)ceil_div(nz_nodes, c);
        const int64_t w = (int64_t)tiles * ceil_div(nz_nodes, zl);
        const double fill = (double)w / (double)(ceil_div(w, slots) * slots);
        const double eff = fill * zl / (zl + 1.0);
        if (eff > best + 1e-12) {
            best = eff;
            best_c = c;
        }
    }
    return (int)ceil_div(nz_nodes, best_c);
}

// the tensor form's grid for the fine level of h (false: the level takes
// another form): tiles in x and y, node planes per workgroup, workgroups
static bool sf_grid(const tm_hierarchy* h, bool fp32, int& tx, int& ty, int& zl, int& nb) {
    const Level& F = h->lv[0];
    if (F.dim != 3 || !h->opt.fine_tensor || !h->sf_ok || (fp32 && h->opt.fine_mfma)) return false;
    // the form reaches the block inverse (six arrays of n_nodes) through a
    // buffer descriptor with 32-bit offsets; setup keeps the vectors below
    // 2 GiB, and an FP64 inverse of a grid beyond that takes the node gather
    if ((int64_t)6 * F.n_nodes * (fp32 ? 4 : 8) >= ((int64_t)1 << 31)) return false;
    tx = sf_tiles(F.nn[0], SF_NX);
    ty = sf_tiles(F.nn[1], SF_NY);
    zl = h->opt.fine_tensor >= 2 ? h->opt.fine_tensor : sf_zlen(tx * ty, F.nn[2], fp32 ? 1024 : 512);
    nb = (int)(tx * ty * ceil_div(F.nn[2], zl));
    return true;
}

// 3D FP32 on the matrix cores, two nodes stacked in z per lane as in
// k_fine3z2 (shared neighbour planes).  Each node's 24x24 KE contraction runs
// on v_mfma_f32_4x4x1 (16 blocks of 4 lanes): in each block, lane 4b+j supplies
// B = one neighbour value of its own node and gets back D[i][j] = sum_k
// A[i][k] B[k][j] for rows i = 0..3, i.e. the three KE-row products of its own
// node (row 3 is padding).  A is broadcast from one block to all 16 (CBSZ = 4,
// ABID = k mod 16), so the 192 KE columns (24 per element corner slot) x 4
// rows sit in 12 registers per lane: register q, block m holds column
// k = 16 q + m.  One accumulator per element slot collects its 24 columns; a
// layer's four slots are scaled by their moduli and added as soon as its two
// planes are done (fixed order: layer below, then layer above; FP32
// accumulation).
typedef float v4f __attribute__((ext_vector_type(4)));

template <int K>
__device__ __forceinline__ v4f mfma_col(const float (&ka)[12], float bv, v4f c) {
    static_assert(K >= 0 && K < 192, "KE column");
    return __builtin_amdgcn_mfma_f32_4x4x1f32(ka[K >> 4], bv, c, 4, K & 15, 0);
}

// plane DZ (relative to the node) of the elements of layer EZ: accumulators
// C[EY * 2 + EX] of that layer
template <int DZ, int EZ>
__device__ __forceinline__ void layer_plane3_mfma(const float (&ka)[12], const float (&w)[9][3], v4f (&C)[4]) {
    constexpr int BZ = DZ - EZ;
    static_assert(BZ >= 0 && BZ <= 1, "plane outside the layer");
    // consecutive instructions go to the 4 different accumulators of the layer
#define TM_MF(EY, EX, BX, BY, D)                                                                  \
    C[EY * 2 + EX] = mfma_col<24 * loc3(1 - EX, 1 - EY, 1 - EZ) + 3 * loc3(BX, BY, BZ) + D>(       \
        ka, w[(EY + BY) * 3 + EX + BX][D], C[EY * 2 + EX]);
#define TM_MF4(BX, BY, D) TM_MF(0, 0, BX, BY, D) TM_MF(0, 1, BX, BY, D) TM_MF(1, 0, BX, BY, D) TM_MF(1, 1, BX, BY, D)
#define TM_MF12(BX, BY) TM_MF4(BX, BY, 0) TM_MF4(BX, BY, 1) TM_MF4(BX, BY, 2)
    TM_MF12(0, 0)
    TM_MF12(1, 0)
    TM_MF12(0, 1)
    TM_MF12(1, 1)
#undef TM_MF12
#undef TM_MF4
#undef TM_MF
}

// acc += sum over the layer's slots (EY, EX) of E[EY][EX] * C[EY * 2 + EX]
__device__ __forceinline__ void layer_reduce(const v4f (&C)[4], const float (&E)[2][2], float (&acc)[3]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float e = E[q >> 1][q & 1];
        acc[0] += e * C[q][0];
        acc[1] += e * C[q][1];
        acc[2] += e * C[q][2];
    }
}

template <int OP, int NB>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(4))) void k_fine3z2_mfma(
    const Pack<OpA<float>, NB> pk, int nx, int ny, int nz, int64_t N64, float omega, double c1, double c2) {
    static_assert(OP != OP_QDOT, "no partial sums in the two-node operator");
    using T = float;
    const OpA<T>& A_ = lane_of(pk);
    const T* __restrict__ E = A_.E;
    const uint8_t* __restrict__ nm = A_.nm;
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
    const float* __restrict__ KA = A_.KA;
    if (done && *done) return;
    // every lane of the wave takes part in the matrix instructions: lanes past
    // the last pair work on pair 0 and store nothing
    const uint32_t lane = threadIdx.x & 63u;
    float ka[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) ka[q] = KA[q * 64 + lane];
    const uint32_t N = (uint32_t)N64;
    const uint32_t NX = nx + 1, NY = ny + 1, NZ = nz + 1, PL = NX * NY;
    const uint32_t NT = PL * ((NZ + 1) / 2);           // threads: z pairs
    const uint32_t p = (uint32_t)xcd_block() * WG + threadIdx.x;
    const bool live = p < NT;
    const uint32_t pp = live ? p : 0u;
    const uint32_t i = pp % NX, tq = pp / NX, j = tq % NY, k = 2u * (tq / NY);
    const bool two = k + 1 < NZ;                        // the upper node exists
    const uint32_t nd0 = k * PL + j * NX + i;
    const uint32_t nd1 = two ? nd0 + PL : nd0;
    constexpr uint32_t NBY = 12u;                       // bytes per node
    uint32_t nb0 = nd0 * NBY;
    asm volatile("" : "+v"(nb0));
    const uint32_t bx[3] = {i ? 0u - NBY : 0u, 0u, i + 1 < NX ? NBY : 0u};
    const uint32_t by[3] = {j ? 0u - NX * NBY : 0u, 0u, j + 1 < NY ? NX * NBY : 0u};
    // planes k-1 .. k+2 relative to node k, clamped into the grid (what lies
    // outside only meets elements of modulus zero)
    const uint32_t bz[4] = {k ? 0u - PL * NBY : 0u, 0u, k + 1 < NZ ? PL * NBY : 0u,
                            k + 2 < NZ ? 2u * PL * NBY : (k + 1 < NZ ? PL * NBY : 0u)};
    const auto xr = buf_rsrc(x, (int64_t)N * NBY);
    const auto er = buf_rsrc(E, (int64_t)nx * ny * nz * 4);
    // moduli of element layers k-1, k, k+1 (index clamped, zero outside)
    const uint32_t EX = (uint32_t)nx, EP = EX * (uint32_t)ny;
    const uint32_t jE = j * EX;
    const uint32_t gx[2] = {i ? i - 1 : 0u, i < EX ? i : i - 1};
    const uint32_t gy[2] = {j ? jE - EX : 0u, j < (uint32_t)ny ? jE : jE - EX};
    float El[3][2][2];
#pragma unroll
    for (int lz = 0; lz < 3; ++lz) {
        const int layer = (int)k - 1 + lz;
        const bool zin = layer >= 0 && layer < nz;
        const uint32_t gz = zin ? (uint32_t)layer * EP : 0u;
#pragma unroll
        for (int ey = 0; ey < 2; ++ey)
#pragma unroll
            for (int ex = 0; ex < 2; ++ex) {
                const bool in = zin && (ex || i) && (ex == 0 || i < (uint32_t)nx) && (ey || j) &&
                                (ey == 0 || j < (uint32_t)ny);
                El[lz][ey][ex] = in ? bld<float>(er, (gz + gy[ey] + gx[ex]) * 4u) : 0.f;
            }
    }
    float w[9][3];
    auto load_plane = [&](int P) {
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const uint32_t rowb = nb0 + bz[P] + by[dy];
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) bld3(xr, rowb + bx[dx], w[dy * 3 + dx]);
        }
    };
    // two sets of four accumulators, reused layer after layer: a layer's
    // slots are scaled and added before its registers take the next layer (the
    // scheduling barriers keep the compiler from starting the next layer's
    // chain early, which would keep three sets live and lower the occupancy)
    const v4f z4 = {0.f, 0.f, 0.f, 0.f};
    float acc0[3] = {0.f, 0.f, 0.f}, acc1[3] = {0.f, 0.f, 0.f};
    float xo0[3], xo1[3];
    v4f A[4] = {z4, z4, z4, z4}, B[4] = {z4, z4, z4, z4};
    load_plane(0);
    layer_plane3_mfma<0, 0>(ka, w, A);                 // node k, layer k-1
    load_plane(1);
#pragma unroll
    for (int c = 0; c < 3; ++c) xo0[c] = w[4][c];
    layer_plane3_mfma<1, 0>(ka, w, A);
    layer_plane3_mfma<1, 1>(ka, w, B);                 // node k, layer k
    layer_reduce(A, El[0], acc0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) A[q] = z4;
    layer_plane3_mfma<0, 0>(ka, w, A);                 // node k+1, layer k
    load_plane(2);
#pragma unroll
    for (int c = 0; c < 3; ++c) xo1[c] = w[4][c];
    layer_plane3_mfma<2, 1>(ka, w, B);
    layer_plane3_mfma<1, 0>(ka, w, A);
    layer_reduce(B, El[1], acc0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) B[q] = z4;
    layer_plane3_mfma<1, 1>(ka, w, B);                 // node k+1, layer k+1
    layer_reduce(A, El[1], acc1);
    // the finishing step's operands, requested while the last plane is used
    FinIn<float, 3> fin0, fin1;
    finish_load<float, 3, OP>(nd0, N, b, dinv, ch, fin0);
    finish_load<float, 3, OP>(nd1, N, b, dinv, ch, fin1);
    const uint8_t m0 = nm[nd0], m1 = nm[nd1];
    load_plane(3);
    layer_plane3_mfma<2, 1>(ka, w, B);
    layer_reduce(B, El[2], acc1);
    double dots[2] = {0.0, 0.0};
    if (live) finish_store<float, 3, OP>(nd0, acc0, xo0, m0, fin0, y, omega, dots, ch);
    if (live && two) finish_store<float, 3, OP>(nd1, acc1, xo1, m1, fin1, y, omega, dots, ch);
}

// 2D: 9 neighbour nodes, 4 elements, 8x8 KE.
template <int R, int S, typename T>
__device__ __forceinline__ void ke_fma2(const KeVals<T>& kc, T& t, T v) {
    constexpr int sg = KE_CLS2.sgn[R][S];
    constexpr int cl = KE_CLS2.cls[R][S];
    if constexpr (sg > 0) t += kc.k[cl] * v;
    else if constexpr (sg < 0) t -= kc.k[cl] * v;
}

template <int A, int EY, int EX, typename T>
__device__ __forceinline__ void elem2(const KeVals<T>& kc, const T (&v)[9][2], T (&t)[2]) {
#define TM_CORNER(BX, BY)                                                                         \
    {                                                                                              \
        constexpr int bb = loc2(BX, BY);                                                           \
        const T* vn = v[(EY + BY) * 3 + EX + BX];                                                  \
        ke_fma2<2 * A + 0, 2 * bb + 0>(kc, t[0], vn[0]);                                            \
        ke_fma2<2 * A + 0, 2 * bb + 1>(kc, t[0], vn[1]);                                            \
        ke_fma2<2 * A + 1, 2 * bb + 0>(kc, t[1], vn[0]);                                            \
        ke_fma2<2 * A + 1, 2 * bb + 1>(kc, t[1], vn[1]);                                            \
    }
    TM_CORNER(0, 0)
    TM_CORNER(1, 0)
    TM_CORNER(0, 1)
    TM_CORNER(1, 1)
#undef TM_CORNER
}

template <typename T, int OP, bool MASK_IN, int NB>
__global__ __launch_bounds__(WG) void k_fine2(const Pack<OpA<T>, NB> pk, const KeVals<T> kc, int nx, int ny,
                                              int64_t N64, T omega, double c1, double c2) {
    const OpA<T>& A_ = lane_of(pk);
    const T* __restrict__ E = A_.E;
    const uint8_t* __restrict__ nm = A_.nm;
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
    double* partials = A_.partials;
    if (done && *done) return;
    const uint32_t N = (uint32_t)N64;
    const uint32_t node = (uint32_t)xcd_block() * WG + threadIdx.x;
    const bool live = node < N;
    const uint32_t NX = nx + 1, NY = ny + 1;
    const uint32_t nd = live ? node : 0u;
    const uint32_t i = nd % NX, j = nd / NX;
    // clamped neighbours by additions; values outside the grid are zeroed
    const uint32_t ox[3] = {i ? 0u - 1u : 0u, 0u, i + 1 < NX ? 1u : 0u};
    const uint32_t oy[3] = {j ? 0u - NX : 0u, 0u, j + 1 < NY ? NX : 0u};
    const bool inx[3] = {i > 0, true, i + 1 < NX}, iny[3] = {j > 0, true, j + 1 < NY};
    const auto xr = buf_rsrc(x, (int64_t)N * 2 * sizeof(T));
    const auto er = buf_rsrc(E, (int64_t)nx * ny * sizeof(T));
    // the finishing step's operands first, so that they arrive with the gather
    FinIn<T, 2> fin;
    finish_load<T, 2, OP>(nd, N, b, dinv, ch, fin);
    const uint8_t mo = nm[nd];
    T v[9][2];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const uint32_t id = nd + oy[dy] + ox[dx];
            T a[2];
            bld2(xr, id * (uint32_t)(2 * sizeof(T)), a);
            const bool in = inx[dx] & iny[dy];
            const uint8_t m = MASK_IN ? nm[id] : (uint8_t)0;
            v[dy * 3 + dx][0] = (in & !(m & 1u)) ? a[0] : T(0);
            v[dy * 3 + dx][1] = (in & !(m & 2u)) ? a[1] : T(0);
        }
    // moduli of the 4 elements around the node (lower corner (i-1+ex, j-1+ey))
    const uint32_t EX = (uint32_t)nx;
    const uint32_t gx[2] = {i ? i - 1 : 0u, i < EX ? i : i - 1};
    const uint32_t gy[2] = {(j ? j - 1 : 0u) * EX, (j < (uint32_t)ny ? j : j - 1) * EX};
    T Ee[2][2];
#pragma unroll
    for (int ey = 0; ey < 2; ++ey)
#pragma unroll
        for (int ex = 0; ex < 2; ++ex) {
            const bool in = (ex || i) && (ex == 0 || i < EX) && (ey || j) && (ey == 0 || j < (uint32_t)ny);
            const T ev = bld<T>(er, (gy[ey] + gx[ex]) * (uint32_t)sizeof(T));
            Ee[ey][ex] = in ? ev : T(0);
        }
    T acc[2] = {0, 0};
#define TM_ELEM(EY, EX)                                                                           \
    {                                                                                              \
        T t[2] = {0, 0};                                                                           \
        elem2<loc2(1 - EX, 1 - EY), EY, EX>(kc, v, t);                                             \
        acc[0] += Ee[EY][EX] * t[0];                                                               \
        acc[1] += Ee[EY][EX] * t[1];                                                               \
    }
    TM_ELEM(0, 0)
    TM_ELEM(0, 1)
    TM_ELEM(1, 0)
    TM_ELEM(1, 1)
#undef TM_ELEM
    T xo[2] = {v[4][0], v[4][1]};                   // this node's own value
    if (MASK_IN) {
        xo[0] = x[2 * nd];
        xo[1] = x[2 * nd + 1];
    }
    double dots[2] = {0.0, 0.0};
    if (live) finish_store<T, 2, OP>(node, acc, xo, mo, fin, y, omega, dots, ch);
    if (OP == OP_QDOT) block_reduce_store<2>(dots, partials);
}

// the first post-smoothing step of the fine level with the prolongation from
// level 1 in it: 3D, the FP32 tensor form, level 1 geometric and every fine
// element count even (level-1 node I sits on fine node 2I)
bool fine_pro_ok(const tm_hierarchy* h) {
    int tx, ty, zl, nb;
    if (h->lv.size() < 2 || h->lv[1].kind != TM_LEVEL_GEOMETRIC) return false;
    if (!sf_grid(h, true, tx, ty, zl, nb)) return false;
    const Level& F = h->lv[0];
    return F.nel[0] % 2 == 0 && F.nel[1] % 2 == 0 && F.nel[2] % 2 == 0;
}

template <int OP, int NB>
static void fine_pro_launch(const LaneIO* L, int n, float omega, double c1, double c2, hipStream_t s) {
    const tm_hierarchy* h = L[0].h;
    const Level& F = h->lv[0];
    Pack<OpA<float>, NB> pk{};
    for (int q = 0; q < n; ++q) {
        const Level& Lq = L[q].h->lv[0];
        OpA<float>& a = pk.a[q];
        a.E = Lq.E32;
        a.nm = Lq.nmask;
        a.x = (const float*)L[q].x;
        a.xc = (const float*)L[q].xc;
        a.b = (const float*)L[q].b;
        a.y = (float*)L[q].y;
        a.dinv = Lq.dinv32;
        a.done = L[q].done;
        a.din = (const float*)L[q].din;
        a.dout = (float*)L[q].dout;
    }
    int tx, ty, zl, nb;
    sf_grid(h, true, tx, ty, zl, nb);
    hipLaunchKernelGGL((k_fine3sf_pro<OP, NB>), dim3((unsigned)nb, n), dim3(SF_TX * SF_TY), 0, s, pk, h->sf32,
                       F.nel[0], F.nel[1], F.nel[2], tx, ty, zl, omega, c1, c2);
}

void launch_fine_pro_b(int op, const LaneIO* L, int n, float omega, double c1, double c2, hipStream_t s) {
    if (op != OP_SMOOTH && op != OP_CHEB) fail(TM_ERR_ARG, "fused prolongation: smoothing steps only");
    for (int q0 = 0; q0 < n; q0 += MAXB) {
        const int m = std::min(MAXB, n - q0);
        if (op == OP_CHEB) {
            if (m == 1) fine_pro_launch<OP_CHEB, 1>(L + q0, 1, omega, c1, c2, s);
            else fine_pro_launch<OP_CHEB, MAXB>(L + q0, m, omega, c1, c2, s);
        } else {
            if (m == 1) fine_pro_launch<OP_SMOOTH, 1>(L + q0, 1, omega, c1, c2, s);
            else fine_pro_launch<OP_SMOOTH, MAXB>(L + q0, m, omega, c1, c2, s);
        }
    }
}

// level 1 in the tensor form for lanes L[0..n) (n <= NB): the lanes' own
// level-1 vectors and block inverses, their fine moduli and supports
template <typename T>
static const SfCoef<T>& pick_sf(const tm_hierarchy* h);
template <>
const SfCoef<float>& pick_sf<float>(const tm_hierarchy* h) { return h->sf32; }
template <>
const SfCoef<double>& pick_sf<double>(const tm_hierarchy* h) { return h->sf64; }

template <typename T, int OP, int NB>
static void coarse1_launch(const LaneIO* L, int n, T omega, double c1, double c2, hipStream_t s) {
    const tm_hierarchy* h = L[0].h;
    const Level& C1 = h->lv[1];
    Pack<OpA<T>, NB> pk{};
    for (int q = 0; q < n; ++q) {
        const Level& F = L[q].h->lv[0];
        const Level& V = L[q].h->lv[1];
        OpA<T>& a = pk.a[q];
        a.E = pick_E<T>(F);
        a.nm = F.nmask;
        a.sub = V.subf;
        a.x = (const T*)L[q].x;
        a.b = (const T*)L[q].b;
        a.y = (T*)L[q].y;
        a.dinv = pick_dinv<T>(V);
        a.done = L[q].done;
        a.din = (const T*)L[q].din;
        a.dout = (T*)L[q].dout;
    }
    const int tx = sf_tiles(C1.nn[0], SF_NX), ty = sf_tiles(C1.nn[1], SF_NY);
    const int zl = sf_zlen(tx * ty, C1.nn[2], 512);
    const dim3 g((unsigned)(tx * ty * ceil_div(C1.nn[2], zl)), n), bk(SF_TX * SF_TY);
    hipLaunchKernelGGL((k_coarse1sf<T, OP, NB>), g, bk, 0, s, pk, pick_sf<T>(h), C1.nel[0], C1.nel[1], C1.nel[2], tx,
                       ty, zl, omega, c1, c2);
}

template <typename T, int OP>
static void coarse1_dispatch(const LaneIO* L, int n, T omega, double c1, double c2, hipStream_t s) {
    for (int q0 = 0; q0 < n; q0 += MAXB) {
        const int m = std::min(MAXB, n - q0);
        if (m == 1) coarse1_launch<T, OP, 1>(L + q0, 1, omega, c1, c2, s);
        else coarse1_launch<T, OP, MAXB>(L + q0, m, omega, c1, c2, s);
    }
}

template <typename T>
void launch_coarse1_tensor_b(int op, const LaneIO* L, int n, T omega, double c1, double c2, hipStream_t s) {
    if (n < 1) return;
    switch (op) {
        case OP_APPLY: coarse1_dispatch<T, OP_APPLY>(L, n, omega, c1, c2, s); break;
        case OP_RESID: coarse1_dispatch<T, OP_RESID>(L, n, omega, c1, c2, s); break;
        case OP_SMOOTH: coarse1_dispatch<T, OP_SMOOTH>(L, n, omega, c1, c2, s); break;
        case OP_CHEB: coarse1_dispatch<T, OP_CHEB>(L, n, omega, c1, c2, s); break;
        default: fail(TM_ERR_ARG, "level-1 tensor form: no partial sums");
    }
}
template void launch_coarse1_tensor_b<float>(int, const LaneIO*, int, float, double, double, hipStream_t);

// workgroups of the FP64 operator with partial sums (q = K~p), i.e. the
// partial sums it leaves per lane
int fine_op_blocks(const tm_hierarchy* h) {
    int tx, ty, zl, nb;
    if (sf_grid(h, false, tx, ty, zl, nb)) return nb;
    return (int)grid_for(h->lv[0].n_nodes);
}

template <typename T>
static const T* pick_E(const Level& L);
template <>
const double* pick_E<double>(const Level& L) { return L.E64; }
template <>
const float* pick_E<float>(const Level& L) { return L.E32; }
template <typename T>
static const KeVals<T>& pick_kc(const tm_hierarchy* h);
template <>
const KeVals<double>& pick_kc<double>(const tm_hierarchy* h) { return h->kc64; }
template <>
const KeVals<float>& pick_kc<float>(const tm_hierarchy* h) { return h->kc32; }
template <typename T>
static const T* pick_dinv(const Level& L);
template <>
const double* pick_dinv<double>(const Level& L) { return L.dinv64; }
template <>
const float* pick_dinv<float>(const Level& L) { return L.dinv32; }

// one launch of the fine operator for lanes L[0..n) (n <= MAXB), all of
// hierarchies with the same fine grid and options
template <typename T, int OP, bool MI, int NB>
static void fine_launch(const LaneIO* L, int n, T omega, double c1, double c2, hipStream_t s) {
    const tm_hierarchy* h = L[0].h;
    const Level& F = h->lv[0];
    Pack<OpA<T>, NB> pk{};
    for (int q = 0; q < n; ++q) {
        const Level& Lq = L[q].h->lv[0];
        OpA<T>& a = pk.a[q];
        a.E = pick_E<T>(Lq);
        a.KA = L[q].h->KA32;
        a.nm = Lq.nmask;
        a.x = (const T*)L[q].x;
        a.b = (const T*)L[q].b;
        a.y = (T*)L[q].y;
        a.dinv = pick_dinv<T>(Lq);
        a.done = L[q].done;
        a.partials = L[q].part;
        a.din = (const T*)L[q].din;
        a.dout = (T*)L[q].dout;
    }
    const dim3 blk(WG);
    if constexpr (!MI && (std::is_same<T, double>::value || OP != OP_QDOT)) {
        int tx, ty, zl, nb;
        if (sf_grid(h, std::is_same<T, float>::value, tx, ty, zl, nb)) {
            const dim3 g((unsigned)nb, n), bk(SF_TX * SF_TY);
            if constexpr (std::is_same<T, float>::value)
                hipLaunchKernelGGL((k_fine3sf<OP, NB>), g, bk, 0, s, pk, h->sf32, F.nel[0], F.nel[1], F.nel[2], tx,
                                   ty, zl, omega, c1, c2);
            else
                hipLaunchKernelGGL((k_fine3sf64<OP, NB>), g, bk, 0, s, pk, h->sf64, F.nel[0], F.nel[1], F.nel[2],
                                   tx, ty, zl, omega, c1, c2);
            return;
        }
    }
    if constexpr (std::is_same<T, float>::value && !MI && OP != OP_QDOT) {
        if (F.dim == 3) {
            const int64_t nt = (int64_t)F.nn[0] * F.nn[1] * ((F.nn[2] + 1) / 2);
            const dim3 g(grid_for(nt), n);
            if (h->opt.fine_mfma)
                hipLaunchKernelGGL((k_fine3z2_mfma<OP, NB>), g, blk, 0, s, pk, F.nel[0], F.nel[1], F.nel[2], F.n_nodes,
                                   omega, c1, c2);
            else
                hipLaunchKernelGGL((k_fine3z2<T, OP, NB>), g, blk, 0, s, pk, pick_kc<T>(h), F.nel[0], F.nel[1],
                                   F.nel[2], F.n_nodes, omega, c1, c2);
            return;
        }
    }
    const dim3 g(grid_for(F.n_nodes), n);
    if (F.dim == 3)
        hipLaunchKernelGGL((k_fine3<T, OP, MI, NB>), g, blk, 0, s, pk, pick_kc<T>(h), F.nel[0], F.nel[1], F.nel[2],
                           F.n_nodes, omega, c1, c2);
    else
        hipLaunchKernelGGL((k_fine2<T, OP, MI, NB>), g, blk, 0, s, pk, pick_kc<T>(h), F.nel[0], F.nel[1], F.n_nodes,
                           omega, c1, c2);
}

template <typename T, int OP, bool MI>
static void fine_dispatch(const LaneIO* L, int n, T omega, double c1, double c2, hipStream_t s) {
    for (int q0 = 0; q0 < n; q0 += MAXB) {
        const int m = std::min(MAXB, n - q0);
        if (m == 1) fine_launch<T, OP, MI, 1>(L + q0, 1, omega, c1, c2, s);
        else fine_launch<T, OP, MI, MAXB>(L + q0, m, omega, c1, c2, s);
    }
}

template <typename T>
void launch_fine_op_b(int op, bool mask_in, const LaneIO* L, int n, T omega, double c1, double c2,
                      hipStream_t s) {
    if (n < 1) return;
    if (mask_in) {
        if (op != OP_APPLY) fail(TM_ERR_ARG, "masked-input fine operator supports apply only");
        fine_dispatch<T, OP_APPLY, true>(L, n, omega, c1, c2, s);
        return;
    }
    switch (op) {
        case OP_APPLY: fine_dispatch<T, OP_APPLY, false>(L, n, omega, c1, c2, s); break;
        case OP_RESID: fine_dispatch<T, OP_RESID, false>(L, n, omega, c1, c2, s); break;
        case OP_SMOOTH: fine_dispatch<T, OP_SMOOTH, false>(L, n, omega, c1, c2, s); break;
        case OP_CHEB: fine_dispatch<T, OP_CHEB, false>(L, n, omega, c1, c2, s); break;
        default:
            for (int q = 0; q < n; ++q)
                if (!L[q].part) fail(TM_ERR_ARG, "q = K~p needs a partial-sum buffer");
            fine_dispatch<T, OP_QDOT, false>(L, n, omega, c1, c2, s);
            break;
    }
}
template void launch_fine_op_b<double>(int, bool, const LaneIO*, int, double, double, double, hipStream_t);
template void launch_fine_op_b<float>(int, bool, const LaneIO*, int, float, double, double, hipStream_t);

template <typename T>
void launch_fine_op(const tm_hierarchy* h, int op, bool mask_in, const T* x, const T* b, T* y,
                    T omega, const int* done, double* partials, hipStream_t s, const ChebArgs& ch) {
    LaneIO l{};
    l.h = h;
    l.x = x;
    l.b = b;
    l.y = y;
    l.done = done;
    l.part = partials;
    l.din = ch.din;
    l.dout = ch.dout;
    launch_fine_op_b<T>(op, mask_in, &l, 1, omega, ch.c1, ch.c2, s);
}
template void launch_fine_op<double>(const tm_hierarchy*, int, bool, const double*, const double*,
                                     double*, double, const int*, double*, hipStream_t, const ChebArgs&);
template void launch_fine_op<float>(const tm_hierarchy*, int, bool, const float*, const float*,
                                    float*, float, const int*, double*, hipStream_t, const ChebArgs&);

}  // namespace tmi
