// Fine-level kernels: SIMP moduli, point-block diagonal and the matrix-free
// operator K~ = M K M + (I - M), K = sum_e E_e L_e^T KE L_e (Sec. 2), applied
// node by node so that every output is summed in a fixed order (deterministic,
// no atomics): node i gathers its 3^dim neighbours once and accumulates
// E_e * KE[rows of i's local corner] * U_e over the 2^dim elements around it.
// KE is read through uniform (scalar) loads; the work is one 2^dim*dim-row
// slice of an element product per element per node, i.e. exactly the flops
// of the element-by-element product, without redundancy.
#include "tm_device.h"

namespace tmi {

// ------------------------------------------------------------ SIMP
__global__ void k_simp(const double* __restrict__ rho, int64_t n, double p, double E0, double Emin,
                       double* __restrict__ E64, float* __restrict__ E32, int* flags) {
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
}

void launch_simp(const double* rho, int64_t n_el, double p, double E0, double Emin, double* E64,
                 float* E32, int* flags, hipStream_t s) {
    hipLaunchKernelGGL(k_simp, dim3(grid_for(n_el)), dim3(WG), 0, s, rho, n_el, p, E0, Emin, E64,
                       E32, flags);
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
template <typename T, int OP, bool MASK_IN>
__global__ __launch_bounds__(WG) void k_fine3(const T* __restrict__ E, const T* __restrict__ KE,
                                              const uint8_t* __restrict__ nm, int nx, int ny, int nz,
                                              int64_t N64, const T* __restrict__ x,
                                              const T* __restrict__ b, T* __restrict__ y,
                                              const T* __restrict__ dinv, T omega,
                                              const int* __restrict__ done, double* partials) {
    if (done && *done) return;
    const uint32_t N = (uint32_t)N64;
    const uint32_t node = (uint32_t)xcd_block() * WG + threadIdx.x;
    const bool live = node < N;
    const uint32_t NX = nx + 1, NY = ny + 1, NZ = nz + 1;
    const uint32_t nd = live ? node : 0u;
    const uint32_t i = nd % NX, tq = nd / NX, j = tq % NY, k = tq / NY;
    const uint32_t cx[3] = {i ? i - 1 : 0u, i, min(i + 1, NX - 1)};
    const uint32_t cy[3] = {j ? j - 1 : 0u, j, min(j + 1, NY - 1)};
    const uint32_t cz[3] = {k ? k - 1 : 0u, k, min(k + 1, NZ - 1)};
    const auto xr = buf_rsrc(x, (int64_t)N * 3 * sizeof(T));
    T v[3][9][3];  // [plane dz+1][(dy+1)*3 + dx+1][component]
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const uint32_t row = (cz[dz] * NY + cy[dy]) * NX;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const uint32_t id = row + cx[dx];
                T a[3];
                bld3(xr, id * (3u * sizeof(T)), a);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (MASK_IN) a[c] = ((nm[id] >> c) & 1u) ? T(0) : a[c];
                    v[dz][dy * 3 + dx][c] = a[c];
                }
            }
        }
    const auto er = buf_rsrc(E, (int64_t)nx * ny * nz * sizeof(T));
    T acc[3] = {0, 0, 0};
#pragma unroll
    for (int ez = 0; ez < 2; ++ez)
#pragma unroll
        for (int ey = 0; ey < 2; ++ey)
#pragma unroll
            for (int ex = 0; ex < 2; ++ex) {
                // element with lower corner (i-1+ex, j-1+ey, k-1+ez)
                const bool in = (ex || i) && (ex == 0 || i < (uint32_t)nx) && (ey || j) &&
                                (ey == 0 || j < (uint32_t)ny) && (ez || k) && (ez == 0 || k < (uint32_t)nz);
                const uint32_t gx = min(i + ex, (uint32_t)nx) - (i + ex > 0 ? 1u : 0u);
                const uint32_t gy = min(j + ey, (uint32_t)ny) - (j + ey > 0 ? 1u : 0u);
                const uint32_t gz = min(k + ez, (uint32_t)nz) - (k + ez > 0 ? 1u : 0u);
                const T Ee = in ? bld<T>(er, ((gz * (uint32_t)ny + gy) * (uint32_t)nx + gx) * (uint32_t)sizeof(T))
                                : T(0);
                const int a = loc3(1 - ex, 1 - ey, 1 - ez);
                T t[3] = {0, 0, 0};
#pragma unroll
                for (int bz = 0; bz < 2; ++bz)
#pragma unroll
                    for (int by = 0; by < 2; ++by)
#pragma unroll
                        for (int bx = 0; bx < 2; ++bx) {
                            const int bb = loc3(bx, by, bz);
                            const T* vn = v[ez + bz][(ey + by) * 3 + ex + bx];
#pragma unroll
                            for (int c = 0; c < 3; ++c)
#pragma unroll
                                for (int d = 0; d < 3; ++d)
                                    t[c] += KE[(3 * a + c) * 24 + 3 * bb + d] * vn[d];
                        }
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[c] += Ee * t[c];
            }
    double dots[2] = {0.0, 0.0};
    if (live) {
        const T xo[3] = {x[3u * node], x[3u * node + 1], x[3u * node + 2]};
        finish_node<T, 3, OP>(node, N, acc, xo, nm[node], b, y, dinv, omega, dots);
    }
    if (OP == OP_QDOT) block_reduce_store<2>(dots, partials);
}

// 2D: 9 neighbour nodes, 4 elements, 8x8 KE.
template <typename T, int OP, bool MASK_IN>
__global__ __launch_bounds__(WG) void k_fine2(const T* __restrict__ E, const T* __restrict__ KE,
                                              const uint8_t* __restrict__ nm, int nx, int ny,
                                              int64_t N, const T* __restrict__ x,
                                              const T* __restrict__ b, T* __restrict__ y,
                                              const T* __restrict__ dinv, T omega,
                                              const int* __restrict__ done, double* partials) {
    if (done && *done) return;
    const int64_t node = xcd_block() * WG + threadIdx.x;
    const bool live = node < N;
    const int NX = nx + 1, NY = ny + 1;
    const int64_t nd = live ? node : 0;
    const int i = (int)(nd % NX);
    const int j = (int)(nd / NX);
    T v[9][2];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const int ii = i + dx - 1, jj = j + dy - 1;
            const bool ok = live && ii >= 0 && ii < NX && jj >= 0 && jj < NY;
            const int64_t id = (int64_t)jj * NX + ii;
            T a0 = 0, a1 = 0;
            if (ok) {
                a0 = x[2 * id];
                a1 = x[2 * id + 1];
                if (MASK_IN) {
                    const uint8_t m = nm[id];
                    if (m & 1) a0 = 0;
                    if (m & 2) a1 = 0;
                }
            }
            v[dy * 3 + dx][0] = a0;
            v[dy * 3 + dx][1] = a1;
        }
    T acc[2] = {0, 0};
#pragma unroll
    for (int ey = 0; ey < 2; ++ey)
#pragma unroll
        for (int ex = 0; ex < 2; ++ex) {
            const int gx = i - 1 + ex, gy = j - 1 + ey;
            const bool ok = live && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
            const T Ee = ok ? E[(int64_t)gy * nx + gx] : T(0);
            const int a = loc2(1 - ex, 1 - ey);
            T t[2] = {0, 0};
#pragma unroll
            for (int by = 0; by < 2; ++by)
#pragma unroll
                for (int bx = 0; bx < 2; ++bx) {
                    const int bb = loc2(bx, by);
                    const T* vn = v[(ey + by) * 3 + ex + bx];
#pragma unroll
                    for (int c = 0; c < 2; ++c)
#pragma unroll
                        for (int d = 0; d < 2; ++d) t[c] += KE[(2 * a + c) * 8 + 2 * bb + d] * vn[d];
                }
#pragma unroll
            for (int c = 0; c < 2; ++c) acc[c] += Ee * t[c];
        }
    double dots[2] = {0.0, 0.0};
    if (live) {
        const T xo[2] = {x[2 * node], x[2 * node + 1]};
        finish_node<T, 2, OP>(node, N, acc, xo, nm[node], b, y, dinv, omega, dots);
    }
    if (OP == OP_QDOT) block_reduce_store<2>(dots, partials);
}

int fine_op_blocks(const tm_hierarchy* h) { return (int)grid_for(h->lv[0].n_nodes); }

template <typename T>
static const T* pick_E(const Level& L);
template <>
const double* pick_E<double>(const Level& L) { return L.E64; }
template <>
const float* pick_E<float>(const Level& L) { return L.E32; }
template <typename T>
static const T* pick_KE(const tm_hierarchy* h);
template <>
const double* pick_KE<double>(const tm_hierarchy* h) { return h->KE64; }
template <>
const float* pick_KE<float>(const tm_hierarchy* h) { return h->KE32; }
template <typename T>
static const T* pick_dinv(const Level& L);
template <>
const double* pick_dinv<double>(const Level& L) { return L.dinv64; }
template <>
const float* pick_dinv<float>(const Level& L) { return L.dinv32; }

template <typename T, int OP, bool MI>
static void fine_dispatch(const tm_hierarchy* h, const T* x, const T* b, T* y, T omega,
                          const int* done, double* partials, hipStream_t s) {
    const Level& L = h->lv[0];
    const dim3 g(grid_for(L.n_nodes)), blk(WG);
    if (L.dim == 3)
        hipLaunchKernelGGL((k_fine3<T, OP, MI>), g, blk, 0, s, pick_E<T>(L), pick_KE<T>(h), L.nmask,
                           L.nel[0], L.nel[1], L.nel[2], L.n_nodes, x, b, y, pick_dinv<T>(L), omega,
                           done, partials);
    else
        hipLaunchKernelGGL((k_fine2<T, OP, MI>), g, blk, 0, s, pick_E<T>(L), pick_KE<T>(h), L.nmask,
                           L.nel[0], L.nel[1], L.n_nodes, x, b, y, pick_dinv<T>(L), omega, done,
                           partials);
}

template <typename T>
void launch_fine_op(const tm_hierarchy* h, int op, bool mask_in, const T* x, const T* b, T* y,
                    T omega, const int* done, double* partials, hipStream_t s) {
    if (mask_in) {
        if (op != OP_APPLY) fail(TM_ERR_ARG, "masked-input fine operator supports apply only");
        fine_dispatch<T, OP_APPLY, true>(h, x, b, y, omega, done, partials, s);
        return;
    }
    switch (op) {
        case OP_APPLY: fine_dispatch<T, OP_APPLY, false>(h, x, b, y, omega, done, partials, s); break;
        case OP_RESID: fine_dispatch<T, OP_RESID, false>(h, x, b, y, omega, done, partials, s); break;
        case OP_SMOOTH: fine_dispatch<T, OP_SMOOTH, false>(h, x, b, y, omega, done, partials, s); break;
        default:
            if (!partials) fail(TM_ERR_ARG, "q = K~p needs a partial-sum buffer");
            fine_dispatch<T, OP_QDOT, false>(h, x, b, y, omega, done, partials, s);
            break;
    }
}
template void launch_fine_op<double>(const tm_hierarchy*, int, bool, const double*, const double*,
                                     double*, double, const int*, double*, hipStream_t);
template void launch_fine_op<float>(const tm_hierarchy*, int, bool, const float*, const float*,
                                    float*, float, const int*, double*, hipStream_t);

}  // namespace tmi
