// Stability eigenproblem (Sec. 2, stability maximisation; Sec. 3, generalized
// Davidson, Algorithm 2): the stress-stiffness matrix and the skinny
// search-space products of the eigensolver, all in FP64.
//
// K_sigma couples every displacement component with itself only, with the
// same scalar weights: K_sigma = G (x) I_dim, where G is a scalar operator on
// the nodes with the 3^dim-point pattern of the grid.  G is stored as a nodal
// stencil [3^dim][n_nodes] (neighbour offset o = (dx+1) + 3 (dy+1) + 9 (dz+1)),
// so the operator reads 27 (9) numbers per node instead of the 81 (18) of a
// block stencil, and is applied to the dim components of a node at once.
//
// G = -sum_e E_sigma(rho_e) g_e(u_e), g_e[a][b] = sum over the Gauss points of
// w |J| grad N_a^T sigma grad N_b with sigma the unit-modulus stress of u_e (the
// textbook geometric stiffness; the minus sign gives compressive states
// positive eigenvalues).  Assembly runs in 2^dim colour passes over the
// elements (elements of one colour share no node), so every stencil entry is
// a plain read-add-write with a fixed summation order: the result is
// deterministic and G[o][I] and G[26-o][J] get bit-identical values.
#include "tm_device.h"

namespace tmi {

// ------------------------------------------------------------ assembly
template <int DIM>
__device__ __forceinline__ double shape_grad(int a, int d, int g, double inv_h) {
    // d N_a / d x_d at Gauss point g (coordinates +-1/sqrt(3) per axis, bit ax
    // of g set = positive side); N_a = prod_e (1 + s_ae xi_e) / 2 on [-1, 1]^dim
    constexpr double GP = 0.57735026918962576451;      // 1 / sqrt(3)
    double v = inv_h;
#pragma unroll
    for (int e = 0; e < DIM; ++e) {
        const double s = corner_coord(a, e) ? 1.0 : -1.0;
        const double xi = ((g >> e) & 1) ? GP : -GP;
        v *= e == d ? s : 0.5 * (1.0 + s * xi);
    }
    return v;
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_gsig_assemble(const double* __restrict__ u, const double* __restrict__ rho,
                                                      double p, double E0, double rho_min, double lam, double mu,
                                                      double h, int nx, int ny, int nz, int cx, int cy, int cz,
                                                      double* __restrict__ G, int64_t n_nodes) {
    constexpr int NPE = 1 << DIM;
    // elements of colour (cx, cy, cz): ex = 2 i + cx, ...
    const int hx = (nx - cx + 1) / 2, hy = (ny - cy + 1) / 2, hz = DIM == 3 ? (nz - cz + 1) / 2 : 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)hx * hy * hz) return;
    const int ex = 2 * (int)(t % hx) + cx;
    const int ey = 2 * (int)((t / hx) % hy) + cy;
    const int ez = DIM == 3 ? 2 * (int)(t / ((int64_t)hx * hy)) + cz : 0;
    const int64_t e = ex + (int64_t)nx * (ey + (int64_t)ny * ez);
    const double r = rho[e];
    if (!(r >= rho_min)) return;                       // E_sigma = 0: no contribution
    const double Es = E0 * pow(r, p);
    const int64_t NX = nx + 1, NY = ny + 1;
    int64_t nd[NPE];
    double ue[NPE][DIM];
#pragma unroll
    for (int a = 0; a < NPE; ++a) {
        nd[a] = (ex + corner_coord(a, 0)) + NX * ((ey + corner_coord(a, 1)) + (DIM == 3 ? NY * (ez + corner_coord(a, 2)) : 0));
#pragma unroll
        for (int c = 0; c < DIM; ++c) ue[a][c] = u[DIM * nd[a] + c];
    }
    const double inv_h = 1.0 / h;
    double wj = 1.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) wj *= 0.5 * h;        // |J| (unit Gauss weights)
    double g[NPE][NPE];
#pragma unroll
    for (int a = 0; a < NPE; ++a)
#pragma unroll
        for (int b = 0; b < NPE; ++b) g[a][b] = 0.0;
#pragma unroll
    for (int gp = 0; gp < NPE; ++gp) {
        double dN[NPE][DIM];
#pragma unroll
        for (int a = 0; a < NPE; ++a)
#pragma unroll
            for (int d = 0; d < DIM; ++d) dN[a][d] = shape_grad<DIM>(a, d, gp, inv_h);
        double F[DIM][DIM];                            // F[c][d] = d u_c / d x_d
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                double s = 0.0;
#pragma unroll
                for (int a = 0; a < NPE; ++a) s += ue[a][c] * dN[a][d];
                F[c][d] = s;
            }
        double tr = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) tr += F[c][c];
        double sg[DIM][DIM];                           // sigma = Es (lam tr(eps) I + 2 mu eps), times w |J|
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int d = 0; d < DIM; ++d)
                sg[c][d] = wj * Es * ((c == d ? lam * tr : 0.0) + mu * (F[c][d] + F[d][c]));
#pragma unroll
        for (int a = 0; a < NPE; ++a) {
            double ta[DIM];
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < DIM; ++c) s += dN[a][c] * sg[c][d];
                ta[d] = s;
            }
#pragma unroll
            for (int b = a; b < NPE; ++b) {
                double s = 0.0;
#pragma unroll
                for (int d = 0; d < DIM; ++d) s += ta[d] * dN[b][d];
                g[a][b] += s;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < NPE; ++a)
#pragma unroll
        for (int b = 0; b < NPE; ++b) {
            const double v = a <= b ? g[a][b] : g[b][a];
            const int o = (corner_coord(b, 0) - corner_coord(a, 0) + 1) + 3 * (corner_coord(b, 1) - corner_coord(a, 1) + 1) +
                          (DIM == 3 ? 9 * (corner_coord(b, 2) - corner_coord(a, 2) + 1) : 0);
            double* dst = G + (int64_t)o * n_nodes + nd[a];
            *dst = *dst - v;
        }
}

void launch_gsig_assemble(const tm_hierarchy* h, const double* u, double rho_min, double* G, hipStream_t s) {
    const Level& L = h->lv[0];
    const double nu = h->mat.nu;
    // unit-modulus Lame constants; plane stress in 2D: sigma = (nu/(1-nu^2)) tr I + (1/(1+nu)) eps
    const double mu = 0.5 / (1.0 + nu);
    const double lam = L.dim == 3 ? nu / ((1.0 + nu) * (1.0 - 2.0 * nu)) : nu / (1.0 - nu * nu);
    const int nst = L.dim == 3 ? 27 : 9;
    launch_fill(G, (int64_t)nst * L.n_nodes * (int64_t)sizeof(double), s);
    const int ncol = L.dim == 3 ? 8 : 4;
    for (int col = 0; col < ncol; ++col) {
        const int cx = col & 1, cy = (col >> 1) & 1, cz = (col >> 2) & 1;
        const int64_t hx = (L.nel[0] - cx + 1) / 2, hy = (L.nel[1] - cy + 1) / 2;
        const int64_t hz = L.dim == 3 ? (L.nel[2] - cz + 1) / 2 : 1;
        const int64_t n = hx * hy * hz;
        if (n == 0) continue;
        if (L.dim == 3)
            hipLaunchKernelGGL(k_gsig_assemble<3>, dim3(grid_for(n)), dim3(WG), 0, s, u, h->rho64, h->mat.p, h->mat.E0,
                               rho_min, lam, mu, h->mesh.h, L.nel[0], L.nel[1], L.nel[2], cx, cy, cz, G, L.n_nodes);
        else
            hipLaunchKernelGGL(k_gsig_assemble<2>, dim3(grid_for(n)), dim3(WG), 0, s, u, h->rho64, h->mat.p, h->mat.E0,
                               rho_min, lam, mu, h->mesh.h, L.nel[0], L.nel[1], 1, cx, cy, 0, G, L.n_nodes);
    }
}

// ------------------------------------------------------------ operator
// y = K_sigma~ x = M (G (x) I) M x: supported dofs (nmask bit c of a node) are
// zero in the output and ignored in the input.
template <int DIM>
__global__ __launch_bounds__(WG) void k_gsig_apply(const double* __restrict__ G, const uint8_t* __restrict__ nm,
                                                   const double* __restrict__ x, double* __restrict__ y, int NX,
                                                   int NY, int NZ, int64_t N) {
    const int64_t node = xcd_block() * WG + threadIdx.x;
    if (node >= N) return;
    const int i = (int)(node % NX), j = (int)((node / NX) % NY), k = DIM == 3 ? (int)(node / ((int64_t)NX * NY)) : 0;
    double acc[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) acc[c] = 0.0;
#pragma unroll
    for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int ii = i + dx, jj = j + dy, kk = k + dz;
                if (ii < 0 || ii >= NX || jj < 0 || jj >= NY || (DIM == 3 && (kk < 0 || kk >= NZ))) continue;
                const int o = (dx + 1) + 3 * (dy + 1) + (DIM == 3 ? 9 * (dz + 1) : 0);
                const double gv = G[(int64_t)o * N + node];
                const int64_t J = ii + (int64_t)NX * (jj + (int64_t)NY * kk);
                const uint8_t mj = nm[J];
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    const double xv = x[DIM * J + c];
                    acc[c] += ((mj >> c) & 1) ? 0.0 : gv * xv;
                }
            }
    const uint8_t mi = nm[node];
#pragma unroll
    for (int c = 0; c < DIM; ++c) y[DIM * node + c] = ((mi >> c) & 1) ? 0.0 : acc[c];
}

void launch_gsig_apply(const tm_hierarchy* h, const double* G, const double* x, double* y, hipStream_t s) {
    const Level& L = h->lv[0];
    if (L.dim == 3)
        hipLaunchKernelGGL(k_gsig_apply<3>, dim3(grid_for(L.n_nodes)), dim3(WG), 0, s, G, L.nmask, x, y, L.nn[0],
                           L.nn[1], L.nn[2], L.n_nodes);
    else
        hipLaunchKernelGGL(k_gsig_apply<2>, dim3(grid_for(L.n_nodes)), dim3(WG), 0, s, G, L.nmask, x, y, L.nn[0],
                           L.nn[1], 1, L.n_nodes);
}

// ------------------------------------------------------------ search-space products
// V is column-major, n rows, leading dimension ld, at most EIG_MAX_COLS columns.
// Rows are split over a grid of eig_blocks(n) workgroups; each workgroup
// writes one partial per column (column-major: part[c * EIG_BLOCKS + block])
// and one workgroup per column adds that column's partials in block order, so
// every sum has a fixed order (deterministic).  Every row's loads of V are
// issued before any of them is used (the column count is a uniform runtime
// value: a load and its use in one guarded block would wait load by load).

// part[c][b] = sum over the rows of block b of V[c][row] w[row] (c < nc), and
// slot EIG_MAX_COLS: z[row] w[row] when z is given.  The columns (z counted as
// column nc) are split into chunks of VTW_CHUNK over blockIdx.y, so a thread
// holds few accumulators and the grid many waves; w is re-read per chunk
// (from cache).
constexpr int VTW_CHUNK = 8;
__global__ __launch_bounds__(WG) void k_vtw(const double* __restrict__ V, int64_t ld, int nc,
                                            const double* __restrict__ w, const double* __restrict__ z, int64_t n,
                                            double* __restrict__ part) {
    const int ntot = nc + (z ? 1 : 0);
    const int c0 = (int)blockIdx.y * VTW_CHUNK;
    double acc[VTW_CHUNK];
#pragma unroll
    for (int k = 0; k < VTW_CHUNK; ++k) acc[k] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x; row < n; row += stride) {
        double v[VTW_CHUNK];
#pragma unroll
        for (int k = 0; k < VTW_CHUNK; ++k) {
            const int c = c0 + k;
            if (c < nc) v[k] = V[c * ld + row];
            else if (c == nc && z) v[k] = z[row];
        }
        const double wv = w[row];
#pragma unroll
        for (int k = 0; k < VTW_CHUNK; ++k)
            if (c0 + k < ntot) acc[k] += v[k] * wv;
    }
    __shared__ double red[WG / 64][VTW_CHUNK];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < VTW_CHUNK; ++k) {
        if (c0 + k < ntot) {
            double v = acc[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) red[wave][k] = v;
        }
    }
    __syncthreads();
    const int k = threadIdx.x;
    if (k < VTW_CHUNK && c0 + k < ntot) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < WG / 64; ++q) v += red[q][k];
        const int slot = c0 + k < nc ? c0 + k : EIG_MAX_COLS;
        part[(int64_t)slot * EIG_BLOCKS + blockIdx.x] = v;
    }
}

// out[c] = sum_b part[c][b]; workgroup g reduces column g (g < nc), or column
// EIG_MAX_COLS for g == nc when with_z
__global__ __launch_bounds__(WG) void k_eig_reduce(const double* __restrict__ part, int nparts, int nc,
                                                   double* __restrict__ out) {
    const int c = (int)blockIdx.x < nc ? (int)blockIdx.x : EIG_MAX_COLS;
    const double* src = part + (int64_t)c * EIG_BLOCKS;
    double v = 0.0;
    for (int b = threadIdx.x; b < nparts; b += WG) v += src[b];
    __shared__ double red[WG / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < WG / 64; ++q) t += red[q];
        out[c] = t;
    }
}

void launch_vtw(const double* V, int64_t ld, int nc, const double* w, const double* z, int64_t n, double* part,
                double* out, hipStream_t s) {
    const int nb = eig_blocks(n), ncols = nc + (z ? 1 : 0);
    if (ncols == 0) return;
    hipLaunchKernelGGL(k_vtw, dim3(nb, (unsigned)ceil_div(ncols, VTW_CHUNK)), dim3(WG), 0, s, V, ld, nc, w, z, n,
                       part);
    hipLaunchKernelGGL(k_eig_reduce, dim3(ncols), dim3(WG), 0, s, part, nb, nc, out);
}

// out[row] = a in[row] + sum_c V[c][row] coef[c]   (in may be NULL, may equal out)
__global__ __launch_bounds__(WG) void k_vupdate(const double* __restrict__ V, int64_t ld, int nc,
                                                const double* __restrict__ coef, double a, const double* in,
                                                double* out, int64_t n) {
    const int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (row >= n) return;
    double v[EIG_MAX_COLS];
#pragma unroll
    for (int c = 0; c < EIG_MAX_COLS; ++c)
        if (c < nc) v[c] = V[c * ld + row];
    double acc = in ? a * in[row] : 0.0;
#pragma unroll
    for (int c = 0; c < EIG_MAX_COLS; ++c)
        if (c < nc) acc += v[c] * coef[c];
    out[row] = acc;
}

void launch_vupdate(const double* V, int64_t ld, int nc, const double* coef, double a, const double* in, double* out,
                    int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_vupdate, dim3(grid_for(n)), dim3(WG), 0, s, V, ld, nc, coef, a, in, out, n);
}

// dst[k][row] = sum_c V[c][row] Y[c + k nc] for k < m: the rows of V times the
// nc x m matrix Y.  Each thread holds its whole row of V before writing, so dst
// may be V itself (the restart V <- V Y).
__global__ __launch_bounds__(WG) void k_vrotate(double* V, int64_t ld, int nc, const double* __restrict__ Y, int m,
                                                double* dst, int64_t ldd, int64_t n) {
    const int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (row >= n) return;
    double v[EIG_MAX_COLS];
#pragma unroll
    for (int c = 0; c < EIG_MAX_COLS; ++c) v[c] = c < nc ? V[c * ld + row] : 0.0;
    for (int k = 0; k < m; ++k) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < EIG_MAX_COLS; ++c)
            if (c < nc) s += v[c] * Y[c + k * nc];
        dst[k * ldd + row] = s;
    }
}

void launch_vrotate(double* V, int64_t ld, int nc, const double* Y, int m, double* dst, int64_t ldd, int64_t n,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_vrotate, dim3(grid_for(n)), dim3(WG), 0, s, V, ld, nc, Y, m, dst, ldd, n);
}

// r = Aq - theta Bq; part[b][0] = sum r^2, part[b][1] = sum Bq^2 over block b
__global__ __launch_bounds__(WG) void k_eig_resid(const double* __restrict__ Aq, const double* __restrict__ Bq,
                                                  double theta, double* __restrict__ r, int64_t n,
                                                  double* __restrict__ part) {
    double rr = 0.0, bb = 0.0;
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x; row < n; row += stride) {
        const double b = Bq[row];
        const double v = Aq[row] - theta * b;
        r[row] = v;
        rr += v * v;
        bb += b * b;
    }
    __shared__ double red[WG / 64][2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        rr += __shfl_xor(rr, off, 64);
        bb += __shfl_xor(bb, off, 64);
    }
    if (lane == 0) {
        red[wave][0] = rr;
        red[wave][1] = bb;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < WG / 64; ++q) v += red[q][threadIdx.x];
        part[(int64_t)threadIdx.x * EIG_BLOCKS + blockIdx.x] = v;
    }
}

void launch_eig_resid(const double* Aq, const double* Bq, double theta, double* r, int64_t n, double* part,
                      double* out, hipStream_t s) {
    const int nb = eig_blocks(n);
    hipLaunchKernelGGL(k_eig_resid, dim3(nb), dim3(WG), 0, s, Aq, Bq, theta, r, n, part);
    hipLaunchKernelGGL(k_eig_reduce, dim3(2), dim3(WG), 0, s, part, nb, 2, out);
}

}  // namespace tmi
