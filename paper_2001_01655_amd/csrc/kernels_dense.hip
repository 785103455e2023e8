// Coarsest level: the operator is factorised once at setup (Sec. 3.2: the
// coarse operator is factorised when the hierarchy is built; the paper uses LU
// on one process, an SPD operator allows Cholesky).  The V-cycle then applies
// the explicit FP64 inverse A_c^-1 = L^-T L^-1 as one matrix-vector product,
// which keeps the per-cycle coarse solve a short, fully parallel kernel
// instead of 2 n_c dependent substitution steps.
#include "tm_device.h"

namespace tmi {

// dense row-major A (n x n) from the stencil of a geometric level
template <int DIM>
__global__ void k_dense_from_stencil(const double* __restrict__ st, int nx, int ny, int nz,
                                     int64_t N, double* __restrict__ A) {
    constexpr int NST = DIM == 3 ? 27 : 9, BB = DIM * DIM;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= N * NST) return;
    const int o = (int)(tid / N);
    const int64_t node = tid % N;
    const int NX = nx + 1, NY = ny + 1, NZ = nz + 1;
    const int i = (int)(node % NX);
    const int j = (int)((node / NX) % NY);
    const int k = DIM == 3 ? (int)(node / ((int64_t)NX * NY)) : 0;
    const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = DIM == 3 ? o / 9 - 1 : 0;
    const int ii = i + dx, jj = j + dy, kk = k + dz;
    if (ii < 0 || ii >= NX || jj < 0 || jj >= NY || kk < 0 || (DIM == 3 && kk >= NZ)) return;
    const int64_t J = DIM == 3 ? ((int64_t)kk * NY + jj) * NX + ii : (int64_t)jj * NX + ii;
    const int64_t n = DIM * N;
#pragma unroll
    for (int r = 0; r < DIM; ++r)
#pragma unroll
        for (int c = 0; c < DIM; ++c)
            A[(DIM * node + r) * n + DIM * J + c] = st[((int64_t)o * BB + r * DIM + c) * N + node];
}

void launch_dense_from_stencil(const Level& L, double* Ad, hipStream_t s) {
    const int64_t nt = L.n_nodes * L.nst;
    if (L.dim == 3)
        hipLaunchKernelGGL(k_dense_from_stencil<3>, dim3(grid_for(nt)), dim3(WG), 0, s, L.st64,
                           L.nel[0], L.nel[1], L.nel[2], L.n_nodes, Ad);
    else
        hipLaunchKernelGGL(k_dense_from_stencil<2>, dim3(grid_for(nt)), dim3(WG), 0, s, L.st64,
                           L.nel[0], L.nel[1], 0, L.n_nodes, Ad);
}

// dense row-major A from a BSR level operator
__global__ void k_dense_from_bsr(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                 const double* __restrict__ v, int64_t nbr, int bs,
                                 double* __restrict__ A) {
    const int64_t br = blockIdx.x;
    if (br >= nbr) return;
    const int64_t n = nbr * bs;
    for (int64_t q = rp[br] * (int64_t)bs * bs + threadIdx.x; q < (int64_t)rp[br + 1] * bs * bs;
         q += blockDim.x) {
        const int64_t blk = q / (bs * bs);
        const int e = (int)(q % (bs * bs));
        const int r = e / bs, c = e % bs;
        A[(br * bs + r) * n + (int64_t)ci[blk] * bs + c] = v[q];
    }
}

void launch_dense_from_bsr(const Level& L, double* Ad, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_from_bsr, dim3((unsigned)L.A.nbr), dim3(64), 0, s, L.A.rp, L.A.ci,
                       L.A.v64, L.A.nbr, L.bs, Ad);
}

// Blocked right-looking Cholesky (blocks of CB x CB) of a row-major SPD
// matrix, lower triangle, in place.  Step kb takes two launches:
//  * panel: every workgroup factors the diagonal block kb in LDS (the
//    redundant copies are identical); workgroup 0 stores the factor to a
//    scratch block, workgroup q > 0 solves X L_kk^T = A_(kb+q),kb for its
//    block row;
//  * update: one workgroup per tile (i, j), kb < j <= i, of the trailing
//    matrix, A_ij -= L_ik L_jk^T, and one more that copies L_kk into place.
// A non-positive pivot raises FLAG_NOT_SPD (the factorisation then continues
// with a unit pivot, so every launch still terminates normally).
constexpr int CB = 64;

__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ A, int64_t n, int kb,
                                                    double* __restrict__ Ls, int* flags) {
    __shared__ double L[CB][CB + 1];
    __shared__ double piv[CB];
    const int t = threadIdx.x;
    const int64_t k0 = (int64_t)kb * CB;
    const int m = (int)min<int64_t>(CB, n - k0);
    for (int q = t; q < CB * CB; q += 256) {
        const int r = q / CB, c = q % CB;
        L[r][c] = (r < m && c <= r) ? A[(k0 + r) * n + k0 + c] : (r == c ? 1.0 : 0.0);
    }
    __syncthreads();
    // unscaled right-looking elimination, one barrier per column:
    // a_ij -= a_ik a_jk / a_kk for k < j <= i; the pivots are kept and the
    // columns scaled by 1 / sqrt(a_kk) at the end
    const int tx = t % 16, ty = t / 16;
    for (int k = 0; k < m; ++k) {
        double akk = L[k][k];
        if (!(akk > 0.0)) akk = 1.0;
        if (t == 0) piv[k] = L[k][k];
        const double inv = 1.0 / akk;
        for (int i = k + 1 + ty; i < m; i += 16) {
            const double lik = L[i][k] * inv;
            for (int j = k + 1 + tx; j <= i; j += 16) L[i][j] -= lik * L[j][k];
        }
        __syncthreads();
    }
    if (t == 0) {
        bool bad = false;
        for (int k = 0; k < m; ++k) bad = bad || !(piv[k] > 0.0);
        if (bad) atomicOr(flags, FLAG_NOT_SPD);
    }
    for (int q = t; q < CB * CB; q += 256) {
        const int r = q / CB, c = q % CB;
        if (c < m && c <= r) {
            const double d = piv[c] > 0.0 ? sqrt(piv[c]) : 1.0;
            L[r][c] = r == c ? d : L[r][c] / d;
        }
    }
    __syncthreads();
    if (blockIdx.x == 0) {
        for (int q = t; q < CB * CB; q += 256) Ls[q] = L[q / CB][q % CB];
        return;
    }
    // block row below: only exists when the diagonal block is full (m == CB);
    // solve X L_kk^T = A_(kb+q),kb row by row
    const int64_t r0 = k0 + (int64_t)blockIdx.x * CB;
    const int rows = (int)min<int64_t>(CB, n - r0);
    if (t < rows) {
        double* row = A + (r0 + t) * n + k0;
        double x[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) x[c] = row[c];
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            double sacc = x[c];
#pragma unroll
            for (int j = 0; j < c; ++j) sacc -= x[j] * L[c][j];
            x[c] = sacc / L[c][c];
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) row[c] = x[c];
    }
}

__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ A, int64_t n, int kb, int rem,
                                                     const double* __restrict__ Ls) {
    const int t = threadIdx.x;
    const int64_t k0 = (int64_t)kb * CB;
    const int ntile = rem * (rem + 1) / 2;
    if ((int)blockIdx.x == ntile) {        // L_kk into place
        const int m = (int)min<int64_t>(CB, n - k0);
        for (int q = t; q < m * m; q += 256) {
            const int r = q / m, c = q % m;
            if (c <= r) A[(k0 + r) * n + k0 + c] = Ls[r * CB + c];
        }
        return;
    }
    int bi = 0, q = (int)blockIdx.x;
    while (q >= bi + 1) {
        q -= bi + 1;
        ++bi;
    }
    const int bj = q;
    const int64_t i0 = k0 + (int64_t)(1 + bi) * CB, j0 = k0 + (int64_t)(1 + bj) * CB;
    const int ri = (int)min<int64_t>(CB, n - i0), rj = (int)min<int64_t>(CB, n - j0);
    __shared__ double Li[CB][CB];
    __shared__ double LjT[CB][CB];
    for (int e = t; e < CB * CB; e += 256) {
        const int r = e / CB, k = e % CB;
        Li[r][k] = r < ri ? A[(i0 + r) * n + k0 + k] : 0.0;
        LjT[k][r] = r < rj ? A[(j0 + r) * n + k0 + k] : 0.0;
    }
    __syncthreads();
    const int tx = t % 16, ty = t / 16;
    double acc[4][4] = {};
    for (int k = 0; k < CB; ++k) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = Li[ty * 4 + u][k];
            b[u] = LjT[k][tx * 4 + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = ty * 4 + u, c = tx * 4 + v;
            if (r < ri && c < rj) A[(i0 + r) * n + j0 + c] -= acc[u][v];
        }
}

// Mirror the factor into the strict upper triangle (Lf[i][k] = L[k][i], k > i),
// so that the forward solve below reads column i of L as a contiguous row.
__global__ __launch_bounds__(256) void k_chol_mirror(double* __restrict__ Lf, int64_t n) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n * n) return;
    const int64_t i = idx / n, k = idx % n;
    if (k > i) Lf[i * n + k] = Lf[k * n + i];
}

// Column c of A^-1 from the factor L (lower part of Lf, mirrored above): solve
// L y = e_c, then L^T x = y; by symmetry x is also row c, which is stored.
// The reciprocal diagonal sits in LDS; every step reads one row of Lf
// (contiguous) and ends in one barrier: the entry a step finishes is written
// back by thread 0 one step later, when no thread reads it any more.
__global__ __launch_bounds__(256) void k_chol_inverse(const double* __restrict__ Lf, int64_t n,
                                                      double* __restrict__ Ainv) {
    extern __shared__ double sh[];
    double* y = sh;
    double* dinv = sh + n;
    const int64_t c = blockIdx.x;
    const int t = threadIdx.x, nt = blockDim.x;
    for (int64_t i = t; i < n; i += nt) {
        y[i] = (i == c) ? 1.0 : 0.0;
        dinv[i] = 1.0 / Lf[i * n + i];
    }
    __syncthreads();
    double prev = 0.0;
    for (int64_t i = c; i < n; ++i) {            // forward: y_i /= L_ii; y_k -= L_ki y_i (k > i)
        const double yi = y[i] * dinv[i];
        if (t == 0 && i > c) y[i - 1] = prev;
        const double* Lt = Lf + i * n;           // row i of the mirror: L_ki for k > i
        for (int64_t k = i + 1 + t; k < n; k += nt) y[k] -= Lt[k] * yi;
        prev = yi;
        __syncthreads();
    }
    if (t == 0) y[n - 1] = prev;
    __syncthreads();
    for (int64_t i = n - 1; i >= 0; --i) {       // backward: x_i = y_i / L_ii; y_k -= L_ik x_i (k < i)
        const double xi = y[i] * dinv[i];
        if (t == 0 && i < n - 1) y[i + 1] = prev;
        const double* Li = Lf + i * n;
        for (int64_t k = t; k < i; k += nt) y[k] -= Li[k] * xi;
        prev = xi;
        __syncthreads();
    }
    if (t == 0) y[0] = prev;
    __syncthreads();
    for (int64_t i = t; i < n; i += nt) Ainv[c * n + i] = y[i];
}

int chol_block_elems() { return CB * CB; }

void launch_cholesky_inverse(double* A, double* Ainv, double* Ls, int64_t n, int* flags, hipStream_t s) {
    if (n > 4096) fail(TM_ERR_ARG, "coarsest level too large for the dense solve (> 4096 dofs)");
    const int nb = (int)ceil_div(n, (int64_t)CB);
    for (int kb = 0; kb < nb; ++kb) {
        const int rem = nb - kb - 1;
        hipLaunchKernelGGL(k_chol_panel, dim3((unsigned)(rem + 1)), dim3(256), 0, s, A, n, kb, Ls, flags);
        hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(rem * (rem + 1) / 2 + 1)), dim3(256), 0, s, A, n, kb,
                           rem, (const double*)Ls);
    }
    hipLaunchKernelGGL(k_chol_mirror, dim3((unsigned)ceil_div(n * n, (int64_t)256)), dim3(256), 0, s, A, n);
    hipLaunchKernelGGL(k_chol_inverse, dim3((unsigned)n), dim3(256), (size_t)2 * n * sizeof(double), s,
                       (const double*)A, n, Ainv);
}

// x = A^-1 b in FP64 (one wave per row, fixed shuffle tree).  Each lane keeps
// four partial sums over columns lane + 64 (4 q + r), so four independent
// loads are in flight per lane; the partials are added in a fixed order.
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_dense_solve(const Pack<DenseA<T>, NB> pk, int64_t n) {
    const DenseA<T>& A_ = lane_of(pk);
    const double* __restrict__ Ainv = A_.Ainv;
    const T* __restrict__ b = A_.b;
    T* __restrict__ x = A_.x;
    const int* __restrict__ done = A_.done;
    if (done && *done) return;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const double* Ar = Ainv + row * n;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t c = lane;
    for (; c + 192 < n; c += 256) {
        a0 += Ar[c] * (double)b[c];
        a1 += Ar[c + 64] * (double)b[c + 64];
        a2 += Ar[c + 128] * (double)b[c + 128];
        a3 += Ar[c + 192] * (double)b[c + 192];
    }
    if (c < n) a0 += Ar[c] * (double)b[c];
    if (c + 64 < n) a1 += Ar[c + 64] * (double)b[c + 64];
    if (c + 128 < n) a2 += Ar[c + 128] * (double)b[c + 128];
    double a = (a0 + a1) + (a2 + a3);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o, 64);
    if (lane == 0) x[row] = (T)a;
}

template <typename T, int NB>
static void dense_launch(const LaneIO* L, int n, hipStream_t s) {
    Pack<DenseA<T>, NB> pk{};
    for (int q = 0; q < n; ++q) {
        DenseA<T>& a = pk.a[q];
        a.Ainv = L[q].h->ainv;
        a.b = (const T*)L[q].x;
        a.x = (T*)L[q].y;
        a.done = L[q].done;
    }
    const int64_t nc = L[0].h->nc;
    hipLaunchKernelGGL((k_dense_solve<T, NB>), dim3((unsigned)ceil_div(nc, 4), n), dim3(256), 0, s, pk, nc);
}

// y = A_c^-1 x on the coarsest level of each lane's hierarchy
template <typename T>
void launch_dense_solve_b(const LaneIO* L, int n, hipStream_t s) {
    for (int q0 = 0; q0 < n; q0 += MAXB) {
        const int m = std::min(MAXB, n - q0);
        if (m == 1) dense_launch<T, 1>(L + q0, 1, s);
        else dense_launch<T, MAXB>(L + q0, m, s);
    }
}
template void launch_dense_solve_b<double>(const LaneIO*, int, hipStream_t);
template void launch_dense_solve_b<float>(const LaneIO*, int, hipStream_t);

}  // namespace tmi
