// Setup of the smoothed-aggregation levels of the hybrid hierarchy (Sec. 3.2
// algebraic multigrid; Sec. 4 block strength of connection with beta, the
// tentative prolongator smoothed by one weighted-Jacobi step, rigid-body
// modes as candidates).  Every result is independent of thread scheduling:
// integer decisions are order-free (min / max / set), and every floating-point
// sum runs over its terms in ascending index order.
//
//  strength      I != J strong iff f_IJ^2 > beta^2 f_II f_JJ, f = squared
//                Frobenius norm of the block; symmetrised (either direction).
//  aggregation   roots = lexicographically-first maximal distance-2
//                independent set under key h(i) = MurmurHash3 fmix32(i),
//                computed by rounds of "undecided local minimum over the
//                distance-2 neighbourhood" (the serial greedy result);
//                pass 1: neighbours of roots; pass 2: remaining nodes join
//                the pass-1 neighbour whose root has the smallest key;
//                aggregate ids by increasing root index.
//  tentative     per aggregate, modified Gram-Schmidt of the candidate rows
//                (members ascending), R_jj >= 0, columns with remaining norm
//                <= 1e-10 of the original set to zero (kept in the pattern).
//  prolongator   P = T - omega D^-1 A T, omega = (4/3) / ||D^-1 A||_inf.
//  coarse        A_c = P^T (A P); exactly-zero diagonal entries set to 1.
#include <cstring>

#include "tm_device.h"

namespace tmi {

// ------------------------------------------------------------------ scan
// exclusive prefix sum of n int32 values (out may alias in), total in *total
constexpr int SCAN_SEG = 4096;

__global__ void k_seg_sums(const int32_t* __restrict__ in, int64_t n, int64_t* __restrict__ bsum) {
    __shared__ int64_t red[WG];
    const int64_t base = (int64_t)blockIdx.x * SCAN_SEG;
    int64_t a = 0;
    for (int64_t i = base + threadIdx.x; i < min(base + SCAN_SEG, n); i += WG) a += in[i];
    red[threadIdx.x] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int w = 0; w < WG; ++w) s += red[w];
        bsum[blockIdx.x] = s;
    }
}

__global__ void k_seg_offsets(int64_t* bsum, int64_t nb, int64_t* total) {
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t v = bsum[b];
            bsum[b] = s;
            s += v;
        }
        *total = s;
    }
}

__global__ void k_seg_scan(const int32_t* in, int64_t n, const int64_t* __restrict__ boff, int32_t* out) {
    // one block per segment, sequential in chunks of WG with a block scan
    __shared__ int64_t sh[WG];
    __shared__ int64_t carry;
    const int64_t base = (int64_t)blockIdx.x * SCAN_SEG;
    if (threadIdx.x == 0) carry = boff[blockIdx.x];
    __syncthreads();
    for (int64_t c0 = base; c0 < min(base + SCAN_SEG, n); c0 += WG) {
        const int64_t i = c0 + threadIdx.x;
        const int64_t v = i < n ? in[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < WG; o <<= 1) {
            const int64_t t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        const int64_t incl = sh[threadIdx.x];
        const int64_t c = carry;
        __syncthreads();
        if (i < n) out[i] = (int32_t)(c + incl - v);
        if (threadIdx.x == WG - 1) carry = c + incl;
        __syncthreads();
    }
}

// scan in place from in[0..n) to out[0..n] (out[n] = total); returns total
int64_t scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int64_t* work, hipStream_t s) {
    const int64_t nb = std::max<int64_t>(1, ceil_div(n, SCAN_SEG));
    int64_t* bsum = work;                 // nb entries
    int64_t* total = work + nb;           // 1 entry
    hipLaunchKernelGGL(k_seg_sums, dim3((unsigned)nb), dim3(WG), 0, s, in, n, bsum);
    hipLaunchKernelGGL(k_seg_offsets, dim3(1), dim3(64), 0, s, bsum, nb, total);
    hipLaunchKernelGGL(k_seg_scan, dim3((unsigned)nb), dim3(WG), 0, s, in, n, (const int64_t*)bsum, out);
    int64_t t = 0;
    TM_HIP(hipMemcpyAsync(&t, total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    TM_HIP(hipStreamSynchronize(s));
    if (t >= ((int64_t)1 << 31)) fail(TM_ERR_ARG, "aggregation structure exceeds int32 indexing");
    const int32_t t32 = (int32_t)t;
    TM_HIP(hipMemcpyAsync(out + n, &t32, sizeof(int32_t), hipMemcpyHostToDevice, s));
    TM_HIP(hipStreamSynchronize(s));
    return t;
}

// ------------------------------------------------------------------ stencil -> BSR
template <int DIM>
__global__ void k_stencil_to_bsr(const double* __restrict__ st, int nx, int ny, int nz, int64_t N,
                                 const int32_t* __restrict__ rp, int32_t* __restrict__ ci,
                                 double* __restrict__ v) {
    constexpr int BB = DIM * DIM;
    const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= N) return;
    const int NX = nx + 1, NY = ny + 1, NZ = nz + 1;
    const int i = (int)(node % NX), j = (int)((node / NX) % NY);
    const int k = DIM == 3 ? (int)(node / ((int64_t)NX * NY)) : 0;
    int32_t q = rp[node];
    for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int ii = i + dx, jj = j + dy, kk = k + dz;
                if (ii < 0 || ii >= NX || jj < 0 || jj >= NY || kk < 0 || (DIM == 3 && kk >= NZ)) continue;
                const int o = DIM == 3 ? (dz + 1) * 9 + (dy + 1) * 3 + dx + 1 : (dy + 1) * 3 + dx + 1;
                ci[q] = (int32_t)(DIM == 3 ? ((int64_t)kk * NY + jj) * NX + ii : (int64_t)jj * NX + ii);
                for (int e = 0; e < BB; ++e) v[(int64_t)q * BB + e] = st[((int64_t)o * BB + e) * N + node];
                ++q;
            }
}

void launch_stencil_to_bsr(const Level& L, const int32_t* rp, int32_t* ci, double* v, hipStream_t s) {
    const dim3 g(grid_for(L.n_nodes)), b(WG);
    if (L.dim == 3)
        hipLaunchKernelGGL(k_stencil_to_bsr<3>, g, b, 0, s, L.st64, L.nel[0], L.nel[1], L.nel[2], L.n_nodes,
                           rp, ci, v);
    else
        hipLaunchKernelGGL(k_stencil_to_bsr<2>, g, b, 0, s, L.st64, L.nel[0], L.nel[1], 0, L.n_nodes, rp, ci,
                           v);
}

// ------------------------------------------------------------------ strength
// squared Frobenius norm of a bs x bs block
__device__ __forceinline__ double fsq(const double* b, int bs) {
    double s = 0.0;
    for (int i = 0; i < bs * bs; ++i) s += b[i] * b[i];
    return s;
}

__device__ __forceinline__ int32_t find_col(const int32_t* ci, int32_t lo, int32_t hi, int32_t c) {
    while (lo < hi) {
        const int32_t m = (lo + hi) >> 1;
        if (ci[m] < c) lo = m + 1;
        else hi = m;
    }
    return lo;
}

__global__ void k_diag_fsq(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const double* __restrict__ v, int64_t n, int bs, double* __restrict__ dn) {
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= n) return;
    const int32_t q = find_col(ci, rp[I], rp[I + 1], (int32_t)I);
    dn[I] = (q < rp[I + 1] && ci[q] == I) ? fsq(v + (int64_t)q * bs * bs, bs) : 0.0;
}

// strong(I,J): the test holds for block (I,J) or for block (J,I)
__device__ __forceinline__ bool strong_pair(const int32_t* rp, const int32_t* ci, const double* v,
                                            const double* dn, int bs, double beta2, int64_t I, int32_t q) {
    const int32_t J = ci[q];
    const double thr = beta2 * (dn[I] * dn[J]);
    const double f1 = fsq(v + (int64_t)q * bs * bs, bs);
    if (f1 * f1 > thr) return true;
    const int32_t p = find_col(ci, rp[J], rp[J + 1], (int32_t)I);
    if (p < rp[J + 1] && ci[p] == (int32_t)I) {
        const double f2 = fsq(v + (int64_t)p * bs * bs, bs);
        if (f2 * f2 > thr) return true;
    }
    return false;
}

template <bool FILL>
__global__ void k_strength(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const double* __restrict__ v, const double* __restrict__ dn, int64_t n, int bs,
                           double beta2, int32_t* __restrict__ cnt, const int32_t* __restrict__ srp,
                           int32_t* __restrict__ sci) {
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= n) return;
    int32_t c = 0;
    for (int32_t q = rp[I]; q < rp[I + 1]; ++q) {
        if (ci[q] == (int32_t)I) continue;
        if (strong_pair(rp, ci, v, dn, bs, beta2, I, q)) {
            if (FILL) sci[srp[I] + c] = ci[q];
            ++c;
        }
    }
    if (!FILL) cnt[I] = c;
}

// ------------------------------------------------------------------ aggregation
constexpr uint64_t KEY_NONE = 1ull << 32;

// m1[i] = min key of undecided nodes in {i} u S(i)
__global__ void k_mis_min(const int32_t* __restrict__ srp, const int32_t* __restrict__ sci, int64_t n,
                          const uint8_t* __restrict__ state, const uint64_t* __restrict__ src,
                          uint64_t* __restrict__ dst, int first) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    auto val = [&](int64_t j) -> uint64_t {
        if (first) return state[j] == 0 ? (uint64_t)fmix32((uint32_t)j) : KEY_NONE;
        return src[j];
    };
    uint64_t m = val(i);
    for (int32_t q = srp[i]; q < srp[i + 1]; ++q) m = min(m, val(sci[q]));
    dst[i] = m;
}

__global__ void k_mis_select(int64_t n, uint8_t* __restrict__ state, const uint64_t* __restrict__ m2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (state[i] == 0 && m2[i] == (uint64_t)fmix32((uint32_t)i)) state[i] = 1;
}

// f[i] = 1 if {i} u S(i) holds a root
__global__ void k_mis_near_root(const int32_t* __restrict__ srp, const int32_t* __restrict__ sci, int64_t n,
                                const uint8_t* __restrict__ state, uint8_t* __restrict__ f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint8_t r = state[i] == 1;
    for (int32_t q = srp[i]; q < srp[i + 1] && !r; ++q) r = state[sci[q]] == 1;
    f[i] = r;
}

__global__ void k_mis_exclude(const int32_t* __restrict__ srp, const int32_t* __restrict__ sci, int64_t n,
                              uint8_t* __restrict__ state, const uint8_t* __restrict__ f,
                              int32_t* __restrict__ undecided) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (state[i] != 0) return;
    bool near = f[i];
    for (int32_t q = srp[i]; q < srp[i + 1] && !near; ++q) near = f[sci[q]];
    if (near)
        state[i] = 2;
    else
        atomicAdd(undecided, 1);
}

__global__ void k_root_flags(int64_t n, const uint8_t* __restrict__ state, int32_t* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = state[i] == 1;
}

// pass 1: roots and their strong neighbours
__global__ void k_agg_pass1(const int32_t* __restrict__ srp, const int32_t* __restrict__ sci, int64_t n,
                            const uint8_t* __restrict__ state, const int32_t* __restrict__ rid,
                            int32_t* __restrict__ agg, int32_t* __restrict__ root) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (state[i] == 1) {
        agg[i] = rid[i];
        root[i] = (int32_t)i;
        return;
    }
    agg[i] = -1;
    root[i] = -1;
    for (int32_t q = srp[i]; q < srp[i + 1]; ++q) {
        const int32_t j = sci[q];
        if (state[j] == 1) {
            agg[i] = rid[j];
            root[i] = j;
            return;
        }
    }
}

// pass 2: join the pass-1 neighbour whose root has the smallest key
__global__ void k_agg_pass2(const int32_t* __restrict__ srp, const int32_t* __restrict__ sci, int64_t n,
                            const int32_t* __restrict__ agg1, const int32_t* __restrict__ root1,
                            int32_t* __restrict__ agg, int32_t* __restrict__ missing) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (agg1[i] >= 0) {
        agg[i] = agg1[i];
        return;
    }
    int32_t best = -1;
    uint32_t bk = 0;
    for (int32_t q = srp[i]; q < srp[i + 1]; ++q) {
        const int32_t j = sci[q];
        if (agg1[j] < 0) continue;
        const int32_t r = root1[j];
        const uint32_t kr = fmix32((uint32_t)r);
        if (best < 0 || kr < bk || (kr == bk && r < best)) {
            best = r;
            bk = kr;
        }
    }
    if (best < 0) {
        agg[i] = -1;
        atomicAdd(missing, 1);
    } else {
        agg[i] = agg1[best];
    }
}

// ------------------------------------------------------------------ members, tentative prolongator
__global__ void k_count_members(int64_t n, const int32_t* __restrict__ agg, int32_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(&cnt[agg[i]], 1);
}
__global__ void k_place_members(int64_t n, const int32_t* __restrict__ agg, const int32_t* __restrict__ off,
                                int32_t* __restrict__ cursor, int32_t* __restrict__ mem) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) mem[off[agg[i]] + atomicAdd(&cursor[agg[i]], 1)] = (int32_t)i;
}
// insertion sort of each segment [off[g], off[g+1])
__global__ void k_sort_segments(int64_t ng, const int32_t* __restrict__ off, int32_t* __restrict__ a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    for (int32_t p = off[g] + 1; p < off[g + 1]; ++p) {
        const int32_t v = a[p];
        int32_t q = p - 1;
        while (q >= off[g] && a[q] > v) {
            a[q + 1] = a[q];
            --q;
        }
        a[q + 1] = v;
    }
}

// Node positions of geometric level l: each coarsening puts coarse node I on
// fine node min(2I, n) of the level above, so node I of level l sits on fine
// node min(2^l I, n0) of its axis (n0 fine elements), at h times that.
struct LevelPos {
    double h;
    int sc;                 // 2^l
    int n0[3];              // fine elements per axis
};

// candidate block of node i: first aggregation step = rigid-body modes at the
// node coordinates of a geometric level, later steps = R factors of the step before
__device__ __forceinline__ double cand(const double* __restrict__ Bprev, int dim, int nx1, int ny1,
                                       const LevelPos& lp, int bs, int k, int64_t i, int r, int c) {
    if (Bprev) return Bprev[((int64_t)i * bs + r) * k + c];
    const int64_t ix = i % nx1, iy = (i / nx1) % ny1, iz = dim == 3 ? i / ((int64_t)nx1 * ny1) : 0;
    const double x = lp.h * (double)min<int64_t>((int64_t)lp.sc * ix, lp.n0[0]);
    const double y = lp.h * (double)min<int64_t>((int64_t)lp.sc * iy, lp.n0[1]);
    const double z = dim == 3 ? lp.h * (double)min<int64_t>((int64_t)lp.sc * iz, lp.n0[2]) : 0.0;
    if (c < dim) return r == c ? 1.0 : 0.0;
    if (dim == 2) return r == 0 ? -y : x;                 // (-y, x)
    if (c == 3) return r == 0 ? 0.0 : (r == 1 ? -z : y);   // (0, -z, y)
    if (c == 4) return r == 0 ? z : (r == 1 ? 0.0 : -x);   // (z, 0, -x)
    return r == 0 ? -y : (r == 1 ? x : 0.0);               // (-y, x, 0)
}

// thread per aggregate: modified Gram-Schmidt on its member rows (in place in T)
__global__ void k_tentative(int64_t ng, const int32_t* __restrict__ off, const int32_t* __restrict__ mem,
                            const double* __restrict__ Bprev, int dim, int nx1, int ny1, const LevelPos lp, int bs,
                            int k, double* __restrict__ T, double* __restrict__ Bc) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const int32_t p0 = off[g], p1 = off[g + 1];
    // T rows of member m: T[(mem * bs + r) * k + c]
    for (int32_t p = p0; p < p1; ++p) {
        const int64_t i = mem[p];
        for (int r = 0; r < bs; ++r)
            for (int c = 0; c < k; ++c) T[((int64_t)i * bs + r) * k + c] = cand(Bprev, dim, nx1, ny1, lp, bs, k, i, r, c);
    }
    double R[6][6];
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) R[a][b] = 0.0;
    for (int j = 0; j < k; ++j) {
        double n0 = 0.0;
        for (int32_t p = p0; p < p1; ++p)
            for (int r = 0; r < bs; ++r) {
                const double v = T[((int64_t)mem[p] * bs + r) * k + j];
                n0 += v * v;
            }
        n0 = sqrt(n0);
        for (int i = 0; i < j; ++i) {
            double d = 0.0;
            for (int32_t p = p0; p < p1; ++p)
                for (int r = 0; r < bs; ++r) {
                    const int64_t row = (int64_t)mem[p] * bs + r;
                    d += T[row * k + i] * T[row * k + j];
                }
            R[i][j] = d;
            for (int32_t p = p0; p < p1; ++p)
                for (int r = 0; r < bs; ++r) {
                    const int64_t row = (int64_t)mem[p] * bs + r;
                    T[row * k + j] -= d * T[row * k + i];
                }
        }
        double nr = 0.0;
        for (int32_t p = p0; p < p1; ++p)
            for (int r = 0; r < bs; ++r) {
                const double v = T[((int64_t)mem[p] * bs + r) * k + j];
                nr += v * v;
            }
        nr = sqrt(nr);
        const bool dead = n0 == 0.0 || nr <= 1e-10 * n0;
        R[j][j] = dead ? 0.0 : nr;
        for (int32_t p = p0; p < p1; ++p)
            for (int r = 0; r < bs; ++r) {
                double& t = T[((int64_t)mem[p] * bs + r) * k + j];
                t = dead ? 0.0 : t / nr;
            }
    }
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) Bc[((int64_t)g * k + a) * k + b] = R[a][b];
}

// ------------------------------------------------------------------ ||D^-1 A||_inf
__global__ void k_dinv_a_rowmax(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                const double* __restrict__ v, const double* __restrict__ dinv, int64_t n, int bs,
                                unsigned long long* __restrict__ out) {
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= n) return;
    double best = 0.0;
    for (int r = 0; r < bs; ++r) {
        double s = 0.0;
        for (int32_t q = rp[I]; q < rp[I + 1]; ++q)
            for (int c = 0; c < bs; ++c) {
                double t = 0.0;
                for (int m = 0; m < bs; ++m)
                    t += dinv[(int64_t)sym_at(r, m, bs) * n + I] * v[((int64_t)q * bs + m) * bs + c];
                s += fabs(t);
            }
        best = fmax(best, s);
    }
    atomicMax(out, (unsigned long long)__double_as_longlong(best));   // non-negative: bit order = value order
}

// ------------------------------------------------------------------ sparse products
// Symbolic phase, one workgroup per output row: mark candidate block columns in
// an LDS bitmap (order-free), then count / emit them in ascending order.
// kind 0: P row I   <- {agg[J] : J in row I of A}
// kind 1: AP row I  <- cols of P rows J in row I of A
// kind 2: Ac row G  <- cols of AP rows I in row G of P^T
struct ProdArgs {
    const int32_t* rp1;   // outer rows
    const int32_t* ci1;
    const int32_t* agg;   // kind 0
    const int32_t* rp2;   // inner rows (kinds 1, 2)
    const int32_t* ci2;
    int32_t ncols;        // size of the column space
};

__device__ void mark_row(const ProdArgs& a, int kind, int64_t row, uint32_t* bits) {
    for (int32_t q = a.rp1[row] + (int32_t)threadIdx.x; q < a.rp1[row + 1]; q += blockDim.x) {
        const int32_t J = a.ci1[q];
        if (kind == 0) {
            const int32_t c = a.agg[J];
            atomicOr(&bits[c >> 5], 1u << (c & 31));
        } else {
            for (int32_t p = a.rp2[J]; p < a.rp2[J + 1]; ++p) {
                const int32_t c = a.ci2[p];
                atomicOr(&bits[c >> 5], 1u << (c & 31));
            }
        }
    }
}

template <bool FILL>
__global__ void k_prod_symbolic(ProdArgs a, int kind, int64_t nrows, int32_t* __restrict__ cnt,
                                const int32_t* __restrict__ orp, int32_t* __restrict__ oci) {
    extern __shared__ uint32_t bits[];
    __shared__ int32_t wsum[WG];
    const int64_t row = blockIdx.x;
    if (row >= nrows) return;
    const int nw = (a.ncols + 31) >> 5;
    for (int w = threadIdx.x; w < nw; w += blockDim.x) bits[w] = 0u;
    __syncthreads();
    mark_row(a, kind, row, bits);
    __syncthreads();
    // per-thread contiguous word range, counts, block prefix
    const int per = (nw + WG - 1) / WG;
    const int w0 = threadIdx.x * per, w1 = min(nw, w0 + per);
    int32_t c = 0;
    for (int w = w0; w < w1; ++w) c += __popc(bits[w]);
    wsum[threadIdx.x] = c;
    __syncthreads();
    if (!FILL) {
        if (threadIdx.x == 0) {
            int32_t t = 0;
            for (int i = 0; i < WG; ++i) t += wsum[i];
            cnt[row] = t;
        }
        return;
    }
    int32_t base = orp[row];
    for (int i = 0; i < (int)threadIdx.x; ++i) base += wsum[i];
    for (int w = w0; w < w1; ++w) {
        uint32_t b = bits[w];
        while (b) {
            const int t = __ffs(b) - 1;
            oci[base++] = (w << 5) + t;
            b &= b - 1;
        }
    }
}

// block row of each stored block
__global__ void k_row_of(const int32_t* __restrict__ rp, int64_t nrows, int32_t* __restrict__ rowof) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    for (int32_t q = rp[r]; q < rp[r + 1]; ++q) rowof[q] = (int32_t)r;
}

// numeric P: block (I, g) = [g == agg[I]] T_I - omega Dinv_I sum_{J in row I, agg[J] = g} A_IJ T_J
__global__ void k_p_numeric(const int32_t* __restrict__ arp, const int32_t* __restrict__ aci,
                            const double* __restrict__ av, const int32_t* __restrict__ agg,
                            const double* __restrict__ T, const double* __restrict__ dinv, int64_t n, int bs, int k,
                            double omega, const int32_t* __restrict__ prow, const int32_t* __restrict__ pci,
                            int64_t nnzb, double* __restrict__ pv) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nnzb) return;
    const int64_t I = prow[b];
    const int32_t g = pci[b];
    double acc[6][6], out[6][6];
    for (int r = 0; r < bs; ++r)
        for (int c = 0; c < k; ++c) acc[r][c] = 0.0;
    for (int32_t q = arp[I]; q < arp[I + 1]; ++q) {
        const int32_t J = aci[q];
        if (agg[J] != g) continue;
        const double* A = av + (int64_t)q * bs * bs;
        const double* TJ = T + (int64_t)J * bs * k;
        for (int r = 0; r < bs; ++r)
            for (int c = 0; c < k; ++c) {
                double t = 0.0;
                for (int m = 0; m < bs; ++m) t += A[r * bs + m] * TJ[m * k + c];
                acc[r][c] += t;
            }
    }
    const double* TI = T + I * bs * k;
    for (int r = 0; r < bs; ++r)
        for (int c = 0; c < k; ++c) {
            double t = 0.0;
            for (int m = 0; m < bs; ++m) t += dinv[(int64_t)sym_at(r, m, bs) * n + I] * acc[m][c];
            out[r][c] = (g == agg[I] ? TI[r * k + c] : 0.0) - omega * t;
        }
    for (int r = 0; r < bs; ++r)
        for (int c = 0; c < k; ++c) pv[(b * bs + r) * k + c] = out[r][c];
}

// transpose of a BSR (br x bc blocks): counts, then placement, then per-row sort
__global__ void k_tr_count(int64_t nnzb, const int32_t* __restrict__ ci, int32_t* __restrict__ cnt) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnzb) atomicAdd(&cnt[ci[q]], 1);
}
__global__ void k_tr_place(int64_t nnzb, const int32_t* __restrict__ rowof, const int32_t* __restrict__ ci,
                           const int32_t* __restrict__ trp, int32_t* __restrict__ cursor,
                           int32_t* __restrict__ tci, int32_t* __restrict__ tsrc) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nnzb) return;
    const int32_t c = ci[q];
    const int32_t p = trp[c] + atomicAdd(&cursor[c], 1);
    tci[p] = rowof[q];
    tsrc[p] = (int32_t)q;
}
// sort each transposed row by column (source row index); keys are unique per row
__global__ void k_tr_sort(int64_t nr, const int32_t* __restrict__ trp, int32_t* __restrict__ tci,
                          int32_t* __restrict__ tsrc) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    for (int32_t p = trp[r] + 1; p < trp[r + 1]; ++p) {
        const int32_t kc = tci[p], ks = tsrc[p];
        int32_t q = p - 1;
        while (q >= trp[r] && tci[q] > kc) {
            tci[q + 1] = tci[q];
            tsrc[q + 1] = tsrc[q];
            --q;
        }
        tci[q + 1] = kc;
        tsrc[q + 1] = ks;
    }
}
__global__ void k_tr_values(int64_t nnzb, const int32_t* __restrict__ tsrc, const double* __restrict__ v, int br,
                            int bc, double* __restrict__ tv) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnzb) return;
    const double* s = v + (int64_t)tsrc[p] * br * bc;
    for (int r = 0; r < bc; ++r)
        for (int c = 0; c < br; ++c) tv[((int64_t)p * bc + r) * br + c] = s[c * bc + r];
}

// numeric C = X Y for one output block (row R, col H):
//   sum_{q in row R of X (ascending)} X_q Y_{ci_x[q], H}  (Y row searched for H)
// X blocks are xr x xc, Y blocks xc x yc.
__global__ void k_prod_numeric(const int32_t* __restrict__ xrp, const int32_t* __restrict__ xci,
                               const double* __restrict__ xv, int xr, int xc, const int32_t* __restrict__ yrp,
                               const int32_t* __restrict__ yci, const double* __restrict__ yv, int yc,
                               const int32_t* __restrict__ crow, const int32_t* __restrict__ cci, int64_t nnzb,
                               double* __restrict__ cv) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nnzb) return;
    const int32_t R = crow[b], H = cci[b];
    double acc[6][6];
    for (int r = 0; r < xr; ++r)
        for (int c = 0; c < yc; ++c) acc[r][c] = 0.0;
    for (int32_t q = xrp[R]; q < xrp[R + 1]; ++q) {
        const int32_t J = xci[q];
        const int32_t p = find_col(yci, yrp[J], yrp[J + 1], H);
        if (p >= yrp[J + 1] || yci[p] != H) continue;
        const double* X = xv + (int64_t)q * xr * xc;
        const double* Y = yv + (int64_t)p * xc * yc;
        for (int r = 0; r < xr; ++r)
            for (int c = 0; c < yc; ++c) {
                double t = 0.0;
                for (int m = 0; m < xc; ++m) t += X[r * xc + m] * Y[m * yc + c];
                acc[r][c] += t;
            }
    }
    for (int r = 0; r < xr; ++r)
        for (int c = 0; c < yc; ++c) cv[(b * xr + r) * yc + c] = acc[r][c];
}

// exactly-zero diagonal entries of a square BSR become 1
__global__ void k_fix_diag(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, int64_t n, int bs,
                           double* __restrict__ v) {
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= n) return;
    const int32_t q = find_col(ci, rp[I], rp[I + 1], (int32_t)I);
    if (q >= rp[I + 1] || ci[q] != I) return;
    for (int r = 0; r < bs; ++r) {
        double& d = v[((int64_t)q * bs + r) * bs + r];
        if (d == 0.0) d = 1.0;
    }
}

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// ------------------------------------------------------------------ host-side launch helpers
void sa_launch_diag_fsq(const BSR& A, int bs, double* dn, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_fsq, dim3(grid_for(A.nbr)), dim3(WG), 0, s, A.rp, A.ci, A.v64, A.nbr, bs, dn);
}
void sa_launch_strength(const BSR& A, int bs, const double* dn, double beta, int32_t* cnt,
                        const int32_t* srp, int32_t* sci, bool fill, hipStream_t s) {
    const double b2 = beta * beta;
    if (fill)
        hipLaunchKernelGGL(k_strength<true>, dim3(grid_for(A.nbr)), dim3(WG), 0, s, A.rp, A.ci, A.v64, dn,
                           A.nbr, bs, b2, cnt, srp, sci);
    else
        hipLaunchKernelGGL(k_strength<false>, dim3(grid_for(A.nbr)), dim3(WG), 0, s, A.rp, A.ci, A.v64, dn,
                           A.nbr, bs, b2, cnt, srp, sci);
}
int sa_mis2(const int32_t* srp, const int32_t* sci, int64_t n, uint8_t* state, uint64_t* m1, uint64_t* m2,
            uint8_t* f, int32_t* counter, hipStream_t s) {
    const dim3 g(grid_for(n)), b(WG);
    TM_HIP(hipMemsetAsync(state, 0, n, s));
    for (int round = 1; round <= 4096; ++round) {
        hipLaunchKernelGGL(k_mis_min, g, b, 0, s, srp, sci, n, state, nullptr, m1, 1);
        hipLaunchKernelGGL(k_mis_min, g, b, 0, s, srp, sci, n, state, (const uint64_t*)m1, m2, 0);
        hipLaunchKernelGGL(k_mis_select, g, b, 0, s, n, state, (const uint64_t*)m2);
        hipLaunchKernelGGL(k_mis_near_root, g, b, 0, s, srp, sci, n, (const uint8_t*)state, f);
        TM_HIP(hipMemsetAsync(counter, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(k_mis_exclude, g, b, 0, s, srp, sci, n, state, (const uint8_t*)f, counter);
        int32_t und = 0;
        TM_HIP(hipMemcpyAsync(&und, counter, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        TM_HIP(hipStreamSynchronize(s));
        if (und == 0) return round;
    }
    fail(TM_ERR_DEVICE, "distance-2 independent set did not finish");
}
void sa_root_flags(int64_t n, const uint8_t* state, int32_t* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_root_flags, dim3(grid_for(n)), dim3(WG), 0, s, n, state, flag);
}
void sa_agg_passes(const int32_t* srp, const int32_t* sci, int64_t n, const uint8_t* state, const int32_t* rid,
                   int32_t* agg1, int32_t* root1, int32_t* agg, int32_t* missing, hipStream_t s) {
    const dim3 g(grid_for(n)), b(WG);
    hipLaunchKernelGGL(k_agg_pass1, g, b, 0, s, srp, sci, n, state, rid, agg1, root1);
    TM_HIP(hipMemsetAsync(missing, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(k_agg_pass2, g, b, 0, s, srp, sci, n, (const int32_t*)agg1, (const int32_t*)root1, agg,
                       missing);
}
void sa_members(int64_t n, int64_t ng, const int32_t* agg, int32_t* cnt_off, int32_t* cursor, int32_t* mem,
                int64_t* work, hipStream_t s) {
    TM_HIP(hipMemsetAsync(cnt_off, 0, sizeof(int32_t) * (ng + 1), s));
    TM_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * ng, s));
    hipLaunchKernelGGL(k_count_members, dim3(grid_for(n)), dim3(WG), 0, s, n, agg, cnt_off);
    scan_exclusive(cnt_off, cnt_off, ng, work, s);
    hipLaunchKernelGGL(k_place_members, dim3(grid_for(n)), dim3(WG), 0, s, n, agg, (const int32_t*)cnt_off,
                       cursor, mem);
    hipLaunchKernelGGL(k_sort_segments, dim3(grid_for(ng)), dim3(WG), 0, s, ng, (const int32_t*)cnt_off, mem);
}
void sa_tentative(int64_t ng, const int32_t* off, const int32_t* mem, const double* Bprev, int dim, int nx1,
                  int ny1, double h, int level, const int* nel0, int bs, int k, double* T, double* Bc, hipStream_t s) {
    LevelPos lp{h, 1 << level, {nel0[0], nel0[1], dim == 3 ? nel0[2] : 0}};
    hipLaunchKernelGGL(k_tentative, dim3(grid_for(ng, 64)), dim3(64), 0, s, ng, off, mem, Bprev, dim, nx1, ny1,
                       lp, bs, k, T, Bc);
}
double sa_jacobi_bound(const BSR& A, int bs, const double* dinv, unsigned long long* work, hipStream_t s) {
    TM_HIP(hipMemsetAsync(work, 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_dinv_a_rowmax, dim3(grid_for(A.nbr)), dim3(WG), 0, s, A.rp, A.ci, A.v64, dinv, A.nbr,
                       bs, work);
    unsigned long long u = 0;
    TM_HIP(hipMemcpyAsync(&u, work, sizeof(u), hipMemcpyDeviceToHost, s));
    TM_HIP(hipStreamSynchronize(s));
    double d;
    memcpy(&d, &u, sizeof(d));
    return d;
}
void sa_symbolic(const int32_t* rp1, const int32_t* ci1, const int32_t* agg, const int32_t* rp2,
                 const int32_t* ci2, int32_t ncols, int kind, int64_t nrows, int32_t* cnt,
                 const int32_t* orp, int32_t* oci, bool fill, hipStream_t s) {
    if (ncols > (1 << 18)) fail(TM_ERR_ARG, "aggregation level too large for the column bitmap (> 262144 blocks)");
    ProdArgs a{rp1, ci1, agg, rp2, ci2, ncols};
    const size_t lds = sizeof(uint32_t) * (size_t)((ncols + 31) / 32 + 1);
    if (fill)
        hipLaunchKernelGGL(k_prod_symbolic<true>, dim3((unsigned)nrows), dim3(WG), lds, s, a, kind, nrows, cnt, orp,
                           oci);
    else
        hipLaunchKernelGGL(k_prod_symbolic<false>, dim3((unsigned)nrows), dim3(WG), lds, s, a, kind, nrows, cnt,
                           orp, oci);
}
void sa_row_of(const int32_t* rp, int64_t nrows, int32_t* rowof, hipStream_t s) {
    hipLaunchKernelGGL(k_row_of, dim3(grid_for(nrows)), dim3(WG), 0, s, rp, nrows, rowof);
}
void sa_p_numeric(const BSR& A, const int32_t* agg, const double* T, const double* dinv, int bs, int k,
                  double omega, const int32_t* prow, const BSR& P, hipStream_t s) {
    hipLaunchKernelGGL(k_p_numeric, dim3(grid_for(P.nnzb, 64)), dim3(64), 0, s, A.rp, A.ci, A.v64, agg, T, dinv,
                       A.nbr, bs, k, omega, prow, P.ci, P.nnzb, P.v64);
}
void sa_transpose(const BSR& P, const int32_t* prow, BSR& PT, int32_t* cursor, int32_t* tsrc, int64_t* work,
                  hipStream_t s) {
    TM_HIP(hipMemsetAsync(PT.rp, 0, sizeof(int32_t) * (PT.nbr + 1), s));
    TM_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * PT.nbr, s));
    hipLaunchKernelGGL(k_tr_count, dim3(grid_for(P.nnzb)), dim3(WG), 0, s, P.nnzb, P.ci, PT.rp);
    scan_exclusive(PT.rp, PT.rp, PT.nbr, work, s);
    hipLaunchKernelGGL(k_tr_place, dim3(grid_for(P.nnzb)), dim3(WG), 0, s, P.nnzb, prow, P.ci,
                       (const int32_t*)PT.rp, cursor, PT.ci, tsrc);
    hipLaunchKernelGGL(k_tr_sort, dim3(grid_for(PT.nbr)), dim3(WG), 0, s, PT.nbr, (const int32_t*)PT.rp, PT.ci,
                       tsrc);
    hipLaunchKernelGGL(k_tr_values, dim3(grid_for(P.nnzb)), dim3(WG), 0, s, P.nnzb, (const int32_t*)tsrc, P.v64,
                       P.br, P.bc, PT.v64);
}
void sa_prod_numeric(const BSR& X, const BSR& Y, const int32_t* crow, BSR& C, hipStream_t s) {
    hipLaunchKernelGGL(k_prod_numeric, dim3(grid_for(C.nnzb, 64)), dim3(64), 0, s, X.rp, X.ci, X.v64, X.br, X.bc,
                       Y.rp, Y.ci, Y.v64, Y.bc, crow, C.ci, C.nnzb, C.v64);
}
void sa_fix_diag(BSR& A, int bs, hipStream_t s) {
    hipLaunchKernelGGL(k_fix_diag, dim3(grid_for(A.nbr)), dim3(WG), 0, s, A.rp, A.ci, A.nbr, bs, A.v64);
}
void sa_to_f32(const double* a, float* b, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(WG), 0, s, a, b, n);
}

}  // namespace tmi
