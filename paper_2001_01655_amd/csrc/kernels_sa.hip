// Setup of the smoothed-aggregation levels of the hybrid hierarchy (Sec. 3.2
// algebraic multigrid; Sec. 4 block strength of connection with beta, the
// tentative prolongator smoothed by one weighted-Jacobi step, rigid-body
// modes as candidates).  Every result is independent of thread scheduling:
// integer decisions are order-free (min / max / set), and every floating-point
// sum runs over its terms in ascending index order.  Rows, aggregates and
// product blocks with long loops take one wave each (64-thread workgroups):
// the lanes compute the terms side by side, and the sums still run in
// ascending order (one lane per output entry, or every lane redundantly).
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

// one wave per row: lane l tests entry q0 + l; the strong entries keep their
// order (ballot prefix counts)
template <bool FILL>
__global__ __launch_bounds__(64) void k_strength(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                 const double* __restrict__ v, const double* __restrict__ dn,
                                                 int64_t n, int bs, double beta2, int32_t* __restrict__ cnt,
                                                 const int32_t* __restrict__ srp, int32_t* __restrict__ sci) {
    const int64_t I = blockIdx.x;
    const int lane = threadIdx.x;
    if (I >= n) return;
    const int32_t q0 = rp[I], q1 = rp[I + 1];
    int32_t c = 0;
    for (int32_t qb = q0; qb < q1; qb += 64) {
        const int32_t q = qb + lane;
        const bool st = q < q1 && ci[q] != (int32_t)I && strong_pair(rp, ci, v, dn, bs, beta2, I, q);
        const uint64_t m = __ballot(st);
        if (FILL && st) sci[srp[I] + c + __popcll(m & ((1ull << lane) - 1ull))] = ci[q];
        c += __popcll(m);
    }
    if (!FILL && lane == 0) cnt[I] = c;
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
// segment [off[g], off[g+1]) of `in` (distinct keys) into `out` in ascending
// order, one wave per segment: each key goes to its rank (the number of
// smaller keys in the segment); optional payload moves with its key
__global__ __launch_bounds__(64) void k_rank_segments(int64_t ng, const int32_t* __restrict__ off,
                                                      const int32_t* __restrict__ in,
                                                      const int32_t* __restrict__ pin, int32_t* __restrict__ out,
                                                      int32_t* __restrict__ pout) {
    const int64_t g = blockIdx.x;
    if (g >= ng) return;
    const int32_t p0 = off[g], p1 = off[g + 1];
    for (int32_t p = p0 + (int32_t)threadIdx.x; p < p1; p += 64) {
        const int32_t key = in[p];
        int32_t rank = 0;
        for (int32_t q = p0; q < p1; ++q) rank += in[q] < key;
        out[p0 + rank] = key;
        if (pin) pout[p0 + rank] = pin[p];
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

// one wave per aggregate: modified Gram-Schmidt on its member rows.  The rows
// (members ascending, then the block's rows) sit in LDS when they fit, else
// they are worked on in T itself; element-wise steps run across the lanes,
// every norm and dot product is summed over the rows in ascending order (by
// every lane alike, so all lanes hold the same value).
constexpr int TENT_LDS = 4096;    // doubles: rows x k of one aggregate

template <bool SH>
__device__ __forceinline__ void mgs_rows(double* __restrict__ W, const int32_t* __restrict__ mem, int32_t p0,
                                         int nrow, int bs, int k, double (&R)[6][6]) {
    // row t of the aggregate: member p0 + t / bs, block row t % bs
    auto at = [&](int t, int c) -> double& {
        if (SH) return W[t * k + c];
        return W[((int64_t)mem[p0 + t / bs] * bs + t % bs) * k + c];
    };
    for (int j = 0; j < k; ++j) {
        double n0 = 0.0;
        for (int t = 0; t < nrow; ++t) {
            const double v = at(t, j);
            n0 += v * v;
        }
        n0 = sqrt(n0);
        for (int i = 0; i < j; ++i) {
            double d = 0.0;
            for (int t = 0; t < nrow; ++t) d += at(t, i) * at(t, j);
            R[i][j] = d;
            __syncthreads();
            for (int t = (int)threadIdx.x; t < nrow; t += 64) at(t, j) -= d * at(t, i);
            __syncthreads();
        }
        double nr = 0.0;
        for (int t = 0; t < nrow; ++t) {
            const double v = at(t, j);
            nr += v * v;
        }
        nr = sqrt(nr);
        const bool dead = n0 == 0.0 || nr <= 1e-10 * n0;
        R[j][j] = dead ? 0.0 : nr;
        __syncthreads();
        for (int t = (int)threadIdx.x; t < nrow; t += 64) {
            double& x = at(t, j);
            x = dead ? 0.0 : x / nr;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void k_tentative(int64_t ng, const int32_t* __restrict__ off,
                                                  const int32_t* __restrict__ mem, const double* __restrict__ Bprev,
                                                  int dim, int nx1, int ny1, const LevelPos lp, int bs, int k,
                                                  double* __restrict__ T, double* __restrict__ Bc, int use_lds) {
    __shared__ double W[TENT_LDS];
    const int64_t g = blockIdx.x;
    if (g >= ng) return;
    const int32_t p0 = off[g], p1 = off[g + 1];
    const int nrow = (p1 - p0) * bs;
    const bool sh = use_lds && nrow * k <= TENT_LDS;
    for (int t = (int)threadIdx.x; t < nrow; t += 64) {
        const int64_t i = mem[p0 + t / bs];
        const int r = t % bs;
        for (int c = 0; c < k; ++c) {
            const double v = cand(Bprev, dim, nx1, ny1, lp, bs, k, i, r, c);
            if (sh) W[t * k + c] = v;
            else T[((int64_t)i * bs + r) * k + c] = v;
        }
    }
    __syncthreads();
    double R[6][6];
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) R[a][b] = 0.0;
    if (sh)
        mgs_rows<true>(W, mem, p0, nrow, bs, k, R);
    else
        mgs_rows<false>(T, mem, p0, nrow, bs, k, R);
    if (sh)
        for (int t = (int)threadIdx.x; t < nrow; t += 64) {
            const int64_t i = mem[p0 + t / bs];
            const int r = t % bs;
            for (int c = 0; c < k; ++c) T[((int64_t)i * bs + r) * k + c] = W[t * k + c];
        }
    if (threadIdx.x == 0)
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) Bc[((int64_t)g * k + a) * k + b] = R[a][b];
}

// ------------------------------------------------------------------ ||D^-1 A||_inf
// one wave per row: lane l forms |(D^-1 A)_{rc}| for block q0 + l, then lane r
// adds its row's terms block by block, column by column (ascending order)
__global__ __launch_bounds__(64) void k_dinv_a_rowmax(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                      const double* __restrict__ v, const double* __restrict__ dinv,
                                                      int64_t n, int bs, unsigned long long* __restrict__ out) {
    __shared__ double u[64][36];
    const int64_t I = blockIdx.x;
    if (I >= n) return;
    const int lane = threadIdx.x;
    const int32_t q0 = rp[I], q1 = rp[I + 1];
    double s = 0.0;
    for (int32_t qb = q0; qb < q1; qb += 64) {
        const int32_t q = qb + lane;
        if (q < q1)
            for (int r = 0; r < bs; ++r)
                for (int c = 0; c < bs; ++c) {
                    double t = 0.0;
                    for (int m = 0; m < bs; ++m)
                        t += dinv[(int64_t)sym_at(r, m, bs) * n + I] * v[((int64_t)q * bs + m) * bs + c];
                    u[lane][r * bs + c] = fabs(t);
                }
        __syncthreads();
        if (lane < bs) {
            const int cnt = min(64, q1 - qb);
            for (int l = 0; l < cnt; ++l)
                for (int c = 0; c < bs; ++c) s += u[l][lane * bs + c];
        }
        __syncthreads();
    }
    // the largest row sum of this block row
    double best = lane < bs ? s : 0.0;
    for (int o = 32; o > 0; o >>= 1) best = fmax(best, __shfl_xor(best, o));
    if (lane == 0)
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

// t = X Y for an XR x XC block X and an XC x YC block Y (row-major), each
// entry summed over m in ascending order
template <int XR, int XC, int YC>
__device__ __forceinline__ void block_mul(const double* __restrict__ X, const double* __restrict__ Y,
                                          double (&t)[XR * YC]) {
    double x[XR * XC], y[XC * YC];
#pragma unroll
    for (int e = 0; e < XR * XC; ++e) x[e] = X[e];
#pragma unroll
    for (int e = 0; e < XC * YC; ++e) y[e] = Y[e];
#pragma unroll
    for (int r = 0; r < XR; ++r)
#pragma unroll
        for (int c = 0; c < YC; ++c) {
            double a = 0.0;
#pragma unroll
            for (int m = 0; m < XC; ++m) a += x[r * XC + m] * y[m * YC + c];
            t[r * YC + c] = a;
        }
}

// numeric P: block (I, g) = [g == agg[I]] T_I - omega Dinv_I sum_{J in row I, agg[J] = g} A_IJ T_J
// One wave per row I: lane l forms A_IJ T_J for entry q0 + l of A's row, lane
// (block, r, c) adds the terms of its aggregate in ascending entry order and
// then finishes its entry.  BS x BS blocks of A, BS x K of T.
constexpr int PN_SLOTS = 64;     // blocks of one P row held in LDS

template <int BS, int K>
__global__ __launch_bounds__(64) void k_p_numeric(const int32_t* __restrict__ arp, const int32_t* __restrict__ aci,
                                                  const double* __restrict__ av, const int32_t* __restrict__ agg,
                                                  const double* __restrict__ T, const double* __restrict__ dinv,
                                                  int64_t n, double omega, const int32_t* __restrict__ prp,
                                                  const int32_t* __restrict__ pci, double* __restrict__ pv, int slots) {
    constexpr int NE = BS * K;
    __shared__ double u[64][NE];
    __shared__ int32_t gq[64];
    __shared__ double sums[PN_SLOTS][NE];
    const int64_t I = blockIdx.x;
    if (I >= n) return;
    const int lane = threadIdx.x;
    const int32_t b0 = prp[I], nb = prp[I + 1] - b0;
    const int32_t q0 = arp[I], q1 = arp[I + 1];
    const double* TI = T + I * NE;
    const int32_t gI = agg[I];
    // blocks of the row in groups of PN_SLOTS (a row has a handful)
    for (int32_t s0 = 0; s0 < nb; s0 += slots) {
        const int ns = min(slots, nb - s0);
        for (int t = lane; t < ns * NE; t += 64) sums[t / NE][t % NE] = 0.0;
        for (int32_t qb = q0; qb < q1; qb += 64) {
            const int32_t q = qb + lane;
            if (q < q1) {
                const int32_t J = aci[q];
                gq[lane] = agg[J];
                double t[NE];
                block_mul<BS, BS, K>(av + (int64_t)q * BS * BS, T + (int64_t)J * NE, t);
#pragma unroll
                for (int e = 0; e < NE; ++e) u[lane][e] = t[e];
            }
            __syncthreads();
            const int cnt = min(64, q1 - qb);
            for (int t = lane; t < ns * NE; t += 64) {
                const int sl = t / NE, e = t % NE;
                const int32_t g = pci[b0 + s0 + sl];
                double a = sums[sl][e];
                for (int l = 0; l < cnt; ++l)
                    if (gq[l] == g) a += u[l][e];
                sums[sl][e] = a;
            }
            __syncthreads();
        }
        for (int t = lane; t < ns * NE; t += 64) {
            const int sl = t / NE, e = t % NE, r = e / K, c = e % K;
            const int32_t g = pci[b0 + s0 + sl];
            double a = 0.0;
#pragma unroll
            for (int mm = 0; mm < BS; ++mm) a += dinv[(int64_t)sym_at(r, mm, BS) * n + I] * sums[sl][mm * K + c];
            pv[(int64_t)(b0 + s0 + sl) * NE + e] = (g == gI ? TI[e] : 0.0) - omega * a;
        }
        __syncthreads();
    }
}

// transpose of a BSR (br x bc blocks): counts, then placement, then each row
// in ascending column order (rank of each key)
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
// X blocks are XR x XC, Y blocks XC x YC (compile-time shapes, so a lane holds
// its two blocks in registers).  One output row per wave (row-by-row
// product): the row's sums sit in LDS (stride NE + 1 against bank
// conflicts); the entries q of X's row are taken in ascending order, and for
// each the lanes take the blocks p of Y's row ci_x[q] (distinct columns, so
// distinct sums): every block adds its terms in ascending q.  A row longer
// than the LDS the launch sized is done block by block, with the same order.
template <int XR, int XC, int YC>
__global__ __launch_bounds__(64) void k_prod_rows(const int32_t* __restrict__ xrp, const int32_t* __restrict__ xci,
                                                  const double* __restrict__ xv, const int32_t* __restrict__ yrp,
                                                  const int32_t* __restrict__ yci, const double* __restrict__ yv,
                                                  const int32_t* __restrict__ crp, const int32_t* __restrict__ cci,
                                                  int64_t nrows, int mcap, double* __restrict__ cv) {
    constexpr int NE = XR * YC, NS = NE + 1;
    extern __shared__ double lds[];
    const int64_t R = blockIdx.x;
    if (R >= nrows) return;
    const int lane = threadIdx.x;
    const int32_t c0 = crp[R], c1 = crp[R + 1];
    const int m = c1 - c0;
    const int32_t q0 = xrp[R], q1 = xrp[R + 1];
    if (m > mcap) {
        // block by block: lane l forms the term of entry q0 + l, lane e adds
        double* u = lds;                                   // [64][NE]
        int* hit = reinterpret_cast<int*>(lds + 64 * NE);  // [64]
        for (int32_t b = c0; b < c1; ++b) {
            const int32_t H = cci[b];
            double acc = 0.0;
            for (int32_t qb = q0; qb < q1; qb += 64) {
                const int32_t q = qb + lane;
                bool h = false;
                if (q < q1) {
                    const int32_t J = xci[q];
                    const int32_t p = find_col(yci, yrp[J], yrp[J + 1], H);
                    h = p < yrp[J + 1] && yci[p] == H;
                    if (h) {
                        double t[NE];
                        block_mul<XR, XC, YC>(xv + (int64_t)q * XR * XC, yv + (int64_t)p * XC * YC, t);
#pragma unroll
                        for (int e = 0; e < NE; ++e) u[lane * NE + e] = t[e];
                    }
                }
                hit[lane] = h;
                __syncthreads();
                if (lane < NE) {
                    const int cnt = min(64, q1 - qb);
                    for (int l = 0; l < cnt; ++l)
                        if (hit[l]) acc += u[l * NE + lane];
                }
                __syncthreads();
            }
            if (lane < NE) cv[(int64_t)b * NE + lane] = acc;
        }
        return;
    }
    double* acc = lds;                                         // [m][NS]
    int32_t* cols = reinterpret_cast<int32_t*>(lds + (size_t)mcap * NS);
    for (int t = lane; t < m * NS; t += 64) acc[t] = 0.0;
    for (int t = lane; t < m; t += 64) cols[t] = cci[c0 + t];
    __syncthreads();
    for (int32_t qb = q0; qb < q1; qb += 64) {
        int32_t pa = 0, pb = 0;
        if (qb + lane < q1) {
            const int32_t J = xci[qb + lane];
            pa = yrp[J];
            pb = yrp[J + 1];
        }
        const int cnt = min(64, q1 - qb);
        for (int l = 0; l < cnt; ++l) {
            const int32_t a0 = __shfl(pa, l), a1 = __shfl(pb, l);
            const double* X = xv + (int64_t)(qb + l) * XR * XC;
            for (int32_t p = a0 + lane; p < a1; p += 64) {
                const int32_t H = yci[p];
                double t[NE];
                block_mul<XR, XC, YC>(X, yv + (int64_t)p * XC * YC, t);
                const int sl = find_col(cols, 0, m, H);
                if (sl < m && cols[sl] == H) {
#pragma unroll
                    for (int e = 0; e < NE; ++e) acc[sl * NS + e] += t[e];
                }
            }
            __syncthreads();
        }
    }
    for (int t = lane; t < m * NE; t += 64) cv[(int64_t)c0 * NE + t] = acc[(t / NE) * NS + t % NE];
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
        hipLaunchKernelGGL(k_strength<true>, dim3((unsigned)A.nbr), dim3(64), 0, s, A.rp, A.ci, A.v64, dn,
                           A.nbr, bs, b2, cnt, srp, sci);
    else
        hipLaunchKernelGGL(k_strength<false>, dim3((unsigned)A.nbr), dim3(64), 0, s, A.rp, A.ci, A.v64, dn,
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
                int32_t* umem, int64_t* work, hipStream_t s) {
    TM_HIP(hipMemsetAsync(cnt_off, 0, sizeof(int32_t) * (ng + 1), s));
    TM_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * ng, s));
    hipLaunchKernelGGL(k_count_members, dim3(grid_for(n)), dim3(WG), 0, s, n, agg, cnt_off);
    scan_exclusive(cnt_off, cnt_off, ng, work, s);
    hipLaunchKernelGGL(k_place_members, dim3(grid_for(n)), dim3(WG), 0, s, n, agg, (const int32_t*)cnt_off,
                       cursor, umem);
    hipLaunchKernelGGL(k_rank_segments, dim3((unsigned)ng), dim3(64), 0, s, ng, (const int32_t*)cnt_off,
                       (const int32_t*)umem, (const int32_t*)nullptr, mem, (int32_t*)nullptr);
}
void sa_tentative(int64_t ng, const int32_t* off, const int32_t* mem, const double* Bprev, int dim, int nx1,
                  int ny1, double h, int level, const int* nel0, int bs, int k, double* T, double* Bc, bool use_lds,
                  hipStream_t s) {
    LevelPos lp{h, 1 << level, {nel0[0], nel0[1], dim == 3 ? nel0[2] : 0}};
    hipLaunchKernelGGL(k_tentative, dim3((unsigned)ng), dim3(64), 0, s, ng, off, mem, Bprev, dim, nx1, ny1,
                       lp, bs, k, T, Bc, (int)use_lds);
}
double sa_jacobi_bound(const BSR& A, int bs, const double* dinv, unsigned long long* work, hipStream_t s) {
    TM_HIP(hipMemsetAsync(work, 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_dinv_a_rowmax, dim3((unsigned)A.nbr), dim3(64), 0, s, A.rp, A.ci, A.v64, dinv, A.nbr,
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
                  double omega, const int32_t* prow, const BSR& P, bool use_lds, hipStream_t s) {
    (void)prow;
    const dim3 g((unsigned)A.nbr), b(64);
#define TM_PN(BS, K)                                                                                     \
    hipLaunchKernelGGL((k_p_numeric<BS, K>), g, b, 0, s, A.rp, A.ci, A.v64, agg, T, dinv, (int64_t)A.nbr, omega, \
                       P.rp, P.ci, P.v64, use_lds ? PN_SLOTS : 1)
    if (bs == 3 && k == 6) TM_PN(3, 6);
    else if (bs == 6 && k == 6) TM_PN(6, 6);
    else if (bs == 2 && k == 3) TM_PN(2, 3);
    else if (bs == 3 && k == 3) TM_PN(3, 3);
    else fail(TM_ERR_ARG, "aggregation block shape not supported");
#undef TM_PN
}
void sa_transpose(const BSR& P, const int32_t* prow, BSR& PT, int32_t* cursor, int32_t* tsrc, int32_t* uci,
                  int32_t* usrc, int64_t* work, hipStream_t s) {
    TM_HIP(hipMemsetAsync(PT.rp, 0, sizeof(int32_t) * (PT.nbr + 1), s));
    TM_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * PT.nbr, s));
    hipLaunchKernelGGL(k_tr_count, dim3(grid_for(P.nnzb)), dim3(WG), 0, s, P.nnzb, P.ci, PT.rp);
    scan_exclusive(PT.rp, PT.rp, PT.nbr, work, s);
    hipLaunchKernelGGL(k_tr_place, dim3(grid_for(P.nnzb)), dim3(WG), 0, s, P.nnzb, prow, P.ci,
                       (const int32_t*)PT.rp, cursor, uci, usrc);
    hipLaunchKernelGGL(k_rank_segments, dim3((unsigned)PT.nbr), dim3(64), 0, s, (int64_t)PT.nbr,
                       (const int32_t*)PT.rp, (const int32_t*)uci, (const int32_t*)usrc, PT.ci, tsrc);
    hipLaunchKernelGGL(k_tr_values, dim3(grid_for(P.nnzb)), dim3(WG), 0, s, P.nnzb, (const int32_t*)tsrc, P.v64,
                       P.br, P.bc, PT.v64);
}
__global__ void k_max_row(const int32_t* __restrict__ rp, int64_t n, int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicMax(out, rp[i + 1] - rp[i]);
}

// LDS of the row form: the longest output row's sums (+ its columns), at most
// 48 KB; longer rows take the block form
template <int XR, int XC, int YC>
static void prod_launch(const BSR& X, const BSR& Y, BSR& C, int32_t mmax, bool use_lds, hipStream_t s) {
    constexpr int NE = XR * YC, NS = NE + 1;
    constexpr size_t CAP = 48 * 1024;
    const size_t block_form = (size_t)64 * NE * sizeof(double) + 64 * sizeof(int);
    int mcap = use_lds ? (int)std::min<int64_t>(mmax, (int64_t)(CAP / (NS * sizeof(double) + sizeof(int32_t)))) : 0;
    size_t lds = (size_t)mcap * (NS * sizeof(double) + sizeof(int32_t));
    lds = std::max(lds, block_form);
    hipLaunchKernelGGL((k_prod_rows<XR, XC, YC>), dim3((unsigned)C.nbr), dim3(64), lds, s, X.rp, X.ci, X.v64, Y.rp,
                       Y.ci, Y.v64, C.rp, C.ci, (int64_t)C.nbr, mcap, C.v64);
}

void sa_prod_numeric(const BSR& X, const BSR& Y, const int32_t* crow, BSR& C, int32_t* dtmp, bool use_lds,
                     hipStream_t s) {
    (void)crow;
    if (C.nbr < 1) return;
    TM_HIP(hipMemsetAsync(dtmp, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(k_max_row, dim3(grid_for(C.nbr)), dim3(WG), 0, s, C.rp, (int64_t)C.nbr, dtmp);
    int32_t mmax = 0;
    TM_HIP(hipMemcpyAsync(&mmax, dtmp, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TM_HIP(hipStreamSynchronize(s));
    const int xr = X.br, xc = X.bc, yc = Y.bc;
    if (Y.br != xc) fail(TM_ERR_ARG, "block shapes of a product do not match");
    if (xr == 3 && xc == 3 && yc == 6) prod_launch<3, 3, 6>(X, Y, C, mmax, use_lds, s);
    else if (xr == 6 && xc == 3 && yc == 6) prod_launch<6, 3, 6>(X, Y, C, mmax, use_lds, s);
    else if (xr == 6 && xc == 6 && yc == 6) prod_launch<6, 6, 6>(X, Y, C, mmax, use_lds, s);
    else if (xr == 2 && xc == 2 && yc == 3) prod_launch<2, 2, 3>(X, Y, C, mmax, use_lds, s);
    else if (xr == 3 && xc == 2 && yc == 3) prod_launch<3, 2, 3>(X, Y, C, mmax, use_lds, s);
    else if (xr == 3 && xc == 3 && yc == 3) prod_launch<3, 3, 3>(X, Y, C, mmax, use_lds, s);
    else fail(TM_ERR_ARG, "aggregation block shape not supported");
}
void sa_fix_diag(BSR& A, int bs, hipStream_t s) {
    hipLaunchKernelGGL(k_fix_diag, dim3(grid_for(A.nbr)), dim3(WG), 0, s, A.rp, A.ci, A.nbr, bs, A.v64);
}
void sa_to_f32(const double* a, float* b, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(WG), 0, s, a, b, n);
}

}  // namespace tmi
