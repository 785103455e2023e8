// Outer Krylov loop (Sec. 3.1): conjugate gradients preconditioned by one
// V-cycle, in FP64.  Every scalar (alpha, beta, residual norms, the stop
// decision) stays on the device, so the host can enqueue many iterations
// without reading anything back; every kernel returns at once when its
// right-hand side has stopped.  Reductions: fixed per-block partial sums, then
// one block sums the partials in a fixed order (bitwise reproducible).
//
// Flexible CG (the V-cycle in FP32 is not an exactly fixed linear operator):
//   alpha = p^T r / p^T q,  beta = - z^T q / p^T q   (p_k K-orthogonal to p_{k-1}).
// Standard PCG: alpha = p^T r / p^T q,  beta = z_k^T r_k / z_{k-1}^T r_{k-1}.
#include "tm_device.h"

namespace tmi {

constexpr int KB_MAX = 2048;   // blocks of the grid-stride vector kernels

int krylov_blocks(int64_t n) { return (int)std::min<int64_t>(ceil_div(n > 0 ? n : 1, WG), KB_MAX); }

// ---------------------------------------------------------------- masks, casts
template <typename T>
__global__ void k_mask_copy(const T* src, T* dst, const uint8_t* __restrict__ nm, int bs,
                            int64_t n) {   // src may equal dst
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint8_t m = nm[i / bs];
    dst[i] = (m & (1u << (i % bs))) ? T(0) : src[i];
}

template <typename T>
void launch_mask_copy(const tm_hierarchy* h, const T* src, T* dst, hipStream_t s) {
    const Level& L = h->lv[0];
    hipLaunchKernelGGL(k_mask_copy<T>, dim3(grid_for(L.n)), dim3(WG), 0, s, src, dst, L.nmask, L.bs, L.n);
}
template void launch_mask_copy<double>(const tm_hierarchy*, const double*, double*, hipStream_t);
template void launch_mask_copy<float>(const tm_hierarchy*, const float*, float*, hipStream_t);

__global__ void k_cast(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}
__global__ void k_cast_back(const float* __restrict__ a, double* __restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}
void launch_cast(const double* a, float* b, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_cast, dim3(grid_for(n)), dim3(WG), 0, s, a, b, n);
}
void launch_cast_back(const float* a, double* b, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_cast_back, dim3(grid_for(n)), dim3(WG), 0, s, a, b, n);
}
__global__ void k_fill(uint32_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}
void launch_fill(void* p, int64_t n_bytes, hipStream_t s) {
    const int64_t n = n_bytes / 4;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(WG), 0, s, (uint32_t*)p, n);
}

// ---------------------------------------------------------------- finalisation
// One block of FB threads sums the per-block partials in a fixed order and
// updates the scalars of its right-hand side.
constexpr int FB = 1024;

// NQ sums of nparts partials each (quantity q at part[q * nparts + i]): every
// thread issues eight loads per quantity before adding them (one round trip
// per 8 * FB partials), then a fixed-shape tree over lanes and waves
template <int NQ>
__device__ __forceinline__ void fin_sums(const double* part, int nparts, double (&out)[NQ]) {
    __shared__ double red[NQ][FB / 64];
    double a[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) a[q] = 0.0;
    for (int i0 = 0; i0 < nparts; i0 += 8 * FB) {
        double v[NQ][8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * FB + (int)threadIdx.x;
#pragma unroll
            for (int q = 0; q < NQ; ++q) v[q][u] = i < nparts ? part[(int64_t)q * nparts + i] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            a[q] += ((v[q][0] + v[q][1]) + (v[q][2] + v[q][3])) + ((v[q][4] + v[q][5]) + (v[q][6] + v[q][7]));
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) a[q] += __shfl_down(a[q], o, 64);
        if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = a[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < FB / 64; ++w) t += red[q][w];
        out[q] = t;
    }
    __syncthreads();
}

struct FinA {
    KScal* sc;
    const double* part;
};

template <int NB>
__global__ __launch_bounds__(FB) void k_finalize(const Pack<FinA, NB> pk, int nparts, int what) {
    KScal* sc = lane_of(pk).sc;
    const double* part = lane_of(pk).part;
    if (sc->done) return;
    if (what == FIN_ALPHA) {
        double t[2];
        fin_sums<2>(part, nparts, t);
        const double pq = t[0], pr = t[1];
        if (threadIdx.x == 0) {
            sc->pq = pq;
            sc->pr = pr;
            if (!(pq > 0.0)) {
                sc->status = TM_ERR_BREAKDOWN;
                sc->done = 1;
                sc->alpha = 0.0;
            } else {
                sc->alpha = pr / pq;
            }
        }
    } else if (what == FIN_RR) {
        double t[1];
        fin_sums<1>(part, nparts, t);
        const double rr = t[0];
        if (threadIdx.x == 0) {
            sc->rr = rr;
            sc->rr_last = rr;
            sc->iter += 1;
            if (rr <= sc->rr_stop) {
                sc->done = 1;
                sc->status = TM_OK;
            } else if (!(rr == rr)) {
                sc->done = 1;
                sc->status = TM_ERR_BREAKDOWN;
            } else if (sc->iter >= sc->max_iters) {
                sc->done = 1;
                sc->status = TM_NOT_CONVERGED;
            }
        }
    } else {
        // beta; on the first call (iter == 0, no previous direction) only z^T r is kept
        double t[2];
        fin_sums<2>(part, nparts, t);
        const double zq = t[0], zr = t[1];
        if (threadIdx.x == 0) {
            sc->zq = zq;
            sc->zr = zr;
            if (sc->outer == TM_OUTER_PCG && !(zr > 0.0)) {
                sc->status = TM_ERR_BREAKDOWN;
                sc->done = 1;
                return;
            }
            if (sc->iter == 0)
                sc->beta = 0.0;
            else if (sc->outer == TM_OUTER_PCG)
                sc->beta = zr / sc->zr_old;
            else
                sc->beta = -zq / sc->pq;
            sc->zr_old = zr;
        }
    }
}

void launch_finalize_b(const LaneIO* L, int n, int nparts, int what, hipStream_t s) {
    for (int q0 = 0; q0 < n; q0 += MAXB) {
        const int m = std::min(MAXB, n - q0);
        if (m == 1) {
            Pack<FinA, 1> pk{{{L[q0].sc, L[q0].part}}};
            hipLaunchKernelGGL((k_finalize<1>), dim3(1, 1), dim3(FB), 0, s, pk, nparts, what);
        } else {
            Pack<FinA, MAXB> pk{};
            for (int q = 0; q < m; ++q) pk.a[q] = FinA{L[q0 + q].sc, L[q0 + q].part};
            hipLaunchKernelGGL((k_finalize<MAXB>), dim3(1, m), dim3(FB), 0, s, pk, nparts, what);
        }
    }
}

void launch_finalize(KScal* sc, const double* part, int nparts, int what, hipStream_t s) {
    LaneIO l{};
    l.sc = sc;
    l.part = const_cast<double*>(part);
    launch_finalize_b(&l, 1, nparts, what, s);
}

// init: ||f||^2 and ||r||^2, then the scalars of a fresh solve
__global__ void k_init_dots(const double* __restrict__ f, const double* __restrict__ r, int64_t n,
                            double* part) {
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) {
        v[0] += f[i] * f[i];
        v[1] += r[i] * r[i];
    }
    block_reduce_store<2>(v, part);
}

__global__ __launch_bounds__(FB) void k_init_scalars(KScal* sc, const double* part, int nparts,
                                                    double rtol, int max_iters, int outer) {
    double t[2];
    fin_sums<2>(part, nparts, t);
    const double ff = t[0], rr = t[1];
    if (threadIdx.x == 0) {
        sc->ff = ff;
        sc->rr = rr;
        sc->rr_last = rr;
        sc->rr_stop = rtol * rtol * ff;
        sc->iter = 0;
        sc->max_iters = max_iters;
        sc->outer = outer;
        sc->fin = 0;
        sc->skipfin = 0;
        sc->status = TM_OK;
        sc->done = (rr <= sc->rr_stop) ? 1 : 0;
        if (!(ff - ff == 0.0) || !(rr - rr == 0.0)) {
            // a load or start vector with an infinity or a NaN: nothing to iterate on
            sc->status = TM_ERR_ARG;
            sc->done = 1;
        }
        sc->alpha = sc->beta = 0.0;
        sc->zr_old = 1.0;
    }
}

void launch_fcg_init(const tm_hierarchy* h, Lane& ln, KScal* sc, int use_u0, double* u, double rtol,
                     int max_iters, int outer, hipStream_t s) {
    const int64_t n = h->n_dof;
    if (use_u0) {
        launch_mask_copy<double>(h, u, u, s);
        launch_fine_op<double>(h, OP_RESID, false, u, ln.f, ln.r, 0.0, nullptr, nullptr, s);
    } else {
        TM_HIP(hipMemsetAsync(u, 0, n * sizeof(double), s));
        TM_HIP(hipMemcpyAsync(ln.r, ln.f, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    const int nb = krylov_blocks(n);
    hipLaunchKernelGGL(k_init_dots, dim3(nb), dim3(WG), 0, s, ln.f, ln.r, n, ln.part);
    hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(FB), 0, s, sc, ln.part, nb, rtol, max_iters, outer);
}

// ---------------------------------------------------------------- u, r update
// Node-parallel: u += alpha p, r -= alpha q, ||r||^2; the r copy handed to the
// V-cycle (FP32 in the mixed path) and the V-cycle's first fine-level sweep
// from zero, x0 = omega D^-1 r, are produced in the same pass.
template <typename TV>
struct UrA {
    double* u;
    double* r;
    const double* p;
    const double* q;
    TV* rv;
    TV* x0;
    const TV* dinv;
    const KScal* sc;
    double* part;
};

// (a function of its own so that the lane's pointers keep their no-alias
// qualifiers: the updates of u and r are in place)
template <typename TV, int BS>
__device__ __forceinline__ void update_ur_body(double* __restrict__ u, double* __restrict__ r,
                                               const double* __restrict__ p, const double* __restrict__ q,
                                               TV* __restrict__ rv, TV* __restrict__ x0,
                                               const TV* __restrict__ dinv, TV omega, int64_t N,
                                               const KScal* __restrict__ sc, double* part) {
    if (sc->done) return;
    const double alpha = sc->alpha;
    const int64_t node = xcd_block() * WG + threadIdx.x;
    double v[1] = {0.0};
    if (node < N) {
        TV rl[BS];
#pragma unroll
        for (int c = 0; c < BS; ++c) {
            const int64_t i = BS * node + c;
            u[i] += alpha * p[i];
            const double ri = r[i] - alpha * q[i];
            r[i] = ri;
            rl[c] = (TV)ri;
            if (sizeof(TV) == 4) rv[i] = rl[c];
            v[0] += ri * ri;
        }
#pragma unroll
        for (int a = 0; a < BS; ++a) {
            TV t = 0;
#pragma unroll
            for (int c = 0; c < BS; ++c) t += dinv[(int64_t)sym_at(a, c, BS) * N + node] * rl[c];
            x0[BS * node + a] = omega * t;
        }
    }
    block_reduce_store<1>(v, part);
}

template <typename TV, int BS, int NB>
__global__ __launch_bounds__(WG) void k_update_ur(const Pack<UrA<TV>, NB> pk, TV omega, int64_t N) {
    const UrA<TV>& A_ = lane_of(pk);
    update_ur_body<TV, BS>(A_.u, A_.r, A_.p, A_.q, A_.rv, A_.x0, A_.dinv, omega, N, A_.sc, A_.part);
}

// one block per WG nodes; its partial sums of |r|^2 are finalised with this count
int update_ur_blocks(const tm_hierarchy* h) { return (int)grid_for(h->lv[0].n_nodes); }

template <typename TV, int BS, int NB>
static void update_ur_launch(const LaneIO* L, int n, bool mixed, hipStream_t s) {
    const tm_hierarchy* h = L[0].h;
    Pack<UrA<TV>, NB> pk{};
    for (int q = 0; q < n; ++q) {
        Lane& ln = *L[q].ln;
        const Level& F = L[q].h->lv[0];
        UrA<TV>& a = pk.a[q];
        a.u = L[q].u;
        a.r = ln.r;
        a.p = ln.p;
        a.q = ln.q;
        a.rv = mixed ? (TV*)ln.r32 : nullptr;
        a.x0 = mixed ? (TV*)ln.v32.x[0] : (TV*)ln.v64.x[0];
        a.dinv = mixed ? (const TV*)F.dinv32 : (const TV*)F.dinv64;
        a.sc = L[q].sc;
        a.part = ln.part;
    }
    const TV w = (TV)first_sweep_weight(h, 0);
    hipLaunchKernelGGL((k_update_ur<TV, BS, NB>), dim3(update_ur_blocks(h), n), dim3(WG), 0, s, pk, w,
                       h->lv[0].n_nodes);
}

template <typename TV>
static void update_ur_t(const LaneIO* L, int n, bool mixed, hipStream_t s) {
    const int bs = L[0].h->lv[0].bs;
    for (int q0 = 0; q0 < n; q0 += MAXB) {
        const int m = std::min(MAXB, n - q0);
        if (bs == 3) {
            if (m == 1) update_ur_launch<TV, 3, 1>(L + q0, 1, mixed, s);
            else update_ur_launch<TV, 3, MAXB>(L + q0, m, mixed, s);
        } else {
            if (m == 1) update_ur_launch<TV, 2, 1>(L + q0, 1, mixed, s);
            else update_ur_launch<TV, 2, MAXB>(L + q0, m, mixed, s);
        }
    }
}

void launch_update_ur_b(const LaneIO* L, int n, bool mixed, hipStream_t s) {
    if (n < 1) return;
    if (mixed) update_ur_t<float>(L, n, true, s);
    else update_ur_t<double>(L, n, false, s);
}

void launch_update_ur(const tm_hierarchy* h, Lane& ln, KScal* sc, double* u, bool mixed, hipStream_t s) {
    LaneIO l{};
    l.h = h;
    l.ln = &ln;
    l.sc = sc;
    l.u = u;
    launch_update_ur_b(&l, 1, mixed, s);
}

// ---------------------------------------------------------------- z dots, beta, p
template <typename TZ>
struct ZdA {
    const TZ* z;
    const double* q;
    const double* r;
    const KScal* sc;
    double* part;
};

template <typename TZ, int NB>
__global__ void k_zdots(const Pack<ZdA<TZ>, NB> pk, int64_t n) {
    const ZdA<TZ>& A_ = lane_of(pk);
    const TZ* __restrict__ z = A_.z;
    const double* __restrict__ q = A_.q;
    const double* __restrict__ r = A_.r;
    const KScal* __restrict__ sc = A_.sc;
    double* part = A_.part;
    if (sc->done) return;
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) {
        const double zi = (double)z[i];
        v[0] += zi * q[i];
        v[1] += zi * r[i];
    }
    block_reduce_store<2>(v, part);
}

template <typename TZ, int NB>
static void zdots_launch(const LaneIO* L, int n, hipStream_t s) {
    Pack<ZdA<TZ>, NB> pk{};
    for (int q = 0; q < n; ++q) {
        Lane& ln = *L[q].ln;
        pk.a[q] = ZdA<TZ>{sizeof(TZ) == 4 ? (const TZ*)ln.z32 : (const TZ*)ln.z64, ln.q, ln.r, L[q].sc, ln.part};
    }
    const int64_t nd = L[0].h->n_dof;
    hipLaunchKernelGGL((k_zdots<TZ, NB>), dim3(krylov_blocks(nd), n), dim3(WG), 0, s, pk, nd);
}

void launch_zdots_b(const LaneIO* L, int n, bool mixed, hipStream_t s) {
    for (int q0 = 0; q0 < n; q0 += MAXB) {
        const int m = std::min(MAXB, n - q0);
        if (mixed) {
            if (m == 1) zdots_launch<float, 1>(L + q0, 1, s);
            else zdots_launch<float, MAXB>(L + q0, m, s);
        } else {
            if (m == 1) zdots_launch<double, 1>(L + q0, 1, s);
            else zdots_launch<double, MAXB>(L + q0, m, s);
        }
    }
}

void launch_zdots(const tm_hierarchy* h, Lane& ln, KScal* sc, bool mixed, hipStream_t s) {
    LaneIO l{};
    l.h = h;
    l.ln = &ln;
    l.sc = sc;
    launch_zdots_b(&l, 1, mixed, s);
}

template <typename TZ>
struct UpA {
    double* p;
    const TZ* z;
    const KScal* sc;
};

template <typename TZ, int NB>
__global__ void k_update_p(const Pack<UpA<TZ>, NB> pk, int64_t n) {
    double* __restrict__ p = lane_of(pk).p;
    const TZ* __restrict__ z = lane_of(pk).z;
    const KScal* __restrict__ sc = lane_of(pk).sc;
    if (sc->done) return;
    const double beta = sc->beta;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG)
        p[i] = (double)z[i] + beta * p[i];
}

template <typename TZ, int NB>
static void update_p_launch(const LaneIO* L, int n, hipStream_t s) {
    Pack<UpA<TZ>, NB> pk{};
    for (int q = 0; q < n; ++q) {
        Lane& ln = *L[q].ln;
        pk.a[q] = UpA<TZ>{ln.p, sizeof(TZ) == 4 ? (const TZ*)ln.z32 : (const TZ*)ln.z64, L[q].sc};
    }
    const int64_t nd = L[0].h->n_dof;
    hipLaunchKernelGGL((k_update_p<TZ, NB>), dim3(krylov_blocks(nd), n), dim3(WG), 0, s, pk, nd);
}

void launch_update_p_b(const LaneIO* L, int n, bool mixed, hipStream_t s) {
    for (int q0 = 0; q0 < n; q0 += MAXB) {
        const int m = std::min(MAXB, n - q0);
        if (mixed) {
            if (m == 1) update_p_launch<float, 1>(L + q0, 1, s);
            else update_p_launch<float, MAXB>(L + q0, m, s);
        } else {
            if (m == 1) update_p_launch<double, 1>(L + q0, 1, s);
            else update_p_launch<double, MAXB>(L + q0, m, s);
        }
    }
}

void launch_update_p(const tm_hierarchy* h, Lane& ln, KScal* sc, bool mixed, hipStream_t s) {
    LaneIO l{};
    l.h = h;
    l.ln = &ln;
    l.sc = sc;
    launch_update_p_b(&l, 1, mixed, s);
}

// ---------------------------------------------------------------- outputs
// true residual ||f - K~u||^2 and compliance f^T u (slots pq / zq once the loop
// is over; fin = 1 marks them).  Gated launches (the end of every batch of
// iterations) compute them only for the lanes that stopped in that batch and
// leave the others as empty launches, so that ending a solve needs no more
// device work.  The gate reads done / fin into skipfin; ungated launches clear
// skipfin themselves.
template <int NB>
__global__ void k_final_gate(const Pack<FinA, NB> pk, int gated) {
    KScal* sc = lane_of(pk).sc;
    sc->skipfin = gated ? (sc->done && !sc->fin ? 0 : 1) : 0;
}

struct FdA {
    const double* f;
    const double* t;
    const double* u;
    double* part;
    const int* skip;
};

template <int NB>
__global__ void k_final_dots(const Pack<FdA, NB> pk, int64_t n) {
    const FdA& a = lane_of(pk);
    if (*a.skip) return;
    const double* __restrict__ f = a.f;
    const double* __restrict__ t = a.t;
    const double* __restrict__ u = a.u;
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) {
        v[0] += t[i] * t[i];
        v[1] += f[i] * u[i];
    }
    block_reduce_store<2>(v, a.part);
}

template <int NB>
__global__ __launch_bounds__(FB) void k_final_scalars(const Pack<FinA, NB> pk, int nparts) {
    KScal* sc = lane_of(pk).sc;
    if (sc->skipfin) return;
    double t2[2];
    fin_sums<2>(lane_of(pk).part, nparts, t2);
    const double tt = t2[0], fu = t2[1];
    if (threadIdx.x == 0) {
        sc->pq = tt;
        sc->zq = fu;
        sc->fin = 1;
    }
}

template <int NB>
static void final_launch(const LaneIO* L, int m, bool gated, hipStream_t s) {
    const tm_hierarchy* h = L[0].h;
    const int64_t n = h->n_dof;
    const int nb = krylov_blocks(n);
    Pack<FinA, NB> pf{};
    Pack<FdA, NB> pd{};
    LaneIO io[NB];
    for (int q = 0; q < m; ++q) {
        Lane& ln = *L[q].ln;
        pf.a[q] = FinA{L[q].sc, ln.part};
        pd.a[q] = FdA{ln.f, ln.q, L[q].u, ln.part, &L[q].sc->skipfin};
        io[q] = LaneIO{};
        io[q].h = L[q].h;
        io[q].x = L[q].u;
        io[q].b = ln.f;
        io[q].y = ln.q;
        io[q].done = &L[q].sc->skipfin;
    }
    hipLaunchKernelGGL((k_final_gate<NB>), dim3(1, m), dim3(1), 0, s, pf, gated ? 1 : 0);
    launch_fine_op_b<double>(OP_RESID, false, io, m, 0.0, 0.0, 0.0, s);
    hipLaunchKernelGGL((k_final_dots<NB>), dim3(nb, m), dim3(WG), 0, s, pd, n);
    hipLaunchKernelGGL((k_final_scalars<NB>), dim3(1, m), dim3(FB), 0, s, pf, nb);
}

void launch_final_residual_b(const LaneIO* L, int n, bool gated, hipStream_t s) {
    for (int q0 = 0; q0 < n; q0 += MAXB) {
        const int m = std::min(MAXB, n - q0);
        if (m == 1) final_launch<1>(L + q0, 1, gated, s);
        else final_launch<MAXB>(L + q0, m, gated, s);
    }
}

void launch_final_residual(const tm_hierarchy* h, Lane& ln, KScal* sc, const double* u,
                           hipStream_t s) {
    LaneIO l{};
    l.h = h;
    l.ln = &ln;
    l.sc = sc;
    l.u = const_cast<double*>(u);
    launch_final_residual_b(&l, 1, false, s);
}

// ---------------------------------------------------------------- eigenvalue estimate
// Start vector of the power iteration for D^-1 A: v_i = 1 + (fmix32(i) mod 2^16) / 2^16,
// zero on supported dofs of the fine level.
__global__ void k_power_start(double* __restrict__ v, int64_t n, const uint8_t* __restrict__ nm, int bs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double val = 1.0 + (double)(fmix32((uint32_t)i) & 0xffffu) / 65536.0;
    if (nm && ((nm[i / bs] >> (i % bs)) & 1u)) val = 0.0;
    v[i] = val;
}

void launch_power_start(double* v, int64_t n, const uint8_t* nmask, int bs, hipStream_t s) {
    hipLaunchKernelGGL(k_power_start, dim3(grid_for(n)), dim3(WG), 0, s, v, n, nmask, bs);
}

// z = D^-1 w per block row; block partials of z.z and v.v
template <int BS>
__global__ __launch_bounds__(WG) void k_power_step(const double* __restrict__ w, const double* __restrict__ dinv,
                                                   const double* __restrict__ v, int64_t N, double* __restrict__ z,
                                                   double* part) {
    const int64_t node = (int64_t)blockIdx.x * WG + threadIdx.x;
    double d[2] = {0.0, 0.0};
    if (node < N) {
#pragma unroll
        for (int r = 0; r < BS; ++r) {
            double t = 0.0;
#pragma unroll
            for (int c = 0; c < BS; ++c) t += dinv[(int64_t)sym_at(r, c, BS) * N + node] * w[BS * node + c];
            z[BS * node + r] = t;
            d[0] += t * t;
            const double vr = v[BS * node + r];
            d[1] += vr * vr;
        }
    }
    block_reduce_store<2>(d, part);
}

void launch_power_step(const Level& L, const double* w, const double* v, double* z, double* part, hipStream_t s) {
    const dim3 g(grid_for(L.n_nodes)), b(WG);
    switch (L.bs) {
        case 2: hipLaunchKernelGGL(k_power_step<2>, g, b, 0, s, w, L.dinv64, v, L.n_nodes, z, part); break;
        case 3: hipLaunchKernelGGL(k_power_step<3>, g, b, 0, s, w, L.dinv64, v, L.n_nodes, z, part); break;
        case 6: hipLaunchKernelGGL(k_power_step<6>, g, b, 0, s, w, L.dinv64, v, L.n_nodes, z, part); break;
        default: fail(TM_ERR_ARG, "block size must be 2, 3 or 6");
    }
}

// theta = factor * sqrt(z.z / v.v) from the last power step's partials: the
// estimate of the largest eigenvalue of D^-1 A times (lower + upper) / 2
// (and, when ninv is given, 1 / ||z|| for keeping the last vector at unit length)
__global__ __launch_bounds__(FB) void k_cheb_theta(const double* part, int nparts, double factor,
                                                   double* theta, double* ninv) {
    double t[2];
    fin_sums<2>(part, nparts, t);
    if (threadIdx.x == 0) {
        *theta = factor * sqrt(t[0] / t[1]);
        if (ninv) *ninv = t[0] > 0.0 ? 1.0 / sqrt(t[0]) : 0.0;
    }
}

void launch_cheb_theta(const double* part, int nparts, double factor, double* theta, double* ninv, hipStream_t s) {
    hipLaunchKernelGGL(k_cheb_theta, dim3(1), dim3(FB), 0, s, part, nparts, factor, theta, ninv);
}

// dst = src * (*scale)
__global__ void k_scale_copy(const double* __restrict__ src, double* __restrict__ dst, int64_t n,
                             const double* __restrict__ scale) {
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i < n) dst[i] = src[i] * *scale;
}

void launch_scale_copy(const double* src, double* dst, int64_t n, const double* scale, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(WG), 0, s, src, dst, n, scale);
}

// D^-1 <- D^-1 / theta (FP64), and its FP32 copy from the result
__global__ void k_scale_dinv(double* __restrict__ d64, float* __restrict__ d32, int64_t n,
                             const double* __restrict__ theta) {
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= n) return;
    const double v = d64[i] / *theta;
    d64[i] = v;
    d32[i] = (float)v;
}

void launch_scale_dinv(Level& L, const double* theta, hipStream_t s) {
    const int64_t n = (int64_t)sym_n(L.bs) * L.n_nodes;
    hipLaunchKernelGGL(k_scale_dinv, dim3(grid_for(n)), dim3(WG), 0, s, L.dinv64, L.dinv32, n, theta);
}

}  // namespace tmi
