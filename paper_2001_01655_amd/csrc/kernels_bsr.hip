// Operators of smoothed-aggregation levels, stored as block sparse rows
// (one bs x bs block per pair of aggregates; int32 block columns), and the
// explicit prolongator P / restriction P^T of the aggregation steps.  Rows of
// aggregation operators and of P^T are long (tens to hundreds of blocks), so
// one wave works on one block row; P rows are short and get one thread each.
// The row owner writes all bs outputs, so the smoother applies the block
// inverse of the point-block Jacobi step directly.
#include "tm_device.h"

namespace tmi {

// One 64-lane wave per block row: lanes split the row's blocks, then a fixed
// shuffle tree sums the bs partial outputs (deterministic), lane 0 finishes.
template <typename T, int BS, int OP>
__global__ __launch_bounds__(WG) void k_bsr_op_wave(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                    const T* __restrict__ v, int64_t nbr, const T* __restrict__ x,
                                                    const T* __restrict__ b, T* __restrict__ y,
                                                    const T* __restrict__ dinv, T omega,
                                                    const int* __restrict__ done, const ChebArgs ch) {
    if (done && *done) return;
    const int64_t row = xcd_block() * (WG / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nbr) return;
    T acc[BS] = {};
    for (int32_t q = rp[row] + lane; q < rp[row + 1]; q += 64) {
        const int64_t c0 = (int64_t)ci[q] * BS;
        T xv[BS];
#pragma unroll
        for (int c = 0; c < BS; ++c) xv[c] = x[c0 + c];
        const T* blk = v + (int64_t)q * BS * BS;
#pragma unroll
        for (int r = 0; r < BS; ++r)
#pragma unroll
            for (int c = 0; c < BS; ++c) acc[r] += blk[r * BS + c] * xv[c];
    }
#pragma unroll
    for (int r = 0; r < BS; ++r)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc[r] += __shfl_down(acc[r], o, 64);
    if (lane != 0) return;
    T xo[BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) xo[c] = x[(int64_t)BS * row + c];
    double dots[2];
    finish_node<T, BS, OP>(row, nbr, acc, xo, 0, b, y, dinv, omega, dots, ch);
}

template <typename T>
static const T* vals_of(const BSR& B);
template <>
const double* vals_of<double>(const BSR& B) { return B.v64; }
template <>
const float* vals_of<float>(const BSR& B) { return B.v32; }
template <typename T>
static const T* dinv_of(const Level& L);
template <>
const double* dinv_of<double>(const Level& L) { return L.dinv64; }
template <>
const float* dinv_of<float>(const Level& L) { return L.dinv32; }

template <typename T, int BS>
static void bsr_op_bs(const Level& L, int op, const T* x, const T* b, T* y, T omega, const int* done,
                      hipStream_t s, const ChebArgs& ch) {
    const dim3 g(grid_for(L.A.nbr, WG / 64)), blk(WG);
    const T* v = vals_of<T>(L.A);
    const T* dv = dinv_of<T>(L);
#define TM_BO(OPV)                                                                                    \
    hipLaunchKernelGGL((k_bsr_op_wave<T, BS, OPV>), g, blk, 0, s, L.A.rp, L.A.ci, v, L.A.nbr, x, b, y, dv, omega, \
                       done, ch)
    switch (op) {
        case OP_APPLY: TM_BO(OP_APPLY); break;
        case OP_RESID: TM_BO(OP_RESID); break;
        case OP_CHEB: TM_BO(OP_CHEB); break;
        default: TM_BO(OP_SMOOTH); break;
    }
#undef TM_BO
}

template <typename T>
void launch_bsr_op(const Level& L, int op, const T* x, const T* b, T* y, T omega, const int* done,
                   hipStream_t s, const ChebArgs& ch) {
    switch (L.bs) {
        case 3: bsr_op_bs<T, 3>(L, op, x, b, y, omega, done, s, ch); break;
        case 6: bsr_op_bs<T, 6>(L, op, x, b, y, omega, done, s, ch); break;
        default: fail(TM_ERR_ARG, "aggregation level block size must be 3 or 6");
    }
}
template void launch_bsr_op<double>(const Level&, int, const double*, const double*, double*, double,
                                    const int*, hipStream_t, const ChebArgs&);
template void launch_bsr_op<float>(const Level&, int, const float*, const float*, float*, float,
                                   const int*, hipStream_t, const ChebArgs&);

// y (+)= B x for a rectangular BSR with BR x BC blocks; optionally x_first = omega D^-1 y
template <typename T, int BR, int BC, bool ADD, bool FIRST>
__global__ __launch_bounds__(WG) void k_bsr_mv(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                               const T* __restrict__ v, int64_t nbr, const T* __restrict__ x,
                                               T* __restrict__ y, T* __restrict__ xf,
                                               const T* __restrict__ dinv, T omega,
                                               const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t row = xcd_block() * WG + threadIdx.x;
    if (row >= nbr) return;
    T acc[BR] = {};
    for (int32_t q = rp[row]; q < rp[row + 1]; ++q) {
        const int64_t c0 = (int64_t)ci[q] * BC;
        const T* blk = v + (int64_t)q * BR * BC;
#pragma unroll
        for (int c = 0; c < BC; ++c) {
            const T xv = x[c0 + c];
#pragma unroll
            for (int r = 0; r < BR; ++r) acc[r] += blk[r * BC + c] * xv;
        }
    }
#pragma unroll
    for (int r = 0; r < BR; ++r) {
        if (ADD)
            y[(int64_t)BR * row + r] += acc[r];
        else
            y[(int64_t)BR * row + r] = acc[r];
    }
    if (FIRST) {
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            T t = 0;
#pragma unroll
            for (int c = 0; c < BR; ++c) t += dinv[(int64_t)sym_at(r, c, BR) * nbr + row] * acc[c];
            xf[(int64_t)BR * row + r] = omega * t;
        }
    }
}

template <typename T, int BR, int BC, bool ADD, bool FIRST>
__global__ __launch_bounds__(WG) void k_bsr_mv_wave(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                    const T* __restrict__ v, int64_t nbr, const T* __restrict__ x,
                                                    T* __restrict__ y, T* __restrict__ xf,
                                                    const T* __restrict__ dinv, T omega,
                                                    const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t row = xcd_block() * (WG / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nbr) return;
    T acc[BR] = {};
    for (int32_t q = rp[row] + lane; q < rp[row + 1]; q += 64) {
        const int64_t c0 = (int64_t)ci[q] * BC;
        const T* blk = v + (int64_t)q * BR * BC;
#pragma unroll
        for (int c = 0; c < BC; ++c) {
            const T xv = x[c0 + c];
#pragma unroll
            for (int r = 0; r < BR; ++r) acc[r] += blk[r * BC + c] * xv;
        }
    }
#pragma unroll
    for (int r = 0; r < BR; ++r)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc[r] += __shfl_down(acc[r], o, 64);
    if (lane != 0) return;
#pragma unroll
    for (int r = 0; r < BR; ++r) {
        if (ADD)
            y[(int64_t)BR * row + r] += acc[r];
        else
            y[(int64_t)BR * row + r] = acc[r];
    }
    if (FIRST) {
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            T t = 0;
#pragma unroll
            for (int c = 0; c < BR; ++c) t += dinv[(int64_t)sym_at(r, c, BR) * nbr + row] * acc[c];
            xf[(int64_t)BR * row + r] = omega * t;
        }
    }
}

template <typename T, int BR, int BC>
static void bsr_mv_shape(const BSR& B, const T* x, T* y, bool add, T* xfirst, const T* dinv, T omega,
                         const int* done, hipStream_t s) {
    const dim3 g(grid_for(B.nbr)), blk(WG);
    const T* v = vals_of<T>(B);
    if (B.nnzb >= 8 * B.nbr) {      // long rows (restriction, smoothed prolongators): one wave per row
        const dim3 gw(grid_for(B.nbr, WG / 64));
        if (add)
            hipLaunchKernelGGL((k_bsr_mv_wave<T, BR, BC, true, false>), gw, blk, 0, s, B.rp, B.ci, v, B.nbr, x, y,
                               xfirst, dinv, omega, done);
        else if (xfirst)
            hipLaunchKernelGGL((k_bsr_mv_wave<T, BR, BC, false, true>), gw, blk, 0, s, B.rp, B.ci, v, B.nbr, x, y,
                               xfirst, dinv, omega, done);
        else
            hipLaunchKernelGGL((k_bsr_mv_wave<T, BR, BC, false, false>), gw, blk, 0, s, B.rp, B.ci, v, B.nbr, x, y,
                               xfirst, dinv, omega, done);
        return;
    }
    if (add)
        hipLaunchKernelGGL((k_bsr_mv<T, BR, BC, true, false>), g, blk, 0, s, B.rp, B.ci, v, B.nbr, x, y,
                           xfirst, dinv, omega, done);
    else if (xfirst)
        hipLaunchKernelGGL((k_bsr_mv<T, BR, BC, false, true>), g, blk, 0, s, B.rp, B.ci, v, B.nbr, x, y,
                           xfirst, dinv, omega, done);
    else
        hipLaunchKernelGGL((k_bsr_mv<T, BR, BC, false, false>), g, blk, 0, s, B.rp, B.ci, v, B.nbr, x, y,
                           xfirst, dinv, omega, done);
}

template <typename T>
static void bsr_mv(const BSR& B, const T* x, T* y, bool add, T* xfirst, const T* dinv, T omega,
                   const int* done, hipStream_t s) {
    const int key = B.br * 10 + B.bc;
    switch (key) {
        case 23: bsr_mv_shape<T, 2, 3>(B, x, y, add, xfirst, dinv, omega, done, s); break;
        case 32: bsr_mv_shape<T, 3, 2>(B, x, y, add, xfirst, dinv, omega, done, s); break;
        case 33: bsr_mv_shape<T, 3, 3>(B, x, y, add, xfirst, dinv, omega, done, s); break;
        case 36: bsr_mv_shape<T, 3, 6>(B, x, y, add, xfirst, dinv, omega, done, s); break;
        case 63: bsr_mv_shape<T, 6, 3>(B, x, y, add, xfirst, dinv, omega, done, s); break;
        case 66: bsr_mv_shape<T, 6, 6>(B, x, y, add, xfirst, dinv, omega, done, s); break;
        default: fail(TM_ERR_ARG, "unsupported prolongator block shape");
    }
}

template <typename T>
void launch_bsr_restrict(const Level& fine, const T* rf, T* bc, const Level& coarse, T* xc_first,
                         T omega, const int* done, hipStream_t s) {
    bsr_mv<T>(fine.PT, rf, bc, false, xc_first, dinv_of<T>(coarse), omega, done, s);
}
template void launch_bsr_restrict<double>(const Level&, const double*, double*, const Level&, double*,
                                          double, const int*, hipStream_t);
template void launch_bsr_restrict<float>(const Level&, const float*, float*, const Level&, float*, float,
                                         const int*, hipStream_t);

template <typename T>
void launch_bsr_prolong(const Level& fine, const T* xc, T* xf, const int* done, hipStream_t s) {
    bsr_mv<T>(fine.P, xc, xf, true, nullptr, nullptr, T(0), done, s);
}
template void launch_bsr_prolong<double>(const Level&, const double*, double*, const int*, hipStream_t);
template void launch_bsr_prolong<float>(const Level&, const float*, float*, const int*, hipStream_t);

// point-block inverse of the diagonal blocks of a BSR level operator
template <int BS>
__global__ void k_bsr_dinv(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const double* __restrict__ v, int64_t nbr, int point,
                           double* __restrict__ d64, float* __restrict__ d32, int* flags) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= nbr) return;
    double D[BS][BS] = {};
    for (int32_t q = rp[row]; q < rp[row + 1]; ++q)
        if (ci[q] == row) {
#pragma unroll
            for (int r = 0; r < BS; ++r)
#pragma unroll
                for (int c = 0; c < BS; ++c) D[r][c] = v[(int64_t)q * BS * BS + r * BS + c];
        }
    store_dinv<BS>(D, point, row, nbr, d64, d32, flags);
}

void launch_bsr_dinv(const Level& L, int point_jacobi, int* flags, hipStream_t s) {
    const dim3 g(grid_for(L.A.nbr)), blk(WG);
    if (L.bs == 3)
        hipLaunchKernelGGL(k_bsr_dinv<3>, g, blk, 0, s, L.A.rp, L.A.ci, L.A.v64, L.A.nbr, point_jacobi,
                           L.dinv64, L.dinv32, flags);
    else if (L.bs == 6)
        hipLaunchKernelGGL(k_bsr_dinv<6>, g, blk, 0, s, L.A.rp, L.A.ci, L.A.v64, L.A.nbr, point_jacobi,
                           L.dinv64, L.dinv32, flags);
    else
        fail(TM_ERR_ARG, "aggregation level block size must be 3 or 6");
}

}  // namespace tmi
