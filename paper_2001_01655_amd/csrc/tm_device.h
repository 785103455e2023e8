// Device helpers shared by the HIP translation units of libtopomg.
#pragma once
#include "tm_internal.h"

namespace tmi {

// ------------------------------------------------------------ block reduce
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], double* partials) {
    // fixed-shape tree: wave shuffles, then one wave over the wave sums
    __shared__ double red[NV][WG / 64];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double a = v[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o, 64);
        if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double a = 0.0;
#pragma unroll
            for (int w = 0; w < WG / 64; ++w) a += red[q][w];
            partials[(int64_t)q * gridDim.x + blockIdx.x] = a;
        }
    }
}

// MurmurHash3's 32-bit finaliser: a bijection of uint32 used as a hash
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// ------------------------------------------------------------ buffer loads
// Raw buffer loads take a 32-bit byte offset from a descriptor held in SGPRs,
// which avoids per-load 64-bit address arithmetic in the gather kernels.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, int64_t bytes) {
    const int nrec = (int)(bytes < 0x7fffffff ? bytes : 0x7fffffff);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, nrec, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bld(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ float bld<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ __forceinline__ double bld<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
// two consecutive values starting at byte offset off: one 8-byte load for FP32,
// one 16-byte load for FP64 (bit casts, no value conversion)
__device__ __forceinline__ void bld2(__amdgpu_buffer_rsrc_t r, uint32_t off, float (&v)[2]) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 t = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    v[0] = t.x;
    v[1] = t.y;
}
__device__ __forceinline__ void bld2(__amdgpu_buffer_rsrc_t r, uint32_t off, double (&v)[2]) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 t = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    v[0] = t.x;
    v[1] = t.y;
}
// three consecutive values starting at byte offset off: one 12-byte load for
// FP32, a 16-byte and an 8-byte load for FP64 (the vector assignments below
// reinterpret the loaded bits; they convert no values)
__device__ __forceinline__ void bld3(__amdgpu_buffer_rsrc_t r, uint32_t off, float (&v)[3]) {
    typedef float f3 __attribute__((ext_vector_type(3)));
    const f3 t = __builtin_amdgcn_raw_buffer_load_b96(r, off, 0, 0);
    v[0] = t.x;
    v[1] = t.y;
    v[2] = t.z;
}
__device__ __forceinline__ void bld3(__amdgpu_buffer_rsrc_t r, uint32_t off, double (&v)[3]) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 t = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    v[0] = t.x;
    v[1] = t.y;
    v[2] = bld<double>(r, off + 16);
}

// ------------------------------------------------------------ grid sums
// Sum over the whole block (fixed wave-shuffle tree, then wave order); every
// thread gets the result.
__device__ __forceinline__ double block_sum_all(double v) {
    __shared__ double red[WG / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < WG / 64; ++w) a += red[w];
    __syncthreads();
    return a;
}

// ------------------------------------------------------------ small SPD inverse
// Inverse of a symmetric positive definite BS x BS block through its Cholesky
// factor: A^-1 = L^-T L^-1.  Returns false on a non-positive pivot.
template <int BS>
__device__ bool spd_inverse(const double (&A)[BS][BS], double (&X)[BS][BS]) {
    double L[BS][BS];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < BS; ++j) {
        double d = A[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        ok = ok && (d > 0.0);
        double ljj = d > 0.0 ? sqrt(d) : 1.0;
        L[j][j] = ljj;
#pragma unroll
        for (int i = j + 1; i < BS; ++i) {
            double t = A[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            L[i][j] = t / ljj;
        }
#pragma unroll
        for (int i = 0; i < j; ++i) L[i][j] = 0.0;
    }
    // W = L^-1 (lower triangular)
    double W[BS][BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) {
#pragma unroll
        for (int i = 0; i < BS; ++i) {
            double t = (i == c) ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < i; ++k) t -= L[i][k] * W[k][c];
            W[i][c] = (i < c) ? 0.0 : t / L[i][i];
        }
    }
    // X = W^T W
#pragma unroll
    for (int i = 0; i < BS; ++i)
#pragma unroll
        for (int j = 0; j < BS; ++j) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < BS; ++k) t += W[k][i] * W[k][j];
            X[i][j] = t;
        }
    return ok;
}

template <int BS>
__device__ void store_dinv(double (&D)[BS][BS], int point, int64_t node, int64_t N,
                          double* __restrict__ d64, float* __restrict__ d32, int* flags) {
    double X[BS][BS];
    if (point) {
#pragma unroll
        for (int i = 0; i < BS; ++i)
#pragma unroll
            for (int j = 0; j < BS; ++j) X[i][j] = (i == j) ? 1.0 / D[i][i] : 0.0;
        bool ok = true;
#pragma unroll
        for (int i = 0; i < BS; ++i) ok = ok && D[i][i] > 0.0;
        if (!ok) atomicOr(flags, FLAG_NOT_SPD);
    } else if (!spd_inverse<BS>(D, X)) {
        atomicOr(flags, FLAG_NOT_SPD);
    }
#pragma unroll
    for (int i = 0; i < BS; ++i)
#pragma unroll
        for (int j = i; j < BS; ++j) {
            d64[(int64_t)sym_at(i, j, BS) * N + node] = X[i][j];
            d32[(int64_t)sym_at(i, j, BS) * N + node] = (float)X[i][j];
        }
}

__device__ __forceinline__ float fma_of(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_of(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ------------------------------------------------------------ operator kernels
// Operands of a node's finishing step, loaded apart from the arithmetic so
// that latency-bound kernels can issue them together with their gathers.
template <typename T, int BS>
struct FinIn {
    T b[BS];
    T dv[sym_n(BS)];      // upper triangle of the block inverse
    T din[BS];
};

template <typename T, int BS, int OP>
__device__ __forceinline__ void finish_load(int64_t node, int64_t N, const T* __restrict__ b,
                                            const T* __restrict__ dinv, const ChebArgs& ch, FinIn<T, BS>& f) {
    if (OP != OP_APPLY) {
#pragma unroll
        for (int c = 0; c < BS; ++c) f.b[c] = b[BS * node + c];
    }
    if (OP == OP_SMOOTH || OP == OP_CHEB) {
#pragma unroll
        for (int e = 0; e < sym_n(BS); ++e) f.dv[e] = dinv[(int64_t)e * N + node];
    }
    if (OP == OP_CHEB) {
        const T* din = (const T*)ch.din;
#pragma unroll
        for (int r = 0; r < BS; ++r) f.din[r] = din[BS * node + r];
    }
}

template <typename T, int BS, int OP>
__device__ __forceinline__ void finish_store(int64_t node, T (&kx)[BS], const T (&xo)[BS], uint8_t m,
                                             const FinIn<T, BS>& f, T* __restrict__ y, T omega,
                                             double (&dots)[2], const ChebArgs& ch) {
#pragma unroll
    for (int c = 0; c < BS; ++c)
        if (m & (1u << c)) kx[c] = xo[c];               // unit row of a supported dof
    if (OP == OP_APPLY) {
#pragma unroll
        for (int c = 0; c < BS; ++c) y[BS * node + c] = kx[c];
    } else if (OP == OP_RESID) {
#pragma unroll
        for (int c = 0; c < BS; ++c) y[BS * node + c] = f.b[c] - kx[c];
    } else if (OP == OP_SMOOTH) {
        T rr[BS];
#pragma unroll
        for (int c = 0; c < BS; ++c) rr[c] = f.b[c] - kx[c];
#pragma unroll
        for (int r = 0; r < BS; ++r) {
            T t = 0;
#pragma unroll
            for (int c = 0; c < BS; ++c) t += f.dv[sym_at(r, c, BS)] * rr[c];
            y[BS * node + r] = xo[r] + omega * t;
        }
    } else if (OP == OP_CHEB) {
        T rr[BS];
#pragma unroll
        for (int c = 0; c < BS; ++c) rr[c] = f.b[c] - kx[c];
        T* dout = (T*)ch.dout;
        const T c1 = (T)ch.c1, c2 = (T)ch.c2;
#pragma unroll
        for (int r = 0; r < BS; ++r) {
            T t = 0;
#pragma unroll
            for (int c = 0; c < BS; ++c) t += f.dv[sym_at(r, c, BS)] * rr[c];
            // the fused multiply-add is written out: c1 din + c2 t has two
            // contractions, and the compiler's pick differs between kernels,
            // while every kernel that runs this step must round alike
            const T dn = fma_of(t, c2, c1 * f.din[r]);
            if (dout) dout[BS * node + r] = dn;           // null: no later step reads it
            y[BS * node + r] = xo[r] + dn;
        }
    } else {  // OP_QDOT: q = K~ p, partial p.q and p.r (b holds r)
#pragma unroll
        for (int c = 0; c < BS; ++c) {
            y[BS * node + c] = kx[c];
            dots[0] += (double)xo[c] * (double)kx[c];
            dots[1] += (double)xo[c] * (double)f.b[c];
        }
    }
}

// y from the operator value kx = (A x)_node: apply, residual, damped block
// Jacobi sweep, Chebyshev step, or q = A p with the partial dots p.q, p.r
template <typename T, int BS, int OP>
__device__ __forceinline__ void finish_node(int64_t node, int64_t N, T (&kx)[BS], const T (&xo)[BS],
                                            uint8_t m, const T* __restrict__ b, T* __restrict__ y,
                                            const T* __restrict__ dinv, T omega, double (&dots)[2],
                                            const ChebArgs& ch = ChebArgs{}) {
    FinIn<T, BS> f;
    finish_load<T, BS, OP>(node, N, b, dinv, ch, f);
    finish_store<T, BS, OP>(node, kx, xo, m, f, y, omega, dots, ch);
}

}  // namespace tmi
