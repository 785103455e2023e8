// Linear density filter rho = S alpha and its transpose (Sec. 2, filtering
// matrix S; Sec. 4, radius 1.5 element sizes): element-parallel stencil over
// the elements whose centres lie closer than the radius.
#include <cmath>
#include <mutex>

#include "tm_device.h"

namespace tmi {

// Fixed scratch of tm_density_filter_noalloc: the scaled input W^-1 x of the
// transpose, one FP64 value per element.  Each GPU holds its own copy of this
// array for the life of the process; host code uses only the device address
// that hipGetSymbolAddress returns for it (taken once per device, with that
// device current), never the array's name.
static __device__ __align__(256) double scratch[FILTER_SCRATCH_MAX];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[MAX_DEVICES] = {};
}  // namespace

double* filter_scratch() {
    int dev = 0;
    TM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) fail(TM_ERR_DEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        TM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(TM_ERR_DEVICE, "no device address for the filter scratch");
        g_scratch_dev[dev] = (double*)p;
    }
    return g_scratch_dev[dev];
}

// cone weights max(0, r - |d|) of the (2R+1)^DIM offsets d, x fastest
template <int DIM, int R>
struct ConeW {
    static constexpr int W = 2 * R + 1;
    static constexpr int N = DIM == 3 ? W * W * W : W * W;
    double h[N];
};

// per-axis in-grid indicators (1.0 / 0.0) of the offsets -R..R from (i, j, k),
// so that the weight of offset d is h_d mx[dx] my[dy] mz[dz] with no branches
template <int DIM, int R>
struct AxisMasks {
    double mx[2 * R + 1], my[2 * R + 1], mz[2 * R + 1];
    __device__ __forceinline__ AxisMasks(int i, int j, int k, int nx, int ny, int nz) {
#pragma unroll
        for (int t = 0; t < 2 * R + 1; ++t) {
            mx[t] = ((i + t - R >= 0) & (i + t - R < nx)) ? 1.0 : 0.0;
            my[t] = ((j + t - R >= 0) & (j + t - R < ny)) ? 1.0 : 0.0;
            mz[t] = DIM == 2 ? (t == R ? 1.0 : 0.0) : (((k + t - R >= 0) & (k + t - R < nz)) ? 1.0 : 0.0);
        }
    }
    __device__ __forceinline__ double in(int tx, int ty, int tz) const { return mx[tx] * my[ty] * mz[tz]; }
};

// sum of H over the row of element (i, j, k): weights of the in-grid offsets
template <int DIM, int R>
__device__ __forceinline__ double cone_rowsum(const ConeW<DIM, R>& cw, const AxisMasks<DIM, R>& m) {
    constexpr int W = 2 * R + 1;
    double w = 0.0;
#pragma unroll
    for (int o = 0; o < ConeW<DIM, R>::N; ++o) {
        const int tx = o % W, ty = (o / W) % W, tz = DIM == 3 ? o / (W * W) : R;
        w += cw.h[o] * m.in(tx, ty, tz);
    }
    return w;
}

// out_e = sum_i H_ei in_i, divided by W_e = sum_i H_ei if NORM; every load
// unconditional (clamped index), outside offsets weighted by zero
template <int DIM, int R, bool NORM>
__global__ __launch_bounds__(WG) void k_filter_apply(const double* __restrict__ in, double* __restrict__ out,
                                                     int nx, int ny, int nz, const ConeW<DIM, R> cw) {
    constexpr int W = 2 * R + 1;
    const uint32_t n = (uint32_t)nx * (uint32_t)ny * (uint32_t)nz;
    const uint32_t e = (uint32_t)xcd_block() * WG + threadIdx.x;
    if (e >= n) return;
    const int i = (int)(e % (uint32_t)nx);
    const int j = (int)((e / (uint32_t)nx) % (uint32_t)ny);
    const int k = DIM == 3 ? (int)(e / ((uint32_t)nx * (uint32_t)ny)) : 0;
    // plane by plane (z); for R >= 2 the planes are not unrolled, so that at
    // most (2R+1)^2 loaded values are live
    constexpr int NP = W * W;
    const AxisMasks<DIM, R> m(i, j, k, nx, ny, nz);
    // clamped neighbour = e + ox[dx] + oy[dy] + oz[dz] (additions per offset)
    int ox[W], oy[W], oz[W];
#pragma unroll
    for (int t = 0; t < W; ++t) {
        ox[t] = min(max(i + t - R, 0), nx - 1) - i;
        oy[t] = (min(max(j + t - R, 0), ny - 1) - j) * nx;
        oz[t] = DIM == 3 ? (min(max(k + t - R, 0), nz - 1) - k) * nx * ny : 0;
    }
    double acc = 0.0, wsum = 0.0;      // wsum: row sum of H over the in-grid offsets
    auto plane = [&](int pz) {
        double v[NP];
#pragma unroll
        for (int o = 0; o < NP; ++o) v[o] = in[(uint32_t)((int)e + oz[pz] + oy[o / W] + ox[o % W])];
#pragma unroll
        for (int o = 0; o < NP; ++o) {
            const double hh = cw.h[pz * NP + o] * m.in(o % W, o / W, DIM == 3 ? pz : R);
            acc += hh * v[o];
            wsum += hh;
        }
    };
    if constexpr (R <= 1) {
#pragma unroll
        for (int pz = 0; pz < (DIM == 3 ? W : 1); ++pz) plane(pz);
    } else {
#pragma unroll 1
        for (int pz = 0; pz < (DIM == 3 ? W : 1); ++pz) plane(pz);
    }
    out[e] = NORM ? acc / wsum : acc;
}

// 3D, radius up to 2 element sizes (R = 1): each thread marches KZ elements up
// a z-column and keeps 3x3 planes of the input in registers (the next one in
// flight), so each output needs 9 (+ the chunk's two extra planes) loads, not 27.  Same sums as
// k_filter_apply<3, 1, NORM> (offsets in the same order).
constexpr int FILTER_KZ = 4;

template <bool NORM>
__global__ __launch_bounds__(WG) void k_filter_zmarch(const double* __restrict__ in, double* __restrict__ out,
                                                      int nx, int ny, int nz, const ConeW<3, 1> cw) {
    const uint32_t cols = (uint32_t)nx * (uint32_t)ny;
    const uint32_t nchunk = ((uint32_t)nz + FILTER_KZ - 1) / FILTER_KZ;
    const uint32_t t = (uint32_t)xcd_block() * WG + threadIdx.x;
    if (t >= cols * nchunk) return;
    const uint32_t col = t % cols, ch = t / cols;
    const int i = (int)(col % (uint32_t)nx), j = (int)(col / (uint32_t)nx);
    const int k0 = (int)ch * FILTER_KZ;
    const int k1 = min(k0 + FILTER_KZ, nz);
    // in-plane clamped offsets and indicators
    int off[9];
    double mxy[9];
#pragma unroll
    for (int o = 0; o < 9; ++o) {
        const int dx = o % 3 - 1, dy = o / 3 - 1;
        const int ii = min(max(i + dx, 0), nx - 1), jj = min(max(j + dy, 0), ny - 1);
        off[o] = jj * nx + ii;
        mxy[o] = ((i + dx >= 0) & (i + dx < nx) & (j + dy >= 0) & (j + dy < ny)) ? 1.0 : 0.0;
    }
    const int plane = nx * ny;
    double P[4][9];                     // planes k-1, k, k+1 (clamped) and k+2 in flight
    auto load = [&](double (&d)[9], int kk) {
        const int kc = min(max(kk, 0), nz - 1);
#pragma unroll
        for (int o = 0; o < 9; ++o) d[o] = in[(uint32_t)(kc * plane + off[o])];
    };
    load(P[0], k0 - 1);
    load(P[1], k0);
    load(P[2], k0 + 1);
    for (int k = k0; k < k1; ++k) {
        load(P[3], k + 2);              // next plane requested before this one is summed
        double acc = 0.0, wsum = 0.0;
#pragma unroll
        for (int pz = 0; pz < 3; ++pz) {
            const double mz = ((k + pz - 1 >= 0) & (k + pz - 1 < nz)) ? 1.0 : 0.0;
#pragma unroll
            for (int o = 0; o < 9; ++o) {
                const double hh = cw.h[pz * 9 + o] * (mxy[o] * mz);
                acc += hh * P[pz][o];
                wsum += hh;
            }
        }
        out[(uint32_t)(k * plane) + col] = NORM ? acc / wsum : acc;
#pragma unroll
        for (int o = 0; o < 9; ++o) {
            P[0][o] = P[1][o];
            P[1][o] = P[2][o];
            P[2][o] = P[3][o];
        }
    }
}

// out_e = in_e / W_e (first half of S^T: S^T x = H (W^-1 x), H symmetric)
template <int DIM, int R>
__global__ __launch_bounds__(WG) void k_filter_scale(const double* __restrict__ in, double* __restrict__ out,
                                                     int nx, int ny, int nz, const ConeW<DIM, R> cw) {
    const uint32_t n = (uint32_t)nx * (uint32_t)ny * (uint32_t)nz;
    const uint32_t e = (uint32_t)xcd_block() * WG + threadIdx.x;
    if (e >= n) return;
    const int i = (int)(e % (uint32_t)nx);
    const int j = (int)((e / (uint32_t)nx) % (uint32_t)ny);
    const int k = DIM == 3 ? (int)(e / ((uint32_t)nx * (uint32_t)ny)) : 0;
    out[e] = in[e] / cone_rowsum<DIM, R>(cw, AxisMasks<DIM, R>(i, j, k, nx, ny, nz));
}

template <int DIM, int R>
static void filter_run(int nx, int ny, int nz, double r, bool tr, const double* in, double* out,
                       double* fixed_scratch, hipStream_t s) {
    constexpr int W = 2 * R + 1;
    ConeW<DIM, R> cw;
    for (int o = 0; o < ConeW<DIM, R>::N; ++o) {
        const int dx = o % W - R, dy = (o / W) % W - R, dz = DIM == 3 ? o / (W * W) - R : 0;
        const double h = r - std::sqrt((double)(dx * dx + dy * dy + dz * dz));
        cw.h[o] = h > 0.0 ? h : 0.0;
    }
    const int64_t n = (int64_t)nx * ny * nz;
    const dim3 g(grid_for(n)), b(WG);
    const int64_t nch = (nz + FILTER_KZ - 1) / FILTER_KZ;
    const dim3 gz(grid_for((int64_t)nx * ny * nch));
    auto apply = [&](const double* src, double* dst, bool norm) {
        if constexpr (DIM == 3 && R == 1) {
            if (norm) hipLaunchKernelGGL((k_filter_zmarch<true>), gz, b, 0, s, src, dst, nx, ny, nz, cw);
            else hipLaunchKernelGGL((k_filter_zmarch<false>), gz, b, 0, s, src, dst, nx, ny, nz, cw);
        } else {
            if (norm) hipLaunchKernelGGL((k_filter_apply<DIM, R, true>), g, b, 0, s, src, dst, nx, ny, nz, cw);
            else hipLaunchKernelGGL((k_filter_apply<DIM, R, false>), g, b, 0, s, src, dst, nx, ny, nz, cw);
        }
    };
    if (!tr) {
        apply(in, out, true);
        return;
    }
    // W^-1 in: the caller's fixed scratch, else stream-ordered scratch; every
    // entry is written by the scaling kernel before it is read
    double* t = fixed_scratch;
    if (!t) TM_HIP(hipMallocAsync((void**)&t, (size_t)n * sizeof(double), s));
    hipLaunchKernelGGL((k_filter_scale<DIM, R>), g, b, 0, s, in, t, nx, ny, nz, cw);
    apply(t, out, false);
    if (!fixed_scratch) TM_HIP(hipFreeAsync(t, s));
}

void launch_density_filter(int dim, const int* nel, double r, bool tr, const double* in, double* out,
                           double* fixed_scratch, hipStream_t s) {
    // stencil half-width: offsets up to ceil(r) - 1 can lie closer than r
    const int R = (int)std::ceil(r) - 1;
    const int nz = dim == 3 ? nel[2] : 1;
#define TM_FL(RR)                                                             \
    if (dim == 3) filter_run<3, RR>(nel[0], nel[1], nz, r, tr, in, out, fixed_scratch, s);   \
    else filter_run<2, RR>(nel[0], nel[1], 1, r, tr, in, out, fixed_scratch, s);
    switch (R) {
        case 0: TM_FL(0) break;
        case 1: TM_FL(1) break;
        case 2: TM_FL(2) break;
        default: TM_FL(3) break;
    }
#undef TM_FL
}

}  // namespace tmi
