// Host orchestration and the C ABI of libtopomg: argument checks, level plan,
// hierarchy setup (Secs. 2, 3.2, 4), the V-cycle of Algorithm 1, the outer
// CG loop driver, solve states for iteration-level scheduling, and exports.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "tm_internal.h"

namespace tmi {

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

struct TmException : std::runtime_error {
    tm_status code;
    TmException(tm_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void fail(tm_status code, const std::string& msg) { throw TmException(code, msg); }

void check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        fail(TM_ERR_OOM, std::string(what) + ": " + hipGetErrorString(e));
    fail(TM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename F>
static tm_status guarded(F&& f) {
    try {
        f();
        return TM_OK;
    } catch (const TmException& e) {
        set_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return TM_ERR_OOM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return TM_ERR_DEVICE;
    }
}

// ------------------------------------------------------------------ memory
// Device memory of a hierarchy comes from the caller's allocator when one was
// given to tm_setup (on the stream of the call that needs it), else hipMalloc.
void* dev_alloc(const tm_hierarchy* h, size_t b) {
    void* p = nullptr;
    if (h->has_alloc) {
        p = h->alloc.alloc(b, (void*)h->cur_stream, h->alloc.ctx);
        if (!p) fail(TM_ERR_OOM, "the caller's allocator returned no memory for " + std::to_string(b) + " bytes");
        return p;
    }
    const hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(TM_ERR_OOM, "hipMalloc of " + std::to_string(b) + " bytes failed");
    }
    return p;
}

// Every block goes back only after the device has finished the work that
// used it: hipFree waits by itself; a caller's free is preceded by a device
// synchronisation (its allocator may hand the block out again at once).
void dev_free_list(const tm_hierarchy* h, std::vector<void*>& list) {
    if (list.empty()) return;
    if (h->has_alloc) {
        (void)hipDeviceSynchronize();
        for (void* p : list) h->alloc.free(p, (void*)h->cur_stream, h->alloc.ctx);
    } else {
        for (void* p : list) (void)hipFree(p);
    }
    list.clear();
}

void* arena_get(const tm_hierarchy* h, Arena& a, size_t bytes) {
    const size_t b = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    a.need += b;
    if (a.used + b <= a.cap) {
        void* p = a.base + a.used;
        a.used += b;
        return p;
    }
    void* p = dev_alloc(h, b);
    a.overflow.push_back(p);
    a.overflow_bytes += b;
    return p;
}

void arena_reset(Arena& a) {
    a.peak = std::max(a.peak, a.need);
    a.need = 0;
    a.used = 0;
}

void arena_prepare(const tm_hierarchy* h, Arena& a) {
    arena_reset(a);
    if (a.overflow.empty()) {
        a.peak = 0;
        return;
    }
    // the last rebuild outgrew the buffer: one buffer for its largest cycle
    // (with headroom), once the device is done with the old blocks
    const size_t want = a.peak + a.peak / 4;
    std::vector<void*> old = a.overflow;
    if (a.base) old.push_back(a.base);
    dev_free_list(h, old);
    a.overflow.clear();
    a.overflow_bytes = 0;
    a.base = nullptr;
    a.cap = 0;
    a.base = (char*)dev_alloc(h, want);
    a.cap = want;
    a.used = 0;
    a.need = 0;
    a.peak = 0;
}

void arena_release(const tm_hierarchy* h, Arena& a) {
    std::vector<void*> all = a.overflow;
    if (a.base) all.push_back(a.base);
    dev_free_list(h, all);
    a = Arena();
}

size_t arena_bytes(const Arena& a) { return a.cap + a.overflow_bytes; }

template <typename T>
static T* dalloc(const tm_hierarchy* h, std::vector<void*>& list, size_t& bytes, size_t n) {
    const size_t b = std::max<size_t>(n, 1) * sizeof(T);
    void* p = dev_alloc(h, b);
    list.push_back(p);
    bytes += b;
    return (T*)p;
}
template <typename T>
static T* halloc(tm_hierarchy* h, size_t n) { return dalloc<T>(h, h->allocs, h->bytes, n); }

static void free_list(const tm_hierarchy* h, std::vector<void*>& list) { dev_free_list(h, list); }

static hipStream_t S(void* s) { return (hipStream_t)s; }

// ------------------------------------------------------------------ element stiffness
// KE for E = 1 of the bilinear / trilinear element on a square / cube of edge h:
// sum over the 2^dim Gauss points of B^T D B |J| (exact for these elements).
// 2D plane stress with unit thickness; 3D isotropic.  Local corner order as
// in loc2 / loc3.
static void element_stiffness(int dim, double nu, double h, std::vector<double>& KE) {
    const int npe = 1 << dim, nd = dim * npe;
    KE.assign((size_t)nd * nd, 0.0);
    int corner[8][3];
    for (int z = 0; z < (dim == 3 ? 2 : 1); ++z)
        for (int y = 0; y < 2; ++y)
            for (int x = 0; x < 2; ++x) {
                const int a = dim == 3 ? loc3(x, y, z) : loc2(x, y);
                corner[a][0] = x;
                corner[a][1] = y;
                corner[a][2] = z;
            }
    const int nv = dim == 2 ? 3 : 6;
    double D[6][6] = {};
    if (dim == 2) {
        const double c = 1.0 / (1.0 - nu * nu);
        D[0][0] = D[1][1] = c;
        D[0][1] = D[1][0] = c * nu;
        D[2][2] = c * (1.0 - nu) / 2.0;
    } else {
        const double c = 1.0 / ((1.0 + nu) * (1.0 - 2.0 * nu));
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) D[i][j] = c * (i == j ? 1.0 - nu : nu);
        for (int i = 3; i < 6; ++i) D[i][i] = c * (1.0 - 2.0 * nu) / 2.0;
    }
    const double g = 1.0 / std::sqrt(3.0);
    const double jac = h / 2.0;
    const double detJ = std::pow(jac, dim);
    const int ngp = 1 << dim;
    for (int gp = 0; gp < ngp; ++gp) {
        double xi[3] = {(gp & 1) ? g : -g, (gp & 2) ? g : -g, (gp & 4) ? g : -g};
        double grad[8][3];
        for (int a = 0; a < npe; ++a)
            for (int d = 0; d < dim; ++d) {
                double v = 1.0 / (1 << dim);
                for (int e = 0; e < dim; ++e) {
                    const double sgn = corner[a][e] ? 1.0 : -1.0;
                    v *= (e == d) ? sgn : (1.0 + sgn * xi[e]);
                }
                grad[a][d] = v / jac;
            }
        double B[6][24] = {};
        for (int a = 0; a < npe; ++a) {
            if (dim == 2) {
                B[0][2 * a] = grad[a][0];
                B[1][2 * a + 1] = grad[a][1];
                B[2][2 * a] = grad[a][1];
                B[2][2 * a + 1] = grad[a][0];
            } else {
                B[0][3 * a] = grad[a][0];
                B[1][3 * a + 1] = grad[a][1];
                B[2][3 * a + 2] = grad[a][2];
                B[3][3 * a + 1] = grad[a][2];
                B[3][3 * a + 2] = grad[a][1];
                B[4][3 * a] = grad[a][2];
                B[4][3 * a + 2] = grad[a][0];
                B[5][3 * a] = grad[a][1];
                B[5][3 * a + 1] = grad[a][0];
            }
        }
        for (int i = 0; i < nd; ++i)
            for (int j = 0; j < nd; ++j) {
                double s = 0.0;
                for (int p = 0; p < nv; ++p)
                    for (int q = 0; q < nv; ++q) s += B[p][i] * D[p][q] * B[q][j];
                KE[(size_t)i * nd + j] += s * detJ;
            }
    }
    for (int i = 0; i < nd; ++i)
        for (int j = 0; j < i; ++j) {
            const double s = 0.5 * (KE[(size_t)i * nd + j] + KE[(size_t)j * nd + i]);
            KE[(size_t)i * nd + j] = KE[(size_t)j * nd + i] = s;
        }
}

// Class values of KE under the symmetries of the square / cube (one value per
// orbit, signs from the compile-time tables); every entry is checked against
// its class value, so the fine operator applies exactly this KE.
template <int DIM>
static void ke_class_values(const KeClasses<DIM>& T, const std::vector<double>& KE, tm_hierarchy* h) {
    constexpr int nd = DIM << DIM;
    double amax = 0.0;
    for (double v : KE) amax = std::max(amax, std::fabs(v));
    bool seen[KE_MAX_CLASSES] = {};
    double kv[KE_MAX_CLASSES] = {};
    for (int r = 0; r < nd; ++r)
        for (int c = 0; c < nd; ++c) {
            const double v = KE[r * nd + c];
            const int k = T.cls[r][c], sg = T.sgn[r][c];
            if (sg == 0) {
                if (std::fabs(v) > 1e-12 * amax) fail(TM_ERR_ARG, "element stiffness lacks its symmetry");
                continue;
            }
            if (!seen[k]) {
                seen[k] = true;
                kv[k] = sg * v;
            } else if (std::fabs(kv[k] - sg * v) > 1e-12 * amax) {
                fail(TM_ERR_ARG, "element stiffness lacks its symmetry");
            }
        }
    for (int k = 0; k < KE_MAX_CLASSES; ++k) {
        h->kc64.k[k] = kv[k];
        h->kc32.k[k] = (float)kv[k];
    }
}

// The 3D KE in the tensor form: C = F KE F^T / 64 per pair of components (F
// the +-1 sum / difference transform of the eight corner values), kept where
// the form has a coupling; every other entry of C must vanish, or the fine
// operator keeps the node gather (sf_ok false).
static void ke_tensor_coefs(const std::vector<double>& KE, tm_hierarchy* h) {
    double F[8][8];
    for (int m = 0; m < 8; ++m)
        for (int lz = 0; lz < 2; ++lz)
            for (int ly = 0; ly < 2; ++ly)
                for (int lx = 0; lx < 2; ++lx) {
                    const int l[3] = {lx, ly, lz};
                    double w = 1.0;
                    for (int k = 0; k < 3; ++k)
                        if ((m >> k) & 1) w *= l[k] ? 1.0 : -1.0;
                    F[m][loc3(lx, ly, lz)] = w;
                }
    double amax = 0.0;
    for (double v : KE) amax = std::max(amax, std::fabs(v));
    bool ok = true;
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d)
            for (int mo = 0; mo < 8; ++mo)
                for (int mi = 0; mi < 8; ++mi) {
                    double v = 0.0;
                    for (int a = 0; a < 8; ++a)
                        for (int b2 = 0; b2 < 8; ++b2) v += F[mo][a] * KE[(3 * a + c) * 24 + 3 * b2 + d] * F[mi][b2];
                    v /= 64.0;
                    const int sl = SF_SLOTS.s[c][d][mi];
                    if (sl >= 0 && sf_out_mode(c, d, mi) == mo) {
                        h->sf64.k[sl] = v;
                        h->sf32.k[sl] = (float)v;
                    }
                    else if (std::fabs(v) > 1e-12 * amax)
                        ok = false;
                }
    h->sf_ok = ok;
}

// Q[c][a][b]: weight of parent corner b at child c's corner a (coarse shape
// functions), child c at offsets (c&1, c>>1&1, c>>2&1) inside its parent.

// ------------------------------------------------------------------ validation / plan
static int64_t nodes_of(const int* nel, int dim) {
    int64_t n = 1;
    for (int d = 0; d < dim; ++d) n *= (int64_t)nel[d] + 1;
    return n;
}

static void check_mesh(const tm_mesh* m) {
    if (!m) fail(TM_ERR_ARG, "mesh is NULL");
    if (m->dim != 2 && m->dim != 3) fail(TM_ERR_ARG, "mesh.dim must be 2 or 3");
    for (int d = 0; d < m->dim; ++d)
        if (m->nel[d] < 1 || m->nel[d] > (1 << 20)) fail(TM_ERR_ARG, "mesh.nel out of range");
    if (!(m->h > 0.0) || !std::isfinite(m->h)) fail(TM_ERR_ARG, "mesh.h must be positive");
    if (nodes_of(m->nel, m->dim) * m->dim >= ((int64_t)1 << 31))
        fail(TM_ERR_ARG, "mesh too large (dofs must fit in int32)");
}

static void check_opts(const tm_options* o) {
    if (!o) fail(TM_ERR_ARG, "options are NULL");
    if (o->n_levels < 0 || o->n_levels > 24) fail(TM_ERR_ARG, "n_levels out of range");
    if (o->n_geometric < 0 || o->n_geometric > 24) fail(TM_ERR_ARG, "n_geometric out of range");
    if (o->n_geometric == 1) fail(TM_ERR_ARG, "aggregation needs an assembled level: n_geometric >= 2");
    if (o->max_coarse < 1) fail(TM_ERR_ARG, "max_coarse must be >= 1");
    if (o->smoother != TM_SMOOTH_BLOCK_JACOBI && o->smoother != TM_SMOOTH_POINT_JACOBI &&
        o->smoother != TM_SMOOTH_CHEBYSHEV)
        fail(TM_ERR_ARG, "smoother must be TM_SMOOTH_BLOCK_JACOBI, TM_SMOOTH_POINT_JACOBI or TM_SMOOTH_CHEBYSHEV");
    if (o->smoother == TM_SMOOTH_CHEBYSHEV && !(o->cheb_lower > 0.0 && o->cheb_lower < 1.0))
        fail(TM_ERR_ARG, "cheb_lower must be in (0, 1)");
    if (o->adapt_iters < 0) fail(TM_ERR_ARG, "adapt_iters must be >= 0");
    if (o->cheb_warm_steps < 0 || o->cheb_warm_steps > 12) fail(TM_ERR_ARG, "cheb_warm_steps must be in 0..12");
    if (o->nu_pre < 1 || o->nu_post < 1 || o->nu_pre > 16 || o->nu_post > 16)
        fail(TM_ERR_ARG, "nu_pre / nu_post must be in 1..16");
    if (!(o->omega > 0.0 && o->omega < 2.0)) fail(TM_ERR_ARG, "omega must be in (0, 2)");
    if (!(o->sa_beta >= 0.0 && o->sa_beta < 1.0)) fail(TM_ERR_ARG, "sa_beta must be in [0, 1)");
    if (o->vcycle_fp != 32 && o->vcycle_fp != 64) fail(TM_ERR_ARG, "vcycle_fp must be 32 or 64");
    if (o->outer != TM_OUTER_FCG && o->outer != TM_OUTER_PCG) fail(TM_ERR_ARG, "outer must be FCG or PCG");
    if (o->max_iters < 1) fail(TM_ERR_ARG, "max_iters must be >= 1");
    if (o->check_every < 0) fail(TM_ERR_ARG, "check_every must be >= 0");
    if (o->fine_mfma != 0 && o->fine_mfma != 1) fail(TM_ERR_ARG, "fine_mfma must be 0 or 1");
    if (o->stencil_kernel < 0 || o->stencil_kernel > 3) fail(TM_ERR_ARG, "stencil_kernel must be 0, 1, 2 or 3");
    if (o->sa_lds < 0 || o->sa_lds > 1) fail(TM_ERR_ARG, "sa_lds must be 0 or 1");
    if (o->fine_tensor < 0 || o->fine_tensor > 4096) fail(TM_ERR_ARG, "fine_tensor must be in 0..4096");
    if (o->n_levels > 0 && o->n_geometric > o->n_levels) fail(TM_ERR_ARG, "n_geometric > n_levels");
}

static void check_material(const tm_material* m) {
    if (!m) fail(TM_ERR_ARG, "material is NULL");
    if (!(m->E0 > 0.0) || !std::isfinite(m->E0)) fail(TM_ERR_ARG, "E0 must be positive");
    if (!(m->Emin > 0.0) || !(m->Emin <= m->E0)) fail(TM_ERR_ARG, "Emin must be in (0, E0]");
    if (!(m->p >= 1.0 && m->p <= 16.0)) fail(TM_ERR_ARG, "p must be in [1, 16]");
    if (!(m->nu > -1.0 && m->nu < 0.5)) fail(TM_ERR_ARG, "nu must be in (-1, 0.5)");
}

// number of geometric levels (fine grid included) and whether aggregation follows
struct Plan {
    int Lg = 1;
    bool sa = false;
    int L_total = 1;        // known for pure geometric hierarchies
};

static Plan plan_levels(const tm_mesh* m, const tm_options* o) {
    Plan p;
    const int dim = m->dim;
    int cur[3] = {m->nel[0], m->nel[1], dim == 3 ? m->nel[2] : 1};
    auto dofs = [&](const int* c) { return nodes_of(c, dim) * dim; };
    // a level coarsens to ceil(n/2) elements per axis (Sec. 4.3); every axis
    // needs at least two elements for that to shrink it
    auto coarsenable = [&](const int* c) {
        for (int d = 0; d < dim; ++d)
            if (c[d] < 2) return false;
        return true;
    };
    if (o->n_geometric > 0) {
        p.Lg = o->n_geometric;
        p.sa = (o->n_levels == 0) || (o->n_levels > o->n_geometric);
    } else if (o->n_levels > 0) {
        p.Lg = o->n_levels;
    } else {
        p.Lg = 1;
        while (dofs(cur) >= o->max_coarse && coarsenable(cur)) {
            for (int d = 0; d < dim; ++d) cur[d] = (cur[d] + 1) / 2;
            ++p.Lg;
        }
        cur[0] = m->nel[0];
        cur[1] = m->nel[1];
        cur[2] = dim == 3 ? m->nel[2] : 1;
    }
    for (int l = 0; l + 1 < p.Lg; ++l) {
        if (!coarsenable(cur))
            fail(TM_ERR_ARG, "too many geometric levels: an axis would be coarsened below one element");
        for (int d = 0; d < dim; ++d) {
            cur[d] = (cur[d] + 1) / 2;
        }
    }
    p.L_total = p.Lg;
    // The operator kernels address the fine vectors and moduli and the first
    // coarse level's stored stencil through buffer descriptors, whose range is
    // below 2 GiB, with 32-bit byte offsets: refuse a mesh whose FP64 copies
    // of those arrays would reach 2 GiB (deeper levels are 8x smaller each).
    const int64_t lim = (int64_t)1 << 31;
    const int64_t nodes0 = nodes_of(m->nel, dim);
    const int64_t n_el = (int64_t)m->nel[0] * m->nel[1] * (dim == 3 ? m->nel[2] : 1);
    if (nodes0 * dim * 8 >= lim || n_el * 8 >= lim)
        fail(TM_ERR_ARG, "mesh too large: an FP64 fine-level vector must stay below 2 GiB (buffer range)");
    if (p.Lg > 1) {
        int c1[3] = {(m->nel[0] + 1) / 2, (m->nel[1] + 1) / 2, dim == 3 ? (m->nel[2] + 1) / 2 : 1};
        const int bb = dim * dim, nst = dim == 3 ? 27 : 9, nq = (nst - 1) / 2 * bb + dim * (dim + 1) / 2;
        if (nodes_of(c1, dim) * nq * 8 >= lim)
            fail(TM_ERR_ARG, "mesh too large: the first coarse level's FP64 stencil must stay below 2 GiB "
                             "(buffer range)");
    }
    return p;
}

}  // namespace tmi

using namespace tmi;

// ============================================================================ setup
namespace tmi {

static void alloc_level_geo(tm_hierarchy* h, Level& L, int l) {
    const int dim = h->dim;
    L.dim = dim;
    L.bs = dim;
    for (int d = 0; d < 3; ++d) {
        int n = d < dim ? h->mesh.nel[d] : 1;
        for (int q = 0; q < l; ++q) n = (n + 1) / 2;          // ceil(n/2) per coarsening
        L.nel[d] = n;
        L.nn[d] = d < dim ? L.nel[d] + 1 : 1;
    }
    L.n_nodes = nodes_of(L.nel, dim);
    L.n = L.n_nodes * dim;
    const int bb = dim * dim;
    L.dinv64 = halloc<double>(h, (size_t)sym_n(dim) * L.n_nodes);
    L.dinv32 = halloc<float>(h, (size_t)sym_n(dim) * L.n_nodes);
    if (l == 0) {
        L.kind = TM_LEVEL_FINE;
        L.E64 = halloc<double>(h, h->n_el);
        L.E32 = halloc<float>(h, h->n_el);
        L.nmask = halloc<uint8_t>(h, L.n_nodes);
    } else {
        L.kind = TM_LEVEL_GEOMETRIC;
        L.nst = dim == 3 ? 27 : 9;
        L.st64 = halloc<double>(h, (size_t)L.nst * bb * L.n_nodes);
        L.nq = (L.nst - 1) / 2 * bb + dim * (dim + 1) / 2;
        L.op_kernel = h->opt.stencil_kernel == 3 ? 0 : h->opt.stencil_kernel;    // 3: level 1 aside, by size
        L.stc64 = halloc<double>(h, (size_t)L.nq * L.n_nodes);
        L.stc32 = halloc<float>(h, (size_t)L.nq * L.n_nodes);
    }
}

static int64_t level_elems(const Level& L, int dim) {
    return (int64_t)L.nel[0] * L.nel[1] * (dim == 3 ? L.nel[2] : 1);
}

static void read_flags(tm_hierarchy* h, hipStream_t s, const char* phase) {
    int f = 0;
    TM_HIP(hipMemcpyAsync(&f, h->flags, sizeof(int), hipMemcpyDeviceToHost, s));
    TM_HIP(hipStreamSynchronize(s));
    if (f & FLAG_BAD_RHO) fail(TM_ERR_ARG, "densities must be finite and in [0, 1]");
    if (f & FLAG_NOT_SPD) fail(TM_ERR_NOT_SPD, std::string("operator not positive definite (") + phase + ")");
}

void build_sa_levels(tm_hierarchy* h, hipStream_t s);      // kernels_sa / host_sa
void numeric_sa_levels(tm_hierarchy* h, hipStream_t s);

static void cheb_interval(tm_hierarchy* h, int l, hipStream_t s, bool warm);

// Numeric setup for densities rho.  With sync the device checks (densities,
// SPD blocks, coarsest factor) are read before returning; without, nothing
// waits for the device and the next solve reads them (flags_pending).
static void numeric_setup(tm_hierarchy* h, const double* rho, hipStream_t s, bool sync = true) {
    ++h->update_seq;
    TM_HIP(hipMemsetAsync(h->flags, 0, sizeof(int), s));
    Level& F = h->lv[0];
    launch_simp(rho, h->n_el, h->mat.p, h->mat.E0, h->mat.Emin, F.E64, F.E32, h->rho64, h->flags, s);
    const int point = h->opt.smoother == TM_SMOOTH_POINT_JACOBI;
    launch_fine_dinv(F, h->KE64, point, h->flags, s);
    if (sync) read_flags(h, s, "fine diagonal");
    int Lg = 0;
    for (auto& L : h->lv)
        if (L.kind != TM_LEVEL_AGGREGATION) ++Lg;
    double* prev = nullptr;
    double* bufs[2] = {h->elem_a, h->elem_b};
    for (int l = 1; l < Lg; ++l) {
        double* cur = bufs[(l - 1) & 1];
        launch_galerkin_elems(h, l - 1, prev, cur, s);
        launch_stencil_assemble(h->lv[l], cur, s);
        launch_stencil_compact(h->lv[l], s);
        launch_stencil_dinv(h->lv[l], point, h->flags, s);
        prev = cur;
    }
    if (h->sa) numeric_sa_levels(h, s);
    if (h->opt.smoother == TM_SMOOTH_CHEBYSHEV) {
        if ((int)h->lv.size() > CHEB_MAX_LEVELS) fail(TM_ERR_ARG, "too many levels for Chebyshev smoothing");
        if (h->opt.cheb_warm_steps > 0 && !h->cheb_v) {
            // one vector per geometric level (their sizes never change)
            int64_t tot = 0;
            h->cheb_off.assign(Lg, 0);
            for (int l = 0; l < Lg; ++l) {
                h->cheb_off[l] = tot;
                tot += h->lv[l].n;
            }
            h->cheb_v = halloc<double>(h, (size_t)tot);
            h->cheb_ninv = halloc<double>(h, CHEB_MAX_LEVELS);
            h->cheb_warm = false;
        }
        const bool warm = h->cheb_v && h->cheb_warm;
        for (int l = 0; l + 1 < (int)h->lv.size(); ++l) cheb_interval(h, l, s, warm && l < Lg);
        if (h->cheb_v) h->cheb_warm = true;
    }
    // coarsest operator: dense FP64, Cholesky, explicit inverse
    Level& C = h->lv.back();
    const int64_t nc = C.n;
    h->nc = nc;
    if (h->dense_cap < (size_t)nc * nc) {
        h->dense_a = halloc<double>(h, (size_t)nc * nc);
        h->dense_cap = (size_t)nc * nc;
    }
    if (!h->chol_ls) h->chol_ls = halloc<double>(h, (size_t)chol_block_elems());
    double* Ad = h->dense_a;
    double* Ls = h->chol_ls;
    TM_HIP(hipMemsetAsync(Ad, 0, (size_t)nc * nc * sizeof(double), s));
    if (C.kind == TM_LEVEL_AGGREGATION)
        launch_dense_from_bsr(C, Ad, s);
    else if (C.kind == TM_LEVEL_GEOMETRIC)
        launch_dense_from_stencil(C, Ad, s);
    else
        fail(TM_ERR_ARG, "a hierarchy needs at least two levels");
    if (h->ainv_cap < (size_t)nc * nc) {
        h->ainv = halloc<double>(h, (size_t)nc * nc);
        h->ainv_cap = (size_t)nc * nc;
    }
    launch_cholesky_inverse(Ad, h->ainv, Ls, nc, h->flags, s);
    if (sync) {
        read_flags(h, s, "coarsest Cholesky");
        TM_HIP(hipStreamSynchronize(s));
    }
    h->flags_pending = !sync;
}

static void destroy_hierarchy(tm_hierarchy* h);

}  // namespace tmi

// ============================================================================ V-cycle
namespace tmi {

template <typename T> static T* vb(Vcyc& V, int l) { return (T*)V.b[l]; }
template <typename T> static T* vx(Vcyc& V, int l) { return (T*)V.x[l]; }
template <typename T> static T* vt(Vcyc& V, int l) { return (T*)V.t[l]; }

static void timed_begin(tm_hierarchy* h, int cls, hipStream_t s, hipEvent_t* e0) {
    if (!h->timing[cls]) return;
    TM_HIP(hipEventCreate(e0));
    TM_HIP(hipEventRecord(*e0, s));
}
static void timed_end(tm_hierarchy* h, int cls, hipStream_t s, hipEvent_t e0) {
    if (!h->timing[cls]) return;
    hipEvent_t e1;
    TM_HIP(hipEventCreate(&e1));
    TM_HIP(hipEventRecord(e1, s));
    h->tev[cls].push_back({e0, e1});
}

// one operator application on level l for lanes io[0..n) (hierarchies with
// the same level structure as io[0].h; Chebyshev coefficients c1, c2 are the
// same for all lanes, the directions are the lanes' own)
template <typename T>
static void level_op_b(int l, int op, const LaneIO* io, int n, hipStream_t s, double c1 = 0.0, double c2 = 0.0) {
    tm_hierarchy* h = const_cast<tm_hierarchy*>(io[0].h);
    Level& L = h->lv[l];
    const T w = (T)h->opt.omega;
    hipEvent_t e0 = nullptr;
    if (L.kind == TM_LEVEL_FINE) {
        timed_begin(h, 1, s, &e0);
        launch_fine_op_b<T>(op, false, io, n, w, c1, c2, s);
        timed_end(h, 1, s, e0);
    } else if (L.kind == TM_LEVEL_GEOMETRIC) {
        const int cls = l == 1 ? 2 : -1;
        if (cls >= 0) timed_begin(h, cls, s, &e0);
        launch_stencil_op_b<T>(l, op, io, n, w, c1, c2, s);
        if (cls >= 0) timed_end(h, cls, s, e0);
    } else {
        // aggregation levels: each lane's own operator (sizes depend on its data)
        for (int q = 0; q < n; ++q) {
            ChebArgs ch;
            ch.din = io[q].din;
            ch.dout = io[q].dout;
            ch.c1 = c1;
            ch.c2 = c2;
            launch_bsr_op<T>(io[q].h->lv[l], op, (const T*)io[q].x, (const T*)io[q].b, (T*)io[q].y, w, io[q].done,
                             s, ch);
        }
    }
}

template <typename T>
static void level_op(tm_hierarchy* h, int l, int op, const T* x, const T* b, T* y, const int* done,
                     hipStream_t s, const ChebArgs& ch = ChebArgs{}) {
    LaneIO io{};
    io.h = h;
    io.x = x;
    io.b = b;
    io.y = y;
    io.done = done;
    io.din = ch.din;
    io.dout = ch.dout;
    level_op_b<T>(l, op, &io, 1, s, ch.c1, ch.c2);
}

// largest eigenvalue of D^-1 A on level l: 12 power steps from a hashed start
// vector (zero on supported dofs), lambda = ||D^-1 A v|| / ||v||, v <- D^-1 A v
// (FP64; block sums added on the host in a fixed order)
// Interval of the Chebyshev smoother on level l: [lower, 1.1] x lambda, lambda
// from 12 power steps on D^-1 A in FP64 (start v_i = 1 + hash(i) / 2^16, zero on
// supported dofs; lambda = |D^-1 A v| / |v| at the last step).  Everything stays
// on the device: theta_l = lambda (lower + 1.1) / 2 goes to cheb_theta[l] and the
// level's D^-1 is divided by it.
// Chebyshev interval centre of level l from power steps on D^-1 A: 12 steps
// from the fixed start vector, or (warm) cheb_warm_steps steps from the level's
// last estimate vector.  A level with a kept vector saves its last iterate at
// unit length for the next design.
static void cheb_interval(tm_hierarchy* h, int l, hipStream_t s, bool warm) {
    Level& L = h->lv[l];
    const int64_t n0 = h->lv[0].n;
    double* v = h->pw;
    double* w = h->pw + n0;
    double* z = h->pw + 2 * n0;
    double* part = h->pw + 3 * n0;
    const int nb = (int)grid_for(L.n_nodes);
    // geometric levels keep their sizes for the hierarchy's life (a demotion
    // turns the last one into aggregation levels, which never keep a vector)
    const bool keep = h->cheb_v && l < (int)h->cheb_off.size() && L.kind != TM_LEVEL_AGGREGATION;
    double* kept = keep ? h->cheb_v + h->cheb_off[l] : nullptr;
    if (warm && keep)
        TM_HIP(hipMemcpyAsync(v, kept, (size_t)L.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    else
        launch_power_start(v, L.n, l == 0 ? L.nmask : nullptr, L.bs, s);
    const int steps = warm && keep ? h->opt.cheb_warm_steps : 12;
    for (int it = 0; it < steps; ++it) {
        level_op<double>(h, l, OP_APPLY, v, v, w, nullptr, s);
        launch_power_step(L, w, v, z, part, s);
        std::swap(v, z);
    }
    launch_cheb_theta(part, nb, 0.5 * (h->opt.cheb_lower + 1.1), h->cheb_theta + l,
                      keep ? h->cheb_ninv + l : nullptr, s);
    if (keep) launch_scale_copy(v, kept, L.n, h->cheb_ninv + l, s);
    launch_scale_dinv(L, h->cheb_theta + l, s);
}

// restriction from level l for lanes io (x: fine residual, y: coarse right-hand
// side, y2: the coarse level's first sweep, or NULL at the coarsest level)
template <typename T>
static void restrict_b(int l, const LaneIO* io, int n, hipStream_t s) {
    const tm_hierarchy* h = io[0].h;
    const T w = (T)first_sweep_weight(h, l + 1);
    if (h->lv[l].xfer_bsr) {
        for (int q = 0; q < n; ++q)
            launch_bsr_restrict<T>(io[q].h->lv[l], (const T*)io[q].x, (T*)io[q].y, io[q].h->lv[l + 1], (T*)io[q].y2, w,
                                   io[q].done, s);
    } else {
        launch_restrict_b<T>(l, io, n, w, s);
    }
}

// prolongation to level l for lanes io (x: coarse correction, y: fine iterate)
template <typename T>
static void prolong_b(int l, const LaneIO* io, int n, hipStream_t s) {
    const tm_hierarchy* h = io[0].h;
    if (h->lv[l].xfer_bsr) {
        for (int q = 0; q < n; ++q)
            launch_bsr_prolong<T>(io[q].h->lv[l], (const T*)io[q].x, (T*)io[q].y, io[q].done, s);
    } else {
        launch_prolong_b<T>(l, io, n, s);
    }
}

// One lane of a batched V-cycle: its hierarchy, work vectors, input (level 0)
// and output.  The lanes of one call share their level structure.
template <typename T>
struct VLane {
    tm_hierarchy* h;
    Vcyc* V;
    const T* b0;
    T* z;
    const int* done;
};

// z = V(b0) on level 0 (Algorithm 1 from x = 0) for every lane, each operation
// one launch for all lanes.  Work vectors of level l: V.b[l] (l > 0), V.x[l],
// V.t[l].  The last post-smoothing sweep writes z.  With first_done the fine
// level's first sweep was produced by the u, r update.
template <typename T>
static void vcycle_b(const VLane<T>* lanes, int n, hipStream_t s, bool first_done = false) {
    tm_hierarchy* h0 = lanes[0].h;
    const int L = (int)h0->lv.size();
    const int npre = h0->opt.nu_pre, npost = h0->opt.nu_post;
    const bool cheb = h0->opt.smoother == TM_SMOOTH_CHEBYSHEV;
    // per level and lane: the iterate and the scratch vector (swapped after each sweep)
    std::vector<std::vector<T*>> xr(L, std::vector<T*>(n)), tr(L, std::vector<T*>(n));
    std::vector<LaneIO> io(n);
    for (int q = 0; q < n; ++q) {
        io[q] = LaneIO{};
        io[q].h = lanes[q].h;
        io[q].done = lanes[q].done;
    }
    auto bvec = [&](int l, int q) -> T* { return l == 0 ? const_cast<T*>(lanes[q].b0) : vb<T>(*lanes[q].V, l); };
    // Chebyshev step k on level l (k = 0: from the current iterate with no
    // previous direction): coefficients of d_k = c1 d_{k-1} + c2 D^-1 r_k.
    // After a zero start the direction d_0 is the first iterate itself.
    // The stored D^-1 is divided by theta_l, so c2 here is the textbook one
    // times theta_l; with sigma = theta / delta = (1.1 + lower) / (1.1 - lower)
    // neither coefficient depends on the eigenvalue estimate.
    auto cheb_coef = [&](int k, double& c1, double& c2) {
        const double lo = h0->opt.cheb_lower, sigma = (1.1 + lo) / (1.1 - lo);
        double rho = 1.0 / sigma;
        c1 = 0.0;
        c2 = 1.0;
        for (int q = 1; q <= k; ++q) {
            const double rn = 1.0 / (2.0 * sigma - rho);
            c1 = rn * rho;
            c2 = 2.0 * rn * sigma;
            rho = rn;
        }
        if (k == 0) c1 = 0.0;
    };
    // one smoothing step on level l from the lanes' x into dst (dst(q))
    auto smooth = [&](int l, int k, bool zero_start, bool last, const std::vector<T*>& x,
                      const std::vector<T*>& dst) {
        double c1 = 0.0, c2 = 0.0;
        if (cheb) cheb_coef(k, c1, c2);
        for (int q = 0; q < n; ++q) {
            io[q].x = x[q];
            io[q].b = bvec(l, q);
            io[q].y = dst[q];
            io[q].din = nullptr;
            io[q].dout = nullptr;
            if (cheb) {
                void* d = lanes[q].V->d[l];
                io[q].din = (k == 0 || (k == 1 && zero_start)) ? (const void*)x[q] : d;
                io[q].dout = last ? nullptr : d;     // the last step of a phase leaves no direction behind
            }
        }
        level_op_b<T>(l, cheb ? OP_CHEB : OP_SMOOTH, io.data(), n, s, c1, c2);
    };
    // a geometric transfer to the coarsest level is restricted inside the
    // coarsest solve's launch
    const bool tail_fused = restrict_solve_ok(h0);
    std::vector<T*> rlast(n, nullptr);
    for (int l = 0; l < L - 1; ++l) {
        std::vector<T*>& x = xr[l];
        std::vector<T*>& t = tr[l];
        for (int q = 0; q < n; ++q) {
            x[q] = vx<T>(*lanes[q].V, l);
            t[q] = vt<T>(*lanes[q].V, l);
        }
        if (l == 0 && !first_done) {
            for (int q = 0; q < n; ++q) {
                io[q].b = bvec(0, q);
                io[q].y = x[q];
            }
            launch_first_smooth_b<T>(0, io.data(), n, (T)first_sweep_weight(h0, 0), s);
        }
        for (int k = 1; k < npre; ++k) {
            // from a zero start the first step's direction is the first iterate
            smooth(l, k, true, k == npre - 1, x, t);
            std::swap(x, t);
        }
        for (int q = 0; q < n; ++q) {
            io[q].x = x[q];
            io[q].b = bvec(l, q);
            io[q].y = t[q];
            io[q].din = nullptr;
            io[q].dout = nullptr;
        }
        level_op_b<T>(l, OP_RESID, io.data(), n, s);
        if (l == L - 2 && tail_fused) {
            for (int q = 0; q < n; ++q) rlast[q] = t[q];
            break;
        }
        for (int q = 0; q < n; ++q) {
            io[q].x = t[q];
            io[q].y = vb<T>(*lanes[q].V, l + 1);
            io[q].y2 = (l + 1 < L - 1) ? vx<T>(*lanes[q].V, l + 1) : nullptr;
        }
        restrict_b<T>(l, io.data(), n, s);
        for (int q = 0; q < n; ++q) io[q].y2 = nullptr;
    }
    for (int q = 0; q < n; ++q) {
        io[q].x = tail_fused ? rlast[q] : vb<T>(*lanes[q].V, L - 1);
        io[q].y = vx<T>(*lanes[q].V, L - 1);
        xr[L - 1][q] = vx<T>(*lanes[q].V, L - 1);
    }
    if (tail_fused)
        launch_restrict_solve_b<T>(io.data(), n, s);
    else
        launch_dense_solve_b<T>(io.data(), n, s);
    for (int l = L - 2; l >= 0; --l) {
        std::vector<T*>& x = xr[l];
        std::vector<T*>& t = tr[l];
        // small geometric levels below a geometric level, and the 3D fine level
        // in the FP32 tensor form, take the prolongation inside their first
        // post-smoothing step
        const bool fine_fused = l == 0 && std::is_same<T, float>::value && fine_pro_ok(h0);
        const bool fused = fine_fused || stencil_pro_ok(h0, l);
        if (!fused) {
            for (int q = 0; q < n; ++q) {
                io[q].x = xr[l + 1][q];
                io[q].y = x[q];
            }
            prolong_b<T>(l, io.data(), n, s);
        }
        for (int k = 0; k < npost; ++k) {
            const bool to_z = l == 0 && k == npost - 1;
            std::vector<T*> dst(n);
            for (int q = 0; q < n; ++q) dst[q] = to_z ? lanes[q].z : t[q];
            if (fused && k == 0) {
                double c1 = 0.0, c2 = 0.0;
                if (cheb) cheb_coef(0, c1, c2);
                for (int q = 0; q < n; ++q) {
                    io[q].x = x[q];
                    io[q].xc = xr[l + 1][q];
                    io[q].b = bvec(l, q);
                    io[q].y = dst[q];
                    io[q].din = nullptr;
                    io[q].dout = cheb && npost > 1 ? lanes[q].V->d[l] : nullptr;
                }
                if (fine_fused) {
                    hipEvent_t e0 = nullptr;
                    timed_begin(h0, 1, s, &e0);
                    launch_fine_pro_b(cheb ? OP_CHEB : OP_SMOOTH, io.data(), n, (float)h0->opt.omega, c1, c2, s);
                    timed_end(h0, 1, s, e0);
                } else
                    launch_stencil_pro_b<T>(l, cheb ? OP_CHEB : OP_SMOOTH, io.data(), n, (T)h0->opt.omega, c1, c2, s);
                for (int q = 0; q < n; ++q) io[q].xc = nullptr;
            } else {
                smooth(l, k, false, k == npost - 1, x, dst);
            }
            if (!to_z) std::swap(x, t);
        }
    }
}

template <typename T>
static void vcycle(tm_hierarchy* h, Vcyc& V, const T* b0, T* z, const int* done, hipStream_t s,
                   bool first_done = false) {
    const VLane<T> ln{h, &V, b0, z, done};
    vcycle_b<T>(&ln, 1, s, first_done);
}

template <typename T>
static void alloc_vcyc(tm_hierarchy* h, Vcyc& V, std::vector<void*>& list, size_t& bytes) {
    const int L = (int)h->lv.size();
    V.b.assign(L, nullptr);
    V.x.assign(L, nullptr);
    V.t.assign(L, nullptr);
    V.d.assign(L, nullptr);
    V.cap.assign(L, 0);
    const bool cheb = h->opt.smoother == TM_SMOOTH_CHEBYSHEV;
    for (int l = 0; l < L; ++l) {
        const size_t n = (size_t)h->lv[l].n;
        V.cap[l] = (int64_t)n;
        if (l > 0) V.b[l] = dalloc<T>(h, list, bytes, n);
        V.x[l] = dalloc<T>(h, list, bytes, n);
        if (l < L - 1) V.t[l] = dalloc<T>(h, list, bytes, n);
        if (cheb && l < L - 1) V.d[l] = dalloc<T>(h, list, bytes, n);
    }
}

}  // namespace tmi

// ============================================================================ solve states
namespace tmi {

static bool mixed_of(const tm_hierarchy* h) { return h->opt.vcycle_fp == 32; }

// partial-sum slots per quantity: every kernel that writes block partials
// launches one of these three grids
static int nparts_cap(const tm_hierarchy* h) {
    return std::max({fine_op_blocks(h), update_ur_blocks(h), krylov_blocks(h->n_dof)});
}

static tm_solve_state* new_state(tm_hierarchy* h, int nrhs) {
    auto* st = new tm_solve_state();
    st->h = h;
    st->nrhs = nrhs;
    const int64_t n = h->n_dof;
    const bool mixed = mixed_of(h);
    try {
        for (int k = 0; k < nrhs; ++k) {
            Lane* ln = new Lane();
            st->lanes.push_back(ln);
            ln->f = dalloc<double>(h, st->allocs, st->bytes, n);
            ln->r = dalloc<double>(h, st->allocs, st->bytes, n);
            ln->p = dalloc<double>(h, st->allocs, st->bytes, n);
            ln->q = dalloc<double>(h, st->allocs, st->bytes, n);
            ln->part = dalloc<double>(h, st->allocs, st->bytes, (size_t)2 * nparts_cap(h));
            if (mixed) {
                ln->r32 = dalloc<float>(h, st->allocs, st->bytes, n);
                ln->z32 = dalloc<float>(h, st->allocs, st->bytes, n);
                alloc_vcyc<float>(h, ln->v32, st->allocs, st->bytes);
            } else {
                ln->z64 = dalloc<double>(h, st->allocs, st->bytes, n);
                alloc_vcyc<double>(h, ln->v64, st->allocs, st->bytes);
            }
        }
        st->sc = dalloc<KScal>(h, st->allocs, st->bytes, nrhs);
        TM_HIP(hipMemset(st->sc, 0, sizeof(KScal) * nrhs));
        TM_HIP(hipHostMalloc((void**)&st->sc_host, sizeof(KScal) * nrhs, hipHostMallocDefault));
        TM_HIP(hipHostMalloc((void**)&st->flags_host, sizeof(int), hipHostMallocDefault));
        TM_HIP(hipEventCreateWithFlags(&st->ev, hipEventDisableTiming));
        TM_HIP(hipEventCreateWithFlags(&st->order, hipEventDisableTiming));
    } catch (...) {
        free_list(st->h, st->allocs);
        for (Lane* ln : st->lanes) delete ln;
        if (st->sc_host) (void)hipHostFree(st->sc_host);
        if (st->flags_host) (void)hipHostFree(st->flags_host);
        if (st->order) (void)hipEventDestroy(st->order);
        if (st->ev) (void)hipEventDestroy(st->ev);
        delete st;
        throw;
    }
    return st;
}

static void delete_state(tm_solve_state* st);

// a state's V-cycle vectors still serve the hierarchy's current levels (an
// update of aggregation levels may change their number or sizes)
static bool state_fits(const tm_hierarchy* h, const tm_solve_state* st) {
    const size_t L = h->lv.size();
    for (const Lane* ln : st->lanes) {
        const Vcyc& V = mixed_of(h) ? ln->v32 : ln->v64;
        if (V.cap.size() != L) return false;
        for (size_t l = 0; l < L; ++l)
            if (V.cap[l] < h->lv[l].n) return false;
    }
    return true;
}

// drop the states whose V-cycle work vectors follow the current level list
void delete_cached_state(tm_hierarchy* h) {
    if (!h) return;
    if (h->cached || !h->pool.empty()) (void)hipDeviceSynchronize();
    if (h->cached) {
        delete_state(h->cached);
        h->cached = nullptr;
    }
    for (tm_solve_state* st : h->pool) delete_state(st);
    h->pool.clear();
}

static void delete_state(tm_solve_state* st) {
    if (!st) return;
    free_list(st->h, st->allocs);
    for (Lane* ln : st->lanes) delete ln;
    if (st->sc_host) (void)hipHostFree(st->sc_host);
    if (st->flags_host) (void)hipHostFree(st->flags_host);
    if (st->ev) (void)hipEventDestroy(st->ev);
    if (st->order) (void)hipEventDestroy(st->order);
    delete st;
}

// the lanes of a state (one per right-hand side) as batched-launch lanes
static void state_lanes(tm_solve_state* st, std::vector<LaneIO>& out) {
    for (int k = 0; k < st->nrhs; ++k) {
        LaneIO l{};
        l.h = st->h;
        l.ln = st->lanes[k];
        l.sc = st->sc + k;
        l.done = &st->sc[k].done;
        l.part = st->lanes[k]->part;
        l.u = st->u + (size_t)k * st->h->n_dof;
        out.push_back(l);
    }
}

// z = V(r) for lanes io; with first_done the fine level's first sweep was
// produced by the u, r update
static void vcycle_lanes(const std::vector<LaneIO>& io, hipStream_t s, bool first_done) {
    const int n = (int)io.size();
    tm_hierarchy* h = const_cast<tm_hierarchy*>(io[0].h);
    if (mixed_of(h)) {
        std::vector<VLane<float>> v(n);
        for (int q = 0; q < n; ++q)
            v[q] = VLane<float>{const_cast<tm_hierarchy*>(io[q].h), &io[q].ln->v32, io[q].ln->r32, io[q].ln->z32,
                                io[q].done};
        vcycle_b<float>(v.data(), n, s, first_done);
    } else {
        std::vector<VLane<double>> v(n);
        for (int q = 0; q < n; ++q)
            v[q] = VLane<double>{const_cast<tm_hierarchy*>(io[q].h), &io[q].ln->v64, io[q].ln->r, io[q].ln->z64,
                                 io[q].done};
        vcycle_b<double>(v.data(), n, s, first_done);
    }
}

static void enqueue_begin(tm_solve_state* st, const double* f, int use_u0) {
    tm_hierarchy* h = st->h;
    const int64_t n = h->n_dof;
    const bool mixed = mixed_of(h);
    hipStream_t s = st->s;
    std::vector<LaneIO> io;
    state_lanes(st, io);
    for (int k = 0; k < st->nrhs; ++k) {
        Lane& ln = *st->lanes[k];
        launch_mask_copy<double>(h, f + (size_t)k * n, ln.f, s);
        launch_fcg_init(h, ln, st->sc + k, use_u0, io[k].u, st->rtol, h->opt.max_iters, h->opt.outer, s);
        if (mixed) launch_cast(ln.r, ln.r32, n, s);
    }
    vcycle_lanes(io, s, false);
    launch_zdots_b(io.data(), st->nrhs, mixed, s);
    launch_finalize_b(io.data(), st->nrhs, krylov_blocks(n), FIN_BETA, s);
    for (int k = 0; k < st->nrhs; ++k) TM_HIP(hipMemsetAsync(st->lanes[k]->p, 0, n * sizeof(double), s));
    launch_update_p_b(io.data(), st->nrhs, mixed, s);
}

// one outer iteration for lanes io (hierarchies with the same level structure
// and options), every operation one launch for all lanes
static void enqueue_iteration_b(const std::vector<LaneIO>& lanes, hipStream_t s) {
    tm_hierarchy* h = const_cast<tm_hierarchy*>(lanes[0].h);
    const int n = (int)lanes.size();
    const int64_t nd = h->n_dof;
    const bool mixed = mixed_of(h);
    std::vector<LaneIO> io(lanes);
    for (int q = 0; q < n; ++q) {
        io[q].x = io[q].ln->p;
        io[q].b = io[q].ln->r;
        io[q].y = io[q].ln->q;
    }
    hipEvent_t e0 = nullptr;
    timed_begin(h, 0, s, &e0);
    launch_fine_op_b<double>(OP_QDOT, false, io.data(), n, 0.0, 0.0, 0.0, s);
    timed_end(h, 0, s, e0);
    launch_finalize_b(io.data(), n, fine_op_blocks(h), FIN_ALPHA, s);
    launch_update_ur_b(io.data(), n, mixed, s);
    launch_finalize_b(io.data(), n, update_ur_blocks(h), FIN_RR, s);
    vcycle_lanes(lanes, s, true);
    launch_zdots_b(io.data(), n, mixed, s);
    launch_finalize_b(io.data(), n, krylov_blocks(nd), FIN_BETA, s);
    launch_update_p_b(io.data(), n, mixed, s);
}

// the pinned mirror of the scalars (and of the device checks of an update
// that did not wait for them) and the completion event of a state, after its
// work enqueued on stream s
static void state_sync_point(tm_solve_state* st, hipStream_t s) {
    TM_HIP(hipMemcpyAsync(st->sc_host, st->sc, sizeof(KScal) * st->nrhs, hipMemcpyDeviceToHost, s));
    st->flags_copied = st->h->flags_pending;
    if (st->flags_copied) {
        TM_HIP(hipMemcpyAsync(st->flags_host, st->h->flags, sizeof(int), hipMemcpyDeviceToHost, s));
        st->flags_seq = st->h->update_seq;
    }
    TM_HIP(hipEventRecord(st->ev, s));
    if (s != st->s) TM_HIP(hipStreamWaitEvent(st->s, st->ev, 0));
    st->pending = true;
}

static void enqueue_advance(tm_solve_state* st, int k_iters) {
    std::vector<LaneIO> io;
    state_lanes(st, io);
    for (int it = 0; it < k_iters; ++it) enqueue_iteration_b(io, st->s);
    launch_final_residual_b(io.data(), (int)io.size(), true, st->s);
    state_sync_point(st, st->s);
}

// Lanes whose hierarchies can share launches: the same level list (kinds,
// sizes, block sizes, transfers, operator kernels, coarsest size) and the same
// solver options and element stiffness.
static std::string shape_key(const tm_hierarchy* h) {
    std::string k;
    auto put = [&](const void* p, size_t n) { k.append((const char*)p, n); };
    const tm_options& o = h->opt;
    const int ints[] = {h->dim, o.smoother, o.nu_pre, o.nu_post, o.vcycle_fp, o.outer, o.fine_mfma, o.fine_tensor,
                        (int)h->lv.size()};
    put(ints, sizeof(ints));
    const double dbl[] = {o.omega, o.cheb_lower};
    put(dbl, sizeof(dbl));
    put(&h->n_dof, sizeof(h->n_dof));
    put(&h->nc, sizeof(h->nc));
    put(h->kc64.k, sizeof(h->kc64.k));
    for (const Level& L : h->lv) {
        const int li[] = {L.kind, L.bs, L.nel[0], L.nel[1], L.nel[2], (int)L.xfer_bsr, L.op_kernel, L.subf ? 1 : 0};
        put(li, sizeof(li));
        put(&L.n, sizeof(L.n));
    }
    return k;
}

static bool state_done(tm_solve_state* st) {
    for (int k = 0; k < st->nrhs; ++k)
        if (!st->sc_host[k].done) return false;
    return true;
}

static void wait_state(tm_solve_state* st) {
    if (st->pending) {
        TM_HIP(hipEventSynchronize(st->ev));
        st->pending = false;
    }
}

// run to completion: chunks of iterations between host checks; the chunk
// length follows the observed convergence rate (extra iterations past the
// stop are empty launches).
static void run_to_completion(tm_solve_state* st) {
    tm_hierarchy* h = st->h;
    int k = h->opt.check_every > 0 ? h->opt.check_every : 6;
    double last_rr = -1.0;
    int last_iter = 0;
    for (;;) {
        enqueue_advance(st, k);
        wait_state(st);
        if (state_done(st)) break;
        if (h->opt.check_every > 0) continue;
        // adapt: estimate iterations left for the slowest right-hand side
        double need = 2.0;
        for (int q = 0; q < st->nrhs; ++q) {
            const KScal& c = st->sc_host[q];
            if (c.done) continue;
            const int di = c.iter - last_iter;
            if (last_rr > 0.0 && di > 0 && c.rr < last_rr && c.rr > 0.0) {
                const double rate = std::log(c.rr / last_rr) / di;         // per iteration (< 0)
                need = std::max(need, std::log(c.rr_stop / c.rr) / rate);
            } else {
                need = std::max(need, (double)k);
            }
        }
        last_rr = st->sc_host[0].rr;
        last_iter = st->sc_host[0].iter;
        k = (int)std::min(64.0, std::max(2.0, std::ceil(need)));
    }
}

static tm_status finish_state(tm_solve_state* st, int32_t* iters, double* compliance, double* relres) {
    tm_hierarchy* h = st->h;
    wait_state(st);
    // the last batch of iterations left the outputs of every right-hand side
    // (and the device checks of the last update, if pending) in the host
    // mirror: nothing to launch or wait for
    bool have = true;
    for (int k = 0; k < st->nrhs; ++k)
        if (!st->sc_host[k].fin) have = false;
    if (h->flags_pending && !(st->flags_copied && st->flags_seq == h->update_seq)) have = false;
    int fl = 0;
    if (have) {
        if (h->flags_pending) fl = *st->flags_host;
    } else {
        std::vector<LaneIO> io;
        state_lanes(st, io);
        launch_final_residual_b(io.data(), (int)io.size(), false, st->s);
        TM_HIP(hipMemcpyAsync(st->sc_host, st->sc, sizeof(KScal) * st->nrhs, hipMemcpyDeviceToHost, st->s));
        if (h->flags_pending) TM_HIP(hipMemcpyAsync(&fl, h->flags, sizeof(int), hipMemcpyDeviceToHost, st->s));
        TM_HIP(hipStreamSynchronize(st->s));
    }
    if (h->flags_pending) {
        // device checks of the last density update, which did not wait for them
        h->flags_pending = false;
        st->ended = true;
        if (fl & FLAG_BAD_RHO) fail(TM_ERR_ARG, "densities of the last update must be finite and in [0, 1]");
        if (fl & FLAG_NOT_SPD) fail(TM_ERR_NOT_SPD, "operator of the last update not positive definite");
    }
    tm_status worst = TM_OK;
    for (int k = 0; k < st->nrhs; ++k) {
        const KScal& c = st->sc_host[k];
        if (iters) iters[k] = c.iter;
        if (h->opt.adapt_iters > 0 && c.iter > h->opt.adapt_iters) h->demote = true;
        if (compliance) compliance[k] = c.zq;
        if (relres) relres[k] = c.ff > 0.0 ? std::sqrt(c.pq / c.ff) : 0.0;
        const tm_status stt = (tm_status)c.status;
        if (stt < 0) {
            worst = stt;
            set_error("right-hand side " + std::to_string(k) + " at iteration " + std::to_string(c.iter) + ": " +
                      (stt == TM_ERR_ARG ? "load or start vector not finite"
                                         : "breakdown (p^T K p <= 0, z^T r <= 0 or a non-finite value)"));
        } else if (stt == TM_NOT_CONVERGED && worst == TM_OK) {
            worst = TM_NOT_CONVERGED;
        }
    }
    st->ended = true;
    return worst;
}

}  // namespace tmi

// ============================================================================ exports helpers
namespace tmi {

static const Level& level_at(const tm_hierarchy* h, int level) {
    if (!h) fail(TM_ERR_ARG, "hierarchy is NULL");
    if (level < 0 || level >= (int)h->lv.size()) fail(TM_ERR_ARG, "level out of range");
    return h->lv[level];
}

// CSR of a geometric level from its FP64 stencil (host copy)
static void stencil_csr(const Level& L, std::vector<int64_t>& rp, std::vector<int32_t>& ci,
                        std::vector<double>& v, bool want_values) {
    const int dim = L.dim, bb = dim * dim;
    std::vector<double> st;
    if (want_values) {
        st.resize((size_t)L.nst * bb * L.n_nodes);
        TM_HIP(hipMemcpy(st.data(), L.st64, st.size() * sizeof(double), hipMemcpyDeviceToHost));
    }
    rp.assign(L.n + 1, 0);
    ci.clear();
    v.clear();
    const int NX = L.nn[0], NY = L.nn[1], NZ = dim == 3 ? L.nn[2] : 1;
    for (int64_t node = 0; node < L.n_nodes; ++node) {
        const int i = (int)(node % NX), j = (int)((node / NX) % NY), k = (int)(node / ((int64_t)NX * NY));
        for (int r = 0; r < dim; ++r) {
            for (int dz = (dim == 3 ? -1 : 0); dz <= (dim == 3 ? 1 : 0); ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int ii = i + dx, jj = j + dy, kk = k + dz;
                        if (ii < 0 || ii >= NX || jj < 0 || jj >= NY || kk < 0 || kk >= NZ) continue;
                        const int o = dim == 3 ? (dz + 1) * 9 + (dy + 1) * 3 + dx + 1 : (dy + 1) * 3 + dx + 1;
                        const int64_t J = ((int64_t)kk * NY + jj) * NX + ii;
                        for (int c = 0; c < dim; ++c) {
                            ci.push_back((int32_t)(dim * J + c));
                            if (want_values) v.push_back(st[((size_t)o * bb + r * dim + c) * L.n_nodes + node]);
                        }
                    }
            rp[dim * node + r + 1] = (int64_t)ci.size();
        }
    }
}

static void bsr_csr(const BSR& B, std::vector<int64_t>& rp, std::vector<int32_t>& ci,
                    std::vector<double>& v) {
    std::vector<int32_t> brp(B.nbr + 1), bci(B.nnzb);
    std::vector<double> bv((size_t)B.nnzb * B.br * B.bc);
    TM_HIP(hipMemcpy(brp.data(), B.rp, brp.size() * 4, hipMemcpyDeviceToHost));
    if (B.nnzb) {
        TM_HIP(hipMemcpy(bci.data(), B.ci, bci.size() * 4, hipMemcpyDeviceToHost));
        TM_HIP(hipMemcpy(bv.data(), B.v64, bv.size() * 8, hipMemcpyDeviceToHost));
    }
    rp.assign(B.nbr * B.br + 1, 0);
    ci.clear();
    v.clear();
    for (int64_t br = 0; br < B.nbr; ++br)
        for (int r = 0; r < B.br; ++r) {
            for (int32_t q = brp[br]; q < brp[br + 1]; ++q)
                for (int c = 0; c < B.bc; ++c) {
                    ci.push_back((int32_t)((int64_t)bci[q] * B.bc + c));
                    v.push_back(bv[((size_t)q * B.br + r) * B.bc + c]);
                }
            rp[br * B.br + r + 1] = (int64_t)ci.size();
        }
}

// geometric prolongator from level l+1 to level l (host), supported fine dofs dropped on level 0
static void geo_prolongator(const tm_hierarchy* h, int l, std::vector<int64_t>& rp,
                            std::vector<int32_t>& ci, std::vector<double>& v) {
    const Level& F = h->lv[l];
    const Level& C = h->lv[l + 1];
    const int dim = F.dim;
    std::vector<uint8_t> nm;
    if (l == 0) {
        nm.resize(F.n_nodes);
        TM_HIP(hipMemcpy(nm.data(), F.nmask, F.n_nodes, hipMemcpyDeviceToHost));
    }
    rp.assign(F.n + 1, 0);
    ci.clear();
    v.clear();
    const int FX = F.nn[0], FY = F.nn[1];
    const int CX = C.nn[0], CY = C.nn[1];
    // per axis: fine node i lies on coarse node i/2 (even i), halfway between
    // (i-1)/2 and (i+1)/2 (odd i), or, for the last node of an odd count, on
    // the last coarse node
    auto parents = [](int i, int nf, int* I, double* w) {
        if ((nf & 1) && i == nf) {
            I[0] = (nf + 1) / 2;
            w[0] = 1.0;
            return 1;
        }
        if (!(i & 1)) {
            I[0] = i / 2;
            w[0] = 1.0;
            return 1;
        }
        I[0] = (i - 1) / 2;
        I[1] = (i + 1) / 2;
        w[0] = w[1] = 0.5;
        return 2;
    };
    for (int64_t node = 0; node < F.n_nodes; ++node) {
        const int i = (int)(node % FX), j = (int)((node / FX) % FY), k = (int)(node / ((int64_t)FX * FY));
        int Ix[2], Iy[2], Iz[2] = {0, 0};
        double wx[2], wy[2], wz[2] = {1.0, 0.0};
        const int nx = parents(i, F.nel[0], Ix, wx), ny = parents(j, F.nel[1], Iy, wy);
        const int nz = dim == 3 ? parents(k, F.nel[2], Iz, wz) : 1;
        for (int r = 0; r < dim; ++r) {
            const bool dropped = l == 0 && (nm[node] & (1u << r));
            if (!dropped) {
                // coarse nodes in ascending id order: z, then y, then x
                for (int c2 = 0; c2 < nz; ++c2)
                    for (int b2 = 0; b2 < ny; ++b2)
                        for (int a2 = 0; a2 < nx; ++a2) {
                            const double w = wx[a2] * wy[b2] * wz[c2];
                            const int64_t Cn = ((int64_t)Iz[c2] * CY + Iy[b2]) * CX + Ix[a2];
                            ci.push_back((int32_t)(dim * Cn + r));
                            v.push_back(w);
                        }
            }
            rp[dim * node + r + 1] = (int64_t)ci.size();
        }
    }
}

}  // namespace tmi

// ============================================================================ stability eigenproblem
namespace tmi {

void free_eig_work(tm_hierarchy* h) {
    if (!h->eig) return;
    (void)hipDeviceSynchronize();
    if (h->eig->host) (void)hipHostFree(h->eig->host);
    free_list(h, h->eig->allocs);
    delete h->eig;
    h->eig = nullptr;
}

// pinned host staging: [0, 33) reduced sums (device to host), then 32
// coefficients and a 32 x 32 block (host to device)
constexpr int EIG_PIN_COEF = EIG_MAX_COLS + 1;
constexpr int EIG_PIN_Y = EIG_PIN_COEF + EIG_MAX_COLS;
constexpr int EIG_PIN_N = EIG_PIN_Y + EIG_MAX_COLS * EIG_MAX_COLS;

static EigWork* eig_work(tm_hierarchy* h, int jmax, int fp) {
    if (h->eig && h->eig->jmax >= jmax && h->eig->fp == fp && h->eig->n == h->n_dof) return h->eig;
    free_eig_work(h);
    auto* w = new EigWork();
    h->eig = w;
    try {
        const size_t n = (size_t)h->n_dof;
        w->n = h->n_dof;
        w->jmax = jmax;
        w->fp = fp;
        auto A = [&](size_t k) { return dalloc<double>(h, w->allocs, w->bytes, k); };
        w->V = A(n * (size_t)jmax);
        w->q = A(n);
        w->Aq = A(n);
        w->Bq = A(n);
        w->r = A(n);
        w->z = A(n);
        w->w = A(n);
        w->part = A((size_t)EIG_BLOCKS * (EIG_MAX_COLS + 1));
        w->red = A(EIG_MAX_COLS + 1);
        w->coef = A(EIG_MAX_COLS);
        w->Y = A(EIG_MAX_COLS * EIG_MAX_COLS);
        if (fp == 64) {
            alloc_vcyc<double>(h, w->vc, w->allocs, w->bytes);
        } else {
            w->r32 = dalloc<float>(h, w->allocs, w->bytes, n);
            w->z32 = dalloc<float>(h, w->allocs, w->bytes, n);
            alloc_vcyc<float>(h, w->vc, w->allocs, w->bytes);
        }
        TM_HIP(hipHostMalloc((void**)&w->host, EIG_PIN_N * sizeof(double), hipHostMallocDefault));
    } catch (...) {
        free_eig_work(h);
        throw;
    }
    return w;
}

// Eigenvalues (descending) and unit eigenvectors (columns of Y, n x n
// column-major) of a small symmetric matrix H (leading dimension ldh) by the
// cyclic Jacobi method in Rutishauser's form: each plane rotation zeroes one
// off-diagonal entry exactly and updates the two diagonal entries by +-t a_pq;
// after a few sweeps, entries that no longer change the diagonal in floating
// point are set to zero; the sweeps end when the off-diagonal part is zero.
static void sym_eig(int n, const std::vector<double>& H, int ldh, std::vector<double>& theta,
                    std::vector<double>& Y) {
    std::vector<double> A((size_t)n * n), Q((size_t)n * n, 0.0);
    auto a = [&](int i, int j) -> double& { return A[i + (size_t)n * j]; };
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) a(i, j) = 0.5 * (H[i + (size_t)ldh * j] + H[j + (size_t)ldh * i]);
    for (int i = 0; i < n; ++i) Q[i + (size_t)n * i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += std::fabs(a(p, q));
        if (off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a(p, q);
                const double g = 100.0 * std::fabs(apq);
                if (sweep > 3 && std::fabs(a(p, p)) + g == std::fabs(a(p, p)) &&
                    std::fabs(a(q, q)) + g == std::fabs(a(q, q))) {
                    a(p, q) = a(q, p) = 0.0;
                    continue;
                }
                if (apq == 0.0) continue;
                const double hd = a(q, q) - a(p, p);
                double t;
                if (std::fabs(hd) + g == std::fabs(hd)) {
                    t = apq / hd;
                } else {
                    const double th = 0.5 * hd / apq;
                    t = 1.0 / (std::fabs(th) + std::sqrt(1.0 + th * th));
                    if (th < 0.0) t = -t;
                }
                const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
                a(p, p) -= t * apq;
                a(q, q) += t * apq;
                a(p, q) = a(q, p) = 0.0;
                for (int r = 0; r < n; ++r) {
                    if (r == p || r == q) continue;
                    const double arp = a(r, p), arq = a(r, q);
                    a(r, p) = a(p, r) = c * arp - sn * arq;
                    a(r, q) = a(q, r) = sn * arp + c * arq;
                }
                for (int r = 0; r < n; ++r) {
                    const double qrp = Q[r + (size_t)n * p], qrq = Q[r + (size_t)n * q];
                    Q[r + (size_t)n * p] = c * qrp - sn * qrq;
                    Q[r + (size_t)n * q] = sn * qrp + c * qrq;
                }
            }
    }
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
        return A[x + (size_t)n * x] > A[y + (size_t)n * y];
    });
    theta.assign(n, 0.0);
    Y.assign((size_t)n * n, 0.0);
    for (int k = 0; k < n; ++k) {
        theta[k] = A[ord[k] + (size_t)n * ord[k]];
        for (int i = 0; i < n; ++i) Y[i + (size_t)n * k] = Q[i + (size_t)n * ord[k]];
    }
}

// Generalized Davidson for K_sigma~ x = theta K~ x (Algorithm 2).  The search
// space V lives on the device (column-major, ld = n_dof) and is K~-orthonormal;
// the projected matrix H = V^T K_sigma~ V (at most 32 x 32) and every decision
// live on the host, which reads a few reduced sums per step.
struct Davidson {
    tm_hierarchy* h;
    EigWork* w;
    hipStream_t s;
    int64_t n;
    int fp, jmax, j = 0;
    std::vector<double> H;                       // jmax x jmax, column-major

    double* col(int c) const { return w->V + (int64_t)c * n; }
    void applyA(const double* x, double* y) { launch_gsig_apply(h, h->gsig, x, y, s); }
    void applyB(const double* x, double* y) {
        launch_fine_op<double>(h, OP_APPLY, true, x, nullptr, y, 0.0, nullptr, nullptr, s);
    }
    // c[i] = V[:, i]^T v for i < nc, and z^T v when z is given
    void dots(int nc, const double* v, const double* z, double* c, double* zz) {
        launch_vtw(w->V, n, nc, v, z, n, w->part, w->red, s);
        TM_HIP(hipMemcpyAsync(w->host, w->red, (EIG_MAX_COLS + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
        TM_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < nc; ++i) c[i] = w->host[i];
        if (zz) *zz = w->host[EIG_MAX_COLS];
    }
    void upload(double* dst, const double* src, int cnt, int pin_off) {
        std::memcpy(w->host + pin_off, src, cnt * sizeof(double));
        TM_HIP(hipMemcpyAsync(dst, w->host + pin_off, cnt * sizeof(double), hipMemcpyHostToDevice, s));
    }
    void precond(const double* r, double* z) {
        if (fp == 64) {
            vcycle<double>(h, w->vc, r, z, nullptr, s);
        } else {
            launch_cast(r, w->r32, n, s);
            vcycle<float>(h, w->vc, w->r32, w->z32, nullptr, s);
            launch_cast_back(w->z32, z, n, s);
        }
    }
    // K~-orthonormalise z against V[:, :j] (classical Gram-Schmidt, repeated
    // once when the norm drops below 1/sqrt(2); the norm after a projection is
    // ||z||^2 - ||c||^2), store it as column j and extend H.  z is overwritten.
    // false: the vector is (numerically) in the span of V.
    bool append(double* z) {
        constexpr double ETA2 = 0.5, BREAK2 = 1e-20;
        double c[EIG_MAX_COLS + 1], coef[EIG_MAX_COLS], zz0 = 0.0, zz = 0.0, beta2 = 0.0;
        applyB(z, w->w);
        dots(j, w->w, z, c, &zz0);
        if (!(zz0 > 0.0)) return false;
        zz = zz0;
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1) {
                applyB(z, w->w);
                dots(j, w->w, z, c, &zz);
            }
            double cc = 0.0;
            for (int i = 0; i < j; ++i) cc += c[i] * c[i];
            beta2 = zz - cc;
            if (beta2 > ETA2 * zz || pass == 1) {
                if (!(beta2 > BREAK2 * zz0)) return false;
                const double inv = 1.0 / std::sqrt(beta2);
                for (int i = 0; i < j; ++i) coef[i] = -c[i] * inv;
                if (j > 0) upload(w->coef, coef, j, EIG_PIN_COEF);
                launch_vupdate(w->V, n, j, w->coef, inv, z, col(j), n, s);     // (z - V c) / beta
                break;
            }
            for (int i = 0; i < j; ++i) coef[i] = -c[i];
            upload(w->coef, coef, j, EIG_PIN_COEF);
            launch_vupdate(w->V, n, j, w->coef, 1.0, z, z, n, s);               // z - V c
        }
        applyA(col(j), w->Aq);
        double hc[EIG_MAX_COLS + 1];
        dots(j + 1, w->Aq, nullptr, hc, nullptr);
        for (int i = 0; i <= j; ++i) {
            H[i + (size_t)jmax * j] = hc[i];
            H[j + (size_t)jmax * i] = hc[i];
        }
        ++j;
        return true;
    }
};

static tm_status run_davidson(tm_hierarchy* h, const tm_eig_options& o, int32_t n_init, const double* v0,
                              double* lambda, double* phi, int32_t* iters_out, int32_t* nconv_out, hipStream_t s) {
    Davidson gd{h, eig_work(h, o.j_max, o.precond_fp), s, h->n_dof, o.precond_fp, o.j_max};
    EigWork* w = gd.w;
    const int64_t n = gd.n;
    gd.H.assign((size_t)o.j_max * o.j_max, 0.0);
    for (int i = 0; i < n_init; ++i) {
        launch_mask_copy<double>(h, v0 + (int64_t)i * n, w->z, s);
        if (!gd.append(w->z)) fail(TM_ERR_ARG, "start vectors are dependent in the K inner product");
    }
    std::vector<double> theta, Y;
    int k = 0, it = 0;
    bool have_prev = false;
    double prev = 0.0;
    for (;;) {
        sym_eig(gd.j, gd.H, o.j_max, theta, Y);
        while (k < o.nev) {
            // Ritz vector q = V y_k, residual r = K_s q - theta K q
            gd.upload(w->coef, Y.data() + (size_t)gd.j * k, gd.j, EIG_PIN_COEF);
            launch_vupdate(w->V, n, gd.j, w->coef, 0.0, nullptr, w->q, n, s);
            gd.applyA(w->q, w->Aq);
            gd.applyB(w->q, w->Bq);
            launch_eig_resid(w->Aq, w->Bq, theta[k], w->r, n, w->part, w->red, s);
            TM_HIP(hipMemcpyAsync(w->host, w->red, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
            TM_HIP(hipStreamSynchronize(s));
            const double rn = std::sqrt(w->host[0]), den = std::fabs(theta[k]) * std::sqrt(w->host[1]);
            const double rel = den > 0.0 ? rn / den : (rn == 0.0 ? 0.0 : HUGE_VAL);
            const bool stag = have_prev && std::fabs(theta[k] - prev) < o.stag_tol * std::fabs(theta[k]);
            if (rel < o.tol || stag) {
                ++k;
                have_prev = false;
                continue;
            }
            break;
        }
        if (k == o.nev || it >= o.max_iters) break;
        prev = theta[k];
        have_prev = true;
        if (gd.j == o.j_max) {
            // restart: keep the j_min leading Ritz vectors
            gd.upload(w->Y, Y.data(), gd.j * o.j_min, EIG_PIN_Y);
            launch_vrotate(w->V, n, gd.j, w->Y, o.j_min, w->V, n, n, s);
            std::fill(gd.H.begin(), gd.H.end(), 0.0);
            for (int i = 0; i < o.j_min; ++i) gd.H[i + (size_t)o.j_max * i] = theta[i];
            gd.j = o.j_min;
        }
        gd.precond(w->r, w->z);
        ++it;
        if (!gd.append(w->z)) fail(TM_ERR_BREAKDOWN, "search space breakdown: the correction lies in the search space");
    }
    sym_eig(gd.j, gd.H, o.j_max, theta, Y);
    for (int i = 0; i < o.nev; ++i) lambda[i] = theta[i];
    if (phi) {
        gd.upload(w->Y, Y.data(), gd.j * o.nev, EIG_PIN_Y);
        launch_vrotate(w->V, n, gd.j, w->Y, o.nev, phi, n, n, s);
    }
    TM_HIP(hipStreamSynchronize(s));
    if (iters_out) *iters_out = it;
    if (nconv_out) *nconv_out = k;
    return k == o.nev ? TM_OK : TM_NOT_CONVERGED;
}

}  // namespace tmi

// ============================================================================ C ABI
extern "C" {

void tm_default_options(tm_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->n_levels = 0;
    o->n_geometric = 0;
    o->max_coarse = 1000;
    o->smoother = TM_SMOOTH_BLOCK_JACOBI;
    o->nu_pre = 1;
    o->nu_post = 1;
    o->omega = 0.5;
    o->sa_beta = 0.003;
    o->vcycle_fp = 32;
    o->outer = TM_OUTER_FCG;
    o->max_iters = 1000;
    o->check_every = 0;
    o->fine_mfma = 0;
    o->cheb_lower = 0.1;
    o->adapt_iters = 0;
    o->cheb_warm_steps = 0;
    o->stencil_kernel = 0;
    o->sa_lds = 0;
    o->fine_tensor = 1;
}

const char* tm_status_string(tm_status s) {
    switch (s) {
        case TM_OK: return "ok";
        case TM_NOT_CONVERGED: return "not converged";
        case TM_ERR_ARG: return "invalid argument";
        case TM_ERR_OOM: return "out of device memory";
        case TM_ERR_DEVICE: return "device error";
        case TM_ERR_NOT_SPD: return "operator not positive definite";
        case TM_ERR_BREAKDOWN: return "Krylov breakdown";
        case TM_ERR_STATE: return "call out of order";
    }
    return "unknown status";
}

const char* tm_last_error(void) { return tmi::g_last_error.c_str(); }

tm_status tm_plan_bytes(const tm_mesh* mesh, const tm_options* opts, int32_t n_rhs, size_t* bytes) {
    return guarded([&] {
        check_mesh(mesh);
        check_opts(opts);
        if (n_rhs < 0) fail(TM_ERR_ARG, "n_rhs must be >= 0");
        if (!bytes) fail(TM_ERR_ARG, "bytes is NULL");
        const Plan p = plan_levels(mesh, opts);
        const int dim = mesh->dim, bb = dim * dim, nd = dim * (1 << dim);
        const int64_t n_el = (int64_t)mesh->nel[0] * mesh->nel[1] * (dim == 3 ? mesh->nel[2] : 1);
        const int64_t nodes0 = nodes_of(mesh->nel, dim);
        // moduli FP64 + FP32, densities FP64, support mask, block inverses FP64 + FP32
        size_t b = (size_t)n_el * 20 + nodes0 * (1 + sym_n(dim) * 12);
        size_t vec = 0, el1 = 0, el2 = 0;
        const bool cheb = opts->smoother == TM_SMOOTH_CHEBYSHEV;
        const size_t vw = opts->vcycle_fp == 32 ? 4 : 8;
        size_t cheb_dir = cheb ? (size_t)nodes0 * dim * vw : 0;    // Chebyshev directions, per RHS
        int nel[3] = {mesh->nel[0], mesh->nel[1], dim == 3 ? mesh->nel[2] : 1};
        const bool mixed = opts->vcycle_fp == 32;
        int64_t last_n = nodes0 * dim;
        for (int l = 1; l < p.Lg; ++l) {
            for (int d = 0; d < dim; ++d) nel[d] = (nel[d] + 1) / 2;
            const int64_t nn = nodes_of(nel, dim);
            const int64_t ne = (int64_t)nel[0] * nel[1] * (dim == 3 ? nel[2] : 1);
            const int nst = dim == 3 ? 27 : 9, nq = (nst - 1) / 2 * bb + dim * (dim + 1) / 2;
            b += (size_t)nn * (bb * 8 * nst + 12 * nq + 12 * sym_n(dim));
            vec += (size_t)nn * dim * (mixed ? 4 : 8) * 3;
            if (cheb && l + 1 < p.Lg) cheb_dir += (size_t)nn * dim * vw;
            if (l == 1) el1 = (size_t)ne * nd * nd * 8;
            if (l == 2) el2 = (size_t)ne * nd * nd * 8;
            last_n = nn * dim;
        }
        if (p.sa) last_n = std::min<int64_t>(last_n, opts->max_coarse * 8);
        b += (size_t)last_n * last_n * 8 * 2 + el1 + el2 + (size_t)(dim == 3 ? 27 : 9) * nd * nd * 8;
        if (opts->smoother == TM_SMOOTH_CHEBYSHEV) b += (size_t)nodes0 * dim * 8 * 3 + (size_t)nodes0 / 16 + 1024;
        if (opts->smoother == TM_SMOOTH_CHEBYSHEV && opts->cheb_warm_steps > 0) b += (size_t)nodes0 * dim * 8 * 2;
        const size_t per_rhs = (size_t)nodes0 * dim * (8 * 4 + (mixed ? 4 * 4 : 8 * 3)) + vec + cheb_dir;
        // every allocation may be rounded up (allocator granularity, partial
        // sums, scalars): one 4 KiB page per allocation of the hierarchy
        // (about 8 per level) and of each right-hand side (about 5 per level)
        const int L_est = p.Lg + (p.sa ? 4 : 0);
        const size_t n_alloc = 32 + 8 * (size_t)L_est + (size_t)n_rhs * (8 + 5 * (size_t)L_est);
        *bytes = b + per_rhs * (size_t)n_rhs + n_alloc * 4096;
    });
}

static void destroy_impl(tm_hierarchy* h) {
    if (!h) return;
    h->cur_stream = nullptr;       // the caller's streams may be gone by now
    tmi::delete_cached_state(h);
    tmi::free_eig_work(h);
    for (int c = 0; c < 3; ++c)
        for (auto& pr : h->tev[c]) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    tmi::free_list(h, h->allocs);
    tmi::arena_release(h, h->sa_keep);
    tmi::arena_release(h, h->sa_tmp);
    tmi::arena_release(h, h->sa_cand[0]);
    tmi::arena_release(h, h->sa_cand[1]);
    delete h;
}

tm_status tm_setup(const tm_mesh* mesh, const tm_material* mat, const double* rho_dev,
                   const tm_bcs* bcs, const tm_options* opts, const tm_allocator* alloc, void* stream,
                   tm_hierarchy** out) {
    tm_hierarchy* h = nullptr;
    tm_status st = guarded([&] {
        if (!out) fail(TM_ERR_ARG, "out is NULL");
        *out = nullptr;
        check_mesh(mesh);
        check_material(mat);
        check_opts(opts);
        if (!rho_dev) fail(TM_ERR_ARG, "rho_dev is NULL");
        if (alloc && (!alloc->alloc || !alloc->free)) fail(TM_ERR_ARG, "allocator needs both alloc and free");
        const Plan plan = plan_levels(mesh, opts);
        const int dim = mesh->dim;
        const int64_t n_nodes = nodes_of(mesh->nel, dim), n_dof = n_nodes * dim;
        std::vector<int64_t> fixed;
        if (bcs && bcs->n > 0) {
            if (!bcs->dofs) fail(TM_ERR_ARG, "bcs.dofs is NULL");
            fixed.assign(bcs->dofs, bcs->dofs + bcs->n);
            for (int64_t d : fixed)
                if (d < 0 || d >= n_dof) fail(TM_ERR_ARG, "support dof id out of range");
            std::sort(fixed.begin(), fixed.end());
            fixed.erase(std::unique(fixed.begin(), fixed.end()), fixed.end());
        }
        if (plan.Lg < 2 && !plan.sa) fail(TM_ERR_ARG, "a hierarchy needs at least two levels");
        hipStream_t s = S(stream);
        h = new tm_hierarchy();
        if (alloc) {
            h->alloc = *alloc;
            h->has_alloc = true;
        }
        h->cur_stream = s;
        h->mesh = *mesh;
        if (dim == 2) h->mesh.nel[2] = 1;
        h->mat = *mat;
        h->opt = *opts;
        h->dim = dim;
        h->n_el = (int64_t)mesh->nel[0] * mesh->nel[1] * (dim == 3 ? mesh->nel[2] : 1);
        h->n_nodes = n_nodes;
        h->n_dof = n_dof;
        h->fixed = fixed;
        h->flags = halloc<int>(h, 4);
        // constants
        std::vector<double> KE;
        element_stiffness(dim, mat->nu, mesh->h, KE);
        if (dim == 3) {
            ke_class_values(KE_CLS3, KE, h);
            ke_tensor_coefs(KE, h);
        } else {
            ke_class_values(KE_CLS2, KE, h);
        }
        h->KE64 = halloc<double>(h, KE.size());
        h->rho64 = halloc<double>(h, (size_t)h->n_el);
        // A operand of the matrix-core operator: register q, lane L holds row
        // L mod 4 (row 3 = 0) of KE column k = 16 q + L/4, k = 24 a + col for
        // element corner slot a; entries rebuilt from the class values
        std::vector<float> KA32;
        if (dim == 3) {
            KA32.assign(12 * 64, 0.f);
            for (int q = 0; q < 12; ++q)
                for (int L = 0; L < 64; ++L) {
                    const int kk = 16 * q + L / 4, a = kk / 24, col = kk % 24, row = L % 4;
                    if (row == 3) continue;
                    const int r = 3 * a + row;
                    KA32[q * 64 + L] = (float)KE_CLS3.sgn[r][col] * h->kc32.k[KE_CLS3.cls[r][col]];
                }
            h->KA32 = halloc<float>(h, KA32.size());
        }
        TM_HIP(hipMemcpyAsync(h->KE64, KE.data(), KE.size() * 8, hipMemcpyHostToDevice, s));
        h->galG = halloc<double>(h, (dim == 3 ? 27 : 9) * KE.size());
        launch_galerkin_unit(dim, h->KE64, h->galG, s);
        if (dim == 3) TM_HIP(hipMemcpyAsync(h->KA32, KA32.data(), KA32.size() * 4, hipMemcpyHostToDevice, s));
        // levels
        h->lv.resize(plan.Lg);
        for (int l = 0; l < plan.Lg; ++l) alloc_level_geo(h, h->lv[l], l);
        std::vector<uint8_t> nm(n_nodes, 0);
        for (int64_t d : fixed) nm[d / dim] |= (uint8_t)(1u << (d % dim));
        TM_HIP(hipMemcpyAsync(h->lv[0].nmask, nm.data(), n_nodes, hipMemcpyHostToDevice, s));
        // level 1 in the tensor form (stencil_kernel 3): 3D, fine element counts
        // even (each level-1 element holds 2 x 2 x 2 fine ones), the form's KE
        // structure
        std::vector<uint8_t> subf;
        if (dim == 3 && plan.Lg > 1 && h->sf_ok && opts->stencil_kernel == 3 &&
            mesh->nel[0] % 2 == 0 && mesh->nel[1] % 2 == 0 && mesh->nel[2] % 2 == 0) {
            const Level& C1 = h->lv[1];
            const int64_t NX = mesh->nel[0] + 1, PLf = NX * (mesh->nel[1] + 1);
            subf.assign((size_t)level_elems(C1, 3), 0);
            for (int cz = 0; cz < C1.nel[2]; ++cz)
                for (int cy = 0; cy < C1.nel[1]; ++cy)
                    for (int cx = 0; cx < C1.nel[0]; ++cx) {
                        uint8_t f = 0;
                        for (int k = 0; k < 8; ++k)
                            for (int c = 0; c < 8; ++c) {
                                const int64_t fx = 2 * cx + (k & 1) + (c & 1), fy = 2 * cy + ((k >> 1) & 1) + ((c >> 1) & 1),
                                              fz = 2 * cz + (k >> 2) + (c >> 2);
                                if (nm[fz * PLf + fy * NX + fx]) f |= (uint8_t)(1u << k);
                            }
                        subf[((size_t)cz * C1.nel[1] + cy) * C1.nel[0] + cx] = f;
                    }
            h->lv[1].subf = halloc<uint8_t>(h, subf.size());
            TM_HIP(hipMemcpyAsync(h->lv[1].subf, subf.data(), subf.size(), hipMemcpyHostToDevice, s));
        }
        const int nd = dim * (1 << dim);
        if (plan.Lg > 1) h->elem_a = halloc<double>(h, (size_t)level_elems(h->lv[1], dim) * nd * nd);
        if (plan.Lg > 2) h->elem_b = halloc<double>(h, (size_t)level_elems(h->lv[2], dim) * nd * nd);
        if (opts->smoother == TM_SMOOTH_CHEBYSHEV) {
            h->cheb_theta = halloc<double>(h, CHEB_MAX_LEVELS);
            h->pw = halloc<double>(h, (size_t)3 * n_dof + 2 * grid_for(n_nodes));
        }
        h->sa = plan.sa;
        if (plan.sa) build_sa_levels(h, s);
        numeric_setup(h, rho_dev, s);
        TM_HIP(hipStreamSynchronize(s));
        *out = h;
    });
    if (st != TM_OK && h) destroy_impl(h);
    return st;
}

tm_status tm_update_density(tm_hierarchy* h, const double* rho_dev, void* stream) {
    return guarded([&] {
        if (!h) fail(TM_ERR_ARG, "hierarchy is NULL");
        if (!rho_dev) fail(TM_ERR_ARG, "rho_dev is NULL");
        if (h->demote) {
            // automated hybrid: one geometric level fewer (at least two stay);
            // the aggregation levels are rebuilt below the new last one
            h->demote = false;
            int Lg = 0;
            for (auto& L : h->lv)
                if (L.kind != TM_LEVEL_AGGREGATION) ++Lg;
            if (Lg > 2) {
                h->lv.resize(Lg - 1);
                h->sa = true;
            }
        }
        // the stress stiffness belongs to the old design; the eigensolver's
        // V-cycle vectors follow the level list, which aggregation rebuilds
        h->gsig_valid = false;
        if (h->sa) free_eig_work(h);
        // without aggregation levels (whose sizes the host must read) the update
        // never waits for the device
        h->cur_stream = S(stream);
        numeric_setup(h, rho_dev, S(stream), h->sa);
    });
}

void tm_destroy(tm_hierarchy* h) { destroy_impl(h); }

int32_t tm_num_levels(const tm_hierarchy* h) { return h ? (int32_t)h->lv.size() : 0; }

tm_status tm_compliance_sensitivity(tm_hierarchy* h, int32_t n_rhs, const double* u_dev, double* dc_dev,
                                    void* stream) {
    return guarded([&] {
        if (!h) fail(TM_ERR_ARG, "hierarchy is NULL");
        if (n_rhs < 1) fail(TM_ERR_ARG, "n_rhs must be >= 1");
        if (!u_dev || !dc_dev) fail(TM_ERR_ARG, "u and dc must be device buffers");
        launch_sensitivity(h, n_rhs, u_dev, dc_dev, S(stream));
        TM_HIP(hipGetLastError());
    });
}

tm_status tm_density_filter(const tm_mesh* mesh, double radius, int32_t transpose, const double* in_dev,
                            double* out_dev, void* stream) {
    return guarded([&] {
        check_mesh(mesh);
        if (!(radius > 0.0 && radius <= 4.0)) fail(TM_ERR_ARG, "radius must be in (0, 4]");
        if (transpose != 0 && transpose != 1) fail(TM_ERR_ARG, "transpose must be 0 or 1");
        if (!in_dev || !out_dev) fail(TM_ERR_ARG, "in and out must be device buffers");
        if (in_dev == out_dev) fail(TM_ERR_ARG, "in and out must not overlap");
        launch_density_filter(mesh->dim, mesh->nel, radius, transpose == 1, in_dev, out_dev, nullptr, S(stream));
        TM_HIP(hipGetLastError());
    });
}

tm_status tm_density_filter_noalloc(const tm_mesh* mesh, double radius, int32_t transpose, const double* in_dev,
                                    double* out_dev, void* stream) {
    return guarded([&] {
        check_mesh(mesh);
        if (!(radius > 0.0 && radius <= 4.0)) fail(TM_ERR_ARG, "radius must be in (0, 4]");
        if (transpose != 0 && transpose != 1) fail(TM_ERR_ARG, "transpose must be 0 or 1");
        if (!in_dev || !out_dev) fail(TM_ERR_ARG, "in and out must be device buffers");
        if (in_dev == out_dev) fail(TM_ERR_ARG, "in and out must not overlap");
        const int64_t n_el = (int64_t)mesh->nel[0] * mesh->nel[1] * (mesh->dim == 3 ? mesh->nel[2] : 1);
        if (n_el > FILTER_SCRATCH_MAX)
            fail(TM_ERR_ARG, "mesh has " + std::to_string(n_el) + " elements; tm_density_filter_noalloc takes at most " +
                                 std::to_string(FILTER_SCRATCH_MAX));
        double* scr = transpose == 1 ? filter_scratch() : nullptr;
        launch_density_filter(mesh->dim, mesh->nel, radius, transpose == 1, in_dev, out_dev, scr, S(stream));
        TM_HIP(hipGetLastError());
    });
}

tm_status tm_hierarchy_bytes(const tm_hierarchy* h, size_t* bytes) {
    return guarded([&] {
        if (!h || !bytes) fail(TM_ERR_ARG, "NULL argument");
        *bytes = h->bytes;
    });
}

static tm_status begin_impl(tm_hierarchy* h, int32_t n_rhs, const double* f_dev, double rtol,
                            int32_t use_u0, double* u_dev, void* stream, tm_solve_state** out,
                            bool cached) {
    return guarded([&] {
        if (!h) fail(TM_ERR_ARG, "hierarchy is NULL");
        if (n_rhs < 1 || n_rhs > 64) fail(TM_ERR_ARG, "n_rhs must be in 1..64");
        if (!f_dev || !u_dev) fail(TM_ERR_ARG, "f_dev / u_dev is NULL");
        if (!(rtol > 0.0 && rtol < 1.0)) fail(TM_ERR_ARG, "rtol must be in (0, 1)");
        tm_solve_state* st = nullptr;
        h->cur_stream = S(stream);
        if (cached) {
            if (h->cached && (h->cached->nrhs != n_rhs || !state_fits(h, h->cached))) {
                delete_state(h->cached);
                h->cached = nullptr;
            }
            if (!h->cached) {
                h->cached = new_state(h, n_rhs);
                h->cached->owned_by_h = true;
            }
            st = h->cached;
        } else {
            for (size_t i = 0; i < h->pool.size();) {
                if (!state_fits(h, h->pool[i])) {          // levels outgrew it
                    delete_state(h->pool[i]);
                    h->pool.erase(h->pool.begin() + i);
                    continue;
                }
                if (!st && h->pool[i]->nrhs == n_rhs) {
                    st = h->pool[i];
                    h->pool.erase(h->pool.begin() + i);
                    continue;
                }
                ++i;
            }
            if (!st) st = new_state(h, n_rhs);
        }
        st->s = S(stream);
        st->rtol = rtol;
        st->use_u0 = use_u0;
        st->u = u_dev;
        st->ended = false;
        st->pending = false;
        try {
            if (st->ev) TM_HIP(hipEventSynchronize(st->ev));   // a reused state may still be draining
            enqueue_begin(st, f_dev, use_u0);
            // outputs of right-hand sides that need no iteration (start already
            // within the tolerance); the host mirror must describe this solve
            // before the first poll
            std::vector<LaneIO> io;
            state_lanes(st, io);
            launch_final_residual_b(io.data(), (int)io.size(), true, st->s);
            std::memset(st->sc_host, 0, sizeof(KScal) * st->nrhs);
            state_sync_point(st, st->s);
        } catch (...) {
            if (!cached) delete_state(st);
            throw;
        }
        *out = st;
    });
}

tm_status tm_solve(tm_hierarchy* h, int32_t n_rhs, const double* f_dev, double rtol, int32_t use_u0,
                   double* u_dev, int32_t* iters, double* compliance, double* relres, void* stream) {
    tm_solve_state* st = nullptr;
    tm_status s0 = begin_impl(h, n_rhs, f_dev, rtol, use_u0, u_dev, stream, &st, true);
    if (s0 != TM_OK) return s0;
    tm_status res = TM_OK;
    const tm_status g = guarded([&] {
        run_to_completion(st);
        res = finish_state(st, iters, compliance, relres);
    });
    return g != TM_OK ? g : res;
}

tm_status tm_solve_begin(tm_hierarchy* h, int32_t n_rhs, const double* f_dev, double rtol,
                         int32_t use_u0, double* u_dev, void* stream, tm_solve_state** st) {
    if (!st) {
        set_error("st is NULL");
        return TM_ERR_ARG;
    }
    return begin_impl(h, n_rhs, f_dev, rtol, use_u0, u_dev, stream, st, false);
}

tm_status tm_solve_advance(tm_solve_state* st, int32_t k_iters) {
    return guarded([&] {
        if (!st || st->ended) fail(TM_ERR_STATE, "state is NULL or ended");
        if (k_iters < 1) fail(TM_ERR_ARG, "k_iters must be >= 1");
        enqueue_advance(st, k_iters);
    });
}

tm_status tm_batch_iterate(int32_t n, tm_solve_state* const* sts, int32_t k_iters, void* stream) {
    return guarded([&] {
        if (n < 0 || (n > 0 && !sts)) fail(TM_ERR_ARG, "bad state list");
        if (k_iters < 1) fail(TM_ERR_ARG, "k_iters must be >= 1");
        for (int i = 0; i < n; ++i)
            if (!sts[i] || sts[i]->ended) fail(TM_ERR_STATE, "state is NULL or ended");
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                if (sts[i] == sts[j]) fail(TM_ERR_ARG, "a state appears twice in the list");
        hipStream_t bs = S(stream);
        // the batch stream continues after the work queued on each state's stream
        for (int i = 0; i < n; ++i)
            if (sts[i]->s != bs) {
                TM_HIP(hipEventRecord(sts[i]->order, sts[i]->s));
                TM_HIP(hipStreamWaitEvent(bs, sts[i]->order, 0));
            }
        // group the lanes of all states by level structure: each group runs an
        // iteration as one launch per operation (MAXB lanes per launch)
        std::vector<std::string> keys;
        std::vector<std::vector<LaneIO>> groups;
        for (int i = 0; i < n; ++i) {
            const std::string key = shape_key(sts[i]->h);
            size_t g = 0;
            while (g < keys.size() && keys[g] != key) ++g;
            if (g == keys.size()) {
                keys.push_back(key);
                groups.emplace_back();
            }
            state_lanes(sts[i], groups[g]);
        }
        for (int it = 0; it < k_iters; ++it)
            for (auto& g : groups) enqueue_iteration_b(g, bs);
        // outputs of the lanes that stopped in this batch
        for (auto& g : groups) launch_final_residual_b(g.data(), (int)g.size(), true, bs);
        for (int i = 0; i < n; ++i) state_sync_point(sts[i], bs);
    });
}

tm_status tm_solve_poll(tm_solve_state* st, int32_t* done) {
    return guarded([&] {
        if (!st || st->ended) fail(TM_ERR_STATE, "state is NULL or ended");
        if (!done) fail(TM_ERR_ARG, "done is NULL");
        *done = -1;
        if (st->pending) {
            const hipError_t q = hipEventQuery(st->ev);
            if (q == hipErrorNotReady) return;
            TM_HIP(q);
            st->pending = false;
        }
        *done = state_done(st) ? 1 : 0;
    });
}

tm_status tm_solve_end(tm_solve_state* st, int32_t* iters, double* compliance, double* relres) {
    if (!st || st->ended) {
        set_error("state is NULL or ended");
        return TM_ERR_STATE;
    }
    tm_status res = TM_OK;
    const tm_status g = guarded([&] { res = finish_state(st, iters, compliance, relres); });
    if (!st->owned_by_h) {
        if (g == TM_OK)
            st->h->pool.push_back(st);       // kept for the next solve on this hierarchy
        else
            delete_state(st);
    }
    return g != TM_OK ? g : res;
}

tm_status tm_apply(tm_hierarchy* h, int32_t level, int32_t fp, const void* x_dev, void* y_dev,
                   void* stream) {
    return guarded([&] {
        const Level& L = level_at(h, level);
        if (fp != 32 && fp != 64) fail(TM_ERR_ARG, "fp must be 32 or 64");
        if (!x_dev || !y_dev) fail(TM_ERR_ARG, "NULL vector");
        hipStream_t s = S(stream);
        if (fp == 64) {
            if (L.kind == TM_LEVEL_FINE)
                launch_fine_op<double>(h, OP_APPLY, true, (const double*)x_dev, nullptr, (double*)y_dev, 0.0,
                                       nullptr, nullptr, s);
            else
                level_op<double>(h, level, OP_APPLY, (const double*)x_dev, nullptr, (double*)y_dev, nullptr, s);
        } else {
            if (L.kind == TM_LEVEL_FINE)
                launch_fine_op<float>(h, OP_APPLY, true, (const float*)x_dev, nullptr, (float*)y_dev, 0.f,
                                      nullptr, nullptr, s);
            else
                level_op<float>(h, level, OP_APPLY, (const float*)x_dev, nullptr, (float*)y_dev, nullptr, s);
        }
        TM_HIP(hipStreamSynchronize(s));
    });
}

tm_status tm_vcycle(tm_hierarchy* h, int32_t fp, const void* b_dev, void* x_dev, void* stream) {
    return guarded([&] {
        if (!h) fail(TM_ERR_ARG, "hierarchy is NULL");
        if (fp != 32 && fp != 64) fail(TM_ERR_ARG, "fp must be 32 or 64");
        if (!b_dev || !x_dev) fail(TM_ERR_ARG, "NULL vector");
        hipStream_t s = S(stream);
        h->cur_stream = s;
        std::vector<void*> list;
        size_t bytes = 0;
        Vcyc V;
        try {
            if (fp == 64) {
                alloc_vcyc<double>(h, V, list, bytes);
                double* bm = dalloc<double>(h, list, bytes, h->n_dof);
                launch_mask_copy<double>(h, (const double*)b_dev, bm, s);
                vcycle<double>(h, V, bm, (double*)x_dev, nullptr, s);
            } else {
                alloc_vcyc<float>(h, V, list, bytes);
                float* bm = dalloc<float>(h, list, bytes, h->n_dof);
                launch_mask_copy<float>(h, (const float*)b_dev, bm, s);
                vcycle<float>(h, V, bm, (float*)x_dev, nullptr, s);
            }
            TM_HIP(hipStreamSynchronize(s));
        } catch (...) {
            (void)hipStreamSynchronize(s);
            free_list(h, list);
            throw;
        }
        free_list(h, list);
    });
}

tm_status tm_level_info(const tm_hierarchy* h, int32_t level, int64_t* n_rows, int64_t* nnz,
                        int32_t* kind, int32_t* block) {
    return guarded([&] {
        const Level& L = level_at(h, level);
        if (n_rows) *n_rows = L.n;
        if (kind) *kind = L.kind;
        if (block) *block = L.bs;
        if (nnz) {
            if (L.kind == TM_LEVEL_AGGREGATION) {
                *nnz = L.A.nnzb * L.bs * L.bs;
            } else {
                // structured stencil: count neighbour blocks inside the grid
                int64_t blocks = 1;
                for (int d = 0; d < L.dim; ++d) blocks *= (int64_t)3 * L.nn[d] - 2;
                *nnz = blocks * L.bs * L.bs;
            }
        }
    });
}

tm_status tm_export_csr(const tm_hierarchy* h, int32_t level, int64_t* rowptr, int32_t* colidx,
                        double* vals) {
    return guarded([&] {
        const Level& L = level_at(h, level);
        if (L.kind == TM_LEVEL_FINE) fail(TM_ERR_ARG, "the fine level is matrix-free");
        std::vector<int64_t> rp;
        std::vector<int32_t> ci;
        std::vector<double> v;
        if (L.kind == TM_LEVEL_GEOMETRIC)
            stencil_csr(L, rp, ci, v, vals != nullptr);
        else
            bsr_csr(L.A, rp, ci, v);
        if (rowptr) std::memcpy(rowptr, rp.data(), rp.size() * 8);
        if (colidx) std::memcpy(colidx, ci.data(), ci.size() * 4);
        if (vals) std::memcpy(vals, v.data(), v.size() * 8);
    });
}

tm_status tm_export_prolongator(const tm_hierarchy* h, int32_t level, int64_t* n_rows, int64_t* nnz,
                                int64_t* rowptr, int32_t* colidx, double* vals) {
    return guarded([&] {
        const Level& L = level_at(h, level);
        if (level + 1 >= (int)h->lv.size()) fail(TM_ERR_ARG, "the coarsest level has no prolongator");
        std::vector<int64_t> rp;
        std::vector<int32_t> ci;
        std::vector<double> v;
        if (L.xfer_bsr)
            bsr_csr(L.P, rp, ci, v);
        else
            geo_prolongator(h, level, rp, ci, v);
        if (n_rows) *n_rows = (int64_t)rp.size() - 1;
        if (nnz) *nnz = (int64_t)ci.size();
        if (rowptr) std::memcpy(rowptr, rp.data(), rp.size() * 8);
        if (colidx) std::memcpy(colidx, ci.data(), ci.size() * 4);
        if (vals) std::memcpy(vals, v.data(), v.size() * 8);
    });
}

tm_status tm_export_aggregates(const tm_hierarchy* h, int32_t level, int32_t* agg_of_node) {
    return guarded([&] {
        const Level& L = level_at(h, level);
        if (!L.agg) fail(TM_ERR_ARG, "level is not an aggregation input level");
        if (!agg_of_node) fail(TM_ERR_ARG, "agg_of_node is NULL");
        TM_HIP(hipMemcpy(agg_of_node, L.agg, L.n_nodes * 4, hipMemcpyDeviceToHost));
    });
}

tm_status tm_export_dinv(const tm_hierarchy* h, int32_t level, double* dinv) {
    return guarded([&] {
        const Level& L = level_at(h, level);
        if (!dinv) fail(TM_ERR_ARG, "dinv is NULL");
        const int bs = L.bs, bb = bs * bs;
        std::vector<double> t((size_t)sym_n(bs) * L.n_nodes);
        TM_HIP(hipMemcpy(t.data(), L.dinv64, t.size() * 8, hipMemcpyDeviceToHost));
        if (h->opt.smoother == TM_SMOOTH_CHEBYSHEV && level + 1 < (int)h->lv.size()) {
            // stored divided by the level's interval centre
            double th = 0.0;
            TM_HIP(hipMemcpy(&th, h->cheb_theta + level, sizeof(double), hipMemcpyDeviceToHost));
            for (double& e : t) e *= th;
        }
        for (int64_t node = 0; node < L.n_nodes; ++node)
            for (int r = 0; r < bs; ++r)
                for (int c = 0; c < bs; ++c)
                    dinv[node * bb + r * bs + c] = t[(size_t)sym_at(r, c, bs) * L.n_nodes + node];
    });
}

tm_status tm_export_coarse_inverse(const tm_hierarchy* h, double* ainv) {
    return guarded([&] {
        if (!h) fail(TM_ERR_ARG, "hierarchy is NULL");
        if (!ainv) fail(TM_ERR_ARG, "ainv is NULL");
        TM_HIP(hipDeviceSynchronize());
        TM_HIP(hipMemcpy(ainv, h->ainv, (size_t)h->nc * h->nc * sizeof(double), hipMemcpyDeviceToHost));
    });
}

tm_status tm_export_connectivity(const tm_mesh* mesh, int32_t* conn) {
    return guarded([&] {
        check_mesh(mesh);
        if (!conn) fail(TM_ERR_ARG, "conn is NULL");
        const int dim = mesh->dim, npe = 1 << dim;
        const int nx = mesh->nel[0], ny = mesh->nel[1], nz = dim == 3 ? mesh->nel[2] : 1;
        const int NX = nx + 1, NY = ny + 1;
        int64_t e = 0;
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i, ++e)
                    for (int z = 0; z < (dim == 3 ? 2 : 1); ++z)
                        for (int y = 0; y < 2; ++y)
                            for (int x = 0; x < 2; ++x) {
                                const int a = dim == 3 ? loc3(x, y, z) : loc2(x, y);
                                conn[e * npe + a] = (int32_t)(((int64_t)(k + z) * NY + (j + y)) * NX + i + x);
                            }
    });
}

tm_status tm_kernel_timing(tm_hierarchy* h, int32_t kernel_class, int32_t enable) {
    return guarded([&] {
        if (!h) fail(TM_ERR_ARG, "hierarchy is NULL");
        if (kernel_class < 0 || kernel_class > 2) fail(TM_ERR_ARG, "kernel_class must be 0, 1 or 2");
        h->timing[kernel_class] = enable != 0;
    });
}

tm_status tm_kernel_timing_read(tm_hierarchy* h, int32_t kernel_class, int64_t* launches,
                                double* total_ms) {
    return guarded([&] {
        if (!h) fail(TM_ERR_ARG, "hierarchy is NULL");
        if (kernel_class < 0 || kernel_class > 2) fail(TM_ERR_ARG, "kernel_class must be 0, 1 or 2");
        double tot = 0.0;
        auto& v = h->tev[kernel_class];
        for (auto& pr : v) {
            TM_HIP(hipEventSynchronize(pr.second));
            float ms = 0.f;
            TM_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
            tot += ms;
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        if (launches) *launches = (int64_t)v.size();
        if (total_ms) *total_ms = tot;
        v.clear();
    });
}

tm_status tm_stress_stiffness(tm_hierarchy* h, const double* u_dev, double rho_min, void* stream) {
    return guarded([&] {
        if (!h) fail(TM_ERR_ARG, "hierarchy is NULL");
        if (!u_dev) fail(TM_ERR_ARG, "u must be a device buffer");
        if (!(rho_min >= 0.0 && rho_min <= 1.0)) fail(TM_ERR_ARG, "rho_min must be in [0, 1]");
        const size_t nst = h->dim == 3 ? 27 : 9;
        h->cur_stream = S(stream);
        if (!h->gsig) h->gsig = halloc<double>(h, nst * (size_t)h->n_nodes);
        h->gsig_valid = false;
        launch_gsig_assemble(h, u_dev, rho_min, h->gsig, S(stream));
        TM_HIP(hipGetLastError());
        h->gsig_valid = true;
    });
}

tm_status tm_apply_stress_stiffness(tm_hierarchy* h, const double* x_dev, double* y_dev, void* stream) {
    return guarded([&] {
        if (!h) fail(TM_ERR_ARG, "hierarchy is NULL");
        if (!x_dev || !y_dev) fail(TM_ERR_ARG, "x and y must be device buffers");
        if (x_dev == y_dev) fail(TM_ERR_ARG, "x and y must not overlap");
        if (!h->gsig_valid) fail(TM_ERR_STATE, "no current stress-stiffness matrix (call tm_stress_stiffness)");
        launch_gsig_apply(h, h->gsig, x_dev, y_dev, S(stream));
        TM_HIP(hipStreamSynchronize(S(stream)));
    });
}

void tm_default_eig_options(tm_eig_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->nev = 6;
    o->j_min = 10;
    o->j_max = 25;
    o->max_iters = 1000;
    o->tol = 1e-6;
    o->stag_tol = 1e-13;
    o->precond_fp = 32;
}

tm_status tm_eigs(tm_hierarchy* h, const tm_eig_options* o, int32_t n_init, const double* v0_dev,
                  double* lambda, double* phi_dev, int32_t* iters, int32_t* n_conv, void* stream) {
    tm_status st = TM_OK;
    const tm_status g = guarded([&] {
        if (!h) fail(TM_ERR_ARG, "hierarchy is NULL");
        if (!o) fail(TM_ERR_ARG, "options are NULL");
        if (!(o->nev >= 1 && o->nev < o->j_min && o->j_min < o->j_max && o->j_max <= EIG_MAX_COLS))
            fail(TM_ERR_ARG, "need 1 <= nev < j_min < j_max <= 32");
        if (o->max_iters < 0) fail(TM_ERR_ARG, "max_iters must be >= 0");
        if (!(o->tol >= 0.0) || !(o->stag_tol >= 0.0)) fail(TM_ERR_ARG, "tolerances must be >= 0");
        if (o->precond_fp != 32 && o->precond_fp != 64) fail(TM_ERR_ARG, "precond_fp must be 32 or 64");
        if (n_init < 1 || n_init > o->j_max) fail(TM_ERR_ARG, "n_init must be in 1..j_max");
        if (!v0_dev || !lambda) fail(TM_ERR_ARG, "start vectors and lambda are required");
        if (!h->gsig_valid) fail(TM_ERR_STATE, "no current stress-stiffness matrix (call tm_stress_stiffness)");
        hipStream_t s = S(stream);
        h->cur_stream = s;
        if (h->flags_pending) {
            h->flags_pending = false;
            read_flags(h, s, "last update");
        }
        st = run_davidson(h, *o, n_init, v0_dev, lambda, phi_dev, iters, n_conv, s);
    });
    return g != TM_OK ? g : st;
}

}  // extern "C"
