// Internal declarations shared by the HIP translation units of libtopomg.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "topomg.h"

namespace tmi {

constexpr int WG = 256;                 // threads per workgroup for node-parallel kernels

// ----------------------------------------------------------------- errors
struct Error {
    tm_status code;
    std::string msg;
};
void set_error(const std::string& msg);
[[noreturn]] void fail(tm_status code, const std::string& msg);
void check_hip(hipError_t e, const char* what);
#define TM_HIP(call) ::tmi::check_hip((call), #call)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline unsigned grid_for(int64_t n, int wg = WG) { return (unsigned)ceil_div(n > 0 ? n : 1, wg); }

// ----------------------------------------------------------------- device helpers
// Logical workgroup index such that consecutive logical indices run on the same
// XCD (hardware dispatches workgroups round-robin over the 8 XCDs).
__device__ __forceinline__ int64_t xcd_block() {
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    const uint32_t q = nb >> 3, r = nb & 7u, x = b & 7u, k = b >> 3;
    return (int64_t)(x * q + (x < r ? x : r) + k);
}

// Block inverses D^-1 are symmetric: only the upper triangle is stored, entry
// (r, c) with r <= c at slot sym_at(r, c, bs) of sym_n(bs), row by row; (c, r)
// reads the same slot.
__host__ __device__ constexpr int sym_n(int bs) { return bs * (bs + 1) / 2; }
__host__ __device__ constexpr int sym_at(int r, int c, int bs) {
    return r <= c ? r * bs - r * (r - 1) / 2 + (c - r) : c * bs - c * (c - 1) / 2 + (r - c);
}

// local index of the element corner at offsets (lx, ly[, lz]) in {0,1}: 2D
// counter-clockwise from the lower-left corner, 3D bottom face then top face.
__host__ __device__ constexpr int loc2(int lx, int ly) { return ly ? (lx ? 2 : 3) : (lx ? 1 : 0); }
__host__ __device__ constexpr int loc3(int lx, int ly, int lz) { return 4 * lz + loc2(lx, ly); }

// Symmetry classes of the element stiffness of a square / cube element of an
// isotropic material.  Each symmetry of the square (8) or cube (48), an axis
// permutation p with reflections m, maps corner a to corner g(a) and dof
// component c to p(c) with sign -1 if axis c is reflected; KE is invariant,
// KE[(a,c),(b,d)] = s_c s_d KE[(g a, p c),(g b, p d)], and symmetric.  The
// orbits of the entries under these maps give cls[r][s] (the class of entry
// (r, s)) and sgn[r][s] (its sign relative to the class value, 0 for an entry
// the symmetries force to zero).  2D has 7 classes, 3D has 12, so the whole
// 8x8 / 24x24 matrix lives in a handful of wave-uniform registers.
template <int DIM>
struct KeClasses {
    static constexpr int NN = 1 << DIM, ND = DIM * NN;
    int8_t cls[ND][ND];
    int8_t sgn[ND][ND];
    int n;
};
constexpr int KE_MAX_CLASSES = 12;

__host__ __device__ constexpr int corner_coord(int a, int ax) {
    const int q = a & 3;
    return ax == 0 ? (q == 1 || q == 2) : ax == 1 ? (q >= 2) : (a >> 2);
}

template <int DIM>
constexpr KeClasses<DIM> make_ke_classes() {
    constexpr int NN = 1 << DIM, ND = DIM * NN;
    constexpr int P3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    constexpr int P2[2][3] = {{0, 1, 2}, {1, 0, 2}};
    const int np = DIM == 3 ? 6 : 2;
    KeClasses<DIM> T{};
    for (int r = 0; r < ND; ++r)
        for (int s = 0; s < ND; ++s) {
            T.cls[r][s] = -1;
            T.sgn[r][s] = 0;
        }
    int n = 0;
    for (int r = 0; r < ND; ++r)
        for (int s = 0; s < ND; ++s) {
            if (T.cls[r][s] >= 0) continue;
            const int a = r / DIM, c = r % DIM, b = s / DIM, d = s % DIM;
            bool zero = false;
            for (int pi = 0; pi < np; ++pi)
                for (int m = 0; m < NN; ++m) {
                    const int* p = DIM == 3 ? P3[pi] : P2[pi];
                    int qa[3] = {0, 0, 0}, qb[3] = {0, 0, 0};
                    for (int ax = 0; ax < DIM; ++ax) {
                        const int fl = (m >> ax) & 1;
                        qa[p[ax]] = fl ? 1 - corner_coord(a, ax) : corner_coord(a, ax);
                        qb[p[ax]] = fl ? 1 - corner_coord(b, ax) : corner_coord(b, ax);
                    }
                    const int a2 = DIM == 3 ? loc3(qa[0], qa[1], qa[2]) : loc2(qa[0], qa[1]);
                    const int b2 = DIM == 3 ? loc3(qb[0], qb[1], qb[2]) : loc2(qb[0], qb[1]);
                    const int sg = (((m >> c) & 1) ? -1 : 1) * (((m >> d) & 1) ? -1 : 1);
                    const int r2 = DIM * a2 + p[c], s2 = DIM * b2 + p[d];
                    const int rr[2] = {r2, s2}, ss[2] = {s2, r2};
                    for (int t = 0; t < 2; ++t) {
                        if (T.cls[rr[t]][ss[t]] == n && T.sgn[rr[t]][ss[t]] != sg) zero = true;
                        T.cls[rr[t]][ss[t]] = (int8_t)n;
                        T.sgn[rr[t]][ss[t]] = (int8_t)sg;
                    }
                }
            if (zero)
                for (int r3 = 0; r3 < ND; ++r3)
                    for (int s3 = 0; s3 < ND; ++s3)
                        if (T.cls[r3][s3] == n) T.sgn[r3][s3] = 0;
            ++n;
        }
    T.n = n;
    return T;
}
inline constexpr KeClasses<2> KE_CLS2 = make_ke_classes<2>();
inline constexpr KeClasses<3> KE_CLS3 = make_ke_classes<3>();
static_assert(KE_CLS2.n <= KE_MAX_CLASSES && KE_CLS3.n <= KE_MAX_CLASSES, "KE class count");

// class values of KE (E = 1), passed to the fine kernels by value
template <typename T>
struct KeVals {
    T k[KE_MAX_CLASSES];
};

// Tensor form of the 3D element stiffness.  Transform the corner values of one
// component to modes, one per choice of sum or difference along each axis
// (bit k of the mode index m set: difference along axis k; for a face of four
// corners, bits 0 and 1; for the element, bit 2 adds z).  The trilinear cube's
// 1D mass matrix is diagonal in these modes and its 1D stiffness and mixed
// matrices map a sum to a difference or back, so KE = F^T C F (F the +-1
// transform per component) with C nonzero only where component d's input mode
// m feeds component c's output mode m (c = d, m != 0) or m with bits c and d
// flipped (c != d, bits c and d of m differ): 21 + 24 = 45 coefficients,
// slot s[c][d][m] (-1: none).
struct SfSlots {
    int8_t s[3][3][8];
    int n;
};
constexpr SfSlots make_sf_slots() {
    SfSlots t{};
    int n = 0;
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d)
            for (int m = 0; m < 8; ++m) {
                const bool on = c == d ? m != 0 : ((m >> c) & 1) != ((m >> d) & 1);
                t.s[c][d][m] = on ? (int8_t)n++ : (int8_t)-1;
            }
    t.n = n;
    return t;
}
inline constexpr SfSlots SF_SLOTS = make_sf_slots();
constexpr int SF_COEFS = 45;
static_assert(SF_SLOTS.n == SF_COEFS, "tensor-form coefficient count");
// output mode of component c fed by input mode m of component d
__host__ __device__ constexpr int sf_out_mode(int c, int d, int m) { return c == d ? m : m ^ (1 << c) ^ (1 << d); }
template <typename T>
struct SfCoef {
    T k[SF_COEFS];
};

// Lane batching: a kernel of the solve path runs the same operation for up to
// MAXB lanes (right-hand sides of one or several hierarchies with the same
// level structure) in one launch; blockIdx.y selects the lane, whose pointers
// travel by value in the kernel arguments.  NB = 1 for single launches.
constexpr int MAXB = 8;
template <typename A, int NB>
struct Pack {
    A a[NB];
};
template <typename A, int NB>
__device__ __forceinline__ const A& lane_of(const Pack<A, NB>& pk) {
    return pk.a[NB == 1 ? 0 : blockIdx.y];
}

// per-lane operands of the level operators (fine matrix-free and stored stencil)
template <typename T>
struct OpA {
    const T* E;          // fine: moduli; stencil: the stored operator
    const float* KA;     // fine FP32 on the matrix cores: KE columns
    const uint8_t* nm;   // fine: support mask
    const T* x;
    const T* b;
    T* y;
    const T* dinv;
    const int* done;
    double* partials;
    const T* din;        // Chebyshev step: previous direction (or the iterate) ...
    T* dout;             // ... and the new direction (NULL: not kept)
    const T* xc;         // fused prolongation: the coarse level's correction
    const uint8_t* sub;  // level 1 in the tensor form: sub-element support flags
};
template <typename T>
struct RestrictA {
    const T* rf;
    const uint8_t* nm;
    T* bc;
    T* xc;
    const T* dinv;
    const int* done;
};
template <typename T>
struct ProlongA {
    const T* xc;
    const uint8_t* nm;
    T* xf;
    const int* done;
};
template <typename T>
struct DenseA {
    const double* Ainv;
    const T* b;
    T* x;
    const int* done;
};
template <typename T>
struct FirstA {
    const T* b;
    const T* dinv;
    T* x;
    const int* done;
};

// Status flags written by kernels (checked by the host after setup phases).
enum : int { FLAG_BAD_RHO = 1, FLAG_NOT_SPD = 2, FLAG_OVERFLOW = 4 };

// Per right-hand-side Krylov scalars, resident on the device.
struct KScal {
    double pq, pr, rr, zq, zr, zr_old;
    double alpha, beta;
    double rr_stop;         // (rtol ||M f||)^2
    double ff;              // ||M f||^2
    double rr_last;         // ||r||^2 after the last completed iteration
    int32_t iter, done, status, max_iters;
    int32_t outer;          // TM_OUTER_*
    int32_t fin;            // pq / zq hold the true residual and compliance of the stopped iterate
    int32_t skipfin;        // gate of the in-batch output kernels (0: compute them for this lane)
    int32_t pad;
};

// ----------------------------------------------------------------- structures
struct BSR {                // block sparse rows, int32 block columns
    int64_t nbr = 0, nbc = 0, nnzb = 0;
    int br = 0, bc = 0;     // block shape
    int32_t* rp = nullptr;  // nbr + 1
    int32_t* ci = nullptr;  // nnzb
    double* v64 = nullptr;  // nnzb * br * bc, row-major blocks
    float* v32 = nullptr;
};

struct Level {
    int kind = TM_LEVEL_FINE;     // TM_LEVEL_*
    int dim = 0;
    int nel[3] = {1, 1, 1};       // elements per axis (geometric levels)
    int nn[3] = {1, 1, 1};        // nodes per axis
    int64_t n_nodes = 0;          // block rows
    int bs = 0;                   // dofs per block row
    int64_t n = 0;                // dofs
    // Chebyshev smoothing interval [theta - delta, theta + delta] for D^-1 A
    // fine level
    double* E64 = nullptr;
    float* E32 = nullptr;
    uint8_t* nmask = nullptr;     // per node: bit c set <=> dof c supported
    // geometric coarse level: stencil [nst][bs*bs][n_nodes] (FP64, setup and exports)
    int nst = 0;
    double* st64 = nullptr;
    // V-cycle copy in symmetric form [nq][n_nodes]: the blocks towards the
    // (nst-1)/2 neighbours after the node in grid order, then the upper
    // triangle of the diagonal block; the other blocks are transposes of the
    // neighbours' stored ones
    int nq = 0;
    int op_kernel = 0;            // stencil operator kernel: 0 by size, 1 large-level, 2 small-level
    // level 1 applied matrix-free in the tensor form (Galerkin product of the
    // fine elements, which an even fine grid nests two per axis in each
    // element): subf[element] bit k set <=> fine sub-element k (x, y, z bits)
    // has a supported dof
    uint8_t* subf = nullptr;
    double* stc64 = nullptr;
    float* stc32 = nullptr;
    // aggregation level operator
    BSR A;
    // point-block Jacobi inverse [bs*bs][n_nodes]
    double* dinv64 = nullptr;
    float* dinv32 = nullptr;
    // transfer to the next coarser level: geometric stencil or explicit P / P^T
    bool xfer_bsr = false;
    BSR P, PT;
    int32_t* agg = nullptr;       // aggregates of this level's nodes (if xfer_bsr)
    int64_t n_agg = 0;
    double* coords = nullptr;     // candidate vectors for aggregation [n][k] (setup only)
};

struct Vcyc {                     // V-cycle work vectors of one precision, per level
    std::vector<void*> b, x, t;   // rhs, iterate, scratch (same length per level)
    std::vector<void*> d;         // Chebyshev update direction (Chebyshev smoothing only)
    std::vector<int64_t> cap;     // entries each vector of a level holds
};

// Grow-only device arena for the aggregation levels, which a density update
// rebuilds with data-dependent sizes: blocks are cut from one buffer in order
// and the arena is emptied (reset) when its contents are no longer needed, in
// stream order.  A request that does not fit gets a block of its own
// (overflow); the next rebuild replaces buffer and overflow blocks by one
// buffer large enough for everything, so rebuilds of steady size allocate and
// free nothing.
struct Arena {
    char* base = nullptr;
    size_t cap = 0, used = 0;
    size_t need = 0;              // bytes asked for since the last reset
    size_t peak = 0;              // largest need of a reset cycle since the last rebuild began
    std::vector<void*> overflow;
    size_t overflow_bytes = 0;
};

struct Lane;                      // one right-hand side of a solve state

// Generalized Davidson (stability eigenproblem): the search space has at most
// EIG_MAX_COLS columns; reductions over rows use at most EIG_BLOCKS workgroups.
constexpr int EIG_MAX_COLS = 32;
constexpr int EIG_BLOCKS = 2048;
inline int eig_blocks(int64_t n) {
    const int64_t b = ceil_div(n > 0 ? n : 1, (int64_t)WG * 2);
    return (int)(b < EIG_BLOCKS ? b : EIG_BLOCKS);
}
struct EigWork {                  // device workspace of tm_eigs, kept by the hierarchy
    int64_t n = 0;
    int jmax = 0, fp = 0;
    double *V = nullptr;          // search space, n x jmax, column-major
    double *q = nullptr, *Aq = nullptr, *Bq = nullptr, *r = nullptr, *z = nullptr, *w = nullptr;
    double *part = nullptr;       // (EIG_MAX_COLS + 1) x EIG_BLOCKS partial sums, column-major
    double *red = nullptr;        // EIG_MAX_COLS + 1 reduced sums
    double *coef = nullptr;       // EIG_MAX_COLS coefficients
    double *Y = nullptr;          // EIG_MAX_COLS^2 Ritz coefficients
    double *rb = nullptr;         // masked V-cycle input (FP64)
    float *r32 = nullptr, *z32 = nullptr;
    double *host = nullptr;       // pinned mirror of red
    Vcyc vc;                      // V-cycle work vectors in the preconditioner's precision
    std::vector<void*> allocs;
    size_t bytes = 0;
};

}  // namespace tmi

struct tm_hierarchy {
    tm_mesh mesh{};
    tm_material mat{};
    tm_options opt{};
    int dim = 0;
    int64_t n_el = 0, n_nodes = 0, n_dof = 0;
    std::vector<int64_t> fixed;
    std::vector<tmi::Level> lv;
    double* KE64 = nullptr;        // element stiffness for E = 1 (device)
    double* galG = nullptr;        // unit Galerkin products Q_k^T KE Q_k per child kind (27 or 9)
    double* rho64 = nullptr;       // densities of the current design (device)
    float* KA32 = nullptr;         // 3D: KE as the broadcast A operand of the matrix-core fine operator
    tmi::KeVals<double> kc64{};       // KE symmetry-class values (fine operator arguments)
    tmi::KeVals<float> kc32{};
    tmi::SfCoef<float> sf32{};        // 3D KE in the tensor form (fine operator arguments)
    tmi::SfCoef<double> sf64{};
    bool sf_ok = false;               // KE has the tensor form's structure
    double* ainv = nullptr;        // inverse of the coarsest operator (FP64, dense)
    float* ainv32 = nullptr;
    int64_t nc = 0;                // coarsest dofs
    size_t ainv_cap = 0;
    bool sa = false;               // smoothed-aggregation levels below the geometric ones
    bool demote = false;           // a solve exceeded adapt_iters: drop a geometric level at the next update
    bool flags_pending = false;    // an update ran without waiting: its device checks are read by the next solve
    uint64_t update_seq = 0;       // numeric setups so far (which update a copy of the checks belongs to)
    double* dense_a = nullptr;     // coarsest operator, dense (setup scratch kept for updates)
    size_t dense_cap = 0;
    double* chol_ls = nullptr;     // blocked Cholesky panel scratch
    int* flags = nullptr;          // device status flags
    // Chebyshev smoothing: centre theta_l of each level's interval (device) and
    // the setup scratch of the power estimate (three fine-size vectors, partials)
    double* cheb_theta = nullptr;
    double* pw = nullptr;
    // warm-started estimates (option cheb_warm_steps): each geometric level's
    // last estimate vector, scaled to unit length, and the scale factors
    double* cheb_v = nullptr;
    std::vector<int64_t> cheb_off;
    double* cheb_ninv = nullptr;
    bool cheb_warm = false;        // cheb_v holds the previous design's vectors
    double* elem_a = nullptr;      // setup workspace: element matrices (ping)
    double* elem_b = nullptr;      // (pong)
    size_t bytes = 0;
    std::vector<void*> allocs;
    // aggregation levels (rebuilt by every numeric setup): level data, the
    // temporaries of one coarsening step, the candidate vectors of two
    // consecutive steps
    tmi::Arena sa_keep, sa_tmp, sa_cand[2];
    size_t sa_bytes = 0;           // the arenas' share of `bytes`
    // kernel timing hooks
    bool timing[3] = {false, false, false};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> tev[3];
    // stability eigenproblem: stress-stiffness stencil [3^dim][n_nodes] of the
    // last tm_stress_stiffness (stale after a density update) and the
    // eigensolver's workspace
    double* gsig = nullptr;
    bool gsig_valid = false;
    tmi::EigWork* eig = nullptr;
    // default solve state (tm_solve) and ended states kept for reuse
    tm_solve_state* cached = nullptr;
    std::vector<tm_solve_state*> pool;
    // device memory source (tm_setup's allocator, else hipMalloc) and the
    // stream of the call in progress, handed to the allocator
    tm_allocator alloc{};
    bool has_alloc = false;
    hipStream_t cur_stream = nullptr;
};

struct tm_solve_state {
    tm_hierarchy* h = nullptr;
    hipStream_t s = nullptr;
    int32_t nrhs = 0;
    double rtol = 0.0;
    int use_u0 = 0;
    double* u = nullptr;           // caller's output (n_dof * nrhs)
    std::vector<tmi::Lane*> lanes;
    tmi::KScal* sc = nullptr;      // device scalars [nrhs]
    tmi::KScal* sc_host = nullptr; // pinned mirror
    hipEvent_t ev = nullptr;       // the scalars' host copy has arrived
    int* flags_host = nullptr;     // pinned copy of the hierarchy's device checks, taken with the scalars
    uint64_t flags_seq = 0;        // update_seq of that copy
    bool flags_copied = false;
    hipEvent_t order = nullptr;    // marks the work queued on s (start of a batch on another stream)
    bool ended = false, pending = false;
    bool owned_by_h = false;
    size_t bytes = 0;
    std::vector<void*> allocs;
};

namespace tmi {
// Weight of the first smoothing step from zero, x = w D^-1 b.  With Chebyshev
// smoothing the stored D^-1 of each level is already divided by theta_l, the
// centre of its interval, so that step has weight 1 (and every later step's
// coefficients depend only on the interval's ratio, known on the host).
inline double first_sweep_weight(const tm_hierarchy* h, int l) {
    (void)l;
    return h->opt.smoother == TM_SMOOTH_CHEBYSHEV ? 1.0 : h->opt.omega;
}
constexpr int CHEB_MAX_LEVELS = 64;
void launch_power_start(double* v, int64_t n, const uint8_t* nmask, int bs, hipStream_t s);
void launch_power_step(const Level& L, const double* w, const double* v, double* z, double* part, hipStream_t s);
void launch_cheb_theta(const double* part, int nparts, double factor, double* theta, double* ninv, hipStream_t s);
void launch_scale_copy(const double* src, double* dst, int64_t n, const double* scale, hipStream_t s);
void launch_scale_dinv(Level& L, const double* theta, hipStream_t s);


struct Lane {
    double *f = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *z64 = nullptr;
    float *r32 = nullptr, *z32 = nullptr;
    double* part = nullptr;        // reduction partials
    Vcyc v32, v64;
};

void delete_cached_state(tm_hierarchy* h);

// One lane of a batched launch (host side): its hierarchy and the vectors the
// operation reads and writes.  Operators: x in, b right-hand side, y out,
// din / dout the Chebyshev directions, part the partial sums; transfers: x in,
// y out, y2 the coarse level's first sweep; dense solve: x = b in, y out;
// Krylov updates: the lane's scalars, vectors and solution.
struct LaneIO {
    const tm_hierarchy* h = nullptr;
    const void* x = nullptr;
    const void* b = nullptr;
    void* y = nullptr;
    void* y2 = nullptr;
    const int* done = nullptr;
    double* part = nullptr;
    const void* din = nullptr;
    void* dout = nullptr;
    const void* xc = nullptr;
    KScal* sc = nullptr;
    Lane* ln = nullptr;
    double* u = nullptr;
};
// batched launchers: n lanes (any number; MAXB per launch) of hierarchies with
// the same level structure and options; the lanes' own pointers differ
template <typename T>
void launch_fine_op_b(int op, bool mask_in, const LaneIO* L, int n, T omega, double c1, double c2, hipStream_t s);
template <typename T>
void launch_stencil_op_b(int level, int op, const LaneIO* L, int n, T omega, double c1, double c2, hipStream_t s);
// level 1 in the tensor form (the level's subf set; FP32 V-cycle): the
// operator from the fine moduli and supports instead of the stored stencil
template <typename T>
void launch_coarse1_tensor_b(int op, const LaneIO* L, int n, T omega, double c1, double c2, hipStream_t s);
template <typename T>
void launch_restrict_b(int fine_level, const LaneIO* L, int n, T omega, hipStream_t s);
// the last restriction and the coarsest solve in one launch (geometric
// transfer to a dense coarsest level)
bool restrict_solve_ok(const tm_hierarchy* h);
template <typename T>
void launch_restrict_solve_b(const LaneIO* L, int n, hipStream_t s);
template <typename T>
void launch_prolong_b(int fine_level, const LaneIO* L, int n, hipStream_t s);
// prolongation fused into the first post-smoothing step (op OP_SMOOTH or
// OP_CHEB from the prolonged iterate) of a small geometric level whose coarse
// level is geometric too; stencil_pro_ok says whether level l qualifies
bool stencil_pro_ok(const tm_hierarchy* h, int level);
// the same on the 3D fine level in the FP32 tensor form (fine_pro_ok says
// whether h qualifies: level 1 geometric, even fine element counts)
bool fine_pro_ok(const tm_hierarchy* h);
void launch_fine_pro_b(int op, const LaneIO* L, int n, float omega, double c1, double c2, hipStream_t s);
template <typename T>
void launch_stencil_pro_b(int level, int op, const LaneIO* L, int n, T omega, double c1, double c2, hipStream_t s);
template <typename T>
void launch_first_smooth_b(int level, const LaneIO* L, int n, T omega, hipStream_t s);
template <typename T>
void launch_dense_solve_b(const LaneIO* L, int n, hipStream_t s);
void launch_finalize_b(const LaneIO* L, int n, int nparts, int what, hipStream_t s);
void launch_update_ur_b(const LaneIO* L, int n, bool mixed, hipStream_t s);
void launch_zdots_b(const LaneIO* L, int n, bool mixed, hipStream_t s);
void launch_update_p_b(const LaneIO* L, int n, bool mixed, hipStream_t s);
// device memory of a hierarchy (host.cpp): from its allocator or hipMalloc;
// a list is returned after the device has finished with it
void* dev_alloc(const tm_hierarchy* h, size_t bytes);
void dev_free_list(const tm_hierarchy* h, std::vector<void*>& list);
// arenas (host.cpp): a block of at least `bytes` (256-byte aligned); reset for
// reuse; prepare for a rebuild (one buffer for the last rebuild's total, only
// if it grew); release everything
void* arena_get(const tm_hierarchy* h, Arena& a, size_t bytes);
void arena_reset(Arena& a);
void arena_prepare(const tm_hierarchy* h, Arena& a);
void arena_release(const tm_hierarchy* h, Arena& a);
size_t arena_bytes(const Arena& a);

// ----------------------------------------------------------------- launchers
// fine level (kernels_fine.hip)
enum { OP_APPLY = 0, OP_RESID = 1, OP_SMOOTH = 2, OP_QDOT = 3, OP_CHEB = 4 };

// OP_CHEB (one Chebyshev step): dout = c1 din + c2 D^-1 (b - A x), y = x + dout.
// din may be x (first step after a zero start) or equal dout (in place).
struct ChebArgs {
    const void* din = nullptr;
    void* dout = nullptr;
    double c1 = 0.0, c2 = 0.0;
};
void launch_simp(const double* rho, int64_t n_el, double p, double E0, double Emin, double* E64,
                 float* E32, double* rho64, int* flags, hipStream_t s);
void launch_sensitivity(const tm_hierarchy* h, int n_rhs, const double* u, double* dc, hipStream_t s);
// fixed_scratch: n_el FP64 device values for the transpose (NULL: stream-ordered
// scratch allocated by the call)
void launch_density_filter(int dim, const int* nel, double r, bool tr, const double* in, double* out,
                           double* fixed_scratch, hipStream_t s);
// largest element count of tm_density_filter_noalloc, and the device address of
// its fixed scratch on the current device
constexpr int64_t FILTER_SCRATCH_MAX = (int64_t)1 << 23;
double* filter_scratch();
void launch_fine_dinv(const Level& L, const double* KE64, int point_jacobi, int* flags,
                      hipStream_t s);
template <typename T>
void launch_fine_op(const tm_hierarchy* h, int op, bool mask_in, const T* x, const T* b, T* y,
                    T omega, const int* done, double* partials, hipStream_t s,
                    const ChebArgs& ch = ChebArgs{});
int update_ur_blocks(const tm_hierarchy* h);
int fine_op_blocks(const tm_hierarchy* h);
// coarse geometric levels (kernels_coarse.hip)
void launch_galerkin_elems(const tm_hierarchy* h, int fine_level, const double* child,
                           double* parent, hipStream_t s);
void launch_galerkin_unit(int dim, const double* KE, double* G, hipStream_t s);
void launch_stencil_assemble(const Level& L, const double* elem, hipStream_t s);
void launch_stencil_compact(const Level& L, hipStream_t s);
void launch_stencil_dinv(const Level& L, int point_jacobi, int* flags, hipStream_t s);
// dense coarsest level (kernels_dense.hip)
void launch_dense_from_stencil(const Level& L, double* Ad, hipStream_t s);
void launch_dense_from_bsr(const Level& L, double* Ad, hipStream_t s);
int chol_block_elems();  // scratch doubles the blocked factorisation needs
void launch_cholesky_inverse(double* A, double* Ainv, double* Ls, int64_t n, int* flags, hipStream_t s);
// aggregation levels (kernels_sa.hip)
template <typename T>
void launch_bsr_op(const Level& L, int op, const T* x, const T* b, T* y, T omega, const int* done,
                   hipStream_t s, const ChebArgs& ch = ChebArgs{});
template <typename T>
void launch_bsr_restrict(const Level& fine, const T* rf, T* bc, const Level& coarse, T* xc_first,
                         T omega, const int* done, hipStream_t s);
template <typename T>
void launch_bsr_prolong(const Level& fine, const T* xc, T* xf, const int* done, hipStream_t s);
void launch_bsr_dinv(const Level& L, int point_jacobi, int* flags, hipStream_t s);
// Krylov (kernels_krylov.hip)
template <typename T>
void launch_mask_copy(const tm_hierarchy* h, const T* src, T* dst, hipStream_t s);
void launch_fcg_init(const tm_hierarchy* h, Lane& ln, KScal* sc, int use_u0, double* u,
                     double rtol, int max_iters, int outer, hipStream_t s);
void launch_update_ur(const tm_hierarchy* h, Lane& ln, KScal* sc, double* u, bool mixed,
                      hipStream_t s);
void launch_zdots(const tm_hierarchy* h, Lane& ln, KScal* sc, bool mixed, hipStream_t s);
// single-block finalisation of the per-block partial sums (fixed order)
enum { FIN_ALPHA = 0, FIN_RR = 1, FIN_BETA = 2 };
void launch_finalize(KScal* sc, const double* part, int nparts, int what, hipStream_t s);
void launch_update_p(const tm_hierarchy* h, Lane& ln, KScal* sc, bool mixed, hipStream_t s);
void launch_final_residual(const tm_hierarchy* h, Lane& ln, KScal* sc, const double* u,
                           hipStream_t s);
// the same for lanes L[0..n) (h, ln, sc, u set); gated: only the lanes that
// have stopped and have no outputs yet (sc->fin == 0), the others stay as they are
void launch_final_residual_b(const LaneIO* L, int n, bool gated, hipStream_t s);
void launch_cast(const double* a, float* b, int64_t n, hipStream_t s);
void launch_cast_back(const float* a, double* b, int64_t n, hipStream_t s);
void launch_fill(void* p, int64_t n_bytes, hipStream_t s);
int krylov_blocks(int64_t n);
// stability eigenproblem (kernels_eigen.hip)
void launch_gsig_assemble(const tm_hierarchy* h, const double* u, double rho_min, double* G, hipStream_t s);
void launch_gsig_apply(const tm_hierarchy* h, const double* G, const double* x, double* y, hipStream_t s);
void launch_vtw(const double* V, int64_t ld, int nc, const double* w, const double* z, int64_t n, double* part,
                double* out, hipStream_t s);
void launch_vupdate(const double* V, int64_t ld, int nc, const double* coef, double a, const double* in, double* out,
                    int64_t n, hipStream_t s);
void launch_vrotate(double* V, int64_t ld, int nc, const double* Y, int m, double* dst, int64_t ldd, int64_t n,
                    hipStream_t s);
void launch_eig_resid(const double* Aq, const double* Bq, double theta, double* r, int64_t n, double* part,
                      double* out, hipStream_t s);

}  // namespace tmi
