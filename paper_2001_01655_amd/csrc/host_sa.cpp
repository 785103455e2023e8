// Smoothed-aggregation levels of the hybrid hierarchy: geometric coarsening on
// the finest levels, then algebraic coarsening of the last geometric level
// until a level has fewer than max_coarse dofs (Sec. 4.3 / 4.4).  The levels
// depend on the densities (strength of connection), so every numeric setup
// rebuilds them; their memory is kept apart from the geometric levels'.
#include <cstring>
#include <string>
#include <vector>

#include "tm_internal.h"

namespace tmi {

// kernels_sa.hip
int64_t scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int64_t* work, hipStream_t s);
void launch_stencil_to_bsr(const Level& L, const int32_t* rp, int32_t* ci, double* v, hipStream_t s);
void sa_launch_diag_fsq(const BSR& A, int bs, double* dn, hipStream_t s);
void sa_launch_strength(const BSR& A, int bs, const double* dn, double beta, int32_t* cnt, const int32_t* srp,
                        int32_t* sci, bool fill, hipStream_t s);
int sa_mis2(const int32_t* srp, const int32_t* sci, int64_t n, uint8_t* state, uint64_t* m1, uint64_t* m2,
            uint8_t* f, int32_t* counter, hipStream_t s);
void sa_root_flags(int64_t n, const uint8_t* state, int32_t* flag, hipStream_t s);
void sa_agg_passes(const int32_t* srp, const int32_t* sci, int64_t n, const uint8_t* state, const int32_t* rid,
                   int32_t* agg1, int32_t* root1, int32_t* agg, int32_t* missing, hipStream_t s);
void sa_members(int64_t n, int64_t ng, const int32_t* agg, int32_t* cnt_off, int32_t* cursor, int32_t* mem,
                int32_t* umem, int64_t* work, hipStream_t s);
void sa_tentative(int64_t ng, const int32_t* off, const int32_t* mem, const double* Bprev, int dim, int nx1,
                  int ny1, double h, int level, const int* nel0, int bs, int k, double* T, double* Bc, bool use_lds,
                  hipStream_t s);
double sa_jacobi_bound(const BSR& A, int bs, const double* dinv, unsigned long long* work, hipStream_t s);
void sa_symbolic(const int32_t* rp1, const int32_t* ci1, const int32_t* agg, const int32_t* rp2,
                 const int32_t* ci2, int32_t ncols, int kind, int64_t nrows, int32_t* cnt, const int32_t* orp,
                 int32_t* oci, bool fill, hipStream_t s);
void sa_row_of(const int32_t* rp, int64_t nrows, int32_t* rowof, hipStream_t s);
void sa_p_numeric(const BSR& A, const int32_t* agg, const double* T, const double* dinv, int bs, int k,
                  double omega, const int32_t* prow, const BSR& P, bool use_lds, hipStream_t s);
void sa_transpose(const BSR& P, const int32_t* prow, BSR& PT, int32_t* cursor, int32_t* tsrc, int32_t* uci,
                  int32_t* usrc, int64_t* work, hipStream_t s);
void sa_prod_numeric(const BSR& X, const BSR& Y, const int32_t* crow, BSR& C, int32_t* dtmp, bool use_lds,
                     hipStream_t s);
void sa_fix_diag(BSR& A, int bs, hipStream_t s);
void sa_to_f32(const double* a, float* b, int64_t n, hipStream_t s);

namespace {

struct Pool {                       // typed blocks from one arena
    const tm_hierarchy* h;
    Arena& a;
    template <typename T>
    T* get(size_t n) {
        return (T*)arena_get(h, a, std::max<size_t>(n, 1) * sizeof(T));
    }
};

// symbolic + allocation of a BSR product/pattern with nrows block rows
void make_pattern(Pool& keep, Pool& tmp, BSR& C, int64_t nrows, int64_t ncols, int br, int bc,
                  const int32_t* rp1, const int32_t* ci1, const int32_t* agg, const int32_t* rp2,
                  const int32_t* ci2, int kind, int64_t* work, hipStream_t s) {
    (void)tmp;
    C.nbr = nrows;
    C.nbc = ncols;
    C.br = br;
    C.bc = bc;
    C.rp = keep.get<int32_t>(nrows + 1);
    sa_symbolic(rp1, ci1, agg, rp2, ci2, (int32_t)ncols, kind, nrows, C.rp, nullptr, nullptr, false, s);
    C.nnzb = scan_exclusive(C.rp, C.rp, nrows, work, s);
    C.ci = keep.get<int32_t>(C.nnzb);
    C.v64 = keep.get<double>((size_t)C.nnzb * br * bc);
    sa_symbolic(rp1, ci1, agg, rp2, ci2, (int32_t)ncols, kind, nrows, nullptr, C.rp, C.ci, true, s);
}

}  // namespace

void build_sa_levels(tm_hierarchy* h, hipStream_t s) {
    (void)h;
    (void)s;   // sizes of aggregation levels are known only after the numeric setup
}

void numeric_sa_levels(tm_hierarchy* h, hipStream_t s) {
    // The new levels overwrite the arenas of the previous ones in stream
    // order: the rebuild waits for the solves of this hierarchy still queued
    // on their own streams (no device-wide wait), and only an arena that the
    // last rebuild outgrew is replaced.
    if (h->cached) TM_HIP(hipStreamWaitEvent(s, h->cached->ev, 0));
    for (tm_solve_state* st : h->pool) TM_HIP(hipStreamWaitEvent(s, st->ev, 0));
    arena_prepare(h, h->sa_keep);
    arena_prepare(h, h->sa_tmp);
    arena_prepare(h, h->sa_cand[0]);
    arena_prepare(h, h->sa_cand[1]);
    int Lg = 0;
    for (auto& L : h->lv)
        if (L.kind != TM_LEVEL_AGGREGATION) ++Lg;
    h->lv.resize(Lg);
    Level& G0 = h->lv[Lg - 1];
    G0.xfer_bsr = false;
    G0.A = BSR();
    G0.P = BSR();
    G0.PT = BSR();
    G0.agg = nullptr;
    G0.n_agg = 0;
    // (solve states keep their V-cycle vectors while the new level sizes fit:
    // checked when the next solve begins)
    auto account = [&] {
        h->bytes -= std::min(h->bytes, h->sa_bytes);
        h->sa_bytes = arena_bytes(h->sa_keep) + arena_bytes(h->sa_tmp) + arena_bytes(h->sa_cand[0]) +
                      arena_bytes(h->sa_cand[1]);
        h->bytes += h->sa_bytes;
    };
    if (G0.n < h->opt.max_coarse) {
        account();
        return;
    }

    Pool keep{h, h->sa_keep};
    int step = 0;
    try {
        const int dim = h->dim;
        const int k = dim == 3 ? 6 : 3;
        // block-CSR copy of the last geometric level (structured pattern)
        {
            Level& G = h->lv[Lg - 1];
            std::vector<int32_t> rp(G.n_nodes + 1, 0);
            const int NX = G.nn[0], NY = G.nn[1], NZ = dim == 3 ? G.nn[2] : 1;
            for (int64_t node = 0; node < G.n_nodes; ++node) {
                const int i = (int)(node % NX), j = (int)((node / NX) % NY), kk = (int)(node / ((int64_t)NX * NY));
                const int cx = 1 + (i > 0) + (i < NX - 1), cy = 1 + (j > 0) + (j < NY - 1);
                const int cz = dim == 3 ? 1 + (kk > 0) + (kk < NZ - 1) : 1;
                rp[node + 1] = rp[node] + cx * cy * cz;
            }
            G.A.nbr = G.A.nbc = G.n_nodes;
            G.A.br = G.A.bc = dim;
            G.A.nnzb = rp[G.n_nodes];
            G.A.rp = keep.get<int32_t>(G.n_nodes + 1);
            G.A.ci = keep.get<int32_t>(G.A.nnzb);
            G.A.v64 = keep.get<double>((size_t)G.A.nnzb * dim * dim);
            TM_HIP(hipMemcpyAsync(G.A.rp, rp.data(), rp.size() * 4, hipMemcpyHostToDevice, s));
            launch_stencil_to_bsr(G, G.A.rp, G.A.ci, G.A.v64, s);
            TM_HIP(hipStreamSynchronize(s));
        }
        const double* Bprev = nullptr;
        int cur = Lg - 1;
        while (h->lv[cur].n >= h->opt.max_coarse) {
            arena_reset(h->sa_tmp);
            Pool tmp{h, h->sa_tmp};
            Level& F = h->lv[cur];
            const int bs = F.bs;
            const int64_t n = F.n_nodes;
            int64_t* work = tmp.get<int64_t>(n / 1024 + 64);
            // strength of connection
            double* dn = tmp.get<double>(n);
            int32_t* srp = tmp.get<int32_t>(n + 1);
            sa_launch_diag_fsq(F.A, bs, dn, s);
            sa_launch_strength(F.A, bs, dn, h->opt.sa_beta, srp, nullptr, nullptr, false, s);
            const int64_t nS = scan_exclusive(srp, srp, n, work, s);
            int32_t* sci = tmp.get<int32_t>(nS);
            sa_launch_strength(F.A, bs, dn, h->opt.sa_beta, nullptr, srp, sci, true, s);
            // roots: lexicographically-first distance-2 independent set
            uint8_t* state = tmp.get<uint8_t>(n);
            uint64_t* m1 = tmp.get<uint64_t>(n);
            uint64_t* m2 = tmp.get<uint64_t>(n);
            uint8_t* fl = tmp.get<uint8_t>(n);
            int32_t* counter = tmp.get<int32_t>(2);
            sa_mis2(srp, sci, n, state, m1, m2, fl, counter, s);
            int32_t* rid = tmp.get<int32_t>(n + 1);
            sa_root_flags(n, state, rid, s);
            const int64_t n_agg = scan_exclusive(rid, rid, n, work, s);
            if (n_agg * k > (int64_t)(0.9 * (double)F.n)) break;      // stagnation: keep this level coarsest
            // aggregates
            int32_t* agg1 = tmp.get<int32_t>(n);
            int32_t* root1 = tmp.get<int32_t>(n);
            int32_t* agg = keep.get<int32_t>(n);
            sa_agg_passes(srp, sci, n, state, rid, agg1, root1, agg, counter, s);
            int32_t missing = 0;
            TM_HIP(hipMemcpyAsync(&missing, counter, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            TM_HIP(hipStreamSynchronize(s));
            if (missing) fail(TM_ERR_DEVICE, "aggregation left nodes unassigned");
            // tentative prolongator
            int32_t* off = tmp.get<int32_t>(n_agg + 1);
            int32_t* cursor = tmp.get<int32_t>(std::max<int64_t>(n_agg, n) + 1);
            int32_t* mem = tmp.get<int32_t>(n);
            int32_t* umem = tmp.get<int32_t>(n);
            sa_members(n, n_agg, agg, off, cursor, mem, umem, work, s);
            double* T = tmp.get<double>((size_t)n * bs * k);
            // this step's candidates (the previous step's stay in the other arena)
            arena_reset(h->sa_cand[step & 1]);
            Pool nextp{h, h->sa_cand[step & 1]};
            double* Bc = nextp.get<double>((size_t)n_agg * k * k);
            sa_tentative(n_agg, off, mem, Bprev, dim, F.nn[0], F.nn[1], h->mesh.h, Lg - 1, h->mesh.nel, bs, k, T, Bc,
                         h->opt.sa_lds == 0, s);
            // smoothed prolongator P = T - omega D^-1 A T
            unsigned long long* mx = tmp.get<unsigned long long>(1);
            const double lam = sa_jacobi_bound(F.A, bs, F.dinv64, mx, s);
            if (!(lam > 0.0)) fail(TM_ERR_NOT_SPD, "aggregation level has a non-positive Jacobi bound");
            const double omega = (4.0 / 3.0) / lam;
            BSR P;
            make_pattern(keep, tmp, P, n, n_agg, bs, k, F.A.rp, F.A.ci, agg, nullptr, nullptr, 0, work, s);
            int32_t* prow = tmp.get<int32_t>(P.nnzb);
            sa_row_of(P.rp, n, prow, s);
            sa_p_numeric(F.A, agg, T, F.dinv64, bs, k, omega, prow, P, h->opt.sa_lds == 0, s);
            // P^T
            BSR PT;
            PT.nbr = n_agg;
            PT.nbc = n;
            PT.br = k;
            PT.bc = bs;
            PT.nnzb = P.nnzb;
            PT.rp = keep.get<int32_t>(n_agg + 1);
            PT.ci = keep.get<int32_t>(P.nnzb);
            PT.v64 = keep.get<double>((size_t)P.nnzb * bs * k);
            int32_t* tsrc = tmp.get<int32_t>(P.nnzb);
            int32_t* uci = tmp.get<int32_t>(P.nnzb);
            int32_t* usrc = tmp.get<int32_t>(P.nnzb);
            sa_transpose(P, prow, PT, cursor, tsrc, uci, usrc, work, s);
            // A P, then A_c = P^T (A P)
            BSR AP;
            make_pattern(tmp, tmp, AP, n, n_agg, bs, k, F.A.rp, F.A.ci, nullptr, P.rp, P.ci, 1, work, s);
            int32_t* aprow = tmp.get<int32_t>(AP.nnzb);
            sa_row_of(AP.rp, n, aprow, s);
            sa_prod_numeric(F.A, P, aprow, AP, counter, h->opt.sa_lds == 0, s);
            BSR Ac;
            make_pattern(keep, tmp, Ac, n_agg, n_agg, k, k, PT.rp, PT.ci, nullptr, AP.rp, AP.ci, 2, work, s);
            int32_t* acrow = tmp.get<int32_t>(Ac.nnzb);
            sa_row_of(Ac.rp, n_agg, acrow, s);
            sa_prod_numeric(PT, AP, acrow, Ac, counter, h->opt.sa_lds == 0, s);
            sa_fix_diag(Ac, k, s);
            // FP32 copies for the V-cycle
            P.v32 = keep.get<float>((size_t)P.nnzb * bs * k);
            PT.v32 = keep.get<float>((size_t)PT.nnzb * bs * k);
            Ac.v32 = keep.get<float>((size_t)Ac.nnzb * k * k);
            sa_to_f32(P.v64, P.v32, P.nnzb * bs * k, s);
            sa_to_f32(PT.v64, PT.v32, PT.nnzb * bs * k, s);
            sa_to_f32(Ac.v64, Ac.v32, Ac.nnzb * k * k, s);
            // the new level
            Level C;
            C.kind = TM_LEVEL_AGGREGATION;
            C.dim = dim;
            C.bs = k;
            C.n_nodes = n_agg;
            C.n = n_agg * k;
            C.A = Ac;
            C.dinv64 = keep.get<double>((size_t)sym_n(k) * n_agg);
            C.dinv32 = keep.get<float>((size_t)sym_n(k) * n_agg);
            TM_HIP(hipMemsetAsync(h->flags, 0, sizeof(int), s));
            launch_bsr_dinv(C, h->opt.smoother == TM_SMOOTH_POINT_JACOBI, h->flags, s);
            int fl_host = 0;
            TM_HIP(hipMemcpyAsync(&fl_host, h->flags, sizeof(int), hipMemcpyDeviceToHost, s));
            TM_HIP(hipStreamSynchronize(s));
            if (fl_host & FLAG_NOT_SPD) fail(TM_ERR_NOT_SPD, "aggregation level diagonal block not positive definite");
            F.xfer_bsr = true;
            F.P = P;
            F.PT = PT;
            F.agg = agg;
            F.n_agg = n_agg;
            h->lv.push_back(C);
            ++cur;
            // candidates of the next step: the R factors
            Bprev = Bc;
            ++step;
        }
        arena_reset(h->sa_tmp);
        account();
    } catch (...) {
        (void)hipStreamSynchronize(s);
        account();
        throw;
    }
}

}  // namespace tmi
