// Host side of libspaimg.so: level hierarchy, cycle orchestration, the solve
// loop with its convergence monitor, mixed-precision refinement and the
// adjoint cycle.  Every arithmetic step on a grid runs in the gfx950 kernels
// of mg_kernels.hip / mg_adjoint.hip; the host only allocates, enqueues and
// reads back one norm per cycle.
//
// Cycle structure (He, Liu and Wang, arXiv 2206.05543, Section 4): V(1,1)
// with full weighting, linear interpolation, rediscretised coarse operators
// and an exact solve at h0 = 1/4; the stopping rule is the reduction of the
// 2-norm of the residual relative to the initial one.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/spaimg.h"
#include "mg_internal.h"

using namespace spaimg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                               \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess)                                                      \
            return fail(MG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kMaxLevels = 20;
constexpr int kTimeKinds = 11;
constexpr long kPartialCap = 1 << 17;  // per batch entry
constexpr long kAdjBlocks = 8192;      // blocks per batch entry of an adjoint sweep

struct Hier {
    Prec p = P64;
    bool scaled = false;
    void* e[kMaxLevels] = {};          // per level; FP64 level 0: only t
    void* b[kMaxLevels] = {};
    void* t[kMaxLevels] = {};
    double* ginv = nullptr;            // sigma_coarsest * A_coarsest^{-1}
    bool ginv_owned = false;           // allocated by alloc_hier
    bool allocated = false;
};

struct TimedLaunch {
    int kind, level;
    hipEvent_t a, b;
};

}  // namespace

struct mg_ctx {
    int N = 0, d = 2, L = 0, batch = 1, prec = MG_PREC_FP64, max_cycles = 100;
    int tail_N = 0;  // 0 = default
    int inner = 0;   // inner cycles per refinement step, 0 = default
    int cycle_kind = MG_CYCLE_V11;
    int ncoef = 3;
    double c[4] = {0, 0, 0, 0};  // centre, faces, diagonals (2D) / edges, corners (3D)
    Hier h64, hlo;
    double* ualt = nullptr;      // FP64 fine ping-pong buffer
    double* psum = nullptr;      // per-block partial sums
    double* pmax = nullptr;      // per-block partial maxima
    double* psum_b = nullptr;    // per-block partial sums of b^2 (||b|| of a solve)
    bool bnorm_req = false;      // the next fused fine pre-smoother sums b^2 too
    int bnorm_parts = 0;         // partials it left in psum_b (0 = none)
    double* dnorm = nullptr;     // device norms: 2 per slot (norm, max)
    double* dscale = nullptr;    // refinement scales per step
    double* hnorm = nullptr;     // coherent pinned host mirror of dnorm
    double* hnorm_dev = nullptr; // its device address
    // partial sums of a finished sweep waiting to be reduced: by the next
    // restriction of cycle() (block 0 of that launch), else by k_finalize
    struct PendingNorm {
        int count = 0;           // partials in psum (0 = nothing pending)
        bool with_max = false;   // also reduce pmax into dnorm[2 slot + 1]
        int slot = -1;
    } pend;
    int norm_slots = 0;
    // adjoint scratch (FP64), allocated on first use; per level
    std::vector<double*> adj_r1, adj_r3, adj_w, adj_ua, adj_ub, adj_uo, adj_bb;
    double* adj_cin = nullptr;   // FP64 copy of an FP32 checkpoint (fine level)
    bool adj_alloc = false;
    double* adj_cacc = nullptr;  // device accumulator of dL/dc (4 doubles)
    double* adj_part = nullptr;  // coefficient-gradient partials of one adjoint cycle
    long adj_pcap = 0;           // its capacity (doubles)
    long adj_poff = 0;           // next free slot
    // timing
    int timing = 0;
    int call_fused = 0;          // fused fine-level launches of this call (mode 3)
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<TimedLaunch> pending;
    double t_ms[kTimeKinds][kMaxLevels] = {};
    int t_cnt[kTimeKinds][kMaxLevels] = {};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

long level_pts(const mg_ctx* h, int l) {
    long n = (h->N >> l) - 1, p = 1;
    for (int a = 0; a < h->d; ++a) p *= n;
    return p;
}
int level_n(const mg_ctx* h, int l) { return (h->N >> l) - 1; }
int level_N(const mg_ctx* h, int l) { return h->N >> l; }

// largest grid of the LDS tail (intervals): 64^2 / 16^3 for V(1,1) and
// W(1,0) cycles.  Measured on a 2D N=4096 W(1,0) solve: a 64^2 tail (its
// top level visited twice inside the workgroup) 30.0 ms, 32^2 with the 64^2
// level launched across the chip 33.4 ms, 16^2 43.1 ms; 3D N=256: 16^3
// 14.6 ms against 17.7 ms for 8^3.
int default_tail_N(int d, int cycle_kind) {
    (void)cycle_kind;
    return d == 2 ? 64 : 16;
}

// low-precision V-cycles per FP64 refinement step.  FP32: six reach about
// what FP32 resolves in one step (~1e-6), so 1e-10 takes two steps; fewer
// per step need more steps, and a last step cut short leaves smooth error
// components that lie below FP32's resolution of the residual (the residual
// norm meets tol while the error stays above the FP64 solve's).  FP16: a
// third cycle gains little.
int inner_cycles(const mg_ctx* h) {
    if (h->inner) return h->inner;
    return h->prec == MG_PREC_FP16_IR ? 2 : 6;
}

// first level whose zero-guess cycles run in the tail kernel
int tail_level(const mg_ctx* h, bool allow_level0) {
    const int tN = h->tail_N ? h->tail_N : default_tail_N(h->d, h->cycle_kind);
    for (int l = allow_level0 ? 0 : 1; l < h->L; ++l)
        if (level_N(h, l) <= tN) return l;
    return h->L - 1;
}

void level_scales(const mg_ctx* h, const Hier& H, int l, double* sA, double* sW,
                  double* pf) {
    const double N = level_N(h, l);
    if (H.scaled) {
        *sA = 1.0;
        *sW = 1.0;
        *pf = 4.0;
    } else {
        *sA = N * N;
        *sW = 1.0 / (N * N);
        *pf = 1.0;
    }
}

}  // namespace

// Inverse of the h-free Laplacian stencil matrix on the 3^d coarsest grid
// (h0 = 1/4, Section 4), times `scale`, by Gauss-Jordan elimination with
// partial pivoting in FP64.  Evaluated at compile time: the host copies it
// into each hierarchy, and the handle-free cycle reads the device tables
// below, so both paths apply the same numbers.
template <int M>
struct StencilInverse {
    double a[M * M];
};

constexpr double abs_cx(double x) { return x < 0 ? -x : x; }

template <int D>
constexpr StencilInverse<D == 2 ? 9 : 27> coarsest_stencil_inverse(double scale) {
    constexpr int n = 3, m = D == 2 ? 9 : 27;
    StencilInverse<m> A{}, I{};
    for (int p = 0; p < m; ++p) {
        const int i = p % n, j = (p / n) % n, k = p / (n * n);
        A.a[p * m + p] = 2.0 * D;
        const int nb[6][3] = {{i - 1, j, k}, {i + 1, j, k}, {i, j - 1, k},
                              {i, j + 1, k}, {i, j, k - 1}, {i, j, k + 1}};
        for (int q = 0; q < 2 * D; ++q) {
            const int x = nb[q][0], y = nb[q][1], z = nb[q][2];
            if (x < 0 || x >= n || y < 0 || y >= n || z < 0 || z >= (D == 3 ? n : 1)) continue;
            A.a[p * m + x + n * (y + n * z)] = -1.0;
        }
        I.a[p * m + p] = 1.0;
    }
    for (int c = 0; c < m; ++c) {
        int piv = c;
        for (int r = c + 1; r < m; ++r)
            if (abs_cx(A.a[r * m + c]) > abs_cx(A.a[piv * m + c])) piv = r;
        for (int q = 0; q < m; ++q) {
            double x = A.a[c * m + q];
            A.a[c * m + q] = A.a[piv * m + q];
            A.a[piv * m + q] = x;
            x = I.a[c * m + q];
            I.a[c * m + q] = I.a[piv * m + q];
            I.a[piv * m + q] = x;
        }
        const double dv = A.a[c * m + c];
        for (int q = 0; q < m; ++q) {
            A.a[c * m + q] = A.a[c * m + q] / dv;
            I.a[c * m + q] = I.a[c * m + q] / dv;
        }
        for (int r = 0; r < m; ++r) {
            if (r == c) continue;
            const double f = A.a[r * m + c];
            if (f == 0.0) continue;
            for (int q = 0; q < m; ++q) {
                A.a[r * m + q] = A.a[r * m + q] - f * A.a[c * m + q];
                I.a[r * m + q] = I.a[r * m + q] - f * I.a[c * m + q];
            }
        }
    }
    for (int q = 0; q < m * m; ++q) I.a[q] = I.a[q] * scale;
    return I;
}

// sigma A_0^{-1} with A_0 = 16 x stencil (N = 4): 1/16 x the stencil
// inverse for the FP64 hierarchy (sigma = 1), the stencil inverse itself for
// the scaled ones (sigma = 16)
constexpr StencilInverse<9> kInv2 = coarsest_stencil_inverse<2>(1.0);
constexpr StencilInverse<27> kInv3 = coarsest_stencil_inverse<3>(1.0);
constexpr StencilInverse<9> kInv2_64 = coarsest_stencil_inverse<2>(1.0 / 16);
constexpr StencilInverse<27> kInv3_64 = coarsest_stencil_inverse<3>(1.0 / 16);

namespace {

void free_hier(Hier& H) {
    for (void** v : {H.e, H.b, H.t})
        for (int l = 0; l < kMaxLevels; ++l) {
            if (v[l]) (void)hipFree(v[l]);
            v[l] = nullptr;
        }
    if (H.ginv && H.ginv_owned) (void)hipFree(H.ginv);
    H.ginv = nullptr;
    H.ginv_owned = false;
    H.allocated = false;
}

int alloc_hier(mg_ctx* h, Hier& H, Prec p) {
    free_hier(H);
    H.p = p;
    H.scaled = p != P64;
    const size_t es = prec_bytes(p);
    for (int l = 0; l < h->L; ++l) {
        const size_t bytes = (size_t)level_pts(h, l) * h->batch * es;
        if (l == 0 && p == P64) {
            HIPCHK(hipMalloc(&H.t[0], bytes));
            continue;
        }
        HIPCHK(hipMalloc(&H.e[l], bytes));
        HIPCHK(hipMalloc(&H.b[l], bytes));
        HIPCHK(hipMalloc(&H.t[l], bytes));
    }
    // exact coarsest solve: sigma * A^{-1}; A = N^2 * stencil (N = 4); in the
    // scaled hierarchy sigma = N^2, so sigma A^{-1} = stencil^{-1}
    const double* G = h->d == 2 ? (H.scaled ? kInv2.a : kInv2_64.a)
                                : (H.scaled ? kInv3.a : kInv3_64.a);
    const size_t gbytes = (h->d == 2 ? 81 : 729) * sizeof(double);
    HIPCHK(hipMalloc(&H.ginv, gbytes));
    H.ginv_owned = true;
    HIPCHK(hipMemcpy(H.ginv, G, gbytes, hipMemcpyHostToDevice));
    H.allocated = true;
    return MG_OK;
}

int alloc_common(mg_ctx* h) {
    if (h->ualt) (void)hipFree(h->ualt);
    if (h->psum) (void)hipFree(h->psum);
    if (h->pmax) (void)hipFree(h->pmax);
    if (h->psum_b) (void)hipFree(h->psum_b);
    if (h->dnorm) (void)hipFree(h->dnorm);
    if (h->dscale) (void)hipFree(h->dscale);
    if (h->hnorm) (void)hipHostFree(h->hnorm);
    h->ualt = h->psum = h->pmax = h->psum_b = h->dnorm = h->dscale = h->hnorm = h->hnorm_dev =
        nullptr;
    const size_t fine = (size_t)level_pts(h, 0) * h->batch * sizeof(double);
    HIPCHK(hipMalloc(&h->ualt, fine));
    HIPCHK(hipMalloc(&h->psum, kPartialCap * h->batch * sizeof(double)));
    HIPCHK(hipMalloc(&h->pmax, kPartialCap * h->batch * sizeof(double)));
    HIPCHK(hipMalloc(&h->psum_b, kPartialCap * h->batch * sizeof(double)));
    h->norm_slots = h->max_cycles + 4;
    HIPCHK(hipMalloc(&h->dnorm, 2 * h->norm_slots * sizeof(double)));
    HIPCHK(hipMalloc(&h->dscale, h->norm_slots * sizeof(double)));
    // coherent: the kernels' system-scope stores of norms reach the host
    // directly, and the solve loops poll the slots (wait_norm)
    HIPCHK(hipHostMalloc(&h->hnorm, 2 * h->norm_slots * sizeof(double), hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer(reinterpret_cast<void**>(&h->hnorm_dev), h->hnorm, 0));
    return MG_OK;
}

void free_adj(mg_ctx* h);

int realloc_all(mg_ctx* h) {
    int rc = alloc_hier(h, h->h64, P64);
    if (rc) return rc;
    if (h->prec != MG_PREC_FP64) {
        rc = alloc_hier(h, h->hlo, h->prec == MG_PREC_FP32_IR ? P32 : P16);
        if (rc) return rc;
    } else {
        free_hier(h->hlo);
    }
    free_adj(h);
    return alloc_common(h);
}

// ---- timing -------------------------------------------------------------

bool timed(mg_ctx* h, int kind, int level) {
    if (h->timing == 2) return true;
    // mode 1: the longest-running kernel of a cycle, the fine level's
    // pre-smoother fused with the restriction (and, in chained 2D solves,
    // with the previous cycle's post-smoother): one event pair per cycle.
    // Mode 3: one of them per call, the second (the first runs right after
    // the caller wrote u, a cache state no later cycle sees).  An event
    // recorded after a large kernel idles the GPU for ~5 us while the
    // caches are written back, so mode 1 costs ~4% of a solve, mode 3 ~0.4%.
    const bool fused = level == 0 && (kind == MG_TIME_SMOOTH_RESTRICT ||
                                      kind == MG_TIME_POST_PRE_RESTRICT);
    if (!fused) return false;
    if (h->timing == 1) return true;
    return h->timing == 3 && h->call_fused++ == 1;
}

int time_begin(mg_ctx* h, int kind, int level, hipStream_t st, TimedLaunch* tl) {
    if (h->ev_used + 2 > h->ev_pool.size()) {
        for (int i = 0; i < 64; ++i) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            h->ev_pool.push_back(e);
        }
    }
    (void)st;
    tl->kind = kind;
    tl->level = level;
    tl->a = h->ev_pool[h->ev_used++];
    tl->b = h->ev_pool[h->ev_used++];
    // the next kernel launched records its own start and end in the pair
    launch_events() = LaunchEvents{tl->a, tl->b};
    return MG_OK;
}

int time_end(mg_ctx* h, TimedLaunch& tl, hipStream_t st) {
    (void)st;
    if (launch_events().start) {
        // nothing was launched (an argument error): nothing to time
        launch_events() = LaunchEvents();
        h->ev_used -= 2;
        return MG_OK;
    }
    h->pending.push_back(tl);
    return MG_OK;
}

// after the stream has been synchronised
int time_collect(mg_ctx* h) {
    for (auto& tl : h->pending) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, tl.a, tl.b));
        h->t_ms[tl.kind][tl.level] += ms;
        h->t_cnt[tl.kind][tl.level] += 1;
    }
    h->pending.clear();
    h->ev_used = 0;
    return MG_OK;
}

// wraps one launch with optional timing events
template <typename F>
int run_timed(mg_ctx* h, int kind, int level, hipStream_t st, F&& launch) {
    TimedLaunch tl;
    const bool on = timed(h, kind, level);
    if (on) {
        int rc = time_begin(h, kind, level, st, &tl);
        if (rc) return rc;
    }
    hipError_t e = launch();
    if (e != hipSuccess) {
        launch_events() = LaunchEvents();
        return fail(MG_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    if (on) return time_end(h, tl, st);
    return MG_OK;
}

// ---- cycle pieces ------------------------------------------------------

Sweep make_sweep(const mg_ctx* h, const Hier& H, int l) {
    Sweep s;
    s.d = h->d;
    s.n = level_n(h, l);
    s.batch = h->batch;
    double pf;
    level_scales(h, H, l, &s.sA, &s.sW, &pf);
    for (int j = 0; j < 4; ++j) s.c[j] = j < h->ncoef ? h->c[j] : 0.0;
    return s;
}

int run_tail(mg_ctx* h, Hier& H, int l, const void* b, void* e, hipStream_t st,
             int wvisits = 0) {
    Tail t;
    t.wvisits = wvisits;
    t.d = h->d;
    t.nt = level_n(h, l);
    t.batch = h->batch;
    t.b = b;
    t.e = e;
    for (int j = 0; j < 4; ++j) t.c[j] = j < h->ncoef ? h->c[j] : 0.0;
    t.ginv = H.ginv;
    t.scaled = H.scaled;
    return run_timed(h, MG_TIME_TAIL, l, st, [&] { return launch_tail(H.p, t, st); });
}

// Where the pre-smoother's residual norm goes (fine FP64 level only).
struct NormReq {
    int slot = -1;                  // dnorm slot, -1 = none
};

// A 3D hierarchy with the 19-/27-point smoother (nonzero edge or corner
// coefficient): its sweeps use the wide variant of the smoother kernel and
// the separate restriction (the fused smoother + restriction kernels carry
// the 7-point stencil only).
bool wide_3d(const mg_ctx* h) { return h->d == 3 && (h->c[2] != 0.0 || h->c[3] != 0.0); }

// Where the zero-guess pre-smoother and the restriction run as one kernel:
// 2D, every level above the tail (a tile kernel; its halo costs 1.3x the
// reads of b); 3D with the 7-point stencil, every level: grids of 200 or
// more nodes per direction in the restriction's march forming e from b on
// the fly (87 against 111 us at n = 255 in FP64, 327 against 478 us at
// n = 511 with FP32 storage), smaller ones in the 3D tile kernel (one
// launch instead of two; the march's twelve-plane unroll made short marches
// slower than the two sweeps, 12.5 against 9.6 us at n = 63).
bool fuse_zero_restrict(const mg_ctx* h, int l) {
    (void)l;
    return h->d == 2 || !wide_3d(h);
}

// Where the pre-smoother from a nonzero iterate (the finest level of every
// cycle, the second coarse visit of a W(1,0) cycle) and the restriction run
// as one kernel: 2D, every level (88 against 136 us at n = 4095); 3D grids
// of 200 or more nodes per direction (108 against 138 us at n = 255; on
// smaller grids the ring-3 halo of its tiles costs what the fusion saves).
bool fuse_smooth_restrict(const mg_ctx* h, int l) {
    return h->d == 2 || (level_n(h, l) >= 200 && !wide_3d(h));
}

// Which part of a cycle to enqueue: all of it, only the pre-smoother (with
// its norm), or everything after the pre-smoother (tmp holds its output).
enum CyclePart { kWhole = 0, kPreOnly = 1, kRest = 2 };

int cycle(mg_ctx* h, Hier& H, int l, const void* u_in, const void* b, void* out, void* tmp,
          const NormReq& nr, hipStream_t st, CyclePart part = kWhole);

// The part of a cycle after the restriction: the coarse visit(s), then
// the post-smoother with the fused correction (V) or the correction alone
// (W).  s holds the level's sweep parameters; tmp the pre-smoothed iterate.
int coarse_and_post(mg_ctx* h, Hier& H, int l, void* tmp, void* out, Sweep s, double pf,
                    bool wcycle, hipStream_t st) {
    int rc;
    if (wcycle) {
        // gamma = 2: the coarse problem twice, the second visit starting from
        // the first's result (both visits in one tail launch at or below the
        // tail size); no post-smoothing: out = tmp + pf P e_{l+1}
        if (l + 1 == h->L - 1 || l + 1 >= tail_level(h, true)) {
            rc = run_tail(h, H, l + 1, H.b[l + 1], H.e[l + 1], st, 2);
        } else {
            rc = cycle(h, H, l + 1, nullptr, H.b[l + 1], H.e[l + 1], H.t[l + 1], NormReq(), st);
            if (rc) return rc;
            rc = cycle(h, H, l + 1, H.e[l + 1], H.b[l + 1], H.e[l + 1], H.t[l + 1], NormReq(),
                       st);
        }
        if (rc) return rc;
        return run_timed(h, MG_TIME_PROLONG, l, st, [&] {
            return launch_prolong_to(H.p, h->d, s.n, h->batch, H.e[l + 1], tmp, out, pf, st);
        });
    }
    rc = cycle(h, H, l + 1, nullptr, H.b[l + 1], H.e[l + 1], H.t[l + 1], NormReq(), st);
    if (rc) return rc;
    s.u = tmp;
    s.out = out;
    // post-smoothing of tmp + pf P e_{l+1}: the correction is fused into the
    // sweep on every level (on small grids it costs no more than a plain
    // sweep, and saves the separate correction launch)
    s.ec = H.e[l + 1];
    s.pf = pf;
    return run_timed(h, MG_TIME_SMOOTH_CORRECT, l, st,
                     [&] { return launch_smooth(H.p, false, false, s, st, nullptr); });
}

// One cycle (V(1,1), or W(1,0) under MG_CYCLE_W10) on hierarchy H at level
// l: out = V(u_in, b), or from a zero guess when u_in is null.  tmp receives
// the pre-smoothed iterate (must differ from u_in, b and out; out may alias
// u_in).  Coarser levels use H.b / H.e / H.t.  Zero-guess cycles at or
// below the tail size run in the single-workgroup LDS tail kernel (the
// coarsest grid is always solved exactly there); above it their
// pre-smoother and restriction are one fused kernel.
int cycle(mg_ctx* h, Hier& H, int l, const void* u_in, const void* b, void* out, void* tmp,
          const NormReq& nr, hipStream_t st, CyclePart part) {
    const bool zero = u_in == nullptr;
    const bool wcycle = h->cycle_kind == MG_CYCLE_W10;
    int rc, nparts = 0;
    // zero-guess cycles at or below the tail size run in the LDS tail
    if (l == h->L - 1 || (zero && l >= tail_level(h, true))) {
        if (part != kWhole) return fail(MG_EINVAL, "split cycle on the tail level");
        if (nr.slot >= 0) {
            // only a single-grid FP64 problem (N = 4) gets here with a norm
            HIPCHK(launch_residual_norm(h->d, level_n(h, l), h->batch,
                                        static_cast<const double*>(u_in),
                                        static_cast<const double*>(b), (double)h->N * h->N,
                                        h->psum, h->pmax, kPartialCap * h->batch, st, &nparts));
            HIPCHK(launch_finalize(h->psum, nullptr, nparts, h->dnorm + 2 * nr.slot, st,
                                   h->hnorm_dev + 2 * nr.slot));
        }
        return run_tail(h, H, l, b, out, st, wcycle ? 1 : 0);
    }
    Sweep s = make_sweep(h, H, l);
    double sA, sW, pf;
    level_scales(h, H, l, &sA, &sW, &pf);
    s.u = u_in;
    s.b = b;
    s.out = tmp;
    const bool norm = nr.slot >= 0 && !zero && H.p == P64;
    s.partials = h->psum;
    s.partials_cap = kPartialCap * h->batch;
    if (zero && part == kWhole && fuse_zero_restrict(h, l)) {
        // zero-guess pre-smoothing and the restriction in one kernel (it
        // also reduces a pending norm in its first workgroup, as the
        // restriction would)
        s.out_c = H.b[l + 1];
        const mg_ctx::PendingNorm pz = h->pend;
        if (pz.count > 0) {
            s.fin_ps = h->psum;
            s.fin_pm = pz.with_max ? h->pmax : nullptr;
            s.fin_count = pz.count;
            s.fin_dev = h->dnorm + 2 * pz.slot;
            s.fin_host = h->hnorm_dev + 2 * pz.slot;
            h->pend = mg_ctx::PendingNorm();
        }
        rc = run_timed(h, MG_TIME_ZERO_SMOOTH_RESTRICT, l, st,
                       [&] { return launch_zero_smooth_restrict(H.p, s, st); });
        if (rc) return rc;
        s.out_c = nullptr;
        s.fin_ps = s.fin_pm = nullptr;
        s.fin_count = 0;
        s.fin_dev = s.fin_host = nullptr;
        return coarse_and_post(h, H, l, tmp, out, s, pf, wcycle, st);
    }
    if (!zero && fuse_smooth_restrict(h, l)) {
        // pre-smoothing and the restriction in one kernel; its norm stays
        // pending for the next restriction-type kernel (or the flush)
        if (part != kRest) {
            s.out_c = H.b[l + 1];
            const bool bn = norm && l == 0 && h->bnorm_req;
            if (bn) s.bparts = h->psum_b;
            rc = run_timed(h, MG_TIME_SMOOTH_RESTRICT, l, st, [&] {
                return launch_smooth_restrict(H.p, norm, s, st, &nparts);
            });
            if (rc) return rc;
            if (bn) {
                h->bnorm_req = false;
                h->bnorm_parts = nparts;
            }
            s.bparts = nullptr;
            if (norm) {
                h->pend.count = nparts;
                h->pend.with_max = false;
                h->pend.slot = nr.slot;
            }
            s.out_c = nullptr;
            if (part == kPreOnly) return MG_OK;
        }
        s.partials = nullptr;
        return coarse_and_post(h, H, l, tmp, out, s, pf, wcycle, st);
    }
    if (part != kRest) {
        rc = run_timed(h, zero ? MG_TIME_SMOOTH_ZERO : MG_TIME_SMOOTH, l, st,
                       [&] { return launch_smooth(H.p, zero, norm, s, st, &nparts); });
        if (rc) return rc;
        if (norm) {
            h->pend.count = nparts;
            h->pend.with_max = false;
            h->pend.slot = nr.slot;
        }
        if (part == kPreOnly) return MG_OK;
    }
    s.u = tmp;
    s.out = H.b[l + 1];
    s.partials = nullptr;
    const mg_ctx::PendingNorm pn = h->pend;
    if (pn.count > 0) {
        // the restriction's first workgroup reduces the pending norm
        s.fin_ps = h->psum;
        s.fin_pm = pn.with_max ? h->pmax : nullptr;
        s.fin_count = pn.count;
        s.fin_dev = h->dnorm + 2 * pn.slot;
        s.fin_host = h->hnorm_dev + 2 * pn.slot;
        h->pend = mg_ctx::PendingNorm();
    }
    rc = run_timed(h, MG_TIME_RESTRICT, l, st, [&] { return launch_restrict(H.p, s, st); });
    if (rc) return rc;
    s.fin_ps = s.fin_pm = nullptr;
    s.fin_count = 0;
    s.fin_dev = s.fin_host = nullptr;
    return coarse_and_post(h, H, l, tmp, out, s, pf, wcycle, st);
}

// Reduces a pending norm that no restriction has picked up (tail-only
// hierarchies) with the standalone kernel and a copy to the host mirror.
int flush_pending_norm(mg_ctx* h, hipStream_t st) {
    const mg_ctx::PendingNorm pn = h->pend;
    if (pn.count == 0) return MG_OK;
    h->pend = mg_ctx::PendingNorm();
    HIPCHK(launch_finalize(h->psum, pn.with_max ? h->pmax : nullptr, pn.count,
                           h->dnorm + 2 * pn.slot, st, h->hnorm_dev + 2 * pn.slot));
    return MG_OK;
}

// One FP64 V(1,1) cycle on the finest grid: u_out = V(u_in, b).  With
// norm_slot >= 0 the pre-smoother also produces ||b - A u_in||_2 into
// dnorm[2 slot] and the host mirror (arm the slot first to poll it).
int fine_cycle64(mg_ctx* h, const double* b, const double* u_in, double* u_out,
                 int norm_slot, hipStream_t st, CyclePart part = kWhole) {
    NormReq nr;
    nr.slot = norm_slot;
    const int rc = cycle(h, h->h64, 0, u_in, b, u_out, h->h64.t[0], nr, st, part);
    if (rc) return rc;
    return flush_pending_norm(h, st);
}

// The solves learn ||r_k|| only while the work that follows it runs, so a
// converged solve normally discards the rest of one cycle.  When the last
// reduction factor predicts ||r_k|| <= kGateSlack tol ||r_0||, the loop
// instead waits for the norm before enqueueing that work (one host round
// trip, against most of a cycle).
constexpr double kGateSlack = 4.0;

// an in-place cycle (no ping-pong) is taken only when the predicted
// ||r_k|| exceeds the tolerance by this factor
constexpr double kFlipMargin = 100.0;

bool predict_final(const std::vector<double>& hist, double tol, double r0) {
    const size_t k = hist.size();
    if (k < 2 || !(hist[k - 2] > 0.0)) return false;
    const double q = hist[k - 1] / hist[k - 2];
    return q < 1.0 && hist[k - 1] * q <= kGateSlack * tol * r0;
}

int check_handle(mg_ctx* h) {
    if (!h) return fail(MG_EINVAL, "null handle");
    return MG_OK;
}

// ||b||_2 over the whole batch for mg_stats: one pass over b at the start
// of a solve into the last norm slot (the solves use slots 0 .. max_cycles
// + 1), copied to the pinned host mirror, read after the final
// synchronisation.
int bnorm_slot(const mg_ctx* h) { return h->norm_slots - 1; }

int enqueue_bnorm(mg_ctx* h, const double* b, hipStream_t st) {
    int np = 0;
    const int sl = bnorm_slot(h);
    HIPCHK(launch_sumsq(b, level_pts(h, 0) * h->batch, h->psum, kPartialCap * h->batch, st, &np));
    HIPCHK(launch_finalize(h->psum, nullptr, np, h->dnorm + 2 * sl, st, h->hnorm_dev + 2 * sl));
    return MG_OK;
}

// The solves ask their first kernel that reads all of b (the first cycle's
// fused fine pre-smoother beside ||r_0||^2; in refinement the residual pass
// or the first step) to sum b^2 too, which saves a pass over b; the
// partials are reduced at the end of the solve, or b gets its own pass if
// no kernel took the request.
void request_bnorm(mg_ctx* h) {
    h->bnorm_req = true;
    h->bnorm_parts = 0;
}

int finish_bnorm(mg_ctx* h, const double* b, hipStream_t st) {
    h->bnorm_req = false;
    if (h->bnorm_parts == 0) return enqueue_bnorm(h, b, st);
    const int sl = bnorm_slot(h);
    HIPCHK(launch_finalize(h->psum_b, nullptr, h->bnorm_parts, h->dnorm + 2 * sl, st,
                           h->hnorm_dev + 2 * sl));
    h->bnorm_parts = 0;
    return MG_OK;
}

// Host hand-off of the per-cycle norms: the kernel that reduces a norm
// stores it into the coherent host mirror with a system-scope store, so the
// host reads it as soon as that workgroup has run, with no event (an event
// after a large kernel idles the GPU ~5 us while the caches are written
// back).  A slot is armed with a value no norm takes before the work that
// fills it is enqueued; wait_norm polls it and, should the stream drain or
// fail first, stops with an error instead of spinning on.
constexpr double kNormPending = -1.0;

void arm_norm(mg_ctx* h, int slot) {
    reinterpret_cast<volatile double*>(h->hnorm)[2 * slot] = kNormPending;
}

int wait_norm(mg_ctx* h, int slot, hipStream_t st, double* out) {
    const volatile double* p = h->hnorm + 2 * slot;
    using clk = std::chrono::steady_clock;
    clk::time_point next = clk::now() + std::chrono::milliseconds(20);
    for (long it = 1;; ++it) {
        const double v = *p;
        if (!(v == kNormPending)) {  // a NaN norm ends the wait as well
            *out = v;
            return MG_OK;
        }
        // The stream is queried only every 20 ms of spinning, far beyond the
        // time a norm takes: the kernel launched after a query (as after an
        // event wait) starts ~5.7 us after its predecessor ends (measured;
        // back-to-back kernels start without a gap), so a normal wait never
        // queries.
        if ((it & 4095) == 0 && clk::now() >= next) {
            next = clk::now() + std::chrono::milliseconds(20);
            const hipError_t e = hipStreamQuery(st);
            if (e == hipSuccess) {
                const double w = *p;
                if (w == kNormPending)
                    return fail(MG_EHIP, "norm slot " + std::to_string(slot) +
                                             " not written by the stream's kernels");
                *out = w;
                return MG_OK;
            }
            if (e != hipErrorNotReady)
                return fail(MG_EHIP, std::string("hipStreamQuery: ") + hipGetErrorString(e));
        }
    }
}

// Checks the problem arguments of mg_setup and mg_vcycle_noalloc.
int check_problem(int N, int d, const double* coeffs, int n_coeffs) {
    if (d != 2 && d != 3) return fail(MG_EINVAL, "d must be 2 or 3");
    if (N < 4 || (N & (N - 1)) != 0) return fail(MG_EINVAL, "N must be a power of two >= 4");
    if ((d == 2 && N > 65536) || (d == 3 && N > 2048)) return fail(MG_EINVAL, "N too large");
    if (!coeffs || (d == 2 && n_coeffs != 3) || (d == 3 && (n_coeffs < 2 || n_coeffs > 4)))
        return fail(MG_EINVAL, d == 2 ? "2D takes 3 coefficients"
                                      : "3D takes 2, 3 or 4 coefficients");
    for (int j = 0; j < n_coeffs; ++j)
        if (!std::isfinite(coeffs[j])) return fail(MG_EINVAL, "coefficients must be finite");
    return MG_OK;
}

// Problem fields of a context (arguments already checked); the level count
// of N <= 65536 stays below kMaxLevels.
void init_problem(mg_ctx* h, int N, int d, const double* coeffs, int n_coeffs) {
    h->N = N;
    h->d = d;
    h->ncoef = n_coeffs;
    for (int j = 0; j < h->ncoef; ++j) h->c[j] = coeffs[j];
    h->L = 0;
    for (int M = N; M >= 4; M /= 2) h->L++;
}

// ---- the handle-free cycle on a static workspace -------------------------

constexpr size_t kScratchBytes = MG_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// Per-device addresses of the static arrays below, looked up once per device
// with that device current (host code never passes the arrays' own names,
// which are host-side stand-ins).
struct StaticDevice {
    bool ready = false;
    unsigned char* scratch = nullptr;
    double* inv2 = nullptr;  // A_0^{-1} of the FP64 hierarchy, 2D (9 x 9)
    double* inv3 = nullptr;  // 3D (27 x 27)
};
StaticDevice g_static[kMaxDevices];
std::mutex g_static_mu;

}  // namespace

// The workspace of mg_vcycle_noalloc: every internal buffer of its cycle
// (the pre-smoothed fine iterate, and the correction, right-hand side and
// pre-smoothed iterate of every coarser level) is carved from this array.
// Each device holds its own copy from module load until the process ends.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
// The coarsest-grid inverses of the FP64 hierarchy, initialised in the code
// object.  Not const: the device compiler drops a const variable that no
// device code reads, and the runtime then cannot resolve the host's lookup.
static __device__ StencilInverse<9> g_inv2_64 = kInv2_64;
static __device__ StencilInverse<27> g_inv3_64 = kInv3_64;

namespace {

int static_setup(int dev, StaticDevice** out) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticDevice& sd = g_static[dev];
    if (!sd.ready) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        sd.scratch = static_cast<unsigned char*>(p);
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(g_inv2_64)));
        sd.inv2 = static_cast<double*>(p);
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(g_inv3_64)));
        sd.inv3 = static_cast<double*>(p);
        sd.ready = true;
    }
    *out = &sd;
    return MG_OK;
}

// Workspace layout of the FP64 cycle: level 0 needs its pre-smoothed
// iterate t, every coarser level e, b and t; each buffer starts on a
// 256-byte boundary.  Returns the bytes needed; with base != nullptr also
// points H's buffers into base.
size_t carve_hier(const mg_ctx* h, Hier* H, unsigned char* base) {
    size_t off = 0;
    auto take = [&](long pts) {
        const size_t at = off;
        off += ((size_t)pts * h->batch * sizeof(double) + 255) / 256 * 256;
        return base ? static_cast<void*>(base + at) : nullptr;
    };
    for (int l = 0; l < h->L; ++l) {
        const long pts = level_pts(h, l);
        if (l > 0) {
            void* e = take(pts);
            void* b = take(pts);
            if (H) {
                H->e[l] = e;
                H->b[l] = b;
            }
        }
        void* t = take(pts);
        if (H) H->t[l] = t;
    }
    return off;
}

}  // namespace

// ============================================================== C ABI

extern "C" {

const char* mg_last_error(void) { return g_err.c_str(); }

int mg_setup(int N, int d, const double* coeffs, int n_coeffs, mg_handle_t* out) {
    if (!out) return fail(MG_EINVAL, "out is NULL");
    *out = nullptr;
    if (check_problem(N, d, coeffs, n_coeffs)) return MG_EINVAL;
    mg_ctx* h = new mg_ctx;
    init_problem(h, N, d, coeffs, n_coeffs);
    int rc = realloc_all(h);
    if (rc) {
        mg_destroy(h);
        return rc;
    }
    hipError_t e1 = hipEventCreate(&h->ev0), e2 = hipEventCreate(&h->ev1);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        mg_destroy(h);
        return fail(MG_EHIP, "hipEventCreate failed");
    }
    *out = h;
    return MG_OK;
}

int mg_set_coeffs(mg_handle_t h, const double* coeffs, int n_coeffs) {
    if (check_handle(h)) return MG_EINVAL;
    if (!coeffs || n_coeffs != h->ncoef) return fail(MG_EINVAL, "wrong coefficient count");
    for (int j = 0; j < n_coeffs; ++j)
        if (!std::isfinite(coeffs[j])) return fail(MG_EINVAL, "coefficients must be finite");
    for (int j = 0; j < n_coeffs; ++j) h->c[j] = coeffs[j];
    return MG_OK;
}

int mg_set_option(mg_handle_t h, int key, double value) {
    if (check_handle(h)) return MG_EINVAL;
    // range first: converting a NaN, an infinity or a value outside the int
    // range to int is undefined
    if (!std::isfinite(value) || std::fabs(value) > 1e9)
        return fail(MG_EINVAL, "option value out of range");
    const int v = (int)value;
    if ((double)v != value) return fail(MG_EINVAL, "option values are integers");
    switch (key) {
        case MG_OPT_PRECISION:
            if (v < MG_PREC_FP64 || v > MG_PREC_FP16_IR) return fail(MG_EINVAL, "bad precision");
            if (v == h->prec) return MG_OK;
            h->prec = v;
            return realloc_all(h);
        case MG_OPT_BATCH:
            if (v < 1 || v > 65535) return fail(MG_EINVAL, "batch must be 1..65535");
            if (v == h->batch) return MG_OK;
            h->batch = v;
            return realloc_all(h);
        case MG_OPT_MAX_CYCLES:
            if (v < 1 || v > 10000) return fail(MG_EINVAL, "max cycles must be 1..10000");
            h->max_cycles = v;
            return alloc_common(h);
        case MG_OPT_TAIL_N: {
            if (v == 0) {
                h->tail_N = 0;
                return MG_OK;
            }
            const int lim = h->d == 2 ? 64 : 16;
            if (v < 4 || v > lim || (v & (v - 1)) != 0)
                return fail(MG_EINVAL, "tail N must be a power of two in 4..64 (2D) or 4..16 (3D)");
            h->tail_N = v;
            return MG_OK;
        }
        case MG_OPT_TIMING:
            if (v < 0 || v > 3) return fail(MG_EINVAL, "timing must be 0, 1, 2 or 3");
            h->timing = v;
            return MG_OK;
        case MG_OPT_INNER_CYCLES:
            if (v < 0 || v > 16) return fail(MG_EINVAL, "inner cycles must be 0..16");
            h->inner = v;
            return MG_OK;
        case MG_OPT_CYCLE:
            if (v != MG_CYCLE_V11 && v != MG_CYCLE_W10)
                return fail(MG_EINVAL, "cycle must be MG_CYCLE_V11 or MG_CYCLE_W10");
            h->cycle_kind = v;
            return MG_OK;
        default:
            return fail(MG_EINVAL, "unknown option");
    }
}

int mg_num_levels(mg_handle_t h) { return h ? h->L : MG_EINVAL; }

int mg_vcycle(mg_handle_t h, const double* b, double* u, void* stream) {
    if (check_handle(h)) return MG_EINVAL;
    if (!b || !u) return fail(MG_EINVAL, "null field pointer");
    hipStream_t st = (hipStream_t)stream;
    // u is updated in place: the post-smoother reads the internal iterate
    // and writes u, and the pre-smoother never writes u
    h->pend = mg_ctx::PendingNorm();
    h->call_fused = 0;
    return fine_cycle64(h, b, u, u, -1, st);
}

int mg_vcycle_noalloc(int N, int d, const double* coeffs, int n_coeffs, int batch,
                      const double* b, double* u, void* stream) {
    if (check_problem(N, d, coeffs, n_coeffs)) return MG_EINVAL;
    if (batch < 1 || batch > 65535) return fail(MG_EINVAL, "batch must be 1..65535");
    if (!b || !u) return fail(MG_EINVAL, "null field pointer");
    // the context lives on the stack: its containers stay empty, timing is
    // off and no norm is requested, so the cycle neither allocates nor
    // synchronises
    mg_ctx h;
    init_problem(&h, N, d, coeffs, n_coeffs);
    h.batch = batch;
    const size_t need = carve_hier(&h, nullptr, nullptr);
    if (need > kScratchBytes)
        return fail(MG_EINVAL, "problem needs " + std::to_string(need) +
                                   " bytes of workspace; the static workspace holds " +
                                   std::to_string(kScratchBytes));
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MG_EINVAL, "device index out of range");
    StaticDevice* sd = nullptr;
    int rc = static_setup(dev, &sd);
    if (rc) return rc;
    Hier& H = h.h64;
    H.p = P64;
    H.scaled = false;
    carve_hier(&h, &H, sd->scratch);
    H.ginv = d == 2 ? sd->inv2 : sd->inv3;
    H.ginv_owned = false;
    H.allocated = true;
    return fine_cycle64(&h, b, u, u, -1, (hipStream_t)stream);
}

int mg_sweep(mg_handle_t h, int op, int level, int prec, const void* u, const void* b,
             void* out, void* stream) {
    if (check_handle(h)) return MG_EINVAL;
    if (prec < MG_PREC_FP64 || prec > MG_PREC_FP16_IR) return fail(MG_EINVAL, "bad precision");
    if (level < 0 || level >= h->L) return fail(MG_EINVAL, "bad level");
    if (!out) return fail(MG_EINVAL, "null output");
    if (op != MG_OP_SMOOTH_ZERO && !u) return fail(MG_EINVAL, "null u");
    if (op != MG_OP_PROLONG_ADD && !b) return fail(MG_EINVAL, "null b");
    if ((op == MG_OP_RESTRICT || op == MG_OP_PROLONG_ADD) && level >= h->L - 1)
        return fail(MG_EINVAL, "no coarser level");
    const Prec p = prec == MG_PREC_FP64 ? P64 : (prec == MG_PREC_FP32_IR ? P32 : P16);
    Hier H;
    H.p = p;
    H.scaled = p != P64;
    Sweep s = make_sweep(h, H, level);
    double sA, sW, pf;
    level_scales(h, H, level, &sA, &sW, &pf);
    hipStream_t st = (hipStream_t)stream;
    s.u = u;
    s.b = b;
    s.out = out;
    hipError_t e;
    switch (op) {
        case MG_OP_SMOOTH: e = launch_smooth(p, false, false, s, st, nullptr); break;
        case MG_OP_SMOOTH_ZERO: e = launch_smooth(p, true, false, s, st, nullptr); break;
        case MG_OP_RESTRICT: e = launch_restrict(p, s, st); break;
        case MG_OP_PROLONG_ADD:
            e = launch_prolong(p, h->d, s.n, h->batch, u, out, pf, st);
            break;
        default: return fail(MG_EINVAL, "bad op");
    }
    if (e != hipSuccess) return fail(MG_EHIP, std::string("launch: ") + hipGetErrorString(e));
    return MG_OK;
}

int mg_sweep_zero_restrict(mg_handle_t h, int level, int prec, const void* b, void* e, void* bc,
                           void* stream) {
    if (check_handle(h)) return MG_EINVAL;
    if (prec < MG_PREC_FP64 || prec > MG_PREC_FP16_IR) return fail(MG_EINVAL, "bad precision");
    if (level < 0 || level >= h->L - 1) return fail(MG_EINVAL, "bad level (no coarser level)");
    if (!b || !e || !bc) return fail(MG_EINVAL, "null field pointer");
    if (wide_3d(h))
        return fail(MG_EINVAL, "the fused smoother + restriction kernels take the 7-point "
                               "3D stencil (edge and corner coefficients must be zero)");
    const Prec p = prec == MG_PREC_FP64 ? P64 : (prec == MG_PREC_FP32_IR ? P32 : P16);
    Hier H;
    H.p = p;
    H.scaled = p != P64;
    Sweep s = make_sweep(h, H, level);
    s.b = b;
    s.out = e;
    s.out_c = bc;
    const hipError_t err = launch_zero_smooth_restrict(p, s, (hipStream_t)stream);
    if (err != hipSuccess) return fail(MG_EHIP, std::string("launch: ") + hipGetErrorString(err));
    return MG_OK;
}

int mg_sweep_smooth_restrict(mg_handle_t h, int level, int prec, const void* u, const void* b,
                             void* out, void* bc, void* stream) {
    if (check_handle(h)) return MG_EINVAL;
    if (prec < MG_PREC_FP64 || prec > MG_PREC_FP16_IR) return fail(MG_EINVAL, "bad precision");
    if (level < 0 || level >= h->L - 1) return fail(MG_EINVAL, "bad level (no coarser level)");
    if (!u || !b || !out || !bc) return fail(MG_EINVAL, "null field pointer");
    if (wide_3d(h))
        return fail(MG_EINVAL, "the fused smoother + restriction kernels take the 7-point "
                               "3D stencil (edge and corner coefficients must be zero)");
    const Prec p = prec == MG_PREC_FP64 ? P64 : (prec == MG_PREC_FP32_IR ? P32 : P16);
    Hier H;
    H.p = p;
    H.scaled = p != P64;
    Sweep s = make_sweep(h, H, level);
    s.u = u;
    s.b = b;
    s.out = out;
    s.out_c = bc;
    const hipError_t err =
        launch_smooth_restrict(p, false, s, (hipStream_t)stream, nullptr);
    if (err != hipSuccess) return fail(MG_EHIP, std::string("launch: ") + hipGetErrorString(err));
    return MG_OK;
}

int mg_sweep_post_pre_restrict(mg_handle_t h, int level, int prec, const void* u,
                               const void* ec, const void* b, void* out, void* out_t, void* bc,
                               void* stream) {
    if (check_handle(h)) return MG_EINVAL;
    if (prec < MG_PREC_FP64 || prec > MG_PREC_FP16_IR) return fail(MG_EINVAL, "bad precision");
    if (level < 0 || level >= h->L - 1) return fail(MG_EINVAL, "bad level (no coarser level)");
    if (!u || !ec || !b || !out || !out_t || !bc) return fail(MG_EINVAL, "null field pointer");
    if (h->d != 2) return fail(MG_EINVAL, "the fused post- and pre-smoother is 2D only");
    const Prec p = prec == MG_PREC_FP64 ? P64 : (prec == MG_PREC_FP32_IR ? P32 : P16);
    Hier H;
    H.p = p;
    H.scaled = p != P64;
    Sweep s = make_sweep(h, H, level);
    double sA, sW, pf;
    level_scales(h, H, level, &sA, &sW, &pf);
    s.u = u;
    s.ec = ec;
    s.pf = pf;
    s.b = b;
    s.out = out;
    s.out_t = out_t;
    s.out_c = bc;
    const hipError_t err =
        launch_post_pre_restrict(p, false, s, (hipStream_t)stream, nullptr);
    if (err != hipSuccess) return fail(MG_EHIP, std::string("launch: ") + hipGetErrorString(err));
    return MG_OK;
}

int mg_sweep_correct(mg_handle_t h, int level, int prec, const void* u, const void* ec,
                     const void* b, void* out, void* stream) {
    if (check_handle(h)) return MG_EINVAL;
    if (prec < MG_PREC_FP64 || prec > MG_PREC_FP16_IR) return fail(MG_EINVAL, "bad precision");
    if (level < 0 || level >= h->L - 1) return fail(MG_EINVAL, "bad level (needs a coarser one)");
    if (!u || !ec || !b || !out) return fail(MG_EINVAL, "null field pointer");
    const Prec p = prec == MG_PREC_FP64 ? P64 : (prec == MG_PREC_FP32_IR ? P32 : P16);
    Hier H;
    H.p = p;
    H.scaled = p != P64;
    Sweep s = make_sweep(h, H, level);
    double sA, sW, pf;
    level_scales(h, H, level, &sA, &sW, &pf);
    s.u = u;
    s.b = b;
    s.out = out;
    s.ec = ec;
    s.pf = pf;
    hipError_t e = launch_smooth(p, false, false, s, (hipStream_t)stream, nullptr);
    if (e != hipSuccess) return fail(MG_EHIP, std::string("launch: ") + hipGetErrorString(e));
    return MG_OK;
}

int mg_coarse_cycle(mg_handle_t h, int level, int prec, const void* b, void* e,
                    void* stream) {
    if (check_handle(h)) return MG_EINVAL;
    if (!b || !e) return fail(MG_EINVAL, "null field pointer");
    if (prec < MG_PREC_FP64 || prec > MG_PREC_FP16_IR) return fail(MG_EINVAL, "bad precision");
    if (level < 0 || level >= h->L) return fail(MG_EINVAL, "bad level");
    Hier* H;
    if (prec == MG_PREC_FP64) {
        H = &h->h64;
    } else {
        if (prec != h->prec) return fail(MG_EINVAL, "set MG_OPT_PRECISION to this precision first");
        H = &h->hlo;
    }
    hipStream_t st = (hipStream_t)stream;
    void* tmp = H->t[level];
    h->pend = mg_ctx::PendingNorm();
    int rc = cycle(h, *H, level, nullptr, b, e, tmp, NormReq(), st);
    if (rc) return rc;
    return MG_OK;
}

int mg_residual_norm(mg_handle_t h, const double* b, const double* u, double* norm,
                     void* stream) {
    if (check_handle(h)) return MG_EINVAL;
    if (!b || !u || !norm) return fail(MG_EINVAL, "null pointer");
    hipStream_t st = (hipStream_t)stream;
    int nparts = 0;
    const double N = h->N;
    int rc = run_timed(h, MG_TIME_RESIDUAL, 0, st, [&] {
        return launch_residual_norm(h->d, level_n(h, 0), h->batch, u, b, N * N, h->psum,
                                    h->pmax, kPartialCap * h->batch, st, &nparts);
    });
    if (rc) return rc;
    HIPCHK(launch_finalize(h->psum, h->pmax, nparts, h->dnorm, st));
    HIPCHK(hipMemcpyAsync(h->hnorm, h->dnorm, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    rc = time_collect(h);
    if (rc) return rc;
    *norm = h->hnorm[0];
    return MG_OK;
}

// FP64 V(1,1) solves in 2D run chained: the post-smoother of cycle k and the
// pre-smoother and restriction of cycle k + 1 are one kernel (it also yields
// ||r_{k+1}|| and writes u_{k+1} straight into the caller's buffer), so a
// cycle is that kernel plus the coarse levels.  Same arithmetic per cycle
// as the separate kernels; the answer is always in u, so neither ping-pong
// nor an in-place cycle is needed.
bool chain_2d(const mg_ctx* h) {
    return h->d == 2 && h->L >= 2 && h->cycle_kind == MG_CYCLE_V11;
}

static int solve64_chain(mg_ctx* h, const double* b, double* u, double tol, mg_stats* st_out,
                         hipStream_t st) {
    Hier& H = h->h64;
    double* tcur = static_cast<double*>(H.t[0]);
    double* tnext = h->ualt;  // free: the iterate never ping-pongs here
    HIPCHK(hipEventRecord(h->ev0, st));
    std::vector<double> hist;
    double r0 = 0.0, rk = 0.0;
    int k = 0, code = MG_OK, run = 0;
    h->bnorm_req = false;
    if (st_out) request_bnorm(h);
    Sweep s = make_sweep(h, H, 0);
    double sA, sW, pf;
    level_scales(h, H, 0, &sA, &sW, &pf);
    s.partials = h->psum;
    s.partials_cap = kPartialCap * h->batch;
    s.b = b;
    s.out_c = H.b[1];
    int nparts = 0, rc;
    auto pend = [&](int slot) {
        h->pend.count = nparts;
        h->pend.with_max = false;
        h->pend.slot = slot;
    };
    // the coarse part of a cycle (its first restriction-type kernel reduces
    // the pending norm), or only the norm's reduction
    auto coarse = [&]() {
        const int r = cycle(h, H, 1, nullptr, H.b[1], H.e[1], H.t[1], NormReq(), st);
        if (r) return r;
        return flush_pending_norm(h, st);
    };
    // cycle 0: pre-smoother and restriction, with ||r_0||
    s.u = u;
    s.out = tcur;
    s.bparts = h->bnorm_req ? h->psum_b : nullptr;
    arm_norm(h, 0);
    rc = run_timed(h, MG_TIME_SMOOTH_RESTRICT, 0, st,
                   [&] { return launch_smooth_restrict(P64, true, s, st, &nparts); });
    if (rc) return rc;
    if (s.bparts) {
        h->bnorm_req = false;
        h->bnorm_parts = nparts;
        s.bparts = nullptr;
    }
    pend(0);
    run = 1;
    bool gate = false;
    rc = coarse();
    if (rc) return rc;
    for (k = 0;; ++k) {
        // u_k is in u; the pre-smoothed iterate of cycle k in tcur, its
        // coarse problem enqueued unless gated
        double nk;
        rc = wait_norm(h, k, st, &nk);
        if (rc) return rc;
        if (!std::isfinite(nk)) {
            code = MG_ENONFINITE;
            rk = nk;
            break;
        }
        if (k == 0) r0 = nk;
        hist.push_back(nk);
        rk = nk;
        if (nk <= tol * r0) break;
        if (k >= h->max_cycles) {
            code = MG_ENOCONV;
            break;
        }
        if (gate) {
            rc = cycle(h, H, 1, nullptr, H.b[1], H.e[1], H.t[1], NormReq(), st);
            if (rc) return rc;
        }
        // post-smoother of cycle k with the coarse correction, then the
        // pre-smoother and restriction of cycle k + 1, with ||r_{k+1}||
        s.u = tcur;
        s.ec = H.e[1];
        s.pf = pf;
        s.out = u;
        s.out_t = tnext;
        arm_norm(h, k + 1);
        rc = run_timed(h, MG_TIME_POST_PRE_RESTRICT, 0, st,
                       [&] { return launch_post_pre_restrict(P64, true, s, st, &nparts); });
        if (rc) return rc;
        pend(k + 1);
        ++run;
        std::swap(tcur, tnext);
        // a cycle predicted to find u_{k+1} converged waits for the norm
        // before its coarse part
        gate = predict_final(hist, tol, r0);
        rc = gate ? flush_pending_norm(h, st) : coarse();
        if (rc) return rc;
    }
    if (st_out) {
        rc = finish_bnorm(h, b, st);
        if (rc) return rc;
    }
    HIPCHK(hipEventRecord(h->ev1, st));
    HIPCHK(hipStreamSynchronize(st));
    rc = time_collect(h);
    if (rc) return rc;
    if (st_out) {
        st_out->cycles = k;
        st_out->cycles_run = run;
        st_out->r0_norm = r0;
        st_out->rk_norm = rk;
        st_out->b_norm = h->hnorm[2 * bnorm_slot(h)];
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
        st_out->elapsed_ms = ms;
        if (st_out->res_hist)
            for (int j = 0; j < (int)hist.size() && j < st_out->hist_cap; ++j)
                st_out->res_hist[j] = hist[j];
    }
    if (code == MG_ENONFINITE) return fail(code, "residual norm is not finite");
    if (code == MG_ENOCONV) return fail(code, "maximum number of cycles reached");
    return MG_OK;
}

static int solve64(mg_ctx* h, const double* b, double* u, double tol, mg_stats* st_out,
                   hipStream_t st) {
    if (chain_2d(h)) return solve64_chain(h, b, u, tol, st_out, st);
    double* X = u;
    double* Y = h->ualt;
    const size_t fine = (size_t)level_pts(h, 0) * h->batch * sizeof(double);
    HIPCHK(hipEventRecord(h->ev0, st));
    std::vector<double> hist;
    double r0 = 0.0, rk = 0.0;
    int k = 0, code = MG_OK, run = 0;
    bool flipped = false;
    h->bnorm_req = false;
    if (st_out) request_bnorm(h);
    for (k = 0;; ++k) {
        // cycle k reads u_k from X and writes u_{k+1} to Y; its pre-smoother
        // also yields ||r_k||.  The host waits only for that norm while the
        // rest of cycle k runs, then decides whether to enqueue cycle k + 1;
        // a cycle predicted to find u_k converged runs its pre-smoother alone
        // first and the rest only if the norm says so.
        const bool gate = h->L > 1 && predict_final(hist, tol, r0);
        // The answer u_K stays where cycle K found it; with ping-pong it
        // lands in the library's buffer for odd K and needs a final copy.
        // One cycle run in place (its post-smoother reads only tmp) flips
        // that parity; it is taken only far from convergence, where u_k
        // cannot be the answer, once the rate predicts K.
        bool inplace = false;
        if (!gate && !flipped && k >= 2 && k < h->max_cycles && hist[k - 2] > 0.0) {
            const double q = hist[k - 1] / hist[k - 2];
            if (tol * r0 > 0.0 && q > 0.0 && q < 0.9 &&
                hist[k - 1] * q >= kFlipMargin * tol * r0) {
                // finite: 0 < tol r0 < hist[k-1] and 0 < q < 0.9
                const int K = k - 1 + (int)std::ceil(std::log(tol * r0 / hist[k - 1]) /
                                                     std::log(q));
                const bool lands_in_u = ((K - k) % 2 == 0) == (X == u);
                inplace = !lands_in_u;
            }
        }
        arm_norm(h, k);
        int rc = fine_cycle64(h, b, X, inplace ? X : Y, k, st, gate ? kPreOnly : kWhole);
        if (rc) return rc;
        ++run;
        double nk;
        rc = wait_norm(h, k, st, &nk);
        if (rc) return rc;
        if (gate && std::isfinite(nk) && nk > tol * r0 && k < h->max_cycles) {
            rc = fine_cycle64(h, b, X, Y, -1, st, kRest);
            if (rc) return rc;
        }
        if (!std::isfinite(nk)) {
            code = MG_ENONFINITE;
            rk = nk;
            break;
        }
        if (k == 0) r0 = nk;
        hist.push_back(nk);
        rk = nk;
        if (inplace && nk <= tol * r0) {
            // the prediction failed: u_k was overwritten by u_{k+1}, which
            // is returned with its own residual (an in-place cycle is never
            // the last one the cycle limit allows)
            int np = 0;
            const double N = h->N;
            HIPCHK(launch_residual_norm(h->d, level_n(h, 0), h->batch, X, b, N * N, h->psum,
                                        h->pmax, kPartialCap * h->batch, st, &np));
            HIPCHK(launch_finalize(h->psum, nullptr, np, h->dnorm, st));
            HIPCHK(hipMemcpyAsync(h->hnorm, h->dnorm, sizeof(double), hipMemcpyDeviceToHost,
                                  st));
            HIPCHK(hipStreamSynchronize(st));
            rk = h->hnorm[0];
            ++k;
            hist.push_back(rk);
            if (rk <= tol * r0) break;
            code = MG_ENOCONV;
            break;
        }
        if (nk <= tol * r0) break;
        if (k >= h->max_cycles) {
            code = MG_ENOCONV;
            break;
        }
        if (inplace)
            flipped = true;
        else
            std::swap(X, Y);
    }
    // u_k is in X
    if (X != u) HIPCHK(hipMemcpyAsync(u, X, fine, hipMemcpyDeviceToDevice, st));
    if (st_out) {
        const int rb = finish_bnorm(h, b, st);
        if (rb) return rb;
    }
    HIPCHK(hipEventRecord(h->ev1, st));
    HIPCHK(hipStreamSynchronize(st));
    int rc = time_collect(h);
    if (rc) return rc;
    if (st_out) {
        st_out->cycles = k;
        st_out->cycles_run = run;
        st_out->r0_norm = r0;
        st_out->rk_norm = rk;
        st_out->b_norm = h->hnorm[2 * bnorm_slot(h)];
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
        st_out->elapsed_ms = ms;
        if (st_out->res_hist)
            for (int j = 0; j < (int)hist.size() && j < st_out->hist_cap; ++j)
                st_out->res_hist[j] = hist[j];
    }
    if (code == MG_ENONFINITE) return fail(code, "residual norm is not finite");
    if (code == MG_ENOCONV) return fail(code, "maximum number of cycles reached");
    return MG_OK;
}

static int solve_ir(mg_ctx* h, const double* b, double* u, double tol, mg_stats* st_out,
                    hipStream_t st) {
    Hier& H = h->hlo;
    double* X = u;
    double* Y = h->ualt;
    const size_t fine = (size_t)level_pts(h, 0) * h->batch * sizeof(double);
    const double N = h->N;
    const double sigma0 = H.scaled ? N * N : 1.0;
    HIPCHK(hipEventRecord(h->ev0, st));
    int nparts = 0, rc;
    // ||b|| from the solve's first pass over b (the residual pass or the
    // first refinement step)
    h->bnorm_req = false;
    if (st_out) request_bnorm(h);
    if (H.p == P16) {
        // FP16 storage needs r_0 scaled into range: a residual pass of the
        // initial guess puts (||r_0||, max|r_0|) in slot 0 for the first step
        double* bp = h->bnorm_req ? h->psum_b : nullptr;
        rc = run_timed(h, MG_TIME_RESIDUAL, 0, st, [&] {
            return launch_residual_norm(h->d, level_n(h, 0), h->batch, X, b, N * N, h->psum,
                                        h->pmax, kPartialCap * h->batch, st, &nparts, bp);
        });
        if (rc) return rc;
        if (bp) {
            h->bnorm_req = false;
            h->bnorm_parts = nparts;
        }
        HIPCHK(launch_finalize(h->psum, h->pmax, nparts, h->dnorm, st));
    } else {
        // FP32 holds r_0 unscaled: max|r| = 0 in slot 0 gives the first step
        // the scale 1
        HIPCHK(hipMemsetAsync(h->dnorm, 0, 2 * sizeof(double), st));
    }
    std::vector<double> hist;
    double r0 = 0.0, rk = 0.0;
    int k = 0, code = MG_OK, run = 0;
    double pred = -1.0;   // predicted ||r_k|| (< 0: no prediction)
    int m_prev = 0;       // inner cycles of the previous step
    for (k = 0;; ++k) {
        const int slot = 1 + k;   // k <= max_cycles < norm_slots - 2
        const int pslot = k;
        IRStep s;
        s.d = h->d;
        s.n = level_n(h, 0);
        s.batch = h->batch;
        s.k = k;
        s.u = X;
        s.unew = Y;
        s.e_lo = k > 0 ? H.e[0] : nullptr;
        s.b = b;
        s.r_lo = H.b[0];
        s.inv_h2 = N * N;
        s.sigma0 = sigma0;
        s.scales = h->dscale;
        s.maxprev = h->dnorm + 2 * pslot + 1;
        s.psum = h->psum;
        s.pmax = h->pmax;
        s.bparts = h->bnorm_req ? h->psum_b : nullptr;
        s.partials_cap = kPartialCap * h->batch;
        arm_norm(h, slot);
        rc = run_timed(h, MG_TIME_IR_STEP, 0, st,
                       [&] { return launch_ir_step(H.p, s, st, &nparts); });
        if (rc) return rc;
        if (s.bparts) {
            h->bnorm_req = false;
            h->bnorm_parts = nparts;
        }
        // (norm, max) of r_k: reduced by the first restriction of the inner
        // cycle, which also writes the host mirror
        h->pend.count = nparts;
        h->pend.with_max = true;
        h->pend.slot = slot;
        // inner low-precision cycles on A e = s r: the first from zero, the
        // others continue from the current e.  The host reads ||r_k|| while
        // the first inner cycle runs and enqueues the others only if the
        // solve goes on, so a converged solve discards one inner cycle --
        // unless the last reduction predicts convergence: then the norm is
        // reduced and read before any inner cycle is enqueued.
        const bool gate = pred >= 0.0 && pred <= kGateSlack * tol * r0;
        if (!gate) {
            rc = cycle(h, H, 0, nullptr, H.b[0], H.e[0], H.t[0], NormReq(), st);
            if (rc) return rc;
        }
        rc = flush_pending_norm(h, st);
        if (rc) return rc;
        ++run;
        double nk;
        rc = wait_norm(h, slot, st, &nk);
        if (rc) return rc;
        if (!std::isfinite(nk)) {
            code = MG_ENONFINITE;
            rk = nk;
            break;
        }
        if (k == 0) r0 = nk;
        hist.push_back(nk);
        rk = nk;
        if (nk <= tol * r0) break;
        if (k >= h->max_cycles) {
            code = MG_ENOCONV;
            break;
        }
        // inner cycles of this step (fixed: the option's count or the
        // default), and the per-cycle reduction observed in the last step,
        // which predicts ||r_{k+1}|| for the gate
        const int m = inner_cycles(h);
        double rho = 1.0;
        if (k > 0) rho = std::pow(nk / hist[k - 1], 1.0 / m_prev);
        pred = k > 0 && rho < 1.0 ? nk * std::pow(rho, m) : -1.0;
        m_prev = m;
        if (gate) {
            rc = cycle(h, H, 0, nullptr, H.b[0], H.e[0], H.t[0], NormReq(), st);
            if (rc) return rc;
        }
        for (int j = 1; j < m; ++j) {
            rc = cycle(h, H, 0, H.e[0], H.b[0], H.e[0], H.t[0], NormReq(), st);
            if (rc) return rc;
        }
        // step 0 applies no correction and leaves u_0 in X
        if (k > 0) std::swap(X, Y);
    }
    // u_k is the refinement step's output: in Y, or u_0 in X after step 0
    double* uk = k > 0 ? Y : X;
    if (uk != u) HIPCHK(hipMemcpyAsync(u, uk, fine, hipMemcpyDeviceToDevice, st));
    if (st_out) {
        rc = finish_bnorm(h, b, st);
        if (rc) return rc;
    }
    HIPCHK(hipEventRecord(h->ev1, st));
    HIPCHK(hipStreamSynchronize(st));
    rc = time_collect(h);
    if (rc) return rc;
    if (st_out) {
        st_out->cycles = k;
        st_out->cycles_run = run;
        st_out->r0_norm = r0;
        st_out->rk_norm = rk;
        st_out->b_norm = h->hnorm[2 * bnorm_slot(h)];
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
        st_out->elapsed_ms = ms;
        if (st_out->res_hist)
            for (int j = 0; j < (int)hist.size() && j < st_out->hist_cap; ++j)
                st_out->res_hist[j] = hist[j];
    }
    if (code == MG_ENONFINITE) return fail(code, "residual norm is not finite");
    if (code == MG_ENOCONV) return fail(code, "maximum number of cycles reached");
    return MG_OK;
}

int mg_solve(mg_handle_t h, const double* b, double* u, double tol, mg_stats* st,
             void* stream) {
    if (check_handle(h)) return MG_EINVAL;
    if (!b || !u) return fail(MG_EINVAL, "null field pointer");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(MG_EINVAL, "tol must be finite and >= 0");
    hipStream_t s = (hipStream_t)stream;
    h->pend = mg_ctx::PendingNorm();  // nothing survives a failed call
    h->call_fused = 0;
    if (h->prec == MG_PREC_FP64) return solve64(h, b, u, tol, st, s);
    return solve_ir(h, b, u, tol, st, s);
}

int mg_get_timing(mg_handle_t h, int kind, int level, double* total_ms, int* count) {
    if (check_handle(h)) return MG_EINVAL;
    if (kind < 0 || kind >= kTimeKinds || level < 0 || level >= kMaxLevels)
        return fail(MG_EINVAL, "bad timing kind or level");
    if (total_ms) *total_ms = h->t_ms[kind][level];
    if (count) *count = h->t_cnt[kind][level];
    return MG_OK;
}

int mg_reset_timing(mg_handle_t h) {
    if (check_handle(h)) return MG_EINVAL;
    std::memset(h->t_ms, 0, sizeof(h->t_ms));
    std::memset(h->t_cnt, 0, sizeof(h->t_cnt));
    return MG_OK;
}

void mg_destroy(mg_handle_t h) {
    if (!h) return;
    free_hier(h->h64);
    free_hier(h->hlo);
    free_adj(h);
    if (h->ualt) (void)hipFree(h->ualt);
    if (h->psum) (void)hipFree(h->psum);
    if (h->pmax) (void)hipFree(h->pmax);
    if (h->psum_b) (void)hipFree(h->psum_b);
    if (h->dnorm) (void)hipFree(h->dnorm);
    if (h->dscale) (void)hipFree(h->dscale);
    if (h->hnorm) (void)hipHostFree(h->hnorm);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    delete h;
}

}  // extern "C"

namespace {
void free_adj(mg_ctx* h) {
    for (auto* v : {&h->adj_r1, &h->adj_r3, &h->adj_w, &h->adj_ua, &h->adj_ub, &h->adj_uo,
                    &h->adj_bb}) {
        for (double* p : *v)
            if (p) (void)hipFree(p);
        v->clear();
    }
    if (h->adj_cacc) (void)hipFree(h->adj_cacc);
    if (h->adj_cin) (void)hipFree(h->adj_cin);
    if (h->adj_part) (void)hipFree(h->adj_part);
    h->adj_cacc = nullptr;
    h->adj_cin = nullptr;
    h->adj_part = nullptr;
    h->adj_pcap = 0;
    h->adj_alloc = false;
}

int alloc_adj(mg_ctx* h) {
    if (h->adj_alloc) return MG_OK;
    free_adj(h);
    for (auto* v : {&h->adj_r1, &h->adj_r3, &h->adj_w, &h->adj_ua, &h->adj_ub, &h->adj_uo,
                    &h->adj_bb})
        v->assign(h->L, nullptr);
    for (int l = 0; l < h->L; ++l) {
        const size_t bytes = (size_t)level_pts(h, l) * h->batch * sizeof(double);
        if (l == 0) HIPCHK(hipMalloc(&h->adj_r1[l], bytes));
        if (l > 0) {
            HIPCHK(hipMalloc(&h->adj_uo[l], bytes));
            HIPCHK(hipMalloc(&h->adj_bb[l], bytes));
        }
        if (l < h->L - 1) {
            HIPCHK(hipMalloc(&h->adj_r3[l], bytes));
            HIPCHK(hipMalloc(&h->adj_ua[l], bytes));
            HIPCHK(hipMalloc(&h->adj_ub[l], bytes));
        }
        // the fine level's post-smoothed iterate of the recomputation (unused)
        if (l == 0 && h->L > 1) HIPCHK(hipMalloc(&h->adj_w[l], bytes));
    }
    HIPCHK(hipMalloc(&h->adj_cacc, 4 * sizeof(double)));
    // two coefficient-gradient sweeps per level above the coarsest, each at
    // most kAdjBlocks blocks per batch entry with 4 partial sums
    h->adj_pcap = 2L * 4 * kAdjBlocks * h->batch * (h->L > 1 ? h->L - 1 : 1);
    HIPCHK(hipMalloc(&h->adj_part, (size_t)h->adj_pcap * sizeof(double)));
    h->adj_alloc = true;
    return MG_OK;
}

// Forward recomputation of one V(1,1) cycle at level l from u_in (null: zero
// guess), keeping what the reverse sweep needs: r1 = b - A u_in (fine
// level; on coarse levels r1 = b), r3 = b - A u2 with u2 = u1 + P e_{l+1},
// and the level output e_l (for the level above).  The residuals are side
// outputs of the cycle's own fused kernels: the pre-smoother (with the
// restriction where the cycle fuses them) writes r1, and the post-smoother
// with the fused correction writes r3 beside e_l.  u_f32: u_in holds FP32
// values (an FP32 checkpoint, read by the fused pre-smoother directly).
int adj_forward(mg_ctx* h, int l, const void* u_in, bool u_f32, const double* bl,
                hipStream_t st) {
    Hier& H = h->h64;
    if (l == h->L - 1) return run_tail(h, H, l, bl, H.e[l], st);
    Sweep s = make_sweep(h, H, l);
    double* t = static_cast<double*>(H.t[l]);
    s.u = u_in;
    s.b = bl;
    s.out = t;
    const bool fused = u_in ? fuse_smooth_restrict(h, l) : fuse_zero_restrict(h, l);
    if (u_f32 && !(fused && u_in)) return fail(MG_EINVAL, "FP32 input without the fused kernel");
    if (fused) {
        s.out_c = H.b[l + 1];
        s.rout = u_in ? h->adj_r1[l] : nullptr;
        s.u_f32 = u_f32;
        HIPCHK(u_in ? launch_smooth_restrict(P64, false, s, st, nullptr)
                    : launch_zero_smooth_restrict(P64, s, st));
    } else {
        s.rout = u_in ? h->adj_r1[l] : nullptr;
        HIPCHK(launch_smooth(P64, u_in == nullptr, false, s, st, nullptr));
        Sweep rs = make_sweep(h, H, l);
        rs.u = t;
        rs.b = bl;
        rs.out = H.b[l + 1];
        HIPCHK(launch_restrict(P64, rs, st));
    }
    int rc = adj_forward(h, l + 1, nullptr, false, static_cast<const double*>(H.b[l + 1]), st);
    if (rc) return rc;
    // post-smoothing of u2 = t + P e_{l+1}; on the fine level only r3 is
    // needed (the cycle's output goes to scratch)
    Sweep q = make_sweep(h, H, l);
    q.u = t;
    q.b = bl;
    q.ec = H.e[l + 1];
    q.pf = 1.0;
    q.rout = h->adj_r3[l];
    q.out = l > 0 ? H.e[l] : h->adj_w[0];
    HIPCHK(launch_smooth(P64, false, false, q, st, nullptr));
    return MG_OK;
}

// Reverse sweep of the cycle at level l: given uo = dL/du_out, accumulates
// bb += dL/db_l and the coefficient gradient, and writes ui = dL/du_in.
int adj_reverse(mg_ctx* h, int l, const double* uo, double* ui, double* bb, const double* r1,
                hipStream_t st) {
    Hier& H = h->h64;
    const int d = h->d, n = level_n(h, l), b = h->batch;
    const double N = level_N(h, l), h2 = 1.0 / (N * N);
    if (l == h->L - 1) {
        // e = A^{-1} b: bbar += A^{-1} ubar_out; the output ignores u_in
        HIPCHK(launch_coarse_matvec(d == 2 ? 9 : 27, b, H.ginv, uo, bb, true, st));
        if (ui) HIPCHK(hipMemsetAsync(ui, 0, (size_t)level_pts(h, l) * b * sizeof(double), st));
        return MG_OK;
    }
    double c[4] = {h->c[0], h->c[1], h->ncoef > 2 ? h->c[2] : 0.0,
                   h->ncoef > 3 ? h->c[3] : 0.0};
    double* ua = h->adj_ua[l];
    double* ub = h->adj_ub[l];
    int np = 0;
    // post-smoothing  u_out = u2 + M r3, r3 = b - A u2: ubar2 = ubar_out -
    // A M ubar_out, bbar += M ubar_out; its coefficient-gradient partials
    // (scaled by h^2) go to their own slots, reduced once per adjoint call in
    // slot order
    HIPCHK(launch_adj_sweep(d, n, b, 0, uo, h->adj_r3[l], nullptr, 0.0, ua, bb,
                            h->adj_part + h->adj_poff, h->adj_pcap - h->adj_poff, N * N, h2, c,
                            st, &np));
    h->adj_poff += 4L * np;
    // correction u2 = u1 + P e_c: ecbar = P^T ubar2 = 2^d R ubar2
    HIPCHK(launch_fw(d, n, b, ua, h->adj_uo[l + 1], d == 2 ? 4.0 : 8.0, st));
    const size_t cbytes = (size_t)level_pts(h, l + 1) * b * sizeof(double);
    HIPCHK(hipMemsetAsync(h->adj_bb[l + 1], 0, cbytes, st));
    int rc = adj_reverse(h, l + 1, h->adj_uo[l + 1], nullptr, h->adj_bb[l + 1],
                         static_cast<const double*>(H.b[l + 1]), st);
    if (rc) return rc;
    // restriction b_c = R (b - A u1): rbar = R^T bcbar = 2^-d P bcbar,
    // interpolated inside the sweep; ubar1 = ubar2 - A rbar, bbar += rbar
    HIPCHK(launch_adj_sweep(d, n, b, 1, ua, nullptr, h->adj_bb[l + 1], d == 2 ? 0.25 : 0.125, ub,
                            bb, nullptr, 0, N * N, h2, c, st, nullptr));
    // pre-smoothing  u1 = u + M r1, r1 = b - A u: ubar = ubar1 - A M ubar1
    // (discarded below the fine level: the coarse cycles start from zero)
    HIPCHK(launch_adj_sweep(d, n, b, 0, ub, r1, nullptr, 0.0, ui ? ui : ua, bb,
                            h->adj_part + h->adj_poff, h->adj_pcap - h->adj_poff, N * N, h2, c,
                            st, &np));
    h->adj_poff += 4L * np;
    return MG_OK;
}
}  // namespace

extern "C" int mg_checkpoint(mg_handle_t h, double* u, void* ckpt, int ckpt_dtype,
                             void* stream) {
    if (check_handle(h)) return MG_EINVAL;
    if (!u || !ckpt) return fail(MG_EINVAL, "null pointer");
    if (ckpt_dtype != MG_CKPT_FP64 && ckpt_dtype != MG_CKPT_FP32)
        return fail(MG_EINVAL, "ckpt_dtype must be MG_CKPT_FP64 or MG_CKPT_FP32");
    hipStream_t st = (hipStream_t)stream;
    const long count = level_pts(h, 0) * h->batch;
    if (ckpt_dtype == MG_CKPT_FP64)
        HIPCHK(hipMemcpyAsync(ckpt, u, count * sizeof(double), hipMemcpyDeviceToDevice, st));
    else
        HIPCHK(launch_ckpt32(u, static_cast<float*>(ckpt), count, st));
    return MG_OK;
}

extern "C" int mg_vcycle_adjoint(mg_handle_t h, const double* b, const void* u_ckpt,
                                 int ckpt_dtype, const double* ubar_out, double* ubar_in,
                                 double* bbar_acc, double* cbar_acc, void* stream) {
    if (check_handle(h)) return MG_EINVAL;
    if (!b || !u_ckpt || !ubar_out || !ubar_in || !bbar_acc || !cbar_acc)
        return fail(MG_EINVAL, "null pointer");
    if (ckpt_dtype != MG_CKPT_FP64 && ckpt_dtype != MG_CKPT_FP32)
        return fail(MG_EINVAL, "ckpt_dtype must be MG_CKPT_FP64 or MG_CKPT_FP32");
    if (h->cycle_kind != MG_CYCLE_V11)
        return fail(MG_EINVAL, "the adjoint is defined for the V(1,1) cycle only");
    hipStream_t st = (hipStream_t)stream;
    int rc = alloc_adj(h);
    if (rc) return rc;
    const void* u_in = u_ckpt;
    bool u_f32 = false;
    if (ckpt_dtype == MG_CKPT_FP32) {
        if (h->L > 1 && fuse_smooth_restrict(h, 0)) {
            // the fused pre-smoother reads the FP32 checkpoint itself
            u_f32 = true;
        } else {
            // the unfused pre-smoother reads FP64: widen into a buffer of
            // its own (allocated on first use)
            if (!h->adj_cin)
                HIPCHK(hipMalloc(&h->adj_cin,
                                 (size_t)level_pts(h, 0) * h->batch * sizeof(double)));
            HIPCHK(launch_widen(static_cast<const float*>(u_ckpt), h->adj_cin,
                                level_pts(h, 0) * h->batch, st));
            u_in = h->adj_cin;
        }
    }
    h->adj_poff = 0;
    if (h->L == 1) {
        // single grid: u_out = A^{-1} b
        HIPCHK(launch_coarse_matvec(h->d == 2 ? 9 : 27, h->batch, h->h64.ginv, ubar_out, bbar_acc,
                                    true, st));
        HIPCHK(hipMemsetAsync(ubar_in, 0, (size_t)level_pts(h, 0) * h->batch * sizeof(double), st));
    } else {
        rc = adj_forward(h, 0, u_in, u_f32, b, st);
        if (rc) return rc;
        rc = adj_reverse(h, 0, ubar_out, ubar_in, bbar_acc, h->adj_r1[0], st);
        if (rc) return rc;
    }
    // dL/dc_j = sum over every smoothing step of its scaled partials
    HIPCHK(launch_reduce_cols(h->adj_part, (int)(h->adj_poff / 4), 4, h->adj_cacc, 1.0, st));
    double hc[4];
    HIPCHK(hipMemcpyAsync(hc, h->adj_cacc, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int j = 0; j < h->ncoef; ++j) cbar_acc[j] += hc[j];
    return MG_OK;
}
