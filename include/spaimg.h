/*
 * spaimg.h -- C ABI of libspaimg.so: geometric multigrid for the Dirichlet
 * Laplacian with the optimised sparse-approximate-inverse (SPAI) smoothers of
 * He, Liu and Wang, "Optimized sparse approximate inverse smoothers for
 * solving Laplacian linear systems" (arXiv 2206.05543), on AMD gfx950 GPUs.
 *
 * Problem (Section 1, eqs. (Poisson), (Ax=b), (A_h)): A_h u = b on the unit
 * square (d = 2, 5-point stencil) or cube (d = 3, 7-point stencil), h = 1/N,
 * unknowns at the (N-1)^d interior nodes.  Dirichlet data g is folded into b
 * by the caller (b_i += g/h^2 at nodes next to the boundary).
 *
 * Smoother (Section 2, eq. (smoother)): u <- u + M (b - A_h u) with
 * M = h^2 (c0 K0 + c1 K1 + c2 K2 [+ c3 K3]), K0 = identity, K1 = sum over the
 * 2d face neighbours, K2 = sum over the 4 diagonal neighbours (2D) or the 12
 * edge neighbours (3D), K3 = sum over the 8 corner neighbours (3D), applied
 * to a residual that is zero outside the grid.  In 3D, c2 and c3 give the
 * wider 19- and 27-point stencils the closing remark of Section 3.2 mentions
 * (c2 = c3 = 0: the 7-point family T).  The coefficients are h-free and
 * include the damping factor omega; the same coefficients are used on every
 * level (rediscretisation, Section 4).  The paper's smoothers:
 *   2D M9 (Theorem 3.1): omega = (309 - 12 sqrt(10))/1720, (c0, c1, c2) =
 *      omega (44, 10, 3)/24 = (0.28891272760249742, 0.065661983546022137,
 *      0.019698595063806643)
 *   3D M7 (Theorem 3.2): omega = 20/73, (c0, c1) = (16/73, 2/73)
 *   damped Jacobi: 2D (0.2, 0, 0), 3D (1/7, 0); best 5-point M5: (12/41,
 *   2/41, 0); additive Vanka: (0.28, 0.04, 0.01) (Section 3.1).
 *
 * Cycle (Section 4): V(1,1) -- one pre- and one post-smoothing step, full
 * weighting restriction of the residual, rediscretised coarse operators with
 * H = 2h, linear (bi-/tri-linear) interpolation, and an exact solve on the
 * grid with h0 = 1/4 (3^d unknowns).  Coarse levels start from zero.
 *
 * Memory layout and ownership: every field argument is a DEVICE pointer owned
 * by the caller, C-contiguous, shape [batch, (N-1)^d] with x fastest (FP64
 * unless stated otherwise).  The library never frees nor retains them past a
 * call.  It owns every internal buffer (allocated in mg_setup and when an
 * option changes the batch or precision; freed in mg_destroy).
 *
 * Streams: every call enqueues its work on `stream` (a hipStream_t; NULL is
 * the null stream) and returns without waiting, except mg_solve,
 * mg_residual_norm and the timing queries, which synchronise that stream.  A
 * handle must not be used from two host threads at once, nor by calls whose
 * work overlaps on two streams.
 *
 * Errors: functions return MG_OK (0) or a negative code; mg_last_error()
 * returns a thread-local message describing the last failure.  Arguments are
 * checked on the host before any work is enqueued.
 */
#ifndef SPAIMG_H
#define SPAIMG_H

#ifdef __cplusplus
extern "C" {
#endif

#define MG_OK 0
#define MG_EINVAL (-1)      /* bad argument or option                        */
#define MG_EHIP (-2)        /* HIP runtime failure (message in mg_last_error) */
#define MG_ENOCONV (-3)     /* max cycles reached before the tolerance       */
#define MG_ENONFINITE (-4)  /* a residual norm is NaN or infinite            */

/* mg_set_option keys */
#define MG_OPT_PRECISION 1  /* MG_PREC_*; used by mg_solve                     */
#define MG_OPT_BATCH 2      /* number of stacked problems, >= 1 (default 1)    */
#define MG_OPT_MAX_CYCLES 3 /* cycle limit of mg_solve, 1..10000 (default 100) */
#define MG_OPT_TAIL_N 4     /* largest coarse grid (intervals, power of two,
                               4..64 in 2D, 4..16 in 3D) solved by the
                               single-workgroup LDS tail kernel; 0 = default:
                               64 in 2D, 16 in 3D                             */
#define MG_OPT_TIMING 5     /* 0 off; 1 time the fine level's fused
                               pre-smoother + restriction with HIP events;
                               2 time every kernel of every level; 3 as 1,
                               but only the second such launch of each
                               mg_solve / mg_vcycle call (an event after a
                               large kernel idles the GPU ~5 us)              */
#define MG_OPT_INNER_CYCLES 6 /* low-precision V-cycles per FP64 refinement
                               step, 1..16; 0 = default (6 for FP32, 2 for
                               FP16)                                          */
#define MG_OPT_CYCLE 7      /* MG_CYCLE_*: the cycle of mg_vcycle, mg_solve
                               and the inner cycles of refinement (default V) */

/* cycles for MG_OPT_CYCLE (Section 4 tests both) */
#define MG_CYCLE_V11 0      /* V(1,1): one pre- and one post-smoothing step   */
#define MG_CYCLE_W10 1      /* W(1,0): one pre-smoothing step, two coarse-grid
                               visits per level, no post-smoothing; both
                               visits of a level at or below the tail size
                               run in one tail launch.  Not available for
                               mg_vcycle_adjoint.                             */

/* precisions for MG_OPT_PRECISION */
#define MG_PREC_FP64 0      /* FP64 V-cycles                                  */
#define MG_PREC_FP32_IR 1   /* FP64 iterative refinement around FP32 V-cycles;
                               the first step stores b - A u_0 unscaled in
                               FP32, so its entries must stay below ~3e38
                               (beyond that mg_solve returns MG_ENONFINITE)  */
#define MG_PREC_FP16_IR 2   /* ... around V-cycles with FP16 storage, FP32
                               arithmetic and per-level power-of-two scaling  */

/* checkpoint storage of mg_checkpoint and mg_vcycle_adjoint */
#define MG_CKPT_FP64 0      /* FP64 copy of the iterate                      */
#define MG_CKPT_FP32 1      /* FP32 rounding (to nearest even) of the iterate */

/* operation codes of mg_sweep */
#define MG_OP_SMOOTH 0       /* out = u + M (b - A u)                          */
#define MG_OP_SMOOTH_ZERO 1  /* out = M b (smoothing from a zero guess)        */
#define MG_OP_RESTRICT 2     /* out (level+1) = R (b - A u)                    */
#define MG_OP_PROLONG_ADD 3  /* out += P u, u on level+1 (in place on out)     */

/* timing kinds for mg_get_timing */
#define MG_TIME_SMOOTH 0      /* smoothing from a guess (pre-smoothing)    */
#define MG_TIME_SMOOTH_ZERO 1
#define MG_TIME_RESTRICT 2
#define MG_TIME_PROLONG 3
#define MG_TIME_TAIL 4
#define MG_TIME_IR_STEP 5
#define MG_TIME_RESIDUAL 6
#define MG_TIME_SMOOTH_CORRECT 7  /* post-smoothing with the fused correction */
#define MG_TIME_ZERO_SMOOTH_RESTRICT 8  /* zero-guess pre-smoothing fused with
                                           the restriction                    */
#define MG_TIME_SMOOTH_RESTRICT 9  /* pre-smoothing from a nonzero iterate
                                      fused with the restriction              */
#define MG_TIME_POST_PRE_RESTRICT 10  /* post-smoothing of one cycle fused
                                         with the next one's pre-smoothing
                                         and restriction (2D solves)      */

typedef struct mg_ctx* mg_handle_t;

typedef struct mg_stats {
    int cycles;        /* cycles k at which ||r_k|| <= tol ||r_0|| (or the
                          limit); u holds u_k                                 */
    int cycles_run;    /* cycles (refinement steps) started: one more than
                          cycles, since u_k is tested by the next cycle's
                          pre-smoother (refinement step); when the previous
                          reduction predicts convergence only that part runs
                          before the host reads the norm                     */
    double r0_norm;    /* ||b - A u_0||_2 (whole batch)                       */
    double rk_norm;    /* ||b - A u_k||_2                                      */
    double b_norm;     /* ||b||_2 (whole batch; one extra pass over b), so
                          that ||r_k|| / ||b|| can be reported beside the
                          stopping rule's ||r_k|| / ||r_0||                   */
    double* res_hist;  /* optional host array: ||r_j||_2, j = 0..cycles       */
    int hist_cap;      /* its capacity (entries)                               */
    double elapsed_ms; /* device time of the whole solve (HIP events)         */
} mg_stats;

/* Creates a solver for N intervals per direction (power of two, 4 <= N <=
 * 65536 in 2D, <= 2048 in 3D) in d = 2 or 3 dimensions with n_coeffs = 3
 * (2D: centre, faces, diagonals) or 2, 3 or 4 (3D: centre, faces[, edges[,
 * corners]]) host FP64 coefficients (see above).  A 3D stencil with a
 * nonzero edge or corner coefficient runs the wide smoother kernel and a
 * separate restriction on every level.  Allocates the level
 * hierarchy (about (1/3 + 1/(2^d - 1)) of one fine field per batch entry plus
 * two fine FP64 fields).  *out receives the handle. */
int mg_setup(int N, int d, const double* spai_coeffs, int n_coeffs, mg_handle_t* out);

/* Sets an option (keys above).  Changing the batch or precision reallocates
 * internal buffers. */
int mg_set_option(mg_handle_t h, int key, double value);

/* Replaces the smoother coefficients (host FP64, n_coeffs equal to
 * mg_setup's). */
int mg_set_coeffs(mg_handle_t h, const double* spai_coeffs, int n_coeffs);

/* One FP64 V(1,1) cycle for every batch entry: u <- V(u, b), in place.
 * (Section 4.) */
int mg_vcycle(mg_handle_t h, const double* b, double* u, void* stream);

/* Bytes of the static per-device workspace of mg_vcycle_noalloc (32 MiB). */
#define MG_NOALLOC_SCRATCH_BYTES (32u << 20)

/* For callers that cannot allocate device memory (work recorded under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * FP64 V(1,1) cycle of mg_vcycle -- same kernels, same launch shapes, same
 * result -- for a problem given by the arguments of mg_setup plus `batch`
 * (1..65535), with default options and without a handle.  u <- V(u, b) in
 * place; b and u are caller-owned device arrays shaped as for mg_vcycle.
 *
 * Allocates nothing: no hipMalloc, hipFree, host heap or library allocator.
 * Every internal buffer lives in one static array of the library
 * (MG_NOALLOC_SCRATCH_BYTES per device, allocated when the code object is
 * loaded and held until the process ends), so the problem's workspace,
 * (N-1)^d + 3 sum_{l>=1} (N/2^l - 1)^d doubles per batch entry (each level
 * buffer rounded up to 256 bytes), must fit in it: e.g. 2D N <= 1024 or 3D
 * N <= 128 at batch 1.  The first call on a device looks up that device's
 * copy of the array (hipGetSymbolAddress); every call then only enqueues
 * kernels on `stream` (a stream of the current device) and returns without
 * waiting.  The cycle writes each workspace element before reading it, so
 * the previous call's contents never matter.  Every call on one device
 * shares that device's array: calls whose work may overlap (two streams,
 * two host threads) race and must be serialised by the caller.
 *
 * Errors: MG_EINVAL for bad N, d, coefficients, batch or null pointers, or
 * a workspace larger than the static array (the message gives both sizes);
 * MG_EHIP for a failed address lookup or kernel launch. */
int mg_vcycle_noalloc(int N, int d, const double* spai_coeffs, int n_coeffs, int batch,
                      const double* b, double* u, void* stream);

/* Cycles from the initial guess in u until ||b - A u_k||_2 <= tol ||b - A
 * u_0||_2 over the whole batch (the stopping rule on the relative residual,
 * Section 4), with the precision set by MG_OPT_PRECISION.  FP64: V(1,1)
 * cycles; st->cycles counts them.  FP32_IR / FP16_IR: each refinement step
 * computes r = b - A u in FP64, scales it by a power of two s (so that
 * max |s r| < 1), runs MG_OPT_INNER_CYCLES low-precision V(1,1) cycles on
 * A e = s r (the first from zero) and updates u += e / s in FP64;
 * st->cycles counts refinement steps.  Synchronises `stream`; the calling
 * thread busy-waits on one pinned host slot per cycle for the norm, which
 * the GPU writes as soon as it is reduced (no event per cycle).  Returns
 * MG_ENOCONV (u = last iterate, st filled) if MG_OPT_MAX_CYCLES is reached,
 * MG_ENONFINITE if a norm is not finite.  st may be NULL. */
int mg_solve(mg_handle_t h, const double* b, double* u, double tol, mg_stats* st,
             void* stream);

/* Per-cycle checkpoint of the cycle-start iterate u (device, batch-shaped
 * FP64) for the adjoint's recomputation: ckpt (device, batch-shaped) receives
 * u in FP64 (MG_CKPT_FP64) or rounded to FP32 (MG_CKPT_FP32).  With FP32 u is
 * replaced in place by the rounded value, so the forward pass continues from
 * exactly what the checkpoint holds and mg_vcycle_adjoint recomputes that
 * cycle's states bit for bit.  The rounding is a non-differentiable step of
 * the forward map; the adjoint passes derivatives through it unchanged
 * (straight-through), which differs from the derivative of the unrounded
 * FP64 map by O(2^-24) relative.  Does not synchronise.  Errors: MG_EINVAL for
 * a null handle or pointer or a bad ckpt_dtype. */
int mg_checkpoint(mg_handle_t h, double* u, void* ckpt, int ckpt_dtype, void* stream);

/* Reverse-mode derivative of one FP64 V(1,1) cycle u_out = V(u_in, b; c)
 * (Section 4 cycle, Section 2 smoother, differentiated by hand): given
 * ubar_out = dL/du_out, writes ubar_in = dL/du_in (may alias ubar_out),
 * accumulates bbar_acc += dL/db (device, batch-shaped) and cbar_acc[j] +=
 * dL/dc_j summed over the batch (HOST FP64 array of mg_setup's n_coeffs).  u_in is the
 * cycle's checkpoint as written by mg_checkpoint: device, batch-shaped, FP64
 * (ckpt_dtype = MG_CKPT_FP64) or FP32 (MG_CKPT_FP32, converted exactly to
 * FP64 as the recomputation reads it).  The forward states of every level are recomputed
 * from it.  Uses A^T = A, M^T = M (symmetric stencils with zero extension),
 * P^T = 2^d R.  Synchronises `stream` (to return cbar_acc on the host).
 * Errors: MG_EINVAL for a null handle or pointer, a bad ckpt_dtype or a
 * W(1,0) cycle setting. */
int mg_vcycle_adjoint(mg_handle_t h, const double* b, const void* u_ckpt, int ckpt_dtype,
                      const double* ubar_out, double* ubar_in, double* bbar_acc,
                      double* cbar_acc, void* stream);

/* One building-block kernel on one level (level 0 = the finest grid, level l
 * has N/2^l intervals), for the whole batch.  prec = MG_PREC_FP64 uses FP64
 * fields in true units.  prec = MG_PREC_FP32_IR (FP32 fields) or
 * MG_PREC_FP16_IR (FP16 fields) uses the scaled storage of the low-precision
 * hierarchies: a correction e on level l is stored as e / h_l^2, the
 * right-hand side unscaled (so A and M need no h factors, and P carries a
 * factor 4 between levels).  op = MG_OP_SMOOTH: out = u + M(b - A u);
 * MG_OP_SMOOTH_ZERO: out = M b (u ignored); MG_OP_RESTRICT: out (shape of
 * level+1) = R (b - A u); MG_OP_PROLONG_ADD: out (level) += P u where u has
 * the shape of level+1 (b ignored).  out must not alias u or b, except for
 * MG_OP_PROLONG_ADD where out is updated in place. */
int mg_sweep(mg_handle_t h, int op, int level, int prec, const void* u, const void* b,
             void* out, void* stream);

/* Zero-guess pre-smoothing fused with the restriction on level `level` in
 * storage precision `prec` (as mg_sweep): e = M b on the level and bc = R (b
 * - A e) on level+1, in one kernel (the kernel mg_solve and mg_vcycle use
 * for zero-guess cycles; Section 4, V-cycle with a zero initial guess on the
 * coarse levels).  b, e: the level's shape; bc: level+1's shape.  Errors:
 * MG_EINVAL for a null handle or pointer, a bad precision, no coarser level,
 * or a 3D 19-/27-point stencil (this kernel carries the 7-point one). */
int mg_sweep_zero_restrict(mg_handle_t h, int level, int prec, const void* b, void* e, void* bc,
                           void* stream);

/* Pre-smoothing from an iterate u fused with the restriction on level
 * `level`, in storage precision `prec` (as mg_sweep): out = u + M (b - A u)
 * on the level and bc = R (b - A out) on level+1, in one kernel (the kernel
 * mg_solve and mg_vcycle use for the finest level's pre-smoothing; Section
 * 4, V(1,1) cycle).  u, b, out: the level's shape, out must not alias u or
 * b; bc: level+1's shape.  Errors: MG_EINVAL for a null handle or pointer, a
 * bad precision, no coarser level, or a 3D 19-/27-point stencil. */
int mg_sweep_smooth_restrict(mg_handle_t h, int level, int prec, const void* u, const void* b,
                             void* out, void* bc, void* stream);

/* The sweeps between two V(1,1) cycles as one kernel, on level `level` of
 * a 2D hierarchy in storage precision `prec` (as mg_sweep): with w = u + P ec
 * (u: the pre-smoothed iterate of cycle k, ec: its coarse-grid correction on
 * level+1), out = w + M (b - A w) is u_{k+1} (post-smoothing), out_t = out +
 * M (b - A out) the pre-smoothed iterate of cycle k+1 and bc = R (b - A
 * out_t) its coarse right-hand side on level+1 (Section 4, V(1,1) cycle;
 * mg_solve uses it between the cycles of 2D FP64 solves).  u, b, out, out_t:
 * the level's shape, out and out_t must not alias each other, u or b; ec,
 * bc: level+1's shape.  Errors: MG_EINVAL for a null handle or pointer, a
 * bad precision, no coarser level or a 3D hierarchy. */
int mg_sweep_post_pre_restrict(mg_handle_t h, int level, int prec, const void* u,
                               const void* ec, const void* b, void* out, void* out_t, void* bc,
                               void* stream);

/* Fused post-smoothing sweep with the coarse-grid correction: with
 * v = u + P ec (ec on level + 1; in the scaled low-precision storage the
 * correction carries the factor 4 between levels), out = v + M (b - A v).
 * out must not alias u, ec or b. */
int mg_sweep_correct(mg_handle_t h, int level, int prec, const void* u, const void* ec,
                     const void* b, void* out, void* stream);

/* Zero-guess V(1,1) cycle from `level` down: e = B_level b, in precision
 * prec (scaled storage as in mg_sweep for the low precisions; for those,
 * MG_OPT_PRECISION must be set to prec first).  Levels at or below the tail
 * size run in the single-workgroup LDS tail kernel. */
int mg_coarse_cycle(mg_handle_t h, int level, int prec, const void* b, void* e,
                    void* stream);

/* ||b - A u||_2 over the whole batch on the finest grid (FP64); writes the
 * host double *norm.  Synchronises `stream`. */
int mg_residual_norm(mg_handle_t h, const double* b, const double* u, double* norm,
                     void* stream);

/* Accumulated device time (ms) and launch count of a timed kernel kind
 * (MG_TIME_*) on `level` since the last reset (MG_OPT_TIMING must be on). */
int mg_get_timing(mg_handle_t h, int kind, int level, double* total_ms, int* count);
int mg_reset_timing(mg_handle_t h);

/* Number of grid levels (finest N down to N = 4). */
int mg_num_levels(mg_handle_t h);

/* Releases every internal buffer of the handle; NULL is ignored. */
void mg_destroy(mg_handle_t h);

/* Thread-local message of the last failing call ("" if none). */
const char* mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SPAIMG_H */
