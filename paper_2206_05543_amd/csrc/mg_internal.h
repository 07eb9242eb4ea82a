// Internal interface between the host orchestration (mg_api.cpp) and the
// gfx950 kernels (mg_kernels.hip).  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace spaimg {

// Event pair in which the next kernel launched by this thread records its own
// start and end (hipExtLaunchKernelGGL: the dispatch's timestamps, with no
// extra command on the stream, so the interval is the kernel alone); the
// launch consumes it.  Null events: an ordinary launch.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
LaunchEvents& launch_events();

// Storage precision of a level hierarchy.  FP64 computes in double; FP32 and
// FP16 (storage) compute in float.
enum Prec : int { P64 = 0, P32 = 1, P16 = 2 };

inline size_t prec_bytes(Prec p) { return p == P64 ? 8 : (p == P32 ? 4 : 2); }

// One stencil sweep over a grid with n = N-1 interior nodes per direction.
// Values are stored scaled by sigma (stored = sigma * true value); the sweep
// uses sA = 1/(h^2 sigma) in front of the Laplacian stencil and
// sW = h^2 sigma in front of the SPAI stencil, so the same code serves the
// unscaled FP64 hierarchy (sigma = 1) and the h-free scaled low-precision
// hierarchies (sigma = 1/h^2, sA = sW = 1).
struct Sweep {
    const void* u = nullptr;     // current iterate (ignored for zero guess)
    bool u_f32 = false;          // u holds FP32 values (the FP64 fused pre-smoother
                                 // with a residual output only: an FP32 checkpoint)
    const void* b = nullptr;     // right-hand side
    void* out = nullptr;         // output (new iterate, or coarse rhs)
    int d = 2;
    int n = 0;                   // interior nodes per direction (fine grid)
    int batch = 1;
    double sA = 0, sW = 0;
    double c[4] = {0, 0, 0, 0};  // SPAI coefficients: centre, faces, then the
                                 // diagonals (2D) or edges and corners (3D)
    double* partials = nullptr;  // per-block sum r^2 (norm variant)
    double* bparts = nullptr;    // per-block sum b^2 beside it (fused pre-smoother, FP64)
    long partials_cap = 0;       // entries available in partials
    // optional fused correction: the sweep reads u + pf * P ec, where ec is a
    // coarse-grid field ((n+1)/2 - 1 interior nodes) of the same storage type
    const void* ec = nullptr;
    double pf = 1.0;
    // optional norm finalisation (restriction only): block 0 reduces the
    // fin_count partial sums (and maxima) of the previous sweep in a fixed
    // order and writes (sqrt(sum), max) to fin_dev and sqrt(sum) to the
    // pinned host mirror fin_host (device address)
    const double* fin_ps = nullptr;
    const double* fin_pm = nullptr;
    int fin_count = 0;
    double* fin_dev = nullptr;
    double* fin_host = nullptr;
    // coarse right-hand side written by the fused zero-guess smoother +
    // restriction ((n+1)/2 - 1 interior nodes per direction)
    void* out_c = nullptr;
    // the next cycle's pre-smoothed iterate, written by the fused
    // post-smoother + pre-smoother + restriction
    void* out_t = nullptr;
    // optional (FP64): the residual b - sA L v that the smoother applies K_c
    // to, stored at every node the sweep owns (the adjoint cycle's forward
    // recomputation keeps it)
    void* rout = nullptr;
};

// Launchers return hipSuccess or the launch error.  *nparts receives the
// number of per-block partial sums written (norm variants).
hipError_t launch_smooth(Prec p, bool zero_guess, bool norm, const Sweep& s,
                         hipStream_t st, int* nparts);
hipError_t launch_restrict(Prec p, const Sweep& s, hipStream_t st);
// zero-guess pre-smoother fused with the restriction (2D): out = sW K b on
// the fine grid, out_c = R (b - sA L out) on the coarse grid (u, ec ignored)
hipError_t launch_zero_smooth_restrict(Prec p, const Sweep& s, hipStream_t st);
// pre-smoother fused with the restriction (nonzero iterate): out = u +
// sW K (b - sA L u) on the fine grid, out_c = R (b - sA L out); the norm
// variant (FP64 only) writes per-block sums of (b - sA L u)^2 to partials
hipError_t launch_smooth_restrict(Prec p, bool norm, const Sweep& s, hipStream_t st,
                                  int* nparts);
// post-smoother of one V(1,1) cycle fused with the pre-smoother and the
// restriction of the next (2D): with w = u + pf P ec (u: the pre-smoothed
// iterate, ec: the coarse correction), out = w + sW K (b - sA L w), out_t =
// out + sW K (b - sA L out), out_c = R (b - sA L out_t); the norm variant
// (FP64 only) writes per-block sums of (b - sA L out)^2 to partials
hipError_t launch_post_pre_restrict(Prec p, bool norm, const Sweep& s, hipStream_t st,
                                    int* nparts);
// u (fine, n interior) += pf * P ec (coarse, n/2 interior)
hipError_t launch_prolong(Prec p, int d, int n, int batch, const void* ec,
                          void* u, double pf, hipStream_t st);
// out = in + pf * P ec (in may equal out)
hipError_t launch_prolong_to(Prec p, int d, int n, int batch, const void* ec, const void* in,
                             void* out, double pf, hipStream_t st);
// Coarse tail: from a level with nt interior nodes down to 3 and back up, in
// one workgroup, for every batch entry.  b and e hold the tail's top level;
// e is written only (every visit sequence starts from a zero guess).
struct Tail {
    int d = 2, nt = 0, batch = 1;
    const void* b = nullptr;
    void* e = nullptr;
    double c[4] = {0, 0, 0, 0};
    const double* ginv = nullptr;  // device: sigma_0 * A_0^{-1}, (3^d)^2
    double sigma_top = 1.0;        // storage scale of the top tail level
    bool scaled = false;           // scaled hierarchy (sigma_l = 1/h_l^2)
    int wvisits = 0;               // 0: V(1,1); 1 or 2: W(1,0) visits of the
                                   // top level, the first from a zero guess
};
hipError_t launch_tail(Prec p, const Tail& t, hipStream_t st);
size_t tail_lds_bytes(Prec p, int d, int nt);

// Deterministic norm finalisation: out[0] = sqrt(sum partials) (fixed order),
// out[1] = max of the max-partials (if maxparts != nullptr); the norm also
// goes to `host` (device address of a coherent pinned mirror) if given.
hipError_t launch_finalize(const double* partials, const double* maxparts,
                           int count, double* out, hipStream_t st, double* host = nullptr);

// Per-block partial sums of v^2 over count doubles (fixed order).
hipError_t launch_sumsq(const double* v, long count, double* partials, long partials_cap,
                        hipStream_t st, int* nparts);

// Fine-grid residual norm of an FP64 iterate: partials of r^2 and max|r|.
hipError_t launch_residual_norm(int d, int n, int batch, const double* u,
                                const double* b, double inv_h2, double* psum,
                                double* pmax, long partials_cap, hipStream_t st,
                                int* nparts, double* bparts = nullptr);

// One FP64 refinement step: unew = u + e_lo * scale_prev (if e_lo), the
// residual r = b - A unew in FP64 and r_lo = s r stored in precision p,
// where s = 2^-ceil(log2(max|r_prev|)) is read from maxprev on the device
// and written to scales[k].  Partials of r^2 and max|r|.
struct IRStep {
    int d = 2, n = 0, batch = 1, k = 0;
    const double* u = nullptr;
    double* unew = nullptr;
    const void* e_lo = nullptr;  // correction from the previous inner cycle
    const double* b = nullptr;
    void* r_lo = nullptr;
    double inv_h2 = 0;
    double sigma0 = 1;           // storage scale of the inner fine level
    double* scales = nullptr;    // device array of refinement scales
    const double* maxprev = nullptr;  // device: max|r_{k-1}|
    double* psum = nullptr;
    double* pmax = nullptr;
    double* bparts = nullptr;    // also partials of b^2 (||b|| of a solve)
    long partials_cap = 0;
};
hipError_t launch_ir_step(Prec p, const IRStep& s, hipStream_t st, int* nparts);

// Kernels of the reverse-mode (adjoint) cycle, FP64, whole batch.
//   mode 0 (the reverse of a smoothing step): w = sW sum_j c_j K_j ubar (K_2:
//   diagonals in 2D, edges in 3D; K_3: corners, 3D), partials[4 i + j] = sW x
//   block sums of (K_j ubar) r over the owned nodes; mode 1 (the reverse of
//   the restricted residual): w = scale P ec (ec on the next coarser grid);
//   then ubar_new = ubar - sA L w and bbar += w.  ubar_new must not alias
//   ubar.  *nparts = blocks.
hipError_t launch_adj_sweep(int d, int n, int batch, int mode, const double* ubar,
                            const double* r, const double* ec, double scale, double* ubar_new,
                            double* bbar, double* partials, long partials_cap, double sA,
                            double sW, const double* c, hipStream_t st, int* nparts);
//   coarse = scale * R fine (full weighting)
hipError_t launch_fw(int d, int n, int batch, const double* fine, double* coarse,
                     double scale, hipStream_t st);
//   acc[j] = scale * sum_i partials[ncols i + j] (fixed order)
hipError_t launch_reduce_cols(const double* partials, int count, int ncols, double* acc,
                              double scale, hipStream_t st);
//   ck = fl32(u), u = (double) ck  (FP32 checkpoint; the forward continues
//   from the rounded iterate)
hipError_t launch_ckpt32(double* u, float* ck, long count, hipStream_t st);
//   u = (double) ck
hipError_t launch_widen(const float* ck, double* u, long count, hipStream_t st);
//   y (+)= G x per batch entry, G m x m (m <= 64)
hipError_t launch_coarse_matvec(int m, int batch, const double* G, const double* x,
                                double* y, bool accumulate, hipStream_t st);

}  // namespace spaimg
