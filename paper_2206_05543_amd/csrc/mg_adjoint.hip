// gfx950 kernels of the reverse-mode (adjoint) V(1,1) cycle, FP64: the
// restriction of the reverse sweep, the coefficient-gradient reduction, the
// checkpoint conversions and the coarsest grid's matrix product.  The
// reverse smoothing steps are marching sweeps in mg_kernels.hip
// (launch_adj_sweep), and the forward recomputation uses the cycle's own
// kernels with their residual side outputs.
//
// The forward cycle (He, Liu and Wang, arXiv 2206.05543, Section 4, with the
// smoother of Section 2, eq. (smoother)) is linear in (u, b) and polynomial
// in the smoother coefficients c.  Its reverse sweep uses A^T = A and
// M^T = M (both stencils are symmetric under zero extension), P^T = 2^d R and
// R^T = 2^-d P for full weighting and linear interpolation.  With
// M = h^2 sum_j c_j K_j, the coefficient gradient of a smoothing step
// u_out = u + M r is dL/dc_j = h^2 <ubar_out, K_j r> = h^2 <K_j ubar_out, r>.
//
// The kernels here are one-node-per-thread (neighbours through L1/L2).
// Reductions are per-block partial sums in a fixed order, so gradients are
// deterministic.
#include <hip/hip_runtime.h>

#include "mg_internal.h"

namespace spaimg {
namespace {

struct Grid {
    int d, n;
    long pts;
    __device__ __forceinline__ void coords(long p, int* i, int* j, int* k) const {
        *i = p % n;
        *j = (p / n) % n;
        *k = d == 3 ? (int)(p / ((long)n * n)) : 0;
    }
    __device__ __forceinline__ double at(const double* a, int i, int j, int k) const {
        if (i < 0 || i >= n || j < 0 || j >= n) return 0.0;
        if (d == 3) {
            if (k < 0 || k >= n) return 0.0;
            return a[((long)k * n + j) * n + i];
        }
        return a[(long)j * n + i];
    }
};


// coarse = scale * R fine (full weighting; scale 2^d gives P^T)
__global__ void __launch_bounds__(256)
k_fw(const double* __restrict__ f, double* __restrict__ c, Grid gf, Grid gc, double scale) {
    const long offf = (long)blockIdx.y * gf.pts, offc = (long)blockIdx.y * gc.pts;
    for (long p = (long)blockIdx.x * 256 + threadIdx.x; p < gc.pts; p += (long)gridDim.x * 256) {
        int i, j, k;
        gc.coords(p, &i, &j, &k);
        const int fi = 2 * i + 1, fj = 2 * j + 1, fk = 2 * k + 1;
        double s = 0.0;
        const int kl = gf.d == 3 ? -1 : 0, kh = gf.d == 3 ? 1 : 0;
        for (int oz = kl; oz <= kh; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    double wt = (ox ? 0.25 : 0.5) * (oy ? 0.25 : 0.5);
                    if (gf.d == 3) wt *= oz ? 0.25 : 0.5;
                    s += wt * gf.at(f + offf, fi + ox, fj + oy, gf.d == 3 ? fk + oz : 0);
                }
        c[offc + p] = scale * s;
    }
}

// acc[j] = scale * sum_i partials[ncols * i + j], one workgroup per column,
// fixed order (each thread a strided subset, then a fixed tree)
__global__ void __launch_bounds__(1024)
k_reduce_cols(const double* __restrict__ partials, int count, int ncols, double* __restrict__ acc,
              double scale) {
    __shared__ double red[16];
    const int jc = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < count; i += 1024) s += partials[(long)ncols * i + jc];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < 16; ++i) t += red[i];
        acc[jc] = scale * t;
    }
}

// y (+)= G x for every batch entry (G: m x m, the exact coarsest solve)
__global__ void __launch_bounds__(64)
k_coarse_matvec(int m, const double* __restrict__ G, const double* __restrict__ x,
                double* __restrict__ y, int accumulate) {
    const long off = (long)blockIdx.x * m;
    const int r = threadIdx.x;
    if (r >= m) return;
    double s = 0.0;
    for (int q = 0; q < m; ++q) s += G[r * m + q] * x[off + q];
    if (accumulate) y[off + r] += s;
    else y[off + r] = s;
}

// Checkpoint of the cycle-start iterate in FP32: ck = fl32(u), and u is
// replaced by the rounded value (round to nearest even both ways), so that
// the forward pass continues from exactly what the checkpoint holds.
__global__ void __launch_bounds__(256)
k_ckpt32(double* __restrict__ u, float* __restrict__ ck, long count) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long)gridDim.x * 256) {
        const float f = (float)u[i];
        ck[i] = f;
        u[i] = (double)f;
    }
}

// FP64 copy of an FP32 checkpoint (exact)
__global__ void __launch_bounds__(256)
k_widen(const float* __restrict__ ck, double* __restrict__ u, long count) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long)gridDim.x * 256)
        u[i] = (double)ck[i];
}

inline Grid make_grid(int d, int n) {
    Grid g;
    g.d = d;
    g.n = n;
    g.pts = d == 3 ? (long)n * n * n : (long)n * n;
    return g;
}

inline dim3 point_grid(long pts, int batch) {
    long blocks = (pts + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    return dim3((unsigned)blocks, batch);
}

}  // namespace

hipError_t launch_fw(int d, int n, int batch, const double* fine, double* coarse, double scale,
                     hipStream_t st) {
    const int nc = (n + 1) / 2 - 1;
    const Grid gf = make_grid(d, n), gc = make_grid(d, nc);
    hipLaunchKernelGGL(k_fw, point_grid(gc.pts, batch), dim3(256), 0, st, fine, coarse, gf, gc, scale);
    return hipGetLastError();
}

hipError_t launch_reduce_cols(const double* partials, int count, int ncols, double* acc,
                              double scale, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_cols, dim3(ncols), dim3(1024), 0, st, partials, count, ncols, acc,
                       scale);
    return hipGetLastError();
}

hipError_t launch_ckpt32(double* u, float* ck, long count, hipStream_t st) {
    hipLaunchKernelGGL(k_ckpt32, point_grid(count, 1), dim3(256), 0, st, u, ck, count);
    return hipGetLastError();
}

hipError_t launch_widen(const float* ck, double* u, long count, hipStream_t st) {
    hipLaunchKernelGGL(k_widen, point_grid(count, 1), dim3(256), 0, st, ck, u, count);
    return hipGetLastError();
}

hipError_t launch_coarse_matvec(int m, int batch, const double* G, const double* x, double* y,
                                bool accumulate, hipStream_t st) {
    if (m > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_coarse_matvec, dim3(batch), dim3(64), 0, st, m, G, x, y, accumulate ? 1 : 0);
    return hipGetLastError();
}

}  // namespace spaimg
