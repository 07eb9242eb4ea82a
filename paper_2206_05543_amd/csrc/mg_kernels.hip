// gfx950 kernels of the SPAI-smoothed geometric multigrid cycle.
//
// Method: He, Liu and Wang, "Optimized sparse approximate inverse smoothers
// for solving Laplacian linear systems" (arXiv 2206.05543).  The 5-/7-point
// Laplacian is eq. (A_h) of Section 1; the smoother is the preconditioned
// Richardson step of Section 2 (eq. (smoother)) with M from the 9-point
// family Upsilon (Section 3.1) or the 7-point family T (Section 3.2); the
// cycle uses full weighting, linear interpolation, rediscretised coarse
// operators and an exact solve at h0 = 1/4 (Section 4).
//
// Layout: interior nodes only, (N-1)^d per grid, x fastest, batch outermost.
// All sweeps are HBM-streaming stencils (about 1 flop per byte), so they are
// written for bandwidth: each workgroup owns an x strip (2D) or an xy tile
// (3D) plus halo rings, and marches through the remaining direction plane by
// plane.  The current plane of u and of the residual live in LDS ring
// buffers; the neighbouring planes live in registers; the next plane is
// prefetched from HBM while the current one is computed; one barrier per
// plane.  Workgroup ids are remapped so that each of the 8 XCDs (own L2)
// receives a contiguous range of tiles, so halo reloads of neighbouring
// tiles hit the same L2.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mg_internal.h"

namespace spaimg {
namespace {

constexpr int kXCD = 8;

// Bijection from hardware workgroup order (round-robin over XCDs) to a
// logical tile order in which every XCD owns one contiguous range.
__device__ __forceinline__ int xcd_remap(int bid, int total) {
    const int per = total / kXCD, rem = total % kXCD;
    const int x = bid % kXCD, i = bid / kXCD;
    return x * per + min(x, rem) + i;
}

template <typename C, typename S>
__device__ __forceinline__ C cvt(S v) { return static_cast<C>(v); }

// Deterministic workgroup sum (fixed shuffle tree, then waves in order).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i) s += red[i];
    return s;
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i) s = fmax(s, red[i]);
    return s;
}

// ---------------------------------------------------------------------------
// 3D fused residual + SPAI smoother:  out = u + sW * K_c (b - sA * L u)
// K_c = c0 I + c1 (6 face neighbours); residual zero outside the grid.
// Tile TX x TY outputs per plane; the residual is computed on the tile plus a
// ring of 1, which needs u on the tile plus a ring of 2 (without corners).
// Output lags the residual by one plane.
// ---------------------------------------------------------------------------
template <typename S, typename C, int TX, int TY, int NT, bool ZG, bool NORM>
__global__ void __launch_bounds__(NT)
k_smooth3d(const S* __restrict__ u, const S* __restrict__ b, S* __restrict__ out,
           int n, int tiles_x, int tiles_y, int zchunk, int nchunks, C sA,
           C sW, C c0, C c1, double* __restrict__ partials) {
    constexpr int RX = TX + 2, RY = TY + 2, NR = RX * RY;
    constexpr int UX = TX + 4, UY = TY + 4, NU = UX * UY;
    constexpr int M = (NR + NT - 1) / NT;
    constexpr int NR2 = 2 * RX + 2 * RY;
    static_assert(NR2 <= NT, "one thread per ring-2 point");
    __shared__ C uL[2][ZG ? 1 : NU];
    __shared__ C rL[2][NR];
    __shared__ double red[NT / 64];

    const int total = tiles_x * tiles_y * nchunks;
    const int lg = xcd_remap(blockIdx.x, total);
    const int tx = lg % tiles_x, ty = (lg / tiles_x) % tiles_y,
              ch = lg / (tiles_x * tiles_y);
    const long plane = (long)n * n;
    const long boff = (long)blockIdx.y * plane * n;
    b += boff;
    out += boff;
    if (!ZG) u += boff;
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = ch * zchunk, z1 = min(z0 + zchunk, n);
    const int t = threadIdx.x;

    int rl[M], ul[M], go[M];
    bool inr[M], val[M], inn[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = t + m * NT;
        inr[m] = i < NR;
        const int lx = i % RX, ly = i / RX;
        const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        val[m] = inr[m] && gx >= 0 && gx < n && gy >= 0 && gy < n;
        inn[m] = val[m] && lx >= 1 && lx <= TX && ly >= 1 && ly <= TY;
        rl[m] = inr[m] ? i : 0;
        ul[m] = inr[m] ? (ly + 1) * UX + lx + 1 : 0;
        go[m] = val[m] ? gy * n + gx : 0;
    }
    int r2l = 0, r2g = 0;
    bool r2v = false;
    if (!ZG && t < NR2) {
        int ux, uy;
        if (t < RX) { ux = 1 + t; uy = 0; }
        else if (t < 2 * RX) { ux = 1 + t - RX; uy = UY - 1; }
        else if (t < 2 * RX + RY) { ux = 0; uy = 1 + t - 2 * RX; }
        else { ux = UX - 1; uy = 1 + t - 2 * RX - RY; }
        const int gx = x0 - 2 + ux, gy = y0 - 2 + uy;
        r2l = uy * UX + ux;
        r2v = gx >= 0 && gx < n && gy >= 0 && gy < n;
        r2g = r2v ? gy * n + gx : 0;
    }
    auto ldu = [&](int p, int m) -> C {
        return (!ZG && val[m] && p >= 0 && p < n) ? cvt<C>(u[p * plane + go[m]]) : C(0);
    };
    auto ldb = [&](int p, int m) -> C {
        return (val[m] && p >= 0 && p < n) ? cvt<C>(b[p * plane + go[m]]) : C(0);
    };
    auto ldr2 = [&](int p) -> C {
        return (!ZG && r2v && p >= 0 && p < n) ? cvt<C>(u[p * plane + r2g]) : C(0);
    };

    C um1[M], u0[M], up1[M], nu[M], b0[M], nb[M], rm2[M], rm1[M], r0[M];
    C urp1 = 0, nur = 0;
    double nacc = 0.0;
    const int s0 = z0 - 1;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        um1[m] = ldu(s0 - 1, m);
        u0[m] = ldu(s0, m);
        up1[m] = ldu(s0 + 1, m);
        b0[m] = ldb(s0, m);
        rm2[m] = rm1[m] = C(0);
    }
    if (!ZG) {
        const C ur0 = ldr2(s0);
        urp1 = ldr2(s0 + 1);
        const int sl = (s0 + 2) & 1;
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (inr[m]) uL[sl][ul[m]] = u0[m];
        if (t < NR2) uL[sl][r2l] = ur0;
    }

    for (int s = s0; s <= z1; ++s) {
        __syncthreads();
        const int cur = (s + 2) & 1;
        // prefetch the planes needed by the next step
#pragma unroll
        for (int m = 0; m < M; ++m) {
            nu[m] = ldu(s + 2, m);
            nb[m] = ldb(s + 1, m);
        }
        if (!ZG && t < NR2) nur = ldr2(s + 2);
        // residual of plane s on the tile plus ring 1
        const bool pin = s >= 0 && s < n;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            C r = C(0);
            if (val[m] && pin) {
                if (ZG) {
                    r = b0[m];
                } else {
                    const C* U = uL[cur];
                    const int q = ul[m];
                    const C lap = C(6) * u0[m] - U[q - 1] - U[q + 1] - U[q - UX] -
                                  U[q + UX] - um1[m] - up1[m];
                    r = b0[m] - sA * lap;
                }
            }
            r0[m] = r;
            if (inr[m]) rL[cur][rl[m]] = r;
        }
        // smoothed plane s - 1
        const int p = s - 1;
        if (p >= z0) {
            const C* R = rL[cur ^ 1];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (!inn[m]) continue;
                const int q = rl[m];
                const C rc = rm1[m];
                const C nbs = R[q - 1] + R[q + 1] + R[q - RX] + R[q + RX] + rm2[m] + r0[m];
                const C v = (ZG ? C(0) : um1[m]) + sW * (c0 * rc + c1 * nbs);
                out[p * plane + go[m]] = static_cast<S>(v);
                if (NORM) nacc += (double)rc * (double)rc;
            }
        }
        // u of plane s + 1 into the other LDS slot
        if (!ZG) {
#pragma unroll
            for (int m = 0; m < M; ++m)
                if (inr[m]) uL[cur ^ 1][ul[m]] = up1[m];
            if (t < NR2) uL[cur ^ 1][r2l] = urp1;
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            um1[m] = u0[m];
            u0[m] = up1[m];
            up1[m] = nu[m];
            b0[m] = nb[m];
            rm2[m] = rm1[m];
            rm1[m] = r0[m];
        }
        urp1 = nur;
    }
    if (NORM) {
        const double s = block_sum<NT>(nacc, red);
        if (t == 0) partials[(long)blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// 2D fused residual + SPAI smoother (9-point M): x strips of TX outputs,
// marching over rows.  The residual of row s is computed on the strip plus a
// ring of 1; output lags by two rows because the 9-point stencil needs the
// residual of rows p-1..p+1 at x-1..x+1 from LDS (4 row slots).
// ---------------------------------------------------------------------------
template <typename S, typename C, int TX, int NT, bool ZG, bool NORM>
__global__ void __launch_bounds__(NT)
k_smooth2d(const S* __restrict__ u, const S* __restrict__ b, S* __restrict__ out,
           int n, int tiles_x, int ychunk, int nchunks, C sA, C sW, C c0, C c1,
           C c2, double* __restrict__ partials) {
    constexpr int RX = TX + 2, UX = TX + 4;
    constexpr int M = (RX + NT - 1) / NT;
    __shared__ C uL[2][ZG ? 1 : UX];
    __shared__ C rL[4][RX];
    __shared__ double red[NT / 64];

    const int total = tiles_x * nchunks;
    const int lg = xcd_remap(blockIdx.x, total);
    const int tx = lg % tiles_x, ch = lg / tiles_x;
    const long area = (long)n * n;
    const long boff = (long)blockIdx.y * area;
    b += boff;
    out += boff;
    if (!ZG) u += boff;
    const int x0 = tx * TX;
    const int y0 = ch * ychunk, y1 = min(y0 + ychunk, n);
    const int t = threadIdx.x;

    int go[M];
    bool inr[M], val[M], inn[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = t + m * NT;
        inr[m] = i < RX;
        const int gx = x0 - 1 + i;
        val[m] = inr[m] && gx >= 0 && gx < n;
        inn[m] = val[m] && i >= 1 && i <= TX;
        go[m] = val[m] ? gx : 0;
    }
    // ring-2 columns x0-2 (thread 0) and x0+TX+1 (thread 1)
    const int r2x = (t == 0) ? x0 - 2 : x0 + TX + 1;
    const int r2l = (t == 0) ? 0 : UX - 1;
    const bool r2v = !ZG && t < 2 && r2x >= 0 && r2x < n;

    auto ldu = [&](int p, int m) -> C {
        return (!ZG && val[m] && p >= 0 && p < n) ? cvt<C>(u[(long)p * n + go[m]]) : C(0);
    };
    auto ldb = [&](int p, int m) -> C {
        return (val[m] && p >= 0 && p < n) ? cvt<C>(b[(long)p * n + go[m]]) : C(0);
    };
    auto ldr2 = [&](int p) -> C {
        return (r2v && p >= 0 && p < n) ? cvt<C>(u[(long)p * n + r2x]) : C(0);
    };

    C um2[M], um1[M], u0[M], up1[M], nu[M], b0[M], nb[M];
    C urp1 = 0, nur = 0;
    double nacc = 0.0;
    const int s0 = y0 - 1;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        um2[m] = C(0);
        um1[m] = ldu(s0 - 1, m);
        u0[m] = ldu(s0, m);
        up1[m] = ldu(s0 + 1, m);
        b0[m] = ldb(s0, m);
    }
    if (!ZG) {
        const C ur0 = ldr2(s0);
        urp1 = ldr2(s0 + 1);
        const int sl = (s0 + 2) & 1;
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (inr[m]) uL[sl][t + m * NT + 1] = u0[m];
        if (t < 2) uL[sl][r2l] = ur0;
    }

    for (int s = s0; s <= y1 + 1; ++s) {
        __syncthreads();
        const int cur = (s + 2) & 1;
        const int rs = (s + 4) & 3;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            nu[m] = ldu(s + 2, m);
            nb[m] = ldb(s + 1, m);
        }
        if (!ZG && t < 2) nur = ldr2(s + 2);
        const bool pin = s >= 0 && s < n;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            C r = C(0);
            const int i = t + m * NT;
            if (val[m] && pin) {
                if (ZG) {
                    r = b0[m];
                } else {
                    const C* U = uL[cur];
                    const C lap = C(4) * u0[m] - U[i] - U[i + 2] - um1[m] - up1[m];
                    r = b0[m] - sA * lap;
                }
            }
            if (inr[m]) rL[rs][i] = r;
        }
        const int p = s - 2;
        if (p >= y0) {
            const C* R0 = rL[(p + 3) & 3];  // row p - 1
            const C* R1 = rL[(p + 4) & 3];  // row p
            const C* R2 = rL[(p + 5) & 3];  // row p + 1
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (!inn[m]) continue;
                const int i = t + m * NT;
                const C rc = R1[i];
                const C fc = R1[i - 1] + R1[i + 1] + R0[i] + R2[i];
                const C cn = R0[i - 1] + R0[i + 1] + R2[i - 1] + R2[i + 1];
                const C v = (ZG ? C(0) : um2[m]) + sW * (c0 * rc + c1 * fc + c2 * cn);
                out[(long)p * n + go[m]] = static_cast<S>(v);
                if (NORM) nacc += (double)rc * (double)rc;
            }
        }
        if (!ZG) {
#pragma unroll
            for (int m = 0; m < M; ++m)
                if (inr[m]) uL[cur ^ 1][t + m * NT + 1] = up1[m];
            if (t < 2) uL[cur ^ 1][r2l] = urp1;
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            um2[m] = um1[m];
            um1[m] = u0[m];
            u0[m] = up1[m];
            up1[m] = nu[m];
            b0[m] = nb[m];
        }
        urp1 = nur;
    }
    if (NORM) {
        const double sum = block_sum<NT>(nacc, red);
        if (t == 0) partials[(long)blockIdx.y * gridDim.x + blockIdx.x] = sum;
    }
}

// ---------------------------------------------------------------------------
// 3D fused residual + full-weighting restriction: bc = R (b - sA L u).
// Coarse tile TXc x TYc (one coarse column per thread); the fine residual is
// computed plane by plane on the (2TXc+1) x (2TYc+1) fine window and reduced
// in xy; the z weights (1/4, 1/2, 1/4) are accumulated in registers.
// ---------------------------------------------------------------------------
template <typename S, typename C, int TXc, int TYc>
__global__ void __launch_bounds__(TXc * TYc)
k_restrict3d(const S* __restrict__ u, const S* __restrict__ b, S* __restrict__ bc,
             int n, int nc, int tiles_x, int tiles_y, int zchunk, int nchunks, C sA) {
    constexpr int NT = TXc * TYc;
    constexpr int FX = 2 * TXc + 1, FY = 2 * TYc + 1, NF = FX * FY;
    constexpr int UX = FX + 2, UY = FY + 2, NU = UX * UY;
    constexpr int M = (NF + NT - 1) / NT;
    constexpr int NR2 = 2 * FX + 2 * FY;
    static_assert(NR2 <= NT, "one thread per ring point");
    __shared__ C uL[2][NU];
    __shared__ C rL[2][NF];

    const int total = tiles_x * tiles_y * nchunks;
    const int lg = xcd_remap(blockIdx.x, total);
    const int tx = lg % tiles_x, ty = (lg / tiles_x) % tiles_y,
              ch = lg / (tiles_x * tiles_y);
    const long plane = (long)n * n, cplane = (long)nc * nc;
    u += (long)blockIdx.y * plane * n;
    b += (long)blockIdx.y * plane * n;
    bc += (long)blockIdx.y * cplane * nc;
    const int cx0 = tx * TXc, cy0 = ty * TYc;
    const int Z0 = ch * zchunk, Z1 = min(Z0 + zchunk, nc);
    const int fx0 = 2 * cx0, fy0 = 2 * cy0;  // fine index of window origin
    const int t = threadIdx.x;

    int ul[M], go[M];
    bool inr[M], val[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = t + m * NT;
        inr[m] = i < NF;
        const int lx = i % FX, ly = i / FX;
        const int gx = fx0 + lx, gy = fy0 + ly;
        val[m] = inr[m] && gx < n && gy < n;
        ul[m] = inr[m] ? (ly + 1) * UX + lx + 1 : 0;
        go[m] = val[m] ? gy * n + gx : 0;
    }
    int r2l = 0, r2g = 0;
    bool r2v = false;
    if (t < NR2) {
        int ux, uy;
        if (t < FX) { ux = 1 + t; uy = 0; }
        else if (t < 2 * FX) { ux = 1 + t - FX; uy = UY - 1; }
        else if (t < 2 * FX + FY) { ux = 0; uy = 1 + t - 2 * FX; }
        else { ux = UX - 1; uy = 1 + t - 2 * FX - FY; }
        const int gx = fx0 - 1 + ux, gy = fy0 - 1 + uy;
        r2l = uy * UX + ux;
        r2v = gx >= 0 && gx < n && gy >= 0 && gy < n;
        r2g = r2v ? gy * n + gx : 0;
    }
    auto ldu = [&](int p, int m) -> C {
        return (val[m] && p >= 0 && p < n) ? cvt<C>(u[p * plane + go[m]]) : C(0);
    };
    auto ldb = [&](int p, int m) -> C {
        return (val[m] && p >= 0 && p < n) ? cvt<C>(b[p * plane + go[m]]) : C(0);
    };
    auto ldr2 = [&](int p) -> C {
        return (r2v && p >= 0 && p < n) ? cvt<C>(u[p * plane + r2g]) : C(0);
    };
    const int cx = t % TXc, cy = t / TXc;
    const bool cval = (cx0 + cx) < nc && (cy0 + cy) < nc;
    const int cgo = (cy0 + cy) * nc + cx0 + cx;

    C um1[M], u0[M], up1[M], nu[M], b0[M], nb[M];
    C urp1 = 0, nur = 0, acc = 0;
    const int f0 = 2 * Z0, f1 = 2 * Z1;  // fine planes f0..f1 contribute
#pragma unroll
    for (int m = 0; m < M; ++m) {
        um1[m] = ldu(f0 - 1, m);
        u0[m] = ldu(f0, m);
        up1[m] = ldu(f0 + 1, m);
        b0[m] = ldb(f0, m);
    }
    {
        const C ur0 = ldr2(f0);
        urp1 = ldr2(f0 + 1);
        const int sl = f0 & 1;
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (inr[m]) uL[sl][ul[m]] = u0[m];
        if (t < NR2) uL[sl][r2l] = ur0;
    }
    for (int s = f0; s <= f1 + 1; ++s) {
        __syncthreads();
        const int cur = s & 1;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            nu[m] = ldu(s + 2, m);
            nb[m] = ldb(s + 1, m);
        }
        if (t < NR2) nur = ldr2(s + 2);
        if (s <= f1) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                C r = C(0);
                if (val[m]) {
                    const C* U = uL[cur];
                    const int q = ul[m];
                    const C lap = C(6) * u0[m] - U[q - 1] - U[q + 1] - U[q - UX] -
                                  U[q + UX] - um1[m] - up1[m];
                    r = b0[m] - sA * lap;
                }
                if (inr[m]) rL[cur][t + m * NT] = r;
            }
        }
        const int f = s - 1;  // fine plane whose residual is reduced now
        if (f >= f0) {
            const C* R = rL[cur ^ 1];
            const int q = (2 * cy + 1) * FX + 2 * cx + 1;
            const C xs = C(0.25) * R[q] +
                         C(0.125) * (R[q - 1] + R[q + 1] + R[q - FX] + R[q + FX]) +
                         C(0.0625) * (R[q - FX - 1] + R[q - FX + 1] + R[q + FX - 1] + R[q + FX + 1]);
            if (((f - f0) & 1) == 0) {
                if (f > f0) {
                    acc += C(0.25) * xs;
                    const int Zc = f / 2 - 1;
                    if (cval) bc[Zc * cplane + cgo] = static_cast<S>(acc);
                }
                acc = C(0.25) * xs;
            } else {
                acc += C(0.5) * xs;
            }
        }
        if (s + 1 <= f1 + 1) {
#pragma unroll
            for (int m = 0; m < M; ++m)
                if (inr[m]) uL[cur ^ 1][ul[m]] = up1[m];
            if (t < NR2) uL[cur ^ 1][r2l] = urp1;
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            um1[m] = u0[m];
            u0[m] = up1[m];
            up1[m] = nu[m];
            b0[m] = nb[m];
        }
        urp1 = nur;
    }
}

// ---------------------------------------------------------------------------
// 2D fused residual + full-weighting restriction: a strip of TXc coarse
// columns (one per thread), marching over fine rows.
// ---------------------------------------------------------------------------
template <typename S, typename C, int TXc>
__global__ void __launch_bounds__(TXc)
k_restrict2d(const S* __restrict__ u, const S* __restrict__ b, S* __restrict__ bc,
             int n, int nc, int tiles_x, int ychunk, int nchunks, C sA) {
    constexpr int NT = TXc;
    constexpr int FX = 2 * TXc + 1, UX = FX + 2;
    constexpr int M = (FX + NT - 1) / NT;
    __shared__ C uL[2][UX];
    __shared__ C rL[2][FX];

    const int total = tiles_x * nchunks;
    const int lg = xcd_remap(blockIdx.x, total);
    const int tx = lg % tiles_x, ch = lg / tiles_x;
    u += (long)blockIdx.y * n * n;
    b += (long)blockIdx.y * n * n;
    bc += (long)blockIdx.y * nc * nc;
    const int cx0 = tx * TXc, fx0 = 2 * cx0;
    const int Y0 = ch * ychunk, Y1 = min(Y0 + ychunk, nc);
    const int t = threadIdx.x;

    int go[M];
    bool inr[M], val[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = t + m * NT;
        inr[m] = i < FX;
        const int gx = fx0 + i;
        val[m] = inr[m] && gx < n;
        go[m] = val[m] ? gx : 0;
    }
    const int r2x = (t == 0) ? fx0 - 1 : fx0 + FX;
    const int r2l = (t == 0) ? 0 : UX - 1;
    const bool r2v = t < 2 && r2x >= 0 && r2x < n;
    auto ldu = [&](int p, int m) -> C {
        return (val[m] && p >= 0 && p < n) ? cvt<C>(u[(long)p * n + go[m]]) : C(0);
    };
    auto ldb = [&](int p, int m) -> C {
        return (val[m] && p >= 0 && p < n) ? cvt<C>(b[(long)p * n + go[m]]) : C(0);
    };
    auto ldr2 = [&](int p) -> C {
        return (r2v && p >= 0 && p < n) ? cvt<C>(u[(long)p * n + r2x]) : C(0);
    };
    const bool cval = (cx0 + t) < nc;

    C um1[M], u0[M], up1[M], nu[M], b0[M], nb[M];
    C urp1 = 0, nur = 0, acc = 0;
    const int f0 = 2 * Y0, f1 = 2 * Y1;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        um1[m] = ldu(f0 - 1, m);
        u0[m] = ldu(f0, m);
        up1[m] = ldu(f0 + 1, m);
        b0[m] = ldb(f0, m);
    }
    {
        const C ur0 = ldr2(f0);
        urp1 = ldr2(f0 + 1);
        const int sl = f0 & 1;
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (inr[m]) uL[sl][t + m * NT + 1] = u0[m];
        if (t < 2) uL[sl][r2l] = ur0;
    }
    for (int s = f0; s <= f1 + 1; ++s) {
        __syncthreads();
        const int cur = s & 1;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            nu[m] = ldu(s + 2, m);
            nb[m] = ldb(s + 1, m);
        }
        if (t < 2) nur = ldr2(s + 2);
        if (s <= f1) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int i = t + m * NT;
                C r = C(0);
                if (val[m]) {
                    const C* U = uL[cur];
                    const C lap = C(4) * u0[m] - U[i] - U[i + 2] - um1[m] - up1[m];
                    r = b0[m] - sA * lap;
                }
                if (inr[m]) rL[cur][i] = r;
            }
        }
        const int f = s - 1;
        if (f >= f0) {
            const C* R = rL[cur ^ 1];
            const int q = 2 * t + 1;
            const C xs = C(0.5) * R[q] + C(0.25) * (R[q - 1] + R[q + 1]);
            if (((f - f0) & 1) == 0) {
                if (f > f0) {
                    acc += C(0.25) * xs;
                    const int Yc = f / 2 - 1;
                    if (cval) bc[(long)Yc * nc + cx0 + t] = static_cast<S>(acc);
                }
                acc = C(0.25) * xs;
            } else {
                acc += C(0.5) * xs;
            }
        }
        if (s + 1 <= f1 + 1) {
#pragma unroll
            for (int m = 0; m < M; ++m)
                if (inr[m]) uL[cur ^ 1][t + m * NT + 1] = up1[m];
            if (t < 2) uL[cur ^ 1][r2l] = urp1;
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            um1[m] = u0[m];
            u0[m] = up1[m];
            up1[m] = nu[m];
            b0[m] = nb[m];
        }
        urp1 = nur;
    }
}

// ---------------------------------------------------------------------------
// Linear interpolation + correction: u += pf * P ec.  One fine node per
// thread; the coarse values (1/2^d of the traffic) come through L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int interp_idx(int i, int nc, int* j0, int* j1) {
    // fine index i (grid coordinate i+1): even coordinate -> one coarse node,
    // odd -> two; returns the count, indices clipped to the coarse interior
    // (-1 marks a boundary node, value 0).
    const int g = i + 1;
    if ((g & 1) == 0) {
        *j0 = g / 2 - 1;
        *j1 = -1;
        return 1;
    }
    const int a = (g - 1) / 2 - 1, c = (g + 1) / 2 - 1;
    *j0 = (a >= 0 && a < nc) ? a : -1;
    *j1 = (c >= 0 && c < nc) ? c : -1;
    return 2;
}

template <typename S, typename C>
__global__ void __launch_bounds__(256)
k_prolong2d(const S* __restrict__ ec, S* __restrict__ u, int n, int nc, C pf) {
    const long area = (long)n * n;
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= area) return;
    u += (long)blockIdx.y * area;
    ec += (long)blockIdx.y * nc * nc;
    const int i = idx % n, j = idx / n;
    int ia, ib, ja, jb;
    const int ni = interp_idx(i, nc, &ia, &ib);
    const int nj = interp_idx(j, nc, &ja, &jb);
    const C wi = ni == 1 ? C(1) : C(0.5), wj = nj == 1 ? C(1) : C(0.5);
    auto e = [&](int x, int y) -> C {
        return (x >= 0 && y >= 0) ? cvt<C>(ec[y * nc + x]) : C(0);
    };
    C s = e(ia, ja);
    if (ni == 2) s += e(ib, ja);
    if (nj == 2) {
        s += e(ia, jb);
        if (ni == 2) s += e(ib, jb);
    }
    u[idx] = static_cast<S>(cvt<C>(u[idx]) + pf * (wi * wj) * s);
}

template <typename S, typename C>
__global__ void __launch_bounds__(256)
k_prolong3d(const S* __restrict__ ec, S* __restrict__ u, int n, int nc, C pf) {
    const long vol = (long)n * n * n;
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= vol) return;
    u += (long)blockIdx.y * vol;
    ec += (long)blockIdx.y * nc * nc * nc;
    const int i = idx % n, j = (idx / n) % n, k = idx / ((long)n * n);
    int xi[2], yj[2], zk[2];
    const int ni = interp_idx(i, nc, &xi[0], &xi[1]);
    const int nj = interp_idx(j, nc, &yj[0], &yj[1]);
    const int nk = interp_idx(k, nc, &zk[0], &zk[1]);
    const C w = (ni == 1 ? C(1) : C(0.5)) * (nj == 1 ? C(1) : C(0.5)) *
                (nk == 1 ? C(1) : C(0.5));
    C s = C(0);
    for (int c = 0; c < nk; ++c)
        for (int bq = 0; bq < nj; ++bq)
            for (int a = 0; a < ni; ++a)
                if (xi[a] >= 0 && yj[bq] >= 0 && zk[c] >= 0)
                    s += cvt<C>(ec[((long)zk[c] * nc + yj[bq]) * nc + xi[a]]);
    u[idx] = static_cast<S>(cvt<C>(u[idx]) + pf * w * s);
}

// ---------------------------------------------------------------------------
// Coarse tail: every level from nt interior nodes per direction down to 3,
// the exact solve on the 3^d grid and back up, in one workgroup with all
// level arrays in LDS.  Coarse levels start from a zero guess (pre-smoothing
// is e = sW K b).
// ---------------------------------------------------------------------------
template <typename C>
struct TailLevel {
    C* e;
    C* b;
    C* r;
    int n;
    C sA, sW;
};

template <typename C>
__device__ __forceinline__ C tget(const C* a, int d, int n, int i, int j, int k) {
    if (i < 0 || i >= n || j < 0 || j >= n) return C(0);
    if (d == 3) {
        if (k < 0 || k >= n) return C(0);
        return a[(k * n + j) * n + i];
    }
    return a[j * n + i];
}

template <typename C>
__device__ __forceinline__ void tdecode(int p, int d, int n, int* i, int* j, int* k) {
    *i = p % n;
    *j = (p / n) % n;
    *k = d == 3 ? p / (n * n) : 0;
}

template <typename C>
__device__ __forceinline__ C tlap(const C* a, int d, int n, int i, int j, int k) {
    C s = C(2 * d) * tget(a, d, n, i, j, k) - tget(a, d, n, i - 1, j, k) -
          tget(a, d, n, i + 1, j, k) - tget(a, d, n, i, j - 1, k) - tget(a, d, n, i, j + 1, k);
    if (d == 3) s -= tget(a, d, n, i, j, k - 1) + tget(a, d, n, i, j, k + 1);
    return s;
}

template <typename C>
__device__ __forceinline__ C tspai(const C* a, int d, int n, int i, int j, int k, C c0,
                                   C c1, C c2) {
    C f = tget(a, d, n, i - 1, j, k) + tget(a, d, n, i + 1, j, k) +
          tget(a, d, n, i, j - 1, k) + tget(a, d, n, i, j + 1, k);
    C v = c0 * tget(a, d, n, i, j, k);
    if (d == 3) {
        f += tget(a, d, n, i, j, k - 1) + tget(a, d, n, i, j, k + 1);
        return v + c1 * f;
    }
    const C cn = tget(a, d, n, i - 1, j - 1, k) + tget(a, d, n, i + 1, j - 1, k) +
                 tget(a, d, n, i - 1, j + 1, k) + tget(a, d, n, i + 1, j + 1, k);
    return v + c1 * f + c2 * cn;
}

template <typename S, typename C>
__global__ void __launch_bounds__(1024)
k_tail(const S* __restrict__ bt, S* __restrict__ et, int d, int nt, C c0, C c1, C c2,
       const double* __restrict__ ginv, int scaled, int Ntop) {
    extern __shared__ unsigned char smem_raw[];
    C* sm = reinterpret_cast<C*>(smem_raw);
    constexpr int NT = 1024;
    const int t = threadIdx.x;
    TailLevel<C> lv[8];
    int L = 0;
    {
        int n = nt, N = Ntop;
        C* p = sm;
        while (true) {
            long pts = 1;
            for (int a = 0; a < d; ++a) pts *= n;
            lv[L].e = p;
            lv[L].b = p + pts;
            lv[L].r = p + 2 * pts;
            lv[L].n = n;
            if (scaled) {
                lv[L].sA = C(1);
                lv[L].sW = C(1);
            } else {
                lv[L].sA = C((double)N * (double)N);
                lv[L].sW = C(1.0 / ((double)N * (double)N));
            }
            p += 3 * pts;
            ++L;
            if (n == 3) break;
            n = (n + 1) / 2 - 1;
            N /= 2;
        }
    }
    const C pf = scaled ? C(4) : C(1);
    auto npts = [&](int n) { return d == 3 ? n * n * n : n * n; };
    {
        const long off = (long)blockIdx.x * npts(nt);
        for (int p = t; p < npts(nt); p += NT) lv[0].b[p] = cvt<C>(bt[off + p]);
    }
    __syncthreads();
    for (int l = 0; l + 1 < L; ++l) {
        TailLevel<C>& A = lv[l];
        TailLevel<C>& B = lv[l + 1];
        const int n = A.n, m = npts(n);
        for (int p = t; p < m; p += NT) {
            int i, j, k;
            tdecode<C>(p, d, n, &i, &j, &k);
            A.e[p] = A.sW * tspai(A.b, d, n, i, j, k, c0, c1, c2);
        }
        __syncthreads();
        for (int p = t; p < m; p += NT) {
            int i, j, k;
            tdecode<C>(p, d, n, &i, &j, &k);
            A.r[p] = A.b[p] - A.sA * tlap(A.e, d, n, i, j, k);
        }
        __syncthreads();
        const int nc = B.n, mc = npts(nc);
        for (int p = t; p < mc; p += NT) {
            int i, j, k;
            tdecode<C>(p, d, nc, &i, &j, &k);
            const int fi = 2 * i + 1, fj = 2 * j + 1, fk = 2 * k + 1;
            C s = C(0);
            const int kl = d == 3 ? -1 : 0, kh = d == 3 ? 1 : 0;
            for (int oz = kl; oz <= kh; ++oz)
                for (int oy = -1; oy <= 1; ++oy)
                    for (int ox = -1; ox <= 1; ++ox) {
                        C w = (ox == 0 ? C(0.5) : C(0.25)) * (oy == 0 ? C(0.5) : C(0.25));
                        if (d == 3) w *= (oz == 0 ? C(0.5) : C(0.25));
                        s += w * tget(A.r, d, n, fi + ox, fj + oy, d == 3 ? fk + oz : 0);
                    }
            B.b[p] = s;
        }
        __syncthreads();
    }
    {
        TailLevel<C>& Z = lv[L - 1];
        const int m = npts(3);
        for (int p = t; p < m; p += NT) {
            double s = 0.0;
            for (int q = 0; q < m; ++q) s += ginv[p * m + q] * (double)Z.b[q];
            Z.e[p] = C(s);
        }
        __syncthreads();
    }
    for (int l = L - 2; l >= 0; --l) {
        TailLevel<C>& A = lv[l];
        TailLevel<C>& B = lv[l + 1];
        const int n = A.n, m = npts(n), nc = B.n;
        for (int p = t; p < m; p += NT) {
            int i, j, k;
            tdecode<C>(p, d, n, &i, &j, &k);
            int xi[2], yj[2], zk[2] = {0, -1};
            const int ni = interp_idx(i, nc, &xi[0], &xi[1]);
            const int nj = interp_idx(j, nc, &yj[0], &yj[1]);
            int nk = 1;
            if (d == 3) nk = interp_idx(k, nc, &zk[0], &zk[1]);
            C w = (ni == 1 ? C(1) : C(0.5)) * (nj == 1 ? C(1) : C(0.5));
            if (d == 3) w *= (nk == 1 ? C(1) : C(0.5));
            C s = C(0);
            for (int c = 0; c < nk; ++c)
                for (int bq = 0; bq < nj; ++bq)
                    for (int a = 0; a < ni; ++a)
                        if (xi[a] >= 0 && yj[bq] >= 0 && zk[c] >= 0)
                            s += B.e[d == 3 ? (zk[c] * nc + yj[bq]) * nc + xi[a]
                                            : yj[bq] * nc + xi[a]];
            A.e[p] += pf * w * s;
        }
        __syncthreads();
        for (int p = t; p < m; p += NT) {
            int i, j, k;
            tdecode<C>(p, d, n, &i, &j, &k);
            A.r[p] = A.b[p] - A.sA * tlap(A.e, d, n, i, j, k);
        }
        __syncthreads();
        for (int p = t; p < m; p += NT) {
            int i, j, k;
            tdecode<C>(p, d, n, &i, &j, &k);
            A.e[p] += A.sW * tspai(A.r, d, n, i, j, k, c0, c1, c2);
        }
        __syncthreads();
    }
    {
        const long off = (long)blockIdx.x * npts(nt);
        for (int p = t; p < npts(nt); p += NT) et[off + p] = static_cast<S>(lv[0].e[p]);
    }
}

// ---------------------------------------------------------------------------
// Norm finalisation in a fixed order (deterministic run to run).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_finalize(const double* __restrict__ ps, const double* __restrict__ pm, int count,
           double* __restrict__ out) {
    __shared__ double red[4];
    double s = 0.0, mx = 0.0;
    for (int i = threadIdx.x; i < count; i += 256) {
        s += ps[i];
        if (pm) mx = fmax(mx, pm[i]);
    }
    const double tot = block_sum<256>(s, red);
    __syncthreads();
    const double tmx = block_max<256>(mx, red);
    if (threadIdx.x == 0) {
        out[0] = sqrt(tot);
        if (pm) out[1] = tmx;
    }
}

// ---------------------------------------------------------------------------
// FP64 refinement step, 3D: unew = u + escale * e (on the fly, halo included),
// r = b - A unew, r_lo = s * r (stored in S), partials of r^2 and max |r|.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double ir_scale(const double* maxprev) {
    const double m = maxprev[0];
    if (!(m > 0.0) || !isfinite(m)) return 1.0;
    int e;
    frexp(m, &e);           // m = f 2^e with f in [0.5, 1)
    return ldexp(1.0, -e);  // s m in [0.5, 1)
}

template <typename S, int TX, int TY>
__global__ void __launch_bounds__(TX * TY)
k_ir3d(const double* __restrict__ u, double* __restrict__ unew, const S* __restrict__ e,
       const double* __restrict__ b, S* __restrict__ rlo, int n, int tiles_x, int tiles_y,
       int zchunk, int nchunks, double inv_h2, double sigma0, int k,
       double* __restrict__ scales, const double* __restrict__ maxprev,
       double* __restrict__ psum, double* __restrict__ pmax) {
    constexpr int NT = TX * TY;
    constexpr int RX = TX + 2, RY = TY + 2, NR = RX * RY;
    constexpr int M = (NR + NT - 1) / NT;
    __shared__ double uL[2][NR];
    __shared__ double red[NT / 64];
    const int total = tiles_x * tiles_y * nchunks;
    const int lg = xcd_remap(blockIdx.x, total);
    const int tx = lg % tiles_x, ty = (lg / tiles_x) % tiles_y,
              ch = lg / (tiles_x * tiles_y);
    const long plane = (long)n * n, boff = (long)blockIdx.y * plane * n;
    u += boff;
    unew += boff;
    b += boff;
    rlo += boff;
    if (e) e += boff;
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = ch * zchunk, z1 = min(z0 + zchunk, n);
    const int t = threadIdx.x;
    const double s_new = ir_scale(maxprev);
    if (blockIdx.x == 0 && blockIdx.y == 0 && t == 0) scales[k] = s_new;
    const double escale = (e && k > 0) ? 1.0 / (sigma0 * scales[k - 1]) : 0.0;

    int go[M];
    bool inr[M], val[M], inn[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = t + m * NT;
        inr[m] = i < NR;
        const int lx = i % RX, ly = i / RX;
        const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        val[m] = inr[m] && gx >= 0 && gx < n && gy >= 0 && gy < n;
        inn[m] = val[m] && lx >= 1 && lx <= TX && ly >= 1 && ly <= TY;
        go[m] = val[m] ? gy * n + gx : 0;
    }
    auto ldU = [&](int p, int m) -> double {
        if (!val[m] || p < 0 || p >= n) return 0.0;
        const long g = p * plane + go[m];
        double v = u[g];
        if (e && k > 0) v += escale * (double)e[g];
        return v;
    };
    double um1[M], u0[M], up1[M], nu[M];
    double acc = 0.0, mx = 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        um1[m] = ldU(z0 - 1, m);
        u0[m] = ldU(z0, m);
        up1[m] = ldU(z0 + 1, m);
        if (inr[m]) uL[z0 & 1][t + m * NT] = u0[m];
    }
    for (int s = z0; s < z1; ++s) {
        __syncthreads();
        const int cur = s & 1;
#pragma unroll
        for (int m = 0; m < M; ++m) nu[m] = ldU(s + 2, m);
        const double* U = uL[cur];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            if (!inn[m]) continue;
            const int q = t + m * NT;
            const long g = s * plane + go[m];
            const double lap = 6.0 * u0[m] - U[q - 1] - U[q + 1] - U[q - RX] - U[q + RX] -
                               um1[m] - up1[m];
            const double r = b[g] - inv_h2 * lap;
            unew[g] = u0[m];
            rlo[g] = static_cast<S>(s_new * r);
            acc += r * r;
            mx = fmax(mx, fabs(r));
        }
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (inr[m]) uL[cur ^ 1][t + m * NT] = up1[m];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            um1[m] = u0[m];
            u0[m] = up1[m];
            up1[m] = nu[m];
        }
    }
    const double ts = block_sum<NT>(acc, red);
    __syncthreads();
    const double tm = block_max<NT>(mx, red);
    if (t == 0) {
        const long pi = (long)blockIdx.y * gridDim.x + blockIdx.x;
        psum[pi] = ts;
        pmax[pi] = tm;
    }
}

template <typename S, int TX>
__global__ void __launch_bounds__(TX)
k_ir2d(const double* __restrict__ u, double* __restrict__ unew, const S* __restrict__ e,
       const double* __restrict__ b, S* __restrict__ rlo, int n, int tiles_x, int ychunk,
       int nchunks, double inv_h2, double sigma0, int k, double* __restrict__ scales,
       const double* __restrict__ maxprev, double* __restrict__ psum,
       double* __restrict__ pmax) {
    constexpr int NT = TX, RX = TX + 2;
    constexpr int M = (RX + NT - 1) / NT;
    __shared__ double uL[2][RX];
    __shared__ double red[NT / 64];
    const int total = tiles_x * nchunks;
    const int lg = xcd_remap(blockIdx.x, total);
    const int tx = lg % tiles_x, ch = lg / tiles_x;
    const long area = (long)n * n, boff = (long)blockIdx.y * area;
    u += boff;
    unew += boff;
    b += boff;
    rlo += boff;
    if (e) e += boff;
    const int x0 = tx * TX;
    const int y0 = ch * ychunk, y1 = min(y0 + ychunk, n);
    const int t = threadIdx.x;
    const double s_new = ir_scale(maxprev);
    if (blockIdx.x == 0 && blockIdx.y == 0 && t == 0) scales[k] = s_new;
    const double escale = (e && k > 0) ? 1.0 / (sigma0 * scales[k - 1]) : 0.0;
    int go[M];
    bool inr[M], val[M], inn[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = t + m * NT;
        inr[m] = i < RX;
        const int gx = x0 - 1 + i;
        val[m] = inr[m] && gx >= 0 && gx < n;
        inn[m] = val[m] && i >= 1 && i <= TX;
        go[m] = val[m] ? gx : 0;
    }
    auto ldU = [&](int p, int m) -> double {
        if (!val[m] || p < 0 || p >= n) return 0.0;
        const long g = (long)p * n + go[m];
        double v = u[g];
        if (e && k > 0) v += escale * (double)e[g];
        return v;
    };
    double um1[M], u0[M], up1[M], nu[M];
    double acc = 0.0, mx = 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        um1[m] = ldU(y0 - 1, m);
        u0[m] = ldU(y0, m);
        up1[m] = ldU(y0 + 1, m);
        if (inr[m]) uL[y0 & 1][t + m * NT] = u0[m];
    }
    for (int s = y0; s < y1; ++s) {
        __syncthreads();
        const int cur = s & 1;
#pragma unroll
        for (int m = 0; m < M; ++m) nu[m] = ldU(s + 2, m);
        const double* U = uL[cur];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            if (!inn[m]) continue;
            const int q = t + m * NT;
            const long g = (long)s * n + go[m];
            const double lap = 4.0 * u0[m] - U[q - 1] - U[q + 1] - um1[m] - up1[m];
            const double r = b[g] - inv_h2 * lap;
            unew[g] = u0[m];
            rlo[g] = static_cast<S>(s_new * r);
            acc += r * r;
            mx = fmax(mx, fabs(r));
        }
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (inr[m]) uL[cur ^ 1][t + m * NT] = up1[m];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            um1[m] = u0[m];
            u0[m] = up1[m];
            up1[m] = nu[m];
        }
    }
    const double ts = block_sum<NT>(acc, red);
    __syncthreads();
    const double tm = block_max<NT>(mx, red);
    if (t == 0) {
        const long pi = (long)blockIdx.y * gridDim.x + blockIdx.x;
        psum[pi] = ts;
        pmax[pi] = tm;
    }
}


// ---------------------------------------------------------------------------
// FP64 residual norm of the fine grid: per-block sum of r^2 and max |r|.
// One node per thread; neighbours come through L1/L2 (used once per solve).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_residual_norm(const double* __restrict__ u, const double* __restrict__ b, int d, int n,
                double inv_h2, double* __restrict__ psum, double* __restrict__ pmax) {
    __shared__ double red[4];
    const long pts = d == 3 ? (long)n * n * n : (long)n * n;
    const long off = (long)blockIdx.y * pts;
    u += off;
    b += off;
    double rr = 0.0, mx = 0.0;
    const long sy = n, sz = (long)n * n;
    for (long idx = (long)blockIdx.x * 256 + threadIdx.x; idx < pts;
         idx += (long)gridDim.x * 256) {
        const int i = idx % n, j = (idx / n) % n;
        const int k = d == 3 ? (int)(idx / ((long)n * n)) : 0;
        double lap = 2.0 * d * u[idx];
        if (i > 0) lap -= u[idx - 1];
        if (i < n - 1) lap -= u[idx + 1];
        if (j > 0) lap -= u[idx - sy];
        if (j < n - 1) lap -= u[idx + sy];
        if (d == 3) {
            if (k > 0) lap -= u[idx - sz];
            if (k < n - 1) lap -= u[idx + sz];
        }
        const double r = b[idx] - inv_h2 * lap;
        rr += r * r;
        mx = fmax(mx, fabs(r));
    }
    const double ts = block_sum<256>(rr, red);
    __syncthreads();
    const double tm = block_max<256>(mx, red);
    if (threadIdx.x == 0) {
        const long pi = (long)blockIdx.y * gridDim.x + blockIdx.x;
        psum[pi] = ts;
        pmax[pi] = tm;
    }
}

// ---------------------------------------------------------------------------
// Launch geometry
// ---------------------------------------------------------------------------
inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// chunk length along the marching direction so that the launch has at least
// `want` workgroups per batch entry, and no chunk shorter than `minc`
inline int pick_chunk(int n, int tiles, int want, int minc) {
    int nch = cdiv(want, tiles);
    int ch = cdiv(n, nch);
    if (ch < minc) ch = minc;
    if (ch > n) ch = n;
    return ch;
}

constexpr int S3_TX = 64, S3_TY = 16, S3_NT = 256;
constexpr int S2_TX = 256, S2_NT = 256;
constexpr int R3_TX = 32, R3_TY = 8;
constexpr int R2_TX = 256;
constexpr int I3_TX = 64, I3_TY = 4;
constexpr int I2_TX = 256;
constexpr int kWantBlocks = 1024;

template <typename S, typename C>
hipError_t smooth_impl(bool zg, bool norm, const Sweep& s, hipStream_t st, int* nparts) {
    const int n = s.n;
    const S* u = static_cast<const S*>(s.u);
    const S* b = static_cast<const S*>(s.b);
    S* out = static_cast<S*>(s.out);
    const C sA = C(s.sA), sW = C(s.sW), c0 = C(s.c[0]), c1 = C(s.c[1]), c2 = C(s.c[2]);
    if (s.d == 3) {
        const int tx = cdiv(n, S3_TX), ty = cdiv(n, S3_TY);
        const int zc = pick_chunk(n, tx * ty, kWantBlocks, 8);
        const int nch = cdiv(n, zc);
        dim3 grid(tx * ty * nch, s.batch);
        if (nparts) *nparts = grid.x * grid.y;
        if (norm && (long)grid.x * grid.y > s.partials_cap) return hipErrorInvalidValue;
#define L3(ZG, NM)                                                                  \
    hipLaunchKernelGGL((k_smooth3d<S, C, S3_TX, S3_TY, S3_NT, ZG, NM>), grid,      \
                       dim3(S3_NT), 0, st, u, b, out, n, tx, ty, zc, nch, sA, sW, c0, \
                       c1, s.partials)
        if (zg) L3(true, false);
        else if (norm) L3(false, true);
        else L3(false, false);
#undef L3
    } else {
        const int tx = cdiv(n, S2_TX);
        const int yc = pick_chunk(n, tx, kWantBlocks, 16);
        const int nch = cdiv(n, yc);
        dim3 grid(tx * nch, s.batch);
        if (nparts) *nparts = grid.x * grid.y;
        if (norm && (long)grid.x * grid.y > s.partials_cap) return hipErrorInvalidValue;
#define L2(ZG, NM)                                                                  \
    hipLaunchKernelGGL((k_smooth2d<S, C, S2_TX, S2_NT, ZG, NM>), grid, dim3(S2_NT), \
                       0, st, u, b, out, n, tx, yc, nch, sA, sW, c0, c1, c2, s.partials)
        if (zg) L2(true, false);
        else if (norm) L2(false, true);
        else L2(false, false);
#undef L2
    }
    return hipGetLastError();
}

template <typename S, typename C>
hipError_t restrict_impl(const Sweep& s, hipStream_t st) {
    const int n = s.n, nc = (n + 1) / 2 - 1;
    const S* u = static_cast<const S*>(s.u);
    const S* b = static_cast<const S*>(s.b);
    S* bc = static_cast<S*>(s.out);
    const C sA = C(s.sA);
    if (s.d == 3) {
        const int tx = cdiv(nc, R3_TX), ty = cdiv(nc, R3_TY);
        const int zc = pick_chunk(nc, tx * ty, kWantBlocks, 4);
        const int nch = cdiv(nc, zc);
        dim3 grid(tx * ty * nch, s.batch);
        hipLaunchKernelGGL((k_restrict3d<S, C, R3_TX, R3_TY>), grid, dim3(R3_TX * R3_TY), 0,
                           st, u, b, bc, n, nc, tx, ty, zc, nch, sA);
    } else {
        const int tx = cdiv(nc, R2_TX);
        const int yc = pick_chunk(nc, tx, kWantBlocks, 8);
        const int nch = cdiv(nc, yc);
        dim3 grid(tx * nch, s.batch);
        hipLaunchKernelGGL((k_restrict2d<S, C, R2_TX>), grid, dim3(R2_TX), 0, st, u, b, bc,
                           n, nc, tx, yc, nch, sA);
    }
    return hipGetLastError();
}

template <typename S, typename C>
hipError_t prolong_impl(int d, int n, int batch, const void* ec, void* u, double pf,
                        hipStream_t st) {
    const int nc = (n + 1) / 2 - 1;
    const long pts = d == 3 ? (long)n * n * n : (long)n * n;
    dim3 grid(cdiv(pts, 256), batch);
    if (d == 3)
        hipLaunchKernelGGL((k_prolong3d<S, C>), grid, dim3(256), 0, st,
                           static_cast<const S*>(ec), static_cast<S*>(u), n, nc, C(pf));
    else
        hipLaunchKernelGGL((k_prolong2d<S, C>), grid, dim3(256), 0, st,
                           static_cast<const S*>(ec), static_cast<S*>(u), n, nc, C(pf));
    return hipGetLastError();
}

template <typename S, typename C>
hipError_t tail_impl(const Tail& t, hipStream_t st) {
    const size_t lds = tail_lds_bytes(sizeof(C) == 8 ? P64 : P32, t.d, t.nt);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_tail<S, C>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((k_tail<S, C>), dim3(t.batch), dim3(1024), lds, st,
                       static_cast<const S*>(t.b), static_cast<S*>(t.e), t.d, t.nt,
                       C(t.c[0]), C(t.c[1]), C(t.c[2]), t.ginv, t.scaled ? 1 : 0, t.N_top);
    return hipGetLastError();
}

template <typename S>
hipError_t ir_impl(const IRStep& s, hipStream_t st, int* nparts) {
    const int n = s.n;
    const S* e = static_cast<const S*>(s.e_lo);
    S* rlo = static_cast<S*>(s.r_lo);
    if (s.d == 3) {
        const int tx = cdiv(n, I3_TX), ty = cdiv(n, I3_TY);
        const int zc = pick_chunk(n, tx * ty, kWantBlocks, 8);
        const int nch = cdiv(n, zc);
        dim3 grid(tx * ty * nch, s.batch);
        if (nparts) *nparts = grid.x * grid.y;
        if ((long)grid.x * grid.y > s.partials_cap) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_ir3d<S, I3_TX, I3_TY>), grid, dim3(I3_TX * I3_TY), 0, st, s.u,
                           s.unew, e, s.b, rlo, n, tx, ty, zc, nch, s.inv_h2, s.sigma0, s.k,
                           s.scales, s.maxprev, s.psum, s.pmax);
    } else {
        const int tx = cdiv(n, I2_TX);
        const int yc = pick_chunk(n, tx, kWantBlocks, 16);
        const int nch = cdiv(n, yc);
        dim3 grid(tx * nch, s.batch);
        if (nparts) *nparts = grid.x * grid.y;
        if ((long)grid.x * grid.y > s.partials_cap) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_ir2d<S, I2_TX>), grid, dim3(I2_TX), 0, st, s.u, s.unew, e, s.b,
                           rlo, n, tx, yc, nch, s.inv_h2, s.sigma0, s.k, s.scales, s.maxprev,
                           s.psum, s.pmax);
    }
    return hipGetLastError();
}

}  // namespace

size_t tail_lds_bytes(Prec p, int d, int nt) {
    long pts = 0;
    for (int n = nt;; n = (n + 1) / 2 - 1) {
        long q = 1;
        for (int a = 0; a < d; ++a) q *= n;
        pts += q;
        if (n <= 3) break;
    }
    return (size_t)(3 * pts) * (p == P64 ? 8 : 4);
}

hipError_t launch_smooth(Prec p, bool zg, bool norm, const Sweep& s, hipStream_t st,
                         int* nparts) {
    switch (p) {
        case P64: return smooth_impl<double, double>(zg, norm, s, st, nparts);
        case P32: return smooth_impl<float, float>(zg, false, s, st, nparts);
        default: return smooth_impl<_Float16, float>(zg, false, s, st, nparts);
    }
}

hipError_t launch_restrict(Prec p, const Sweep& s, hipStream_t st) {
    switch (p) {
        case P64: return restrict_impl<double, double>(s, st);
        case P32: return restrict_impl<float, float>(s, st);
        default: return restrict_impl<_Float16, float>(s, st);
    }
}

hipError_t launch_prolong(Prec p, int d, int n, int batch, const void* ec, void* u,
                          double pf, hipStream_t st) {
    switch (p) {
        case P64: return prolong_impl<double, double>(d, n, batch, ec, u, pf, st);
        case P32: return prolong_impl<float, float>(d, n, batch, ec, u, pf, st);
        default: return prolong_impl<_Float16, float>(d, n, batch, ec, u, pf, st);
    }
}

hipError_t launch_tail(Prec p, const Tail& t, hipStream_t st) {
    switch (p) {
        case P64: return tail_impl<double, double>(t, st);
        case P32: return tail_impl<float, float>(t, st);
        default: return tail_impl<_Float16, float>(t, st);
    }
}

hipError_t launch_finalize(const double* partials, const double* maxparts, int count,
                           double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, partials, maxparts, count, out);
    return hipGetLastError();
}

hipError_t launch_residual_norm(int d, int n, int batch, const double* u, const double* b,
                                double inv_h2, double* psum, double* pmax, long partials_cap,
                                hipStream_t st, int* nparts) {
    const long pts = d == 3 ? (long)n * n * n : (long)n * n;
    dim3 grid(std::min(cdiv(pts, 256), 4096), batch);
    if (nparts) *nparts = grid.x * grid.y;
    if ((long)grid.x * grid.y > partials_cap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_residual_norm, grid, dim3(256), 0, st, u, b, d, n, inv_h2, psum, pmax);
    return hipGetLastError();
}

hipError_t launch_ir_step(Prec p, const IRStep& s, hipStream_t st, int* nparts) {
    switch (p) {
        case P32: return ir_impl<float>(s, st, nparts);
        case P16: return ir_impl<_Float16>(s, st, nparts);
        default: return ir_impl<double>(s, st, nparts);
    }
}

}  // namespace spaimg
