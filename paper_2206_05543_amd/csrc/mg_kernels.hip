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
#include <hip/hip_ext.h>

#include <algorithm>

#include "mg_internal.h"

namespace spaimg {

LaunchEvents& launch_events() {
    static thread_local LaunchEvents ev;
    return ev;
}

namespace {

// Every kernel of this file is launched here: with the thread's pending
// event pair (launch_events) the launch records the kernel's own start and
// end in it, otherwise it is an ordinary launch.
template <typename K, typename... A>
void mg_launch(K kernel, dim3 grid, dim3 block, unsigned lds, hipStream_t st, A... args) {
    LaunchEvents& ev = launch_events();
    if (ev.start) {
        const LaunchEvents e = ev;
        ev = LaunchEvents();
        hipExtLaunchKernelGGL(kernel, grid, block, lds, st, e.start, e.stop, 0u, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
    }
}

constexpr int kXCD = 8;

// compile-time position of a step within the unrolled marching loops
template <int K>
struct Par {
    static constexpr int k = K;
};

// Runs f(s, Par<0>), f(s+1, Par<1>), ..., f(s+R-1, Par<R-1>) for s = first,
// first+R, ... while s <= last: the body of a marching loop unrolled R times,
// so that every prefetch slot index is a compile-time constant.  Groups are
// always run whole (the step function ignores steps past `last`): a loop
// with a single latch keeps the prefetch registers in place, where an exit
// in the middle of a group makes the compiler copy loads still in flight.
template <int R, int K = 0, typename F>
__device__ __forceinline__ void unroll_step(int s, F&& f) {
    if constexpr (K < R) {
        f(s + K, Par<K>());
        unroll_step<R, K + 1>(s, f);
    }
}
template <int R, typename F>
__device__ __forceinline__ void march(int first, int last, F&& f) {
    for (int s = first; s <= last; s += R) unroll_step<R>(s, f);
}

// Bijection from hardware workgroup order (round-robin over XCDs) to a
// logical tile order in which every XCD owns one contiguous range.
__device__ __forceinline__ int xcd_remap(int bid, int total) {
    const int per = total / kXCD, rem = total % kXCD;
    const int x = bid % kXCD, i = bid / kXCD;
    return x * per + min(x, rem) + i;
}

template <typename C, typename S>
__device__ __forceinline__ C cvt(S v) { return static_cast<C>(v); }

// Output stores of large grids are non-temporal: the field is consumed by a
// later kernel from HBM anyway, and keeping the write stream out of the
// caches lets the two read streams run at full rate (measured on MI355X: a
// 2-read/1-write stream goes from ~5.4 to ~7.0 TB/s).  Small grids, which
// the next kernel reads back from L2, use ordinary stores.
constexpr long kNtMinPts = 1L << 22;

template <typename S>
__device__ __forceinline__ void st_out(S* p, S v, bool nt) {
    if (nt) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// ---------------------------------------------------------------------------
// Raw buffer access.  The marching kernels read and write through buffer
// resources, one per field and workgroup, that cover the window of lines
// [first, first + count) (planes in 3D, rows in 2D) the workgroup's march
// touches.  A line is addressed by a 32-bit offset (one scalar multiply); a
// line outside the caller's range gets the offset kOobLine and a lane
// outside the grid the offset kOob.  kOobLine added to an in-line offset
// (below one line's bytes) or to kOob, and kOob added to an in-range line's
// offset, stay at or above num_records and below 2^32, so all of these read
// as zero and their stores are dropped by the hardware range check.  This
// replaces per-lane index clamps, 64-bit address arithmetic and exec-mask
// branches by one 32-bit offset per point, and a resource per line and
// field (a 64-bit address, two selects and the descriptor words) by one per
// field.  The host keeps count * line bytes <= kWinMax.
// ---------------------------------------------------------------------------
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr unsigned kOob = 0x80000000u;
constexpr int kRsrcWord3 = 0x00020000;  // raw (untyped) buffer, gfx9-family layout
typedef int int2v __attribute__((ext_vector_type(2)));

constexpr unsigned kOobLine = 0x7FF00000u;
constexpr long kWinMax = kOobLine;
template <typename S>
struct Win {
    rsrc_t r;
    int first;
    int lb;  // line bytes
    __device__ __forceinline__ Win(const S* base, long len, int first_, int count)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<S*>(base + (long)first_ * len), 0,
                                              count > 0 ? (int)(count * len * (long)sizeof(S)) : 0,
                                              kRsrcWord3)),
          first(first_), lb((int)(len * (long)sizeof(S))) {}
    // line p's offset; `in` must imply first <= p < first + count
    __device__ __forceinline__ unsigned at(int p, bool in) const {
        return in ? (unsigned)((p - first) * lb) : kOobLine;
    }
};

template <typename S>
__device__ __forceinline__ S bload(rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ double bload<double>(rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ float bload<float>(rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ __forceinline__ _Float16 bload<_Float16>(rsrc_t r, unsigned off) {
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
}
// NTS selects the non-temporal store (cache policy bit 1)
template <bool NTS>
__device__ __forceinline__ void bstore(double v, rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(int2v, v), r, off, 0, NTS ? 2 : 0);
}
template <bool NTS>
__device__ __forceinline__ void bstore(float v, rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, off, 0, NTS ? 2 : 0);
}
template <bool NTS>
__device__ __forceinline__ void bstore(_Float16 v, rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(short, v), r, off, 0, NTS ? 2 : 0);
}
template <bool B>
struct Bool {
    static constexpr bool value = B;
};

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

// The host mirror of a norm lives in coherent (fine-grained) pinned memory:
// a system-scope store reaches the host without a cache flush, and the host
// polls the slot for it instead of waiting for the stream.
__device__ __forceinline__ void store_host_norm(double* host, double v) {
    __hip_atomic_store(host, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Norm of a finished sweep from its per-block partials, in a fixed order
// (deterministic run to run): (sqrt(sum ps), max pm) to dev, sqrt(sum ps)
// to the pinned host mirror `host`.  Run by one whole workgroup of the
// kernel that follows the sweep, which saves a reduction launch and a copy.
template <int NT>
__device__ void finalize_norm(const double* ps, const double* pm, int count, double* dev,
                              double* host, double* red) {
    double s = 0.0, mx = 0.0;
    for (int i = threadIdx.x; i < count; i += NT) {
        s += ps[i];
        if (pm) mx = fmax(mx, pm[i]);
    }
    const double tot = block_sum<NT>(s, red);
    __syncthreads();
    const double tmx = block_max<NT>(mx, red);
    if (threadIdx.x == 0) {
        const double nrm = sqrt(tot);
        dev[0] = nrm;
        if (pm) dev[1] = tmx;
        if (host) store_host_norm(host, nrm);
    }
}

// ---------------------------------------------------------------------------
// Software pipeline of the marching kernels.  Global loads of the plane that
// will be consumed PD steps later are issued at the top of each step into
// raw storage-typed registers; they are converted (and combined with the
// fused coarse correction) only when the plane is consumed, so no arithmetic
// waits on a load in flight.
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// 3D fused residual + SPAI smoother:  out = v + sW * K_c (b - sA * L v)
// with v = u (PRO = false), v = 0 (ZG), or v = u + pf * P ec (PRO: the
// coarse-grid correction fused into the post-smoother).  K_c = c0 I +
// c1 (6 face neighbours); the residual is zero outside the grid.  Tile
// TX x TY outputs per plane; the residual is computed on the tile plus a
// ring of 1, which needs v on the tile plus a ring of 2 (without corners).
// Output lags the residual by one plane.  For PRO, the coarse plane under
// each even fine plane is staged once into an LDS tile, and every column
// keeps the bilinear value of the last coarse plane in a register, so the
// trilinear correction costs one coarse read per coarse node.
//
// Every lane executes the same instruction stream: global accesses go
// through the per-field plane windows (off-grid reads are zero, off-tile
// stores are dropped), LDS writes of lanes past the tile land in a scratch area,
// and the residual outside the grid is cleared with a select.
//
// WIDE: the 19-/27-point SPAI stencils (K_c + c2 x 12 edge neighbours + c3 x
// 8 corner neighbours), which need the in-plane neighbours of all three
// residual planes around an output plane: the residual planes live in a
// ring of four LDS slots and the output lags the residual by two planes, so
// every plane a step reads was written before that step's barrier.
// ---------------------------------------------------------------------------
template <typename S, typename C, int TX, int TY, int NT, int PD, int UN, bool ZG, bool NORM,
          bool PRO, bool NTS, bool WIDE = false, bool ROUT = false>
__global__ void __launch_bounds__(NT)
k_smooth3d(const S* __restrict__ u, const S* __restrict__ b, S* __restrict__ out,
           int n, int tiles_x, int tiles_y, int zchunk, int nchunks, C sA,
           C sW, C c0, C c1, double* __restrict__ partials,
           const S* __restrict__ ec, int nc, C pf, C c2 = C(0), C c3 = C(0),
           S* __restrict__ rout = nullptr) {
    constexpr int RX = TX + 2, RY = TY + 2, NR = RX * RY;
    constexpr int UX = TX + 4, UY = TY + 4, NU = UX * UY;
    constexpr int M = (NR + NT - 1) / NT;
    constexpr int NR2 = 2 * RX + 2 * RY;
    constexpr int CX = TX / 2 + 4, CY = TY / 2 + 4, NC = CX * CY;
    constexpr int MC = (NC + NT - 1) / NT;
    // residual planes: slot t + m * NT at offset RP, padded by RX + 1 on
    // both sides so that neighbour reads of every lane stay in bounds
    constexpr int RP = RX + 1, RSZ = RP + M * NT + RX + 1;
    // u planes: lanes past the tile write (and read around) UD + lane
    constexpr int UD = NU + UX, USZ = NU + 2 * UX + 65;
    static_assert(NR2 <= NT, "one thread per ring-2 point");
    static_assert(TX % 2 == 0 && TY % 2 == 0, "even tiles");
    __shared__ C uL[2][ZG ? 1 : USZ];
    __shared__ C rL[WIDE ? 4 : 2][RSZ];
    __shared__ C cL[PRO ? MC * NT : 1];
    __shared__ double red[NT / 64];

    const int total = tiles_x * tiles_y * nchunks;
    const int lg = xcd_remap(blockIdx.x, total);
    const int tx = lg % tiles_x, ty = (lg / tiles_x) % tiles_y,
              ch = lg / (tiles_x * tiles_y);
    const long plane = (long)n * n;
    const long boff = (long)blockIdx.y * plane * n;
    b += boff;
    out += boff;
    if (ROUT) rout += boff;
    if (!ZG) u += boff;
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = ch * zchunk, z1 = min(z0 + zchunk, n);
    const int t = threadIdx.x;
    const int lane = t & 63;

    int ul[M];
    unsigned gb[M];  // byte offset in the plane, kOob off the grid
    bool val[M], inn[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = t + m * NT;
        const bool inr = i < NR;
        const int lx = i % RX, ly = i / RX;
        const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        val[m] = inr && gx >= 0 && gx < n && gy >= 0 && gy < n;
        inn[m] = val[m] && lx >= 1 && lx <= TX && ly >= 1 && ly <= TY;
        ul[m] = inr ? (ly + 1) * UX + lx + 1 : UD + lane;
        gb[m] = val[m] ? (unsigned)((gy * n + gx) * (int)sizeof(S)) : kOob;
    }
    int r2l = UD + lane, r2x = 0, r2y = 0;
    unsigned r2b = kOob;
    const bool r2in = !ZG && t < NR2;
    if (r2in) {
        int ux, uy;
        if (t < RX) { ux = 1 + t; uy = 0; }
        else if (t < 2 * RX) { ux = 1 + t - RX; uy = UY - 1; }
        else if (t < 2 * RX + RY) { ux = 0; uy = 1 + t - 2 * RX; }
        else { ux = UX - 1; uy = 1 + t - 2 * RX - RY; }
        r2x = x0 - 2 + ux;
        r2y = y0 - 2 + uy;
        r2l = uy * UX + ux;
        if (r2x >= 0 && r2x < n && r2y >= 0 && r2y < n)
            r2b = (unsigned)((r2y * n + r2x) * (int)sizeof(S));
    }

    // ---- fused coarse correction (PRO): per lane, the LDS index of the
    // lower coarse neighbour plus two flags (second node in x, in y)
    const long cplane = (long)nc * nc;
    const int cx0 = x0 / 2 - 2, cy0 = y0 / 2 - 2;  // coarse tile origin
    int cc[M + 1];
    C qprev[M + 1];
    unsigned cgb[MC];
    // coarse planes are loaded CD even steps ahead into RCS register slots
    constexpr int RCS = UN / 2, CD = RCS >= 2 ? 2 : 1;
    S rc[RCS][MC];
    if (PRO) {
        ec += (long)blockIdx.y * cplane * nc;
        auto setup = [&](int k, bool ok, int gx, int gy) {
            const int g = gx + 1, h = gy + 1;  // grid coordinates
            const int lx = (g >> 1) - 1 - cx0, ly = (h >> 1) - 1 - cy0;
            cc[k] = ok ? (ly * CX + lx) | ((g & 1) << 16) | ((h & 1) << 17) : 0;
            qprev[k] = C(0);
        };
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int i = t + m * NT;
            setup(m, i < NR, x0 - 1 + i % RX, y0 - 1 + i / RX);
        }
        setup(M, r2in, r2x, r2y);
#pragma unroll
        for (int j = 0; j < MC; ++j) {
            const int i = t + j * NT;
            const int gx = cx0 + i % CX, gy = cy0 + i / CX;
            const bool ok = i < NC && gx >= 0 && gx < nc && gy >= 0 && gy < nc;
            cgb[j] = ok ? (unsigned)((gy * nc + gx) * (int)sizeof(S)) : kOob;
        }
    }
    // planes any output depends on: v up to z1 + 1, b up to z1, coarse
    // planes up to (z1 + 1) / 2 (later planes read as zero); one window of
    // fine planes z0 - 2 .. ulast serves every fine field
    const int ulast = min(n - 1, z1 + 1), blast = min(n - 1, z1);
    const int clast = min(nc - 1, z1 / 2 + 1), cf0 = max(0, z0 / 2 - 2);
    const int f0 = max(0, z0 - 2), fcnt = ulast - f0 + 1;
    const Win<S> wu(ZG ? b : u, plane, f0, fcnt), wb(b, plane, f0, fcnt);
    const Win<S> wo(out, plane, f0, fcnt), wro(ROUT ? rout : out, plane, f0, fcnt);
    const Win<S> wec(PRO ? ec : b, cplane, cf0, clast - cf0 + 1);
    auto c_issue = [&](int Z, int sl) {
        const unsigned o = wec.at(Z, Z >= 0 && Z <= clast);
#pragma unroll
        for (int j = 0; j < MC; ++j) rc[sl][j] = bload<S>(wec.r, o + cgb[j]);
    };
    auto c_write = [&](int sl) {
#pragma unroll
        for (int j = 0; j < MC; ++j) cL[t + j * NT] = cvt<C>(rc[sl][j]);
    };
    // bilinear value at lane k of a coarse plane staged in LDS at `base`:
    // the same sum order and weights as the explicit interpolation operator
    auto q_at = [&](const C* base, int k) -> C {
        const int i = cc[k] & 0xffff;
        const bool hx = cc[k] & 0x10000, hy = cc[k] & 0x20000;
        C q = base[i];
        q += hx ? base[i + 1] : C(0);
        q += hy ? base[i + CX] : C(0);
        q += (hx && hy) ? base[i + CX + 1] : C(0);
        return (hx ? C(0.5) : C(1)) * (hy ? C(0.5) : C(1)) * q;
    };

    // ---- prefetch ring: raw u (and ring-2 value) of plane p and raw b of
    // plane p live in slot (p - s0) % (PD + 1); written by the loads, read
    // once when consumed.  b is consumed PD steps after its load, u PD + 1.
    // The marching loop is unrolled UN times: a multiple of the ring length
    // and of the PRO parity keeps every slot index static, and a multiple of
    // 3 (the u/r plane rotation) leaves no register copies at the latch.
    constexpr int RS = PD + 1;
    constexpr int UR = UN;
    static_assert(UN % RS == 0 && UN % 2 == 0, "unroll covers the prefetch ring and parity");
    S ru[RS][M], rb[RS][M], rr2[RS];
    auto issue_u = [&](int p, int k) {
        const unsigned o = wu.at(p, p >= 0 && p <= ulast);
#pragma unroll
        for (int m = 0; m < M; ++m) ru[k][m] = bload<S>(wu.r, o + gb[m]);
        rr2[k] = bload<S>(wu.r, o + r2b);
    };
    auto issue_b = [&](int p, int k) {
        const unsigned o = wb.at(p, p >= 0 && p <= blast);
#pragma unroll
        for (int m = 0; m < M; ++m) rb[k][m] = bload<S>(wb.r, o + gb[m]);
    };
    // consume raw plane p: v = u + pf * P ec; qh holds the bilinear coarse
    // values of plane p/2 when p is even
    auto take_raw = [&](int p, const S* raw, S raw2, const C* qh, C* dst, C& rdst) {
#pragma unroll
        for (int m = 0; m < M + 1; ++m) {
            C v = cvt<C>(m < M ? raw[m] : raw2);
            if (PRO) {
                C pe;
                if ((p & 1) == 0) {
                    pe = C(0.5) * (qprev[m] + qh[m]);
                    qprev[m] = qh[m];
                } else {
                    pe = qprev[m];
                }
                v += pf * pe;
            }
            if (m < M) dst[m] = v; else rdst = v;
        }
    };
    auto take_u = [&](int p, int sl, const C* qh, C* dst, C& rdst) {
        take_raw(p, ru[sl], rr2[sl], qh, dst, rdst);
    };

    C um2[M], um1[M], u0[M], up1[M], rm2[M], rm1[M], r0[M];
    C ur0 = 0, urp1 = 0;
    double nacc = 0.0;
    const int s0 = z0 - 1;
    // prologue: every load is issued before the first wait.  v of planes
    // s0-1, s0, s0+1, b of plane s0 (and the next PD-1), and for PRO the
    // coarse planes (s0-1)/2 - 1 .. (s0+1)/2, staged in the residual LDS
    // (not in use before the loop) to interpolate the first three planes.
    static_assert(!PRO || 3 * MC * NT <= 2 * RSZ, "coarse staging fits the residual LDS");
    {
#pragma unroll
        for (int q = 0; q < PD; ++q) issue_b(s0 + q, q);
        S pu[3][M], pr2[3];
        if (!ZG) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int p = s0 - 1 + q;
                const unsigned o = wu.at(p, p >= 0 && p <= ulast);
#pragma unroll
                for (int m = 0; m < M; ++m) pu[q][m] = bload<S>(wu.r, o + gb[m]);
                pr2[q] = bload<S>(wu.r, o + r2b);
            }
        }
        C qs[3][M + 1];
        if (PRO) {
            const int Zb = (s0 - 1) / 2;  // s0 is odd
            S pc[3][MC];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int Z = Zb - 1 + q;
                const unsigned o = wec.at(Z, Z >= 0 && Z <= clast);
#pragma unroll
                for (int j = 0; j < MC; ++j) pc[q][j] = bload<S>(wec.r, o + cgb[j]);
            }
            C* cs = &rL[0][0];
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int j = 0; j < MC; ++j) cs[q * MC * NT + t + j * NT] = cvt<C>(pc[q][j]);
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int k = 0; k < M + 1; ++k) qs[q][k] = q_at(cs + q * MC * NT, k);
#pragma unroll
            for (int k = 0; k < M + 1; ++k) qprev[k] = qs[0][k];
        }
        if (!ZG) {
            C dummy;
            take_raw(s0 - 1, pu[0], pr2[0], qs[1], um1, dummy);
            take_raw(s0, pu[1], pr2[1], qs[1], u0, ur0);
            take_raw(s0 + 1, pu[2], pr2[2], qs[2], up1, urp1);
        }
#pragma unroll
        for (int m = 0; m < M; ++m) rm2[m] = rm1[m] = um2[m] = C(0);
        if (!ZG) {
#pragma unroll
            for (int q = 0; q < PD; ++q) issue_u(s0 + 2 + q, (2 + q) % RS);
        }
        // s0 is odd (the launch uses even chunks); coarse plane (s0+3)/2 + j
        // goes to the slot of the even step that would have issued it
        if (PRO) {
#pragma unroll
            for (int j = 0; j < CD; ++j)
                c_issue((s0 + 3) / 2 + j, (((1 + 2 * j - 2 * CD + 2 * UN) % UN) >> 1) % RCS);
        }
    }
    if (!ZG) {
        const int sl = (s0 + 2) & 1;
#pragma unroll
        for (int m = 0; m < M; ++m) uL[sl][ul[m]] = u0[m];
        uL[sl][r2l] = ur0;
    }

    auto step = [&](int s, auto kc) {
        constexpr int k = decltype(kc)::k;  // (s - s0) % UR
        __syncthreads();
        const int cur = (s + 2) & 1;
        // prefetch: v plane s+2+PD and b plane s+PD into the slots consumed
        // last step; coarse plane for PRO
        if (!ZG) issue_u(s + 2 + PD, (k + 1) % RS);
        issue_b(s + PD, (k + PD) % RS);
        // s even (s0 odd): coarse plane needed 2 CD steps later
        if (PRO && (k & 1) == 1) c_issue((s + 2 + 2 * CD) / 2, (k >> 1) % RCS);
        // residual of plane s on the tile plus ring 1
        const bool pin = s >= 0 && s < n;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            C r = cvt<C>(rb[k % RS][m]);
            if (!ZG) {
                const C* U = uL[cur];
                const int q = ul[m];
                const C lap = C(6) * u0[m] - U[q - 1] - U[q + 1] - U[q - UX] - U[q + UX] -
                              um1[m] - up1[m];
                r = (pin && val[m]) ? r - sA * lap : C(0);
            }
            r0[m] = r;
            rL[WIDE ? (s & 3) : cur][RP + t + m * NT] = r;
        }
        if constexpr (WIDE) {
            // smoothed plane s - 2 from residual planes s - 3, s - 2, s - 1
            const int p = s - 2;
            if (p >= z0 && p < z1) {
                const C* Rm = rL[(s - 3) & 3];
                const C* R0 = rL[(s - 2) & 3];
                const C* Rp = rL[(s - 1) & 3];
                const unsigned ro = wo.at(p, true);
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const int q = RP + t + m * NT;
                    const C rc0 = R0[q];
                    const C fc = R0[q - 1] + R0[q + 1] + R0[q - RX] + R0[q + RX] + Rm[q] + Rp[q];
                    const C ed = R0[q - RX - 1] + R0[q - RX + 1] + R0[q + RX - 1] +
                                 R0[q + RX + 1] + Rm[q - 1] + Rm[q + 1] + Rm[q - RX] +
                                 Rm[q + RX] + Rp[q - 1] + Rp[q + 1] + Rp[q - RX] + Rp[q + RX];
                    const C cn = Rm[q - RX - 1] + Rm[q - RX + 1] + Rm[q + RX - 1] +
                                 Rm[q + RX + 1] + Rp[q - RX - 1] + Rp[q - RX + 1] +
                                 Rp[q + RX - 1] + Rp[q + RX + 1];
                    const C v = (ZG ? C(0) : um2[m]) +
                                sW * (c0 * rc0 + c1 * fc + c2 * ed + c3 * cn);
                    bstore<NTS>(static_cast<S>(v), wo.r, ro + (inn[m] ? gb[m] : kOob));
                    if (ROUT)
                        bstore<false>(static_cast<S>(rc0), wro.r, ro + (inn[m] ? gb[m] : kOob));
                    if (NORM) nacc += inn[m] ? (double)rc0 * (double)rc0 : 0.0;
                }
            }
        } else {
            // smoothed plane s - 1
            const int p = s - 1;
            if (p >= z0 && p < z1) {
                const C* R = rL[cur ^ 1];
                const unsigned ro = wo.at(p, true);
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const int q = RP + t + m * NT;
                    const C rc0 = rm1[m];
                    const C nbs = R[q - 1] + R[q + 1] + R[q - RX] + R[q + RX] + rm2[m] + r0[m];
                    const C v = (ZG ? C(0) : um1[m]) + sW * (c0 * rc0 + c1 * nbs);
                    bstore<NTS>(static_cast<S>(v), wo.r, ro + (inn[m] ? gb[m] : kOob));
                    if (ROUT)
                        bstore<false>(static_cast<S>(rc0), wro.r, ro + (inn[m] ? gb[m] : kOob));
                    if (NORM) nacc += inn[m] ? (double)rc0 * (double)rc0 : 0.0;
                }
            }
        }
        // v of plane s + 1 into the other LDS slot
        if (!ZG) {
#pragma unroll
            for (int m = 0; m < M; ++m) uL[cur ^ 1][ul[m]] = up1[m];
            uL[cur ^ 1][r2l] = urp1;
        }
        // rotate: consume plane s+2 of v
        C qh[M + 1];
        if (PRO && (k & 1) == 1) {  // s even
#pragma unroll
            for (int j = 0; j < M + 1; ++j) qh[j] = q_at(cL, j);
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            if (WIDE) um2[m] = um1[m];
            um1[m] = u0[m];
            u0[m] = up1[m];
            rm2[m] = rm1[m];
            rm1[m] = r0[m];
        }
        if (!ZG) take_u(s + 2, (k + 2) % RS, qh, up1, urp1);
        // s odd: stage coarse plane (s+3)/2, loaded 2 CD - 1 steps ago
        if (PRO && (k & 1) == 0) c_write((((k - 2 * CD + 1 + UN) % UN) >> 1) % RCS);
    };
    // WIDE outputs lag one more plane: the last one, z1 - 1, at step z1 + 1
    march<UR>(s0, WIDE ? z1 + 1 : z1, step);
    if (NORM) {
        const double sm = block_sum<NT>(nacc, red);
        if (t == 0) partials[(long)blockIdx.y * gridDim.x + blockIdx.x] = sm;
    }
}

// ---------------------------------------------------------------------------
// 2D fused residual + SPAI smoother (9-point M), same scheme: x strips of TX
// outputs marching over rows.  The residual of row s is computed on the
// strip plus a ring of 1; output lags by two rows because the 9-point
// stencil needs the residual of rows p-1..p+1 at x-1..x+1 from LDS (4 row
// slots).  PRO stages the coarse row under each even fine row in LDS.  As in
// 3D, every lane runs the same instruction stream (per-field row windows,
// LDS scratch slots for lanes past the strip, selects for off-grid points).
// ---------------------------------------------------------------------------
template <typename S, typename C, int TX, int NT, int PD, int UN, bool ZG, bool NORM, bool PRO,
          bool NTS, bool ROUT = false>
__global__ void __launch_bounds__(NT)
k_smooth2d(const S* __restrict__ u, const S* __restrict__ b, S* __restrict__ out,
           int n, int tiles_x, int ychunk, int nchunks, C sA, C sW, C c0, C c1,
           C c2, double* __restrict__ partials, const S* __restrict__ ec, int nc, C pf,
           S* __restrict__ rout = nullptr) {
    constexpr int RX = TX + 2, UX = TX + 4;
    constexpr int M = (RX + NT - 1) / NT;
    constexpr int CX = TX / 2 + 4;
    constexpr int MC = (CX + NT - 1) / NT;
    // residual rows: slot t + m * NT at offset 1, one guard entry each side;
    // u rows: column x0 - 2 + j at j, lanes past the strip use UD + lane
    constexpr int RSZ = M * NT + 2;
    constexpr int UD = UX + 1, USZ = UD + 65;
    static_assert(TX % 2 == 0, "even strips");
    __shared__ C uL[2][ZG ? 1 : USZ];
    __shared__ C rL[4][RSZ];
    __shared__ C cL[PRO ? MC * NT : 1];
    __shared__ double red[NT / 64];

    const int total = tiles_x * nchunks;
    const int lg = xcd_remap(blockIdx.x, total);
    const int tx = lg % tiles_x, ch = lg / tiles_x;
    const long area = (long)n * n;
    const long boff = (long)blockIdx.y * area;
    b += boff;
    out += boff;
    if (ROUT) rout += boff;
    if (!ZG) u += boff;
    const int x0 = tx * TX;
    const int y0 = ch * ychunk, y1 = min(y0 + ychunk, n);
    const int t = threadIdx.x;
    const int lane = t & 63;

    int ul[M];
    unsigned gb[M];
    bool val[M], inn[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = t + m * NT;
        const bool inr = i < RX;
        const int gx = x0 - 1 + i;
        val[m] = inr && gx >= 0 && gx < n;
        inn[m] = val[m] && i >= 1 && i <= TX;
        ul[m] = inr ? i + 1 : UD + lane;
        gb[m] = val[m] ? (unsigned)(gx * (int)sizeof(S)) : kOob;
    }
    // ring-2 columns x0-2 (thread 0) and x0+TX+1 (thread 1)
    const bool r2in = !ZG && t < 2;
    const int r2x = (t == 0) ? x0 - 2 : x0 + TX + 1;
    const int r2l = r2in ? (t == 0 ? 0 : UX - 1) : UD + lane;
    const unsigned r2b =
        (r2in && r2x >= 0 && r2x < n) ? (unsigned)(r2x * (int)sizeof(S)) : kOob;

    // fused coarse correction: LDS index of the left coarse neighbour and a
    // flag for the second node
    const int cx0 = x0 / 2 - 2;
    int cc[M + 1];
    C qprev[M + 1];
    unsigned cgb[MC];
    // coarse planes are loaded CD even steps ahead into RCS register slots
    constexpr int RCS = UN / 2, CD = RCS >= 2 ? 2 : 1;
    S rc[RCS][MC];
    if (PRO) {
        ec += (long)blockIdx.y * nc * nc;
        auto setup = [&](int k, bool ok, int gx) {
            const int g = gx + 1;
            cc[k] = ok ? ((g >> 1) - 1 - cx0) | ((g & 1) << 16) : 0;
            qprev[k] = C(0);
        };
#pragma unroll
        for (int m = 0; m < M; ++m) setup(m, t + m * NT < RX, x0 - 1 + t + m * NT);
        setup(M, r2in, r2x);
#pragma unroll
        for (int j = 0; j < MC; ++j) {
            const int i = t + j * NT;
            const int gx = cx0 + i;
            cgb[j] = (i < CX && gx >= 0 && gx < nc) ? (unsigned)(gx * (int)sizeof(S)) : kOob;
        }
    }
    // rows any output depends on: v up to y1 + 1, b up to y1, coarse rows
    // up to (y1 + 1) / 2 (later rows read as zero); one window of fine rows
    // y0 - 2 .. ulast serves every fine field
    const int ulast = min(n - 1, y1 + 1), blast = min(n - 1, y1);
    const int clast = min(nc - 1, y1 / 2 + 1), cf0 = max(0, y0 / 2 - 2);
    const int f0 = max(0, y0 - 2), fcnt = ulast - f0 + 1;
    const Win<S> wu(ZG ? b : u, n, f0, fcnt), wb(b, n, f0, fcnt);
    const Win<S> wo(out, n, f0, fcnt), wro(ROUT ? rout : out, n, f0, fcnt);
    const Win<S> wec(PRO ? ec : b, nc, cf0, clast - cf0 + 1);
    auto c_issue = [&](int Y, int sl) {
        const unsigned o = wec.at(Y, Y >= 0 && Y <= clast);
#pragma unroll
        for (int j = 0; j < MC; ++j) rc[sl][j] = bload<S>(wec.r, o + cgb[j]);
    };
    auto c_write = [&](int sl) {
#pragma unroll
        for (int j = 0; j < MC; ++j) cL[t + j * NT] = cvt<C>(rc[sl][j]);
    };
    auto q_at = [&](const C* base, int k) -> C {
        const int i = cc[k] & 0xffff;
        const bool hx = cc[k] & 0x10000;
        C q = base[i];
        q += hx ? base[i + 1] : C(0);
        return (hx ? C(0.5) : C(1)) * q;
    };

    // prefetch ring, as in 3D: u of row p and b of row p in slot
    // (p - s0) % (PD + 1); b is consumed PD steps after its load.  Unrolled
    // UN times (a multiple of 4 matches the four-row rotation)
    constexpr int RS = PD + 1;
    constexpr int UR = UN;
    static_assert(UN % RS == 0 && UN % 2 == 0, "unroll covers the prefetch ring and parity");
    S ru[RS][M], rb[RS][M], rr2[RS];
    auto issue_u = [&](int p, int k) {
        const unsigned o = wu.at(p, p >= 0 && p <= ulast);
#pragma unroll
        for (int m = 0; m < M; ++m) ru[k][m] = bload<S>(wu.r, o + gb[m]);
        rr2[k] = bload<S>(wu.r, o + r2b);
    };
    auto issue_b = [&](int p, int k) {
        const unsigned o = wb.at(p, p >= 0 && p <= blast);
#pragma unroll
        for (int m = 0; m < M; ++m) rb[k][m] = bload<S>(wb.r, o + gb[m]);
    };
    auto take_raw = [&](int p, const S* raw, S raw2, const C* qh, C* dst, C& rdst) {
#pragma unroll
        for (int m = 0; m < M + 1; ++m) {
            C v = cvt<C>(m < M ? raw[m] : raw2);
            if (PRO) {
                C pe;
                if ((p & 1) == 0) {
                    pe = C(0.5) * (qprev[m] + qh[m]);
                    qprev[m] = qh[m];
                } else {
                    pe = qprev[m];
                }
                v += pf * pe;
            }
            if (m < M) dst[m] = v; else rdst = v;
        }
    };
    auto take_u = [&](int p, int sl, const C* qh, C* dst, C& rdst) {
        take_raw(p, ru[sl], rr2[sl], qh, dst, rdst);
    };

    C um2[M], um1[M], u0[M], up1[M];
    C ur0 = 0, urp1 = 0;
    double nacc = 0.0;
    const int s0 = y0 - 1;
    // prologue: all loads before the first wait (see the 3D kernel)
    static_assert(!PRO || 3 * MC <= 4 * M, "coarse staging fits the residual LDS");
    {
#pragma unroll
        for (int q = 0; q < PD; ++q) issue_b(s0 + q, q);
        S pu[3][M], pr2[3];
        if (!ZG) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int p = s0 - 1 + q;
                const unsigned o = wu.at(p, p >= 0 && p <= ulast);
#pragma unroll
                for (int m = 0; m < M; ++m) pu[q][m] = bload<S>(wu.r, o + gb[m]);
                pr2[q] = bload<S>(wu.r, o + r2b);
            }
        }
        C qs[3][M + 1];
        if (PRO) {
            const int Yb = (s0 - 1) / 2;  // s0 is odd
            S pc[3][MC];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int Y = Yb - 1 + q;
                const unsigned o = wec.at(Y, Y >= 0 && Y <= clast);
#pragma unroll
                for (int j = 0; j < MC; ++j) pc[q][j] = bload<S>(wec.r, o + cgb[j]);
            }
            C* cs = &rL[0][0];
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int j = 0; j < MC; ++j) cs[q * MC * NT + t + j * NT] = cvt<C>(pc[q][j]);
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int k = 0; k < M + 1; ++k) qs[q][k] = q_at(cs + q * MC * NT, k);
#pragma unroll
            for (int k = 0; k < M + 1; ++k) qprev[k] = qs[0][k];
        }
        if (!ZG) {
            C dummy;
            take_raw(s0 - 1, pu[0], pr2[0], qs[1], um1, dummy);
            take_raw(s0, pu[1], pr2[1], qs[1], u0, ur0);
            take_raw(s0 + 1, pu[2], pr2[2], qs[2], up1, urp1);
        }
#pragma unroll
        for (int m = 0; m < M; ++m) um2[m] = C(0);
        if (!ZG) {
#pragma unroll
            for (int q = 0; q < PD; ++q) issue_u(s0 + 2 + q, (2 + q) % RS);
        }
        // s0 is odd (the launch uses even chunks); coarse plane (s0+3)/2 + j
        // goes to the slot of the even step that would have issued it
        if (PRO) {
#pragma unroll
            for (int j = 0; j < CD; ++j)
                c_issue((s0 + 3) / 2 + j, (((1 + 2 * j - 2 * CD + 2 * UN) % UN) >> 1) % RCS);
        }
    }
    if (!ZG) {
        const int sl = (s0 + 2) & 1;
#pragma unroll
        for (int m = 0; m < M; ++m) uL[sl][ul[m]] = u0[m];
        uL[sl][r2l] = ur0;
    }

    auto step = [&](int s, auto kc) {
        constexpr int k = decltype(kc)::k;  // (s - s0) % UR
        __syncthreads();
        const int cur = (s + 2) & 1;
        const int rs = (s + 4) & 3;
        if (!ZG) issue_u(s + 2 + PD, (k + 1) % RS);
        issue_b(s + PD, (k + PD) % RS);
        // s even (s0 odd): coarse plane needed 2 CD steps later
        if (PRO && (k & 1) == 1) c_issue((s + 2 + 2 * CD) / 2, (k >> 1) % RCS);
        const bool pin = s >= 0 && s < n;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            C r = cvt<C>(rb[k % RS][m]);
            if (!ZG) {
                const C* U = uL[cur];
                const int q = ul[m];
                const C lap = C(4) * u0[m] - U[q - 1] - U[q + 1] - um1[m] - up1[m];
                r = (pin && val[m]) ? r - sA * lap : C(0);
            }
            rL[rs][1 + t + m * NT] = r;
        }
        const int p = s - 2;
        if (p >= y0 && p < y1) {
            const C* R0 = rL[(p + 3) & 3];  // row p - 1
            const C* R1 = rL[(p + 4) & 3];  // row p
            const C* R2 = rL[(p + 5) & 3];  // row p + 1
            const unsigned ro = wo.at(p, true);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int q = 1 + t + m * NT;
                const C rcc = R1[q];
                const C fc = R1[q - 1] + R1[q + 1] + R0[q] + R2[q];
                const C cn = R0[q - 1] + R0[q + 1] + R2[q - 1] + R2[q + 1];
                const C v = (ZG ? C(0) : um2[m]) + sW * (c0 * rcc + c1 * fc + c2 * cn);
                bstore<NTS>(static_cast<S>(v), wo.r, ro + (inn[m] ? gb[m] : kOob));
                if (ROUT)
                    bstore<false>(static_cast<S>(rcc), wro.r, ro + (inn[m] ? gb[m] : kOob));
                if (NORM) nacc += inn[m] ? (double)rcc * (double)rcc : 0.0;
            }
        }
        if (!ZG) {
#pragma unroll
            for (int m = 0; m < M; ++m) uL[cur ^ 1][ul[m]] = up1[m];
            uL[cur ^ 1][r2l] = urp1;
        }
        C qh[M + 1];
        if (PRO && (k & 1) == 1) {  // s even
#pragma unroll
            for (int j = 0; j < M + 1; ++j) qh[j] = q_at(cL, j);
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            um2[m] = um1[m];
            um1[m] = u0[m];
            u0[m] = up1[m];
        }
        if (!ZG) take_u(s + 2, (k + 2) % RS, qh, up1, urp1);
        // s odd: stage coarse plane (s+3)/2, loaded 2 CD - 1 steps ago
        if (PRO && (k & 1) == 0) c_write((((k - 2 * CD + 1 + UN) % UN) >> 1) % RCS);
    };
    march<UR>(s0, y1 + 1, step);
    if (NORM) {
        const double sm = block_sum<NT>(nacc, red);
        if (t == 0) partials[(long)blockIdx.y * gridDim.x + blockIdx.x] = sm;
    }
}

// ---------------------------------------------------------------------------
// 3D fused residual + full-weighting restriction: bc = R (b - sA L u).
// Coarse tile TXc x TYc; the fine residual is computed plane by plane on the
// (2TXc+1) x (2TYc+1) fine window (lanes own window points, NT chosen so
// that about two points per lane cover it) and reduced in xy by one thread
// per coarse column; the z weights (1/4, 1/2, 1/4) are accumulated in
// registers.  Same branch-free buffer addressing and prefetch ring as the
// smoothers.
// ---------------------------------------------------------------------------
template <typename S, typename C, int TXc, int TYc, int NT, int UN>
__global__ void __launch_bounds__(NT)
k_restrict3d(const S* __restrict__ u, const S* __restrict__ b, S* __restrict__ bc,
             int n, int nc, int tiles_x, int tiles_y, int zchunk, int nchunks, C sA,
             const double* __restrict__ fin_ps, const double* __restrict__ fin_pm, int fin_count,
             double* __restrict__ fin_dev, double* __restrict__ fin_host) {
    constexpr int FX = 2 * TXc + 1, FY = 2 * TYc + 1, NF = FX * FY;
    constexpr int UX = FX + 2, UY = FY + 2, NU = UX * UY;
    constexpr int M = (NF + NT - 1) / NT;
    constexpr int NR2 = 2 * FX + 2 * FY;
    constexpr int RP = FX + 1, RSZ = RP + M * NT + FX + 1;
    constexpr int UD = NU + UX, USZ = NU + 2 * UX + 65;
    constexpr int RS = 2;  // prefetch ring: one plane ahead
    static_assert(NR2 <= NT && TXc * TYc <= NT, "ring and coarse columns fit the workgroup");
    static_assert(UN % 2 == 0, "unroll covers the prefetch ring and the plane parity");
    __shared__ C uL[2][USZ];
    __shared__ C rL[2][RSZ];
    __shared__ double red[NT / 64];
    if (fin_count > 0 && blockIdx.x == 0 && blockIdx.y == 0)
        finalize_norm<NT>(fin_ps, fin_pm, fin_count, fin_dev, fin_host, red);

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
    const int lane = t & 63;

    int ul[M];
    unsigned gb[M];
    bool val[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = t + m * NT;
        const bool inr = i < NF;
        const int lx = i % FX, ly = i / FX;
        const int gx = fx0 + lx, gy = fy0 + ly;
        val[m] = inr && gx < n && gy < n;
        ul[m] = inr ? (ly + 1) * UX + lx + 1 : UD + lane;
        gb[m] = val[m] ? (unsigned)((gy * n + gx) * (int)sizeof(S)) : kOob;
    }
    int r2l = UD + lane;
    unsigned r2b = kOob;
    if (t < NR2) {
        int ux, uy;
        if (t < FX) { ux = 1 + t; uy = 0; }
        else if (t < 2 * FX) { ux = 1 + t - FX; uy = UY - 1; }
        else if (t < 2 * FX + FY) { ux = 0; uy = 1 + t - 2 * FX; }
        else { ux = UX - 1; uy = 1 + t - 2 * FX - FY; }
        const int gx = fx0 - 1 + ux, gy = fy0 - 1 + uy;
        r2l = uy * UX + ux;
        if (gx >= 0 && gx < n && gy >= 0 && gy < n) r2b = (unsigned)((gy * n + gx) * (int)sizeof(S));
    }
    // fine planes 2 Z0 - 1 .. 2 Z1 + 1 feed the residuals of planes 2 Z0 ..
    // 2 Z1 (later planes read as zero), in one window per field
    const int ulast = min(n - 1, 2 * Z1 + 1), blast = min(n - 1, 2 * Z1);
    const int w0 = max(0, 2 * Z0 - 1), wcnt = ulast - w0 + 1;
    const Win<S> wu(u, plane, w0, wcnt), wb(b, plane, w0, wcnt), wbc(bc, cplane, Z0, Z1 - Z0);
    S ru[RS][M], rb[RS][M], rr2[RS];
    auto issue_u = [&](int p, int k) {
        const unsigned o = wu.at(p, p >= 0 && p <= ulast);
#pragma unroll
        for (int m = 0; m < M; ++m) ru[k][m] = bload<S>(wu.r, o + gb[m]);
        rr2[k] = bload<S>(wu.r, o + r2b);
    };
    auto issue_b = [&](int p, int k) {
        const unsigned o = wb.at(p, p >= 0 && p <= blast);
#pragma unroll
        for (int m = 0; m < M; ++m) rb[k][m] = bload<S>(wb.r, o + gb[m]);
    };
    // coarse column of this thread and its window centre
    const int cx = t % TXc, cy = t / TXc;
    const bool cin = t < TXc * TYc;
    const unsigned cgb = (cin && cx0 + cx < nc && cy0 + cy < nc)
                             ? (unsigned)(((cy0 + cy) * nc + cx0 + cx) * (int)sizeof(S))
                             : kOob;
    const int cq = RP + (cin ? (2 * cy + 1) * FX + 2 * cx + 1 : FX + 1);

    C um1[M], u0[M], up1[M];
    C ur0 = 0, urp1 = 0, acc = 0;
    const int f0 = 2 * Z0, f1 = 2 * Z1;  // fine planes f0..f1 contribute
    {
        // all prologue loads before the first wait
        issue_b(f0, 0);
        S pu[3][M], pr2[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int p = f0 - 1 + q;
            const unsigned o = wu.at(p, p >= 0 && p <= ulast);
#pragma unroll
            for (int m = 0; m < M; ++m) pu[q][m] = bload<S>(wu.r, o + gb[m]);
            pr2[q] = bload<S>(wu.r, o + r2b);
        }
        C dummy;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            C* dst = q == 0 ? um1 : (q == 1 ? u0 : up1);
#pragma unroll
            for (int m = 0; m < M; ++m) dst[m] = cvt<C>(pu[q][m]);
            (q == 1 ? ur0 : (q == 2 ? urp1 : dummy)) = cvt<C>(pr2[q]);
        }
        issue_u(f0 + 2, 0);
        const int sl = f0 & 1;
#pragma unroll
        for (int m = 0; m < M; ++m) uL[sl][ul[m]] = u0[m];
        uL[sl][r2l] = ur0;
    }
    auto step = [&](int s, auto kc) {
        constexpr int k = decltype(kc)::k;  // (s - f0) % UN
        __syncthreads();
        const int cur = s & 1;
        issue_u(s + 3, (k + 1) % RS);
        issue_b(s + 1, (k + 1) % RS);
        // residual of fine plane s on the window
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const C* U = uL[cur];
            const int q = ul[m];
            const C lap = C(6) * u0[m] - U[q - 1] - U[q + 1] - U[q - UX] - U[q + UX] - um1[m] -
                          up1[m];
            const C r = cvt<C>(rb[k % RS][m]) - sA * lap;
            rL[cur][RP + t + m * NT] = val[m] ? r : C(0);
        }
        const int f = s - 1;  // fine plane whose residual is reduced now
        if (f >= f0 && f <= f1) {
            const C* R = rL[cur ^ 1];
            const int q = cq;
            const C xs = C(0.25) * R[q] +
                         C(0.125) * (R[q - 1] + R[q + 1] + R[q - FX] + R[q + FX]) +
                         C(0.0625) * (R[q - FX - 1] + R[q - FX + 1] + R[q + FX - 1] + R[q + FX + 1]);
            if ((k & 1) == 1) {  // f - f0 even
                if (f > f0) {
                    acc += C(0.25) * xs;
                    bstore<false>(static_cast<S>(acc), wbc.r, wbc.at(f / 2 - 1, true) + cgb);
                }
                acc = C(0.25) * xs;
            } else {
                acc += C(0.5) * xs;
            }
        }
#pragma unroll
        for (int m = 0; m < M; ++m) uL[cur ^ 1][ul[m]] = up1[m];
        uL[cur ^ 1][r2l] = urp1;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            um1[m] = u0[m];
            u0[m] = up1[m];
            up1[m] = cvt<C>(ru[k % RS][m]);
        }
        urp1 = cvt<C>(rr2[k % RS]);
    };
    march<UN>(f0, f1 + 1, step);
}

// ---------------------------------------------------------------------------
// 3D zero-guess pre-smoothing fused with the restriction: e = sW K_c b and
// bc = R (b - sA L e) in one march over fine planes, on the restriction's
// window (the (2 TXc + 1) x (2 TYc + 1) fine footprint of a coarse column
// tile).  L e there needs e on the footprint plus a ring of 1 without
// corners (the "e points"); e at those takes b on a ring of 2 in the plane
// (LDS, one plane per slot, three slots) and b one plane below and above
// (registers at the e points, a ring of four planes).  e is formed one plane
// ahead of the residual, b loaded three planes ahead; e is zero outside the
// grid and is written on the fine nodes the workgroup owns.  The unroll
// covers the register rings (4 and 2), the LDS ring (3) and the parity.
// ---------------------------------------------------------------------------
template <typename S, typename C, int TXc, int TYc, int NT, int UN>
__global__ void __launch_bounds__(NT)
k_zrestrict3d(const S* __restrict__ b, S* __restrict__ e, S* __restrict__ bc, int n, int nc,
              int tiles_x, int tiles_y, int zchunk, int nchunks, C sA, C sW, C c0, C c1,
              const double* __restrict__ fin_ps, const double* __restrict__ fin_pm,
              int fin_count, double* __restrict__ fin_dev, double* __restrict__ fin_host) {
    constexpr int FX = 2 * TXc + 1, FY = 2 * TYc + 1, NF = FX * FY;
    constexpr int UX = FX + 2, UY = FY + 2, NU = UX * UY;  // e window
    constexpr int BX = FX + 4, BY = FY + 4, NB = BX * BY;  // b window
    constexpr int M = (NF + NT - 1) / NT;
    constexpr int NR2 = 2 * FX + 2 * FY;  // ring-1 e points (no corners)
    constexpr int NX = NR2 + 4;           // b beyond the e points: ring 2, ring-1 corners
    constexpr int RP = FX + 1, RSZ = RP + M * NT + FX + 1;
    constexpr int UD = NU + UX, USZ = NU + 2 * UX + 65;
    constexpr int BD = NB + BX, BSZ = NB + 2 * BX + 65;
    static_assert(NX <= NT && TXc * TYc <= NT, "ring and coarse columns fit the workgroup");
    static_assert(UN % 12 == 0, "unroll covers the rings of 4, 3 and 2 planes");
    __shared__ C uL[2][USZ];
    __shared__ C bL[3][BSZ];
    __shared__ C rL[2][RSZ];
    __shared__ double red[NT / 64];
    if (fin_count > 0 && blockIdx.x == 0 && blockIdx.y == 0)
        finalize_norm<NT>(fin_ps, fin_pm, fin_count, fin_dev, fin_host, red);

    const int total = tiles_x * tiles_y * nchunks;
    const int lg = xcd_remap(blockIdx.x, total);
    const int tx = lg % tiles_x, ty = (lg / tiles_x) % tiles_y,
              ch = lg / (tiles_x * tiles_y);
    const long plane = (long)n * n, cplane = (long)nc * nc;
    b += (long)blockIdx.y * plane * n;
    e += (long)blockIdx.y * plane * n;
    bc += (long)blockIdx.y * cplane * nc;
    const int cx0 = tx * TXc, cy0 = ty * TYc;
    const int Z0 = ch * zchunk, Z1 = min(Z0 + zchunk, nc);
    const int fx0 = 2 * cx0, fy0 = 2 * cy0;
    // fine nodes owned: [f0, 2 (c0 + T)) per direction, the last tile up to n
    const int ox1 = cx0 + TXc >= nc ? n : fx0 + 2 * TXc;
    const int oy1 = cy0 + TYc >= nc ? n : fy0 + 2 * TYc;
    const int t = threadIdx.x;
    const int lane = t & 63;

    // interior e points: window index, b-window index, global offset, flags
    int li[M], lbi[M];
    unsigned gi[M];
    bool val[M], own[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = t + m * NT;
        const bool inr = i < NF;
        const int lx = i % FX, ly = i / FX;
        const int gx = fx0 + lx, gy = fy0 + ly;
        val[m] = inr && gx < n && gy < n;
        own[m] = inr && gx < ox1 && gy < oy1;
        li[m] = inr ? (ly + 1) * UX + lx + 1 : UD + lane;
        lbi[m] = inr ? (ly + 2) * BX + lx + 2 : BD + lane;
        gi[m] = val[m] ? (unsigned)((gy * n + gx) * (int)sizeof(S)) : kOob;
    }
    // ring-1 e point (no corners) of threads t < NR2
    int l1 = UD + lane, lb1 = BD + lane;
    unsigned g1 = kOob;
    bool v1 = false;
    if (t < NR2) {
        int ux, uy;
        if (t < FX) { ux = 1 + t; uy = 0; }
        else if (t < 2 * FX) { ux = 1 + t - FX; uy = UY - 1; }
        else if (t < 2 * FX + FY) { ux = 0; uy = 1 + t - 2 * FX; }
        else { ux = UX - 1; uy = 1 + t - 2 * FX - FY; }
        const int gx = fx0 - 1 + ux, gy = fy0 - 1 + uy;
        l1 = uy * UX + ux;
        lb1 = (uy + 1) * BX + ux + 1;
        v1 = gx >= 0 && gx < n && gy >= 0 && gy < n;
        if (v1) g1 = (unsigned)((gy * n + gx) * (int)sizeof(S));
    }
    // b point beyond the e points of threads t < NX: ring 2 without corners
    // (where the ring-1 e points reach) and the four ring-1 corners
    int lbx = BD + lane;
    unsigned gxo = kOob;
    if (t < NX) {
        int bx, by;
        if (t < FX) { bx = 2 + t; by = 0; }
        else if (t < 2 * FX) { bx = 2 + t - FX; by = BY - 1; }
        else if (t < 2 * FX + FY) { bx = 0; by = 2 + t - 2 * FX; }
        else if (t < NR2) { bx = BX - 1; by = 2 + t - 2 * FX - FY; }
        else {
            const int c = t - NR2;
            bx = (c & 1) ? BX - 2 : 1;
            by = (c & 2) ? BY - 2 : 1;
        }
        const int gx = fx0 - 2 + bx, gy = fy0 - 2 + by;
        lbx = by * BX + bx;
        if (gx >= 0 && gx < n && gy >= 0 && gy < n) gxo = (unsigned)((gy * n + gx) * (int)sizeof(S));
    }
    // b planes 2 Z0 - 2 .. 2 Z1 + 2 feed e up to plane 2 Z1 + 1 and the
    // residuals up to 2 Z1 (later planes read as zero); e is stored on the
    // owned planes 2 Z0 .. blast
    const int blast = min(n - 1, 2 * Z1 + 2);
    const int w0 = max(0, 2 * Z0 - 2), wcnt = blast - w0 + 1;
    const Win<S> wb(b, plane, w0, wcnt), we(e, plane, w0, wcnt), wbc(bc, cplane, Z0, Z1 - Z0);
    S rbi[4][M], rb1[4], rbx[2];
    auto issue = [&](int p, int q4, int q2) {
        const rsrc_t r = wb.r;
        const unsigned o = wb.at(p, p >= 0 && p <= blast);
#pragma unroll
        for (int m = 0; m < M; ++m) rbi[q4][m] = bload<S>(r, o + gi[m]);
        rb1[q4] = bload<S>(r, o + g1);
        rbx[q2] = bload<S>(r, o + gxo);
    };
    // e at the e points of plane p from the b window in slot B and b below
    // (slot dn) and above (slot up) in registers
    auto form_e = [&](int p, const C* B, int dn, int up, C* ei, C& e1) {
        const bool pin = p >= 0 && p < n;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int q = lbi[m];
            const C f = B[q - 1] + B[q + 1] + B[q - BX] + B[q + BX] + cvt<C>(rbi[dn][m]) +
                        cvt<C>(rbi[up][m]);
            const C v = sW * (c0 * B[q] + c1 * f);
            ei[m] = (pin && val[m]) ? v : C(0);
        }
        const int q = lb1;
        const C f = B[q - 1] + B[q + 1] + B[q - BX] + B[q + BX] + cvt<C>(rb1[dn]) + cvt<C>(rb1[up]);
        const C v = sW * (c0 * B[q] + c1 * f);
        e1 = (pin && v1) ? v : C(0);
    };
    auto put_b = [&](C* B, int q4, int q2) {
#pragma unroll
        for (int m = 0; m < M; ++m) B[lbi[m]] = cvt<C>(rbi[q4][m]);
        B[lb1] = cvt<C>(rb1[q4]);
        B[lbx] = cvt<C>(rbx[q2]);
    };
    auto store_e = [&](int p, const C* ei) {
        const bool pown = p >= 2 * Z0 && p < n && (p < 2 * Z1 || Z1 == nc);
        const unsigned o = we.at(p, pown);
#pragma unroll
        for (int m = 0; m < M; ++m)
            bstore<false>(static_cast<S>(ei[m]), we.r, o + (own[m] ? gi[m] : kOob));
    };
    const int cx = t % TXc, cy = t / TXc;
    const bool cin = t < TXc * TYc;
    const unsigned cgb = (cin && cx0 + cx < nc && cy0 + cy < nc)
                             ? (unsigned)(((cy0 + cy) * nc + cx0 + cx) * (int)sizeof(S))
                             : kOob;
    const int cq = RP + (cin ? (2 * cy + 1) * FX + 2 * cx + 1 : FX + 1);

    C um1[M], u0[M], up1[M];
    C ur0 = 0, urp1 = 0, acc = 0;
    const int f0 = 2 * Z0, f1 = 2 * Z1;
    {
        // planes f0-2 .. f0+2; register slot of plane p is (p - f0) mod 4
        // (mod 2 for the b beyond the e points), LDS slot (p - f0) mod 3
        S tmi[2][M], tm1[2], tx0, tx1;
        {
            const unsigned o0 = wb.at(f0 - 2, f0 - 2 >= 0), o1 = wb.at(f0 - 1, f0 - 1 >= 0);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                tmi[0][m] = bload<S>(wb.r, o0 + gi[m]);
                tmi[1][m] = bload<S>(wb.r, o1 + gi[m]);
            }
            tm1[0] = bload<S>(wb.r, o0 + g1);
            tm1[1] = bload<S>(wb.r, o1 + g1);
        }
        issue(f0, 0, 0);
        tx0 = rbx[0];
        issue(f0 + 1, 1, 1);
        tx1 = rbx[1];
        issue(f0 + 2, 2, 0);
        // LDS: slot 2 <- plane f0-1 (e points only), slot 0 <- f0, slot 1 <- f0+1
#pragma unroll
        for (int m = 0; m < M; ++m) bL[2][lbi[m]] = cvt<C>(tmi[1][m]);
        bL[2][lb1] = cvt<C>(tm1[1]);
#pragma unroll
        for (int m = 0; m < M; ++m) bL[0][lbi[m]] = cvt<C>(rbi[0][m]);
        bL[0][lb1] = cvt<C>(rb1[0]);
        bL[0][lbx] = cvt<C>(tx0);
#pragma unroll
        for (int m = 0; m < M; ++m) bL[1][lbi[m]] = cvt<C>(rbi[1][m]);
        bL[1][lb1] = cvt<C>(rb1[1]);
        bL[1][lbx] = cvt<C>(tx1);
        __syncthreads();
        // e(f0 - 1) at the interior: b below from the prologue registers,
        // above = plane f0 (slot 0)
        {
            const bool pin = f0 - 1 >= 0;
            const C* B = bL[2];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int q = lbi[m];
                const C f = B[q - 1] + B[q + 1] + B[q - BX] + B[q + BX] + cvt<C>(tmi[0][m]) +
                            cvt<C>(rbi[0][m]);
                const C v = sW * (c0 * B[q] + c1 * f);
                um1[m] = (pin && val[m]) ? v : C(0);
            }
        }
        // e(f0) at the e points: below = plane f0-1 (prologue), above = f0+1
        {
            const C* B = bL[0];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int q = lbi[m];
                const C f = B[q - 1] + B[q + 1] + B[q - BX] + B[q + BX] + cvt<C>(tmi[1][m]) +
                            cvt<C>(rbi[1][m]);
                const C v = sW * (c0 * B[q] + c1 * f);
                u0[m] = val[m] ? v : C(0);
            }
            const int q = lb1;
            const C f = B[q - 1] + B[q + 1] + B[q - BX] + B[q + BX] + cvt<C>(tm1[1]) +
                        cvt<C>(rb1[1]);
            const C v = sW * (c0 * B[q] + c1 * f);
            ur0 = v1 ? v : C(0);
        }
#pragma unroll
        for (int m = 0; m < M; ++m) uL[0][li[m]] = u0[m];
        uL[0][l1] = ur0;
        store_e(f0, u0);
    }
    auto step = [&](int s, auto kc) {
        constexpr int k = decltype(kc)::k;  // (s - f0) % UN
        constexpr int cu = k & 1, nx = (k + 1) & 1;
        __syncthreads();
        issue(s + 3, (k + 3) % 4, (k + 3) % 2);
        // e of plane s + 1 (one plane ahead of the residual)
        form_e(s + 1, bL[(k + 1) % 3], k % 4, (k + 2) % 4, up1, urp1);
        // residual of fine plane s on the window
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const C* U = uL[cu];
            const int q = li[m];
            const C lap = C(6) * u0[m] - U[q - 1] - U[q + 1] - U[q - UX] - U[q + UX] - um1[m] -
                          up1[m];
            const C r = cvt<C>(rbi[k % 4][m]) - sA * lap;
            rL[cu][RP + t + m * NT] = val[m] ? r : C(0);
        }
        const int f = s - 1;  // fine plane whose residual is reduced now
        if (f >= f0 && f <= f1) {
            const C* R = rL[nx];
            const int q = cq;
            const C xs = C(0.25) * R[q] +
                         C(0.125) * (R[q - 1] + R[q + 1] + R[q - FX] + R[q + FX]) +
                         C(0.0625) * (R[q - FX - 1] + R[q - FX + 1] + R[q + FX - 1] + R[q + FX + 1]);
            if ((k & 1) == 1) {  // f - f0 even
                if (f > f0) {
                    acc += C(0.25) * xs;
                    bstore<false>(static_cast<S>(acc), wbc.r, wbc.at(f / 2 - 1, true) + cgb);
                }
                acc = C(0.25) * xs;
            } else {
                acc += C(0.5) * xs;
            }
        }
#pragma unroll
        for (int m = 0; m < M; ++m) uL[nx][li[m]] = up1[m];
        uL[nx][l1] = urp1;
        store_e(s + 1, up1);
        put_b(bL[(k + 2) % 3], (k + 2) % 4, k % 2);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            um1[m] = u0[m];
            u0[m] = up1[m];
        }
    };
    march<UN>(f0, f1 + 1, step);
}

// ---------------------------------------------------------------------------
// 2D fused residual + full-weighting restriction: a strip of TXc coarse
// columns (window of 2 TXc + 1 fine columns owned by NT lanes), marching
// over fine rows.
// ---------------------------------------------------------------------------
template <typename S, typename C, int TXc, int NT, int UN>
__global__ void __launch_bounds__(NT)
k_restrict2d(const S* __restrict__ u, const S* __restrict__ b, S* __restrict__ bc,
             int n, int nc, int tiles_x, int ychunk, int nchunks, C sA,
             const double* __restrict__ fin_ps, const double* __restrict__ fin_pm, int fin_count,
             double* __restrict__ fin_dev, double* __restrict__ fin_host) {
    constexpr int FX = 2 * TXc + 1, UX = FX + 2;
    constexpr int M = (FX + NT - 1) / NT;
    constexpr int RSZ = M * NT + 2;
    constexpr int UD = UX + 1, USZ = UD + 65;
    constexpr int RS = 2;
    static_assert(TXc <= NT, "one thread per coarse column");
    static_assert(UN % 2 == 0, "unroll covers the prefetch ring and the row parity");
    __shared__ C uL[2][USZ];
    __shared__ C rL[2][RSZ];
    __shared__ double red[NT / 64];
    if (fin_count > 0 && blockIdx.x == 0 && blockIdx.y == 0)
        finalize_norm<NT>(fin_ps, fin_pm, fin_count, fin_dev, fin_host, red);

    const int total = tiles_x * nchunks;
    const int lg = xcd_remap(blockIdx.x, total);
    const int tx = lg % tiles_x, ch = lg / tiles_x;
    u += (long)blockIdx.y * n * n;
    b += (long)blockIdx.y * n * n;
    bc += (long)blockIdx.y * nc * nc;
    const int cx0 = tx * TXc, fx0 = 2 * cx0;
    const int Y0 = ch * ychunk, Y1 = min(Y0 + ychunk, nc);
    const int t = threadIdx.x;
    const int lane = t & 63;

    int ul[M];
    unsigned gb[M];
    bool val[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = t + m * NT;
        const bool inr = i < FX;
        const int gx = fx0 + i;
        val[m] = inr && gx < n;
        ul[m] = inr ? i + 1 : UD + lane;
        gb[m] = val[m] ? (unsigned)(gx * (int)sizeof(S)) : kOob;
    }
    const int r2x = (t == 0) ? fx0 - 1 : fx0 + FX;
    const int r2l = t < 2 ? (t == 0 ? 0 : UX - 1) : UD + lane;
    const unsigned r2b =
        (t < 2 && r2x >= 0 && r2x < n) ? (unsigned)(r2x * (int)sizeof(S)) : kOob;
    // fine rows 2 Y0 - 1 .. 2 Y1 + 1 feed the residuals of rows 2 Y0 .. 2 Y1
    // (later rows read as zero), in one window per field
    const int ulast = min(n - 1, 2 * Y1 + 1), blast = min(n - 1, 2 * Y1);
    const int w0 = max(0, 2 * Y0 - 1), wcnt = ulast - w0 + 1;
    const Win<S> wu(u, n, w0, wcnt), wb(b, n, w0, wcnt), wbc(bc, nc, Y0, Y1 - Y0);
    S ru[RS][M], rb[RS][M], rr2[RS];
    auto issue_u = [&](int p, int k) {
        const unsigned o = wu.at(p, p >= 0 && p <= ulast);
#pragma unroll
        for (int m = 0; m < M; ++m) ru[k][m] = bload<S>(wu.r, o + gb[m]);
        rr2[k] = bload<S>(wu.r, o + r2b);
    };
    auto issue_b = [&](int p, int k) {
        const unsigned o = wb.at(p, p >= 0 && p <= blast);
#pragma unroll
        for (int m = 0; m < M; ++m) rb[k][m] = bload<S>(wb.r, o + gb[m]);
    };
    const unsigned cgb =
        (t < TXc && cx0 + t < nc) ? (unsigned)((cx0 + t) * (int)sizeof(S)) : kOob;
    const int cq = 1 + (t < TXc ? 2 * t + 1 : 1);

    C um1[M], u0[M], up1[M];
    C ur0 = 0, urp1 = 0, acc = 0;
    const int f0 = 2 * Y0, f1 = 2 * Y1;
    {
        // all prologue loads before the first wait
        issue_b(f0, 0);
        S pu[3][M], pr2[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int p = f0 - 1 + q;
            const unsigned o = wu.at(p, p >= 0 && p <= ulast);
#pragma unroll
            for (int m = 0; m < M; ++m) pu[q][m] = bload<S>(wu.r, o + gb[m]);
            pr2[q] = bload<S>(wu.r, o + r2b);
        }
        C dummy;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            C* dst = q == 0 ? um1 : (q == 1 ? u0 : up1);
#pragma unroll
            for (int m = 0; m < M; ++m) dst[m] = cvt<C>(pu[q][m]);
            (q == 1 ? ur0 : (q == 2 ? urp1 : dummy)) = cvt<C>(pr2[q]);
        }
        issue_u(f0 + 2, 0);
        const int sl = f0 & 1;
#pragma unroll
        for (int m = 0; m < M; ++m) uL[sl][ul[m]] = u0[m];
        uL[sl][r2l] = ur0;
    }
    auto step = [&](int s, auto kc) {
        constexpr int k = decltype(kc)::k;  // (s - f0) % UN
        __syncthreads();
        const int cur = s & 1;
        issue_u(s + 3, (k + 1) % RS);
        issue_b(s + 1, (k + 1) % RS);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const C* U = uL[cur];
            const int q = ul[m];
            const C lap = C(4) * u0[m] - U[q - 1] - U[q + 1] - um1[m] - up1[m];
            const C r = cvt<C>(rb[k % RS][m]) - sA * lap;
            rL[cur][1 + t + m * NT] = val[m] ? r : C(0);
        }
        const int f = s - 1;
        if (f >= f0 && f <= f1) {
            const C* R = rL[cur ^ 1];
            const C xs = C(0.5) * R[cq] + C(0.25) * (R[cq - 1] + R[cq + 1]);
            if ((k & 1) == 1) {  // f - f0 even
                if (f > f0) {
                    acc += C(0.25) * xs;
                    bstore<false>(static_cast<S>(acc), wbc.r, wbc.at(f / 2 - 1, true) + cgb);
                }
                acc = C(0.25) * xs;
            } else {
                acc += C(0.5) * xs;
            }
        }
#pragma unroll
        for (int m = 0; m < M; ++m) uL[cur ^ 1][ul[m]] = up1[m];
        uL[cur ^ 1][r2l] = urp1;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            um1[m] = u0[m];
            u0[m] = up1[m];
            up1[m] = cvt<C>(ru[k % RS][m]);
        }
        urp1 = cvt<C>(rr2[k % RS]);
    };
    march<UN>(f0, f1 + 1, step);
}

// ---------------------------------------------------------------------------
// Linear interpolation + correction: out = in + pf * P ec (in may be out).
// One fine node per thread; the coarse values (1/2^d of the traffic) come
// through L2.
// ---------------------------------------------------------------------------
template <typename S, typename C>
__global__ void __launch_bounds__(256)
k_prolong2d(const S* __restrict__ ec, const S* in, S* out, int n, int nc, C pf) {
    const long area = (long)n * n;
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= area) return;
    in += (long)blockIdx.y * area;
    out += (long)blockIdx.y * area;
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
    st_out(&out[idx], static_cast<S>(cvt<C>(in[idx]) + pf * (wi * wj) * s), area >= kNtMinPts);
}

template <typename S, typename C>
__global__ void __launch_bounds__(256)
k_prolong3d(const S* __restrict__ ec, const S* in, S* out, int n, int nc, C pf) {
    const long vol = (long)n * n * n;
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= vol) return;
    in += (long)blockIdx.y * vol;
    out += (long)blockIdx.y * vol;
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
    st_out(&out[idx], static_cast<S>(cvt<C>(in[idx]) + pf * w * s), vol >= kNtMinPts);
}

// ---------------------------------------------------------------------------
// Zero-guess pre-smoothing fused with the restriction (2D coarse levels):
// e = sW K_c b, r = b - sA L e, bc = R r.  A workgroup owns a tile of coarse
// nodes; it stages b on the tile's fine footprint plus a ring of 3 in LDS
// (zero outside the grid), forms e on the footprint plus a ring of 1 (zero
// outside the grid), r on the footprint, and writes e on the fine nodes it
// owns and bc on its coarse nodes.  The halo costs re-reads (mostly L2 hits)
// and recomputation of e, against a whole launch and one pass over b and e
// in HBM saved.  Arithmetic in the order of the separate sweeps.  Block 0
// reduces a pending norm like the restriction does.
// ---------------------------------------------------------------------------
template <typename S, typename C, int CX, int CY, int NT>
__global__ void __launch_bounds__(NT)
k_zsr2d(const S* __restrict__ b, S* __restrict__ e, S* __restrict__ bc, int n, int nc,
        int tiles_x, int tiles_y, C sA, C sW, C c0, C c1, C c2,
        const double* __restrict__ fin_ps, const double* __restrict__ fin_pm, int fin_count,
        double* __restrict__ fin_dev, double* __restrict__ fin_host) {
    constexpr int RX = 2 * CX + 1, RY = 2 * CY + 1;  // r: the fine footprint
    constexpr int EX = RX + 2, EY = RY + 2;          // e: footprint + 1
    constexpr int BX = RX + 4, BY = RY + 4;          // b: footprint + 2 (+ 1 for e)
    __shared__ C bL[BX * BY];
    __shared__ C eL[EX * EY];
    __shared__ C rL[RX * RY];
    __shared__ double red[NT / 64];
    if (fin_count > 0 && blockIdx.x == 0 && blockIdx.y == 0)
        finalize_norm<NT>(fin_ps, fin_pm, fin_count, fin_dev, fin_host, red);
    const int lg = xcd_remap(blockIdx.x, tiles_x * tiles_y);
    const int cx0 = (lg % tiles_x) * CX, cy0 = (lg / tiles_x) * CY;
    const int fx0 = 2 * cx0, fy0 = 2 * cy0;
    const long area = (long)n * n;
    b += (long)blockIdx.y * area;
    e += (long)blockIdx.y * area;
    bc += (long)blockIdx.y * nc * nc;
    // fine nodes owned: [fx0, 2 (cx0 + CX)), the last tile up to n
    const int ox1 = cx0 + CX >= nc ? n : fx0 + 2 * CX;
    const int oy1 = cy0 + CY >= nc ? n : fy0 + 2 * CY;
    const int t = threadIdx.x;
    {
        // every load in flight before the first wait
        constexpr int NB = (BX * BY + NT - 1) / NT;
        S v[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i = t + j * NT;
            const int lx = i % BX, ly = i / BX;
            const int gx = fx0 - 2 + lx, gy = fy0 - 2 + ly;
            const bool in = i < BX * BY && gx >= 0 && gx < n && gy >= 0 && gy < n;
            v[j] = in ? b[(long)gy * n + gx] : S(0);
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i = t + j * NT;
            if (i < BX * BY) bL[i] = cvt<C>(v[j]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < (EX * EY + NT - 1) / NT; ++j) {
        const int i = t + j * NT;
        if (i >= EX * EY) break;
        const int lx = i % EX, ly = i / EX;
        const int gx = fx0 - 1 + lx, gy = fy0 - 1 + ly;
        const int q = (ly + 1) * BX + lx + 1;
        const C f = bL[q - 1] + bL[q + 1] + bL[q - BX] + bL[q + BX];
        const C cn = bL[q - BX - 1] + bL[q - BX + 1] + bL[q + BX - 1] + bL[q + BX + 1];
        const C v = sW * (c0 * bL[q] + c1 * f + c2 * cn);
        const bool in = gx >= 0 && gx < n && gy >= 0 && gy < n;
        eL[i] = in ? v : C(0);
        if (gx >= fx0 && gx < ox1 && gy >= fy0 && gy < oy1)
            e[(long)gy * n + gx] = static_cast<S>(v);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < (RX * RY + NT - 1) / NT; ++j) {
        const int i = t + j * NT;
        if (i >= RX * RY) break;
        const int lx = i % RX, ly = i / RX;
        const int qe = (ly + 1) * EX + lx + 1, qb = (ly + 2) * BX + lx + 2;
        const C lap = C(4) * eL[qe] - eL[qe - 1] - eL[qe + 1] - eL[qe - EX] - eL[qe + EX];
        const C r = bL[qb] - sA * lap;
        rL[i] = (fx0 + lx < n && fy0 + ly < n) ? r : C(0);
    }
    __syncthreads();
    for (int i = t; i < CX * CY; i += NT) {
        const int lx = i % CX, ly = i / CX;
        const int ci = cx0 + lx, cj = cy0 + ly;
        if (ci >= nc || cj >= nc) continue;
        const int q = (2 * ly + 1) * RX + 2 * lx + 1;
        auto xs = [&](int c) { return C(0.5) * rL[c] + C(0.25) * (rL[c - 1] + rL[c + 1]); };
        C acc = C(0.25) * xs(q - RX);
        acc += C(0.5) * xs(q);
        acc += C(0.25) * xs(q + RX);
        bc[(long)cj * nc + ci] = static_cast<S>(acc);
    }
}

// ---------------------------------------------------------------------------
// The same fusion on 3D coarse grids (7-point K_c and L): a workgroup owns a
// CX x CY x CZ block of coarse nodes, stages b on the block's fine footprint
// plus a ring of 2 in LDS (zero outside the grid), forms e on the footprint
// plus a ring of 1, r on the footprint and the 27-point full weighting, and
// writes e on the fine nodes it owns and bc on its coarse nodes.  One
// launch and no march per level, where the marching pair (smoother, then
// restriction) costs two launch latencies.  e enters r as stored (rounded
// to S), r is written over b in place (each node reads only its own b), and
// every sum runs in the order of the separate sweeps, so the results equal
// theirs.  Block 0 reduces a pending norm like the restriction does.
// ---------------------------------------------------------------------------
template <typename S, typename C, int CX, int CY, int CZ, int NT>
__global__ void __launch_bounds__(NT)
k_zsr3d(const S* __restrict__ b, S* __restrict__ e, S* __restrict__ bc, int n, int nc,
        int tiles_x, int tiles_y, int tiles_z, C sA, C sW, C c0, C c1,
        const double* __restrict__ fin_ps, const double* __restrict__ fin_pm, int fin_count,
        double* __restrict__ fin_dev, double* __restrict__ fin_host) {
    constexpr int RX = 2 * CX + 1, RY = 2 * CY + 1, RZ = 2 * CZ + 1;  // the fine footprint
    constexpr int EX = RX + 2, EY = RY + 2, EZ = RZ + 2;              // e: footprint + 1
    constexpr int BX = RX + 4, BY = RY + 4, BZ = RZ + 4;              // b: footprint + 2
    constexpr int BP = BX * BY, EP = EX * EY;
    __shared__ C bL[BP * BZ];  // b, then r on the footprint
    __shared__ C eL[EP * EZ];
    __shared__ double red[NT / 64];
    if (fin_count > 0 && blockIdx.x == 0 && blockIdx.y == 0)
        finalize_norm<NT>(fin_ps, fin_pm, fin_count, fin_dev, fin_host, red);
    const int lg = xcd_remap(blockIdx.x, tiles_x * tiles_y * tiles_z);
    const int cx0 = (lg % tiles_x) * CX, cy0 = ((lg / tiles_x) % tiles_y) * CY,
              cz0 = (lg / (tiles_x * tiles_y)) * CZ;
    const int fx0 = 2 * cx0, fy0 = 2 * cy0, fz0 = 2 * cz0;
    const long vol = (long)n * n * n;
    b += (long)blockIdx.y * vol;
    e += (long)blockIdx.y * vol;
    bc += (long)blockIdx.y * nc * nc * nc;
    // fine nodes owned: [fx0, 2 (cx0 + CX)), the last block up to n
    const int ox1 = cx0 + CX >= nc ? n : fx0 + 2 * CX;
    const int oy1 = cy0 + CY >= nc ? n : fy0 + 2 * CY;
    const int oz1 = cz0 + CZ >= nc ? n : fz0 + 2 * CZ;
    const int t = threadIdx.x;
    {
        // every load in flight before the first wait (a loop that waits for
        // each load in turn costs one memory latency per iteration)
        constexpr int NB = (BP * BZ + NT - 1) / NT;
        S v[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i = t + j * NT;
            const int lx = i % BX, ly = (i / BX) % BY, lz = i / BP;
            const int gx = fx0 - 2 + lx, gy = fy0 - 2 + ly, gz = fz0 - 2 + lz;
            const bool in = i < BP * BZ && gx >= 0 && gx < n && gy >= 0 && gy < n && gz >= 0 &&
                            gz < n;
            v[j] = in ? b[((long)gz * n + gy) * n + gx] : S(0);
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i = t + j * NT;
            if (i < BP * BZ) bL[i] = cvt<C>(v[j]);
        }
    }
    __syncthreads();
    // fixed trip counts, unrolled: LDS reads of later points issue ahead
#pragma unroll
    for (int j = 0; j < (EP * EZ + NT - 1) / NT; ++j) {
        const int i = t + j * NT;
        if (i >= EP * EZ) break;
        const int lx = i % EX, ly = (i / EX) % EY, lz = i / EP;
        const int gx = fx0 - 1 + lx, gy = fy0 - 1 + ly, gz = fz0 - 1 + lz;
        const int q = (lz + 1) * BP + (ly + 1) * BX + lx + 1;
        const C f = bL[q - 1] + bL[q + 1] + bL[q - BX] + bL[q + BX] + bL[q - BP] + bL[q + BP];
        const S v = static_cast<S>(sW * (c0 * bL[q] + c1 * f));
        const bool in = gx >= 0 && gx < n && gy >= 0 && gy < n && gz >= 0 && gz < n;
        eL[i] = in ? cvt<C>(v) : C(0);
        if (gx >= fx0 && gx < ox1 && gy >= fy0 && gy < oy1 && gz >= fz0 && gz < oz1)
            e[((long)gz * n + gy) * n + gx] = v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < (RX * RY * RZ + NT - 1) / NT; ++j) {
        const int i = t + j * NT;
        if (i >= RX * RY * RZ) break;
        const int lx = i % RX, ly = (i / RX) % RY, lz = i / (RX * RY);
        const int qe = (lz + 1) * EP + (ly + 1) * EX + lx + 1;
        const int qb = (lz + 2) * BP + (ly + 2) * BX + lx + 2;
        const C lap = C(6) * eL[qe] - eL[qe - 1] - eL[qe + 1] - eL[qe - EX] - eL[qe + EX] -
                      eL[qe - EP] - eL[qe + EP];
        const C r = bL[qb] - sA * lap;
        bL[qb] = (fx0 + lx < n && fy0 + ly < n && fz0 + lz < n) ? r : C(0);
    }
    __syncthreads();
    for (int i = t; i < CX * CY * CZ; i += NT) {
        const int lx = i % CX, ly = (i / CX) % CY, lz = i / (CX * CY);
        const int ci = cx0 + lx, cj = cy0 + ly, ck = cz0 + lz;
        if (ci >= nc || cj >= nc || ck >= nc) continue;
        // coarse node over footprint point (2 lx + 1, 2 ly + 1, 2 lz + 1)
        const int q = (2 * lz + 3) * BP + (2 * ly + 3) * BX + 2 * lx + 3;
        auto xs = [&](int c) {
            return C(0.25) * bL[c] + C(0.125) * (bL[c - 1] + bL[c + 1] + bL[c - BX] + bL[c + BX]) +
                   C(0.0625) * (bL[c - BX - 1] + bL[c - BX + 1] + bL[c + BX - 1] + bL[c + BX + 1]);
        };
        C acc = C(0.25) * xs(q - BP);
        acc += C(0.5) * xs(q);
        acc += C(0.25) * xs(q + BP);
        bc[((long)ck * nc + cj) * nc + ci] = static_cast<S>(acc);
    }
}

// ---------------------------------------------------------------------------
// Post-smoothing with the fused coarse correction on small 3D grids (7-point
// K_c and L), as a tile kernel: v = u + pf P ec on the tile plus a ring of
// 2, r = b - sA L v on the tile plus a ring of 1 (zero outside the grid),
// out = v + sW K_c r on the tile.  A workgroup loads u, b and the coarse
// block under its tile with every load in flight before the first wait,
// stages the coarse block and v in LDS and needs no march: one launch
// latency per level where a march pays its pipeline fill.  The trilinear
// value is formed as the marching kernel forms it (bilinear in the plane,
// then the mean of two coarse planes between them) and every sum runs in
// that kernel's order; the compiler's fused multiply-adds may still differ,
// so results agree with the march's to rounding, not bit for bit.
// ---------------------------------------------------------------------------
template <typename S, typename C, int TX, int TY, int TZ, int NT>
__global__ void __launch_bounds__(NT)
k_pro3d(const S* __restrict__ u, const S* __restrict__ b, S* __restrict__ out,
        const S* __restrict__ ec, int n, int nc, int tiles_x, int tiles_y, int tiles_z, C sA,
        C sW, C c0, C c1, C pf) {
    constexpr int VX = TX + 4, VY = TY + 4, VZ = TZ + 4, VP = VX * VY, NV = VP * VZ;
    constexpr int RX = TX + 2, RY = TY + 2, RZ = TZ + 2, RP = RX * RY, NR = RP * RZ;
    constexpr int CX = TX / 2 + 4, CY = TY / 2 + 4, CZ = TZ / 2 + 4, CP = CX * CY;
    constexpr int NCB = CP * CZ;
    constexpr int MV = (NV + NT - 1) / NT, MR = (NR + NT - 1) / NT, MCB = (NCB + NT - 1) / NT;
    static_assert(TX % 2 == 0 && TY % 2 == 0 && TZ % 2 == 0, "even tiles");
    __shared__ C cL[NCB];
    __shared__ C vL[NV];
    __shared__ C rL[NR];
    const int lg = xcd_remap(blockIdx.x, tiles_x * tiles_y * tiles_z);
    const int x0 = (lg % tiles_x) * TX, y0 = ((lg / tiles_x) % tiles_y) * TY,
              z0 = (lg / (tiles_x * tiles_y)) * TZ;
    const long vol = (long)n * n * n;
    u += (long)blockIdx.y * vol;
    b += (long)blockIdx.y * vol;
    out += (long)blockIdx.y * vol;
    ec += (long)blockIdx.y * nc * nc * nc;
    // coarse block origin: the lower coarse neighbour of fine index x0 - 2
    const int cx0 = x0 / 2 - 2, cy0 = y0 / 2 - 2, cz0 = z0 / 2 - 2;
    const int t = threadIdx.x;
    auto fin = [&](int gx, int gy, int gz) {
        return gx >= 0 && gx < n && gy >= 0 && gy < n && gz >= 0 && gz < n;
    };
    S ru[MV], rb[MR], rc[MCB];
#pragma unroll
    for (int j = 0; j < MV; ++j) {
        const int i = t + j * NT;
        const int gx = x0 - 2 + i % VX, gy = y0 - 2 + (i / VX) % VY, gz = z0 - 2 + i / VP;
        ru[j] = (i < NV && fin(gx, gy, gz)) ? u[((long)gz * n + gy) * n + gx] : S(0);
    }
#pragma unroll
    for (int j = 0; j < MR; ++j) {
        const int i = t + j * NT;
        const int gx = x0 - 1 + i % RX, gy = y0 - 1 + (i / RX) % RY, gz = z0 - 1 + i / RP;
        rb[j] = (i < NR && fin(gx, gy, gz)) ? b[((long)gz * n + gy) * n + gx] : S(0);
    }
#pragma unroll
    for (int j = 0; j < MCB; ++j) {
        const int i = t + j * NT;
        const int kx = cx0 + i % CX, ky = cy0 + (i / CX) % CY, kz = cz0 + i / CP;
        const bool in = i < NCB && kx >= 0 && kx < nc && ky >= 0 && ky < nc && kz >= 0 &&
                        kz < nc;
        rc[j] = in ? ec[((long)kz * nc + ky) * nc + kx] : S(0);
    }
#pragma unroll
    for (int j = 0; j < MCB; ++j)
        if (t + j * NT < NCB) cL[t + j * NT] = cvt<C>(rc[j]);
    __syncthreads();
    // v = u + pf P ec on the tile + 2
#pragma unroll
    for (int j = 0; j < MV; ++j) {
        const int i = t + j * NT;
        if (i >= NV) break;
        const int G = x0 - 1 + i % VX, H = y0 - 1 + (i / VX) % VY, Z = z0 - 1 + i / VP;
        const int lx = (G >> 1) - 1 - cx0, ly = (H >> 1) - 1 - cy0, lz = (Z >> 1) - 1 - cz0;
        const bool hx = G & 1, hy = H & 1;
        auto q_at = [&](int kz) {
            const int c = kz * CP + ly * CX + lx;
            C q = cL[c];
            q += hx ? cL[c + 1] : C(0);
            q += hy ? cL[c + CX] : C(0);
            q += (hx && hy) ? cL[c + CX + 1] : C(0);
            return (hx ? C(0.5) : C(1)) * (hy ? C(0.5) : C(1)) * q;
        };
        const C pe = (Z & 1) ? C(0.5) * (q_at(lz) + q_at(lz + 1)) : q_at(lz);
        vL[i] = cvt<C>(ru[j]) + pf * pe;
    }
    __syncthreads();
    // r = b - sA L v on the tile + 1
#pragma unroll
    for (int j = 0; j < MR; ++j) {
        const int i = t + j * NT;
        if (i >= NR) break;
        const int lx = i % RX, ly = (i / RX) % RY, lz = i / RP;
        const int q = (lz + 1) * VP + (ly + 1) * VX + lx + 1;
        const C lap = C(6) * vL[q] - vL[q - 1] - vL[q + 1] - vL[q - VX] - vL[q + VX] -
                      vL[q - VP] - vL[q + VP];
        const C r = cvt<C>(rb[j]) - sA * lap;
        rL[i] = fin(x0 - 1 + lx, y0 - 1 + ly, z0 - 1 + lz) ? r : C(0);
    }
    __syncthreads();
    // out = v + sW K_c r on the tile
#pragma unroll
    for (int j = 0; j < (TX * TY * TZ + NT - 1) / NT; ++j) {
        const int i = t + j * NT;
        if (i >= TX * TY * TZ) break;
        const int lx = i % TX, ly = (i / TX) % TY, lz = i / (TX * TY);
        const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
        if (gx >= n || gy >= n || gz >= n) continue;
        const int q = (lz + 1) * RP + (ly + 1) * RX + lx + 1;
        const int qv = (lz + 2) * VP + (ly + 2) * VX + lx + 2;
        const C nbs = rL[q - 1] + rL[q + 1] + rL[q - RX] + rL[q + RX] + rL[q - RP] + rL[q + RP];
        const C v = vL[qv] + sW * (c0 * rL[q] + c1 * nbs);
        out[((long)gz * n + gy) * n + gx] = static_cast<S>(v);
    }
}

// ---------------------------------------------------------------------------
// Pre-smoothing fused with the restriction (2D, any iterate):
// out = u + sW K_c (b - sA L u) and bc = R (b - sA L out).  x strips of TX
// fine columns march over rows; a row passes four stages, each one row
// behind the last, so that one barrier per row suffices: at step s the
// residual of row s (strip + ring 2, from u on strip + ring 3), the new
// iterate of row s-2 (strip + ring 1, from residual rows s-3..s-1), the new
// residual of row s-3 (the strip + the column right of it, where the
// coarse nodes' full-weighting stencils reach) and its restriction one step
// later.  Residuals and iterates outside the grid are zero.  The new
// iterate enters the second residual as stored (rounded to S), as it would
// from HBM.  The norm variant sums (b - sA L u)^2 over the owned nodes (the
// residual of the incoming iterate).  Against the separate smoother and
// restriction, one pass over u and b and one launch are saved for ring-3
// halo columns (L2 hits) and three extra rows per chunk.
// ---------------------------------------------------------------------------
template <typename S, typename C, int TX, int NT, int PD, int UN, bool NTS, bool NORM,
          bool ROUT = false, typename SU = S>
__global__ void __launch_bounds__(NT)
k_sr2d(const SU* __restrict__ u, const S* __restrict__ b, S* __restrict__ out,
       S* __restrict__ bc, int n, int nc, int tiles_x, int ychunk, int nchunks, C sA, C sW,
       C c0, C c1, C c2, double* __restrict__ partials, S* __restrict__ rout = nullptr,
       double* __restrict__ bparts = nullptr) {
    constexpr int W = TX + 7;             // columns x0-3 .. x0+TX+3
    constexpr int M = (W + NT - 1) / NT;
    constexpr int LW = W + 2 + 65;        // one guard each side, scratch for idle lanes
    constexpr int HC = TX / 2;            // coarse columns per strip
    constexpr int MC = (HC + NT - 1) / NT;
    constexpr int RS = PD + 1;
    static_assert(TX % 2 == 0, "even strips");
    static_assert(UN % RS == 0, "unroll covers the prefetch ring");
    __shared__ C uL[2][LW];
    __shared__ C rL[4][LW];
    __shared__ C vL[2][LW];
    __shared__ C wL[2][LW];
    __shared__ double red[NT / 64];

    const int total = tiles_x * nchunks;
    const int lg = xcd_remap(blockIdx.x, total);
    const int tx = lg % tiles_x, ch = lg / tiles_x;
    const long area = (long)n * n;
    u += (long)blockIdx.y * area;
    b += (long)blockIdx.y * area;
    out += (long)blockIdx.y * area;
    if (ROUT) rout += (long)blockIdx.y * area;
    bc += (long)blockIdx.y * nc * nc;
    const int x0 = tx * TX;
    const int Y0 = ch * ychunk, Y1 = min(Y0 + ychunk, nc);
    // fine rows owned: [2 Y0, 2 Y1), the last chunk up to n
    const int o0 = 2 * Y0, o1 = Y1 == nc ? n : 2 * Y1;
    const int t = threadIdx.x;
    const int lane = t & 63;

    int li[M];
    unsigned gb[M], gu[M];
    bool col[M], own[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int j = t + m * NT;
        const bool inr = j < W;
        const int gx = x0 - 3 + j;
        col[m] = inr && gx >= 0 && gx < n;
        own[m] = col[m] && gx >= x0 && gx < x0 + TX;
        li[m] = inr ? j + 1 : W + 2 + lane;
        gb[m] = col[m] ? (unsigned)(gx * (int)sizeof(S)) : kOob;
        gu[m] = col[m] ? (unsigned)(gx * (int)sizeof(SU)) : kOob;
    }
    // coarse column x0/2 + i sits over local column 2 i + 4
    int cq[MC];
    unsigned cgb[MC];
#pragma unroll
    for (int q = 0; q < MC; ++q) {
        const int i = t + q * NT;
        const bool ok = i < HC && x0 / 2 + i < nc;
        cq[q] = i < HC ? 2 * i + 5 : W + 2 + lane;
        cgb[q] = ok ? (unsigned)((x0 / 2 + i) * (int)sizeof(S)) : kOob;
    }

    // rows any output depends on: u up to 2 Y1 + 3, b up to 2 Y1 + 2; the
    // whole unrolled groups and the prefetch run past them, and rows
    // outside these ranges read as zero without touching memory
    const int ulast = min(n - 1, 2 * Y1 + 3), blast = min(n - 1, 2 * Y1 + 2);
    // one window of fine rows 2 Y0 - 3 .. ulast serves every fine field
    const int f0 = max(0, 2 * Y0 - 3), fcnt = ulast - f0 + 1;
    const Win<SU> wu(u, n, f0, fcnt);
    const Win<S> wb(b, n, f0, fcnt), wo(out, n, f0, fcnt);
    const Win<S> wro(ROUT ? rout : out, n, f0, fcnt), wbc(bc, nc, Y0, Y1 - Y0);
    SU ru[RS][M];
    S rb[RS][M];
    auto issue_u = [&](int p, int k) {
        const unsigned o = wu.at(p, p >= 0 && p <= ulast);
#pragma unroll
        for (int m = 0; m < M; ++m) ru[k][m] = bload<SU>(wu.r, o + gu[m]);
    };
    auto issue_b = [&](int p, int k) {
        const unsigned o = wb.at(p, p >= 0 && p <= blast);
#pragma unroll
        for (int m = 0; m < M; ++m) rb[k][m] = bload<S>(wb.r, o + gb[m]);
    };

    // u rows s-2..s+1, b rows s-1..s-3, residual rows s-1..s-3 and new
    // iterate rows s-3, s-4 at this thread's columns (step s, on entry)
    C um2[M], um1[M], u0[M], up1[M];
    C b1[M], b2[M], b3[M];
    C r1[M], r2[M], r3[M];
    C v1[M], v2[M];
    C acc[MC];
    double nacc = 0.0, bacc = 0.0;
    const int s0 = 2 * Y0 - 2, s1 = 2 * Y1 + 4;
    {
        // all prologue loads before the first wait
        SU pu[3][M];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int p = s0 - 1 + q;
            const unsigned o = wu.at(p, p >= 0 && p <= ulast);
#pragma unroll
            for (int m = 0; m < M; ++m) pu[q][m] = bload<SU>(wu.r, o + gu[m]);
        }
#pragma unroll
        for (int q = 0; q < PD; ++q) {
            issue_u(s0 + 2 + q, q);
            issue_b(s0 + q, q);
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            um2[m] = C(0);
            um1[m] = cvt<C>(pu[0][m]);
            u0[m] = cvt<C>(pu[1][m]);
            up1[m] = cvt<C>(pu[2][m]);
            b1[m] = b2[m] = b3[m] = C(0);
            r1[m] = r2[m] = r3[m] = C(0);
            v1[m] = v2[m] = C(0);
            uL[s0 & 1][li[m]] = u0[m];
        }
#pragma unroll
        for (int q = 0; q < MC; ++q) acc[q] = C(0);
    }

    auto step = [&](int s, auto kc) {
        constexpr int k = decltype(kc)::k;  // (s - s0) % UN
        __syncthreads();
        issue_u(s + 2 + PD, (k + PD) % RS);
        issue_b(s + PD, (k + PD) % RS);
        // residual of row s
        const bool sin = s >= 0 && s < n;
        const bool sown = s >= o0 && s < o1;
        C r0[M], b0[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const C* U = uL[s & 1];
            const int q = li[m];
            b0[m] = cvt<C>(rb[k % RS][m]);
            const C lap = C(4) * u0[m] - U[q - 1] - U[q + 1] - um1[m] - up1[m];
            const C r = (sin && col[m]) ? b0[m] - sA * lap : C(0);
            r0[m] = r;
            rL[s & 3][q] = r;
            if (NORM) {
                nacc += (sown && own[m]) ? (double)r * (double)r : 0.0;
                bacc += (sown && own[m]) ? (double)b0[m] * (double)b0[m] : 0.0;
            }
            if (ROUT)
                bstore<false>(static_cast<S>(r), wro.r,
                              wro.at(s, sown) + (own[m] ? gb[m] : kOob));
        }
        // new iterate of row s-2 (residual rows s-3, s-2, s-1)
        const int p = s - 2;
        const bool pin = p >= 0 && p < n;
        const unsigned ro = wo.at(p, p >= o0 && p < o1);
        C v0[M];
        {
            const C* R0 = rL[(s + 1) & 3];  // row s - 3
            const C* R1 = rL[(s + 2) & 3];  // row s - 2
            const C* R2 = rL[(s + 3) & 3];  // row s - 1
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int q = li[m];
                const C fc = R1[q - 1] + R1[q + 1] + r3[m] + r1[m];
                const C cn = R0[q - 1] + R0[q + 1] + R2[q - 1] + R2[q + 1];
                const C v = um2[m] + sW * (c0 * r2[m] + c1 * fc + c2 * cn);
                const S vs = static_cast<S>(v);
                bstore<NTS>(vs, wo.r, ro + (own[m] ? gb[m] : kOob));
                v0[m] = (pin && col[m]) ? cvt<C>(vs) : C(0);
                vL[p & 1][q] = v0[m];
            }
        }
        // residual of row s-3 at the new iterate (rows s-4, s-3, s-2)
        {
            const C* V = vL[(s + 1) & 1];  // row s - 3
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int q = li[m];
                const C lap = C(4) * v1[m] - V[q - 1] - V[q + 1] - v2[m] - v0[m];
                wL[(s + 1) & 1][q] = b3[m] - sA * lap;
            }
        }
        // restriction of row f = s-4 (written by the previous step)
        const int f = s - 4;
        if (f >= 2 * Y0 && f <= 2 * Y1) {
            const C* R = wL[f & 1];
            const unsigned rc = wbc.at(f / 2 - 1, true);
#pragma unroll
            for (int q = 0; q < MC; ++q) {
                const int c = cq[q];
                const C xs = C(0.5) * R[c] + C(0.25) * (R[c - 1] + R[c + 1]);
                if ((f & 1) == 0) {
                    if (f > 2 * Y0) {
                        acc[q] += C(0.25) * xs;
                        bstore<false>(static_cast<S>(acc[q]), wbc.r, rc + cgb[q]);
                    }
                    acc[q] = C(0.25) * xs;
                } else {
                    acc[q] += C(0.5) * xs;
                }
            }
        }
        // u of row s+1 for the next step's neighbours; shift the histories
#pragma unroll
        for (int m = 0; m < M; ++m) {
            uL[(s + 1) & 1][li[m]] = up1[m];
            um2[m] = um1[m];
            um1[m] = u0[m];
            u0[m] = up1[m];
            up1[m] = cvt<C>(ru[k % RS][m]);
            b3[m] = b2[m];
            b2[m] = b1[m];
            b1[m] = b0[m];
            r3[m] = r2[m];
            r2[m] = r1[m];
            r1[m] = r0[m];
            v2[m] = v1[m];
            v1[m] = v0[m];
        }
    };
    march<UN>(s0, s1, step);
    if (NORM) {
        const double sm = block_sum<NT>(nacc, red);
        if (t == 0) partials[(long)blockIdx.y * gridDim.x + blockIdx.x] = sm;
        if (bparts) {  // sum b^2 as well (||b|| of a solve, in its first cycle)
            __syncthreads();
            const double sb = block_sum<NT>(bacc, red);
            if (t == 0) bparts[(long)blockIdx.y * gridDim.x + blockIdx.x] = sb;
        }
    }
}

// ---------------------------------------------------------------------------
// Post-smoothing of one V(1,1) cycle fused with the pre-smoothing and the
// restriction of the next (2D): from the pre-smoothed iterate t and the
// coarse correction ec,
//   w  = t + pf P ec,  uo = w + sW K_c (b - sA L w)         (end of cycle k)
//   t2 = uo + sW K_c (b - sA L uo),  bc = R (b - sA L t2)    (cycle k + 1)
// and the norm variant sums (b - sA L uo)^2 over the owned nodes (the
// residual of u_{k+1}).  x strips march over rows through seven stages,
// each one or two rows behind the one it reads, with one barrier per row: at
// step s the interpolated iterate of row s, the first residual of row s-1,
// the new iterate of row s-3, its residual of row s-4, the next
// pre-smoothed iterate of row s-6, its residual of row s-7 and the
// restriction of row s-8.  u is loaded on the strip plus a ring of 5 (each
// stage is valid one column further in).  Stored values enter later stages
// as stored.  The coarse correction is read per lane (one or two coarse
// values per row pair, L2 hits) two row pairs ahead.
// ---------------------------------------------------------------------------
template <typename S, typename C, int TX, int NT, int PD, int UN, bool NTS, bool NORM>
__global__ void __launch_bounds__(NT)
k_psr2d(const S* __restrict__ t, const S* __restrict__ ec, const S* __restrict__ b,
        S* __restrict__ uo, S* __restrict__ t2, S* __restrict__ bc, int n, int nc,
        int tiles_x, int ychunk, int nchunks, C sA, C sW, C c0, C c1, C c2, C pf,
        double* __restrict__ partials) {
    constexpr int W = TX + 11;            // columns x0-5 .. x0+TX+5
    constexpr int M = (W + NT - 1) / NT;
    constexpr int LW = W + 2 + 65;        // one guard each side, scratch for idle lanes
    constexpr int HC = TX / 2;
    constexpr int MC = (HC + NT - 1) / NT;
    constexpr int RS = PD + 1;
    static_assert(TX % 2 == 0, "even strips");
    static_assert(UN % RS == 0 && UN % 4 == 0, "unroll covers the rings and the row pairs");
    __shared__ C wL[2][LW];   // interpolated iterate
    __shared__ C aL[4][LW];   // its residual
    __shared__ C kL[2][LW];   // new iterate u_{k+1}
    __shared__ C gL[4][LW];   // its residual
    __shared__ C oL[2][LW];   // next pre-smoothed iterate
    __shared__ C fL[2][LW];   // its residual
    __shared__ double red[NT / 64];

    const int total = tiles_x * nchunks;
    const int lg = xcd_remap(blockIdx.x, total);
    const int tx = lg % tiles_x, ch = lg / tiles_x;
    const long area = (long)n * n;
    t += (long)blockIdx.y * area;
    b += (long)blockIdx.y * area;
    uo += (long)blockIdx.y * area;
    t2 += (long)blockIdx.y * area;
    ec += (long)blockIdx.y * nc * nc;
    bc += (long)blockIdx.y * nc * nc;
    const int x0 = tx * TX;
    const int Y0 = ch * ychunk, Y1 = min(Y0 + ychunk, nc);
    const int o0 = 2 * Y0, o1 = Y1 == nc ? n : 2 * Y1;
    const int th = threadIdx.x;
    const int lane = th & 63;

    int li[M];
    unsigned gb[M], ca[M], cb[M];
    bool col[M], own[M], odd[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int j = th + m * NT;
        const bool inr = j < W;
        const int gx = x0 - 5 + j;
        col[m] = inr && gx >= 0 && gx < n;
        own[m] = col[m] && gx >= x0 && gx < x0 + TX;
        li[m] = inr ? j + 1 : W + 2 + lane;
        gb[m] = col[m] ? (unsigned)(gx * (int)sizeof(S)) : kOob;
        // linear interpolation in x: grid coordinate g = gx + 1; even g sits
        // on coarse node g/2 - 1, odd g between (g-1)/2 - 1 and (g+1)/2 - 1
        const int g = gx + 1;
        odd[m] = (g & 1) != 0;
        const int ia = odd[m] ? (g - 1) / 2 - 1 : g / 2 - 1;
        const int ib = odd[m] ? (g + 1) / 2 - 1 : ia;
        ca[m] = (inr && ia >= 0 && ia < nc && g >= 0) ? (unsigned)(ia * (int)sizeof(S)) : kOob;
        cb[m] = (inr && ib >= 0 && ib < nc && g >= 0) ? (unsigned)(ib * (int)sizeof(S)) : kOob;
    }
    int cq[MC];
    unsigned cgb[MC];
#pragma unroll
    for (int q = 0; q < MC; ++q) {
        const int i = th + q * NT;
        const bool ok = i < HC && x0 / 2 + i < nc;
        cq[q] = i < HC ? 2 * i + 7 : W + 2 + lane;  // local column 2 i + 6, guard + 1
        cgb[q] = ok ? (unsigned)((x0 / 2 + i) * (int)sizeof(S)) : kOob;
    }

    // rows any output depends on, and the windows holding them: fine rows
    // 2 Y0 - 5 .. tlast (every row read or written), coarse correction rows
    // Y0 - 3 .. clast, coarse right-hand side rows Y0 .. Y1 - 1
    const int tlast = min(n - 1, 2 * Y1 + 5), blast = min(n - 1, 2 * Y1 + 4);
    const int clast = min(nc - 1, Y1 + 2);
    const int f0 = max(0, 2 * Y0 - 5), c0r = max(0, Y0 - 3);
    const Win<S> wt(t, n, f0, tlast - f0 + 1), wb(b, n, f0, tlast - f0 + 1);
    const Win<S> wuo(uo, n, f0, tlast - f0 + 1), wt2(t2, n, f0, tlast - f0 + 1);
    const Win<S> wec(ec, nc, c0r, clast - c0r + 1), wbc(bc, nc, Y0, Y1 - Y0);
    S rt[RS][M], rb[RS][M], rca[2][M], rcb[2][M];
    auto issue_t = [&](int p, int k) {
        const unsigned o = wt.at(p, p >= 0 && p <= tlast);
#pragma unroll
        for (int m = 0; m < M; ++m) rt[k][m] = bload<S>(wt.r, o + gb[m]);
    };
    auto issue_b = [&](int p, int k) {
        const unsigned o = wb.at(p, p >= 0 && p <= blast);
#pragma unroll
        for (int m = 0; m < M; ++m) rb[k][m] = bload<S>(wb.r, o + gb[m]);
    };
    auto issue_c = [&](int Y, int k) {
        const unsigned o = wec.at(Y, Y >= 0 && Y <= clast);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            rca[k][m] = bload<S>(wec.r, o + ca[m]);
            rcb[k][m] = bload<S>(wec.r, o + cb[m]);
        }
    };
    // x-interpolated coarse value (the same sums as the interpolation operator)
    auto qx = [&](S a, S bb, int m) -> C {
        C q = cvt<C>(a);
        q += odd[m] ? cvt<C>(bb) : C(0);
        return (odd[m] ? C(0.5) : C(1)) * q;
    };

    // histories at this lane's columns, on entry to step s:
    //   w rows s-1..s-3, first residual rows s-2..s-4, u_{k+1} rows
    //   s-4..s-6, its residual rows s-5..s-7, t2 rows s-7, s-8, b rows
    //   s-1..s-7, and the x-interpolated coarse row of the last even row
    C w1[M], w2[M], w3[M], a1[M], a2[M], a3[M], k1[M], k2[M], k3[M];
    C g1[M], g2[M], g3[M], o1v[M], o2v[M], qprev[M];
    C bh[7][M];
    C acc[MC];
    double nacc = 0.0;
    const int s0 = 2 * Y0 - 5, s1 = 2 * Y1 + 8;
    {
        // coarse row Y0-3 (interpolation of row s0), row Y0-2 (first even
        // step), then the rolling prefetch
        S pa[M], pb[M];
        {
            const int Y = Y0 - 3;
            const unsigned o = wec.at(Y, Y >= 0 && Y <= clast);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                pa[m] = bload<S>(wec.r, o + ca[m]);
                pb[m] = bload<S>(wec.r, o + cb[m]);
            }
        }
        issue_c(Y0 - 2, 0);
#pragma unroll
        for (int q = 0; q < PD; ++q) {
            issue_t(s0 + q, q);
            issue_b(s0 + q, q);
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            qprev[m] = qx(pa[m], pb[m], m);
            w1[m] = w2[m] = w3[m] = a1[m] = a2[m] = a3[m] = C(0);
            k1[m] = k2[m] = k3[m] = g1[m] = g2[m] = g3[m] = o1v[m] = o2v[m] = C(0);
#pragma unroll
            for (int q = 0; q < 7; ++q) bh[q][m] = C(0);
        }
#pragma unroll
        for (int q = 0; q < MC; ++q) acc[q] = C(0);
        for (int i = th; i < LW; i += NT) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                wL[q][i] = kL[q][i] = oL[q][i] = fL[q][i] = C(0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) aL[q][i] = gL[q][i] = C(0);
        }
    }

    auto step = [&](int s, auto kc) {
        constexpr int k = decltype(kc)::k;  // (s - s0) % UN; s0 is odd
        __syncthreads();
        issue_t(s + PD, (k + PD) % RS);
        issue_b(s + PD, (k + PD) % RS);
        // odd s: coarse row (s+3)/2, consumed at the even step s+3
        if ((k & 1) == 0) issue_c((s + 3) / 2, ((k + 2) / 2) % 2);
        // interpolated iterate of row s
        const bool sin = s >= 0 && s < n;
        C w0[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            C pe;
            if ((k & 1) == 1) {  // s even: between coarse rows s/2 - 1 and s/2
                const C qn = qx(rca[((k - 1) / 2) % 2][m], rcb[((k - 1) / 2) % 2][m], m);
                pe = C(0.5) * (qprev[m] + qn);
                qprev[m] = qn;
            } else {             // s odd: on coarse row (s-1)/2
                pe = qprev[m];
            }
            const C v = cvt<C>(rt[k % RS][m]) + pf * pe;
            w0[m] = (sin && col[m]) ? v : C(0);
            wL[s & 1][li[m]] = w0[m];
        }
        // first residual of row s-1
        {
            const bool pin = s - 1 >= 0 && s - 1 < n;
            const C* Wr = wL[(s + 1) & 1];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int q = li[m];
                const C lap = C(4) * w1[m] - Wr[q - 1] - Wr[q + 1] - w2[m] - w0[m];
                const C r = (pin && col[m]) ? bh[0][m] - sA * lap : C(0);
                aL[(s + 3) & 3][q] = r;
                a3[m] = a2[m];
                a2[m] = a1[m];
                a1[m] = r;  // rows s-1, s-2, s-3 after this
            }
        }
        // new iterate of row s-3 (first residual rows s-4, s-3, s-2)
        C kn[M];
        {
            const int p = s - 3;
            const bool pin = p >= 0 && p < n;
            const C* R0 = aL[(s + 0) & 3];  // row s - 4
            const C* R1 = aL[(s + 1) & 3];  // row s - 3
            const C* R2 = aL[(s + 2) & 3];  // row s - 2
            const unsigned ro = wuo.at(p, p >= o0 && p < o1);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int q = li[m];
                // a1 = row s-1 now, a2 = s-2, a3 = s-3; row s-4 from LDS
                const C fc = R1[q - 1] + R1[q + 1] + R0[q] + a2[m];
                const C cn = R0[q - 1] + R0[q + 1] + R2[q - 1] + R2[q + 1];
                const C v = w3[m] + sW * (c0 * a3[m] + c1 * fc + c2 * cn);
                const S vs = static_cast<S>(v);
                bstore<NTS>(vs, wuo.r, ro + (own[m] ? gb[m] : kOob));
                kn[m] = (pin && col[m]) ? cvt<C>(vs) : C(0);
                kL[p & 1][q] = kn[m];
            }
        }
        // its residual, row s-4 (new iterate rows s-5, s-4, s-3)
        {
            const int p = s - 4;
            const bool pin = p >= 0 && p < n;
            const bool pown = p >= o0 && p < o1;
            const C* K = kL[p & 1];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int q = li[m];
                const C lap = C(4) * k1[m] - K[q - 1] - K[q + 1] - k2[m] - kn[m];
                const C r = (pin && col[m]) ? bh[3][m] - sA * lap : C(0);
                gL[p & 3][q] = r;
                if (NORM) nacc += (pown && own[m]) ? (double)r * (double)r : 0.0;
                g3[m] = g2[m];
                g2[m] = g1[m];
                g1[m] = r;  // rows s-4, s-5, s-6 after this
            }
        }
        // next pre-smoothed iterate of row s-6 (residual rows s-7, s-6, s-5)
        C on[M];
        {
            const int p = s - 6;
            const bool pin = p >= 0 && p < n;
            const C* Q0 = gL[(s + 1) & 3];  // row s - 7
            const C* Q1 = gL[(s + 2) & 3];  // row s - 6
            const C* Q2 = gL[(s + 3) & 3];  // row s - 5
            const unsigned ro = wt2.at(p, p >= o0 && p < o1);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int q = li[m];
                // g1 = row s-4, g2 = s-5, g3 = s-6; row s-7 from LDS
                const C fc = Q1[q - 1] + Q1[q + 1] + Q0[q] + g2[m];
                const C cn = Q0[q - 1] + Q0[q + 1] + Q2[q - 1] + Q2[q + 1];
                const C v = k3[m] + sW * (c0 * g3[m] + c1 * fc + c2 * cn);
                const S vs = static_cast<S>(v);
                bstore<NTS>(vs, wt2.r, ro + (own[m] ? gb[m] : kOob));
                on[m] = (pin && col[m]) ? cvt<C>(vs) : C(0);
                oL[p & 1][q] = on[m];
            }
        }
        // its residual, row s-7 (rows s-8, s-7, s-6)
        {
            const C* O = oL[(s + 1) & 1];  // row s - 7
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int q = li[m];
                const C lap = C(4) * o1v[m] - O[q - 1] - O[q + 1] - o2v[m] - on[m];
                fL[(s + 1) & 1][q] = bh[6][m] - sA * lap;
            }
        }
        // restriction of row f = s-8 (written by the previous step)
        const int f = s - 8;
        if (f >= 2 * Y0 && f <= 2 * Y1) {
            const C* R = fL[f & 1];
            const unsigned rc = wbc.at(f / 2 - 1, true);
#pragma unroll
            for (int q = 0; q < MC; ++q) {
                const int c = cq[q];
                const C xs = C(0.5) * R[c] + C(0.25) * (R[c - 1] + R[c + 1]);
                if ((f & 1) == 0) {
                    if (f > 2 * Y0) {
                        acc[q] += C(0.25) * xs;
                        bstore<false>(static_cast<S>(acc[q]), wbc.r, rc + cgb[q]);
                    }
                    acc[q] = C(0.25) * xs;
                } else {
                    acc[q] += C(0.5) * xs;
                }
            }
        }
        // shift the histories; b of row s enters
#pragma unroll
        for (int m = 0; m < M; ++m) {
            w3[m] = w2[m];
            w2[m] = w1[m];
            w1[m] = w0[m];
            k3[m] = k2[m];
            k2[m] = k1[m];
            k1[m] = kn[m];
            o2v[m] = o1v[m];
            o1v[m] = on[m];
#pragma unroll
            for (int q = 6; q > 0; --q) bh[q][m] = bh[q - 1][m];
            bh[0][m] = cvt<C>(rb[k % RS][m]);
        }
    };
    march<UN>(s0, s1, step);
    if (NORM) {
        const double sm = block_sum<NT>(nacc, red);
        if (th == 0) partials[(long)blockIdx.y * gridDim.x + blockIdx.x] = sm;
    }
}

// ---------------------------------------------------------------------------
// Pre-smoothing fused with the restriction (3D, any iterate):
// out = u + sW K_c (b - sA L u) and bc = R (b - sA L out).  A workgroup owns
// a TX x TY tile of fine columns and marches over planes; every lane keeps
// its points of the tile plus a ring of 3 (u there; the residual is valid on
// the ring of 2, the new iterate on the ring of 1, the second residual on
// the tile plus the row and column after it, where the coarse nodes'
// stencils reach).  The 7-point M and A couple planes only through the same
// column, so the stages lag by one plane each: at step s the residual of
// plane s, the new iterate of plane s-1, the second residual of plane s-2
// and the restriction of plane s-3, with one barrier per plane (in-plane
// neighbours from LDS, the planes above and below from registers).
// Residuals and iterates outside the grid are zero; the new iterate enters
// the second residual as stored.  The norm variant sums (b - sA L u)^2 over
// the owned nodes.
// ---------------------------------------------------------------------------
template <typename S, typename C, int TX, int TY, int NT, int PD, int UN, bool NTS, bool NORM,
          bool ROUT = false, typename SU = S>
__global__ void __launch_bounds__(NT)
k_sr3d(const SU* __restrict__ u, const S* __restrict__ b, S* __restrict__ out,
       S* __restrict__ bc, int n, int nc, int tiles_x, int tiles_y, int zchunk, int nchunks,
       C sA, C sW, C c0, C c1, double* __restrict__ partials, S* __restrict__ rout = nullptr,
       double* __restrict__ bparts = nullptr) {
    constexpr int WX = TX + 7, WY = TY + 7, NW = WX * WY;  // x0-3 .. x0+TX+3
    constexpr int M = (NW + NT - 1) / NT;
    constexpr int WP = WX + 1;                             // guard row of neighbours
    // FP64: idle lanes (past the window) write, and read around, slots of
    // their own (SCR + lane), so that no LDS write of the march needs an exec
    // mask (1% faster at n = 255); FP32/FP16 storage: idle lanes skip their
    // writes (3% faster at n = 511)
    constexpr bool SCRW = sizeof(S) == 8;
    constexpr int SCR = NW + 2 * WP + WX + 1;
    constexpr int LSZ = SCRW ? SCR + 64 + WX + 1 : NW + 2 * WP;
    constexpr int HX = TX / 2, HY = TY / 2, NCC = HX * HY;  // coarse columns per tile
    constexpr int MC = (NCC + NT - 1) / NT;
    constexpr int RS = PD + 1;
    static_assert(TX % 2 == 0 && TY % 2 == 0, "even tiles");
    static_assert(UN % RS == 0, "unroll covers the prefetch ring");
    __shared__ C uL[2][LSZ];
    __shared__ C rL[2][LSZ];
    __shared__ C vL[2][LSZ];
    __shared__ C wL[2][LSZ];
    __shared__ double red[NT / 64];

    const int total = tiles_x * tiles_y * nchunks;
    const int lg = xcd_remap(blockIdx.x, total);
    const int tx = lg % tiles_x, ty = (lg / tiles_x) % tiles_y,
              ch = lg / (tiles_x * tiles_y);
    const long plane = (long)n * n, cplane = (long)nc * nc;
    u += (long)blockIdx.y * plane * n;
    b += (long)blockIdx.y * plane * n;
    out += (long)blockIdx.y * plane * n;
    if (ROUT) rout += (long)blockIdx.y * plane * n;
    bc += (long)blockIdx.y * cplane * nc;
    const int x0 = tx * TX, y0 = ty * TY;
    const int Z0 = ch * zchunk, Z1 = min(Z0 + zchunk, nc);
    // fine planes owned: [2 Z0, 2 Z1), the last chunk up to n
    const int o0 = 2 * Z0, o1 = Z1 == nc ? n : 2 * Z1;
    const int t = threadIdx.x;

    int li[M];
    unsigned gb[M], gu[M];
    bool col[M], own[M], wr[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = t + m * NT;
        wr[m] = i < NW;
        const int lx = i % WX, ly = i / WX;
        const int gx = x0 - 3 + lx, gy = y0 - 3 + ly;
        col[m] = wr[m] && gx >= 0 && gx < n && gy >= 0 && gy < n;
        own[m] = col[m] && gx >= x0 && gx < x0 + TX && gy >= y0 && gy < y0 + TY;
        li[m] = wr[m] ? WP + i : (SCRW ? SCR + (t & 63) : WP);
        gb[m] = col[m] ? (unsigned)((gy * n + gx) * (int)sizeof(S)) : kOob;
        gu[m] = col[m] ? (unsigned)((gy * n + gx) * (int)sizeof(SU)) : kOob;
    }
    // coarse column (x0/2 + i, y0/2 + j) sits over window point (2i+4, 2j+4)
    int cq[MC];
    unsigned cgb[MC];
#pragma unroll
    for (int q = 0; q < MC; ++q) {
        const int k = t + q * NT;
        const int i = k % HX, j = k / HX;
        const bool ok = k < NCC && x0 / 2 + i < nc && y0 / 2 + j < nc;
        cq[q] = k < NCC ? WP + (2 * j + 4) * WX + 2 * i + 4 : WP + WX + 1;
        cgb[q] = ok ? (unsigned)(((y0 / 2 + j) * nc + x0 / 2 + i) * (int)sizeof(S)) : kOob;
    }

    // planes any output depends on: u up to 2 Z1 + 3, b up to 2 Z1 + 2 (as
    // in 2D, later planes read as zero without touching memory); one window
    // of fine planes 2 Z0 - 3 .. ulast serves every fine field
    const int ulast = min(n - 1, 2 * Z1 + 3), blast = min(n - 1, 2 * Z1 + 2);
    const int f0 = max(0, 2 * Z0 - 3), fcnt = ulast - f0 + 1;
    const Win<SU> wu(u, plane, f0, fcnt);
    const Win<S> wb(b, plane, f0, fcnt), wo(out, plane, f0, fcnt);
    const Win<S> wro(ROUT ? rout : out, plane, f0, fcnt), wbc(bc, cplane, Z0, Z1 - Z0);
    SU ru[RS][M];
    S rb[RS][M];
    auto issue_u = [&](int p, int k) {
        const unsigned o = wu.at(p, p >= 0 && p <= ulast);
#pragma unroll
        for (int m = 0; m < M; ++m) ru[k][m] = bload<SU>(wu.r, o + gu[m]);
    };
    auto issue_b = [&](int p, int k) {
        const unsigned o = wb.at(p, p >= 0 && p <= blast);
#pragma unroll
        for (int m = 0; m < M; ++m) rb[k][m] = bload<S>(wb.r, o + gb[m]);
    };

    // on entry to step s: u planes s-1..s+1, b planes s-1, s-2, residual
    // planes s-1, s-2 and new iterate planes s-2, s-3 at this lane's points
    C um1[M], u0[M], up1[M], b1[M], b2[M], r1[M], r2[M], v1[M], v2[M];
    C acc[MC];
    double nacc = 0.0, bacc = 0.0;
    const int s0 = 2 * Z0 - 2, s1 = 2 * Z1 + 3;
    {
        SU pu[3][M];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int p = s0 - 1 + q;
            const unsigned o = wu.at(p, p >= 0 && p <= ulast);
#pragma unroll
            for (int m = 0; m < M; ++m) pu[q][m] = bload<SU>(wu.r, o + gu[m]);
        }
#pragma unroll
        for (int q = 0; q < PD; ++q) {
            issue_u(s0 + 2 + q, q);
            issue_b(s0 + q, q);
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            um1[m] = cvt<C>(pu[0][m]);
            u0[m] = cvt<C>(pu[1][m]);
            up1[m] = cvt<C>(pu[2][m]);
            b1[m] = b2[m] = r1[m] = r2[m] = v1[m] = v2[m] = C(0);
            if (SCRW || wr[m]) uL[s0 & 1][li[m]] = u0[m];
        }
#pragma unroll
        for (int q = 0; q < MC; ++q) acc[q] = C(0);
        // the planes a first step reads before any step wrote them
        for (int i = t; i < LSZ; i += NT) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                rL[j][i] = C(0);
                vL[j][i] = C(0);
                wL[j][i] = C(0);
            }
        }
    }

    auto step = [&](int s, auto kc) {
        constexpr int k = decltype(kc)::k;  // (s - s0) % UN
        __syncthreads();
        issue_u(s + 2 + PD, (k + PD) % RS);
        issue_b(s + PD, (k + PD) % RS);
        // residual of plane s
        const bool sin = s >= 0 && s < n;
        const bool sown = s >= o0 && s < o1;
        C r0[M], b0[M];
        {
            const C* U = uL[s & 1];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int q = li[m];
                b0[m] = cvt<C>(rb[k % RS][m]);
                const C lap = C(6) * u0[m] - U[q - 1] - U[q + 1] - U[q - WX] - U[q + WX] -
                              um1[m] - up1[m];
                const C r = (sin && col[m]) ? b0[m] - sA * lap : C(0);
                r0[m] = r;
                if (SCRW || wr[m]) rL[s & 1][q] = r;
                if (NORM) {
                    nacc += (sown && own[m]) ? (double)r * (double)r : 0.0;
                    bacc += (sown && own[m]) ? (double)b0[m] * (double)b0[m] : 0.0;
                }
                if (ROUT)
                    bstore<false>(static_cast<S>(r), wro.r,
                                  wro.at(s, sown) + (own[m] ? gb[m] : kOob));
            }
        }
        // new iterate of plane s-1 (residual planes s-2, s-1, s)
        const int p = s - 1;
        const bool pin = p >= 0 && p < n;
        C v0[M];
        {
            const C* R = rL[(s + 1) & 1];  // plane s - 1
            const unsigned ro = wo.at(p, p >= o0 && p < o1);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int q = li[m];
                const C nbs = R[q - 1] + R[q + 1] + R[q - WX] + R[q + WX] + r2[m] + r0[m];
                const C v = um1[m] + sW * (c0 * r1[m] + c1 * nbs);
                const S vs = static_cast<S>(v);
                bstore<NTS>(vs, wo.r, ro + (own[m] ? gb[m] : kOob));
                v0[m] = (pin && col[m]) ? cvt<C>(vs) : C(0);
                if (SCRW || wr[m]) vL[p & 1][q] = v0[m];
            }
        }
        // residual of plane s-2 at the new iterate (planes s-3, s-2, s-1)
        {
            const C* V = vL[s & 1];  // plane s - 2
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int q = li[m];
                const C lap = C(6) * v1[m] - V[q - 1] - V[q + 1] - V[q - WX] - V[q + WX] -
                              v2[m] - v0[m];
                if (SCRW || wr[m]) wL[s & 1][q] = b2[m] - sA * lap;
            }
        }
        // restriction of plane f = s-3 (written by the previous step)
        const int f = s - 3;
        if (f >= 2 * Z0 && f <= 2 * Z1) {
            const C* R = wL[f & 1];
            const unsigned rc = wbc.at(f / 2 - 1, true);
#pragma unroll
            for (int q = 0; q < MC; ++q) {
                const int c = cq[q];
                const C xs = C(0.25) * R[c] +
                             C(0.125) * (R[c - 1] + R[c + 1] + R[c - WX] + R[c + WX]) +
                             C(0.0625) * (R[c - WX - 1] + R[c - WX + 1] + R[c + WX - 1] +
                                          R[c + WX + 1]);
                if ((f & 1) == 0) {
                    if (f > 2 * Z0) {
                        acc[q] += C(0.25) * xs;
                        bstore<false>(static_cast<S>(acc[q]), wbc.r, rc + cgb[q]);
                    }
                    acc[q] = C(0.25) * xs;
                } else {
                    acc[q] += C(0.5) * xs;
                }
            }
        }
        // u of plane s+1 for the next step's neighbours; shift the histories
#pragma unroll
        for (int m = 0; m < M; ++m) {
            if (SCRW || wr[m]) uL[(s + 1) & 1][li[m]] = up1[m];
            um1[m] = u0[m];
            u0[m] = up1[m];
            up1[m] = cvt<C>(ru[k % RS][m]);
            b2[m] = b1[m];
            b1[m] = b0[m];
            r2[m] = r1[m];
            r1[m] = r0[m];
            v2[m] = v1[m];
            v1[m] = v0[m];
        }
    };
    march<UN>(s0, s1, step);
    if (NORM) {
        const double sm = block_sum<NT>(nacc, red);
        if (t == 0) partials[(long)blockIdx.y * gridDim.x + blockIdx.x] = sm;
        if (bparts) {  // sum b^2 as well (||b|| of a solve, in its first cycle)
            __syncthreads();
            const double sb = block_sum<NT>(bacc, red);
            if (t == 0) bparts[(long)blockIdx.y * gridDim.x + blockIdx.x] = sb;
        }
    }
}

// ---------------------------------------------------------------------------
// Reverse-mode sweeps of the adjoint cycle as marches (FP64), one barrier
// per plane (row).  MODE 0, the reverse of a smoothing step u_out = u + M r
// (r = b - A u): w = sW K_c ubar on the tile plus a ring of 1 from ubar
// staged in LDS on the tile plus a ring of 2, the coefficient partials
// sW sum (K_j ubar) r over the owned nodes, then ubar_new = ubar - sA L w
// and bbar += w at the owned nodes, one plane (row) behind.  MODE 1, the
// reverse of the restriction of the residual: the same update with w =
// scale P bbar_c, the linear interpolation of the coarse field ec (scale =
// 2^-d gives R^T), gathered from L2 once per coarse plane (row) and node
// column and combined with the interpolation operator's weights.  ubar and
// w are zero outside the grid (zero extension).  Loads of plane (row) s+1
// are issued during step s.
// ---------------------------------------------------------------------------
template <int TX, int TY, int NT, bool WIDE, int MODE>
__global__ void __launch_bounds__(NT)
k_adj_sweep3d(const double* __restrict__ ub, const double* __restrict__ r,
              const double* __restrict__ ec, double* __restrict__ ub_new,
              double* __restrict__ bb, double* __restrict__ partials, int n, int tiles_x,
              int tiles_y, int zchunk, int nchunks, double sA, double sW, double c0, double c1,
              double c2, double c3, double scale) {
    constexpr int UX = TX + 4, UY = TY + 4, NU = UX * UY;  // ubar: tile + ring 2
    constexpr int RX = TX + 2, RY = TY + 2, NR = RX * RY;  // w: tile + ring 1
    constexpr int MU = (NU + NT - 1) / NT, MW = (NR + NT - 1) / NT;
    constexpr int UP = UX + 1, USZ = UP + MU * NT + UX + 1;  // guards for neighbour reads
    constexpr int WP = RX + 1, WSZ = WP + MW * NT + RX + 1;
    __shared__ double uL[MODE == 0 ? 4 : 1][MODE == 0 ? USZ : 1];
    __shared__ double wL[2][WSZ];
    __shared__ double red[NT / 64];

    const int total = tiles_x * tiles_y * nchunks;
    const int lg = xcd_remap(blockIdx.x, total);
    const int tx = lg % tiles_x, ty = (lg / tiles_x) % tiles_y, ch = lg / (tiles_x * tiles_y);
    const long plane = (long)n * n;
    const long boff = (long)blockIdx.y * plane * n;
    const int nc = (n + 1) / 2 - 1;
    const long cplane = (long)nc * nc;
    ub += boff;
    ub_new += boff;
    bb += boff;
    if (MODE == 0) r += boff;
    else ec += (long)blockIdx.y * cplane * nc;
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = ch * zchunk, z1 = min(z0 + zchunk, n);
    const int t = threadIdx.x;

    unsigned ugb[MU];
    int uli[MU];
#pragma unroll
    for (int m = 0; m < MU; ++m) {
        const int i = t + m * NT;
        const int gx = x0 - 2 + i % UX, gy = y0 - 2 + i / UX;
        const bool ok = i < NU && gx >= 0 && gx < n && gy >= 0 && gy < n;
        ugb[m] = ok ? (unsigned)((gy * n + gx) * 8) : kOob;
        uli[m] = UP + (i < NU ? i : NU);  // idle lanes write a guard slot
    }
    unsigned wgb[MW];
    int wq[MW], wuq[MW];
    bool wval[MW], own[MW];
#pragma unroll
    for (int m = 0; m < MW; ++m) {
        const int i = t + m * NT;
        const bool in = i < NR;
        const int lx = in ? i % RX : 0, ly = in ? i / RX : 0;  // idle lanes read a valid node
        const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        wval[m] = in && gx >= 0 && gx < n && gy >= 0 && gy < n;
        own[m] = wval[m] && lx >= 1 && lx <= TX && ly >= 1 && ly <= TY;
        wgb[m] = wval[m] ? (unsigned)((gy * n + gx) * 8) : kOob;
        wq[m] = WP + (in ? i : NR);
        wuq[m] = UP + (ly + 1) * UX + lx + 1;  // the same node in the ubar window
    }
    // MODE 1: the coarse nodes of each w node's interpolation in the plane:
    // grid coordinate g = gx + 1 lies on or between coarse nodes g/2 and
    // (g+1)/2 (interior indices one less; 0 and nc+1 are boundary nodes)
    unsigned cof[MW][4];
    if (MODE == 1) {
#pragma unroll
        for (int m = 0; m < MW; ++m) {
            const int i = t + m * NT;
            const bool in = i < NR;
            const int gx = x0 - 1 + (in ? i % RX : 0) + 1, gy = y0 - 1 + (in ? i / RX : 0) + 1;
            const int xa = gx / 2 - 1, xb = (gx + 1) / 2 - 1, ya = gy / 2 - 1, yb = (gy + 1) / 2 - 1;
            auto off = [&](int cx, int cy) -> unsigned {
                return (wval[m] && cx >= 0 && cx < nc && cy >= 0 && cy < nc)
                           ? (unsigned)((cy * nc + cx) * 8) : kOob;
            };
            cof[m][0] = off(xa, ya);
            cof[m][1] = off(xb, ya);
            cof[m][2] = off(xa, yb);
            cof[m][3] = off(xb, yb);
        }
    }

    // one buffer resource per field over the planes this march touches:
    // ubar from z0 - 2 to z1 + 3, the other fields inside that range; the
    // coarse planes up to z1 / 2
    const int wf0 = max(0, z0 - 2), wfl = min(n - 1, z1 + 3), wfc = wfl - wf0 + 1;
    const Win<double> wub(ub, plane, wf0, wfc), wrr(MODE == 0 ? r : ub, plane, wf0, wfc);
    const Win<double> wbb(bb, plane, wf0, wfc), wun(ub_new, plane, wf0, wfc);
    const int wc0 = max(0, ((z0 - 1) >> 1) - 1), wcl = min(nc - 1, z1 >> 1);
    const Win<double> wec(MODE == 1 ? ec : ub, cplane, wc0, wcl - wc0 + 1);
    auto ld_plane = [&](const Win<double>& w, int p, unsigned off) {
        return bload<double>(w.r, w.at(p, p >= 0 && p <= wfl) + off);
    };
    // the in-plane part of a w node's interpolation: the four coarse values
    // of coarse plane k around it (a node on a coarse line counts its value
    // twice).  Fine plane s (grid coordinate s + 1) lies between coarse
    // planes s/2 - 1 and s/2 when s is even and on plane (s - 1)/2 when s is
    // odd (counted twice), so each coarse plane is gathered once, at the even
    // step that first needs it, and serves three fine planes.
    auto bilin = [&](int k, int m) -> double {
        const unsigned o = wec.at(k, k >= 0 && k <= wcl);
        return bload<double>(wec.r, o + cof[m][0]) + bload<double>(wec.r, o + cof[m][1]) +
               bload<double>(wec.r, o + cof[m][2]) + bload<double>(wec.r, o + cof[m][3]);
    };
    // w of plane s at step s (s = z0-1 .. z1), outputs of plane s-1
    const int s0 = z0 - 1, s1 = z1;
    double pu[MU];
    if (MODE == 0) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int p = s0 - 1 + q;
#pragma unroll
            for (int m = 0; m < MU; ++m) uL[p & 3][uli[m]] = ld_plane(wub, p, ugb[m]);
        }
#pragma unroll
        for (int m = 0; m < MU; ++m) pu[m] = ld_plane(wub, s0 + 2, ugb[m]);
    }
    // per-step loads, one step ahead: r (MODE 0) of plane s, or (MODE 1) at
    // even s the in-plane interpolation of coarse plane s/2; ubar (MODE 1)
    // and bbar of plane s - 1
    double nr[MW], nw[MW], nu[MW], nb[MW];
    auto issue = [&](int s) {
        const int p = s - 1;
        const bool pout = p >= z0 && p < z1, sown = s >= z0 && s < z1;
#pragma unroll
        for (int m = 0; m < MW; ++m) {
            nr[m] = MODE == 0 ? ld_plane(wrr, s, sown && own[m] ? wgb[m] : kOob) : 0.0;
            if (MODE == 1 && (s & 1) == 0) nw[m] = bilin(s >> 1, m);
            nu[m] = MODE == 1 ? ld_plane(wub, p, pout && own[m] ? wgb[m] : kOob) : 0.0;
            nb[m] = ld_plane(wbb, p, pout && own[m] ? wgb[m] : kOob);
        }
    };
    // MODE 1: in-plane interpolations of the coarse planes below and above
    // (or on) the current fine plane; before the first step, the coarse
    // plane the first step needs besides the one it gathers itself
    double bpre[MW], bcur[MW];
#pragma unroll
    for (int m = 0; m < MW; ++m) {
        bpre[m] = 0.0;
        nw[m] = 0.0;
        bcur[m] = MODE == 1 ? bilin((s0 & 1) ? (s0 >> 1) : (s0 >> 1) - 1, m) : 0.0;
    }
    issue(s0);
    double wm1[MW], wm2[MW];
#pragma unroll
    for (int m = 0; m < MW; ++m) wm1[m] = wm2[m] = 0.0;
    for (int i = t; i < WSZ; i += NT) wL[0][i] = wL[1][i] = 0.0;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;

    for (int s = s0; s <= s1; ++s) {
        __syncthreads();
        double rv[MW], ws[MW], uo[MW], bo[MW];
#pragma unroll
        for (int m = 0; m < MW; ++m) {
            rv[m] = nr[m];
            if (MODE == 1) {
                if ((s & 1) == 0) {
                    bpre[m] = bcur[m];
                    bcur[m] = nw[m];
                    ws[m] = bpre[m] + bcur[m];
                } else {
                    ws[m] = bcur[m] + bcur[m];
                }
            }
            uo[m] = nu[m];
            bo[m] = nb[m];
        }
        if (s < s1) issue(s + 1);
        if (MODE == 0) {
#pragma unroll
            for (int m = 0; m < MU; ++m) uL[(s + 2) & 3][uli[m]] = pu[m];
#pragma unroll
            for (int m = 0; m < MU; ++m) pu[m] = ld_plane(wub, s + 3, ugb[m]);
        }
        const int p = s - 1;
        const bool pout = p >= z0 && p < z1;
        // w of plane s
        double w0[MW];
        const bool sin = s >= 0 && s < n, sown = s >= z0 && s < z1;
#pragma unroll
        for (int m = 0; m < MW; ++m) {
            double w = 0.0;
            if (MODE == 0) {
                const double* Um = uL[(s + 3) & 3];  // plane s - 1
                const double* U0 = uL[s & 3];
                const double* Up = uL[(s + 1) & 3];
                const int q = wuq[m];
                const double k0 = U0[q];
                const double k1 = U0[q - 1] + U0[q + 1] + U0[q - UX] + U0[q + UX] + Um[q] + Up[q];
                double k2 = 0.0, k3 = 0.0;
                if (WIDE) {
                    k2 = U0[q - UX - 1] + U0[q - UX + 1] + U0[q + UX - 1] + U0[q + UX + 1] +
                         Um[q - 1] + Um[q + 1] + Um[q - UX] + Um[q + UX] + Up[q - 1] + Up[q + 1] +
                         Up[q - UX] + Up[q + UX];
                    k3 = Um[q - UX - 1] + Um[q - UX + 1] + Um[q + UX - 1] + Um[q + UX + 1] +
                         Up[q - UX - 1] + Up[q - UX + 1] + Up[q + UX - 1] + Up[q + UX + 1];
                }
                w = sW * (c0 * k0 + c1 * k1 + c2 * k2 + c3 * k3);
                if (sown && own[m]) {
                    a0 += k0 * rv[m];
                    a1 += k1 * rv[m];
                    a2 += k2 * rv[m];
                    a3 += k3 * rv[m];
                }
            } else {
                w = scale * (0.125 * ws[m]);
            }
            w0[m] = (sin && wval[m]) ? w : 0.0;
            wL[s & 1][wq[m]] = w0[m];
        }
        // outputs of plane s - 1
        if (pout) {
            const double* W1 = wL[(s + 1) & 1];  // plane s - 1
            const unsigned oo = wun.at(p, true);  // the same offset in wbb
#pragma unroll
            for (int m = 0; m < MW; ++m) {
                const int q = wq[m];
                const double lw = 6.0 * wm1[m] - W1[q - 1] - W1[q + 1] - W1[q - RX] - W1[q + RX] -
                                  wm2[m] - w0[m];
                const double u = MODE == 0 ? uL[(s + 3) & 3][wuq[m]] : uo[m];
                bstore<false>(u - sA * lw, wun.r, oo + (own[m] ? wgb[m] : kOob));
                bstore<false>(bo[m] + wm1[m], wbb.r, oo + (own[m] ? wgb[m] : kOob));
            }
        }
#pragma unroll
        for (int m = 0; m < MW; ++m) {
            wm2[m] = wm1[m];
            wm1[m] = w0[m];
        }
    }
    if (MODE == 0) {
        // fixed-order block sums of the four coefficient partials
        const double s_0 = block_sum<NT>(a0, red);
        __syncthreads();
        const double s_1 = block_sum<NT>(a1, red);
        __syncthreads();
        const double s_2 = block_sum<NT>(a2, red);
        __syncthreads();
        const double s_3 = block_sum<NT>(a3, red);
        if (t == 0) {
            double* pp = partials + 4 * ((long)blockIdx.y * gridDim.x + blockIdx.x);
            pp[0] = sW * s_0;
            pp[1] = sW * s_1;
            pp[2] = sW * s_2;
            pp[3] = sW * s_3;
        }
    }
}

// 2D: x strips of TX outputs marching over rows; K_c is the 9-point stencil.
template <int TX, int NT, int MODE>
__global__ void __launch_bounds__(NT)
k_adj_sweep2d(const double* __restrict__ ub, const double* __restrict__ r,
              const double* __restrict__ ec, double* __restrict__ ub_new,
              double* __restrict__ bb, double* __restrict__ partials, int n, int tiles_x,
              int ychunk, int nchunks, double sA, double sW, double c0, double c1, double c2,
              double scale) {
    constexpr int UX = TX + 4, RX = TX + 2;
    constexpr int MU = (UX + NT - 1) / NT, MW = (RX + NT - 1) / NT;
    constexpr int USZ = 1 + MU * NT + 1, WSZ = 1 + MW * NT + 1;
    __shared__ double uL[MODE == 0 ? 4 : 1][MODE == 0 ? USZ : 1];
    __shared__ double wL[2][WSZ];
    __shared__ double red[NT / 64];

    const int total = tiles_x * nchunks;
    const int lg = xcd_remap(blockIdx.x, total);
    const int tx = lg % tiles_x, ch = lg / tiles_x;
    const long area = (long)n * n;
    const long boff = (long)blockIdx.y * area;
    const int nc = (n + 1) / 2 - 1;
    ub += boff;
    ub_new += boff;
    bb += boff;
    if (MODE == 0) r += boff;
    else ec += (long)blockIdx.y * nc * nc;
    const int x0 = tx * TX;
    const int z0 = ch * ychunk, z1 = min(z0 + ychunk, n);
    const int t = threadIdx.x;

    unsigned ugb[MU];
    int uli[MU];
#pragma unroll
    for (int m = 0; m < MU; ++m) {
        const int i = t + m * NT;
        const int gx = x0 - 2 + i;
        ugb[m] = (i < UX && gx >= 0 && gx < n) ? (unsigned)(gx * 8) : kOob;
        uli[m] = 1 + (i < UX ? i : UX);
    }
    unsigned wgb[MW];
    int wq[MW], wuq[MW];
    bool wval[MW], own[MW];
#pragma unroll
    for (int m = 0; m < MW; ++m) {
        const int i = t + m * NT;
        const bool in = i < RX;
        const int lx = in ? i : 0;
        const int gx = x0 - 1 + lx;
        wval[m] = in && gx >= 0 && gx < n;
        own[m] = wval[m] && lx >= 1 && lx <= TX;
        wgb[m] = wval[m] ? (unsigned)(gx * 8) : kOob;
        wq[m] = 1 + (in ? i : RX);
        wuq[m] = 1 + lx + 1;
    }
    // MODE 1: the coarse columns of each w node's interpolation
    unsigned cof[MW][2];
    if (MODE == 1) {
#pragma unroll
        for (int m = 0; m < MW; ++m) {
            const int i = t + m * NT;
            const int g = x0 - 1 + (i < RX ? i : 0) + 1;
            const int xa = g / 2 - 1, xb = (g + 1) / 2 - 1;
            cof[m][0] = (wval[m] && xa >= 0 && xa < nc) ? (unsigned)(xa * 8) : kOob;
            cof[m][1] = (wval[m] && xb >= 0 && xb < nc) ? (unsigned)(xb * 8) : kOob;
        }
    }
    // one buffer resource per field over the rows this march touches (as
    // in 3D)
    const int wf0 = max(0, z0 - 2), wfl = min(n - 1, z1 + 3), wfc = wfl - wf0 + 1;
    const Win<double> wub(ub, n, wf0, wfc), wrr(MODE == 0 ? r : ub, n, wf0, wfc);
    const Win<double> wbb(bb, n, wf0, wfc), wun(ub_new, n, wf0, wfc);
    const int wc0 = max(0, ((z0 - 1) >> 1) - 1), wcl = min(nc - 1, z1 >> 1);
    const Win<double> wec(MODE == 1 ? ec : ub, nc, wc0, wcl - wc0 + 1);
    auto ld_row = [&](const Win<double>& w, int p, unsigned off) {
        return bload<double>(w.r, w.at(p, p >= 0 && p <= wfl) + off);
    };
    // the x part of a w node's interpolation: the two coarse values of
    // coarse row k around it; each coarse row is gathered once, at the even
    // step that first needs it, and serves three fine rows (as in 3D)
    auto lin = [&](int k, int m) -> double {
        const unsigned o = wec.at(k, k >= 0 && k <= wcl);
        return bload<double>(wec.r, o + cof[m][0]) + bload<double>(wec.r, o + cof[m][1]);
    };
    const int s0 = z0 - 1, s1 = z1;
    double pu[MU];
    if (MODE == 0) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int p = s0 - 1 + q;
#pragma unroll
            for (int m = 0; m < MU; ++m) uL[p & 3][uli[m]] = ld_row(wub, p, ugb[m]);
        }
#pragma unroll
        for (int m = 0; m < MU; ++m) pu[m] = ld_row(wub, s0 + 2, ugb[m]);
    }
    double nr[MW], nw[MW], nu[MW], nb[MW];
    auto issue = [&](int s) {
        const int p = s - 1;
        const bool pout = p >= z0 && p < z1, sown = s >= z0 && s < z1;
#pragma unroll
        for (int m = 0; m < MW; ++m) {
            nr[m] = MODE == 0 ? ld_row(wrr, s, sown && own[m] ? wgb[m] : kOob) : 0.0;
            if (MODE == 1 && (s & 1) == 0) nw[m] = lin(s >> 1, m);
            nu[m] = MODE == 1 ? ld_row(wub, p, pout && own[m] ? wgb[m] : kOob) : 0.0;
            nb[m] = ld_row(wbb, p, pout && own[m] ? wgb[m] : kOob);
        }
    };
    double bpre[MW], bcur[MW];
#pragma unroll
    for (int m = 0; m < MW; ++m) {
        bpre[m] = 0.0;
        nw[m] = 0.0;
        bcur[m] = MODE == 1 ? lin((s0 & 1) ? (s0 >> 1) : (s0 >> 1) - 1, m) : 0.0;
    }
    issue(s0);
    double wm1[MW], wm2[MW];
#pragma unroll
    for (int m = 0; m < MW; ++m) wm1[m] = wm2[m] = 0.0;
    for (int i = t; i < WSZ; i += NT) wL[0][i] = wL[1][i] = 0.0;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;

    for (int s = s0; s <= s1; ++s) {
        __syncthreads();
        double rv[MW], ws[MW], uo[MW], bo[MW];
#pragma unroll
        for (int m = 0; m < MW; ++m) {
            rv[m] = nr[m];
            if (MODE == 1) {
                if ((s & 1) == 0) {
                    bpre[m] = bcur[m];
                    bcur[m] = nw[m];
                    ws[m] = bpre[m] + bcur[m];
                } else {
                    ws[m] = bcur[m] + bcur[m];
                }
            }
            uo[m] = nu[m];
            bo[m] = nb[m];
        }
        if (s < s1) issue(s + 1);
        if (MODE == 0) {
#pragma unroll
            for (int m = 0; m < MU; ++m) uL[(s + 2) & 3][uli[m]] = pu[m];
#pragma unroll
            for (int m = 0; m < MU; ++m) pu[m] = ld_row(wub, s + 3, ugb[m]);
        }
        const int p = s - 1;
        const bool pout = p >= z0 && p < z1;
        double w0[MW];
        const bool sin = s >= 0 && s < n, sown = s >= z0 && s < z1;
#pragma unroll
        for (int m = 0; m < MW; ++m) {
            double w = 0.0;
            if (MODE == 0) {
                const double* Um = uL[(s + 3) & 3];  // row s - 1
                const double* U0 = uL[s & 3];
                const double* Up = uL[(s + 1) & 3];
                const int q = wuq[m];
                const double k0 = U0[q];
                const double k1 = U0[q - 1] + U0[q + 1] + Um[q] + Up[q];
                const double k2 = Um[q - 1] + Um[q + 1] + Up[q - 1] + Up[q + 1];
                w = sW * (c0 * k0 + c1 * k1 + c2 * k2);
                if (sown && own[m]) {
                    a0 += k0 * rv[m];
                    a1 += k1 * rv[m];
                    a2 += k2 * rv[m];
                }
            } else {
                w = scale * (0.25 * ws[m]);
            }
            w0[m] = (sin && wval[m]) ? w : 0.0;
            wL[s & 1][wq[m]] = w0[m];
        }
        if (pout) {
            const double* W1 = wL[(s + 1) & 1];  // row s - 1
            const unsigned oo = wun.at(p, true);  // the same offset in wbb
#pragma unroll
            for (int m = 0; m < MW; ++m) {
                const int q = wq[m];
                const double lw = 4.0 * wm1[m] - W1[q - 1] - W1[q + 1] - wm2[m] - w0[m];
                const double u = MODE == 0 ? uL[(s + 3) & 3][wuq[m]] : uo[m];
                bstore<false>(u - sA * lw, wun.r, oo + (own[m] ? wgb[m] : kOob));
                bstore<false>(bo[m] + wm1[m], wbb.r, oo + (own[m] ? wgb[m] : kOob));
            }
        }
#pragma unroll
        for (int m = 0; m < MW; ++m) {
            wm2[m] = wm1[m];
            wm1[m] = w0[m];
        }
    }
    if (MODE == 0) {
        const double s_0 = block_sum<NT>(a0, red);
        __syncthreads();
        const double s_1 = block_sum<NT>(a1, red);
        __syncthreads();
        const double s_2 = block_sum<NT>(a2, red);
        if (t == 0) {
            double* pp = partials + 4 * ((long)blockIdx.y * gridDim.x + blockIdx.x);
            pp[0] = sW * s_0;
            pp[1] = sW * s_1;
            pp[2] = sW * s_2;
            pp[3] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// Coarse tail: every level from nt interior nodes per direction down to 3,
// the exact solve on the 3^d grid and back up, in one workgroup of 1024
// threads with all level arrays in LDS, as a V(1,1) cycle or (WC) wvisits
// W(1,0) visits of the top level.  Each level's first visit starts from a
// zero guess (pre-smoothing is e = sW K b).  Every LDS array carries a ring of
// zeros, so stencils need no bounds checks; threads map to nodes through
// power-of-two boxes (2D: 64 x 16 per pass, 3D: 16 x 16 x 4), so no
// divisions are needed.
// ---------------------------------------------------------------------------
__host__ __device__ inline int tail_levels(int nt) {
    int L = 1;
    for (int n = nt; n > 3; n = (n + 1) / 2 - 1) ++L;
    return L;
}

__host__ __device__ inline long tail_padded(int d, int n) {
    const long p = n + 2;
    return d == 3 ? p * p * p : p * p;
}

template <int D>
struct TailMap;
template <>
struct TailMap<2> {
    // lane -> x, wave -> row
    static __device__ __forceinline__ int x0() { return threadIdx.x & 63; }
    static __device__ __forceinline__ int y0() { return threadIdx.x >> 6; }
    static constexpr int YS = 16;
};
template <>
struct TailMap<3> {
    static __device__ __forceinline__ int x0() { return threadIdx.x & 15; }
    static __device__ __forceinline__ int y0() { return (threadIdx.x >> 4) & 15; }
    static __device__ __forceinline__ int z0() { return threadIdx.x >> 8; }
    static constexpr int ZS = 4;
};

// calls f(i, j, k) for every node of an n-grid owned by this thread
template <int D, typename F>
__device__ __forceinline__ void tail_for(int n, F&& f) {
    if (D == 2) {
        const int i = TailMap<2>::x0();
        if (i >= n) return;
        for (int j = TailMap<2>::y0(); j < n; j += TailMap<2>::YS) f(i, j, 0);
    } else {
        const int i = TailMap<3>::x0(), j = TailMap<3>::y0();
        if (i >= n || j >= n) return;
        for (int k = TailMap<3>::z0(); k < n; k += TailMap<3>::ZS) f(i, j, k);
    }
}

// byte offset of the FP64 coarsest-grid inverse behind the level arrays
__host__ __device__ inline size_t tail_ginv_offset(size_t level_bytes) {
    return (level_bytes + 7) & ~size_t(7);
}

// Compile-time geometry of a tail whose top level has 2^KT - 1 interior
// nodes per direction: level l (0 = top) has 2^(KT-l) - 1, down to 3 at
// l = KT - 2; arrays e, b, r of (n_l + 2)^D each, level after level.  With
// every size, pitch and offset a constant, a phase is a short straight-line
// stretch of code (the tail's phases are bound by their instruction count
// and latency, not by LDS bandwidth).
template <int D, int KT>
struct TailGeo {
    static constexpr int L = KT - 1;
    static constexpr int n(int l) { return (1 << (KT - l)) - 1; }
    static constexpr int P(int l) { return n(l) + 2; }
    static constexpr long pad(int l) {
        return D == 3 ? (long)P(l) * P(l) * P(l) : (long)P(l) * P(l);
    }
    static constexpr long base(int l) {
        long b = 0;
        for (int k = 0; k < l; ++k) b += 3 * pad(k);
        return b;
    }
};

template <typename S, typename C, int D, bool WC, int KT>
__global__ void __launch_bounds__(1024)
k_tail(const S* __restrict__ bt, S* __restrict__ et, C c0, C c1, C c2, C c3,
       const double* __restrict__ ginv, int scaled, int wvisits) {
    using G = TailGeo<D, KT>;
    constexpr int L = G::L, nt = G::n(0);
    extern __shared__ unsigned char smem_raw[];
    C* sm = reinterpret_cast<C*>(smem_raw);
    const int t = threadIdx.x;
    constexpr long tot = G::base(L);
    for (long q = t; q < tot; q += 1024) sm[q] = C(0);
    constexpr int m3 = D == 2 ? 9 : 27;
    double* gl = reinterpret_cast<double*>(smem_raw + tail_ginv_offset(tot * sizeof(C)));
    for (int q = t; q < m3 * m3; q += 1024) gl[q] = ginv[q];
    auto pidx = [&](int i, int j, int k, int P) -> int {
        return D == 3 ? ((k + 1) * P + j + 1) * P + i + 1 : (j + 1) * P + i + 1;
    };
    __syncthreads();
    {
        const long off = (long)blockIdx.x * (D == 3 ? (long)nt * nt * nt : (long)nt * nt);
        C* B = sm + G::pad(0);
        tail_for<D>(nt, [&](int i, int j, int k) {
            const long g = D == 3 ? ((long)k * nt + j) * nt + i : (long)j * nt + i;
            B[pidx(i, j, k, G::P(0))] = cvt<C>(bt[off + g]);
        });
    }
    __syncthreads();
    // sA = 1/(h_l^2 sigma_l), sW = h_l^2 sigma_l: N_l^2 and 1/N_l^2 (N_l =
    // 2^(KT - l)) unscaled, 1 for the scaled low-precision hierarchies
    auto level_consts = [&](auto lc, C* sA, C* sW) {
        constexpr int l = decltype(lc)::k;
        constexpr double N2 = (double)(1L << (2 * (KT - l)));
        *sA = scaled ? C(1) : C(N2);
        *sW = scaled ? C(1) : C(1.0 / N2);
    };
    const C pf = scaled ? C(4) : C(1);
    // stencils on a padded array at flat index q with pitches 1, P, P^2
    auto lap = [&](const C* a, int q, int P) -> C {
        C s = C(2 * D) * a[q] - a[q - 1] - a[q + 1] - a[q - P] - a[q + P];
        if (D == 3) s -= a[q - P * P] + a[q + P * P];
        return s;
    };
    // the 19-/27-point 3D stencils: edge and corner terms
    const bool wide = D == 3 && (c2 != C(0) || c3 != C(0));
    auto spai = [&](const C* a, int q, int P) -> C {
        C f = a[q - 1] + a[q + 1] + a[q - P] + a[q + P];
        if (D == 3) {
            const int P2 = P * P;
            f += a[q - P2] + a[q + P2];
            if (!wide) return c0 * a[q] + c1 * f;
            const C ed = a[q - P - 1] + a[q - P + 1] + a[q + P - 1] + a[q + P + 1] +
                         a[q - P2 - 1] + a[q - P2 + 1] + a[q - P2 - P] + a[q - P2 + P] +
                         a[q + P2 - 1] + a[q + P2 + 1] + a[q + P2 - P] + a[q + P2 + P];
            const C cn = a[q - P2 - P - 1] + a[q - P2 - P + 1] + a[q - P2 + P - 1] +
                         a[q - P2 + P + 1] + a[q + P2 - P - 1] + a[q + P2 - P + 1] +
                         a[q + P2 + P - 1] + a[q + P2 + P + 1];
            return c0 * a[q] + c1 * f + c2 * ed + c3 * cn;
        }
        const C cn = a[q - P - 1] + a[q - P + 1] + a[q + P - 1] + a[q + P + 1];
        return c0 * a[q] + c1 * f + c2 * cn;
    };
    // runs f over the nodes of an n-grid, then a workgroup barrier
    auto nodes = [&](int n, auto&& f) {
        tail_for<D>(n, f);
        __syncthreads();
    };
    // ---- phases on level l (each ends with a barrier)
    // zero-guess pre-smoothing: E = sW K B
    auto smooth_zero = [&](auto lc) {
        constexpr int l = decltype(lc)::k, n = G::n(l), P = G::P(l);
        C* E = sm + G::base(l);
        const C* B = E + G::pad(l);
        C sA, sW;
        level_consts(lc, &sA, &sW);
        nodes(n, [&](int i, int j, int k) {
            const int q = pidx(i, j, k, P);
            E[q] = sW * spai(B, q, P);
        });
    };
    // R = B - sA A E
    auto residual = [&](auto lc) {
        constexpr int l = decltype(lc)::k, n = G::n(l), P = G::P(l);
        const C* E = sm + G::base(l);
        const C* B = E + G::pad(l);
        C* R = sm + G::base(l) + 2 * G::pad(l);
        C sA, sW;
        level_consts(lc, &sA, &sW);
        nodes(n, [&](int i, int j, int k) {
            const int q = pidx(i, j, k, P);
            R[q] = B[q] - sA * lap(E, q, P);
        });
    };
    // E += sW K R (after residual)
    auto update = [&](auto lc) {
        constexpr int l = decltype(lc)::k, n = G::n(l), P = G::P(l);
        C* E = sm + G::base(l);
        const C* R = E + 2 * G::pad(l);
        C sA, sW;
        level_consts(lc, &sA, &sW);
        nodes(n, [&](int i, int j, int k) {
            const int q = pidx(i, j, k, P);
            E[q] += sW * spai(R, q, P);
        });
    };
    // B_{l+1} = full weighting of R_l
    auto restrict_r = [&](auto lc) {
        constexpr int l = decltype(lc)::k, P = G::P(l), nc = G::n(l + 1), Pc = G::P(l + 1);
        const C* R = sm + G::base(l) + 2 * G::pad(l);
        C* Bc = sm + G::base(l + 1) + G::pad(l + 1);
        nodes(nc, [&](int i, int j, int k) {
            const int q = pidx(2 * i + 1, 2 * j + 1, D == 3 ? 2 * k + 1 : 0, P);
            C s;
            if (D == 2) {
                s = C(0.25) * R[q] + C(0.125) * (R[q - 1] + R[q + 1] + R[q - P] + R[q + P]) +
                    C(0.0625) * (R[q - P - 1] + R[q - P + 1] + R[q + P - 1] + R[q + P + 1]);
            } else {
                constexpr int P2 = P * P;
                s = C(0);
                for (int oz = -1; oz <= 1; ++oz) {
                    const int qz = q + oz * P2;
                    const C pl = C(0.25) * R[qz] +
                                 C(0.125) * (R[qz - 1] + R[qz + 1] + R[qz - P] + R[qz + P]) +
                                 C(0.0625) * (R[qz - P - 1] + R[qz - P + 1] + R[qz + P - 1] +
                                              R[qz + P + 1]);
                    s += (oz == 0 ? C(0.5) : C(0.25)) * pl;
                }
            }
            Bc[pidx(i, j, k, Pc)] = s;
        });
    };
    // exact solve on the 3^d grid (level L-1) with the FP64 inverse
    auto exact = [&]() {
        constexpr int m = D == 2 ? 9 : 27, P = 5;
        C* E = sm + G::base(L - 1);
        const C* B = E + G::pad(L - 1);
        if (t < m) {
            const int i = t % 3, j = (t / 3) % 3, k = t / 9;
            double s = 0.0;
            for (int q = 0; q < m; ++q) {
                const int qi = q % 3, qj = (q / 3) % 3, qk = q / 9;
                s += gl[t * m + q] * (double)B[pidx(qi, qj, qk, P)];
            }
            E[pidx(i, j, k, P)] = C(s);
        }
        __syncthreads();
    };
    // E_l += pf P E_{l+1} (linear interpolation: fine node i, at grid
    // coordinate i+1, takes the coarse node (i+1)/2 if even, the mean of
    // (i/2, i/2+1) if odd; in padded coarse coordinates the coarse node G
    // sits at index G, and the ring supplies the zero boundary values)
    auto correct = [&](auto lc) {
        constexpr int l = decltype(lc)::k, n = G::n(l), P = G::P(l), Pc = G::P(l + 1);
        C* E = sm + G::base(l);
        const C* Ec = sm + G::base(l + 1);
        nodes(n, [&](int i, int j, int k) {
            const int gi = i + 1, gj = j + 1, gk = k + 1;
            const int ia = gi >> 1, ib = (gi + 1) >> 1;
            const int ja = gj >> 1, jb = (gj + 1) >> 1;
            C v;
            if (D == 2) {
                v = C(0.25) * (Ec[ja * Pc + ia] + Ec[ja * Pc + ib] + Ec[jb * Pc + ia] +
                               Ec[jb * Pc + ib]);
            } else {
                const int ka = gk >> 1, kb = (gk + 1) >> 1;
                constexpr int P2 = Pc * Pc;
                v = C(0.125) * (Ec[ka * P2 + ja * Pc + ia] + Ec[ka * P2 + ja * Pc + ib] +
                                Ec[ka * P2 + jb * Pc + ia] + Ec[ka * P2 + jb * Pc + ib] +
                                Ec[kb * P2 + ja * Pc + ia] + Ec[kb * P2 + ja * Pc + ib] +
                                Ec[kb * P2 + jb * Pc + ia] + Ec[kb * P2 + jb * Pc + ib]);
            }
            E[pidx(i, j, k, P)] += pf * v;
        });
    };

    if constexpr (!WC) {
        // V(1,1) from a zero guess: down through the levels, the exact solve,
        // back up, as compile-time recursion
        auto visit = [&](auto self, auto lc) -> void {
            constexpr int l = decltype(lc)::k;
            if constexpr (l == L - 1) {
                exact();
            } else {
                smooth_zero(lc);
                residual(lc);
                restrict_r(lc);
                self(self, Par<l + 1>{});
                correct(lc);
                residual(lc);
                update(lc);
            }
        };
        visit(visit, Par<0>{});
    } else {
        // W(1,0): each visit of level l < L-1 pre-smooths (from zero on a
        // level's first visit, from its current E on the second), restricts,
        // visits level l+1 twice and adds the interpolated correction.  A
        // second visit of the 3^d grid repeats an exact solve of unchanged
        // data and is skipped.  The top level is visited wvisits times.  The
        // visit order is compile-time recursion; `first` is uniform.
        auto visit = [&](auto self, auto lc, bool first) -> void {
            constexpr int l = decltype(lc)::k;
            if constexpr (l == L - 1) {
                if (first) exact();
            } else {
                if (first) {
                    smooth_zero(lc);
                } else {
                    residual(lc);
                    update(lc);
                }
                residual(lc);
                restrict_r(lc);
                self(self, Par<l + 1>{}, true);
                self(self, Par<l + 1>{}, false);
                correct(lc);
            }
        };
        visit(visit, Par<0>{}, true);
        if (wvisits > 1) visit(visit, Par<0>{}, false);
    }
    __syncthreads();
    {
        const long off = (long)blockIdx.x * (D == 3 ? (long)nt * nt * nt : (long)nt * nt);
        const C* E = sm;
        tail_for<D>(nt, [&](int i, int j, int k) {
            const long g = D == 3 ? ((long)k * nt + j) * nt + i : (long)j * nt + i;
            et[off + g] = static_cast<S>(E[pidx(i, j, k, G::P(0))]);
        });
    }
}

// ---------------------------------------------------------------------------
// Norm finalisation in a fixed order (deterministic run to run).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_finalize(const double* __restrict__ ps, const double* __restrict__ pm, int count,
           double* __restrict__ out, double* __restrict__ host) {
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
        const double nrm = sqrt(tot);
        out[0] = nrm;
        if (pm) out[1] = tmx;
        if (host) store_host_norm(host, nrm);
    }
}

// Sum of squares of a vector as per-block partials: block i owns the i-th
// contiguous chunk and its lanes stride through it, then a fixed shuffle
// tree, so the result is the same run to run.  (||b||_2 of a solve.)
__global__ void __launch_bounds__(256)
k_sumsq(const double* __restrict__ v, long count, long per, double* __restrict__ partials) {
    __shared__ double red[4];
    const long a = (long)blockIdx.x * per, e = min(count, a + per);
    double s0 = 0.0, s1 = 0.0;
    long i = a + threadIdx.x;
    for (; i + 256 < e; i += 512) {
        const double x = v[i], y = v[i + 256];
        s0 += x * x;
        s1 += y * y;
    }
    if (i < e) s0 += v[i] * v[i];
    const double tot = block_sum<256>(s0 + s1, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// ---------------------------------------------------------------------------
// FP64 refinement step, 3D: unew = u + escale * e (on the fly, halo included),
// r = b - A unew, r_lo = s * r (stored in S), partials of r^2 and max |r|.
// Without a correction (the first step) unew equals u and is not stored.
// Same scheme as the smoothers: per-field plane windows (e reads as zero when
// there is no correction yet), an unrolled marching loop over planes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double ir_scale(const double* maxprev) {
    const double m = maxprev[0];
    if (!(m > 0.0) || !isfinite(m)) return 1.0;
    int e;
    frexp(m, &e);           // m = f 2^e with f in [0.5, 1)
    return ldexp(1.0, -e);  // s m in [0.5, 1)
}

// RES: residual norm only (no e, no stores, no scale): the initial residual
// pass of a solve and mg_residual_norm
template <typename S, int TX, int TY, int NT, int UN, bool NTS, bool RES>
__global__ void __launch_bounds__(NT)
k_ir3d(const double* __restrict__ u, double* __restrict__ unew, const S* __restrict__ e,
       const double* __restrict__ b, S* __restrict__ rlo, int n, int tiles_x, int tiles_y,
       int zchunk, int nchunks, double inv_h2, double sigma0, int k,
       double* __restrict__ scales, const double* __restrict__ maxprev,
       double* __restrict__ psum, double* __restrict__ pmax, double* __restrict__ bparts) {
    constexpr int RX = TX + 2, RY = TY + 2, NR = RX * RY;
    constexpr int M = (NR + NT - 1) / NT;
    constexpr int RP = RX + 1, RSZ = RP + M * NT + RX + 1;
    constexpr int RS = 2;
    static_assert(UN % 2 == 0, "unroll covers the prefetch ring");
    __shared__ double uL[2][RSZ];
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
    const bool hase = !RES && e != nullptr && k > 0;
    if (hase) e += boff;
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = ch * zchunk, z1 = min(z0 + zchunk, n);
    const int t = threadIdx.x;
    const double s_new = RES ? 1.0 : ir_scale(maxprev);
    if (!RES && blockIdx.x == 0 && blockIdx.y == 0 && t == 0) scales[k] = s_new;
    const double escale = hase ? 1.0 / (sigma0 * scales[k - 1]) : 0.0;

    unsigned gu[M], ge[M], gi[M];  // byte offsets: u (ring), e (ring), interior
    bool inn[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = t + m * NT;
        const int lx = i % RX, ly = i / RX;
        const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        const bool val = i < NR && gx >= 0 && gx < n && gy >= 0 && gy < n;
        inn[m] = val && lx >= 1 && lx <= TX && ly >= 1 && ly <= TY;
        const int g = gy * n + gx;
        gu[m] = val ? (unsigned)(g * 8) : kOob;
        ge[m] = val ? (unsigned)(g * (int)sizeof(S)) : kOob;
        gi[m] = inn[m] ? (unsigned)(g * 8) : kOob;
    }
    // planes z0 - 1 .. z1 of u (and e) feed the residuals of planes z0 ..
    // z1 - 1, b up to z1 - 1 (later planes read as zero); one window per field
    const int ulast = min(n - 1, z1), blast = z1 - 1;
    const int w0 = max(0, z0 - 1), wcnt = ulast - w0 + 1;
    const Win<double> wu(u, plane, w0, wcnt), wb(b, plane, w0, wcnt);
    const Win<double> wn(RES ? u : unew, plane, w0, wcnt);
    const Win<S> we(hase ? e : rlo, plane, w0, wcnt), wr(rlo, plane, w0, wcnt);
    double ru[RS][M], rb[RS][M];
    S re[RS][M];
    auto issue = [&](int p, int q) {
        const bool pin = p >= 0 && p <= ulast;
        const unsigned oa = wu.at(p, pin), oc = we.at(p, pin && hase);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            ru[q][m] = bload<double>(wu.r, oa + gu[m]);
            re[q][m] = bload<S>(we.r, oc + ge[m]);
        }
    };
    auto issue_b = [&](int p, int q) {
        const unsigned o = wb.at(p, p >= 0 && p <= blast);
#pragma unroll
        for (int m = 0; m < M; ++m) rb[q][m] = bload<double>(wb.r, o + gi[m]);
    };
    auto take = [&](double* dst, const double* raw, const S* rawe) {
#pragma unroll
        for (int m = 0; m < M; ++m) dst[m] = raw[m] + escale * (double)rawe[m];
    };
    double um1[M], u0[M], up1[M];
    double acc = 0.0, mx = 0.0, bacc = 0.0;  // bacc: b^2, kept only with bparts
    {
        // all prologue loads before the first wait
        issue_b(z0, 0);
        double pu[3][M];
        S pe[3][M];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int p = z0 - 1 + q;
            const bool pin = p >= 0 && p <= ulast;
            const unsigned oa = wu.at(p, pin), oc = we.at(p, pin && hase);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                pu[q][m] = bload<double>(wu.r, oa + gu[m]);
                pe[q][m] = bload<S>(we.r, oc + ge[m]);
            }
        }
        take(um1, pu[0], pe[0]);
        take(u0, pu[1], pe[1]);
        take(up1, pu[2], pe[2]);
        issue(z0 + 2, 0);
#pragma unroll
        for (int m = 0; m < M; ++m) uL[z0 & 1][RP + t + m * NT] = u0[m];
    }
    auto step = [&](int s, auto kc) {
        constexpr int k = decltype(kc)::k;  // (s - z0) % UN
        __syncthreads();
        const int cur = s & 1;
        issue(s + 3, (k + 1) % RS);
        issue_b(s + 1, (k + 1) % RS);
        if (s < z1) {
            const double* U = uL[cur];
            const unsigned ow = wn.at(s, hase), orl = wr.at(s, true);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int q = RP + t + m * NT;
                const double lap = 6.0 * u0[m] - U[q - 1] - U[q + 1] - U[q - RX] - U[q + RX] -
                                   um1[m] - up1[m];
                const double r = rb[k % RS][m] - inv_h2 * lap;
                if (!RES) {
                    bstore<NTS>(u0[m], wn.r, ow + gi[m]);
                    bstore<NTS>(static_cast<S>(s_new * r), wr.r, orl + (inn[m] ? ge[m] : kOob));
                }
                acc += inn[m] ? r * r : 0.0;
                bacc += inn[m] ? rb[k % RS][m] * rb[k % RS][m] : 0.0;
                mx = fmax(mx, inn[m] ? fabs(r) : 0.0);
            }
        }
#pragma unroll
        for (int m = 0; m < M; ++m) uL[cur ^ 1][RP + t + m * NT] = up1[m];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            um1[m] = u0[m];
            u0[m] = up1[m];
        }
        take(up1, ru[k % RS], re[k % RS]);
    };
    march<UN>(z0, z1 - 1, step);
    const double ts = block_sum<NT>(acc, red);
    __syncthreads();
    const double tm = block_max<NT>(mx, red);
    if (t == 0) {
        const long pi = (long)blockIdx.y * gridDim.x + blockIdx.x;
        psum[pi] = ts;
        pmax[pi] = tm;
    }
    if (bparts) {  // sum b^2 as well (||b|| of a solve, in its first pass over b)
        __syncthreads();
        const double sb = block_sum<NT>(bacc, red);
        if (t == 0) bparts[(long)blockIdx.y * gridDim.x + blockIdx.x] = sb;
    }
}

template <typename S, int TX, int NT, int UN, bool NTS, bool RES>
__global__ void __launch_bounds__(NT)
k_ir2d(const double* __restrict__ u, double* __restrict__ unew, const S* __restrict__ e,
       const double* __restrict__ b, S* __restrict__ rlo, int n, int tiles_x, int ychunk,
       int nchunks, double inv_h2, double sigma0, int k, double* __restrict__ scales,
       const double* __restrict__ maxprev, double* __restrict__ psum,
       double* __restrict__ pmax, double* __restrict__ bparts) {
    constexpr int RX = TX + 2;
    constexpr int M = (RX + NT - 1) / NT;
    constexpr int RSZ = M * NT + 2;
    constexpr int RS = 2;
    static_assert(UN % 2 == 0, "unroll covers the prefetch ring");
    __shared__ double uL[2][RSZ];
    __shared__ double red[NT / 64];
    const int total = tiles_x * nchunks;
    const int lg = xcd_remap(blockIdx.x, total);
    const int tx = lg % tiles_x, ch = lg / tiles_x;
    const long area = (long)n * n, boff = (long)blockIdx.y * area;
    u += boff;
    unew += boff;
    b += boff;
    rlo += boff;
    const bool hase = !RES && e != nullptr && k > 0;
    if (hase) e += boff;
    const int x0 = tx * TX;
    const int y0 = ch * ychunk, y1 = min(y0 + ychunk, n);
    const int t = threadIdx.x;
    const double s_new = RES ? 1.0 : ir_scale(maxprev);
    if (!RES && blockIdx.x == 0 && blockIdx.y == 0 && t == 0) scales[k] = s_new;
    const double escale = hase ? 1.0 / (sigma0 * scales[k - 1]) : 0.0;
    unsigned gu[M], ge[M], gi[M];
    bool inn[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = t + m * NT;
        const int gx = x0 - 1 + i;
        const bool val = i < RX && gx >= 0 && gx < n;
        inn[m] = val && i >= 1 && i <= TX;
        gu[m] = val ? (unsigned)(gx * 8) : kOob;
        ge[m] = val ? (unsigned)(gx * (int)sizeof(S)) : kOob;
        gi[m] = inn[m] ? (unsigned)(gx * 8) : kOob;
    }
    // rows y0 - 1 .. y1 of u (and e) feed the residuals of rows y0 .. y1 - 1,
    // b up to y1 - 1 (later rows read as zero); one window per field
    const int ulast = min(n - 1, y1), blast = y1 - 1;
    const int w0 = max(0, y0 - 1), wcnt = ulast - w0 + 1;
    const Win<double> wu(u, n, w0, wcnt), wb(b, n, w0, wcnt), wn(RES ? u : unew, n, w0, wcnt);
    const Win<S> we(hase ? e : rlo, n, w0, wcnt), wr(rlo, n, w0, wcnt);
    double ru[RS][M], rb[RS][M];
    S re[RS][M];
    auto issue = [&](int p, int q) {
        const bool pin = p >= 0 && p <= ulast;
        const unsigned oa = wu.at(p, pin), oc = we.at(p, pin && hase);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            ru[q][m] = bload<double>(wu.r, oa + gu[m]);
            re[q][m] = bload<S>(we.r, oc + ge[m]);
        }
    };
    auto issue_b = [&](int p, int q) {
        const unsigned o = wb.at(p, p >= 0 && p <= blast);
#pragma unroll
        for (int m = 0; m < M; ++m) rb[q][m] = bload<double>(wb.r, o + gi[m]);
    };
    auto take = [&](double* dst, const double* raw, const S* rawe) {
#pragma unroll
        for (int m = 0; m < M; ++m) dst[m] = raw[m] + escale * (double)rawe[m];
    };
    double um1[M], u0[M], up1[M];
    double acc = 0.0, mx = 0.0, bacc = 0.0;  // bacc: b^2, kept only with bparts
    {
        issue_b(y0, 0);
        double pu[3][M];
        S pe[3][M];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int p = y0 - 1 + q;
            const bool pin = p >= 0 && p <= ulast;
            const unsigned oa = wu.at(p, pin), oc = we.at(p, pin && hase);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                pu[q][m] = bload<double>(wu.r, oa + gu[m]);
                pe[q][m] = bload<S>(we.r, oc + ge[m]);
            }
        }
        take(um1, pu[0], pe[0]);
        take(u0, pu[1], pe[1]);
        take(up1, pu[2], pe[2]);
        issue(y0 + 2, 0);
#pragma unroll
        for (int m = 0; m < M; ++m) uL[y0 & 1][1 + t + m * NT] = u0[m];
    }
    auto step = [&](int s, auto kc) {
        constexpr int k = decltype(kc)::k;  // (s - y0) % UN
        __syncthreads();
        const int cur = s & 1;
        issue(s + 3, (k + 1) % RS);
        issue_b(s + 1, (k + 1) % RS);
        if (s < y1) {
            const double* U = uL[cur];
            const unsigned ow = wn.at(s, hase), orl = wr.at(s, true);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int q = 1 + t + m * NT;
                const double lap = 4.0 * u0[m] - U[q - 1] - U[q + 1] - um1[m] - up1[m];
                const double r = rb[k % RS][m] - inv_h2 * lap;
                if (!RES) {
                    bstore<NTS>(u0[m], wn.r, ow + gi[m]);
                    bstore<NTS>(static_cast<S>(s_new * r), wr.r, orl + (inn[m] ? ge[m] : kOob));
                }
                acc += inn[m] ? r * r : 0.0;
                bacc += inn[m] ? rb[k % RS][m] * rb[k % RS][m] : 0.0;
                mx = fmax(mx, inn[m] ? fabs(r) : 0.0);
            }
        }
#pragma unroll
        for (int m = 0; m < M; ++m) uL[cur ^ 1][1 + t + m * NT] = up1[m];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            um1[m] = u0[m];
            u0[m] = up1[m];
        }
        take(up1, ru[k % RS], re[k % RS]);
    };
    march<UN>(y0, y1 - 1, step);
    const double ts = block_sum<NT>(acc, red);
    __syncthreads();
    const double tm = block_max<NT>(mx, red);
    if (t == 0) {
        const long pi = (long)blockIdx.y * gridDim.x + blockIdx.x;
        psum[pi] = ts;
        pmax[pi] = tm;
    }
    if (bparts) {  // sum b^2 as well (||b|| of a solve, in its first pass over b)
        __syncthreads();
        const double sb = block_sum<NT>(bacc, red);
        if (t == 0) bparts[(long)blockIdx.y * gridDim.x + blockIdx.x] = sb;
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

// the fused-correction sweep assumes every chunk starts on an even plane
inline int even_chunk(int c) { return c + (c & 1); }

// chunk c capped so that a window of per * c + extra lines of line_bytes
// each stays within kWinMax bytes; 0 when not even one chunk line fits
inline int win_chunk(int c, long line_bytes, int per, int extra) {
    const long cap = (kWinMax / line_bytes - extra) / per;
    return (int)std::max(0L, std::min((long)c, cap));
}

// Launch configurations of the marching sweeps by grid size, measured on
// MI355X in FP64 (the same shapes serve FP32/FP16 storage unless noted).  `want` is the
// number of marches (workgroups) per batch entry: one long march per CU on
// large grids, where halo planes cost bandwidth, more and shorter ones on
// smaller grids, where latency dominates.
//   smoother 3D  n >= 200: 64x16 tiles / 640 threads, unrolled 6, 256 marches
//                (FP32/FP16 storage: 256x8 / 1024, 1024 marches: 4- and 2-byte
//                rows need long row segments)
//                n >= 100: 32x16 / 320, 512 marches;  else 32x16 / 320, 256
//   smoother 2D  n >= 3000: 1024-wide strips / 576 threads, unrolled 4, 256
//                n >= 1500: 512 / 320, 512 marches;  n >= 700: 256 / 320, 512;
//                else 128 / 192, 512
//   restriction  3D n >= 200: 32x8 coarse columns / 576, unrolled 6, 256
//                (FP32/FP16: 64x8 / 768, 512);
//                else 32x4 / 320, 512;  2D n >= 3000: 512 / 576, unrolled 6,
//                256; n >= 700: 256 / 320, 512; else 128 / 192, 512
template <typename S, typename C, int TX, int TY, int NT, int UN, bool NTS>
hipError_t launch_smooth3d(bool zg, bool norm, const Sweep& s, int want, int minc,
                           hipStream_t st, int* nparts) {
    if (s.u_f32) return hipErrorInvalidValue;  // FP32 input: fused pre-smoother only
    const int n = s.n, nc = (n + 1) / 2 - 1;
    const S* u = static_cast<const S*>(s.u);
    const S* b = static_cast<const S*>(s.b);
    S* out = static_cast<S*>(s.out);
    const S* ec = static_cast<const S*>(s.ec);
    const bool pro = ec != nullptr;
    const C sA = C(s.sA), sW = C(s.sW), c0 = C(s.c[0]), c1 = C(s.c[1]), pf = C(s.pf);
    const C c2 = C(s.c[2]), c3 = C(s.c[3]);
    const int tx = cdiv(n, TX), ty = cdiv(n, TY);
    // a chunk's window of zc + 4 planes stays within kWinMax bytes
    const long zcap = min((long)n + 1, kWinMax / ((long)n * n * (long)sizeof(S)) - 4) & ~1L;
    if (zcap < 2) return hipErrorInvalidValue;
    const int zc = min(even_chunk(pick_chunk(n, tx * ty, want, minc)), (int)zcap);
    const int nch = cdiv(n, zc);
    dim3 grid(tx * ty * nch, s.batch);
    if (nparts) *nparts = grid.x * grid.y;
    if (norm && (long)grid.x * grid.y > s.partials_cap) return hipErrorInvalidValue;
    constexpr int PDC = UN % 3 == 0 ? 2 : 1;  // deeper prefetch for the fused correction
#define L3(PD, ZG, NM, PR, WD)                                                                 \
    mg_launch((k_smooth3d<S, C, TX, TY, NT, PD, UN, ZG, NM, PR, NTS, WD>), grid,       \
                       dim3(NT), 0, st, u, b, out, n, tx, ty, zc, nch, sA, sW, c0, c1,         \
                       s.partials, ec, nc, pf, c2, c3, static_cast<S*>(nullptr))
#define L3R(PD, PR, WD)                                                                        \
    mg_launch((k_smooth3d<S, C, TX, TY, NT, PD, UN, false, false, PR, NTS, WD, true>), \
                       grid, dim3(NT), 0, st, u, b, out, n, tx, ty, zc, nch, sA, sW, c0, c1,  \
                       s.partials, ec, nc, pf, c2, c3, static_cast<S*>(s.rout))
    if constexpr (sizeof(S) == 8) {
        if (s.rout) {  // residual side output (from a guess, or with the correction)
            if (zg || norm) return hipErrorInvalidValue;
            const bool wide = s.c[2] != 0.0 || s.c[3] != 0.0;
            if (pro && wide) L3R(PDC, true, true);
            else if (pro) L3R(PDC, true, false);
            else if (wide) L3R(1, false, true);
            else L3R(1, false, false);
            return hipGetLastError();
        }
    }
#undef L3R
    if (s.c[2] != 0.0 || s.c[3] != 0.0) {  // 19-/27-point stencil
        if (zg) L3(1, true, false, false, true);
        else if (norm) L3(1, false, true, false, true);
        else if (pro) L3(PDC, false, false, true, true);
        else L3(1, false, false, false, true);
    } else {
        if (zg) L3(1, true, false, false, false);
        else if (norm) L3(1, false, true, false, false);
        else if (pro) L3(PDC, false, false, true, false);
        else L3(1, false, false, false, false);
    }
#undef L3
    return hipGetLastError();
}

template <typename S, typename C, int TX, int NT, int UN, bool NTS>
hipError_t launch_smooth2d(bool zg, bool norm, const Sweep& s, int want, int minc,
                           hipStream_t st, int* nparts) {
    if (s.u_f32) return hipErrorInvalidValue;  // FP32 input: fused pre-smoother only
    const int n = s.n, nc = (n + 1) / 2 - 1;
    const S* u = static_cast<const S*>(s.u);
    const S* b = static_cast<const S*>(s.b);
    S* out = static_cast<S*>(s.out);
    const S* ec = static_cast<const S*>(s.ec);
    const bool pro = ec != nullptr;
    const C sA = C(s.sA), sW = C(s.sW), c0 = C(s.c[0]), c1 = C(s.c[1]), c2 = C(s.c[2]);
    const C pf = C(s.pf);
    const int tx = cdiv(n, TX);
    // a chunk's window of yc + 4 rows stays within kWinMax bytes
    const long ycap = min((long)n + 1, kWinMax / ((long)n * (long)sizeof(S)) - 4) & ~1L;
    if (ycap < 2) return hipErrorInvalidValue;
    const int yc = min(even_chunk(pick_chunk(n, tx, want, minc)), (int)ycap);
    const int nch = cdiv(n, yc);
    dim3 grid(tx * nch, s.batch);
    if (nparts) *nparts = grid.x * grid.y;
    if (norm && (long)grid.x * grid.y > s.partials_cap) return hipErrorInvalidValue;
#define L2(ZG, NM, PR)                                                                      \
    mg_launch((k_smooth2d<S, C, TX, NT, 1, UN, ZG, NM, PR, NTS>), grid, dim3(NT), 0, \
                       st, u, b, out, n, tx, yc, nch, sA, sW, c0, c1, c2, s.partials, ec, nc, pf, \
                       static_cast<S*>(nullptr))
    if constexpr (sizeof(S) == 8) {
        if (s.rout) {  // residual side output (from a guess, or with the correction)
            if (zg || norm) return hipErrorInvalidValue;
            if (pro)
                mg_launch((k_smooth2d<S, C, TX, NT, 1, UN, false, false, true, NTS, true>),
                                   grid, dim3(NT), 0, st, u, b, out, n, tx, yc, nch, sA, sW, c0,
                                   c1, c2, s.partials, ec, nc, pf, static_cast<S*>(s.rout));
            else
                mg_launch((k_smooth2d<S, C, TX, NT, 1, UN, false, false, false, NTS, true>),
                                   grid, dim3(NT), 0, st, u, b, out, n, tx, yc, nch, sA, sW, c0,
                                   c1, c2, s.partials, ec, nc, pf, static_cast<S*>(s.rout));
            return hipGetLastError();
        }
    }
    if (zg) L2(true, false, false);
    else if (norm) L2(false, true, false);
    else if (pro) L2(false, false, true);
    else L2(false, false, false);
#undef L2
    return hipGetLastError();
}

template <typename S, typename C>
hipError_t smooth_impl(bool zg, bool norm, const Sweep& s, hipStream_t st, int* nparts) {
    const int n = s.n;
    const bool pro = s.ec != nullptr;
    if (zg && (norm || pro)) return hipErrorInvalidValue;
    if (norm && pro) return hipErrorInvalidValue;
    // buffer offsets are 32-bit byte offsets within one plane
    if (s.d == 3 && (long)n * n * (long)sizeof(S) > 0x7fffffffL) return hipErrorInvalidValue;
    // the large configurations (at least 200^3 or 3000^2 > 2^22 nodes)
    // store non-temporally
    if (s.d == 3) {
        // FP32 / FP16 storage: 256x8 tiles on 1024 threads and 1024 marches
        // (4-byte and 2-byte rows need longer row segments and more waves in
        // flight; 11% faster than 128x16 tiles measured cold at n = 511).
        // FP16 storage: 128x8 tiles on 512 threads and 512 marches, two
        // workgroups per CU (the post-smoother with the correction at n =
        // 511 in the refinement loop: 311 against 359 us; 64x16 on 512 352,
        // 128x16 on 1024 345, 64x8 on 256 351 us; FP32 storage is slower on
        // every one of these shapes than on 256x8)
        if constexpr (sizeof(S) == 2) {
            if (n >= 200)
                return launch_smooth3d<S, C, 128, 8, 512, 6, true>(zg, norm, s, 512, 32, st,
                                                                    nparts);
        }
        if constexpr (sizeof(S) < 8) {
            if (n >= 200)
                return launch_smooth3d<S, C, 256, 8, 1024, 6, true>(zg, norm, s, 1024, 32, st,
                                                                     nparts);
        }
        if (n >= 200) return launch_smooth3d<S, C, 64, 16, 640, 6, true>(zg, norm, s, 256, 32, st, nparts);
        // n = 127 (the post-smoother with the correction): 32x16 tiles and
        // 512 marches 16.4-16.7 us, 64x16 with 256 marches 17.3-18.1, with
        // 512 marches 22.2, 32x32 17.3-17.6
        if (n >= 100) return launch_smooth3d<S, C, 32, 16, 320, 2, false>(zg, norm, s, 512, 2, st, nparts);
        if (n < 50 && pro && !norm && !s.rout && !s.u_f32 && s.c[2] == 0.0 && s.c[3] == 0.0) {
            // the post-smoother with the correction as a tile kernel below 50
            // nodes per side (FP64, 3D N=256: n = 31 4.7 against 6.3 us for
            // the march; at n = 63 the march is faster, 6.4 against 6.8 us
            // on 8x8x8 tiles and 7.9 us on 8x8x4)
            const int nc = (n + 1) / 2 - 1;
#define PRO3(TX, TY, TZ, NT)                                                                    \
    do {                                                                                       \
        const int tx = cdiv(n, TX), ty = cdiv(n, TY), tz = cdiv(n, TZ);                        \
        if (nparts) *nparts = 0;                                                               \
        mg_launch((k_pro3d<S, C, TX, TY, TZ, NT>), dim3(tx * ty * tz, s.batch), dim3(NT), 0,  \
                  st, static_cast<const S*>(s.u), static_cast<const S*>(s.b),                  \
                  static_cast<S*>(s.out), static_cast<const S*>(s.ec), n, nc, tx, ty, tz,      \
                  C(s.sA), C(s.sW), C(s.c[0]), C(s.c[1]), C(s.pf));                            \
    } while (0)
            PRO3(8, 8, 8, 512);
#undef PRO3
            return hipGetLastError();
        }
        return launch_smooth3d<S, C, 32, 16, 320, 2, false>(zg, norm, s, 256, 2, st, nparts);
    }
    if (n >= 3000) return launch_smooth2d<S, C, 1024, 576, 4, true>(zg, norm, s, 256, 32, st, nparts);
    if (n >= 1500) return launch_smooth2d<S, C, 512, 320, 2, false>(zg, norm, s, 512, 2, st, nparts);
    // n = 1023: 256-wide strips (the post-smoother with the correction 10.5
    // against 11.4 us on 512-wide ones; at n = 2047 512 stays, 24.2 against
    // 24.7 us)
    if (n >= 700) return launch_smooth2d<S, C, 256, 320, 2, false>(zg, norm, s, 512, 2, st, nparts);
    return launch_smooth2d<S, C, 128, 192, 2, false>(zg, norm, s, 512, 2, st, nparts);
}

template <typename S, typename C, int TXc, int TYc, int NT, int UN>
hipError_t launch_restrict3d(const Sweep& s, int want, int minc, hipStream_t st) {
    const int n = s.n, nc = (n + 1) / 2 - 1;
    const int tx = cdiv(nc, TXc), ty = cdiv(nc, TYc);
    const int zc = win_chunk(pick_chunk(nc, tx * ty, want, minc), (long)n * n * sizeof(S), 2, 3);
    if (zc < 1) return hipErrorInvalidValue;
    const int nch = cdiv(nc, zc);
    dim3 grid(tx * ty * nch, s.batch);
    mg_launch((k_restrict3d<S, C, TXc, TYc, NT, UN>), grid, dim3(NT), 0, st,
                       static_cast<const S*>(s.u), static_cast<const S*>(s.b),
                       static_cast<S*>(s.out), n, nc, tx, ty, zc, nch, C(s.sA), s.fin_ps,
                       s.fin_pm, s.fin_count, s.fin_dev, s.fin_host);
    return hipGetLastError();
}

template <typename S, typename C, int TXc, int NT, int UN>
hipError_t launch_restrict2d(const Sweep& s, int want, int minc, hipStream_t st) {
    const int n = s.n, nc = (n + 1) / 2 - 1;
    const int tx = cdiv(nc, TXc);
    const int yc = win_chunk(pick_chunk(nc, tx, want, minc), (long)n * sizeof(S), 2, 3);
    if (yc < 1) return hipErrorInvalidValue;
    const int nch = cdiv(nc, yc);
    dim3 grid(tx * nch, s.batch);
    mg_launch((k_restrict2d<S, C, TXc, NT, UN>), grid, dim3(NT), 0, st,
                       static_cast<const S*>(s.u), static_cast<const S*>(s.b),
                       static_cast<S*>(s.out), n, nc, tx, yc, nch, C(s.sA), s.fin_ps,
                       s.fin_pm, s.fin_count, s.fin_dev, s.fin_host);
    return hipGetLastError();
}

template <typename S, typename C>
hipError_t restrict_impl(const Sweep& s, hipStream_t st) {
    const int n = s.n;
    if (s.d == 3 && (long)n * n * (long)sizeof(S) > 0x7fffffffL) return hipErrorInvalidValue;
    if (s.d == 3) {
        if (sizeof(S) < 8 && n >= 200) return launch_restrict3d<S, C, 64, 8, 768, 6>(s, 512, 8, st);
        if (n >= 200) return launch_restrict3d<S, C, 32, 8, 576, 6>(s, 256, 8, st);
        return launch_restrict3d<S, C, 32, 4, 320, 2>(s, 512, 1, st);
    }
    if (n >= 3000) return launch_restrict2d<S, C, 512, 576, 6>(s, 256, 8, st);
    if (n >= 700) return launch_restrict2d<S, C, 256, 320, 2>(s, 512, 1, st);
    return launch_restrict2d<S, C, 128, 192, 2>(s, 512, 1, st);
}

template <typename S, typename C>
hipError_t prolong_impl(int d, int n, int batch, const void* ec, const void* in, void* out,
                        double pf, hipStream_t st) {
    const int nc = (n + 1) / 2 - 1;
    const long pts = d == 3 ? (long)n * n * n : (long)n * n;
    dim3 grid(cdiv(pts, 256), batch);
    if (d == 3)
        mg_launch((k_prolong3d<S, C>), grid, dim3(256), 0, st,
                           static_cast<const S*>(ec), static_cast<const S*>(in),
                           static_cast<S*>(out), n, nc, C(pf));
    else
        mg_launch((k_prolong2d<S, C>), grid, dim3(256), 0, st,
                           static_cast<const S*>(ec), static_cast<const S*>(in),
                           static_cast<S*>(out), n, nc, C(pf));
    return hipGetLastError();
}

template <typename S, typename C, int D, bool WC, int KT>
hipError_t tail_launch(const Tail& t, size_t lds, hipStream_t st) {
    static bool attr_set = false;  // the dynamic LDS limit, once per instantiation
    if (!attr_set) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_tail<S, C, D, WC, KT>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    mg_launch((k_tail<S, C, D, WC, KT>), dim3(t.batch), dim3(1024), lds, st,
              static_cast<const S*>(t.b), static_cast<S*>(t.e), C(t.c[0]), C(t.c[1]),
              C(t.c[2]), C(t.c[3]), t.ginv, t.scaled ? 1 : 0, WC ? t.wvisits : 0);
    return hipGetLastError();
}

// the top tail level has nt = 2^KT - 1 nodes per direction (3 .. 63 in 2D,
// 3 .. 15 in 3D), a compile-time parameter of the kernel
template <typename S, typename C, int D, bool WC>
hipError_t tail_impl_w(const Tail& t, size_t lds, hipStream_t st) {
    switch (t.nt) {
        case 3: return tail_launch<S, C, D, WC, 2>(t, lds, st);
        case 7: return tail_launch<S, C, D, WC, 3>(t, lds, st);
        case 15: return tail_launch<S, C, D, WC, 4>(t, lds, st);
        default: break;
    }
    if constexpr (D == 2) {
        if (t.nt == 31) return tail_launch<S, C, D, WC, 5>(t, lds, st);
        if (t.nt == 63) return tail_launch<S, C, D, WC, 6>(t, lds, st);
    }
    return hipErrorInvalidValue;
}

template <typename S, typename C, int D>
hipError_t tail_impl_d(const Tail& t, size_t lds, hipStream_t st) {
    return t.wvisits > 0 ? tail_impl_w<S, C, D, true>(t, lds, st)
                         : tail_impl_w<S, C, D, false>(t, lds, st);
}

template <typename S, typename C>
hipError_t tail_impl(const Tail& t, hipStream_t st) {
    const size_t lds = tail_lds_bytes(sizeof(C) == 8 ? P64 : P32, t.d, t.nt);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    // the thread boxes cover at most 64 (2D) or 16 (3D) nodes per direction
    if ((t.d == 2 && t.nt > 63) || (t.d == 3 && t.nt > 15)) return hipErrorInvalidValue;
    return t.d == 3 ? tail_impl_d<S, C, 3>(t, lds, st) : tail_impl_d<S, C, 2>(t, lds, st);
}

template <typename S, bool RES>
hipError_t ir_impl(const IRStep& s, hipStream_t st, int* nparts) {
    const int n = s.n;
    const S* e = static_cast<const S*>(s.e_lo);
    S* rlo = static_cast<S*>(s.r_lo);
    if (s.d == 3 && (long)n * n * 8L > 0x7fffffffL) return hipErrorInvalidValue;
    const bool large = s.d == 3 ? n >= 200 : n >= 3000;
    // same shapes as the FP64 smoothers; large grids: one long march per CU,
    // unrolled 6 times, non-temporal stores (256x4 tiles were faster alone,
    // measured cold, but not inside the refinement loop, and slower with
    // FP16 corrections)
#define IR3(TX, TY, NT, UN, NTS, WANT, MINC)                                                    \
    do {                                                                                       \
        const int tx = cdiv(n, TX), ty = cdiv(n, TY);                                          \
        const int zc = win_chunk(pick_chunk(n, tx * ty, WANT, MINC), 8L * n * n, 1, 2);        \
        if (zc < 1) return hipErrorInvalidValue;                                               \
        const int nch = cdiv(n, zc);                                                           \
        dim3 grid(tx * ty * nch, s.batch);                                                     \
        if (nparts) *nparts = grid.x * grid.y;                                                 \
        if ((long)grid.x * grid.y > s.partials_cap) return hipErrorInvalidValue;               \
        mg_launch((k_ir3d<S, TX, TY, NT, UN, NTS, RES>), grid, dim3(NT), 0, st, s.u, s.unew, \
                           e, s.b, rlo, n, tx, ty, zc, nch, s.inv_h2, s.sigma0, s.k, s.scales,  \
                           s.maxprev, s.psum, s.pmax, s.bparts);                                \
    } while (0)
#define IR2(TX, NT, UN, NTS, WANT, MINC)                                                        \
    do {                                                                                       \
        const int tx = cdiv(n, TX);                                                            \
        const int yc = win_chunk(pick_chunk(n, tx, WANT, MINC), 8L * n, 1, 2);                 \
        if (yc < 1) return hipErrorInvalidValue;                                               \
        const int nch = cdiv(n, yc);                                                           \
        dim3 grid(tx * nch, s.batch);                                                          \
        if (nparts) *nparts = grid.x * grid.y;                                                 \
        if ((long)grid.x * grid.y > s.partials_cap) return hipErrorInvalidValue;               \
        mg_launch((k_ir2d<S, TX, NT, UN, NTS, RES>), grid, dim3(NT), 0, st, s.u, s.unew, e, \
                           s.b, rlo, n, tx, yc, nch, s.inv_h2, s.sigma0, s.k, s.scales,         \
                           s.maxprev, s.psum, s.pmax, s.bparts);                                \
    } while (0)
    if (s.d == 3) {
        if (large) IR3(64, 16, 640, 6, true, 256, 32);
        else IR3(32, 16, 320, 2, false, 512, 1);
    } else {
        if (large) IR2(1024, 576, 6, true, 256, 32);
        else IR2(128, 192, 2, false, 512, 1);
    }
#undef IR3
#undef IR2
    return hipGetLastError();
}

}  // namespace

size_t tail_lds_bytes(Prec p, int d, int nt) {
    long tot = 0;
    for (int n = nt;; n = (n + 1) / 2 - 1) {
        tot += 3 * tail_padded(d, n);
        if (n <= 3) break;
    }
    const int m = d == 2 ? 9 : 27;
    return tail_ginv_offset((size_t)tot * (p == P64 ? 8 : 4)) + (size_t)m * m * 8;
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

template <typename S, typename C, int TXc, int TYc, int NT>
hipError_t launch_zrestrict3d(const Sweep& s, int want, int minc, hipStream_t st) {
    const int n = s.n, nc = (n + 1) / 2 - 1;
    const int tx = cdiv(nc, TXc), ty = cdiv(nc, TYc);
    const int zc = win_chunk(pick_chunk(nc, tx * ty, want, minc), (long)n * n * sizeof(S), 2, 5);
    if (zc < 1) return hipErrorInvalidValue;
    const int nch = cdiv(nc, zc);
    mg_launch((k_zrestrict3d<S, C, TXc, TYc, NT, 12>), dim3(tx * ty * nch, s.batch),
                       dim3(NT), 0, st, static_cast<const S*>(s.b), static_cast<S*>(s.out),
                       static_cast<S*>(s.out_c), n, nc, tx, ty, zc, nch, C(s.sA), C(s.sW),
                       C(s.c[0]), C(s.c[1]), s.fin_ps, s.fin_pm, s.fin_count, s.fin_dev,
                       s.fin_host);
    return hipGetLastError();
}

template <typename S, typename C>
hipError_t zsr_impl(const Sweep& s, hipStream_t st) {
    const int n = s.n, nc = (n + 1) / 2 - 1;
    if (nc < 1 || !s.out_c) return hipErrorInvalidValue;
    if (s.d == 3) {
        if ((long)n * n * (long)sizeof(S) > 0x7fffffffL) return hipErrorInvalidValue;
        // the restriction's shapes
        if constexpr (sizeof(S) < 8) {
            if (n >= 200) return launch_zrestrict3d<S, C, 64, 8, 768>(s, 512, 8, st);
        }
        if (n >= 200) return launch_zrestrict3d<S, C, 32, 8, 576>(s, 256, 8, st);
        if (s.c[2] != 0.0 || s.c[3] != 0.0) return hipErrorInvalidValue;  // 7-point only
        const C sA = C(s.sA), sW = C(s.sW), c0 = C(s.c[0]), c1 = C(s.c[1]);
#define ZSR3(CX, CY, CZ, NT)                                                                    \
    do {                                                                                       \
        const int tx = cdiv(nc, CX), ty = cdiv(nc, CY), tz = cdiv(nc, CZ);                     \
        mg_launch((k_zsr3d<S, C, CX, CY, CZ, NT>), dim3(tx * ty * tz, s.batch), dim3(NT), 0,  \
                  st, static_cast<const S*>(s.b), static_cast<S*>(s.out),                      \
                  static_cast<S*>(s.out_c), n, nc, tx, ty, tz, sA, sW, c0, c1, s.fin_ps,       \
                  s.fin_pm, s.fin_count, s.fin_dev, s.fin_host);                               \
    } while (0)
        // blocks measured on MI355X in FP64 (3D N=256 levels 1-3): 8x8x4 coarse
        // nodes on 1024 threads at n = 127 (20.5 against 21.2 us for the
        // smoother and the restriction; 512 threads 22.2, 8x8x8 22.4, 16x8x4
        // 22.3 us), 4x4x4 on 512 below (n = 63: 6.1 against 8.9 us, n = 31:
        // 4.4 against 8.4 us)
        if (n >= 100) ZSR3(8, 8, 4, 1024);
        else ZSR3(4, 4, 4, 512);
#undef ZSR3
        return hipGetLastError();
    }
    const S* b = static_cast<const S*>(s.b);
    S* e = static_cast<S*>(s.out);
    S* bc = static_cast<S*>(s.out_c);
    const C sA = C(s.sA), sW = C(s.sW), c0 = C(s.c[0]), c1 = C(s.c[1]), c2 = C(s.c[2]);
    // tiles measured on MI355X: 32x16 coarse nodes on 1024 threads from
    // n = 1023 up (21 us at n = 2047 against 27 us for 16x16 on 256), 16x16
    // on 512 below
#define ZSR(CX, CY, NT)                                                                         \
    do {                                                                                       \
        const int tx = cdiv(nc, CX), ty = cdiv(nc, CY);                                        \
        mg_launch((k_zsr2d<S, C, CX, CY, NT>), dim3(tx * ty, s.batch), dim3(NT), 0,   \
                           st, b, e, bc, n, nc, tx, ty, sA, sW, c0, c1, c2, s.fin_ps,          \
                           s.fin_pm, s.fin_count, s.fin_dev, s.fin_host);                      \
    } while (0)
    if (n >= 1000)
        ZSR(32, 16, 1024);
    else
        ZSR(16, 16, 512);
#undef ZSR
    return hipGetLastError();
}

template <typename S, typename C, int TX, int NT, int PD, int UN, bool NTS>
hipError_t launch_sr2d(const Sweep& s, bool norm, int want, int minc, hipStream_t st,
                       int* nparts) {
    // an FP32 input iterate only in FP64 with the residual output
    if (s.u_f32 && (sizeof(S) != 8 || !s.rout)) return hipErrorInvalidValue;
    const int n = s.n, nc = (n + 1) / 2 - 1;
    const int tx = cdiv(n, TX);
    // a chunk's window of 2 yc + 7 rows stays within kWinMax bytes
    const int yc = (int)min((long)pick_chunk(nc, tx, want, minc),
                            (kWinMax / ((long)n * (long)sizeof(S)) - 7) / 2);
    if (yc < 1) return hipErrorInvalidValue;
    const int nch = cdiv(nc, yc);
    dim3 grid(tx * nch, s.batch);
    if (nparts) *nparts = grid.x * grid.y;
    if (norm && (long)grid.x * grid.y > s.partials_cap) return hipErrorInvalidValue;
    const S* u = static_cast<const S*>(s.u);
    const S* b = static_cast<const S*>(s.b);
    S* out = static_cast<S*>(s.out);
    S* bc = static_cast<S*>(s.out_c);
    const C sA = C(s.sA), sW = C(s.sW), c0 = C(s.c[0]), c1 = C(s.c[1]), c2 = C(s.c[2]);
#define SR2(NM)                                                                              \
    mg_launch((k_sr2d<S, C, TX, NT, PD, UN, NTS, NM>), grid, dim3(NT), 0, st, u, b,  \
                       out, bc, n, nc, tx, yc, nch, sA, sW, c0, c1, c2, s.partials,          \
                       static_cast<S*>(nullptr), NM ? s.bparts : nullptr)
    if constexpr (sizeof(S) == 8) {
        if (s.rout) {  // residual side output
            if (norm) return hipErrorInvalidValue;
            if (s.u_f32)  // the iterate as stored in an FP32 checkpoint
                mg_launch((k_sr2d<S, C, TX, NT, PD, UN, NTS, false, true, float>), grid,
                          dim3(NT), 0, st, static_cast<const float*>(s.u), b, out, bc, n, nc,
                          tx, yc, nch, sA, sW, c0, c1, c2, s.partials, static_cast<S*>(s.rout),
                          static_cast<double*>(nullptr));
            else
                mg_launch((k_sr2d<S, C, TX, NT, PD, UN, NTS, false, true>), grid, dim3(NT), 0,
                          st, u, b, out, bc, n, nc, tx, yc, nch, sA, sW, c0, c1, c2,
                          s.partials, static_cast<S*>(s.rout), static_cast<double*>(nullptr));
            return hipGetLastError();
        }
    }
    if (norm) SR2(true);
    else SR2(false);
#undef SR2
    return hipGetLastError();
}

template <typename S, typename C, int TX, int TY, int NT, int PD, int UN, bool NTS>
hipError_t launch_sr3d(const Sweep& s, bool norm, int want, int minc, hipStream_t st,
                       int* nparts) {
    // an FP32 input iterate only in FP64 with the residual output
    if (s.u_f32 && (sizeof(S) != 8 || !s.rout)) return hipErrorInvalidValue;
    const int n = s.n, nc = (n + 1) / 2 - 1;
    const int tx = cdiv(n, TX), ty = cdiv(n, TY);
    // a chunk's window of 2 zc + 7 planes stays within kWinMax bytes
    const int zc = (int)min((long)pick_chunk(nc, tx * ty, want, minc),
                            (kWinMax / ((long)n * n * (long)sizeof(S)) - 7) / 2);
    if (zc < 1) return hipErrorInvalidValue;
    const int nch = cdiv(nc, zc);
    dim3 grid(tx * ty * nch, s.batch);
    if (nparts) *nparts = grid.x * grid.y;
    if (norm && (long)grid.x * grid.y > s.partials_cap) return hipErrorInvalidValue;
    const S* u = static_cast<const S*>(s.u);
    const S* b = static_cast<const S*>(s.b);
    S* out = static_cast<S*>(s.out);
    S* bc = static_cast<S*>(s.out_c);
    const C sA = C(s.sA), sW = C(s.sW), c0 = C(s.c[0]), c1 = C(s.c[1]);
#define SR3(NM)                                                                             \
    mg_launch((k_sr3d<S, C, TX, TY, NT, PD, UN, NTS, NM>), grid, dim3(NT), 0, st,     \
                       u, b, out, bc, n, nc, tx, ty, zc, nch, sA, sW, c0, c1, s.partials,   \
                       static_cast<S*>(nullptr), NM ? s.bparts : nullptr)
    if constexpr (sizeof(S) == 8) {
        if (s.rout) {  // residual side output
            if (norm) return hipErrorInvalidValue;
            if (s.u_f32)  // the iterate as stored in an FP32 checkpoint
                mg_launch((k_sr3d<S, C, TX, TY, NT, PD, UN, NTS, false, true, float>), grid,
                          dim3(NT), 0, st, static_cast<const float*>(s.u), b, out, bc, n, nc,
                          tx, ty, zc, nch, sA, sW, c0, c1, s.partials, static_cast<S*>(s.rout),
                          static_cast<double*>(nullptr));
            else
                mg_launch((k_sr3d<S, C, TX, TY, NT, PD, UN, NTS, false, true>), grid,
                          dim3(NT), 0, st, u, b, out, bc, n, nc, tx, ty, zc, nch, sA, sW,
                          c0, c1, s.partials, static_cast<S*>(s.rout),
                          static_cast<double*>(nullptr));
            return hipGetLastError();
        }
    }
    if (norm) SR3(true);
    else SR3(false);
#undef SR3
    return hipGetLastError();
}

template <typename S, typename C>
hipError_t sr_impl(const Sweep& s, bool norm, hipStream_t st, int* nparts) {
    const int n = s.n, nc = (n + 1) / 2 - 1;
    if (nc < 1 || !s.out_c || !s.u) return hipErrorInvalidValue;
    if (s.d == 3) {
        // buffer offsets are 32-bit byte offsets within one plane
        if ((long)n * n * (long)sizeof(S) > 0x7fffffffL) return hipErrorInvalidValue;
        // shapes measured on MI355X in FP64: 32x32 tiles (ring 3: 1.49x the
        // tile's points) with two points per lane; n = 255: 106 us against
        // 128 us for the separate smoother and restriction, n = 511: 758
        // against 1058 us.  64x16 tiles were 3-4% slower, non-temporal
        // stores 4-5% slower, one u and one residual plane in LDS (two
        // workgroups per CU, a second barrier per plane) 2-3% slower.  Below
        // 200 nodes the fused kernel is not faster than the two sweeps (22-33
        // against 24 us at n = 127); the cycle uses it from 200 up.
        // FP32 / FP16 storage: 64x32 tiles on 1024 threads (4- and 2-byte
        // rows need longer row segments; n = 511: 448 / 346 us against 566 /
        // 406 us for the separate sweeps, where 32x32 tiles take 486 / 477)
        if constexpr (sizeof(S) < 8) {
            return launch_sr3d<S, C, 64, 32, 1024, 2, 6, false>(s, norm, n >= 200 ? 256 : 512,
                                                                4, st, nparts);
        }
        if (n >= 200) return launch_sr3d<S, C, 32, 32, 768, 2, 6, false>(s, norm, 256, 8, st, nparts);
        return launch_sr3d<S, C, 32, 32, 768, 1, 2, false>(s, norm, 512, 4, st, nparts);
    }
    // shapes measured on MI355X in FP64 (n = 4095: 90 us against 127 us for
    // the separate smoother and restriction; 1024-wide strips with two
    // columns per lane beat 512- and 256-wide ones by 8-10%; n = 2047: 25
    // against 35 us; n = 1023: 15 against 16 us)
    if (n >= 3000) return launch_sr2d<S, C, 1024, 576, 2, 6, true>(s, norm, 256, 16, st, nparts);
    if (n >= 1500) return launch_sr2d<S, C, 1024, 576, 2, 6, false>(s, norm, 512, 8, st, nparts);
    if (n >= 700) return launch_sr2d<S, C, 256, 320, 2, 6, false>(s, norm, 1024, 4, st, nparts);
    return launch_sr2d<S, C, 128, 192, 2, 6, false>(s, norm, 1024, 2, st, nparts);
}

hipError_t launch_smooth_restrict(Prec p, bool norm, const Sweep& s, hipStream_t st,
                                  int* nparts) {
    switch (p) {
        case P64: return sr_impl<double, double>(s, norm, st, nparts);
        case P32:
            if (norm) return hipErrorInvalidValue;
            return sr_impl<float, float>(s, false, st, nparts);
        default:
            if (norm) return hipErrorInvalidValue;
            return sr_impl<_Float16, float>(s, false, st, nparts);
    }
}

template <typename S, typename C, int TX, int NT, int PD, int UN, bool NTS>
hipError_t launch_psr2d(const Sweep& s, bool norm, int want, int minc, hipStream_t st,
                        int* nparts) {
    if (s.u_f32) return hipErrorInvalidValue;
    const int n = s.n, nc = (n + 1) / 2 - 1;
    const int tx = cdiv(n, TX);
    // a chunk's window of 2 yc + 11 fine rows stays within kWinMax bytes
    const int yc = min(pick_chunk(nc, tx, want, minc),
                       (int)((kWinMax / ((long)n * sizeof(S)) - 11) / 2));
    if (yc < 1) return hipErrorInvalidValue;
    const int nch = cdiv(nc, yc);
    dim3 grid(tx * nch, s.batch);
    if (nparts) *nparts = grid.x * grid.y;
    if (norm && (long)grid.x * grid.y > s.partials_cap) return hipErrorInvalidValue;
    const S* u = static_cast<const S*>(s.u);
    const S* ec = static_cast<const S*>(s.ec);
    const S* b = static_cast<const S*>(s.b);
    S* out = static_cast<S*>(s.out);
    S* out_t = static_cast<S*>(s.out_t);
    S* bc = static_cast<S*>(s.out_c);
    const C sA = C(s.sA), sW = C(s.sW), c0 = C(s.c[0]), c1 = C(s.c[1]), c2 = C(s.c[2]);
    const C pf = C(s.pf);
#define PSR2(NM)                                                                              \
    mg_launch((k_psr2d<S, C, TX, NT, PD, UN, NTS, NM>), grid, dim3(NT), 0, st, u, ec, \
                       b, out, out_t, bc, n, nc, tx, yc, nch, sA, sW, c0, c1, c2, pf,         \
                       s.partials)
    if (norm) PSR2(true);
    else PSR2(false);
#undef PSR2
    return hipGetLastError();
}

template <typename S, typename C>
hipError_t psr_impl(const Sweep& s, bool norm, hipStream_t st, int* nparts) {
    const int n = s.n, nc = (n + 1) / 2 - 1;
    if (nc < 1 || s.d != 2 || !s.u || !s.ec || !s.out || !s.out_t || !s.out_c)
        return hipErrorInvalidValue;
    // shapes measured on MI355X in FP64: 512-wide strips, one column per
    // lane (two spill), prefetch two rows ahead; n = 4095: 139 us against
    // 170 us for the post-smoother and the fused pre-smoother + restriction
    // (256-wide strips 151 us, prefetch one row ahead 152-164 us); n = 2047:
    // 47 against 50 us
    if (n >= 1500) return launch_psr2d<S, C, 512, 576, 2, 12, true>(s, norm, 256, 16, st, nparts);
    if (n >= 700) return launch_psr2d<S, C, 256, 320, 1, 4, false>(s, norm, 512, 4, st, nparts);
    return launch_psr2d<S, C, 128, 192, 1, 4, false>(s, norm, 1024, 2, st, nparts);
}

hipError_t launch_post_pre_restrict(Prec p, bool norm, const Sweep& s, hipStream_t st,
                                    int* nparts) {
    switch (p) {
        case P64: return psr_impl<double, double>(s, norm, st, nparts);
        case P32:
            if (norm) return hipErrorInvalidValue;
            return psr_impl<float, float>(s, false, st, nparts);
        default:
            if (norm) return hipErrorInvalidValue;
            return psr_impl<_Float16, float>(s, false, st, nparts);
    }
}

hipError_t launch_zero_smooth_restrict(Prec p, const Sweep& s, hipStream_t st) {
    switch (p) {
        case P64: return zsr_impl<double, double>(s, st);
        case P32: return zsr_impl<float, float>(s, st);
        default: return zsr_impl<_Float16, float>(s, st);
    }
}

hipError_t launch_prolong(Prec p, int d, int n, int batch, const void* ec, void* u,
                          double pf, hipStream_t st) {
    return launch_prolong_to(p, d, n, batch, ec, u, u, pf, st);
}

hipError_t launch_prolong_to(Prec p, int d, int n, int batch, const void* ec, const void* in,
                             void* out, double pf, hipStream_t st) {
    switch (p) {
        case P64: return prolong_impl<double, double>(d, n, batch, ec, in, out, pf, st);
        case P32: return prolong_impl<float, float>(d, n, batch, ec, in, out, pf, st);
        default: return prolong_impl<_Float16, float>(d, n, batch, ec, in, out, pf, st);
    }
}

hipError_t launch_tail(Prec p, const Tail& t, hipStream_t st) {
    switch (p) {
        case P64: return tail_impl<double, double>(t, st);
        case P32: return tail_impl<float, float>(t, st);
        default: return tail_impl<_Float16, float>(t, st);
    }
}

hipError_t launch_adj_sweep(int d, int n, int batch, int mode, const double* ubar,
                            const double* r, const double* ec, double scale, double* ubar_new,
                            double* bbar, double* partials, long partials_cap, double sA,
                            double sW, const double* c, hipStream_t st, int* nparts) {
    if (mode != 0 && mode != 1) return hipErrorInvalidValue;
    if ((long)n * n * 8 > 0x7fffffffL) return hipErrorInvalidValue;  // 32-bit plane offsets
    dim3 grid;
    int tx = 0, ty = 1, zc = 0, nch = 0;
    // about 2048 marches over the whole batch, none shorter than 8 planes
    // (rows): each march re-reads three planes of ubar and computes one
    // plane of w more than it owns
    const int want = std::max(64, 2048 / std::max(1, batch));
    if (d == 3) {
        // 32 x 16 tiles on 512 threads (ubar on 36 x 20 per plane in LDS)
        tx = cdiv(n, 32);
        ty = cdiv(n, 16);
        zc = win_chunk(pick_chunk(n, tx * ty, want, 8), 8L * n * n, 1, 6);
    } else {
        // 256-wide strips on 320 threads
        tx = cdiv(n, 256);
        zc = win_chunk(pick_chunk(n, tx, want, 8), 8L * n, 1, 6);
    }
    if (zc < 1) return hipErrorInvalidValue;
    nch = cdiv(n, zc);
    grid = dim3(tx * ty * nch, batch);
    if (nparts) *nparts = grid.x * grid.y;
    if (mode == 0 && 4L * grid.x * grid.y > partials_cap) return hipErrorInvalidValue;
    const bool wide = d == 3 && (c[2] != 0.0 || c[3] != 0.0);
#define AS3(WD, MD)                                                                             \
    mg_launch((k_adj_sweep3d<32, 16, 512, WD, MD>), grid, dim3(512), 0, st, ubar, r, ec, \
                       ubar_new, bbar, partials, n, tx, ty, zc, nch, sA, sW, c[0], c[1], c[2], \
                       c[3], scale)
#define AS2(MD)                                                                               \
    mg_launch((k_adj_sweep2d<256, 320, MD>), grid, dim3(320), 0, st, ubar, r, ec,     \
                       ubar_new, bbar, partials, n, tx, zc, nch, sA, sW, c[0], c[1], c[2], scale)
    if (d == 3) {
        if (mode == 1) AS3(false, 1);
        else if (wide) AS3(true, 0);
        else AS3(false, 0);
    } else {
        if (mode == 1) AS2(1);
        else AS2(0);
    }
#undef AS3
#undef AS2
    return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, const double* maxparts, int count,
                           double* out, hipStream_t st, double* host) {
    mg_launch(k_finalize, dim3(1), dim3(256), 0, st, partials, maxparts, count, out,
                       host);
    return hipGetLastError();
}

hipError_t launch_sumsq(const double* v, long count, double* partials, long partials_cap,
                        hipStream_t st, int* nparts) {
    long blocks = std::min<long>(2048, std::max<long>(1, (count + 4095) / 4096));
    if (blocks > partials_cap) blocks = partials_cap;
    const long per = (count + blocks - 1) / blocks;
    mg_launch(k_sumsq, dim3((unsigned)blocks), dim3(256), 0, st, v, count, per, partials);
    if (nparts) *nparts = (int)blocks;
    return hipGetLastError();
}

hipError_t launch_residual_norm(int d, int n, int batch, const double* u, const double* b,
                                double inv_h2, double* psum, double* pmax, long partials_cap,
                                hipStream_t st, int* nparts, double* bparts) {
    // the marching refinement-step kernel without its stores
    IRStep s;
    s.d = d;
    s.n = n;
    s.batch = batch;
    s.u = u;
    s.b = b;
    s.inv_h2 = inv_h2;
    s.psum = psum;
    s.pmax = pmax;
    s.bparts = bparts;
    s.partials_cap = partials_cap;
    return ir_impl<double, true>(s, st, nparts);
}

hipError_t launch_ir_step(Prec p, const IRStep& s, hipStream_t st, int* nparts) {
    switch (p) {
        case P32: return ir_impl<float, false>(s, st, nparts);
        case P16: return ir_impl<_Float16, false>(s, st, nparts);
        default: return ir_impl<double, false>(s, st, nparts);
    }
}

}  // namespace spaimg
