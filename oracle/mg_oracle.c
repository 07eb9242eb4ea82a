/*
 * mg_oracle.c -- plain FP64 CPU oracle for the SPAI-smoothed geometric
 * multigrid cycle of He, Liu and Wang, "Optimized sparse approximate inverse
 * smoothers for solving Laplacian linear systems" (arXiv 2206.05543).
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists to check the GPU library.  Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or helper with the GPU path.
 * Built with -O2 -ffp-contract=off so that every product and sum is rounded
 * exactly as written; loops are plain and unfused.  A second build with
 * -fopenmp (the all-core CPU baseline) splits the outer grid loops of the
 * stencil and transfer operators and the element-wise loops across threads;
 * every output element is still computed by one thread with the same
 * operations, and the reductions (norms, dot products) and scatter loops
 * stay serial, so both builds give bit-identical results.
 *
 * Grid convention (Section 1, eqs. (Ax=b) and (A_h)): the unit square/cube
 * with N intervals per direction, h = 1/N, unknowns on the n = N-1 interior
 * nodes per direction, Dirichlet value 0 outside.  Arrays hold interior nodes
 * only, x fastest: index = i + n*(j + n*k) for the node at ((i+1)h, (j+1)h,
 * (k+1)h).  Batched arrays are stacked with the batch index outermost.
 *
 * Smoother coefficients c (Section 3): the stencil of M with h^2 taken out
 * and the damping factor omega folded in, i.e. M = h^2 * sum_j c_j K_j with
 * K_0 the identity, K_1 the sum over the 2d face neighbours and K_2 the sum
 * over the 4 diagonal neighbours (2D); in 3D K_2 is the sum over the 12 edge
 * neighbours and K_3 the sum over the 8 corner neighbours, the wider
 * 19- and 27-point stencils the closing remark of Section 3.2 mentions
 * (c_2 = c_3 = 0 gives the 7-point family T).  c holds 3 entries in 2D and 4
 * in 3D.  M acts on a residual that is zero outside the interior (zero
 * extension).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* threads the loops below run on: 1 in the plain build */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ grid */

static long npts(int d, int N)
{
    long n = N - 1, p = 1;
    for (int a = 0; a < d; a++) p *= n;
    return p;
}

/* Value of a grid function at interior index (i,j,k); zero for any node on
 * or outside the boundary.  In 2D, k is ignored. */
static double at(const double *v, int d, int N, int i, int j, int k)
{
    int n = N - 1;
    if (i < 0 || i >= n || j < 0 || j >= n) return 0.0;
    if (d == 3) {
        if (k < 0 || k >= n) return 0.0;
        return v[i + (long)n * (j + (long)n * k)];
    }
    return v[i + (long)n * j];
}

static long idx(int d, int N, int i, int j, int k)
{
    long n = N - 1;
    return d == 3 ? i + n * (j + n * k) : i + n * j;
}

/* ------------------------------------------------------ stencil operators */

/* out = A_h v: the 5-point (2D) or 7-point (3D) negative Laplacian,
 * (A_h v)_p = (2d v_p - sum of the 2d face neighbours) / h^2
 * (Section 1, eq. (A_h)). */
void or_apply_A(int d, int N, const double *v, double *out)
{
    int n = N - 1;
    double inv_h2 = (double)N * (double)N;
    int nk = (d == 3) ? n : 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nk; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                double s = 2.0 * d * at(v, d, N, i, j, k);
                s -= at(v, d, N, i - 1, j, k);
                s -= at(v, d, N, i + 1, j, k);
                s -= at(v, d, N, i, j - 1, k);
                s -= at(v, d, N, i, j + 1, k);
                if (d == 3) {
                    s -= at(v, d, N, i, j, k - 1);
                    s -= at(v, d, N, i, j, k + 1);
                }
                out[idx(d, N, i, j, k)] = s * inv_h2;
            }
}

/* out = K_which v with zero extension: K_0 = identity, K_1 = sum of the
 * face neighbours, K_2 = sum of the four diagonal neighbours (2D) or of the
 * twelve edge neighbours (3D: offsets with two nonzero components), K_3 =
 * sum of the eight corner neighbours (3D only: three nonzero components).
 * These are the building blocks of the 9-point family Upsilon(alpha, beta,
 * gamma) (Section 3.1), the 7-point family T(alpha, beta) (Section 3.2) and
 * its 19- and 27-point extensions. */
void or_apply_K(int d, int N, int which, const double *v, double *out)
{
    int n = N - 1;
    int nk = (d == 3) ? n : 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nk; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                double s = 0.0;
                if (which == 0) {
                    s = at(v, d, N, i, j, k);
                } else if (which == 1) {
                    s += at(v, d, N, i - 1, j, k);
                    s += at(v, d, N, i + 1, j, k);
                    s += at(v, d, N, i, j - 1, k);
                    s += at(v, d, N, i, j + 1, k);
                    if (d == 3) {
                        s += at(v, d, N, i, j, k - 1);
                        s += at(v, d, N, i, j, k + 1);
                    }
                } else if (d == 2) {
                    s += at(v, d, N, i - 1, j - 1, k);
                    s += at(v, d, N, i + 1, j - 1, k);
                    s += at(v, d, N, i - 1, j + 1, k);
                    s += at(v, d, N, i + 1, j + 1, k);
                } else {
                    /* every offset (a, b, c) in {-1, 0, 1}^3 with exactly
                     * `which` nonzero components (2: edges, 3: corners) */
                    for (int c = -1; c <= 1; c++)
                        for (int b = -1; b <= 1; b++)
                            for (int a = -1; a <= 1; a++)
                                if ((a != 0) + (b != 0) + (c != 0) == which)
                                    s += at(v, d, N, i + a, j + b, k + c);
                }
                out[idx(d, N, i, j, k)] = s;
            }
}

static int ncoef(int d) { return d == 2 ? 3 : 4; }

/* out = M v = h^2 * sum_j c_j K_j v (Section 3.1: Upsilon; Section 3.2: T
 * and its wider extensions).  A zero coefficient of the 3D edge or corner
 * term is skipped: its term adds nothing. */
void or_apply_W(int d, int N, const double *c, const double *v, double *out)
{
    long P = npts(d, N);
    double h2 = 1.0 / ((double)N * (double)N);
    double *t = malloc(sizeof(double) * P);
    memset(out, 0, sizeof(double) * P);
    for (int j = 0; j < ncoef(d); j++) {
        if (d == 3 && j >= 2 && c[j] == 0.0) continue;
        or_apply_K(d, N, j, v, t);
#pragma omp parallel for schedule(static)
        for (long p = 0; p < P; p++) out[p] += c[j] * t[p];
    }
#pragma omp parallel for schedule(static)
    for (long p = 0; p < P; p++) out[p] *= h2;
    free(t);
}

/* r = b - A_h u */
void or_residual(int d, int N, const double *u, const double *b, double *r)
{
    long P = npts(d, N);
    or_apply_A(d, N, u, r);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < P; p++) r[p] = b[p] - r[p];
}

/* One step of the preconditioned Richardson smoother, out of place:
 * out = u + M (b - A_h u) (Section 2, eq. (smoother), omega folded into M). */
void or_smooth(int d, int N, const double *c, const double *u,
               const double *b, double *out)
{
    long P = npts(d, N);
    double *r = malloc(sizeof(double) * P);
    double *w = malloc(sizeof(double) * P);
    or_residual(d, N, u, b, r);
    or_apply_W(d, N, c, r, w);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < P; p++) out[p] = u[p] + w[p];
    free(r);
    free(w);
}

/* ------------------------------------------------------ grid transfers */

/* 1D full-weighting weight for offset o in {-1, 0, 1}. */
static double fw(int o) { return o == 0 ? 0.5 : 0.25; }

/* rc = R r: full-weighting restriction to the grid with N/2 intervals
 * (Section 4, multigrid setup).  The coarse node J sits on fine node 2J;
 * in 0-based interior indices coarse index jc maps to fine index 2 jc + 1. */
void or_restrict(int d, int N, const double *r, double *rc)
{
    int Nc = N / 2, nc = Nc - 1;
    int nk = (d == 3) ? nc : 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int kc = 0; kc < nk; kc++)
        for (int jc = 0; jc < nc; jc++)
            for (int ic = 0; ic < nc; ic++) {
                double s = 0.0;
                int ok_lo = (d == 3) ? -1 : 0, ok_hi = (d == 3) ? 1 : 0;
                for (int ok = ok_lo; ok <= ok_hi; ok++)
                    for (int oj = -1; oj <= 1; oj++)
                        for (int oi = -1; oi <= 1; oi++) {
                            double w = fw(oi) * fw(oj);
                            if (d == 3) w *= fw(ok);
                            s += w * at(r, d, N, 2 * ic + 1 + oi, 2 * jc + 1 + oj,
                                        2 * kc + 1 + ok);
                        }
                rc[idx(d, Nc, ic, jc, kc)] = s;
            }
}

/* Coarse nodes and weights that linear interpolation uses for the fine node
 * with grid coordinate g (1..N-1): an even g coincides with coarse node g/2,
 * an odd g lies halfway between coarse nodes (g-1)/2 and (g+1)/2.  Returns
 * the count; coarse coordinates 0 and N/2 are boundary nodes (value 0). */
static int interp1d(int g, int G[2], double w[2])
{
    if (g % 2 == 0) {
        G[0] = g / 2;
        w[0] = 1.0;
        return 1;
    }
    G[0] = (g - 1) / 2;
    G[1] = (g + 1) / 2;
    w[0] = w[1] = 0.5;
    return 2;
}

/* u += P ec: bilinear (2D) / trilinear (3D) interpolation from the grid with
 * N/2 intervals, coarse boundary values 0 (Section 4, multigrid setup). */
void or_prolong_add(int d, int N, const double *ec, double *u)
{
    int n = N - 1, Nc = N / 2;
    int nk = (d == 3) ? n : 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nk; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                int Gi[2], Gj[2], Gk[2] = {0, 0};
                double wi[2], wj[2], wk[2] = {1.0, 1.0};
                int ni = interp1d(i + 1, Gi, wi);
                int nj = interp1d(j + 1, Gj, wj);
                int nkk = 1;
                if (d == 3) nkk = interp1d(k + 1, Gk, wk);
                double s = 0.0;
                for (int c = 0; c < nkk; c++)
                    for (int b = 0; b < nj; b++)
                        for (int a = 0; a < ni; a++) {
                            double w = wi[a] * wj[b];
                            int kk = 0;
                            if (d == 3) {
                                w *= wk[c];
                                kk = Gk[c] - 1;
                            }
                            s += w * at(ec, d, Nc, Gi[a] - 1, Gj[b] - 1, kk);
                        }
                u[idx(d, N, i, j, k)] += s;
            }
}

/* rf += R^T bc, written as a scatter of the full-weighting weights (the
 * transpose of or_restrict, coded independently of or_prolong_add). */
void or_restrict_T_add(int d, int N, const double *bc, double *rf)
{
    int Nc = N / 2, nc = Nc - 1;
    int nk = (d == 3) ? nc : 1;
    for (int kc = 0; kc < nk; kc++)
        for (int jc = 0; jc < nc; jc++)
            for (int ic = 0; ic < nc; ic++) {
                double v = bc[idx(d, Nc, ic, jc, kc)];
                int ok_lo = (d == 3) ? -1 : 0, ok_hi = (d == 3) ? 1 : 0;
                for (int ok = ok_lo; ok <= ok_hi; ok++)
                    for (int oj = -1; oj <= 1; oj++)
                        for (int oi = -1; oi <= 1; oi++) {
                            double w = fw(oi) * fw(oj);
                            if (d == 3) w *= fw(ok);
                            rf[idx(d, N, 2 * ic + 1 + oi, 2 * jc + 1 + oj,
                                   d == 3 ? 2 * kc + 1 + ok : 0)] += w * v;
                        }
            }
}

/* ec += P^T uf: the transpose of linear interpolation, as a scatter from
 * each fine node to the coarse nodes it was interpolated from. */
void or_prolong_T_add(int d, int N, const double *uf, double *ec)
{
    int n = N - 1, Nc = N / 2;
    int nk = (d == 3) ? n : 1;
    for (int k = 0; k < nk; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                int Gi[2], Gj[2], Gk[2] = {1, 1};
                double wi[2], wj[2], wk[2] = {1.0, 1.0};
                int ni = interp1d(i + 1, Gi, wi);
                int nj = interp1d(j + 1, Gj, wj);
                int nkk = 1;
                if (d == 3) nkk = interp1d(k + 1, Gk, wk);
                double v = uf[idx(d, N, i, j, k)];
                for (int c = 0; c < nkk; c++)
                    for (int b = 0; b < nj; b++)
                        for (int a = 0; a < ni; a++) {
                            int I = Gi[a], J = Gj[b], K = Gk[c];
                            if (I < 1 || I > Nc - 1 || J < 1 || J > Nc - 1) continue;
                            if (d == 3 && (K < 1 || K > Nc - 1)) continue;
                            double w = wi[a] * wj[b] * wk[c];
                            ec[idx(d, Nc, I - 1, J - 1, d == 3 ? K - 1 : 0)] += w * v;
                        }
            }
}

/* ------------------------------------------------------ coarsest solve */

/* x = A_h^{-1} b by a dense Cholesky factorisation of the stencil matrix
 * (the exact solve on the coarsest grid, h0 = 1/4, Section 4).  Works for
 * any N; intended for N = 4 (9 or 27 unknowns) and small test grids. */
void or_direct_solve(int d, int N, const double *b, double *x)
{
    long P = npts(d, N);
    int n = N - 1;
    double inv_h2 = (double)N * (double)N;
    double *L = calloc((size_t)(P * P), sizeof(double));
    /* assemble A row by row from the stencil definition */
    int nk = (d == 3) ? n : 1;
    for (int k = 0; k < nk; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                long p = idx(d, N, i, j, k);
                L[p * P + p] = 2.0 * d * inv_h2;
                int nb[6][3] = {{i - 1, j, k}, {i + 1, j, k}, {i, j - 1, k},
                                {i, j + 1, k}, {i, j, k - 1}, {i, j, k + 1}};
                for (int q = 0; q < 2 * d; q++) {
                    int a = nb[q][0], bb = nb[q][1], cc = nb[q][2];
                    if (a < 0 || a >= n || bb < 0 || bb >= n) continue;
                    if (d == 3 && (cc < 0 || cc >= n)) continue;
                    L[p * P + idx(d, N, a, bb, cc)] = -inv_h2;
                }
            }
    /* in-place Cholesky, lower triangle: A = L L^T */
    for (long c = 0; c < P; c++) {
        double s = L[c * P + c];
        for (long q = 0; q < c; q++) s -= L[c * P + q] * L[c * P + q];
        double dia = sqrt(s);
        L[c * P + c] = dia;
        for (long r = c + 1; r < P; r++) {
            double t = L[r * P + c];
            for (long q = 0; q < c; q++) t -= L[r * P + q] * L[c * P + q];
            L[r * P + c] = t / dia;
        }
    }
    /* forward then backward substitution */
    double *y = malloc(sizeof(double) * P);
    for (long r = 0; r < P; r++) {
        double t = b[r];
        for (long q = 0; q < r; q++) t -= L[r * P + q] * y[q];
        y[r] = t / L[r * P + r];
    }
    for (long r = P - 1; r >= 0; r--) {
        double t = y[r];
        for (long q = r + 1; q < P; q++) t -= L[q * P + r] * x[q];
        x[r] = t / L[r * P + r];
    }
    free(y);
    free(L);
}

/* ------------------------------------------------------ cycles */

double or_norm2(long n, const double *v)
{
    double s = 0.0;
    for (long p = 0; p < n; p++) s += v[p] * v[p];
    return sqrt(s);
}

/* One multigrid cycle on the grid with N intervals, in place on u
 * (Section 4, multigrid setup): nu1 pre-smoothing steps, the residual
 * restricted by full weighting, gamma recursive cycles on the coarse grid
 * (rediscretised A with H = 2h) from a zero initial guess, bilinear/trilinear
 * correction, nu2 post-smoothing steps.  The grid with N = 4 (h0 = 1/4) is
 * solved exactly.  gamma = 1 is the V-cycle, gamma = 2 the W-cycle. */
void or_cycle(int d, int N, const double *c, int nu1, int nu2, int gamma,
              double *u, const double *b)
{
    if (N <= 4) {
        or_direct_solve(d, N, b, u);
        return;
    }
    long P = npts(d, N), Pc = npts(d, N / 2);
    double *t = malloc(sizeof(double) * P);
    for (int s = 0; s < nu1; s++) {
        or_smooth(d, N, c, u, b, t);
        memcpy(u, t, sizeof(double) * P);
    }
    or_residual(d, N, u, b, t);
    double *bc = malloc(sizeof(double) * Pc);
    double *ec = calloc((size_t)Pc, sizeof(double));
    or_restrict(d, N, t, bc);
    for (int g = 0; g < gamma; g++) or_cycle(d, N / 2, c, nu1, nu2, gamma, ec, bc);
    or_prolong_add(d, N, ec, u);
    for (int s = 0; s < nu2; s++) {
        or_smooth(d, N, c, u, b, t);
        memcpy(u, t, sizeof(double) * P);
    }
    free(bc);
    free(ec);
    free(t);
}

void or_vcycle(int d, int N, const double *c, double *u, const double *b)
{
    or_cycle(d, N, c, 1, 1, 1, u, b);
}

/* Cycles until ||b - A u_k||_2 <= tol * ||b - A u_0||_2 (the stopping rule
 * on the reduction of the relative residual, Section 4).  hist[k] receives
 * ||r_k||_2 for k = 0..cycles (capacity maxc + 1).  Returns the number of
 * cycles taken, or -maxc if the tolerance was not met. */
int or_solve(int d, int N, const double *c, int nu1, int nu2, int gamma,
             double *u, const double *b, double tol, int maxc, double *hist)
{
    long P = npts(d, N);
    double *r = malloc(sizeof(double) * P);
    or_residual(d, N, u, b, r);
    double r0 = or_norm2(P, r);
    hist[0] = r0;
    int k = 0, done = (r0 == 0.0);
    while (!done && k < maxc) {
        or_cycle(d, N, c, nu1, nu2, gamma, u, b);
        k++;
        or_residual(d, N, u, b, r);
        hist[k] = or_norm2(P, r);
        if (hist[k] <= tol * r0) done = 1;
    }
    free(r);
    return done ? k : -maxc;
}

/* ------------------------------------------------------ adjoint cycle */

static double dot(long n, const double *a, const double *b)
{
    double s = 0.0;
    for (long p = 0; p < n; p++) s += a[p] * b[p];
    return s;
}

/* cbar[j] += h^2 <ubar, K_j r>: derivative of <ubar, M r> with respect to the
 * coefficient c_j of M = h^2 sum_j c_j K_j. */
static void coef_grad(int d, int N, const double *ubar, const double *r,
                      double *cbar)
{
    long P = npts(d, N);
    double h2 = 1.0 / ((double)N * (double)N);
    double *t = malloc(sizeof(double) * P);
    for (int j = 0; j < ncoef(d); j++) {
        or_apply_K(d, N, j, r, t);
        cbar[j] += h2 * dot(P, ubar, t);
    }
    free(t);
}

/* Reverse-mode derivative of one V(1,1) cycle u_out = V(u, b; c) on the grid
 * with N intervals.  Given ubar_out = dL/du_out, writes ubar_in = dL/du and
 * accumulates bbar += dL/db and cbar[j] += dL/dc_j.  The forward states are
 * recomputed first; the reverse sweep walks the cycle backwards, using
 * A^T = A, M^T = M (symmetric stencils under zero extension) and the explicit
 * transposes of the transfer operators. */
void or_vcycle_adjoint(int d, int N, const double *c, const double *u,
                       const double *b, const double *ubar_out,
                       double *ubar_in, double *bbar, double *cbar)
{
    long P = npts(d, N);
    if (N <= 4) {
        /* u_out = A^{-1} b does not depend on u; dL/db = A^{-1} ubar_out */
        double *t = malloc(sizeof(double) * P);
        or_direct_solve(d, N, ubar_out, t);
        for (long p = 0; p < P; p++) {
            bbar[p] += t[p];
            ubar_in[p] = 0.0;
        }
        free(t);
        return;
    }
    long Pc = npts(d, N / 2);
    double *r1 = malloc(sizeof(double) * P);
    double *u1 = malloc(sizeof(double) * P);
    double *u2 = malloc(sizeof(double) * P);
    double *r3 = malloc(sizeof(double) * P);
    double *t = malloc(sizeof(double) * P);
    double *w = malloc(sizeof(double) * P);
    double *bc = malloc(sizeof(double) * Pc);
    double *ec = calloc((size_t)Pc, sizeof(double));
    /* forward recomputation */
    or_residual(d, N, u, b, r1);
    or_apply_W(d, N, c, r1, t);
    for (long p = 0; p < P; p++) u1[p] = u[p] + t[p];
    or_residual(d, N, u1, b, t);
    or_restrict(d, N, t, bc);
    or_vcycle(d, N / 2, c, ec, bc);
    memcpy(u2, u1, sizeof(double) * P);
    or_prolong_add(d, N, ec, u2);
    or_residual(d, N, u2, b, r3);

    /* reverse: post-smoothing u_out = u2 + M r3, r3 = b - A u2 */
    double *ubar2 = malloc(sizeof(double) * P);
    coef_grad(d, N, ubar_out, r3, cbar);
    or_apply_W(d, N, c, ubar_out, w);
    or_apply_A(d, N, w, t);
    for (long p = 0; p < P; p++) {
        bbar[p] += w[p];
        ubar2[p] = ubar_out[p] - t[p];
    }
    /* correction u2 = u1 + P ec */
    double *ecbar = calloc((size_t)Pc, sizeof(double));
    double *bcbar = calloc((size_t)Pc, sizeof(double));
    double *ucbar = malloc(sizeof(double) * Pc);
    double *zero_c = calloc((size_t)Pc, sizeof(double));
    or_prolong_T_add(d, N, ubar2, ecbar);
    /* coarse cycle ec = V(0, bc) */
    or_vcycle_adjoint(d, N / 2, c, zero_c, bc, ecbar, ucbar, bcbar, cbar);
    /* restriction bc = R (b - A u1) */
    double *rbar = calloc((size_t)P, sizeof(double));
    or_restrict_T_add(d, N, bcbar, rbar);
    or_apply_A(d, N, rbar, t);
    double *ubar1 = malloc(sizeof(double) * P);
    for (long p = 0; p < P; p++) {
        bbar[p] += rbar[p];
        ubar1[p] = ubar2[p] - t[p];
    }
    /* pre-smoothing u1 = u + M r1, r1 = b - A u */
    coef_grad(d, N, ubar1, r1, cbar);
    or_apply_W(d, N, c, ubar1, w);
    or_apply_A(d, N, w, t);
    for (long p = 0; p < P; p++) {
        bbar[p] += w[p];
        ubar_in[p] = ubar1[p] - t[p];
    }
    free(r1); free(u1); free(u2); free(r3); free(t); free(w);
    free(bc); free(ec); free(ubar2); free(ecbar); free(bcbar); free(ucbar);
    free(zero_c); free(rbar); free(ubar1);
}
