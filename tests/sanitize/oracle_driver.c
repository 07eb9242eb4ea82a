/* Runs every entry point of oracle/mg_oracle.c on small 2D and 3D grids, so
 * that a build with -fsanitize=address,undefined checks the oracle's memory
 * accesses and arithmetic (tests/test_sanitize.py).  Prints nothing on
 * success; the exit status is 0 when every call returned. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

void or_apply_A(int d, int N, const double *v, double *out);
void or_apply_K(int d, int N, int which, const double *v, double *out);
void or_apply_W(int d, int N, const double *c, const double *v, double *out);
void or_residual(int d, int N, const double *u, const double *b, double *r);
void or_smooth(int d, int N, const double *c, const double *u, const double *b, double *out);
void or_restrict(int d, int N, const double *r, double *rc);
void or_prolong_add(int d, int N, const double *ec, double *u);
void or_restrict_T_add(int d, int N, const double *bc, double *rf);
void or_prolong_T_add(int d, int N, const double *uf, double *ec);
void or_direct_solve(int d, int N, const double *b, double *x);
double or_norm2(long n, const double *v);
void or_cycle(int d, int N, const double *c, int nu1, int nu2, int gamma, double *u,
              const double *b);
void or_vcycle(int d, int N, const double *c, double *u, const double *b);
int or_solve(int d, int N, const double *c, int nu1, int nu2, int gamma, double *u,
             const double *b, double tol, int maxc, double *hist);
void or_vcycle_adjoint(int d, int N, const double *c, const double *u, const double *b,
                       const double *ubar_out, double *ubar_in, double *bbar, double *cbar);
int or_num_threads(void);

static long pts(int d, int N)
{
    long p = 1;
    for (int a = 0; a < d; a++) p *= N - 1;
    return p;
}

static double *field(long n, unsigned *seed)
{
    double *v = malloc(sizeof(double) * n);
    for (long i = 0; i < n; i++) {
        *seed = *seed * 1103515245u + 12345u;
        v[i] = (double)(*seed >> 8) / (double)(1u << 24) - 0.5;
    }
    return v;
}

static int run(int d, int N)
{
    const double c2[3] = {0.28891272760249742, 0.065661983546022137, 0.019698595063806643};
    /* 3D: centre, faces, edges, corners (a 27-point stencil, so that the
     * edge and corner terms run too) */
    const double c3[4] = {0.1966, 0.0397, 0.0115, 0.0037};
    const double *c = d == 2 ? c2 : c3;
    unsigned seed = 7u + (unsigned)(d * 100 + N);
    long P = pts(d, N), Pc = pts(d, N / 2);
    double *u = field(P, &seed), *b = field(P, &seed), *t = field(P, &seed);
    double *w = field(P, &seed), *bc = field(Pc, &seed), *ec = field(Pc, &seed);
    double *ub = field(P, &seed), *ui = field(P, &seed), *bb = field(P, &seed);
    double cb[4] = {0, 0, 0, 0};
    double hist[64];
    for (int k = 0; k < (d == 2 ? 3 : 4); k++) {
        or_apply_K(d, N, k, u, t);
    }
    or_apply_A(d, N, u, t);
    or_apply_W(d, N, c, u, t);
    or_residual(d, N, u, b, t);
    or_smooth(d, N, c, u, b, w);
    or_restrict(d, N, t, bc);
    or_prolong_add(d, N, ec, w);
    or_restrict_T_add(d, N, bc, w);
    or_prolong_T_add(d, N, u, ec);
    or_direct_solve(d, 4, b, t);
    or_cycle(d, N, c, 1, 0, 2, u, b);
    or_vcycle(d, N, c, u, b);
    free(u);
    u = field(P, &seed);  /* a fresh guess: the cycles above may have solved exactly */
    int k = or_solve(d, N, c, 1, 1, 1, u, b, 1e-10, 60, hist);
    or_vcycle_adjoint(d, N, c, u, b, ub, ui, bb, cb);
    or_vcycle_adjoint(d, 4, c, u, b, ub, ui, bb, cb);
    int ok = k > 0 && isfinite(or_norm2(P, ui)) && isfinite(cb[0]) && or_num_threads() >= 1;
    free(u); free(b); free(t); free(w); free(bc); free(ec); free(ub); free(ui); free(bb);
    return ok;
}

int main(void)
{
    if (!run(2, 4) || !run(2, 16) || !run(2, 32) || !run(3, 8) || !run(3, 16)) {
        fprintf(stderr, "an oracle call returned an unexpected result\n");
        return 1;
    }
    return 0;
}
