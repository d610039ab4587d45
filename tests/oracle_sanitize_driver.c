/*
 * Driver for the sanitizer build of the oracle (tests/test_oracle_sanitize.py):
 * calls every entry point of oracle/oracle.c on small lattices -- 4^4 with 2^4
 * blocks and complex boundary phases, and an anisotropic 4x2x4x8 lattice -- so
 * that AddressSanitizer and UndefinedBehaviorSanitizer see every loop, index
 * and buffer the oracle has.  Links are near the identity (a small random
 * deformation, 1 + C positive definite); sources are random.  Checks a few
 * results (the solve converges, the residuals are finite) and exits 0.
 */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex cplx;

typedef struct {
    int L[4], blk[4];
    double kappa, csw, phase_re[4], phase_im[4];
    int n_sap, n_jac;
} orc_params;

void orc_gamma(int mu, double *out);
int orc_site_colour(const orc_params *p, long n);
void orc_clover_field(const orc_params *p, const cplx *U, cplx *C);
int orc_clover_inverse(const orc_params *p, const cplx *C, cplx *Cinv);
void orc_hop(const orc_params *p, const cplx *U, const cplx *x, cplx *y, int part);
void orc_dirac_D(const orc_params *p, const cplx *U, const cplx *C, const cplx *x, cplx *y);
void orc_dirac_A(const orc_params *p, const cplx *U, const cplx *Cinv, const cplx *x, cplx *y);
void orc_dirac_D_sites(const orc_params *p, const cplx *U, const cplx *x, const long *sites, long ns, cplx *y);
int orc_dirac_A_sites(const orc_params *p, const cplx *U, const cplx *x, const long *sites, long ns, cplx *y);
void orc_block_apply(const orc_params *p, const cplx *U, const cplx *Cinv, const cplx *x, cplx *y, int colour,
                     int part);
void orc_jacobi(const orc_params *p, const cplx *U, const cplx *Cinv, const cplx *b, cplx *x, int colour);
void orc_sap(const orc_params *p, const cplx *U, const cplx *Cinv, const cplx *b, cplx *x);
void orc_amsap(const orc_params *p, const cplx *U, const cplx *Cinv, const cplx *b, cplx *x);
int orc_bicgstab(const orc_params *p, const cplx *U, const cplx *C, const cplx *Cinv, int op, const cplx *b, cplx *x,
                 double tol, int maxiter, int *iters, double *relres);
int orc_dci(const orc_params *p, const cplx *U, const cplx *C, const cplx *Cinv, const cplx *b, cplx *x, double tol,
            double inner_tol, int inner_maxiter, int inner_op, int round_sp, int max_outer, int *outer_iters,
            int *inner_iters_total, double *relres);
void orc_force(const orc_params *p, const cplx *U, const cplx *psi, const cplx *chi, cplx *W);
double orc_dcsw(const orc_params *p, const cplx *U, const cplx *psi, const cplx *chi);

static unsigned long long rng_state = 88172645463325252ULL;
static double urand(void) /* xorshift64, uniform in [-1, 1) */
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

static int finite_all(const cplx *v, long n)
{
    for (long i = 0; i < n; ++i)
        if (!isfinite(creal(v[i])) || !isfinite(cimag(v[i]))) return 0;
    return 1;
}

static int run(const int L[4], const int blk[4])
{
    orc_params p = {{L[0], L[1], L[2], L[3]}, {blk[0], blk[1], blk[2], blk[3]}, 0.12, 1.3,
                    {1.0, cos(0.4), 1.0, -cos(0.2)}, {0.0, sin(0.4), 0.0, -sin(0.2)}, 2, 3};
    long V = (long)L[0] * L[1] * L[2] * L[3], N = 12 * V;
    cplx *U = malloc(sizeof(cplx) * 36 * V), *C = malloc(sizeof(cplx) * 144 * V), *Ci = malloc(sizeof(cplx) * 144 * V);
    cplx *b = malloc(sizeof(cplx) * N), *x = malloc(sizeof(cplx) * N), *y = malloc(sizeof(cplx) * N);
    cplx *W = malloc(sizeof(cplx) * 36 * V);
    double g[32];
    int bad = 0;
    for (long k = 0; k < 4 * V; ++k)
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) U[k * 9 + a * 3 + c] = (a == c ? 1.0 : 0.0) + 0.05 * (urand() + I * urand());
    for (long i = 0; i < N; ++i) b[i] = urand() + I * urand();
    for (int mu = 0; mu < 5; ++mu) orc_gamma(mu, g);
    for (long n = 0; n < V; ++n) bad |= orc_site_colour(&p, n) & ~1;
    orc_clover_field(&p, U, C);
    bad |= orc_clover_inverse(&p, C, Ci) != 0;
    for (int part = 0; part < 3; ++part) orc_hop(&p, U, b, y, part);
    orc_dirac_D(&p, U, C, b, y);
    orc_dirac_A(&p, U, Ci, b, y);
    long sites[3] = {0, V / 2, V - 1};
    orc_dirac_D_sites(&p, U, b, sites, 3, y);
    bad |= orc_dirac_A_sites(&p, U, b, sites, 3, y) != 0;
    for (int colour = 0; colour < 2; ++colour) {
        for (int part = 1; part <= 2; ++part) orc_block_apply(&p, U, Ci, b, y, colour, part);
        orc_jacobi(&p, U, Ci, b, x, colour);
    }
    orc_sap(&p, U, Ci, b, x);
    orc_amsap(&p, U, Ci, b, y);
    bad |= !finite_all(x, N) || !finite_all(y, N);
    int it = 0, no = 0, ni = 0;
    double rr = 1.0;
    for (int op = 0; op < 3; ++op) {
        bad |= orc_bicgstab(&p, U, C, Ci, op, b, x, 1e-10, 2000, &it, &rr) != 0;
        bad |= !(rr < 1e-10);
    }
    bad |= orc_dci(&p, U, C, Ci, b, x, 1e-10, 1e-6, 500, 2, 1, 20, &no, &ni, &rr) != 0 || !(rr < 1e-10);
    bad |= orc_dci(&p, U, C, Ci, b, x, 1e-10, 1e-6, 500, 1, 0, 20, &no, &ni, &rr) != 0 || !(rr < 1e-10);
    orc_force(&p, U, b, x, W);
    bad |= !finite_all(W, 36 * V) || !isfinite(orc_dcsw(&p, U, b, x));
    printf("lattice %dx%dx%dx%d: %s\n", L[0], L[1], L[2], L[3], bad ? "FAILED" : "ok");
    free(U);
    free(C);
    free(Ci);
    free(b);
    free(x);
    free(y);
    free(W);
    return bad;
}

int main(void)
{
    const int L1[4] = {4, 4, 4, 4}, B1[4] = {2, 2, 2, 2};
    const int L2[4] = {4, 2, 4, 8}, B2[4] = {2, 1, 2, 2};
    int bad = run(L1, B1);
    bad |= run(L2, B2);
    return bad ? 1 : 0;
}
