/*
 * oracle.c -- plain, slow, FP64 CPU reference for the Clover-Wilson quark
 * solver of "102 PFLOPS Lattice QCD quark solver on Fugaku" (arXiv 2109.10687).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker that the GPU path is
 * compared against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the HIP library.
 *
 * Everything is written as the definition reads: full 4x4 spin matrices, full
 * 3x3 colour matrices, a full 12x12 clover block per site, full-lattice
 * vectors with colour masks for the Schwarz blocks.  No spin projection, no
 * compressed storage, no fused steps.
 *
 * Conventions (Appendix "Clover-Wilson Dirac operator"):
 *   site n = (x,y,z,t), index  x + Lx*(y + Ly*(z + Lz*t));  mu = 0..3 is the
 *   paper's mu = 1..4, so mu = 3 is the direction of the diagonal gamma_4.
 *   spinor element (n, colour a, spin alpha) at  n*12 + a*4 + alpha
 *   (colour outer, spin inner, as in the K-computer layout of Sec. 4).
 *   link U_mu(n)[a][b] at  ((mu*V + n)*9 + a*3 + b).
 *
 * Boundary phases are not in the paper (it never states boundary
 * conditions): a hop that crosses the lattice edge in direction mu picks up
 * phase_mu going forward and conj(phase_mu) going backward.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* loops over fewer sites than this run on one thread (thread start-up costs more) */
#define PAR_MIN 4096

typedef struct {
    int L[4];            /* Lx, Ly, Lz, Lt */
    int blk[4];          /* Schwarz block extent per direction */
    double kappa;
    double csw;
    double phase_re[4];  /* boundary phase per direction */
    double phase_im[4];
    int n_sap;           /* loop count of the SAP preconditioner (Alg. 1) */
    int n_jac;           /* number of A_EE applications in Alg. 2 */
} orc_params;

/* ---------------------------------------------------------------------- */
/* gamma matrices exactly as printed in the appendix (Dirac representation) */
static const double GRE[4][4][4] = {
    {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{0, 0, 0, 1}, {0, 0, -1, 0}, {0, -1, 0, 0}, {1, 0, 0, 0}},
    {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, -1, 0}, {0, 0, 0, -1}},
};
static const double GIM[4][4][4] = {
    {{0, 0, 0, 1}, {0, 0, 1, 0}, {0, -1, 0, 0}, {-1, 0, 0, 0}},
    {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{0, 0, 1, 0}, {0, 0, 0, -1}, {-1, 0, 0, 0}, {0, 1, 0, 0}},
    {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}},
};

static cplx gam(int mu, int a, int b) { return GRE[mu][a][b] + I * GIM[mu][a][b]; }

/* gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 (not defined in the paper) */
static void gamma5(cplx g5[4][4])
{
    cplx t1[4][4], t2[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += gam(0, i, k) * gam(1, k, j);
            t1[i][j] = s;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += t1[i][k] * gam(2, k, j);
            t2[i][j] = s;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += t2[i][k] * gam(3, k, j);
            g5[i][j] = s;
        }
}

/* export: gamma_mu (mu = 0..3) or gamma_5 (mu = 4) as 16 complex numbers */
void orc_gamma(int mu, double *out)
{
    cplx g[4][4];
    if (mu == 4) {
        gamma5(g);
    } else {
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) g[i][j] = gam(mu, i, j);
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            out[2 * (i * 4 + j)] = creal(g[i][j]);
            out[2 * (i * 4 + j) + 1] = cimag(g[i][j]);
        }
}

/* ---------------------------------------------------------------------- */
/* geometry */

static long volume(const orc_params *p) { return (long)p->L[0] * p->L[1] * p->L[2] * p->L[3]; }

static void coords(const orc_params *p, long n, int c[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = (int)(n % p->L[mu]);
        n /= p->L[mu];
    }
}

static long index_of(const orc_params *p, const int c[4])
{
    return c[0] + (long)p->L[0] * (c[1] + (long)p->L[1] * (c[2] + (long)p->L[2] * c[3]));
}

/* neighbour n + dir*mu_hat with periodic wrap */
static long shift(const orc_params *p, long n, int mu, int dir)
{
    int c[4];
    coords(p, n, c);
    c[mu] = (c[mu] + dir + p->L[mu]) % p->L[mu];
    return index_of(p, c);
}

static cplx phase(const orc_params *p, int mu) { return p->phase_re[mu] + I * p->phase_im[mu]; }

/* factor on the forward hop n -> n+mu (phase_mu when it crosses the edge) */
static cplx fwd_phase(const orc_params *p, long n, int mu)
{
    int c[4];
    coords(p, n, c);
    return (c[mu] == p->L[mu] - 1) ? phase(p, mu) : 1.0;
}

/* factor on the backward hop n -> n-mu (conjugate phase when it crosses) */
static cplx bwd_phase(const orc_params *p, long n, int mu)
{
    int c[4];
    coords(p, n, c);
    return (c[mu] == 0) ? conj(phase(p, mu)) : 1.0;
}

/* Schwarz block of a site and its colour (parity of the block coordinates),
 * Sec. 3: domains coloured by the even- or oddness of their indices. */
static long block_of(const orc_params *p, long n)
{
    int c[4];
    coords(p, n, c);
    long b = 0, stride = 1;
    for (int mu = 0; mu < 4; ++mu) {
        b += (c[mu] / p->blk[mu]) * stride;
        stride *= p->L[mu] / p->blk[mu];
    }
    return b;
}

int orc_site_colour(const orc_params *p, long n)
{
    int c[4];
    coords(p, n, c);
    int s = 0;
    for (int mu = 0; mu < 4; ++mu) s += c[mu] / p->blk[mu];
    return s & 1;
}

/* ---------------------------------------------------------------------- */
/* 3x3 colour algebra */

static const cplx *link(const cplx *U, long V, int mu, long n) { return U + ((long)mu * V + n) * 9; }

static void mat_mul(const cplx *A, const cplx *B, cplx *C)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[k * 3 + j];
            C[i * 3 + j] = s;
        }
}

static void mat_dag(const cplx *A, cplx *B)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[i * 3 + j] = conj(A[j * 3 + i]);
}

/* product of four matrices, each optionally daggered */
static void mat_prod4(const cplx *M[4], const int dag[4], cplx *out)
{
    cplx acc[9], tmp[9], m[9];
    for (int i = 0; i < 9; ++i) acc[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int k = 0; k < 4; ++k) {
        if (dag[k])
            mat_dag(M[k], m);
        else
            memcpy(m, M[k], sizeof m);
        mat_mul(acc, m, tmp);
        memcpy(acc, tmp, sizeof acc);
    }
    memcpy(out, acc, sizeof acc);
}

/* ---------------------------------------------------------------------- */
/* clover term (Appendix): C = (i/2) kappa c_SW sigma_{mu nu} F_{mu nu}, summed
 * over all ordered pairs, sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu].  F is the
 * field strength; the paper gives no formula for it, and this oracle takes the
 * four-leaf clover:  Q = sum of the four counter-clockwise plaquettes in the
 * (mu,nu) plane that start and end at n,  F = (Q - Q^dagger)/8. */

static void clover_Q(const orc_params *p, const cplx *U, long n, int mu, int nu, cplx Q[9])
{
    long V = volume(p);
    long n_pm = shift(p, n, mu, +1), n_pn = shift(p, n, nu, +1);
    long n_mm = shift(p, n, mu, -1), n_mn = shift(p, n, nu, -1);
    long n_mm_pn = shift(p, n_mm, nu, +1);
    long n_mm_mn = shift(p, n_mm, nu, -1);
    long n_pm_mn = shift(p, n_pm, nu, -1);
    cplx leaf[9];
    for (int i = 0; i < 9; ++i) Q[i] = 0;

    /* leaf 1: n -> n+mu -> n+mu+nu -> n+nu -> n */
    const cplx *l1[4] = {link(U, V, mu, n), link(U, V, nu, n_pm), link(U, V, mu, n_pn), link(U, V, nu, n)};
    const int d1[4] = {0, 0, 1, 1};
    mat_prod4(l1, d1, leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];

    /* leaf 2: n -> n+nu -> n-mu+nu -> n-mu -> n */
    const cplx *l2[4] = {link(U, V, nu, n), link(U, V, mu, n_mm_pn), link(U, V, nu, n_mm), link(U, V, mu, n_mm)};
    const int d2[4] = {0, 1, 1, 0};
    mat_prod4(l2, d2, leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];

    /* leaf 3: n -> n-mu -> n-mu-nu -> n-nu -> n */
    const cplx *l3[4] = {link(U, V, mu, n_mm), link(U, V, nu, n_mm_mn), link(U, V, mu, n_mm_mn), link(U, V, nu, n_mn)};
    const int d3[4] = {1, 1, 0, 0};
    mat_prod4(l3, d3, leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];

    /* leaf 4: n -> n-nu -> n+mu-nu -> n+mu -> n */
    const cplx *l4[4] = {link(U, V, nu, n_mn), link(U, V, mu, n_mn), link(U, V, nu, n_pm_mn), link(U, V, mu, n)};
    const int d4[4] = {1, 0, 0, 1};
    mat_prod4(l4, d4, leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];
}

/* the clover block C(n) (without the identity) as a 12x12 matrix, row index
 * a*4+alpha, column index b*4+beta */
static void clover_site(const orc_params *p, const cplx *U, long n, cplx C[144])
{
    for (int i = 0; i < 144; ++i) C[i] = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu) {
            if (mu == nu) continue;
            cplx Q[9], F[9];
            clover_Q(p, U, n, mu, nu, Q);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) F[a * 3 + b] = (Q[a * 3 + b] - conj(Q[b * 3 + a])) / 8.0;
            cplx sig[4][4];
            for (int al = 0; al < 4; ++al)
                for (int be = 0; be < 4; ++be) {
                    cplx c = 0;
                    for (int k = 0; k < 4; ++k) c += gam(mu, al, k) * gam(nu, k, be) - gam(nu, al, k) * gam(mu, k, be);
                    sig[al][be] = 0.5 * I * c;
                }
            cplx pref = 0.5 * I * p->kappa * p->csw;
            for (int a = 0; a < 3; ++a)
                for (int al = 0; al < 4; ++al)
                    for (int b = 0; b < 3; ++b)
                        for (int be = 0; be < 4; ++be) C[(a * 4 + al) * 12 + b * 4 + be] += pref * sig[al][be] * F[a * 3 + b];
        }
}

void orc_clover_field(const orc_params *p, const cplx *U, cplx *C)
{
    long V = volume(p);
#pragma omp parallel for schedule(static) if (V >= PAR_MIN)
    for (long n = 0; n < V; ++n) clover_site(p, U, n, C + n * 144);
}

/* inverse of a 12x12 complex matrix by Gauss-Jordan elimination with partial
 * pivoting; returns 0 on success, 1 if a pivot vanishes */
static int invert12(const cplx *M, cplx *Minv)
{
    cplx a[12][24];
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) {
            a[i][j] = M[i * 12 + j];
            a[i][12 + j] = (i == j) ? 1.0 : 0.0;
        }
    for (int col = 0; col < 12; ++col) {
        int piv = col;
        for (int r = col + 1; r < 12; ++r)
            if (cabs(a[r][col]) > cabs(a[piv][col])) piv = r;
        if (cabs(a[piv][col]) == 0.0) return 1;
        if (piv != col)
            for (int j = 0; j < 24; ++j) {
                cplx t = a[col][j];
                a[col][j] = a[piv][j];
                a[piv][j] = t;
            }
        cplx inv = 1.0 / a[col][col];
        for (int j = 0; j < 24; ++j) a[col][j] *= inv;
        for (int r = 0; r < 12; ++r) {
            if (r == col) continue;
            cplx f = a[r][col];
            if (f == 0) continue;
            for (int j = 0; j < 24; ++j) a[r][j] -= f * a[col][j];
        }
    }
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) Minv[i * 12 + j] = a[i][12 + j];
    return 0;
}

/* C_inv = (1 + C)^{-1} per site; returns the number of singular sites */
int orc_clover_inverse(const orc_params *p, const cplx *C, cplx *Cinv)
{
    long V = volume(p);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad) if (V >= PAR_MIN)
    for (long n = 0; n < V; ++n) {
        cplx M[144];
        for (int i = 0; i < 144; ++i) M[i] = C[n * 144 + i] + ((i % 13 == 0) ? 1.0 : 0.0);
        bad += invert12(M, Cinv + n * 144);
    }
    return bad;
}

/* ---------------------------------------------------------------------- */
/* hopping term (Sec. 3 and the appendix):
 *   (H x)(n) = sum_mu [ (1 - gamma_mu) U_mu(n) x(n+mu)
 *                      + (1 + gamma_mu) U_mu(n-mu)^dagger x(n-mu) ]
 * part = 0: every hop;  1: only hops inside one Schwarz block;
 *        2: only hops between different blocks.                            */

enum { PART_ALL = 0, PART_IN = 1, PART_OUT = 2 };

static int hop_selected(const orc_params *p, long n, long m, int part)
{
    if (part == PART_ALL) return 1;
    int same = block_of(p, n) == block_of(p, m);
    return part == PART_IN ? same : !same;
}

/* ys[0..11] += coef * sum of the selected hops of x into site n */
static void hop_site(const orc_params *p, const cplx *U, const cplx *x, long n, int part, cplx coef, cplx *ys)
{
    long V = volume(p);
    for (int mu = 0; mu < 4; ++mu) {
        for (int dir = +1; dir >= -1; dir -= 2) {
            long m = shift(p, n, mu, dir);
            if (!hop_selected(p, n, m, part)) continue;
            cplx W[9]; /* colour matrix acting on x(m) */
            cplx ph;
            if (dir > 0) {
                memcpy(W, link(U, V, mu, n), sizeof W);
                ph = fwd_phase(p, n, mu);
            } else {
                mat_dag(link(U, V, mu, m), W);
                ph = bwd_phase(p, n, mu);
            }
            /* colour step: w[a][beta] = sum_b W[a][b] x(m)[b][beta] */
            cplx w[12];
            for (int a = 0; a < 3; ++a)
                for (int be = 0; be < 4; ++be) {
                    cplx s = 0;
                    for (int b = 0; b < 3; ++b) s += W[a * 3 + b] * x[m * 12 + b * 4 + be];
                    w[a * 4 + be] = s;
                }
            /* spin step: (1 -/+ gamma_mu)[alpha][beta] */
            for (int a = 0; a < 3; ++a)
                for (int al = 0; al < 4; ++al) {
                    cplx s = 0;
                    for (int be = 0; be < 4; ++be) {
                        cplx P = ((al == be) ? 1.0 : 0.0) - (double)dir * gam(mu, al, be);
                        s += P * w[a * 4 + be];
                    }
                    ys[a * 4 + al] += coef * ph * s;
                }
        }
    }
}

void orc_hop(const orc_params *p, const cplx *U, const cplx *x, cplx *y, int part)
{
    long V = volume(p);
#pragma omp parallel for schedule(static) if (V >= PAR_MIN)
    for (long n = 0; n < V; ++n) {
        for (int i = 0; i < 12; ++i) y[n * 12 + i] = 0;
        hop_site(p, U, x, n, part, 1.0, y + n * 12);
    }
}

static void mat12_vec(const cplx *M, const cplx *v, cplx *out)
{
    for (int i = 0; i < 12; ++i) {
        cplx s = 0;
        for (int j = 0; j < 12; ++j) s += M[i * 12 + j] * v[j];
        out[i] = s;
    }
}

/* D x = (1 + C) x - kappa H x   (appendix) */
void orc_dirac_D(const orc_params *p, const cplx *U, const cplx *C, const cplx *x, cplx *y)
{
    long V = volume(p);
#pragma omp parallel for schedule(static) if (V >= PAR_MIN)
    for (long n = 0; n < V; ++n) {
        cplx cx[12];
        mat12_vec(C + n * 144, x + n * 12, cx);
        for (int i = 0; i < 12; ++i) y[n * 12 + i] = x[n * 12 + i] + cx[i];
        hop_site(p, U, x, n, PART_ALL, -p->kappa, y + n * 12);
    }
}

/* A x = x - kappa C_inv H x   (Sec. 3, A = C_inv D) */
void orc_dirac_A(const orc_params *p, const cplx *U, const cplx *Cinv, const cplx *x, cplx *y)
{
    long V = volume(p);
#pragma omp parallel for schedule(static) if (V >= PAR_MIN)
    for (long n = 0; n < V; ++n) {
        cplx h[12], ch[12];
        for (int i = 0; i < 12; ++i) h[i] = 0;
        hop_site(p, U, x, n, PART_ALL, 1.0, h);
        mat12_vec(Cinv + n * 144, h, ch);
        for (int i = 0; i < 12; ++i) y[n * 12 + i] = x[n * 12 + i] - p->kappa * ch[i];
    }
}

/* (D x)(n) at a list of sites, building the clover of each listed site on
 * the fly from U (no V*144 clover array), for lattices too large to hold the
 * full clover field in host memory. */
void orc_dirac_D_sites(const orc_params *p, const cplx *U, const cplx *x, const long *sites, long ns, cplx *y)
{
#pragma omp parallel for schedule(dynamic, 16) if (ns >= 64)
    for (long k = 0; k < ns; ++k) {
        long n = sites[k];
        cplx C[144], cx[12], acc[12];
        clover_site(p, U, n, C);
        mat12_vec(C, x + n * 12, cx);
        for (int i = 0; i < 12; ++i) acc[i] = x[n * 12 + i] + cx[i];
        hop_site(p, U, x, n, PART_ALL, -p->kappa, acc);
        for (int i = 0; i < 12; ++i) y[k * 12 + i] = acc[i];
    }
}

/* (A x)(n) = x(n) - kappa C_inv(n) (H x)(n) at a list of sites (Sec. 3), the clover
 * of each listed site built on the fly and inverted there (Gauss-Jordan, as
 * orc_clover_inverse); returns the number of sites where 1 + C was singular. */
int orc_dirac_A_sites(const orc_params *p, const cplx *U, const cplx *x, const long *sites, long ns, cplx *y)
{
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) if (ns >= 64) reduction(+ : bad)
    for (long k = 0; k < ns; ++k) {
        long n = sites[k];
        cplx C[144], Ci[144], hx[12], t[12];
        clover_site(p, U, n, C);
        for (int i = 0; i < 12; ++i) C[i * 12 + i] += 1.0;
        if (invert12(C, Ci)) ++bad;
        for (int i = 0; i < 12; ++i) hx[i] = 0;
        hop_site(p, U, x, n, PART_ALL, 1.0, hx);
        mat12_vec(Ci, hx, t);
        for (int i = 0; i < 12; ++i) y[k * 12 + i] = x[n * 12 + i] - p->kappa * t[i];
    }
    return bad;
}

/* ---------------------------------------------------------------------- */
/* Schwarz block pieces of A (Sec. 3, 2x2 block form):
 *   part IN : y(n) = x(n) - kappa C_inv(n) sum_{hops inside n's block} ...   = (A_cc x)(n)
 *   part OUT: y(n) =      - kappa C_inv(n) sum_{hops from other blocks} ...  = (A_{c,c'} x)(n)
 * Only rows n of colour `colour` are written; other rows of y are untouched.
 * The block neighbours across a block face always have the other colour,
 * because every direction holds an even number of blocks. */
void orc_block_apply(const orc_params *p, const cplx *U, const cplx *Cinv, const cplx *x, cplx *y, int colour, int part)
{
    long V = volume(p);
#pragma omp parallel for schedule(static) if (V >= PAR_MIN)
    for (long n = 0; n < V; ++n) {
        if (orc_site_colour(p, n) != colour) continue;
        cplx h[12], ch[12];
        for (int i = 0; i < 12; ++i) h[i] = 0;
        hop_site(p, U, x, n, part, 1.0, h);
        mat12_vec(Cinv + n * 144, h, ch);
        for (int i = 0; i < 12; ++i) {
            cplx diag = (part == PART_IN) ? x[n * 12 + i] : 0.0;
            y[n * 12 + i] = diag - p->kappa * ch[i];
        }
    }
}

/* ---------------------------------------------------------------------- */
/* vector helpers over the rows of one colour (colour < 0: every row) */

static int row_on(const orc_params *p, long n, int colour) { return colour < 0 || orc_site_colour(p, n) == colour; }

/* Alg. 2: x_c = B_cc b_c, the Jacobi (truncated Neumann) approximation of
 * A_cc^{-1} with n_jac applications of A_cc */
void orc_jacobi(const orc_params *p, const cplx *U, const cplx *Cinv, const cplx *b, cplx *x, int colour)
{
    long V = volume(p);
    cplx *q = calloc((size_t)V * 12, sizeof(cplx));
    orc_block_apply(p, U, Cinv, b, q, colour, PART_IN);
#pragma omp parallel for schedule(static) if (V >= PAR_MIN)
    for (long n = 0; n < V; ++n)
        if (row_on(p, n, colour))
            for (int i = 0; i < 12; ++i) x[n * 12 + i] = 2.0 * b[n * 12 + i] - q[n * 12 + i];
    for (int j = 1; j < p->n_jac; ++j) {
        orc_block_apply(p, U, Cinv, x, q, colour, PART_IN);
#pragma omp parallel for schedule(static) if (V >= PAR_MIN)
        for (long n = 0; n < V; ++n)
            if (row_on(p, n, colour))
                for (int i = 0; i < 12; ++i) x[n * 12 + i] = x[n * 12 + i] + b[n * 12 + i] - q[n * 12 + i];
    }
    free(q);
}

/* s_c = s_c + b_c - q_c */
static void upd_add(const orc_params *p, cplx *s, const cplx *b, const cplx *q, int colour)
{
    long V = volume(p);
#pragma omp parallel for schedule(static) if (V >= PAR_MIN)
    for (long n = 0; n < V; ++n)
        if (row_on(p, n, colour))
            for (int i = 0; i < 12; ++i) s[n * 12 + i] += b[n * 12 + i] - q[n * 12 + i];
}

/* s_c = s_c - A_{c,c'} x_{c'} */
static void upd_sub_out(const orc_params *p, const cplx *U, const cplx *Cinv, cplx *s, const cplx *x, cplx *tmp, int colour)
{
    long V = volume(p);
    orc_block_apply(p, U, Cinv, x, tmp, colour, PART_OUT);
#pragma omp parallel for schedule(static) if (V >= PAR_MIN)
    for (long n = 0; n < V; ++n)
        if (row_on(p, n, colour))
            for (int i = 0; i < 12; ++i) s[n * 12 + i] -= tmp[n * 12 + i];
}

/* Alg. 1: x = M_SAP b, with E = colour 0, O = colour 1 */
void orc_sap(const orc_params *p, const cplx *U, const cplx *Cinv, const cplx *b, cplx *x)
{
    long V = volume(p);
    size_t bytes = (size_t)V * 12 * sizeof(cplx);
    cplx *s = malloc(bytes), *q = calloc((size_t)V * 12, sizeof(cplx)), *tmp = calloc((size_t)V * 12, sizeof(cplx));
    memcpy(s, b, bytes);
    memset(x, 0, bytes);
    const int E = 0, O = 1;
    for (int i = 0; i < p->n_sap; ++i) {
        orc_jacobi(p, U, Cinv, s, x, E);                 /* x_E = B_EE s_E       */
        orc_block_apply(p, U, Cinv, x, q, E, PART_IN);   /* q_E = A_EE x_E       */
        upd_add(p, s, b, q, E);                          /* s_E = s_E + b_E - q_E */
        upd_sub_out(p, U, Cinv, s, x, tmp, O);           /* s_O = s_O - A_OE x_E */
        orc_jacobi(p, U, Cinv, s, x, O);                 /* x_O = B_OO s_O       */
        orc_block_apply(p, U, Cinv, x, q, O, PART_IN);   /* q_O = A_OO x_O       */
        upd_add(p, s, b, q, O);                          /* s_O = s_O + b_O - q_O */
        upd_sub_out(p, U, Cinv, s, x, tmp, E);           /* s_E = s_E - A_EO x_O */
    }
    orc_jacobi(p, U, Cinv, s, x, E);        /* x_E = B_EE s_E       */
    upd_sub_out(p, U, Cinv, s, x, tmp, O);  /* s_O = s_O - A_OE x_E */
    orc_jacobi(p, U, Cinv, s, x, O);        /* x_O = B_OO s_O       */
    free(s);
    free(q);
    free(tmp);
}

/* Alg. 3: x = A M_SAP b, computed as A applied to the output of Alg. 1 */
void orc_amsap(const orc_params *p, const cplx *U, const cplx *Cinv, const cplx *b, cplx *x)
{
    long V = volume(p);
    cplx *m = malloc((size_t)V * 12 * sizeof(cplx));
    orc_sap(p, U, Cinv, b, m);
    orc_dirac_A(p, U, Cinv, m, x);
    free(m);
}

/* ---------------------------------------------------------------------- */
/* BiCGStab, Alg. 5.  <a|b> = sum conj(a_i) b_i.
 * op = 0: D (plain);  1: A = C_inv D (plain);  2: A M_SAP (right-
 * preconditioned: solves A M y = b, returns x = M y, Sec. 3). */

typedef struct {
    const orc_params *p;
    const cplx *U, *C, *Cinv;
    int op;
} orc_system;

static void apply_op(const orc_system *s, const cplx *in, cplx *out)
{
    if (s->op == 0)
        orc_dirac_D(s->p, s->U, s->C, in, out);
    else if (s->op == 1)
        orc_dirac_A(s->p, s->U, s->Cinv, in, out);
    else
        orc_amsap(s->p, s->U, s->Cinv, in, out);
}

static cplx dotc(long N, const cplx *a, const cplx *b)
{
    double sr = 0, si = 0;
#pragma omp parallel for schedule(static) reduction(+ : sr, si) if (N >= 12 * PAR_MIN)
    for (long i = 0; i < N; ++i) {
        cplx t = conj(a[i]) * b[i];
        sr += creal(t);
        si += cimag(t);
    }
    return sr + I * si;
}

static double norm2(long N, const cplx *a) { return creal(dotc(N, a, a)); }

/* returns 0 converged, 1 maxiter reached, 2 breakdown; *iters = loop passes */
int orc_bicgstab(const orc_params *p, const cplx *U, const cplx *C, const cplx *Cinv, int op, const cplx *b, cplx *x,
                 double tol, int maxiter, int *iters, double *relres)
{
    long N = volume(p) * 12;
    size_t bytes = (size_t)N * sizeof(cplx);
    orc_system sys = {p, U, C, Cinv, op};
    cplx *r = malloc(bytes), *pv = malloc(bytes), *rt = malloc(bytes), *q = malloc(bytes), *t = malloc(bytes);
    cplx *y = calloc((size_t)N, sizeof(cplx));
    memcpy(r, b, bytes);
    memcpy(pv, b, bytes);
    memcpy(rt, b, bytes);
    double bnorm2 = norm2(N, b);
    cplx rho0 = bnorm2;
    int status = 1, it = 0;
    double rnorm2 = bnorm2;
    if (bnorm2 == 0.0) {
        status = 0;
        goto done;
    }
    for (it = 0; it < maxiter; ++it) {
        apply_op(&sys, pv, q);
        cplx rq = dotc(N, rt, q);
        if (rq == 0) {
            status = 2;
            break;
        }
        cplx alpha = rho0 / rq;
        for (long i = 0; i < N; ++i) {
            y[i] += alpha * pv[i];
            r[i] -= alpha * q[i];
        }
        rnorm2 = norm2(N, r);
        if (sqrt(rnorm2 / bnorm2) < tol) {
            status = 0;
            ++it;
            break;
        }
        apply_op(&sys, r, t);
        double tt = norm2(N, t);
        if (tt == 0.0) {
            status = 2;
            break;
        }
        cplx omega = dotc(N, t, r) / tt;
        for (long i = 0; i < N; ++i) {
            y[i] += omega * r[i];
            r[i] -= omega * t[i];
        }
        rnorm2 = norm2(N, r);
        cplx rho = dotc(N, rt, r);
        if (sqrt(rnorm2 / bnorm2) < tol) {
            status = 0;
            ++it;
            break;
        }
        if (omega == 0 || rho0 == 0) {
            status = 2;
            break;
        }
        cplx beta = alpha * rho / (rho0 * omega);
        rho0 = rho;
        for (long i = 0; i < N; ++i) pv[i] = r[i] + beta * (pv[i] - omega * q[i]);
    }
done:
    if (op == 2)
        orc_sap(p, U, Cinv, y, x); /* x = M_SAP y */
    else
        memcpy(x, y, bytes);
    if (iters) *iters = it;
    if (relres) *relres = sqrt(rnorm2 / (bnorm2 > 0 ? bnorm2 : 1.0));
    free(r);
    free(pv);
    free(rt);
    free(q);
    free(t);
    free(y);
    return status;
}

/* ---------------------------------------------------------------------- */
/* Alg. 4: defect correction for D x = b.  The outer residual is the true
 * residual r = b - D x.  The inner solver works on A = C_inv D, whose source
 * for the outer residual r is C_inv r; the rescaling by err keeps the inner
 * source at unit norm.  inner_op selects the inner solver (1: plain A,
 * 2: A M_SAP).  When round_sp is set, the inner source and the inner solution
 * are rounded to single precision (R_SP, P_DP) component by component.
 * Returns 0 converged, 1 outer limit reached. */
int orc_dci(const orc_params *p, const cplx *U, const cplx *C, const cplx *Cinv, const cplx *b, cplx *x, double tol,
            double inner_tol, int inner_maxiter, int inner_op, int round_sp, int max_outer, int *outer_iters,
            int *inner_iters_total, double *relres)
{
    long V = volume(p), N = V * 12;
    size_t bytes = (size_t)N * sizeof(cplx);
    cplx *r = malloc(bytes), *c = malloc(bytes), *d = malloc(bytes), *Dx = malloc(bytes);
    memset(x, 0, bytes);
    memcpy(r, b, bytes);
    double bnorm = sqrt(norm2(N, b));
    double err = bnorm;
    int outer = 0, inner_total = 0, status = 1;
    if (bnorm == 0.0) {
        status = 0;
        goto done;
    }
    while (outer < max_outer) {
        /* p = R_SP(C_inv r / err) */
        for (long n = 0; n < V; ++n) {
            cplx v[12];
            for (int i = 0; i < 12; ++i) v[i] = r[n * 12 + i] / err;
            mat12_vec(Cinv + n * 144, v, c + n * 12);
        }
        if (round_sp)
            for (long i = 0; i < N; ++i) c[i] = (double)(float)creal(c[i]) + I * (double)(float)cimag(c[i]);
        int it = 0;
        double rr;
        orc_bicgstab(p, U, C, Cinv, inner_op, c, d, inner_tol, inner_maxiter, &it, &rr);
        inner_total += it;
        if (round_sp)
            for (long i = 0; i < N; ++i) d[i] = (double)(float)creal(d[i]) + I * (double)(float)cimag(d[i]);
        for (long i = 0; i < N; ++i) x[i] += err * d[i]; /* x = x + err P_DP(q) */
        orc_dirac_D(p, U, C, x, Dx);
        for (long i = 0; i < N; ++i) r[i] = b[i] - Dx[i];
        err = sqrt(norm2(N, r));
        ++outer;
        if (err / bnorm < tol) {
            status = 0;
            break;
        }
    }
done:
    if (outer_iters) *outer_iters = outer;
    if (inner_iters_total) *inner_iters_total = inner_total;
    if (relres) *relres = err / (bnorm > 0 ? bnorm : 1.0);
    free(r);
    free(c);
    free(d);
    free(Dx);
    return status;
}

/* ---------------------------------------------------------------------- */
/* Derivative of L = |D^{-1} phi|^2 with respect to the links (fermion force).
 * With psi = D^{-1} phi and chi = D^{-dagger} psi, dL = -2 Re <chi| dD psi>.
 * Written as dL = Re sum_links tr(dU_mu(n) W_mu(n)); this function returns W.
 *   hop part:    W += 2 kappa phase * ( [(1 - gamma_mu) psi(n+mu)] chi(n)^dagger
 *                                     + ( [(1 + gamma_mu) psi(n)] chi(n+mu)^dagger )^dagger )
 *   clover part: C = i kappa c_SW sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu} with
 *                F = (Q - Q^dagger)/8 gives dL = Re sum tr(dQ_{mu nu}(n) Y_{mu nu}(n)),
 *                Y = (-i kappa c_SW / 4) (Lambda + Lambda^dagger),
 *                Lambda_{ba} = sum_{alpha beta} sigma[alpha][beta] psi_{b beta} conj(chi_{a alpha});
 *                a leaf written A U B (U at one position) adds B Y A to W of that
 *                link, a leaf written A U^dagger B adds (B Y A)^dagger.
 * The clover part is accumulated by visiting every base site, plane, leaf and
 * position in turn (sequential: positions of different sites hit the same link). */

static void mat_mul_acc(const cplx *A, const cplx *B, cplx *C) /* C = A B */
{
    cplx t[9];
    mat_mul(A, B, t);
    memcpy(C, t, sizeof t);
}

void orc_force(const orc_params *p, const cplx *U, const cplx *psi, const cplx *chi, cplx *W)
{
    long V = volume(p);
    memset(W, 0, (size_t)4 * V * 9 * sizeof(cplx));
    /* hop part */
    for (long n = 0; n < V; ++n)
        for (int mu = 0; mu < 4; ++mu) {
            long m = shift(p, n, mu, +1);
            cplx ph = fwd_phase(p, n, mu);
            cplx Pm[12], Pp[12]; /* (1 - gamma) psi(n+mu), (1 + gamma) psi(n) as [colour][spin] */
            for (int a = 0; a < 3; ++a)
                for (int al = 0; al < 4; ++al) {
                    cplx s1 = 0, s2 = 0;
                    for (int be = 0; be < 4; ++be) {
                        cplx g = gam(mu, al, be);
                        cplx d = (al == be) ? 1.0 : 0.0;
                        s1 += (d - g) * psi[m * 12 + a * 4 + be];
                        s2 += (d + g) * psi[n * 12 + a * 4 + be];
                    }
                    Pm[a * 4 + al] = s1;
                    Pp[a * 4 + al] = s2;
                }
            cplx *w = W + ((long)mu * V + n) * 9;
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) {
                    cplx F = 0, G = 0; /* F_ba, G_ab */
                    for (int al = 0; al < 4; ++al) {
                        F += Pm[b * 4 + al] * conj(chi[n * 12 + a * 4 + al]);
                        G += Pp[a * 4 + al] * conj(chi[m * 12 + b * 4 + al]);
                    }
                    /* W_ba += 2 kappa ph (F_ba + conj(G_ab)) */
                    w[b * 3 + a] += 2.0 * p->kappa * ph * (F + conj(G));
                }
        }
    /* clover part */
    if (p->csw == 0.0) return;
    for (long n = 0; n < V; ++n)
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                cplx sig[4][4];
                for (int al = 0; al < 4; ++al)
                    for (int be = 0; be < 4; ++be) {
                        cplx c = 0;
                        for (int k = 0; k < 4; ++k) c += gam(mu, al, k) * gam(nu, k, be) - gam(nu, al, k) * gam(mu, k, be);
                        sig[al][be] = 0.5 * I * c;
                    }
                cplx Lam[9], Y[9];
                for (int b = 0; b < 3; ++b)
                    for (int a = 0; a < 3; ++a) {
                        cplx s = 0;
                        for (int al = 0; al < 4; ++al)
                            for (int be = 0; be < 4; ++be) s += sig[al][be] * psi[n * 12 + b * 4 + be] * conj(chi[n * 12 + a * 4 + al]);
                        Lam[b * 3 + a] = s;
                    }
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) Y[i * 3 + j] = (-0.25 * I * p->kappa * p->csw) * (Lam[i * 3 + j] + conj(Lam[j * 3 + i]));
                /* the four leaves of Q_{mu nu}(n), as in clover_Q: (site, direction, daggered) */
                long n_pm = shift(p, n, mu, +1), n_pn = shift(p, n, nu, +1);
                long n_mm = shift(p, n, mu, -1), n_mn = shift(p, n, nu, -1);
                long n_mm_pn = shift(p, n_mm, nu, +1), n_mm_mn = shift(p, n_mm, nu, -1);
                long n_pm_mn = shift(p, n_pm, nu, -1);
                const long ls[4][4] = {{n, n_pm, n_pn, n}, {n, n_mm_pn, n_mm, n_mm}, {n_mm, n_mm_mn, n_mm_mn, n_mn},
                                       {n_mn, n_mn, n_pm_mn, n}};
                const int ld[4][4] = {{mu, nu, mu, nu}, {nu, mu, nu, mu}, {mu, nu, mu, nu}, {nu, mu, nu, mu}};
                const int lg[4][4] = {{0, 0, 1, 1}, {0, 1, 1, 0}, {1, 1, 0, 0}, {1, 0, 0, 1}};
                for (int lf = 0; lf < 4; ++lf) {
                    cplx M[4][9];
                    for (int k = 0; k < 4; ++k) {
                        const cplx *Uk = link(U, V, ld[lf][k], ls[lf][k]);
                        if (lg[lf][k])
                            mat_dag(Uk, M[k]);
                        else
                            memcpy(M[k], Uk, sizeof M[k]);
                    }
                    for (int pos = 0; pos < 4; ++pos) {
                        cplx A[9], B[9], T[9], R[9];
                        for (int i = 0; i < 9; ++i) A[i] = B[i] = (i % 4 == 0) ? 1.0 : 0.0;
                        for (int k = 0; k < pos; ++k) mat_mul_acc(A, M[k], A);
                        for (int k = pos + 1; k < 4; ++k) mat_mul_acc(B, M[k], B);
                        mat_mul(B, Y, T);
                        mat_mul(T, A, R); /* B Y A */
                        cplx *w = W + ((long)ld[lf][pos] * V + ls[lf][pos]) * 9;
                        if (lg[lf][pos]) {
                            for (int i = 0; i < 3; ++i)
                                for (int j = 0; j < 3; ++j) w[i * 3 + j] += conj(R[j * 3 + i]);
                        } else {
                            for (int i = 0; i < 9; ++i) w[i] += R[i];
                        }
                    }
                }
            }
}

/* dL/dc_SW = -2 Re <chi| (C / c_SW) psi>, C the clover field (appendix); C / c_SW is
 * the clover block built with c_SW = 1, so the derivative is defined at c_SW = 0 too */
double orc_dcsw(const orc_params *p, const cplx *U, const cplx *psi, const cplx *chi)
{
    long V = volume(p);
    orc_params p1 = *p;
    p1.csw = 1.0;
    double s = 0;
    cplx C1[144];
    for (long n = 0; n < V; ++n) {
        cplx cx[12];
        clover_site(&p1, U, n, C1);
        mat12_vec(C1, psi + n * 12, cx);
        for (int i = 0; i < 12; ++i) s += creal(conj(chi[n * 12 + i]) * cx[i]);
    }
    return -2.0 * s;
}
