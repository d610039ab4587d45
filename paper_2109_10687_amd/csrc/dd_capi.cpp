// dd_capi.cpp -- the C ABI of include/ddsolve.h: context and field ownership,
// gauge loading, the Dirac and SAP entry points, and the solver loops:
//   plain FP64 BiCGStab on D (Alg. 5 without preconditioner),
//   FP32 BiCGStab on A M_SAP (Alg. 5 with Alg. 1 as right preconditioner),
//   FP64 defect correction (Alg. 4) around the FP32 solver with an FP16 SAP;
// the adjoint solve D^dagger x = b through D^dagger = gamma_5 D gamma_5, and the
// fermion force of L = |D^{-1} phi|^2 (dd_force.hip).
// Every step of the path runs in the kernels of dd_kernels.hip; this file
// only sequences launches and evaluates the BiCGStab scalars.
#include <hip/hip_runtime.h>

#include <array>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ddsolve.h"
#include "dd_launch.h"

using dd::Geom;
using cplx = std::complex<double>;

namespace {

constexpr int N64 = 7, N32 = 10, N16 = 5;
constexpr int RED_MAX = 64;  // longest reduction result (doubles): GCR cycle, or 3 per batched right-hand side
constexpr int BATCH_MAX = 16;  // right-hand sides of one batched solve

struct TimerRec {
    int cls;
    hipEvent_t a, b;
    double bytes, flops;
};

}  // namespace

struct dd_ctx {
    dd_params prm{};
    Geom g{};
    hipStream_t stream = nullptr;
    std::string err;
    bool gauge = false;
    int verbose = 0;  // DD_VERBOSE=1: one progress line per outer pass and per 100 inner iterations
    dd::Phase4 phase{};
    // packed gauge fields
    void *U64 = nullptr, *U32 = nullptr, *U16 = nullptr;
    void *clov64 = nullptr, *cinv32 = nullptr, *cinv16 = nullptr;
    void *yforce = nullptr;  // force work field (54 complex per site), allocated by the first dd_force
    // batched right-hand sides: contiguous arrays of per-RHS internal fields, allocated by the
    // first batched call and grown on demand (kinds: see BK_* below)
    int bcap = 0;
    std::vector<void *> bk;
    int mrhs_force = -1;                // multi-RHS kernel variant forced by the caller (-1: autotune)
    int mrhs_tuned[13] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};  // per right-hand sides in a tile
    double mrhs_ms[13][16] = {};         // autotuner timings (ms per launch) per variant
    // work vectors
    void *f64[N64] = {}, *f32[N32] = {}, *f16[N16] = {};
    void *gz[dd::GCR_MAX_NKV] = {}, *gp[dd::GCR_MAX_NKV] = {};  // GCR images (FP32), directions (FP16)
    double *partials = nullptr, *red = nullptr, *red_host = nullptr;
    int *flag = nullptr;
    // kernel timing
    bool timing = false;
    std::vector<TimerRec> recs;
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
    long long launches[DD_KT_COUNT] = {};
    double ms[DD_KT_COUNT] = {}, bytes[DD_KT_COUNT] = {}, flops[DD_KT_COUNT] = {};
};

namespace {

dd_status fail(dd_ctx *c, dd_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

#define HIPCK(c, call)                                                                                   \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess) return fail((c), DD_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

hipEvent_t take_event(dd_ctx *c)
{
    if (c->pool_used == c->pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->pool.push_back(e);
    }
    return c->pool[c->pool_used++];
}

// run `launch` and, when timing is on, bracket it with events on the stream;
// bytes and flops are the launch's algorithmic traffic and arithmetic
template <typename F> hipError_t timed(dd_ctx *c, int cls, double bytes, double flops, F &&launch)
{
    if (!c->timing) return launch();
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) return launch();
    (void)hipEventRecord(a, c->stream);
    hipError_t e = launch();
    (void)hipEventRecord(b, c->stream);
    c->recs.push_back({cls, a, b, bytes, flops});
    return e;
}

hipError_t flush_timing(dd_ctx *c)
{
    if (c->recs.empty()) return hipSuccess;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return e;
    for (auto &r : c->recs) {
        float t = 0;
        if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
            c->ms[r.cls] += t;
            c->launches[r.cls] += 1;
            c->bytes[r.cls] += r.bytes;
            c->flops[r.cls] += r.flops;
        }
    }
    c->recs.clear();
    c->pool_used = 0;
    return hipSuccess;
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int v)
{
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

size_t spinor_bytes(const Geom &g, int prec)
{
    if (prec == DD_F64) return (size_t)g.V * 12 * 16;
    if (prec == DD_F32) return (size_t)g.V * 12 * 8;
    return (size_t)g.V * (12 * 4 + 4);
}

// ---- algorithmic bytes and flops per site (each field read or written once)
double sp_b(int prec) { return prec == 0 ? 192.0 : prec == 1 ? 96.0 : 52.0; }   // spinor (+ FP16 scale)
double lk_b(int prec) { return prec == 0 ? 144.0 : prec == 1 ? 72.0 : 24.0; }    // one link (FP16: 12 reals)
double cl_b(int prec) { return prec == 0 ? 576.0 : prec == 1 ? 288.0 : 144.0; }  // clover / C_inv block pair
const double HOPF[4] = {168, 168, 168, 156};                                      // flops of one hop per direction
constexpr double CLOVF = 600;                                                      // clover multiply + combine
// fermion force, counted flops (complex multiply 6, add 2; a 3x3 product 198, C += A B 216):
// per link 6 plaquettes x 1854 + hop outer products 730; per site the Y planes 6 x 400
// and, for dL/dc_SW, the six field strengths and traces 6 x 2500
constexpr double FORCE_LINK_FLOPS = 6 * 1854.0 + 730.0;
constexpr double FORCE_Y_FLOPS = 6 * 400.0, FORCE_DCSW_FLOPS = 6 * 2500.0;

// hop flops per site that stay inside a block, and those that leave it
double hops_in(const Geom &g)
{
    double f = 0;
    for (int mu = 0; mu < 4; ++mu) f += 2.0 * (g.b[mu] - 1) / g.b[mu] * HOPF[mu];
    return f;
}
double hops_out(const Geom &g)
{
    double f = 0;
    for (int mu = 0; mu < 4; ++mu) f += 2.0 / g.b[mu] * HOPF[mu];
    return f;
}

// gamma matrices of the paper's appendix (Dirac representation, gamma_4 diagonal),
// used here only to form the sigma blocks of the clover setup
void gamma_table(cplx gm[4][4][4])
{
    const cplx I(0, 1);
    cplx g1[4][4] = {{0, 0, 0, I}, {0, 0, I, 0}, {0, -I, 0, 0}, {-I, 0, 0, 0}};
    cplx g2[4][4] = {{0, 0, 0, 1}, {0, 0, -1, 0}, {0, -1, 0, 0}, {1, 0, 0, 0}};
    cplx g3[4][4] = {{0, 0, I, 0}, {0, 0, 0, -I}, {-I, 0, 0, 0}, {0, I, 0, 0}};
    cplx g4[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, -1, 0}, {0, 0, 0, -1}};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            gm[0][i][j] = g1[i][j];
            gm[1][i][j] = g2[i][j];
            gm[2][i][j] = g3[i][j];
            gm[3][i][j] = g4[i][j];
        }
}

// sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] rotated by P = [[1,1],[1,-1]]/sqrt2
// (spin pairs) into the basis where gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 is
// diagonal; sigma commutes with gamma_5, so only the two 2x2 diagonal blocks survive
bool sigma_blocks(dd::SigmaBlocks &sb)
{
    cplx gm[4][4][4];
    gamma_table(gm);
    const double r = 1.0 / std::sqrt(2.0);
    double P[4][4] = {{r, 0, r, 0}, {0, r, 0, r}, {r, 0, -r, 0}, {0, r, 0, -r}};
    int plane = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu, ++plane) {
            cplx s[4][4], t[4][4], u[4][4];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    cplx c = 0;
                    for (int k = 0; k < 4; ++k) c += gm[mu][i][k] * gm[nu][k][j] - gm[nu][i][k] * gm[mu][k][j];
                    s[i][j] = cplx(0, 0.5) * c;
                }
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    cplx c = 0;
                    for (int k = 0; k < 4; ++k) c += P[i][k] * s[k][j];
                    t[i][j] = c;
                }
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    cplx c = 0;
                    for (int k = 0; k < 4; ++k) c += t[i][k] * P[k][j];
                    u[i][j] = c;
                }
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    if (std::abs(u[i][j + 2]) > 1e-12 || std::abs(u[i + 2][j]) > 1e-12) return false;
                    sb.re[plane][0][i][j] = u[i][j].real();
                    sb.im[plane][0][i][j] = u[i][j].imag();
                    sb.re[plane][1][i][j] = u[i + 2][j + 2].real();
                    sb.im[plane][1][i][j] = u[i + 2][j + 2].imag();
                }
        }
    return true;
}

// ------------------------------------------------------------------ launch helpers

dd_status k_dirac(dd_ctx *c, void *out, const void *in, int pin, int pout, int pg, int op)
{
    dd::DiracArgs a{};
    a.out = out;
    a.in = in;
    a.pin = pin;
    a.pout = pout;
    a.pg = pg;
    a.op = op;
    a.kappa = c->prm.kappa;
    a.phase = c->phase;
    if (pg == 0) {
        a.links = c->U64;
        a.clover = c->clov64;
    } else if (pg == 1) {
        a.links = c->U32;
        a.clover = c->cinv32;
    } else {
        a.links = c->U16;
        a.clover = c->cinv16;
    }
    int cls = pg == 0 ? DD_KT_DIRAC_F64 : pg == 2 ? DD_KT_DIRAC_F16 : pin == 2 ? DD_KT_DIRAC_F16IN : DD_KT_DIRAC_F32;
    const double V = (double)c->g.V;
    const double bytes = V * (sp_b(pin) + sp_b(pout) + 4 * lk_b(pg) + cl_b(pg));
    const double flops = V * (hops_in(c->g) + hops_out(c->g) + CLOVF);
    hipError_t e = timed(c, cls, bytes, flops, [&] { return dd::launch_dirac(c->g, c->stream, a); });
    if (e != hipSuccess) return fail(c, DD_ERR_HIP, std::string("dirac launch: ") + hipGetErrorString(e));
    return DD_OK;
}

// x = M_SAP b at storage precision prec (1 FP32, 2 FP16), work vector s
dd_status k_sap(dd_ctx *c, int prec, const void *b, void *x, void *s)
{
    dd::SapArgs a{};
    a.b = b;
    a.s = s;
    a.x = x;
    a.prec = prec;
    a.links = prec == 1 ? c->U32 : c->U16;
    a.cinv = prec == 1 ? c->cinv32 : c->cinv16;
    a.n_jac = c->prm.n_jac;
    a.kappa = c->prm.kappa;
    a.phase = c->phase;
    const int E = 0, O = 1;
    const int n = c->prm.n_sap;
    const Geom &g = c->g;
    auto half = [&](int colour, int flags) -> dd_status {
        // per site of the swept colour: source, links, C_inv, x written; without
        // TAIL also b read and s written; with PRE the neighbour-block face
        // spinors and the links that point into the block from outside
        const bool tail = flags & dd::SAP_TAIL, pre = flags & dd::SAP_PRE, first = flags & dd::SAP_FIRST;
        double face_sp = 0, face_lk = 0;
        for (int mu = 0; mu < 4; ++mu) {
            face_sp += 2.0 / g.b[mu];
            face_lk += 1.0 / g.b[mu];
        }
        double per = sp_b(prec) + 4 * lk_b(prec) + cl_b(prec) + sp_b(prec);
        if (!tail) per += (first ? 0.0 : sp_b(prec)) + sp_b(prec);
        if (pre) per += face_sp * sp_b(prec) + face_lk * lk_b(prec);
        double fl = c->prm.n_jac * (hops_in(g) + CLOVF);
        if (!tail) fl += hops_in(g) + CLOVF + 48;
        if (pre) fl += hops_out(g) + CLOVF;
        const double sites = 0.5 * (double)g.V;
        const bool pk = prec == 2 && c->prm.sap_fp16_arith;
        hipError_t e = timed(c, DD_KT_SAP, sites * per, sites * fl, [&] {
            return pk ? dd::launch_sap_half_pk(c->g, c->stream, a, colour, flags)
                      : dd::launch_sap_half(c->g, c->stream, a, colour, flags);
        });
        if (e != hipSuccess) return fail(c, DD_ERR_HIP, std::string("sap launch: ") + hipGetErrorString(e));
        return DD_OK;
    };
    dd_status st;
    for (int i = 0; i < n; ++i) {
        if ((st = half(E, i == 0 ? dd::SAP_FIRST : dd::SAP_PRE)) != DD_OK) return st;
        if ((st = half(O, i == 0 ? (dd::SAP_FIRST | dd::SAP_PRE) : dd::SAP_PRE)) != DD_OK) return st;
    }
    if ((st = half(E, dd::SAP_TAIL | (n == 0 ? dd::SAP_FIRST : dd::SAP_PRE))) != DD_OK) return st;
    if ((st = half(O, dd::SAP_TAIL | dd::SAP_PRE | (n == 0 ? dd::SAP_FIRST : 0))) != DD_OK) return st;
    return DD_OK;
}

dd_status blas(dd_ctx *c, dd::BlasArgs a)
{
    a.partials = c->partials;
    // vectors read + written per site, and flops per site
    double rw = 0, fl = 0;
    const double P0 = sp_b(a.p[0]), P1 = sp_b(a.p[1]), P2 = sp_b(a.p[2]);
    switch (a.kind) {
    case dd::BLAS_DOT: rw = P0 + P1; fl = 96; break;
    case dd::BLAS_DOT_NORM: rw = P0 + P1; fl = 144; break;
    case dd::BLAS_NORM2: rw = P0; fl = 48; break;
    case dd::BLAS_UPDATE1: rw = 2 * P0 + P1 + 3 * P2; fl = 240; break;
    case dd::BLAS_UPDATE2: rw = 2 * P0 + P1 + 4 * P2; fl = 336; break;
    case dd::BLAS_PUPDATE: rw = 4 * P0; fl = 192; break;
    case dd::BLAS_AXPBY: rw = P0 + (a.c[1] != 0.0 ? 2 : 1) * P1; fl = 72; break;
    case dd::BLAS_SUB_NORM: rw = 3 * P0; fl = 72; break;
    case dd::BLAS_CONVERT: rw = P0 + P1; break;
    case dd::BLAS_CINV_SRC: rw = sp_b(1) + P1 + cl_b(1); fl = CLOVF; break;
    }
    const double V = (double)c->g.V;
    hipError_t e = timed(c, DD_KT_BLAS, V * rw, V * fl, [&] { return dd::launch_blas(c->g, c->stream, a); });
    if (e != hipSuccess) return fail(c, DD_ERR_HIP, std::string("vector kernel: ") + hipGetErrorString(e));
    return DD_OK;
}

// run a reducing vector kernel and bring its nv sums to the host
dd_status reduce(dd_ctx *c, dd::BlasArgs a, int nv, double *out)
{
    dd_status st = blas(c, a);
    if (st != DD_OK) return st;
    HIPCK(c, dd::launch_finalize(c->stream, c->partials, dd::blas_grid(c->g), nv, c->red));
    HIPCK(c, hipMemcpyAsync(c->red_host, c->red, nv * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < nv; ++k) out[k] = c->red_host[k];
    return DD_OK;
}

dd::BlasArgs mkb(int kind, std::initializer_list<void *> v, std::initializer_list<int> p,
                 std::initializer_list<double> cc = {})
{
    dd::BlasArgs a{};
    a.kind = kind;
    int i = 0;
    for (void *x : v) a.v[i++] = x;
    i = 0;
    for (int x : p) a.p[i++] = x;
    i = 0;
    for (double x : cc) a.c[i++] = x;
    return a;
}

dd_status norm2(dd_ctx *c, void *v, int prec, double *out)
{
    return reduce(c, mkb(dd::BLAS_NORM2, {v}, {prec}), 1, out);
}

dd_status copy(dd_ctx *c, void *dst, int pd, void *src, int ps)
{
    if (ps == 2 || pd == 2) return blas(c, mkb(dd::BLAS_CONVERT, {src, dst}, {ps, pd}));
    return blas(c, mkb(dd::BLAS_AXPBY, {src, dst}, {ps, pd}, {1.0, 0.0}));
}

bool is_fin(double v) { return std::isfinite(v); }
bool is_fin(cplx v) { return std::isfinite(v.real()) && std::isfinite(v.imag()); }

// r = b - D x (FP64) ; returns |r|^2
dd_status residual64(dd_ctx *c, void *r, void *b, void *x, void *tmp, double *rn2)
{
    dd_status st = k_dirac(c, tmp, x, 0, 0, 0, 0);
    if (st != DD_OK) return st;
    return reduce(c, mkb(dd::BLAS_SUB_NORM, {r, b, tmp}, {0, 0, 0}), 1, rn2);
}

// ------------------------------------------------------------------ solvers

struct SolveOut {
    int iters = 0;
    double relres = 0;
    int detail = 0;
};

// plain BiCGStab (Alg. 5, M = I) on D in FP64; x holds the initial guess.
// At a recursive exit the true residual is recomputed; if it misses tol the
// iteration restarts from it.
dd_status solve_plain64(dd_ctx *c, void *x, void *b, double tol, int maxiter, SolveOut &o)
{
    void *r = c->f64[2], *rt = c->f64[3], *p = c->f64[4], *q = c->f64[5], *t = c->f64[6];
    double bn2;
    dd_status st = norm2(c, b, 0, &bn2);
    if (st != DD_OK) return st;
    if (!is_fin(bn2)) return fail(c, DD_ERR_NONFINITE, "source holds NaN or Inf");
    if (bn2 == 0.0) {
        HIPCK(c, hipMemsetAsync(x, 0, spinor_bytes(c->g, DD_F64), c->stream));
        o.relres = 0;
        return DD_OK;
    }
    int it = 0;
    for (int restart = 0; restart < 20; ++restart) {
        double rn2;
        if ((st = residual64(c, r, b, x, q, &rn2)) != DD_OK) return st;
        o.relres = std::sqrt(rn2 / bn2);
        if (o.relres < tol) {
            o.iters = it;
            return DD_OK;
        }
        if (it >= maxiter) break;
        if ((st = copy(c, rt, 0, r, 0)) != DD_OK) return st;
        if ((st = copy(c, p, 0, r, 0)) != DD_OK) return st;
        cplx rho0 = rn2;
        bool conv = false;
        while (it < maxiter) {
            ++it;
            if ((st = k_dirac(c, q, p, 0, 0, 0, 0)) != DD_OK) return st;
            double d[3];
            if ((st = reduce(c, mkb(dd::BLAS_DOT, {rt, q}, {0, 0}), 2, d)) != DD_OK) return st;
            cplx rq(d[0], d[1]);
            if (rq == 0.0 || !is_fin(rq)) {
                o.iters = it;
                o.detail = rq == 0.0 ? 1 : 4;
                return DD_BREAKDOWN;
            }
            cplx alpha = rho0 / rq;
            if ((st = reduce(c, mkb(dd::BLAS_UPDATE1, {x, p, r, q}, {0, 0, 0}, {alpha.real(), alpha.imag()}), 1,
                             &rn2)) != DD_OK)
                return st;
            if (std::sqrt(rn2 / bn2) < tol) {
                conv = true;
                break;
            }
            if (c->verbose && it % 500 == 0) {
                std::fprintf(stderr, "[ddsolve] FP64 iteration %d: relative residual %.3e\n", it, std::sqrt(rn2 / bn2));
                std::fflush(stderr);
            }
            if ((st = k_dirac(c, t, r, 0, 0, 0, 0)) != DD_OK) return st;
            if ((st = reduce(c, mkb(dd::BLAS_DOT_NORM, {t, r}, {0, 0}), 3, d)) != DD_OK) return st;
            if (d[2] == 0.0 || !is_fin(d[2])) {
                o.iters = it;
                o.detail = d[2] == 0.0 ? 2 : 4;
                return DD_BREAKDOWN;
            }
            cplx omega = cplx(d[0], d[1]) / d[2];
            if ((st = reduce(c, mkb(dd::BLAS_UPDATE2, {x, r, r, t, rt}, {0, 0, 0}, {omega.real(), omega.imag()}), 3,
                             d)) != DD_OK)
                return st;
            rn2 = d[0];
            cplx rho(d[1], d[2]);
            if (std::sqrt(rn2 / bn2) < tol) {
                conv = true;
                break;
            }
            if (omega == 0.0) {
                o.iters = it;
                o.detail = 3;
                return DD_BREAKDOWN;
            }
            cplx beta = (alpha / omega) * (rho / rho0);
            if (!is_fin(beta)) {
                o.iters = it;
                o.detail = 4;
                return DD_BREAKDOWN;
            }
            rho0 = rho;
            if ((st = blas(c, mkb(dd::BLAS_PUPDATE, {p, r, q}, {0, 0, 0},
                                  {beta.real(), beta.imag(), omega.real(), omega.imag()}))) != DD_OK)
                return st;
        }
        if (!conv) break;
    }
    o.iters = it;
    double rn2;
    if ((st = residual64(c, r, b, x, q, &rn2)) != DD_OK) return st;
    o.relres = std::sqrt(rn2 / bn2);
    return o.relres < tol ? DD_OK : DD_NOT_CONVERGED;
}

// FP32 BiCGStab on A M_SAP (Alg. 5 with Alg. 1 as right preconditioner) for the
// source src (FP32, internal); the solution accumulates the preconditioned
// directions, y += alpha M p + omega M r, which equals M_SAP applied to Alg. 5's
// iterate when M is linear and stays consistent with the recursive residual
// when M is computed in rounded FP16.  prec = SAP storage precision (1 or 2).
dd_status solve_sap32(dd_ctx *c, int prec, void *src, void *y, double tol, int maxiter, SolveOut &o)
{
    void *r = c->f32[2], *rt = c->f32[3], *p = c->f32[4], *q = c->f32[5], *t = c->f32[6];
    void *Mp = prec == 1 ? c->f32[7] : c->f16[2];
    void *Mr = prec == 1 ? c->f32[8] : c->f16[3];
    void *s = prec == 1 ? c->f32[9] : c->f16[4];
    void *p16 = c->f16[0], *r16 = c->f16[1];
    dd_status st;
    HIPCK(c, hipMemsetAsync(y, 0, spinor_bytes(c->g, DD_F32), c->stream));
    double bn2;
    if ((st = norm2(c, src, 1, &bn2)) != DD_OK) return st;
    if (!is_fin(bn2)) return fail(c, DD_ERR_NONFINITE, "inner source holds NaN or Inf");
    o.iters = 0;
    o.relres = 0;
    if (bn2 == 0.0) return DD_OK;
    if ((st = copy(c, r, 1, src, 1)) != DD_OK) return st;
    if ((st = copy(c, p, 1, src, 1)) != DD_OK) return st;
    if ((st = copy(c, rt, 1, src, 1)) != DD_OK) return st;
    cplx rho0 = bn2;
    double rn2 = bn2;
    auto precond = [&](void *in, void *in16, void *Mout, void *Aout) -> dd_status {
        dd_status s2;
        const void *bsrc = in;
        if (prec == 2) {
            if ((s2 = copy(c, in16, 2, in, 1)) != DD_OK) return s2;
            bsrc = in16;
        }
        if ((s2 = k_sap(c, prec, bsrc, Mout, s)) != DD_OK) return s2;
        return k_dirac(c, Aout, Mout, prec, 1, 1, 1);
    };
    for (int it = 0; it < maxiter; ++it) {
        o.iters = it + 1;
        if ((st = precond(p, p16, Mp, q)) != DD_OK) return st;
        double d[3];
        if ((st = reduce(c, mkb(dd::BLAS_DOT, {rt, q}, {1, 1}), 2, d)) != DD_OK) return st;
        cplx rq(d[0], d[1]);
        if (rq == 0.0 || !is_fin(rq)) {
            o.detail = rq == 0.0 ? 1 : 4;
            o.relres = std::sqrt(rn2 / bn2);
            return DD_BREAKDOWN;
        }
        cplx alpha = rho0 / rq;
        if ((st = reduce(c, mkb(dd::BLAS_UPDATE1, {y, Mp, r, q}, {1, prec, 1}, {alpha.real(), alpha.imag()}), 1,
                         &rn2)) != DD_OK)
            return st;
        o.relres = std::sqrt(rn2 / bn2);
        if (o.relres < tol) return DD_OK;
        if (c->verbose && (it + 1) % 100 == 0) {
            std::fprintf(stderr, "[ddsolve] inner iteration %d: relative residual %.3e\n", it + 1, o.relres);
            std::fflush(stderr);
        }
        if ((st = precond(r, r16, Mr, t)) != DD_OK) return st;
        if ((st = reduce(c, mkb(dd::BLAS_DOT_NORM, {t, r}, {1, 1}), 3, d)) != DD_OK) return st;
        if (d[2] == 0.0 || !is_fin(d[2])) {
            o.detail = d[2] == 0.0 ? 2 : 4;
            return DD_BREAKDOWN;
        }
        cplx omega = cplx(d[0], d[1]) / d[2];
        if ((st = reduce(c, mkb(dd::BLAS_UPDATE2, {y, Mr, r, t, rt}, {1, prec, 1}, {omega.real(), omega.imag()}), 3,
                         d)) != DD_OK)
            return st;
        rn2 = d[0];
        cplx rho(d[1], d[2]);
        o.relres = std::sqrt(rn2 / bn2);
        if (o.relres < tol) return DD_OK;
        if (omega == 0.0) {
            o.detail = 3;
            return DD_BREAKDOWN;
        }
        cplx beta = (alpha / omega) * (rho / rho0);
        if (!is_fin(beta)) {
            o.detail = 4;
            return DD_BREAKDOWN;
        }
        rho0 = rho;
        if ((st = blas(c, mkb(dd::BLAS_PUPDATE, {p, r, q}, {1, 1, 1},
                              {beta.real(), beta.imag(), omega.real(), omega.imag()}))) != DD_OK)
            return st;
    }
    return DD_NOT_CONVERGED;
}

// bring nv finalized sums of `partials` (nwg workgroups) to the host
dd_status fetch(dd_ctx *c, int nv, double *out)
{
    HIPCK(c, dd::launch_finalize(c->stream, c->partials, dd::blas_grid(c->g), nv, c->red));
    HIPCK(c, hipMemcpyAsync(c->red_host, c->red, nv * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < nv; ++k) out[k] = c->red_host[k];
    return DD_OK;
}

// Restarted flexible GCR on A M (M = FP16 SAP) for the FP32 source src.  Each
// iteration: p_k = M r (FP16), z_k = A p_k (FP32), z_k orthonormalised against
// z_0..z_{k-1} (classical Gram-Schmidt, FP64 sums), r -= <z_k|r> z_k.  At the end
// of a cycle y += sum_k alpha_k p_k with alpha from the triangular relation
// A p_k = b_k z_k + sum_{j<k} a_jk z_j.  The directions are stored, so M may
// differ from one application to the next.
dd_status solve_gcr32(dd_ctx *c, void *src, void *y, double tol, int maxiter, SolveOut &o)
{
    const Geom &g = c->g;
    const int nkv = c->prm.gcr_nkv;
    void *r = c->f32[2], *r16 = c->f16[1], *s = c->f16[4];
    const double V = (double)g.V;
    dd_status st;
    HIPCK(c, hipMemsetAsync(y, 0, spinor_bytes(g, DD_F32), c->stream));
    double bn2;
    if ((st = norm2(c, src, 1, &bn2)) != DD_OK) return st;
    if (!is_fin(bn2)) return fail(c, DD_ERR_NONFINITE, "inner source holds NaN or Inf");
    o.iters = 0;
    o.relres = 0;
    if (bn2 == 0.0) return DD_OK;
    if ((st = copy(c, r, 1, src, 1)) != DD_OK) return st;
    double rn2 = bn2;
    std::vector<cplx> a((size_t)nkv * nkv), cc(nkv), alpha(nkv);
    std::vector<double> bk(nkv);
    bool done = false;
    while (!done) {
        int n = 0;
        for (int k = 0; k < nkv; ++k) {
            // p_k = M r,  z_k = A p_k
            if ((st = copy(c, r16, 2, r, 1)) != DD_OK) return st;
            if ((st = k_sap(c, 2, r16, c->gp[k], s)) != DD_OK) return st;
            if ((st = k_dirac(c, c->gz[k], c->gp[k], 2, 1, 1, 1)) != DD_OK) return st;
            dd::VecSet zs{};
            for (int j = 0; j < k; ++j) zs.v[j] = c->gz[j];
            double d[2 * dd::GCR_MAX_NKV];
            if (k > 0) {
                hipError_t e = timed(c, DD_KT_BLAS, V * 96.0 * (k + 1), V * 96.0 * k,
                                     [&] { return dd::launch_multidot(g, c->stream, zs, k, c->gz[k], c->partials); });
                if (e != hipSuccess) return fail(c, DD_ERR_HIP, std::string("multidot: ") + hipGetErrorString(e));
                if ((st = fetch(c, 2 * k, d)) != DD_OK) return st;
                for (int j = 0; j < k; ++j) {
                    a[(size_t)j * nkv + k] = cplx(d[2 * j], d[2 * j + 1]);
                    zs.re[j] = d[2 * j];
                    zs.im[j] = d[2 * j + 1];
                }
            }
            hipError_t e = timed(c, DD_KT_BLAS, V * 96.0 * (k + 3), V * 96.0 * (k + 1), [&] {
                return dd::launch_gcr_orth(g, c->stream, zs, k, c->gz[k], r, c->partials);
            });
            if (e != hipSuccess) return fail(c, DD_ERR_HIP, std::string("gcr orth: ") + hipGetErrorString(e));
            if ((st = fetch(c, 3, d)) != DD_OK) return st;
            if (!(d[0] > 0.0) || !is_fin(d[0])) {
                o.detail = d[0] == 0.0 ? 2 : 4;
                done = true;
                if (k == 0) return DD_BREAKDOWN;
                break;
            }
            bk[k] = std::sqrt(d[0]);
            cc[k] = cplx(d[1], d[2]) / bk[k];
            e = timed(c, DD_KT_BLAS, V * 96.0 * 4, V * 96.0, [&] {
                return dd::launch_gcr_rupdate(g, c->stream, c->gz[k], r, 1.0 / bk[k], cc[k].real(), cc[k].imag(),
                                              c->partials);
            });
            if (e != hipSuccess) return fail(c, DD_ERR_HIP, std::string("gcr update: ") + hipGetErrorString(e));
            if ((st = fetch(c, 1, &rn2)) != DD_OK) return st;
            n = k + 1;
            ++o.iters;
            o.relres = std::sqrt(rn2 / bn2);
            if (c->verbose && o.iters % 100 == 0) {
                std::fprintf(stderr, "[ddsolve] GCR iteration %d: relative residual %.3e\n", o.iters, o.relres);
                std::fflush(stderr);
            }
            if (o.relres < tol || o.iters >= maxiter) {
                done = true;
                break;
            }
        }
        if (n == 0) break;
        // back substitution: alpha_j = (c_j - sum_{k>j} a_jk alpha_k) / b_j
        for (int j = n - 1; j >= 0; --j) {
            cplx t = cc[j];
            for (int k = j + 1; k < n; ++k) t -= a[(size_t)j * nkv + k] * alpha[k];
            alpha[j] = t / bk[j];
        }
        dd::VecSet ps{};
        for (int j = 0; j < n; ++j) {
            ps.v[j] = c->gp[j];
            ps.re[j] = alpha[j].real();
            ps.im[j] = alpha[j].imag();
        }
        hipError_t e = timed(c, DD_KT_BLAS, V * (52.0 * n + 192.0), V * 96.0 * n,
                             [&] { return dd::launch_multi_axpy(g, c->stream, ps, n, 2, y); });
        if (e != hipSuccess) return fail(c, DD_ERR_HIP, std::string("gcr solution update: ") + hipGetErrorString(e));
    }
    return o.relres < tol ? DD_OK : (o.detail ? DD_BREAKDOWN : DD_NOT_CONVERGED);
}

}  // namespace

namespace {

// ------------------------------------------------------------------ batched right-hand sides

// kinds of per-RHS fields in the batch buffers (each kind: nrhs fields one after another)
enum { BK_B64, BK_X64, BK_R64, BK_T64, BK_SRC, BK_Y, BK_R, BK_RT, BK_P, BK_Q, BK_T, BK_MP, BK_MR, BK_IN, BK_OUT,
       BK_COUNT };

int bk_prec(int k) { return k <= BK_T64 ? DD_F64 : DD_F32; }

dd_status batch_alloc(dd_ctx *c, int n)
{
    if (n <= c->bcap) return DD_OK;
    for (void *p : c->bk)
        if (p) (void)hipFree(p);
    c->bk.assign(BK_COUNT, nullptr);
    c->bcap = 0;
    for (int k = 0; k < BK_COUNT; ++k)
        if (hipMalloc(&c->bk[k], (size_t)n * spinor_bytes(c->g, bk_prec(k))) != hipSuccess) {
            (void)hipGetLastError();
            for (void *&p : c->bk)
                if (p) {
                    (void)hipFree(p);
                    p = nullptr;
                }
            return fail(c, DD_ERR_NOMEM, "batch work fields");
        }
    c->bcap = n;
    return DD_OK;
}

// field r of kind k
void *bf(dd_ctx *c, int k, int r) { return (char *)c->bk[k] + (size_t)r * spinor_bytes(c->g, bk_prec(k)); }

// run a reducing vector kernel on right-hand side r and leave its nv sums at red[off..]
dd_status reduce_to(dd_ctx *c, dd::BlasArgs a, int nv, int off)
{
    dd_status st = blas(c, a);
    if (st != DD_OK) return st;
    HIPCK(c, dd::launch_finalize(c->stream, c->partials, dd::blas_grid(c->g), nv, c->red + off));
    return DD_OK;
}

dd_status fetch_red(dd_ctx *c, int n, double *out)
{
    HIPCK(c, hipMemcpyAsync(c->red_host, c->red, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < n; ++k) out[k] = c->red_host[k];
    return DD_OK;
}

// out = A in for n FP32 batched fields (internal layout, contiguous), tiles of up to 12 on the
// matrix cores; the variant is the caller's, or the autotuner's choice for this tile size
dd_status mrhs_launch(dd_ctx *c, int v, void *out, const void *in, int n)
{
    dd::MrhsArgs a{};
    a.in = (const float2 *)in;
    a.out = (float2 *)out;
    a.u = (const float2 *)c->U32;
    a.cinv = (const float2 *)c->cinv32;
    a.nrhs = n;
    a.kappa = c->prm.kappa;
    a.phase = c->phase;
    const double V = (double)c->g.V;
    const double bytes = V * (n * 2.0 * sp_b(DD_F32) + 4 * lk_b(DD_F32) + cl_b(DD_F32));
    const double flops = V * n * (hops_in(c->g) + hops_out(c->g) + CLOVF);
    hipError_t e = timed(c, DD_KT_DIRAC_MRHS, bytes, flops, [&] { return dd::launch_dirac_mrhs(c->g, c->stream, a, v); });
    if (e != hipSuccess) return fail(c, DD_ERR_HIP, std::string("multi-RHS dirac launch: ") + hipGetErrorString(e));
    return DD_OK;
}

// time every variant on this tile (two warm-up launches, three timed) and keep the fastest
dd_status mrhs_tune(dd_ctx *c, int n, void *out, const void *in)
{
    const int nv = dd::mrhs_variant_count();
    hipEvent_t e0, e1;
    HIPCK(c, hipEventCreate(&e0));
    HIPCK(c, hipEventCreate(&e1));
    const bool timing = c->timing;
    c->timing = false;
    int best = 0;
    for (int v = 0; v < nv; ++v) {
        dd_status st;
        for (int k = 0; k < 2; ++k)
            if ((st = mrhs_launch(c, v, out, in, n)) != DD_OK) return st;
        HIPCK(c, hipEventRecord(e0, c->stream));
        for (int k = 0; k < 3; ++k)
            if ((st = mrhs_launch(c, v, out, in, n)) != DD_OK) return st;
        HIPCK(c, hipEventRecord(e1, c->stream));
        HIPCK(c, hipEventSynchronize(e1));
        float ms = 0;
        HIPCK(c, hipEventElapsedTime(&ms, e0, e1));
        c->mrhs_ms[n][v] = ms / 3.0;
        if (c->mrhs_ms[n][v] < c->mrhs_ms[n][best]) best = v;
    }
    c->timing = timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->mrhs_tuned[n] = best;
    return DD_OK;
}

dd_status k_dirac_mrhs(dd_ctx *c, void *out, const void *in, int n)
{
    const size_t fb = spinor_bytes(c->g, DD_F32);
    for (int r0 = 0; r0 < n; r0 += 12) {
        const int m = n - r0 < 12 ? n - r0 : 12;
        void *o = (char *)out + r0 * fb;
        const void *i = (const char *)in + r0 * fb;
        int v = c->mrhs_force;
        if (v < 0) {
            if (c->mrhs_tuned[m] < 0) {
                dd_status st = mrhs_tune(c, m, o, i);
                if (st != DD_OK) return st;
            }
            v = c->mrhs_tuned[m];
        }
        dd_status st = mrhs_launch(c, v, o, i, m);
        if (st != DD_OK) return st;
    }
    return DD_OK;
}

struct BRhs {
    bool active = false;
    cplx rho0 = 0.0;
    double bn2 = 0, rn2 = 0, tol = 0;
    SolveOut o;
    dd_status st = DD_OK;
};

// FP32 BiCGStab for n right-hand sides in lockstep (Alg. 5 per right-hand side, each with
// its own scalars and exit), on A M with M = the FP16-storage SAP of each right-hand side
// (sap) or M = I; every A application is one batched launch over all n.  Sources: BK_SRC, solutions:
// BK_Y (flexible accumulation as in the single right-hand-side solver).
dd_status solve_batch32(dd_ctx *c, int n, bool sap, std::vector<BRhs> &R, int maxiter)
{
    const size_t f32 = spinor_bytes(c->g, DD_F32);
    dd_status st;
    HIPCK(c, hipMemsetAsync(c->bk[BK_Y], 0, n * f32, c->stream));
    for (int r = 0; r < n; ++r)
        if ((st = reduce_to(c, mkb(dd::BLAS_NORM2, {bf(c, BK_SRC, r)}, {1}), 1, r)) != DD_OK) return st;
    double red[3 * BATCH_MAX];
    if ((st = fetch_red(c, n, red)) != DD_OK) return st;
    int nact = 0;
    for (int r = 0; r < n; ++r) {
        BRhs &b = R[r];
        b.o = SolveOut{};
        b.bn2 = b.rn2 = red[r];
        b.rho0 = red[r];
        b.st = DD_OK;
        if (!is_fin(red[r])) return fail(c, DD_ERR_NONFINITE, "inner source holds NaN or Inf");
        b.active = red[r] > 0.0;
        nact += b.active;
        if (!b.active) continue;
        for (int k : {BK_R, BK_P, BK_RT})
            if ((st = copy(c, bf(c, k, r), 1, bf(c, BK_SRC, r), 1)) != DD_OK) return st;
    }
    const int mp = sap ? BK_MP : BK_P, mr = sap ? BK_MR : BK_R;
    // M = the FP16-storage SAP of each right-hand side (as in the single right-hand-side
    // mixed solver), its output widened to FP32 for the batched A
    auto precond = [&](int from, int to) -> dd_status {
        if (!sap) return DD_OK;
        void *in16 = c->f16[0], *out16 = c->f16[2], *s16 = c->f16[4];
        for (int r = 0; r < n; ++r) {
            if (!R[r].active) continue;
            dd_status s2;
            if ((s2 = copy(c, in16, 2, bf(c, from, r), 1)) != DD_OK) return s2;
            if ((s2 = k_sap(c, 2, in16, out16, s16)) != DD_OK) return s2;
            if ((s2 = copy(c, bf(c, to, r), 1, out16, 2)) != DD_OK) return s2;
        }
        return DD_OK;
    };
    auto stop = [&](BRhs &b, dd_status s2, int detail) {
        b.active = false;
        b.st = s2;
        b.o.detail = detail;
        --nact;
    };
    for (int it = 0; it < maxiter && nact > 0; ++it) {
        if ((st = precond(BK_P, BK_MP)) != DD_OK) return st;
        if ((st = k_dirac_mrhs(c, c->bk[BK_Q], c->bk[mp], n)) != DD_OK) return st;
        for (int r = 0; r < n; ++r)
            if (R[r].active &&
                (st = reduce_to(c, mkb(dd::BLAS_DOT, {bf(c, BK_RT, r), bf(c, BK_Q, r)}, {1, 1}), 2, 2 * r)) != DD_OK)
                return st;
        if ((st = fetch_red(c, 2 * n, red)) != DD_OK) return st;
        std::vector<cplx> alpha(n);
        for (int r = 0; r < n; ++r) {
            BRhs &b = R[r];
            if (!b.active) continue;
            b.o.iters = it + 1;
            cplx rq(red[2 * r], red[2 * r + 1]);
            if (rq == 0.0 || !is_fin(rq)) {
                stop(b, DD_BREAKDOWN, rq == 0.0 ? 1 : 4);
                continue;
            }
            alpha[r] = b.rho0 / rq;
            if ((st = reduce_to(c, mkb(dd::BLAS_UPDATE1, {bf(c, BK_Y, r), bf(c, mp, r), bf(c, BK_R, r), bf(c, BK_Q, r)},
                                       {1, 1, 1}, {alpha[r].real(), alpha[r].imag()}),
                                1, r)) != DD_OK)
                return st;
        }
        if ((st = fetch_red(c, n, red)) != DD_OK) return st;
        for (int r = 0; r < n; ++r) {
            BRhs &b = R[r];
            if (!b.active) continue;
            b.rn2 = red[r];
            b.o.relres = std::sqrt(b.rn2 / b.bn2);
            if (b.o.relres < b.tol) stop(b, DD_OK, 0);
        }
        if (nact == 0) break;
        if ((st = precond(BK_R, BK_MR)) != DD_OK) return st;
        if ((st = k_dirac_mrhs(c, c->bk[BK_T], c->bk[mr], n)) != DD_OK) return st;
        for (int r = 0; r < n; ++r)
            if (R[r].active &&
                (st = reduce_to(c, mkb(dd::BLAS_DOT_NORM, {bf(c, BK_T, r), bf(c, BK_R, r)}, {1, 1}), 3, 3 * r)) != DD_OK)
                return st;
        if ((st = fetch_red(c, 3 * n, red)) != DD_OK) return st;
        std::vector<cplx> omega(n);
        for (int r = 0; r < n; ++r) {
            BRhs &b = R[r];
            if (!b.active) continue;
            const double *d = red + 3 * r;
            if (d[2] == 0.0 || !is_fin(d[2])) {
                stop(b, DD_BREAKDOWN, d[2] == 0.0 ? 2 : 4);
                continue;
            }
            omega[r] = cplx(d[0], d[1]) / d[2];
            if ((st = reduce_to(c, mkb(dd::BLAS_UPDATE2,
                                       {bf(c, BK_Y, r), bf(c, mr, r), bf(c, BK_R, r), bf(c, BK_T, r), bf(c, BK_RT, r)},
                                       {1, 1, 1}, {omega[r].real(), omega[r].imag()}),
                                3, 3 * r)) != DD_OK)
                return st;
        }
        if ((st = fetch_red(c, 3 * n, red)) != DD_OK) return st;
        for (int r = 0; r < n; ++r) {
            BRhs &b = R[r];
            if (!b.active) continue;
            const double *d = red + 3 * r;
            b.rn2 = d[0];
            cplx rho(d[1], d[2]);
            b.o.relres = std::sqrt(b.rn2 / b.bn2);
            if (b.o.relres < b.tol) {
                stop(b, DD_OK, 0);
                continue;
            }
            if (omega[r] == 0.0) {
                stop(b, DD_BREAKDOWN, 3);
                continue;
            }
            cplx beta = (alpha[r] / omega[r]) * (rho / b.rho0);
            if (!is_fin(beta)) {
                stop(b, DD_BREAKDOWN, 4);
                continue;
            }
            b.rho0 = rho;
            if ((st = blas(c, mkb(dd::BLAS_PUPDATE, {bf(c, BK_P, r), bf(c, BK_R, r), bf(c, BK_Q, r)}, {1, 1, 1},
                                  {beta.real(), beta.imag(), omega[r].real(), omega[r].imag()}))) != DD_OK)
                return st;
        }
        if (c->verbose && (it + 1) % 100 == 0) {
            std::fprintf(stderr, "[ddsolve] batched inner iteration %d: %d right-hand sides still running\n", it + 1, nact);
            std::fflush(stderr);
        }
    }
    for (int r = 0; r < n; ++r)
        if (R[r].active) {
            R[r].active = false;
            R[r].st = DD_NOT_CONVERGED;
        }
    return DD_OK;
}

// r = b - D x for every right-hand side (FP64), |r|^2 into rn2
dd_status residual64_batch(dd_ctx *c, int n, double *rn2)
{
    dd_status st;
    for (int r = 0; r < n; ++r) {
        if ((st = k_dirac(c, bf(c, BK_T64, r), bf(c, BK_X64, r), 0, 0, 0, 0)) != DD_OK) return st;
        if ((st = reduce_to(c, mkb(dd::BLAS_SUB_NORM, {bf(c, BK_R64, r), bf(c, BK_B64, r), bf(c, BK_T64, r)}, {0, 0, 0}), 1,
                            r)) != DD_OK)
            return st;
    }
    return fetch_red(c, n, rn2);
}

}  // namespace

// ====================================================================== several lattices

struct dd_multi {
    std::vector<dd_ctx *> L;
    hipStream_t stream = nullptr;
    std::string err;
    int *counter = nullptr;                      // work-queue head of the multi-lattice launch
    dd::LatDesc *desc_dev = nullptr;             // three descriptor tables: the caller's apply, A Mp, A Mr
    dd::LatDesc *desc_host = nullptr;            // pinned staging for the caller's apply
    int total = 0;                               // work items (256-site chunks) over all lattices
};

namespace {

dd_status mfail(dd_multi *m, dd_status s, const std::string &msg)
{
    if (m) m->err = msg;
    return s;
}

#define MHIPCK(m, call)                                                                                   \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess) return mfail((m), DD_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// a lattice's own failure, reported on the multi-lattice handle
dd_status lat_fail(dd_multi *m, int k, dd_status s)
{
    if (s < 0) m->err = "lattice " + std::to_string(k) + ": " + m->L[k]->err;
    return s;
}

void fill_desc(dd_multi *m, dd::LatDesc *d, const std::vector<const void *> &in, const std::vector<void *> &out)
{
    int item = 0;
    for (size_t k = 0; k < m->L.size(); ++k) {
        dd_ctx *c = m->L[k];
        d[k].g = c->g;
        d[k].in = in[k];
        d[k].out = out[k];
        d[k].u = c->U32;
        d[k].cinv = c->cinv32;
        d[k].phase = c->phase;
        d[k].kappa = c->prm.kappa;
        d[k].item0 = item;
        item += (int)((c->g.V + 255) / 256);
    }
}

// one launch of A over every lattice with descriptor table t (0 caller, 1 A Mp, 2 A Mr)
dd_status multi_launch(dd_multi *m, int t, int pin)
{
    const int n = (int)m->L.size();
    double bytes = 0, flops = 0;
    for (dd_ctx *c : m->L) {
        const double V = (double)c->g.V;
        bytes += V * (sp_b(pin) + sp_b(DD_F32) + 4 * lk_b(DD_F32) + cl_b(DD_F32));
        flops += V * (hops_in(c->g) + hops_out(c->g) + CLOVF);
    }
    dd_ctx *c0 = m->L[0];  // the timers of the first lattice's context hold the multi-lattice launches
    hipError_t e = timed(c0, DD_KT_DIRAC_MULTI, bytes, flops, [&] {
        return dd::launch_dirac_multi(m->stream, m->desc_dev + t * n, n, m->total, pin, m->counter);
    });
    if (e != hipSuccess) return mfail(m, DD_ERR_HIP, std::string("multi-lattice dirac launch: ") + hipGetErrorString(e));
    return DD_OK;
}

// bring the first nv reduction results of every lattice's context to the host (one sync)
dd_status multi_fetch(dd_multi *m, int nv, std::vector<std::array<double, 3>> &out)
{
    for (dd_ctx *c : m->L)
        MHIPCK(m, hipMemcpyAsync(c->red_host, c->red, nv * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    MHIPCK(m, hipStreamSynchronize(m->stream));
    for (size_t k = 0; k < m->L.size(); ++k)
        for (int v = 0; v < nv; ++v) out[k][v] = m->L[k]->red_host[v];
    return DD_OK;
}

// the inner FP32 BiCGStab of every lattice in lockstep (Alg. 5 on A M_SAP with the FP16
// SAP of each lattice, as in the single-lattice mixed solver, flexible accumulation):
// per lattice its own fields and scalars, the A applications of a step as one launch
dd_status solve_multi32(dd_multi *m, std::vector<BRhs> &R, int maxiter)
{
    const int n = (int)m->L.size();
    dd_status st;
    std::vector<std::array<double, 3>> red(n);
    // fields per lattice (as in solve_sap32 with FP16 SAP storage)
    auto F = [&](int k, int which) -> void * {
        dd_ctx *c = m->L[k];
        switch (which) {
        case 0: return c->f32[0];  // src
        case 1: return c->f32[1];  // y
        case 2: return c->f32[2];  // r
        case 3: return c->f32[3];  // rt
        case 4: return c->f32[4];  // p
        case 5: return c->f32[5];  // q
        case 6: return c->f32[6];  // t
        case 7: return c->f16[2];  // M p
        case 8: return c->f16[3];  // M r
        case 9: return c->f16[4];  // SAP work
        case 10: return c->f16[0]; // p in FP16
        default: return c->f16[1]; // r in FP16
        }
    };
    int nact = 0;
    for (int k = 0; k < n; ++k) {
        dd_ctx *c = m->L[k];
        MHIPCK(m, hipMemsetAsync(F(k, 1), 0, spinor_bytes(c->g, DD_F32), m->stream));
        if ((st = reduce_to(c, mkb(dd::BLAS_NORM2, {F(k, 0)}, {1}), 1, 0)) != DD_OK) return lat_fail(m, k, st);
    }
    if ((st = multi_fetch(m, 1, red)) != DD_OK) return st;
    for (int k = 0; k < n; ++k) {
        BRhs &b = R[k];
        b.o = SolveOut{};
        b.bn2 = b.rn2 = red[k][0];
        b.rho0 = red[k][0];
        b.st = DD_OK;
        if (!is_fin(red[k][0])) return mfail(m, DD_ERR_NONFINITE, "inner source holds NaN or Inf");
        b.active = red[k][0] > 0.0;
        nact += b.active;
        if (!b.active) continue;
        dd_ctx *c = m->L[k];
        for (int w : {2, 4, 3})
            if ((st = copy(c, F(k, w), 1, F(k, 0), 1)) != DD_OK) return lat_fail(m, k, st);
    }
    auto precond = [&](int from, int from16, int to) -> dd_status {
        for (int k = 0; k < n; ++k) {
            if (!R[k].active) continue;
            dd_ctx *c = m->L[k];
            dd_status s2;
            if ((s2 = copy(c, F(k, from16), 2, F(k, from), 1)) != DD_OK) return lat_fail(m, k, s2);
            if ((s2 = k_sap(c, 2, F(k, from16), F(k, to), F(k, 9))) != DD_OK) return lat_fail(m, k, s2);
        }
        return DD_OK;
    };
    auto stop = [&](BRhs &b, dd_status s2, int detail) {
        b.active = false;
        b.st = s2;
        b.o.detail = detail;
        --nact;
    };
    std::vector<cplx> alpha(n), omega(n);
    for (int it = 0; it < maxiter && nact > 0; ++it) {
        if ((st = precond(4, 10, 7)) != DD_OK) return st;
        if ((st = multi_launch(m, 1, 2)) != DD_OK) return st;  // q = A M p, every lattice
        for (int k = 0; k < n; ++k)
            if (R[k].active && (st = reduce_to(m->L[k], mkb(dd::BLAS_DOT, {F(k, 3), F(k, 5)}, {1, 1}), 2, 0)) != DD_OK)
                return lat_fail(m, k, st);
        if ((st = multi_fetch(m, 2, red)) != DD_OK) return st;
        for (int k = 0; k < n; ++k) {
            BRhs &b = R[k];
            if (!b.active) continue;
            b.o.iters = it + 1;
            cplx rq(red[k][0], red[k][1]);
            if (rq == 0.0 || !is_fin(rq)) {
                stop(b, DD_BREAKDOWN, rq == 0.0 ? 1 : 4);
                continue;
            }
            alpha[k] = b.rho0 / rq;
            if ((st = reduce_to(m->L[k], mkb(dd::BLAS_UPDATE1, {F(k, 1), F(k, 7), F(k, 2), F(k, 5)}, {1, 2, 1},
                                             {alpha[k].real(), alpha[k].imag()}),
                                1, 0)) != DD_OK)
                return lat_fail(m, k, st);
        }
        if ((st = multi_fetch(m, 1, red)) != DD_OK) return st;
        for (int k = 0; k < n; ++k) {
            BRhs &b = R[k];
            if (!b.active) continue;
            b.rn2 = red[k][0];
            b.o.relres = std::sqrt(b.rn2 / b.bn2);
            if (b.o.relres < b.tol) stop(b, DD_OK, 0);
        }
        if (nact == 0) break;
        if ((st = precond(2, 11, 8)) != DD_OK) return st;
        if ((st = multi_launch(m, 2, 2)) != DD_OK) return st;  // t = A M r, every lattice
        for (int k = 0; k < n; ++k)
            if (R[k].active &&
                (st = reduce_to(m->L[k], mkb(dd::BLAS_DOT_NORM, {F(k, 6), F(k, 2)}, {1, 1}), 3, 0)) != DD_OK)
                return lat_fail(m, k, st);
        if ((st = multi_fetch(m, 3, red)) != DD_OK) return st;
        for (int k = 0; k < n; ++k) {
            BRhs &b = R[k];
            if (!b.active) continue;
            const double *d = red[k].data();
            if (d[2] == 0.0 || !is_fin(d[2])) {
                stop(b, DD_BREAKDOWN, d[2] == 0.0 ? 2 : 4);
                continue;
            }
            omega[k] = cplx(d[0], d[1]) / d[2];
            if ((st = reduce_to(m->L[k], mkb(dd::BLAS_UPDATE2, {F(k, 1), F(k, 8), F(k, 2), F(k, 6), F(k, 3)}, {1, 2, 1},
                                             {omega[k].real(), omega[k].imag()}),
                                3, 0)) != DD_OK)
                return lat_fail(m, k, st);
        }
        if ((st = multi_fetch(m, 3, red)) != DD_OK) return st;
        for (int k = 0; k < n; ++k) {
            BRhs &b = R[k];
            if (!b.active) continue;
            const double *d = red[k].data();
            b.rn2 = d[0];
            cplx rho(d[1], d[2]);
            b.o.relres = std::sqrt(b.rn2 / b.bn2);
            if (b.o.relres < b.tol) {
                stop(b, DD_OK, 0);
                continue;
            }
            if (omega[k] == 0.0) {
                stop(b, DD_BREAKDOWN, 3);
                continue;
            }
            cplx beta = (alpha[k] / omega[k]) * (rho / b.rho0);
            if (!is_fin(beta)) {
                stop(b, DD_BREAKDOWN, 4);
                continue;
            }
            b.rho0 = rho;
            if ((st = blas(m->L[k], mkb(dd::BLAS_PUPDATE, {F(k, 4), F(k, 2), F(k, 5)}, {1, 1, 1},
                                        {beta.real(), beta.imag(), omega[k].real(), omega[k].imag()}))) != DD_OK)
                return lat_fail(m, k, st);
        }
    }
    for (int k = 0; k < n; ++k)
        if (R[k].active) {
            R[k].active = false;
            R[k].st = DD_NOT_CONVERGED;
        }
    return DD_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

dd_status dd_create(const dd_params *prm, void *hip_stream, dd_ctx **out)
{
    if (!prm || !out) return DD_ERR_ARG;
    *out = nullptr;
    dd_ctx *c = new (std::nothrow) dd_ctx;
    if (!c) return DD_ERR_NOMEM;
    c->prm = *prm;
    if (c->prm.inner_tol <= 0) c->prm.inner_tol = 1e-6;
    if (c->prm.inner_maxiter <= 0) c->prm.inner_maxiter = 2000;
    if (c->prm.gcr_nkv <= 0) c->prm.gcr_nkv = dd::GCR_MAX_NKV;
    if (c->prm.gcr_nkv > dd::GCR_MAX_NKV) {
        delete c;
        return DD_ERR_ARG;
    }
    Geom &g = c->g;
    long long V = 1;
    int bvol = 1, nblk = 1;
    for (int mu = 0; mu < 4; ++mu) {
        int L = prm->dims[mu], b = prm->block[mu];
        if (L <= 0 || !pow2(b) || b < 2 || b > 16 || L % (2 * b) != 0) {
            delete c;
            return DD_ERR_GEOMETRY;
        }
        g.L[mu] = L;
        g.b[mu] = b;
        g.NB[mu] = L / b;
        V *= L;
        bvol *= b;
        nblk *= L / b;
    }
    if (bvol > dd::MAX_BLOCK_VOLUME || prm->n_sap < 0 || prm->n_jac < 1 || !(prm->kappa >= 0) || !std::isfinite(prm->csw)) {
        delete c;
        return bvol > dd::MAX_BLOCK_VOLUME ? DD_ERR_GEOMETRY : DD_ERR_ARG;
    }
    g.bvol = bvol;
    g.lbvol = ilog2(bvol);
    g.nblk = nblk;
    g.V = V;
    g.sh[0] = 0;
    for (int mu = 1; mu < 4; ++mu) g.sh[mu] = g.sh[mu - 1] + ilog2(g.b[mu - 1]);
    g.bstride[0] = 1;
    for (int mu = 1; mu < 4; ++mu) g.bstride[mu] = g.bstride[mu - 1] * g.NB[mu - 1];
    for (int mu = 0; mu < 4; ++mu) {
        c->phase.re[mu] = prm->phase_re[mu];
        c->phase.im[mu] = prm->phase_im[mu];
    }
    c->stream = (hipStream_t)hip_stream;
    if (const char *v = std::getenv("DD_VERBOSE")) c->verbose = std::atoi(v);

    auto alloc = [&](void **p, size_t bytes) -> bool { return hipMalloc(p, bytes) == hipSuccess; };
    bool ok = alloc(&c->U64, (size_t)V * 36 * 16) && alloc(&c->U32, (size_t)V * 36 * 8) &&
              alloc(&c->U16, (size_t)V * 24 * 4) && alloc(&c->clov64, (size_t)V * 36 * 16) &&
              alloc(&c->cinv32, (size_t)V * 36 * 8) && alloc(&c->cinv16, (size_t)V * 36 * 4);
    for (int i = 0; ok && i < N64; ++i) ok = alloc(&c->f64[i], spinor_bytes(g, DD_F64));
    for (int i = 0; ok && i < N32; ++i) ok = alloc(&c->f32[i], spinor_bytes(g, DD_F32));
    for (int i = 0; ok && i < N16; ++i) ok = alloc(&c->f16[i], spinor_bytes(g, DD_F16));
    for (int i = 0; ok && i < c->prm.gcr_nkv; ++i)
        ok = alloc(&c->gz[i], spinor_bytes(g, DD_F32)) && alloc(&c->gp[i], spinor_bytes(g, DD_F16));
    ok = ok && alloc((void **)&c->partials, dd::MAX_PARTIALS * sizeof(double)) &&
         alloc((void **)&c->red, RED_MAX * sizeof(double)) && alloc((void **)&c->flag, 4 * sizeof(int)) &&
         hipHostMalloc((void **)&c->red_host, RED_MAX * sizeof(double), hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        dd_destroy(c);
        return DD_ERR_NOMEM;
    }
    *out = c;
    return DD_OK;
}

dd_status dd_destroy(dd_ctx *c)
{
    if (!c) return DD_OK;
    (void)hipStreamSynchronize(c->stream);
    void *bufs[] = {c->U64, c->U32, c->U16, c->clov64, c->cinv32, c->cinv16, c->yforce, c->partials, c->red, c->flag};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
    for (void *p : c->f64)
        if (p) (void)hipFree(p);
    for (void *p : c->f32)
        if (p) (void)hipFree(p);
    for (void *p : c->f16)
        if (p) (void)hipFree(p);
    for (void *p : c->gz)
        if (p) (void)hipFree(p);
    for (void *p : c->gp)
        if (p) (void)hipFree(p);
    for (void *p : c->bk)
        if (p) (void)hipFree(p);
    if (c->red_host) (void)hipHostFree(c->red_host);
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    delete c;
    return DD_OK;
}

const char *dd_last_error(const dd_ctx *c) { return c ? c->err.c_str() : "null context"; }

dd_status dd_load_gauge(dd_ctx *c, const void *U)
{
    if (!c || !U) return fail(c, DD_ERR_ARG, "null argument");
    HIPCK(c, hipMemsetAsync(c->flag, 0, 4 * sizeof(int), c->stream));
    HIPCK(c, dd::launch_pack_links(c->g, c->stream, U, c->U64, c->U32, c->U16, c->flag));
    dd::SigmaBlocks sb{};
    if (!sigma_blocks(sb)) return fail(c, DD_ERR_ARG, "sigma blocks not block diagonal");
    HIPCK(c, dd::launch_clover(c->g, c->stream, c->U64, sb, c->prm.kappa * c->prm.csw, c->clov64, c->cinv32,
                               c->cinv16, c->flag + 1));
    int fl[2] = {0, 0};
    HIPCK(c, hipMemcpyAsync(fl, c->flag, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    c->gauge = false;
    if (fl[0]) return fail(c, DD_ERR_NONFINITE, "gauge field holds NaN or Inf");
    if (fl[1]) return fail(c, DD_ERR_CLOVER_NOT_PD, "1 + C is not positive definite at some site");
    c->gauge = true;
    return DD_OK;
}

long long dd_field_bytes(const dd_ctx *c, dd_prec prec)
{
    if (!c || prec < DD_F64 || prec > DD_F16) return -1;
    return (long long)spinor_bytes(c->g, prec);
}

dd_status dd_pack_spinor(dd_ctx *c, void *dst, const void *src, dd_prec prec)
{
    if (!c || !dst || !src || prec < DD_F64 || prec > DD_F16) return fail(c, DD_ERR_ARG, "bad argument");
    HIPCK(c, dd::launch_pack_spinor(c->g, c->stream, prec, dst, src));
    return DD_OK;
}

dd_status dd_unpack_spinor(dd_ctx *c, void *dst, const void *src, dd_prec prec)
{
    if (!c || !dst || !src || prec < DD_F64 || prec > DD_F16) return fail(c, DD_ERR_ARG, "bad argument");
    HIPCK(c, dd::launch_unpack_spinor(c->g, c->stream, prec, dst, src));
    return DD_OK;
}

static dd_status check_op(dd_ctx *c, dd_prec prec, dd_op op)
{
    if (!c->gauge) return fail(c, DD_ERR_STATE, "no gauge field loaded");
    if (op == DD_OP_A && (prec == DD_F32 || prec == DD_F16)) return DD_OK;
    if ((op == DD_OP_D || op == DD_OP_DDAG) && prec == DD_F64) return DD_OK;
    return fail(c, DD_ERR_ARG, "operator not available at this precision (D, D^dagger: FP64; A: FP32, FP16)");
}

dd_status dirac_apply_packed(dd_ctx *c, void *out, const void *in, dd_prec prec, dd_op op)
{
    if (!c || !out || !in) return fail(c, DD_ERR_ARG, "null argument");
    dd_status st = check_op(c, prec, op);
    if (st != DD_OK) return st;
    return k_dirac(c, out, in, prec, prec, prec, op);
}

dd_status dirac_apply(dd_ctx *c, void *out, const void *in, dd_prec prec, dd_op op)
{
    if (!c || !out || !in) return fail(c, DD_ERR_ARG, "null argument");
    dd_status st = check_op(c, prec, op);
    if (st != DD_OK) return st;
    void *ti = c->f64[5], *to = c->f64[6];
    HIPCK(c, dd::launch_pack_spinor(c->g, c->stream, prec, ti, in));
    if ((st = k_dirac(c, to, ti, prec, prec, prec, op)) != DD_OK) return st;
    HIPCK(c, dd::launch_unpack_spinor(c->g, c->stream, prec, out, to));
    return DD_OK;
}

dd_status sap_precondition(dd_ctx *c, void *x, const void *b, dd_prec prec)
{
    if (!c || !x || !b) return fail(c, DD_ERR_ARG, "null argument");
    if (!c->gauge) return fail(c, DD_ERR_STATE, "no gauge field loaded");
    if (prec != DD_F32 && prec != DD_F16) return fail(c, DD_ERR_ARG, "SAP is available at FP32 and FP16");
    void *tb = c->f64[5], *tx = c->f64[6], *ts = c->f64[4];
    HIPCK(c, dd::launch_pack_spinor(c->g, c->stream, prec, tb, b));
    dd_status st = k_sap(c, prec, tb, tx, ts);
    if (st != DD_OK) return st;
    HIPCK(c, dd::launch_unpack_spinor(c->g, c->stream, prec, x, tx));
    return DD_OK;
}

// D x = b, or D^dagger x = b when dagger is set: D^dagger = gamma_5 D gamma_5, so
// y = gamma_5 x solves D y = gamma_5 b; the gamma_5 is applied while packing b
// and x and while unpacking the result
static dd_status solve_entry(dd_ctx *c, void *x_dev, const void *b_dev, double tol, int maxiter, dd_solve_mode mode,
                             dd_solve_info *info, bool dagger)
{
    if (!c || !x_dev || !b_dev) return fail(c, DD_ERR_ARG, "null argument");
    if (!(tol > 0) || maxiter < 0 || mode < DD_SOLVE_F64_PLAIN || mode > DD_SOLVE_MIXED_GCR)
        return fail(c, DD_ERR_ARG, "bad tolerance, maxiter or mode");
    if (!c->gauge) return fail(c, DD_ERR_STATE, "no gauge field loaded");
    auto t0 = std::chrono::steady_clock::now();
    dd_solve_info inf{};
    void *b = c->f64[0], *x = c->f64[1];
    HIPCK(c, dd::launch_pack_spinor(c->g, c->stream, DD_F64, b, b_dev, dagger));
    double bn2;
    dd_status st = norm2(c, b, 0, &bn2);
    if (st != DD_OK) return st;
    if (!is_fin(bn2)) return fail(c, DD_ERR_NONFINITE, "source holds NaN or Inf");
    dd_status res = DD_OK;
    if (mode == DD_SOLVE_F64_PLAIN) {
        HIPCK(c, dd::launch_pack_spinor(c->g, c->stream, DD_F64, x, x_dev, dagger));
        SolveOut o;
        res = solve_plain64(c, x, b, tol, maxiter, o);
        if (res < 0) return res;
        inf.iters_outer = 1;
        inf.iters_inner_total = o.iters;
        inf.relres_inner_last = o.relres;
        inf.status_detail = o.detail;
    } else if (mode == DD_SOLVE_F32_SAP) {
        void *src = c->f32[0], *y = c->f32[1];
        if ((st = blas(c, mkb(dd::BLAS_CINV_SRC, {src, b, c->cinv32}, {1, 0}, {1.0}))) != DD_OK) return st;
        SolveOut o;
        res = solve_sap32(c, 1, src, y, tol, maxiter, o);
        if (res < 0) return res;
        if ((st = copy(c, x, 0, y, 1)) != DD_OK) return st;
        inf.iters_outer = 1;
        inf.iters_inner_total = o.iters;
        inf.relres_inner_last = o.relres;
        inf.status_detail = o.detail;
    } else {
        // Alg. 4: x += err * P_DP(A_SP^{-1} R_SP(C_inv r / err)), r = b - D x in FP64
        HIPCK(c, dd::launch_pack_spinor(c->g, c->stream, DD_F64, x, x_dev, dagger));
        void *r = c->f64[2], *tmp = c->f64[3];
        void *src = c->f32[0], *y = c->f32[1];
        double rn2;
        if ((st = residual64(c, r, b, x, tmp, &rn2)) != DD_OK) return st;
        double prev = rn2;
        int stall = 0, outer = 0;
        res = DD_NOT_CONVERGED;
        if (bn2 == 0.0) HIPCK(c, hipMemsetAsync(x, 0, spinor_bytes(c->g, DD_F64), c->stream));
        while (true) {
            if (bn2 == 0.0 || std::sqrt(rn2 / bn2) < tol) {
                res = DD_OK;
                break;
            }
            if (outer >= maxiter) break;
            double err = std::sqrt(rn2);
            if ((st = blas(c, mkb(dd::BLAS_CINV_SRC, {src, r, c->cinv32}, {1, 0}, {1.0 / err}))) != DD_OK) return st;
            // each pass reduces the residual by inner_tol, except that the last
            // pass stops once the outer target is met (with a factor 2 margin)
            const double need = 0.5 * tol * std::sqrt(bn2) / err;
            const double itol = need > c->prm.inner_tol ? (need < 0.1 ? need : 0.1) : c->prm.inner_tol;
            SolveOut o;
            dd_status si = mode == DD_SOLVE_MIXED_GCR ? solve_gcr32(c, src, y, itol, c->prm.inner_maxiter, o)
                                                      : solve_sap32(c, 2, src, y, itol, c->prm.inner_maxiter, o);
            if (si < 0) return si;
            inf.iters_inner_total += o.iters;
            inf.relres_inner_last = o.relres;
            if ((st = blas(c, mkb(dd::BLAS_AXPBY, {y, x}, {1, 0}, {err, 1.0}))) != DD_OK) return st;
            if ((st = residual64(c, r, b, x, tmp, &rn2)) != DD_OK) return st;
            ++outer;
            if (!is_fin(rn2) || rn2 >= prev) {
                // the correction made the true residual worse (inner solve failed):
                // take it back, so x stays the best iterate, and stop
                if ((st = blas(c, mkb(dd::BLAS_AXPBY, {y, x}, {1, 0}, {-err, 1.0}))) != DD_OK) return st;
                if ((st = residual64(c, r, b, x, tmp, &rn2)) != DD_OK) return st;
                inf.status_detail = is_fin(rn2) ? 5 : 4;
                res = DD_BREAKDOWN;
                break;
            }
            if (c->verbose) {
                std::fprintf(stderr, "[ddsolve] outer pass %d: %d inner iterations (inner tol %.1e, reached %.2e), "
                             "true residual %.3e\n", outer, o.iters, itol, o.relres, std::sqrt(rn2 / bn2));
                std::fflush(stderr);
            }
            stall = rn2 > 0.81 * prev ? stall + 1 : 0;  // |r| fell by less than 10%
            prev = rn2;
            if (stall >= 2) {
                inf.status_detail = 5;
                res = DD_BREAKDOWN;
                break;
            }
        }
        inf.iters_outer = outer;
    }
    // true FP64 residual of the returned x
    {
        double rn2;
        if ((st = residual64(c, c->f64[2], b, x, c->f64[3], &rn2)) != DD_OK) return st;
        inf.relres_true = bn2 > 0 ? std::sqrt(rn2 / bn2) : 0.0;
    }
    HIPCK(c, dd::launch_unpack_spinor(c->g, c->stream, DD_F64, x_dev, x, dagger));
    HIPCK(c, hipStreamSynchronize(c->stream));
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return res;
}

dd_status bicgstab_solve(dd_ctx *c, void *x_dev, const void *b_dev, double tol, int maxiter, dd_solve_mode mode,
                         dd_solve_info *info)
{
    return solve_entry(c, x_dev, b_dev, tol, maxiter, mode, info, false);
}

dd_status bicgstab_solve_dagger(dd_ctx *c, void *x_dev, const void *b_dev, double tol, int maxiter,
                                dd_solve_mode mode, dd_solve_info *info)
{
    return solve_entry(c, x_dev, b_dev, tol, maxiter, mode, info, true);
}

dd_status dd_spinor_norm2(dd_ctx *c, const void *x_dev, double *out)
{
    if (!c || !x_dev || !out) return fail(c, DD_ERR_ARG, "null argument");
    void *t = c->f64[5];
    HIPCK(c, dd::launch_pack_spinor(c->g, c->stream, DD_F64, t, x_dev));
    return norm2(c, t, 0, out);
}

dd_status dd_set_csw(dd_ctx *c, double csw)
{
    if (!c) return DD_ERR_ARG;
    if (!std::isfinite(csw)) return fail(c, DD_ERR_ARG, "c_SW must be finite");
    c->prm.csw = csw;
    c->gauge = false;  // the clover blocks depend on c_SW: dd_load_gauge again
    return DD_OK;
}

dd_status dd_force(dd_ctx *c, void *out_dev, double *dcsw, const void *psi_dev, const void *chi_dev, int su3)
{
    if (!c || !out_dev || !psi_dev || !chi_dev) return fail(c, DD_ERR_ARG, "null argument");
    if (su3 != 0 && su3 != 1) return fail(c, DD_ERR_ARG, "su3 must be 0 or 1");
    if (!c->gauge) return fail(c, DD_ERR_STATE, "no gauge field loaded");
    const Geom &g = c->g;
    if (!c->yforce && hipMalloc(&c->yforce, (size_t)g.V * 54 * 16) != hipSuccess) {
        (void)hipGetLastError();
        c->yforce = nullptr;
        return fail(c, DD_ERR_NOMEM, "force work field");
    }
    dd::ForceArgs a{};
    a.psi = c->f64[0];
    a.chi = c->f64[1];
    HIPCK(c, dd::launch_pack_spinor(g, c->stream, DD_F64, c->f64[0], psi_dev));
    HIPCK(c, dd::launch_pack_spinor(g, c->stream, DD_F64, c->f64[1], chi_dev));
    a.u64 = c->U64;
    a.y = c->yforce;
    a.out = out_dev;
    a.partials = dcsw ? c->partials : nullptr;
    a.dcsw = c->red;
    if (!sigma_blocks(a.sig)) return fail(c, DD_ERR_ARG, "sigma blocks not block diagonal");
    a.kcsw = c->prm.kappa * c->prm.csw;
    a.kappa = c->prm.kappa;
    a.phase = c->phase;
    a.su3 = su3;
    // per site: psi, chi, four links and the six Y planes read twice over (once
    // written), the output links written; flops of the hop outer products, the
    // 24 leaves per link (nine 3x3 products per plaquette) and the dcsw traces
    const double V = (double)g.V;
    const double bytes = V * (2 * 192.0 + 4 * 144.0 + 2 * 864.0 + 4 * 144.0 + (dcsw ? 4 * 144.0 : 0.0));
    const double flops = V * (4 * FORCE_LINK_FLOPS + FORCE_Y_FLOPS + (dcsw ? FORCE_DCSW_FLOPS : 0.0));
    hipError_t e = timed(c, DD_KT_FORCE, bytes, flops, [&] { return dd::launch_force(g, c->stream, a); });
    if (e != hipSuccess) return fail(c, DD_ERR_HIP, std::string("force launch: ") + hipGetErrorString(e));
    if (dcsw) {
        HIPCK(c, hipMemcpyAsync(c->red_host, c->red, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCK(c, hipStreamSynchronize(c->stream));
        *dcsw = c->red_host[0];
    } else {
        HIPCK(c, hipStreamSynchronize(c->stream));
    }
    return DD_OK;
}

dd_status dirac_apply_batch(dd_ctx *c, void *out, const void *in, int nrhs, dd_prec prec, dd_op op)
{
    if (!c || !out || !in) return fail(c, DD_ERR_ARG, "null argument");
    if (nrhs < 1) return fail(c, DD_ERR_ARG, "nrhs must be at least 1");
    dd_status st = check_op(c, prec, op);
    if (st != DD_OK) return st;
    if (prec == DD_F16) return fail(c, DD_ERR_ARG, "batched apply: DD_F64 (D, D^dagger) or DD_F32 (A)");
    const size_t cb = (size_t)c->g.V * 12 * 16;  // canonical field bytes
    if (prec == DD_F64) {
        for (int r = 0; r < nrhs; ++r)
            if ((st = dirac_apply(c, (char *)out + r * cb, (const char *)in + r * cb, prec, op)) != DD_OK) return st;
        return DD_OK;
    }
    const int tile = nrhs < 12 ? nrhs : 12;
    if ((st = batch_alloc(c, tile)) != DD_OK) return st;
    const size_t fb = spinor_bytes(c->g, DD_F32);
    for (int r0 = 0; r0 < nrhs; r0 += 12) {
        const int m = nrhs - r0 < 12 ? nrhs - r0 : 12;
        for (int r = 0; r < m; ++r)
            HIPCK(c, dd::launch_pack_spinor(c->g, c->stream, DD_F32, (char *)c->bk[BK_IN] + r * fb,
                                            (const char *)in + (r0 + r) * cb));
        if ((st = k_dirac_mrhs(c, c->bk[BK_OUT], c->bk[BK_IN], m)) != DD_OK) return st;
        for (int r = 0; r < m; ++r)
            HIPCK(c, dd::launch_unpack_spinor(c->g, c->stream, DD_F32, (char *)out + (r0 + r) * cb,
                                              (char *)c->bk[BK_OUT] + r * fb));
    }
    return DD_OK;
}

dd_status dd_batch_set_variant(dd_ctx *c, int variant)
{
    if (!c) return DD_ERR_ARG;
    if (variant < -1 || variant >= dd::mrhs_variant_count()) return fail(c, DD_ERR_ARG, "no such variant");
    c->mrhs_force = variant;
    return DD_OK;
}

dd_status dd_batch_tuning(dd_ctx *c, int nrhs, int *variant, double *ms, int n_ms)
{
    if (!c || nrhs < 1 || nrhs > 12) return fail(c, DD_ERR_ARG, "nrhs must be 1..12");
    if (variant) *variant = c->mrhs_force >= 0 ? c->mrhs_force : c->mrhs_tuned[nrhs];
    const int nv = dd::mrhs_variant_count();
    for (int v = 0; ms && v < n_ms; ++v) ms[v] = v < nv ? c->mrhs_ms[nrhs][v] : 0.0;
    return DD_OK;
}

const char *dd_batch_variant_name(int variant) { return dd::mrhs_variant_name(variant); }

dd_status bicgstab_solve_batch(dd_ctx *c, void *x_dev, const void *b_dev, int nrhs, double tol, int maxiter,
                               dd_batch_inner inner, dd_solve_info *info)
{
    if (!c || !x_dev || !b_dev) return fail(c, DD_ERR_ARG, "null argument");
    if (nrhs < 1 || nrhs > BATCH_MAX) return fail(c, DD_ERR_ARG, "nrhs must be 1..16");
    if (!(tol > 0) || maxiter < 0 || (inner != DD_BATCH_INNER_SAP && inner != DD_BATCH_INNER_PLAIN))
        return fail(c, DD_ERR_ARG, "bad tolerance, maxiter or inner solver");
    if (!c->gauge) return fail(c, DD_ERR_STATE, "no gauge field loaded");
    auto t0 = std::chrono::steady_clock::now();
    dd_status st = batch_alloc(c, nrhs);
    if (st != DD_OK) return st;
    const int n = nrhs;
    const size_t cb = (size_t)c->g.V * 12 * 16;
    std::vector<dd_solve_info> inf(n);
    std::vector<BRhs> R(n);
    double bn2[BATCH_MAX], rn2[BATCH_MAX], prev[BATCH_MAX];
    for (int r = 0; r < n; ++r) {
        HIPCK(c, dd::launch_pack_spinor(c->g, c->stream, DD_F64, bf(c, BK_B64, r), (const char *)b_dev + r * cb));
        HIPCK(c, dd::launch_pack_spinor(c->g, c->stream, DD_F64, bf(c, BK_X64, r), (const char *)x_dev + r * cb));
        if ((st = reduce_to(c, mkb(dd::BLAS_NORM2, {bf(c, BK_B64, r)}, {0}), 1, r)) != DD_OK) return st;
    }
    if ((st = fetch_red(c, n, bn2)) != DD_OK) return st;
    for (int r = 0; r < n; ++r)
        if (!is_fin(bn2[r])) return fail(c, DD_ERR_NONFINITE, "a source holds NaN or Inf");
    for (int r = 0; r < n; ++r)
        if (bn2[r] == 0.0) HIPCK(c, hipMemsetAsync(bf(c, BK_X64, r), 0, spinor_bytes(c->g, DD_F64), c->stream));
    if ((st = residual64_batch(c, n, rn2)) != DD_OK) return st;
    // per right-hand side: 0 running, 1 converged, 2 stopped (breakdown or stagnation)
    std::vector<int> state(n, 0);
    std::vector<int> stall(n, 0);
    std::vector<dd_status> res(n, DD_NOT_CONVERGED);
    for (int r = 0; r < n; ++r) prev[r] = rn2[r];
    const size_t f32 = spinor_bytes(c->g, DD_F32);
    for (int outer = 0;; ++outer) {
        int running = 0;
        for (int r = 0; r < n; ++r) {
            if (state[r] != 0) continue;
            if (bn2[r] == 0.0 || std::sqrt(rn2[r] / bn2[r]) < tol) {
                state[r] = 1;
                res[r] = DD_OK;
            } else
                ++running;
        }
        if (running == 0 || outer >= maxiter) break;
        // inner sources C_inv r / err for the running right-hand sides, zero for the others
        double err[BATCH_MAX];
        for (int r = 0; r < n; ++r) {
            err[r] = std::sqrt(rn2[r]);
            R[r].tol = 1.0;
            if (state[r] != 0) {
                HIPCK(c, hipMemsetAsync(bf(c, BK_SRC, r), 0, f32, c->stream));
                continue;
            }
            if ((st = blas(c, mkb(dd::BLAS_CINV_SRC, {bf(c, BK_SRC, r), bf(c, BK_R64, r), c->cinv32}, {1, 0},
                                  {1.0 / err[r]}))) != DD_OK)
                return st;
            const double need = 0.5 * tol * std::sqrt(bn2[r]) / err[r];
            R[r].tol = need > c->prm.inner_tol ? (need < 0.1 ? need : 0.1) : c->prm.inner_tol;
        }
        if ((st = solve_batch32(c, n, inner == DD_BATCH_INNER_SAP, R, c->prm.inner_maxiter)) != DD_OK) return st;
        for (int r = 0; r < n; ++r) {
            if (state[r] != 0) continue;
            inf[r].iters_inner_total += R[r].o.iters;
            inf[r].relres_inner_last = R[r].o.relres;
            if ((st = blas(c, mkb(dd::BLAS_AXPBY, {bf(c, BK_Y, r), bf(c, BK_X64, r)}, {1, 0}, {err[r], 1.0}))) != DD_OK)
                return st;
        }
        if ((st = residual64_batch(c, n, rn2)) != DD_OK) return st;
        for (int r = 0; r < n; ++r) {
            if (state[r] != 0) continue;
            inf[r].iters_outer = outer + 1;
            if (!is_fin(rn2[r]) || rn2[r] >= prev[r]) {
                // the correction made the true residual worse: take it back and stop this one
                if ((st = blas(c, mkb(dd::BLAS_AXPBY, {bf(c, BK_Y, r), bf(c, BK_X64, r)}, {1, 0}, {-err[r], 1.0}))) !=
                    DD_OK)
                    return st;
                state[r] = 2;
                res[r] = DD_BREAKDOWN;
                inf[r].status_detail = is_fin(rn2[r]) ? 5 : 4;
                continue;
            }
            stall[r] = rn2[r] > 0.81 * prev[r] ? stall[r] + 1 : 0;
            prev[r] = rn2[r];
            if (stall[r] >= 2) {
                state[r] = 2;
                res[r] = DD_BREAKDOWN;
                inf[r].status_detail = 5;
            }
        }
        if (c->verbose) {
            int conv = 0;
            for (int r = 0; r < n; ++r) conv += state[r] == 1 || (bn2[r] > 0 && std::sqrt(rn2[r] / bn2[r]) < tol);
            std::fprintf(stderr, "[ddsolve] batched outer pass %d: %d of %d right-hand sides at tolerance\n", outer + 1,
                         conv, n);
            std::fflush(stderr);
        }
    }
    // true FP64 residuals of the returned solutions
    if ((st = residual64_batch(c, n, rn2)) != DD_OK) return st;
    dd_status worst = DD_OK;
    for (int r = 0; r < n; ++r) {
        inf[r].relres_true = bn2[r] > 0 ? std::sqrt(rn2[r] / bn2[r]) : 0.0;
        if (res[r] == DD_NOT_CONVERGED && inf[r].relres_true < tol) res[r] = DD_OK;
        if (res[r] > worst) worst = res[r];
        HIPCK(c, dd::launch_unpack_spinor(c->g, c->stream, DD_F64, (char *)x_dev + r * cb, bf(c, BK_X64, r)));
    }
    HIPCK(c, hipStreamSynchronize(c->stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int r = 0; r < n; ++r) {
        inf[r].seconds = secs;
        if (res[r] == DD_BREAKDOWN && inf[r].status_detail == 0) inf[r].status_detail = 4;
        if (info) info[r] = inf[r];
    }
    return worst;
}

dd_status dd_multi_create(const dd_params *params, int nlat, void *hip_stream, dd_multi **out)
{
    if (!params || !out || nlat < 1 || nlat > 64) return DD_ERR_ARG;
    *out = nullptr;
    dd_multi *m = new (std::nothrow) dd_multi;
    if (!m) return DD_ERR_NOMEM;
    m->stream = (hipStream_t)hip_stream;
    for (int k = 0; k < nlat; ++k) {
        dd_ctx *c = nullptr;
        dd_status st = dd_create(&params[k], hip_stream, &c);
        if (st != DD_OK) {
            dd_multi_destroy(m);
            return st;
        }
        m->L.push_back(c);
        m->total += (int)((c->g.V + 255) / 256);
    }
    bool ok = hipMalloc((void **)&m->counter, sizeof(int)) == hipSuccess &&
              hipMalloc((void **)&m->desc_dev, 3 * nlat * sizeof(dd::LatDesc)) == hipSuccess &&
              hipHostMalloc((void **)&m->desc_host, 3 * nlat * sizeof(dd::LatDesc), hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        dd_multi_destroy(m);
        return DD_ERR_NOMEM;
    }
    *out = m;
    return DD_OK;
}

dd_status dd_multi_destroy(dd_multi *m)
{
    if (!m) return DD_OK;
    if (!m->L.empty()) (void)hipStreamSynchronize(m->stream);  // no device call when nothing was created
    for (dd_ctx *c : m->L) dd_destroy(c);
    if (m->counter) (void)hipFree(m->counter);
    if (m->desc_dev) (void)hipFree(m->desc_dev);
    if (m->desc_host) (void)hipHostFree(m->desc_host);
    delete m;
    return DD_OK;
}

const char *dd_multi_last_error(const dd_multi *m) { return m ? m->err.c_str() : "null handle"; }

dd_ctx *dd_multi_context(dd_multi *m, int lat)
{
    if (!m || lat < 0 || lat >= (int)m->L.size()) return nullptr;
    return m->L[lat];
}

dd_status dd_multi_load_gauge(dd_multi *m, int lat, const void *U)
{
    if (!m || lat < 0 || lat >= (int)m->L.size()) return mfail(m, DD_ERR_ARG, "no such lattice");
    return lat_fail(m, lat, dd_load_gauge(m->L[lat], U));
}

static dd_status multi_ready(dd_multi *m)
{
    for (size_t k = 0; k < m->L.size(); ++k)
        if (!m->L[k]->gauge) return mfail(m, DD_ERR_STATE, "lattice " + std::to_string(k) + ": no gauge field loaded");
    return DD_OK;
}

dd_status dirac_apply_multi(dd_multi *m, void *const *out, const void *const *in)
{
    if (!m || !out || !in) return mfail(m, DD_ERR_ARG, "null argument");
    const int n = (int)m->L.size();
    for (int k = 0; k < n; ++k)
        if (!out[k] || !in[k]) return mfail(m, DD_ERR_ARG, "null field");
    dd_status st = multi_ready(m);
    if (st != DD_OK) return st;
    std::vector<const void *> vin(n);
    std::vector<void *> vout(n);
    for (int k = 0; k < n; ++k) {
        dd_ctx *c = m->L[k];
        vin[k] = c->f32[7];
        vout[k] = c->f32[8];
        MHIPCK(m, dd::launch_pack_spinor(c->g, m->stream, DD_F32, c->f32[7], in[k]));
    }
    fill_desc(m, m->desc_host, vin, vout);
    MHIPCK(m, hipMemcpyAsync(m->desc_dev, m->desc_host, n * sizeof(dd::LatDesc), hipMemcpyHostToDevice, m->stream));
    if ((st = multi_launch(m, 0, 1)) != DD_OK) return st;
    for (int k = 0; k < n; ++k)
        MHIPCK(m, dd::launch_unpack_spinor(m->L[k]->g, m->stream, DD_F32, out[k], m->L[k]->f32[8]));
    MHIPCK(m, hipStreamSynchronize(m->stream));  // the staging table is reused by the next call
    return DD_OK;
}

dd_status bicgstab_solve_multi(dd_multi *m, void *const *x_dev, const void *const *b_dev, double tol, int maxiter,
                               dd_solve_info *info)
{
    if (!m || !x_dev || !b_dev) return mfail(m, DD_ERR_ARG, "null argument");
    if (!(tol > 0) || maxiter < 0) return mfail(m, DD_ERR_ARG, "bad tolerance or maxiter");
    const int n = (int)m->L.size();
    for (int k = 0; k < n; ++k)
        if (!x_dev[k] || !b_dev[k]) return mfail(m, DD_ERR_ARG, "null field");
    dd_status st = multi_ready(m);
    if (st != DD_OK) return st;
    auto t0 = std::chrono::steady_clock::now();
    // descriptor tables of the two A applications of a BiCGStab step: M p -> q, M r -> t
    {
        std::vector<const void *> i1(n), i2(n);
        std::vector<void *> o1(n), o2(n);
        for (int k = 0; k < n; ++k) {
            dd_ctx *c = m->L[k];
            i1[k] = c->f16[2];
            o1[k] = c->f32[5];
            i2[k] = c->f16[3];
            o2[k] = c->f32[6];
        }
        fill_desc(m, m->desc_host + n, i1, o1);
        fill_desc(m, m->desc_host + 2 * n, i2, o2);
        MHIPCK(m, hipMemcpyAsync(m->desc_dev + n, m->desc_host + n, 2 * n * sizeof(dd::LatDesc), hipMemcpyHostToDevice,
                                 m->stream));
        MHIPCK(m, hipStreamSynchronize(m->stream));
    }
    std::vector<dd_solve_info> inf(n);
    std::vector<BRhs> R(n);
    std::vector<double> bn2(n), rn2(n), prev(n);
    std::vector<int> state(n, 0), stall(n, 0);
    std::vector<dd_status> res(n, DD_NOT_CONVERGED);
    for (int k = 0; k < n; ++k) {
        dd_ctx *c = m->L[k];
        MHIPCK(m, dd::launch_pack_spinor(c->g, m->stream, DD_F64, c->f64[0], b_dev[k]));
        MHIPCK(m, dd::launch_pack_spinor(c->g, m->stream, DD_F64, c->f64[1], x_dev[k]));
        if ((st = norm2(c, c->f64[0], 0, &bn2[k])) != DD_OK) return lat_fail(m, k, st);
        if (!is_fin(bn2[k])) return mfail(m, DD_ERR_NONFINITE, "a source holds NaN or Inf");
        if (bn2[k] == 0.0) MHIPCK(m, hipMemsetAsync(c->f64[1], 0, spinor_bytes(c->g, DD_F64), m->stream));
        if ((st = residual64(c, c->f64[2], c->f64[0], c->f64[1], c->f64[3], &rn2[k])) != DD_OK) return lat_fail(m, k, st);
        prev[k] = rn2[k];
    }
    for (int outer = 0;; ++outer) {
        int running = 0;
        for (int k = 0; k < n; ++k) {
            if (state[k] != 0) continue;
            if (bn2[k] == 0.0 || std::sqrt(rn2[k] / bn2[k]) < tol) {
                state[k] = 1;
                res[k] = DD_OK;
            } else
                ++running;
        }
        if (running == 0 || outer >= maxiter) break;
        std::vector<double> err(n);
        for (int k = 0; k < n; ++k) {
            dd_ctx *c = m->L[k];
            err[k] = std::sqrt(rn2[k]);
            R[k].tol = 1.0;
            if (state[k] != 0) {
                MHIPCK(m, hipMemsetAsync(c->f32[0], 0, spinor_bytes(c->g, DD_F32), m->stream));
                continue;
            }
            if ((st = blas(c, mkb(dd::BLAS_CINV_SRC, {c->f32[0], c->f64[2], c->cinv32}, {1, 0}, {1.0 / err[k]}))) != DD_OK)
                return lat_fail(m, k, st);
            const double need = 0.5 * tol * std::sqrt(bn2[k]) / err[k];
            R[k].tol = need > c->prm.inner_tol ? (need < 0.1 ? need : 0.1) : c->prm.inner_tol;
        }
        if ((st = solve_multi32(m, R, m->L[0]->prm.inner_maxiter)) != DD_OK) return st;
        for (int k = 0; k < n; ++k) {
            if (state[k] != 0) continue;
            dd_ctx *c = m->L[k];
            inf[k].iters_inner_total += R[k].o.iters;
            inf[k].relres_inner_last = R[k].o.relres;
            if ((st = blas(c, mkb(dd::BLAS_AXPBY, {c->f32[1], c->f64[1]}, {1, 0}, {err[k], 1.0}))) != DD_OK)
                return lat_fail(m, k, st);
            if ((st = residual64(c, c->f64[2], c->f64[0], c->f64[1], c->f64[3], &rn2[k])) != DD_OK)
                return lat_fail(m, k, st);
            inf[k].iters_outer = outer + 1;
            if (!is_fin(rn2[k]) || rn2[k] >= prev[k]) {
                if ((st = blas(c, mkb(dd::BLAS_AXPBY, {c->f32[1], c->f64[1]}, {1, 0}, {-err[k], 1.0}))) != DD_OK)
                    return lat_fail(m, k, st);
                state[k] = 2;
                res[k] = DD_BREAKDOWN;
                inf[k].status_detail = is_fin(rn2[k]) ? 5 : 4;
                continue;
            }
            stall[k] = rn2[k] > 0.81 * prev[k] ? stall[k] + 1 : 0;
            prev[k] = rn2[k];
            if (stall[k] >= 2) {
                state[k] = 2;
                res[k] = DD_BREAKDOWN;
                inf[k].status_detail = 5;
            }
        }
    }
    dd_status worst = DD_OK;
    for (int k = 0; k < n; ++k) {
        dd_ctx *c = m->L[k];
        if ((st = residual64(c, c->f64[2], c->f64[0], c->f64[1], c->f64[3], &rn2[k])) != DD_OK) return lat_fail(m, k, st);
        inf[k].relres_true = bn2[k] > 0 ? std::sqrt(rn2[k] / bn2[k]) : 0.0;
        if (res[k] == DD_NOT_CONVERGED && inf[k].relres_true < tol) res[k] = DD_OK;
        if (res[k] > worst) worst = res[k];
        MHIPCK(m, dd::launch_unpack_spinor(c->g, m->stream, DD_F64, x_dev[k], c->f64[1]));
    }
    MHIPCK(m, hipStreamSynchronize(m->stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int k = 0; k < n; ++k) {
        inf[k].seconds = secs;
        if (res[k] == DD_BREAKDOWN && inf[k].status_detail == 0) inf[k].status_detail = 4;
        if (info) info[k] = inf[k];
    }
    return worst;
}

dd_status dd_timing_enable(dd_ctx *c, int on)
{
    if (!c) return DD_ERR_ARG;
    HIPCK(c, flush_timing(c));
    c->timing = on != 0;
    for (int k = 0; k < DD_KT_COUNT; ++k) {
        c->launches[k] = 0;
        c->ms[k] = c->bytes[k] = c->flops[k] = 0;
    }
    return DD_OK;
}

dd_status dd_timing_query(dd_ctx *c, dd_kernel_class cls, long long *launches, double *ms, double *bytes,
                          double *flops)
{
    if (!c || cls < 0 || cls >= DD_KT_COUNT) return fail(c, DD_ERR_ARG, "bad kernel class");
    HIPCK(c, flush_timing(c));
    if (launches) *launches = c->launches[cls];
    if (ms) *ms = c->ms[cls];
    if (bytes) *bytes = c->bytes[cls];
    if (flops) *flops = c->flops[cls];
    return DD_OK;
}

}  // extern "C"
