// dd_solvers.cpp -- the single right-hand-side solver loops:
//   plain FP64 BiCGStab on D (Alg. 5 without preconditioner),
//   FP32 BiCGStab on A M_SAP (Alg. 5 with Alg. 1 as right preconditioner),
//   restarted flexible GCR on A M_SAP (FP16 SAP).
// The kernels do every step; these loops sequence launches and evaluate the scalars.
#include "dd_host.h"

namespace ddh {

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
    // FP16 SAP: the updates that produce r and p also write their FP16 copies (the SAP's
    // inputs), and y takes alpha Mp + omega Mr in one pass per iteration
    const bool fused = prec == 2;
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
    if (fused && (st = copy(c, p16, 2, src, 1)) != DD_OK) return st;
    cplx rho0 = bn2;
    double rn2 = bn2;
    Stall stall{c->prm.stall_window};
    auto precond = [&](void *in, void *in16, void *Mout, void *Aout) -> dd_status {
        dd_status s2;
        const void *bsrc = in;
        if (prec == 2) {
            if (!fused && (s2 = copy(c, in16, 2, in, 1)) != DD_OK) return s2;
            bsrc = in16;
        }
        if ((s2 = k_sap(c, prec, bsrc, Mout, s)) != DD_OK) return s2;
        return k_dirac(c, Aout, Mout, prec, 1, 1, 1);
    };
    cplx alpha = 0.0;
    // with the fused updates y lacks alpha Mp between the two half steps: add it on an exit there
    auto settle_y = [&]() -> dd_status {
        if (!fused) return DD_OK;
        return blas(c, mkb(dd::BLAS_CAXPY, {y, Mp}, {1, prec}, {alpha.real(), alpha.imag()}));
    };
    for (int it = 0; it < maxiter; ++it) {
        o.iters = it + 1;
        c->hist_inner.push_back(std::sqrt(rn2 / bn2));  // one entry per iteration: its last residual
        if ((st = precond(p, p16, Mp, q)) != DD_OK) return st;
        double d[3];
        if ((st = reduce(c, mkb(dd::BLAS_DOT, {rt, q}, {1, 1}), 2, d)) != DD_OK) return st;
        cplx rq(d[0], d[1]);
        if (rq == 0.0 || !is_fin(rq)) {
            o.detail = rq == 0.0 ? 1 : 4;
            o.relres = std::sqrt(rn2 / bn2);
            return DD_BREAKDOWN;
        }
        alpha = rho0 / rq;
        if (fused)
            st = reduce(c, mkb(dd::BLAS_UPDATE1_H, {r, q, r16}, {1, 1, 2}, {alpha.real(), alpha.imag()}), 1, &rn2);
        else
            st = reduce(c, mkb(dd::BLAS_UPDATE1, {y, Mp, r, q}, {1, prec, 1}, {alpha.real(), alpha.imag()}), 1, &rn2);
        if (st != DD_OK) return st;
        o.relres = std::sqrt(rn2 / bn2);
        c->hist_inner.back() = o.relres;
        if (o.relres < tol) return settle_y();
        if (c->verbose && (it + 1) % 100 == 0) {
            std::fprintf(stderr, "[ddsolve] inner iteration %d: relative residual %.3e\n", it + 1, o.relres);
            std::fflush(stderr);
        }
        if ((st = precond(r, r16, Mr, t)) != DD_OK) return st;
        if ((st = reduce(c, mkb(dd::BLAS_DOT_NORM, {t, r}, {1, 1}), 3, d)) != DD_OK) return st;
        if (d[2] == 0.0 || !is_fin(d[2])) {
            o.detail = d[2] == 0.0 ? 2 : 4;
            if ((st = settle_y()) != DD_OK) return st;
            return DD_BREAKDOWN;
        }
        cplx omega = cplx(d[0], d[1]) / d[2];
        if (fused)
            st = reduce(c, mkb(dd::BLAS_UPDATE2_MM, {y, Mp, Mr, r, t, rt}, {1, prec, 1, 1, 1, 1},
                               {alpha.real(), alpha.imag(), omega.real(), omega.imag()}),
                        3, d);
        else
            st = reduce(c, mkb(dd::BLAS_UPDATE2, {y, Mr, r, t, rt}, {1, prec, 1}, {omega.real(), omega.imag()}), 3, d);
        if (st != DD_OK) return st;
        rn2 = d[0];
        cplx rho(d[1], d[2]);
        o.relres = std::sqrt(rn2 / bn2);
        c->hist_inner.back() = o.relres;
        if (o.relres < tol) return DD_OK;
        if (stall.hit(it + 1, o.relres)) {  // y is complete here: both half steps are in
            o.detail = DETAIL_INNER_STALL;
            return DD_BREAKDOWN;
        }
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
        if (fused)
            st = blas(c, mkb(dd::BLAS_PUPDATE_H, {p, r, q, p16}, {1, 1, 1, 2},
                             {beta.real(), beta.imag(), omega.real(), omega.imag()}));
        else
            st = blas(c, mkb(dd::BLAS_PUPDATE, {p, r, q}, {1, 1, 1}, {beta.real(), beta.imag(), omega.real(), omega.imag()}));
        if (st != DD_OK) return st;
    }
    return DD_NOT_CONVERGED;
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
    Stall stall{c->prm.stall_window};
    bool stalled = false;
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
            c->hist_inner.push_back(o.relres);
            if (c->verbose && o.iters % 100 == 0) {
                std::fprintf(stderr, "[ddsolve] GCR iteration %d: relative residual %.3e\n", o.iters, o.relres);
                std::fflush(stderr);
            }
            stalled = o.relres >= tol && stall.hit(o.iters, o.relres);
            if (o.relres < tol || o.iters >= maxiter || stalled) {
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
    if (stalled) o.detail = DETAIL_INNER_STALL;
    return o.relres < tol ? DD_OK : (o.detail ? DD_BREAKDOWN : DD_NOT_CONVERGED);
}

}  // namespace ddh
