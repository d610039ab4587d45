// dd_solvers.cpp -- the single right-hand-side solver loops:
//   plain FP64 BiCGStab on D (Alg. 5 without preconditioner),
//   FP32 BiCGStab on A M_SAP (Alg. 5 with Alg. 1 as right preconditioner),
//   restarted flexible GCR on A M_SAP (FP16 SAP).
// The kernels do every step; these loops sequence launches and evaluate the scalars.
#include <algorithm>

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
            Range range("ddsolve: FP64 BiCGStab iteration");
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
        // FP32 SAP: A M_SAP by the fused tail of Alg. 3 when asked for; FP16 SAP: the FP32 operator
        // applied to the FP16-stored M output (the inner recursion needs A to FP32 accuracy)
        if (prec == 1 && c->prm.sap_fused_tail) return k_sap(c, 1, bsrc, Mout, s, Aout);
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
        Range range("ddsolve: inner BiCGStab iteration");
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
        if (c->prm.debug_flags & (prec == 2 ? DD_DEBUG_ZERO_OMEGA_F16 : DD_DEBUG_ZERO_OMEGA_F32)) omega = 0.0;
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

dd_status ensure_gcr(dd_ctx *c)
{
    for (int i = 0; i < c->prm.gcr_nkv; ++i) {
        if (!c->gz[i] && hipMalloc(&c->gz[i], spinor_bytes(c->g, DD_F32)) != hipSuccess) c->gz[i] = nullptr;
        if (!c->gp[i] && hipMalloc(&c->gp[i], spinor_bytes(c->g, DD_F16)) != hipSuccess) c->gp[i] = nullptr;
        if (!c->gz[i] || !c->gp[i]) {
            (void)hipGetLastError();
            return fail(c, DD_ERR_NOMEM, "GCR fields");
        }
    }
    return DD_OK;
}

// The flexible GMRES basis takes the FP64 work vectors that neither the outer loop (b, x, the
// product D z) nor the inner FP32 solve touch, and the directions the FP32 vectors of the
// FP32-storage SAP (the inner solve runs the FP16 SAP); only the rest is allocated.
dd_status ensure_fgmres(dd_ctx *c)
{
    const int m = c->prm.fgmres_nkv;
    void *v_alias[] = {c->f64[2], c->f64[4], c->f64[5], c->f64[6]};
    void *z_alias[] = {c->f32[7], c->f32[8], c->f32[9]};
    constexpr int NVA = sizeof(v_alias) / sizeof(v_alias[0]), NZA = sizeof(z_alias) / sizeof(z_alias[0]);
    for (int i = 0; i <= m; ++i) {
        if (i < NVA) {
            c->fv[i] = v_alias[i];
        } else {
            if (!c->fv_own[i] && hipMalloc(&c->fv_own[i], spinor_bytes(c->g, DD_F64)) != hipSuccess)
                c->fv_own[i] = nullptr;
            c->fv[i] = c->fv_own[i];
        }
        if (i == m) break;
        if (i < NZA) {
            c->fz[i] = z_alias[i];
        } else {
            if (!c->fz_own[i] && hipMalloc(&c->fz_own[i], spinor_bytes(c->g, DD_F32)) != hipSuccess)
                c->fz_own[i] = nullptr;
            c->fz[i] = c->fz_own[i];
        }
        if (!c->fv[i] || !c->fz[i]) {
            (void)hipGetLastError();
            return fail(c, DD_ERR_NOMEM, "flexible GMRES fields");
        }
    }
    if (!c->fv[m]) {
        (void)hipGetLastError();
        return fail(c, DD_ERR_NOMEM, "flexible GMRES fields");
    }
    return DD_OK;
}

// Restarted flexible GMRES (Saad's FGMRES, the flexible outer loop Sec. 3 names) on D x = b
// in FP64.  A cycle starts from r = b - D x, v_0 = r / |r|; iteration j preconditions the
// Arnoldi vector by an inner FP32 solve, z_j ~ D^{-1} v_j (BiCGStab on A M_SAP with the FP16
// SAP for A z = C_inv v_j, A = C_inv D), keeps z_j, and orthogonalises w = D z_j against
// v_0 .. v_j (classical Gram-Schmidt applied twice, FP64 sums) into H and v_{j+1}; Givens
// rotations keep the least-squares residual |beta e_0 - H y| at hand.  At the cycle's end
// x += sum_j y_j z_j.  The kept z_j make the varying preconditioner harmless: x minimises
// the FP64 residual over x_0 + span{z_j} whatever the inner solves returned.
dd_status solve_fgmres64(dd_ctx *c, void *x, void *b, double bn2, double tol, int maxiter, OuterOut &o)
{
    const Geom &g = c->g;
    const int m = c->prm.fgmres_nkv;
    const double V = (double)g.V, bnorm = std::sqrt(bn2);
    void *tmp = c->f64[3], *src = c->f32[0];
    dd_status st;
    std::vector<cplx> H((size_t)(m + 1) * m), gv(m + 1), cs(m), sn(m), yv(m);
    auto h_at = [&](int i, int j) -> cplx & { return H[(size_t)i * m + j]; };
    double rn2 = 0, prev = 0;
    int stall = 0;
    for (int cycle = 0;; ++cycle) {
        if ((st = residual64(c, c->fv[0], b, x, tmp, &rn2)) != DD_OK) return st;
        const double beta = std::sqrt(rn2);
        if (!is_fin(rn2)) {
            o.detail = 4;
            return DD_BREAKDOWN;
        }
        if (cycle == 0)
            c->hist_outer.push_back(beta / bnorm);
        else
            c->hist_outer.back() = beta / bnorm;  // the true residual in place of the estimate
        if (beta / bnorm < tol) return DD_OK;
        if (cycle > 0) {
            stall = rn2 > 0.81 * prev ? stall + 1 : 0;  // a cycle lowered |r| by less than 10%
            if (stall >= 2) {
                o.detail = DETAIL_OUTER_STALL;
                return DD_BREAKDOWN;
            }
        }
        prev = rn2;
        if (o.outer >= maxiter) return DD_NOT_CONVERGED;
        if ((st = blas(c, mkb(dd::BLAS_AXPBY, {c->fv[0], c->fv[0]}, {0, 0}, {1.0 / beta, 0.0}))) != DD_OK) return st;
        std::fill(gv.begin(), gv.end(), cplx(0.0));
        gv[0] = beta;
        double resid = beta;
        int n = 0;
        for (int j = 0; j < m && o.outer < maxiter; ++j) {
            // z_j = M v_j: the inner solve of A z = C_inv v_j to the reduction still needed
            const double need = 0.5 * tol * bnorm / resid;
            const double itol = need > c->prm.inner_tol ? (need < 0.1 ? need : 0.1) : c->prm.inner_tol;
            Range range("ddsolve: flexible GMRES iteration");
            if ((st = blas(c, mkb(dd::BLAS_CINV_SRC, {src, c->fv[j], c->cinv32}, {1, 0}, {1.0}))) != DD_OK) return st;
            SolveOut io;
            dd_status si = solve_sap32(c, 2, src, c->fz[j], itol, c->prm.inner_maxiter, io);
            if (si < 0) return si;
            ++o.outer;
            o.inner += io.iters;
            o.inner_last = io.relres;
            // w = D z_j, orthogonalised against v_0 .. v_j
            if ((st = copy(c, tmp, 0, c->fz[j], 1)) != DD_OK) return st;
            if ((st = k_dirac(c, c->fv[j + 1], tmp, 0, 0, 0, 0)) != DD_OK) return st;
            dd::VecSet vs{};
            for (int i = 0; i <= j; ++i) vs.v[i] = c->fv[i];
            double wn2 = 0;
            for (int pass = 0; pass < 2; ++pass) {
                double d[2 * dd::GCR_MAX_NKV];
                hipError_t e = timed(c, DD_KT_BLAS, V * 192.0 * (j + 2), V * 96.0 * (j + 1), [&] {
                    return dd::launch_multidot(g, c->stream, vs, j + 1, c->fv[j + 1], c->partials, 0);
                });
                if (e != hipSuccess) return fail(c, DD_ERR_HIP, std::string("multidot: ") + hipGetErrorString(e));
                if ((st = fetch(c, 2 * (j + 1), d)) != DD_OK) return st;
                for (int i = 0; i <= j; ++i) {
                    const cplx hij(d[2 * i], d[2 * i + 1]);
                    h_at(i, j) = pass == 0 ? hij : h_at(i, j) + hij;
                    vs.re[i] = hij.real();
                    vs.im[i] = hij.imag();
                }
                e = timed(c, DD_KT_BLAS, V * 192.0 * (j + 3), V * 96.0 * (j + 2), [&] {
                    return dd::launch_orth64(g, c->stream, vs, j + 1, c->fv[j + 1], c->partials);
                });
                if (e != hipSuccess) return fail(c, DD_ERR_HIP, std::string("orthogonalise: ") + hipGetErrorString(e));
                if ((st = fetch(c, 1, &wn2)) != DD_OK) return st;
            }
            if (!is_fin(wn2)) {
                o.detail = 4;
                return DD_BREAKDOWN;
            }
            const double hn = std::sqrt(wn2);
            // earlier rotations on column j, then the one that removes h_{j+1,j}
            for (int i = 0; i < j; ++i) {
                const cplx a = h_at(i, j), bb = h_at(i + 1, j);
                h_at(i, j) = cs[i] * a + sn[i] * bb;
                h_at(i + 1, j) = -std::conj(sn[i]) * a + cs[i] * bb;
            }
            const cplx a = h_at(j, j);
            const double rho = std::sqrt(std::norm(a) + hn * hn);
            if (std::abs(a) == 0.0) {
                cs[j] = 0.0;
                sn[j] = 1.0;
            } else {
                cs[j] = std::abs(a) / rho;
                sn[j] = (a / std::abs(a)) * hn / rho;
            }
            h_at(j, j) = cs[j] * a + sn[j] * hn;
            gv[j + 1] = -std::conj(sn[j]) * gv[j];
            gv[j] = cs[j] * gv[j];
            n = j + 1;
            resid = std::abs(gv[j + 1]);
            c->hist_outer.push_back(resid / bnorm);
            if (c->verbose) {
                std::fprintf(stderr, "[ddsolve] FGMRES iteration %d: %d inner iterations (inner tol %.1e), "
                             "residual estimate %.3e\n", o.outer, io.iters, itol, resid / bnorm);
                std::fflush(stderr);
            }
            if (hn == 0.0 || resid / bnorm < tol) break;  // exact in the subspace, or converged
            if ((st = blas(c, mkb(dd::BLAS_AXPBY, {c->fv[j + 1], c->fv[j + 1]}, {0, 0}, {1.0 / hn, 0.0}))) != DD_OK)
                return st;
        }
        // y = R^{-1} g (R: the rotated, upper-triangular H), x += sum_j y_j z_j
        for (int i = n - 1; i >= 0; --i) {
            cplx t = gv[i];
            for (int k = i + 1; k < n; ++k) t -= h_at(i, k) * yv[k];
            if (h_at(i, i) == 0.0 || !is_fin(t)) {
                o.detail = 4;
                return DD_BREAKDOWN;
            }
            yv[i] = t / h_at(i, i);
        }
        dd::VecSet zs{};
        for (int i = 0; i < n; ++i) {
            zs.v[i] = c->fz[i];
            zs.re[i] = yv[i].real();
            zs.im[i] = yv[i].imag();
        }
        hipError_t e = timed(c, DD_KT_BLAS, V * (2 * 192.0 + 96.0 * n), V * 96.0 * n,
                             [&] { return dd::launch_multi_axpy64(g, c->stream, zs, n, x); });
        if (e != hipSuccess) return fail(c, DD_ERR_HIP, std::string("solution update: ") + hipGetErrorString(e));
    }
}

}  // namespace ddh
