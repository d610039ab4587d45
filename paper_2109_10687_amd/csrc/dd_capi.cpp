// dd_capi.cpp -- the core of the C ABI of include/ddsolve.h: context and field
// ownership, gauge loading, the Dirac and SAP entry points, the solve entry
// points (FP64 defect correction, Alg. 4, around the FP32 solvers of
// dd_solvers.cpp with an FP16 SAP; the adjoint solve D^dagger x = b through
// D^dagger = gamma_5 D gamma_5), the fermion force of L = |D^{-1} phi|^2
// (dd_force.hip), and kernel timing.  Batched and multi-lattice entry points
// are in dd_batch.cpp.  Every step of the path runs in the HIP kernels; the
// host code only sequences launches and evaluates the BiCGStab scalars.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "dd_host.h"

using namespace ddh;

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
    if (c->prm.stall_window == 0) c->prm.stall_window = 200;
    if (c->prm.fgmres_nkv <= 0) c->prm.fgmres_nkv = 4;
    if (c->prm.gcr_nkv > dd::GCR_MAX_NKV || c->prm.fgmres_nkv > dd::GCR_MAX_NKV) {
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
    bool ok = alloc(&c->U64, (size_t)V * 36 * 16) && alloc(&c->U32, (size_t)V * 24 * 8) &&
              alloc(&c->U16, (size_t)V * 24 * 4) && alloc(&c->clov64, (size_t)V * 36 * 16) &&
              alloc(&c->cinv32, (size_t)V * 36 * 8) && alloc(&c->cinv16, (size_t)V * 36 * 4) &&
              alloc(&c->CPsap, (size_t)V * 36 * 4) &&
              alloc(&c->faces, dd::sap_face_bytes(g));
    for (int i = 0; ok && i < N64; ++i) ok = alloc(&c->f64[i], spinor_bytes(g, DD_F64));
    for (int i = 0; ok && i < N32; ++i) ok = alloc(&c->f32[i], spinor_bytes(g, DD_F32));
    for (int i = 0; ok && i < N16; ++i) ok = alloc(&c->f16[i], spinor_bytes(g, DD_F16));
    ok = ok && alloc((void **)&c->partials, dd::MAX_PARTIALS * sizeof(double)) &&
         alloc((void **)&c->red, RED_MAX * sizeof(double)) && alloc((void **)&c->flag, 4 * sizeof(int)) &&
         hipHostMalloc((void **)&c->red_host, RED_MAX * sizeof(double), hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        dd_destroy(c);
        return DD_ERR_NOMEM;
    }
    // the device address of dd_force_noalloc's work array on this (the current) device;
    // a failed lookup is reported by that entry point, not here
    c->yscratch_err = dd::force_scratch_address(&c->yscratch);
    if (c->yscratch_err != hipSuccess) c->yscratch = nullptr;
    *out = c;
    return DD_OK;
}

dd_status dd_destroy(dd_ctx *c)
{
    if (!c) return DD_OK;
    (void)hipStreamSynchronize(c->stream);
    void *bufs[] = {c->U64,   c->U32,     c->U16,      c->clov64, c->cinv32, c->cinv16,
                    c->CPsap, c->faces, c->yforce, c->partials, c->red,    c->flag};
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
    for (void *p : c->fv_own)
        if (p) (void)hipFree(p);
    for (void *p : c->fz_own)
        if (p) (void)hipFree(p);
    for (void *p : c->bk)
        if (p) (void)hipFree(p);
    if (c->bfaces) (void)hipFree(c->bfaces);
    if (c->red_host) (void)hipHostFree(c->red_host);
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    delete c;
    return DD_OK;
}

const char *dd_last_error(const dd_ctx *c) { return c ? c->err.c_str() : "null context"; }

dd_status dd_solve_history(dd_ctx *c, int which, double *out, int cap, int *n)
{
    if (!c || !n || (which != 0 && which != 1) || cap < 0 || (cap > 0 && !out))
        return fail(c, DD_ERR_ARG, "bad argument");
    const std::vector<double> &h = which == 0 ? c->hist_outer : c->hist_inner;
    *n = (int)h.size();
    for (int k = 0; k < cap && k < (int)h.size(); ++k) out[k] = h[k];
    return DD_OK;
}

dd_status dd_load_gauge(dd_ctx *c, const void *U)
{
    if (!c || !U) return fail(c, DD_ERR_ARG, "null argument");
    HIPCK(c, hipMemsetAsync(c->flag, 0, 4 * sizeof(int), c->stream));
    HIPCK(c, dd::launch_pack_links(c->g, c->stream, U, c->U64, c->U32, c->U16, c->flag));
    dd::SigmaBlocks sb{};
    if (!sigma_blocks(sb)) return fail(c, DD_ERR_ARG, "sigma blocks not block diagonal");
    HIPCK(c, dd::launch_clover(c->g, c->stream, c->U64, sb, c->prm.kappa * c->prm.csw, c->clov64, c->cinv32,
                               c->cinv16, c->flag + 1));
    HIPCK(c, dd::launch_sap_prep(c->g, c->stream, c->cinv16, c->CPsap));
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

dd_status dirac_apply_packed(dd_ctx *c, void *out, const void *in, dd_prec prec, dd_op op)
{
    if (!c || !out || !in) return fail(c, DD_ERR_ARG, "null argument");
    dd_status st = check_op(c, prec, op);
    if (st != DD_OK) return st;
    return k_dirac(c, out, in, prec, prec, prec, op);
}

dd_status dirac_apply_packed_f16in(dd_ctx *c, void *out, const void *in)
{
    if (!c || !out || !in) return fail(c, DD_ERR_ARG, "null argument");
    if (!c->gauge) return fail(c, DD_ERR_STATE, "no gauge field loaded");
    return k_dirac(c, out, in, DD_F16, DD_F32, DD_F32, DD_OP_A);
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

dd_status sap_precondition_amsap(dd_ctx *c, void *ax, const void *b, dd_prec prec)
{
    if (!c || !ax || !b) return fail(c, DD_ERR_ARG, "null argument");
    if (!c->gauge) return fail(c, DD_ERR_STATE, "no gauge field loaded");
    if (prec != DD_F32 && prec != DD_F16) return fail(c, DD_ERR_ARG, "A M_SAP is available at FP32 and FP16");
    void *tb = c->f64[5], *tx = c->f64[6], *ts = c->f64[4], *tax = c->f64[3];
    HIPCK(c, dd::launch_pack_spinor(c->g, c->stream, prec, tb, b));
    dd_status st;
    if (prec == DD_F32) {
        if ((st = k_sap(c, 1, tb, tx, ts, tax)) != DD_OK) return st;
    } else {
        if ((st = k_sap(c, 2, tb, tx, ts)) != DD_OK) return st;
        if ((st = k_dirac(c, tax, tx, DD_F16, DD_F32, DD_F32, DD_OP_A)) != DD_OK) return st;
    }
    HIPCK(c, dd::launch_unpack_spinor(c->g, c->stream, DD_F32, ax, tax));
    return DD_OK;
}

// D x = b, or D^dagger x = b when dagger is set: D^dagger = gamma_5 D gamma_5, so
// y = gamma_5 x solves D y = gamma_5 b; the gamma_5 is applied while packing b
// and x and while unpacking the result
static dd_status solve_entry(dd_ctx *c, void *x_dev, const void *b_dev, double tol, int maxiter, dd_solve_mode mode,
                             dd_solve_info *info, bool dagger)
{
    if (!c || !x_dev || !b_dev) return fail(c, DD_ERR_ARG, "null argument");
    if (!(tol > 0) || maxiter < 0 || mode < DD_SOLVE_F64_PLAIN || mode > DD_SOLVE_FGMRES)
        return fail(c, DD_ERR_ARG, "bad tolerance, maxiter or mode");
    if (!c->gauge) return fail(c, DD_ERR_STATE, "no gauge field loaded");
    Range range(dagger ? "ddsolve: adjoint solve" : "ddsolve: solve");
    auto t0 = std::chrono::steady_clock::now();
    dd_solve_info inf{};
    c->hist_outer.clear();
    c->hist_inner.clear();
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
    } else if (mode == DD_SOLVE_FGMRES) {
        if ((st = ensure_fgmres(c)) != DD_OK) return st;
        HIPCK(c, dd::launch_pack_spinor(c->g, c->stream, DD_F64, x, x_dev, dagger));
        if (bn2 == 0.0) HIPCK(c, hipMemsetAsync(x, 0, spinor_bytes(c->g, DD_F64), c->stream));
        OuterOut o;
        res = bn2 == 0.0 ? DD_OK : solve_fgmres64(c, x, b, bn2, tol, maxiter, o);
        if (res < 0) return res;
        inf.iters_outer = o.outer;
        inf.iters_inner_total = o.inner;
        inf.relres_inner_last = o.inner_last;
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
        if (mode == DD_SOLVE_MIXED_GCR && (st = ensure_gcr(c)) != DD_OK) return st;
        HIPCK(c, dd::launch_pack_spinor(c->g, c->stream, DD_F64, x, x_dev, dagger));
        void *r = c->f64[2], *tmp = c->f64[3];
        void *src = c->f32[0], *y = c->f32[1];
        double rn2;
        if ((st = residual64(c, r, b, x, tmp, &rn2)) != DD_OK) return st;
        if (bn2 > 0) c->hist_outer.push_back(std::sqrt(rn2 / bn2));
        double prev = rn2;
        int stall = 0, outer = 0;
        // 0: the mode's own inner solver (FP16 SAP), 1: FP32 SAP-BiCGStab, 2: plain FP64 BiCGStab
        int level = 0;
        bool restarted = false;  // this level has had its one restart after a broken-down pass
        // a stagnating pass or a broken-down inner solve: fall back one level, or stop
        auto give_up = [&](int detail) -> bool {
            if (c->prm.no_fallback || level == 2) {
                inf.status_detail = detail;
                res = DD_BREAKDOWN;
                return true;
            }
            ++level;
            stall = 0;
            restarted = false;
            if (c->verbose) {
                std::fprintf(stderr, "[ddsolve] falling back to %s after outer pass %d\n",
                             level == 1 ? "FP32 SAP-BiCGStab" : "plain FP64 BiCGStab", outer);
                std::fflush(stderr);
            }
            return false;
        };
        res = DD_NOT_CONVERGED;
        if (bn2 == 0.0) HIPCK(c, hipMemsetAsync(x, 0, spinor_bytes(c->g, DD_F64), c->stream));
        while (true) {
            if (bn2 == 0.0 || std::sqrt(rn2 / bn2) < tol) {
                res = DD_OK;
                break;
            }
            if (outer >= maxiter) break;
            if (level == 2) {
                // the last level: plain FP64 BiCGStab on D x = b from the current x
                SolveOut o;
                Range pass("ddsolve: FP64 fallback solve");
                dd_status sp = solve_plain64(c, x, b, tol, c->prm.inner_maxiter, o);
                if (sp < 0) return sp;
                ++outer;
                inf.iters_inner_total += o.iters;
                inf.relres_inner_last = o.relres;
                const double before = rn2;
                if ((st = residual64(c, r, b, x, tmp, &rn2)) != DD_OK) return st;
                c->hist_outer.push_back(std::sqrt(rn2 / bn2));
                if (sp == DD_BREAKDOWN && !restarted && rn2 <= 1e-2 * before) {
                    restarted = true;  // broke down after a 10x gain: restart once from the new x
                    continue;
                }
                if (sp != DD_OK || std::sqrt(rn2 / bn2) >= tol) {
                    res = sp == DD_OK ? DD_NOT_CONVERGED : sp;
                    inf.status_detail = o.detail;
                    break;
                }
                continue;
            }
            double err = std::sqrt(rn2);
            if ((st = blas(c, mkb(dd::BLAS_CINV_SRC, {src, r, c->cinv32}, {1, 0}, {1.0 / err}))) != DD_OK) return st;
            // each pass reduces the residual by inner_tol, except that the last
            // pass stops once the outer target is met (with a factor 2 margin)
            const double need = 0.5 * tol * std::sqrt(bn2) / err;
            const double itol = need > c->prm.inner_tol ? (need < 0.1 ? need : 0.1) : c->prm.inner_tol;
            SolveOut o;
            Range pass("ddsolve: defect-correction pass");
            dd_status si = level == 1                    ? solve_sap32(c, 1, src, y, itol, c->prm.inner_maxiter, o)
                           : mode == DD_SOLVE_MIXED_GCR ? solve_gcr32(c, src, y, itol, c->prm.inner_maxiter, o)
                                                        : solve_sap32(c, 2, src, y, itol, c->prm.inner_maxiter, o);
            if (si < 0) return si;
            inf.iters_inner_total += o.iters;
            inf.relres_inner_last = o.relres;
            if ((st = blas(c, mkb(dd::BLAS_AXPBY, {y, x}, {1, 0}, {err, 1.0}))) != DD_OK) return st;
            if ((st = residual64(c, r, b, x, tmp, &rn2)) != DD_OK) return st;
            ++outer;
            if (!is_fin(rn2) || rn2 >= prev) {
                // the correction made the true residual worse (inner solve failed):
                // take it back, so x stays the best iterate
                if ((st = blas(c, mkb(dd::BLAS_AXPBY, {y, x}, {1, 0}, {-err, 1.0}))) != DD_OK) return st;
                if ((st = residual64(c, r, b, x, tmp, &rn2)) != DD_OK) return st;
                if (give_up(is_fin(rn2) ? DETAIL_OUTER_STALL : 4)) break;
                continue;
            }
            c->hist_outer.push_back(std::sqrt(rn2 / bn2));
            if (c->verbose) {
                std::fprintf(stderr, "[ddsolve] outer pass %d: %d inner iterations (inner tol %.1e, reached %.2e), "
                             "true residual %.3e\n", outer, o.iters, itol, o.relres, std::sqrt(rn2 / bn2));
                std::fflush(stderr);
            }
            if (si == DD_BREAKDOWN && std::sqrt(rn2 / bn2) >= tol) {
                // the inner solve broke down or stagnated (its stall window).  The first time
                // at a level, a pass that still gained 10x is followed by a pass of the same
                // inner solver (restarted, with a fresh shadow residual, as after any pass);
                // otherwise the next passes run one level up.  Without the fallback, a
                // stagnated pass that gained less than 10x ends the solve (further passes
                // would crawl at that rate)
                const bool gained = rn2 <= 1e-2 * prev;
                if (!c->prm.no_fallback && level < 2) {
                    if (gained && !restarted) {
                        restarted = true;
                    } else {
                        prev = rn2;
                        give_up(o.detail);
                        continue;
                    }
                } else if (o.detail == DETAIL_INNER_STALL && !gained) {
                    inf.status_detail = DETAIL_INNER_STALL;
                    res = DD_BREAKDOWN;
                    break;
                }
            }
            stall = rn2 > 0.81 * prev ? stall + 1 : 0;  // |r| fell by less than 10%
            prev = rn2;
            if (stall >= 2 && give_up(DETAIL_OUTER_STALL)) break;
        }
        inf.iters_outer = outer;
        inf.precision_level = level;
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
    inf.status = res;
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

// the force of dd_force and dd_force_noalloc with the work field y (54 complex doubles
// per site); timed = false launches without the kernel timers (whose event pool may grow)
static dd_status force_entry(dd_ctx *c, void *out_dev, double *dcsw, const void *psi_dev, const void *chi_dev,
                             int su3, void *y, bool timed_launch)
{
    const Geom &g = c->g;
    dd::ForceArgs a{};
    a.psi = c->f64[0];
    a.chi = c->f64[1];
    HIPCK(c, dd::launch_pack_spinor(g, c->stream, DD_F64, c->f64[0], psi_dev));
    HIPCK(c, dd::launch_pack_spinor(g, c->stream, DD_F64, c->f64[1], chi_dev));
    a.u64 = c->U64;
    a.y = y;
    a.out = out_dev;
    a.partials = dcsw ? c->partials : nullptr;
    a.dcsw = c->red;
    if (!sigma_blocks(a.sig)) return fail(c, DD_ERR_ARG, "sigma blocks not block diagonal");
    a.kcsw = c->prm.kappa * c->prm.csw;
    a.kappa = c->prm.kappa;
    a.csw = c->prm.csw;
    a.clov64 = c->clov64;
    a.phase = c->phase;
    a.su3 = su3;
    // per site: psi, chi, four links and the six Y planes read twice over (once
    // written), the output links written; flops of the hop outer products, the
    // 24 leaves per link (nine 3x3 products per plaquette) and the dcsw traces
    const double V = (double)g.V;
    const bool csw_from_clover = c->prm.csw != 0.0;
    const double bytes = V * (2 * 192.0 + 4 * 144.0 + 2 * 864.0 + 4 * 144.0 +
                              (dcsw ? (csw_from_clover ? 576.0 : 4 * 144.0) : 0.0));
    const double flops = V * (4 * FORCE_LINK_FLOPS + FORCE_Y_FLOPS +
                              (dcsw ? (csw_from_clover ? FORCE_DCSW_CLOVER_FLOPS : FORCE_DCSW_FLOPS) : 0.0));
    hipError_t e = timed_launch ? timed(c, DD_KT_FORCE, bytes, flops, [&] { return dd::launch_force(g, c->stream, a); })
                                : dd::launch_force(g, c->stream, a);
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

dd_status dd_force(dd_ctx *c, void *out_dev, double *dcsw, const void *psi_dev, const void *chi_dev, int su3)
{
    if (!c || !out_dev || !psi_dev || !chi_dev) return fail(c, DD_ERR_ARG, "null argument");
    if (su3 != 0 && su3 != 1) return fail(c, DD_ERR_ARG, "su3 must be 0 or 1");
    if (!c->gauge) return fail(c, DD_ERR_STATE, "no gauge field loaded");
    if (!c->yforce && hipMalloc(&c->yforce, (size_t)c->g.V * 54 * 16) != hipSuccess) {
        (void)hipGetLastError();
        c->yforce = nullptr;
        return fail(c, DD_ERR_NOMEM, "force work field");
    }
    return force_entry(c, out_dev, dcsw, psi_dev, chi_dev, su3, c->yforce, true);
}

dd_status dd_force_noalloc(dd_ctx *c, void *out_dev, double *dcsw, const void *psi_dev, const void *chi_dev, int su3)
{
    if (!c || !out_dev || !psi_dev || !chi_dev) return fail(c, DD_ERR_ARG, "null argument");
    if (su3 != 0 && su3 != 1) return fail(c, DD_ERR_ARG, "su3 must be 0 or 1");
    if (!c->gauge) return fail(c, DD_ERR_STATE, "no gauge field loaded");
    const size_t need = (size_t)c->g.V * 54 * 16;
    if (need > dd::FORCE_SCRATCH_BYTES)
        return fail(c, DD_ERR_ARG, "lattice too large for dd_force_noalloc: " + std::to_string(c->g.V) +
                                       " sites need " + std::to_string(need) + " bytes of work space, the fixed "
                                       "array holds " + std::to_string(dd::FORCE_SCRATCH_BYTES) + " (at most " +
                                       std::to_string(dd::FORCE_SCRATCH_BYTES / (54 * 16)) + " sites)");
    if (!c->yscratch)
        return fail(c, DD_ERR_HIP, std::string("work array address: ") + hipGetErrorString(c->yscratch_err));
    return force_entry(c, out_dev, dcsw, psi_dev, chi_dev, su3, c->yscratch, false);
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
