// dd_batch.cpp -- batched right-hand sides (one launch of the multi-RHS A for
// all of them, each with its own BiCGStab scalars) and several lattices in one
// work-queue launch: the internals and their C entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>

#include "dd_host.h"

using namespace ddh;

namespace ddh {

dd_status batch_alloc(dd_ctx *c, int n)
{
    if (n <= c->bcap) return DD_OK;
    for (void *p : c->bk)
        if (p) (void)hipFree(p);
    if (c->bfaces) (void)hipFree(c->bfaces);
    c->bfaces = nullptr;
    c->bk.assign(BK_COUNT, nullptr);
    c->bcap = 0;
    if (hipMalloc(&c->bfaces, (size_t)n * dd::sap_face_bytes(c->g)) != hipSuccess) {
        (void)hipGetLastError();
        c->bfaces = nullptr;
        return fail(c, DD_ERR_NOMEM, "batch face terms");
    }
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

// out = A in for n batched fields (internal layout, contiguous) at input precision pin (FP32,
// or FP16 storage), FP32 output; FP32 inputs run the variant v
dd_status mrhs_launch(dd_ctx *c, int v, void *out, const void *in, int n, int pin = DD_F32)
{
    dd::MrhsArgs a{};
    a.in = (const float2 *)in;
    a.in16 = in;
    a.pin = pin;
    a.out = (float2 *)out;
    a.u = (const float2 *)c->U32;
    a.cinv = (const float2 *)c->cinv32;
    a.nrhs = n;
    a.kappa = c->prm.kappa;
    a.phase = c->phase;
    const double V = (double)c->g.V;
    const double bytes = V * (n * (sp_b(pin) + sp_b(DD_F32)) + 4 * lk_b(DD_F32) + cl_b(DD_F32));
    const double flops = V * n * (hops_in(c->g) + hops_out(c->g) + CLOVF);
    hipError_t e = timed(c, DD_KT_DIRAC_MRHS, bytes, flops, [&] { return dd::launch_dirac_mrhs(c->g, c->stream, a, v); });
    if (e != hipSuccess) return fail(c, DD_ERR_HIP, std::string("multi-RHS dirac launch: ") + hipGetErrorString(e));
    return DD_OK;
}

// time every variant that takes inputs of precision pin on this tile (two warm-up
// launches, three timed) and keep the fastest
dd_status mrhs_tune(dd_ctx *c, int n, void *out, const void *in, int pin)
{
    const int nv = dd::mrhs_variant_count();
    const int v0 = pin == DD_F16 ? dd::MRHS_FIRST_VECTOR : 0;  // FP16 inputs: the vector variants
    double *ms_tab = pin == DD_F16 ? c->mrhs_ms16[n] : c->mrhs_ms[n];
    hipEvent_t e0, e1;
    HIPCK(c, hipEventCreate(&e0));
    HIPCK(c, hipEventCreate(&e1));
    const bool timing = c->timing;
    c->timing = false;
    int best = v0;
    for (int v = v0; v < nv; ++v) {
        dd_status st;
        for (int k = 0; k < 2; ++k)
            if ((st = mrhs_launch(c, v, out, in, n, pin)) != DD_OK) return st;
        HIPCK(c, hipEventRecord(e0, c->stream));
        for (int k = 0; k < 3; ++k)
            if ((st = mrhs_launch(c, v, out, in, n, pin)) != DD_OK) return st;
        HIPCK(c, hipEventRecord(e1, c->stream));
        HIPCK(c, hipEventSynchronize(e1));
        float ms = 0;
        HIPCK(c, hipEventElapsedTime(&ms, e0, e1));
        ms_tab[v] = ms / 3.0;
        if (ms_tab[v] < ms_tab[best]) best = v;
    }
    c->timing = timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (pin == DD_F16 ? c->mrhs_tuned16 : c->mrhs_tuned)[n] = best;
    return DD_OK;
}

dd_status k_dirac_mrhs(dd_ctx *c, void *out, const void *in, int n, int pin)
{
    const size_t fb = spinor_bytes(c->g, DD_F32), fi = spinor_bytes(c->g, pin);
    int *tuned = pin == DD_F16 ? c->mrhs_tuned16 : c->mrhs_tuned;
    for (int r0 = 0; r0 < n; r0 += 12) {
        const int m = n - r0 < 12 ? n - r0 : 12;
        void *o = (char *)out + r0 * fb;
        const void *i = (const char *)in + r0 * fi;
        int v = c->mrhs_force;
        if (v >= 0 && pin == DD_F16 && v < dd::MRHS_FIRST_VECTOR) v = -1;  // a forced matrix-core variant: FP32 only
        if (v < 0) {
            if (tuned[m] < 0) {
                dd_status st = mrhs_tune(c, m, o, i, pin);
                if (st != DD_OK) return st;
            }
            v = tuned[m];
        }
        dd_status st = mrhs_launch(c, v, o, i, m, pin);
        if (st != DD_OK) return st;
    }
    return DD_OK;
}



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
        b.stall = Stall{c->prm.stall_window};
        if (!is_fin(red[r])) return fail(c, DD_ERR_NONFINITE, "inner source holds NaN or Inf");
        b.active = red[r] > 0.0;
        nact += b.active;
        if (!b.active) continue;
        for (int k : {BK_R, BK_P, BK_RT})
            if ((st = copy(c, bf(c, k, r), 1, bf(c, BK_SRC, r), 1)) != DD_OK) return st;
        if (sap && (st = copy(c, bf(c, BK_P16, r), 2, bf(c, BK_SRC, r), 1)) != DD_OK) return st;
    }
    const int mp = sap ? BK_MP16 : BK_P, mr = sap ? BK_MR16 : BK_R;
    // M = the FP16-storage SAP of each right-hand side (as in the single right-hand-side
    // mixed solver), reading the FP16 copies of r and p that the updates write and writing
    // FP16 fields that the batched A reads as they are
    // all active right-hand sides in one launch per half-sweep: a block's links and C_inv are
    // staged once for all of them
    auto precond = [&](int from16, int to16) -> dd_status {
        if (!sap) return DD_OK;
        dd::SapRhs rhs{};
        for (int r = 0; r < n; ++r)
            if (R[r].active) rhs.idx[rhs.n++] = r;
        rhs.sp_stride = (long long)spinor_bytes(c->g, DD_F16);
        rhs.face_stride = (long long)dd::sap_face_bytes(c->g);
        return k_sap_batch(c, rhs, bf(c, from16, 0), bf(c, to16, 0), bf(c, BK_S16, 0), c->bfaces);
    };
    // with the SAP, y takes alpha Mp + omega Mr in one pass; a right-hand side that stops
    // between the two half steps gets its alpha Mp here
    auto settle_y = [&](int r, cplx al) -> dd_status {
        if (!sap) return DD_OK;
        return blas(c, mkb(dd::BLAS_CAXPY, {bf(c, BK_Y, r), bf(c, BK_MP16, r)}, {1, 2}, {al.real(), al.imag()}));
    };
    auto stop = [&](BRhs &b, dd_status s2, int detail) {
        b.active = false;
        b.st = s2;
        b.o.detail = detail;
        --nact;
    };
    for (int it = 0; it < maxiter && nact > 0; ++it) {
        if ((st = precond(BK_P16, BK_MP16)) != DD_OK) return st;
        if ((st = k_dirac_mrhs(c, c->bk[BK_Q], c->bk[mp], n, sap ? DD_F16 : DD_F32)) != DD_OK) return st;
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
            if (sap)
                st = reduce_to(c, mkb(dd::BLAS_UPDATE1_H, {bf(c, BK_R, r), bf(c, BK_Q, r), bf(c, BK_R16, r)}, {1, 1, 2},
                                      {alpha[r].real(), alpha[r].imag()}),
                               1, r);
            else
                st = reduce_to(c, mkb(dd::BLAS_UPDATE1, {bf(c, BK_Y, r), bf(c, mp, r), bf(c, BK_R, r), bf(c, BK_Q, r)},
                                      {1, 1, 1}, {alpha[r].real(), alpha[r].imag()}),
                               1, r);
            if (st != DD_OK) return st;
        }
        if ((st = fetch_red(c, n, red)) != DD_OK) return st;
        for (int r = 0; r < n; ++r) {
            BRhs &b = R[r];
            if (!b.active) continue;
            b.rn2 = red[r];
            b.o.relres = std::sqrt(b.rn2 / b.bn2);
            if (b.o.relres < b.tol) {
                if ((st = settle_y(r, alpha[r])) != DD_OK) return st;
                stop(b, DD_OK, 0);
            }
        }
        if (nact == 0) break;
        if ((st = precond(BK_R16, BK_MR16)) != DD_OK) return st;
        if ((st = k_dirac_mrhs(c, c->bk[BK_T], c->bk[mr], n, sap ? DD_F16 : DD_F32)) != DD_OK) return st;
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
                if ((st = settle_y(r, alpha[r])) != DD_OK) return st;
                stop(b, DD_BREAKDOWN, d[2] == 0.0 ? 2 : 4);
                continue;
            }
            omega[r] = cplx(d[0], d[1]) / d[2];
            if (sap)
                st = reduce_to(c, mkb(dd::BLAS_UPDATE2_MM,
                                      {bf(c, BK_Y, r), bf(c, BK_MP16, r), bf(c, BK_MR16, r), bf(c, BK_R, r),
                                       bf(c, BK_T, r), bf(c, BK_RT, r)},
                                      {1, 2, 2, 1, 1, 1},
                                      {alpha[r].real(), alpha[r].imag(), omega[r].real(), omega[r].imag()}),
                               3, 3 * r);
            else
                st = reduce_to(c, mkb(dd::BLAS_UPDATE2,
                                      {bf(c, BK_Y, r), bf(c, mr, r), bf(c, BK_R, r), bf(c, BK_T, r), bf(c, BK_RT, r)},
                                      {1, 1, 1}, {omega[r].real(), omega[r].imag()}),
                               3, 3 * r);
            if (st != DD_OK) return st;
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
            if (b.stall.hit(it + 1, b.o.relres)) {
                stop(b, DD_BREAKDOWN, DETAIL_INNER_STALL);
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
            if (sap)
                st = blas(c, mkb(dd::BLAS_PUPDATE_H, {bf(c, BK_P, r), bf(c, BK_R, r), bf(c, BK_Q, r), bf(c, BK_P16, r)},
                                 {1, 1, 1, 2}, {beta.real(), beta.imag(), omega[r].real(), omega[r].imag()}));
            else
                st = blas(c, mkb(dd::BLAS_PUPDATE, {bf(c, BK_P, r), bf(c, BK_R, r), bf(c, BK_Q, r)}, {1, 1, 1},
                                 {beta.real(), beta.imag(), omega[r].real(), omega[r].imag()}));
            if (st != DD_OK) return st;
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


}  // namespace ddh

namespace {

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

// a reducing vector kernel on lattice k whose nv sums go to that lattice's slots of the
// multi-lattice result array
static dd_status multi_reduce(dd_multi *m, int k, dd::BlasArgs a, int nv)
{
    dd_ctx *c = m->L[k];
    dd_status st = blas(c, a);
    if (st != DD_OK) return lat_fail(m, k, st);
    MHIPCK(m, dd::launch_finalize(m->stream, c->partials, dd::blas_grid(c->g), nv, m->red_all + 3 * k));
    return DD_OK;
}

// bring the first nv results of every lattice's last multi_reduce or multi_blas to the host (one copy,
// one sync)
dd_status multi_fetch(dd_multi *m, int nv, std::vector<std::array<double, 3>> &out)
{
    const size_t n = m->L.size();
    MHIPCK(m, hipMemcpyAsync(m->red_all_host, m->red_all, 3 * n * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    MHIPCK(m, hipStreamSynchronize(m->stream));
    for (size_t k = 0; k < n; ++k)
        for (int v = 0; v < nv; ++v) out[k][v] = m->red_all_host[3 * k + v];
    return DD_OK;
}

// one vector kernel of the lockstep solver on the lattices ks (fields and coefficients from
// mk(k)), in table launches of up to MULTI_BLAS_MAX lattices whose partials fit the first
// lattice's partials array; with nv > 0 each lattice's nv sums are finalised into its slots
// of the result array (multi_fetch brings them over).  Timed on the first lattice's timers.
static dd_status multi_blas(dd_multi *m, int kind, const std::vector<int> &ks,
                            const std::function<dd::BlasArgs(int)> &mk, int nv)
{
    dd_ctx *c0 = m->L[0];
    size_t i = 0;
    while (i < ks.size()) {
        dd::MultiBlasTab t{};
        int slot[dd::MULTI_BLAS_MAX];
        int total = 0;
        long long poff = 0;
        double bytes = 0, flops = 0;
        for (; i < ks.size() && t.n < dd::MULTI_BLAS_MAX; ++i) {
            dd_ctx *c = m->L[ks[i]];
            const int nwg = dd::blas_grid(c->g);
            const long long need = (long long)nwg * (nv > 0 ? nv : 1);
            if (t.n > 0 && poff + need > dd::MAX_PARTIALS) break;
            const dd::BlasArgs a = mk(ks[i]);
            dd::MultiBlasLat &e = t.e[t.n];
            e.g = c->g;
            for (int j = 0; j < 6; ++j) e.v[j] = a.v[j];
            for (int j = 0; j < 4; ++j) e.c[j] = a.c[j];
            e.item0 = total;
            e.nwg = nwg;
            e.poff = poff;
            slot[t.n] = ks[i];
            total += nwg;
            poff += need;
            ++t.n;
            double rw, fl;
            blas_cost(a, rw, fl);
            bytes += rw * (double)c->g.V;
            flops += fl * (double)c->g.V;
        }
        hipError_t e = timed(c0, DD_KT_BLAS, bytes, flops,
                             [&] { return dd::launch_blas_multi(m->stream, kind, t, total, c0->partials); });
        if (e != hipSuccess) return mfail(m, DD_ERR_HIP, std::string("multi-lattice vector kernel: ") + hipGetErrorString(e));
        if (nv > 0) MHIPCK(m, dd::launch_finalize_multi(m->stream, t, slot, c0->partials, nv, m->red_all));
    }
    return DD_OK;
}

// the packed-FP16 SAP of the lattices of every group, one launch per half-sweep and group
// (table v: 0 the SAP of p16 into M p, 1 of r16 into M r)
static dd_status sap_multi(dd_multi *m, int v)
{
    Range range("ddsolve: multi-lattice SAP preconditioner");
    dd_ctx *t0 = m->L[0];  // the first lattice's timers hold the multi-lattice launches
    for (const auto &gr : m->sap_groups) {
        dd_ctx *c0 = m->L[gr.lat[0]];
        const dd::SapLat *tab = m->sap_host + (size_t)v * m->L.size() + gr.off;
        dd_status st = sap_schedule(c0->prm.n_sap, true, false, [&](int colour, int flags) -> dd_status {
            double bytes = 0, flops = 0;
            for (int k : gr.lat) {
                double b, f;
                sap_half_cost(m->L[k]->g, 2, true, flags, 1.0, m->L[k]->prm.n_jac, b, f);
                bytes += b;
                flops += f;
            }
            hipError_t e = timed(t0, DD_KT_SAP, bytes, flops, [&] {
                return dd::launch_sap_half_pk_multi(c0->g, m->stream, tab, (int)gr.lat.size(), colour, flags);
            });
            if (e != hipSuccess)
                return mfail(m, DD_ERR_HIP, std::string("multi-lattice sap launch: ") + hipGetErrorString(e));
            return DD_OK;
        });
        if (st != DD_OK) return st;
    }
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
    std::vector<cplx> alpha(n), omega(n), beta_k(n);
    for (int k = 0; k < n; ++k) {
        dd_ctx *c = m->L[k];
        MHIPCK(m, hipMemsetAsync(F(k, 1), 0, spinor_bytes(c->g, DD_F32), m->stream));
        if ((st = multi_reduce(m, k, mkb(dd::BLAS_NORM2, {F(k, 0)}, {1}), 1)) != DD_OK) return st;
    }
    if ((st = multi_fetch(m, 1, red)) != DD_OK) return st;
    for (int k = 0; k < n; ++k) {
        BRhs &b = R[k];
        b.o = SolveOut{};
        b.bn2 = b.rn2 = red[k][0];
        b.rho0 = red[k][0];
        b.st = DD_OK;
        b.stall = Stall{m->L[k]->prm.stall_window};
        if (!is_fin(red[k][0])) return mfail(m, DD_ERR_NONFINITE, "inner source holds NaN or Inf");
        b.active = red[k][0] > 0.0;
        nact += b.active;
        if (!b.active) continue;
        dd_ctx *c = m->L[k];
        for (int w : {2, 4, 3})
            if ((st = copy(c, F(k, w), 1, F(k, 0), 1)) != DD_OK) return lat_fail(m, k, st);
        if ((st = copy(c, F(k, 10), 2, F(k, 0), 1)) != DD_OK) return lat_fail(m, k, st);
    }
    // the FP16 SAP of each lattice reads the FP16 copies of p and r that the fused updates
    // write (as in solve_sap32); y takes alpha Mp + omega Mr in one pass
    // (one launch per half-sweep for the lattices of the shared SAP, converged ones included)
    std::vector<char> shared(n, 0);
    for (const auto &gr : m->sap_groups)
        for (int k : gr.lat) shared[k] = 1;
    auto precond = [&](int from16, int to) -> dd_status {
        dd_status s2;
        if ((s2 = sap_multi(m, from16 == 10 ? 0 : 1)) != DD_OK) return s2;
        for (int k = 0; k < n; ++k) {
            if (!R[k].active || shared[k]) continue;
            if ((s2 = k_sap(m->L[k], 2, F(k, from16), F(k, to), F(k, 9))) != DD_OK) return lat_fail(m, k, s2);
        }
        return DD_OK;
    };
    auto settle_y = [&](int k) -> dd_status {  // a lattice stopping between the half steps gets its alpha Mp
        return blas(m->L[k], mkb(dd::BLAS_CAXPY, {F(k, 1), F(k, 7)}, {1, 2}, {alpha[k].real(), alpha[k].imag()}));
    };
    auto stop = [&](BRhs &b, dd_status s2, int detail) {
        b.active = false;
        b.st = s2;
        b.o.detail = detail;
        --nact;
    };
    // the active lattices, for the table launches of the vector kernels
    auto active = [&]() {
        std::vector<int> ks;
        for (int k = 0; k < n; ++k)
            if (R[k].active) ks.push_back(k);
        return ks;
    };
    for (int it = 0; it < maxiter && nact > 0; ++it) {
        if ((st = precond(10, 7)) != DD_OK) return st;
        if ((st = multi_launch(m, 1, 2)) != DD_OK) return st;  // q = A M p, every lattice
        if ((st = multi_blas(m, dd::BLAS_DOT, active(), [&](int k) { return mkb(dd::BLAS_DOT, {F(k, 3), F(k, 5)}, {1, 1}); },
                             2)) != DD_OK)
            return st;
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
        }
        if ((st = multi_blas(m, dd::BLAS_UPDATE1_H, active(), [&](int k) {
                 return mkb(dd::BLAS_UPDATE1_H, {F(k, 2), F(k, 5), F(k, 11)}, {1, 1, 2}, {alpha[k].real(), alpha[k].imag()});
             }, 1)) != DD_OK)
            return st;
        if ((st = multi_fetch(m, 1, red)) != DD_OK) return st;
        for (int k = 0; k < n; ++k) {
            BRhs &b = R[k];
            if (!b.active) continue;
            b.rn2 = red[k][0];
            b.o.relres = std::sqrt(b.rn2 / b.bn2);
            if (b.o.relres < b.tol) {
                if ((st = settle_y(k)) != DD_OK) return lat_fail(m, k, st);
                stop(b, DD_OK, 0);
            }
        }
        if (nact == 0) break;
        if ((st = precond(11, 8)) != DD_OK) return st;
        if ((st = multi_launch(m, 2, 2)) != DD_OK) return st;  // t = A M r, every lattice
        if ((st = multi_blas(m, dd::BLAS_DOT_NORM, active(),
                             [&](int k) { return mkb(dd::BLAS_DOT_NORM, {F(k, 6), F(k, 2)}, {1, 1}); }, 3)) != DD_OK)
            return st;
        if ((st = multi_fetch(m, 3, red)) != DD_OK) return st;
        for (int k = 0; k < n; ++k) {
            BRhs &b = R[k];
            if (!b.active) continue;
            const double *d = red[k].data();
            if (d[2] == 0.0 || !is_fin(d[2])) {
                if ((st = settle_y(k)) != DD_OK) return lat_fail(m, k, st);
                stop(b, DD_BREAKDOWN, d[2] == 0.0 ? 2 : 4);
                continue;
            }
            omega[k] = cplx(d[0], d[1]) / d[2];
        }
        if ((st = multi_blas(m, dd::BLAS_UPDATE2_MM, active(), [&](int k) {
                 return mkb(dd::BLAS_UPDATE2_MM, {F(k, 1), F(k, 7), F(k, 8), F(k, 2), F(k, 6), F(k, 3)}, {1, 2, 2, 1, 1, 1},
                            {alpha[k].real(), alpha[k].imag(), omega[k].real(), omega[k].imag()});
             }, 3)) != DD_OK)
            return st;
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
            if (b.stall.hit(it + 1, b.o.relres)) {
                stop(b, DD_BREAKDOWN, DETAIL_INNER_STALL);
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
            beta_k[k] = beta;
        }
        if ((st = multi_blas(m, dd::BLAS_PUPDATE_H, active(), [&](int k) {
                 return mkb(dd::BLAS_PUPDATE_H, {F(k, 4), F(k, 2), F(k, 5), F(k, 10)}, {1, 1, 1, 2},
                            {beta_k[k].real(), beta_k[k].imag(), omega[k].real(), omega[k].imag()});
             }, 0)) != DD_OK)
            return st;
    }
    for (int k = 0; k < n; ++k)
        if (R[k].active) {
            R[k].active = false;
            R[k].st = DD_NOT_CONVERGED;
        }
    return DD_OK;
}



}  // namespace

extern "C" {

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
        if ((st = k_dirac_mrhs(c, c->bk[BK_OUT], c->bk[BK_IN], m, DD_F32)) != DD_OK) return st;
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

dd_status sap_precondition_batch(dd_ctx *c, void *x_dev, const void *b_dev, int nrhs)
{
    if (!c || !x_dev || !b_dev) return fail(c, DD_ERR_ARG, "null argument");
    if (nrhs < 1 || nrhs > BATCH_MAX) return fail(c, DD_ERR_ARG, "nrhs must be 1..16");
    if (!c->gauge) return fail(c, DD_ERR_STATE, "no gauge field loaded");
    dd_status st = batch_alloc(c, nrhs);
    if (st != DD_OK) return st;
    const size_t cb = (size_t)c->g.V * 12 * 16;
    dd::SapRhs rhs{};
    for (int r = 0; r < nrhs; ++r) {
        HIPCK(c, dd::launch_pack_spinor(c->g, c->stream, DD_F16, bf(c, BK_P16, r), (const char *)b_dev + r * cb));
        rhs.idx[rhs.n++] = r;
    }
    rhs.sp_stride = (long long)spinor_bytes(c->g, DD_F16);
    rhs.face_stride = (long long)dd::sap_face_bytes(c->g);
    if ((st = k_sap_batch(c, rhs, bf(c, BK_P16, 0), bf(c, BK_MP16, 0), bf(c, BK_S16, 0), c->bfaces)) != DD_OK)
        return st;
    for (int r = 0; r < nrhs; ++r)
        HIPCK(c, dd::launch_unpack_spinor(c->g, c->stream, DD_F16, (char *)x_dev + r * cb, bf(c, BK_MP16, r)));
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
                inf[r].status_detail = is_fin(rn2[r]) ? DETAIL_OUTER_STALL : 4;
                continue;
            }
            if (R[r].o.detail == DETAIL_INNER_STALL && rn2[r] > 1e-2 * prev[r]) {
                state[r] = 2;
                res[r] = DD_BREAKDOWN;
                inf[r].status_detail = DETAIL_INNER_STALL;
                continue;
            }
            stall[r] = rn2[r] > 0.81 * prev[r] ? stall[r] + 1 : 0;
            prev[r] = rn2[r];
            if (stall[r] >= 2) {
                state[r] = 2;
                res[r] = DD_BREAKDOWN;
                inf[r].status_detail = DETAIL_OUTER_STALL;
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
        inf[r].status = res[r];
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
              hipHostMalloc((void **)&m->desc_host, 3 * nlat * sizeof(dd::LatDesc), hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void **)&m->sap_host, 2 * nlat * sizeof(dd::SapLat), hipHostMallocDefault) == hipSuccess &&
              hipMalloc((void **)&m->red_all, 3 * nlat * sizeof(double)) == hipSuccess &&
              hipHostMalloc((void **)&m->red_all_host, 3 * nlat * sizeof(double), hipHostMallocDefault) == hipSuccess;
    // the groups of lattices whose SAP half-sweeps share one launch (same block shape and
    // n_sap, packed-FP16 arithmetic)
    int off = 0;
    for (int k = 0; k < nlat; ++k) {
        const dd_ctx *c = m->L[k];
        if (!c->prm.sap_fp16_arith) continue;
        dd_multi::SapGroup *grp = nullptr;
        for (auto &gr : m->sap_groups) {
            const dd_ctx *c0 = m->L[gr.lat[0]];
            if (c0->prm.n_sap == c->prm.n_sap && std::equal(c0->g.b, c0->g.b + 4, c->g.b)) grp = &gr;
        }
        if (!grp) {
            m->sap_groups.emplace_back();
            grp = &m->sap_groups.back();
        }
        grp->lat.push_back(k);
        grp->items += dd::sap_multi_items(c->g);
    }
    for (auto &gr : m->sap_groups) {
        gr.off = off;
        off += (int)gr.lat.size();
    }
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
    if (m->sap_host) (void)hipHostFree(m->sap_host);
    if (m->red_all) (void)hipFree(m->red_all);
    if (m->red_all_host) (void)hipHostFree(m->red_all_host);
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
        // the shared SAP launches: p16 -> M p and r16 -> M r, the SAP work vector
        for (int v = 0; v < 2; ++v)
            for (const auto &gr : m->sap_groups) {
                int item0 = 0;
                for (size_t q = 0; q < gr.lat.size(); ++q) {
                    dd_ctx *c = m->L[gr.lat[q]];
                    dd::SapArgs a{};
                    a.b = c->f16[v];
                    a.x = c->f16[2 + v];
                    a.s = c->f16[4];
                    a.prec = 2;
                    a.links = c->U16;
                    a.cinv = c->CPsap;
                    a.n_jac = c->prm.n_jac;
                    a.kappa = c->prm.kappa;
                    a.phase = c->phase;
                    a.faces = c->faces;
                    m->sap_host[v * n + gr.off + q] = dd::sap_lat(c->g, a, item0);
                    item0 += dd::sap_multi_items(c->g);
                }
            }
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
                inf[k].status_detail = is_fin(rn2[k]) ? DETAIL_OUTER_STALL : 4;
                continue;
            }
            if (R[k].o.detail == DETAIL_INNER_STALL && rn2[k] > 1e-2 * prev[k]) {
                state[k] = 2;
                res[k] = DD_BREAKDOWN;
                inf[k].status_detail = DETAIL_INNER_STALL;
                continue;
            }
            stall[k] = rn2[k] > 0.81 * prev[k] ? stall[k] + 1 : 0;
            prev[k] = rn2[k];
            if (stall[k] >= 2) {
                state[k] = 2;
                res[k] = DD_BREAKDOWN;
                inf[k].status_detail = DETAIL_OUTER_STALL;
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
        inf[k].status = res[k];
        if (info) info[k] = inf[k];
    }
    return worst;
}


}  // extern "C"
