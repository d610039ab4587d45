// dd_ops.cpp -- launches of the single-field kernels with their algorithmic
// byte and flop counts (kernel timing), the vector kernels and reductions, and
// the sigma blocks of the clover setup.
#include <functional>

#include "dd_host.h"

using namespace ddh;

namespace {

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

}  // namespace

namespace ddh {

dd_status fail(dd_ctx *c, dd_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

dd_status mfail(dd_multi *m, dd_status s, const std::string &msg)
{
    if (m) m->err = msg;
    return s;
}

hipEvent_t take_event(dd_ctx *c)
{
    if (c->pool_used == c->pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->pool.push_back(e);
    }
    return c->pool[c->pool_used++];
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

// x = M_SAP b at storage precision prec (1 FP32, 2 FP16), work vector s; rhs.n > 0 sweeps the
// listed right-hand sides of a batch in each launch (packed FP16 only), faces: their face terms
// algorithmic bytes and counted flops per swept site of one half-sweep with these flags
// (nr right-hand sides), for the kernel timers
void sap_half_cost(const Geom &g, int prec, bool pk, int flags, double nr, int n_jac, double &bytes, double &flops)
{
    // per site of the swept colour: source (s, or b in the first), links, C_inv; without
    // TAIL also b read and s written.  FP32 arithmetic: x written, and with PRE the
    // neighbour-block face spinors and the links that point into the block from outside.
    // Packed FP16: x written by the tails only; with PRE the face hop terms read (6 half2
    // per face site, the neighbour block's scale), with FACES_OUT this block's written
    const bool tail = flags & dd::SAP_TAIL, pre = flags & dd::SAP_PRE, first = flags & dd::SAP_FIRST;
    double face_sp = 0, face_lk = 0;
    for (int mu = 0; mu < 4; ++mu) {
        face_sp += 2.0 / g.b[mu];
        face_lk += 1.0 / g.b[mu];
    }
    const double stat = 4 * lk_b(prec) + cl_b(prec);  // links and C_inv, once for all right-hand sides
    double per = sp_b(prec);
    if (!tail) per += (first ? 0.0 : sp_b(prec)) + sp_b(prec);
    if (!pk || tail) per += sp_b(prec);
    if (pk) {
        const double term = 6 * 4.0 + 4.0 / g.bvol;
        if (pre) per += face_sp * term;
        if (flags & dd::SAP_FACES_OUT) per += face_sp * term;
    } else if (pre) {
        per += face_sp * sp_b(prec) + face_lk * lk_b(prec);
    }
    double fl = n_jac * (hops_in(g) + CLOVF);
    if (!tail) fl += hops_in(g) + CLOVF + 48;
    if (pre) fl += hops_out(g) + CLOVF;
    if (flags & dd::SAP_AMSAP) {  // Alg. 3: one more in-block sweep, ax written
        per += sp_b(prec);
        fl += hops_in(g) + CLOVF + 48;
        if (flags & dd::SAP_AMSAP_PRE) {  // and the cross-block hops formed again
            per += face_sp * sp_b(prec) + face_lk * lk_b(prec);
            fl += hops_out(g);
        }
    }
    if (flags & dd::SAP_CROSS_ONLY) {  // the cross-block hops of the final x into ax (read, written)
        per = face_sp * sp_b(prec) + face_lk * lk_b(prec) + 2 * sp_b(prec);
        fl = hops_out(g) + CLOVF + 24;
    }
    const double sites = 0.5 * (double)g.V;
    bytes = sites * (nr * per + stat);
    flops = sites * nr * fl;
}

// The half-sweeps of one application of Alg. 1 (loop count n_sap) in order: half(colour,
// flags).  The packed-FP16 half-sweeps (pk) hand the cross-block term on as face hop terms:
// every half-sweep but the last leaves them.  With amsap, the fused tail of Alg. 3: the
// tails also write their rows of A x, and one more launch adds the even rows' cross-block
// term of the final odd x.
dd_status sap_schedule(int n_sap, bool pk, bool amsap, const std::function<dd_status(int, int)> &half)
{
    const int E = 0, O = 1;
    const int out = pk ? dd::SAP_FACES_OUT : 0;
    dd_status st;
    for (int i = 0; i < n_sap; ++i) {
        if ((st = half(E, (i == 0 ? dd::SAP_FIRST : dd::SAP_PRE) | out)) != DD_OK) return st;
        if ((st = half(O, (i == 0 ? (dd::SAP_FIRST | dd::SAP_PRE) : dd::SAP_PRE) | out)) != DD_OK) return st;
    }
    const int am = amsap ? dd::SAP_AMSAP : 0;
    if ((st = half(E, dd::SAP_TAIL | (n_sap == 0 ? dd::SAP_FIRST : dd::SAP_PRE) | out | am)) != DD_OK) return st;
    if ((st = half(O, dd::SAP_TAIL | dd::SAP_PRE | (n_sap == 0 ? dd::SAP_FIRST : 0) | am |
                          (amsap ? dd::SAP_AMSAP_PRE : 0))) != DD_OK)
        return st;
    if (amsap && (st = half(E, dd::SAP_CROSS_ONLY)) != DD_OK) return st;
    return DD_OK;
}

static dd_status sap_sweeps(dd_ctx *c, int prec, const void *b, void *x, void *s, void *faces,
                            const dd::SapRhs &rhs, void *ax = nullptr)
{
    Range range("ddsolve: SAP preconditioner");
    dd::SapArgs a{};
    a.rhs = rhs;
    a.ax = ax;
    a.b = b;
    a.s = s;
    a.x = x;
    a.prec = prec;
    const bool pk = prec == 2 && c->prm.sap_fp16_arith;
    a.links = prec == 1 ? c->U32 : c->U16;
    a.cinv = prec == 1 ? c->cinv32 : pk ? c->CPsap : c->cinv16;
    a.n_jac = c->prm.n_jac;
    a.kappa = c->prm.kappa;
    a.phase = c->phase;
    a.faces = faces;
    const double nr = rhs.n > 0 ? rhs.n : 1;  // right-hand sides per launch
    return sap_schedule(c->prm.n_sap, pk, ax != nullptr, [&](int colour, int flags) -> dd_status {
        double bytes, flops;
        sap_half_cost(c->g, prec, pk, flags, nr, c->prm.n_jac, bytes, flops);
        hipError_t e = timed(c, DD_KT_SAP, bytes, flops, [&] {
            return pk ? dd::launch_sap_half_pk(c->g, c->stream, a, colour, flags)
                      : dd::launch_sap_half(c->g, c->stream, a, colour, flags);
        });
        if (e != hipSuccess) return fail(c, DD_ERR_HIP, std::string("sap launch: ") + hipGetErrorString(e));
        return DD_OK;
    });
}

dd_status k_sap(dd_ctx *c, int prec, const void *b, void *x, void *s, void *ax)
{
    if (ax && prec != 1)
        return fail(c, DD_ERR_ARG, "the fused A M_SAP is available with FP32 storage");
    return sap_sweeps(c, prec, b, x, s, c->faces, dd::SapRhs{}, ax);
}

dd_status k_sap_batch(dd_ctx *c, const dd::SapRhs &rhs, const void *b, void *x, void *s, void *faces)
{
    if (rhs.n <= 0) return DD_OK;
    if (c->prm.sap_fp16_arith) return sap_sweeps(c, 2, b, x, s, faces, rhs);
    // FP32 arithmetic on FP16 storage: one SAP per right-hand side
    for (int k = 0; k < rhs.n; ++k) {
        const long long o = rhs.idx[k] * rhs.sp_stride;
        dd_status st = sap_sweeps(c, 2, (const char *)b + o, (char *)x + o, (char *)s + o, c->faces, dd::SapRhs{});
        if (st != DD_OK) return st;
    }
    return DD_OK;
}

// bytes read + written per site, and flops per site, of a vector kernel
void blas_cost(const dd::BlasArgs &a, double &rw, double &fl)
{
    rw = 0;
    fl = 0;
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
    case dd::BLAS_UPDATE1_H: rw = 3 * sp_b(1) + sp_b(2); fl = 144; break;                 // r r/w, q, r16 written
    case dd::BLAS_UPDATE2_MM: rw = 4 * sp_b(1) + 2 * P1 + 2 * sp_b(1); fl = 432; break;  // y, r r/w; Mp, Mr; t, rt
    case dd::BLAS_PUPDATE_H: rw = 4 * sp_b(1) + sp_b(2); fl = 192; break;                 // p r/w, r, q, p16 written
    case dd::BLAS_CAXPY: rw = 2 * sp_b(1) + P1; fl = 96; break;
    }
}

dd_status blas(dd_ctx *c, dd::BlasArgs a)
{
    a.partials = c->partials;
    double rw, fl;
    blas_cost(a, rw, fl);
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
                 std::initializer_list<double> cc)
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


// r = b - D x (FP64) ; returns |r|^2
dd_status residual64(dd_ctx *c, void *r, void *b, void *x, void *tmp, double *rn2)
{
    Range range("ddsolve: FP64 residual");
    dd_status st = k_dirac(c, tmp, x, 0, 0, 0, 0);
    if (st != DD_OK) return st;
    return reduce(c, mkb(dd::BLAS_SUB_NORM, {r, b, tmp}, {0, 0, 0}), 1, rn2);
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

dd_status check_op(dd_ctx *c, dd_prec prec, dd_op op)
{
    if (!c->gauge) return fail(c, DD_ERR_STATE, "no gauge field loaded");
    if (op == DD_OP_A && (prec == DD_F32 || prec == DD_F16)) return DD_OK;
    if ((op == DD_OP_D || op == DD_OP_DDAG) && prec == DD_F64) return DD_OK;
    return fail(c, DD_ERR_ARG, "operator not available at this precision (D, D^dagger: FP64; A: FP32, FP16)");
}

}  // namespace ddh
