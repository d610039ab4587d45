// dd_host.h -- host-side state and helpers shared by the C ABI's translation
// units: the context and multi-lattice handles, kernel timing, the per-site
// byte and flop counts of each launch, and the launch, vector-kernel and solver
// helpers (dd_ops.cpp, dd_solvers.cpp, dd_batch.cpp).  Internal to the library.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <complex>
#include <functional>
#include <initializer_list>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/ddsolve.h"
#include "dd_launch.h"

namespace ddh {

// a roctx range around a solver phase (seen by rocprofv3 --marker-trace; free otherwise)
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

using dd::Geom;
using cplx = std::complex<double>;

constexpr int N64 = 7, N32 = 10, N16 = 5;
constexpr int RED_MAX = 64;  // longest reduction result (doubles): GCR cycle, or 3 per batched right-hand side
constexpr int BATCH_MAX = 16;  // right-hand sides of one batched solve

struct TimerRec {
    int cls;
    hipEvent_t a, b;
    double bytes, flops;
};

}  // namespace ddh

struct dd_ctx {
    dd_params prm{};
    dd::Geom g{};
    hipStream_t stream = nullptr;
    std::string err;
    bool gauge = false;
    int verbose = 0;  // DD_VERBOSE=1: one progress line per outer pass and per 100 inner iterations
    dd::Phase4 phase{};
    // packed gauge fields
    void *U64 = nullptr, *U32 = nullptr, *U16 = nullptr;
    void *clov64 = nullptr, *cinv32 = nullptr, *cinv16 = nullptr;
    void *CPsap = nullptr;  // SAP-ready FP16 C_inv (launch_sap_prep)
    void *faces = nullptr;  // face hop terms of the packed-FP16 SAP half-sweeps
    void *yforce = nullptr;  // force work field (54 complex per site), allocated by the first dd_force
    void *yscratch = nullptr;       // the fixed device array that dd_force_noalloc uses instead
    hipError_t yscratch_err = hipSuccess;  // the result of looking its address up in dd_create
    // batched right-hand sides: contiguous arrays of per-RHS internal fields, allocated by the
    // first batched call and grown on demand (kinds: see BK_* below)
    int bcap = 0;
    std::vector<void *> bk;
    void *bfaces = nullptr;  // the packed-FP16 SAP's face terms, one set per right-hand side
    int mrhs_force = -1;                // multi-RHS kernel variant forced by the caller (-1: autotune)
    int mrhs_tuned[13] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};  // per right-hand sides in a tile
    double mrhs_ms[13][16] = {};         // autotuner timings (ms per launch) per variant
    // the same for FP16-storage inputs (the SAP-preconditioned batched solve), where only the
    // vector variants apply
    int mrhs_tuned16[13] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
    double mrhs_ms16[13][16] = {};
    // work vectors
    void *f64[ddh::N64] = {}, *f32[ddh::N32] = {}, *f16[ddh::N16] = {};
    void *gz[dd::GCR_MAX_NKV] = {}, *gp[dd::GCR_MAX_NKV] = {};  // GCR images (FP32), directions (FP16)
    // flexible GMRES basis (FP64) and directions (FP32): the first ones alias work vectors the
    // inner solve never touches, the rest are allocated by the first such solve (fv_own, fz_own)
    void *fv[dd::GCR_MAX_NKV + 1] = {}, *fz[dd::GCR_MAX_NKV] = {};
    void *fv_own[dd::GCR_MAX_NKV + 1] = {}, *fz_own[dd::GCR_MAX_NKV] = {};
    double *partials = nullptr, *red = nullptr, *red_host = nullptr;
    int *flag = nullptr;
    // kernel timing
    bool timing = false;
    std::vector<ddh::TimerRec> recs;
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
    long long launches[DD_KT_COUNT] = {};
    double ms[DD_KT_COUNT] = {}, bytes[DD_KT_COUNT] = {}, flops[DD_KT_COUNT] = {};
    // residual history of the last single-field solve: true FP64 residual per outer pass,
    // recursive inner residual per inner iteration
    std::vector<double> hist_outer, hist_inner;
};

struct dd_multi {
    std::vector<dd_ctx *> L;
    hipStream_t stream = nullptr;
    std::string err;
    int *counter = nullptr;                      // work-queue head of the multi-lattice launch
    dd::LatDesc *desc_dev = nullptr;             // three descriptor tables: the caller's apply, A Mp, A Mr
    dd::LatDesc *desc_host = nullptr;            // pinned staging for the caller's apply
    int total = 0;                               // work items (256-site chunks) over all lattices
    // the multi-lattice packed-FP16 SAP: lattices with the same block shape and n_sap (and
    // packed-FP16 arithmetic) share one launch per half-sweep; two tables of nlat entries (the
    // SAP of p and of r in the inner solve), each group's lattices consecutive in them
    struct SapGroup {
        std::vector<int> lat;  // lattice indices
        int items = 0;         // work items of a launch
        int off = 0;           // first table entry
    };
    dd::SapLat *sap_host = nullptr;  // the multi-lattice half-sweep tables (kernel arguments)
    std::vector<SapGroup> sap_groups;
    double *red_all = nullptr, *red_all_host = nullptr;  // three reduction results per lattice
};

namespace ddh {

// record msg on the context (if any) and return s
dd_status fail(dd_ctx *c, dd_status s, const std::string &msg);
dd_status mfail(dd_multi *m, dd_status s, const std::string &msg);

#define HIPCK(c, call)                                                                                   \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess) return fail((c), DD_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define MHIPCK(m, call)                                                                                   \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess) return mfail((m), DD_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

hipEvent_t take_event(dd_ctx *c);

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

// fold the recorded launch timings into the per-class totals
hipError_t flush_timing(dd_ctx *c);

inline bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
inline int ilog2(int v)
{
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

inline size_t spinor_bytes(const Geom &g, int prec)
{
    if (prec == DD_F64) return (size_t)g.V * 12 * 16;
    if (prec == DD_F32) return (size_t)g.V * 12 * 8;
    return (size_t)g.V * (12 * 4 + 4);
}

// ---- algorithmic bytes and flops per site (each field read or written once)
inline double sp_b(int prec) { return prec == 0 ? 192.0 : prec == 1 ? 96.0 : 52.0; }   // spinor (+ FP16 scale)
inline double lk_b(int prec) { return prec == 0 ? 144.0 : prec == 1 ? 48.0 : 24.0; }    // one link (FP32, FP16: 12 reals)
inline double cl_b(int prec) { return prec == 0 ? 576.0 : prec == 1 ? 288.0 : 144.0; }  // clover / C_inv block pair
constexpr double HOPF[4] = {168, 168, 168, 156};                                            // flops of one hop per direction
constexpr double CLOVF = 600;                                                      // clover multiply + combine
// fermion force, counted flops (complex multiply 6, add 2; a 3x3 product 198, C += A B 216):
// per link 6 plaquettes x (4 products + 4 accumulated products) + the hop term (four spin
// projections of 12 flops and two 9-entry traces over two spins, 22 flops an entry); per site
// the Y planes 6 x 400 and, for dL/dc_SW, either the six field strengths and traces 6 x 2500
// (c_SW = 0) or the clover product, 12 complex differences and 12 real parts of conjugate
// products summed (600 + 24 + 48)
constexpr double FORCE_LINK_FLOPS = 6 * (4 * 198.0 + 4 * 216.0) + (4 * 12.0 + 2 * 9 * 22.0);
constexpr double FORCE_Y_FLOPS = 6 * 400.0, FORCE_DCSW_FLOPS = 6 * 2500.0;
constexpr double FORCE_DCSW_CLOVER_FLOPS = 600.0 + 24.0 + 48.0;

// hop flops per site that stay inside a block, and those that leave it
inline double hops_in(const Geom &g)
{
    double f = 0;
    for (int mu = 0; mu < 4; ++mu) f += 2.0 * (g.b[mu] - 1) / g.b[mu] * HOPF[mu];
    return f;
}
inline double hops_out(const Geom &g)
{
    double f = 0;
    for (int mu = 0; mu < 4; ++mu) f += 2.0 / g.b[mu] * HOPF[mu];
    return f;
}

inline bool is_fin(double v) { return std::isfinite(v); }
inline bool is_fin(cplx v) { return std::isfinite(v.real()) && std::isfinite(v.imag()); }

// ---- dd_ops.cpp: launches of the single-field kernels and the reductions

// sigma_mu_nu in the chiral basis (the clover's 2x2 spin blocks); false if not block diagonal
bool sigma_blocks(dd::SigmaBlocks &sb);
// operator op at input / output / gauge precisions pin, pout, pg (0 FP64, 1 FP32, 2 FP16)
dd_status k_dirac(dd_ctx *c, void *out, const void *in, int pin, int pout, int pg, int op);
// x = M_SAP b at storage precision prec (1 FP32, 2 FP16), work vector s; with ax (FP32 only)
// also ax = A M_SAP b by the fused tail of Alg. 3
dd_status k_sap(dd_ctx *c, int prec, const void *b, void *x, void *s, void *ax = nullptr);
// the half-sweeps of one SAP application in order, and the timer figures of one of them
dd_status sap_schedule(int n_sap, bool pk, bool amsap, const std::function<dd_status(int, int)> &half);
void sap_half_cost(const Geom &g, int prec, bool pk, int flags, double nr, int n_jac, double &bytes, double &flops);
// the same for the right-hand sides rhs.idx[0 .. n) of a batch of FP16 fields (the packed-FP16
// SAP: one launch per half-sweep for all of them; otherwise one SAP per right-hand side):
// field r of b, x and s at byte offset r * spinor_bytes(FP16), face terms per right-hand side
dd_status k_sap_batch(dd_ctx *c, const dd::SapRhs &rhs, const void *b, void *x, void *s, void *faces);
dd_status blas(dd_ctx *c, dd::BlasArgs a);
// run a reducing vector kernel and bring its nv sums to the host
dd_status reduce(dd_ctx *c, dd::BlasArgs a, int nv, double *out);
void blas_cost(const dd::BlasArgs &a, double &rw, double &fl);
dd::BlasArgs mkb(int kind, std::initializer_list<void *> v, std::initializer_list<int> p,
                 std::initializer_list<double> cc = {});
dd_status norm2(dd_ctx *c, void *v, int prec, double *out);
dd_status copy(dd_ctx *c, void *dst, int pd, void *src, int ps);
// r = b - D x (FP64) ; returns |r|^2
dd_status residual64(dd_ctx *c, void *r, void *b, void *x, void *tmp, double *rn2);
// bring nv finalized sums of `partials` to the host
dd_status fetch(dd_ctx *c, int nv, double *out);
// the operator / precision pairs the apply entry points accept, and a loaded gauge field
dd_status check_op(dd_ctx *c, dd_prec prec, dd_op op);

// ---- dd_solvers.cpp

struct SolveOut {
    int iters = 0;
    double relres = 0;
    int detail = 0;
};

constexpr int DETAIL_OUTER_STALL = 5;  // a defect-correction pass gained nothing (or twice < 10%)
constexpr int DETAIL_INNER_STALL = 6;  // an inner solve hit its stall window and its pass gained < 10x

// Stall window of an inner solve: hit() is true once the relative residual has not
// fallen 10x below the last point where it did so within `window` iterations.
struct Stall {
    int window = 0;  // <= 0: never
    int ref_it = 0;
    double ref = 1.0;
    bool hit(int it, double relres)
    {
        if (window <= 0) return false;
        if (relres < 0.1 * ref) {
            ref = relres;
            ref_it = it;
            return false;
        }
        return it - ref_it >= window;
    }
};

// plain FP64 BiCGStab on D (x: initial guess and result)
dd_status solve_plain64(dd_ctx *c, void *x, void *b, double tol, int maxiter, SolveOut &o);
// FP32 BiCGStab on A M_SAP (SAP storage precision prec) for the source src, y = the solution
dd_status solve_sap32(dd_ctx *c, int prec, void *src, void *y, double tol, int maxiter, SolveOut &o);
// flexible GCR on A M_SAP with the FP16 SAP
dd_status solve_gcr32(dd_ctx *c, void *src, void *y, double tol, int maxiter, SolveOut &o);
// the GCR and flexible GMRES fields, allocated on the first solve of that mode
dd_status ensure_gcr(dd_ctx *c);
dd_status ensure_fgmres(dd_ctx *c);

struct OuterOut {
    int outer = 0, inner = 0;
    double inner_last = 0;
    int detail = 0;
};
// restarted flexible GMRES on D x = b in FP64 (x: initial guess and result), preconditioned by
// the FP32 SAP-BiCGStab with the FP16 SAP; |b|^2 = bn2 > 0
dd_status solve_fgmres64(dd_ctx *c, void *x, void *b, double bn2, double tol, int maxiter, OuterOut &o);

// ---- dd_batch.cpp: batched right-hand sides and several lattices

// kinds of per-RHS fields in the batch buffers (each kind: nrhs fields one after another)
enum { BK_B64, BK_X64, BK_R64, BK_T64, BK_SRC, BK_Y, BK_R, BK_RT, BK_P, BK_Q, BK_T, BK_IN, BK_OUT,
       BK_R16, BK_P16, BK_MP16, BK_MR16, BK_S16, BK_COUNT };

inline int bk_prec(int k) { return k <= BK_T64 ? DD_F64 : k >= BK_R16 ? DD_F16 : DD_F32; }

dd_status batch_alloc(dd_ctx *c, int n);
// field r of kind k
void *bf(dd_ctx *c, int k, int r);
// run a reducing vector kernel on right-hand side r and leave its nv sums at red[off..]
dd_status reduce_to(dd_ctx *c, dd::BlasArgs a, int nv, int off);
dd_status fetch_red(dd_ctx *c, int n, double *out);
// out = A in for n batched fields at input precision pin (DD_F32 or DD_F16), FP32 output,
// in tiles of up to 12
dd_status k_dirac_mrhs(dd_ctx *c, void *out, const void *in, int n, int pin);

struct BRhs {
    bool active = false;
    cplx rho0 = 0.0;
    double bn2 = 0, rn2 = 0, tol = 0;
    SolveOut o;
    Stall stall;
    dd_status st = DD_OK;
};

// lockstep FP32 BiCGStab for n right-hand sides (sources BK_SRC, solutions BK_Y)
dd_status solve_batch32(dd_ctx *c, int n, bool sap, std::vector<BRhs> &R, int maxiter);
// BK_R64 = BK_B64 - D BK_X64 for each right-hand side; rn2 = their squared norms
dd_status residual64_batch(dd_ctx *c, int n, double *rn2);

}  // namespace ddh
