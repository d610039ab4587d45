// dd_kernels.hip -- gfx950 kernels of the Clover-Wilson quark solver and their
// host launchers.
//
//  * pack / unpack between the canonical layout and the block-major internal
//    layout (FP64, FP32, per-site-scaled FP16);
//  * link packing (FP64, FP32 18-real, FP16 12-real) and the clover setup
//    (four-leaf field strength, 1 + C as two 6x6 Hermitian blocks, Cholesky
//    inverse) in FP64 -- appendix "Clover-Wilson Dirac operator";
//  * the full-lattice apply of D = 1 + C - kappa H, A = I - kappa C_inv H
//    (Sec. 3) and gamma_5 D gamma_5: one thread per site, coalesced
//    block-major loads, spin-projected hops, FP64 or FP32 arithmetic;
//  * the SAP half-sweep (Alg. 1 with the Jacobi of Alg. 2): one workgroup per
//    Schwarz block, the block's links and the current Jacobi iterate staged
//    in LDS, the cross-block term read from the neighbouring blocks;
//  * vector updates and reductions of BiCGStab (Alg. 5) with FP64
//    accumulation: wavefront shuffles, then LDS, then one partial per
//    workgroup, summed in a fixed order by a one-workgroup kernel.
#include "dd_device.h"
#include "dd_gauge.h"
#include "dd_launch.h"

namespace dd {

// ============================================================ pack / unpack

// canonical [Lt][Lz][Ly][Lx][3][4] complex double  ->  internal at precision P,
// with gamma_5 applied on the way when g5 is set
template <int P>
__global__ void __launch_bounds__(256) k_pack_spinor(Geom g, SpinorField<P> dst, const double2 *src, int g5)
{
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= g.V) return;
    Site st;
    decode(g, i, st);
    long long n = lex_index(g, st);
    Spinor<double> x;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double2 t = src[n * 12 + c * 4 + a];
            x.v[a][c] = {t.x, t.y};
        }
    if (g5) gamma5(x);
    dst.store(g, st.l, st.s, x);
}

template <int P>
__global__ void __launch_bounds__(256) k_unpack_spinor(Geom g, double2 *dst, SpinorField<P> src, int g5)
{
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= g.V) return;
    Site st;
    decode(g, i, st);
    long long n = lex_index(g, st);
    Spinor<double> x;
    src.load(g, st.l, st.s, x);
    if (g5) gamma5(x);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) dst[n * 12 + c * 4 + a] = make_double2(x.v[a][c].re, x.v[a][c].im);
}

// canonical links [4][Lt][Lz][Ly][Lx][3][3] -> FP64 (18 reals), FP32 and FP16 (rows 0 and
// 1, 12 reals); flags non-finite entries
__global__ void __launch_bounds__(256)
    k_pack_links(Geom g, const double2 *src, double2 *u64, float2 *u32, __half2 *u16, int *bad)
{
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= g.V) return;
    Site st;
    decode(g, i, st);
    long long n = lex_index(g, st);
    int nonfinite = 0;
    for (int mu = 0; mu < 4; ++mu) {
        const double2 *m = src + ((long long)mu * g.V + n) * 9;
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            double2 t = m[e];
            if (!isfinite(t.x) || !isfinite(t.y)) nonfinite = 1;
            u64[elem(g, st.l, st.s, 36, mu * 9 + e)] = t;
            if (e < 6) {
                u32[elem(g, st.l, st.s, 24, mu * 6 + e)] = make_float2((float)t.x, (float)t.y);
                u16[elem(g, st.l, st.s, 24, mu * 6 + e)] = __floats2half2_rn((float)t.x, (float)t.y);
            }
        }
    }
    if (nonfinite) atomicOr(bad, 1);
}

// ============================================================ clover setup

// Cholesky inverse of a Hermitian positive definite 6x6 matrix (full storage);
// returns false when a pivot is not positive
DD_INL bool hpd_inverse6(cx<double> (&M)[6][6], cx<double> (&Minv)[6][6])
{
    cx<double> L[6][6];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) L[i][j] = {0, 0};
    for (int j = 0; j < 6; ++j) {
        double d = M[j][j].re;
        for (int k = 0; k < j; ++k) d -= norm2(L[j][k]);
        if (!(d > 0.0)) return false;
        double ljj = sqrt(d);
        L[j][j] = {ljj, 0};
        for (int i = j + 1; i < 6; ++i) {
            cx<double> s = M[i][j];
            for (int k = 0; k < j; ++k) s = s - L[i][k] * conj(L[j][k]);
            L[i][j] = (1.0 / ljj) * s;
        }
    }
    // Linv = L^{-1} (lower triangular) by forward substitution
    cx<double> Li[6][6];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) Li[i][j] = {0, 0};
    for (int j = 0; j < 6; ++j) {
        Li[j][j] = {1.0 / L[j][j].re, 0};
        for (int i = j + 1; i < 6; ++i) {
            cx<double> s = {0, 0};
            for (int k = j; k < i; ++k) s = s + L[i][k] * Li[k][j];
            Li[i][j] = (-1.0 / L[i][i].re) * s;
        }
    }
    // M^{-1} = Linv^dagger Linv
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            cx<double> s = {0, 0};
            for (int k = (i > j ? i : j); k < 6; ++k) s = s + cmulc(Li[k][i], Li[k][j]);
            Minv[i][j] = s;
        }
    return true;
}

template <typename V2> DD_INL V2 mk2(double a, double b);
template <> DD_INL double2 mk2<double2>(double a, double b) { return make_double2(a, b); }
template <> DD_INL float2 mk2<float2>(double a, double b) { return make_float2((float)a, (float)b); }
template <> DD_INL __half2 mk2<__half2>(double a, double b) { return __floats2half2_rn((float)a, (float)b); }

// store a Hermitian 6x6 pair (blocks + and -) scaled by `f` in the clover layout
template <typename V2>
DD_INL void store_clov(V2 *dst, const Geom &g, int l, int s, cx<double> (&M)[2][6][6], double f)
{
    for (int b = 0; b < 2; ++b) {
        for (int j = 0; j < 3; ++j)
            dst[elem(g, l, s, 36, b * 18 + j)] = mk2<V2>(f * M[b][2 * j][2 * j].re, f * M[b][2 * j + 1][2 * j + 1].re);
        for (int i = 0; i < 6; ++i)
            for (int j = i + 1; j < 6; ++j) {
                cx<double> v = M[b][i][j];
                dst[elem(g, l, s, 36, b * 18 + 3 + upper_index(i, j))] = mk2<V2>(f * v.re, f * v.im);
            }
    }
}

// 1 + C in the gamma_5-diagonal basis is diag(M+, M-) with
//   M_pm = 1 + i kappa c_SW sum_{mu<nu} sigma^pm_{mu nu} (x) F_{mu nu},
// sigma^pm the 2x2 diagonal blocks of P sigma_{mu nu} P, P = [[1,1],[1,-1]]/sqrt 2.
// Stored: N = M/2 (so that 1 + C = Q diag(N+, N-) Q, Q = [[1,1],[1,-1]]) in FP64,
// and M^{-1}/2 (C_inv = Q diag(M+^{-1}/2, M-^{-1}/2) Q) in FP32 and FP16.
__global__ void __launch_bounds__(64) k_clover(Geom g, const double2 *u64, SigmaBlocks sig, double kcsw,
                                               double2 *clov64, float2 *cinv32, __half2 *cinv16, int *bad)
{
    long long i = (long long)blockIdx.x * 64 + threadIdx.x;
    if (i >= g.V) return;
    int l = (int)(i >> g.lbvol), s = (int)(i & (g.bvol - 1));
    cx<double> M[2][6][6];
    for (int b = 0; b < 2; ++b)
        for (int p = 0; p < 6; ++p)
            for (int q = 0; q < 6; ++q) M[b][p][q] = {p == q ? 1.0 : 0.0, 0.0};
    int plane = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu, ++plane) {
            Mat3<double> F;
            field_strength(g, u64, i, mu, nu, F);
            for (int b = 0; b < 2; ++b)
                for (int s1 = 0; s1 < 2; ++s1)
                    for (int s2 = 0; s2 < 2; ++s2) {
                        cx<double> sg = {sig.re[plane][b][s1][s2], sig.im[plane][b][s1][s2]};
                        if (sg.re == 0.0 && sg.im == 0.0) continue;
                        cx<double> pre = cx<double>{0.0, kcsw} * sg;  // i kappa c_SW sigma
                        for (int a = 0; a < 3; ++a)
                            for (int c = 0; c < 3; ++c)
                                M[b][s1 * 3 + a][s2 * 3 + c] = M[b][s1 * 3 + a][s2 * 3 + c] + pre * F.m[a][c];
                    }
        }
    store_clov(clov64, g, l, s, M, 0.5);
    cx<double> Mi[2][6][6];
    bool ok = hpd_inverse6(M[0], Mi[0]) && hpd_inverse6(M[1], Mi[1]);
    if (!ok) {
        atomicOr(bad, 1);
        for (int b = 0; b < 2; ++b)
            for (int p = 0; p < 6; ++p)
                for (int q = 0; q < 6; ++q) Mi[b][p][q] = {0, 0};
    }
    store_clov(cinv32, g, l, s, Mi, 0.5);
    store_clov(cinv16, g, l, s, Mi, 0.5);
}

// ============================================================ Dirac apply

template <int P> DD_INL SpinorField<P> sf_at(void *p, const Geom &g);
template <> DD_INL SpinorField<1> sf_at<1>(void *p, const Geom &) { return SpinorField<1>{(float2 *)p}; }
template <> DD_INL SpinorField<2> sf_at<2>(void *p, const Geom &g)
{
    return SpinorField<2>{(__half2 *)p, (float *)((char *)p + 12 * g.V * sizeof(__half2))};
}

template <int PIN, int PG> struct Acc { using T = float; };
template <int PG> struct Acc<0, PG> { using T = double; };
template <> struct Acc<1, 0> { using T = double; };
template <> struct Acc<2, 0> { using T = double; };

// out = op(in) on the full lattice, one thread per site; op 0 = D, 1 = A, 2 = D^dagger
// out(i) = op(in)(i) for one site i
template <int PIN, int POUT, int PG, int OP>
DD_INL void dirac_site(const Geom &g, const SpinorField<POUT> &out, const SpinorField<PIN> &in, const LinkField<PG> &U,
                       const CloverField<PG> &C, const Phase4 &ph, double kappa, long long i)
{
    using R = typename Acc<PIN, PG>::T;
    Site st;
    decode(g, i, st);
    Spinor<R> acc;
    zero(acc);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
        for (int dir = 1; dir >= -1; dir -= 2) {
            bool wrap, inblk;
            long long j = neighbour(g, st, mu, dir, wrap, inblk);
            int lj = (int)(j >> g.lbvol), sj = (int)(j & (g.bvol - 1));
            Spinor<R> psi;
            in.load(g, lj, sj, psi);
            if (OP == 2) gamma5(psi);
            Mat3<R> W;
            if (dir > 0)
                U.load(g, st.l, st.s, mu, W);
            else
                U.load(g, lj, sj, mu, W);
            cx<R> phase = {R(ph.re[mu]), R(dir > 0 ? ph.im[mu] : -ph.im[mu])};
            hop(mu, dir, W, psi, wrap, phase, acc);
        }
    }
    Spinor<R> x, t, o;
    in.load(g, st.l, st.s, x);
    if (OP == 2) gamma5(x);
    Clov<R> cl;
    C.load(g, st.l, st.s, cl);
    const R k = R(kappa);
    if (OP == 1) {
        clover_mul(cl, acc, t);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) o.v[a][c] = x.v[a][c] - k * t.v[a][c];
    } else {
        clover_mul(cl, x, t);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) o.v[a][c] = t.v[a][c] - k * acc.v[a][c];
        if (OP == 2) gamma5(o);
    }
    out.store(g, st.l, st.s, o, true);
}

// B > 0: the block shape is B^4, known at compile time (strides and block volume fold)
template <int PIN, int POUT, int PG, int OP, int B>
__global__ void __launch_bounds__(256) k_dirac(Geom gin, SpinorField<POUT> out, SpinorField<PIN> in, LinkField<PG> U,
                                               CloverField<PG> C, Phase4 ph, double kappa)
{
    const Geom g = fixed_shape<B>(gin);
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    const long long i = (long long)w * 256 + threadIdx.x;
    if (i >= g.V) return;
    dirac_site<PIN, POUT, PG, OP>(g, out, in, U, C, ph, kappa, i);
}

// ---- the same operator streamed along t (4^4 blocks)
// A workgroup walks `ns` consecutive blocks of one column (fixed block x, y, z) in t:
//  * the block's input spinor is staged in LDS, and in-block neighbours come from there
//    (one HBM/L2 read per site instead of one per hop);
//  * the top slice computes the next block's backward t hop term, U_t^dagger times the
//    projected spinor (the same arithmetic the hop does), so the next block reads neither
//    that face's spinor nor its links: a block-per-workgroup launch reads them a second
//    time, too long after the block itself for the L2 to still hold them.
// The next block's t' = 0 slice, which the top slice reads for its forward hop, is read again
// by the next step rather than kept in LDS: the neighbouring columns read it at that time too
// (their x, y and z faces), and those reads then share the L2 lines (measured: keeping it was
// no faster).
// Columns are taken x fastest, then the two columns of a z pair, then y, then the z pairs:
// consecutive workgroups (which one XCD runs side by side) then hold a column's x neighbours,
// its y neighbours 2 NB_x items away and, for one of its two z faces, its z neighbour NB_x
// items away, so those faces come from the L2 while the neighbour's block is still there.  A
// face's sites are short runs of a block's site-major storage (four sites for a y face,
// sixteen for a z face), so a face read that misses the L2 fetches whole lines of which it
// uses a quarter or a half.  Against the plain lexicographic order (whose z neighbours are
// NB_x NB_y items away) with walks of 4, this order with walks of 2 takes 64^3x128 from 4.39
// to 4.26-4.29 ms (FP16-input A), 5.20-5.22 to 5.12-5.14 ms (FP32 A) and 10.43-10.46 to
// 10.33-10.39 ms (FP64 D); 2x2 or 4x4 tiles of (y, z) columns and longer z runs gain less or
// lose.
// The hop order and arithmetic are those of dirac_site; results agree to FP32 (FP64) rounding,
// not bit for bit, since the compiler fuses multiply-adds differently in the two kernels.
template <int P> struct StoreT;
template <> struct StoreT<0> { using T = double2; };
template <> struct StoreT<1> { using T = float2; };
template <> struct StoreT<2> { using T = __half2; };

// one site's spinor as stored: 12 elements (256 apart in a 4^4 block) and the FP16 scale
template <int P> struct RawSp {
    typename StoreT<P>::T e[12];
    float sc;
};

template <int P> DD_INL void raw_load(const typename StoreT<P>::T *p, const float *sp, RawSp<P> &r)
{
#pragma unroll
    for (int e = 0; e < 12; ++e) r.e[e] = p[e * 256];
    r.sc = P == 2 ? *sp : 1.f;
}

// the conversion SpinorField<P>::load applies
template <int P, typename R> DD_INL void raw_to(const RawSp<P> &r, Spinor<R> &x)
{
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if constexpr (P == 2) {
                float2 t = __half22float2(r.e[a * 3 + c]);
                x.v[a][c] = {R(t.x * r.sc), R(t.y * r.sc)};
            } else {
                x.v[a][c] = {R(r.e[a * 3 + c].x), R(r.e[a * 3 + c].y)};
            }
        }
}

template <int PIN, int POUT, int PG, int OP>
__global__ void __launch_bounds__(256) k_dirac_ts(Geom gin, SpinorField<POUT> out, SpinorField<PIN> in, LinkField<PG> U,
                                                  CloverField<PG> C, Phase4 ph, double kappa, int ns)
{
    using R = typename Acc<PIN, PG>::T;
    using T = typename StoreT<PIN>::T;
    const Geom g = fixed_shape<4>(gin);
    __shared__ T tile[12][256];                     // this block's input
    __shared__ float tsc[PIN == 2 ? 256 : 1];
    __shared__ cx<R> carry[2][6][64];               // backward t hop terms, by step parity
    wg_skew();
    const int ncol = g.bstride[3];
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    const int seg = w / ncol, q = w - seg * ncol;
    int col;  // item q -> column: x fastest, then z within a pair, then y, then the z pair
    {
        const int nx = g.NB[0], ny = g.NB[1];
        int r = q / nx;
        const int bx = q - r * nx;
        const int zl = r & 1;
        r >>= 1;
        const int zp = r / ny, by = r - zp * ny;
        col = bx + nx * (by + ny * (2 * zp + zl));
    }
    const int s = threadIdx.x, tw = __builtin_amdgcn_readfirstlane(s >> 6);  // t' of the site: one per wavefront
    // the FP16 scale of internal site i (FP32 / FP64 inputs have none)
    auto scale_at = [&](long long i) -> const float * {
        if constexpr (PIN == 2)
            return in.scale + i;
        else
            return nullptr;
    };
    const int bt0 = seg * ns;
    for (int k = 0; k < ns; ++k) {
        // the site is decoded afresh in every step, from a thread index the compiler cannot
        // follow across steps: otherwise it keeps every hop's addresses from one step to the
        // next in registers (some 40 VGPRs, one wavefront per SIMD less)
        int sl = s;
        asm volatile("" : "+v"(sl));
        Site st;
        decode(g, ((long long)(col + (bt0 + k) * ncol) << 8) + sl, st);
        // stage the block
        {
            RawSp<PIN> own;
            raw_load<PIN>(&in.p[elem(g, st.l, sl, 12, 0)], scale_at(((long long)st.l << 8) + sl), own);
#pragma unroll
            for (int e = 0; e < 12; ++e) tile[e][sl] = own.e[e];
            if constexpr (PIN == 2) tsc[sl] = own.sc;
        }
        wg_barrier();
        Spinor<R> acc;
        zero(acc);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
            for (int dir = 1; dir >= -1; dir -= 2) {
                if (mu == 3 && dir < 0 && tw == 0 && k > 0) {  // computed by the previous block's top slice
                    Half<R> kk;
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int c = 0; c < 3; ++c) kk.v[a][c] = carry[k & 1][a * 3 + c][sl];
                    reconstruct(3, -1, kk, acc);
                    continue;
                }
                bool wrap, inblk;
                const long long j = neighbour(g, st, mu, dir, wrap, inblk);
                const int lj = (int)(j >> 8), sj = (int)(j & 255);
                // one load path for both sources: LDS and HBM hold the elements 256 apart
                RawSp<PIN> r;
                raw_load<PIN>(inblk ? &tile[0][sj] : &in.p[elem(g, lj, sj, 12, 0)],
                              inblk ? &tsc[PIN == 2 ? sj : 0] : scale_at(j), r);
                Spinor<R> psi;
                raw_to<PIN>(r, psi);
                if (OP == 2) gamma5(psi);
                Mat3<R> W;
                if (dir > 0)
                    U.load(g, st.l, sl, mu, W);
                else
                    U.load(g, lj, sj, mu, W);
                cx<R> phase = {R(ph.re[mu]), R(dir > 0 ? ph.im[mu] : -ph.im[mu])};
                hop(mu, dir, W, psi, wrap, phase, acc);
            }
        }
        Spinor<R> x, t, o;
        {
            RawSp<PIN> r;
            raw_load<PIN>(&tile[0][sl], &tsc[PIN == 2 ? sl : 0], r);
            raw_to<PIN>(r, x);
        }
        if (OP == 2) gamma5(x);
        Clov<R> cl;
        C.load(g, st.l, sl, cl);
        const R kr = R(kappa);
        if (OP == 1) {
            clover_mul(cl, acc, t);
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) o.v[a][c] = x.v[a][c] - kr * t.v[a][c];
        } else {
            clover_mul(cl, x, t);
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) o.v[a][c] = t.v[a][c] - kr * acc.v[a][c];
            if (OP == 2) gamma5(o);
        }
        out.store(g, st.l, sl, o, true);
        // the next block's backward t hop term from this block's top slice
        if (tw == 3 && k + 1 < ns) {
            Mat3<R> W;
            U.load(g, st.l, sl, 3, W);
            Half<R> h, kk;
            project(3, -1, x, h);
            mat_half(W, true, h, kk);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) carry[(k + 1) & 1][a * 3 + c][sl - 192] = kk.v[a][c];
        }
        wg_barrier();
    }
}

// A = I - kappa C_inv H (FP32 links and C_inv, FP32 output, input at precision PIN) on
// several lattices in one persistent launch: the work items are (lattice, 256-site
// chunk) pairs numbered lattice by lattice; each workgroup takes the next item from
// a global counter until none is left, so lattices of uneven size share the chip
// without a launch (or an idle tail) per lattice.  Every workgroup leaves once the
// counter passes the item count.
template <int PIN>
__global__ void __launch_bounds__(256) k_dirac_multi(const LatDesc *desc, int nlat, int total, int *counter)
{
    __shared__ int item_s;
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(counter, 1);
        wg_barrier();
        const int item = item_s;
        wg_barrier();
        if (item >= total) break;
        int lat = 0;
        while (lat + 1 < nlat && item >= desc[lat + 1].item0) ++lat;
        const LatDesc &d = desc[lat];
        const long long i = (long long)(item - d.item0) * 256 + threadIdx.x;
        if (i < d.g.V) {
            SpinorField<PIN> in = sf_at<PIN>((void *)d.in, d.g);
            SpinorField<1> out{(float2 *)d.out};
            dirac_site<PIN, 1, 1, 1>(d.g, out, in, LinkField<1>{(const float2 *)d.u},
                                     CloverField<1>{(const float2 *)d.cinv}, d.phase, d.kappa, i);
        }
    }
}

// ============================================================ SAP half-sweep

// where the SAP kernel reads the block's links from: the FP16 copy (rows 0 and
// 1, 24 half2 per site, 24 KB for a 4^4 block) is staged in LDS as is and the
// third row is rebuilt at each use (staging full 3x3 matrices measured slower:
// the extra LDS reads cost more than the rebuild); FP32 links are read from
// global memory through the caches, which keeps that workgroup's LDS at 24 KB
template <int P> struct SapLinks;
template <> struct SapLinks<1> {
    static constexpr int E = 0;  // nothing staged
    using T = float2;
    LinkField<1> U;
    DD_INL void stage(T *, const Geom &, int, int) const {}
    DD_INL void load(const T *, const Geom &g, int l, int s, int mu, Mat3<float> &W) const { U.load(g, l, s, mu, W); }
};
template <> struct SapLinks<2> {
    static constexpr int E = 24;
    using T = __half2;
    const __half2 *p;
    DD_INL void stage(T *lds, const Geom &g, int l, int s) const
    {
        for (int e = 0; e < E; ++e) lds[e * g.bvol + s] = p[elem(g, l, s, E, e)];
    }
    DD_INL void load(const T *lds, const Geom &g, int, int s, int mu, Mat3<float> &U) const
    {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                float2 t = __half22float2(lds[(mu * 6 + a * 3 + b) * g.bvol + s]);
                U.m[a][b] = {t.x, t.y};
            }
        su3_row3(U);
    }
};

DD_INL void lds_store_spinor(float2 *xs, int bvol, int s, const Spinor<float> &x)
{
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) xs[(a * 3 + c) * bvol + s] = make_float2(x.v[a][c].re, x.v[a][c].im);
}

DD_INL void lds_load_spinor(const float2 *xs, int bvol, int s, Spinor<float> &x)
{
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float2 t = xs[(a * 3 + c) * bvol + s];
            x.v[a][c] = {t.x, t.y};
        }
}

// acc = H_in x: the hops that stay inside the block (Dirichlet at the block
// faces), neighbours from LDS; in-block hops never cross the lattice edge, so
// they carry no boundary phase
template <int P>
DD_INL void inblock_hops(const float2 *xs, const SapLinks<P> &lk, const typename SapLinks<P>::T *ul, const Geom &g,
                         const Site &st, Spinor<float> &acc)
{
    zero(acc);
    const int bvol = g.bvol;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int stride = 1 << g.sh[mu];
#pragma unroll
        for (int dir = 1; dir >= -1; dir -= 2) {
            int c = st.c[mu] + dir;
            if (c < 0 || c >= g.b[mu]) continue;
            int m = st.s + dir * stride;
            Spinor<float> psi;
            lds_load_spinor(xs, bvol, m, psi);
            Mat3<float> W;
            lk.load(ul, g, st.l, dir > 0 ? st.s : m, mu, W);
            hop(mu, dir, W, psi, false, cx<float>{1.f, 0.f}, acc);
        }
    }
}

// One half-sweep of Alg. 1 for the blocks of one colour c (E = 0, O = 1):
//   [PRE]   s_c <- s_c - A_{c c'} x_{c'}     (cross-block hops from the other colour)
//           x_c  = B_cc s_c                   (Alg. 2: x = s + K x, n_jac times, K = kappa C_inv H_in)
//   [!TAIL] s_c <- s_c + b_c - A_cc x_c      (A_cc x = x - K x)
// FIRST takes s_c from b (s = b at the start of Alg. 1).  The fused tail of Alg. 3 (A M_SAP b,
// written to ax): with TAIL, AMSAP also writes ax_c = A_cc x_c, AMSAP_PRE includes the
// cross-block term A_{c c'} x_{c'} (the odd tail, whose neighbours already hold the final even
// x), and a CROSS_ONLY launch on the even blocks then adds A_{c c'} x_{c'} of the final odd x.  One
// workgroup per block, one thread per site; blockDim.x == block volume.
template <int P, int B>
__global__ void __launch_bounds__(256) k_sap_half(Geom gin, int colour, int flags, SpinorField<P> bsrc,
                                                  SpinorField<P> sw, SpinorField<P> xw, SapLinks<P> lk,
                                                  LinkField<P> U, CloverField<P> Ci, Phase4 ph, float kappa,
                                                  int n_jac, SpinorField<P> axw)
{
    const Geom g = fixed_shape<B>(gin);
    using LT = typename SapLinks<P>::T;
    extern __shared__ float4 smem_raw[];
    const int bvol = g.bvol;
    float2 *xs = reinterpret_cast<float2 *>(smem_raw);
    LT *ul = reinterpret_cast<LT *>(xs + 12 * bvol);
    wg_skew();

    const int w = xcd_remap(blockIdx.x, gridDim.x);
    Site st;
    st.l = colour_block(g, colour, w);
    st.s = threadIdx.x;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) st.c[mu] = (st.s >> g.sh[mu]) & (g.b[mu] - 1);
    block_coords(g, st.l, st.B);

    const bool cross_only = (flags & SAP_CROSS_ONLY) != 0;
    if (!cross_only) lk.stage(ul, g, st.l, st.s);

    Clov<float> cl;
    Ci.load(g, st.l, st.s, cl);
    Spinor<float> src;
    if (!cross_only) {
        if (flags & SAP_FIRST)
            bsrc.load(g, st.l, st.s, src);
        else
            sw.load(g, st.l, st.s, src);
    }

    // acc += H_{c c'} x_{c'} at this site: the hops that come from the neighbouring blocks
    auto cross_hops = [&](Spinor<float> &acc) {
        for (int mu = 0; mu < 4; ++mu) {
            for (int dir = 1; dir >= -1; dir -= 2) {
                int c = st.c[mu] + dir;
                if (c >= 0 && c < g.b[mu]) continue;
                bool wrap, inblk;
                long long j = neighbour(g, st, mu, dir, wrap, inblk);
                int lj = (int)(j >> g.lbvol), sj = (int)(j & (bvol - 1));
                Spinor<float> psi;
                xw.load(g, lj, sj, psi);
                Mat3<float> W;
                if (dir > 0)
                    U.load(g, st.l, st.s, mu, W);
                else
                    U.load(g, lj, sj, mu, W);
                cx<float> phase = {(float)ph.re[mu], (float)(dir > 0 ? ph.im[mu] : -ph.im[mu])};
                hop(mu, dir, W, psi, wrap, phase, acc);
            }
        }
    };
    Spinor<float> acc, t;
    if ((flags & SAP_PRE) || cross_only) {
        zero(acc);
        cross_hops(acc);
        clover_mul(cl, acc, t);
        if (cross_only) {  // ax_c += A_{c c'} x_{c'} = -kappa C_inv H_{c c'} x_{c'}
            Spinor<float> q;
            axw.load(g, st.l, st.s, q);
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) q.v[a][c] = q.v[a][c] - kappa * t.v[a][c];
            axw.store(g, st.l, st.s, q);
            return;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) src.v[a][c] = src.v[a][c] + kappa * t.v[a][c];
    }

    Spinor<float> x = src;
    for (int j = 0; j < n_jac; ++j) {
        wg_barrier();  // previous readers of xs are done (and links staged)
        lds_store_spinor(xs, bvol, st.s, x);
        wg_barrier();
        inblock_hops<P>(xs, lk, ul, g, st, acc);
        clover_mul(cl, acc, t);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) x.v[a][c] = src.v[a][c] + kappa * t.v[a][c];
    }
    if (!(flags & SAP_TAIL)) {
        wg_barrier();
        lds_store_spinor(xs, bvol, st.s, x);
        wg_barrier();
        inblock_hops<P>(xs, lk, ul, g, st, acc);
        clover_mul(cl, acc, t);
        Spinor<float> b;
        bsrc.load(g, st.l, st.s, b);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                src.v[a][c] = src.v[a][c] + b.v[a][c] - x.v[a][c] + kappa * t.v[a][c];
        sw.store(g, st.l, st.s, src);
    } else if (flags & SAP_AMSAP) {
        // Alg. 3: this colour's rows of A x, x - kappa C_inv (H_in x + H_{c c'} x_{c'}): the
        // in-block hops of the final x, and with AMSAP_PRE the hops from the other colour's final
        // x, the same ones this launch's prologue read (formed again here rather than kept
        // through the sweeps), all under one C_inv product as in the Dirac apply
        wg_barrier();
        lds_store_spinor(xs, bvol, st.s, x);
        wg_barrier();
        inblock_hops<P>(xs, lk, ul, g, st, acc);
        if (flags & SAP_AMSAP_PRE) cross_hops(acc);
        clover_mul(cl, acc, t);
        Spinor<float> q;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) q.v[a][c] = x.v[a][c] - kappa * t.v[a][c];
        axw.store(g, st.l, st.s, q);
    }
    xw.store(g, st.l, st.s, x);
}

// ============================================================ vector kernels

template <int P> struct Elem;
template <> struct Elem<0> {
    DD_INL static cx<double> get(const SpinorField<0> &f, const Geom &, long long o)
    {
        double2 t = f.p[o];
        return {t.x, t.y};
    }
    DD_INL static void put(const SpinorField<0> &f, const Geom &, long long o, cx<double> v)
    {
        f.p[o] = make_double2(v.re, v.im);
    }
};
template <> struct Elem<1> {
    DD_INL static cx<double> get(const SpinorField<1> &f, const Geom &, long long o)
    {
        float2 t = f.p[o];
        return {(double)t.x, (double)t.y};
    }
    DD_INL static void put(const SpinorField<1> &f, const Geom &, long long o, cx<double> v)
    {
        f.p[o] = make_float2((float)v.re, (float)v.im);
    }
};
template <> struct Elem<2> {  // read only: the scale belongs to the whole site
    DD_INL static cx<double> get(const SpinorField<2> &f, const Geom &g, long long o)
    {
        long long blk12 = o >> g.lbvol;  // l*12 + e
        long long site = ((blk12 / 12) << g.lbvol) + (o & (g.bvol - 1));
        float sc = f.scale[site];
        float2 t = __half22float2(f.p[o]);
        return {(double)(t.x * sc), (double)(t.y * sc)};
    }
};

// sum the per-workgroup partials in a fixed order: out[k] = sum_w partials[w*nv + k]
__global__ void __launch_bounds__(256) k_finalize(const double *partials, int nwg, int nv, double *out)
{
    __shared__ double sh[256];
    for (int k = 0; k < nv; ++k) {
        double t = 0;
        for (int w = threadIdx.x; w < nwg; w += 256) t += partials[(long long)w * nv + k];
        sh[threadIdx.x] = t;
        wg_barrier();
        for (int h = 128; h >= 1; h >>= 1) {
            if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
            wg_barrier();
        }
        if (threadIdx.x == 0) out[k] = sh[0];
        wg_barrier();
    }
}

#define GRID_STRIDE(o, N) for (long long o = (long long)blockIdx.x * BLAS_WG + threadIdx.x; o < (N); o += (long long)gridDim.x * BLAS_WG)
// the same loop for workgroup wid of nwg (the bodies below, shared by the single-lattice
// kernels and the multi-lattice launch)
#define GRID_STRIDE_W(o, N) for (long long o = (long long)wid * BLAS_WG + threadIdx.x; o < (N); o += (long long)nwg * BLAS_WG)

// <a|b> (2 values) and, with NV = 3, |a|^2 as the third
template <int PA, int PB, int NV>
DD_INL void dot_body(const Geom &g, SpinorField<PA> a, SpinorField<PB> b, double *partials, int wid, int nwg)
{
    double v[NV] = {};
    GRID_STRIDE_W(o, 12 * g.V)
    {
        cx<double> x = Elem<PA>::get(a, g, o), y = Elem<PB>::get(b, g, o);
        cx<double> d = cmulc(x, y);
        v[0] += d.re;
        v[1] += d.im;
        if (NV == 3) v[2] += norm2(x);
    }
    wg_reduce_store_at<NV>(v, partials, wid);
}

template <int PA, int PB, int NV>
__global__ void __launch_bounds__(BLAS_WG) k_dot(Geom g, SpinorField<PA> a, SpinorField<PB> b, double *partials)
{
    dot_body<PA, PB, NV>(g, a, b, partials, blockIdx.x, gridDim.x);
}

template <int PA>
__global__ void __launch_bounds__(BLAS_WG) k_norm2(Geom g, SpinorField<PA> a, double *partials)
{
    double v[1] = {0};
    GRID_STRIDE(o, 12 * g.V) v[0] += norm2(Elem<PA>::get(a, g, o));
    wg_reduce_store<1>(v, partials);
}

// x += alpha y ; r -= alpha q ; partial |r|^2
template <int PX, int PY, int PR>
__global__ void __launch_bounds__(BLAS_WG) k_update1(Geom g, SpinorField<PX> x, SpinorField<PY> y, SpinorField<PR> r,
                                                     SpinorField<PR> q, double are, double aim, double *partials)
{
    double v[1] = {0};
    const cx<double> al = {are, aim};
    GRID_STRIDE(o, 12 * g.V)
    {
        Elem<PX>::put(x, g, o, Elem<PX>::get(x, g, o) + al * Elem<PY>::get(y, g, o));
        cx<double> rr = Elem<PR>::get(r, g, o) - al * Elem<PR>::get(q, g, o);
        Elem<PR>::put(r, g, o, rr);
        rr = Elem<PR>::get(r, g, o);  // norm of the stored (rounded) value
        v[0] += norm2(rr);
    }
    wg_reduce_store<1>(v, partials);
}

// x += omega y ; r -= omega t ; partial |r|^2 and <rt|r>
template <int PX, int PY, int PR>
__global__ void __launch_bounds__(BLAS_WG) k_update2(Geom g, SpinorField<PX> x, SpinorField<PY> y, SpinorField<PR> r,
                                                     SpinorField<PR> t, SpinorField<PR> rt, double ore, double oim,
                                                     double *partials)
{
    double v[3] = {0, 0, 0};
    const cx<double> om = {ore, oim};
    GRID_STRIDE(o, 12 * g.V)
    {
        Elem<PX>::put(x, g, o, Elem<PX>::get(x, g, o) + om * Elem<PY>::get(y, g, o));
        cx<double> rr = Elem<PR>::get(r, g, o) - om * Elem<PR>::get(t, g, o);
        Elem<PR>::put(r, g, o, rr);
        rr = Elem<PR>::get(r, g, o);
        v[0] += norm2(rr);
        cx<double> d = cmulc(Elem<PR>::get(rt, g, o), rr);
        v[1] += d.re;
        v[2] += d.im;
    }
    wg_reduce_store<3>(v, partials);
}

// p = r + beta (p - omega q)
template <int PR>
__global__ void __launch_bounds__(BLAS_WG) k_pupdate(Geom g, SpinorField<PR> p, SpinorField<PR> r, SpinorField<PR> q,
                                                     double bre, double bim, double ore, double oim)
{
    const cx<double> be = {bre, bim}, om = {ore, oim};
    GRID_STRIDE(o, 12 * g.V)
    {
        cx<double> pv = Elem<PR>::get(p, g, o);
        Elem<PR>::put(p, g, o, Elem<PR>::get(r, g, o) + be * (pv - om * Elem<PR>::get(q, g, o)));
    }
}

// Fused updates of the mixed-precision BiCGStab (FP32 vectors, FP16-storage SAP
// inputs and outputs): the FP16 copy of r or p that the next SAP application reads
// is written by the update that produces the vector, one site per thread (the FP16
// storage scale belongs to the whole site), instead of by a separate conversion
// pass that reads the vector again.  The grid is the vector kernels' grid, so the
// partial sums line up with the finalising reduction.
#define SITE_STRIDE_W(i) for (long long i = (long long)wid * BLAS_WG + threadIdx.x; i < g.V; i += (long long)nwg * BLAS_WG)

// r -= alpha q ; partial |r|^2 ; r16 = r
DD_INL void update1_h_body(const Geom &g, SpinorField<1> r, SpinorField<1> q, SpinorField<2> r16, double are, double aim,
                           double *partials, int wid, int nwg)
{
    double v[1] = {0};
    const cx<double> al = {are, aim};
    SITE_STRIDE_W(i)
    {
        const int l = (int)(i >> g.lbvol), s = (int)(i & (g.bvol - 1));
        Spinor<float> rs;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long long o = elem(g, l, s, 12, a * 3 + c);
                const cx<double> rr = Elem<1>::get(r, g, o) - al * Elem<1>::get(q, g, o);
                Elem<1>::put(r, g, o, rr);
                rs.v[a][c] = {(float)rr.re, (float)rr.im};  // the stored (rounded) value
                v[0] += norm2(cx<double>{(double)rs.v[a][c].re, (double)rs.v[a][c].im});
            }
        r16.store(g, l, s, rs);
    }
    wg_reduce_store_at<1>(v, partials, wid);
}

__global__ void __launch_bounds__(BLAS_WG) k_update1_h(Geom g, SpinorField<1> r, SpinorField<1> q, SpinorField<2> r16,
                                                       double are, double aim, double *partials)
{
    update1_h_body(g, r, q, r16, are, aim, partials, blockIdx.x, gridDim.x);
}

// x += alpha y1 + omega y2 ; r -= omega t ; partial |r|^2 and <rt|r>.  A thread takes whole sites (as the other
// updates do): an FP16 operand's scale is read once per site, and no element index is divided back into its site.
template <int PY>
DD_INL void update2_mm_body(const Geom &g, SpinorField<1> x, SpinorField<PY> y1, SpinorField<PY> y2, SpinorField<1> r,
                            SpinorField<1> t, SpinorField<1> rt, double are, double aim, double ore, double oim,
                            double *partials, int wid, int nwg)
{
    double v[3] = {0, 0, 0};
    const cx<double> al = {are, aim}, om = {ore, oim};
    SITE_STRIDE_W(i)
    {
        const int l = (int)(i >> g.lbvol), s = (int)(i & (g.bvol - 1));
        Spinor<float> u1, u2;  // as stored (FP16: times the site scale, in FP32)
        y1.load(g, l, s, u1);
        y2.load(g, l, s, u2);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long long o = elem(g, l, s, 12, a * 3 + c);
                const cx<double> w1 = {(double)u1.v[a][c].re, (double)u1.v[a][c].im};
                const cx<double> w2 = {(double)u2.v[a][c].re, (double)u2.v[a][c].im};
                Elem<1>::put(x, g, o, Elem<1>::get(x, g, o) + al * w1 + om * w2);
                const cx<double> rr = Elem<1>::get(r, g, o) - om * Elem<1>::get(t, g, o);
                Elem<1>::put(r, g, o, rr);
                const cx<double> rs = {(double)(float)rr.re, (double)(float)rr.im};  // the stored (rounded) value
                v[0] += norm2(rs);
                const cx<double> d = cmulc(Elem<1>::get(rt, g, o), rs);
                v[1] += d.re;
                v[2] += d.im;
            }
    }
    wg_reduce_store_at<3>(v, partials, wid);
}

template <int PY>
__global__ void __launch_bounds__(BLAS_WG) k_update2_mm(Geom g, SpinorField<1> x, SpinorField<PY> y1, SpinorField<PY> y2,
                                                        SpinorField<1> r, SpinorField<1> t, SpinorField<1> rt,
                                                        double are, double aim, double ore, double oim, double *partials)
{
    update2_mm_body<PY>(g, x, y1, y2, r, t, rt, are, aim, ore, oim, partials, blockIdx.x, gridDim.x);
}

// p = r + beta (p - omega q) ; p16 = p
DD_INL void pupdate_h_body(const Geom &g, SpinorField<1> p, SpinorField<1> r, SpinorField<1> q, SpinorField<2> p16,
                           double bre, double bim, double ore, double oim, int wid, int nwg)
{
    const cx<double> be = {bre, bim}, om = {ore, oim};
    SITE_STRIDE_W(i)
    {
        const int l = (int)(i >> g.lbvol), s = (int)(i & (g.bvol - 1));
        Spinor<float> ps;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long long o = elem(g, l, s, 12, a * 3 + c);
                const cx<double> pv = Elem<1>::get(r, g, o) + be * (Elem<1>::get(p, g, o) - om * Elem<1>::get(q, g, o));
                Elem<1>::put(p, g, o, pv);
                ps.v[a][c] = {(float)pv.re, (float)pv.im};
            }
        p16.store(g, l, s, ps);
    }
}

__global__ void __launch_bounds__(BLAS_WG) k_pupdate_h(Geom g, SpinorField<1> p, SpinorField<1> r, SpinorField<1> q,
                                                       SpinorField<2> p16, double bre, double bim, double ore, double oim)
{
    pupdate_h_body(g, p, r, q, p16, bre, bim, ore, oim, blockIdx.x, gridDim.x);
}

// The vector kernels of the lockstep multi-lattice solver, one launch for the lattices of a
// table (each with its own fields, coefficients, workgroups and partials)
template <int KIND>
__global__ void __launch_bounds__(BLAS_WG) k_blas_multi(MultiBlasTab t, double *partials)
{
    int k = 0;
    while (k + 1 < t.n && (int)blockIdx.x >= t.e[k + 1].item0) ++k;
    const MultiBlasLat &L = t.e[k];
    const Geom &g = L.g;
    const int wid = (int)blockIdx.x - L.item0, nwg = L.nwg;
    double *pp = partials + L.poff;
    auto f1 = [&](int i) { return SpinorField<1>{(float2 *)L.v[i]}; };
    auto f2 = [&](int i) {
        return SpinorField<2>{(__half2 *)L.v[i], (float *)((char *)L.v[i] + 12 * g.V * sizeof(__half2))};
    };
    if constexpr (KIND == BLAS_DOT)
        dot_body<1, 1, 2>(g, f1(0), f1(1), pp, wid, nwg);
    else if constexpr (KIND == BLAS_DOT_NORM)
        dot_body<1, 1, 3>(g, f1(0), f1(1), pp, wid, nwg);
    else if constexpr (KIND == BLAS_UPDATE1_H)
        update1_h_body(g, f1(0), f1(1), f2(2), L.c[0], L.c[1], pp, wid, nwg);
    else if constexpr (KIND == BLAS_UPDATE2_MM)
        update2_mm_body<2>(g, f1(0), f2(1), f2(2), f1(3), f1(4), f1(5), L.c[0], L.c[1], L.c[2], L.c[3], pp, wid, nwg);
    else
        pupdate_h_body(g, f1(0), f1(1), f1(2), f2(3), L.c[0], L.c[1], L.c[2], L.c[3], wid, nwg);
}

// per lattice of a table: out[3 slot + q] = sum_w partials[poff + w nv + q], one workgroup
// per lattice, the fixed order of k_finalize
struct MultiFin {
    long long poff[MULTI_BLAS_MAX];
    int nwg[MULTI_BLAS_MAX], slot[MULTI_BLAS_MAX];
};

__global__ void __launch_bounds__(256) k_finalize_multi(MultiFin f, const double *partials, int nv, double *out)
{
    __shared__ double sh[256];
    const int k = blockIdx.x;
    const double *pp = partials + f.poff[k];
    for (int q = 0; q < nv; ++q) {
        double t = 0;
        for (int w = threadIdx.x; w < f.nwg[k]; w += 256) t += pp[(long long)w * nv + q];
        sh[threadIdx.x] = t;
        wg_barrier();
        for (int h = 128; h >= 1; h >>= 1) {
            if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
            wg_barrier();
        }
        if (threadIdx.x == 0) out[3 * f.slot[k] + q] = sh[0];
        wg_barrier();
    }
}

// x += alpha y (complex alpha)
template <int PY>
__global__ void __launch_bounds__(BLAS_WG) k_caxpy(Geom g, SpinorField<1> x, SpinorField<PY> y, double are, double aim)
{
    const cx<double> al = {are, aim};
    GRID_STRIDE(o, 12 * g.V) Elem<1>::put(x, g, o, Elem<1>::get(x, g, o) + al * Elem<PY>::get(y, g, o));
}

// y = a (copy with precision conversion; FP16 targets go through a per-site kernel)
template <int PA, int PY>
__global__ void __launch_bounds__(BLAS_WG) k_copy(Geom g, SpinorField<PY> y, SpinorField<PA> a)
{
    GRID_STRIDE(o, 12 * g.V) Elem<PY>::put(y, g, o, Elem<PA>::get(a, g, o));
}

// y = alpha a + beta y (real coefficients)
template <int PA, int PY>
__global__ void __launch_bounds__(BLAS_WG) k_axpby(Geom g, double alpha, SpinorField<PA> a, double beta, SpinorField<PY> y)
{
    GRID_STRIDE(o, 12 * g.V)
    {
        cx<double> yv = beta == 0.0 ? cx<double>{0, 0} : Elem<PY>::get(y, g, o);
        Elem<PY>::put(y, g, o, alpha * Elem<PA>::get(a, g, o) + beta * yv);
    }
}

// r = b - a ; partial |r|^2
template <int P>
__global__ void __launch_bounds__(BLAS_WG) k_sub_norm(Geom g, SpinorField<P> r, SpinorField<P> b, SpinorField<P> a,
                                                      double *partials)
{
    double v[1] = {0};
    GRID_STRIDE(o, 12 * g.V)
    {
        cx<double> d = Elem<P>::get(b, g, o) - Elem<P>::get(a, g, o);
        Elem<P>::put(r, g, o, d);
        v[0] += norm2(d);
    }
    wg_reduce_store<1>(v, partials);
}

// per-site conversion into another storage precision (any target, FP16 included)
template <int PA, int PY>
__global__ void __launch_bounds__(256) k_convert(Geom g, SpinorField<PY> y, SpinorField<PA> a)
{
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= g.V) return;
    int l = (int)(i >> g.lbvol), s = (int)(i & (g.bvol - 1));
    Spinor<float> x;
    a.load(g, l, s, x);
    y.store(g, l, s, x);
}

// c = C_inv (scale * r): the inner source of the defect correction, C_inv in FP32
template <int PR>
__global__ void __launch_bounds__(256) k_cinv_src(Geom g, SpinorField<1> c, SpinorField<PR> r, CloverField<1> Ci,
                                                  double scale)
{
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= g.V) return;
    int l = (int)(i >> g.lbvol), s = (int)(i & (g.bvol - 1));
    Spinor<double> x;
    r.load(g, l, s, x);
    Spinor<float> xf, o;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) xf.v[a][cc] = {(float)(scale * x.v[a][cc].re), (float)(scale * x.v[a][cc].im)};
    Clov<float> cl;
    Ci.load(g, l, s, cl);
    clover_mul(cl, xf, o);
    c.store(g, l, s, o);
}



// load a spinor from a raw field pointer at precision P
template <int P> DD_INL void sf_load(void *p, const Geom &g, int l, int s, Spinor<float> &x);
template <> DD_INL void sf_load<1>(void *p, const Geom &g, int l, int s, Spinor<float> &x)
{
    SpinorField<1>{(float2 *)p}.load(g, l, s, x);
}
template <> DD_INL void sf_load<2>(void *p, const Geom &g, int l, int s, Spinor<float> &x)
{
    SpinorField<2>{(__half2 *)p, (float *)((char *)p + 12 * g.V * sizeof(__half2))}.load(g, l, s, x);
}

// ------------------------------------------------------------ flexible GCR kernels
// The k previous images z_j are FP32 fields passed by value (pointer set); the
// reductions accumulate in FP64 like every other reduction here.

template <int NV> DD_INL void wg_reduce_store_dyn(double (&v)[NV], int nv, double *partials)
{
    __shared__ double red[NV][BLAS_WG / 64];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        if (q >= nv) break;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int q = 0; q < nv; ++q) red[q][wave] = v[q];
    wg_barrier();
    if (threadIdx.x == 0)
        for (int q = 0; q < nv; ++q) {
            double t = 0;
            for (int w = 0; w < BLAS_WG / 64; ++w) t += red[q][w];
            partials[(long long)blockIdx.x * nv + q] = t;
        }
}

// <z_j | z> for j < k; T2 = float2 (GCR images) or double2 (the FP64 basis of flexible GMRES)
template <typename T2>
__global__ void __launch_bounds__(BLAS_WG) k_multidot(Geom g, VecSet zs, int k, const T2 *z, double *partials)
{
    double v[2 * GCR_MAX_NKV];
#pragma unroll
    for (int q = 0; q < 2 * GCR_MAX_NKV; ++q) v[q] = 0;
    GRID_STRIDE(o, 12 * g.V)
    {
        const T2 zo = z[o];
#pragma unroll
        for (int j = 0; j < GCR_MAX_NKV; ++j) {
            if (j >= k) break;
            const T2 a = ((const T2 *)zs.v[j])[o];
            v[2 * j] += (double)a.x * zo.x + (double)a.y * zo.y;
            v[2 * j + 1] += (double)a.x * zo.y - (double)a.y * zo.x;
        }
    }
    wg_reduce_store_dyn<2 * GCR_MAX_NKV>(v, 2 * k, partials);
}

// ------------------------------------------------------------ flexible GMRES (FP64 basis)

// w -= sum_j coef_j v_j (j < k, FP64); partial |w|^2
__global__ void __launch_bounds__(BLAS_WG) k_orth64(Geom g, VecSet vs, int k, double2 *w, double *partials)
{
    double v[1] = {0};
    GRID_STRIDE(o, 12 * g.V)
    {
        double2 wo = w[o];
        for (int j = 0; j < k; ++j) {
            const double2 a = ((const double2 *)vs.v[j])[o];
            wo.x -= vs.re[j] * a.x - vs.im[j] * a.y;
            wo.y -= vs.re[j] * a.y + vs.im[j] * a.x;
        }
        w[o] = wo;
        v[0] += wo.x * wo.x + wo.y * wo.y;
    }
    wg_reduce_store<1>(v, partials);
}

// x (FP64) += sum_j coef_j z_j (j < k, FP32)
__global__ void __launch_bounds__(BLAS_WG) k_multi_axpy64(Geom g, VecSet zs, int k, double2 *x)
{
    GRID_STRIDE(o, 12 * g.V)
    {
        double2 xo = x[o];
        for (int j = 0; j < k; ++j) {
            const float2 a = ((const float2 *)zs.v[j])[o];
            xo.x += zs.re[j] * a.x - zs.im[j] * a.y;
            xo.y += zs.re[j] * a.y + zs.im[j] * a.x;
        }
        x[o] = xo;
    }
}

__global__ void __launch_bounds__(BLAS_WG)
    k_gcr_orth(Geom g, VecSet zs, int k, float2 *z, const float2 *r, double *partials)
{
    double v[3] = {0, 0, 0};
    GRID_STRIDE(o, 12 * g.V)
    {
        float2 zo = z[o];
        double zr = zo.x, zi = zo.y;
        for (int j = 0; j < k; ++j) {
            const float2 a = ((const float2 *)zs.v[j])[o];
            zr -= zs.re[j] * a.x - zs.im[j] * a.y;
            zi -= zs.re[j] * a.y + zs.im[j] * a.x;
        }
        zo = make_float2((float)zr, (float)zi);
        z[o] = zo;
        const float2 ro = r[o];
        v[0] += (double)zo.x * zo.x + (double)zo.y * zo.y;
        v[1] += (double)zo.x * ro.x + (double)zo.y * ro.y;
        v[2] += (double)zo.x * ro.y - (double)zo.y * ro.x;
    }
    wg_reduce_store<3>(v, partials);
}

__global__ void __launch_bounds__(BLAS_WG)
    k_gcr_rupdate(Geom g, float2 *z, float2 *r, double inv_bn, double cre, double cim, double *partials)
{
    double v[1] = {0};
    GRID_STRIDE(o, 12 * g.V)
    {
        float2 zo = z[o];
        const double zr = zo.x * inv_bn, zi = zo.y * inv_bn;
        z[o] = make_float2((float)zr, (float)zi);
        float2 ro = r[o];
        ro = make_float2((float)(ro.x - (cre * zr - cim * zi)), (float)(ro.y - (cre * zi + cim * zr)));
        r[o] = ro;
        v[0] += (double)ro.x * ro.x + (double)ro.y * ro.y;
    }
    wg_reduce_store<1>(v, partials);
}

// y += sum_j coef_j p_j, one thread per site (FP16 p_j carry a per-site scale)
template <int PP>
__global__ void __launch_bounds__(256) k_multi_axpy(Geom g, VecSet ps, int k, float2 *y)
{
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= g.V) return;
    int l = (int)(i >> g.lbvol), s = (int)(i & (g.bvol - 1));
    double acc[12][2];
    for (int e = 0; e < 12; ++e) {
        float2 t = y[elem(g, l, s, 12, e)];
        acc[e][0] = t.x;
        acc[e][1] = t.y;
    }
    for (int j = 0; j < k; ++j) {
        Spinor<float> p;
        sf_load<PP>(ps.v[j], g, l, s, p);
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 3; ++c) {
                const int e = a * 3 + c;
                acc[e][0] += ps.re[j] * p.v[a][c].re - ps.im[j] * p.v[a][c].im;
                acc[e][1] += ps.re[j] * p.v[a][c].im + ps.im[j] * p.v[a][c].re;
            }
    }
    for (int e = 0; e < 12; ++e) y[elem(g, l, s, 12, e)] = make_float2((float)acc[e][0], (float)acc[e][1]);
}

// ============================================================ host launchers

static inline int grid_sites(long long V, int wg) { return (int)((V + wg - 1) / wg); }

template <int P> static SpinorField<P> sf(void *p, const Geom &g);
template <> SpinorField<0> sf<0>(void *p, const Geom &) { return SpinorField<0>{(double2 *)p}; }
template <> SpinorField<1> sf<1>(void *p, const Geom &) { return SpinorField<1>{(float2 *)p}; }
template <> SpinorField<2> sf<2>(void *p, const Geom &g)
{
    return SpinorField<2>{(__half2 *)p, (float *)((char *)p + 12 * g.V * sizeof(__half2))};
}

#define DISPATCH_P(P, ...)                                    \
    switch (P) {                                              \
    case 0: { constexpr int P_ = 0; __VA_ARGS__; } break;     \
    case 1: { constexpr int P_ = 1; __VA_ARGS__; } break;     \
    default: { constexpr int P_ = 2; __VA_ARGS__; } break;    \
    }

hipError_t launch_pack_spinor(const Geom &g, hipStream_t st, int prec, void *dst, const void *src, bool g5)
{
    DISPATCH_P(prec, hipLaunchKernelGGL(k_pack_spinor<P_>, dim3(grid_sites(g.V, 256)), dim3(256), 0, st, g,
                                        sf<P_>(dst, g), (const double2 *)src, (int)g5));
    return hipGetLastError();
}

hipError_t launch_unpack_spinor(const Geom &g, hipStream_t st, int prec, void *dst, const void *src, bool g5)
{
    DISPATCH_P(prec, hipLaunchKernelGGL(k_unpack_spinor<P_>, dim3(grid_sites(g.V, 256)), dim3(256), 0, st, g,
                                        (double2 *)dst, sf<P_>((void *)src, g), (int)g5));
    return hipGetLastError();
}

hipError_t launch_pack_links(const Geom &g, hipStream_t st, const void *src, void *u64, void *u32, void *u16, int *bad)
{
    hipLaunchKernelGGL(k_pack_links, dim3(grid_sites(g.V, 256)), dim3(256), 0, st, g, (const double2 *)src,
                       (double2 *)u64, (float2 *)u32, (__half2 *)u16, bad);
    return hipGetLastError();
}

hipError_t launch_clover(const Geom &g, hipStream_t st, const void *u64, const SigmaBlocks &sig, double kcsw,
                         void *clov64, void *cinv32, void *cinv16, int *bad)
{
    hipLaunchKernelGGL(k_clover, dim3(grid_sites(g.V, 64)), dim3(64), 0, st, g, (const double2 *)u64, sig, kcsw,
                       (double2 *)clov64, (float2 *)cinv32, (__half2 *)cinv16, bad);
    return hipGetLastError();
}

// blocks per workgroup of the t-streamed apply, 0 for a block per workgroup: 2 (the blocks in t
// are even) as long as that leaves 1024 workgroups (four per CU) to fill the chip; smaller
// lattices keep a block per workgroup.  Measured on 64^3x128 with the z-pair column order: walks
// of 2 beat 4 (FP64 D by 2 %, the others by up to 0.5 %) and 8; longer walks let the workgroups
// of neighbouring columns drift apart.
static int dirac_stream_len(const Geom &g)
{
    return g.nblk / 2 >= 1024 ? 2 : 0;
}

// one operator / precision combination: the t-streamed kernel where dirac_stream_len allows it
// (not for the all-FP16 operator, whose faces are small: there the block-per-workgroup kernel
// holds more wavefronts per SIMD), else one block per workgroup, specialised for 4^4 blocks
// except in FP64 (which gains nothing from it)
template <int PIN, int POUT, int PG, int OP>
static void dirac_launch(const Geom &g, hipStream_t st, const DiracArgs &a, bool cube4, int ns)
{
    const SpinorField<POUT> out = sf<POUT>(a.out, g);
    const SpinorField<PIN> in = sf<PIN>((void *)a.in, g);
    const LinkField<PG> U{(decltype(LinkField<PG>::p))a.links};
    const CloverField<PG> C{(decltype(CloverField<PG>::p))a.clover};
    if constexpr (PG != 2) {
        if (ns > 1) {
            hipLaunchKernelGGL((k_dirac_ts<PIN, POUT, PG, OP>), dim3(g.nblk / ns), dim3(256), 0, st, g, out, in, U, C,
                               a.phase, a.kappa, ns);
            return;
        }
    }
    const dim3 grid(grid_sites(g.V, 256));
    if (cube4)
        hipLaunchKernelGGL((k_dirac<PIN, POUT, PG, OP, (PG != 0 ? 4 : 0)>), grid, dim3(256), 0, st, g, out, in, U, C,
                           a.phase, a.kappa);
    else
        hipLaunchKernelGGL((k_dirac<PIN, POUT, PG, OP, 0>), grid, dim3(256), 0, st, g, out, in, U, C, a.phase, a.kappa);
}

hipError_t launch_dirac(const Geom &g, hipStream_t st, const DiracArgs &a)
{
    const bool cube4 = g.b[0] == 4 && g.b[1] == 4 && g.b[2] == 4 && g.b[3] == 4;
    const int ns = cube4 ? dirac_stream_len(g) : 0;
    if (a.pin == 0 && a.pout == 0 && a.pg == 0) {
        if (a.op == 0)
            dirac_launch<0, 0, 0, 0>(g, st, a, cube4, ns);
        else if (a.op == 2)
            dirac_launch<0, 0, 0, 2>(g, st, a, cube4, ns);
        else
            return hipErrorInvalidValue;
    } else if (a.op != 1) {
        return hipErrorInvalidValue;
    } else if (a.pin == 1 && a.pout == 1 && a.pg == 1) {
        dirac_launch<1, 1, 1, 1>(g, st, a, cube4, ns);
    } else if (a.pin == 2 && a.pout == 1 && a.pg == 1) {
        dirac_launch<2, 1, 1, 1>(g, st, a, cube4, ns);
    } else if (a.pin == 2 && a.pout == 2 && a.pg == 2) {
        dirac_launch<2, 2, 2, 1>(g, st, a, cube4, ns);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dirac_multi(hipStream_t st, const LatDesc *desc_dev, int nlat, int total, int pin, int *counter)
{
    hipError_t e = hipMemsetAsync(counter, 0, sizeof(int), st);
    if (e != hipSuccess) return e;
    const int nwg = total < 2048 ? total : 2048;
    if (pin == 2)
        hipLaunchKernelGGL(k_dirac_multi<2>, dim3(nwg), dim3(256), 0, st, desc_dev, nlat, total, counter);
    else
        hipLaunchKernelGGL(k_dirac_multi<1>, dim3(nwg), dim3(256), 0, st, desc_dev, nlat, total, counter);
    return hipGetLastError();
}

size_t sap_lds_bytes(const Geom &g, int prec)
{
    size_t link = prec == 1 ? 0 : SapLinks<2>::E * sizeof(__half2);
    return (size_t)g.bvol * (12 * sizeof(float2) + link);
}

hipError_t launch_sap_half(const Geom &g, hipStream_t st, const SapArgs &a, int colour, int flags)
{
    if ((flags & (SAP_AMSAP | SAP_CROSS_ONLY)) && !a.ax) return hipErrorInvalidValue;
    const int nwg = g.nblk / 2;
    const size_t lds = sap_lds_bytes(g, a.prec);
    const bool cube4 = g.b[0] == 4 && g.b[1] == 4 && g.b[2] == 4 && g.b[3] == 4;
    if (a.prec == 1) {
        hipLaunchKernelGGL((cube4 ? k_sap_half<1, 4> : k_sap_half<1, 0>), dim3(nwg), dim3(g.bvol), lds, st, g, colour, flags, sf<1>((void *)a.b, g),
                           sf<1>(a.s, g), sf<1>(a.x, g), SapLinks<1>{LinkField<1>{(const float2 *)a.links}},
                           LinkField<1>{(const float2 *)a.links}, CloverField<1>{(const float2 *)a.cinv}, a.phase,
                           (float)a.kappa, a.n_jac, sf<1>(a.ax, g));
    } else if (a.prec == 2) {
        hipLaunchKernelGGL((cube4 ? k_sap_half<2, 4> : k_sap_half<2, 0>), dim3(nwg), dim3(g.bvol), lds, st, g, colour, flags, sf<2>((void *)a.b, g),
                           sf<2>(a.s, g), sf<2>(a.x, g), SapLinks<2>{(const __half2 *)a.links},
                           LinkField<2>{(const __half2 *)a.links}, CloverField<2>{(const __half2 *)a.cinv}, a.phase,
                           (float)a.kappa, a.n_jac, sf<2>(a.ax, g));
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int blas_grid(const Geom &g)
{
    long long n = (12 * g.V + BLAS_WG - 1) / BLAS_WG;
    return (int)(n < BLAS_MAX_WG ? n : BLAS_MAX_WG);
}

int blas_grid_sites(const Geom &g)
{
    long long n = (g.V + BLAS_WG - 1) / BLAS_WG;
    return (int)(n < BLAS_MAX_WG ? n : BLAS_MAX_WG);
}

hipError_t launch_finalize(hipStream_t st, const double *partials, int nwg, int nv, double *out)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, partials, nwg, nv, out);
    return hipGetLastError();
}

hipError_t launch_blas_multi(hipStream_t st, int kind, const MultiBlasTab &t, int total, double *partials)
{
    if (t.n <= 0 || t.n > MULTI_BLAS_MAX || total <= 0) return hipErrorInvalidValue;
    const dim3 G(total), B(BLAS_WG);
    switch (kind) {
    case BLAS_DOT: hipLaunchKernelGGL(k_blas_multi<BLAS_DOT>, G, B, 0, st, t, partials); break;
    case BLAS_DOT_NORM: hipLaunchKernelGGL(k_blas_multi<BLAS_DOT_NORM>, G, B, 0, st, t, partials); break;
    case BLAS_UPDATE1_H: hipLaunchKernelGGL(k_blas_multi<BLAS_UPDATE1_H>, G, B, 0, st, t, partials); break;
    case BLAS_UPDATE2_MM: hipLaunchKernelGGL(k_blas_multi<BLAS_UPDATE2_MM>, G, B, 0, st, t, partials); break;
    case BLAS_PUPDATE_H: hipLaunchKernelGGL(k_blas_multi<BLAS_PUPDATE_H>, G, B, 0, st, t, partials); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_finalize_multi(hipStream_t st, const MultiBlasTab &t, const int *slot, const double *partials, int nv,
                                 double *out)
{
    if (t.n <= 0 || t.n > MULTI_BLAS_MAX || nv < 1 || nv > 3) return hipErrorInvalidValue;
    MultiFin f{};
    for (int k = 0; k < t.n; ++k) {
        f.poff[k] = t.e[k].poff;
        f.nwg[k] = t.e[k].nwg;
        f.slot[k] = slot[k];
    }
    hipLaunchKernelGGL(k_finalize_multi, dim3(t.n), dim3(256), 0, st, f, partials, nv, out);
    return hipGetLastError();
}

hipError_t launch_blas(const Geom &g, hipStream_t st, const BlasArgs &a)
{
    const int nwg = blas_grid(g);
    const dim3 G(nwg), B(BLAS_WG);
    switch (a.kind) {
    case BLAS_DOT:  // <v0|v1>, precisions p0 == p1
        DISPATCH_P(a.p[0], hipLaunchKernelGGL((k_dot<P_, P_, 2>), G, B, 0, st, g, sf<P_>(a.v[0], g),
                                              sf<P_>(a.v[1], g), a.partials));
        break;
    case BLAS_DOT_NORM:  // <v0|v1>, |v0|^2
        DISPATCH_P(a.p[0], hipLaunchKernelGGL((k_dot<P_, P_, 3>), G, B, 0, st, g, sf<P_>(a.v[0], g),
                                              sf<P_>(a.v[1], g), a.partials));
        break;
    case BLAS_NORM2:
        DISPATCH_P(a.p[0], hipLaunchKernelGGL((k_norm2<P_>), G, B, 0, st, g, sf<P_>(a.v[0], g), a.partials));
        break;
    case BLAS_UPDATE1:  // v0 += c0 v1 ; v2 -= c0 v3   (p0 = x, p1 = y, p2 = r/q)
        if (a.p[0] == 0 && a.p[1] == 0 && a.p[2] == 0)
            hipLaunchKernelGGL((k_update1<0, 0, 0>), G, B, 0, st, g, sf<0>(a.v[0], g), sf<0>(a.v[1], g),
                               sf<0>(a.v[2], g), sf<0>(a.v[3], g), a.c[0], a.c[1], a.partials);
        else if (a.p[0] == 1 && a.p[1] == 1 && a.p[2] == 1)
            hipLaunchKernelGGL((k_update1<1, 1, 1>), G, B, 0, st, g, sf<1>(a.v[0], g), sf<1>(a.v[1], g),
                               sf<1>(a.v[2], g), sf<1>(a.v[3], g), a.c[0], a.c[1], a.partials);
        else if (a.p[0] == 1 && a.p[1] == 2 && a.p[2] == 1)
            hipLaunchKernelGGL((k_update1<1, 2, 1>), G, B, 0, st, g, sf<1>(a.v[0], g), sf<2>(a.v[1], g),
                               sf<1>(a.v[2], g), sf<1>(a.v[3], g), a.c[0], a.c[1], a.partials);
        else
            return hipErrorInvalidValue;
        break;
    case BLAS_UPDATE2:  // v0 += c0 v1 ; v2 -= c0 v3 ; <v4|v2>
        if (a.p[0] == 0 && a.p[1] == 0 && a.p[2] == 0)
            hipLaunchKernelGGL((k_update2<0, 0, 0>), G, B, 0, st, g, sf<0>(a.v[0], g), sf<0>(a.v[1], g),
                               sf<0>(a.v[2], g), sf<0>(a.v[3], g), sf<0>(a.v[4], g), a.c[0], a.c[1], a.partials);
        else if (a.p[0] == 1 && a.p[1] == 1 && a.p[2] == 1)
            hipLaunchKernelGGL((k_update2<1, 1, 1>), G, B, 0, st, g, sf<1>(a.v[0], g), sf<1>(a.v[1], g),
                               sf<1>(a.v[2], g), sf<1>(a.v[3], g), sf<1>(a.v[4], g), a.c[0], a.c[1], a.partials);
        else if (a.p[0] == 1 && a.p[1] == 2 && a.p[2] == 1)
            hipLaunchKernelGGL((k_update2<1, 2, 1>), G, B, 0, st, g, sf<1>(a.v[0], g), sf<2>(a.v[1], g),
                               sf<1>(a.v[2], g), sf<1>(a.v[3], g), sf<1>(a.v[4], g), a.c[0], a.c[1], a.partials);
        else
            return hipErrorInvalidValue;
        break;
    case BLAS_PUPDATE:  // v0 = v1 + c01 (v0 - c23 v2)
        DISPATCH_P(a.p[0], if (P_ == 2) return hipErrorInvalidValue;
                   hipLaunchKernelGGL((k_pupdate<P_ == 2 ? 1 : P_>), G, B, 0, st, g, sf<P_ == 2 ? 1 : P_>(a.v[0], g),
                                      sf<P_ == 2 ? 1 : P_>(a.v[1], g), sf<P_ == 2 ? 1 : P_>(a.v[2], g), a.c[0],
                                      a.c[1], a.c[2], a.c[3]));
        break;
    case BLAS_AXPBY:  // v1 = c0 v0 + c1 v1 (p0 source, p1 target in {0, 1})
        if (a.p[0] == 1 && a.p[1] == 0)
            hipLaunchKernelGGL((k_axpby<1, 0>), G, B, 0, st, g, a.c[0], sf<1>(a.v[0], g), a.c[1], sf<0>(a.v[1], g));
        else if (a.p[0] == 0 && a.p[1] == 0)
            hipLaunchKernelGGL((k_axpby<0, 0>), G, B, 0, st, g, a.c[0], sf<0>(a.v[0], g), a.c[1], sf<0>(a.v[1], g));
        else if (a.p[0] == 1 && a.p[1] == 1)
            hipLaunchKernelGGL((k_axpby<1, 1>), G, B, 0, st, g, a.c[0], sf<1>(a.v[0], g), a.c[1], sf<1>(a.v[1], g));
        else if (a.p[0] == 0 && a.p[1] == 1)
            hipLaunchKernelGGL((k_axpby<0, 1>), G, B, 0, st, g, a.c[0], sf<0>(a.v[0], g), a.c[1], sf<1>(a.v[1], g));
        else
            return hipErrorInvalidValue;
        break;
    case BLAS_SUB_NORM:  // v0 = v1 - v2 ; |v0|^2 (FP64)
        hipLaunchKernelGGL((k_sub_norm<0>), G, B, 0, st, g, sf<0>(a.v[0], g), sf<0>(a.v[1], g), sf<0>(a.v[2], g),
                           a.partials);
        break;
    case BLAS_CONVERT: {  // v1 = v0 with precisions p0 -> p1 (per site)
        const dim3 Gs(grid_sites(g.V, 256)), Bs(256);
        if (a.p[0] == 1 && a.p[1] == 2)
            hipLaunchKernelGGL((k_convert<1, 2>), Gs, Bs, 0, st, g, sf<2>(a.v[1], g), sf<1>(a.v[0], g));
        else if (a.p[0] == 2 && a.p[1] == 1)
            hipLaunchKernelGGL((k_convert<2, 1>), Gs, Bs, 0, st, g, sf<1>(a.v[1], g), sf<2>(a.v[0], g));
        else if (a.p[0] == 0 && a.p[1] == 1)
            hipLaunchKernelGGL((k_convert<0, 1>), Gs, Bs, 0, st, g, sf<1>(a.v[1], g), sf<0>(a.v[0], g));
        else if (a.p[0] == 1 && a.p[1] == 0)
            hipLaunchKernelGGL((k_convert<1, 0>), Gs, Bs, 0, st, g, sf<0>(a.v[1], g), sf<1>(a.v[0], g));
        else
            return hipErrorInvalidValue;
        break;
    }
    case BLAS_CINV_SRC: {  // v0 (FP32) = C_inv (c0 * v1), v1 at precision p1
        const dim3 Gs(grid_sites(g.V, 256)), Bs(256);
        if (a.p[1] == 0)
            hipLaunchKernelGGL((k_cinv_src<0>), Gs, Bs, 0, st, g, sf<1>(a.v[0], g), sf<0>(a.v[1], g),
                               CloverField<1>{(const float2 *)a.v[2]}, a.c[0]);
        else
            return hipErrorInvalidValue;
        break;
    }
    case BLAS_UPDATE1_H:  // r -= c01 q ; |r|^2 ; v2 = r (FP16)
        hipLaunchKernelGGL(k_update1_h, G, B, 0, st, g, sf<1>(a.v[0], g), sf<1>(a.v[1], g), sf<2>(a.v[2], g), a.c[0],
                           a.c[1], a.partials);
        break;
    case BLAS_UPDATE2_MM:  // y += c01 v1 + c23 v2 ; r -= c23 t ; |r|^2, <rt|r>
        if (a.p[1] == 2)
            hipLaunchKernelGGL((k_update2_mm<2>), G, B, 0, st, g, sf<1>(a.v[0], g), sf<2>(a.v[1], g), sf<2>(a.v[2], g),
                               sf<1>(a.v[3], g), sf<1>(a.v[4], g), sf<1>(a.v[5], g), a.c[0], a.c[1], a.c[2], a.c[3],
                               a.partials);
        else if (a.p[1] == 1)
            hipLaunchKernelGGL((k_update2_mm<1>), G, B, 0, st, g, sf<1>(a.v[0], g), sf<1>(a.v[1], g), sf<1>(a.v[2], g),
                               sf<1>(a.v[3], g), sf<1>(a.v[4], g), sf<1>(a.v[5], g), a.c[0], a.c[1], a.c[2], a.c[3],
                               a.partials);
        else
            return hipErrorInvalidValue;
        break;
    case BLAS_PUPDATE_H:  // p = r + c01 (p - c23 q) ; v3 = p (FP16)
        hipLaunchKernelGGL(k_pupdate_h, G, B, 0, st, g, sf<1>(a.v[0], g), sf<1>(a.v[1], g), sf<1>(a.v[2], g),
                           sf<2>(a.v[3], g), a.c[0], a.c[1], a.c[2], a.c[3]);
        break;
    case BLAS_CAXPY:  // v0 += c01 v1
        if (a.p[1] == 2)
            hipLaunchKernelGGL((k_caxpy<2>), G, B, 0, st, g, sf<1>(a.v[0], g), sf<2>(a.v[1], g), a.c[0], a.c[1]);
        else if (a.p[1] == 1)
            hipLaunchKernelGGL((k_caxpy<1>), G, B, 0, st, g, sf<1>(a.v[0], g), sf<1>(a.v[1], g), a.c[0], a.c[1]);
        else
            return hipErrorInvalidValue;
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_multidot(const Geom &g, hipStream_t st, const VecSet &zs, int k, void *z, double *partials, int prec)
{
    if (k < 1 || k > GCR_MAX_NKV) return hipErrorInvalidValue;
    if (prec == 0)
        hipLaunchKernelGGL(k_multidot<double2>, dim3(blas_grid(g)), dim3(BLAS_WG), 0, st, g, zs, k, (const double2 *)z,
                           partials);
    else if (prec == 1)
        hipLaunchKernelGGL(k_multidot<float2>, dim3(blas_grid(g)), dim3(BLAS_WG), 0, st, g, zs, k, (const float2 *)z,
                           partials);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_orth64(const Geom &g, hipStream_t st, const VecSet &vs, int k, void *w, double *partials)
{
    if (k < 0 || k > GCR_MAX_NKV) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_orth64, dim3(blas_grid(g)), dim3(BLAS_WG), 0, st, g, vs, k, (double2 *)w, partials);
    return hipGetLastError();
}

hipError_t launch_multi_axpy64(const Geom &g, hipStream_t st, const VecSet &zs, int k, void *x)
{
    if (k < 1 || k > GCR_MAX_NKV) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_multi_axpy64, dim3(blas_grid(g)), dim3(BLAS_WG), 0, st, g, zs, k, (double2 *)x);
    return hipGetLastError();
}

hipError_t launch_gcr_orth(const Geom &g, hipStream_t st, const VecSet &zs, int k, void *z, void *r, double *partials)
{
    if (k < 0 || k > GCR_MAX_NKV) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gcr_orth, dim3(blas_grid(g)), dim3(BLAS_WG), 0, st, g, zs, k, (float2 *)z,
                       (const float2 *)r, partials);
    return hipGetLastError();
}

hipError_t launch_gcr_rupdate(const Geom &g, hipStream_t st, void *z, void *r, double inv_bn, double cre, double cim,
                              double *partials)
{
    hipLaunchKernelGGL(k_gcr_rupdate, dim3(blas_grid(g)), dim3(BLAS_WG), 0, st, g, (float2 *)z, (float2 *)r, inv_bn,
                       cre, cim, partials);
    return hipGetLastError();
}

hipError_t launch_multi_axpy(const Geom &g, hipStream_t st, const VecSet &ps, int k, int pp, void *y)
{
    if (k < 1 || k > GCR_MAX_NKV) return hipErrorInvalidValue;
    const dim3 G(grid_sites(g.V, 256)), B(256);
    if (pp == 2)
        hipLaunchKernelGGL(k_multi_axpy<2>, G, B, 0, st, g, ps, k, (float2 *)y);
    else if (pp == 1)
        hipLaunchKernelGGL(k_multi_axpy<1>, G, B, 0, st, g, ps, k, (float2 *)y);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace dd
