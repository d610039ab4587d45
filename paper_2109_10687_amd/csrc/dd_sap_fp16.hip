// dd_sap_fp16.hip -- SAP half-sweep (Alg. 1 with the Jacobi of Alg. 2) with
// FP16 storage and packed FP16 arithmetic.
//
// The block-local work of a half-sweep is N_JAC + 1 applications of
// K = kappa C_inv H_in, all inside one workgroup.  Here every spinor is kept in
// "pair form": for each colour c the spin pairs (psi0, psi1) and (psi2, psi3)
// are two complex pairs, each stored as two half2 (real parts, imaginary
// parts).  A spin-projected half spinor is then one complex pair per colour, so
// a link entry, broadcast to both halves, multiplies both spins of the half
// spinor in one packed FMA: a hop's two 3x3 complex products take 36 packed
// FMAs.  The clover block (two 6x6 Hermitian blocks in the gamma_5-diagonal
// basis) is rearranged once per gauge field, from its FP16 storage, into pair
// coefficients (k_sap_prep),
//   w_pair[c] = sum_c' A[c][c'] (.) z_pair[c'] + B[c][c'] (.) swap(z_pair[c']).
// The cross-block term of Alg. 1 (the neighbouring blocks' x_{c'} hopping into
// the block) travels between half-sweeps as face hop terms: each half-sweep leaves,
// at the faces of its blocks, the projected half spinors of its result (multiplied
// by its own link for the hops that run backwards into the neighbour), straight
// from LDS in packed FP16, and the next half-sweep of the other colour reads them
// instead of its neighbours' whole spinors and links.  x itself is written only by
// the last two half-sweeps (the preconditioner's output).  With h = H_{c c'} x_{c'}
// the updated source x0 = s_c + kappa C_inv h takes one clover product (it is the
// first Jacobi step, from x = 0), and every later step is x <- x0 + kappa C_inv H_in x,
// which equals s_c + kappa C_inv (H_in x + h).  The face terms are summed per site in
// FP32 (each neighbouring block has its own scale).  FP16 range: the block's
// source and h are scaled by 1 / max|component| before the sweeps (the sweeps
// are linear) and the result is scaled back in FP32; the final s update of
// Alg. 1 is evaluated in FP32.
#include "dd_device.h"
#include "dd_launch.h"

namespace dd {

typedef __half2 h2;

struct PC {  // a pair of complex numbers: re = (z0.re, z1.re), im = (z0.im, z1.im)
    h2 re, im;
};
struct SpH {  // spinor in pair form: u[c] = (psi0, psi1)[c], l[c] = (psi2, psi3)[c]
    PC u[3], l[3];
};

DD_INL h2 lo2(h2 a) { return __low2half2(a); }
DD_INL h2 hi2(h2 a) { return __high2half2(a); }
DD_INL h2 swp(h2 a) { return __lowhigh2highlow(a); }
DD_INL h2 fma2(h2 a, h2 b, h2 c) { return __hfma2(a, b, c); }
DD_INL h2 neg2(h2 a) { return __hneg2(a); }
DD_INL h2 add2(h2 a, h2 b) { return __hadd2(a, b); }
DD_INL h2 sub2(h2 a, h2 b) { return __hsub2(a, b); }
DD_INL h2 mul2(h2 a, h2 b) { return __hmul2(a, b); }
DD_INL h2 zero2() { return __float2half2_rn(0.f); }

DD_INL void zero(SpH &s)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) s.u[c] = s.l[c] = PC{zero2(), zero2()};
}

// k = W h for a half spinor in pair form; W = U (dag = false) or U^dagger.
// U[a][b] holds (re, im) in one half2.
DD_INL void mat_pair(const h2 (&U)[3][3], bool dag, const PC (&h)[3], PC (&k)[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        h2 kr = zero2(), ki = zero2();
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const h2 e = dag ? U[b][a] : U[a][b];
            const h2 er = lo2(e), ei = dag ? neg2(hi2(e)) : hi2(e);
            kr = fma2(er, h[b].re, kr);
            kr = fma2(neg2(ei), h[b].im, kr);
            ki = fma2(er, h[b].im, ki);
            ki = fma2(ei, h[b].re, ki);
        }
        k[a] = PC{kr, ki};
    }
}

// half spinor (h0, h1) of (1 - s gamma_mu) p, pair form, for the gamma matrices of the appendix;
// for mu = 3 (gamma_4 diagonal) the surviving spin pair itself: the factor 2 of (1 - s gamma_4)
// is applied when the hop is rebuilt (recon_pair, recon_mix)
DD_INL void proj_pair(int mu, int s, const SpH &p, PC (&h)[3])
{
    const h2 S = __float2half2_rn((float)s);                      // (s, s)
    const h2 Cm = __floats2half2_rn(-(float)s, (float)s);         // (-s, s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (mu == 0) {  // (h0, h1) = (psi0, psi1) - s i (psi3, psi2)
            h[c].re = fma2(S, swp(p.l[c].im), p.u[c].re);
            h[c].im = fma2(neg2(S), swp(p.l[c].re), p.u[c].im);
        } else if (mu == 1) {  // (h0, h1) = (psi0, psi1) + (-s, s) (psi3, psi2)
            h[c].re = fma2(Cm, swp(p.l[c].re), p.u[c].re);
            h[c].im = fma2(Cm, swp(p.l[c].im), p.u[c].im);
        } else if (mu == 2) {  // (h0, h1) = (psi0, psi1) + i (-s, s) (psi2, psi3)
            h[c].re = fma2(neg2(Cm), p.l[c].im, p.u[c].re);
            h[c].im = fma2(Cm, p.l[c].re, p.u[c].im);
        } else {  // gamma_4 diagonal: the surviving spin pair (the factor 2 comes later)
            h[c] = s > 0 ? p.l[c] : p.u[c];
        }
    }
}

// acc += (1 - s gamma_mu) rebuilt from k = W h, pair form
DD_INL void recon_pair(int mu, int s, const PC (&k)[3], SpH &acc)
{
    const h2 S = __float2half2_rn((float)s);                      // (s, s)
    const h2 Cp = __floats2half2_rn((float)s, -(float)s);         // (s, -s)
    const h2 TWO = __float2half2_rn(2.f);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (mu == 3) {  // twice the rebuilt pair (the factor 2 of 1 - s gamma_4, see proj_pair)
            PC &t = s > 0 ? acc.l[c] : acc.u[c];
            t.re = fma2(TWO, k[c].re, t.re);
            t.im = fma2(TWO, k[c].im, t.im);
            continue;
        }
        acc.u[c].re = add2(acc.u[c].re, k[c].re);
        acc.u[c].im = add2(acc.u[c].im, k[c].im);
        if (mu == 0) {  // (acc2, acc3) += s i (k1, k0)
            acc.l[c].re = fma2(neg2(S), swp(k[c].im), acc.l[c].re);
            acc.l[c].im = fma2(S, swp(k[c].re), acc.l[c].im);
        } else if (mu == 1) {  // (acc2, acc3) += (s, -s) (k1, k0)
            acc.l[c].re = fma2(Cp, swp(k[c].re), acc.l[c].re);
            acc.l[c].im = fma2(Cp, swp(k[c].im), acc.l[c].im);
        } else {  // (acc2, acc3) += i (s, -s) (k0, k1)
            acc.l[c].re = fma2(neg2(Cp), k[c].im, acc.l[c].re);
            acc.l[c].im = fma2(Cp, k[c].re, acc.l[c].im);
        }
    }
}

// acc += (1 - s gamma_mu) W psi, pair form
DD_INL void hop_pair(int mu, int s, const h2 (&U)[3][3], const SpH &p, SpH &acc)
{
    PC h[3], k[3];
    proj_pair(mu, s, p, h);
    mat_pair(U, s < 0, h, k);
    recon_pair(mu, s, k, acc);
}

// clover block in pair form.  For chiral block blk with Hermitian 6x6 entries H,
//   A[c][d] = (H(c, d), H(3+c, 3+d)),  B[c][d] = (H(c, 3+d), H(3+c, d))   (lane 0, lane 1)
// and w_pair[c] = sum_d A[c][d] (.) z_pair[d] + B[c][d] (.) swap(z_pair[d]).  Hermiticity
// fixes half of them: A[d][c] = conj(A[c][d]) lane by lane, A[c][c] is real, and
// B[d][c] = conj(swap(B[c][d])), B[c][c] = (w, conj w) with w = H(c, 3+c).  Only the
// diagonal and the upper entries are kept (36 registers instead of 72).
struct ClovPair {
    h2 Ad[2][3];  // real parts of A[c][c]
    PC Au[2][3];  // A[0][1], A[0][2], A[1][2]
    h2 Bd[2][3];  // w = H(c, 3+c) as (re, im)
    PC Bu[2][3];  // B[0][1], B[0][2], B[1][2]
};

DD_INL int upper3(int c, int d) { return c + d - 1; }  // (0,1) -> 0, (0,2) -> 1, (1,2) -> 2

// the pair coefficients of the site's FP16 C_inv (the stored entries are only
// regrouped: no rounding)
DD_INL void clov_pairs_ld(const CloverField<2> &Ci, const Geom &g, int l, int s, ClovPair &P)
{
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        h2 dg[3], up[15];
#pragma unroll
        for (int j = 0; j < 3; ++j) dg[j] = ld_stream(&Ci.p[elem(g, l, s, 36, blk * 18 + j)]);
#pragma unroll
        for (int j = 0; j < 15; ++j) up[j] = ld_stream(&Ci.p[elem(g, l, s, 36, blk * 18 + 3 + j)]);
        auto diag = [&](int i) { return (i & 1) ? __high2half(dg[i >> 1]) : __low2half(dg[i >> 1]); };
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            P.Ad[blk][c] = __halves2half2(diag(c), diag(3 + c));
            P.Bd[blk][c] = up[upper_index(c, 3 + c)];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int d = c + 1; d < 3; ++d) {
                const h2 a = up[upper_index(c, d)], b = up[upper_index(3 + c, 3 + d)];
                P.Au[blk][upper3(c, d)] = PC{__lows2half2(a, b), __highs2half2(a, b)};
                // B[c][d] = (H(c, 3+d), conj H(d, 3+c))
                const h2 e = up[upper_index(c, 3 + d)], f = up[upper_index(d, 3 + c)];
                P.Bu[blk][upper3(c, d)] = PC{__lows2half2(e, f), __halves2half2(__high2half(e), __hneg(__high2half(f)))};
            }
    }
}

// The SAP-ready copy of C_inv holds these coefficients per site, 18 half2 per chiral
// block: Ad[0..2], Au[0..2] (re, im), Bd[0..2], Bu[0..2] (re, im)
DD_INL void clov_pairs_put(__half2 *p, const Geom &g, int l, int s, const ClovPair &P)
{
#pragma unroll
    for (int blk = 0; blk < 2; ++blk)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int o = blk * 18;
            p[elem(g, l, s, 36, o + c)] = P.Ad[blk][c];
            p[elem(g, l, s, 36, o + 3 + 2 * c)] = P.Au[blk][c].re;
            p[elem(g, l, s, 36, o + 4 + 2 * c)] = P.Au[blk][c].im;
            p[elem(g, l, s, 36, o + 9 + c)] = P.Bd[blk][c];
            p[elem(g, l, s, 36, o + 12 + 2 * c)] = P.Bu[blk][c].re;
            p[elem(g, l, s, 36, o + 13 + 2 * c)] = P.Bu[blk][c].im;
        }
}

DD_INL void clov_pairs_get(const __half2 *p, const Geom &g, int l, int s, ClovPair &P)
{
#pragma unroll
    for (int blk = 0; blk < 2; ++blk)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int o = blk * 18;
            P.Ad[blk][c] = ld_stream(&p[elem(g, l, s, 36, o + c)]);
            P.Au[blk][c] = PC{ld_stream(&p[elem(g, l, s, 36, o + 3 + 2 * c)]), ld_stream(&p[elem(g, l, s, 36, o + 4 + 2 * c)])};
            P.Bd[blk][c] = ld_stream(&p[elem(g, l, s, 36, o + 9 + c)]);
            P.Bu[blk][c] = PC{ld_stream(&p[elem(g, l, s, 36, o + 12 + 2 * c)]), ld_stream(&p[elem(g, l, s, 36, o + 13 + 2 * c)])};
        }
}

// (a (.) z): complex product lane by lane, accumulated into r
DD_INL void cmac_pair(const PC &a, const PC &z, PC &r)
{
    r.re = fma2(a.re, z.re, r.re);
    r.re = fma2(neg2(a.im), z.im, r.re);
    r.im = fma2(a.re, z.im, r.im);
    r.im = fma2(a.im, z.re, r.im);
}

// r += conj(a) (.) z lane by lane
DD_INL void cmac_pair_conj(const PC &a, const PC &z, PC &r)
{
    r.re = fma2(a.re, z.re, r.re);
    r.re = fma2(a.im, z.im, r.re);
    r.im = fma2(a.re, z.im, r.im);
    r.im = fma2(neg2(a.im), z.re, r.im);
}

// out = Q diag(N+, N-) Q in, pair form (Q = [[1, 1], [1, -1]] on the spin pairs)
DD_INL void clover_pair(const ClovPair &P, const SpH &in, SpH &out)
{
    PC z[2][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        z[0][c] = PC{add2(in.u[c].re, in.l[c].re), add2(in.u[c].im, in.l[c].im)};
        z[1][c] = PC{sub2(in.u[c].re, in.l[c].re), sub2(in.u[c].im, in.l[c].im)};
    }
    PC w[2][3];
#pragma unroll
    for (int blk = 0; blk < 2; ++blk)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            PC r{zero2(), zero2()};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const PC &zd = z[blk][d];
                const PC zs{swp(zd.re), swp(zd.im)};
                if (d == c) {
                    // A[c][c] real; B[c][c] = (w, conj w): re pair (w.re, w.re), im pair (w.im, -w.im)
                    const h2 wb = P.Bd[blk][c];
                    r.re = fma2(P.Ad[blk][c], zd.re, r.re);
                    r.im = fma2(P.Ad[blk][c], zd.im, r.im);
                    cmac_pair(PC{lo2(wb), __halves2half2(__high2half(wb), __hneg(__high2half(wb)))}, zs, r);
                } else if (d > c) {
                    cmac_pair(P.Au[blk][upper3(c, d)], zd, r);
                    cmac_pair(P.Bu[blk][upper3(c, d)], zs, r);
                } else {
                    cmac_pair_conj(P.Au[blk][upper3(d, c)], zd, r);
                    const PC &b = P.Bu[blk][upper3(d, c)];
                    cmac_pair_conj(PC{swp(b.re), swp(b.im)}, zs, r);
                }
            }
            w[blk][c] = r;
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        out.u[c] = PC{add2(w[0][c].re, w[1][c].re), add2(w[0][c].im, w[1][c].im)};
        out.l[c] = PC{sub2(w[0][c].re, w[1][c].re), sub2(w[0][c].im, w[1][c].im)};
    }
}

// conversions between the FP32 spinor (times a scale) and pair form
DD_INL void to_pair(const Spinor<float> &x, float sc, SpH &p)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        p.u[c] = PC{__floats2half2_rn(sc * x.v[0][c].re, sc * x.v[1][c].re),
                    __floats2half2_rn(sc * x.v[0][c].im, sc * x.v[1][c].im)};
        p.l[c] = PC{__floats2half2_rn(sc * x.v[2][c].re, sc * x.v[3][c].re),
                    __floats2half2_rn(sc * x.v[2][c].im, sc * x.v[3][c].im)};
    }
}

DD_INL void from_pair(const SpH &p, float sc, Spinor<float> &x)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float2 ur = __half22float2(p.u[c].re), ui = __half22float2(p.u[c].im);
        float2 lr = __half22float2(p.l[c].re), li = __half22float2(p.l[c].im);
        x.v[0][c] = {sc * ur.x, sc * ui.x};
        x.v[1][c] = {sc * ur.y, sc * ui.y};
        x.v[2][c] = {sc * lr.x, sc * li.x};
        x.v[3][c] = {sc * lr.y, sc * li.y};
    }
}

// one site of an FP16-storage spinor in pair form, as stored (relative to the
// site's scale); returns the scale
DD_INL float load_pair(const SpinorField<2> &f, const Geom &g, int l, int s, SpH &p)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const h2 a0 = f.p[elem(g, l, s, 12, c)], a1 = f.p[elem(g, l, s, 12, 3 + c)];
        const h2 a2 = f.p[elem(g, l, s, 12, 6 + c)], a3 = f.p[elem(g, l, s, 12, 9 + c)];
        p.u[c] = PC{__lows2half2(a0, a1), __highs2half2(a0, a1)};
        p.l[c] = PC{__lows2half2(a2, a3), __highs2half2(a2, a3)};
    }
    return f.scale[((long long)l << g.lbvol) + s];
}

// pair form times an FP32 factor, rounded once per component
DD_INL void scale_pair(const SpH &a, float f, SpH &r)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float2 ur = __half22float2(a.u[c].re), ui = __half22float2(a.u[c].im);
        const float2 lr = __half22float2(a.l[c].re), li = __half22float2(a.l[c].im);
        r.u[c] = PC{__floats2half2_rn(f * ur.x, f * ur.y), __floats2half2_rn(f * ui.x, f * ui.y)};
        r.l[c] = PC{__floats2half2_rn(f * lr.x, f * lr.y), __floats2half2_rn(f * li.x, f * li.y)};
    }
}

// an FP16 link as a 3x3 of (re, im) half2: rows 0 and 1 as stored (link_rows), row 2 =
// conj(row0 x row1) accumulated in FP32 from the FP16 entries (mixed-precision
// FMAs) and rounded once (link_row2)
DD_INL void link_rows(const __half2 *u16, const Geom &g, int l, int s, int mu, h2 (&U)[3][3])
{
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) U[a][b] = u16[elem(g, l, s, 24, mu * 6 + a * 3 + b)];
}

DD_INL void link_row2(h2 (&U)[3][3])
{
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int b1 = (b + 1) % 3, b2 = (b + 2) % 3;
        const h2 p = U[0][b1], q = U[1][b2], r = U[0][b2], t = U[1][b1];  // conj(p q - r t)
        const float pr = __low2float(p), pi = __high2float(p), qr = __low2float(q), qi = __high2float(q);
        const float rr = __low2float(r), ri = __high2float(r), tr = __low2float(t), ti = __high2float(t);
        const float re = pr * qr - pi * qi - rr * tr + ri * ti;
        const float im = pr * qi + pi * qr - rr * ti - ri * tr;
        U[2][b] = __floats2half2_rn(re, -im);
    }
}

// The SAP-ready copy of C_inv, written once per gauge field: its pair coefficients
// (clov_pairs_put), so a half-sweep loads them without regrouping.
__global__ void __launch_bounds__(256) k_sap_prep(Geom g, CloverField<2> Ci, __half2 *cpsap)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= g.V) return;
    const int l = (int)(i >> g.lbvol), s = (int)(i & (g.bvol - 1));
    ClovPair P;
    clov_pairs_ld(Ci, g, l, s, P);
    clov_pairs_put(cpsap, g, l, s, P);
}

// o = fa a + fb b + fx x + ft t, component by component, accumulated in FP32 from the
// FP16 pair-form inputs
DD_INL void combine_pair(const SpH &a, float fa, const SpH &b, float fb, const SpH &x, float fx, const SpH &t,
                         float ft, Spinor<float> &o)
{
    auto lo = [&](h2 A, h2 B, h2 X, h2 T) {
        return fa * __low2float(A) + fb * __low2float(B) + fx * __low2float(X) + ft * __low2float(T);
    };
    auto hi = [&](h2 A, h2 B, h2 X, h2 T) {
        return fa * __high2float(A) + fb * __high2float(B) + fx * __high2float(X) + ft * __high2float(T);
    };
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        o.v[0][c] = {lo(a.u[c].re, b.u[c].re, x.u[c].re, t.u[c].re), lo(a.u[c].im, b.u[c].im, x.u[c].im, t.u[c].im)};
        o.v[1][c] = {hi(a.u[c].re, b.u[c].re, x.u[c].re, t.u[c].re), hi(a.u[c].im, b.u[c].im, x.u[c].im, t.u[c].im)};
        o.v[2][c] = {lo(a.l[c].re, b.l[c].re, x.l[c].re, t.l[c].re), lo(a.l[c].im, b.l[c].im, x.l[c].im, t.l[c].im)};
        o.v[3][c] = {hi(a.l[c].re, b.l[c].re, x.l[c].re, t.l[c].re), hi(a.l[c].im, b.l[c].im, x.l[c].im, t.l[c].im)};
    }
}

// acc += f (1 - s gamma_mu) rebuilt from the pair-form half spinor k, accumulated in
// FP32 straight from the FP16 parts (mixed-precision FMAs)
DD_INL void recon_mix(int mu, int s, const PC (&k)[3], float f, Spinor<float> &acc)
{
    const float fs = s > 0 ? f : -f;
    auto add = [](cx<float> &a, float fr, float fi) { a = {a.re + fr, a.im + fi}; };
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float r0 = __low2float(k[c].re), r1 = __high2float(k[c].re);
        const float i0 = __low2float(k[c].im), i1 = __high2float(k[c].im);
        if (mu == 3) {  // twice the pair (the factor 2 of 1 - s gamma_4, see proj_pair)
            const int o = s > 0 ? 2 : 0;
            add(acc.v[o][c], 2.f * f * r0, 2.f * f * i0);
            add(acc.v[o + 1][c], 2.f * f * r1, 2.f * f * i1);
            continue;
        }
        add(acc.v[0][c], f * r0, f * i0);
        add(acc.v[1][c], f * r1, f * i1);
        if (mu == 0) {  // (acc2, acc3) += s i (k1, k0)
            add(acc.v[2][c], -fs * i1, fs * r1);
            add(acc.v[3][c], -fs * i0, fs * r0);
        } else if (mu == 1) {  // (acc2, acc3) += s (k1, -k0)
            add(acc.v[2][c], fs * r1, fs * i1);
            add(acc.v[3][c], -fs * r0, -fs * i0);
        } else {  // (acc2, acc3) += s i (k0, -k1)
            add(acc.v[2][c], -fs * i0, fs * r0);
            add(acc.v[3][c], fs * i1, -fs * r1);
        }
    }
}

// LDS: the Jacobi iterate as 3 x uint4 per site (one colour: u.re, u.im, l.re, l.im)
DD_INL void lds_put(uint4 *xs, int bvol, int s, const SpH &p)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        uint4 v;
        v.x = *reinterpret_cast<const unsigned *>(&p.u[c].re);
        v.y = *reinterpret_cast<const unsigned *>(&p.u[c].im);
        v.z = *reinterpret_cast<const unsigned *>(&p.l[c].re);
        v.w = *reinterpret_cast<const unsigned *>(&p.l[c].im);
        xs[c * bvol + s] = v;
    }
}

DD_INL void lds_get(const uint4 *xs, int bvol, int s, SpH &p)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const uint4 v = xs[c * bvol + s];
        p.u[c].re = *reinterpret_cast<const h2 *>(&v.x);
        p.u[c].im = *reinterpret_cast<const h2 *>(&v.y);
        p.l[c].re = *reinterpret_cast<const h2 *>(&v.z);
        p.l[c].im = *reinterpret_cast<const h2 *>(&v.w);
    }
}

// staged links: U_mu(s) entry (a, b) as one half2 (re, im) at [(mu*9 + a*3 + b)][s]
DD_INL void lds_link(const h2 *ul, int bvol, int s, int mu, h2 (&U)[3][3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) U[a][b] = ul[(mu * 9 + a * 3 + b) * bvol + s];
}

// acc = H_in x in pair form (hops inside the block, Dirichlet at its faces); bvol is
// the block volume (a compile-time constant where the kernel is specialised for it)
DD_INL void inblock_pair(const uint4 *xs, const h2 *ul, const Geom &g, int bvol, const Site &st, SpH &acc)
{
    zero(acc);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int stride = 1 << g.sh[mu];
#pragma unroll
        for (int dir = 1; dir >= -1; dir -= 2) {
            const int c = st.c[mu] + dir;
            if (c < 0 || c >= g.b[mu]) continue;
            const int m = st.s + dir * stride;
            SpH p;
            lds_get(xs, bvol, m, p);
            h2 U[3][3];
            lds_link(ul, bvol, dir > 0 ? st.s : m, mu, U);
            hop_pair(mu, dir, U, p, acc);
        }
    }
}

// log2 of the block extent in direction nu
DD_INL int log2b(const Geom &g, int nu) { return (nu < 3 ? g.sh[nu + 1] : g.lbvol) - g.sh[nu]; }

// first face hop of face q = 2 mu + side (side 0: the +mu face, 1: the -mu face);
// faces are numbered in that order, face q holds bvol / b[mu] hops
DD_INL int face_offset(const Geom &g, int mu, int side)
{
    int o = 0;
#pragma unroll
    for (int nu = 0; nu < 4; ++nu)
        if (nu < mu) o += 2 * (g.bvol >> log2b(g, nu));
    return o + side * (g.bvol >> log2b(g, mu));
}

// Face hop terms.  A half-sweep that is followed by one of the other colour leaves, for
// every site m of each of its block's faces, the part of that site's hop into the
// neighbouring block that it can form from its own data (pair form, relative to the
// block normalisation of its x, which is stored once per block):
//   +mu face (slot face_offset(mu, 0) + kk): the neighbour block l + mu takes x(m) by a
//     backward hop, U_mu(m)^dagger (1 + gamma_mu) x(m) -- the link is this block's own;
//   -mu face (slot face_offset(mu, 1) + kk): the neighbour block l - mu takes x(m) by a
//     forward hop, U_mu(m - mu) (1 - gamma_mu) x(m) -- the link belongs to the receiver,
//     which multiplies it in; the term is the projection alone.
// kk numbers the face's sites by their other three in-block coordinates in order, so a
// face site and the site across the face share it.
template <int MU, int SIDE>
DD_INL void face_out(const Geom &g, int l, int kk, int p, int P, const uint4 *xs, const h2 *ul, int bvol, h2 *ft)
{
    int m = (SIDE == 0 ? g.b[MU] - 1 : 0) << g.sh[MU];
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == MU) continue;
        m += (kk & (g.b[nu] - 1)) << g.sh[nu];
        kk >>= log2b(g, nu);
    }
    SpH xp;
    lds_get(xs, bvol, m, xp);
    PC k[3];
    if (SIDE == 0) {
        PC h[3];
        h2 U[3][3];
        proj_pair(MU, -1, xp, h);
        lds_link(ul, bvol, m, MU, U);
        mat_pair(U, true, h, k);
    } else {
        proj_pair(MU, +1, xp, k);
    }
    h2 *dst = ft + (long long)l * 6 * P + p;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        dst[(2 * c) * P] = k[c].re;
        dst[(2 * c + 1) * P] = k[c].im;
    }
}

// the face term at slot `slot` of block l and the scale of that block
DD_INL float face_in(const h2 *ft, const float *fs, int l, int slot, int P, PC (&k)[3])
{
    const h2 *src = ft + (long long)l * 6 * P + slot;
#pragma unroll
    for (int c = 0; c < 3; ++c) k[c] = PC{src[(2 * c) * P], src[(2 * c + 1) * P]};
    return fs[l];
}

// k times the boundary phase (re, im) of a hop that crosses the lattice edge
DD_INL void phase_pair(PC (&k)[3], float re, float im)
{
    const h2 pr = __float2half2_rn(re), pi = __float2half2_rn(im);
#pragma unroll
    for (int c = 0; c < 3; ++c) k[c] = PC{fma2(pr, k[c].re, mul2(neg2(pi), k[c].im)), fma2(pr, k[c].im, mul2(pi, k[c].re))};
}

// the field of right-hand side r of a batch whose fields lie `off` bytes apart
DD_INL SpinorField<2> rhs_field(const SpinorField<2> &f, long long off)
{
    return SpinorField<2>{(__half2 *)((char *)f.p + off), (float *)((char *)f.scale + off)};
}

// One half-sweep with FP16 arithmetic; same flags and result (up to FP16 rounding) as
// k_sap_half<2>, except that the cross-block term comes from the face hop terms of the
// previous half-sweep (faces: the terms, then one scale per block) and that x is written
// only by the tails of Alg. 1 (a middle half-sweep's x is only ever read through those
// terms).  FACES_OUT leaves this half-sweep's terms for the next one.  The workgroup sweeps
// its block for every right-hand side of `rhs` in turn (b, s, x and the face terms of each
// at their own offsets) with the block's links staged and its C_inv loaded once.  B > 0
// (4 or 2) fixes the block shape to B^4 at compile time: the block extents, in-block strides and the
// block volume become constants, so every LDS offset of the sweeps is an immediate instead
// of a register and the face index arithmetic folds; B = 0 takes the shape from the geometry.
// blocks per workgroup of the packed-FP16 half-sweep: blocks of fewer than 64 sites share
// one wavefront (a block volume is a power of two, at least 16)
DD_HDI int sap_blocks_per_wg(int bvol) { return bvol < 64 ? 64 / bvol : 1; }

// The body of the half-sweep for the w-th block of the swept colour; the kernels below
// take w from their launch (one lattice) or from a table of lattices.
template <int B, bool ONE>
DD_INL void sap_half_pk_body(Geom gin, int w, int colour, int flags, SpinorField<2> bsrc, SpinorField<2> sw,
                             SpinorField<2> xw, const __half2 *u16, const __half2 *cpsap, Phase4 ph, float kappa,
                             int n_jac, h2 *ft, SapRhs rhs)
{
    extern __shared__ uint4 smem_pk[];
    const Geom g = fixed_shape<B>(gin);
    const int bvol = g.bvol;
    // blocks smaller than a wavefront are packed, several to a workgroup (one wavefront):
    // block q of the workgroup is the work item's block bpw w + q, its sites lanes q bvol ..
    const int bpw = sap_blocks_per_wg(bvol);
    const int q = bpw > 1 ? (int)(threadIdx.x >> g.lbvol) : 0;
    const int tid = bpw > 1 ? (int)(threadIdx.x & (bvol - 1)) : (int)threadIdx.x;  // site in the block
    uint4 *xs = smem_pk + (size_t)q * 12 * bvol;            // 3 x bvol uint4
    h2 *ul = reinterpret_cast<h2 *>(xs + 3 * bvol);         // 36 x bvol half2
    __shared__ float wmax[4];
    const int P = face_offset(g, 3, 1) + (bvol >> log2b(g, 3));  // face sites of a block
    wg_skew();

    Site st;
    st.l = colour_block(g, colour, w * bpw + q);
    st.s = tid;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) st.c[mu] = (st.s >> g.sh[mu]) & (g.b[mu] - 1);
    block_coords(g, st.l, st.B);

    // stage the block's links in LDS as full 3x3 FP16 matrices (row 2 rebuilt from the two stored
    // rows) and load its C_inv pair coefficients from the SAP-ready copy, once for all right-hand
    // sides; all loads first, then row 2 and the LDS stores: where the pointers come from a table
    // (the multi-lattice kernel) the loads are flat, and an LDS store right after each would wait
    // for it
    ClovPair CP;
    {
        h2 lk[4][3][3];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) link_rows(u16, g, st.l, st.s, mu, lk[mu]);
        clov_pairs_get(cpsap, g, st.l, st.s, CP);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            link_row2(lk[mu]);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) ul[(mu * 9 + a * 3 + b) * bvol + st.s] = lk[mu][a][b];
        }
    }
    const bool pre = (flags & SAP_PRE) != 0;

    // ONE: the fields as given, a single right-hand side (no loop for the compiler to hoist
    // the neighbour blocks' addresses out of, which would spill them)
    const int nrhs = ONE ? 1 : rhs.n;
    for (int ri = 0; ri < nrhs; ++ri) {
        if (ri > 0) wg_barrier();  // the previous right-hand side is done with LDS
        const long long ridx = ONE ? 0 : rhs.idx[ri];
        const long long off = ONE ? 0 : ridx * rhs.sp_stride;
        const SpinorField<2> b_r = rhs_field(bsrc, off), s_r = rhs_field(sw, off), x_r = rhs_field(xw, off);
        h2 *ft_r = ONE ? ft : (h2 *)((char *)ft + ridx * rhs.face_stride);
        float *fs_r = reinterpret_cast<float *>(ft_r + (long long)g.nblk * 6 * P);  // one scale per block

        // s_c as stored: pair form relative to the site scale ssc
        SpH sraw;
        const float ssc = load_pair((flags & SAP_FIRST) ? b_r : s_r, g, st.l, st.s, sraw);

        // With PRE, h = H_{c c'} x_{c'} at this site: the hops from the neighbouring blocks, taken
        // from the terms they left at the shared faces -- on the +mu face the projection of the
        // neighbour's x, multiplied here by this site's U_mu; on the -mu face the finished
        // backward term -- summed in FP32 with each neighbour block's scale.
        Spinor<float> hc;
        zero(hc);
        if (pre) {
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) {
                const int c = st.c[mu];
                int kk = 0, w8 = 0;
#pragma unroll
                for (int nu = 0; nu < 4; ++nu) {
                    if (nu == mu) continue;
                    kk += st.c[nu] << w8;
                    w8 += log2b(g, nu);
                }
                if (c == g.b[mu] - 1) {  // forward hop from block l + mu, whose -mu face holds the projection
                    const bool edge = st.B[mu] == g.NB[mu] - 1;
                    const int lj = st.l + (edge ? (1 - g.NB[mu]) : 1) * g.bstride[mu];
                    PC t[3], k[3];
                    const float sc = face_in(ft_r, fs_r, lj, face_offset(g, mu, 1) + kk, P, t);
                    h2 U[3][3];
                    lds_link(ul, bvol, st.s, mu, U);  // this site's own link, staged by this thread
                    mat_pair(U, false, t, k);
                    if (edge) phase_pair(k, (float)ph.re[mu], (float)ph.im[mu]);
                    recon_mix(mu, 1, k, sc, hc);
                }
                if (c == 0) {  // backward hop from block l - mu, whose +mu face holds U^dagger times the projection
                    const bool edge = st.B[mu] == 0;
                    const int lj = st.l - (edge ? (1 - g.NB[mu]) : 1) * g.bstride[mu];
                    PC k[3];
                    const float sc = face_in(ft_r, fs_r, lj, face_offset(g, mu, 0) + kk, P, k);
                    if (edge) phase_pair(k, (float)ph.re[mu], (float)-ph.im[mu]);
                    recon_mix(mu, -1, k, sc, hc);
                }
            }
        }

        // block normalisation: scale s_c and h to max |component| <= 1 (a stored FP16
        // spinor has max |component| = 1 relative to its scale)
        float m = ssc;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) m = fmaxf(m, fmaxf(fabsf(hc.v[a][c].re), fabsf(hc.v[a][c].im)));
        const int wv = bvol < 64 ? bvol : 64;  // lanes of one block in one wavefront
        for (int o2 = wv / 2; o2 >= 1; o2 >>= 1) m = fmaxf(m, __shfl_xor(m, o2, wv));
        if (bvol >= 64 && (threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
        wg_barrier();  // also: every link is staged
        if (bvol >= 64) {  // smaller blocks have their maximum from the shuffles
            m = 0.f;
            for (int k = 0; k < bvol / 64; ++k) m = fmaxf(m, wmax[k]);
        }
        const float sc = m > 0.f ? 1.f / m : 0.f;

        // x0 = s_c + kappa C_inv h (normalised): the first Jacobi step from x = 0; every later
        // step is x <- x0 + kappa C_inv H_in x
        SpH x0, x, acc, t;
        scale_pair(sraw, ssc * sc, x0);
        const h2 K = __float2half2_rn(kappa);
        if (pre) {
            SpH hp;
            to_pair(hc, sc, hp);
            clover_pair(CP, hp, t);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                x0.u[c] = PC{fma2(K, t.u[c].re, x0.u[c].re), fma2(K, t.u[c].im, x0.u[c].im)};
                x0.l[c] = PC{fma2(K, t.l[c].re, x0.l[c].re), fma2(K, t.l[c].im, x0.l[c].im)};
            }
        }
        x = x0;
        for (int j = 0; j < n_jac; ++j) {
            wg_barrier();
            lds_put(xs, bvol, st.s, x);
            wg_barrier();
            inblock_pair(xs, ul, g, bvol, st, acc);
            clover_pair(CP, acc, t);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                x.u[c] = PC{fma2(K, t.u[c].re, x0.u[c].re), fma2(K, t.u[c].im, x0.u[c].im)};
                x.l[c] = PC{fma2(K, t.l[c].re, x0.l[c].re), fma2(K, t.l[c].im, x0.l[c].im)};
            }
        }
        const float inv = m;  // undo the normalisation
        if (!(flags & SAP_TAIL)) {
            // s_c <- (s_c + kappa C_inv h) + b_c - x_c + kappa C_inv H_in x_c, in FP32
            wg_barrier();
            lds_put(xs, bvol, st.s, x);
            wg_barrier();
            inblock_pair(xs, ul, g, bvol, st, acc);
            clover_pair(CP, acc, t);
            SpH braw;
            const float sb = load_pair(b_r, g, st.l, st.s, braw);
            Spinor<float> snew;
            combine_pair(x0, inv, braw, sb, x, -inv, t, kappa * inv, snew);
            s_r.store(g, st.l, st.s, snew);
        } else {
            Spinor<float> xf;
            from_pair(x, inv, xf);
            x_r.store(g, st.l, st.s, xf);
            if (flags & SAP_FACES_OUT) {
                wg_barrier();
                lds_put(xs, bvol, st.s, x);
            }
        }
        if (flags & SAP_FACES_OUT) {
            // this block's face terms from x in LDS (put there by the s update, or just above),
            // spread evenly over the workgroup
            wg_barrier();
            const bool equal_faces = g.b[0] == g.b[1] && g.b[1] == g.b[2] && g.b[2] == g.b[3];
            const int lnf = g.lbvol - log2b(g, 0);  // log2 of the sites per face
            for (int p = tid; p < P; p += bvol) {
                int q = 0, base = 0;
                if (equal_faces) {  // hypercubic block: face q holds sites q * nf ... q * nf + nf - 1
                    q = p >> lnf;
                    base = q << lnf;
                } else {
#pragma unroll
                    for (int qq = 0; qq < 7; ++qq) {
                        const int n = bvol >> log2b(g, qq >> 1);
                        if (q == qq && p >= base + n) {
                            base += n;
                            q = qq + 1;
                        }
                    }
                }
                const int kk = p - base;
                switch (q) {  // faces in order +x, -x, +y, -y, +z, -z, +t, -t
                case 0: face_out<0, 0>(g, st.l, kk, p, P, xs, ul, bvol, ft_r); break;
                case 1: face_out<0, 1>(g, st.l, kk, p, P, xs, ul, bvol, ft_r); break;
                case 2: face_out<1, 0>(g, st.l, kk, p, P, xs, ul, bvol, ft_r); break;
                case 3: face_out<1, 1>(g, st.l, kk, p, P, xs, ul, bvol, ft_r); break;
                case 4: face_out<2, 0>(g, st.l, kk, p, P, xs, ul, bvol, ft_r); break;
                case 5: face_out<2, 1>(g, st.l, kk, p, P, xs, ul, bvol, ft_r); break;
                case 6: face_out<3, 0>(g, st.l, kk, p, P, xs, ul, bvol, ft_r); break;
                default: face_out<3, 1>(g, st.l, kk, p, P, xs, ul, bvol, ft_r); break;
                }
            }
            if (tid == 0) fs_r[st.l] = inv;
        }
    }
}

template <int B, bool ONE>
__global__ void __launch_bounds__(256) k_sap_half_pk(Geom gin, int colour, int flags, SpinorField<2> bsrc,
                                                     SpinorField<2> sw, SpinorField<2> xw, const __half2 *u16,
                                                     const __half2 *cpsap, Phase4 ph, float kappa, int n_jac, h2 *ft,
                                                     SapRhs rhs)
{
    sap_half_pk_body<B, ONE>(gin, xcd_remap(blockIdx.x, gridDim.x), colour, flags, bsrc, sw, xw, u16, cpsap, ph, kappa,
                        n_jac, ft, rhs);
}

// The same half-sweep on several lattices of one block shape in one launch: the work items
// are the workgroups' shares of the blocks of the swept colour (sap_multi_items per lattice),
// numbered lattice by lattice (item0 of each table entry); a workgroup finds its lattice in
// the table and sweeps its blocks there.  One right-hand side per lattice.  The table comes by
// value in the kernel arguments, so the fields' pointers are known to be global ones (from a
// table in device memory every access would be a flat one).
template <int B>
__global__ void __launch_bounds__(256) k_sap_half_pk_multi(SapLatTab t, int colour, int flags)
{
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    int k = 0;
    while (k + 1 < t.n && w >= t.e[k + 1].item0) ++k;
    const SapLat &L = t.e[k];
    SapRhs one{};
    one.n = 1;
    sap_half_pk_body<B, true>(L.g, w - L.item0, colour, flags, L.b, L.s, L.x, L.u16, L.cpsap, L.ph, L.kappa, L.n_jac, L.ft,
                        one);
}

// face sites of one block, and the bytes of the face terms of a lattice (6 half2 per face
// site, one FP32 scale per block)
static size_t face_sites(const Geom &g)
{
    size_t faces = 0;
    for (int mu = 0; mu < 4; ++mu) faces += 2 * (size_t)(g.bvol / g.b[mu]);
    return faces;
}

size_t sap_face_bytes(const Geom &g)
{
    return (size_t)g.nblk * (face_sites(g) * 6 * sizeof(__half2) + sizeof(float));
}

size_t sap_pk_lds_bytes(const Geom &g)
{
    // the Jacobi iterate and the staged links
    return (size_t)g.bvol * (3 * sizeof(uint4) + 36 * sizeof(__half2));
}

hipError_t launch_sap_half_pk(const Geom &g, hipStream_t st, const SapArgs &a, int colour, int flags)
{
    if (a.prec != 2 || !a.faces) return hipErrorInvalidValue;
    auto sfh = [&](void *p) {
        return SpinorField<2>{(__half2 *)p, (float *)((char *)p + 12 * g.V * sizeof(__half2))};
    };
    const bool cube4 = g.b[0] == 4 && g.b[1] == 4 && g.b[2] == 4 && g.b[3] == 4;
    const bool cube2 = g.b[0] == 2 && g.b[1] == 2 && g.b[2] == 2 && g.b[3] == 2;
    SapRhs rhs = a.rhs;
    const bool one = rhs.n <= 0;  // one right-hand side (the fields as given)
    if (one) {
        rhs = SapRhs{};
        rhs.n = 1;
    }
    if (rhs.n > SAP_RHS_MAX) return hipErrorInvalidValue;
    auto kern = cube4   ? (one ? k_sap_half_pk<4, true> : k_sap_half_pk<4, false>)
                : cube2 ? (one ? k_sap_half_pk<2, true> : k_sap_half_pk<2, false>)
                        : (one ? k_sap_half_pk<0, true> : k_sap_half_pk<0, false>);
    const int bpw = sap_blocks_per_wg(g.bvol);  // (g.nblk / 2 is a multiple of 8: every direction holds an even
                                                 // number of blocks)
    hipLaunchKernelGGL(kern, dim3(g.nblk / 2 / bpw), dim3(g.bvol * bpw), bpw * sap_pk_lds_bytes(g), st, g, colour, flags,
                       sfh((void *)a.b), sfh(a.s), sfh(a.x), (const __half2 *)a.links, (const __half2 *)a.cinv, a.phase,
                       (float)a.kappa, a.n_jac, (h2 *)a.faces, rhs);
    return hipGetLastError();
}

hipError_t launch_sap_prep(const Geom &g, hipStream_t st, const void *cinv16, void *cpsap)
{
    hipLaunchKernelGGL(k_sap_prep, dim3((unsigned)((g.V + 255) / 256)), dim3(256), 0, st, g,
                       CloverField<2>{(const __half2 *)cinv16}, (__half2 *)cpsap);
    return hipGetLastError();
}

SapLat sap_lat(const Geom &g, const SapArgs &a, int item0)
{
    auto sfh = [&](void *p) {
        return SpinorField<2>{(__half2 *)p, (float *)((char *)p + 12 * g.V * sizeof(__half2))};
    };
    SapLat L{};
    L.g = g;
    L.b = sfh((void *)a.b);
    L.s = sfh(a.s);
    L.x = sfh(a.x);
    L.u16 = (const __half2 *)a.links;
    L.cpsap = (const __half2 *)a.cinv;
    L.ph = a.phase;
    L.kappa = (float)a.kappa;
    L.n_jac = a.n_jac;
    L.ft = (h2 *)a.faces;
    L.item0 = item0;
    return L;
}

int sap_multi_items(const Geom &g) { return g.nblk / 2 / sap_blocks_per_wg(g.bvol); }

hipError_t launch_sap_half_pk_multi(const Geom &g, hipStream_t st, const SapLat *lat, int nlat, int colour, int flags)
{
    if (nlat <= 0) return hipSuccess;
    const bool cube4 = g.b[0] == 4 && g.b[1] == 4 && g.b[2] == 4 && g.b[3] == 4;
    const bool cube2 = g.b[0] == 2 && g.b[1] == 2 && g.b[2] == 2 && g.b[3] == 2;
    const int bpw = sap_blocks_per_wg(g.bvol);
    auto kern = cube4 ? k_sap_half_pk_multi<4> : cube2 ? k_sap_half_pk_multi<2> : k_sap_half_pk_multi<0>;
    for (int k0 = 0; k0 < nlat; k0 += SAP_MULTI_MAX) {  // up to SAP_MULTI_MAX lattices per launch
        SapLatTab t{};
        int items = 0;
        for (; t.n < SAP_MULTI_MAX && k0 + t.n < nlat; ++t.n) {
            t.e[t.n] = lat[k0 + t.n];
            t.e[t.n].item0 = items;
            items += sap_multi_items(t.e[t.n].g);
        }
        hipLaunchKernelGGL(kern, dim3(items), dim3(g.bvol * bpw), bpw * sap_pk_lds_bytes(g), st, t, colour, flags);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace dd
