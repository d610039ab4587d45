// dd_sap_fp16.hip -- SAP half-sweep (Alg. 1 with the Jacobi of Alg. 2) with
// FP16 storage and packed FP16 arithmetic for the block-local sweeps.
//
// The block-local work of a half-sweep is N_JAC + 1 applications of
// K = kappa C_inv H_in, all inside one workgroup.  Here every spinor is kept in
// "pair form": for each colour c the spin pairs (psi0, psi1) and (psi2, psi3)
// are two complex pairs, each stored as two half2 (real parts, imaginary
// parts).  A spin-projected half spinor is then one complex pair per colour, so
// a link entry, broadcast to both halves, multiplies both spins of the half
// spinor in one packed FMA: a hop's two 3x3 complex products take 36 packed
// FMAs.  The clover block (two 6x6 Hermitian blocks in the gamma_5-diagonal
// basis) is rearranged once per launch into pair coefficients,
//   w_pair[c] = sum_c' A[c][c'] (.) z_pair[c'] + B[c][c'] (.) swap(z_pair[c']).
// FP16 range: the block's source is scaled by 1 / max|component| before the
// sweeps (the sweeps are linear) and the result is scaled back in FP32.  The
// cross-block prologue (A_{c c'} x_{c'}, the previous half-sweep's output read
// from the neighbouring blocks) and the final s update stay in FP32.
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

// acc += (1 - s gamma_mu) W psi, pair form, for the gamma matrices of the appendix
DD_INL void hop_pair(int mu, int s, const h2 (&U)[3][3], const SpH &p, SpH &acc)
{
    const h2 S = __float2half2_rn((float)s);                      // (s, s)
    const h2 Cm = __floats2half2_rn(-(float)s, (float)s);         // (-s, s)
    PC h[3], k[3];
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
        } else {  // gamma_4 diagonal: twice the surviving spin pair
            const PC &q = s > 0 ? p.l[c] : p.u[c];
            h[c].re = add2(q.re, q.re);
            h[c].im = add2(q.im, q.im);
        }
    }
    mat_pair(U, s < 0, h, k);
    const h2 Cp = __floats2half2_rn((float)s, -(float)s);  // (s, -s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (mu == 3) {
            PC &t = s > 0 ? acc.l[c] : acc.u[c];
            t.re = add2(t.re, k[c].re);
            t.im = add2(t.im, k[c].im);
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

// clover block in pair form: for each chiral block, A[c][c'] and B[c][c']
struct ClovPair {
    PC A[2][3][3], B[2][3][3];
};

// element (i, j) of the Hermitian 6x6 block blk
DD_INL cx<float> herm_elem(const Clov<float> &C, int blk, int i, int j)
{
    if (i == j) return {C.d[blk][i], 0.f};
    if (i < j) return C.h[blk][upper_index(i, j)];
    return conj(C.h[blk][upper_index(j, i)]);
}

DD_INL PC pair_of(cx<float> a, cx<float> b) { return PC{__floats2half2_rn(a.re, b.re), __floats2half2_rn(a.im, b.im)}; }

DD_INL void clov_pairs(const Clov<float> &C, ClovPair &P)
{
#pragma unroll
    for (int blk = 0; blk < 2; ++blk)
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                P.A[blk][c][d] = pair_of(herm_elem(C, blk, c, d), herm_elem(C, blk, 3 + c, 3 + d));
                P.B[blk][c][d] = pair_of(herm_elem(C, blk, c, 3 + d), herm_elem(C, blk, 3 + c, d));
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
                cmac_pair(P.A[blk][c][d], z[blk][d], r);
                cmac_pair(P.B[blk][c][d], PC{swp(z[blk][d].re), swp(z[blk][d].im)}, r);
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

// acc = H_in x in pair form (hops inside the block, Dirichlet at its faces)
DD_INL void inblock_pair(const uint4 *xs, const h2 *ul, const Geom &g, const Site &st, SpH &acc)
{
    zero(acc);
    const int bvol = g.bvol;
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

// One half-sweep with FP16 arithmetic in the block-local part; same flags and
// result (up to FP16 rounding) as k_sap_half<2>.
__global__ void __launch_bounds__(256) k_sap_half_pk(Geom g, int colour, int flags, SpinorField<2> bsrc,
                                                     SpinorField<2> sw, SpinorField<2> xw, const __half2 *u16,
                                                     CloverField<2> Ci, Phase4 ph, float kappa, int n_jac)
{
    extern __shared__ uint4 smem_pk[];
    const int bvol = g.bvol;
    uint4 *xs = smem_pk;                                    // 3 x bvol uint4
    h2 *ul = reinterpret_cast<h2 *>(xs + 3 * bvol);         // 36 x bvol half2
    __shared__ float wmax[4];

    const int w = xcd_remap(blockIdx.x, gridDim.x);
    Site st;
    st.l = colour_block(g, colour, w);
    st.s = threadIdx.x;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) st.c[mu] = (st.s >> g.sh[mu]) & (g.b[mu] - 1);
    block_coords(g, st.l, st.B);

    const LinkField<2> U16{u16};
    Clov<float> cl;
    Ci.load(g, st.l, st.s, cl);

    Spinor<float> src;
    if (flags & SAP_FIRST)
        bsrc.load(g, st.l, st.s, src);
    else
        sw.load(g, st.l, st.s, src);

    if (flags & SAP_PRE) {  // s_c += kappa C_inv (cross-block hops of x_{c'}), FP32
        // Each (direction, side, face site) hop once, spread evenly over the workgroup: a
        // per-site loop would run all eight hop bodies in every wavefront with most lanes
        // idle.  The hops' half spinors are parked in LDS (the link staging area, not in
        // use yet) and summed per site afterwards.
        float2 *fb = reinterpret_cast<float2 *>(ul);  // [6][P] complex
        int off[9];
        off[0] = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) off[q + 1] = off[q] + bvol / g.b[q >> 1];
        const int P = off[8];
        for (int p = threadIdx.x; p < P; p += bvol) {
            int q = 0;
            while (q < 7 && p >= off[q + 1]) ++q;
            const int mu = q >> 1, dir = (q & 1) ? -1 : 1;
            int kk = p - off[q];
            Site fs;
            fs.l = st.l;
            fs.s = 0;
#pragma unroll
            for (int nu = 0; nu < 4; ++nu) {
                fs.B[nu] = st.B[nu];
                if (nu == mu) {
                    fs.c[nu] = dir > 0 ? g.b[nu] - 1 : 0;
                } else {
                    fs.c[nu] = kk & (g.b[nu] - 1);
                    kk >>= log2b(g, nu);
                }
                fs.s += fs.c[nu] << g.sh[nu];
            }
            bool wrap, inblk;
            const long long j = neighbour(g, fs, mu, dir, wrap, inblk);
            const int lj = (int)(j >> g.lbvol), sj = (int)(j & (bvol - 1));
            Spinor<float> psi;
            xw.load(g, lj, sj, psi);
            Mat3<float> W;
            if (dir > 0)
                U16.load(g, st.l, fs.s, mu, W);
            else
                U16.load(g, lj, sj, mu, W);
            Half<float> h, k;
            project(mu, dir, psi, h);
            mat_half(W, dir < 0, h, k);
            if (wrap) {
                const cx<float> phase = {(float)ph.re[mu], (float)(dir > 0 ? ph.im[mu] : -ph.im[mu])};
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int c = 0; c < 3; ++c) k.v[a][c] = k.v[a][c] * phase;
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) fb[(a * 3 + c) * P + p] = make_float2(k.v[a][c].re, k.v[a][c].im);
        }
        __syncthreads();
        Spinor<float> acc, t;
        zero(acc);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
            for (int dir = 1; dir >= -1; dir -= 2) {
                const int c = st.c[mu] + dir;
                if (c >= 0 && c < g.b[mu]) continue;
                // index of this site on the face: the other three coordinates in order
                int kk = 0, w8 = 0;
#pragma unroll
                for (int nu = 0; nu < 4; ++nu) {
                    if (nu == mu) continue;
                    kk += st.c[nu] << w8;
                    w8 += log2b(g, nu);
                }
                const int p = off[2 * mu + (dir > 0 ? 0 : 1)] + kk;
                Half<float> k;
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) {
                        const float2 v = fb[(a * 3 + cc) * P + p];
                        k.v[a][cc] = {v.x, v.y};
                    }
                reconstruct(mu, dir, k, acc);
            }
        }
        clover_mul(cl, acc, t);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) src.v[a][c] = src.v[a][c] + kappa * t.v[a][c];
        __syncthreads();  // the face buffer is about to become the link staging area
    }

    // stage the block's links as full 3x3 FP16 matrices
    for (int mu = 0; mu < 4; ++mu) {
        Mat3<float> U;
        U16.load(g, st.l, st.s, mu, U);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) ul[(mu * 9 + a * 3 + b) * bvol + st.s] = __floats2half2_rn(U.m[a][b].re, U.m[a][b].im);
    }

    ClovPair CP;
    clov_pairs(cl, CP);

    // block normalisation: scale the source to max |component| = 1
    float m = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) m = fmaxf(m, fmaxf(fabsf(src.v[a][c].re), fabsf(src.v[a][c].im)));
    const int wv = bvol < 64 ? bvol : 64;  // lanes of this workgroup in one wavefront
    for (int off = wv / 2; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, wv));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    m = 0.f;
    for (int q = 0; q < (bvol + 63) / 64; ++q) m = fmaxf(m, wmax[q]);
    const float sc = m > 0.f ? 1.f / m : 0.f;

    SpH sh, x, acc, t;
    to_pair(src, sc, sh);
    x = sh;
    const h2 K = __float2half2_rn(kappa);
    for (int j = 0; j < n_jac; ++j) {
        __syncthreads();
        lds_put(xs, bvol, st.s, x);
        __syncthreads();
        inblock_pair(xs, ul, g, st, acc);
        clover_pair(CP, acc, t);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x.u[c].re = fma2(K, t.u[c].re, sh.u[c].re);
            x.u[c].im = fma2(K, t.u[c].im, sh.u[c].im);
            x.l[c].re = fma2(K, t.l[c].re, sh.l[c].re);
            x.l[c].im = fma2(K, t.l[c].im, sh.l[c].im);
        }
    }
    const float inv = m;  // undo the normalisation
    Spinor<float> xf;
    from_pair(x, inv, xf);
    if (!(flags & SAP_TAIL)) {
        __syncthreads();
        lds_put(xs, bvol, st.s, x);
        __syncthreads();
        inblock_pair(xs, ul, g, st, acc);
        clover_pair(CP, acc, t);
        Spinor<float> tf, b;
        from_pair(t, inv, tf);
        bsrc.load(g, st.l, st.s, b);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                src.v[a][c] = src.v[a][c] + b.v[a][c] - xf.v[a][c] + kappa * tf.v[a][c];
        sw.store(g, st.l, st.s, src);
    }
    xw.store(g, st.l, st.s, xf);
}

size_t sap_pk_lds_bytes(const Geom &g)
{
    // the Jacobi iterate, then the larger of the link staging area and the face buffer of
    // the cross-block prologue (6 FP32 complex per face hop)
    size_t faces = 0;
    for (int mu = 0; mu < 4; ++mu) faces += 2 * (size_t)(g.bvol / g.b[mu]);
    const size_t links = (size_t)g.bvol * 36 * sizeof(__half2), fbuf = faces * 6 * sizeof(float2);
    return (size_t)g.bvol * 3 * sizeof(uint4) + (links > fbuf ? links : fbuf);
}

hipError_t launch_sap_half_pk(const Geom &g, hipStream_t st, const SapArgs &a, int colour, int flags)
{
    if (a.prec != 2) return hipErrorInvalidValue;
    auto sfh = [&](void *p) {
        return SpinorField<2>{(__half2 *)p, (float *)((char *)p + 12 * g.V * sizeof(__half2))};
    };
    hipLaunchKernelGGL(k_sap_half_pk, dim3(g.nblk / 2), dim3(g.bvol), sap_pk_lds_bytes(g), st, g, colour, flags,
                       sfh((void *)a.b), sfh(a.s), sfh(a.x), (const __half2 *)a.links,
                       CloverField<2>{(const __half2 *)a.cinv}, a.phase, (float)a.kappa, a.n_jac);
    return hipGetLastError();
}

}  // namespace dd
