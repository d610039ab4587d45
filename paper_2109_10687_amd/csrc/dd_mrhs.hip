// dd_mrhs.hip -- the FP32 operator A = I - kappa C_inv H (Sec. 3) applied to a
// batch of up to 12 right-hand sides at once, with the link products on the
// matrix cores.
//
// With several right-hand sides, each hop multiplies one 3x3 link by a 3 x 24
// block of projected half spinors (3 colours x 2 half-spin components x 12
// right-hand sides).  In real form this is a 6x6 by 6x24 product.  The
// v_mfma_f32_4x4x1_16b_f32 instruction performs sixteen independent 4x4x1
// outer-product updates per wavefront, so one wavefront handles sixteen sites
// at a time, a group of four lanes per site: two 4-row tiles (rows 6 and 7
// zero), six 4-column tiles, six steps over k.  Nothing is packed
// block-diagonally, so only the row padding (6 of 8 rows used) is wasted.
//
// Lane q of a site's group supplies rows q and q+4 of the link's real form and
// columns q, q+4, ..., q+20 of the half-spinor block; column c holds
// right-hand side c/2 and half-spin component c%2, so lanes q and q^1 carry
// the two half-spin components of the same six right-hand sides.  After each
// hop a lane adds its component of W h into partial sums of the output spin
// components it touches (its own, and the lower-half components that its
// half-spin component feeds); one exchange between the lane pair at the end
// completes the lower half, and a second exchange gives each lane the full
// chiral 6-vector for the clover block C_inv.
//
// Batched fields: nrhs FP32 internal-layout spinors, one after another
// (stride 12 V complex).  Right-hand sides beyond nrhs in the last tile are
// never written (their lanes read the last right-hand side instead).
#include "dd_device.h"
#include "dd_launch.h"

namespace dd {

typedef float f4_t __attribute__((ext_vector_type(4)));

namespace {

struct Cf {
    float re, im;
};
DD_INL Cf cadd(Cf a, Cf b) { return {a.re + b.re, a.im + b.im}; }
DD_INL Cf cmul(Cf a, Cf b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
DD_INL Cf cmulc_(Cf a, Cf b) { return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; }  // conj(a) b
DD_INL Cf ld2(const float2 *p);

// entry (a, b) of an FP32 link stored as rows 0 and 1; row 2 = conj(row0 x row1)
DD_INL Cf link32(const float2 *u, const Geom &g, int l, int s, int mu, int a, int b)
{
    auto e = [&](int r, int c) { return ld2(&u[elem(g, l, s, 24, mu * 6 + r * 3 + c)]); };
    if (a < 2) return e(a, b);
    const int b1 = (b + 1) % 3, b2 = (b + 2) % 3;
    const Cf p = e(0, b1), q = e(1, b2), r = e(0, b2), t = e(1, b1);
    return {p.re * q.re - p.im * q.im - r.re * t.re + r.im * t.im, -(p.re * q.im + p.im * q.re - r.re * t.im - r.im * t.re)};
}

DD_INL Cf ld2(const float2 *p)
{
    float2 t = *p;
    return {t.x, t.y};
}
DD_INL Cf shfl1(Cf a) { return {__shfl_xor(a.re, 1, 64), __shfl_xor(a.im, 1, 64)}; }

}  // namespace

// NTP: column tiles per pass (a lane carries NTP right-hand sides per pass; the
// group of four lanes 2 NTP; 6 passes / NTP cover twelve).  WGS: threads per workgroup.
// BS: block side when the block shape is fixed at compile time (0: taken from the geometry).
template <int NTP, int WGS, int BS>
__global__ void __launch_bounds__(WGS) k_dirac_mrhs(Geom gin, MrhsArgs a)
{
    const Geom g = fixed_shape<BS>(gin);
    constexpr int NPASS = 6 / NTP;
    const int nwg = gridDim.x;
    const int w = xcd_remap(blockIdx.x, nwg);
    const int lane = threadIdx.x & 63;
    const int q = lane & 3, s = q & 1;
    const long long i = (long long)w * (WGS / 4) + (threadIdx.x >> 2);  // site of this lane's group
    if (i >= g.V) return;                                              // whole groups leave together
    Site st;
    decode(g, i, st);
    const long long RS = 12 * g.V;  // stride between right-hand sides (complex)
    const float kap = (float)a.kappa;

#pragma unroll 1
    for (int pass = 0; pass < NPASS; ++pass) {
        // this lane's right-hand sides: rhs(nt) = 2 (pass*NTP + nt) + (q >> 1)
        // (a right-hand side beyond nrhs reads the last one and is not stored: every
        // load stays unconditional, so no branch splits the loads of a hop)
        int rhs[NTP], rld[NTP];
        bool on[NTP];
#pragma unroll
        for (int nt = 0; nt < NTP; ++nt) {
            rhs[nt] = 2 * (pass * NTP + nt) + (q >> 1);
            on[nt] = rhs[nt] < a.nrhs;
            rld[nt] = on[nt] ? rhs[nt] : a.nrhs - 1;
        }
        // partial sums: P0 = spin component s, P2 / P3 = components 2 / 3
        Cf P0[NTP][3], P2[NTP][3], P3[NTP][3];
#pragma unroll
        for (int nt = 0; nt < NTP; ++nt)
#pragma unroll
            for (int c = 0; c < 3; ++c) P0[nt][c] = P2[nt][c] = P3[nt][c] = {0.f, 0.f};

        // hops one at a time: the unrolled form keeps every hop's operands live and spills
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu) {
#pragma unroll 1
            for (int dir = 1; dir >= -1; dir -= 2) {
                bool wrap, inblk;
                const long long j = neighbour(g, st, mu, dir, wrap, inblk);
                const int lj = (int)(j >> g.lbvol), sj = (int)(j & (g.bvol - 1));
                // ---- A: rows q and q+4 of the real form of W (U forward, U^dagger backward)
                float A[2][6];
                {
                    const int ll = dir > 0 ? st.l : lj, ss = dir > 0 ? st.s : sj;
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt) {
                        const int r = q + 4 * mt;  // rows 6 and 7 are padding: loaded from row 0, zeroed
                        const bool pad = r >= 6;
                        const int rr = pad ? 0 : r % 3;
                        const bool rim = r >= 3;
#pragma unroll
                        for (int kk = 0; kk < 3; ++kk) {
                            // W[rr][kk]: U[rr][kk] or conj(U[kk][rr])
                            Cf u = dir > 0 ? link32(a.u, g, ll, ss, mu, rr, kk) : link32(a.u, g, ll, ss, mu, kk, rr);
                            if (dir < 0) u.im = -u.im;
                            // real form [[Re, -Im], [Im, Re]]
                            A[mt][kk] = pad ? 0.f : (rim ? u.im : u.re);
                            A[mt][kk + 3] = pad ? 0.f : (rim ? u.re : -u.im);
                        }
                    }
                }
                // ---- B: this lane's half-spin component s of the projected neighbour spinor
                // h_s = psi_{i1} + f * psi_{i2} (spin projection of (1 - dir gamma_mu))
                int i1, i2;
                Cf f1 = {1.f, 0.f}, f2 = {0.f, 0.f};
                const float sr = (float)dir;
                if (mu == 0) {
                    i1 = s;
                    i2 = 3 - s;
                    f2 = {0.f, -sr};
                } else if (mu == 1) {
                    i1 = s;
                    i2 = 3 - s;
                    f2 = {s ? sr : -sr, 0.f};
                } else if (mu == 2) {
                    i1 = s;
                    i2 = 2 + s;
                    f2 = {0.f, s ? sr : -sr};
                } else {
                    i1 = (dir > 0 ? 2 : 0) + s;
                    i2 = i1;
                    f1 = {2.f, 0.f};
                }
                float B[NTP][6];
#pragma unroll
                for (int nt = 0; nt < NTP; ++nt) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float2 *base = a.in + rld[nt] * RS;
                        Cf p1 = ld2(&base[elem(g, lj, sj, 12, i1 * 3 + c)]);
                        Cf p2 = ld2(&base[elem(g, lj, sj, 12, i2 * 3 + c)]);  // i2 = i1 for mu = 3 (f2 = 0)
                        Cf h = cadd(cmul(f1, p1), cmul(f2, p2));
                        B[nt][c] = h.re;
                        B[nt][c + 3] = h.im;
                    }
                }
                // ---- C = A B on the matrix cores: per column tile, two row tiles, six k steps
                f4_t C[NTP][2];
#pragma unroll
                for (int nt = 0; nt < NTP; ++nt)
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt) {
                        f4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int k = 0; k < 6; ++k) acc = __builtin_amdgcn_mfma_f32_4x4x1f32(A[mt][k], B[nt][k], acc, 0, 0, 0);
                        C[nt][mt] = acc;
                    }
                // ---- reconstruct: k_s[colour] = (Re: rows 0..2, Im: rows 3..5) of column (nt, q)
                Cf ph = {1.f, 0.f};
                if (wrap) ph = {(float)a.phase.re[mu], (float)(dir > 0 ? a.phase.im[mu] : -a.phase.im[mu])};
                // factors into P0, P2, P3 for this (mu, dir, s)
                Cf g0 = {1.f, 0.f}, g2 = {0.f, 0.f}, g3 = {0.f, 0.f};
                if (mu == 0) {
                    if (s == 0) g3 = {0.f, sr}; else g2 = {0.f, sr};
                } else if (mu == 1) {
                    if (s == 0) g3 = {-sr, 0.f}; else g2 = {sr, 0.f};
                } else if (mu == 2) {
                    if (s == 0) g2 = {0.f, sr}; else g3 = {0.f, -sr};
                } else {
                    if (dir > 0) {
                        g0 = {0.f, 0.f};
                        if (s == 0) g2 = {1.f, 0.f}; else g3 = {1.f, 0.f};
                    }
                }
#pragma unroll
                for (int nt = 0; nt < NTP; ++nt) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        Cf k = {C[nt][0][c], c == 0 ? C[nt][0][3] : C[nt][1][c - 1]};
                        k = cmul(ph, k);
                        P0[nt][c] = cadd(P0[nt][c], cmul(g0, k));
                        P2[nt][c] = cadd(P2[nt][c], cmul(g2, k));
                        P3[nt][c] = cadd(P3[nt][c], cmul(g3, k));
                    }
                }
            }
        }
        // ---- epilogue per column tile: complete the lower components across the lane
        // pair (lane s then owns spins s and s+2), form the chiral vectors
        // u = H_a + H_{a+2}, u2 = H_a - H_{a+2} (lane s holds a = s, its partner the
        // other half), apply rows 3s..3s+2 of the two C_inv blocks, out = in - kappa C_inv H
#pragma unroll
        for (int nt = 0; nt < NTP; ++nt) {
            Cf U1[3], U2[3], V1[3], V2[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Cf send = s == 0 ? P3[nt][c] : P2[nt][c];
                Cf recv = shfl1(send);
                Cf h = P0[nt][c];
                Cf h2 = s == 0 ? cadd(P2[nt][c], recv) : cadd(P3[nt][c], recv);
                U1[c] = cadd(h, h2);
                U2[c] = {h.re - h2.re, h.im - h2.im};
                V1[c] = shfl1(U1[c]);
                V2[c] = shfl1(U2[c]);
            }
            float2 *ob = a.out + rld[nt] * RS;
            const float2 *ib = a.in + rld[nt] * RS;
#pragma unroll
            for (int rr = 0; rr < 3; ++rr) {
                const int r = 3 * s + rr;
                Cf w1 = {0.f, 0.f}, w2 = {0.f, 0.f};
#pragma unroll
                for (int cc = 0; cc < 6; ++cc) {
                    // entry (r, cc) of N+ (block 0) and N- (block 1): Hermitian, stored as the
                    // real diagonal (pairs) and the upper triangle
                    // (one unconditional load per block: the element index and the
                    // interpretation are selected, not branched on)
                    const bool dg = cc == r;
                    const int e = dg ? r / 2 : 3 + (cc > r ? upper_index(r, cc) : upper_index(cc, r));
                    const float2 t0 = a.cinv[elem(g, st.l, st.s, 36, e)];
                    const float2 t1 = a.cinv[elem(g, st.l, st.s, 36, 18 + e)];
                    const float cj = cc < r ? -1.f : 1.f;
                    Cf np = dg ? Cf{(r & 1) ? t0.y : t0.x, 0.f} : Cf{t0.x, cj * t0.y};
                    Cf nm = dg ? Cf{(r & 1) ? t1.y : t1.x, 0.f} : Cf{t1.x, cj * t1.y};
                    // the chiral 6-vector: entries 0..2 belong to lane s = 0, 3..5 to s = 1
                    const bool mine = (cc < 3) == (s == 0);
                    const int c3 = cc % 3;
                    w1 = cadd(w1, cmul(np, mine ? U1[c3] : V1[c3]));
                    w2 = cadd(w2, cmul(nm, mine ? U2[c3] : V2[c3]));
                }
                // (C_inv H)_s = w1 + w2, (C_inv H)_{s+2} = w1 - w2
                Cf xs = ld2(&ib[elem(g, st.l, st.s, 12, s * 3 + rr)]);
                Cf xs2 = ld2(&ib[elem(g, st.l, st.s, 12, (s + 2) * 3 + rr)]);
                if (on[nt]) {
                    ob[elem(g, st.l, st.s, 12, s * 3 + rr)] =
                        make_float2(xs.re - kap * (w1.re + w2.re), xs.im - kap * (w1.im + w2.im));
                    ob[elem(g, st.l, st.s, 12, (s + 2) * 3 + rr)] =
                        make_float2(xs2.re - kap * (w1.re - w2.re), xs2.im - kap * (w1.im - w2.im));
                }
            }
        }
    }
}

// The vector alternative for the autotuner: one thread per site and group of NR
// right-hand sides (each link and the C_inv block are loaded once per group), the
// groups' workgroups of a block launched back to back on the same XCD, so the block's
// links and C_inv come from HBM once and from L2 for the other groups (loaded with
// ordinary, cached loads for that reason).  PIN: input storage precision (1 FP32,
// 2 FP16 with per-site scales).
template <int B, int PIN, int NR>
__global__ void __launch_bounds__(256) k_dirac_rhs_vec(Geom gin, MrhsArgs a)
{
    const Geom g = fixed_shape<B>(gin);
    const int ngrp = (a.nrhs + NR - 1) / NR;
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    const int blk = w / ngrp, grp = w - blk * ngrp;
    const int r0 = grp * NR, cnt = a.nrhs - r0 < NR ? a.nrhs - r0 : NR;
    const long long i = (long long)blk * 256 + threadIdx.x;
    if (i >= g.V) return;
    Site st;
    decode(g, i, st);
    const long long RS = 12 * g.V;
    auto in_of = [&](int r) {
        if constexpr (PIN == 1) {
            return SpinorField<1>{(float2 *)(a.in + r * RS)};
        } else {
            __half2 *h = (__half2 *)((char *)a.in16 + r * g.V * (12 * sizeof(__half2) + sizeof(float)));
            return SpinorField<2>{h, (float *)(h + RS)};
        }
    };
    LinkField<1> U{a.u};
    Spinor<float> acc[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) zero(acc[q]);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
        for (int dir = 1; dir >= -1; dir -= 2) {
            bool wrap, inblk;
            const long long j = neighbour(g, st, mu, dir, wrap, inblk);
            const int lj = (int)(j >> g.lbvol), sj = (int)(j & (g.bvol - 1));
            Mat3<float> W;
            if (dir > 0)
                U.load(g, st.l, st.s, mu, W);
            else
                U.load(g, lj, sj, mu, W);
            const cx<float> phase = {(float)a.phase.re[mu], (float)(dir > 0 ? a.phase.im[mu] : -a.phase.im[mu])};
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                if (q >= cnt) break;
                Spinor<float> psi;
                in_of(r0 + q).load(g, lj, sj, psi);
                hop(mu, dir, W, psi, wrap, phase, acc[q]);
            }
        }
    }
    Clov<float> cl;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
            float2 t = a.cinv[elem(g, st.l, st.s, 36, b * 18 + jj)];
            cl.d[b][2 * jj] = t.x;
            cl.d[b][2 * jj + 1] = t.y;
        }
#pragma unroll
        for (int jj = 0; jj < 15; ++jj) {
            float2 t = a.cinv[elem(g, st.l, st.s, 36, b * 18 + 3 + jj)];
            cl.h[b][jj] = {t.x, t.y};
        }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        if (q >= cnt) break;
        Spinor<float> x, t, o;
        in_of(r0 + q).load(g, st.l, st.s, x);
        clover_mul(cl, acc[q], t);
#pragma unroll
        for (int aa = 0; aa < 4; ++aa)
#pragma unroll
            for (int c = 0; c < 3; ++c) o.v[aa][c] = x.v[aa][c] - (float)a.kappa * t.v[aa][c];
        SpinorField<1>{a.out + (r0 + q) * RS}.store(g, st.l, st.s, o, true);
    }
}

// The batched A with the block's links and C_inv resident for the whole tile (4^4 blocks): a
// workgroup per block, a thread per site.  The block's forward links (their two stored rows)
// are staged in LDS, where the in-block backward hops find them as well, and each thread keeps
// its C_inv blocks in registers.  The right-hand sides then follow one another: each is staged
// in LDS as stored (FP16 with its site scales, or FP32); in-block neighbours and backward links
// are read from LDS and the others (sites on the block's faces) from global memory; row 2 of a
// link is rebuilt where it is used.  The vector kernels read every link and C_inv block again,
// from L2, for each group of right-hand sides; here the block's own fields are read once per
// tile, and a right-hand side costs its own spinor, its cross-block neighbours (with their
// links) and the output.
template <int PIN> struct ResT;
template <> struct ResT<1> { using T = float2; };
template <> struct ResT<2> { using T = __half2; };

template <int PIN>
__global__ void __launch_bounds__(256) k_dirac_rhs_res(Geom gin, MrhsArgs a)
{
    using T = typename ResT<PIN>::T;
    const Geom g = fixed_shape<4>(gin);
    __shared__ float2 lk[4][6][256];  // rows 0 and 1 of U_mu at each site of the block
    __shared__ T tile[12][256];       // the right-hand side in turn, as stored
    __shared__ float tsc[PIN == 2 ? 256 : 1];
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    const int s = threadIdx.x;
    Site st;
    decode(g, ((long long)w << 8) + s, st);
    const long long RS = 12 * g.V;
    auto elems = [&](int r) -> const T * {
        if constexpr (PIN == 1)
            return a.in + r * RS;
        else
            return (const T *)((const char *)a.in16 + r * g.V * (12 * sizeof(__half2) + sizeof(float)));
    };
    auto scales = [&](int r) -> const float * {
        if constexpr (PIN == 1)
            return nullptr;
        else
            return (const float *)(elems(r) + RS);
    };
    // the block's fields, once for the tile
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int e = 0; e < 6; ++e) lk[mu][e][s] = a.u[elem(g, st.l, s, 24, mu * 6 + e)];
    Clov<float> cl;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
            float2 t = a.cinv[elem(g, st.l, s, 36, b * 18 + jj)];
            cl.d[b][2 * jj] = t.x;
            cl.d[b][2 * jj + 1] = t.y;
        }
#pragma unroll
        for (int jj = 0; jj < 15; ++jj) {
            float2 t = a.cinv[elem(g, st.l, s, 36, b * 18 + 3 + jj)];
            cl.h[b][jj] = {t.x, t.y};
        }
    }
    // one stored spinor from 12 elements 256 apart (LDS or global) and its scale
    auto get = [&](const T *p, const float *sp, Spinor<float> &x) {
        const float sc = PIN == 2 ? *sp : 1.f;
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            float2 t;
            if constexpr (PIN == 2)
                t = __half22float2(p[e * 256]);
            else
                t = p[e * 256];
            x.v[e / 3][e % 3] = {t.x * sc, t.y * sc};
        }
    };
    for (int r = 0; r < a.nrhs; ++r) {
        wg_barrier();  // the fields are staged; the previous right-hand side is done with the tile
        // the site is decoded afresh for each right-hand side, from an index the compiler cannot
        // follow across them: otherwise it keeps every hop's addresses in registers throughout
        int sl = s;
        asm volatile("" : "+v"(sl));
        decode(g, ((long long)w << 8) + sl, st);
        {
            const T *p = elems(r) + elem(g, st.l, s, 12, 0);
#pragma unroll
            for (int e = 0; e < 12; ++e) tile[e][s] = p[e * 256];
            if constexpr (PIN == 2) tsc[s] = scales(r)[((long long)st.l << 8) + s];
        }
        wg_barrier();
        Spinor<float> acc;
        zero(acc);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
            for (int dir = 1; dir >= -1; dir -= 2) {
                bool wrap, inblk;
                const long long j = neighbour(g, st, mu, dir, wrap, inblk);
                const int lj = (int)(j >> 8), sj = (int)(j & 255);
                // in-block neighbours from LDS, the others from global memory (two paths: a
                // pointer that may be either would make every read a flat load)
                Spinor<float> psi;
                Mat3<float> W;
                if (inblk) {
                    get(&tile[0][sj], PIN == 2 ? &tsc[sj] : nullptr, psi);
#pragma unroll
                    for (int e = 0; e < 6; ++e) {
                        const float2 t = lk[mu][e][dir > 0 ? s : sj];
                        W.m[e / 3][e % 3] = {t.x, t.y};
                    }
                } else {
                    get(elems(r) + elem(g, lj, sj, 12, 0), PIN == 2 ? scales(r) + j : nullptr, psi);
#pragma unroll
                    for (int e = 0; e < 6; ++e) {
                        const float2 t = dir > 0 ? lk[mu][e][s] : a.u[elem(g, lj, sj, 24, mu * 6 + e)];
                        W.m[e / 3][e % 3] = {t.x, t.y};
                    }
                }
                su3_row3(W);
                const cx<float> phase = {(float)a.phase.re[mu], (float)(dir > 0 ? a.phase.im[mu] : -a.phase.im[mu])};
                hop(mu, dir, W, psi, wrap, phase, acc);
            }
        }
        Spinor<float> x, t, o;
        get(&tile[0][s], PIN == 2 ? &tsc[s] : nullptr, x);
        clover_mul(cl, acc, t);
#pragma unroll
        for (int aa = 0; aa < 4; ++aa)
#pragma unroll
            for (int c = 0; c < 3; ++c) o.v[aa][c] = x.v[aa][c] - (float)a.kappa * t.v[aa][c];
        SpinorField<1>{a.out + r * RS}.store(g, st.l, s, o, true);
    }
}

// variants 0-7: column tiles per pass (1, 2, 3 or 6: 2, 4, 6 or 12 right-hand sides per
// pass) x workgroup size (64 or 256 threads); variants 8-11: the vector kernel above with
// 1, 2, 3 or 4 right-hand sides per thread; variant 12: the resident-field kernel (4^4 blocks;
// other block shapes run variant 8 in its place).  Fewer right-hand sides per pass or thread
// need fewer registers, so more wavefronts hide the load latency, at the price of
// reading the links and C_inv more often.
int mrhs_variant_count() { return 13; }

const char *mrhs_variant_name(int v)
{
    static const char *names[] = {"mfma4x4x1 2 rhs/pass, 64-thread wg",  "mfma4x4x1 2 rhs/pass, 256-thread wg",
                                  "mfma4x4x1 4 rhs/pass, 64-thread wg",  "mfma4x4x1 4 rhs/pass, 256-thread wg",
                                  "mfma4x4x1 6 rhs/pass, 64-thread wg",  "mfma4x4x1 6 rhs/pass, 256-thread wg",
                                  "mfma4x4x1 12 rhs/pass, 64-thread wg", "mfma4x4x1 12 rhs/pass, 256-thread wg",
                                  "vector, 1 rhs per thread",            "vector, 2 rhs per thread",
                                  "vector, 3 rhs per thread",            "vector, 4 rhs per thread",
                                  "resident links and C_inv, rhs in turn"};
    return (v >= 0 && v < 13) ? names[v] : "?";
}

// the vector kernel with NR right-hand sides per thread, FP32 or FP16 inputs
template <int PIN, int NR> static void launch_vec(const Geom &g, hipStream_t st, const MrhsArgs &a, bool cube4)
{
    const dim3 G((unsigned)((g.V + 255) / 256 * ((a.nrhs + NR - 1) / NR))), T(256);
    if (cube4)
        hipLaunchKernelGGL((k_dirac_rhs_vec<4, PIN, NR>), G, T, 0, st, g, a);
    else
        hipLaunchKernelGGL((k_dirac_rhs_vec<0, PIN, NR>), G, T, 0, st, g, a);
}

// the resident-field kernel: a workgroup per 4^4 block; other block shapes take the vector
// kernel with one right-hand side per thread
template <int PIN> static void launch_res(const Geom &g, hipStream_t st, const MrhsArgs &a, bool cube4)
{
    if (cube4)
        hipLaunchKernelGGL((k_dirac_rhs_res<PIN>), dim3((unsigned)g.nblk), dim3(256), 0, st, g, a);
    else
        launch_vec<PIN, 1>(g, st, a, cube4);
}

hipError_t launch_dirac_mrhs(const Geom &g, hipStream_t st, const MrhsArgs &a, int variant)
{
    auto grid = [&](int wgs) { return dim3((unsigned)((g.V * 4 + wgs - 1) / wgs)); };
    // the vector kernels run with the block shape fixed at compile time for 4^4 blocks (fewer
    // registers); the matrix-core kernels' registers are their accumulators, they stay generic
    const bool cube4 = g.b[0] == 4 && g.b[1] == 4 && g.b[2] == 4 && g.b[3] == 4;
    if (a.pin == 2) {  // FP16-storage inputs: the vector kernels only
        switch (variant) {
        case 12: launch_res<2>(g, st, a, cube4); break;
        case 9: launch_vec<2, 2>(g, st, a, cube4); break;
        case 10: launch_vec<2, 3>(g, st, a, cube4); break;
        case 11: launch_vec<2, 4>(g, st, a, cube4); break;
        default: launch_vec<2, 1>(g, st, a, cube4); break;
        }
        return hipGetLastError();
    }
    if (a.pin != 1) return hipErrorInvalidValue;
    switch (variant) {
    case 0: hipLaunchKernelGGL((k_dirac_mrhs<1, 64, 0>), grid(64), dim3(64), 0, st, g, a); break;
    case 1: hipLaunchKernelGGL((k_dirac_mrhs<1, 256, 0>), grid(256), dim3(256), 0, st, g, a); break;
    case 2: hipLaunchKernelGGL((k_dirac_mrhs<2, 64, 0>), grid(64), dim3(64), 0, st, g, a); break;
    case 3: hipLaunchKernelGGL((k_dirac_mrhs<2, 256, 0>), grid(256), dim3(256), 0, st, g, a); break;
    case 4: hipLaunchKernelGGL((k_dirac_mrhs<3, 64, 0>), grid(64), dim3(64), 0, st, g, a); break;
    case 5: hipLaunchKernelGGL((k_dirac_mrhs<3, 256, 0>), grid(256), dim3(256), 0, st, g, a); break;
    case 6: hipLaunchKernelGGL((k_dirac_mrhs<6, 64, 0>), grid(64), dim3(64), 0, st, g, a); break;
    case 7: hipLaunchKernelGGL((k_dirac_mrhs<6, 256, 0>), grid(256), dim3(256), 0, st, g, a); break;
    case 12: launch_res<1>(g, st, a, cube4); break;
    case 9: launch_vec<1, 2>(g, st, a, cube4); break;
    case 10: launch_vec<1, 3>(g, st, a, cube4); break;
    case 11: launch_vec<1, 4>(g, st, a, cube4); break;
    default: launch_vec<1, 1>(g, st, a, cube4); break;
    }
    return hipGetLastError();
}

}  // namespace dd
