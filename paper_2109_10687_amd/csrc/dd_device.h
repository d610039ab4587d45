// dd_device.h -- device-side building blocks of the gfx950 Clover-Wilson path:
// complex arithmetic, the block-major site geometry, storage accessors for
// spinors, links and the clover blocks, the spin-projected hop and the
// chiral-block clover multiply.
//
// Internal layout (block-major structure of arrays, "AoSoA"):
//   the lattice is cut into SAP blocks of extent b[mu] (powers of two);
//   blocks are numbered lexicographically, l = Bx + NBx*(By + NBy*(Bz + NBz*Bt));
//   a site inside a block has index s = x' + bx*(y' + by*(z' + bz*t'));
//   internal site index i = l*bvol + s.
//   A field with E complex elements per site stores element e of site (l, s)
//   at ((l*E + e) * bvol + s): consecutive lanes read consecutive addresses.
//   spinor   E = 12, element k = spin*3 + colour
//   link     E = 4*9  (element (mu*9 + a*3 + b)),  FP16 copy E = 4*6 (rows 0,1)
//   clover   E = 36: two 6x6 Hermitian blocks (gamma_5-diagonal basis), each
//            3 complex holding the 6 real diagonal entries pairwise, then the
//            15 upper off-diagonal entries row by row.
//   FP16 spinors carry one FP32 scale per site (max |component|), stored after
//   the 12*V half2 elements.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dd {

#define DD_INL __device__ __forceinline__
#define DD_HDI __host__ __device__ __forceinline__

// ------------------------------------------------------------------ LDS race check
// Compiled with -DDD_RACE_CHECK=n (n > 0), the kernels that share LDS between the
// wavefronts of a workgroup let wavefront w of W wait n*(W-1-w) sleep periods (about
// 3.4 us each) at entry and after every workgroup barrier, so the wavefronts run each
// phase between barriers in the reverse of their usual order.  A missing barrier then
// changes what a wavefront reads; the results of such a build must equal the normal
// build's bit for bit.  n = 0 (the product build) compiles the waits away.
#ifndef DD_RACE_CHECK
#define DD_RACE_CHECK 0
#endif

DD_INL void wg_skew()
{
    if constexpr (DD_RACE_CHECK > 0) {
        const unsigned nthr = blockDim.x * blockDim.y * blockDim.z;
        const unsigned tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
        const int nw = (int)((nthr + 63) >> 6), w = (int)(tid >> 6);
        for (int i = 0; i < (nw - 1 - w) * DD_RACE_CHECK; ++i) __builtin_amdgcn_s_sleep(127);
    }
}

// workgroup barrier (plus the race check's wait)
DD_INL void wg_barrier()
{
    __syncthreads();
    wg_skew();
}

// ------------------------------------------------------------------ complex
template <typename R>
struct cx {
    R re, im;
};

template <typename R> DD_HDI cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R> DD_HDI cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> DD_HDI cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> DD_HDI cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <typename R> DD_HDI cx<R> operator*(cx<R> a, cx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> DD_HDI cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R> DD_HDI cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename R> DD_HDI cx<R> cmulc(cx<R> a, cx<R> b)
{
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R> DD_HDI cx<R> itimes(cx<R> a) { return {-a.im, a.re}; }
template <typename R> DD_HDI R norm2(cx<R> a) { return a.re * a.re + a.im * a.im; }

template <typename R>
struct Spinor {
    cx<R> v[4][3];  // [spin][colour]
};

template <typename R>
struct Half {  // spin-projected half spinor: two spins x three colours
    cx<R> v[2][3];
};

template <typename R>
struct Mat3 {
    cx<R> m[3][3];
};

template <typename R>
struct Clov {  // two Hermitian 6x6 blocks: real diagonal + 15 upper entries
    R d[2][6];
    cx<R> h[2][15];
};

template <typename R> DD_INL void zero(Spinor<R> &s)
{
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) s.v[a][c] = {R(0), R(0)};
}

// ------------------------------------------------------------------ geometry
struct Geom {
    int L[4];        // lattice extents
    int b[4];        // block extents (powers of two)
    int sh[4];       // bit offset of the in-block coordinate mu inside s
    int NB[4];       // blocks per direction (even)
    int bstride[4];  // lexicographic block strides
    int bvol, lbvol, nblk;
    long long V;
};

struct Site {
    int l, s;
    int c[4];  // in-block coordinates
    int B[4];  // block coordinates
};

DD_INL void decode(const Geom &g, long long i, Site &st)
{
    st.l = (int)(i >> g.lbvol);
    st.s = (int)(i & (g.bvol - 1));
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) st.c[mu] = (st.s >> g.sh[mu]) & (g.b[mu] - 1);
    unsigned l = (unsigned)st.l;
    st.B[0] = (int)(l % (unsigned)g.NB[0]);
    l /= (unsigned)g.NB[0];
    st.B[1] = (int)(l % (unsigned)g.NB[1]);
    l /= (unsigned)g.NB[1];
    st.B[2] = (int)(l % (unsigned)g.NB[2]);
    st.B[3] = (int)(l / (unsigned)g.NB[2]);
}

// block coordinates of lexicographic block l
DD_INL void block_coords(const Geom &g, int l, int B[4])
{
    unsigned u = (unsigned)l;
    B[0] = (int)(u % (unsigned)g.NB[0]);
    u /= (unsigned)g.NB[0];
    B[1] = (int)(u % (unsigned)g.NB[1]);
    u /= (unsigned)g.NB[1];
    B[2] = (int)(u % (unsigned)g.NB[2]);
    B[3] = (int)(u / (unsigned)g.NB[2]);
}

// the w-th block of colour `colour` (colour = parity of the block coordinates)
DD_INL int colour_block(const Geom &g, int colour, int w)
{
    int B[4];
    block_coords(g, 2 * w, B);  // NB[0] is even: blocks 2w and 2w+1 differ only in Bx
    int j = (colour + B[0] + B[1] + B[2] + B[3]) & 1;
    return 2 * w + j;
}

// neighbour of a decoded site in direction mu (dir = +1/-1); `wrap` tells
// whether the hop crosses the lattice edge; `inblk` whether it stays in the block
DD_INL long long neighbour(const Geom &g, const Site &st, int mu, int dir, bool &wrap, bool &inblk)
{
    int c = st.c[mu] + dir;
    int stride = 1 << g.sh[mu];
    if (c >= 0 && c < g.b[mu]) {
        wrap = false;
        inblk = true;
        return ((long long)st.l << g.lbvol) + st.s + dir * stride;
    }
    inblk = false;
    int B = st.B[mu] + dir;
    int l = st.l + dir * g.bstride[mu];
    wrap = false;
    if (B < 0) {
        l += g.NB[mu] * g.bstride[mu];
        wrap = true;
    } else if (B >= g.NB[mu]) {
        l -= g.NB[mu] * g.bstride[mu];
        wrap = true;
    }
    int s = st.s - dir * (g.b[mu] - 1) * stride;
    return ((long long)l << g.lbvol) + s;
}

// lexicographic index of a decoded site
DD_INL long long lex_index(const Geom &g, const Site &st)
{
    long long x[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) x[mu] = (long long)st.B[mu] * g.b[mu] + st.c[mu];
    return x[0] + g.L[0] * (x[1] + (long long)g.L[1] * (x[2] + (long long)g.L[2] * x[3]));
}

DD_INL long long elem(const Geom &g, int l, int s, int E, int e)
{
    return (((long long)l * E + e) << g.lbvol) + s;
}

// The geometry with the block shape fixed to B^4 at compile time (B = 2, 4, 8):
// block extents, in-block strides and the block volume become constants, so the
// compiler folds the in-block index arithmetic and turns offsets into immediates.
// B = 0 keeps the run-time shape.
template <int B> DD_INL Geom fixed_shape(const Geom &gin)
{
    static_assert(B == 0 || B == 2 || B == 4 || B == 8, "block side");
    Geom g = gin;
    if (B > 0) {
        constexpr int lb = B == 2 ? 1 : B == 4 ? 2 : 3;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            g.b[mu] = B;
            g.sh[mu] = mu * lb;
        }
        g.bvol = B * B * B * B;
        g.lbvol = 4 * lb;
    }
    return g;
}

// workgroup id -> work item, spreading consecutive items over one XCD: the
// hardware deals workgroups round-robin to the 8 XCDs, so item
// (w % 8) * (n / 8) + w / 8 keeps neighbouring items on the same L2.
DD_INL int xcd_remap(int w, int n)
{
    if (n % 8 != 0) return w;
    return (w & 7) * (n >> 3) + (w >> 3);
}

// ------------------------------------------------------------------ streaming access
// Non-temporal loads and stores for data a kernel touches once (the clover
// blocks, the Dirac apply's output): they do not displace the spinors and links
// that neighbouring sites read again from L2.
typedef double d2nt_t __attribute__((ext_vector_type(2)));
typedef float f2nt_t __attribute__((ext_vector_type(2)));
DD_INL double2 ld_stream(const double2 *p)
{
    d2nt_t v = __builtin_nontemporal_load((const d2nt_t *)p);
    return make_double2(v.x, v.y);
}
DD_INL float2 ld_stream(const float2 *p)
{
    f2nt_t v = __builtin_nontemporal_load((const f2nt_t *)p);
    return make_float2(v.x, v.y);
}
DD_INL __half2 ld_stream(const __half2 *p)
{
    unsigned int v = __builtin_nontemporal_load((const unsigned int *)p);
    return *reinterpret_cast<__half2 *>(&v);
}
DD_INL void st_stream(double2 *p, double2 x)
{
    d2nt_t v = {x.x, x.y};
    __builtin_nontemporal_store(v, (d2nt_t *)p);
}
DD_INL void st_stream(float2 *p, float2 x)
{
    f2nt_t v = {x.x, x.y};
    __builtin_nontemporal_store(v, (f2nt_t *)p);
}
DD_INL void st_stream(__half2 *p, __half2 x) { __builtin_nontemporal_store(*reinterpret_cast<unsigned int *>(&x), (unsigned int *)p); }
DD_INL void st_stream(float *p, float x) { __builtin_nontemporal_store(x, p); }

// ------------------------------------------------------------------ storage
// precision tags: 0 = FP64, 1 = FP32, 2 = FP16 (per-site scaled spinors,
// 12-real links, FP16 clover)
template <int P> struct Real;
template <> struct Real<0> { using T = double; };
template <> struct Real<1> { using T = float; };
template <> struct Real<2> { using T = float; };

template <int P> struct SpinorField;

template <> struct SpinorField<0> {
    double2 *p;
    template <typename R> DD_INL void load(const Geom &g, int l, int s, Spinor<R> &x) const
    {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double2 t = p[elem(g, l, s, 12, a * 3 + c)];
                x.v[a][c] = {R(t.x), R(t.y)};
            }
    }
    template <typename R> DD_INL void store(const Geom &g, int l, int s, const Spinor<R> &x, bool stream = false) const
    {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double2 v = make_double2(x.v[a][c].re, x.v[a][c].im);
                if (stream)
                    st_stream(&p[elem(g, l, s, 12, a * 3 + c)], v);
                else
                    p[elem(g, l, s, 12, a * 3 + c)] = v;
            }
    }
};

template <> struct SpinorField<1> {
    float2 *p;
    template <typename R> DD_INL void load(const Geom &g, int l, int s, Spinor<R> &x) const
    {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float2 t = p[elem(g, l, s, 12, a * 3 + c)];
                x.v[a][c] = {R(t.x), R(t.y)};
            }
    }
    template <typename R> DD_INL void store(const Geom &g, int l, int s, const Spinor<R> &x, bool stream = false) const
    {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float2 v = make_float2((float)x.v[a][c].re, (float)x.v[a][c].im);
                if (stream)
                    st_stream(&p[elem(g, l, s, 12, a * 3 + c)], v);
                else
                    p[elem(g, l, s, 12, a * 3 + c)] = v;
            }
    }
};

template <> struct SpinorField<2> {
    __half2 *p;    // 12 * V half2
    float *scale;  // V scales, right after the half2 block
    template <typename R> DD_INL void load(const Geom &g, int l, int s, Spinor<R> &x) const
    {
        float sc = scale[((long long)l << g.lbvol) + s];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float2 t = __half22float2(p[elem(g, l, s, 12, a * 3 + c)]);
                x.v[a][c] = {R(t.x * sc), R(t.y * sc)};
            }
    }
    template <typename R> DD_INL void store(const Geom &g, int l, int s, const Spinor<R> &x, bool stream = false) const
    {
        float m = 0.f;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                m = fmaxf(m, fabsf((float)x.v[a][c].re));
                m = fmaxf(m, fabsf((float)x.v[a][c].im));
            }
        float inv = m > 0.f ? 1.0f / m : 0.f;
        if (stream)
            st_stream(&scale[((long long)l << g.lbvol) + s], m);
        else
            scale[((long long)l << g.lbvol) + s] = m;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                __half2 v = __floats2half2_rn((float)x.v[a][c].re * inv, (float)x.v[a][c].im * inv);
                if (stream)
                    st_stream(&p[elem(g, l, s, 12, a * 3 + c)], v);
                else
                    p[elem(g, l, s, 12, a * 3 + c)] = v;
            }
    }
};

template <int P> struct LinkField;

template <> struct LinkField<0> {
    const double2 *p;
    template <typename R> DD_INL void load(const Geom &g, int l, int s, int mu, Mat3<R> &U) const
    {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                double2 t = p[elem(g, l, s, 36, mu * 9 + a * 3 + b)];
                U.m[a][b] = {R(t.x), R(t.y)};
            }
    }
};

// third row of an SU(3) matrix from its first two: conj(row0 x row1)
template <typename R> DD_INL void su3_row3(Mat3<R> &U)
{
    U.m[2][0] = conj(U.m[0][1] * U.m[1][2] - U.m[0][2] * U.m[1][1]);
    U.m[2][1] = conj(U.m[0][2] * U.m[1][0] - U.m[0][0] * U.m[1][2]);
    U.m[2][2] = conj(U.m[0][0] * U.m[1][1] - U.m[0][1] * U.m[1][0]);
}

// FP32 links: rows 0 and 1 as stored (12 reals, elem(l, s, 24, mu * 6 + a * 3 + b)), row 2
// rebuilt in FP32 (the traffic of the FP32 and FP16-input applies is HBM-bound; the
// rebuild is ALU work they have to spare)
template <> struct LinkField<1> {
    const float2 *p;
    template <typename R> DD_INL void load(const Geom &g, int l, int s, int mu, Mat3<R> &U) const
    {
        Mat3<float> W;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                float2 t = p[elem(g, l, s, 24, mu * 6 + a * 3 + b)];
                W.m[a][b] = {t.x, t.y};
            }
        su3_row3(W);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) U.m[a][b] = {R(W.m[a][b].re), R(W.m[a][b].im)};
    }
};

template <> struct LinkField<2> {
    const __half2 *p;
    template <typename R> DD_INL void load(const Geom &g, int l, int s, int mu, Mat3<R> &U) const
    {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                float2 t = __half22float2(p[elem(g, l, s, 24, mu * 6 + a * 3 + b)]);
                U.m[a][b] = {R(t.x), R(t.y)};
            }
        su3_row3(U);
    }
};

template <int P> struct CloverField;

template <typename R, typename V2> DD_INL void clov_from(const V2 *p, const Geom &g, int l, int s, Clov<R> &C)
{
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            V2 t = ld_stream(&p[elem(g, l, s, 36, blk * 18 + j)]);
            C.d[blk][2 * j] = R(t.x);
            C.d[blk][2 * j + 1] = R(t.y);
        }
#pragma unroll
        for (int j = 0; j < 15; ++j) {
            V2 t = ld_stream(&p[elem(g, l, s, 36, blk * 18 + 3 + j)]);
            C.h[blk][j] = {R(t.x), R(t.y)};
        }
    }
}

template <> struct CloverField<0> {
    const double2 *p;
    template <typename R> DD_INL void load(const Geom &g, int l, int s, Clov<R> &C) const { clov_from(p, g, l, s, C); }
};
template <> struct CloverField<1> {
    const float2 *p;
    template <typename R> DD_INL void load(const Geom &g, int l, int s, Clov<R> &C) const { clov_from(p, g, l, s, C); }
};
template <> struct CloverField<2> {
    const __half2 *p;
    template <typename R> DD_INL void load(const Geom &g, int l, int s, Clov<R> &C) const
    {
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                float2 t = __half22float2(ld_stream(&p[elem(g, l, s, 36, blk * 18 + j)]));
                C.d[blk][2 * j] = R(t.x);
                C.d[blk][2 * j + 1] = R(t.y);
            }
#pragma unroll
            for (int j = 0; j < 15; ++j) {
                float2 t = __half22float2(ld_stream(&p[elem(g, l, s, 36, blk * 18 + 3 + j)]));
                C.h[blk][j] = {R(t.x), R(t.y)};
            }
        }
    }
};

// ------------------------------------------------------------------ operators
// index of the upper entry (i < j) of a 6x6 Hermitian block, row by row
DD_HDI int upper_index(int i, int j) { return i * 6 - i * (i + 1) / 2 + (j - i - 1); }

// w = N u for one Hermitian 6x6 block
template <typename R> DD_INL void herm6(const R *d, const cx<R> *h, const cx<R> *u, cx<R> *w)
{
#pragma unroll
    for (int i = 0; i < 6; ++i) w[i] = d[i] * u[i];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i + 1; j < 6; ++j) {
            cx<R> hij = h[upper_index(i, j)];
            w[i] = w[i] + hij * u[j];
            w[j] = w[j] + cmulc(hij, u[i]);
        }
}

// out = Q diag(N+, N-) Q in, Q = [[1, 1], [1, -1]] on the spin pairs (0,1)/(2,3):
// the clover block applied in the basis where gamma_5 is diagonal
template <typename R> DD_INL void clover_mul(const Clov<R> &C, const Spinor<R> &in, Spinor<R> &out)
{
    cx<R> u[6], w[6], u2[6], w2[6];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            u[a * 3 + c] = in.v[a][c] + in.v[a + 2][c];
            u2[a * 3 + c] = in.v[a][c] - in.v[a + 2][c];
        }
    herm6(C.d[0], C.h[0], u, w);
    herm6(C.d[1], C.h[1], u2, w2);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            out.v[a][c] = w[a * 3 + c] + w2[a * 3 + c];
            out.v[a + 2][c] = w[a * 3 + c] - w2[a * 3 + c];
        }
}

// k = W h with W = U (dag = false) or U^dagger (dag = true), per spin of the half spinor
template <typename R> DD_INL void mat_half(const Mat3<R> &U, bool dag, const Half<R> &h, Half<R> &k)
{
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            cx<R> acc = {R(0), R(0)};
#pragma unroll
            for (int j = 0; j < 3; ++j) acc = acc + (dag ? cmulc(U.m[j][i], h.v[a][j]) : U.m[i][j] * h.v[a][j]);
            k.v[a][i] = acc;
        }
}

// spin projection h = upper two rows of (1 - s gamma_mu) psi, s = +1 forward,
// -1 backward, for the gamma matrices of the appendix.  For mu = 3 (gamma_4
// diagonal) the half spinor is the surviving spin pair scaled by 2.
template <typename R> DD_INL void project(int mu, int s, const Spinor<R> &p, Half<R> &h)
{
    R sr = R(s);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (mu == 0) {  // gamma_1: X = [[0, i], [i, 0]]
            h.v[0][c] = p.v[0][c] - sr * itimes(p.v[3][c]);
            h.v[1][c] = p.v[1][c] - sr * itimes(p.v[2][c]);
        } else if (mu == 1) {  // gamma_2: X = [[0, 1], [-1, 0]]
            h.v[0][c] = p.v[0][c] - sr * p.v[3][c];
            h.v[1][c] = p.v[1][c] + sr * p.v[2][c];
        } else if (mu == 2) {  // gamma_3: X = [[i, 0], [0, -i]]
            h.v[0][c] = p.v[0][c] - sr * itimes(p.v[2][c]);
            h.v[1][c] = p.v[1][c] + sr * itimes(p.v[3][c]);
        } else {  // gamma_4 = diag(1, 1, -1, -1)
            int o = s > 0 ? 2 : 0;
            h.v[0][c] = R(2) * p.v[o][c];
            h.v[1][c] = R(2) * p.v[o + 1][c];
        }
    }
}

// acc += (1 - s gamma_mu) rebuilt from k = W h
template <typename R> DD_INL void reconstruct(int mu, int s, const Half<R> &k, Spinor<R> &acc)
{
    R sr = R(s);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (mu == 0) {
            acc.v[0][c] = acc.v[0][c] + k.v[0][c];
            acc.v[1][c] = acc.v[1][c] + k.v[1][c];
            acc.v[2][c] = acc.v[2][c] + sr * itimes(k.v[1][c]);
            acc.v[3][c] = acc.v[3][c] + sr * itimes(k.v[0][c]);
        } else if (mu == 1) {
            acc.v[0][c] = acc.v[0][c] + k.v[0][c];
            acc.v[1][c] = acc.v[1][c] + k.v[1][c];
            acc.v[2][c] = acc.v[2][c] + sr * k.v[1][c];
            acc.v[3][c] = acc.v[3][c] - sr * k.v[0][c];
        } else if (mu == 2) {
            acc.v[0][c] = acc.v[0][c] + k.v[0][c];
            acc.v[1][c] = acc.v[1][c] + k.v[1][c];
            acc.v[2][c] = acc.v[2][c] + sr * itimes(k.v[0][c]);
            acc.v[3][c] = acc.v[3][c] - sr * itimes(k.v[1][c]);
        } else {
            int o = s > 0 ? 2 : 0;
            acc.v[o][c] = acc.v[o][c] + k.v[0][c];
            acc.v[o + 1][c] = acc.v[o + 1][c] + k.v[1][c];
        }
    }
}

// acc += (1 - s gamma_mu) W psi * phase   (W = U forward, U^dagger backward)
template <typename R>
DD_INL void hop(int mu, int s, const Mat3<R> &U, const Spinor<R> &psi, bool use_phase, cx<R> phase, Spinor<R> &acc)
{
    Half<R> h, k;
    project(mu, s, psi, h);
    mat_half(U, s < 0, h, k);
    if (use_phase) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) k.v[a][c] = k.v[a][c] * phase;
    }
    reconstruct(mu, s, k, acc);
}

// gamma_5 = [[0, 1], [1, 0]] on the spin pairs: swaps spins (0,1) and (2,3)
template <typename R> DD_INL void gamma5(Spinor<R> &p)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cx<R> t0 = p.v[0][c], t1 = p.v[1][c];
        p.v[0][c] = p.v[2][c];
        p.v[1][c] = p.v[3][c];
        p.v[2][c] = t0;
        p.v[3][c] = t1;
    }
}

}  // namespace dd
