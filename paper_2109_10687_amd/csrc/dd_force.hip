// dd_force.hip -- derivative of L = |D^{-1} phi|^2 with respect to the gauge
// links and to c_SW: the fermion-force bilinear of the operator of the
// appendix, D = 1 + C - kappa H.
//
// With psi = D^{-1} phi and chi = D^{-dagger} psi (D^dagger = gamma_5 D gamma_5),
// dL = -2 Re <chi| dD psi>.  Per link U_mu(n) the kernels build the 3x3 matrix
// W_mu(n) with dL = Re sum tr(dU_mu(n) W_mu(n)):
//
//   hop:    W += 2 kappa phase_mu(n) ( [(1 - gamma_mu) psi(n+mu)] chi(n)^dagger
//                                    + ( [(1 + gamma_mu) psi(n)] chi(n+mu)^dagger )^dagger )
//           (outer products over colour, summed over spin);
//   clover: C = i kappa c_SW sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu},
//           F = (Q - Q^dagger)/8, gives dL = Re sum tr(dQ_{mu nu}(n) Y_{mu nu}(n)) with
//           Y = (-i kappa c_SW / 4)(Lambda + Lambda^dagger), anti-Hermitian, and
//           Lambda_{ba} = sum_{alpha beta} sigma_{alpha beta} psi_{b beta} conj(chi_{a alpha}).
//           Every plaquette through the link contributes: for the closed path
//           U Z2 Z3 Z4 (corners d1 = n, d2 = n+mu, d3, d4) the derivative with
//           respect to U is  Y(d2) Z2 Z3 Z4 + Z2 Y(d3) Z3 Z4 + Z2 Z3 Y(d4) Z4 + Z2 Z3 Z4 Y(d1),
//           with Y of the plane taken with the sign of the orientation: + for the
//           plaquette n -> n+mu -> n+mu+nu -> n+nu when mu < nu, and the sign
//           flips with nu > mu and for the plaquette on the -nu side.  Six
//           plaquettes per link (two per other direction), each seen from its
//           four corners: the 24 leaves a link enters.
//   c_SW:   dL/dc_SW = -2 Re <chi| (C / c_SW) psi> = 2 kappa sum_{n, mu<nu} Im tr(F_{mu nu} Lambda_{mu nu}).
//
// Output per link: G = W^dagger, the gradient dL/dRe U + i dL/dIm U entry by
// entry, or (su(3) form) the traceless Hermitian F_mu(n) = (i/2)(X - X^dagger)
// - tr/3, X = U W, with dL = tr(omega F) for U -> exp(i omega) U.
//
// Two kernels: k_force_y computes Y for the six planes of every site (FP64,
// 54 complex per site, block-major like every other field) and the c_SW sum;
// k_force_w gathers per link.  Both in FP64: the force is taken once per solve.
#include <mutex>

#include "dd_device.h"
#include "dd_gauge.h"
#include "dd_launch.h"

namespace dd {

// Work field of the force for the entry point that allocates nothing: a fixed
// file-scope device array (each GPU holds its own copy, at its own address, until
// the process ends).  Host code never passes `scratch` itself to a kernel -- on the
// host that name is only a stand-in -- but the device address looked up below.
static __device__ __align__(256) unsigned char scratch[FORCE_SCRATCH_BYTES];

hipError_t force_scratch_address(void **ptr)
{
    // once per device, with that device current
    static std::mutex mu;
    static void *addr[MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

// chiral components of a spinor: u[blk][s][c] = psi_s + (-1)^blk psi_{s+2}
// (the rotation P = [[1, 1], [1, -1]] / sqrt 2 without the 1/sqrt 2)
DD_INL void chiral(const Spinor<double> &p, cx<double> (&u)[2][2][3])
{
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            u[0][s][c] = p.v[s][c] + p.v[s + 2][c];
            u[1][s][c] = p.v[s][c] - p.v[s + 2][c];
        }
}

// dL/dc_SW: with c_SW != 0 from the clover blocks already built, -(2 / c_SW) Re <chi| C psi>
// with C psi = (1 + C) psi - psi per site; at c_SW = 0 (no clover to read it from) from the
// field strength, 2 kappa sum Im tr(F Lambda) over the planes
__global__ void __launch_bounds__(BLAS_WG) k_force_y(Geom g, SpinorField<0> psi, SpinorField<0> chi,
                                                     const double2 *u64, CloverField<0> clov, SigmaBlocks sig,
                                                     double kcsw, double kappa, double csw, double2 *Y,
                                                     double *partials)
{
    const bool from_clover = csw != 0.0;
    double v[1] = {0.0};
    for (long long i = (long long)blockIdx.x * BLAS_WG + threadIdx.x; i < g.V; i += (long long)gridDim.x * BLAS_WG) {
        const int l = (int)(i >> g.lbvol), s = (int)(i & (g.bvol - 1));
        Spinor<double> p, x;
        psi.load(g, l, s, p);
        chi.load(g, l, s, x);
        cx<double> up[2][2][3], ux[2][2][3];
        chiral(p, up);
        chiral(x, ux);
        int plane = 0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu, ++plane) {
                // sigma = P u P with u = diag(sig blocks), P symmetric: the bilinear in
                // the chiral components carries a factor 1/2
                cx<double> lam[3][3];
                for (int b = 0; b < 3; ++b)
                    for (int a = 0; a < 3; ++a) lam[b][a] = {0.0, 0.0};
                for (int blk = 0; blk < 2; ++blk)
                    for (int s1 = 0; s1 < 2; ++s1)
                        for (int s2 = 0; s2 < 2; ++s2) {
                            cx<double> sg = {0.5 * sig.re[plane][blk][s1][s2], 0.5 * sig.im[plane][blk][s1][s2]};
                            if (sg.re == 0.0 && sg.im == 0.0) continue;
                            for (int b = 0; b < 3; ++b) {
                                cx<double> t = sg * up[blk][s2][b];
                                for (int a = 0; a < 3; ++a) lam[b][a] = lam[b][a] + cmulc(ux[blk][s1][a], t);
                            }
                        }
                // Y = (-i kcsw / 4)(lam + lam^dagger)
                const double f = 0.25 * kcsw;
                for (int b = 0; b < 3; ++b)
                    for (int a = 0; a < 3; ++a) {
                        cx<double> h = lam[b][a] + conj(lam[a][b]);
                        Y[elem(g, l, s, 54, plane * 9 + b * 3 + a)] = make_double2(f * h.im, -f * h.re);
                    }
                if (partials && !from_clover) {
                    Mat3<double> F;
                    field_strength(g, u64, i, mu, nu, F);
                    cx<double> tr = {0.0, 0.0};
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) tr = tr + F.m[a][b] * lam[b][a];
                    v[0] += 2.0 * kappa * tr.im;
                }
            }
        if (partials && from_clover) {
            Clov<double> cl;
            clov.load(g, l, s, cl);
            Spinor<double> t;
            clover_mul(cl, p, t);
            double re = 0.0;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) re += cmulc(x.v[a][c], t.v[a][c] - p.v[a][c]).re;
            v[0] -= (2.0 / csw) * re;
        }
    }
    if (partials) wg_reduce_store<1>(v, partials);
}

DD_INL void load_y(const Geom &g, const double2 *Y, long long i, int plane, double sign, Mat3<double> &M)
{
    const int l = (int)(i >> g.lbvol), s = (int)(i & (g.bvol - 1));
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        double2 t = Y[elem(g, l, s, 54, plane * 9 + e)];
        M.m[e / 3][e % 3] = {sign * t.x, sign * t.y};
    }
}

// element (i, k) of A or of A^dagger
template <bool DAG> DD_INL cx<double> el(const Mat3<double> &A, int i, int k)
{
    return DAG ? conj(A.m[k][i]) : A.m[i][k];
}

// C = op(A) op(B), op the dagger where asked (no daggered copy is formed)
template <bool DA, bool DB> DD_INL void mulx(const Mat3<double> &A, const Mat3<double> &B, Mat3<double> &C)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> s = el<DA>(A, i, 0) * el<DB>(B, 0, j);
            s = s + el<DA>(A, i, 1) * el<DB>(B, 1, j);
            C.m[i][j] = s + el<DA>(A, i, 2) * el<DB>(B, 2, j);
        }
}

// C += op(A) op(B)
template <bool DA, bool DB> DD_INL void maddx(const Mat3<double> &A, const Mat3<double> &B, Mat3<double> &C)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> s = C.m[i][j] + el<DA>(A, i, 0) * el<DB>(B, 0, j);
            s = s + el<DA>(A, i, 1) * el<DB>(B, 1, j);
            C.m[i][j] = s + el<DA>(A, i, 2) * el<DB>(B, 2, j);
        }
}

// W += f sum_k conj(a[k][col]) b[k][row] over the two spins of two half spinors: the spin
// trace of an outer product of two projected spinors
DD_INL void half_outer(const Half<double> &a, const Half<double> &b, cx<double> f, Mat3<double> &W)
{
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cx<double> s = cmulc(a.v[0][c], b.v[0][r]);
            s = s + cmulc(a.v[1][c], b.v[1][r]);
            W.m[r][c] = W.m[r][c] + f * s;
        }
}

DD_INL int plane_index(int a, int b)  // a < b
{
    return a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
}

// the derivative of the plaquettes through U_mu(n) in the (mu, nu) plane on the sd side,
// with Y of that plane (sign sgn) at its corners: for the closed path U Z2 Z3 Z4,
// W += Y(d2) S + S Y(d1) + Z2 (Z3 Y(d4) Z4 + Y(d3) Z3 Z4), S = Z2 Z3 Z4.  Z3 = U_mu(.)^dagger
// always; Z2 is daggered on the -nu side and Z4 on the +nu side.  Eight 3x3 products per
// plaquette, no daggered copies formed.
template <int SD>
DD_INL void staple_force(const Geom &g, const double2 *u64, const double2 *Y, long long i, long long j, int mu,
                         int nu, int plane, double sgn, Mat3<double> &W)
{
    constexpr bool DZ2 = SD < 0, DZ4 = SD > 0;
    const long long n_s = step(g, i, nu, SD);  // n + sd nu
    const long long j_s = step(g, j, nu, SD);  // n + mu + sd nu
    Mat3<double> L4, L3, T, A, B;
    load_link64(g, u64, SD > 0 ? i : n_s, nu, L4);  // Z4 = U_nu(n)^dagger, or U_nu(n - nu)
    load_y(g, Y, n_s, plane, sgn, T);               // Y(d4), d4 = n + sd nu
    {
        Mat3<double> t;
        mulx<false, DZ4>(T, L4, t);                 // Y(d4) Z4
        load_link64(g, u64, n_s, mu, L3);           // Z3 = U_mu(n + sd nu)^dagger
        mulx<true, DZ4>(L3, L4, A);                 // A = Z3 Z4
        mulx<true, false>(L3, t, B);                // B = Z3 Y(d4) Z4
    }
    Mat3<double> &L2 = L3;
    load_y(g, Y, j_s, plane, sgn, T);               // Y(d3), d3 = n + mu + sd nu
    load_link64(g, u64, SD > 0 ? j : j_s, nu, L2);  // Z2 = U_nu(n + mu), or U_nu(n + mu - nu)^dagger
    maddx<false, false>(T, A, B);                   // B += Y(d3) Z3 Z4
    maddx<DZ2, false>(L2, B, W);                    // W += Z2 B
    Mat3<double> &S = B;
    mulx<DZ2, false>(L2, A, S);                     // S = Z2 Z3 Z4
    Mat3<double> &T1 = A;
    load_y(g, Y, j, plane, sgn, T);                 // Y(d2), d2 = n + mu
    load_y(g, Y, i, plane, sgn, T1);                // Y(d1), d1 = n
    maddx<false, false>(T, S, W);
    maddx<false, false>(S, T1, W);
}

// one thread per site, blockIdx.y = mu; writes the canonical [4][Lt][Lz][Ly][Lx][3][3]
__global__ void __launch_bounds__(256) k_force_w(Geom g, SpinorField<0> psi, SpinorField<0> chi, const double2 *u64,
                                                 const double2 *Y, Phase4 ph, double kappa, int su3, double2 *out)
{
    const int mu = blockIdx.y;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= g.V) return;
    Site st;
    decode(g, i, st);
    bool wrap, inblk;
    const long long j = neighbour(g, st, mu, +1, wrap, inblk);
    const int lj = (int)(j >> g.lbvol), sj = (int)(j & (g.bvol - 1));

    // ---- hop term: 2 kappa phase times the spin traces of
    //   [(1 - gamma_mu) psi(n+mu)] chi(n)^dagger  and  ([(1 + gamma_mu) psi(n)] chi(n+mu)^dagger)^dagger,
    // each the trace over the two projected spins (1 -+ gamma_mu is twice a projector: the
    // trace equals sum_k conj(P chi)_k (P psi)_k for mu < 3, half of it for mu = 3, where the
    // projection carries the factor 2)
    Mat3<double> W;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) W.m[a][b] = {0.0, 0.0};
    {
        const cx<double> phase = wrap ? cx<double>{ph.re[mu], ph.im[mu]} : cx<double>{1.0, 0.0};
        const cx<double> k2 = ((mu == 3 ? 1.0 : 2.0) * kappa) * phase;
        Spinor<double> p;
        Half<double> hp, hx;
        psi.load(g, lj, sj, p);
        project(mu, +1, p, hp);        // P^- psi(n+mu)
        chi.load(g, st.l, st.s, p);
        project(mu, +1, p, hx);        // P^- chi(n)
        half_outer(hx, hp, k2, W);     // W[b][a] += k2 sum conj(hx_a) hp_b
        psi.load(g, st.l, st.s, p);
        project(mu, -1, p, hp);        // P^+ psi(n)
        chi.load(g, lj, sj, p);
        project(mu, -1, p, hx);        // P^+ chi(n+mu)
        half_outer(hp, hx, k2, W);     // W[b][a] += k2 sum conj(hp_a) hx_b
    }

    // ---- clover term: the six plaquettes through the link, staple by staple
    if (Y) {
#pragma unroll 1
        for (int nu = 0; nu < 4; ++nu) {
            if (nu == mu) continue;
            const int plane = mu < nu ? plane_index(mu, nu) : plane_index(nu, mu);
            const double orient = mu < nu ? 1.0 : -1.0;
            staple_force<+1>(g, u64, Y, i, j, mu, nu, plane, orient, W);
            staple_force<-1>(g, u64, Y, i, j, mu, nu, plane, -orient, W);
        }
    }

    // ---- output
    Mat3<double> O;
    if (su3) {
        Mat3<double> U, X;
        load_link64(g, u64, i, mu, U);
        mul3(U, W, X);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                cx<double> d = X.m[a][b] - conj(X.m[b][a]);
                O.m[a][b] = {-0.5 * d.im, 0.5 * d.re};  // (i/2) d
            }
        const double tr = (O.m[0][0].re + O.m[1][1].re + O.m[2][2].re) / 3.0;
        for (int a = 0; a < 3; ++a) O.m[a][a].re -= tr;
    } else {
        dag3(W, O);
    }
    const long long n = lex_index(g, st);
    double2 *dst = out + ((long long)mu * g.V + n) * 9;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) dst[a * 3 + b] = make_double2(O.m[a][b].re, O.m[a][b].im);
}

hipError_t launch_force(const Geom &g, hipStream_t st, const ForceArgs &a)
{
    const int nwg = blas_grid_sites(g);
    hipLaunchKernelGGL(k_force_y, dim3(nwg), dim3(BLAS_WG), 0, st, g, SpinorField<0>{(double2 *)a.psi},
                       SpinorField<0>{(double2 *)a.chi}, (const double2 *)a.u64,
                       CloverField<0>{(const double2 *)a.clov64}, a.sig, a.kcsw, a.kappa, a.csw, (double2 *)a.y,
                       a.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.partials) {
        e = launch_finalize(st, a.partials, nwg, 1, a.dcsw);
        if (e != hipSuccess) return e;
    }
    const dim3 grid((unsigned)((g.V + 255) / 256), 4);
    hipLaunchKernelGGL(k_force_w, grid, dim3(256), 0, st, g, SpinorField<0>{(double2 *)a.psi},
                       SpinorField<0>{(double2 *)a.chi}, (const double2 *)a.u64,
                       a.kcsw != 0.0 ? (const double2 *)a.y : nullptr, a.phase, a.kappa, a.su3, (double2 *)a.out);
    return hipGetLastError();
}

}  // namespace dd
