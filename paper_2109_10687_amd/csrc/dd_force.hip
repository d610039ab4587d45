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

__global__ void __launch_bounds__(BLAS_WG) k_force_y(Geom g, SpinorField<0> psi, SpinorField<0> chi,
                                                     const double2 *u64, SigmaBlocks sig, double kcsw, double kappa,
                                                     double2 *Y, double *partials)
{
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
                if (partials) {
                    Mat3<double> F;
                    field_strength(g, u64, i, mu, nu, F);
                    cx<double> tr = {0.0, 0.0};
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) tr = tr + F.m[a][b] * lam[b][a];
                    v[0] += 2.0 * kappa * tr.im;
                }
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

// C += A B
DD_INL void madd3(Mat3<double> &C, const Mat3<double> &A, const Mat3<double> &B)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cx<double> s = C.m[i][j];
            for (int k = 0; k < 3; ++k) s = s + A.m[i][k] * B.m[k][j];
            C.m[i][j] = s;
        }
}

DD_INL int plane_index(int a, int b)  // a < b
{
    return a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
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

    // ---- hop term
    Mat3<double> W;
    {
        Spinor<double> pn, pj, xn, xj, t1, t2;
        psi.load(g, st.l, st.s, pn);
        psi.load(g, lj, sj, pj);
        chi.load(g, st.l, st.s, xn);
        chi.load(g, lj, sj, xj);
        Half<double> h;
        zero(t1);
        zero(t2);
        project(mu, +1, pj, h);
        reconstruct(mu, +1, h, t1);  // (1 - gamma_mu) psi(n+mu)
        project(mu, -1, pn, h);
        reconstruct(mu, -1, h, t2);  // (1 + gamma_mu) psi(n)
        cx<double> phase = wrap ? cx<double>{ph.re[mu], ph.im[mu]} : cx<double>{1.0, 0.0};
        const cx<double> k2 = (2.0 * kappa) * phase;
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                cx<double> s = {0.0, 0.0};
                for (int al = 0; al < 4; ++al) {
                    s = s + cmulc(xn.v[al][a], t1.v[al][b]);  // t1_b conj(chi(n)_a)
                    s = s + cmulc(t2.v[al][a], xj.v[al][b]);  // conj(t2_a) chi(n+mu)_b
                }
                W.m[b][a] = k2 * s;
            }
    }

    // ---- clover term
    if (Y) {
        for (int nu = 0; nu < 4; ++nu) {
            if (nu == mu) continue;
            const int plane = mu < nu ? plane_index(mu, nu) : plane_index(nu, mu);
            const double orient = mu < nu ? 1.0 : -1.0;
            for (int sd = 1; sd >= -1; sd -= 2) {
                // the staple path n+mu -> n+mu+sd*nu -> n+sd*nu -> n
                const long long n_s = step(g, i, nu, sd);    // n + sd nu
                const long long j_s = step(g, j, nu, sd);    // n + mu + sd nu
                Mat3<double> Z2, Z3, Z4, m;
                if (sd > 0) {
                    load_link64(g, u64, j, nu, m);
                    Z2 = m;                                  // U_nu(n+mu)
                    load_link64(g, u64, n_s, mu, m);
                    dag3(m, Z3);                             // U_mu(n+nu)^dagger
                    load_link64(g, u64, i, nu, m);
                    dag3(m, Z4);                             // U_nu(n)^dagger
                } else {
                    load_link64(g, u64, j_s, nu, m);
                    dag3(m, Z2);                             // U_nu(n+mu-nu)^dagger
                    load_link64(g, u64, n_s, mu, m);
                    dag3(m, Z3);                             // U_mu(n-nu)^dagger
                    load_link64(g, u64, n_s, nu, Z4);        // U_nu(n-nu)
                }
                const double sgn = orient * (double)sd;
                Mat3<double> T34, Z23, S, Yc, t;
                mul3(Z3, Z4, T34);
                mul3(Z2, Z3, Z23);
                // Z2 Z3 Y(d4) Z4, d4 = n + sd nu
                load_y(g, Y, n_s, plane, sgn, Yc);
                mul3(Yc, Z4, t);
                madd3(W, Z23, t);
                // Z2 Y(d3) Z3 Z4, d3 = n + mu + sd nu
                load_y(g, Y, j_s, plane, sgn, Yc);
                mul3(Yc, T34, t);
                madd3(W, Z2, t);
                mul3(Z2, T34, S);
                // Y(d2) S, d2 = n + mu
                load_y(g, Y, j, plane, sgn, Yc);
                madd3(W, Yc, S);
                // S Y(d1), d1 = n
                load_y(g, Y, i, plane, sgn, Yc);
                madd3(W, S, Yc);
            }
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
                       SpinorField<0>{(double2 *)a.chi}, (const double2 *)a.u64, a.sig, a.kcsw, a.kappa,
                       (double2 *)a.y, a.partials);
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
