// dd_gauge.h -- FP64 gauge-field helpers shared by the clover setup and the
// fermion force: neighbour stepping on internal site indices, 3x3 complex
// products and the four-leaf clover field strength (appendix "Clover-Wilson
// Dirac operator").
#pragma once

#include "dd_device.h"

namespace dd {

// site index of a neighbour given as an internal index (re-decoded)
DD_INL long long step(const Geom &g, long long i, int mu, int dir)
{
    Site st;
    decode(g, i, st);
    bool w, ib;
    return neighbour(g, st, mu, dir, w, ib);
}

DD_INL void load_link64(const Geom &g, const double2 *u, long long i, int mu, Mat3<double> &U)
{
    LinkField<0> f{u};
    f.load(g, (int)(i >> g.lbvol), (int)(i & (g.bvol - 1)), mu, U);
}

DD_INL void mul3(const Mat3<double> &A, const Mat3<double> &B, Mat3<double> &C)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cx<double> s = {0, 0};
            for (int k = 0; k < 3; ++k) s = s + A.m[i][k] * B.m[k][j];
            C.m[i][j] = s;
        }
}

DD_INL void dag3(const Mat3<double> &A, Mat3<double> &B)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B.m[i][j] = conj(A.m[j][i]);
}

// product of four links, each daggered or not, accumulated into Q
DD_INL void leaf(const Mat3<double> *M, const int *dg, Mat3<double> &Q)
{
    Mat3<double> acc, t, m;
    if (dg[0]) dag3(M[0], acc); else acc = M[0];
    for (int k = 1; k < 4; ++k) {
        if (dg[k]) dag3(M[k], m); else m = M[k];
        mul3(acc, m, t);
        acc = t;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Q.m[i][j] = Q.m[i][j] + acc.m[i][j];
}

// F_{mu nu}(n) = (Q - Q^dagger) / 8 with Q the four counter-clockwise
// plaquettes of the (mu, nu) plane through n
DD_INL void field_strength(const Geom &g, const double2 *u, long long n, int mu, int nu, Mat3<double> &F)
{
    long long n_pm = step(g, n, mu, +1), n_pn = step(g, n, nu, +1);
    long long n_mm = step(g, n, mu, -1), n_mn = step(g, n, nu, -1);
    long long n_mm_pn = step(g, n_mm, nu, +1), n_mm_mn = step(g, n_mm, nu, -1);
    long long n_pm_mn = step(g, n_pm, nu, -1);
    Mat3<double> Q;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Q.m[i][j] = {0, 0};
    Mat3<double> M[4];
    {
        load_link64(g, u, n, mu, M[0]); load_link64(g, u, n_pm, nu, M[1]);
        load_link64(g, u, n_pn, mu, M[2]); load_link64(g, u, n, nu, M[3]);
        const int dg[4] = {0, 0, 1, 1};
        leaf(M, dg, Q);
    }
    {
        load_link64(g, u, n, nu, M[0]); load_link64(g, u, n_mm_pn, mu, M[1]);
        load_link64(g, u, n_mm, nu, M[2]); load_link64(g, u, n_mm, mu, M[3]);
        const int dg[4] = {0, 1, 1, 0};
        leaf(M, dg, Q);
    }
    {
        load_link64(g, u, n_mm, mu, M[0]); load_link64(g, u, n_mm_mn, nu, M[1]);
        load_link64(g, u, n_mm_mn, mu, M[2]); load_link64(g, u, n_mn, nu, M[3]);
        const int dg[4] = {1, 1, 0, 0};
        leaf(M, dg, Q);
    }
    {
        load_link64(g, u, n_mn, nu, M[0]); load_link64(g, u, n_mn, mu, M[1]);
        load_link64(g, u, n_pm_mn, nu, M[2]); load_link64(g, u, n, mu, M[3]);
        const int dg[4] = {1, 0, 0, 1};
        leaf(M, dg, Q);
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) F.m[i][j] = 0.125 * (Q.m[i][j] - conj(Q.m[j][i]));
}

}  // namespace dd
