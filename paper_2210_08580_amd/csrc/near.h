// Quadrature of self and adjacent panel pairs (shared by the assembly and by
// the finite-difference derivative of the near blocks in the adjoint pass).
#pragma once
#include "fds_internal.h"
#include "hankel.h"

namespace fds {

struct W8 {
    double wp0[8];   // w_b psi_0(xi_b)
    double wp1[8];   // w_b psi_1(xi_b)
};

__device__ __forceinline__ double2 fma_cr(double s, double2 a, double2 acc) {
    return make_double2(fma(s, a.x, acc.x), fma(s, a.y, acc.y));
}

// Linear shape functions of a panel as c0 + c1 s, s = fraction of length from
// the shared node; `end` = the shared node is the panel's end (xi = 1).
__device__ __forceinline__ void corner_lin(bool end, int al, double& c0, double& c1) {
    if (end) {   // psi_0 = s, psi_1 = 1 - s
        c0 = al == 0 ? 0.0 : 1.0;
        c1 = al == 0 ? 1.0 : -1.0;
    } else {     // psi_0 = 1 - s, psi_1 = s
        c0 = al == 0 ? 1.0 : 0.0;
        c1 = al == 0 ? -1.0 : 1.0;
    }
}

// Blocks of a self (s = 1) or adjacent (s = 0: q = p - 1, s = 2: q = p + 1) panel
// pair: S_ab = int int psi_a psi_b g and D_ab = int int psi_a psi_b dg/dn_y, with
// the logarithmic parts integrated exactly (closed form on a self pair, Duffy's
// corner split with 32 points in the angle on adjacent pairs) and the smooth
// remainders by the 8 x 8 rule. px, py / qx, qy: the 8 Gauss points of the panels.
// YUK: the Yukawa kernel (1/2pi) K0(k R) instead of g (tab is then the K0 table);
// it has the same logarithmic part, its S block is real and no D block is formed.
template <bool WANT_D, bool YUK = false>
__device__ __forceinline__ void near_pair_blocks(const double* px, const double* py, const double* qx,
                                                 const double* qy, double hp, double hq, double nxp, double nyp,
                                                 double nxq, double nyq, int s, double k,
                                                 const double* __restrict__ tab, const double* __restrict__ gl32,
                                                 const W8& wt, double2 (&So)[2][2], double2 (&Do)[2][2]) {
    double2 Sr[2][2], Dr[2][2];
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
        for (int b2 = 0; b2 < 2; ++b2) {
            Sr[a2][b2] = make_double2(0.0, 0.0);
            Dr[a2][b2] = make_double2(0.0, 0.0);
        }
    for (int a = 0; a < 8; ++a) {
        const double xa = px[a], ya = py[a];
        for (int b = 0; b < 8; ++b) {
            const double dx = xa - qx[b], dy = ya - qy[b];
            const double R = sqrt(fma(dx, dx, dy * dy));
            const double2 g = YUK ? make_double2(yukawa_reg(k, R, tab), 0.0) : green_reg(k, R, tab);
            const double wa[2] = {wt.wp0[a], wt.wp1[a]};
            const double wb[2] = {wt.wp0[b], wt.wp1[b]};
            double2 rem = make_double2(0.0, 0.0);
            if (WANT_D && !YUK && s != 1) {
                const double2 r0 = dlayer_rem(k, R, tab);
                const double dn = fma(dx, nxq, dy * nyq) / R;
                rem = cscale(r0, dn);
            }
#pragma unroll
            for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
                for (int b2 = 0; b2 < 2; ++b2) {
                    Sr[a2][b2] = fma_cr(wa[a2] * wb[b2], g, Sr[a2][b2]);
                    Dr[a2][b2] = fma_cr(wa[a2] * wb[b2], rem, Dr[a2][b2]);
                }
        }
    }
    const double hh = hp * hq;
    double Lg[2][2], Dl[2][2];
    if (s == 1) {
        // int int psi_a psi_b log|x - y| = h^2 (log(h)/4 + J_ab), J_00 = J_11 = -7/16, J_01 = -5/16
        const double lh = 0.25 * log(hp);
        Lg[0][0] = Lg[1][1] = hp * hp * (lh - 7.0 / 16.0);
        Lg[0][1] = Lg[1][0] = hp * hp * (lh - 5.0 / 16.0);
        Dl[0][0] = Dl[0][1] = Dl[1][0] = Dl[1][1] = 0.0;
    } else {
        // directions from the shared node: tau = (-ny, nx)
        const double tpx = -nyp, tpy = nxp, tqx = -nyq, tqy = nxq;
        const bool end_x = (s == 2);   // q = p+1: shared node is the end of p, start of q
        const double ax = end_x ? -tpx : tpx, ay = end_x ? -tpy : tpy;
        const double bx = end_x ? tqx : -tqx, by = end_x ? tqy : -tqy;
        const double ab = ax * bx + ay * by;
        const double anq = ax * nxq + ay * nyq;
#pragma unroll
        for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
            for (int b2 = 0; b2 < 2; ++b2) {
                Lg[a2][b2] = 0.0;
                Dl[a2][b2] = 0.0;
            }
        for (int it = 0; it < 32; ++it) {
            const double tt = gl32[it], wtt = gl32[32 + it];
            const double f1 = hp * hp + hq * hq * tt * tt - 2.0 * hp * hq * tt * ab;
            const double f2 = hp * hp * tt * tt + hq * hq - 2.0 * hp * hq * tt * ab;
            const double lf1 = 0.5 * log(f1), lf2 = 0.5 * log(f2);
#pragma unroll
            for (int a2 = 0; a2 < 2; ++a2) {
                double a0, a1;
                corner_lin(end_x, a2, a0, a1);
#pragma unroll
                for (int b2 = 0; b2 < 2; ++b2) {
                    double b0, b1;
                    corner_lin(!end_x, b2, b0, b1);
                    const double c10 = a0 * b0, c11 = a1 * b0 + a0 * b1 * tt, c12 = a1 * b1 * tt;
                    const double c20 = a0 * b0, c21 = a1 * b0 * tt + a0 * b1, c22 = a1 * b1 * tt;
                    // int_0^1 rho^(m+1)(log rho + log f) = -1/(m+2)^2 + log f/(m+2)
                    const double g1 = c10 * (-0.25 + 0.5 * lf1) + c11 * (-1.0 / 9.0 + lf1 / 3.0) +
                                      c12 * (-1.0 / 16.0 + 0.25 * lf1);
                    const double g2 = c20 * (-0.25 + 0.5 * lf2) + c21 * (-1.0 / 9.0 + lf2 / 3.0) +
                                      c22 * (-1.0 / 16.0 + 0.25 * lf2);
                    Lg[a2][b2] += wtt * (g1 + g2);
                    const double d1 = (c10 + 0.5 * c11 + c12 / 3.0) * (hp * anq / f1);
                    const double d2 = (c20 + 0.5 * c21 + c22 / 3.0) * (hp * anq * tt / f2);
                    Dl[a2][b2] += wtt * (d1 + d2);
                }
            }
        }
#pragma unroll
        for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
            for (int b2 = 0; b2 < 2; ++b2) {
                Lg[a2][b2] *= hh;
                Dl[a2][b2] *= hh * kInv2Pi;
            }
    }
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
        for (int b2 = 0; b2 < 2; ++b2) {
            const double2 sv = cscale(Sr[a2][b2], hh);
            So[a2][b2] = make_double2(sv.x - kInv2Pi * Lg[a2][b2], sv.y);
            const double2 dv = cscale(Dr[a2][b2], hh);
            Do[a2][b2] = make_double2(dv.x + Dl[a2][b2], dv.y);
        }
}

}  // namespace fds
