// Far-field objective of the inverse-problem use case and its adjoint gradient.
//
// Forward model: the unfiltered Galerkin TE-EFIE N j_r = -f_r (paper, Notation
// and Background), solved by the filtered fast solver as preconditioner and
// refinement against the unfiltered operator. Far field of u = -j (sound-hard
// boundary, Green's representation as the double layer of the total field):
//     u_inf(theta) = e^{i pi/4}/sqrt(8 pi k) int (-i k th.n_y) e^{-i k th.y} u(y) ds_y,
// with the 8-point Gauss rule per panel; as a matrix, (F j)_l.
// Objective J = sum_r sum_l |(F j_r)_l - T_lr|^2 and, with e_r = F j_r - T_r,
// N^H lambda_r = F^H e_r (N is complex symmetric, so mu_r = conj(lambda_r)
// solves N mu_r = conj(F^H e_r)),
//     dJ/dx = sum_r 2 Re[e_r^H (dF/dx) j_r] - 2 Re[mu_r^T (df_r/dx + (dN/dx) j_r)].
// The operator term is sum_ij M_ij dN_ij/dx with M = sum_r mu_r j_r^T (one GEMM);
// it is evaluated pair by pair with the kernel recomputed on the fly (no N x N
// derivative is stored):
//   far panel pairs: analytically. With e_p = P_{p+1} - P_p and Maue's form,
//     N^{pq}_ab = sum_{al,be} w_al w_be g(R) [s_a s_b - k^2 (e_p.e_q) psi_a(xi_al) psi_b(xi_be)],
//     so only g(|x_al - y_be|) and e_p.e_q depend on the nodes; dg/dx = -c (x - y),
//     c = (ik/4) H1(kR)/R.
//   self and adjacent pairs: fourth-order central differences of the same
//     singular quadrature (steps 1e-3 and 2e-3 of the shorter panel), which is
//     analytic in the nodes.
// The S and N bands |i - j| <= 2 are symmetrised in the assembly, so M enters
// there as (M_ij + M_ji)/2. Amplitudes: J is quadratic in A_r, F j_r = A_r a_r,
//     dJ/dRe A_r + i dJ/dIm A_r = 2 sum_l e_lr conj(a_lr).
#include <cmath>

#include "fds_internal.h"
#include "hankel.h"
#include "linalg.h"
#include "lowrank.h"
#include "near.h"
#include "pipeline.h"

namespace fds {

static const double2 kOne = {1.0, 0.0};
static const double2 kZero = {0.0, 0.0};
constexpr double kSqrtHalfA = 0.70710678118654752440;

struct Rule8A {
    double xi[8];
    double w[8];
};

// far-pair rules of the assembly (orders 8, 4, 3): xi and w
struct FarRules {
    double x8[8], w8[8], x4[4], w4[4], x3[3], w3[3];
};
static_assert(sizeof(FarRules) == 30 * sizeof(double), "FarRules is copied as 30 doubles");

__device__ __forceinline__ double2 c_inf(double k) {
    const double s = 1.0 / sqrt(8.0 * kPi * k);
    return make_double2(kSqrtHalfA * s, kSqrtHalfA * s);
}

__device__ __forceinline__ double2 cexpi(double ph) {
    double s, c;
    sincos(ph, &s, &c);
    return make_double2(c, s);
}

// ------------------------------------------------------------------ far-field matrix
// F[l + i nang] = c_inf (i k) sum_{p in {i-1, i}} (th_l . (h n)_p) sum_al w psi e^{-i k th_l . x_al},
// (h n)_p = (e_y, -e_x) for the edge e = P_{p+1} - P_p.
__global__ __launch_bounds__(256) void farfield_matrix_kernel(const double* __restrict__ nodes, int n, const double* __restrict__ thetas,
                                       int nang, double k, Rule8A r, double2* __restrict__ F) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * nang) return;
    const int l = (int)(t % nang);
    const int i = (int)(t / nang);
    double ts, tc;
    sincos(thetas[l], &ts, &tc);
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int p = side == 0 ? i : (i == 0 ? n - 1 : i - 1);
        const int p1 = p + 1 == n ? 0 : p + 1;
        const double x0 = nodes[2 * p], y0 = nodes[2 * p + 1];
        const double ex = nodes[2 * p1] - x0, ey = nodes[2 * p1 + 1] - y0;
        const double tn = tc * ey - ts * ex;
        double2 s = make_double2(0.0, 0.0);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const double psi = side == 0 ? 1.0 - r.xi[a] : r.xi[a];
            const double2 E = cexpi(-k * (tc * (x0 + r.xi[a] * ex) + ts * (y0 + r.xi[a] * ey)));
            s = fma_cr(r.w[a] * psi, E, s);
        }
        acc = fma_cr(tn, s, acc);
    }
    // c_inf * (i k) * acc
    const double2 ci = c_inf(k);
    F[t] = cmul(cmul(ci, make_double2(0.0, k)), acc);
}

// ------------------------------------------------------------------ small reductions
// out[0] = sum |E|^2 over n values (one workgroup)
__global__ void sumsq_kernel(const double2* __restrict__ E, int64_t n, double* __restrict__ out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < n; t += blockDim.x) s += E[t].x * E[t].x + E[t].y * E[t].y;
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// gA[r] = 2 / conj(A_r) sum_l E_lr conj(FJ_lr)
__global__ void amp_grad_kernel(const double2* __restrict__ E, const double2* __restrict__ FJ, int nang,
                                const double2* __restrict__ amps, double2* __restrict__ gA) {
    __shared__ double sx[256], sy[256];
    const int r = blockIdx.x;
    double ax = 0.0, ay = 0.0;
    for (int l = threadIdx.x; l < nang; l += blockDim.x) {
        const double2 v = cmul(E[(int64_t)r * nang + l], cconj(FJ[(int64_t)r * nang + l]));
        ax += v.x;
        ay += v.y;
    }
    sx[threadIdx.x] = ax;
    sy[threadIdx.x] = ay;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sx[threadIdx.x] += sx[threadIdx.x + st];
            sy[threadIdx.x] += sy[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double2 a = cconj(amps[r]);
        const double den = a.x * a.x + a.y * a.y;
        const double2 inv = make_double2(a.x / den, -a.y / den);
        gA[r] = cscale(cmul(inv, make_double2(sx[0], sy[0])), 2.0);
    }
}

// ------------------------------------------------------------------ per-panel terms
// Far-field term +2 Re sum_l sum_i Q_li dF_li/dx and right-hand-side term
// -2 Re sum_r sum_i mu_ri df_ri/dx, each a sum over panels p of a function of
// (P_p, P_{p+1}). gp[p] = {d/dP_p (x, y), d/dP_{p+1} (x, y)}.
__global__ __launch_bounds__(64) void panel_grad_kernel(const double* __restrict__ nodes, int n, double k, Rule8A r,
                                  const double* __restrict__ thetas, int nang,
                                  const double2* __restrict__ Qp,   // E J^H: Q_li = conj(Qp[l + i nang])
                                  const double* __restrict__ angles, const double2* __restrict__ amps, int nrhs,
                                  const double2* __restrict__ mu, double* __restrict__ gp) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int p1 = p + 1 == n ? 0 : p + 1;
    const double x0 = nodes[2 * p], y0 = nodes[2 * p + 1];
    const double ex = nodes[2 * p1] - x0, ey = nodes[2 * p1 + 1] - y0;
    // complex gradient accumulators: d/dP_p (x, y), d/dP_{p+1} (x, y)
    double2 g0x = make_double2(0.0, 0.0), g0y = g0x, g1x = g0x, g1y = g0x;
    double2 h0x = g0x, h0y = g0x, h1x = g0x, h1y = g0x;   // right-hand-side term
    const double2 ci = cmul(c_inf(k), make_double2(0.0, k));
    for (int l = 0; l < nang; ++l) {
        double ts, tc;
        sincos(thetas[l], &ts, &tc);
        const double2 qa = cconj(Qp[(int64_t)p * nang + l]), qb = cconj(Qp[(int64_t)p1 * nang + l]);
        const double tpx = -ts, tpy = tc;                 // theta_perp
        const double et = ex * tpx + ey * tpy;            // e . theta_perp = theta . (h n)
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const double xi = r.xi[a];
            const double2 X = cexpi(-k * (tc * (x0 + xi * ex) + ts * (y0 + xi * ey)));
            const double2 cl = cmul(ci, cscale(cadd(cscale(qa, 1.0 - xi), cscale(qb, xi)), r.w[a]));
            const double2 cX = cmul(cl, X);
            // d/dx_al of X = -i k th X
            const double2 ikX = make_double2(k * cX.y, -k * cX.x);   // -i k cX
            g0x = cadd(g0x, cadd(cscale(cX, -tpx), cscale(ikX, et * (1.0 - xi) * tc)));
            g0y = cadd(g0y, cadd(cscale(cX, -tpy), cscale(ikX, et * (1.0 - xi) * ts)));
            g1x = cadd(g1x, cadd(cscale(cX, tpx), cscale(ikX, et * xi * tc)));
            g1y = cadd(g1y, cadd(cscale(cX, tpy), cscale(ikX, et * xi * ts)));
        }
    }
    for (int rr = 0; rr < nrhs; ++rr) {
        double ds, dc;
        sincos(angles[rr], &ds, &dc);
        const double2 ma = mu[(int64_t)rr * n + p], mb = mu[(int64_t)rr * n + p1];
        const double2 ikA = cmul(make_double2(0.0, k), amps[rr]);
        const double dpx = -ds, dpy = dc;                 // d_perp
        const double ed = ex * dpx + ey * dpy;            // e . d_perp = (h n) . d
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const double xi = r.xi[a];
            const double2 E = cexpi(k * (dc * (x0 + xi * ex) + ds * (y0 + xi * ey)));
            const double2 cr = cmul(ikA, cscale(cadd(cscale(ma, 1.0 - xi), cscale(mb, xi)), r.w[a]));
            const double2 cE = cmul(cr, E);
            const double2 ikE = make_double2(-k * cE.y, k * cE.x);   // i k cE
            h0x = cadd(h0x, cadd(cscale(cE, -dpx), cscale(ikE, ed * (1.0 - xi) * dc)));
            h0y = cadd(h0y, cadd(cscale(cE, -dpy), cscale(ikE, ed * (1.0 - xi) * ds)));
            h1x = cadd(h1x, cadd(cscale(cE, dpx), cscale(ikE, ed * xi * dc)));
            h1y = cadd(h1y, cadd(cscale(cE, dpy), cscale(ikE, ed * xi * ds)));
        }
    }
    double* o = gp + 4 * (int64_t)p;
    o[0] = 2.0 * (g0x.x - h0x.x);
    o[1] = 2.0 * (g0y.x - h0y.x);
    o[2] = 2.0 * (g1x.x - h1x.x);
    o[3] = 2.0 * (g1y.x - h1y.x);
}

// grad[i] += gp[i] (node p part) + gp[i - 1] (node p+1 part)
__global__ void panel_combine_kernel(const double* __restrict__ gp, int n, double* __restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int im = i == 0 ? n - 1 : i - 1;
    grad[2 * i] += gp[4 * (int64_t)i] + gp[4 * (int64_t)im + 2];
    grad[2 * i + 1] += gp[4 * (int64_t)i + 1] + gp[4 * (int64_t)im + 3];
}

// ------------------------------------------------------------------ operator term
__device__ __forceinline__ int cyc_dist(int i, int j, int n) {
    int d = i - j;
    d = d < 0 ? -d : d;
    return d < n - d ? d : n - d;
}

// M entry as seen by the assembled N: symmetrised on the band |i - j| <= 2
__device__ __forceinline__ double2 m_eff(const double2* __restrict__ M, int n, int i, int j) {
    const double2 a = M[i + (int64_t)j * n];
    if (cyc_dist(i, j, n) > 2) return a;
    return cscale(cadd(a, M[j + (int64_t)i * n]), 0.5);
}

__device__ __forceinline__ double wsum(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int PG_BS = 256;   // column panels per workgroup
constexpr int PG_RB = 32;    // row panels per workgroup

// -2 Re sum over far ordered panel pairs (p, q) of d/dx [sum_ab M_eff(p+a, q+b) N^{pq}_ab].
__global__ __launch_bounds__(PG_BS) void pair_grad_far_kernel(const double* __restrict__ nodes,
                                                              const double* __restrict__ h, int n, double k,
                                                              const double* __restrict__ tab, FarRules fr,
                                                              const double2* __restrict__ M,
                                                              double* __restrict__ grad) {
    __shared__ double red[4][PG_BS / 64];
    __shared__ FarRules rs;
    const int tid = threadIdx.x;
    if (tid < 30) reinterpret_cast<double*>(&rs)[tid] = reinterpret_cast<const double*>(&fr)[tid];
    __syncthreads();
    const int q = blockIdx.x * PG_BS + tid;
    const bool qv = q < n;
    const int qq = qv ? q : 0;
    const int q1 = qq + 1 == n ? 0 : qq + 1;
    const double qx0 = nodes[2 * qq], qy0 = nodes[2 * qq + 1];
    const double eqx = nodes[2 * q1] - qx0, eqy = nodes[2 * q1 + 1] - qy0;
    const double hq = h[qq];
    double gq[4] = {0.0, 0.0, 0.0, 0.0};   // d/dP_q (x, y), d/dP_{q+1} (x, y)
    const int pbeg = blockIdx.y * PG_RB, pend = min(n, pbeg + PG_RB);
    for (int p = pbeg; p < pend; ++p) {
        double gpl[4] = {0.0, 0.0, 0.0, 0.0};
        const int p1 = p + 1 == n ? 0 : p + 1;
        if (qv && cyc_dist(p, qq, n) >= 2) {
            const double px0 = nodes[2 * p], py0 = nodes[2 * p + 1];
            const double epx = nodes[2 * p1] - px0, epy = nodes[2 * p1 + 1] - py0;
            const double hp = h[p];
            // same rule choice as the assembly's far kernel
            const double hm = fmax(hp, hq);
            const double dist =
                hypot(px0 + 0.5 * epx - qx0 - 0.5 * eqx, py0 + 0.5 * epy - qy0 - 0.5 * eqy) - 0.5 * (hp + hq);
            int no = 8;
            if (k * hm <= 0.1 && dist >= 96.0 * hm) no = 4;
            if (k * hm <= 0.016 && dist >= 512.0 * hm) no = 3;
            const double* xs = no == 8 ? rs.x8 : (no == 4 ? rs.x4 : rs.x3);
            const double* ws = no == 8 ? rs.w8 : (no == 4 ? rs.w4 : rs.w3);
            const double2 M00 = m_eff(M, n, p, qq), M01 = m_eff(M, n, p, q1);
            const double2 M10 = m_eff(M, n, p1, qq), M11 = m_eff(M, n, p1, q1);
            const double2 AM = cadd(csub(M00, M01), csub(M11, M10));
            const double Epq = epx * eqx + epy * eqy;
            const double k2 = k * k;
            double2 dxs[2] = {make_double2(0, 0), make_double2(0, 0)};   // sum (1-xi) dPhi/dx_al (x comp)
            double2 dys[2] = {make_double2(0, 0), make_double2(0, 0)};
            double2 qxs[2] = {make_double2(0, 0), make_double2(0, 0)};
            double2 qys[2] = {make_double2(0, 0), make_double2(0, 0)};
            double2 dE = make_double2(0.0, 0.0);
            for (int al = 0; al < no; ++al) {
                const double xa = xs[al];
                const double X = px0 + xa * epx, Y = py0 + xa * epy;
                // B row: psi_0(xa) M0b + psi_1(xa) M1b
                const double2 Br0 = cadd(cscale(M00, 1.0 - xa), cscale(M10, xa));
                const double2 Br1 = cadd(cscale(M01, 1.0 - xa), cscale(M11, xa));
                double2 fx = make_double2(0, 0), fy = make_double2(0, 0);
                for (int be = 0; be < no; ++be) {
                    const double xb = xs[be];
                    const double dx = X - (qx0 + xb * eqx), dy = Y - (qy0 + xb * eqy);
                    const double R = sqrt(fma(dx, dx, dy * dy));
                    const Bessel01 bs = hk_eval_hot(k * R, tab);
                    const double2 g = make_double2(-0.25 * bs.y0, 0.25 * bs.j0);
                    const double kr = 0.25 * k / R;
                    const double2 c = make_double2(-kr * bs.y1, kr * bs.j1);
                    const double2 B = cadd(cscale(Br0, 1.0 - xb), cscale(Br1, xb));
                    const double ww = ws[al] * ws[be];
                    const double2 coef = cscale(csub(AM, cscale(B, k2 * Epq)), ww);
                    const double2 cc = cmul(coef, c);
                    // dPhi/dx_al += -cc d ; dPhi/dy_be += +cc d
                    fx = fma_cr(-dx, cc, fx);
                    fy = fma_cr(-dy, cc, fy);
                    qxs[0] = fma_cr(dx * (1.0 - xb), cc, qxs[0]);
                    qys[0] = fma_cr(dy * (1.0 - xb), cc, qys[0]);
                    qxs[1] = fma_cr(dx * xb, cc, qxs[1]);
                    qys[1] = fma_cr(dy * xb, cc, qys[1]);
                    dE = fma_cr(ww, cmul(g, B), dE);
                }
                dxs[0] = fma_cr(1.0 - xa, fx, dxs[0]);
                dys[0] = fma_cr(1.0 - xa, fy, dys[0]);
                dxs[1] = fma_cr(xa, fx, dxs[1]);
                dys[1] = fma_cr(xa, fy, dys[1]);
            }
            const double2 dPhidE = cscale(dE, -k2);
            // -2 Re of the node derivatives
            gpl[0] = -2.0 * (dxs[0].x - eqx * dPhidE.x);
            gpl[1] = -2.0 * (dys[0].x - eqy * dPhidE.x);
            gpl[2] = -2.0 * (dxs[1].x + eqx * dPhidE.x);
            gpl[3] = -2.0 * (dys[1].x + eqy * dPhidE.x);
            gq[0] += -2.0 * (qxs[0].x - epx * dPhidE.x);
            gq[1] += -2.0 * (qys[0].x - epy * dPhidE.x);
            gq[2] += -2.0 * (qxs[1].x + epx * dPhidE.x);
            gq[3] += -2.0 * (qys[1].x + epy * dPhidE.x);
        }
        // reduce the row-panel part over the workgroup
#pragma unroll
        for (int t = 0; t < 4; ++t) gpl[t] = wsum(gpl[t]);
        if ((tid & 63) == 0) {
#pragma unroll
            for (int t = 0; t < 4; ++t) red[t][tid >> 6] = gpl[t];
        }
        __syncthreads();
        if (tid < 4) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < PG_BS / 64; ++w) s += red[tid][w];
            const int node = tid < 2 ? p : p1;
            atomicAdd(grad + 2 * node + (tid & 1), s);
        }
        __syncthreads();
    }
    if (qv) {
        atomicAdd(grad + 2 * qq, gq[0]);
        atomicAdd(grad + 2 * qq + 1, gq[1]);
        atomicAdd(grad + 2 * q1, gq[2]);
        atomicAdd(grad + 2 * q1 + 1, gq[3]);
    }
}

// N block of a self / adjacent pair from the node coordinates (Maue form from S).
__device__ void near_n_block(const double (&P)[4][2], int s, double k, const double* __restrict__ tab,
                             const double* __restrict__ gl32, const Rule8A& r, const W8& wt, double2 (&Nb)[2][2]) {
    // P[0], P[1]: panel p; P[2], P[3]: panel q
    double px[8], py[8], qx[8], qy[8];
    const double epx = P[1][0] - P[0][0], epy = P[1][1] - P[0][1];
    const double eqx = P[3][0] - P[2][0], eqy = P[3][1] - P[2][1];
    const double hp = hypot(epx, epy), hq = hypot(eqx, eqy);
    const double tpx = epx / hp, tpy = epy / hp, tqx = eqx / hq, tqy = eqy / hq;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        px[a] = P[0][0] + r.xi[a] * (hp * tpx);
        py[a] = P[0][1] + r.xi[a] * (hp * tpy);
        qx[a] = P[2][0] + r.xi[a] * (hq * tqx);
        qy[a] = P[2][1] + r.xi[a] * (hq * tqy);
    }
    double2 So[2][2], Do[2][2];
    near_pair_blocks<false>(px, py, qx, qy, hp, hq, tpy, -tpx, tqy, -tqx, s, k, tab, gl32, wt, So, Do);
    const double2 I0 = cadd(cadd(So[0][0], So[0][1]), cadd(So[1][0], So[1][1]));
    const double2 I0h = cscale(I0, 1.0 / (hp * hq));
    const double kk = -k * k * (tpy * tqy + tpx * tqx);
    Nb[0][0] = cadd(I0h, cscale(So[0][0], kk));
    Nb[0][1] = csub(cscale(So[0][1], kk), I0h);
    Nb[1][0] = csub(cscale(So[1][0], kk), I0h);
    Nb[1][1] = cadd(I0h, cscale(So[1][1], kk));
}

// -2 Re d/dx [sum_ab M_eff(p+a, q+b) N^{pq}_ab] for the ordered near pairs
// (q = p - 1, p, p + 1), by central differences in each node coordinate.
__global__ __launch_bounds__(64) void pair_grad_near_kernel(const double* __restrict__ nodes, int n, double k,
                                      const double* __restrict__ tab, const double* __restrict__ gl32, Rule8A r,
                                      W8 wt, const double2* __restrict__ M, double* __restrict__ grad) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * n) return;
    const int p = t / 3, s = t - 3 * (t / 3);
    const int q = s == 0 ? (p == 0 ? n - 1 : p - 1) : (s == 1 ? p : (p + 1 == n ? 0 : p + 1));
    const int p1 = p + 1 == n ? 0 : p + 1, q1 = q + 1 == n ? 0 : q + 1;
    const int nid[4] = {p, p1, q, q1};
    double P[4][2];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        P[v][0] = nodes[2 * nid[v]];
        P[v][1] = nodes[2 * nid[v] + 1];
    }
    const double2 Mw[2][2] = {{m_eff(M, n, p, q), m_eff(M, n, p, q1)}, {m_eff(M, n, p1, q), m_eff(M, n, p1, q1)}};
    const double hmin = fmin(hypot(P[1][0] - P[0][0], P[1][1] - P[0][1]), hypot(P[3][0] - P[2][0], P[3][1] - P[2][1]));
    // Fourth-order central difference, f' = (8 (f(d) - f(-d)) - (f(2d) - f(-2d))) / (12 d),
    // with d = 1e-3 of the shorter panel: the blocks are analytic in the node
    // coordinates on the scale of the panel length h, so the truncation error is
    // ~(d/h)^4 / 30 ~ 3e-14 and the rounding error ~1.5 u / (d/h) ~ 2e-13 of the
    // block scale (a second-order difference at this accuracy would need d ~ 1e-6 h,
    // where rounding alone reaches 1e-10).
    const double del = 1e-3 * hmin;
    const double offs[4] = {del, -del, 2.0 * del, -2.0 * del};
    // distinct nodes of the pair: perturbing one moves every slot that holds it
    for (int v = 0; v < 4; ++v) {
        bool dup = false;
        for (int u = 0; u < v; ++u) dup = dup || nid[u] == nid[v];
        if (dup) continue;
        for (int ax = 0; ax < 2; ++ax) {
            double ph[4];
            for (int sg = 0; sg < 4; ++sg) {
                double Q[4][2];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    Q[u][0] = P[u][0];
                    Q[u][1] = P[u][1];
                    if (nid[u] == nid[v]) Q[u][ax] += offs[sg];
                }
                double2 Nb[2][2];
                near_n_block(Q, s, k, tab, gl32, r, wt, Nb);
                double2 phi = make_double2(0.0, 0.0);
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) phi = cadd(phi, cmul(Mw[a][b], Nb[a][b]));
                ph[sg] = phi.x;
            }
            const double d1 = (8.0 * (ph[0] - ph[1]) - (ph[2] - ph[3])) / (12.0 * del);
            atomicAdd(grad + 2 * nid[v] + ax, -2.0 * d1);
        }
    }
}

__global__ void zero_kernel(double* __restrict__ x, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] = 0.0;
}

static inline unsigned nb(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

static Rule8A rule8(const Op& op) {
    Rule8A r;
    for (int a = 0; a < 8; ++a) {
        r.xi[a] = op.rule.xi[a];
        r.w[a] = op.rule.w[a];
    }
    return r;
}

void launch_farfield_matrix(Op& op, const double* thetas, int nang, double2* F) {
    Ctx& c = *op.ctx;
    const int64_t tot = op.n * (int64_t)nang;
    {
        KScope _ks(c, "farfield");
        hipLaunchKernelGGL(farfield_matrix_kernel, dim3(nb(tot, 256)), dim3(256), 0, c.stream, op.nodes, (int)op.n,
                           thetas, nang, op.k, rule8(op), F);
    }
    FDS_HIP_TRY(hipGetLastError());
}

void run_farfield(Op& op, const double2* J, int64_t nrhs, const double* thetas, int nang, double2* out) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    double2* F = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * nang));
    launch_farfield_matrix(op, thetas, nang, F);
    zgemm(c, OP_N, OP_N, nang, (int)nrhs, n, kOne, F, nang, J, n, kZero, out, nang);
    c.dfree(F);
}

void run_farfield_grad(Op& op, const double* angles, const double2* amps, int64_t nrhs, const double* thetas,
                       int nang, const double2* T, int max_iters, double tol, double* Jout, double* grad,
                       double2* gamp, double2* ff_out, fds_solve_stats* stats) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    const size_t blk = sizeof(double2) * (size_t)n * nrhs;
    const size_t fblk = sizeof(double2) * (size_t)nang * nrhs;
    // forward: N j = -f, refined against the unfiltered operator
    double2* f = static_cast<double2*>(c.dmalloc(blk));
    launch_rhs_planewave(op, angles, amps, nrhs, f, nullptr);
    double2* J = static_cast<double2*>(c.dmalloc(blk));
    fds_solve_stats st{};
    run_solve(op, f, nullptr, nrhs, J, nullptr, max_iters, tol, stats ? stats : &st, true);
    // far fields, residual, objective, amplitude gradient
    double2* F = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * nang));
    launch_farfield_matrix(op, thetas, nang, F);
    double2* FJ = static_cast<double2*>(c.dmalloc(fblk));
    zgemm(c, OP_N, OP_N, nang, (int)nrhs, n, kOne, F, nang, J, n, kZero, FJ, nang);
    if (ff_out) FDS_HIP_TRY(hipMemcpyAsync(ff_out, FJ, fblk, hipMemcpyDeviceToDevice, c.stream));
    double2* E = static_cast<double2*>(c.dmalloc(fblk));
    FDS_HIP_TRY(hipMemcpyAsync(E, FJ, fblk, hipMemcpyDeviceToDevice, c.stream));
    axpby(c, make_double2(-1.0, 0.0), T, kOne, E, (int64_t)nang * nrhs);
    double* dj = static_cast<double*>(c.dmalloc(sizeof(double)));
    {
        KScope _ks(c, "objective");
        hipLaunchKernelGGL(sumsq_kernel, dim3(1), dim3(256), 0, c.stream, E, (int64_t)nang * nrhs, dj);
        hipLaunchKernelGGL(amp_grad_kernel, dim3((unsigned)nrhs), dim3(256), 0, c.stream, E, FJ, nang, amps, gamp);
    }
    FDS_HIP_TRY(hipGetLastError());
    // adjoint: N mu = conj(F^H e), solved as the EFIE with f = -conj(F^H e)
    double2* b = static_cast<double2*>(c.dmalloc(blk));
    zgemm(c, OP_C, OP_N, n, (int)nrhs, nang, kOne, F, nang, E, nang, kZero, b, n);
    conj_copy(c, b, f, (int64_t)n * nrhs);
    axpby(c, kZero, f, make_double2(-1.0, 0.0), f, (int64_t)n * nrhs);
    double2* mu = b;
    fds_solve_stats st2{};
    run_solve(op, f, nullptr, nrhs, mu, nullptr, max_iters, tol, &st2, true);
    // gradient in the node coordinates
    {
        KScope _ks(c, "adjoint_grad");
        hipLaunchKernelGGL(zero_kernel, dim3(nb(2 * (int64_t)n, 256)), dim3(256), 0, c.stream, grad, 2 * (int64_t)n);
    }
    FDS_HIP_TRY(hipGetLastError());
    double2* M = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * n));
    zgemm(c, OP_N, OP_T, n, n, (int)nrhs, kOne, mu, n, J, n, kZero, M, n);
    double2* Qp = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)nang * n));
    zgemm(c, OP_N, OP_C, nang, n, (int)nrhs, kOne, E, nang, J, n, kZero, Qp, nang);
    FarRules fr;
    gauss_legendre_01(8, fr.x8, fr.w8);
    gauss_legendre_01(4, fr.x4, fr.w4);
    gauss_legendre_01(3, fr.x3, fr.w3);
    W8 wt;
    for (int a = 0; a < 8; ++a) {
        wt.wp0[a] = op.rule.w[a] * (1.0 - op.rule.xi[a]);
        wt.wp1[a] = op.rule.w[a] * op.rule.xi[a];
    }
    double* gp = static_cast<double*>(c.dmalloc(sizeof(double) * 4 * (size_t)n));
    {
        KScope _ks(c, "adjoint_grad");
        hipLaunchKernelGGL(pair_grad_far_kernel, dim3(nb(n, PG_BS), nb(n, PG_RB)), dim3(PG_BS), 0, c.stream,
                           op.nodes, op.h, n, op.k, c.hk_tab, fr, M, grad);
        hipLaunchKernelGGL(pair_grad_near_kernel, dim3(nb(3 * (int64_t)n, 64)), dim3(64), 0, c.stream, op.nodes, n,
                           op.k, c.hk_tab, c.gl32, rule8(op), wt, M, grad);
        hipLaunchKernelGGL(panel_grad_kernel, dim3(nb(n, 64)), dim3(64), 0, c.stream, op.nodes, n, op.k, rule8(op),
                           thetas, nang, Qp, angles, amps, (int)nrhs, mu, gp);
        hipLaunchKernelGGL(panel_combine_kernel, dim3(nb(n, 256)), dim3(256), 0, c.stream, gp, n, grad);
    }
    FDS_HIP_TRY(hipGetLastError());
    FDS_HIP_TRY(hipMemcpyAsync(Jout, dj, sizeof(double), hipMemcpyDeviceToHost, c.stream));
    FDS_HIP_TRY(hipStreamSynchronize(c.stream));
    for (void* ptr : {(void*)f, (void*)J, (void*)F, (void*)FJ, (void*)E, (void*)dj, (void*)b, (void*)M, (void*)Qp,
                      (void*)gp})
        c.dfree(ptr);
}

}  // namespace fds
