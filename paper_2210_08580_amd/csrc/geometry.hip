// Geometry, Gram / Laplacian, plane-wave right-hand sides and the special-
// function test kernels.
//
// Mesh (paper, Notation and Background): straight segments joining
// consecutive nodes of a closed curve; panel p runs from node p to node p+1
// (mod n) with length h_p, outward normal n_p = (tau_y, -tau_x) for
// counter-clockwise nodes, and 8 Gauss points x_p(xi_a) = node_p + xi_a h_p tau_p.
// P1 hat basis: on panel p, psi_0 = 1 - xi (node p), psi_1 = xi (node p+1).
#include <cmath>

#include "fds_internal.h"
#include "hankel.h"

namespace fds {

// ----------------------------------------------------------------- host Gauss rule
// Gauss-Legendre nodes/weights on [0,1] by Newton's method on P_n.
void gauss_legendre_01(int n, double* x, double* w) {
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= n; ++j) {
                const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            const double pn = (n == 0) ? 1.0 : p1;
            const double pnm1 = p0;
            dp = n * (z * pn - pnm1) / (z * z - 1.0);
            const double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        // recompute derivative at the converged node
        double p0 = 1.0, p1 = z;
        for (int j = 2; j <= n; ++j) {
            const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        // ascending order on [0,1]
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
}

// ----------------------------------------------------------------- kernels
struct Rule8Arg {
    double xi[8];
};

__global__ void geometry_kernel(const double* __restrict__ nodes, int n, Rule8Arg r,
                                double* __restrict__ h, double* __restrict__ nx,
                                double* __restrict__ ny, double* __restrict__ gx,
                                double* __restrict__ gy) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int q = (p + 1 == n) ? 0 : p + 1;
    const double x0 = nodes[2 * p], y0 = nodes[2 * p + 1];
    const double dx = nodes[2 * q] - x0, dy = nodes[2 * q + 1] - y0;
    const double len = hypot(dx, dy);
    const double tx = dx / len, ty = dy / len;
    h[p] = len;
    nx[p] = ty;
    ny[p] = -tx;
    const double ex = len * tx, ey = len * ty;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        gx[8 * p + a] = x0 + r.xi[a] * ex;
        gy[8 * p + a] = y0 + r.xi[a] * ey;
    }
}

__global__ void sparse_kernel(const double* __restrict__ h, int n, double* __restrict__ gd,
                              double* __restrict__ go, double* __restrict__ ld,
                              double* __restrict__ lo) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double hm = h[i == 0 ? n - 1 : i - 1], hi = h[i];
    gd[i] = (hm + hi) / 3.0;
    go[i] = hi / 6.0;
    ld[i] = 1.0 / hm + 1.0 / hi;
    lo[i] = -1.0 / hi;
}

// f_i = <phi_i, du/dn>, h_i = <phi_i, u>, u = A exp(i k d.x), du/dn = i k (n.d) u.
__global__ __launch_bounds__(256) void rhs_planewave_kernel(const double* __restrict__ gx, const double* __restrict__ gy,
                                     const double* __restrict__ h, const double* __restrict__ nx,
                                     const double* __restrict__ ny, int n, double k, Rule8Arg wr,
                                     Rule8Arg xr, const double* __restrict__ angles,
                                     const double2* __restrict__ amps, int64_t nrhs,
                                     double2* __restrict__ f, double2* __restrict__ hh) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * nrhs) return;
    const int i = (int)(t % n);
    const int64_t r = t / n;
    double s, c;
    sincos(angles[r], &s, &c);
    const double2 A = amps[r];
    double2 fs = make_double2(0.0, 0.0), hs = fs;
    // panel i carries psi_0 of node i; panel i-1 carries psi_1 of node i
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int p = side == 0 ? i : (i == 0 ? n - 1 : i - 1);
        double2 lf = make_double2(0.0, 0.0), lh = lf;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const double psi = side == 0 ? 1.0 - xr.xi[a] : xr.xi[a];
            const double ph = k * (gx[8 * p + a] * c + gy[8 * p + a] * s);
            double sp, cp;
            sincos(ph, &sp, &cp);
            const double2 u = cmul(A, make_double2(cp, sp));
            const double wp = wr.xi[a] * psi;
            lh.x += wp * u.x;
            lh.y += wp * u.y;
            lf.x += wp * u.x;
            lf.y += wp * u.y;
        }
        const double nd = nx[p] * c + ny[p] * s;
        // du/dn moment = i k (n.d) * (moment of u)
        const double2 dl = make_double2(-k * nd * lf.y, k * nd * lf.x);
        hs = cadd(hs, cscale(lh, h[p]));
        fs = cadd(fs, cscale(dl, h[p]));
    }
    if (f) f[r * n + i] = fs;
    if (hh) hh[r * n + i] = hs;
}

__global__ void hankel_eval_kernel(const double* __restrict__ x, int64_t n,
                                   const double* __restrict__ tab, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Bessel01 b = hf_eval(x[i], tab);
    out[4 * i + 0] = b.j0;
    out[4 * i + 1] = b.y0;
    out[4 * i + 2] = b.j1;
    out[4 * i + 3] = b.y1;
}

__global__ void hankel_eval_f32_kernel(const double* __restrict__ x, int64_t n, const float* __restrict__ tab,
                                       float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Bessel01f b = hf32_eval(x[i], tab);
    out[4 * i + 0] = b.j0;
    out[4 * i + 1] = b.y0;
    out[4 * i + 2] = b.j1;
    out[4 * i + 3] = b.y1;
}

__global__ void kernel_eval_kernel(double k, const double* __restrict__ Rs, int64_t n,
                                   const double* __restrict__ tab, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double R = Rs[i];
    double* o = out + 8 * i;
    if (R > 0.0) {
        const Bessel01 b = hk_eval(k * R, tab);
        o[0] = -0.25 * b.y0;
        o[1] = 0.25 * b.j0;
        o[4] = -0.25 * k * b.y1 / R;
        o[5] = 0.25 * k * b.j1 / R;
        const double2 rem = dlayer_rem(k, R, tab);
        o[6] = rem.x / R;
        o[7] = rem.y / R;
    } else {
        o[0] = o[1] = o[4] = o[5] = o[6] = o[7] = 0.0;
    }
    const double2 gr = green_reg(k, R, tab);
    o[2] = gr.x;
    o[3] = gr.y;
}

// Yukawa kernel values at distances R: out[i] = ((1/2pi) K0(kappa R) (R > 0, else 0),
// (1/2pi)(K0(kappa R) + log R), continuous at R = 0).
__global__ void yukawa_eval_kernel(double kappa, const double* __restrict__ Rs, int64_t n,
                                   const double* __restrict__ ytab, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double R = Rs[i];
    out[2 * i] = R > 0.0 ? kInv2Pi * yk_k0(kappa * R, ytab) : 0.0;
    out[2 * i + 1] = yukawa_reg(kappa, R, ytab);
}

// ----------------------------------------------------------------- launchers
static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_geometry(Op& op) {
    const int n = (int)op.n;
    Rule8Arg r;
    for (int a = 0; a < 8; ++a) r.xi[a] = op.rule.xi[a];
    {
        KScope _ks(*op.ctx, "geometry");
        hipLaunchKernelGGL(geometry_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, op.ctx->stream,
                       op.nodes, n, r, op.h, op.nx, op.ny, op.gx, op.gy);
    }
    FDS_HIP_TRY(hipGetLastError());
    {
        KScope _ks(*op.ctx, "geometry");
        hipLaunchKernelGGL(sparse_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, op.ctx->stream,
                       op.h, n, op.g_diag, op.g_off, op.l_diag, op.l_off);
    }
    FDS_HIP_TRY(hipGetLastError());
}

void launch_rhs_planewave(Op& op, const double* angles, const double2* amps, int64_t nrhs,
                          double2* f, double2* hh) {
    Rule8Arg wr, xr;
    for (int a = 0; a < 8; ++a) {
        wr.xi[a] = op.rule.w[a];
        xr.xi[a] = op.rule.xi[a];
    }
    const int64_t tot = op.n * nrhs;
    {
        KScope _ks(*op.ctx, "rhs_planewave");
        hipLaunchKernelGGL(rhs_planewave_kernel, dim3(blocks_for(tot, 256)), dim3(256), 0,
                       op.ctx->stream, op.gx, op.gy, op.h, op.nx, op.ny, (int)op.n, op.k, wr, xr,
                       angles, amps, nrhs, f, hh);
    }
    FDS_HIP_TRY(hipGetLastError());
}

void launch_hankel_eval(Ctx& c, const double* x, int64_t n, double* out) {
    {
        KScope _ks(c, "hankel_eval");
        hipLaunchKernelGGL(hankel_eval_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, c.stream, x, n,
                       c.hf_tab, out);
    }
    FDS_HIP_TRY(hipGetLastError());
}

void launch_hankel_eval_f32(Ctx& c, const double* x, int64_t n, float* out) {
    {
        KScope _ks(c, "hankel_eval");
        hipLaunchKernelGGL(hankel_eval_f32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, c.stream, x, n,
                           c.hf_tab32, out);
    }
    FDS_HIP_TRY(hipGetLastError());
}

void launch_yukawa_eval(Ctx& c, double kappa, const double* R, int64_t n, double* out) {
    {
        KScope _ks(c, "yukawa_eval");
        hipLaunchKernelGGL(yukawa_eval_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, c.stream, kappa, R, n,
                           c.yk_tab, out);
    }
    FDS_HIP_TRY(hipGetLastError());
}

void launch_kernel_eval(Ctx& c, double k, const double* R, int64_t n, double* out) {
    {
        KScope _ks(c, "kernel_eval");
        hipLaunchKernelGGL(kernel_eval_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, c.stream, k, R,
                       n, c.hk_tab, out);
    }
    FDS_HIP_TRY(hipGetLastError());
}

}  // namespace fds
