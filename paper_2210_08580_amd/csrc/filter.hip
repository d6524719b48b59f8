// Laplacian filter basis (paper, Laplacian Filters, 2D case, eq. LapFilter,
// with the orthonormalised Laplacian G^{-1/2} L G^{-1/2} for non-uniform
// meshes): the n smallest eigenpairs of the periodic tridiagonal pencil
// L v = lambda G v (P1 stiffness and mass matrices). With V_g the
// G-orthonormal generalised eigenvectors, V_n = G^{1/2} V_g are the
// orthonormal eigenvectors of G^{-1/2} L G^{-1/2}.
//
// Eigenvalues: bisection on Sylvester inertia counts. The periodic
// tridiagonal L - sigma G is reordered as a block tridiagonal matrix of 2x2
// blocks by pairing node k with node n-1-k; the block LDL^T recurrence
// A_{k+1} = D_{k+1} - E_k A_k^{-1} E_k then gives the count of negative
// eigenvalues as the sum over blocks. One wavefront refines one eigenvalue,
// its 64 lanes evaluating 64 shifts per round (multisection).
// Eigenvectors: inverse iteration (L - lambda G) x_new = G x_old with a banded
// LU with partial pivoting of the same folded ordering (bandwidth 2), one
// thread per eigenvalue, G-Gram-Schmidt inside clusters of close eigenvalues,
// and a final CholeskyQR in the G inner product.
#include <algorithm>
#include <cmath>
#include <vector>

#include "fds_internal.h"
#include "linalg.h"

namespace fds {

struct Pencil {
    const double* __restrict__ ld;
    const double* __restrict__ lo;
    const double* __restrict__ gd;
    const double* __restrict__ go;
    int n;
};

__device__ __forceinline__ double pm(const Pencil& P, int i, double s) { return P.ld[i] - s * P.gd[i]; }
__device__ __forceinline__ double pf(const Pencil& P, int i, double s) { return P.lo[i] - s * P.go[i]; }

// number of eigenvalues of the pencil below s
__device__ int pencil_count(const Pencil& P, double s) {
    const int n = P.n;
    const int K = n / 2;                       // node pairs (k, n-1-k)
    const bool odd = (n & 1) != 0;
    const double tiny = 1e-290;
    double a = pm(P, 0, s), c = pm(P, n - 1, s), b = pf(P, n - 1, s);
    if (!odd && K == 1) b += pf(P, 0, s);
    int cnt = 0;
    for (int k = 0;; ++k) {
        double det = a * c - b * b;
        if (fabs(det) < tiny) det = det < 0.0 ? -tiny : tiny;
        cnt += det < 0.0 ? 1 : (a < 0.0 ? 2 : 0);
        if (k == K - 1) {
            if (odd) {
                const int sN = (n - 1) / 2;
                const double u1 = pf(P, sN - 1, s), u2 = pf(P, sN, s);
                const double val = pm(P, sN, s) - (u1 * u1 * c - 2.0 * u1 * u2 * b + u2 * u2 * a) / det;
                cnt += val < 0.0 ? 1 : 0;
            }
            break;
        }
        const double e1 = pf(P, k, s), e2 = pf(P, n - 2 - k, s);
        const double inv = 1.0 / det;
        const double an = pm(P, k + 1, s) - e1 * e1 * c * inv;
        const double cn = pm(P, n - 2 - k, s) - e2 * e2 * a * inv;
        double bn = e1 * e2 * b * inv;
        if (!odd && k + 1 == K - 1) bn += pf(P, K - 1, s);   // nodes n/2-1 and n/2 are adjacent
        a = an;
        b = bn;
        c = cn;
    }
    return cnt;
}

// one wavefront per eigenvalue index (first + i)
__global__ void bisect_kernel(Pencil P, double glo, double ghi, double rtol, double atol, int first, int nw,
                              double* __restrict__ lam) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (i >= nw) return;
    const int idx = first + i;
    double lo = glo, hi = ghi;
    for (int it = 0; it < 64; ++it) {
        const double w = hi - lo;
        if (w <= fmax(rtol * fmax(fabs(lo), fabs(hi)), atol)) break;
        const double s = lo + w * (double)(lane + 1) / 65.0;
        const int cnt = pencil_count(P, s);
        const unsigned long long mask = __ballot(cnt > idx);
        const int l = mask ? (__ffsll(mask) - 1) : 64;
        const double nlo = (l == 0) ? lo : lo + w * (double)l / 65.0;
        const double nhi = (l == 64) ? hi : lo + w * (double)(l + 1) / 65.0;
        if (!(nhi - nlo < w)) break;
        lo = nlo;
        hi = nhi;
    }
    if (lane == 0) lam[i] = 0.5 * (lo + hi);
}

// ---------------------------------------------------------------- folded ordering
__device__ __forceinline__ int node_of(int r, int n) {
    if ((n & 1) && r == n - 1) return (n - 1) / 2;
    return (r & 1) ? n - 1 - (r >> 1) : (r >> 1);
}

// entries M[node(r)][node(r + d)] for d = -2..2 (zero outside the matrix)
__device__ void band_row(const Pencil& P, int r, double s, double out[5]) {
    const int n = P.n;
    const int a = node_of(r, n);
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        const int cpos = r + t - 2;
        double v = 0.0;
        if (cpos >= 0 && cpos < n) {
            const int b = node_of(cpos, n);
            if (b == a) v = pm(P, a, s);
            else if (b == (a + 1 == n ? 0 : a + 1)) v = pf(P, a, s);
            else if (a == (b + 1 == n ? 0 : b + 1)) v = pf(P, b, s);
        }
        out[t] = v;
    }
}

// Banded LU with partial pivoting of the folded L - sigma_i G (thread per eigenvalue).
// fac layout: [(j*7 + t) * nw + i], t = 0..4: U row j at columns j..j+4, t = 5,6: multipliers.
__global__ void invit_factor_kernel(Pencil P, const double* __restrict__ sig, int nw, double pivmin,
                                    double* __restrict__ fac, unsigned char* __restrict__ pv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw) return;
    const int n = P.n;
    const double s = sig[i];
    double w0[5], w1[5], w2[5], tmp[5];
    band_row(P, 0, s, tmp);
    w0[0] = tmp[2]; w0[1] = tmp[3]; w0[2] = tmp[4]; w0[3] = 0.0; w0[4] = 0.0;
    band_row(P, 1, s, tmp);
    w1[0] = tmp[1]; w1[1] = tmp[2]; w1[2] = tmp[3]; w1[3] = tmp[4]; w1[4] = 0.0;
    band_row(P, 2, s, w2);
    for (int j = 0; j < n; ++j) {
        const bool v1 = j + 1 < n, v2 = j + 2 < n;
        int p = 0;
        double best = fabs(w0[0]);
        if (v1 && fabs(w1[0]) > best) { p = 1; best = fabs(w1[0]); }
        if (v2 && fabs(w2[0]) > best) { p = 2; }
        if (p == 1) {
#pragma unroll
            for (int t = 0; t < 5; ++t) { const double q = w0[t]; w0[t] = w1[t]; w1[t] = q; }
        } else if (p == 2) {
#pragma unroll
            for (int t = 0; t < 5; ++t) { const double q = w0[t]; w0[t] = w2[t]; w2[t] = q; }
        }
        if (fabs(w0[0]) < pivmin) w0[0] = w0[0] < 0.0 ? -pivmin : pivmin;
        const double inv = 1.0 / w0[0];
        const double l1 = v1 ? w1[0] * inv : 0.0, l2 = v2 ? w2[0] * inv : 0.0;
#pragma unroll
        for (int t = 1; t < 5; ++t) {
            w1[t] -= l1 * w0[t];
            w2[t] -= l2 * w0[t];
        }
#pragma unroll
        for (int t = 0; t < 5; ++t) fac[((int64_t)j * 7 + t) * nw + i] = w0[t];
        fac[((int64_t)j * 7 + 5) * nw + i] = l1;
        fac[((int64_t)j * 7 + 6) * nw + i] = l2;
        pv[(int64_t)j * nw + i] = (unsigned char)p;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            w0[t] = w1[t + 1];
            w1[t] = w2[t + 1];
        }
        w0[4] = 0.0;
        w1[4] = 0.0;
        if (j + 3 < n) band_row(P, j + 3, s, w2);
        else
#pragma unroll
            for (int t = 0; t < 5; ++t) w2[t] = 0.0;
    }
}

// One inverse-iteration step per eigenvalue: W = G X; X <- M^{-1} W; X /= ||X||_G.
// X, W: [nw][n] node-indexed vectors.
__global__ void invit_step_kernel(Pencil P, int nw, const double* __restrict__ fac,
                                  const unsigned char* __restrict__ pv, double* __restrict__ X,
                                  double* __restrict__ Wk) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw) return;
    const int n = P.n;
    double* x = X + (int64_t)i * n;
    double* w = Wk + (int64_t)i * n;
    for (int k = 0; k < n; ++k) {
        const int km = k == 0 ? n - 1 : k - 1, kp = k + 1 == n ? 0 : k + 1;
        w[k] = P.gd[k] * x[k] + P.go[km] * x[km] + P.go[k] * x[kp];
    }
    // forward elimination on the folded right-hand side; z_j stored at node_of(j)
    double y0 = w[node_of(0, n)], y1 = w[node_of(1, n)], y2 = w[node_of(2, n)];
    for (int j = 0; j < n; ++j) {
        const int p = pv[(int64_t)j * nw + i];
        if (p == 1) { const double q = y0; y0 = y1; y1 = q; }
        else if (p == 2) { const double q = y0; y0 = y2; y2 = q; }
        const double l1 = fac[((int64_t)j * 7 + 5) * nw + i], l2 = fac[((int64_t)j * 7 + 6) * nw + i];
        y1 -= l1 * y0;
        y2 -= l2 * y0;
        x[node_of(j, n)] = y0;
        y0 = y1;
        y1 = y2;
        y2 = (j + 3 < n) ? w[node_of(j + 3, n)] : 0.0;
    }
    double x1 = 0.0, x2 = 0.0, x3 = 0.0, x4 = 0.0;
    for (int j = n - 1; j >= 0; --j) {
        const int nd = node_of(j, n);
        const double* u = fac + (int64_t)j * 7 * nw + i;
        const double v = (x[nd] - u[nw] * x1 - u[2 * nw] * x2 - u[3 * nw] * x3 - u[4 * nw] * x4) / u[0];
        x[nd] = v;
        x4 = x3;
        x3 = x2;
        x2 = x1;
        x1 = v;
    }
    double nrm = 0.0;
    for (int k = 0; k < n; ++k) {
        const int km = k == 0 ? n - 1 : k - 1, kp = k + 1 == n ? 0 : k + 1;
        nrm += x[k] * (P.gd[k] * x[k] + P.go[km] * x[km] + P.go[k] * x[kp]);
    }
    const double sc = 1.0 / sqrt(nrm);
    for (int k = 0; k < n; ++k) x[k] *= sc;
}

__device__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// G-inner product Gram-Schmidt inside each cluster [cb[c], cb[c+1]) (workgroup per cluster).
__global__ void cluster_gs_kernel(Pencil P, const int* __restrict__ cb, double* __restrict__ X) {
    __shared__ double sh[256];
    const int n = P.n;
    const int c0 = cb[blockIdx.x], c1 = cb[blockIdx.x + 1];
    for (int j = c0; j < c1; ++j) {
        double* xj = X + (int64_t)j * n;
        for (int i = c0; i <= j; ++i) {
            const double* xi = X + (int64_t)i * n;
            double part = 0.0;
            for (int k = threadIdx.x; k < n; k += blockDim.x) {
                const int km = k == 0 ? n - 1 : k - 1, kp = k + 1 == n ? 0 : k + 1;
                part += xi[k] * (P.gd[k] * xj[k] + P.go[km] * xj[km] + P.go[k] * xj[kp]);
            }
            const double dot = block_sum(part, sh);
            if (i < j) {
                for (int k = threadIdx.x; k < n; k += blockDim.x) xj[k] -= dot * xi[k];
            } else {
                const double sc = 1.0 / sqrt(dot);
                for (int k = threadIdx.x; k < n; k += blockDim.x) xj[k] *= sc;
            }
            __syncthreads();
        }
    }
}

__global__ void init_vectors_kernel(double* __restrict__ X, int n, int nw) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * nw) return;
    uint64_t z = (uint64_t)t * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    X[t] = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

// ---------------------------------------------------------------- host driver
void compute_filter_basis(Op& op, int n_modes, bool keep_null, double cluster_rtol) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    // bounds of the pencil's spectrum: 0 <= lambda <= max_i 4/(h_{i-1} h_i) / lambda_min(G) (Gershgorin)
    std::vector<double> hd(4 * (size_t)n);
    FDS_HIP_TRY(hipMemcpyAsync(hd.data(), op.g_diag, sizeof(double) * n, hipMemcpyDeviceToHost, c.stream));
    FDS_HIP_TRY(hipMemcpyAsync(hd.data() + n, op.g_off, sizeof(double) * n, hipMemcpyDeviceToHost, c.stream));
    FDS_HIP_TRY(hipMemcpyAsync(hd.data() + 2 * n, op.l_diag, sizeof(double) * n, hipMemcpyDeviceToHost, c.stream));
    FDS_HIP_TRY(hipMemcpyAsync(hd.data() + 3 * n, op.l_off, sizeof(double) * n, hipMemcpyDeviceToHost, c.stream));
    FDS_HIP_TRY(hipStreamSynchronize(c.stream));
    double gmin = 1e300, gmax = 0.0, lmax = 0.0;
    for (int i = 0; i < n; ++i) {
        const int im = i == 0 ? n - 1 : i - 1;
        const double gd = hd[i], go1 = std::fabs(hd[n + im]), go2 = std::fabs(hd[n + i]);
        gmin = std::min(gmin, gd - go1 - go2);
        gmax = std::max(gmax, gd + go1 + go2);
        lmax = std::max(lmax, std::fabs(hd[2 * n + i]) + std::fabs(hd[3 * n + im]) + std::fabs(hd[3 * n + i]));
    }
    op.cheb_lo = gmin;
    op.cheb_hi = gmax;
    const double lam_hi = 1.01 * lmax / gmin;
    const double mnorm = lmax + lam_hi * gmax;

    Pencil P{op.l_diag, op.l_off, op.g_diag, op.g_off, n};
    const int start = keep_null ? 0 : 1;
    int want = keep_null ? n_modes : n_modes - 1;
    FDS_REQUIRE(want >= 1 && start + want <= n, FDS_ERR_ARG, "n_modes out of range");
    // eigenvalues start .. start+nw-1 (a few beyond the cut for the cluster guard)
    std::vector<double> lam;
    int nw = 0;
    int extra = 8;
    for (;;) {
        nw = std::min(n - start, want + extra);
        double* dlam = static_cast<double*>(c.dmalloc(sizeof(double) * nw));
        const int wpb = 4;
        hipLaunchKernelGGL(bisect_kernel, dim3((nw + wpb - 1) / wpb), dim3(64 * wpb), 0, c.stream, P,
                           -1e-3 * lam_hi, lam_hi, 4e-15, 4e-16 * lam_hi, start, nw, dlam);
        FDS_HIP_TRY(hipGetLastError());
        lam.assign(nw, 0.0);
        FDS_HIP_TRY(hipMemcpyAsync(lam.data(), dlam, sizeof(double) * nw, hipMemcpyDeviceToHost, c.stream));
        FDS_HIP_TRY(hipStreamSynchronize(c.stream));
        c.dfree(dlam);
        int ne = want;
        while (ne < nw) {
            const double a = lam[ne - 1], b = lam[ne];
            if (b - a > cluster_rtol * std::max(std::fabs(a), std::fabs(b))) break;
            ++ne;
        }
        if (ne < nw || start + nw == n) {
            want = std::min(ne, nw);
            break;
        }
        extra *= 4;
    }
    const int ne = want;
    op.filt_lam = lam;
    lam.resize(ne);
    // clusters for the inverse iteration: relative gaps below 1e-5 of the scale
    const double scale = std::max(lam[ne - 1], 1e-300);
    std::vector<int> cb{0};
    for (int i = 1; i < ne; ++i)
        if (lam[i] - lam[i - 1] > 1e-5 * scale) cb.push_back(i);
    cb.push_back(ne);
    const int ncl = (int)cb.size() - 1;

    double* dsig = static_cast<double*>(c.dmalloc(sizeof(double) * ne));
    FDS_HIP_TRY(hipMemcpyAsync(dsig, lam.data(), sizeof(double) * ne, hipMemcpyHostToDevice, c.stream));
    int* dcb = static_cast<int*>(c.dmalloc(sizeof(int) * (ncl + 1)));
    FDS_HIP_TRY(hipMemcpyAsync(dcb, cb.data(), sizeof(int) * (ncl + 1), hipMemcpyHostToDevice, c.stream));
    double* fac = static_cast<double*>(c.dmalloc(sizeof(double) * 7 * (size_t)n * ne));
    unsigned char* pv = static_cast<unsigned char*>(c.dmalloc((size_t)n * ne));
    double* X = static_cast<double*>(c.dmalloc(sizeof(double) * (size_t)n * ne));
    double* Wk = static_cast<double*>(c.dmalloc(sizeof(double) * (size_t)n * ne));
    hipLaunchKernelGGL(init_vectors_kernel, dim3((unsigned)(((int64_t)n * ne + 255) / 256)), dim3(256), 0,
                       c.stream, X, n, ne);
    FDS_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(invit_factor_kernel, dim3((ne + 63) / 64), dim3(64), 0, c.stream, P, dsig, ne,
                       1e-15 * mnorm, fac, pv);
    FDS_HIP_TRY(hipGetLastError());
    for (int it = 0; it < 3; ++it) {
        hipLaunchKernelGGL(invit_step_kernel, dim3((ne + 63) / 64), dim3(64), 0, c.stream, P, ne, fac, pv, X,
                           Wk);
        FDS_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(cluster_gs_kernel, dim3(ncl), dim3(256), 0, c.stream, P, dcb, X);
        FDS_HIP_TRY(hipGetLastError());
    }
    // CholeskyQR (twice) in the G inner product: V <- V R^{-1}, R^T R = V^T G V
    double* M = static_cast<double*>(c.dmalloc(sizeof(double) * (size_t)ne * ne));
    int* info = static_cast<int*>(c.dmalloc(sizeof(int)));
    for (int pass = 0; pass < 2; ++pass) {
        gram_mul<double>(c, op.g_diag, op.g_off, n, X, ne, n, 1.0, 0.0, Wk, n);
        dgemm(c, OP_T, OP_N, ne, ne, n, 1.0, X, n, Wk, n, 0.0, M, ne);
        FDS_HIP_TRY(hipMemsetAsync(info, 0, sizeof(int), c.stream));
        chol_upper(c, M, ne, info);
        trsm_right_upper(c, M, ne, X, n);
    }
    int hinfo = 0;
    FDS_HIP_TRY(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    FDS_HIP_TRY(hipStreamSynchronize(c.stream));
    c.dfree(M);
    c.dfree(info);
    c.dfree(Wk);
    c.dfree(fac);
    c.dfree(pv);
    c.dfree(dsig);
    c.dfree(dcb);
    FDS_REQUIRE(hinfo == 0, FDS_ERR_SINGULAR, "filter basis lost G-orthogonality (Cholesky failed)");
    c.dfree(op.Vg);
    c.dfree(op.Vn);
    op.Vn = nullptr;
    op.Vg = X;
    op.n_eff = ne;
}

}  // namespace fds
