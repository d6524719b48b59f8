// Adaptive cross approximation of the filtered compact part (paper, Inversion of
// the structured matrices: the skeleton C = U V^T comes from a skeleton-detecting
// algorithm; Bebendorf's ACA with partial pivoting is one of the two it cites).
//
// The matrix is A_y = V_n B_y (N x N, y coordinates), never formed: V_n (n_eff
// orthonormal real vectors) and B_y = G^{-1/2} Bt (n_eff rows of length N) give
//   row i:    A_y[i, j] = sum_m V_n[m][i] B_y[m][j]   (one thread per j)
//   column j: A_y[i, j] = sum_m V_n[m][i] B_y[m][j]   (one thread per i)
// and each step subtracts the crosses found so far in the same pass. Step k:
// residual row i_k, its largest entry outside the used columns (pivot p at j_k),
// b_k = row / p, a_k = residual column j_k, the Frobenius-norm estimate of the
// sum S_k from the inner products with the earlier crosses, stop once
// ||a_k|| ||b_k|| <= tol ||S_k||_F or k = rank_cap, next row = the largest entry of
// a_k outside the used rows. The pivot search and the divisions stay on the
// device; the host reads one small record per step to decide on stopping.
#include <cmath>
#include <vector>

#include "fds_internal.h"
#include "linalg.h"
#include "pipeline.h"

namespace fds {

namespace {

constexpr int ACA_BS = 256;

struct Pivot {          // result of a masked arg-max
    int idx;
    int pad;
    double mag;
    double2 val;
};

struct StepRec {        // what the host reads after each step
    Pivot col;          // pivot of the residual row (column j_k, entry p)
    Pivot row;          // largest entry of a_k outside the used rows (next row)
    double na2, nb2;    // ||a_k||^2, ||b_k||^2
};

// residual row i of A_y - sum_{l<k} a_l b_l^T, or residual column j (COL)
template <bool COL>
__global__ void aca_line_kernel(int n, int ne, int k, int fixed_host, const Pivot* __restrict__ fixed_dev,
                                const double* __restrict__ Vn, const double2* __restrict__ By,
                                const double2* __restrict__ AK, const double2* __restrict__ BK,
                                double2* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int f = fixed_dev ? fixed_dev->idx : fixed_host;   // the fixed row (COL = false) or column
    const int i = COL ? t : f, j = COL ? f : t;
    double2 acc = make_double2(0.0, 0.0);
    for (int m = 0; m < ne; ++m) {
        const double v = Vn[(int64_t)m * n + i];
        const double2 b = By[(int64_t)m * n + j];
        acc.x = fma(v, b.x, acc.x);
        acc.y = fma(v, b.y, acc.y);
    }
    for (int l = 0; l < k; ++l) {
        const double2 a = AK[(int64_t)l * n + i], b = BK[(int64_t)l * n + j];
        acc.x -= a.x * b.x - a.y * b.y;
        acc.y -= a.x * b.y + a.y * b.x;
    }
    out[t] = acc;
}

// masked arg-max of |x| (mask[i] != 0 excluded), lowest index among equal magnitudes;
// one block of ACA_BS threads
__global__ void aca_argmax_kernel(int n, const double2* __restrict__ x, const unsigned char* __restrict__ mask,
                                  Pivot* __restrict__ out) {
    __shared__ double sm[ACA_BS];
    __shared__ int si[ACA_BS];
    double best = -1.0;
    int bi = n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        if (mask[i]) continue;
        const double m = hypot(x[i].x, x[i].y);
        if (m > best) {
            best = m;
            bi = i;
        }
    }
    sm[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const double o = sm[threadIdx.x + s];
            const int oi = si[threadIdx.x + s];
            if (o > sm[threadIdx.x] || (o == sm[threadIdx.x] && oi < si[threadIdx.x])) {
                sm[threadIdx.x] = o;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        Pivot p;
        p.idx = si[0] < n ? si[0] : 0;
        p.pad = 0;
        p.mag = si[0] < n ? sm[0] : 0.0;
        p.val = si[0] < n ? x[si[0]] : make_double2(0.0, 0.0);
        *out = p;
    }
}

// b_k = row / p (p = the pivot found in the row); marks the pivot column used.
// A vanishing pivot leaves b_k zero and the column free (the host skips the step).
__global__ void aca_scale_kernel(int n, const double2* __restrict__ row, const Pivot* __restrict__ pv,
                                 double2* __restrict__ bk, unsigned char* __restrict__ used_c) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const Pivot p = *pv;
    if (!(p.mag > 0.0)) {
        bk[j] = make_double2(0.0, 0.0);
        return;
    }
    const double d = p.val.x * p.val.x + p.val.y * p.val.y;
    const double2 r = row[j];
    // r / p = r conj(p) / |p|^2
    bk[j] = make_double2((r.x * p.val.x + r.y * p.val.y) / d, (r.y * p.val.x - r.x * p.val.y) / d);
    if (j == p.idx) used_c[j] = 1;
}

// dots[l] = (a_l^H a_k, b_l^H b_k) for l < k (one block each); block k: ||a_k||^2, ||b_k||^2
__global__ void aca_dots_kernel(int n, int k, const double2* __restrict__ AK, const double2* __restrict__ BK,
                                double2* __restrict__ dots, StepRec* __restrict__ rec) {
    __shared__ double red[4][ACA_BS];
    const int l = blockIdx.x;
    const double2* ak = AK + (int64_t)k * n;
    const double2* bk = BK + (int64_t)k * n;
    const double2* al = AK + (int64_t)l * n;
    const double2* bl = BK + (int64_t)l * n;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double2 x = al[i], y = ak[i], u = bl[i], v = bk[i];
        s0 += x.x * y.x + x.y * y.y;   // conj(x) y
        s1 += x.x * y.y - x.y * y.x;
        s2 += u.x * v.x + u.y * v.y;
        s3 += u.x * v.y - u.y * v.x;
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    red[2][threadIdx.x] = s2;
    red[3][threadIdx.x] = s3;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (l < k) {
            dots[2 * l] = make_double2(red[0][0], red[1][0]);
            dots[2 * l + 1] = make_double2(red[2][0], red[3][0]);
        } else {
            rec->na2 = red[0][0];
            rec->nb2 = red[2][0];
        }
    }
}

__global__ void aca_set_flag_kernel(unsigned char* __restrict__ f, int i) { f[i] = 1; }

}  // namespace

void run_compress_aca(Op& op, int rank_cap, double tol) {
    FDS_REQUIRE(rank_cap >= 1 && tol >= 0.0 && std::isfinite(tol), FDS_ERR_ARG, "bad compression options");
    Ctx& c = *op.ctx;
    if (op.owns_uw) {
        c.dfree(op.U);
        c.dfree(op.W);
    }
    op.U = op.W = nullptr;
    op.owns_uw = false;
    op.sv.clear();
    const int n = (int)op.n, ne = op.n_eff;
    FDS_REQUIRE(ne >= 1, FDS_ERR_STATE, "empty filter basis");
    const int cap = std::min(rank_cap, n);
    const double* Vn = filter_basis_view(op);
    // B_y = G^{-1/2} Bt (n_eff rows of length n)
    double2* By = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * ne));
    FDS_HIP_TRY(hipMemcpyAsync(By, op.Bt, sizeof(double2) * (size_t)n * ne, hipMemcpyDeviceToDevice, c.stream));
    apply_gram_power(op, -1, By, ne);
    double2* AK = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * cap));
    double2* BK = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * cap));
    double2* row = static_cast<double2*>(c.dmalloc(sizeof(double2) * n));
    double2* dots = static_cast<double2*>(c.dmalloc(sizeof(double2) * 2 * (size_t)cap));
    StepRec* drec = static_cast<StepRec*>(c.dmalloc(sizeof(StepRec)));
    unsigned char* used = static_cast<unsigned char*>(c.dmalloc(2 * (size_t)n));   // rows, then columns
    unsigned char* used_r = used;
    unsigned char* used_c = used + n;
    {
        // masks start clear (a fill kernel, not a memset)
        std::vector<unsigned char> z(2 * (size_t)n, 0);
        FDS_HIP_TRY(hipMemcpyAsync(used, z.data(), 2 * (size_t)n, hipMemcpyHostToDevice, c.stream));
        FDS_HIP_TRY(hipStreamSynchronize(c.stream));
    }
    std::vector<bool> hused(n, false);
    std::vector<double2> hdots(2 * (size_t)cap);
    const unsigned nb = (unsigned)((n + ACA_BS - 1) / ACA_BS);
    double s2 = 0.0;
    int k = 0, i = 0;
    {
        KScope _ks(c, "aca");
        while (k < cap) {
            hused[i] = true;
            hipLaunchKernelGGL(aca_set_flag_kernel, dim3(1), dim3(1), 0, c.stream, used_r, i);
            hipLaunchKernelGGL((aca_line_kernel<false>), dim3(nb), dim3(ACA_BS), 0, c.stream, n, ne, k, i,
                               (const Pivot*)nullptr, Vn, By, AK, BK, row);
            hipLaunchKernelGGL(aca_argmax_kernel, dim3(1), dim3(ACA_BS), 0, c.stream, n, row, used_c, &drec->col);
            double2* bk = BK + (int64_t)k * n;
            double2* ak = AK + (int64_t)k * n;
            hipLaunchKernelGGL(aca_scale_kernel, dim3(nb), dim3(ACA_BS), 0, c.stream, n, row, &drec->col, bk,
                               used_c);
            hipLaunchKernelGGL((aca_line_kernel<true>), dim3(nb), dim3(ACA_BS), 0, c.stream, n, ne, k, 0,
                               &drec->col, Vn, By, AK, BK, ak);
            hipLaunchKernelGGL(aca_dots_kernel, dim3(k + 1), dim3(ACA_BS), 0, c.stream, n, k, AK, BK, dots, drec);
            hipLaunchKernelGGL(aca_argmax_kernel, dim3(1), dim3(ACA_BS), 0, c.stream, n, ak, used_r, &drec->row);
            FDS_HIP_TRY(hipGetLastError());
            StepRec rec;
            FDS_HIP_TRY(hipMemcpyAsync(&rec, drec, sizeof(StepRec), hipMemcpyDeviceToHost, c.stream));
            if (k > 0)
                FDS_HIP_TRY(hipMemcpyAsync(hdots.data(), dots, sizeof(double2) * 2 * (size_t)k,
                                           hipMemcpyDeviceToHost, c.stream));
            FDS_HIP_TRY(hipStreamSynchronize(c.stream));
            if (!(rec.col.mag > 0.0)) {
                // the residual row vanishes outside the used columns: next unused row
                int nx = -1;
                for (int q = 0; q < n; ++q)
                    if (!hused[q]) {
                        nx = q;
                        break;
                    }
                if (nx < 0) break;
                i = nx;
                continue;
            }
            double cross = 0.0;
            for (int l = 0; l < k; ++l) {
                const double2 x = hdots[2 * l], y = hdots[2 * l + 1];
                cross += 2.0 * (x.x * y.x - x.y * y.y);   // Re((a_l^H a_k)(b_l^H b_k))
            }
            const double nab = std::sqrt(rec.na2 * rec.nb2);
            s2 += cross + rec.na2 * rec.nb2;
            op.sv.push_back(nab);
            ++k;
            if (nab <= tol * std::sqrt(std::max(s2, 0.0))) break;
            if (!(rec.row.mag >= 0.0) || hused[rec.row.idx]) break;   // every row used
            i = rec.row.idx;
        }
    }
    const int r = k;
    if (r > 0) {
        // U_j = G^{-1/2} A_K, W_j^T = G^{1/2} B_K
        op.U = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * r));
        op.W = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * r));
        FDS_HIP_TRY(hipMemcpyAsync(op.U, AK, sizeof(double2) * (size_t)n * r, hipMemcpyDeviceToDevice, c.stream));
        FDS_HIP_TRY(hipMemcpyAsync(op.W, BK, sizeof(double2) * (size_t)n * r, hipMemcpyDeviceToDevice, c.stream));
        apply_gram_power(op, -1, op.U, r);
        apply_gram_power(op, 1, op.W, r);
        op.owns_uw = true;
    }
    c.dfree(By);
    c.dfree(AK);
    c.dfree(BK);
    c.dfree(row);
    c.dfree(dots);
    c.dfree(drec);
    c.dfree(used);
    op.rank = r;
    op.stage = Stage::Compressed;
}

}  // namespace fds
