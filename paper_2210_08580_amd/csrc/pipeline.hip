// Orchestration of the filtered fast direct solve on the device.
//
// The paper's normalised unknown is y = G^{1/2} j and its filtered system is
// (beta I + P C) y = v with P = V_n V_n^T (paper, Filters Based Fast Direct
// Solver, 2D case). This library works in the current coefficients j instead:
// with V_g = G^{-1/2} V_n (G-orthonormal generalised Laplacian eigenvectors)
// the same system reads
//     (beta I + V_g Bt^T) j = w,   w = G^{-1/2} v,
// where, for the EFIE part, Bt = G^{1/2} (V_n^T C)^T = N^T G^{-1} S^T V_g - G V_g / 4,
// for the MFIE part Bt = -D^T V_g, and
//     EFIE  w = -G^{-1} S G^{-1} f,   MFIE  w = -G^{-1} h.
// Every product is a similarity transform of the paper's by G^{1/2}, so the
// solution is identical up to rounding, but no square root of G is needed on
// the solve path: only tridiagonal G^{-1} solves and G products. Residual
// norms are measured in the y metric, ||r_y||^2 = r_j^H G r_j.
// The skeleton U W of the filtered compact part is likewise stored as
// U_j = G^{-1/2} U_y, W_j = W_y G^{1/2}; the Woodbury core I + W U/beta is the
// same in both coordinates (paper, Inversion of the structured matrices).
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "fds_internal.h"
#include "linalg.h"
#include "lowrank.h"
#include "pipeline.h"

namespace fds {

static const double2 kOne = {1.0, 0.0};
static const double2 kZero = {0.0, 0.0};

void compute_filter_basis(Op& op, int n_modes, bool keep_null, double cluster_rtol);
void prefetch_filter_eigs(Op& op, int n_modes);

// Y = alpha op(M) X + beta Y for the column-major view M of a stored operator
// (which: 0 = S, 1 = N, 2 = D; the row-major n x n matrix read column-major is
// its transpose). X, Y: n x ncols complex128. Complex64 operators are widened on
// load and multiplied in FP64: N is hypersingular and the filtered products
// apply it to smooth vectors, where FP32 accumulation (or FP32 rounding of the
// vectors) would be amplified by ||N|| / |lambda_N(low modes)| ~ 1/h.
// The complex128 band of N (half-width w) replaces the zeros of the complex64
// matrix on load (N is symmetric, so op(N) = N for OP_N and OP_T).
// Formulation helpers: the EFIE part is present in EFIE, CFIE and the
// Yukawa-Calderon CFIE, the MFIE part in MFIE, CFIE and YCFIE; the single layer
// of the Calderon product is S (operator 0) or the Yukawa S_y (operator 3).
static inline bool has_efie(int f) { return f == FDS_EFIE || f == FDS_CFIE || f == FDS_YCFIE; }
static inline bool has_mfie(int f) { return f == FDS_MFIE || f == FDS_CFIE || f == FDS_YCFIE; }
static inline int s_op(int f) { return f == FDS_YCFIE ? 3 : 0; }

// Assembles the Yukawa single layer (kernel (1/2pi) K0(k R)) on first use.
void ensure_yukawa(Op& op) {
    if (op.Sy) return;
    Ctx& c = *op.ctx;
    op.Sy = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)op.n * op.n));
    launch_assemble_yukawa(op, op.k, op.Sy);
}

static void op_gemm(Op& op, int which, int opa, int64_t ncols, double2 alpha, const double2* X, double2 beta,
                    double2* Y) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    if (which == 3) {   // the symmetric Yukawa single layer, FP64 in every precision
        FDS_REQUIRE(op.Sy != nullptr, FDS_ERR_STATE, "Yukawa operator not assembled");
        GemmTag tag(c, "gemm_op_y");
        zgemm(c, OP_N, OP_N, n, (int)ncols, n, alpha, op.Sy, n, X, n, beta, Y, n);
        return;
    }
    // S and N are stored exactly symmetric (mirror writes of one value, symmetrised
    // near band), so their transposed products are the untransposed ones
    if (which != 2 && opa == OP_T) opa = OP_N;
    GemmTag tag(c, opa == OP_N ? "gemm_op" : "gemm_op_t");   // n x n operator products
    if (op.prec == FDS_FP32) {
        const float2* M = which == 0 ? op.S32 : (which == 1 ? op.N32 : op.D32);
        BandA band;
        if (which == 1) {
            FDS_REQUIRE(opa != OP_C, FDS_ERR_ARG, "conjugated product with N");
            band.nb = op.Nband;
            band.w = op.nbw;
            band.n = n;
        }
        zgemm_a32(c, opa, OP_N, n, (int)ncols, n, alpha, M, n, X, n, beta, Y, n, band);
        return;
    }
    const double2* M = which == 0 ? op.S : (which == 1 ? op.Nm : op.D);
    zgemm(c, opa, OP_N, n, (int)ncols, n, alpha, M, n, X, n, beta, Y, n);
}

// Y = alpha M V_g + beta Y for a stored operator M (column-major view, OP_N) and
// the real filter basis V_g (n x n_eff): the complex-by-real kernel (half the
// MFMAs of a complex product) when the shape allows it, else the complex copy.
static void op_gemm_vg(Op& op, int which, double2 alpha, double2 beta, double2* Y) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n, ne = op.n_eff;
    bool done;
    {
        GemmTag tag(c, "gemm_op_vg");
        if (which == 3) {
            FDS_REQUIRE(op.Sy != nullptr, FDS_ERR_STATE, "Yukawa operator not assembled");
            done = zgemm_real_b(c, n, ne, n, alpha, op.Sy, n, op.Vg, n, beta, Y, n);
        } else if (op.prec == FDS_FP32) {
            const float2* M = which == 0 ? op.S32 : (which == 1 ? op.N32 : op.D32);
            BandA band;
            if (which == 1) {
                band.nb = op.Nband;
                band.w = op.nbw;
                band.n = n;
            }
            done = zgemm_a32_real_b(c, n, ne, n, alpha, M, n, op.Vg, n, beta, Y, n, band);
        } else {
            const double2* M = which == 0 ? op.S : (which == 1 ? op.Nm : op.D);
            done = zgemm_real_b(c, n, ne, n, alpha, M, n, op.Vg, n, beta, Y, n);
        }
    }
    if (!done) op_gemm(op, which, OP_N, ne, alpha, op.Vgc, beta, Y);
}

// per-column sqrt(x^H G x)
__global__ void gnorm_kernel(const double* __restrict__ d, const double* __restrict__ e, int n,
                             const double2* __restrict__ X, int64_t ncols, double* __restrict__ out) {
    __shared__ double sh[256];
    const int64_t c = blockIdx.x;
    if (c >= ncols) return;
    const double2* x = X + c * n;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int im = i == 0 ? n - 1 : i - 1, ip = i + 1 == n ? 0 : i + 1;
        const double2 gx = make_double2(d[i] * x[i].x + e[im] * x[im].x + e[i] * x[ip].x,
                                        d[i] * x[i].y + e[im] * x[im].y + e[i] * x[ip].y);
        s += x[i].x * gx.x + x[i].y * gx.y;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sqrt(fmax(sh[0], 0.0));
}

static void gnorms(Op& op, const double2* X, int64_t ncols, double* out) {
    {
        KScope _ks(*op.ctx, "gnorm");
        hipLaunchKernelGGL(gnorm_kernel, dim3((unsigned)ncols), dim3(256), 0, op.ctx->stream, op.g_diag, op.g_off,
                       (int)op.n, X, ncols, out);
    }
    FDS_HIP_TRY(hipGetLastError());
}

// G^{-1}: banded inverse when every consecutive panel-length ratio is below 4.5
// (then the truncation error of the band is below 1e-18 relative, see
// gram_band_kernel), the exact cyclic Thomas algorithm otherwise.
void ensure_gram_factor(Op& op) {
    if (op.gfac || op.gband) return;
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    bool band = n > 4 * GW;
    if (band) {
        const std::vector<double>& h = op.h_host;
        for (int i = 0; i < n && band; ++i) {
            const double a = h[i == 0 ? n - 1 : i - 1], b = h[i];
            if (a > 4.5 * b || b > 4.5 * a) band = false;
        }
    }
    if (band) {
        op.gband = static_cast<double*>(c.dmalloc(sizeof(double) * (2 * GW + 1) * (size_t)n));
        gram_band_build(c, op.g_diag, op.g_off, n, op.gband);
    } else {
        op.gfac = static_cast<double*>(c.dmalloc(sizeof(double) * (3 * (size_t)n + 2)));
        gram_factor(c, op.g_diag, op.g_off, n, op.gfac);
    }
}

// Y = G^{-1} X for ncols vectors (Y may alias X)
void gram_inv(Op& op, const double2* X, int64_t ncols, double2* Y) {
    ensure_gram_factor(op);
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    const size_t bytes = sizeof(double2) * (size_t)n * ncols;
    if (op.gband) {
        if (X == Y) {
            double2* t = static_cast<double2*>(c.dmalloc(bytes));
            FDS_HIP_TRY(hipMemcpyAsync(t, X, bytes, hipMemcpyDeviceToDevice, c.stream));
            gram_band_apply<double2>(c, op.gband, n, t, ncols, Y);
            c.dfree(t);
        } else {
            gram_band_apply<double2>(c, op.gband, n, X, ncols, Y);
        }
        return;
    }
    if (X != Y) FDS_HIP_TRY(hipMemcpyAsync(Y, X, bytes, hipMemcpyDeviceToDevice, c.stream));
    gram_solve<double2>(c, op.g_off, op.gfac, n, Y, ncols, n);
}

// Gershgorin interval of G (P1 mass matrix: diagonal (h_{i-1} + h_i)/3, off-diagonal
// h_i/6) from the host panel lengths, widened by 1e-12 relative so that rounding
// differences between the host and the device lengths cannot put an eigenvalue outside.
void gram_gershgorin(const std::vector<double>& h, double& lo, double& hi) {
    const size_t n = h.size();
    lo = 1e300;
    hi = 0.0;
    for (size_t i = 0; i < n; ++i) {
        const double hm = h[i == 0 ? n - 1 : i - 1], hp = h[i];
        const double d = (hm + hp) / 3.0, r = hm / 6.0 + hp / 6.0;
        lo = std::min(lo, d - r);
        hi = std::max(hi, d + r);
    }
    lo *= 1.0 - 1e-12;
    hi *= 1.0 + 1e-12;
}

void ensure_cheb_bounds(Op& op) {
    if (op.cheb_hi > 0.0) return;
    gram_gershgorin(op.h_host, op.cheb_lo, op.cheb_hi);
}

// The band of G^{p/2} (p = +-1) on a homogeneous mesh large enough for the band
// (n > 4 GW, like the banded G^{-1}); null otherwise (Chebyshev series then).
static const double* gram_circ(Op& op, int p) {
    if (!op.homog || op.n <= 4 * GW) return nullptr;
    double*& b = op.gpow[p > 0 ? 1 : 0];
    if (!b) {
        b = static_cast<double*>(op.ctx->dmalloc(sizeof(double) * (2 * GW + 1) * (size_t)op.n));
        gram_circ_band(*op.ctx, op.h_mean, (int)op.n, p, b);
    }
    return b;
}

void apply_gram_power(Op& op, int p, double2* X, int64_t ncols) {
    if (p == -2) {
        gram_inv(op, X, ncols, X);
        return;
    }
    FDS_REQUIRE(p == 1 || p == -1, FDS_ERR_ARG, "p must be -2, -1 or 1");
    if (ncols <= 0) return;
    if (const double* band = gram_circ(op, p)) {
        Ctx& c = *op.ctx;
        const size_t bytes = sizeof(double2) * (size_t)op.n * ncols;
        double2* t = static_cast<double2*>(c.dmalloc(bytes));
        gram_band_apply<double2>(c, band, (int)op.n, X, ncols, t);
        FDS_HIP_TRY(hipMemcpyAsync(X, t, bytes, hipMemcpyDeviceToDevice, c.stream));
        c.dfree(t);
        return;
    }
    ensure_cheb_bounds(op);
    gram_pow_half<double2>(*op.ctx, op.g_diag, op.g_off, (int)op.n, op.cheb_lo, op.cheb_hi, p, X, ncols);
}

const double* filter_basis_view(Op& op) {
    if (!op.Vn) {
        Ctx& c = *op.ctx;
        const size_t bytes = sizeof(double) * (size_t)op.n * op.n_eff;
        op.Vn = static_cast<double*>(c.dmalloc(bytes));
        if (const double* band = gram_circ(op, 1)) {
            gram_band_apply<double>(c, band, (int)op.n, op.Vg, op.n_eff, op.Vn);
        } else {
            FDS_HIP_TRY(hipMemcpyAsync(op.Vn, op.Vg, bytes, hipMemcpyDeviceToDevice, c.stream));
            ensure_cheb_bounds(op);
            gram_pow_half<double>(c, op.g_diag, op.g_off, (int)op.n, op.cheb_lo, op.cheb_hi, 1, op.Vn,
                                  op.n_eff);
        }
    }
    return op.Vn;
}

// The first bisection of the Laplacian eigensolver (filtering point n_modes, null
// mode kept), enqueued on the side stream after the mesh event: it overlaps the
// dense assembly that the caller enqueues next on the main stream. The main
// stream is joined to it by the filter's own side-stream scope.
void prefetch_filter(Op& op, int n_modes) {
    if (op.homog) return;   // the DFT basis of a homogeneous mesh needs no eigensolver
    Ctx& c = *op.ctx;
    if (!op.ev_mesh) FDS_HIP_TRY(hipEventCreateWithFlags(&op.ev_mesh, hipEventDisableTiming));
    if (!op.ev_mesh_fresh) {
        FDS_HIP_TRY(hipEventRecord(op.ev_mesh, c.stream));
        op.ev_mesh_fresh = true;
    }
    SideStream side(c, op.ev_mesh, false);
    ensure_gram_factor(op);
    prefetch_filter_eigs(op, n_modes);
}

static void filter_prepare(Op& op, int form, double alpha, int n_modes, bool keep_null, double cluster_rtol) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    // The eigensolver and the Gram factor need only the mesh: right after the
    // assembly they run on the side stream beside the still-running dense
    // assembly kernels (their chains are latency-bound and leave most of the
    // chip idle); a later call orders them after all earlier work instead.
    if (!op.ev_mesh) FDS_HIP_TRY(hipEventCreateWithFlags(&op.ev_mesh, hipEventDisableTiming));
    if (!op.ev_mesh_fresh) FDS_HIP_TRY(hipEventRecord(op.ev_mesh, c.stream));
    op.ev_mesh_fresh = false;
    {
        SideStream side(c, op.ev_mesh);
        ensure_gram_factor(op);
        compute_filter_basis(op, n_modes, keep_null, cluster_rtol);
    }
    const int ne = op.n_eff;
    op.form = form;
    op.alpha = alpha;
    op.beta = form == FDS_EFIE ? 0.25 : (form == FDS_MFIE ? 0.5 : (1.0 + 2.0 * alpha) / 4.0);
    c.dfree(op.Vgc);
    c.dfree(op.Bt);
    op.Vgc = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * ne));
    op.Bt = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * ne));
    real_to_complex(c, op.Vg, op.Vgc, (int64_t)n * ne);
}

void run_filter(Op& op, int form, double alpha, int n_modes, bool keep_null, double cluster_rtol) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    if (form == FDS_YCFIE) ensure_yukawa(op);   // enqueued first: it runs beside the eigensolver
    filter_prepare(op, form, alpha, n_modes, keep_null, cluster_rtol);
    const int ne = op.n_eff;
    if (has_efie(form)) {
        // Bt = N^T G^{-1} S^T Vg - G Vg / 4  (S, N stored row-major: as column-major arrays they are S^T, N^T;
        // S_y in place of S for the Yukawa-Calderon CFIE)
        double2* X = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * ne));
        op_gemm_vg(op, s_op(form), kOne, kZero, X);
        gram_inv(op, X, ne, X);
        op_gemm(op, 1, OP_N, ne, kOne, X, kZero, op.Bt);
        gram_mul<double2>(c, op.g_diag, op.g_off, n, op.Vgc, ne, n, -0.25, 0.0, X, n);
        axpby(c, kOne, X, kOne, op.Bt, (int64_t)n * ne);
        c.dfree(X);
        if (form == FDS_CFIE || form == FDS_YCFIE)   // + alpha * (-D^T Vg)
            op_gemm_vg(op, 2, make_double2(-alpha, 0.0), kOne, op.Bt);
    } else {
        op_gemm_vg(op, 2, make_double2(-1.0, 0.0), kZero, op.Bt);
    }
    op.stage = Stage::Filtered;
    op.rank = 0;
}

// Several FP64 operators: per-operator eigensolver, then each dense product
// stage of all operators as one grouped GEMM launch.
void run_filter_batch(Op* const* ops, int count, int form, double alpha, const int* n_modes, bool keep_null,
                      double cluster_rtol) {
    if (count <= 0) return;
    Ctx& c = *ops[0]->ctx;
    for (int j = 0; j < count; ++j) {
        FDS_REQUIRE(ops[j]->prec == FDS_FP64, FDS_ERR_NOTIMPL, "batched filter is FP64 only");
        filter_prepare(*ops[j], form, alpha, n_modes[j], keep_null, cluster_rtol);
    }
    std::vector<double2*> X(count, nullptr);
    std::vector<GemmSpec> g;
    if (form == FDS_EFIE || form == FDS_CFIE) {
        for (int j = 0; j < count; ++j) {
            Op& op = *ops[j];
            const int n = (int)op.n, ne = op.n_eff;
            X[j] = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * ne));
            g.push_back({n, ne, n, kOne, kZero, op.S, n, op.Vgc, n, X[j], n});
        }
        zgemm_grouped_nn(c, g);
        g.clear();
        for (int j = 0; j < count; ++j) {
            Op& op = *ops[j];
            const int n = (int)op.n, ne = op.n_eff;
            gram_inv(op, X[j], ne, X[j]);
            g.push_back({n, ne, n, kOne, kZero, op.Nm, n, X[j], n, op.Bt, n});
        }
        zgemm_grouped_nn(c, g);
        g.clear();
        for (int j = 0; j < count; ++j) {
            Op& op = *ops[j];
            const int n = (int)op.n, ne = op.n_eff;
            gram_mul<double2>(c, op.g_diag, op.g_off, n, op.Vgc, ne, n, -0.25, 0.0, X[j], n);
            axpby(c, kOne, X[j], kOne, op.Bt, (int64_t)n * ne);
            c.dfree(X[j]);
        }
    }
    if (form == FDS_MFIE || form == FDS_CFIE) {
        const double a = form == FDS_MFIE ? -1.0 : -alpha;
        const double2 b = form == FDS_MFIE ? kZero : kOne;
        for (int j = 0; j < count; ++j) {
            Op& op = *ops[j];
            const int n = (int)op.n, ne = op.n_eff;
            g.push_back({n, ne, n, make_double2(a, 0.0), b, op.D, n, op.Vgc, n, op.Bt, n});
        }
        zgemm_grouped_nn(c, g);
    }
    for (int j = 0; j < count; ++j) {
        ops[j]->stage = Stage::Filtered;
        ops[j]->rank = 0;
    }
}

// Truncation of the projected block's singular values (descending):
// r = min(rank_cap, #{s_i > max(tol, 1e-13) s_0}), lowered while s_{r-1} < (1 + 1e-6) s_r
// so that a numerically repeated singular value is never split.
static int truncation_rank(const std::vector<double>& s, int rank_cap, double tol) {
    if (s.empty() || !(s[0] > 0.0)) return 0;
    const double thr = std::max(tol, 1e-13) * s[0];
    int cnt = 0;
    for (double v : s) cnt += v > thr ? 1 : 0;
    int r = std::min(rank_cap, cnt);
    while (r > 0 && r < (int)s.size() && s[r - 1] < (1.0 + 1e-6) * s[r]) --r;
    return r;
}

void run_compress(Op& op, int rank_cap, int oversample, int power_iters, double tol, uint64_t seed,
                  bool householder) {
    const int ne = op.n_eff;
    const int ell = rank_cap + oversample;
    FDS_REQUIRE(rank_cap >= 1 && oversample >= 0 && power_iters >= 0 && tol >= 0.0, FDS_ERR_ARG,
                "bad compression options");
    Ctx& c = *op.ctx;
    if (op.owns_uw) {
        c.dfree(op.U);
        c.dfree(op.W);
    }
    op.U = op.W = nullptr;
    op.owns_uw = false;
    op.sv.clear();
    if (tol == 0.0 && rank_cap >= ne && ell >= ne) {
        // The filtered compact part V_n B has rank <= n_eff and a sketch of width
        // l >= n_eff spans its whole range, so the randomised skeleton is exact:
        // U_j = V_g, W_j = Bt^T (rank n_eff), no sketch needs to be formed.
        op.U = op.Vgc;
        op.W = op.Bt;
        op.rank = ne;
        op.stage = Stage::Compressed;
        return;
    }
    FDS_REQUIRE(ne >= 1, FDS_ERR_STATE, "empty filter basis");
    const int n = (int)op.n;
    const bool sketched = ell < ne;     // else the range of the compact part is found exactly
    FDS_REQUIRE(!sketched || ell <= n, FDS_ERR_ARG, "rank_cap + oversample exceeds the system size");
    const int m = sketched ? ell : ne;  // width of the final projected block
    const size_t nm = (size_t)n * m;
    // B_y^H = G^{-1/2} conj(Bt)  (N x n_eff): A_y = V_n B_y is the filtered compact part
    double2* cBt = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * ne));
    conj_copy(c, op.Bt, cBt, (int64_t)n * ne);
    double2* Z = static_cast<double2*>(c.dmalloc(sizeof(double2) * nm));
    double2* tau = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)std::max(m, ne)));
    double2* Qz = nullptr;   // n_eff x ell orthonormal range coordinates (Q = V_n Qz)
    if (sketched) {
        // Randomised subspace iteration (Halko, Martinsson & Tropp 2011) in the
        // coordinates of V_n: A_y X = V_n (B_y X), A_y^H V_n Y = B_y^H Y, and
        // orth(V_n Y) = V_n orth(Y).
        double2* T = static_cast<double2*>(c.dmalloc(sizeof(double2) * nm));
        double2* X = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)ne * m));
        Qz = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)ne * m));
        double2* Qp = static_cast<double2*>(c.dmalloc(sizeof(double2) * nm));
        sketch(c, seed, n, m, T);
        for (int it = 0;; ++it) {
            // X = B_y T = Bt^T G^{-1/2} T ; Qz = orth(X)
            apply_gram_power(op, -1, T, m);
            {
                GemmTag tg(c, "gemm_sketch");
                // n_eff x l output, inner dimension N: few tiles, so the inner
                // dimension is split into chunks of about 256 (at most 64 parts)
                SplitHint sh(c, std::max(1, std::min(64, n / 256)));
                zgemm(c, OP_T, OP_N, ne, m, n, kOne, op.Bt, n, T, n, kZero, X, ne);
            }
            // the intermediate bases only carry the span forward; the last Q_z is the
            // orthonormal range basis of the projection
            qr_explicit(c, X, ne, m, tau, Qz, !householder, it < power_iters);
            if (it == power_iters) break;
            // Z = B_y^H Qz ; T = orth(Z)
            {
                GemmTag tg(c, "gemm_sketch");
                SplitHint sh(c, 2);   // 3 N/128 tiles: two K parts balance them over the chip
                zgemm(c, OP_N, OP_N, n, m, ne, kOne, cBt, n, Qz, ne, kZero, Z, n);
            }
            apply_gram_power(op, -1, Z, m);
            qr_explicit(c, Z, n, m, tau, Qp, !householder, true);
            std::swap(T, Qp);
        }
        // projected block B = Q^H A_y = Qz^H B_y, held as B^H = B_y^H Qz
        {
            GemmTag tg(c, "gemm_sketch");
            SplitHint sh(c, 2);
            zgemm(c, OP_N, OP_N, n, m, ne, kOne, cBt, n, Qz, ne, kZero, Z, n);
        }
        apply_gram_power(op, -1, Z, m);
        c.dfree(T);
        c.dfree(X);
        c.dfree(Qp);
    } else {
        FDS_HIP_TRY(hipMemcpyAsync(Z, cBt, sizeof(double2) * nm, hipMemcpyDeviceToDevice, c.stream));
        apply_gram_power(op, -1, Z, m);
    }
    c.dfree(cBt);
    // B^H = Q_P R (Householder), R^H = Uh diag(s) Vh^H (Jacobi):
    //     B = Uh diag(s) (Q_P Vh)^H
    double2* QP = static_cast<double2*>(c.dmalloc(sizeof(double2) * nm));
    qr_explicit(c, Z, n, m, tau, QP, !householder);
    double2* RH = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)m * m));
    r_adjoint(c, Z, n, m, RH);
    c.dfree(Z);
    c.dfree(tau);
    double2* Uh = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)m * m));
    double2* Vh = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)m * m));
    double* sg = static_cast<double*>(c.dmalloc(sizeof(double) * (size_t)m));
    jacobi_svd(c, RH, m, Uh, Vh, sg, 60);
    c.dfree(RH);
    op.sv.assign(m, 0.0);
    FDS_HIP_TRY(hipMemcpyAsync(op.sv.data(), sg, sizeof(double) * m, hipMemcpyDeviceToHost, c.stream));
    FDS_HIP_TRY(hipStreamSynchronize(c.stream));
    const int r = truncation_rank(op.sv, rank_cap, tol);
    if (r > 0) {
        // U_j = G^{-1/2} V_n Qz Uh_r diag(s_r) = V_g (Qz Uh_r) diag(s_r)
        double2* Ur = Uh;
        double2* T1 = nullptr;
        if (Qz) {
            T1 = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)ne * r));
            zgemm(c, OP_N, OP_N, ne, r, m, kOne, Qz, ne, Uh, m, kZero, T1, ne);
            Ur = T1;
        }
        scale_cols(c, Ur, ne, r, sg);
        op.U = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * r));
        if (!zgemm_real_a(c, n, r, ne, kOne, op.Vg, n, Ur, ne, kZero, op.U, n))
            zgemm(c, OP_N, OP_N, n, r, ne, kOne, op.Vgc, n, Ur, ne, kZero, op.U, n);
        if (T1) c.dfree(T1);
        // W_j^T = (W_y G^{1/2})^T = G^{1/2} conj(Q_P Vh_r)
        double2* T2 = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * r));
        zgemm(c, OP_N, OP_N, n, r, m, kOne, QP, n, Vh, m, kZero, T2, n);
        op.W = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * r));
        conj_copy(c, T2, op.W, (int64_t)n * r);
        c.dfree(T2);
        apply_gram_power(op, 1, op.W, r);
        op.owns_uw = true;
    }
    if (Qz) c.dfree(Qz);
    c.dfree(QP);
    c.dfree(Uh);
    c.dfree(Vh);
    c.dfree(sg);
    op.rank = r;
    op.stage = Stage::Compressed;
}

// X (n x m column-major, i.e. m vectors of length n) -> Y = X^T (m x n column-major)
__global__ void ctranspose_kernel(const double2* __restrict__ X, int n, int m, double2* __restrict__ Y) {
    __shared__ double2 t[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;   // bx over n, by over m
    for (int k = threadIdx.y; k < 32; k += blockDim.y) {
        const int i = bx + threadIdx.x, j = by + k;
        if (i < n && j < m) t[k][threadIdx.x] = X[(int64_t)j * n + i];
    }
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += blockDim.y) {
        const int j = by + threadIdx.x, i = bx + k;
        if (i < n && j < m) Y[(int64_t)i * m + j] = t[threadIdx.x][k];
    }
}

static double2* ctranspose(Ctx& c, const double2* X, int n, int m) {
    double2* Y = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * m));
    {
        KScope _ks(c, "transpose");
        hipLaunchKernelGGL(ctranspose_kernel, dim3((n + 31) / 32, (m + 31) / 32), dim3(32, 8), 0, c.stream, X, n, m,
                           Y);
    }
    FDS_HIP_TRY(hipGetLastError());
    return Y;
}

// The rows of Bt^T and of W as column-major matrices, so that the products with
// them in the factor and the solves run untransposed (Gauss's three products,
// row-contiguous loads).
static void make_rows(Op& op) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    if (op.Wr != op.Btr) c.dfree(op.Wr);
    c.dfree(op.Btr);
    op.Btr = ctranspose(c, op.Bt, n, op.n_eff);
    op.Wr = op.W == op.Bt ? op.Btr : (op.rank > 0 ? ctranspose(c, op.W, n, op.rank) : nullptr);
}

void run_factor(Op& op) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n, r = op.rank;
    c.dfree(op.K);
    c.dfree(op.Up);
    op.K = nullptr;
    op.Up = nullptr;
    make_rows(op);
    if (r == 0) {
        op.stage = Stage::Factored;
        return;
    }
    FDS_REQUIRE(r <= 2048, FDS_ERR_NOTIMPL, "skeleton rank above 2048");
    // K = I + beta^{-1} W_j U_j ; W_j as the r x n matrix Wr
    double2* K = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)r * r));
    // the exact skeleton has U = V_g (held as its complex copy): the real V_g then
    // serves as the real operand of both products with U
    const bool ureal = op.U == op.Vgc && op.Vg != nullptr;
    if (!(ureal && zgemm_real_b(c, r, r, n, make_double2(1.0 / op.beta, 0.0), op.Wr, r, op.Vg, n, kZero, K, r)))
        zgemm(c, OP_N, OP_N, r, r, n, make_double2(1.0 / op.beta, 0.0), op.Wr, r, op.U, n, kZero, K, r);
    add_diag(c, K, r, 1.0);
    op.K = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)r * r));
    double hs[2];
    gj_inverse(c, K, op.K, r, hs);
    c.dfree(K);
    FDS_REQUIRE(hs[0] >= 64.0 * 2.220446049250313e-16 * hs[1], FDS_ERR_SINGULAR,
                "Woodbury core is numerically singular");
    // fold the core into U: Up = U K^{-1}
    op.Up = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)n * r));
    if (!(ureal && zgemm_real_a(c, n, r, r, kOne, op.Vg, n, op.K, r, kZero, op.Up, n)))
        zgemm(c, OP_N, OP_N, n, r, r, kOne, op.U, n, op.K, r, kZero, op.Up, n);
    op.stage = Stage::Factored;
}

// b <- Woodbury solve of (beta I + U W) x = b, in place on b (n x nrhs); z: r x nrhs scratch
//      x = b/beta - (U K^{-1}) (W b) / beta^2
static void woodbury_apply(Op& op, double2* b, int64_t nrhs, double2* z) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n, r = op.rank;
    const double ib = 1.0 / op.beta;
    if (r > 0) {
        {
            // r x nrhs output with the long inner dimension n: 256-long chunks of it
            SplitHint sh(c, std::max(1, std::min(64, n / 256)));
            zgemm(c, OP_N, OP_N, r, (int)nrhs, n, kOne, op.Wr, r, b, n, kZero, z, r);
        }
        zgemm(c, OP_N, OP_N, n, (int)nrhs, r, make_double2(-ib * ib, 0.0), op.Up, n, z, r,
              make_double2(ib, 0.0), b, n);
    } else {
        axpby(c, kZero, b, make_double2(ib, 0.0), b, (int64_t)n * nrhs);
    }
}

// The adjoint system. With y = G^{1/2} u, the adjoint (beta I + P C)^H y = v of the
// paper's filtered system reads, in the coordinates u (the adjoint's current
// coefficients),
//     (beta I + G^{-1} conj(Bt) V_g^T G) u = w' = G^{-1/2} v,
// and its skeleton form beta I + G^{-1} W_j^H U_j^H G has the Woodbury inverse
//     b/beta - beta^{-2} G^{-1} W_j^H (K^{-1})^H U_j^H G b
// with the same core K = I + W_j U_j/beta, ((U_j K^{-1})^H = Up^H).
// b <- that inverse applied to b (n x nrhs); z: r x nrhs, t: n x nrhs scratch.
static void woodbury_apply_adj(Op& op, double2* b, int64_t nrhs, double2* z, double2* t) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n, r = op.rank;
    const double ib = 1.0 / op.beta;
    if (r > 0) {
        gram_mul<double2>(c, op.g_diag, op.g_off, n, b, nrhs, n, 1.0, 0.0, t, n);
        zgemm(c, OP_C, OP_N, r, (int)nrhs, n, kOne, op.Up, n, t, n, kZero, z, r);
        zgemm(c, OP_C, OP_N, n, (int)nrhs, r, kOne, op.Wr, r, z, r, kZero, t, n);
        gram_inv(op, t, nrhs, t);
        axpby(c, make_double2(-ib * ib, 0.0), t, make_double2(ib, 0.0), b, (int64_t)n * nrhs);
    } else {
        axpby(c, kZero, b, make_double2(ib, 0.0), b, (int64_t)n * nrhs);
    }
}

// res = w' - (beta I + G^{-1} conj(Bt) V_g^T G) u  (filtered adjoint; z: n_eff x nrhs, t: n x nrhs)
static void filtered_residual_adj(Op& op, const double2* w, const double2* u, int64_t nrhs, double2* res,
                                  double2* z, double2* t) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n, ne = op.n_eff;
    const int64_t tot = (int64_t)n * nrhs;
    gram_mul<double2>(c, op.g_diag, op.g_off, n, u, nrhs, n, 1.0, 0.0, t, n);
    zgemm(c, OP_T, OP_N, ne, (int)nrhs, n, kOne, op.Vgc, n, t, n, kZero, z, ne);
    zgemm(c, OP_C, OP_N, n, (int)nrhs, ne, kOne, op.Btr, ne, z, ne, kZero, t, n);
    gram_inv(op, t, nrhs, t);
    FDS_HIP_TRY(hipMemcpyAsync(res, w, sizeof(double2) * tot, hipMemcpyDeviceToDevice, c.stream));
    axpby(c, make_double2(-op.beta, 0.0), u, kOne, res, tot);
    axpby(c, make_double2(-1.0, 0.0), t, kOne, res, tot);
}

// res = w' - (beta I + C_u^H) u for the unfiltered operator in the adjoint coordinates:
// C_u^H u = G^{-1} N^H G^{-1} S^H u - u/4 (EFIE part), -G^{-1} D^H u (MFIE part).
// S, N are complex symmetric and G real, so with u~ = conj(u) the products are
// conj(G^{-1} N G^{-1} S u~) and conj(G^{-1} D^T u~): the stored operators are used
// untransposed (as for the forward residual), and complex64 ones through their
// FP64 band as well. t0, t1, t2: n x nrhs scratch.
static void unfiltered_residual_adj(Op& op, const double2* w, const double2* u, int64_t nrhs, double2* res,
                                    double2* t0, double2* t1, double2* t2) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    const int64_t tot = (int64_t)n * nrhs;
    conj_copy(c, u, t0, tot);                                            // u~
    bool any = false;
    if (has_efie(op.form)) {
        op_gemm(op, s_op(op.form), OP_T, nrhs, kOne, t0, kZero, t1);     // S u~ (S_y for YCFIE)
        gram_inv(op, t1, nrhs, t1);
        op_gemm(op, 1, OP_T, nrhs, kOne, t1, kZero, t2);                 // N G^-1 S u~
        gram_inv(op, t2, nrhs, t2);
        any = true;
    }
    if (has_mfie(op.form)) {
        const double a = op.form == FDS_MFIE ? 1.0 : op.alpha;
        op_gemm(op, 2, OP_N, nrhs, kOne, t0, kZero, t1);                 // D^T u~ (column-major view of D)
        gram_inv(op, t1, nrhs, t1);
        if (any) axpby(c, make_double2(-a, 0.0), t1, kOne, t2, tot);     // E - alpha M
        else axpby(c, make_double2(-a, 0.0), t1, kZero, t2, tot);        // -M
    }
    conj_copy(c, t2, t1, tot);
    FDS_HIP_TRY(hipMemcpyAsync(res, w, sizeof(double2) * tot, hipMemcpyDeviceToDevice, c.stream));
    const double bu = has_efie(op.form) ? op.beta - 0.25 : op.beta;
    axpby(c, make_double2(-bu, 0.0), u, kOne, res, tot);
    axpby(c, make_double2(-1.0, 0.0), t1, kOne, res, tot);
}

// r = w - (beta I + C_j) j with the unfiltered compact part in j coordinates,
// C_j = G^{-1} S G^{-1} N - I/4 (EFIE), -G^{-1} D (MFIE), EFIE + alpha MFIE (CFIE).
static void unfiltered_residual(Op& op, const double2* w, const double2* jv, int64_t nrhs, double2* res,
                                double2* t1, double2* t2) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    const int64_t tot = (int64_t)n * nrhs;
    const size_t blk = sizeof(double2) * (size_t)tot;
    FDS_HIP_TRY(hipMemcpyAsync(res, w, blk, hipMemcpyDeviceToDevice, c.stream));
    axpby(c, make_double2(-op.beta, 0.0), jv, kOne, res, tot);
    if (has_efie(op.form)) {
        op_gemm(op, 1, OP_T, nrhs, kOne, jv, kZero, t1);          // N j
        gram_inv(op, t1, nrhs, t1);
        op_gemm(op, s_op(op.form), OP_T, nrhs, kOne, t1, kZero, t2);   // S G^-1 N j (S_y for YCFIE)
        gram_inv(op, t2, nrhs, t2);
        axpby(c, make_double2(-1.0, 0.0), t2, kOne, res, tot);
        axpby(c, make_double2(0.25, 0.0), jv, kOne, res, tot);
    }
    if (has_mfie(op.form)) {
        const double a = op.form == FDS_MFIE ? 1.0 : op.alpha;
        op_gemm(op, 2, OP_T, nrhs, kOne, jv, kZero, t1);          // D j
        gram_inv(op, t1, nrhs, t1);
        axpby(c, make_double2(a, 0.0), t1, kOne, res, tot);
    }
}

// Right-hand side in j coordinates, w = G^{-1/2} v: -G^{-1} S G^{-1} f (EFIE),
// -G^{-1} h (MFIE), the EFIE one + alpha times the MFIE one (CFIE). Needs only the
// assembled operator.
// Split-K factor of the right-hand-side product S (G^{-1} f): about 4096 work items
// (128 x 64 output tiles times K parts), at most 8 parts.
static int rhs_split(int n, int64_t nrhs) {
    const int64_t tiles = ((int64_t)(n + 127) / 128) * ((nrhs + 63) / 64);
    return (int)std::max<int64_t>(1, std::min<int64_t>(8, 4096 / std::max<int64_t>(tiles, 1)));
}

void run_rhs_system(Op& op, int form, double alpha, const double2* f, const double2* h, int64_t nrhs,
                    double2* w) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    const size_t blk = sizeof(double2) * (size_t)n * nrhs;
    if (form == FDS_YCFIE) ensure_yukawa(op);
    double2* t = static_cast<double2*>(c.dmalloc(blk));
    if (has_efie(form)) {
        FDS_REQUIRE(f != nullptr, FDS_ERR_ARG, "f is required for the EFIE/CFIE");
        gram_inv(op, f, nrhs, t);
        // S = (S stored row-major)^T as a column-major array (S_y for YCFIE). Split K
        // (rhs_split): the output tiles of this product alone fill the chip with one
        // workgroup per compute unit, each holding a whole unit's registers, so
        // latency-bound kernels that run beside it (the filter's eigensolver on the side
        // stream) would wait for a whole tile; with more, shorter work items they keep a
        // few units and the product flows around them (at N = 8192 and 256 right-hand
        // sides 8 parts: 10.05-10.06 ms per step, against 10.08 with 16 parts, which
        // write twice the partial sums, and 10.09-10.11 with 4).
        SplitHint sh(c, rhs_split(n, nrhs));
        op_gemm(op, s_op(form), OP_T, nrhs, make_double2(-1.0, 0.0), t, kZero, w);
        gram_inv(op, w, nrhs, w);
    }
    if (has_mfie(form)) {
        FDS_REQUIRE(h != nullptr, FDS_ERR_ARG, "h is required for the MFIE/CFIE");
        gram_inv(op, h, nrhs, t);
        if (form == FDS_MFIE) axpby(c, make_double2(-1.0, 0.0), t, kZero, w, (int64_t)n * nrhs);
        else axpby(c, make_double2(-alpha, 0.0), t, kOne, w, (int64_t)n * nrhs);
    }
    c.dfree(t);
}

void run_solve(Op& op, const double2* f, const double2* h, int64_t nrhs, double2* j_out, double2* y_out,
               int max_iters, double tol, fds_solve_stats* stats, bool unfiltered) {
    Ctx& c = *op.ctx;
    double2* w = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)op.n * nrhs));
    try {
        run_rhs_system(op, op.form, op.alpha, f, h, nrhs, w);
        run_solve_system(op, w, nrhs, j_out, y_out, max_iters, tol, stats, unfiltered);
    } catch (...) {
        c.dfree(w);
        throw;
    }
    c.dfree(w);
}

// The Woodbury solve and refinement from w (j coordinates, the filter's form).
void run_solve_system(Op& op, const double2* w, int64_t nrhs, double2* j_out, double2* y_out, int max_iters,
                      double tol, fds_solve_stats* stats, bool unfiltered, bool adjoint) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n, ne = op.n_eff;
    const size_t blk = sizeof(double2) * (size_t)n * nrhs;
    double2* res = static_cast<double2*>(c.dmalloc(blk));
    double2* z = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)std::max(op.rank, ne) * nrhs));
    double2* ta = adjoint ? static_cast<double2*>(c.dmalloc(blk)) : nullptr;   // adjoint Woodbury scratch
    auto precond = [&](double2* b) {
        if (adjoint) woodbury_apply_adj(op, b, nrhs, z, ta);
        else woodbury_apply(op, b, nrhs, z);
    };
    // ---- Woodbury solve
    double2* jv = j_out;
    FDS_HIP_TRY(hipMemcpyAsync(jv, w, blk, hipMemcpyDeviceToDevice, c.stream));
    precond(jv);
    // ---- refinement against beta I + V_g Bt^T (the uncompressed filtered operator)
    double* nrm = static_cast<double*>(c.dmalloc(sizeof(double) * 2 * nrhs));
    std::vector<double> hn(2 * nrhs);
    int iters = 0;
    double rel = 0.0;
    bool conv = false;
    if (stats) {
        std::fill(stats->history, stats->history + 32, 0.0);
        gnorms(op, w, nrhs, nrm + nrhs);
    }
    double2* t1 = nullptr;
    double2* t2 = nullptr;
    double2* t0 = nullptr;
    if (unfiltered || adjoint) {
        t1 = static_cast<double2*>(c.dmalloc(blk));
        t2 = static_cast<double2*>(c.dmalloc(blk));
    }
    if (unfiltered && adjoint) t0 = static_cast<double2*>(c.dmalloc(blk));
    for (int it = 0;; ++it) {
        if (!stats && it >= max_iters) break;
        if (adjoint && unfiltered) {
            unfiltered_residual_adj(op, w, jv, nrhs, res, t0, t1, t2);
        } else if (adjoint) {
            filtered_residual_adj(op, w, jv, nrhs, res, z, t1);
        } else if (unfiltered) {
            unfiltered_residual(op, w, jv, nrhs, res, t1, t2);
        } else {
            // res = w - beta j - V_g (Bt^T j)
            FDS_HIP_TRY(hipMemcpyAsync(res, w, blk, hipMemcpyDeviceToDevice, c.stream));
            axpby(c, make_double2(-op.beta, 0.0), jv, kOne, res, (int64_t)n * nrhs);
            {
                SplitHint sh(c, std::max(1, std::min(64, n / 256)));
                zgemm(c, OP_N, OP_N, ne, (int)nrhs, n, kOne, op.Btr, ne, jv, n, kZero, z, ne);
            }
            if (!zgemm_real_a(c, n, (int)nrhs, ne, make_double2(-1.0, 0.0), op.Vg, n, z, ne, kOne, res, n))
                zgemm(c, OP_N, OP_N, n, (int)nrhs, ne, make_double2(-1.0, 0.0), op.Vgc, n, z, ne, kOne, res, n);
        }
        if (stats) {
            gnorms(op, res, nrhs, nrm);
            FDS_HIP_TRY(hipMemcpyAsync(hn.data(), nrm, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, c.stream));
            FDS_HIP_TRY(hipStreamSynchronize(c.stream));
            rel = 0.0;
            for (int64_t k = 0; k < nrhs; ++k) {
                const double den = hn[nrhs + k] > 0.0 ? hn[nrhs + k] : 1.0;
                rel = std::max(rel, hn[k] / den);
            }
            if (it < 32) stats->history[it] = rel;
            if (rel <= tol) {
                conv = true;
                break;
            }
        }
        if (it >= max_iters) break;
        precond(res);
        axpby(c, kOne, res, kOne, jv, (int64_t)n * nrhs);
        ++iters;
    }
    if (y_out) {
        FDS_HIP_TRY(hipMemcpyAsync(y_out, jv, blk, hipMemcpyDeviceToDevice, c.stream));
        apply_gram_power(op, 1, y_out, nrhs);
    }
    c.dfree(nrm);
    c.dfree(res);
    c.dfree(z);
    c.dfree(t0);
    c.dfree(t1);
    c.dfree(t2);
    c.dfree(ta);
    if (stats) {
        stats->iters = iters;
        stats->converged = conv ? 1 : 0;
        stats->relres = rel;
        FDS_REQUIRE(conv, FDS_ERR_NOCONV, "refinement did not reach the requested tolerance");
    }
}

// The adjoint solve (beta I + P C)^H y = v (or of the unfiltered operator) from v
// in the normalised coordinates: u = G^{-1/2} y is solved for with w' = G^{-1/2} v.
void run_solve_adjoint(Op& op, const double2* v, int64_t nrhs, double2* y_out, double2* u_out, int max_iters,
                       double tol, fds_solve_stats* stats, bool unfiltered) {
    Ctx& c = *op.ctx;
    const size_t blk = sizeof(double2) * (size_t)op.n * nrhs;
    double2* wv = static_cast<double2*>(c.dmalloc(blk));
    double2* u = u_out ? u_out : static_cast<double2*>(c.dmalloc(blk));
    try {
        FDS_HIP_TRY(hipMemcpyAsync(wv, v, blk, hipMemcpyDeviceToDevice, c.stream));
        apply_gram_power(op, -1, wv, nrhs);
        run_solve_system(op, wv, nrhs, u, y_out, max_iters, tol, stats, unfiltered, true);
    } catch (...) {
        c.dfree(wv);
        if (!u_out) c.dfree(u);
        throw;
    }
    c.dfree(wv);
    if (!u_out) c.dfree(u);
}

// ---------------------------------------------------------------- allocation-free solve
// Scratch of fds_solve_system_noalloc: a file-scope device array, one copy on
// each GPU, held until the process ends. Its host-side name is not a device
// address: each device's address is obtained once, at context creation with
// that device current, and kept in Ctx::scratch; kernels only ever receive
// that address.
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void init_noalloc_scratch(Ctx& c) {
    static std::mutex mu;
    static std::map<int, void*> addr;   // device -> address of its copy of `scratch`
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(c.device);
    if (it == addr.end()) {
        void* p = nullptr;
        FDS_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        it = addr.emplace(c.device, p).first;
    }
    c.scratch = it->second;
}

// fds_solve_system with stats == NULL, y_out == NULL, the filtered refinement and
// max_iters = sweeps, without device allocations: the right-hand sides are taken
// in column blocks whose residual (n x cb) and small products (r x cb) fit three
// quarters of the scratch array; the rest holds the split-K partial sums.
void run_solve_system_noalloc(Op& op, const double2* w, int64_t nrhs, double2* j_out, int sweeps) {
    Ctx& c = *op.ctx;
    FDS_REQUIRE(c.scratch != nullptr, FDS_ERR_STATE, "scratch array not initialised");
    run_solve_system_ws(op, w, nrhs, j_out, sweeps, c.scratch, kScratchBytes);
}

// The same solve on a caller-given workspace: up to 3/4 of it holds the residual
// and the small products of a block of right-hand sides, the rest the GEMMs'
// split-K partial sums. Every device allocation in between raises an error.
void run_solve_system_ws(Op& op, const double2* w, int64_t nrhs, double2* j_out, int sweeps, void* ws,
                         size_t ws_bytes) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n, ne = op.n_eff;
    const int zr = std::max(op.rank, sweeps > 0 ? ne : 0);
    const size_t col = sizeof(double2) * ((size_t)n + (size_t)std::max(zr, 1));
    const int64_t cb = std::min<int64_t>(nrhs, (int64_t)((ws_bytes / 4 * 3) / col));
    FDS_REQUIRE(cb >= 1, FDS_ERR_ARG,
                "system too large for the allocation-free solve: 16 (n + max(rank, n_eff)) bytes per right-hand "
                "side must fit 3/4 of the workspace");
    double2* res = static_cast<double2*>(ws);
    double2* z = res + (size_t)n * cb;
    const size_t used = (sizeof(double2) * ((size_t)n + std::max(zr, 1)) * cb + 255) / 256 * 256;
    NoAlloc na(c, static_cast<unsigned char*>(ws) + used, ws_bytes - used);
    for (int64_t c0 = 0; c0 < nrhs; c0 += cb) {
        const int64_t nb = std::min(cb, nrhs - c0);
        const int64_t tot = (int64_t)n * nb;
        const double2* wv = w + (size_t)c0 * n;
        double2* jv = j_out + (size_t)c0 * n;
        FDS_HIP_TRY(hipMemcpyAsync(jv, wv, sizeof(double2) * tot, hipMemcpyDeviceToDevice, c.stream));
        woodbury_apply(op, jv, nb, z);
        for (int it = 0; it < sweeps; ++it) {
            // res = w - beta j - V_g (Bt^T j); j += Woodbury(res)
            FDS_HIP_TRY(hipMemcpyAsync(res, wv, sizeof(double2) * tot, hipMemcpyDeviceToDevice, c.stream));
            axpby(c, make_double2(-op.beta, 0.0), jv, kOne, res, tot);
            zgemm(c, OP_N, OP_N, ne, (int)nb, n, kOne, op.Btr, ne, jv, n, kZero, z, ne);
            if (!zgemm_real_a(c, n, (int)nb, ne, make_double2(-1.0, 0.0), op.Vg, n, z, ne, kOne, res, n))
                zgemm(c, OP_N, OP_N, n, (int)nb, ne, make_double2(-1.0, 0.0), op.Vgc, n, z, ne, kOne, res, n);
            woodbury_apply(op, res, nb, z);
            axpby(c, kOne, res, kOne, jv, tot);
        }
    }
}

// The right-hand side w of the filter's form from f and h with caller-owned
// workspace t (n x nrhs); f is overwritten. Makes no allocation (split-K partial
// sums go to the context's workspace while one is set).
static void rhs_system_ws(Op& op, double2* f, const double2* h, int64_t nrhs, double2* w, double2* t) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    const int form = op.form;
    if (has_efie(form)) {
        gram_inv(op, f, nrhs, t);
        {
            SplitHint sh(c, 4);   // the batch's products run side by side in graph branches
            op_gemm(op, s_op(form), OP_T, nrhs, make_double2(-1.0, 0.0), t, kZero, f);
        }
        gram_inv(op, f, nrhs, w);
    }
    if (has_mfie(form)) {
        gram_inv(op, h, nrhs, t);
        if (form == FDS_MFIE) axpby(c, make_double2(-1.0, 0.0), t, kZero, w, (int64_t)n * nrhs);
        else axpby(c, make_double2(-op.alpha, 0.0), t, kOne, w, (int64_t)n * nrhs);
    }
}

// One problem of a batch: plane-wave right-hand sides, w, the Woodbury solve and
// `sweeps` filtered refinement sweeps, with no allocation and no host read, so
// that the launches can be recorded into a graph.
void run_batch_item(Op& op, const BatchItem& it, int sweeps, void* ws, size_t ws_bytes) {
    Ctx& c = *op.ctx;
    {
        NoAlloc na(c, ws, ws_bytes);
        launch_rhs_planewave(op, it.angles, it.amps, it.nrhs, it.f, it.h);
        rhs_system_ws(op, it.f, it.h, it.nrhs, it.w, it.t);
    }
    run_solve_system_ws(op, it.w, it.nrhs, it.j, sweeps, ws, ws_bytes);
}

}  // namespace fds
