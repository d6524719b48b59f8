// Dense building blocks of the truncating skeleton compression: the counter-
// based sketch, the QR factorisation of tall complex blocks with the explicit
// orthonormal factor (CholeskyQR2 on the matrix cores, certified, with blocked
// Householder QR as the fallback), and the one-sided (Hestenes) Jacobi SVD of
// small square blocks.
//
// Householder QR follows the standard complex reflector construction
// (Golub & Van Loan, Matrix Computations, sec. 5.1-5.2): column j is mapped to
// beta e_j by H_j = I - tau_j v_j v_j^H with v_j(j) = 1 and real beta, A is
// overwritten by R (upper triangle) and the v_j (below it), and
// Q = H_0 H_1 ... H_{m-1} [I; 0] is formed explicitly. Within a panel, one
// launch per column: the workgroup owning a column applies the previous
// reflector to it and the owner of the next pivot column then builds the next
// reflector, so no two workgroups ever touch the same column within a launch;
// the panel's reflectors then update the rest of the block in compact WY form.
//
// One-sided Jacobi (Hestenes 1958; Demmel & Veselic, SIAM J. Matrix Anal.
// Appl. 13, 1992) rotates pairs of columns of X until they are mutually
// orthogonal: X V = U Sigma with V unitary. Up to 312 columns the columns are
// grouped in blocks of 8 and the block pairs visited in the round-robin (circle)
// order, one launch per round, each workgroup rotating the 16 columns of its
// pair in LDS; wider matrices go pair by pair (m/2 disjoint pairs per launch,
// one workgroup per pair).
// The relative accuracy of small singular values is what the truncation rule
// needs, which a Gram-matrix eigensolver would not deliver.
#include <algorithm>
#include <cmath>

#include "fds_internal.h"
#include "linalg.h"
#include "lowrank.h"

namespace fds {

static constexpr int LR_BS = 256;
// Householder steps stream whole columns of a tall block through one workgroup
// each; 1024 threads with four rows in flight per thread keep enough loads
// outstanding for a single CU to run near its share of the memory bandwidth.
static constexpr int HH_BS = 1024;

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup of up to 4 values (BS threads). sh: 4 * (BS/64) doubles.
template <int K, int BS = LR_BS>
__device__ __forceinline__ void block_sum_k(double (&v)[K], double* sh) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int NW = BS / 64;
#pragma unroll
    for (int t = 0; t < K; ++t) v[t] = wave_sum(v[t]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int t = 0; t < K; ++t) sh[t * NW + wv] = v[t];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < K; ++t) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += sh[t * NW + w];
        v[t] = s;
    }
}

// 1/sqrt(x) and 1/x for x > 0: hardware estimates and two Newton steps each
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return y;
}

__device__ __forceinline__ double recip_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    y = fma(y, fma(-x, y, 1.0), y);
    return y;
}

// ----------------------------------------------------------------- sketch
// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), one output step of state z.
__device__ __forceinline__ uint64_t splitmix64_out(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Omega (n x ell, column-major): entry (i, j) from state seed ^ (i ell + j),
// ((1 - 2 b0) + i (1 - 2 b1)) / sqrt(2) with b0, b1 the two low output bits.
__global__ void sketch_kernel(uint64_t seed, int64_t n, int ell, double2* __restrict__ Om) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * ell) return;
    const int64_t j = t / n, i = t % n;
    const uint64_t z = splitmix64_out(seed ^ ((uint64_t)i * (uint64_t)ell + (uint64_t)j));
    const double r = 0.70710678118654752440;
    Om[t] = make_double2((z & 1ull) ? -r : r, (z & 2ull) ? -r : r);
}

void sketch(Ctx& c, uint64_t seed, int64_t n, int ell, double2* Om) {
    const int64_t tot = n * ell;
    {
        KScope _ks(c, "sketch");
        hipLaunchKernelGGL(sketch_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c.stream, seed, n,
                           ell, Om);
    }
    FDS_HIP_TRY(hipGetLastError());
}

// ----------------------------------------------------------------- Householder QR
// Blocked Householder QR with the compact WY form (Schreiber & Van Loan 1989):
// the reflectors H_j = I - tau_j v_j v_j^H of a panel of QR_NB columns are found
// column by column (hh_step_kernel), their product is I - V T V^H with T upper
// triangular, and the columns right of the panel are updated by
// A2 <- (I - V T^H V^H) A2 in three matrix-core products. Q = H_0 H_1 ... [I; 0]
// is formed panel by panel from the right, Q2 <- (I - V T V^H) Q2.
constexpr int QR_NB = 32;

// Launch j (panel starting at column j0): workgroup b owns column c = j + b.
// For j > j0 it applies H_{j-1}^H (a <- a - conj(tau) v (v^H a)) to its column
// over rows j-1..M-1; the owner of column j then builds H_j from rows j..M-1.
// Every thread walks the same rows in every loop, so it only re-reads what it
// wrote itself.
__global__ __launch_bounds__(HH_BS) void hh_step_kernel(double2* __restrict__ A, int64_t lda, int M, int j, int j0,
                                                        double2* __restrict__ tau) {
    __shared__ double sh[4 * (HH_BS / 64)];
    __shared__ double2 alpha_sh;
    const int c = j + blockIdx.x;
    const int tid = threadIdx.x;
    double2* a = A + (int64_t)c * lda;
    const bool apply = j > j0;
    const int base = apply ? j - 1 : j;
    double nrm2 = 0.0;
    if (apply) {
        const double2* v = A + (int64_t)(j - 1) * lda;
        const double2 tj = tau[j - 1];
        double s[2] = {0.0, 0.0};
#pragma unroll 4
        for (int r = base + tid; r < M; r += HH_BS) {
            const double2 vr = r == j - 1 ? make_double2(1.0, 0.0) : v[r];
            const double2 ar = a[r];
            s[0] += vr.x * ar.x + vr.y * ar.y;     // conj(v) a
            s[1] += vr.x * ar.y - vr.y * ar.x;
        }
        block_sum_k<2, HH_BS>(s, sh);
        const double2 f = cmul(cconj(tj), make_double2(s[0], s[1]));
#pragma unroll 4
        for (int r = base + tid; r < M; r += HH_BS) {
            const double2 vr = r == j - 1 ? make_double2(1.0, 0.0) : v[r];
            const double2 ar = csub(a[r], cmul(vr, f));
            a[r] = ar;
            if (c == j) {
                if (r == j) alpha_sh = ar;
                else if (r > j) nrm2 += ar.x * ar.x + ar.y * ar.y;
            }
        }
    } else {
#pragma unroll 4
        for (int r = j + tid; r < M; r += HH_BS) {
            const double2 ar = a[r];
            if (r == j) alpha_sh = ar;
            else nrm2 += ar.x * ar.x + ar.y * ar.y;
        }
    }
    if (c != j) return;
    double t[1] = {nrm2};
    block_sum_k<1, HH_BS>(t, sh);            // contains a barrier: alpha_sh is visible afterwards
    const double2 alpha = alpha_sh;
    nrm2 = t[0];
    if (nrm2 == 0.0 && alpha.y == 0.0) {
        if (tid == 0) tau[j] = make_double2(0.0, 0.0);
        return;
    }
    const double beta = -copysign(sqrt(alpha.x * alpha.x + alpha.y * alpha.y + nrm2), alpha.x);
    const double2 tj = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
    const double2 d = make_double2(alpha.x - beta, alpha.y);
    const double dd = d.x * d.x + d.y * d.y;
    const double2 sc = make_double2(d.x / dd, -d.y / dd);   // 1 / (alpha - beta)
#pragma unroll 4
    for (int r = base + tid; r < M; r += HH_BS) {
        if (r > j) a[r] = cmul(a[r], sc);
        else if (r == j) a[r] = make_double2(beta, 0.0);
    }
    if (tid == 0) tau[j] = tj;
}

// The reflectors of columns k0..k0+kb-1 as an explicit (M - k0) x kb block:
// unit diagonal, zeros above it.
__global__ void hh_panel_v_kernel(const double2* __restrict__ A, int64_t lda, int M, int k0, int kb,
                                  double2* __restrict__ V) {
    const int Mv = M - k0;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)Mv * kb) return;
    const int cc = (int)(t / Mv), r = (int)(t % Mv);
    V[t] = r < cc ? make_double2(0.0, 0.0)
                  : (r == cc ? make_double2(1.0, 0.0) : A[(int64_t)(k0 + cc) * lda + k0 + r]);
}

// T (kb x kb, column-major, upper triangular) with H_k0 ... H_{k0+kb-1} = I - V T V^H,
// from tau and the Gram matrix VV = V^H V: T_ii = tau_i,
// T[0:i, i] = -tau_i T[0:i, 0:i] VV[0:i, i].
__global__ __launch_bounds__(64) void hh_larft_kernel(const double2* __restrict__ tau, int kb,
                                                      const double2* __restrict__ VV, double2* __restrict__ T) {
    __shared__ double2 ts[QR_NB][QR_NB + 1];   // ts[row][col]
    const int r = threadIdx.x;
    for (int i = 0; i < kb; ++i) {
        const double2 ti = tau[i];
        double2 v = make_double2(0.0, 0.0);
        if (r < i) {
            double2 s = make_double2(0.0, 0.0);
            for (int l = r; l < i; ++l) s = cadd(s, cmul(ts[r][l], VV[(int64_t)i * kb + l]));
            v = make_double2(-(ti.x * s.x - ti.y * s.y), -(ti.x * s.y + ti.y * s.x));
        } else if (r == i) {
            v = ti;
        }
        if (r < kb) ts[r][i] = v;
        __syncthreads();
    }
    for (int t = r; t < kb * kb; t += 64) T[t] = ts[t % kb][t / kb];
}

// Q <- [I; 0] (M x m)
__global__ void eye_kernel(double2* __restrict__ Q, int64_t ldq, int M, int m) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)M * m) return;
    const int64_t c = t / M, r = t % M;
    Q[c * ldq + r] = make_double2(r == c ? 1.0 : 0.0, 0.0);
}

// X (m x m) = R^H, R the upper triangle of the factored A
__global__ void r_adjoint_kernel(const double2* __restrict__ A, int64_t lda, int m, double2* __restrict__ X) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * m) return;
    const int c = (int)(t / m), r = (int)(t % m);
    X[t] = c <= r ? cconj(A[(int64_t)r * lda + c]) : make_double2(0.0, 0.0);
}

static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

static void householder_qr(Ctx& c, double2* A, int M, int m, double2* tau, double2* Q) {
    FDS_REQUIRE(m >= 1 && M >= m, FDS_ERR_ARG, "Householder QR needs rows >= columns >= 1");
    const int npan = (m + QR_NB - 1) / QR_NB;
    const bool blocks = npan > 1 || Q;
    // per panel k (columns k0 = k QR_NB ..): V_k ((M - k0) x kb at V + k0 M) and T_k
    double2* V = blocks ? static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)M * m)) : nullptr;
    double2* T = blocks ? static_cast<double2*>(c.dmalloc(sizeof(double2) * QR_NB * QR_NB * (size_t)npan)) : nullptr;
    double2* VV = blocks ? static_cast<double2*>(c.dmalloc(sizeof(double2) * QR_NB * QR_NB)) : nullptr;
    double2* W = blocks ? static_cast<double2*>(c.dmalloc(sizeof(double2) * QR_NB * (size_t)m)) : nullptr;
    double2* W2 = blocks ? static_cast<double2*>(c.dmalloc(sizeof(double2) * QR_NB * (size_t)m)) : nullptr;
    const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0), mone = make_double2(-1.0, 0.0);
    GemmTag tg(c, "qr_update");   // the compact-WY products
    for (int k = 0; k < npan; ++k) {
        const int k0 = k * QR_NB, kb = std::min(QR_NB, m - k0), Mv = M - k0, mt = m - k0 - kb;
        {
            KScope _ks(c, "qr_householder");
            for (int j = k0; j < k0 + kb; ++j) {
                const unsigned g = j == k0 ? 1u : (unsigned)(k0 + kb - j);
                hipLaunchKernelGGL(hh_step_kernel, dim3(g), dim3(HH_BS), 0, c.stream, A, (int64_t)M, M, j, k0,
                                   tau);
            }
        }
        FDS_HIP_TRY(hipGetLastError());
        if (!blocks) break;
        double2* Vk = V + (size_t)k0 * M;
        double2* Tk = T + (size_t)k * QR_NB * QR_NB;
        {
            KScope _ks(c, "qr_householder");
            hipLaunchKernelGGL(hh_panel_v_kernel, dim3(nblk((int64_t)Mv * kb, 256)), dim3(256), 0, c.stream, A,
                               (int64_t)M, M, k0, kb, Vk);
        }
        FDS_HIP_TRY(hipGetLastError());
        zgemm(c, OP_C, OP_N, kb, kb, Mv, one, Vk, Mv, Vk, Mv, zero, VV, kb);
        {
            KScope _ks(c, "qr_householder");
            hipLaunchKernelGGL(hh_larft_kernel, dim3(1), dim3(64), 0, c.stream, tau + k0, kb, VV, Tk);
        }
        FDS_HIP_TRY(hipGetLastError());
        if (mt > 0) {
            // A2 <- A2 - V (T^H (V^H A2)), A2 = rows k0.., columns k0 + kb..
            double2* A2 = A + (int64_t)(k0 + kb) * M + k0;
            zgemm(c, OP_C, OP_N, kb, mt, Mv, one, Vk, Mv, A2, M, zero, W, kb);
            zgemm(c, OP_C, OP_N, kb, mt, kb, one, Tk, kb, W, kb, zero, W2, kb);
            zgemm(c, OP_N, OP_N, Mv, mt, kb, mone, Vk, Mv, W2, kb, one, A2, M);
        }
    }
    if (Q) {
        {
            KScope _ks(c, "qr_form_q");
            hipLaunchKernelGGL(eye_kernel, dim3(nblk((int64_t)M * m, 256)), dim3(256), 0, c.stream, Q, (int64_t)M,
                               M, m);
        }
        FDS_HIP_TRY(hipGetLastError());
        for (int k = npan - 1; k >= 0; --k) {
            // Q2 <- Q2 - V (T (V^H Q2)), Q2 = rows k0.., columns k0.. (the columns
            // left of k0 are still zero in those rows)
            const int k0 = k * QR_NB, kb = std::min(QR_NB, m - k0), Mv = M - k0, mq = m - k0;
            const double2* Vk = V + (size_t)k0 * M;
            const double2* Tk = T + (size_t)k * QR_NB * QR_NB;
            double2* Q2 = Q + (int64_t)k0 * M + k0;
            zgemm(c, OP_C, OP_N, kb, mq, Mv, one, Vk, Mv, Q2, M, zero, W, kb);
            zgemm(c, OP_N, OP_N, kb, mq, kb, one, Tk, kb, W, kb, zero, W2, kb);
            zgemm(c, OP_N, OP_N, Mv, mq, kb, mone, Vk, Mv, W2, kb, one, Q2, M);
        }
    }
    if (blocks) {
        c.dfree(V);
        c.dfree(T);
        c.dfree(VV);
        c.dfree(W);
        c.dfree(W2);
    }
}

// ----------------------------------------------------------------- Cholesky QR
// CholeskyQR2 (Fukaya, Nakatsukasa, Yanagisawa & Yamamoto, ScalA 2014):
// G1 = A^H A = R1^H R1, Q1 = A R1^{-1}; G2 = Q1^H Q1 = R2^H R2, Q = Q1 R2^{-1};
// R = R2 R1. The Gram products and the right-multiplications are matrix-core
// GEMMs; each Cholesky factor and its triangular inverse come from one
// workgroup holding the packed lower triangle of the Gram matrix in LDS.
// The first pass leaves Q1 with ||Q1^H Q1 - I|| of order kappa(A)^2 u, and the
// second pass, started from a well-conditioned Q1, is accurate to unit
// roundoff. The second Gram matrix certifies the first pass: ||G2 - I||_F < 1/2
// bounds kappa(Q1)^2 by 3. When that check or a pivot fails the blocked
// Householder factorisation runs instead.
constexpr int CQ_BS = 512;
constexpr int CQ_MAX = 140;   // packed triangle (157,920 B) and the buffers below fit 160 KiB of LDS
constexpr int CQ_TRI = CQ_MAX * (CQ_MAX + 1) / 2;

// packed column-major lower triangle: column c holds rows c..m-1
__device__ __forceinline__ int cq_idx(int m, int r, int c) { return c * (2 * m - c - 1) / 2 + r; }

// Sums over groups of Ls consecutive lanes (Ls a power of two <= 16) by DPP
// moves within rows of 16 lanes: lane ^ 1, lane ^ 2, then the mirror images in
// the half row and in the row; every lane of a group ends with the group's sum.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(bits & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double group_sum(double v, int Ls) {
    if (Ls >= 2) v += dpp_mov<0xB1>(v);    // quad_perm(1, 0, 3, 2)
    if (Ls >= 4) v += dpp_mov<0x4E>(v);    // quad_perm(2, 3, 0, 1)
    if (Ls >= 8) v += dpp_mov<0x141>(v);   // row_half_mirror
    if (Ls >= 16) v += dpp_mov<0x140>(v);  // row_mirror
    return v;
}

typedef double cgd4 __attribute__((ext_vector_type(4)));
constexpr int CB = 16;   // columns per step of the factorisation

// G (m x m Hermitian, column-major, ld m) = L L^H. Writes R = L^H (m x m upper
// triangular, zeros below). flag: set to 1 when a pivot is not positive or, with
// check, when ||G - I||_F >= 1/2; with check the previous flag is kept (or-ed),
// without it the flag is overwritten.
//
// CB columns per step. The inner products over finished columns are a small
// matrix product on the FP64 matrix cores (one 16-row tile per wavefront); the
// step's CB x CB diagonal block is then factored by wavefront 0 and the rest of
// the step solved one row per thread.
__global__ __launch_bounds__(CQ_BS) void chol_kernel(const double2* __restrict__ G, int m, int check,
                                                     double2* __restrict__ R, int* __restrict__ flag) {
    __shared__ double2 L[CQ_TRI];       // packed lower triangle
    __shared__ double pv[CQ_MAX];       // 1 / pivot
    __shared__ double2 colc[CB];        // a column of the diagonal block
    __shared__ double red[CQ_BS / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double dev = 0.0;
    // whole-matrix loops: column c per wavefront, rows by lane
    for (int c = wave; c < m; c += CQ_BS / 64)
        for (int r = lane; r < m; r += 64) {
            const double2 g = G[(size_t)c * m + r];
            if (r >= c) L[cq_idx(m, r, c)] = g;
            const double ex = g.x - (r == c ? 1.0 : 0.0);
            dev += ex * ex + g.y * g.y;
        }
    {
        double v[1] = {dev};
        block_sum_k<1, CQ_BS>(v, red);   // barriers: L is complete afterwards
        dev = v[0];
    }
    int bad = check && !(dev < 0.25);

    // Cholesky, Crout order, unnormalised: with d_l the pivots,
    //   Lh(r, c) = G(r, c) - sum_{l<c} Lh(r, l) conj(Lh(c, l)) / d_l,  d_c = Lh(c, c),
    // and L(r, c) = Lh(r, c) / sqrt(d_c).
    for (int j = 0; j < m; j += CB) {
        const int bw = min(CB, m - j), u = m - j;
        {   // rows r >= j, the step's columns, terms l < j, on the FP64 matrix cores: one
            // 16-row tile per wavefront, S = Lh[rows, :j] (conj(Lh[j + c, :j]) / d)^T by
            // Gauss's three products (T1 = ar br, T2 = ai bi, T3 = (ar + ai)(br + bi))
            const int nrt = (u + 15) / 16, ln = lane & 15, lk = lane >> 4;
            for (int rt = wave; rt < nrt && j > 0; rt += CQ_BS / 64) {   // uniform per wavefront
                const int r0 = j + rt * 16, ra = r0 + ln;
                cgd4 t1 = {0.0, 0.0, 0.0, 0.0}, t2 = {0.0, 0.0, 0.0, 0.0}, t3 = {0.0, 0.0, 0.0, 0.0};
                for (int l0 = 0; l0 < j; l0 += 4) {   // j is a multiple of 16
                    const int l = l0 + lk;
                    const double2* col = L + cq_idx(m, 0, l);   // column l, indexed by row
                    const double2 av = ra < m ? col[ra] : make_double2(0.0, 0.0);
                    const double2 bv = ln < bw ? col[j + ln] : make_double2(0.0, 0.0);
                    const double w = pv[l];
                    const double br = w * bv.x, bi = -w * bv.y;
                    t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, br, t1, 0, 0, 0);
                    t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bi, t2, 0, 0, 0);
                    t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x + av.y, br + bi, t3, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {   // element v: row r0 + lk + 4 v, column ln
                    const int r = r0 + lk + 4 * v, c = ln;
                    if (r < m && c < bw && j + c <= r) {
                        double2& x = L[cq_idx(m, r, j + c)];
                        x.x -= t1[v] - t2[v];
                        x.y -= t3[v] - t1[v] - t2[v];
                    }
                }
            }
        }
        __syncthreads();
        if (wave == 0) {
            // the diagonal block, right-looking, in the registers of wavefront 0:
            // lane 4a + q holds D(a, q + 4k), k = 0..3; column c goes round through colc
            const int a = lane >> 2, q = lane & 3;
            double2 x[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int e = q + 4 * k;
                x[k] = (a < bw && e <= a) ? L[cq_idx(m, j + a, j + e)] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                if (c < bw) {   // uniform
                    if (q == (c & 3)) colc[a] = x[c >> 2];
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    const double id = recip_nr(colc[c].x);
                    const double2 la = colc[a];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int e = q + 4 * k;
                        if (c < e && e <= a && a < bw) {   // D(a, e) -= D(a, c) conj(D(e, c)) / d_c
                            const double2 le = colc[e];
                            x[k].x -= id * (la.x * le.x + la.y * le.y);
                            x[k].y -= id * (la.y * le.x - la.x * le.y);
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                    __builtin_amdgcn_wave_barrier();   // colc is rewritten by the next column
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int e = q + 4 * k;
                if (a < bw && e <= a) L[cq_idx(m, j + a, j + e)] = x[k];
                if (a < bw && e == a) pv[j + a] = 1.0 / x[k].x;
            }
        }
        __syncthreads();
        {   // rows below the block: the triangular part, one row per thread
            const int r = j + bw + tid;
            if (r < m) {
                int cb[CB];   // the block's columns, indexed by row
#pragma unroll
                for (int c = 0; c < CB; ++c) cb[c] = cq_idx(m, 0, min(j + c, m - 1));
                double2 p[CB];
#pragma unroll
                for (int c = 0; c < CB; ++c) p[c] = c < bw ? L[cb[c] + r] : make_double2(0.0, 0.0);
#pragma unroll
                for (int c = 1; c < CB; ++c) {
                    if (c < bw) {
#pragma unroll
                        for (int e = 0; e < c; ++e) {   // p[c] -= p[e] conj(Lh(j+c, j+e)) / d_{j+e}
                            const double2 v = L[cb[e] + j + c];
                            const double w = pv[j + e];
                            p[c].x -= w * (p[e].x * v.x + p[e].y * v.y);
                            p[c].y -= w * (p[e].y * v.x - p[e].x * v.y);
                        }
                    }
                }
#pragma unroll
                for (int c = 0; c < CB; ++c)
                    if (c < bw) L[cb[c] + r] = p[c];
            }
        }
        __syncthreads();
    }
    // normalise: L(r, l) = Lh(r, l) / sqrt(d_l), L(l, l) = sqrt(d_l)
    for (int c = wave; c < m; c += CQ_BS / 64) {
        const double sc = sqrt(pv[c]);
        for (int r = c + lane; r < m; r += 64) {
            double2& x = L[cq_idx(m, r, c)];
            if (r == c) {
                if (!(x.x > 0.0)) bad = 1;
                x = make_double2(sqrt(x.x), 0.0);
            } else {
                x.x *= sc;
                x.y *= sc;
            }
        }
    }
    bad = __syncthreads_or(bad);
    for (int c = wave; c < m; c += CQ_BS / 64)
        for (int r = lane; r < m; r += 64)
            R[(size_t)c * m + r] = r < c ? cconj(L[cq_idx(m, c, r)])
                                         : make_double2(r == c ? L[cq_idx(m, r, r)].x : 0.0, 0.0);
    if (tid == 0) *flag = (check ? *flag : 0) | bad;
}

// Y = R^{-1} for R upper triangular (m x m, column-major, ld m) from Y R = I,
// whose rows are independent: workgroup w forms rows r0 = 16 w .. r0 + 15,
// column blocks C = c0 .. c0 + 15 from the left (c0 >= r0):
//   T = -Y[rows, r0 : c0] R[r0 : c0, C]                    (one entry per thread)
//   y(i, c) = (T(i, c) + [r0 + i == c] - sum_{q in C, q < c} y(i, q) R(q, c)) / R(c, c)
// the latter one row per thread, left to right. Entries left of the diagonal are 0.
constexpr int TI_B = 16;

__global__ __launch_bounds__(256) void tri_inv_kernel(const double2* __restrict__ R, int m,
                                                      double2* __restrict__ Y) {
    __shared__ double2 ys[TI_B][CQ_MAX];        // this workgroup's rows of Y
    __shared__ double2 rb[CQ_MAX][TI_B + 1];    // the column block of R, rows r0 .. c0 + 15
    __shared__ double2 ts[TI_B][TI_B + 1];
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * TI_B;
    for (int t = tid; t < TI_B * m; t += 256) ys[t / m][t % m] = make_double2(0.0, 0.0);
    for (int c0 = r0; c0 < m; c0 += TI_B) {
        const int cw = min(TI_B, m - c0), lend = c0 + cw;
        __syncthreads();   // the previous block's ys and rb reads are done
        for (int t = tid; t < (lend - r0) * cw; t += 256) {
            const int j = t / (lend - r0), l = r0 + t % (lend - r0);
            rb[l][j] = R[(size_t)(c0 + j) * m + l];
        }
        __syncthreads();
        {
            const int i = tid / TI_B, j = tid % TI_B;
            double2 acc = make_double2(0.0, 0.0);
            if (j < cw)
                for (int l = r0; l < c0; ++l) {
                    const double2 a = ys[i][l], b = rb[l][j];
                    acc.x -= a.x * b.x - a.y * b.y;
                    acc.y -= a.x * b.y + a.y * b.x;
                }
            ts[i][j] = acc;
        }
        __syncthreads();
        if (tid < TI_B && r0 + tid < m) {
            const int i = tid, r = r0 + i;
            double2 yv[TI_B];
#pragma unroll
            for (int j = 0; j < TI_B; ++j) {
                yv[j] = make_double2(0.0, 0.0);
                const int c = c0 + j;
                if (j >= cw || c < r) continue;
                double2 sacc = ts[i][j];
                if (c == r) sacc.x += 1.0;
#pragma unroll
                for (int q = 0; q < j; ++q) {
                    const double2 b = rb[c0 + q][j];
                    sacc.x -= yv[q].x * b.x - yv[q].y * b.y;
                    sacc.y -= yv[q].x * b.y + yv[q].y * b.x;
                }
                const double2 d = rb[c][j];   // real positive diagonal of a Cholesky factor
                const double id = 1.0 / d.x;
                yv[j] = make_double2(sacc.x * id, sacc.y * id);
            }
#pragma unroll
            for (int j = 0; j < TI_B; ++j)
                if (j < cw) ys[i][c0 + j] = yv[j];
        }
    }
    __syncthreads();
    for (int t = tid; t < TI_B * m; t += 256) {
        const int i = t % TI_B, c = t / TI_B;
        if (r0 + i < m) Y[(size_t)c * m + r0 + i] = ys[i][c];
    }
}

// Gram matrix G = A^H A of a tall block (M x m, m <= GT_COLS, column-major, ld
// lda) on the FP64 matrix cores. Workgroup b sums the GT_ROWS-row chunks b,
// b + grid, ... into the 45 lower 16 x 16 tiles of its partial (the columns zero-padded to
// GT_COLS); gram_tall_reduce_kernel adds the partials in a fixed order and fills
// the upper triangle by conjugate symmetry. Per tile, Gauss's three real products
// with a = conj(A(k, i)), b = A(k, j): T1 = ar br, T2 = ai bi,
// T3 = (ar - ai)(br + bi); Re G = T1 + T2, Im G = T3 - T1 + T2.
typedef double gd4 __attribute__((ext_vector_type(4)));
constexpr int GT_COLS = 144;                      // 9 column blocks of 16 (>= CQ_MAX)
constexpr int GT_T = GT_COLS / 16;
constexpr int GT_NTILE = GT_T * (GT_T + 1) / 2;   // 45 lower tiles
constexpr int GT_ROWS = 64;
constexpr int GT_WAVES = 8;
constexpr int GT_TPW = (GT_NTILE + GT_WAVES - 1) / GT_WAVES;   // tiles per wavefront (6)

__global__ __launch_bounds__(64 * GT_WAVES) void gram_tall_kernel(const double2* __restrict__ A, int64_t lda, int M,
                                                                  int m, double2* __restrict__ part) {
    __shared__ double sr[GT_ROWS][GT_COLS + 1];
    __shared__ double si[GT_ROWS][GT_COLS + 1];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // this wavefront's tiles: w, w + GT_WAVES, ... in the row-major order of the lower triangle
    int ti[GT_TPW], tj[GT_TPW];
#pragma unroll
    for (int u = 0; u < GT_TPW; ++u) {
        int t = w + u * GT_WAVES, i = 0;
        while (t > i) { t -= i + 1; ++i; }   // t-th entry of row i: (i, t), t <= i
        ti[u] = i;
        tj[u] = t;
    }
    gd4 t1[GT_TPW], t2[GT_TPW], t3[GT_TPW];
#pragma unroll
    for (int u = 0; u < GT_TPW; ++u) {
        t1[u] = gd4{0.0, 0.0, 0.0, 0.0};
        t2[u] = gd4{0.0, 0.0, 0.0, 0.0};
        t3[u] = gd4{0.0, 0.0, 0.0, 0.0};
    }
    const int ln = lane & 15, lk = lane >> 4;
    const int nchunk = (M + GT_ROWS - 1) / GT_ROWS;
    for (int ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {   // chunks of GT_ROWS rows
        const int r0 = ch * GT_ROWS;
        __syncthreads();   // the previous chunk's reads are done
        for (int t = tid; t < GT_ROWS * GT_COLS; t += 64 * GT_WAVES) {
            const int k = t % GT_ROWS, c = t / GT_ROWS;   // consecutive threads: consecutive rows of a column
            const double2 v = (r0 + k < M && c < m) ? A[(int64_t)c * lda + r0 + k] : make_double2(0.0, 0.0);
            sr[k][c] = v.x;
            si[k][c] = v.y;
        }
        __syncthreads();
        for (int kk = 0; kk < GT_ROWS; kk += 4) {
            const int k = kk + lk;
#pragma unroll
            for (int u = 0; u < GT_TPW; ++u) {
                if (w + u * GT_WAVES >= GT_NTILE) continue;   // uniform
                const int ci = ti[u] * 16 + ln, cj = tj[u] * 16 + ln;
                const double ar = sr[k][ci], ai = si[k][ci], br = sr[k][cj], bi = si[k][cj];
                t1[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, t1[u], 0, 0, 0);
                t2[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, t2[u], 0, 0, 0);
                t3[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar - ai, br + bi, t3[u], 0, 0, 0);
            }
        }
    }
    double2* P = part + (int64_t)blockIdx.x * GT_COLS * GT_COLS;   // column-major GT_COLS x GT_COLS
#pragma unroll
    for (int u = 0; u < GT_TPW; ++u) {
        if (w + u * GT_WAVES >= GT_NTILE) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = ti[u] * 16 + lk + 4 * v, j = tj[u] * 16 + ln;
            P[(int64_t)j * GT_COLS + i] = make_double2(t1[u][v] + t2[u][v], t3[u][v] - t1[u][v] + t2[u][v]);
        }
    }
}

// G (m x m, ld m) = sum of the nb partials' lower tiles, upper triangle by
// symmetry. Workgroup j takes column j of the stored tiles (rows from the first
// row of its tile block on, contiguous in every partial) and writes G(i, j) and
// G(j, i) = conj(G(i, j)).
__global__ __launch_bounds__(GT_COLS) void gram_tall_reduce_kernel(const double2* __restrict__ part, int nb, int m,
                                                                   double2* __restrict__ G) {
    const int j = blockIdx.x;
    const int i = (j / 16) * 16 + threadIdx.x;
    if (i >= m) return;
    // eight partial sums (partials b = 8q + u go to sum u) keep eight loads in flight
    const double2* src = part + (int64_t)j * GT_COLS + i;
    constexpr int64_t ST = (int64_t)GT_COLS * GT_COLS;
    double sx[8], sy[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) sx[u] = sy[u] = 0.0;
    int b = 0;
    for (; b + 8 <= nb; b += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double2 v = src[(b + u) * ST];
            sx[u] += v.x;
            sy[u] += v.y;
        }
    }
    for (int u = 0; b < nb; ++b, ++u) {
        const double2 v = src[b * ST];
        sx[u] += v.x;
        sy[u] += v.y;
    }
    const double2 s = make_double2(((sx[0] + sx[1]) + (sx[2] + sx[3])) + ((sx[4] + sx[5]) + (sx[6] + sx[7])),
                                   ((sy[0] + sy[1]) + (sy[2] + sy[3])) + ((sy[4] + sy[5]) + (sy[6] + sy[7])));
    G[(int64_t)j * m + i] = s;
    if (i / 16 != j / 16) G[(int64_t)i * m + j] = make_double2(s.x, -s.y);   // the diagonal tiles are stored whole
}

// workgroups of the tall Gram kernel (and partials): one per 64-row chunk, at most 512
static inline int gram_tall_groups(int M) { return std::min(512, (M + GT_ROWS - 1) / GT_ROWS); }

static void gram_tall(Ctx& c, const double2* A, int M, int m, double2* G, double2* part) {
    const int nb = gram_tall_groups(M);
    KScope _ks(c, "qr_gram");
    hipLaunchKernelGGL(gram_tall_kernel, dim3((unsigned)nb), dim3(64 * GT_WAVES), 0, c.stream, A, (int64_t)M, M, m,
                       part);
    hipLaunchKernelGGL(gram_tall_reduce_kernel, dim3((unsigned)m), dim3(GT_COLS), 0, c.stream, part, nb, m, G);
}

// flag |= (||G - I||_F >= 1/2), G m x m (column-major, ld m)
__global__ __launch_bounds__(256) void gram_check_kernel(const double2* __restrict__ G, int m, int* __restrict__ flag) {
    __shared__ double sh[4 * 4];
    double v[1] = {0.0};
    for (int t = threadIdx.x; t < m * m; t += 256) {
        const double2 g = G[t];
        const double ex = g.x - (t % m == t / m ? 1.0 : 0.0);
        v[0] += ex * ex + g.y * g.y;
    }
    block_sum_k<1, 256>(v, sh);
    if (threadIdx.x == 0 && !(v[0] < 0.25)) *flag = 1;
}

// CholeskyQR2 of A (M x m): Q receives the orthonormal factor and the upper
// triangle of A the R factor. With basis_only the first pass is the result:
// Q = A R1^{-1} spans range(A) with ||Q^H Q - I||_F < 1/2 (certified by its
// Gram matrix), which is what a subspace iteration step needs. Returns false,
// with A unchanged, when the factorisation does not certify itself.
static bool cholesky_qr2(Ctx& c, double2* A, int M, int m, double2* Q, bool basis_only) {
    if (m > CQ_MAX) return false;
    const size_t mm = (size_t)m * m;
    double2* G = static_cast<double2*>(c.dmalloc(sizeof(double2) * mm * 4));
    double2 *R1 = G + mm, *R2 = G + 2 * mm, *Ri = G + 3 * mm;
    double2* Q1 = basis_only ? nullptr : static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)M * m));
    int* flag = static_cast<int*>(c.dmalloc(sizeof(int)));
    // partial Gram matrices, one per workgroup of the tall Gram kernel
    double2* part = static_cast<double2*>(c.dmalloc(sizeof(double2) * GT_COLS * GT_COLS * (size_t)gram_tall_groups(M)));
    const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
    GemmTag tg(c, "qr_gram");
    double2* R[2] = {R1, R2};
    const double2* in[2] = {A, Q1};
    double2* out[2] = {Q1, Q};
    if (basis_only) out[0] = Q;
    for (int pass = 0; pass < 2; ++pass) {
        gram_tall(c, in[pass], M, m, G, part);
        if (basis_only && pass == 1) {
            KScope _ks(c, "qr_cholesky");
            hipLaunchKernelGGL(gram_check_kernel, dim3(1), dim3(256), 0, c.stream, G, m, flag);
            break;
        }
        {
            KScope _ks(c, "qr_cholesky");
            hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(CQ_BS), 0, c.stream, G, m, pass, R[pass], flag);
            hipLaunchKernelGGL(tri_inv_kernel, dim3((unsigned)((m + TI_B - 1) / TI_B)), dim3(256), 0, c.stream,
                               R[pass], m, Ri);
        }
        FDS_HIP_TRY(hipGetLastError());
        zgemm(c, OP_N, OP_N, M, m, m, one, in[pass], M, Ri, m, zero, out[pass], M);
        if (basis_only) in[1] = Q;
    }
    int bad = 1;
    FDS_HIP_TRY(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    FDS_HIP_TRY(hipStreamSynchronize(c.stream));
    if (!bad) {
        if (basis_only)
            FDS_HIP_TRY(hipMemcpy2DAsync(A, sizeof(double2) * (size_t)M, R1, sizeof(double2) * (size_t)m,
                                         sizeof(double2) * (size_t)m, (size_t)m, hipMemcpyDeviceToDevice, c.stream));
        else
            zgemm(c, OP_N, OP_N, m, m, m, one, R2, m, R1, m, zero, A, M);
    }
    c.dfree(G);
    c.dfree(Q1);
    c.dfree(flag);
    c.dfree(part);
    return !bad;
}

bool qr_explicit(Ctx& c, double2* A, int M, int m, double2* tau, double2* Q, bool cholesky, bool basis_only) {
    FDS_REQUIRE(m >= 1 && M >= m && Q, FDS_ERR_ARG, "QR needs rows >= columns >= 1 and an output");
    if (cholesky && cholesky_qr2(c, A, M, m, Q, basis_only)) return true;
    householder_qr(c, A, M, m, tau, Q);
    return false;
}

void r_adjoint(Ctx& c, const double2* A, int M, int m, double2* X) {
    {
        KScope _ks(c, "qr_form_q");
        hipLaunchKernelGGL(r_adjoint_kernel, dim3(nblk((int64_t)m * m, 256)), dim3(256), 0, c.stream, A,
                           (int64_t)M, m, X);
    }
    FDS_HIP_TRY(hipGetLastError());
}

// ----------------------------------------------------------------- one-sided Jacobi
// Round `round` of the circle method on mpad (even) players: pair 0 is
// (round, mpad-1), pair k > 0 is ((round+k) mod (mpad-1), (round-k) mod (mpad-1)).
// Columns >= m are absent (odd m). The rotation
//     [x_p', x_q'] = [x_p, x_q] [[c, s], [-s e, c e]],   e = conj(g)/|g|, g = x_p^H x_q,
// with t = tan(theta) the smaller root of t^2 + 2 zeta t - 1 = 0,
// zeta = (|x_q|^2 - |x_p|^2) / (2|g|), makes the pair orthogonal; V gets the
// same rotation.
__global__ __launch_bounds__(LR_BS) void jacobi_round_kernel(double2* __restrict__ X, int rows,
                                                             double2* __restrict__ V, int m, int mpad,
                                                             int round, double tol, int* __restrict__ counter) {
    __shared__ double sh[4 * (LR_BS / 64)];
    const int k = blockIdx.x;
    const int L = mpad - 1;
    int p, q;
    if (k == 0) {
        p = round;
        q = L;
    } else {
        p = (round + k) % L;
        q = (round - k + L) % L;
    }
    if (p >= m || q >= m) return;
    const int tid = threadIdx.x;
    double2* xp = X + (int64_t)p * rows;
    double2* xq = X + (int64_t)q * rows;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = tid; r < rows; r += LR_BS) {
        const double2 a = xp[r], b = xq[r];
        s[0] += a.x * a.x + a.y * a.y;
        s[1] += b.x * b.x + b.y * b.y;
        s[2] += a.x * b.x + a.y * b.y;   // conj(a) b
        s[3] += a.x * b.y - a.y * b.x;
    }
    block_sum_k<4>(s, sh);
    const double al = s[0], be = s[1];
    const double ag = hypot(s[2], s[3]);
    if (!(al > 0.0 && be > 0.0) || !(ag > tol * sqrt(al) * sqrt(be))) return;
    const double zeta = (be - al) / (2.0 * ag);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
    const double2 e = make_double2(s[2] / ag, -s[3] / ag);
    const double2 se = cscale(e, sn), ce = cscale(e, cs);
    for (int r = tid; r < rows; r += LR_BS) {
        const double2 a = xp[r], b = xq[r];
        xp[r] = csub(cscale(a, cs), cmul(se, b));
        xq[r] = cadd(cscale(a, sn), cmul(ce, b));
    }
    double2* vp = V + (int64_t)p * m;
    double2* vq = V + (int64_t)q * m;
    for (int r = tid; r < m; r += LR_BS) {
        const double2 a = vp[r], b = vq[r];
        vp[r] = csub(cscale(a, cs), cmul(se, b));
        vq[r] = cadd(cscale(a, sn), cmul(ce, b));
    }
    if (tid == 0) atomicAdd(counter, 1);
}

// Block one-sided Jacobi (the columns grouped in blocks of JB; block pairs in the
// circle order, one launch per round): workgroup k takes its pair of blocks,
// holds their 2 JB columns of X and of V in LDS and rotates the JB x JB cross
// pairs of the two blocks (JB inner rounds, one wavefront per pair), in the
// sweep's first round also the pairs within each block, with the threshold and
// rotation of jacobi_round_kernel. A sweep (every block pair once) visits every
// column pair exactly once, so it is a cyclic Jacobi ordering.
// rows held in LDS for blocks of B columns: X and V columns of two blocks,
// 2 x 2B x rows x 16 B within 156 KiB (312 rows for B = 8, 156 for B = 16)
template <int B>
constexpr int jb_maxrows() { return 159744 / (2 * 2 * B * 16); }
template <int B>
constexpr int jb_ld() { return (2 * B * jb_maxrows<B>() + 64 * B - 1) / (64 * B); }   // entries per thread

// sum over the wavefront without LDS traffic: DPP sums within rows of 16 lanes,
// then the four row sums read out of lanes 0, 16, 32 and 48
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v = group_sum(v, 16);
    const long long b = __double_as_longlong(v);
    double t = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 16 * r);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 16 * r);
        t += __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
    }
    return t;
}

// columns c of the block pair (2 JB of them, rows entries each) between global
// memory and LDS, all loads of a thread issued before its LDS stores
template <int JB, bool LOAD>
__device__ __forceinline__ void jb_move(double2* __restrict__ G, int64_t ld, int rows, int m, int P, int Q,
                                        double2 (*S)[jb_maxrows<JB>()]) {
    constexpr int JB_LD = jb_ld<JB>();
    double2 buf[JB_LD];
#pragma unroll
    for (int u = 0; u < JB_LD; ++u) {
        const int i = threadIdx.x + u * 64 * JB;
        const int c = i / rows, r = i - c * rows;
        const int g = (c < JB ? P : Q) * JB + (c % JB);
        const bool ok = c < 2 * JB && g < m;
        if (LOAD) buf[u] = ok ? G[(int64_t)g * ld + r] : make_double2(0.0, 0.0);
        else if (ok) G[(int64_t)g * ld + r] = S[c][r];
    }
    if (LOAD) {
#pragma unroll
        for (int u = 0; u < JB_LD; ++u) {
            const int i = threadIdx.x + u * 64 * JB;
            const int c = i / rows, r = i - c * rows;
            if (c < 2 * JB) S[c][r] = buf[u];
        }
    }
}

template <int JB>
__global__ __launch_bounds__(64 * JB) void jacobi_block_kernel(double2* __restrict__ X, int rows,
                                                               double2* __restrict__ V, int m, int nbp, int round,
                                                               double tol, int* __restrict__ counter) {
    constexpr int MR = jb_maxrows<JB>();
    __shared__ double2 xs[2 * JB][MR];
    __shared__ double2 vs[2 * JB][MR];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int k = blockIdx.x, L = nbp - 1;
    const int P = k == 0 ? round : (round + k) % L;
    const int Q = k == 0 ? L : (round - k + L) % L;
    auto gcol = [&](int c) { return (c < JB ? P : Q) * JB + (c % JB); };
    jb_move<JB, true>(X, rows, rows, m, P, Q, xs);
    jb_move<JB, true>(V, m, m, m, P, Q, vs);
    __syncthreads();
    int rot = 0;
    // one rotation of local columns p and q by the calling wavefront
    auto rotate = [&](int p, int q) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int r = lane; r < rows; r += 64) {
            const double2 a = xs[p][r], b = xs[q][r];
            s0 += a.x * a.x + a.y * a.y;
            s1 += b.x * b.x + b.y * b.y;
            s2 += a.x * b.x + a.y * b.y;   // conj(a) b
            s3 += a.x * b.y - a.y * b.x;
        }
        const double al = wave_sum_dpp(s0), be = wave_sum_dpp(s1), gr = wave_sum_dpp(s2), gi = wave_sum_dpp(s3);
        const double ag2 = gr * gr + gi * gi;
        if (!(al > 0.0 && be > 0.0 && ag2 > tol * tol * al * be)) return;
        // the rotation of jacobi_round_kernel, with square roots and quotients
        // from the hardware estimates refined by Newton steps
        const double iag = rsqrt_nr(ag2);
        const double zeta = (be - al) * 0.5 * iag;
        const double q1 = 1.0 + zeta * zeta;
        const double sq = q1 * rsqrt_nr(q1);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) * recip_nr(fabs(zeta) + sq);
        const double cs = rsqrt_nr(1.0 + t * t), sn = cs * t;
        const double2 e = make_double2(gr * iag, -gi * iag);
        const double2 se = cscale(e, sn), ce = cscale(e, cs);
        for (int r = lane; r < rows; r += 64) {
            const double2 a = xs[p][r], b = xs[q][r];
            xs[p][r] = csub(cscale(a, cs), cmul(se, b));
            xs[q][r] = cadd(cscale(a, sn), cmul(ce, b));
        }
        for (int r = lane; r < m; r += 64) {
            const double2 a = vs[p][r], b = vs[q][r];
            vs[p][r] = csub(cscale(a, cs), cmul(se, b));
            vs[q][r] = cadd(cscale(a, sn), cmul(ce, b));
        }
        ++rot;
    };
    // the pairs within each block once per sweep (in the sweep's first round every
    // block sits in exactly one workgroup): circle order on the JB columns of a
    // block, JB / 2 wavefronts per block
    if (round == 0) {
        const int base = (w / (JB / 2)) * JB, pw = w % (JB / 2);
        for (int ir = 0; ir < JB - 1; ++ir) {
            const int p = base + (pw == 0 ? ir : (ir + pw) % (JB - 1));
            const int q = base + (pw == 0 ? JB - 1 : (ir - pw + JB - 1) % (JB - 1));
            if (gcol(p) < m && gcol(q) < m) rotate(p, q);   // uniform within the wavefront
            __syncthreads();
        }
    }
    // the cross pairs of the two blocks: JB rounds, wavefront w pairs column w of
    // the first block with column (w + s) mod JB of the second
    for (int sft = 0; sft < JB; ++sft) {
        const int p = w, q = JB + (w + sft) % JB;
        if (gcol(p) < m && gcol(q) < m) rotate(p, q);
        __syncthreads();
    }
    jb_move<JB, false>(X, rows, rows, m, P, Q, xs);
    jb_move<JB, false>(V, m, m, m, P, Q, vs);
    if (lane == 0 && rot > 0) atomicAdd(counter, rot);
}

__global__ void colnorm_kernel(const double2* __restrict__ X, int rows, double* __restrict__ out) {
    __shared__ double sh[4 * (LR_BS / 64)];
    const double2* x = X + (int64_t)blockIdx.x * rows;
    double s[1] = {0.0};
    for (int r = threadIdx.x; r < rows; r += LR_BS) s[0] += x[r].x * x[r].x + x[r].y * x[r].y;
    block_sum_k<1>(s, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = sqrt(s[0]);
}

// position of column c in the descending order of sigma (ties by index)
__global__ void sort_rank_kernel(const double* __restrict__ sig, int m, int* __restrict__ pos) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    const double v = sig[c];
    int r = 0;
    for (int k = 0; k < m; ++k) {
        const double w = sig[k];
        r += (w > v || (w == v && k < c)) ? 1 : 0;
    }
    pos[c] = r;
}

// sorted outputs: U(:, pos c) = X(:, c) / sigma_c, V(:, pos c) = V(:, c), sigma sorted
__global__ void svd_gather_kernel(const double2* __restrict__ X, int rows, const double2* __restrict__ V, int m,
                                  const double* __restrict__ sig, const int* __restrict__ pos,
                                  double2* __restrict__ Uo, double2* __restrict__ Vo, double* __restrict__ so) {
    const int c = blockIdx.x;
    const int d = pos[c];
    const double sc = sig[c] > 0.0 ? 1.0 / sig[c] : 0.0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x)
        Uo[(int64_t)d * rows + r] = cscale(X[(int64_t)c * rows + r], sc);
    for (int r = threadIdx.x; r < m; r += blockDim.x) Vo[(int64_t)d * m + r] = V[(int64_t)c * m + r];
    if (threadIdx.x == 0) so[d] = sig[c];
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

int jacobi_svd(Ctx& c, double2* X, int m, double2* Uo, double2* Vo, double* sig, int max_sweeps) {
    FDS_REQUIRE(m >= 1, FDS_ERR_ARG, "empty Jacobi SVD");
    double2* V = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)m * m));
    double* sw = static_cast<double*>(c.dmalloc(sizeof(double) * (size_t)m));
    int* iw = static_cast<int*>(c.dmalloc(sizeof(int) * ((size_t)m + 1)));
    int* counter = iw + m;
    const int mpad = m + (m & 1);
    // blocks of 8 columns (16-column blocks, 5 workgroups of 16 wavefronts at 138
    // columns, took 4.1 ms against 3.0 ms: fewer workgroups, twice the rounds per launch)
    constexpr int jb = 8;
    const int nb = (m + jb - 1) / jb, nbp = std::max(2, nb + (nb & 1));   // blocks, padded to even
    const double tol = 2.0 * std::sqrt((double)m) * 2.220446049250313e-16;
    hipLaunchKernelGGL(eye_kernel, dim3(nblk((int64_t)m * m, 256)), dim3(256), 0, c.stream, V, (int64_t)m, m, m);
    FDS_HIP_TRY(hipGetLastError());
    int sweeps = 0;
    bool conv = m == 1;
    while (!conv && sweeps < max_sweeps) {
        {
            KScope _ks(c, "svd_jacobi");
            hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, c.stream, counter);
            if (m <= jb_maxrows<jb>()) {
                for (int rd = 0; rd < nbp - 1; ++rd)
                    hipLaunchKernelGGL(jacobi_block_kernel<jb>, dim3((unsigned)(nbp / 2)), dim3(64 * jb), 0, c.stream,
                                       X, m, V, m, nbp, rd, tol, counter);
            } else {
                for (int rd = 0; rd < mpad - 1; ++rd)
                    hipLaunchKernelGGL(jacobi_round_kernel, dim3((unsigned)(mpad / 2)), dim3(LR_BS), 0, c.stream, X,
                                       m, V, m, mpad, rd, tol, counter);
            }
        }
        FDS_HIP_TRY(hipGetLastError());
        int hc = 0;
        FDS_HIP_TRY(hipMemcpyAsync(&hc, counter, sizeof(int), hipMemcpyDeviceToHost, c.stream));
        FDS_HIP_TRY(hipStreamSynchronize(c.stream));
        ++sweeps;
        conv = hc == 0;
    }
    if (!conv) {
        c.dfree(V);
        c.dfree(sw);
        c.dfree(iw);
        throw Error{FDS_ERR_NOCONV, "Jacobi SVD did not converge"};
    }
    {
        KScope _ks(c, "svd_jacobi");
        hipLaunchKernelGGL(colnorm_kernel, dim3((unsigned)m), dim3(LR_BS), 0, c.stream, X, m, sw);
        hipLaunchKernelGGL(sort_rank_kernel, dim3(nblk(m, 256)), dim3(256), 0, c.stream, sw, m, iw);
        hipLaunchKernelGGL(svd_gather_kernel, dim3((unsigned)m), dim3(256), 0, c.stream, X, m, V, m, sw, iw, Uo, Vo,
                           sig);
    }
    FDS_HIP_TRY(hipGetLastError());
    c.dfree(V);
    c.dfree(sw);
    c.dfree(iw);
    return sweeps;
}

// ----------------------------------------------------------------- small elementwise helpers
__global__ void conj_kernel(const double2* __restrict__ x, double2* __restrict__ y, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = cconj(x[t]);
}

__global__ void scale_cols_kernel(double2* __restrict__ X, int64_t rows, int cols, const double* __restrict__ s) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * cols) return;
    X[t] = cscale(X[t], s[t / rows]);
}

void conj_copy(Ctx& c, const double2* x, double2* y, int64_t n) {
    {
        KScope _ks(c, "elementwise");
        hipLaunchKernelGGL(conj_kernel, dim3(nblk(n, 256)), dim3(256), 0, c.stream, x, y, n);
    }
    FDS_HIP_TRY(hipGetLastError());
}

void scale_cols(Ctx& c, double2* X, int64_t rows, int cols, const double* s) {
    {
        KScope _ks(c, "elementwise");
        hipLaunchKernelGGL(scale_cols_kernel, dim3(nblk(rows * cols, 256)), dim3(256), 0, c.stream, X, rows, cols, s);
    }
    FDS_HIP_TRY(hipGetLastError());
}

}  // namespace fds
