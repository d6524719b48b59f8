// Dense and sparse linear algebra on the device:
//   * complex (and real) GEMM on FP64 MFMA (v_mfma_f64_16x16x4f64) and complex64
//     GEMM on FP32 MFMA (v_mfma_f32_16x16x4f32, FP32 accumulation), column-major,
//     op(A), op(B) in {N, T, C}, optional split-K with a deterministic reduction;
//   * the periodic tridiagonal Gram matrix G: factorisation (cyclic Thomas with
//     a Sherman-Morrison correction), block solves G^{-1} X, block products G X;
//   * Chebyshev-series application of G^{+-1/2} (Clenshaw recurrence);
//   * small dense factorisations in one workgroup: Cholesky (real), LU with
//     partial pivoting (complex), block triangular solves.
#include <cmath>
#include <cstdio>
#include <type_traits>
#include <typeinfo>
#include <vector>

#include "fds_internal.h"
#include "linalg.h"

namespace fds {

typedef double d4 __attribute__((ext_vector_type(4)));

// ============================================================ GEMM
// 64 x 64 output tile per workgroup of 4 wavefronts (2 x 2 of 32 x 32), K staged
// through LDS 16 at a time; each wavefront holds 2 x 2 MFMA 16 x 16 accumulators
// (real and imaginary parts separately: 4 real MFMAs per complex product).
constexpr int GB_M = 64, GB_N = 64, GB_K = 16, G_PAD = 2;

typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct GT;
template <>
struct GT<double> {
    typedef double R;
    typedef d4 Acc;
    static constexpr bool CPLX = false;
};
template <>
struct GT<double2> {
    typedef double R;
    typedef d4 Acc;
    static constexpr bool CPLX = true;
};
template <>
struct GT<float2> {
    typedef float R;
    typedef f4 Acc;
    static constexpr bool CPLX = true;
};

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// Row of accumulator register v of a lane within the 16 x 16 tile (column = lane & 15):
// v_mfma_f64_16x16x4f64 places D[i][j] in lane j + 16 (i % 4), register i / 4;
// v_mfma_f32_16x16x4f32 places it in lane j + 16 (i / 4), register i % 4.
__device__ __forceinline__ int acc_row(double, int lane, int v) { return (lane >> 4) + 4 * v; }
__device__ __forceinline__ int acc_row(float, int lane, int v) { return 4 * (lane >> 4) + v; }

__device__ __forceinline__ double2 ld_op(const double2* p, int op) {
    double2 v = *p;
    if (op == OP_C) v.y = -v.y;
    return v;
}
__device__ __forceinline__ float2 ld_op(const float2* p, int op) {
    float2 v = *p;
    if (op == OP_C) v.y = -v.y;
    return v;
}
__device__ __forceinline__ double ld_op(const double* p, int) { return *p; }
// complex64 operand widened to complex128 on load (FP64 arithmetic on FP32-stored matrices)
__device__ __forceinline__ void ld_into(const float2* p, int op, double2& v) {
    const float2 f = *p;
    v = make_double2(f.x, op == OP_C ? -f.y : f.y);
}
template <typename T>
__device__ __forceinline__ void ld_into(const T* p, int op, T& v) { v = ld_op(p, op); }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ bool nonzero(double2 b) { return b.x != 0.0 || b.y != 0.0; }
__device__ __forceinline__ bool nonzero(float2 b) { return b.x != 0.0f || b.y != 0.0f; }
__device__ __forceinline__ bool nonzero(double b) { return b != 0.0; }
__device__ __forceinline__ double cmul(double a, double b) { return a * b; }
__device__ __forceinline__ double cadd(double a, double b) { return a + b; }

// Grouped GEMM problem descriptor (complex128, op N x N).
struct GemmProblem {
    int m, n, k;
    double2 alpha, beta;
    const double2* A;
    int64_t lda;
    const double2* B;
    int64_t ldb;
    double2* C;
    int64_t ldc;
    int64_t tile_begin;
};

// One 64 x 64 output tile (bx, by) and K-range bz of C = alpha op(A) op(B) + beta C.
template <typename T, typename TA, int OPA, int OPB>
__device__ __forceinline__ void gemm_tile(int m, int n, int k, T alpha, const TA* __restrict__ A, int64_t lda,
                                          const T* __restrict__ B, int64_t ldb, T beta, T* __restrict__ C,
                                          int64_t ldc, int kchunk, T* __restrict__ part, int bx, int by, int bz,
                                          T (&sA)[GB_K][GB_M + G_PAD], T (&sB)[GB_K][GB_N + G_PAD]) {
    typedef typename GT<T>::R RT;
    typedef typename GT<T>::Acc Acc;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int row0 = bx * GB_M, col0 = by * GB_N;
    const int kbeg = bz * kchunk;
    const int kend = min(k, kbeg + kchunk);

    Acc accR[2][2], accI[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            accR[a][b] = Acc{0, 0, 0, 0};
            accI[a][b] = Acc{0, 0, 0, 0};
        }

    for (int kk = kbeg; kk < kend; kk += GB_K) {
        // ---- stage A tile: op(A)[row0 + i][kk + p], i < 64, p < 16
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int i, p;
            if (OPA == OP_N) {
                i = tid & 63;
                p = (tid >> 6) + 4 * e;
            } else {
                p = tid & 15;
                i = (tid >> 4) + 16 * e;
            }
            const int gi = row0 + i, gp = kk + p;
            T v{};
            if (gi < m && gp < kend) {
                const TA* src = (OPA == OP_N) ? A + gi + (int64_t)gp * lda : A + gp + (int64_t)gi * lda;
                ld_into(src, OPA, v);
            }
            sA[p][i] = v;
        }
        // ---- stage B tile: op(B)[kk + p][col0 + j], p < 16, j < 64
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int j, p;
            if (OPB == OP_N) {
                p = tid & 15;
                j = (tid >> 4) + 16 * e;
            } else {
                j = tid & 63;
                p = (tid >> 6) + 4 * e;
            }
            const int gj = col0 + j, gp = kk + p;
            T v{};
            if (gj < n && gp < kend) {
                const T* src = (OPB == OP_N) ? B + gp + (int64_t)gj * ldb : B + gj + (int64_t)gp * ldb;
                v = ld_op(src, OPB);
            }
            sB[p][j] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kc = 0; kc < GB_K / 4; ++kc) {
            const int pr = kc * 4 + (lane >> 4);
            T a[2], b[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) a[r] = sA[pr][wm * 32 + r * 16 + (lane & 15)];
#pragma unroll
            for (int c = 0; c < 2; ++c) b[c] = sB[pr][wn * 32 + c * 16 + (lane & 15)];
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    if constexpr (GT<T>::CPLX) {
                        accR[r][c] = mfma16(a[r].x, b[c].x, accR[r][c]);
                        accR[r][c] = mfma16(-a[r].y, b[c].y, accR[r][c]);
                        accI[r][c] = mfma16(a[r].x, b[c].y, accI[r][c]);
                        accI[r][c] = mfma16(a[r].y, b[c].x, accI[r][c]);
                    } else {
                        accR[r][c] = mfma16(a[r], b[c], accR[r][c]);
                    }
                }
        }
        __syncthreads();
    }
    // ---- epilogue
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = row0 + wm * 32 + r * 16 + acc_row(RT{}, lane, v);
                const int gj = col0 + wn * 32 + c * 16 + (lane & 15);
                if (gi >= m || gj >= n) continue;
                T acc;
                if constexpr (GT<T>::CPLX) {
                    acc.x = accR[r][c][v];
                    acc.y = accI[r][c][v];
                } else {
                    acc = accR[r][c][v];
                }
                if (part) {
                    part[(int64_t)bz * m * n + gi + (int64_t)gj * m] = acc;
                } else {
                    T o = cmul(alpha, acc);
                    if (nonzero(beta)) o = cadd(o, cmul(beta, C[gi + (int64_t)gj * ldc]));
                    C[gi + (int64_t)gj * ldc] = o;
                }
            }
}

template <typename T, typename TA, int OPA, int OPB>
__global__ __launch_bounds__(256) void gemm_kernel(int m, int n, int k, T alpha, const TA* __restrict__ A,
                                                   int64_t lda, const T* __restrict__ B, int64_t ldb, T beta,
                                                   T* __restrict__ C, int64_t ldc, int kchunk,
                                                   T* __restrict__ part) {
    __shared__ T sA[GB_K][GB_M + G_PAD];
    __shared__ T sB[GB_K][GB_N + G_PAD];
    gemm_tile<T, TA, OPA, OPB>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, blockIdx.x, blockIdx.y,
                               blockIdx.z, sA, sB);
}

// Large problems: 128 x 64 output tile per workgroup (4 wavefronts of 64 x 32,
// 4 x 2 MFMA tiles each), the next K slice loaded into registers while the
// matrix cores work on the current one (complex128 output; A may be complex64,
// widened on load).
constexpr int BB_M = 128, BB_N = 64, BB_K = 16, BB_PAD = 2;

template <typename TA, int OPA, int OPB>
__global__ __launch_bounds__(256) void gemm_big_kernel(int m, int n, int k, double2 alpha,
                                                       const TA* __restrict__ A, int64_t lda,
                                                       const double2* __restrict__ B, int64_t ldb, double2 beta,
                                                       double2* __restrict__ C, int64_t ldc, int kchunk,
                                                       double2* __restrict__ part) {
    __shared__ double2 sA[BB_K][BB_M + BB_PAD];
    __shared__ double2 sB[BB_K][BB_N + BB_PAD];
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int row0 = blockIdx.x * BB_M, col0 = blockIdx.y * BB_N;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(k, kbeg + kchunk);
    d4 accR[4][2], accI[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            accR[a][b] = d4{0.0, 0.0, 0.0, 0.0};
            accI[a][b] = d4{0.0, 0.0, 0.0, 0.0};
        }
    double2 ra[8], rb[4];
    auto loadAB = [&](int kk) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            int i, p;
            if (OPA == OP_N) {
                i = tid & 127;
                p = (tid >> 7) + 2 * e;
            } else {
                p = tid & 15;
                i = (tid >> 4) + 16 * e;
            }
            const int gi = row0 + i, gp = kk + p;
            double2 v = make_double2(0.0, 0.0);
            if (gi < m && gp < kend) {
                const TA* src = (OPA == OP_N) ? A + gi + (int64_t)gp * lda : A + gp + (int64_t)gi * lda;
                ld_into(src, OPA, v);
            }
            ra[e] = v;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int j, p;
            if (OPB == OP_N) {
                p = tid & 15;
                j = (tid >> 4) + 16 * e;
            } else {
                j = tid & 63;
                p = (tid >> 6) + 4 * e;
            }
            const int gj = col0 + j, gp = kk + p;
            double2 v = make_double2(0.0, 0.0);
            if (gj < n && gp < kend) {
                const double2* src = (OPB == OP_N) ? B + gp + (int64_t)gj * ldb : B + gj + (int64_t)gp * ldb;
                v = ld_op(src, OPB);
            }
            rb[e] = v;
        }
    };
    if (kbeg < kend) loadAB(kbeg);
    for (int kk = kbeg; kk < kend; kk += BB_K) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if (OPA == OP_N) sA[(tid >> 7) + 2 * e][tid & 127] = ra[e];
            else sA[tid & 15][(tid >> 4) + 16 * e] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (OPB == OP_N) sB[tid & 15][(tid >> 4) + 16 * e] = rb[e];
            else sB[(tid >> 6) + 4 * e][tid & 63] = rb[e];
        }
        __syncthreads();
        if (kk + BB_K < kend) loadAB(kk + BB_K);
#pragma unroll
        for (int kc = 0; kc < BB_K / 4; ++kc) {
            const int pr = kc * 4 + (lane >> 4);
            double2 a[4], b[2];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = sA[pr][wm * 64 + r * 16 + (lane & 15)];
#pragma unroll
            for (int c = 0; c < 2; ++c) b[c] = sB[pr][wn * 32 + c * 16 + (lane & 15)];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    accR[r][c] = mfma16(a[r].x, b[c].x, accR[r][c]);
                    accR[r][c] = mfma16(-a[r].y, b[c].y, accR[r][c]);
                    accI[r][c] = mfma16(a[r].x, b[c].y, accI[r][c]);
                    accI[r][c] = mfma16(a[r].y, b[c].x, accI[r][c]);
                }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = row0 + wm * 64 + r * 16 + acc_row(0.0, lane, v);
                const int gj = col0 + wn * 32 + c * 16 + (lane & 15);
                if (gi >= m || gj >= n) continue;
                const double2 acc = make_double2(accR[r][c][v], accI[r][c][v]);
                if (part) {
                    part[(int64_t)blockIdx.z * m * n + gi + (int64_t)gj * m] = acc;
                } else {
                    double2 o = cmul(alpha, acc);
                    if (beta.x != 0.0 || beta.y != 0.0) o = cadd(o, cmul(beta, C[gi + (int64_t)gj * ldc]));
                    C[gi + (int64_t)gj * ldc] = o;
                }
            }
}

// Grouped GEMM: problems of uneven sizes in one launch; workgroup b takes tile
// b - tile_begin[g] of the problem g with tile_begin[g] <= b < tile_begin[g + 1].
__global__ __launch_bounds__(256) void gemm_grouped_kernel_nn(const GemmProblem* __restrict__ probs, int count) {
    __shared__ double2 sA[GB_K][GB_M + G_PAD];
    __shared__ double2 sB[GB_K][GB_N + G_PAD];
    const int64_t b = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (probs[mid].tile_begin <= b) lo = mid;
        else hi = mid - 1;
    }
    const GemmProblem& P = probs[lo];
    const int64_t t = b - P.tile_begin;
    const int gm = (P.m + GB_M - 1) / GB_M;
    const int bx = (int)(t % gm), by = (int)(t / gm);
    gemm_tile<double2, double2, OP_N, OP_N>(P.m, P.n, P.k, P.alpha, P.A, P.lda, P.B, P.ldb, P.beta, P.C, P.ldc,
                                            P.k + GB_K, nullptr, bx, by, 0, sA, sB);
}

template <typename T>
__global__ void splitk_reduce_kernel(int m, int n, int nz, T alpha, const T* __restrict__ part, T beta,
                                     T* __restrict__ C, int64_t ldc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * n) return;
    const int i = (int)(t % m);
    const int64_t j = t / m;
    T s{};
    for (int z = 0; z < nz; ++z) s = cadd(s, part[(int64_t)z * m * n + t]);
    T o = cmul(alpha, s);
    if (nonzero(beta)) o = cadd(o, cmul(beta, C[i + j * ldc]));
    C[i + j * ldc] = o;
}

template <typename T, typename TA, int OPA, int OPB>
static void gemm_launch(Ctx& c, int m, int n, int k, T alpha, const TA* A, int64_t lda, const T* B, int64_t ldb,
                        T beta, T* C, int64_t ldc, int nz);

static int bucket(int v) {   // shape classes: powers of two
    int b = 1;
    while (b < v) b <<= 1;
    return b;
}

// Split-K factor: a heuristic (split when the output tiles cannot fill the chip),
// or, with autotuning on, the fastest of the candidates timed once per shape
// class (operand types, ops, m, n, k rounded up to powers of two) on a scratch
// output, and cached in the context. Never tunes while the stream is captured.
template <typename T, typename TA>
static constexpr bool big_ok() {
    return std::is_same<T, double2>::value;
}

// Kernel configuration: split-K factor (bits 0..7) and the 128 x 128 tile (bit 8).
// Heuristic: large tiles when both dimensions reach 128 (complex128 output), and
// split K when the output tiles alone cannot fill the chip; or, with autotuning
// on, the fastest candidate timed once per shape class (operand types, ops, m, n,
// k rounded up to powers of two) on a scratch output, cached in the context.
// Never tunes while the stream is being captured.
template <typename T, typename TA, int OPA, int OPB>
static int choose_config(Ctx& c, int m, int n, int k, const TA* A, int64_t lda, const T* B, int64_t ldb) {
    auto split_for = [&](int tiles) {
        int nz = 1;
        if (tiles < 512 && k > 4 * GB_K) nz = std::max(1, std::min((512 + tiles - 1) / tiles, (k + 255) / 256));
        return std::min(nz, 64);
    };
    const bool bigp = big_ok<T, TA>() && m >= BB_M && n >= BB_N;
    int cfg;
    if (bigp) {
        const int tb = ((m + BB_M - 1) / BB_M) * ((n + BB_N - 1) / BB_N);
        cfg = 256 | split_for(4 * tb);
    } else {
        cfg = split_for(((m + GB_M - 1) / GB_M) * ((n + GB_N - 1) / GB_N));
    }
    if (!c.autotune) return cfg;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(c.stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return cfg;
    char key[160];
    snprintf(key, sizeof(key), "%s/%s/%d%d/%d/%d/%d", typeid(T).name(), typeid(TA).name(), OPA, OPB, bucket(m),
             bucket(n), bucket(k));
    auto it = c.tuned.find(key);
    if (it != c.tuned.end()) return it->second;
    std::vector<int> cand;
    for (int big = 0; big <= (bigp ? 1 : 0); ++big) {
        const int tiles = big ? ((m + BB_M - 1) / BB_M) * ((n + BB_N - 1) / BB_N)
                              : ((m + GB_M - 1) / GB_M) * ((n + GB_N - 1) / GB_N);
        for (int z = 1; z <= 64; z *= 2) {
            if (z > 1 && ((int64_t)z * 2 * GB_K > k || (int64_t)z * m * n * sizeof(T) > ((int64_t)1 << 29) ||
                          (int64_t)tiles * z > 8192))
                continue;
            cand.push_back((big ? 256 : 0) | z);
        }
    }
    T* scratch = static_cast<T*>(c.dmalloc(sizeof(T) * (size_t)m * n));
    hipEvent_t e0, e1;
    FDS_HIP_TRY(hipEventCreate(&e0));
    FDS_HIP_TRY(hipEventCreate(&e1));
    const bool prof = c.prof;
    c.prof = false;
    float best = 1e30f;
    int bc = cfg;
    T one{}, zero{};
    if constexpr (GT<T>::CPLX) one.x = 1; else one = 1;
    for (int z : cand) {
        gemm_launch<T, TA, OPA, OPB>(c, m, n, k, one, A, lda, B, ldb, zero, scratch, m, z);   // warm
        FDS_HIP_TRY(hipEventRecord(e0, c.stream));
        for (int rep = 0; rep < 3; ++rep)
            gemm_launch<T, TA, OPA, OPB>(c, m, n, k, one, A, lda, B, ldb, zero, scratch, m, z);
        FDS_HIP_TRY(hipEventRecord(e1, c.stream));
        FDS_HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.0f;
        FDS_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
            best = ms;
            bc = z;
        }
    }
    c.prof = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c.dfree(scratch);
    c.tuned[key] = bc;
    return bc;
}

template <typename T, typename TA, int OPA, int OPB>
static void gemm_dispatch(Ctx& c, int m, int n, int k, T alpha, const TA* A, int64_t lda, const T* B, int64_t ldb,
                          T beta, T* C, int64_t ldc) {
    const int cfg = choose_config<T, TA, OPA, OPB>(c, m, n, k, A, lda, B, ldb);
    gemm_launch<T, TA, OPA, OPB>(c, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, cfg);
}

template <typename T, typename TA, int OPA, int OPB>
static void gemm_launch(Ctx& c, int m, int n, int k, T alpha, const TA* A, int64_t lda, const T* B, int64_t ldb,
                        T beta, T* C, int64_t ldc, int cfg) {
    const bool big = big_ok<T, TA>() && (cfg & 256);
    const int bm = big ? BB_M : GB_M, bn = big ? BB_N : GB_N;
    const int gm = (m + bm - 1) / bm, gn = (n + bn - 1) / bn;
    int nz = std::max(1, cfg & 255);
    int kchunk = (k + nz - 1) / nz;
    kchunk = (kchunk + GB_K - 1) / GB_K * GB_K;
    nz = (k + kchunk - 1) / kchunk;
    T* part = nullptr;
    if (nz > 1) part = static_cast<T*>(c.dmalloc(sizeof(T) * (size_t)nz * m * n));
    {
        KScope _ks(c, std::is_same<T, float2>::value ? "gemm_c64" : "gemm");
        if constexpr (big_ok<T, TA>()) {
            if (big) {
                hipLaunchKernelGGL((gemm_big_kernel<TA, OPA, OPB>), dim3(gm, gn, nz), dim3(256), 0, c.stream, m, n, k,
                                   alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part);
            } else {
                hipLaunchKernelGGL((gemm_kernel<T, TA, OPA, OPB>), dim3(gm, gn, nz), dim3(256), 0, c.stream, m, n, k,
                                   alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part);
            }
        } else {
            hipLaunchKernelGGL((gemm_kernel<T, TA, OPA, OPB>), dim3(gm, gn, nz), dim3(256), 0, c.stream, m, n, k,
                               alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part);
        }
    }
    FDS_HIP_TRY(hipGetLastError());
    if (part) {
        const int64_t tot = (int64_t)m * n;
        {
            KScope _ks(c, "gemm_splitk_reduce");
            hipLaunchKernelGGL(splitk_reduce_kernel<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c.stream,
                               m, n, nz, alpha, part, beta, C, ldc);
        }
        FDS_HIP_TRY(hipGetLastError());
        c.dfree(part);
    }
}

template <typename T, typename TA = T>
static void gemm_any(Ctx& c, int opa, int opb, int m, int n, int k, T alpha, const TA* A, int64_t lda, const T* B,
                     int64_t ldb, T beta, T* C, int64_t ldc) {
    if (m <= 0 || n <= 0) return;
#define FDS_G(a, b)                                                                    \
    if (opa == a && opb == b) {                                                        \
        gemm_dispatch<T, TA, a, b>(c, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);   \
        return;                                                                        \
    }
    FDS_G(OP_N, OP_N) FDS_G(OP_N, OP_T) FDS_G(OP_N, OP_C)
    FDS_G(OP_T, OP_N) FDS_G(OP_T, OP_T) FDS_G(OP_T, OP_C)
    FDS_G(OP_C, OP_N) FDS_G(OP_C, OP_T) FDS_G(OP_C, OP_C)
#undef FDS_G
    throw Error{FDS_ERR_ARG, "bad GEMM op"};
}

void zgemm(Ctx& c, int opa, int opb, int m, int n, int k, double2 alpha, const double2* A, int64_t lda,
           const double2* B, int64_t ldb, double2 beta, double2* C, int64_t ldc) {
    gemm_any<double2>(c, opa, opb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

void zgemm_a32(Ctx& c, int opa, int opb, int m, int n, int k, double2 alpha, const float2* A, int64_t lda,
               const double2* B, int64_t ldb, double2 beta, double2* C, int64_t ldc) {
    gemm_any<double2, float2>(c, opa, opb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

int autotune_entries(Ctx& c, int cap, char* keys, int* values) {
    int i = 0;
    for (const auto& kv : c.tuned) {
        if (i < cap) {
            if (keys) snprintf(keys + 160 * i, 160, "%s", kv.first.c_str());
            if (values) values[i] = kv.second;
        }
        ++i;
    }
    return i;
}

void zgemm_grouped_nn(Ctx& c, const std::vector<GemmSpec>& specs) {
    std::vector<GemmProblem> probs;
    int64_t tiles = 0;
    for (const auto& g : specs) {
        if (g.m <= 0 || g.n <= 0) continue;
        GemmProblem P;
        P.m = g.m; P.n = g.n; P.k = g.k;
        P.alpha = g.alpha; P.beta = g.beta;
        P.A = g.A; P.lda = g.lda; P.B = g.B; P.ldb = g.ldb; P.C = g.C; P.ldc = g.ldc;
        P.tile_begin = tiles;
        tiles += (int64_t)((g.m + GB_M - 1) / GB_M) * ((g.n + GB_N - 1) / GB_N);
        probs.push_back(P);
    }
    if (probs.empty()) return;
    FDS_REQUIRE(tiles < (int64_t)1 << 31, FDS_ERR_ARG, "grouped GEMM too large");
    GemmProblem* d = static_cast<GemmProblem*>(c.dmalloc(sizeof(GemmProblem) * probs.size()));
    FDS_HIP_TRY(hipMemcpyAsync(d, probs.data(), sizeof(GemmProblem) * probs.size(), hipMemcpyHostToDevice, c.stream));
    FDS_HIP_TRY(hipStreamSynchronize(c.stream));   // the host table goes out of scope below
    {
        KScope _ks(c, "gemm_grouped");
        hipLaunchKernelGGL(gemm_grouped_kernel_nn, dim3((unsigned)tiles), dim3(256), 0, c.stream, d, (int)probs.size());
    }
    FDS_HIP_TRY(hipGetLastError());
    c.dfree(d);
}

void cgemm(Ctx& c, int opa, int opb, int m, int n, int k, float2 alpha, const float2* A, int64_t lda,
           const float2* B, int64_t ldb, float2 beta, float2* C, int64_t ldc) {
    gemm_any<float2>(c, opa, opb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

void dgemm(Ctx& c, int opa, int opb, int m, int n, int k, double alpha, const double* A, int64_t lda,
           const double* B, int64_t ldb, double beta, double* C, int64_t ldc) {
    if (opa == OP_C) opa = OP_T;
    if (opb == OP_C) opb = OP_T;
    gemm_any<double>(c, opa, opb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

// ============================================================ periodic tridiagonal G
// G = T + u v^T with u = (g, 0..0, e_{n-1}), v = (1, 0..0, e_{n-1}/g), g = -d_0, so
// that T is tridiagonal (corners removed, T_00 = d_0 - g, T_{n-1,n-1} = d_{n-1} - e_{n-1}^2/g).
// Layout of fac: [0,n) 1/den_i, [n,2n) cp_i, [2n,3n) z = T^{-1} u, [3n] vcoef, [3n+1] 1/(1+v.z).
__global__ void gram_factor_kernel(const double* __restrict__ d, const double* __restrict__ e, int n,
                                   double* __restrict__ fac) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double* inv = fac;
    double* cp = fac + n;
    double* z = fac + 2 * n;
    const double g = -d[0];
    const double en = e[n - 1];
    double den = d[0] - g;
    inv[0] = 1.0 / den;
    cp[0] = e[0] * inv[0];
    for (int i = 1; i < n; ++i) {
        double di = d[i];
        if (i == n - 1) di -= en * en / g;
        den = di - e[i - 1] * cp[i - 1];
        inv[i] = 1.0 / den;
        cp[i] = (i < n - 1) ? e[i] * inv[i] : 0.0;
    }
    // z = T^{-1} u, u = (g, 0, ..., 0, en)
    double y = g * inv[0];
    z[0] = y;
    for (int i = 1; i < n; ++i) {
        const double ui = (i == n - 1) ? en : 0.0;
        y = (ui - e[i - 1] * y) * inv[i];
        z[i] = y;
    }
    for (int i = n - 2; i >= 0; --i) z[i] -= cp[i] * z[i + 1];
    const double vcoef = en / g;
    fac[3 * n] = vcoef;
    fac[3 * n + 1] = 1.0 / (1.0 + z[0] + vcoef * z[n - 1]);
}

// X[c][0..n) <- G^{-1} X[c] for each vector c (thread per vector).
template <typename T>
__global__ void gram_solve_kernel(const double* __restrict__ e, const double* __restrict__ fac, int n,
                                  T* __restrict__ X, int64_t ncols, int64_t ld) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    T* x = X + c * ld;
    const double* inv = fac;
    const double* cp = fac + n;
    const double* z = fac + 2 * n;
    const double vcoef = fac[3 * n], f = fac[3 * n + 1];
    T y = x[0] * inv[0];
    x[0] = y;
    for (int i = 1; i < n; ++i) {
        y = (x[i] - y * e[i - 1]) * inv[i];
        x[i] = y;
    }
    for (int i = n - 2; i >= 0; --i) {
        y = x[i] - y * cp[i];
        x[i] = y;
    }
    const T s = (x[0] + x[n - 1] * vcoef) * f;
    for (int i = 0; i < n; ++i) x[i] = x[i] - s * z[i];
}

// Y = a G X + b X (element-parallel; Y may not alias X).
template <typename T>
__global__ void gram_mul_kernel(const double* __restrict__ d, const double* __restrict__ e, int n,
                                const T* __restrict__ X, int64_t ncols, int64_t ldx, double a, double b,
                                T* __restrict__ Y, int64_t ldy) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * ncols) return;
    const int i = (int)(t % n);
    const int64_t c = t / n;
    const T* x = X + c * ldx;
    const int im = i == 0 ? n - 1 : i - 1, ip = i + 1 == n ? 0 : i + 1;
    const T gx = x[i] * d[i] + x[im] * e[im] + x[ip] * e[i];
    Y[c * ldy + i] = gx * a + x[i] * b;
}

void gram_factor(Ctx& c, const double* d, const double* e, int n, double* fac) {
    {
        KScope _ks(c, "gram_factor");
        hipLaunchKernelGGL(gram_factor_kernel, dim3(1), dim3(64), 0, c.stream, d, e, n, fac);
    }
    FDS_HIP_TRY(hipGetLastError());
}

template <typename T>
void gram_solve(Ctx& c, const double* e, const double* fac, int n, T* X, int64_t ncols, int64_t ld) {
    if (ncols <= 0) return;
    {
        KScope _ks(c, "gram_solve");
        hipLaunchKernelGGL(gram_solve_kernel<T>, dim3((unsigned)((ncols + 63) / 64)), dim3(64), 0, c.stream, e, fac,
                       n, X, ncols, ld);
    }
    FDS_HIP_TRY(hipGetLastError());
}
template void gram_solve<double>(Ctx&, const double*, const double*, int, double*, int64_t, int64_t);
template void gram_solve<double2>(Ctx&, const double*, const double*, int, double2*, int64_t, int64_t);

template <typename T>
void gram_mul(Ctx& c, const double* d, const double* e, int n, const T* X, int64_t ncols, int64_t ldx,
              double a, double b, T* Y, int64_t ldy) {
    const int64_t tot = (int64_t)n * ncols;
    if (tot <= 0) return;
    {
        KScope _ks(c, "gram_mul");
        hipLaunchKernelGGL(gram_mul_kernel<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c.stream, d, e, n,
                       X, ncols, ldx, a, b, Y, ldy);
    }
    FDS_HIP_TRY(hipGetLastError());
}
template void gram_mul<double>(Ctx&, const double*, const double*, int, const double*, int64_t, int64_t, double,
                               double, double*, int64_t);
template void gram_mul<double2>(Ctx&, const double*, const double*, int, const double2*, int64_t, int64_t,
                                double, double, double2*, int64_t);

// ------------------------------------------------------------ banded G^{-1}
// G is strongly diagonally dominant: each row satisfies |e_{i-1}| + |e_i| =
// d_i / 2, and the elimination multipliers e_i / (d_i - e_{i-1} c_{i-1}) stay
// below 1/2 for any panel lengths. Entries of G^{-1} therefore decay at least
// like 2^{-|i-j|} away from the (periodic) diagonal, and G^{-1} restricted to
// the band |i - j| <= GW (GW = 64) equals G^{-1} to a relative 2^{-64}.
// Row i of the band is computed by a Thomas solve of G x = e_i on the window
// i-GW .. i+GW (periodic indices, couplings outside the window dropped), whose
// truncation error is of the same order. band layout: [t][i], t = k + GW.
__global__ void gram_band_kernel(const double* __restrict__ d, const double* __restrict__ e, int n,
                                 double* __restrict__ band, double* __restrict__ scr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int M = 2 * GW + 1;
    double* cp = scr;                 // [M][n]
    double* z = scr + (int64_t)M * n; // [M][n]
    double cprev = 0.0, zprev = 0.0;
    for (int t = 0; t < M; ++t) {
        int j = i + t - GW;
        j = j < 0 ? j + n : (j >= n ? j - n : j);
        const int jm = j == 0 ? n - 1 : j - 1;
        const double lower = t > 0 ? e[jm] : 0.0;
        const double den = d[j] - lower * cprev;
        const double upper = t < M - 1 ? e[j] : 0.0;
        const double cpt = upper / den;
        const double rhs = t == GW ? 1.0 : 0.0;
        const double zt = (rhs - lower * zprev) / den;
        cp[(int64_t)t * n + i] = cpt;
        z[(int64_t)t * n + i] = zt;
        cprev = cpt;
        zprev = zt;
    }
    double x = 0.0;
    for (int t = M - 1; t >= 0; --t) {
        x = z[(int64_t)t * n + i] - cp[(int64_t)t * n + i] * x;
        band[(int64_t)t * n + i] = x;
    }
}

// Y = G^{-1} X (out of place) with the band: workgroup = 256 rows of one vector.
template <typename T>
__global__ __launch_bounds__(256) void gram_band_apply_kernel(const double* __restrict__ band, int n,
                                                              const T* __restrict__ X, T* __restrict__ Y) {
    __shared__ T xs[256 + 2 * GW];
    const int64_t col = blockIdx.y;
    const int r0 = blockIdx.x * 256;
    const T* x = X + col * n;
    for (int t = threadIdx.x; t < 256 + 2 * GW; t += 256) {
        int j = r0 - GW + t;
        j = ((j % n) + n) % n;
        xs[t] = x[j];
    }
    __syncthreads();
    const int i = r0 + threadIdx.x;
    if (i >= n) return;
    T acc{};
#pragma unroll 8
    for (int t = 0; t < 2 * GW + 1; ++t) acc = acc + xs[threadIdx.x + t] * band[(int64_t)t * n + i];
    Y[col * n + i] = acc;
}

void gram_band_build(Ctx& c, const double* d, const double* e, int n, double* band) {
    double* scr = static_cast<double*>(c.dmalloc(sizeof(double) * 2 * (2 * GW + 1) * (size_t)n));
    {
        KScope _ks(c, "gram_band_build");
        hipLaunchKernelGGL(gram_band_kernel, dim3((n + 127) / 128), dim3(128), 0, c.stream, d, e, n, band, scr);
    }
    FDS_HIP_TRY(hipGetLastError());
    c.dfree(scr);
}

template <typename T>
void gram_band_apply(Ctx& c, const double* band, int n, const T* X, int64_t ncols, T* Y) {
    if (ncols <= 0) return;
    {
        KScope _ks(c, "gram_inv");
        hipLaunchKernelGGL(gram_band_apply_kernel<T>, dim3((n + 255) / 256, (unsigned)ncols), dim3(256), 0,
                           c.stream, band, n, X, Y);
    }
    FDS_HIP_TRY(hipGetLastError());
}
template void gram_band_apply<double>(Ctx&, const double*, int, const double*, int64_t, double*);
template void gram_band_apply<double2>(Ctx&, const double*, int, const double2*, int64_t, double2*);

// ============================================================ Chebyshev G^{p/2}
// f(x) = x^{p/2} on [lo, hi] expanded in Chebyshev polynomials of
// t = (2x - lo - hi)/(hi - lo); coefficients by interpolation at Chebyshev points.
std::vector<double> cheb_coeffs(int p, double lo, double hi) {
    const int M = 400;
    std::vector<double> fv(M), a(M);
    for (int j = 0; j < M; ++j) {
        const double t = std::cos(kPiHost * (j + 0.5) / M);
        const double x = 0.5 * (hi + lo) + 0.5 * (hi - lo) * t;
        fv[j] = std::pow(x, 0.5 * p);
    }
    for (int i = 0; i < M; ++i) {
        double s = 0.0;
        for (int j = 0; j < M; ++j) s += fv[j] * std::cos(kPiHost * i * (j + 0.5) / M);
        a[i] = s * 2.0 / M;
    }
    a[0] *= 0.5;
    int deg = M - 1;
    const double a0 = std::fabs(a[0]);
    while (deg > 1 && std::fabs(a[deg]) < 1e-18 * a0 && std::fabs(a[deg - 1]) < 1e-18 * a0) --deg;
    a.resize(deg + 1);
    return a;
}

// One Clenshaw step for all vectors:
//   bj = a_j X + 2 That(b1) - b2,  That(v) = (2 G v - (lo+hi) v)/(hi-lo)
// final (last=1): Y = a_0 X + That(b1) - b2
template <typename T>
__global__ void clenshaw_kernel(const double* __restrict__ d, const double* __restrict__ e, int n,
                                const T* __restrict__ X, const T* __restrict__ b1, const T* __restrict__ b2,
                                T* __restrict__ out, int64_t ncols, double aj, double s1, double s0,
                                double tw) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * ncols) return;
    const int i = (int)(t % n);
    const int64_t c = t / n;
    const int64_t o = c * n;
    const int im = i == 0 ? n - 1 : i - 1, ip = i + 1 == n ? 0 : i + 1;
    const T gb = b1[o + i] * d[i] + b1[o + im] * e[im] + b1[o + ip] * e[i];
    // That(b1) = s1 * G b1 + s0 * b1
    const T th = gb * s1 + b1[o + i] * s0;
    out[o + i] = X[o + i] * aj + th * tw - b2[o + i];
}

template <typename T>
void gram_pow_half(Ctx& c, const double* d, const double* e, int n, double lo, double hi, int p,
                   T* X, int64_t ncols) {
    if (ncols <= 0) return;
    const std::vector<double> a = cheb_coeffs(p, lo, hi);
    const int deg = (int)a.size() - 1;
    const size_t bytes = sizeof(T) * (size_t)n * ncols;
    T* bufs[3];
    for (int i = 0; i < 3; ++i) bufs[i] = static_cast<T*>(c.dmalloc(bytes));
    FDS_HIP_TRY(hipMemsetAsync(bufs[1], 0, bytes, c.stream));
    FDS_HIP_TRY(hipMemsetAsync(bufs[2], 0, bytes, c.stream));
    const double s1 = 2.0 / (hi - lo), s0 = -(hi + lo) / (hi - lo);
    const int64_t tot = (int64_t)n * ncols;
    const unsigned nb = (unsigned)((tot + 255) / 256);
    // rotate: cur = b_j, p1 = b_{j+1}, p2 = b_{j+2}
    int cur = 0, p1 = 1, p2 = 2;
    for (int j = deg; j >= 1; --j) {
        {
        KScope _ks(c, "gram_pow_half");
        hipLaunchKernelGGL(clenshaw_kernel<T>, dim3(nb), dim3(256), 0, c.stream, d, e, n, X, bufs[p1], bufs[p2],
                           bufs[cur], ncols, a[j], s1, s0, 2.0);
    }
        FDS_HIP_TRY(hipGetLastError());
        const int t = p2;
        p2 = p1;
        p1 = cur;
        cur = t;
    }
    {
        KScope _ks(c, "gram_pow_half");
        hipLaunchKernelGGL(clenshaw_kernel<T>, dim3(nb), dim3(256), 0, c.stream, d, e, n, X, bufs[p1], bufs[p2],
                       bufs[cur], ncols, a[0], s1, s0, 1.0);
    }
    FDS_HIP_TRY(hipGetLastError());
    FDS_HIP_TRY(hipMemcpyAsync(X, bufs[cur], bytes, hipMemcpyDeviceToDevice, c.stream));
    for (int i = 0; i < 3; ++i) c.dfree(bufs[i]);
}
template void gram_pow_half<double>(Ctx&, const double*, const double*, int, double, double, int, double*,
                                    int64_t);
template void gram_pow_half<double2>(Ctx&, const double*, const double*, int, double, double, int, double2*,
                                     int64_t);

// ============================================================ small dense
// Cholesky A = R^T R of a real SPD matrix (column-major n x n, in place: the upper
// triangle receives R, the strict lower triangle is zeroed). One workgroup.
__global__ void chol_kernel(double* __restrict__ A, int n, int* __restrict__ info) {
    __shared__ double piv;
    for (int j = 0; j < n; ++j) {
        if (threadIdx.x == 0) {
            const double v = A[j + (int64_t)j * n];
            if (!(v > 0.0)) info[0] = j + 1;
            piv = sqrt(fmax(v, 1e-300));
            A[j + (int64_t)j * n] = piv;
        }
        __syncthreads();
        for (int cidx = j + 1 + threadIdx.x; cidx < n; cidx += blockDim.x) A[j + (int64_t)cidx * n] /= piv;
        __syncthreads();
        const int m = n - j - 1;
        for (int64_t t = threadIdx.x; t < (int64_t)m * m; t += blockDim.x) {
            const int r = j + 1 + (int)(t % m), cc = j + 1 + (int)(t / m);
            if (r <= cc) A[r + (int64_t)cc * n] -= A[j + (int64_t)r * n] * A[j + (int64_t)cc * n];
        }
        __syncthreads();
    }
    for (int64_t t = threadIdx.x; t < (int64_t)n * n; t += blockDim.x) {
        const int r = (int)(t % n), cc = (int)(t / n);
        if (r > cc) A[t] = 0.0;
    }
}

// X <- X R^{-1} for R upper triangular (n x n column-major); X has `rows` rows
// (ld = rows), i.e. each row x solves y R = x. Thread per row.
__global__ void trsm_right_upper_kernel(const double* __restrict__ R, int n, double* __restrict__ X,
                                        int64_t rows) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    for (int cidx = 0; cidx < n; ++cidx) {
        double s = X[r + cidx * rows];
        for (int i = 0; i < cidx; ++i) s -= X[r + i * rows] * R[i + (int64_t)cidx * n];
        X[r + cidx * rows] = s / R[cidx + (int64_t)cidx * n];
    }
}

// LU with partial pivoting of a complex n x n column-major matrix (one workgroup).
// piv[j] = row swapped with j at step j. minpiv[0] = min |U_jj|, maxabs[0] = max |A|.
__global__ void lu_kernel(double2* __restrict__ A, int n, int* __restrict__ piv, double* __restrict__ stats) {
    __shared__ double sv[1024];
    __shared__ int si[1024];
    __shared__ int prow;
    __shared__ double2 pval;
    // max |A| before factorisation
    double mx = 0.0;
    for (int64_t t = threadIdx.x; t < (int64_t)n * n; t += blockDim.x) mx = fmax(mx, hypot(A[t].x, A[t].y));
    sv[threadIdx.x] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sv[threadIdx.x] = fmax(sv[threadIdx.x], sv[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        stats[1] = sv[0];
        stats[0] = 1e300;
    }
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        double best = -1.0;
        int bi = j;
        for (int r = j + threadIdx.x; r < n; r += blockDim.x) {
            const double2 v = A[r + (int64_t)j * n];
            const double av = fabs(v.x) + fabs(v.y);
            if (av > best) {
                best = av;
                bi = r;
            }
        }
        sv[threadIdx.x] = best;
        si[threadIdx.x] = bi;
        __syncthreads();
        for (int s = blockDim.x / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) {
                const double o = sv[threadIdx.x + s];
                const int oi = si[threadIdx.x + s];
                if (o > sv[threadIdx.x] || (o == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                    sv[threadIdx.x] = o;
                    si[threadIdx.x] = oi;
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            prow = si[0];
            piv[j] = prow;
        }
        __syncthreads();
        const int pr = prow;
        if (pr != j)
            for (int cidx = threadIdx.x; cidx < n; cidx += blockDim.x) {
                const double2 t = A[j + (int64_t)cidx * n];
                A[j + (int64_t)cidx * n] = A[pr + (int64_t)cidx * n];
                A[pr + (int64_t)cidx * n] = t;
            }
        __syncthreads();
        if (threadIdx.x == 0) {
            pval = A[j + (int64_t)j * n];
            stats[0] = fmin(stats[0], hypot(pval.x, pval.y));
        }
        __syncthreads();
        const double2 p = pval;
        const double den = p.x * p.x + p.y * p.y;
        const double2 pinv = den > 0.0 ? make_double2(p.x / den, -p.y / den) : make_double2(0.0, 0.0);
        for (int r = j + 1 + threadIdx.x; r < n; r += blockDim.x) A[r + (int64_t)j * n] = cmul(A[r + (int64_t)j * n], pinv);
        __syncthreads();
        const int m = n - j - 1;
        for (int64_t t = threadIdx.x; t < (int64_t)m * m; t += blockDim.x) {
            const int r = j + 1 + (int)(t % m), cc = j + 1 + (int)(t / m);
            A[r + (int64_t)cc * n] = csub(A[r + (int64_t)cc * n], cmul(A[r + (int64_t)j * n], A[j + (int64_t)cc * n]));
        }
        __syncthreads();
    }
}

// Gauss-Jordan inverse with partial pivoting of a complex r x r column-major
// matrix (one workgroup). A is overwritten; Ainv receives A^{-1}.
// stats[0] = min |pivot|, stats[1] = max |A| (before elimination).
__global__ void gj_inverse_kernel(double2* __restrict__ A, double2* __restrict__ Ainv, int r,
                                  double* __restrict__ stats) {
    extern __shared__ double2 fcol[];          // r entries: column j before elimination
    __shared__ double sv[1024];
    __shared__ int si[1024];
    __shared__ int prow;
    double mx = 0.0;
    for (int64_t t = threadIdx.x; t < (int64_t)r * r; t += blockDim.x) {
        mx = fmax(mx, hypot(A[t].x, A[t].y));
        Ainv[t] = make_double2((t % r) == (t / r) ? 1.0 : 0.0, 0.0);
    }
    sv[threadIdx.x] = mx;
    __syncthreads();
    for (int s2 = blockDim.x / 2; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2) sv[threadIdx.x] = fmax(sv[threadIdx.x], sv[threadIdx.x + s2]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        stats[1] = sv[0];
        stats[0] = 1e300;
    }
    __syncthreads();
    for (int j = 0; j < r; ++j) {
        double best = -1.0;
        int bi = j;
        for (int i = j + threadIdx.x; i < r; i += blockDim.x) {
            const double2 v = A[i + (int64_t)j * r];
            const double av = fabs(v.x) + fabs(v.y);
            if (av > best) {
                best = av;
                bi = i;
            }
        }
        sv[threadIdx.x] = best;
        si[threadIdx.x] = bi;
        __syncthreads();
        for (int s2 = blockDim.x / 2; s2 > 0; s2 >>= 1) {
            if (threadIdx.x < s2) {
                const double o = sv[threadIdx.x + s2];
                const int oi = si[threadIdx.x + s2];
                if (o > sv[threadIdx.x] || (o == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                    sv[threadIdx.x] = o;
                    si[threadIdx.x] = oi;
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) prow = si[0];
        __syncthreads();
        const int p = prow;
        if (p != j)
            for (int cc = threadIdx.x; cc < 2 * r; cc += blockDim.x) {
                double2* M = cc < r ? A : Ainv;
                const int col = cc < r ? cc : cc - r;
                const double2 t = M[j + (int64_t)col * r];
                M[j + (int64_t)col * r] = M[p + (int64_t)col * r];
                M[p + (int64_t)col * r] = t;
            }
        __syncthreads();
        const double2 pv = A[j + (int64_t)j * r];
        const double den = pv.x * pv.x + pv.y * pv.y;
        const double2 pinv = den > 0.0 ? make_double2(pv.x / den, -pv.y / den) : make_double2(0.0, 0.0);
        if (threadIdx.x == 0) stats[0] = fmin(stats[0], sqrt(den));
        __syncthreads();
        for (int cc = threadIdx.x; cc < 2 * r; cc += blockDim.x) {
            double2* M = cc < r ? A : Ainv;
            const int col = cc < r ? cc : cc - r;
            M[j + (int64_t)col * r] = cmul(M[j + (int64_t)col * r], pinv);
        }
        for (int i = threadIdx.x; i < r; i += blockDim.x) fcol[i] = A[i + (int64_t)j * r];
        __syncthreads();
        for (int64_t t = threadIdx.x; t < (int64_t)r * 2 * r; t += blockDim.x) {
            const int i = (int)(t % r);
            const int cc = (int)(t / r);
            if (i == j) continue;
            double2* M = cc < r ? A : Ainv;
            const int col = cc < r ? cc : cc - r;
            if (cc < r && col < j) continue;          // already eliminated columns stay zero
            const double2 f = fcol[i];
            M[i + (int64_t)col * r] = csub(M[i + (int64_t)col * r], cmul(f, M[j + (int64_t)col * r]));
        }
        __syncthreads();
    }
}

// One Gauss-Jordan step with partial pivoting on the augmented r x 2r matrix
// [A | X] (column-major, ld r), out of place (ping-pong buffers): every
// workgroup finds the same pivot in column j, then updates its own slab of
// GJ_CW columns. pabs[j] receives |pivot|.
constexpr int GJ_CW = 16;
__global__ __launch_bounds__(256) void gj_step_kernel(const double2* __restrict__ Min, double2* __restrict__ Mout,
                                                      int r, int j, double* __restrict__ pabs) {
    extern __shared__ double2 col[];     // column j of Min (r entries)
    __shared__ double sv[256];
    __shared__ int si[256];
    for (int i = threadIdx.x; i < r; i += blockDim.x) col[i] = Min[i + (int64_t)j * r];
    __syncthreads();
    double best = -1.0;
    int bi = j;
    for (int i = j + threadIdx.x; i < r; i += blockDim.x) {
        const double av = fabs(col[i].x) + fabs(col[i].y);
        if (av > best) {
            best = av;
            bi = i;
        }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s2 = blockDim.x / 2; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2) {
            const double o = sv[threadIdx.x + s2];
            const int oi = si[threadIdx.x + s2];
            if (o > sv[threadIdx.x] || (o == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                sv[threadIdx.x] = o;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    const int p = si[0];
    const double2 pv = col[p];
    const double den = pv.x * pv.x + pv.y * pv.y;
    const double2 pinv = den > 0.0 ? make_double2(pv.x / den, -pv.y / den) : make_double2(0.0, 0.0);
    if (blockIdx.x == 0 && threadIdx.x == 0) pabs[j] = sqrt(den);
    const int c0 = blockIdx.x * GJ_CW;
    for (int t = threadIdx.x; t < GJ_CW * r; t += blockDim.x) {
        const int i = t % r;
        const int cc = c0 + t / r;
        if (cc >= 2 * r) continue;
        const double2 prow = cmul(Min[p + (int64_t)cc * r], pinv);   // scaled pivot row
        double2 v;
        if (i == j) {
            v = prow;
        } else {
            const int src = (i == p) ? j : i;                        // rows j and p swapped
            v = csub(Min[src + (int64_t)cc * r], cmul(col[src], prow));
        }
        Mout[i + (int64_t)cc * r] = v;
    }
}

__global__ void gj_init_kernel(const double2* __restrict__ A, double2* __restrict__ M, int r) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * (int64_t)r * r) return;
    const int i = (int)(t % r);
    const int64_t cc = t / r;
    M[t] = cc < r ? A[t] : make_double2(i == (int)(cc - r) ? 1.0 : 0.0, 0.0);
}

__global__ void gj_stats_kernel(const double2* __restrict__ A, const double* __restrict__ pabs, int r,
                                double* __restrict__ stats) {
    __shared__ double smax[256], smin[256];
    double mx = 0.0, mn = 1e300;
    for (int64_t t = threadIdx.x; t < (int64_t)r * r; t += blockDim.x) mx = fmax(mx, hypot(A[t].x, A[t].y));
    for (int t = threadIdx.x; t < r; t += blockDim.x) mn = fmin(mn, pabs[t]);
    smax[threadIdx.x] = mx;
    smin[threadIdx.x] = mn;
    __syncthreads();
    for (int s2 = blockDim.x / 2; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s2]);
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s2]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        stats[0] = smin[0];
        stats[1] = smax[0];
    }
}

void gj_inverse(Ctx& c, double2* A, double2* Ainv, int r, double* stats) {
    // augmented [A | I] ping-pong; the inverse ends in the right half
    double2* M0 = static_cast<double2*>(c.dmalloc(sizeof(double2) * 2 * (size_t)r * r));
    double2* M1 = static_cast<double2*>(c.dmalloc(sizeof(double2) * 2 * (size_t)r * r));
    double* pabs = static_cast<double*>(c.dmalloc(sizeof(double) * r));
    const int64_t tot = 2 * (int64_t)r * r;
    {
        KScope _ks(c, "gj_inverse");
        hipLaunchKernelGGL(gj_init_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c.stream, A, M0, r);
        const unsigned nb = (unsigned)((2 * r + GJ_CW - 1) / GJ_CW);
        for (int j = 0; j < r; ++j) {
            const double2* in = (j & 1) ? M1 : M0;
            double2* out = (j & 1) ? M0 : M1;
            hipLaunchKernelGGL(gj_step_kernel, dim3(nb), dim3(256), sizeof(double2) * r, c.stream, in, out, r, j,
                               pabs);
        }
        hipLaunchKernelGGL(gj_stats_kernel, dim3(1), dim3(256), 0, c.stream, A, pabs, r, stats);
    }
    FDS_HIP_TRY(hipGetLastError());
    const double2* fin = (r & 1) ? M1 : M0;
    FDS_HIP_TRY(hipMemcpyAsync(Ainv, fin + (size_t)r * r, sizeof(double2) * (size_t)r * r, hipMemcpyDeviceToDevice,
                               c.stream));
    c.dfree(M0);
    c.dfree(M1);
    c.dfree(pabs);
}

// Solve LU x = P b for each column of B (n x ncols, ld = n), thread per column.
__global__ void lu_solve_kernel(const double2* __restrict__ LU, const int* __restrict__ piv, int n,
                                double2* __restrict__ B, int64_t ncols) {
    const int64_t cidx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cidx >= ncols) return;
    double2* b = B + cidx * n;
    for (int j = 0; j < n; ++j) {
        const int p = piv[j];
        if (p != j) {
            const double2 t = b[j];
            b[j] = b[p];
            b[p] = t;
        }
    }
    for (int j = 0; j < n; ++j) {
        const double2 bj = b[j];
        for (int r = j + 1; r < n; ++r) b[r] = csub(b[r], cmul(LU[r + (int64_t)j * n], bj));
    }
    for (int j = n - 1; j >= 0; --j) {
        const double2 u = LU[j + (int64_t)j * n];
        const double den = u.x * u.x + u.y * u.y;
        const double2 xj = cmul(b[j], make_double2(u.x / den, -u.y / den));
        b[j] = xj;
        for (int r = 0; r < j; ++r) b[r] = csub(b[r], cmul(LU[r + (int64_t)j * n], xj));
    }
}

void chol_upper(Ctx& c, double* A, int n, int* info) {
    {
        KScope _ks(c, "chol");
        hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(1024), 0, c.stream, A, n, info);
    }
    FDS_HIP_TRY(hipGetLastError());
}

void trsm_right_upper(Ctx& c, const double* R, int n, double* X, int64_t rows) {
    {
        KScope _ks(c, "trsm");
        hipLaunchKernelGGL(trsm_right_upper_kernel, dim3((unsigned)((rows + 127) / 128)), dim3(128), 0, c.stream, R,
                       n, X, rows);
    }
    FDS_HIP_TRY(hipGetLastError());
}

void lu_factor(Ctx& c, double2* A, int n, int* piv, double* stats) {
    {
        KScope _ks(c, "lu_factor");
        hipLaunchKernelGGL(lu_kernel, dim3(1), dim3(1024), 0, c.stream, A, n, piv, stats);
    }
    FDS_HIP_TRY(hipGetLastError());
}

void lu_solve(Ctx& c, const double2* LU, const int* piv, int n, double2* B, int64_t ncols) {
    if (ncols <= 0) return;
    {
        KScope _ks(c, "lu_solve");
        hipLaunchKernelGGL(lu_solve_kernel, dim3((unsigned)((ncols + 63) / 64)), dim3(64), 0, c.stream, LU, piv, n, B,
                       ncols);
    }
    FDS_HIP_TRY(hipGetLastError());
}

// ============================================================ element-wise helpers
__global__ void real_to_complex_kernel(const double* __restrict__ x, double2* __restrict__ y, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = make_double2(x[t], 0.0);
}

// y = a x + b y  (complex scalars a, b)
__global__ void axpby_kernel(double2 a, const double2* __restrict__ x, double2 b, double2* __restrict__ y,
                             int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = cadd(cmul(a, x[t]), cmul(b, y[t]));
}

__global__ void daxpby_kernel(double a, const double* __restrict__ x, double b, double* __restrict__ y, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = a * x[t] + b * y[t];
}

void daxpby(Ctx& c, double a, const double* x, double b, double* y, int64_t n) {
    if (n <= 0) return;
    {
        KScope _ks(c, "elementwise");
        hipLaunchKernelGGL(daxpby_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, a, x, b, y, n);
    }
    FDS_HIP_TRY(hipGetLastError());
}

void real_to_complex(Ctx& c, const double* x, double2* y, int64_t n) {
    if (n <= 0) return;
    {
        KScope _ks(c, "elementwise");
        hipLaunchKernelGGL(real_to_complex_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, x, y, n);
    }
    FDS_HIP_TRY(hipGetLastError());
}

void axpby(Ctx& c, double2 a, const double2* x, double2 b, double2* y, int64_t n) {
    if (n <= 0) return;
    {
        KScope _ks(c, "elementwise");
        hipLaunchKernelGGL(axpby_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, a, x, b, y, n);
    }
    FDS_HIP_TRY(hipGetLastError());
}

// add `s` to the diagonal of an n x n column-major matrix
__global__ void add_diag_kernel(double2* __restrict__ A, int n, double s) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) A[t + (int64_t)t * n].x += s;
}

void add_diag(Ctx& c, double2* A, int n, double s) {
    {
        KScope _ks(c, "elementwise");
        hipLaunchKernelGGL(add_diag_kernel, dim3((n + 255) / 256), dim3(256), 0, c.stream, A, n, s);
    }
    FDS_HIP_TRY(hipGetLastError());
}

}  // namespace fds
