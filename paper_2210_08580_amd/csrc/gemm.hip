// Complex (and real) GEMM on the matrix cores, column-major, op(A), op(B) in
// {N, T, C}: FP64 MFMA (v_mfma_f64_16x16x4f64) for complex128 and real FP64,
// complex128 with a complex64 A operand widened on load (optionally with a
// complex128 band), complex64 on FP32 MFMA (v_mfma_f32_16x16x4f32, FP32
// accumulation); optional split-K with a deterministic reduction, a 128 x 64
// tile for large complex128 products, a grouped launch over problems of uneven
// sizes, and a split-K / tile autotuner.
#include <algorithm>
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

// complex128 value of a raw A element under op (conjugated for OP_C)
__device__ __forceinline__ double2 widen_op(float2 f, int op) { return make_double2(f.x, op == OP_C ? -f.y : f.y); }
__device__ __forceinline__ double2 widen_op(double2 d, int op) { return op == OP_C ? make_double2(d.x, -d.y) : d; }
__device__ __forceinline__ float2 conj_op(float2 f, int op) { return op == OP_C ? make_float2(f.x, -f.y) : f; }

// op(A)[gi][gp] from the complex128 band when |gp - gi| (cyclic) <= w
__device__ __forceinline__ bool band_lookup(const BandA& bd, int gi, int gp, double2& v) {
    int d = gp - gi;
    d = d < 0 ? d + bd.n : d;
    d = 2 * d > bd.n ? d - bd.n : d;
    if ((d < 0 ? -d : d) > bd.w) return false;
    v = bd.nb[(int64_t)gi * (2 * bd.w + 1) + d + bd.w];
    return true;
}
// element (gi, gp) of op(A), source pointer src
template <typename T, typename TA>
__device__ __forceinline__ void ld_a(const TA* src, int op, int gi, int gp, const BandA& bd, T& v) {
    if constexpr (std::is_same<TA, float2>::value && std::is_same<T, double2>::value) {
        if (bd.nb && band_lookup(bd, gi, gp, v)) return;
    }
    ld_into(src, op, v);
}

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
                                          T (&sA)[GB_K][GB_M + G_PAD], T (&sB)[GB_K][GB_N + G_PAD],
                                          const BandA& bd) {
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
                ld_a(src, OPA, gi, gp, bd, v);
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
                                                   T* __restrict__ part, BandA bd) {
    __shared__ T sA[GB_K][GB_M + G_PAD];
    __shared__ T sB[GB_K][GB_N + G_PAD];
    gemm_tile<T, TA, OPA, OPB>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, blockIdx.x, blockIdx.y,
                               blockIdx.z, sA, sB, bd);
}

// Large problems: 128 x 64 output tile per workgroup (4 wavefronts of 64 x 32,
// 4 x 2 MFMA tiles each). The K slices pass through registers (loaded two
// slices ahead) into two alternating LDS buffers, so the matrix cores work on
// one slice while the next is staged (complex128 output; A may be complex64,
// widened when staged).
constexpr int BB_M = 128, BB_N = 64, BB_K = 16, BB_PAD = 2;

// TB = double: a real B operand (two real MFMAs per complex-by-real tile step).
// WN = 2: 128 x 64 tile, 2 x 2 wavefronts of 64 x 32; WN = 1 (narrow outputs of at
// most 32 columns): 128 x 32 tile, 4 x 1 wavefronts of 32 x 32.
// AL32 (complex64 A without a complex128 band): A stays complex64 in LDS and is
// widened when read from it, which halves its LDS footprint. A complex B then
// takes K slices of 32 (half the barriers per matrix-core step, one slice of
// loads in flight for twice as long); a real B keeps slices of 16 and fits two
// workgroups per compute unit (registers capped at two wavefronts per SIMD).
// TA = double: a real A (the filter basis) against a complex B, two real MFMAs per
// step (accR = a br, accI = a bi), two workgroups per compute unit as well.
template <typename TA, typename TB>
constexpr int gb_waves() {
    return (std::is_same<TA, double>::value || (std::is_same<TA, float2>::value && std::is_same<TB, double>::value))
               ? 2 : 1;
}
template <typename TA, typename TB, int OPA, int OPB, int WN = 2, bool AL32 = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(gb_waves<TA, TB>(), gb_waves<TA, TB>())))
void gemm_big_kernel(int m, int n, int k, double2 alpha, const TA* __restrict__ A, int64_t lda,
                     const TB* __restrict__ B, int64_t ldb, double2 beta, double2* __restrict__ C, int64_t ldc,
                     int kchunk, double2* __restrict__ part, BandA bd) {
    constexpr bool BCPLX = std::is_same<TB, double2>::value;
    constexpr bool ACPLX = !std::is_same<TA, double>::value;
    static_assert(!AL32 || std::is_same<TA, float2>::value, "complex64 LDS staging needs a complex64 A");
    static_assert(ACPLX || (BCPLX && OPA == OP_N), "a real A: untransposed, against a complex B");
    // transposed-A loads leave no registers for a third product
    constexpr bool GAUSS3 = ACPLX && BCPLX && OPA == OP_N;
    constexpr int KS = (AL32 && BCPLX) ? 32 : BB_K; // K slice depth
    constexpr int BN = 32 * WN;             // tile columns
    constexpr int WM = 4 / WN;              // wavefronts along the rows
    constexpr int RT = BB_M / (16 * WM);    // 16-row MFMA tiles per wavefront
    constexpr int EA = KS * BB_M / 256;     // A elements staged per thread and slice
    constexpr int EB = KS * BN / 256;       // B elements staged per thread and slice
    typedef typename std::conditional<AL32, float2, typename std::conditional<ACPLX, double2, double>::type>::type SA;
    typedef typename std::conditional<ACPLX, double2, double>::type FA;   // A fragment in registers
    // two LDS buffers: slice i is multiplied from one while slice i + 1 is staged into the other
    __shared__ SA sA[2][KS][BB_M + BB_PAD];
    __shared__ TB sB[2][KS][BN + BB_PAD];
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int wm = w % WM, wn = w / WM;
    const int row0 = blockIdx.x * BB_M, col0 = blockIdx.y * BN;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(k, kbeg + kchunk);
    // complex B and untransposed A: Gauss's three products per tile, T1 = ar br,
    // T2 = ai bi, T3 = (ar + ai)(br + bi); Re = T1 - T2, Im = T3 - T1 - T2 (the sums
    // are formed after the LDS reads). Other complex cases: four products. Real B:
    // accR = ar b, accI = ai b.
    d4 accR[RT][2], accI[RT][2], acc3[RT][2];
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            accR[a][b] = d4{0.0, 0.0, 0.0, 0.0};
            accI[a][b] = d4{0.0, 0.0, 0.0, 0.0};
            acc3[a][b] = d4{0.0, 0.0, 0.0, 0.0};
        }
    // raw operands in flight (complex64 A is widened when staged to LDS, or when
    // read from it under AL32, so the loads of the next slice are not waited on
    // while the current one computes)
    TA ra[EA];
    TB rb[EB];
    // staging maps: element e of a thread is row i / column j, slice row p
    auto amap = [&](int e, int& i, int& p) {
        if (OPA == OP_N) {
            i = tid & 127;
            p = (tid >> 7) + 2 * e;
        } else {
            p = tid % KS;
            i = tid / KS + (256 / KS) * e;
        }
    };
    auto bmap = [&](int e, int& j, int& p) {
        if (OPB == OP_N) {
            p = tid % KS;
            j = tid / KS + (256 / KS) * e;
        } else {
            j = tid % BN;
            p = tid / BN + (256 / BN) * e;
        }
    };
    auto loadAB = [&](int kk) {
#pragma unroll
        for (int e = 0; e < EA; ++e) {
            int i, p;
            amap(e, i, p);
            const int gi = row0 + i, gp = kk + p;
            TA v{};
            if (gi < m && gp < kend) v = (OPA == OP_N) ? A[gi + (int64_t)gp * lda] : A[gp + (int64_t)gi * lda];
            ra[e] = v;
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            int j, p;
            bmap(e, j, p);
            const int gj = col0 + j, gp = kk + p;
            TB v{};
            if (gj < n && gp < kend) {
                const TB* src = (OPB == OP_N) ? B + gp + (int64_t)gj * ldb : B + gj + (int64_t)gp * ldb;
                v = ld_op(src, OPB);
            }
            rb[e] = v;
        }
    };
    // does the K slice [kk, kk + KS) meet the band of the row block (uniform)?
    auto band_slice = [&](int kk) {
        if (!bd.nb) return false;
        const int dmin = kk - (row0 + BB_M - 1), dmax = kk + KS - 1 - row0;
        for (int q = -1; q <= 1; ++q)
            if (dmax >= q * bd.n - bd.w && dmin <= q * bd.n + bd.w) return true;
        return false;
    };
    auto stage = [&](int kk, int buf) {
        const bool bsl = !AL32 && std::is_same<TA, float2>::value && band_slice(kk);
#pragma unroll
        for (int e = 0; e < EA; ++e) {
            int i, p;
            amap(e, i, p);
            if constexpr (AL32) {
                sA[buf][p][i] = conj_op(ra[e], OPA);
            } else if constexpr (!ACPLX) {
                sA[buf][p][i] = ra[e];
            } else {
                double2 v = widen_op(ra[e], OPA);
                if (bsl && row0 + i < m && kk + p < kend) band_lookup(bd, row0 + i, kk + p, v);
                sA[buf][p][i] = v;
            }
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            int j, p;
            bmap(e, j, p);
            sB[buf][p][j] = rb[e];
        }
    };
    auto compute = [&](int buf) {
        // two k-steps per iteration: a full unroll makes the compiler hoist the LDS
        // fragments of all four, and the extra live registers then spill to AGPRs
        // (moves every slice)
#pragma unroll 2
        for (int kc = 0; kc < KS / 4; ++kc) {
            const int pr = kc * 4 + (lane >> 4);
            FA a[RT];
            TB b[2];
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const SA av = sA[buf][pr][wm * (16 * RT) + r * 16 + (lane & 15)];
                if constexpr (ACPLX) a[r] = make_double2(av.x, av.y);
                else a[r] = av;
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) b[c] = sB[buf][pr][wn * 32 + c * 16 + (lane & 15)];
            if constexpr (!ACPLX) {
#pragma unroll
                for (int r = 0; r < RT; ++r)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        accR[r][c] = mfma16(a[r], b[c].x, accR[r][c]);
                        accI[r][c] = mfma16(a[r], b[c].y, accI[r][c]);
                    }
            } else if constexpr (GAUSS3) {
                double as[RT], bs[2];
#pragma unroll
                for (int r = 0; r < RT; ++r) as[r] = a[r].x + a[r].y;
#pragma unroll
                for (int c = 0; c < 2; ++c) bs[c] = b[c].x + b[c].y;
#pragma unroll
                for (int r = 0; r < RT; ++r)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        accR[r][c] = mfma16(a[r].x, b[c].x, accR[r][c]);
                        accI[r][c] = mfma16(a[r].y, b[c].y, accI[r][c]);
                        acc3[r][c] = mfma16(as[r], bs[c], acc3[r][c]);
                    }
            } else if constexpr (BCPLX) {
#pragma unroll
                for (int r = 0; r < RT; ++r)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        accR[r][c] = mfma16(a[r].x, b[c].x, accR[r][c]);
                        accR[r][c] = mfma16(-a[r].y, b[c].y, accR[r][c]);
                        accI[r][c] = mfma16(a[r].x, b[c].y, accI[r][c]);
                        accI[r][c] = mfma16(a[r].y, b[c].x, accI[r][c]);
                    }
            } else {
#pragma unroll
                for (int r = 0; r < RT; ++r)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        accR[r][c] = mfma16(a[r].x, b[c], accR[r][c]);
                        accI[r][c] = mfma16(a[r].y, b[c], accI[r][c]);
                    }
            }
        }
    };
    // slice i in buffer i & 1; one barrier per slice: every wavefront has finished
    // multiplying from a buffer before anyone stages into it again
    if (kbeg < kend) {
        loadAB(kbeg);
        stage(kbeg, 0);
        if (kbeg + KS < kend) loadAB(kbeg + KS);
        __syncthreads();
    }
    int buf = 0;
    for (int kk = kbeg; kk < kend; kk += KS) {
        compute(buf);
        if (kk + KS < kend) {
            stage(kk + KS, buf ^ 1);
            if (kk + 2 * KS < kend) loadAB(kk + 2 * KS);
        }
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = row0 + wm * (16 * RT) + r * 16 + acc_row(0.0, lane, v);
                const int gj = col0 + wn * 32 + c * 16 + (lane & 15);
                if (gi >= m || gj >= n) continue;
                const double2 acc = GAUSS3 ? make_double2(accR[r][c][v] - accI[r][c][v],
                                                         acc3[r][c][v] - accR[r][c][v] - accI[r][c][v])
                                          : make_double2(accR[r][c][v], accI[r][c][v]);
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
                                            P.k + GB_K, nullptr, bx, by, 0, sA, sB, BandA());
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
                        T beta, T* C, int64_t ldc, int cfg, const BandA& bd);

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
static int choose_config(Ctx& c, int m, int n, int k, const TA* A, int64_t lda, const T* B, int64_t ldb,
                         const BandA& bd) {
    auto split_for = [&](int tiles) {
        int nz = 1;
        if (tiles < 512 && k > 4 * GB_K) nz = std::max(1, std::min((512 + tiles - 1) / tiles, (k + 255) / 256));
        return std::min(nz, 64);
    };
    const bool bigp = big_ok<T, TA>() && m >= BB_M && n >= BB_N;
    // outputs of at most 32 columns: the 128 x 32 tile (a 64 x 64 tile would leave half
    // of its wavefronts without columns)
    const bool narrowp = big_ok<T, TA>() && m >= BB_M && n <= 32;
    int cfg;
    if (bigp) {
        const int tb = ((m + BB_M - 1) / BB_M) * ((n + BB_N - 1) / BB_N);
        cfg = 256 | split_for(4 * tb);
    } else if (narrowp) {
        cfg = 512 | split_for(4 * ((m + BB_M - 1) / BB_M));
    } else {
        cfg = split_for(((m + GB_M - 1) / GB_M) * ((n + GB_N - 1) / GB_N));
    }
    if (c.split_hint > 0) return (cfg & 768) | std::min(std::max(cfg & 255, c.split_hint), 64);
    if (!c.autotune || c.noalloc) return cfg;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(c.stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return cfg;
    char key[160];
    snprintf(key, sizeof(key), "%s/%s/%d%d/%d/%d/%d", typeid(T).name(), typeid(TA).name(), OPA, OPB, bucket(m),
             bucket(n), bucket(k));
    auto it = c.tuned.find(key);
    if (it != c.tuned.end()) return it->second;
    std::vector<int> cand;
    for (int big = 0; big <= (bigp || narrowp ? 1 : 0); ++big) {
        const int tiles = big ? ((m + BB_M - 1) / BB_M) * (narrowp ? 1 : (n + BB_N - 1) / BB_N)
                              : ((m + GB_M - 1) / GB_M) * ((n + GB_N - 1) / GB_N);
        for (int z = 1; z <= 64; z *= 2) {
            if (z > 1 && ((int64_t)z * 2 * GB_K > k || (int64_t)z * m * n * sizeof(T) > ((int64_t)1 << 29) ||
                          (int64_t)tiles * z > 8192))
                continue;
            cand.push_back((big ? (narrowp ? 512 : 256) : 0) | z);
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
        gemm_launch<T, TA, OPA, OPB>(c, m, n, k, one, A, lda, B, ldb, zero, scratch, m, z, bd);   // warm
        FDS_HIP_TRY(hipEventRecord(e0, c.stream));
        for (int rep = 0; rep < 3; ++rep)
            gemm_launch<T, TA, OPA, OPB>(c, m, n, k, one, A, lda, B, ldb, zero, scratch, m, z, bd);
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
                          T beta, T* C, int64_t ldc, const BandA& bd) {
    const int cfg = choose_config<T, TA, OPA, OPB>(c, m, n, k, A, lda, B, ldb, bd);
    gemm_launch<T, TA, OPA, OPB>(c, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, cfg, bd);
}

template <typename T, typename TA, int OPA, int OPB>
static void gemm_launch(Ctx& c, int m, int n, int k, T alpha, const TA* A, int64_t lda, const T* B, int64_t ldb,
                        T beta, T* C, int64_t ldc, int cfg, const BandA& bd) {
    const bool big = big_ok<T, TA>() && (cfg & 256);
    const bool narrow = big_ok<T, TA>() && (cfg & 512);
    const int bm = big || narrow ? BB_M : GB_M, bn = narrow ? 32 : (big ? BB_N : GB_N);
    const int gm = (m + bm - 1) / bm, gn = (n + bn - 1) / bn;
    int nz = std::max(1, cfg & 255);
    if (c.noalloc && nz > 1) {   // the partial sums must fit the caller's workspace
        const size_t per = sizeof(T) * (size_t)m * n;
        nz = std::max(1, std::min<int>(nz, (int)std::min<size_t>(c.ws_bytes / per, 64)));
    }
    // a complex64 A without a complex128 band stays complex64 in LDS (K slices of 32)
    const bool al32 = std::is_same<TA, float2>::value && !bd.nb && (big || narrow);
    const int kq = al32 ? 2 * GB_K : GB_K;
    int kchunk = (k + nz - 1) / nz;
    kchunk = (kchunk + kq - 1) / kq * kq;
    nz = (k + kchunk - 1) / kchunk;
    T* part = nullptr;
    if (nz > 1)
        part = c.noalloc ? static_cast<T*>(c.ws) : static_cast<T*>(c.dmalloc(sizeof(T) * (size_t)nz * m * n));
    {
        KScope _ks(c, c.gemm_tag ? c.gemm_tag : (std::is_same<T, float2>::value ? "gemm_c64" : "gemm"));
        if constexpr (big_ok<T, TA>()) {
            bool done = false;
            if constexpr (std::is_same<TA, float2>::value) {
                if (al32) {
                    if (narrow)
                        hipLaunchKernelGGL((gemm_big_kernel<TA, double2, OPA, OPB, 1, true>), dim3(gm, gn, nz),
                                           dim3(256), 0, c.stream, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                                           kchunk, part, bd);
                    else
                        hipLaunchKernelGGL((gemm_big_kernel<TA, double2, OPA, OPB, 2, true>), dim3(gm, gn, nz),
                                           dim3(256), 0, c.stream, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                                           kchunk, part, bd);
                    done = true;
                }
            }
            if (done) {
            } else if (narrow) {
                hipLaunchKernelGGL((gemm_big_kernel<TA, double2, OPA, OPB, 1>), dim3(gm, gn, nz), dim3(256), 0, c.stream,
                                   m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, bd);
            } else if (big) {
                hipLaunchKernelGGL((gemm_big_kernel<TA, double2, OPA, OPB>), dim3(gm, gn, nz), dim3(256), 0, c.stream, m, n, k,
                                   alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, bd);
            } else {
                hipLaunchKernelGGL((gemm_kernel<T, TA, OPA, OPB>), dim3(gm, gn, nz), dim3(256), 0, c.stream, m, n, k,
                                   alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, bd);
            }
        } else {
            hipLaunchKernelGGL((gemm_kernel<T, TA, OPA, OPB>), dim3(gm, gn, nz), dim3(256), 0, c.stream, m, n, k,
                               alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, bd);
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
        if (!c.noalloc) c.dfree(part);
    }
}

template <typename T, typename TA = T>
static void gemm_any(Ctx& c, int opa, int opb, int m, int n, int k, T alpha, const TA* A, int64_t lda, const T* B,
                     int64_t ldb, T beta, T* C, int64_t ldc, const BandA& bd = BandA()) {
    if (m <= 0 || n <= 0) return;
#define FDS_G(a, b)                                                                    \
    if (opa == a && opb == b) {                                                        \
        gemm_dispatch<T, TA, a, b>(c, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, bd); \
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
               const double2* B, int64_t ldb, double2 beta, double2* C, int64_t ldc, const BandA& band) {
    if (band.nb) {
        FDS_REQUIRE(m == band.n && k == band.n && opa != OP_C && band.w >= 0 && 2 * band.w < band.n, FDS_ERR_ARG,
                    "banded complex64 GEMM: square symmetric operand, no conjugate");
    }
    gemm_any<double2, float2>(c, opa, opb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, band);
}

// C = alpha A B + beta C (no transposes) with a complex A (complex128, or complex64
// with an optional complex128 band) and a real B, on the 128 x 64 tile kernel;
// false (nothing launched) when the output is smaller than one tile.
template <typename TA>
static bool gemm_real_b(Ctx& c, int m, int n, int k, double2 alpha, const TA* A, int64_t lda, const double* B,
                        int64_t ldb, double2 beta, double2* C, int64_t ldc, const BandA& bd) {
    if (m < BB_M || n < BB_N || k <= 0) return false;
    const int gm = (m + BB_M - 1) / BB_M, gn = (n + BB_N - 1) / BB_N;
    // complex64 A without a band: complex64 in LDS, two workgroups per compute unit,
    // so split K until about 512 workgroups are in flight; else one per compute unit
    const bool al32 = std::is_same<TA, float2>::value && !bd.nb;
    const int want = al32 ? 512 : 128;
    int nz = 1;
    if (gm * gn < want && k > 4 * GB_K) nz = std::max(1, std::min((want + gm * gn - 1) / (gm * gn), (k + 255) / 256));
    nz = std::min(nz, 64);
    int kchunk = (k + nz - 1) / nz;
    kchunk = (kchunk + GB_K - 1) / GB_K * GB_K;
    nz = (k + kchunk - 1) / kchunk;
    double2* part = nullptr;
    if (nz > 1) part = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)nz * m * n));
    {
        KScope _ks(c, c.gemm_tag ? c.gemm_tag : "gemm");
        bool done = false;
        if constexpr (std::is_same<TA, float2>::value) {
            if (al32) {
                hipLaunchKernelGGL((gemm_big_kernel<TA, double, OP_N, OP_N, 2, true>), dim3(gm, gn, nz), dim3(256), 0,
                                   c.stream, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, bd);
                done = true;
            }
        }
        if (!done)
            hipLaunchKernelGGL((gemm_big_kernel<TA, double, OP_N, OP_N>), dim3(gm, gn, nz), dim3(256), 0, c.stream, m,
                               n, k, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, bd);
    }
    FDS_HIP_TRY(hipGetLastError());
    if (part) {
        const int64_t tot = (int64_t)m * n;
        {
            KScope _ks(c, "gemm_splitk_reduce");
            hipLaunchKernelGGL(splitk_reduce_kernel<double2>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                               c.stream, m, n, nz, alpha, part, beta, C, ldc);
        }
        FDS_HIP_TRY(hipGetLastError());
        c.dfree(part);
    }
    return true;
}

bool zgemm_real_b(Ctx& c, int m, int n, int k, double2 alpha, const double2* A, int64_t lda, const double* B,
                  int64_t ldb, double2 beta, double2* C, int64_t ldc) {
    return gemm_real_b<double2>(c, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, BandA());
}

bool zgemm_a32_real_b(Ctx& c, int m, int n, int k, double2 alpha, const float2* A, int64_t lda, const double* B,
                      int64_t ldb, double2 beta, double2* C, int64_t ldc, const BandA& band) {
    if (band.nb) {
        FDS_REQUIRE(m == band.n && k == band.n && band.w >= 0 && 2 * band.w < band.n, FDS_ERR_ARG,
                    "banded complex64 GEMM: square symmetric operand");
    }
    return gemm_real_b<float2>(c, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, band);
}

bool zgemm_real_a(Ctx& c, int m, int n, int k, double2 alpha, const double* A, int64_t lda, const double2* B,
                  int64_t ldb, double2 beta, double2* C, int64_t ldc) {
    const bool narrow = n <= 32;
    if (m < BB_M || n <= 0 || k <= 0 || (!narrow && n < BB_N)) return false;
    const int bn = narrow ? 32 : BB_N;
    const int gm = (m + BB_M - 1) / BB_M, gn = (n + bn - 1) / bn;
    // two workgroups per compute unit: split K until about 512 are in flight
    int nz = 1;
    if (gm * gn < 512 && k > 4 * GB_K) nz = std::max(1, std::min((512 + gm * gn - 1) / (gm * gn), (k + 255) / 256));
    nz = std::min(nz, 64);
    if (c.noalloc && nz > 1) {   // the partial sums must fit the caller's workspace
        const size_t per = sizeof(double2) * (size_t)m * n;
        nz = std::max(1, std::min<int>(nz, (int)std::min<size_t>(c.ws_bytes / per, 64)));
    }
    int kchunk = (k + nz - 1) / nz;
    kchunk = (kchunk + GB_K - 1) / GB_K * GB_K;
    nz = (k + kchunk - 1) / kchunk;
    double2* part = nullptr;
    if (nz > 1)
        part = c.noalloc ? static_cast<double2*>(c.ws)
                         : static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)nz * m * n));
    {
        KScope _ks(c, c.gemm_tag ? c.gemm_tag : "gemm");
        if (narrow)
            hipLaunchKernelGGL((gemm_big_kernel<double, double2, OP_N, OP_N, 1>), dim3(gm, gn, nz), dim3(256), 0,
                               c.stream, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, BandA());
        else
            hipLaunchKernelGGL((gemm_big_kernel<double, double2, OP_N, OP_N, 2>), dim3(gm, gn, nz), dim3(256), 0,
                               c.stream, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, BandA());
    }
    FDS_HIP_TRY(hipGetLastError());
    if (part) {
        const int64_t tot = (int64_t)m * n;
        {
            KScope _ks(c, "gemm_splitk_reduce");
            hipLaunchKernelGGL(splitk_reduce_kernel<double2>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                               c.stream, m, n, nz, alpha, part, beta, C, ldc);
        }
        FDS_HIP_TRY(hipGetLastError());
        if (!c.noalloc) c.dfree(part);
    }
    return true;
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

}  // namespace fds
