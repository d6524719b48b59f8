// Device linear-algebra building blocks (see linalg.hip).
#pragma once
#include <vector>

#include "fds_internal.h"

namespace fds {

enum { OP_N = 0, OP_T = 1, OP_C = 2 };
constexpr double kPiHost = 3.14159265358979323846;

// C = alpha op(A) op(B) + beta C, column-major, m x n result, inner dimension k.
void zgemm(Ctx& c, int opa, int opb, int m, int n, int k, double2 alpha, const double2* A, int64_t lda,
           const double2* B, int64_t ldb, double2 beta, double2* C, int64_t ldc);
// Grouped complex GEMM C_g = alpha_g A_g B_g + beta_g C_g (no transposes), one launch.
struct GemmSpec {
    int m, n, k;
    double2 alpha, beta;
    const double2* A;
    int64_t lda;
    const double2* B;
    int64_t ldb;
    double2* C;
    int64_t ldc;
};
void zgemm_grouped_nn(Ctx& c, const std::vector<GemmSpec>& specs);
// Split-K autotuner cache: number of entries; keys: cap x 160 chars, values: cap ints.
int autotune_entries(Ctx& c, int cap, char* keys, int* values);
// Complex128 band of a square, symmetric complex64-stored operand: the entries
// of op(A) with cyclic |column - row| <= w are read as nb[row * (2w + 1) + column
// - row + w] instead of from A (nb == nullptr: no band).
struct BandA {
    const double2* nb = nullptr;
    int w = -1;
    int n = 0;
};
// zgemm with a complex64 A operand, widened to complex128 on load (FP64 MFMA),
// optionally with a complex128 band (requires m == k == band.n and opa != C).
void zgemm_a32(Ctx& c, int opa, int opb, int m, int n, int k, double2 alpha, const float2* A, int64_t lda,
               const double2* B, int64_t ldb, double2 beta, double2* C, int64_t ldc, const BandA& band = BandA());
// C = alpha A B + beta C (no transposes) with a real B (two real MFMAs per complex-by-real
// step instead of four); returns false without launching when m < 128 or n < 64.
bool zgemm_real_b(Ctx& c, int m, int n, int k, double2 alpha, const double2* A, int64_t lda, const double* B,
                  int64_t ldb, double2 beta, double2* C, int64_t ldc);
bool zgemm_a32_real_b(Ctx& c, int m, int n, int k, double2 alpha, const float2* A, int64_t lda, const double* B,
                      int64_t ldb, double2 beta, double2* C, int64_t ldc, const BandA& band = BandA());
// C = alpha A B + beta C (no transposes) with a real A (the filter basis) and a
// complex B: two real MFMAs per step instead of three; returns false without
// launching when m < 128, or n < 64 with n > 32.
bool zgemm_real_a(Ctx& c, int m, int n, int k, double2 alpha, const double* A, int64_t lda, const double2* B,
                  int64_t ldb, double2 beta, double2* C, int64_t ldc);
// Complex64 variant on the FP32 matrix cores (FP32 accumulation).
void cgemm(Ctx& c, int opa, int opb, int m, int n, int k, float2 alpha, const float2* A, int64_t lda,
           const float2* B, int64_t ldb, float2 beta, float2* C, int64_t ldc);
void dgemm(Ctx& c, int opa, int opb, int m, int n, int k, double alpha, const double* A, int64_t lda,
           const double* B, int64_t ldb, double beta, double* C, int64_t ldc);

// Periodic tridiagonal Gram matrix (diag d, off e with e[i] = G[i][i+1 mod n]).
void gram_factor(Ctx& c, const double* d, const double* e, int n, double* fac /* 3n+2 */);
template <typename T>
void gram_solve(Ctx& c, const double* e, const double* fac, int n, T* X, int64_t ncols, int64_t ld);
template <typename T>
void gram_mul(Ctx& c, const double* d, const double* e, int n, const T* X, int64_t ncols, int64_t ldx,
              double a, double b, T* Y, int64_t ldy);
constexpr int GW = 64;   // half-bandwidth of the truncated G^{-1}
void gram_band_build(Ctx& c, const double* d, const double* e, int n, double* band /* (2GW+1) n */);
template <typename T>
void gram_band_apply(Ctx& c, const double* band, int n, const T* X, int64_t ncols, T* Y);
std::vector<double> cheb_coeffs(int p, double lo, double hi);
// G^{p/2} (p = +-1) of a homogeneous mesh (panel length h) as a band (gram_band_apply layout)
void gram_circ_band(Ctx& c, double h, int n, int p, double* band /* (2GW+1) n */);
template <typename T>
void gram_pow_half(Ctx& c, const double* d, const double* e, int n, double lo, double hi, int p, T* X,
                   int64_t ncols);

// Inverse of a complex r x r column-major matrix (A is left unchanged).
// stats[0] = min |pivot|, stats[1] = max |A|.
// stats (host, 2): min |pivot| and max |A| entry; waits for the device
void gj_inverse(Ctx& c, double2* A, double2* Ainv, int r, double* stats);

void real_to_complex(Ctx& c, const double* x, double2* y, int64_t n);
void daxpby(Ctx& c, double a, const double* x, double b, double* y, int64_t n);
void axpby(Ctx& c, double2 a, const double2* x, double2 b, double2* y, int64_t n);
void add_diag(Ctx& c, double2* A, int n, double s);

}  // namespace fds
