// Dense building blocks of the truncating skeleton compression (lowrank.hip).
#pragma once
#include "fds_internal.h"

namespace fds {

// Omega (n x ell, column-major) of the counter-based SplitMix64 sketch.
void sketch(Ctx& c, uint64_t seed, int64_t n, int ell, double2* Om);

// QR of A (M x m column-major, ld M, M >= m) with the explicit orthonormal
// factor Q (M x m): CholeskyQR2 (when allowed) if it certifies itself, else blocked
// Householder. The upper triangle of A receives R; what lies below it is left
// unspecified. tau[m] is workspace.
// Returns true when CholeskyQR2 produced the result.
// basis_only: Q need only be a well-conditioned basis of range(A) (the
// CholeskyQR path then stops after its first pass, certified ||Q^H Q - I||_F < 1/2;
// A = Q R still holds); Householder always returns an orthonormal Q.
bool qr_explicit(Ctx& c, double2* A, int M, int m, double2* tau, double2* Q, bool cholesky = true,
                 bool basis_only = false);
// X (m x m) = R^H from a factored A.
void r_adjoint(Ctx& c, const double2* A, int M, int m, double2* X);

// One-sided Jacobi SVD of the square X (m x m, overwritten): X = U diag(sig) V^H
// with sig descending. Uo, Vo: m x m outputs. Returns the sweep count;
// throws FDS_ERR_NOCONV after max_sweeps.
int jacobi_svd(Ctx& c, double2* X, int m, double2* Uo, double2* Vo, double* sig, int max_sweeps);

void conj_copy(Ctx& c, const double2* x, double2* y, int64_t n);
void scale_cols(Ctx& c, double2* X, int64_t rows, int cols, const double* s);

}  // namespace fds
