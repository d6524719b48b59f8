// Dense building blocks of the truncating skeleton compression (lowrank.hip).
#pragma once
#include "fds_internal.h"

namespace fds {

// Omega (n x ell, column-major) of the counter-based SplitMix64 sketch.
void sketch(Ctx& c, uint64_t seed, int64_t n, int ell, double2* Om);

// Householder QR of A (M x m column-major, ld M, M >= m): A is overwritten by
// R (upper triangle) and the reflectors; tau[m]. If Q is not null it receives
// the explicit M x m orthonormal factor.
void householder_qr(Ctx& c, double2* A, int M, int m, double2* tau, double2* Q);
// X (m x m) = R^H from a factored A.
void r_adjoint(Ctx& c, const double2* A, int M, int m, double2* X);

// One-sided Jacobi SVD of the square X (m x m, overwritten): X = U diag(sig) V^H
// with sig descending. Uo, Vo: m x m outputs. Returns the sweep count;
// throws FDS_ERR_NOCONV after max_sweeps.
int jacobi_svd(Ctx& c, double2* X, int m, double2* Uo, double2* Vo, double* sig, int max_sweeps);

void conj_copy(Ctx& c, const double2* x, double2* y, int64_t n);
void scale_cols(Ctx& c, double2* X, int64_t rows, int cols, const double* s);

}  // namespace fds
