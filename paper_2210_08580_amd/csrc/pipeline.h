// Pipeline stages behind the C ABI (see pipeline.hip).
#pragma once
#include "fds_internal.h"

namespace fds {

void ensure_gram_factor(Op& op);
void apply_gram_power(Op& op, int p, double2* X, int64_t ncols);
const double* filter_basis_view(Op& op);
void run_filter(Op& op, int form, double alpha, int n_modes, bool keep_null, double cluster_rtol);
void prefetch_filter(Op& op, int n_modes);
void run_filter_batch(Op* const* ops, int count, int form, double alpha, const int* n_modes, bool keep_null,
                      double cluster_rtol);
void run_compress(Op& op, int rank_cap, int oversample, int power_iters, double tol, uint64_t seed,
                  bool householder = false);
void run_compress_aca(Op& op, int rank_cap, double tol);   // aca.hip
void run_factor(Op& op);
void run_rhs_system(Op& op, int form, double alpha, const double2* f, const double2* h, int64_t nrhs,
                    double2* w);
void run_solve_system(Op& op, const double2* w, int64_t nrhs, double2* j_out, double2* y_out, int max_iters,
                      double tol, fds_solve_stats* stats, bool unfiltered, bool adjoint = false);
void run_solve(Op& op, const double2* f, const double2* h, int64_t nrhs, double2* j_out, double2* y_out,
               int max_iters, double tol, fds_solve_stats* stats, bool unfiltered = false);
void gram_inv(Op& op, const double2* X, int64_t ncols, double2* Y);
void run_solve_adjoint(Op& op, const double2* v, int64_t nrhs, double2* y_out, double2* u_out, int max_iters,
                       double tol, fds_solve_stats* stats, bool unfiltered);
// allocation-free Woodbury solve + filtered refinement sweeps (static scratch array)
void init_noalloc_scratch(Ctx& c);
void run_solve_system_noalloc(Op& op, const double2* w, int64_t nrhs, double2* j_out, int sweeps);
void run_solve_system_ws(Op& op, const double2* w, int64_t nrhs, double2* j_out, int sweeps, void* ws,
                         size_t ws_bytes);
// one problem of a batch (capture-safe: no allocation, no host read)
struct BatchItem {
    const double* angles;
    const double2* amps;
    int64_t nrhs;
    double2 *f, *h, *w, *t, *j;
};
void run_batch_item(Op& op, const BatchItem& it, int sweeps, void* ws, size_t ws_bytes);
// adjoint.hip
void run_farfield(Op& op, const double2* J, int64_t nrhs, const double* thetas, int nang, double2* out);
void run_farfield_grad(Op& op, const double* angles, const double2* amps, int64_t nrhs, const double* thetas,
                       int nang, const double2* T, int max_iters, double tol, double* Jout, double* grad,
                       double2* gamp, double2* ff_out, fds_solve_stats* stats);

}  // namespace fds
