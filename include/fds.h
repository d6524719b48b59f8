/*
 * fds.h -- C ABI of the filtered fast direct solver for the 2D TE-EFIE /
 * TE-MFIE / TE-CFIE on AMD Instinct MI355X (gfx950).
 *
 * Method: C. Henry et al., "Fast Direct Solvers for Integral Equations at
 * Low-Frequency Based on Operator Filtering" (arXiv 2210.08580). Section
 * names below refer to that paper.
 *
 * Pipeline and state machine (calls out of order return FDS_ERR_STATE):
 *     fds_assemble -> fds_filter -> fds_compress -> fds_factor -> fds_solve
 * fds_rhs_planewave and the fds_op_* views are valid from ASSEMBLED on.
 *
 * Conventions
 *   - Every pointer argument named "device" is a device address on the
 *     context's GPU; "host" pointers are ordinary host memory.
 *   - Complex numbers are interleaved (re, im) doubles (complex128).
 *   - N x N operator matrices are row-major. Blocks of vectors (right-hand
 *     sides, solutions, filter basis) are stored vector after vector: a block
 *     of m vectors of length N is m contiguous runs of N entries.
 *   - All work is enqueued on the context's HIP stream and is asynchronous
 *     unless stated otherwise; fds_sync waits for it and reports
 *     asynchronous device errors.
 *   - Inputs are borrowed: the library never frees caller memory. An fds_op
 *     owns its device workspace until fds_op_destroy.
 *   - No C++ exception crosses this interface. On failure a call returns a
 *     non-zero status and fds_last_error() (thread-local) describes it.
 */
#ifndef FDS_H
#define FDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fds_status {
    FDS_OK = 0,
    FDS_ERR_ARG = 1,       /* invalid argument (sizes, NULL, bad geometry)       */
    FDS_ERR_ALLOC = 2,     /* device allocation failed                            */
    FDS_ERR_HIP = 3,       /* a HIP runtime call failed                           */
    FDS_ERR_STATE = 4,     /* call made out of pipeline order                     */
    FDS_ERR_SINGULAR = 5,  /* Woodbury core numerically singular                  */
    FDS_ERR_NOCONV = 6,    /* refinement did not reach the requested tolerance    */
    FDS_ERR_NOTIMPL = 7    /* option not implemented                              */
} fds_status;

typedef struct fds_ctx_s* fds_ctx;
typedef struct fds_op_s* fds_op;

/* Optional device allocator (e.g. a framework's caching allocator). alloc
 * returns a device pointer of at least `bytes` usable on `stream`, or NULL. */
typedef struct fds_allocator {
    void* (*alloc)(size_t bytes, void* stream, void* user);
    void (*release)(void* ptr, void* stream, void* user);
    void* user;
} fds_allocator;

typedef enum fds_form {
    FDS_EFIE = 0,   /* normalised Calderon TE-EFIE, beta = 1/4                 */
    FDS_MFIE = 1,   /* normalised TE-MFIE, beta = 1/2                          */
    FDS_CFIE = 2,   /* EFIE + alpha MFIE, beta = (1 + 2 alpha)/4                */
    FDS_YCFIE = 3   /* filtered Yukawa-Calderon TE-CFIE (paper, Filters Based
                       Fast Direct Solver, 2D case): the CFIE with the single
                       layer of the Calderon product and of v_e taken at the
                       imaginary wavenumber i k, kernel (1/2 pi) K0(k R);
                       beta = (1 + 2 alpha)/4. The Yukawa operator is assembled
                       (FP64) by the first fds_rhs_system or fds_filter call
                       with this form; not available in fds_filter_batch
                       (fds_batch_create filters such batches per problem). */
} fds_form;

/* Arithmetic of the stored operators. There is no reduced-precision sketch:
 * the randomised range finder works in the coordinates of the kept filter
 * modes, where each sketch product is N x n_eff x l (a small fraction of the
 * N^2 operator products), and its accuracy bounds the skeleton, whose errors
 * only the full-cost refinement sweeps could remove. */
typedef enum fds_precision { FDS_FP64 = 0, FDS_FP32 = 1 } fds_precision;

typedef struct fds_asm_opts {
    int32_t nquad;       /* Gauss points per panel; only 8 is supported          */
    int32_t precision;   /* FDS_FP64: complex128 operators;
                            FDS_FP32: complex64 operators, far-pair kernel values
                            and accumulation in FP32 (distances and Bessel
                            arguments in FP64), self/adjacent-pair quadrature in
                            FP64, N and S near the diagonal in FP64 (band_width);
                            the products with S, N, D widen the complex64
                            operands and run on the FP64 matrix cores        */
    int32_t band_width;  /* FDS_FP32 only: half-width w of the cyclic band
                            |i - j| <= w on which N (and S) are computed in FP64,
                            N kept in complex128 (fds_op_nband); 0 = default
                            (63 up to 8192 panels, n/64 - 1 above); clipped to
                            (n-1)/2 */
    int32_t filter_modes; /* 0, or the filtering point n_modes of a coming
                            fds_filter (null mode kept): the Laplacian
                            eigensolver needs only the mesh, so its bisection
                            is started here on the context's second stream and
                            runs beside the dense assembly; fds_filter with
                            that n_modes and keep_nullspace = 1 continues from
                            it (any other filter call discards it) */
    int32_t reserved[4];
} fds_asm_opts;

typedef struct fds_filter_opts {
    int32_t n_modes;          /* filtering point n: number of kept Laplacian modes */
    int32_t keep_nullspace;   /* 1: keep the constant (null) mode (default)        */
    double cluster_rtol;      /* grow n while the cut splits eigenvalues closer
                                 than this relative gap (default 1e-6)            */
} fds_filter_opts;

typedef struct fds_compress_opts {
    int32_t rank_cap;      /* r: maximal skeleton rank                           */
    int32_t oversample;    /* p: sketch width l = r + p                          */
    int32_t power_iters;   /* q: subspace iterations                             */
    int32_t precision;     /* FDS_FP64                                           */
    double tol;            /* eps: keep sigma_i > eps sigma_1 (0: rank cap only)  */
    uint64_t seed;         /* sketch seed (SplitMix64 counter rule)              */
    int32_t qr;            /* orthonormalisation of the sketch and projected
                              blocks: FDS_QR_AUTO (CholeskyQR2 when the block
                              has at most 140 columns and the factorisation
                              certifies itself, else Householder) or
                              FDS_QR_HOUSEHOLDER (always blocked Householder) */
    int32_t reserved;
} fds_compress_opts;

enum { FDS_QR_AUTO = 0, FDS_QR_HOUSEHOLDER = 1 };

typedef struct fds_solve_opts {
    int32_t max_iters;     /* refinement sweeps after the Woodbury solve          */
    int32_t precision;     /* FDS_FP64                                           */
    double tol;            /* stop when max_r ||v_r - A y_r|| / ||v_r|| <= tol    */
    int32_t unfiltered;    /* 0: refine against the filtered operator beta I + P C
                              (the paper's filtered solution); 1: against the
                              unfiltered beta I + C, so that the iteration
                              converges to the Galerkin solution of N j = -f
                              (EFIE), (G/2 - D) j = -h (MFIE); the filtered
                              Woodbury solve is then the preconditioner        */
    int32_t reserved;
} fds_solve_opts;

typedef struct fds_solve_stats {
    int32_t iters;         /* refinement sweeps done                              */
    int32_t converged;     /* 1 if the tolerance was met                          */
    double relres;         /* final max relative residual                         */
    double history[32];    /* residual after the Woodbury solve and each sweep    */
} fds_solve_stats;

/* ---------------------------------------------------------------- context */

/* Creates a context on GPU `device`; all work is ordered on `hip_stream`
 * (a hipStream_t; NULL = the default stream). `alloc` may be NULL (the
 * library then uses hipMalloc/hipFree). Device memory that the library frees
 * stays in the context's cache (per stream and size class) for its next
 * allocations; the cache is handed back to `alloc` when an allocation fails
 * and when the context is destroyed. Allocations made while the stream is
 * being captured into a graph bypass the cache. */
fds_status fds_ctx_create(int device, void* hip_stream, const fds_allocator* alloc,
                          fds_ctx* out);
/* Waits for the context's streams, returns its cached memory and destroys it
 * (operators of the context must be destroyed first). */
fds_status fds_ctx_destroy(fds_ctx ctx);
/* Waits for all enqueued work; reports asynchronous device errors. */
fds_status fds_sync(fds_ctx ctx);
/* Thread-local description of the last failure of this thread. */
const char* fds_last_error(void);

/* Per-kernel timing with HIP events on the context's stream (off by default).
 * While enabled, every kernel launch of the library is bracketed by two
 * events; fds_profile_read resolves them (it synchronises the stream),
 * accumulates per kernel name and clears the accumulators.
 * names: host buffer of cap x 32 chars (NUL-terminated names), total_ms and
 * launches: host arrays of cap entries; *count receives the number of names. */
fds_status fds_profile_enable(fds_ctx ctx, int32_t on);
fds_status fds_profile_read(fds_ctx ctx, int32_t cap, char* names, double* total_ms,
                            int64_t* launches, int32_t* count);

/* GEMM autotuning (off by default). When on, the first GEMM of each shape
 * class (operand types, ops, m, n, k rounded up to powers of two) times the
 * split-K candidates 1, 2, 4, ... (the K extent per workgroup) on a scratch
 * output, synchronising, and caches the fastest in the context; later GEMMs of
 * the class reuse it. Nothing is tuned while the stream is being captured. */
fds_status fds_autotune(fds_ctx ctx, int32_t on);
/* Copies the cache: keys (host, cap x 160 chars, may be NULL), split_k (host,
 * cap ints, may be NULL); *count receives the number of entries. */
fds_status fds_autotune_read(fds_ctx ctx, int32_t cap, char* keys, int32_t* split_k, int32_t* count);

/* ------------------------------------------------------- special functions */

/* Bessel functions of the Hankel kernel (paper, Notation and Background:
 * g2 = (i/4) H0^(1)(k|r - r'|)), by the FP64 evaluator of the far-pair assembly.
 * x: device [n] doubles, x > 0. out: device [n][4] doubles = J0, Y0, J1, Y1 at each x. */
fds_status fds_hankel_eval(fds_ctx ctx, const double* x, int64_t n, double* out);

/* Single-precision evaluation used by the FP32 far-field assembly (scaled
 * error below 2e-7 max(|f|, 1)); x: device [n] doubles, out: device [n][4] floats. */
fds_status fds_hankel_eval_f32(fds_ctx ctx, const double* x, int64_t n, float* out);

/* Kernel values used by the Galerkin quadrature at distances R (device [n],
 * R >= 0). out: device [n][8] doubles =
 *   g(R) = (i/4) H0^(1)(kR)                           (re, im)  (R > 0)
 *   g(R) + log(R)/(2 pi), continuous at R = 0          (re, im)
 *   c(R) = (ik/4) H1^(1)(kR)/R, dg/dn_y = c (x-y).n_y  (re, im)  (R > 0)
 *   c(R) - 1/(2 pi R^2)                                (re, im)  (R > 0)  */
fds_status fds_kernel_eval(fds_ctx ctx, double k, const double* R, int64_t n,
                           double* out);

/* The Yukawa kernel of the Yukawa-Calderon TE-CFIE (the 2D Helmholtz kernel at
 * the imaginary wavenumber i kappa) at distances R (device [n], R >= 0).
 * out: device [n][2] doubles =
 *   (1/2 pi) K0(kappa R)                               (R > 0; 0 at R = 0)
 *   (1/2 pi) (K0(kappa R) + log R), continuous at R = 0 */
fds_status fds_yukawa_eval(fds_ctx ctx, double kappa, const double* R, int64_t n, double* out);

/* ------------------------------------------------------------ mesh generation */

/* Equal-chord (homogeneous) mesh of a closed curve (paper, Laplacian Filters,
 * Two-Dimensional Case: on a homogeneously discretised curve the filter is
 * diagonalised by the DFT; fds_filter then builds it in closed form). The curve
 * is the trigonometric polynomial
 *     x(t) = sum_{m=0}^{degree} ax[m] cos(m t) + bx[m] sin(m t),  y(t) likewise,
 * t in [0, 2 pi), counter-clockwise and simple. Returns in nodes (host, [n][2])
 * the points r(t_0 = 0), r(t_1), ..., r(t_{n-1}), 0 < t_1 < ... < t_{n-1} < 2 pi,
 * whose n chords |r(t_{i+1}) - r(t_i)| (cyclic) are equal, and that length in
 * *chord (may be NULL). ax, bx, ay, by: host [degree + 1] doubles (bx[0], by[0]
 * unused). 4 <= n <= 2^24, 1 <= degree <= 4096. Runs on the host (no context,
 * no GPU); FDS_ERR_ARG if no such mesh is found (e.g. a self-intersecting curve). */
fds_status fds_equal_chord_nodes(int32_t degree, const double* ax, const double* bx, const double* ay,
                                 const double* by, int64_t n, double* nodes, double* chord);

/* Complex GEMM on the FP64 matrix cores (the dense contractions of the
 * compression and solve stages run on this kernel):
 *   C = alpha op(A) op(B) + beta C,  column-major, C is m x n, inner size k,
 *   op in {0: none, 1: transpose, 2: conjugate transpose}.
 * A, B, C: device complex128 with leading dimensions lda, ldb, ldc; alpha and
 * beta: host complex128 (2 doubles each). C must not alias A or B. */
fds_status fds_zgemm(fds_ctx ctx, int32_t opa, int32_t opb, int64_t m, int64_t n, int64_t k,
                     const double* alpha, const void* A, int64_t lda, const void* B, int64_t ldb,
                     const double* beta, void* C, int64_t ldc);

/* Inverse of a dense complex128 r x r matrix by the routine that inverts the
 * Woodbury core I + W U / beta (paper, Inversion of the structured matrices):
 * blocked Gauss-Jordan, first without row interchanges and kept when
 * max |A Ainv - I| <= 8 eps r, else with partial pivoting. A and Ainv: device,
 * column-major, leading dimension r, caller-owned, not aliased (A is not
 * modified). stats (host, 2 doubles, may be NULL): min |pivot| and max |A|; a
 * caller treats A as singular when stats[0] < 64 eps stats[1].
 * FDS_ERR_ARG for r < 1 or NULL pointers, FDS_ERR_NOTIMPL for r > 2048.
 * Synchronises the context stream. Test and diagnostic entry point. */
fds_status fds_zinv(fds_ctx ctx, int64_t r, const void* A, void* Ainv, double* stats);

/* QR of a dense complex128 M x m matrix (M >= m >= 1) with the explicit
 * orthonormal factor, by the routine that orthonormalises the sketch and the
 * projected block in fds_compress (paper, Inversion of the structured
 * matrices: the orthonormal basis of the sampled range). method: FDS_QR_AUTO
 * (CholeskyQR2 for m <= 140 when ||Q1^H Q1 - I||_F < 1/2 after its first pass
 * and every pivot is positive, else Householder) or FDS_QR_HOUSEHOLDER.
 * A: device, column-major, leading dimension M, caller-owned; overwritten, its
 * upper triangle receives R (what lies below is unspecified). Q: device, M x m,
 * leading dimension M, caller-owned, not aliased with A. householder_used
 * (host, may be NULL): 1 when the Householder factorisation produced the
 * result. FDS_ERR_ARG for bad sizes, NULL pointers or method. Synchronises the
 * context stream. Test and diagnostic entry point. */
fds_status fds_zqr(fds_ctx ctx, int64_t M, int64_t m, void* A, void* Q, int32_t method,
                   int32_t* householder_used);

/* fds_zgemm for complex64 operands on the FP32 matrix cores (FP32 accumulation);
 * alpha and beta: host complex64 (2 floats each). */
fds_status fds_cgemm(fds_ctx ctx, int32_t opa, int32_t opb, int64_t m, int64_t n, int64_t k,
                     const float* alpha, const void* A, int64_t lda, const void* B, int64_t ldb,
                     const float* beta, void* C, int64_t ldc);

/* ---------------------------------------------------------------- assembly */

/* Dense Galerkin assembly (paper, Notation and Background: [S]_ij, [N]_ij,
 * [D]_ij with the P1 hat basis on a straight-segment mesh; N in Maue's
 * integrated-by-parts form) plus the Gram matrix G and the Laplacian L
 * (paper, Laplacian Filters, 2D case).
 * nodes: device [n][2] doubles, counter-clockwise, closed (panel i joins
 *        node i to node i+1 mod n), no repeated node; 8 <= n.
 * k:     wave number > 0.
 * opts:  may be NULL (defaults: nquad 8, FP64).
 * out:   receives a new operator owning S, N, D (3 n^2 complex128, or
 *        complex64 with FDS_FP32).
 * Errors: FDS_ERR_ARG for bad sizes/k or a zero-length / non-finite panel,
 * FDS_ERR_ALLOC when the matrices do not fit. */
fds_status fds_assemble(fds_ctx ctx, const double* nodes, int64_t n, double k,
                        const fds_asm_opts* opts, fds_op* out);
fds_status fds_op_destroy(fds_op op);

/* Batched assembly of `count` FP64 operators of uneven sizes (nodes[j]: device
 * [n[j]][2], k[j]; host arrays of pointers / sizes / wave numbers): the far
 * panel pairs of all operators are processed by one persistent launch whose
 * wavefronts draw 63 x 63 half-tiles from a shared work queue; the near pairs
 * and band corrections follow per operator. Same results as fds_assemble on
 * each operator. out: host array of `count` handles; on error none is created. */
fds_status fds_assemble_batch(fds_ctx ctx, int32_t count, const double* const* nodes, const int64_t* n,
                              const double* k, fds_op* out);

/* ------------------------------------------------------------------ batches
 * Many problems in one call (paper, Filters Based Fast Direct Solver: the
 * factorisation is computed once per geometry and reused for every right-hand
 * side; Inversion of the structured matrices). A batch assembles the operators
 * of all curves by one persistent far-field launch, filters, compresses and
 * factors each of them, and then records the plane-wave right-hand sides, the
 * Woodbury solves and a fixed number of refinement sweeps of every problem in
 * one HIP graph, which each fds_batch_replay launches at once. The set-up is
 * not in the graph: the number of kept modes (cut guard) and the skeleton rank
 * are decided from computed eigenvalues and singular values. */
typedef struct fds_problem {
    const double* nodes;   /* device [n][2], as for fds_assemble                 */
    int64_t n;             /* panels, >= 8                                       */
    double k;              /* wave number > 0                                    */
    int32_t n_modes;       /* filtering point n in [1, n]                        */
    int32_t nrhs;          /* plane waves, >= 1                                  */
    const double* angles;  /* device [nrhs] directions (radians); read at every
                              replay                                             */
    const void* amps;      /* device [nrhs] complex128 amplitudes; read at every
                              replay                                             */
    void* j_out;           /* device [nrhs][n] complex128: the current
                              coefficients j, written at every replay            */
} fds_problem;

typedef struct fds_batch_opts {
    int32_t precision;     /* FDS_FP64 or FDS_FP32 (as fds_asm_opts.precision;
                              default band width)                                */
    int32_t form;          /* fds_form                                           */
    double alpha;          /* CFIE coupling (FDS_CFIE, FDS_YCFIE)                */
    int32_t rank_cap;      /* skeleton rank cap; 0: each problem's n_eff (exact
                              skeleton)                                          */
    int32_t oversample;    /* p (fds_compress_opts)                              */
    int32_t power_iters;   /* q                                                  */
    int32_t sweeps;        /* refinement sweeps after each Woodbury solve, against
                              the filtered operator (fixed count, no residual
                              test: nothing is read back by the host)            */
    double tol;            /* compression tolerance eps                          */
    uint64_t seed;         /* sketch seed                                        */
    int32_t reserved[4];
} fds_batch_opts;

typedef struct fds_batch_s* fds_batch;

/* Builds the batch: batched assembly (all far tiles of all problems in one
 * persistent launch; FP32 operators add their FP64 band of N per problem),
 * filter (FP64 EFIE/MFIE/CFIE: grouped products over all problems), skeleton
 * compression and Woodbury factor per problem, one eager run of every solve,
 * then the capture of those solves into one graph. Right-hand-side and
 * solution buffers are the caller's (probs[i].angles, amps, j_out) and must
 * stay valid until fds_batch_destroy; the library allocates the per-problem
 * right-hand-side workspace (4 n nrhs complex128 per problem, 3 for the EFIE)
 * and the workspace of the graph's branches: the problems are spread over up
 * to 8 independent branches (largest n^2 nrhs first, each to the least loaded
 * branch), which the device may run side by side. Replays of one batch must
 * not overlap each other. Errors: FDS_ERR_ARG for bad sizes or options,
 * FDS_ERR_SINGULAR from a factor, FDS_ERR_HIP if the capture fails; on error
 * nothing is created. Synchronises the stream. */
fds_status fds_batch_create(fds_ctx ctx, int64_t nb, const fds_problem* probs, const fds_batch_opts* opts,
                            fds_batch* out);
/* One launch of the recorded graph on the context's stream: the right-hand
 * sides from the current angles and amplitudes, the Woodbury solve and the
 * sweeps of every problem, j written to each j_out. Asynchronous. */
fds_status fds_batch_replay(fds_batch b);
/* Borrowed operator of problem i (for fds_op_info and the views); valid until
 * fds_batch_destroy. */
fds_status fds_batch_op(fds_batch b, int64_t i, fds_op* op);
/* Waits for the context's stream, then frees the graph, the operators and the
 * workspace. */
fds_status fds_batch_destroy(fds_batch b);
/* fds_batch_create, one fds_batch_replay, a stream synchronisation and
 * fds_batch_destroy: the nb problems solved end to end in one call. */
fds_status fds_batch_run(fds_ctx ctx, int64_t nb, const fds_problem* probs, const fds_batch_opts* opts);

/* Sizes: n, kept filter modes (0 before fds_filter), skeleton rank (0 before
 * fds_compress). Any output pointer may be NULL. Host call, no sync. */
fds_status fds_op_info(fds_op op, int64_t* n, int32_t* n_eff, int32_t* rank);

/* Borrowed device views of S, N, D ([n][n] row-major; complex128, or
 * complex64 for an operator assembled with FDS_FP32). */
fds_status fds_op_matrices(fds_op op, void** S, void** Nmat, void** D);

/* FP32 operators only (NULL and width 0 otherwise): borrowed device view of
 * N on the cyclic band |d| <= w, w = min(63, (n - 1)/2), in complex128:
 * [n][2w + 1] with N[i][(i + d) mod n] at [i][d + w]. The complex64 N returned
 * by fds_op_matrices holds zeros on this band. The Galerkin matrix of the
 * hypersingular operator has O(1) entries near the diagonal but eigenvalues
 * O(h) on smooth vectors, so FP32 errors there would be amplified by 1/h;
 * the band is computed and kept in FP64. Host call. */
fds_status fds_op_nband(fds_op op, const void** Nband, int32_t* width);

/* Borrowed device view of the Yukawa single layer S_y of the Yukawa-Calderon
 * TE-CFIE ([n][n] row-major complex128 with zero imaginary parts), or NULL
 * before the first fds_rhs_system / fds_filter call with FDS_YCFIE. Host call. */
fds_status fds_op_yukawa(fds_op op, const void** Sy);

/* Storage precision of S, N, D (FDS_FP64 or FDS_FP32). Host call. */
fds_status fds_op_precision(fds_op op, int32_t* precision);

/* Borrowed device views of the periodic tridiagonal G and L: diag[i] and
 * off[i] = M[i][i+1 mod n] ([n] doubles each). */
fds_status fds_op_sparse(fds_op op, const double** g_diag, const double** g_off,
                         const double** l_diag, const double** l_off);

/* X <- G^{p/2} X for p in {-2, -1, 1} (G^{-1}, G^{-1/2}, G^{1/2}); X: device,
 * ncols complex128 vectors of length n, in place. Used by the normalised
 * formulations (paper, Notation and Background). */
fds_status fds_apply_gram(fds_op op, int32_t p, void* X, int64_t ncols);

/* ------------------------------------------------------------------ filter */

/* Laplacian filter P = V_n V_n^T (paper, Laplacian Filters, eq. LapFilter,
 * with the orthonormalised Laplacian G^{-1/2} L G^{-1/2} for non-uniform
 * meshes) and the compact part of the chosen formulation (paper, Filters
 * Based Fast Direct Solver, 2D case). Builds B = V_n^T C (n_eff x n).
 * n_eff (host, may be NULL) receives the number of kept modes after the
 * cluster guard. Errors: FDS_ERR_ARG for n_modes outside [1, n], or for a CFIE
 * with alpha = -1/2 (beta = 0: no second-kind part). */
fds_status fds_filter(fds_op op, fds_form form, double alpha,
                      const fds_filter_opts* opts, int32_t* n_eff);

/* fds_filter on `count` FP64 operators of one context (uneven sizes): the
 * eigensolver runs per operator and every dense product stage of all operators
 * is one grouped GEMM launch. opts: host array of `count` (one keep_nullspace
 * and cluster_rtol per batch, taken from opts[0]); n_eff: host [count] or NULL. */
fds_status fds_filter_batch(int32_t count, fds_op* ops, fds_form form, double alpha,
                            const fds_filter_opts* opts, int32_t* n_eff);

/* Borrowed device view of V_n: n_eff orthonormal real vectors of length n. */
fds_status fds_op_filter_basis(fds_op op, const double** Vn);

/* Eigenvalues of the generalised Laplacian pencil L v = lambda G v found by the
 * last fds_filter call (ascending; kept modes first, then up to a few beyond
 * the cut). Host call: copies min(cap, available) values to host `out` and
 * stores that number in *count. Available even when fds_filter failed after
 * the eigenvalue stage. */
fds_status fds_op_filter_eigenvalues(fds_op op, double* out, int32_t cap, int32_t* count);

/* ------------------------------------------------------------- compression */

/* Randomised skeleton C_f ~ U W of the filtered compact part (paper,
 * Inversion of the structured matrices; randomised range finder with
 * subspace iteration of Halko, Martinsson & Tropp). With l = rank_cap +
 * oversample:
 *   - tol == 0, rank_cap >= n_eff, l >= n_eff: C_f has rank <= n_eff and the
 *     sketch spans its range, so the skeleton is exact (rank n_eff, no sketch
 *     is formed);
 *   - l < n_eff: Y = C_f Omega with the SplitMix64 sketch Omega (n x l,
 *     fds_compress_opts.seed), power_iters subspace iterations with
 *     re-orthonormalisation (fds_compress_opts.qr), B = Q^H C_f, SVD of B;
 *   - otherwise (l >= n_eff but truncating): SVD of C_f itself.
 * The rank is r = min(rank_cap, #{sigma_i > max(tol, 1e-13) sigma_1}), lowered
 * while sigma_r < (1 + 1e-6) sigma_{r+1} (no split of a repeated value).
 * Synchronises. rank_out (host, may be NULL) receives r. Errors: FDS_ERR_ARG
 * if l > n on the sketched branch or qr is not one of FDS_QR_*; FDS_ERR_NOCONV if the Jacobi SVD of the
 * projected block does not converge. */
fds_status fds_compress(fds_op op, const fds_compress_opts* opts, int32_t* rank_out);

/* The skeleton by adaptive cross approximation instead (paper, Inversion of the
 * structured matrices: Bebendorf's ACA is the other skeleton-detecting algorithm
 * it cites). ACA with partial pivoting of the filtered compact part in the
 * normalised coordinates, A_y = V_n B_y (N x N, read by rows and columns through
 * its two factors, never formed): first row 0; each step takes the residual
 * row, its largest entry outside the used columns as pivot, b = row / pivot, the
 * residual pivot column as a, and the next row at the largest entry of a outside
 * the used rows; it stops once ||a|| ||b|| <= tol ||S||_F (S the sum of the
 * crosses so far) or after rank_cap crosses. A residual row that vanishes is
 * skipped for the lowest unused row. fds_op_singular_values then returns the
 * cross norms ||a_k|| ||b_k||. Same stage rules and views as fds_compress.
 * Synchronises (once per cross). rank_out (host, may be NULL) receives r.
 * Errors: FDS_ERR_ARG if rank_cap < 1 or tol < 0. */
fds_status fds_compress_aca(fds_op op, int32_t rank_cap, double tol, int32_t* rank_out);

/* Singular values (descending) of the projected block B of the last
 * truncating fds_compress call (none after the exact skeleton), or after
 * fds_compress_aca the cross norms ||a_k|| ||b_k|| in step order. Host call:
 * copies min(cap, available) values to host `out`, the number to *count. */
fds_status fds_op_singular_values(fds_op op, double* out, int32_t cap, int32_t* count);

/* Borrowed device views of the skeleton in current-coefficient coordinates:
 * with U_y W_y the skeleton of the filtered compact part of the normalised
 * system (unknown y = G^{1/2} j), U = G^{-1/2} U_y (r vectors of length n) and
 * W = W_y G^{1/2}, returned transposed (r vectors of length n holding the rows
 * of W). Both complex128. The Woodbury core I_r + W U / beta is the same in
 * both coordinates. */
fds_status fds_op_factors(fds_op op, const void** U, const void** W, int32_t* rank);

/* ----------------------------------------------------------------- factor */

/* Inverse of the Woodbury core K = I_r + beta^{-1} W U (paper, Inversion of
 * the structured matrices) by blocked Gauss-Jordan elimination: first without
 * row interchanges, kept when max |K K^{-1} - I| <= 8 eps r; otherwise redone
 * with partial pivoting. K^{-1} is folded into the skeleton (U K^{-1}), so a
 * solve is two products. Synchronises once to check the residual and the
 * pivots; FDS_ERR_SINGULAR if min|pivot| < 64 eps max|K|. */
fds_status fds_factor(fds_op op);

/* -------------------------------------------------------------------- RHS */

/* Plane waves u = A exp(i k d.x), d = (cos phi, sin phi) (paper, Notation and
 * Background: e_2, h_2 moments; plane waves stand in for the paper's dipole).
 * angles: device [nrhs] doubles; amps: device [nrhs] complex128.
 * f_out: device [nrhs][n] complex128, f_i = <phi_i, du/dn>   (may be NULL)
 * h_out: device [nrhs][n] complex128, h_i = <phi_i, u>       (may be NULL) */
fds_status fds_rhs_planewave(fds_op op, const double* angles, const void* amps,
                             int64_t nrhs, void* f_out, void* h_out);

/* ------------------------------------------------------------------ solve */

/* Solves (beta I + P C) y = v for nrhs right-hand sides built from f and h
 * (EFIE v = -G^{-1/2} S G^{-1} f, MFIE v = -G^{-1/2} h, CFIE v_e + alpha v_h)
 * with the Woodbury inverse of beta I + U W, then FP64 iterative refinement
 * against beta I + P C, and returns j = G^{-1/2} y.
 * f, h: device [nrhs][n] complex128 (the one the formulation does not use may
 * be NULL). j_out, y_out: device [nrhs][n] complex128 (y_out may be NULL).
 * opts may be NULL (defaults: max_iters 4, tol 1e-12). stats (host, may be
 * NULL) makes the call synchronous and reports the residual history.
 * FDS_ERR_NOCONV if stats is given and the tolerance was not met. */
fds_status fds_solve(fds_op op, const void* f, const void* h, int64_t nrhs,
                     void* j_out, void* y_out, const fds_solve_opts* opts,
                     fds_solve_stats* stats);

/* The solve in two parts, so that the dense right-hand-side product can be
 * enqueued right after fds_assemble and run on the device beside the filter's
 * eigensolver (whose kernels leave most of the chip idle).
 *
 * fds_rhs_system: w = G^{-1/2} v, the right-hand side in current coefficients
 * (paper, Notation and Background: the moments e_2, h_2 and the Calderon
 * normalisation): EFIE w = -G^{-1} S G^{-1} f, MFIE w = -G^{-1} h, CFIE the EFIE
 * one + alpha times the MFIE one. Valid from ASSEMBLED on; form and alpha must
 * be those the later fds_filter call uses. f, h, w_out: device [nrhs][n]
 * complex128 (the input the formulation does not use may be NULL; w_out may
 * not alias f or h). Asynchronous.
 *
 * fds_solve_system: fds_solve from w (fds_rhs_system output): the Woodbury
 * solve, refinement, outputs, opts and stats exactly as fds_solve. */
fds_status fds_rhs_system(fds_op op, fds_form form, double alpha, const void* f, const void* h,
                          int64_t nrhs, void* w_out);
fds_status fds_solve_system(fds_op op, const void* w, int64_t nrhs, void* j_out, void* y_out,
                            const fds_solve_opts* opts, fds_solve_stats* stats);

/* The adjoint solve (paper, Inversion of the structured matrices: the Woodbury
 * identity of beta I + U W, here of its conjugate transpose beta I + W^H U^H):
 * solves (beta I + P C)^H y = v for the filtered operator of the last
 * fds_filter call (opts->unfiltered = 1: of beta I + C, the operator of the
 * normalised formulation, whose adjoint solution is that of the Galerkin system
 * transposed and conjugated). The adjoint Woodbury solve with the conjugated
 * skeleton and core, then FP64 refinement against the adjoint operator
 * (max_iters, tol as in fds_solve), in y-coordinates (the paper's normalised
 * unknowns, y = G^{1/2} j). v: device [nrhs][n] complex128; y_out: device
 * [nrhs][n] complex128; u_out: device [nrhs][n] complex128 or NULL, receives
 * G^{-1/2} y (the adjoint's current coefficients). Outputs may not alias v.
 * opts may be NULL (max_iters 4, tol 1e-12). stats: as in fds_solve
 * (FDS_ERR_NOCONV if given and the tolerance was not met). Requires a factored
 * operator. */
fds_status fds_solve_adjoint(fds_op op, const void* v, int64_t nrhs, void* y_out, void* u_out,
                             const fds_solve_opts* opts, fds_solve_stats* stats);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): fds_solve_system with
 * stats == NULL, y_out == NULL, refinement against the filtered operator and
 * max_iters = sweeps, computed without any device allocation. Its work space
 * is a static device array of 32 MiB inside the library (one per GPU, held
 * until the process ends): the right-hand sides are processed in blocks of cb
 * columns, 16 (n + max(rank, n_eff)) cb bytes in 24 MiB of it, the split-K
 * partial sums of the products in the rest. Calls that overlap on one GPU
 * (from several threads or streams, any context) share that array and race;
 * the caller serialises them. w, j_out: device [nrhs][n] complex128 (j_out may
 * not alias w). Asynchronous. Requires a factored operator. Errors:
 * FDS_ERR_ARG for sweeps outside [0, 1000] or when one right-hand side does
 * not fit (16 (n + max(rank, n_eff)) > 24 MiB). */
fds_status fds_solve_system_noalloc(fds_op op, const void* w, int64_t nrhs, void* j_out, int32_t sweeps);

/* --------------------------------------------------------- inverse problem */

/* Far fields of currents j (device [nrhs][n] complex128) at angles thetas
 * (device [nang] doubles): out (device [nrhs][nang] complex128),
 *   u_inf(theta) = e^{i pi/4}/sqrt(8 pi k) int (-i k th.n_y) e^{-i k th.y} u(y) ds_y,
 * u = -sum_i j_i phi_i (the total field on the sound-hard boundary, sign of the
 * paper's TE-MFIE), th = (cos theta, sin theta), 8-point Gauss rule per panel.
 * The paper names inverse problems as a use case (Introduction) but fixes no
 * far-field formula; this is the standard 2D one (convention u_s ~ u_inf
 * e^{ikr}/sqrt(r)). */
fds_status fds_farfield(fds_op op, const void* j, int64_t nrhs, const double* thetas, int64_t nang, void* out);

/* Objective J = sum_r sum_l |u_inf,r(theta_l) - T_lr|^2 of the unfiltered
 * Galerkin TE-EFIE N j_r = -f_r with plane waves (angles [nrhs] doubles, amps
 * [nrhs] complex128, both device), and its gradient by the adjoint method:
 * one forward and one adjoint solve (the filtered Woodbury solve as the
 * preconditioner, refinement against the unfiltered operator with opts:
 * max_iters, tol), one GEMM M = mu J^T and one pass over all panel pairs that
 * recomputes the kernel (far pairs analytically, self/adjacent pairs by central
 * differences of their singular quadrature).
 * Requires a factored EFIE operator. target: device [nrhs][nang] complex128.
 * J: host double. grad_nodes: device [n][2] doubles, dJ/d(node coordinates).
 * grad_amps: device [nrhs] complex128, dJ/dRe A_r + i dJ/dIm A_r.
 * farfield_out: device [nrhs][nang] complex128 or NULL. stats: host, forward
 * solve, may be NULL. Synchronises. */
fds_status fds_farfield_objective_grad(fds_op op, const double* angles, const void* amps, int64_t nrhs,
                                       const double* thetas, int64_t nang, const void* target,
                                       const fds_solve_opts* opts, double* J, double* grad_nodes,
                                       void* grad_amps, void* farfield_out, fds_solve_stats* stats);

#ifdef __cplusplus
}
#endif
#endif /* FDS_H */
