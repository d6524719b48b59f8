// Internal declarations shared by the HIP translation units of libfds.
#pragma once
#include <hip/hip_runtime.h>
#include <algorithm>

#include <cstdint>
#include <map>
#include <mutex>
#include <unordered_map>
#include <string>
#include <vector>

#include "../../include/fds.h"

namespace fds {

// ------------------------------------------------------------------ errors
struct Error {
    fds_status code;
    std::string msg;
};

void set_error(const std::string& msg);

#define FDS_HIP_TRY(expr)                                                         \
    do {                                                                          \
        hipError_t _e = (expr);                                                   \
        if (_e != hipSuccess)                                                     \
            throw ::fds::Error{FDS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)}; \
    } while (0)

#define FDS_REQUIRE(cond, code, text)                                             \
    do {                                                                          \
        if (!(cond)) throw ::fds::Error{code, text};                              \
    } while (0)

// ------------------------------------------------------------------ complex
__host__ __device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__host__ __device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// ------------------------------------------------------------------ context / operator
struct ProfRec {
    const char* name;
    hipEvent_t a, b;
};

struct Ctx {
    int device = 0;
    bool prof = false;                                    // per-kernel event timing on/off
    std::vector<ProfRec> pending;                         // recorded, not yet resolved
    std::map<std::string, std::pair<double, int64_t>> acc;  // name -> (total ms, launches)
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;   // non-blocking, default priority: work that only needs the mesh
    fds_allocator alloc{};
    bool has_alloc = false;
    const char* gemm_tag = nullptr;            // profiling name of GEMM launches (nullptr: "gemm")
    int split_hint = 0;                        // least split-K factor of the next GEMMs (0: heuristic)
    bool autotune = false;                     // time GEMM split-K candidates on first use
    std::map<std::string, int> tuned;          // shape class -> chosen split-K factor
    double* hk_tab = nullptr;     // device copy of the Bessel coefficient table
    double* hf_tab = nullptr;     // device copies of the far-field sets (quarter intervals)
    float* hf_tab32 = nullptr;
    double* gl32 = nullptr;       // 32-point Gauss-Legendre rule on [0,1]: x[32], w[32]
    double* yk_tab = nullptr;     // device copy of the K0 coefficient table (Yukawa kernel)
    float* yk_tab32 = nullptr;    // device copy of the float32 K0 interval table
    // Pinned host buffer for small device-to-host reads that are waited on at once
    // (nothing is in flight from it between uses, so it can be regrown freely).
    void* host_pin = nullptr;
    size_t host_pin_bytes = 0;
    void* pinned_host(size_t bytes) {
        if (bytes > host_pin_bytes) {
            if (host_pin) (void)hipHostFree(host_pin);
            host_pin = nullptr;
            host_pin_bytes = 0;
            const size_t nb = std::max<size_t>(bytes, 4096);
            if (hipHostMalloc(&host_pin, nb, hipHostMallocDefault) != hipSuccess) {
                host_pin = nullptr;
                return nullptr;
            }
            host_pin_bytes = nb;
        }
        return host_pin;
    }
    // Allocation-free calls (fds_solve_system_noalloc): `scratch` is this device's
    // address of the library's static scratch array (set once per device at context
    // creation). While `noalloc` is set every device allocation is refused, the
    // split-K partial sums of the GEMMs go to ws (ws_bytes) and nothing is autotuned.
    void* scratch = nullptr;
    bool noalloc = false;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // Device memory: a size-class cache in front of the allocator callback (or
    // hipMalloc), one free list per stream, so that a block is reused only on the
    // stream it was last allocated on (stream order then separates its old and new
    // uses). While the stream is being captured into a graph, allocations go to the
    // allocator directly and cached blocks freed meanwhile are never reused.
    struct Block {
        size_t bytes;
        hipStream_t stream;
        bool pooled;
    };
    std::mutex pool_mu;
    std::unordered_map<void*, Block> live;
    std::map<std::pair<hipStream_t, size_t>, std::vector<void*>> cache;
    std::vector<std::pair<void*, hipStream_t>> held;
    void* dmalloc(size_t bytes);
    void dfree(void* p);
    void release_cache();         // hands every cached (and held) block back to the allocator
    void* raw_alloc(size_t bytes, hipStream_t s);
    void raw_free(void* p, hipStream_t s);
};

// Brackets the launches made during its lifetime with two events on the
// context's stream when profiling is enabled (the times are resolved lazily).
struct KScope {
    Ctx* c = nullptr;
    const char* name = nullptr;
    hipEvent_t a = nullptr;
    KScope(Ctx& ctx, const char* n) {
        if (!ctx.prof) return;
        c = &ctx;
        name = n;
        if (hipEventCreate(&a) != hipSuccess || hipEventRecord(a, ctx.stream) != hipSuccess) a = nullptr;
    }
    ~KScope() {
        if (!a) return;
        hipEvent_t b = nullptr;
        if (hipEventCreate(&b) == hipSuccess && hipEventRecord(b, c->stream) == hipSuccess)
            c->pending.push_back({name, a, b});
    }
    KScope(const KScope&) = delete;
    KScope& operator=(const KScope&) = delete;
};

// Moves the context onto its side stream for the enclosed work, which is
// ordered after the event `after` (recorded on the main stream); on exit the
// main stream is ordered after everything the enclosed work launched. Every
// launch, copy, allocation and timing made through the context in between goes
// to the side stream, so the main stream's queued kernels keep running beside it.
// With join = false the main stream is not ordered after the enclosed work
// (a later SideStream scope, or an explicit wait, must do it).
struct SideStream {
    Ctx& c;
    hipStream_t main;
    bool join;
    SideStream(Ctx& ctx, hipEvent_t after, bool join_on_exit = true) : c(ctx), main(ctx.stream), join(join_on_exit) {
        if (!c.side && hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking) != hipSuccess) {
            c.side = nullptr;
            throw Error{FDS_ERR_HIP, "hipStreamCreateWithFlags failed"};
        }
        if (hipStreamWaitEvent(c.side, after, 0) != hipSuccess)
            throw Error{FDS_ERR_HIP, "hipStreamWaitEvent failed"};
        c.stream = c.side;
    }
    ~SideStream() {
        c.stream = main;
        if (!join) return;
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess && hipEventRecord(e, c.side) == hipSuccess &&
            hipStreamWaitEvent(main, e, 0) == hipSuccess) {
            (void)hipEventDestroy(e);
            return;
        }
        if (e) (void)hipEventDestroy(e);
        (void)hipStreamSynchronize(c.side);
    }
    SideStream(const SideStream&) = delete;
    SideStream& operator=(const SideStream&) = delete;
};

// Allocation-free mode for the enclosed work (see Ctx::noalloc).
struct NoAlloc {
    Ctx& c;
    NoAlloc(Ctx& ctx, void* ws, size_t ws_bytes) : c(ctx) {
        c.noalloc = true;
        c.ws = ws;
        c.ws_bytes = ws_bytes;
    }
    ~NoAlloc() {
        c.noalloc = false;
        c.ws = nullptr;
        c.ws_bytes = 0;
    }
    NoAlloc(const NoAlloc&) = delete;
    NoAlloc& operator=(const NoAlloc&) = delete;
};

// Sets the profiling name of the GEMM launches made during its lifetime.
struct GemmTag {
    Ctx& c;
    const char* old;
    GemmTag(Ctx& ctx, const char* t) : c(ctx), old(ctx.gemm_tag) { ctx.gemm_tag = t; }
    ~GemmTag() { c.gemm_tag = old; }
    GemmTag(const GemmTag&) = delete;
    GemmTag& operator=(const GemmTag&) = delete;
};

// Raises the split-K factor of the GEMMs enqueued in its scope to at least z.
struct SplitHint {
    Ctx& c;
    int old;
    SplitHint(Ctx& ctx, int z) : c(ctx), old(ctx.split_hint) { ctx.split_hint = z; }
    ~SplitHint() { c.split_hint = old; }
    SplitHint(const SplitHint&) = delete;
    SplitHint& operator=(const SplitHint&) = delete;
};

enum class Stage : int { Assembled = 1, Filtered = 2, Compressed = 3, Factored = 4 };

struct GaussRule8 {
    double xi[8];
    double w[8];
};

struct Op {
    Ctx* ctx = nullptr;
    int64_t n = 0;
    double k = 0.0;
    Stage stage = Stage::Assembled;
    // geometry (device)
    double* nodes = nullptr;      // [n][2]
    double* h = nullptr;          // [n]
    double* nx = nullptr;         // [n]
    double* ny = nullptr;         // [n]
    double* gx = nullptr;         // [n][8]
    double* gy = nullptr;         // [n][8]
    double* g_diag = nullptr;     // Gram diag / off
    double* g_off = nullptr;
    double* l_diag = nullptr;     // Laplacian diag / off
    double* l_off = nullptr;
    std::vector<double> h_host;   // panel lengths computed on the host from the caller's nodes: the
                                  // mesh bounds (Gershgorin, perimeter, h_max) need no device copy
    GaussRule8 rule{};
    // recorded on the main stream once the mesh arrays above are built; the first
    // filter call orders its eigensolver after it alone, not after the dense assembly
    hipEvent_t ev_mesh = nullptr;
    bool ev_mesh_fresh = false;
    // dense operators (device, row-major): complex128, or complex64 when prec == FDS_FP32
    int prec = FDS_FP64;
    double2* S = nullptr;
    double2* Nm = nullptr;
    double2* D = nullptr;
    float2* S32 = nullptr;
    float2* N32 = nullptr;
    float2* D32 = nullptr;
    double2* Sy = nullptr;        // Yukawa single layer (kernel (1/2pi) K0(k R)), complex128 with zero
                                  // imaginary parts; built by the first Yukawa-Calderon CFIE call
    double2* Nband = nullptr;     // FP32 operators: N on the cyclic band |d| <= nbw in complex128,
                                  // [n][2 nbw + 1] (N[i][(i + d) mod n] at [i][d + nbw]); N32 is zero there
    int nbw = 0;
    // filter / compact part
    int form = 0;
    double alpha = 1.0;
    double beta = 0.25;
    int32_t n_eff = 0;
    // Laplacian eigensolver started by fds_assemble (filtering-point hint) on the
    // side stream: the folded bands, the Sturm steps and the first bisection launch
    // for eigenvalues pre_start .. pre_start + pre_nw - 1, picked up by the filter
    bool pre_active = false;
    int pre_modes = 0, pre_nw = 0, pre_extra = 0;
    double* pre_Lb = nullptr;
    double* pre_Gb = nullptr;
    void* pre_steps = nullptr;
    double* pre_lam = nullptr;
    std::vector<double> filt_lam; // pencil eigenvalues of the last filter call (host)
    double* lam_dev = nullptr;    // Rayleigh-Ritz values of the kept modes, copied into filt_lam
    int32_t lam_dev_n = 0;        //   on first read (0: filt_lam is current)
    double* Vn = nullptr;         // [n_eff][n]  orthonormal eigenvectors of G^-1/2 L G^-1/2
    double* Vg = nullptr;         // [n_eff][n]  G^-1/2 Vn (G-orthonormal generalised eigenvectors)
    double2* Vgc = nullptr;       // [n_eff][n]  V_g as complex128
    double2* Bt = nullptr;        // [n_eff][n]  G^{1/2} (V_n^T C)^T (filtered compact part, j coordinates)
    // Gram power workspace: periodic tridiagonal factorisation of G
    double* gfac = nullptr;       // exact cyclic Thomas factors of G [3n+2] (small or irregular meshes)
    double* gband = nullptr;      // banded G^{-1} [(2 GW + 1) n] (regular meshes)
    double cheb_lo = 0.0, cheb_hi = 0.0;
    // homogeneous (equal-chord) mesh: all panel lengths within kHomogTol of their mean
    // h_mean; G and L are then circulant, the filter modes are the DFT modes, and
    // G^{+-1/2} are circulants applied as bands (gpow[0]: p = -1, gpow[1]: p = +1)
    bool homog = false;
    double h_mean = 0.0;
    double* gpow[2] = {nullptr, nullptr};
    // skeleton and Woodbury core
    int32_t rank = 0;
    std::vector<double> sv;       // singular values of the last truncating compression (host)
    double2* U = nullptr;         // [rank][n]  U_j = G^{-1/2} U_y
    double2* W = nullptr;         // [rank][n]  row t of W_j = W_y G^{1/2} (stored as W_j^T, n x rank)
    bool owns_uw = false;         // U/W are separate allocations (else views of Vgc/Bt)
    double2* K = nullptr;         // [rank][rank] Woodbury core inverse K^{-1} (column-major)
    double2* Up = nullptr;        // [rank][n]  U_j K^{-1}
    double2* Btr = nullptr;       // Bt as an n_eff x n column-major matrix (rows of Bt^T), for untransposed products
    double2* Wr = nullptr;        // W likewise, rank x n (aliases Btr when W is Bt)
    int32_t* piv = nullptr;       // [rank]
    ~Op();
};

// ------------------------------------------------------------------ launchers
// geometry.hip
void launch_geometry(Op& op);
void launch_rhs_planewave(Op& op, const double* angles, const double2* amps, int64_t nrhs,
                          double2* f, double2* h);
void launch_hankel_eval(Ctx& c, const double* x, int64_t n, double* out);
void launch_hankel_eval_f32(Ctx& c, const double* x, int64_t n, float* out);
void launch_kernel_eval(Ctx& c, double k, const double* R, int64_t n, double* out);
void launch_yukawa_eval(Ctx& c, double kappa, const double* R, int64_t n, double* out);
// Relative spread of the panel lengths below which a mesh counts as homogeneous.
constexpr double kHomogTol = 1e-10;
// Equal-chord mesh of a trigonometric-polynomial curve (host, mesher.hip).
void equal_chord_mesh(int d, const double* ax, const double* bx, const double* ay, const double* by, int64_t n,
                      double* nodes, double* chord);
// pipeline.hip: Gershgorin interval of the Gram matrix from host panel lengths
void gram_gershgorin(const std::vector<double>& h, double& lo, double& hi);
// assemble.hip
void launch_assemble(Op& op);
void launch_assemble_batch(Ctx& c, Op* const* ops, int nops);
void launch_assemble_yukawa(Op& op, double kappa, double2* Sy);
// gauss rules (host)
void gauss_legendre_01(int n, double* x, double* w);

}  // namespace fds

struct fds_ctx_s {
    fds::Ctx impl;
};
struct fds_op_s {
    fds::Op impl;
};
