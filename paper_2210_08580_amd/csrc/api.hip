// C ABI of libfds: argument checking, the pipeline state machine, device
// memory ownership and error reporting. All numerical work is in the kernels
// of the other translation units; this file only orchestrates them on the
// context's stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "fds_internal.h"
#include "hankel.h"
#include "linalg.h"
#include "lowrank.h"
#include "pipeline.h"

namespace fds {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

void* Ctx::raw_alloc(size_t bytes, hipStream_t s) {
    void* p = nullptr;
    if (has_alloc) {
        p = alloc.alloc(bytes, (void*)s, alloc.user);
        if (!p) throw Error{FDS_ERR_ALLOC, "allocator callback returned NULL"};
        return p;
    }
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{FDS_ERR_ALLOC, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    }
    return p;
}

void Ctx::raw_free(void* p, hipStream_t s) {
    if (has_alloc) {
        alloc.release(p, (void*)s, alloc.user);
        return;
    }
    (void)hipFree(p);
}

// size classes: powers of two up to 1 MiB, then multiples of 2 MiB
static size_t size_class(size_t b) {
    if (b <= ((size_t)1 << 20)) {
        size_t c = 512;
        while (c < b) c <<= 1;
        return c;
    }
    const size_t g = (size_t)2 << 20;
    return (b + g - 1) / g * g;
}

static bool capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

void* Ctx::dmalloc(size_t bytes) {
    if (noalloc) throw Error{FDS_ERR_STATE, "internal error: device allocation inside an allocation-free call"};
    if (bytes == 0) bytes = 16;
    std::lock_guard<std::mutex> lk(pool_mu);
    if (capturing(stream)) {
        void* p = raw_alloc(bytes, stream);
        live[p] = Block{bytes, stream, false};
        return p;
    }
    const size_t cls = size_class(bytes);
    void* p = nullptr;
    auto it = cache.find({stream, cls});
    if (it != cache.end() && !it->second.empty()) {
        p = it->second.back();
        it->second.pop_back();
    } else {
        try {
            p = raw_alloc(cls, stream);
        } catch (const Error&) {
            // give the cached blocks back and try once more
            for (auto& kv : cache)
                for (void* q : kv.second) raw_free(q, kv.first.first);
            cache.clear();
            p = raw_alloc(cls, stream);
        }
    }
    live[p] = Block{cls, stream, true};
    return p;
}

void Ctx::dfree(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(pool_mu);
    auto it = live.find(p);
    if (it == live.end()) {   // not from dmalloc: hand it straight back
        raw_free(p, stream);
        return;
    }
    const Block b = it->second;
    live.erase(it);
    if (!b.pooled) {
        raw_free(p, b.stream);
    } else if (capturing(stream)) {
        held.push_back({p, b.stream});
    } else {
        cache[{b.stream, b.bytes}].push_back(p);
    }
}

void Ctx::release_cache() {
    std::lock_guard<std::mutex> lk(pool_mu);
    for (auto& kv : cache)
        for (void* q : kv.second) raw_free(q, kv.first.first);
    cache.clear();
    for (auto& h : held) raw_free(h.first, h.second);
    held.clear();
}

Op::~Op() {
    if (!ctx) return;
    if (pre_active && ctx->side) (void)hipStreamSynchronize(ctx->side);
    void* ptrs[] = {pre_Lb, pre_Gb, pre_steps, pre_lam,nodes, h, nx, ny, gx, gy, g_diag, g_off, l_diag, l_off, S, Nm, D, S32, N32, D32, Nband,
                    Vn, Vg, Vgc, Bt, gfac, gband, K, Up, piv, lam_dev, Sy, gpow[0], gpow[1], Btr};
    for (void* p : ptrs) ctx->dfree(p);
    if (owns_uw) {
        ctx->dfree(U);
        ctx->dfree(W);
    }
    if (Wr != Btr) ctx->dfree(Wr);
    if (ev_mesh) (void)hipEventDestroy(ev_mesh);
}

template <typename F>
static fds_status guarded(F&& f) {
    try {
        f();
        return FDS_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return FDS_ERR_ALLOC;
    } catch (...) {
        set_error("unexpected internal error");
        return FDS_ERR_HIP;
    }
}

static void require_stage(const Op& op, Stage s, const char* what) {
    if ((int)op.stage < (int)s)
        throw Error{FDS_ERR_STATE, std::string(what) + " called before the required pipeline stage"};
}

void resolve_profile(Ctx& c) {
    for (auto& r : c.pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            auto& e = c.acc[r.name];
            e.first += ms;
            e.second += 1;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    c.pending.clear();
}

}  // namespace fds

using namespace fds;

extern "C" {

const char* fds_last_error(void) { return g_last_error.c_str(); }

fds_status fds_ctx_create(int device, void* hip_stream, const fds_allocator* alloc, fds_ctx* out) {
    return guarded([&] {
        FDS_REQUIRE(out != nullptr, FDS_ERR_ARG, "out is NULL");
        *out = nullptr;
        int count = 0;
        FDS_HIP_TRY(hipGetDeviceCount(&count));
        FDS_REQUIRE(device >= 0 && device < count, FDS_ERR_ARG, "device index out of range");
        FDS_HIP_TRY(hipSetDevice(device));
        auto* c = new fds_ctx_s();
        Ctx& x = c->impl;
        x.device = device;
        x.stream = (hipStream_t)hip_stream;
        if (alloc && alloc->alloc && alloc->release) {
            x.alloc = *alloc;
            x.has_alloc = true;
        }
        try {
            x.hk_tab = (double*)x.dmalloc(sizeof(double) * HK_TAB_DOUBLES);
            FDS_HIP_TRY(hipMemcpyAsync(x.hk_tab, &HK_TAB[0][0][0], sizeof(double) * HK_TAB_DOUBLES,
                                       hipMemcpyHostToDevice, x.stream));
            x.hf_tab = (double*)x.dmalloc(sizeof(double) * HF_TAB_DOUBLES);
            FDS_HIP_TRY(hipMemcpyAsync(x.hf_tab, &HF_TAB[0][0][0], sizeof(double) * HF_TAB_DOUBLES,
                                       hipMemcpyHostToDevice, x.stream));
            x.hf_tab32 = (float*)x.dmalloc(sizeof(float) * HF32_TAB_FLOATS);
            FDS_HIP_TRY(hipMemcpyAsync(x.hf_tab32, &HF32_TAB[0][0][0], sizeof(float) * HF32_TAB_FLOATS,
                                       hipMemcpyHostToDevice, x.stream));
            std::vector<double> yk(YK_ALL_DOUBLES);
            std::copy(&YK_TAB[0][0], &YK_TAB[0][0] + YK_TAB_DOUBLES, yk.begin());
            std::copy(YK_SER_I0, YK_SER_I0 + YK_NSER, yk.begin() + YK_OFF_I0);
            std::copy(YK_SER_K0, YK_SER_K0 + YK_NSER, yk.begin() + YK_OFF_K0);
            std::copy(YK_ASY, YK_ASY + YK_NASY, yk.begin() + YK_OFF_ASY);
            x.yk_tab = (double*)x.dmalloc(sizeof(double) * YK_ALL_DOUBLES);
            FDS_HIP_TRY(hipMemcpyAsync(x.yk_tab, yk.data(), sizeof(double) * YK_ALL_DOUBLES, hipMemcpyHostToDevice,
                                       x.stream));
            x.yk_tab32 = (float*)x.dmalloc(sizeof(float) * YK32_TAB_FLOATS);
            FDS_HIP_TRY(hipMemcpyAsync(x.yk_tab32, &YK32_TAB[0][0], sizeof(float) * YK32_TAB_FLOATS,
                                       hipMemcpyHostToDevice, x.stream));
            double g[64];
            gauss_legendre_01(32, g, g + 32);
            x.gl32 = (double*)x.dmalloc(sizeof(double) * 64);
            FDS_HIP_TRY(hipMemcpyAsync(x.gl32, g, sizeof(g), hipMemcpyHostToDevice, x.stream));
            FDS_HIP_TRY(hipStreamSynchronize(x.stream));
            init_noalloc_scratch(x);
        } catch (...) {
            x.dfree(x.hk_tab);
            x.dfree(x.hf_tab);
            x.dfree(x.hf_tab32);
            x.dfree(x.gl32);
            x.dfree(x.yk_tab);
            x.dfree(x.yk_tab32);
            delete c;
            throw;
        }
        *out = c;
    });
}

fds_status fds_ctx_destroy(fds_ctx ctx) {
    return guarded([&] {
        if (!ctx) return;
        (void)hipStreamSynchronize(ctx->impl.stream);
        if (ctx->impl.side) (void)hipStreamSynchronize(ctx->impl.side);
        resolve_profile(ctx->impl);
        ctx->impl.dfree(ctx->impl.hk_tab);
        ctx->impl.dfree(ctx->impl.hf_tab);
        ctx->impl.dfree(ctx->impl.hf_tab32);
        ctx->impl.dfree(ctx->impl.gl32);
        ctx->impl.dfree(ctx->impl.yk_tab);
        ctx->impl.dfree(ctx->impl.yk_tab32);
        ctx->impl.release_cache();
        if (ctx->impl.host_pin) (void)hipHostFree(ctx->impl.host_pin);
        ctx->impl.host_pin = nullptr;
        if (ctx->impl.side) {
            (void)hipStreamDestroy(ctx->impl.side);
            ctx->impl.side = nullptr;
        }
        delete ctx;
    });
}

fds_status fds_sync(fds_ctx ctx) {
    return guarded([&] {
        FDS_REQUIRE(ctx != nullptr, FDS_ERR_ARG, "ctx is NULL");
        FDS_HIP_TRY(hipStreamSynchronize(ctx->impl.stream));
        FDS_HIP_TRY(hipGetLastError());
    });
}

fds_status fds_profile_enable(fds_ctx ctx, int32_t on) {
    return guarded([&] {
        FDS_REQUIRE(ctx != nullptr, FDS_ERR_ARG, "ctx is NULL");
        ctx->impl.prof = on != 0;
    });
}

fds_status fds_profile_read(fds_ctx ctx, int32_t cap, char* names, double* total_ms, int64_t* launches,
                            int32_t* count) {
    return guarded([&] {
        FDS_REQUIRE(ctx && cap >= 0 && (cap == 0 || (names && total_ms && launches)), FDS_ERR_ARG,
                    "bad argument");
        Ctx& c = ctx->impl;
        resolve_profile(c);
        int32_t i = 0;
        for (const auto& kv : c.acc) {
            if (i >= cap) break;
            std::strncpy(names + 32 * i, kv.first.c_str(), 31);
            names[32 * i + 31] = 0;
            total_ms[i] = kv.second.first;
            launches[i] = kv.second.second;
            ++i;
        }
        if (count) *count = i;
        c.acc.clear();
    });
}

fds_status fds_autotune(fds_ctx ctx, int32_t on) {
    return guarded([&] {
        FDS_REQUIRE(ctx != nullptr, FDS_ERR_ARG, "ctx is NULL");
        ctx->impl.autotune = on != 0;
    });
}

fds_status fds_autotune_read(fds_ctx ctx, int32_t cap, char* keys, int32_t* split_k, int32_t* count) {
    return guarded([&] {
        FDS_REQUIRE(ctx && count && cap >= 0, FDS_ERR_ARG, "bad argument");
        *count = autotune_entries(ctx->impl, cap, keys, split_k);
    });
}

fds_status fds_hankel_eval(fds_ctx ctx, const double* x, int64_t n, double* out) {
    return guarded([&] {
        FDS_REQUIRE(ctx && x && out && n >= 0, FDS_ERR_ARG, "bad argument");
        if (n == 0) return;
        launch_hankel_eval(ctx->impl, x, n, out);
    });
}

fds_status fds_hankel_eval_f32(fds_ctx ctx, const double* x, int64_t n, float* out) {
    return guarded([&] {
        FDS_REQUIRE(ctx && x && out && n >= 0, FDS_ERR_ARG, "bad argument");
        if (n == 0) return;
        launch_hankel_eval_f32(ctx->impl, x, n, out);
    });
}

fds_status fds_yukawa_eval(fds_ctx ctx, double kappa, const double* R, int64_t n, double* out) {
    return guarded([&] {
        FDS_REQUIRE(ctx && R && out && n >= 0, FDS_ERR_ARG, "bad argument");
        FDS_REQUIRE(std::isfinite(kappa) && kappa > 0.0, FDS_ERR_ARG, "kappa must be finite and > 0");
        if (n == 0) return;
        launch_yukawa_eval(ctx->impl, kappa, R, n, out);
    });
}

fds_status fds_equal_chord_nodes(int32_t degree, const double* ax, const double* bx, const double* ay,
                                 const double* by, int64_t n, double* nodes, double* chord) {
    return guarded([&] { equal_chord_mesh(degree, ax, bx, ay, by, n, nodes, chord); });
}

fds_status fds_kernel_eval(fds_ctx ctx, double k, const double* R, int64_t n, double* out) {
    return guarded([&] {
        FDS_REQUIRE(ctx && R && out && n >= 0, FDS_ERR_ARG, "bad argument");
        FDS_REQUIRE(std::isfinite(k) && k > 0.0, FDS_ERR_ARG, "k must be finite and > 0");
        if (n == 0) return;
        launch_kernel_eval(ctx->impl, k, R, n, out);
    });
}

fds_status fds_zgemm(fds_ctx ctx, int32_t opa, int32_t opb, int64_t m, int64_t n, int64_t k,
                     const double* alpha, const void* A, int64_t lda, const void* B, int64_t ldb,
                     const double* beta, void* C, int64_t ldc) {
    return guarded([&] {
        FDS_REQUIRE(ctx && alpha && beta && C, FDS_ERR_ARG, "NULL argument");
        FDS_REQUIRE(opa >= 0 && opa <= 2 && opb >= 0 && opb <= 2, FDS_ERR_ARG, "op must be 0, 1 or 2");
        FDS_REQUIRE(m >= 0 && n >= 0 && k >= 0 && m < (1 << 30) && n < (1 << 30) && k < (1 << 30),
                    FDS_ERR_ARG, "bad sizes");
        if (m == 0 || n == 0) return;
        FDS_REQUIRE(A && B, FDS_ERR_ARG, "NULL operand");
        const int64_t ra = opa == 0 ? m : k, rb = opb == 0 ? k : n;
        FDS_REQUIRE(lda >= std::max<int64_t>(1, ra) && ldb >= std::max<int64_t>(1, rb) && ldc >= m,
                    FDS_ERR_ARG, "leading dimension too small");
        zgemm(ctx->impl, opa, opb, (int)m, (int)n, (int)k, make_double2(alpha[0], alpha[1]),
              (const double2*)A, lda, (const double2*)B, ldb, make_double2(beta[0], beta[1]), (double2*)C, ldc);
    });
}

fds_status fds_zinv(fds_ctx ctx, int64_t r, const void* A, void* Ainv, double* stats) {
    return guarded([&] {
        FDS_REQUIRE(ctx && A && Ainv && r >= 1, FDS_ERR_ARG, "bad argument");
        FDS_REQUIRE(r <= 2048, FDS_ERR_NOTIMPL, "dense inverse of order above 2048");
        Ctx& c = ctx->impl;
        double hs[2];
        gj_inverse(c, (double2*)const_cast<void*>(A), (double2*)Ainv, (int)r, hs);
        if (stats) {
            stats[0] = hs[0];
            stats[1] = hs[1];
        }
    });
}

fds_status fds_zqr(fds_ctx ctx, int64_t M, int64_t m, void* A, void* Q, int32_t method,
                   int32_t* householder_used) {
    return guarded([&] {
        FDS_REQUIRE(ctx && A && Q && A != Q, FDS_ERR_ARG, "bad argument");
        FDS_REQUIRE(m >= 1 && M >= m && M < (1 << 30), FDS_ERR_ARG, "QR needs rows >= columns >= 1");
        FDS_REQUIRE(method == FDS_QR_AUTO || method == FDS_QR_HOUSEHOLDER, FDS_ERR_ARG, "bad qr method");
        Ctx& c = ctx->impl;
        double2* tau = static_cast<double2*>(c.dmalloc(sizeof(double2) * (size_t)m));
        bool chol = false;
        try {
            chol = qr_explicit(c, static_cast<double2*>(A), (int)M, (int)m, tau, static_cast<double2*>(Q),
                               method == FDS_QR_AUTO);
            FDS_HIP_TRY(hipStreamSynchronize(c.stream));
        } catch (...) {
            c.dfree(tau);
            throw;
        }
        c.dfree(tau);
        if (householder_used) *householder_used = chol ? 0 : 1;
    });
}

fds_status fds_cgemm(fds_ctx ctx, int32_t opa, int32_t opb, int64_t m, int64_t n, int64_t k,
                     const float* alpha, const void* A, int64_t lda, const void* B, int64_t ldb,
                     const float* beta, void* C, int64_t ldc) {
    return guarded([&] {
        FDS_REQUIRE(ctx && alpha && beta && C, FDS_ERR_ARG, "NULL argument");
        FDS_REQUIRE(opa >= 0 && opa <= 2 && opb >= 0 && opb <= 2, FDS_ERR_ARG, "op must be 0, 1 or 2");
        FDS_REQUIRE(m >= 0 && n >= 0 && k >= 0 && m < (1 << 30) && n < (1 << 30) && k < (1 << 30),
                    FDS_ERR_ARG, "bad sizes");
        if (m == 0 || n == 0) return;
        FDS_REQUIRE(A && B, FDS_ERR_ARG, "NULL operand");
        const int64_t ra = opa == 0 ? m : k, rb = opb == 0 ? k : n;
        FDS_REQUIRE(lda >= std::max<int64_t>(1, ra) && ldb >= std::max<int64_t>(1, rb) && ldc >= m,
                    FDS_ERR_ARG, "leading dimension too small");
        cgemm(ctx->impl, opa, opb, (int)m, (int)n, (int)k, make_float2(alpha[0], alpha[1]),
              (const float2*)A, lda, (const float2*)B, ldb, make_float2(beta[0], beta[1]), (float2*)C, ldc);
    });
}

// Validates the geometry, allocates the operator and builds its panels, Gram
// and Laplacian matrices; the dense assembly is left to the caller.
static fds_op_s* new_operator(Ctx& c, const double* nodes, int64_t n, double k, const fds_asm_opts* opts) {
    FDS_REQUIRE(nodes != nullptr, FDS_ERR_ARG, "NULL nodes");
    FDS_REQUIRE(n >= 8 && n <= (int64_t)1 << 20, FDS_ERR_ARG, "n must be in [8, 2^20]");
    FDS_REQUIRE(std::isfinite(k) && k > 0.0, FDS_ERR_ARG, "k must be finite and > 0");
    if (opts) {
        FDS_REQUIRE(opts->nquad == 0 || opts->nquad == 8, FDS_ERR_NOTIMPL,
                    "only the 8-point rule is implemented");
        FDS_REQUIRE(opts->precision == FDS_FP64 || opts->precision == FDS_FP32, FDS_ERR_NOTIMPL,
                    "assembly precision must be FDS_FP64 or FDS_FP32");
        FDS_REQUIRE(opts->band_width >= 0, FDS_ERR_ARG, "band_width must be >= 0");
    }
    // host-side geometry validation (O(n) copy)
    std::vector<double> hn(2 * n);
    FDS_HIP_TRY(hipMemcpyAsync(hn.data(), nodes, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, c.stream));
    FDS_HIP_TRY(hipStreamSynchronize(c.stream));
    double area = 0.0;
    std::vector<double> hh(n);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t j = (i + 1) % n;
        const double x0 = hn[2 * i], y0 = hn[2 * i + 1], x1 = hn[2 * j], y1 = hn[2 * j + 1];
        FDS_REQUIRE(std::isfinite(x0) && std::isfinite(y0), FDS_ERR_ARG, "non-finite node");
        hh[i] = std::hypot(x1 - x0, y1 - y0);
        FDS_REQUIRE(hh[i] > 0.0, FDS_ERR_ARG, "zero-length panel");
        area += x0 * y1 - x1 * y0;
    }
    FDS_REQUIRE(area > 0.0, FDS_ERR_ARG, "nodes must be counter-clockwise");

    auto* o = new fds_op_s();
    Op& op = o->impl;
    op.ctx = &c;
    op.n = n;
    op.k = k;
    op.prec = opts ? opts->precision : FDS_FP64;
    {
        double hmin = 1e300, hmax = 0.0, hsum = 0.0;
        for (double v : hh) {
            hmin = std::min(hmin, v);
            hmax = std::max(hmax, v);
            hsum += v;
        }
        op.h_mean = hsum / (double)n;
        op.homog = hmax - hmin <= kHomogTol * op.h_mean;
    }
    op.h_host = std::move(hh);
    try {
        const size_t nd = sizeof(double) * n;
        op.nodes = (double*)c.dmalloc(2 * nd);
        op.h = (double*)c.dmalloc(nd);
        op.nx = (double*)c.dmalloc(nd);
        op.ny = (double*)c.dmalloc(nd);
        op.gx = (double*)c.dmalloc(8 * nd);
        op.gy = (double*)c.dmalloc(8 * nd);
        op.g_diag = (double*)c.dmalloc(nd);
        op.g_off = (double*)c.dmalloc(nd);
        op.l_diag = (double*)c.dmalloc(nd);
        op.l_off = (double*)c.dmalloc(nd);
        if (op.prec == FDS_FP32) {
            const size_t mat = sizeof(float2) * (size_t)n * (size_t)n;
            op.S32 = (float2*)c.dmalloc(mat);
            op.N32 = (float2*)c.dmalloc(mat);
            op.D32 = (float2*)c.dmalloc(mat);
            // cyclic band |d| <= nbw, with 2 nbw + 1 <= n so that the taps are distinct
            // default half-width: the FP32 rounding of N beyond the band reaches the solution
            // amplified ~1/(w h) (measured on the ellipse 2 x 0.5 at 16384 panels: 2.1e-6,
            // 1.0e-6, 4.6e-7, 2.1e-7 for w = 63, 127, 255, 511), so w grows with n
            const int64_t req = opts && opts->band_width > 0 ? opts->band_width : (n > 8192 ? n / 64 - 1 : 63);
            op.nbw = (int)std::min<int64_t>(req, (n - 1) / 2);
            op.Nband = (double2*)c.dmalloc(sizeof(double2) * (2 * op.nbw + 1) * (size_t)n);
        } else {
            const size_t mat = sizeof(double2) * (size_t)n * (size_t)n;
            op.S = (double2*)c.dmalloc(mat);
            op.Nm = (double2*)c.dmalloc(mat);
            op.D = (double2*)c.dmalloc(mat);
        }
        FDS_HIP_TRY(hipMemcpyAsync(op.nodes, nodes, 2 * nd, hipMemcpyDeviceToDevice, c.stream));
        gauss_legendre_01(8, op.rule.xi, op.rule.w);
        launch_geometry(op);
        FDS_HIP_TRY(hipEventCreateWithFlags(&op.ev_mesh, hipEventDisableTiming));
        FDS_HIP_TRY(hipEventRecord(op.ev_mesh, c.stream));
        op.ev_mesh_fresh = true;
    } catch (...) {
        delete o;
        throw;
    }
    return o;
}

fds_status fds_assemble(fds_ctx ctx, const double* nodes, int64_t n, double k,
                        const fds_asm_opts* opts, fds_op* out) {
    return guarded([&] {
        FDS_REQUIRE(ctx && nodes && out, FDS_ERR_ARG, "NULL argument");
        *out = nullptr;
        FDS_REQUIRE(!opts || (opts->filter_modes >= 0 && opts->filter_modes <= n), FDS_ERR_ARG,
                    "filter_modes must be in [0, n]");
        fds_op_s* o = new_operator(ctx->impl, nodes, n, k, opts);
        try {
            if (opts && opts->filter_modes > 0) prefetch_filter(o->impl, opts->filter_modes);
            launch_assemble(o->impl);
            o->impl.stage = Stage::Assembled;
        } catch (...) {
            delete o;
            throw;
        }
        *out = o;
    });
}

fds_status fds_assemble_batch(fds_ctx ctx, int32_t count, const double* const* nodes, const int64_t* n,
                              const double* k, fds_op* out) {
    return guarded([&] {
        FDS_REQUIRE(ctx && nodes && n && k && out && count >= 1, FDS_ERR_ARG, "bad argument");
        for (int32_t j = 0; j < count; ++j) out[j] = nullptr;
        std::vector<fds_op_s*> made;
        try {
            for (int32_t j = 0; j < count; ++j) made.push_back(new_operator(ctx->impl, nodes[j], n[j], k[j], nullptr));
            std::vector<Op*> ops;
            for (auto* o : made) ops.push_back(&o->impl);
            launch_assemble_batch(ctx->impl, ops.data(), count);
            for (auto* o : made) o->impl.stage = Stage::Assembled;
        } catch (...) {
            for (auto* o : made) delete o;
            throw;
        }
        for (int32_t j = 0; j < count; ++j) out[j] = made[j];
    });
}

fds_status fds_op_destroy(fds_op op) {
    return guarded([&] {
        if (!op) return;
        (void)hipStreamSynchronize(op->impl.ctx->stream);
        delete op;
    });
}

fds_status fds_op_info(fds_op op, int64_t* n, int32_t* n_eff, int32_t* rank) {
    return guarded([&] {
        FDS_REQUIRE(op != nullptr, FDS_ERR_ARG, "op is NULL");
        if (n) *n = op->impl.n;
        if (n_eff) *n_eff = op->impl.n_eff;
        if (rank) *rank = op->impl.rank;
    });
}

fds_status fds_op_matrices(fds_op op, void** S, void** Nmat, void** D) {
    return guarded([&] {
        FDS_REQUIRE(op != nullptr, FDS_ERR_ARG, "op is NULL");
        const bool f32 = op->impl.prec == FDS_FP32;
        if (S) *S = f32 ? (void*)op->impl.S32 : (void*)op->impl.S;
        if (Nmat) *Nmat = f32 ? (void*)op->impl.N32 : (void*)op->impl.Nm;
        if (D) *D = f32 ? (void*)op->impl.D32 : (void*)op->impl.D;
    });
}

fds_status fds_op_nband(fds_op op, const void** Nband, int32_t* width) {
    return guarded([&] {
        FDS_REQUIRE(op && Nband && width, FDS_ERR_ARG, "NULL argument");
        *Nband = op->impl.Nband;
        *width = op->impl.nbw;
    });
}

fds_status fds_op_yukawa(fds_op op, const void** Sy) {
    return guarded([&] {
        FDS_REQUIRE(op && Sy, FDS_ERR_ARG, "NULL argument");
        *Sy = op->impl.Sy;
    });
}

fds_status fds_op_precision(fds_op op, int32_t* precision) {
    return guarded([&] {
        FDS_REQUIRE(op && precision, FDS_ERR_ARG, "NULL argument");
        *precision = op->impl.prec;
    });
}

fds_status fds_op_sparse(fds_op op, const double** g_diag, const double** g_off,
                         const double** l_diag, const double** l_off) {
    return guarded([&] {
        FDS_REQUIRE(op != nullptr, FDS_ERR_ARG, "op is NULL");
        if (g_diag) *g_diag = op->impl.g_diag;
        if (g_off) *g_off = op->impl.g_off;
        if (l_diag) *l_diag = op->impl.l_diag;
        if (l_off) *l_off = op->impl.l_off;
    });
}

fds_status fds_rhs_planewave(fds_op op, const double* angles, const void* amps, int64_t nrhs,
                             void* f_out, void* h_out) {
    return guarded([&] {
        FDS_REQUIRE(op && angles && amps && nrhs >= 0, FDS_ERR_ARG, "bad argument");
        require_stage(op->impl, Stage::Assembled, "fds_rhs_planewave");
        if (nrhs == 0 || (!f_out && !h_out)) return;
        launch_rhs_planewave(op->impl, angles, (const double2*)amps, nrhs, (double2*)f_out,
                             (double2*)h_out);
    });
}

fds_status fds_apply_gram(fds_op op, int32_t p, void* X, int64_t ncols) {
    return guarded([&] {
        FDS_REQUIRE(op && X && ncols >= 0, FDS_ERR_ARG, "bad argument");
        if (ncols == 0) return;
        apply_gram_power(op->impl, p, (double2*)X, ncols);
    });
}

fds_status fds_filter(fds_op op, fds_form form, double alpha, const fds_filter_opts* opts,
                      int32_t* n_eff) {
    return guarded([&] {
        FDS_REQUIRE(op != nullptr, FDS_ERR_ARG, "op is NULL");
        require_stage(op->impl, Stage::Assembled, "fds_filter");
        FDS_REQUIRE(form == FDS_EFIE || form == FDS_MFIE || form == FDS_CFIE || form == FDS_YCFIE, FDS_ERR_ARG,
                    "bad form");
        FDS_REQUIRE(std::isfinite(alpha), FDS_ERR_ARG, "alpha must be finite");
        int nm = 21;
        bool keep = true;
        double crt = 1e-6;
        if (opts) {
            nm = opts->n_modes;
            keep = opts->keep_nullspace != 0;
            crt = opts->cluster_rtol > 0.0 ? opts->cluster_rtol : 1e-6;
        }
        FDS_REQUIRE(nm >= 1 && nm <= op->impl.n, FDS_ERR_ARG, "n_modes must be in [1, n]");
        FDS_REQUIRE(keep || nm >= 2, FDS_ERR_ARG, "n_modes must be >= 2 without the null mode");
        if (form == FDS_CFIE || form == FDS_YCFIE)
            FDS_REQUIRE(std::fabs(1.0 + 2.0 * alpha) > 1e-12, FDS_ERR_ARG, "CFIE with beta = 0");
        run_filter(op->impl, form, alpha, nm, keep, crt);
        if (n_eff) *n_eff = op->impl.n_eff;
    });
}

fds_status fds_filter_batch(int32_t count, fds_op* ops, fds_form form, double alpha,
                            const fds_filter_opts* opts, int32_t* n_eff) {
    return guarded([&] {
        FDS_REQUIRE(ops && opts && count >= 1, FDS_ERR_ARG, "bad argument");
        FDS_REQUIRE(form == FDS_EFIE || form == FDS_MFIE || form == FDS_CFIE, FDS_ERR_ARG, "bad form");
        FDS_REQUIRE(std::isfinite(alpha), FDS_ERR_ARG, "alpha must be finite");
        if (form == FDS_CFIE)
            FDS_REQUIRE(std::fabs(1.0 + 2.0 * alpha) > 1e-12, FDS_ERR_ARG, "CFIE with beta = 0");
        std::vector<Op*> v(count);
        std::vector<int> nm(count);
        for (int32_t j = 0; j < count; ++j) {
            FDS_REQUIRE(ops[j] != nullptr, FDS_ERR_ARG, "NULL operator");
            FDS_REQUIRE(ops[j]->impl.ctx == ops[0]->impl.ctx, FDS_ERR_ARG, "operators of different contexts");
            require_stage(ops[j]->impl, Stage::Assembled, "fds_filter_batch");
            v[j] = &ops[j]->impl;
            nm[j] = opts[j].n_modes;
            FDS_REQUIRE(nm[j] >= 1 && nm[j] <= v[j]->n, FDS_ERR_ARG, "n_modes must be in [1, n]");
            FDS_REQUIRE(opts[j].keep_nullspace == opts[0].keep_nullspace, FDS_ERR_ARG,
                        "one null-space choice per batch");
        }
        const bool keep = opts[0].keep_nullspace != 0;
        FDS_REQUIRE(keep || *std::min_element(nm.begin(), nm.end()) >= 2, FDS_ERR_ARG,
                    "n_modes must be >= 2 without the null mode");
        const double crt = opts[0].cluster_rtol > 0.0 ? opts[0].cluster_rtol : 1e-6;
        run_filter_batch(v.data(), count, form, alpha, nm.data(), keep, crt);
        if (n_eff)
            for (int32_t j = 0; j < count; ++j) n_eff[j] = v[j]->n_eff;
    });
}

fds_status fds_op_filter_basis(fds_op op, const double** Vn) {
    return guarded([&] {
        FDS_REQUIRE(op != nullptr, FDS_ERR_ARG, "op is NULL");
        require_stage(op->impl, Stage::Filtered, "fds_op_filter_basis");
        const double* v = filter_basis_view(op->impl);
        if (Vn) *Vn = v;
    });
}

fds_status fds_op_filter_eigenvalues(fds_op op, double* out, int32_t cap, int32_t* count) {
    return guarded([&] {
        FDS_REQUIRE(op && out && cap >= 0, FDS_ERR_ARG, "bad argument");
        Op& o = op->impl;
        if (o.lam_dev_n > 0) {
            FDS_HIP_TRY(hipMemcpyAsync(o.filt_lam.data(), o.lam_dev, sizeof(double) * o.lam_dev_n,
                                       hipMemcpyDeviceToHost, o.ctx->stream));
            FDS_HIP_TRY(hipStreamSynchronize(o.ctx->stream));
            o.lam_dev_n = 0;
        }
        const auto& v = o.filt_lam;
        const int32_t m = (int32_t)std::min<size_t>(v.size(), (size_t)cap);
        for (int32_t i = 0; i < m; ++i) out[i] = v[i];
        if (count) *count = m;
    });
}

fds_status fds_compress(fds_op op, const fds_compress_opts* opts, int32_t* rank_out) {
    return guarded([&] {
        FDS_REQUIRE(op && opts, FDS_ERR_ARG, "NULL argument");
        require_stage(op->impl, Stage::Filtered, "fds_compress");
        FDS_REQUIRE(opts->precision == FDS_FP64, FDS_ERR_NOTIMPL, "only FP64 compression is implemented");
        FDS_REQUIRE(opts->qr == FDS_QR_AUTO || opts->qr == FDS_QR_HOUSEHOLDER, FDS_ERR_ARG, "bad qr method");
        run_compress(op->impl, opts->rank_cap, opts->oversample, opts->power_iters, opts->tol, opts->seed,
                     opts->qr == FDS_QR_HOUSEHOLDER);
        if (rank_out) *rank_out = op->impl.rank;
    });
}

fds_status fds_compress_aca(fds_op op, int32_t rank_cap, double tol, int32_t* rank_out) {
    return guarded([&] {
        FDS_REQUIRE(op != nullptr, FDS_ERR_ARG, "op is NULL");
        require_stage(op->impl, Stage::Filtered, "fds_compress_aca");
        run_compress_aca(op->impl, rank_cap, tol);
        if (rank_out) *rank_out = op->impl.rank;
    });
}

fds_status fds_op_singular_values(fds_op op, double* out, int32_t cap, int32_t* count) {
    return guarded([&] {
        FDS_REQUIRE(op && count && cap >= 0 && (out || cap == 0), FDS_ERR_ARG, "bad argument");
        require_stage(op->impl, Stage::Compressed, "fds_op_singular_values");
        const auto& sv = op->impl.sv;
        const int32_t k = std::min<int32_t>(cap, (int32_t)sv.size());
        for (int32_t i = 0; i < k; ++i) out[i] = sv[i];
        *count = k;
    });
}

fds_status fds_op_factors(fds_op op, const void** U, const void** W, int32_t* rank) {
    return guarded([&] {
        FDS_REQUIRE(op != nullptr, FDS_ERR_ARG, "op is NULL");
        require_stage(op->impl, Stage::Compressed, "fds_op_factors");
        if (U) *U = op->impl.U;
        if (W) *W = op->impl.W;
        if (rank) *rank = op->impl.rank;
    });
}

fds_status fds_factor(fds_op op) {
    return guarded([&] {
        FDS_REQUIRE(op != nullptr, FDS_ERR_ARG, "op is NULL");
        require_stage(op->impl, Stage::Compressed, "fds_factor");
        run_factor(op->impl);
    });
}

fds_status fds_solve(fds_op op, const void* f, const void* h, int64_t nrhs, void* j_out,
                     void* y_out, const fds_solve_opts* opts, fds_solve_stats* stats) {
    return guarded([&] {
        FDS_REQUIRE(op && j_out && nrhs >= 0, FDS_ERR_ARG, "bad argument");
        require_stage(op->impl, Stage::Factored, "fds_solve");
        int it = 4;
        double tol = 1e-12;
        bool unf = false;
        if (opts) {
            FDS_REQUIRE(opts->precision == FDS_FP64, FDS_ERR_NOTIMPL, "only FP64 solves are implemented");
            it = opts->max_iters;
            tol = opts->tol;
            unf = opts->unfiltered != 0;
        }
        FDS_REQUIRE(it >= 0 && it <= 1000, FDS_ERR_ARG, "max_iters out of range");
        if (nrhs == 0) return;
        run_solve(op->impl, (const double2*)f, (const double2*)h, nrhs, (double2*)j_out,
                  (double2*)y_out, it, tol, stats, unf);
    });
}

fds_status fds_rhs_system(fds_op op, fds_form form, double alpha, const void* f, const void* h, int64_t nrhs,
                          void* w_out) {
    return guarded([&] {
        FDS_REQUIRE(op && w_out && nrhs >= 0, FDS_ERR_ARG, "bad argument");
        require_stage(op->impl, Stage::Assembled, "fds_rhs_system");
        FDS_REQUIRE(form == FDS_EFIE || form == FDS_MFIE || form == FDS_CFIE || form == FDS_YCFIE, FDS_ERR_ARG,
                    "bad form");
        FDS_REQUIRE(std::isfinite(alpha), FDS_ERR_ARG, "alpha must be finite");
        if (nrhs == 0) return;
        run_rhs_system(op->impl, form, alpha, (const double2*)f, (const double2*)h, nrhs, (double2*)w_out);
    });
}

fds_status fds_solve_system(fds_op op, const void* w, int64_t nrhs, void* j_out, void* y_out,
                            const fds_solve_opts* opts, fds_solve_stats* stats) {
    return guarded([&] {
        FDS_REQUIRE(op && w && j_out && nrhs >= 0, FDS_ERR_ARG, "bad argument");
        require_stage(op->impl, Stage::Factored, "fds_solve_system");
        int it = 4;
        double tol = 1e-12;
        bool unf = false;
        if (opts) {
            FDS_REQUIRE(opts->precision == FDS_FP64, FDS_ERR_NOTIMPL, "only FP64 solves are implemented");
            it = opts->max_iters;
            tol = opts->tol;
            unf = opts->unfiltered != 0;
        }
        FDS_REQUIRE(it >= 0 && it <= 1000, FDS_ERR_ARG, "max_iters out of range");
        if (nrhs == 0) return;
        run_solve_system(op->impl, (const double2*)w, nrhs, (double2*)j_out, (double2*)y_out, it, tol, stats, unf);
    });
}

fds_status fds_solve_adjoint(fds_op op, const void* v, int64_t nrhs, void* y_out, void* u_out,
                             const fds_solve_opts* opts, fds_solve_stats* stats) {
    return guarded([&] {
        FDS_REQUIRE(op && v && y_out && nrhs >= 0, FDS_ERR_ARG, "bad argument");
        FDS_REQUIRE(v != y_out && v != u_out, FDS_ERR_ARG, "outputs may not alias v");
        require_stage(op->impl, Stage::Factored, "fds_solve_adjoint");
        int it = 4;
        double tol = 1e-12;
        bool unf = false;
        if (opts) {
            FDS_REQUIRE(opts->precision == FDS_FP64, FDS_ERR_NOTIMPL, "only FP64 solves are implemented");
            it = opts->max_iters;
            tol = opts->tol;
            unf = opts->unfiltered != 0;
        }
        FDS_REQUIRE(it >= 0 && it <= 1000, FDS_ERR_ARG, "max_iters out of range");
        if (nrhs == 0) return;
        run_solve_adjoint(op->impl, (const double2*)v, nrhs, (double2*)y_out, (double2*)u_out, it, tol, stats, unf);
    });
}

fds_status fds_solve_system_noalloc(fds_op op, const void* w, int64_t nrhs, void* j_out, int32_t sweeps) {
    return guarded([&] {
        FDS_REQUIRE(op && w && j_out && nrhs >= 0, FDS_ERR_ARG, "bad argument");
        require_stage(op->impl, Stage::Factored, "fds_solve_system_noalloc");
        FDS_REQUIRE(sweeps >= 0 && sweeps <= 1000, FDS_ERR_ARG, "sweeps out of range");
        if (nrhs == 0) return;
        run_solve_system_noalloc(op->impl, (const double2*)w, nrhs, (double2*)j_out, sweeps);
    });
}

// ------------------------------------------------------------------ batches
struct fds_batch_s {
    Ctx* c = nullptr;
    std::vector<fds_op_s*> ops;
    std::vector<BatchItem> items;
    std::vector<int> chain;          // chain (graph branch) of each problem
    std::vector<void*> chain_ws;     // workspace of each chain
    std::vector<size_t> chain_bytes;
    std::vector<void*> bufs;
    int sweeps = 0;
    hipGraphExec_t exec = nullptr;
    ~fds_batch_s() {
        if (c) (void)hipStreamSynchronize(c->stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        for (void* b : bufs) c->dfree(b);
        for (auto* o : ops) delete o;
    }
};

constexpr int kBatchChains = 8;

// Records the solves of every problem into one graph. The problems are split
// into up to kBatchChains chains (longest first, each to the least loaded chain
// by n^2 nrhs), each captured on its own stream forked from and joined back to
// the origin stream, so that the graph's branches run side by side; each chain
// has its own workspace. Private streams are used because the context's stream
// may be the legacy default stream, which cannot be captured.
static hipGraphExec_t capture_batch(fds_batch_s& b) {
    Ctx& c = *b.c;
    const int nch = (int)b.chain_ws.size();
    FDS_HIP_TRY(hipStreamSynchronize(c.stream));
    std::vector<hipStream_t> st(nch + 1, nullptr);
    std::vector<hipEvent_t> ev(nch + 1, nullptr);
    const hipStream_t old = c.stream;
    const bool prof = c.prof;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    bool capturing = false;
    auto cleanup = [&]() {
        c.stream = old;
        c.prof = prof;
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto s : st)
            if (s) (void)hipStreamDestroy(s);
    };
    try {
        for (int i = 0; i <= nch; ++i) {
            FDS_HIP_TRY(hipStreamCreateWithFlags(&st[i], hipStreamNonBlocking));
            FDS_HIP_TRY(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
        }
        c.prof = false;   // no timing events inside the graph
        FDS_HIP_TRY(hipStreamBeginCapture(st[nch], hipStreamCaptureModeThreadLocal));
        capturing = true;
        FDS_HIP_TRY(hipEventRecord(ev[nch], st[nch]));
        for (int i = 0; i < nch; ++i) FDS_HIP_TRY(hipStreamWaitEvent(st[i], ev[nch], 0));
        for (size_t i = 0; i < b.items.size(); ++i) {
            const int ch = b.chain[i];
            c.stream = st[ch];
            run_batch_item(b.ops[i]->impl, b.items[i], b.sweeps, b.chain_ws[ch], b.chain_bytes[ch]);
        }
        for (int i = 0; i < nch; ++i) {
            FDS_HIP_TRY(hipEventRecord(ev[i], st[i]));
            FDS_HIP_TRY(hipStreamWaitEvent(st[nch], ev[i], 0));
        }
        c.stream = old;
        capturing = false;
        FDS_HIP_TRY(hipStreamEndCapture(st[nch], &g));
        FDS_HIP_TRY(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    } catch (...) {
        if (capturing) {
            hipGraph_t bad = nullptr;
            (void)hipStreamEndCapture(st[nch], &bad);
            if (bad) (void)hipGraphDestroy(bad);
        }
        if (g) (void)hipGraphDestroy(g);
        cleanup();
        throw;
    }
    (void)hipGraphDestroy(g);
    cleanup();
    return ge;
}

static fds_batch_s* make_batch(fds_ctx ctx, int64_t nb, const fds_problem* probs, const fds_batch_opts* o) {
    FDS_REQUIRE(ctx && probs && o && nb >= 1 && nb <= (1 << 16), FDS_ERR_ARG, "bad argument");
    FDS_REQUIRE(o->precision == FDS_FP64 || o->precision == FDS_FP32, FDS_ERR_ARG, "precision must be FP64 or FP32");
    const int form = o->form;
    FDS_REQUIRE(form == FDS_EFIE || form == FDS_MFIE || form == FDS_CFIE || form == FDS_YCFIE, FDS_ERR_ARG,
                "bad form");
    FDS_REQUIRE(std::isfinite(o->alpha), FDS_ERR_ARG, "alpha must be finite");
    if (form == FDS_CFIE || form == FDS_YCFIE)
        FDS_REQUIRE(std::fabs(1.0 + 2.0 * o->alpha) > 1e-12, FDS_ERR_ARG, "CFIE with beta = 0");
    FDS_REQUIRE(o->rank_cap >= 0 && o->oversample >= 0 && o->power_iters >= 0 && o->tol >= 0.0, FDS_ERR_ARG,
                "bad compression options");
    FDS_REQUIRE(o->sweeps >= 0 && o->sweeps <= 1000, FDS_ERR_ARG, "sweeps out of range");
    for (int64_t i = 0; i < nb; ++i) {
        const fds_problem& p = probs[i];
        FDS_REQUIRE(p.nodes && p.angles && p.amps && p.j_out, FDS_ERR_ARG, "NULL pointer in a problem");
        FDS_REQUIRE(p.n >= 8 && p.n <= (int64_t)1 << 20, FDS_ERR_ARG, "n must be in [8, 2^20]");
        FDS_REQUIRE(p.n_modes >= 1 && p.n_modes <= p.n, FDS_ERR_ARG, "n_modes must be in [1, n]");
        FDS_REQUIRE(p.nrhs >= 1, FDS_ERR_ARG, "nrhs must be >= 1");
    }
    Ctx& c = ctx->impl;
    auto* b = new fds_batch_s();
    b->c = &c;
    b->sweeps = o->sweeps;
    try {
        fds_asm_opts ao{};
        ao.precision = o->precision;
        for (int64_t i = 0; i < nb; ++i)
            b->ops.push_back(new_operator(c, probs[i].nodes, probs[i].n, probs[i].k, &ao));
        std::vector<Op*> ops;
        for (auto* op : b->ops) ops.push_back(&op->impl);
        launch_assemble_batch(c, ops.data(), (int)nb);
        for (Op* op : ops) op->stage = Stage::Assembled;
        std::vector<int> nm(nb);
        for (int64_t i = 0; i < nb; ++i) nm[i] = probs[i].n_modes;
        if (o->precision == FDS_FP64 && form != FDS_YCFIE) {
            run_filter_batch(ops.data(), (int)nb, form, o->alpha, nm.data(), true, 1e-6);
        } else {
            for (int64_t i = 0; i < nb; ++i) run_filter(*ops[i], form, o->alpha, nm[i], true, 1e-6);
        }
        for (Op* op : ops) {
            run_compress(*op, o->rank_cap > 0 ? o->rank_cap : op->n_eff, o->oversample, o->power_iters, o->tol,
                         o->seed);
            run_factor(*op);
        }
        for (int64_t i = 0; i < nb; ++i) {
            const fds_problem& p = probs[i];
            const size_t blk = sizeof(double2) * (size_t)p.n * (size_t)p.nrhs;
            BatchItem it{};
            it.angles = p.angles;
            it.amps = static_cast<const double2*>(p.amps);
            it.nrhs = p.nrhs;
            it.j = static_cast<double2*>(p.j_out);
            double2** slots[4] = {&it.f, &it.h, &it.w, &it.t};
            for (int s = 0; s < 4; ++s) {
                if (s == 1 && !(form == FDS_MFIE || form == FDS_CFIE || form == FDS_YCFIE)) continue;
                *slots[s] = static_cast<double2*>(c.dmalloc(blk));
                b->bufs.push_back(*slots[s]);
            }
            b->items.push_back(it);
        }
        // chains: longest problems first, each to the least loaded chain
        const int nch = (int)std::min<int64_t>(nb, kBatchChains);
        std::vector<int64_t> order(nb);
        for (int64_t i = 0; i < nb; ++i) order[i] = i;
        auto cost = [&](int64_t i) { return (double)probs[i].n * (double)probs[i].n * (double)probs[i].nrhs; };
        std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t z) { return cost(a) > cost(z); });
        std::vector<double> load(nch, 0.0);
        b->chain.assign(nb, 0);
        b->chain_bytes.assign(nch, 0);
        for (int64_t i : order) {
            const int ch = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            load[ch] += cost(i);
            b->chain[i] = ch;
            // residual and small products (3/4 of the workspace), then room for the
            // split-K partial sums of the right-hand-side product (4 n nrhs complex)
            const Op& op = *ops[i];
            const size_t zr = (size_t)std::max({op.rank, op.n_eff, 1});
            const size_t need = (size_t)16 * probs[i].nrhs * ((size_t)op.n + zr) / 3 * 4 +
                                (size_t)64 * op.n * probs[i].nrhs + ((size_t)4 << 20);
            b->chain_bytes[ch] = std::max(b->chain_bytes[ch], (need + 255) / 256 * 256);
        }
        for (int ch = 0; ch < nch; ++ch) {
            b->chain_ws.push_back(c.dmalloc(b->chain_bytes[ch]));
            b->bufs.push_back(b->chain_ws.back());
        }
        // one eager run: builds whatever the solves create lazily and checks
        // that nothing allocates before anything is recorded
        for (int64_t i = 0; i < nb; ++i)
            run_batch_item(*ops[i], b->items[i], b->sweeps, b->chain_ws[b->chain[i]], b->chain_bytes[b->chain[i]]);
        b->exec = capture_batch(*b);
    } catch (...) {
        delete b;
        throw;
    }
    return b;
}

fds_status fds_batch_create(fds_ctx ctx, int64_t nb, const fds_problem* probs, const fds_batch_opts* opts,
                            fds_batch* out) {
    return guarded([&] {
        FDS_REQUIRE(out != nullptr, FDS_ERR_ARG, "out is NULL");
        *out = nullptr;
        *out = make_batch(ctx, nb, probs, opts);
    });
}

fds_status fds_batch_replay(fds_batch b) {
    return guarded([&] {
        FDS_REQUIRE(b && b->exec, FDS_ERR_ARG, "bad batch");
        FDS_HIP_TRY(hipGraphLaunch(b->exec, b->c->stream));
    });
}

fds_status fds_batch_op(fds_batch b, int64_t i, fds_op* op) {
    return guarded([&] {
        FDS_REQUIRE(b && op && i >= 0 && i < (int64_t)b->ops.size(), FDS_ERR_ARG, "bad argument");
        *op = b->ops[i];
    });
}

fds_status fds_batch_destroy(fds_batch b) {
    return guarded([&] { delete b; });
}

fds_status fds_batch_run(fds_ctx ctx, int64_t nb, const fds_problem* probs, const fds_batch_opts* opts) {
    return guarded([&] {
        std::unique_ptr<fds_batch_s> b(make_batch(ctx, nb, probs, opts));
        FDS_HIP_TRY(hipGraphLaunch(b->exec, b->c->stream));
        FDS_HIP_TRY(hipStreamSynchronize(b->c->stream));
    });
}

fds_status fds_farfield(fds_op op, const void* j, int64_t nrhs, const double* thetas, int64_t nang, void* out) {
    return guarded([&] {
        FDS_REQUIRE(op && j && thetas && out && nrhs >= 0 && nang >= 0 && nang < (1 << 24), FDS_ERR_ARG,
                    "bad argument");
        if (nrhs == 0 || nang == 0) return;
        run_farfield(op->impl, (const double2*)j, nrhs, thetas, (int)nang, (double2*)out);
    });
}

fds_status fds_farfield_objective_grad(fds_op op, const double* angles, const void* amps, int64_t nrhs,
                                       const double* thetas, int64_t nang, const void* target,
                                       const fds_solve_opts* opts, double* J, double* grad_nodes,
                                       void* grad_amps, void* farfield_out, fds_solve_stats* stats) {
    return guarded([&] {
        FDS_REQUIRE(op && angles && amps && thetas && target && J && grad_nodes && grad_amps, FDS_ERR_ARG,
                    "NULL argument");
        FDS_REQUIRE(nrhs >= 1 && nang >= 1 && nang < (1 << 24) && nrhs < (1 << 24), FDS_ERR_ARG, "bad sizes");
        require_stage(op->impl, Stage::Factored, "fds_farfield_objective_grad");
        FDS_REQUIRE(op->impl.form == FDS_EFIE, FDS_ERR_NOTIMPL, "the adjoint gradient uses the EFIE model");
        int it = 8;
        double tol = 1e-12;
        if (opts) {
            FDS_REQUIRE(opts->precision == FDS_FP64, FDS_ERR_NOTIMPL, "only FP64 solves are implemented");
            it = opts->max_iters;
            tol = opts->tol;
        }
        FDS_REQUIRE(it >= 0 && it <= 1000, FDS_ERR_ARG, "max_iters out of range");
        run_farfield_grad(op->impl, angles, (const double2*)amps, nrhs, thetas, (int)nang, (const double2*)target,
                          it, tol, J, grad_nodes, (double2*)grad_amps, (double2*)farfield_out, stats);
    });
}

}  // extern "C"
