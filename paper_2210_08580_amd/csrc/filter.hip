// Laplacian filter basis (paper, Laplacian Filters, 2D case, eq. LapFilter,
// with the orthonormalised Laplacian G^{-1/2} L G^{-1/2} for non-uniform
// meshes): the n smallest eigenpairs of the periodic tridiagonal pencil
// L v = lambda G v (P1 stiffness and mass matrices). With V_g the
// G-orthonormal generalised eigenvectors, V_n = G^{1/2} V_g are the
// orthonormal eigenvectors of G^{-1/2} L G^{-1/2}.
//
// Eigenvalues: bisection on Sylvester inertia counts. The periodic
// tridiagonal L - sigma G is reordered as a block tridiagonal matrix of 2x2
// blocks by pairing node k with node n-1-k; the block LDL^T recurrence
// A_{k+1} = D_{k+1} - E_k A_k^{-1} E_k then gives the count of negative
// eigenvalues as the sum over blocks; it runs from both ends of the block
// sequence at once (two chains of half the length per lane, then the meeting
// block). One workgroup of four wavefronts refines one eigenvalue, its 256 lanes
// evaluating 256 shifts per round (multisection).
// Eigenvectors: inverse iteration (L - lambda G) x_new = G x_old with a banded
// LU with partial pivoting of the same folded ordering (bandwidth 2), run from
// both ends of the band at once (one thread per eigenvalue and half, a 4 x 4
// interface system in the middle), G-Gram-Schmidt inside clusters of close
// eigenvalues, and a final Newton-Schulz orthonormalisation in the G inner product.
#include <algorithm>
#include <cmath>
#include <vector>

#include "fds_internal.h"
#include "linalg.h"

namespace fds {

struct Pencil {
    const double* __restrict__ ld;
    const double* __restrict__ lo;
    const double* __restrict__ gd;
    const double* __restrict__ go;
    int n;
};

__device__ __forceinline__ double pm(const Pencil& P, int i, double s) { return P.ld[i] - s * P.gd[i]; }
__device__ __forceinline__ double pf(const Pencil& P, int i, double s) { return P.lo[i] - s * P.go[i]; }

// number of eigenvalues of the pencil below s
__device__ int pencil_count(const Pencil& P, double s) {
    const int n = P.n;
    const int K = n / 2;                       // node pairs (k, n-1-k)
    const bool odd = (n & 1) != 0;
    const double tiny = 1e-290;
    double a = pm(P, 0, s), c = pm(P, n - 1, s), b = pf(P, n - 1, s);
    if (!odd && K == 1) b += pf(P, 0, s);
    int cnt = 0;
    for (int k = 0;; ++k) {
        double det = a * c - b * b;
        if (fabs(det) < tiny) det = det < 0.0 ? -tiny : tiny;
        cnt += det < 0.0 ? 1 : (a < 0.0 ? 2 : 0);
        if (k == K - 1) {
            if (odd) {
                const int sN = (n - 1) / 2;
                const double u1 = pf(P, sN - 1, s), u2 = pf(P, sN, s);
                const double val = pm(P, sN, s) - (u1 * u1 * c - 2.0 * u1 * u2 * b + u2 * u2 * a) / det;
                cnt += val < 0.0 ? 1 : 0;
            }
            break;
        }
        const double e1 = pf(P, k, s), e2 = pf(P, n - 2 - k, s);
        const double inv = 1.0 / det;
        const double an = pm(P, k + 1, s) - e1 * e1 * c * inv;
        const double cn = pm(P, n - 2 - k, s) - e2 * e2 * a * inv;
        double bn = e1 * e2 * b * inv;
        if (!odd && k + 1 == K - 1) bn += pf(P, K - 1, s);   // nodes n/2-1 and n/2 are adjacent
        a = an;
        b = bn;
        c = cn;
    }
    return cnt;
}

__device__ __forceinline__ double bcast(double v, int l) {
    const uint64_t u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Inertia count for the shift s held by this lane; the whole wave walks the
// same block sequence, so the pencil entries of 64 consecutive block steps are
// loaded once (one step per lane) and broadcast from registers.
__device__ int pencil_count_wave(const Pencil& P, double s) {
    const int n = P.n;
    const int K = n / 2;
    const bool odd = (n & 1) != 0;
    const double tiny = 1e-290;
    const int lane = threadIdx.x & 63;
    double a = pm(P, 0, s), c = pm(P, n - 1, s), b = pf(P, n - 1, s);
    int cnt = 0;
    for (int k0 = 0; k0 < K; k0 += 64) {
        // step k (k0 <= k < K-1) needs f(k), f(n-2-k), m(k+1), m(n-2-k)
        const int kk = min(k0 + lane, K - 1);
        const double lo1 = P.lo[kk], go1 = P.go[kk], lo2 = P.lo[n - 2 - kk], go2 = P.go[n - 2 - kk];
        const double ld1 = P.ld[min(kk + 1, n - 1)], gd1 = P.gd[min(kk + 1, n - 1)];
        const double ld2 = P.ld[n - 2 - kk], gd2 = P.gd[n - 2 - kk];
        const int kend = min(64, K - k0);
        for (int l = 0; l < kend; ++l) {
            const int k = k0 + l;
            double det = a * c - b * b;
            if (fabs(det) < tiny) det = det < 0.0 ? -tiny : tiny;
            cnt += det < 0.0 ? 1 : (a < 0.0 ? 2 : 0);
            if (k == K - 1) {
                if (odd) {
                    const int sN = (n - 1) / 2;
                    const double u1 = pf(P, sN - 1, s), u2 = pf(P, sN, s);
                    const double val = pm(P, sN, s) - (u1 * u1 * c - 2.0 * u1 * u2 * b + u2 * u2 * a) / det;
                    cnt += val < 0.0 ? 1 : 0;
                }
                break;
            }
            const double e1 = bcast(lo1, l) - s * bcast(go1, l);
            const double e2 = bcast(lo2, l) - s * bcast(go2, l);
            const double m1 = bcast(ld1, l) - s * bcast(gd1, l);
            const double m2 = bcast(ld2, l) - s * bcast(gd2, l);
            const double inv = 1.0 / det;
            const double an = m1 - e1 * e1 * c * inv;
            const double cn = m2 - e2 * e2 * a * inv;
            double bn = e1 * e2 * b * inv;
            if (!odd && k + 1 == K - 1) bn += pf(P, K - 1, s);   // nodes n/2-1 and n/2 are adjacent
            a = an;
            b = bn;
            c = cn;
        }
    }
    return cnt;
}

// one wavefront per eigenvalue index (first + i)
__global__ __launch_bounds__(64) void bisect_kernel(Pencil P, double glo, double ghi, double rtol, double atol,
                                                    int first, int nw, double* __restrict__ lam) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x;
    if (i >= nw) return;
    const int idx = first + i;
    double lo = glo, hi = ghi;
    for (int it = 0; it < 64; ++it) {
        const double w = hi - lo;
        if (w <= fmax(rtol * fmax(fabs(lo), fabs(hi)), atol)) break;
        const double s = lo + w * (double)(lane + 1) / 65.0;
        const int cnt = pencil_count_wave(P, s);
        const unsigned long long mask = __ballot(cnt > idx);
        const int l = mask ? (__ffsll(mask) - 1) : 64;
        const double nlo = (l == 0) ? lo : lo + w * (double)l / 65.0;
        const double nhi = (l == 64) ? hi : lo + w * (double)(l + 1) / 65.0;
        if (!(nhi - nlo < w)) break;
        lo = nlo;
        hi = nhi;
    }
    if (lane == 0) lam[i] = 0.5 * (lo + hi);
}

// ---------------------------------------------------------------- scaled inertia count
// Step k (0 <= k < K-1) of the block recurrence over the node pairs (k, n-1-k):
// coupling E_k = diag(f(k), f(n-2-k)), next diagonal block D = [[m(k+1), x], [x, m(n-2-k)]]
// with x = f(K-1) on the last step of an even n (the middle nodes are adjacent), else 0.
struct SturmStep {
    double lo1, go1, lo2, go2, ld1, gd1, ld2, gd2, xl, xg;
};

// Entry k (0 <= k < K) of the table of the bottom-up recurrence: the coupling
// E_k = diag(f(k), f(n-2-k)) to block k+1 and the diagonal block
// D_k = [[m(k), x_k], [x_k, m(n-1-k)]] (x_0 = f(n-1), x_{K-1} = f(K-1) for an even
// n, else 0), in the fields (lo1, go1), (lo2, go2), (ld1, gd1), (ld2, gd2), (xl, xg).
__global__ void sturm_steps_kernel(Pencil P, SturmStep* __restrict__ st, SturmStep* __restrict__ sb) {
    const int n = P.n, K = n / 2;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const bool odd = (n & 1) != 0;
    if (k < K && k + 1 < n) {
        SturmStep b;
        b.lo1 = P.lo[k];
        b.go1 = P.go[k];
        b.lo2 = P.lo[n - 2 - k];
        b.go2 = P.go[n - 2 - k];
        b.ld1 = P.ld[k];
        b.gd1 = P.gd[k];
        b.ld2 = P.ld[n - 1 - k];
        b.gd2 = P.gd[n - 1 - k];
        const bool xk = k == 0 || (!odd && k == K - 1);
        const int xo = k == 0 ? n - 1 : K - 1;
        b.xl = xk ? P.lo[xo] : 0.0;
        b.xg = xk ? P.go[xo] : 0.0;
        sb[k] = b;
    }
    if (k >= K - 1) return;
    SturmStep t;
    t.lo1 = P.lo[k];
    t.go1 = P.go[k];
    t.lo2 = P.lo[n - 2 - k];
    t.go2 = P.go[n - 2 - k];
    t.ld1 = P.ld[k + 1];
    t.gd1 = P.gd[k + 1];
    t.ld2 = P.ld[n - 2 - k];
    t.gd2 = P.gd[n - 2 - k];
    const bool mid = !odd && k + 1 == K - 1;
    t.xl = mid ? P.lo[K - 1] : 0.0;
    t.xg = mid ? P.go[K - 1] : 0.0;
    st[k] = t;
}

// Number of eigenvalues of the pencil below s by the block LDL^T recurrence
// A_{k+1} = D_{k+1} - E_k A_k^{-1} E_k carried without division: B_k = s_k A_k with
//     B_{k+1} = det(B_k) D_{k+1} - s_k E_k adj(B_k) E_k,   s_{k+1} = det(B_k),
// (a block's inertia is read from sign det(B_k) = sign det(A_k) and
// sign(b11) sign(s_k) = sign(a_k)), and B_k, s_k rescaled together by a power
// of two after every step. The dependency chain per step is a few FMAs.
// Power-of-two factor 2^-e with e the binary exponent of v (v > 0 finite).
__device__ __forceinline__ double inv_pow2_of(double v) {
    const long long bits = __double_as_longlong(v);
    const long long e = (bits >> 52) & 0x7ff;             // biased exponent of v
    return __longlong_as_double((2046 - e) << 52);          // 2^(1023 - (e - 1023)) = 2^-(e-1023)
}

constexpr int BS_WAVES = 4;            // wavefronts per eigenvalue: 256 shifts per round
constexpr int BS_CHUNK = 64 * BS_WAVES;  // recurrence steps staged in LDS at a time

__device__ int pencil_count_scaled(const Pencil& P, const SturmStep* __restrict__ st, double sig,
                                   SturmStep* __restrict__ sh) {
    const int n = P.n;
    const int K = n / 2;
    const bool odd = (n & 1) != 0;
    double b11 = pm(P, 0, sig), b22 = pm(P, n - 1, sig), b12 = pf(P, n - 1, sig), sc = 1.0;
    int cnt = 0;
    for (int k0 = 0; k0 < K - 1; k0 += BS_CHUNK) {
        const int kend = min(K - 1, k0 + BS_CHUNK);
        __syncthreads();
        if (k0 + (int)threadIdx.x < kend) sh[threadIdx.x] = st[k0 + threadIdx.x];
        __syncthreads();
        // Two steps per iteration with two coefficient sets: the set of step k + 1 is
        // read from LDS while step k runs and that of k + 2 while k + 1 runs, so the
        // loads overlap the arithmetic and no register copies are needed. B and s are
        // rescaled every fourth step (one step changes their magnitude by well under
        // 1e40, far inside the exponent range). An exactly singular leading block
        // (det = 0) counts as a tiny positive determinant.
        auto step = [&](const SturmStep& t, int k) {
            double det = fma(b11, b22, -b12 * b12);
            det = det == 0.0 ? 1e-300 : det;
            cnt += det < 0.0 ? 1 : ((b11 < 0.0) != (sc < 0.0) ? 2 : 0);
            const double e1 = fma(-sig, t.go1, t.lo1), e2 = fma(-sig, t.go2, t.lo2);
            const double m1 = fma(-sig, t.gd1, t.ld1), m2 = fma(-sig, t.gd2, t.ld2);
            const double x = fma(-sig, t.xg, t.xl);
            const double s1 = sc * e1, s2 = sc * e2;
            const double n11 = fma(det, m1, -(s1 * e1) * b22);
            const double n22 = fma(det, m2, -(s2 * e2) * b11);
            const double n12 = fma(det, x, (s1 * e2) * b12);
            if ((k & 3) == 3) {
                const double f = inv_pow2_of(fmax(fmax(fabs(n11), fabs(n22)), fmax(fabs(n12), 1e-300)));
                b11 = n11 * f;
                b22 = n22 * f;
                b12 = n12 * f;
                sc = det * f;
            } else {
                b11 = n11;
                b22 = n22;
                b12 = n12;
                sc = det;
            }
        };
        SturmStep ta = sh[0];
        int k = k0;
        for (; k + 1 < kend; k += 2) {
            const SturmStep tb = sh[k + 1 - k0];
            step(ta, k);
            ta = sh[min(k + 2, kend - 1) - k0];
            step(tb, k + 1);
        }
        if (k < kend) step(ta, k);
    }
    double det = fma(b11, b22, -b12 * b12);
    det = det == 0.0 ? 1e-300 : det;
    cnt += det < 0.0 ? 1 : ((b11 < 0.0) != (sc < 0.0) ? 2 : 0);
    if (odd) {
        // middle node: val = m - (u1^2 c - 2 u1 u2 b + u2^2 a)/det(A), with A = B/sc
        const int sN = (n - 1) / 2;
        const double u1 = pf(P, sN - 1, sig), u2 = pf(P, sN, sig);
        const double q = u1 * u1 * b22 - 2.0 * u1 * u2 * b12 + u2 * u2 * b11;
        const double v = fma(pm(P, sN, sig), det, -sc * q);
        cnt += ((v < 0.0) != (det < 0.0)) ? 1 : 0;
    }
    return cnt;
}

// One step of the scaled block recurrence (top-down from block k to k+1, or
// bottom-up from block k+1 to k with the bottom table): counts the inertia of the
// current block B / s, then B <- det(B) D - s E adj(B) E, s <- det(B), rescaled by
// a power of two when `rescale`.
__device__ __forceinline__ void sturm_step(const SturmStep& t, double sig, bool rescale, double& b11, double& b22,
                                           double& b12, double& sc, int& cnt) {
    double det = fma(b11, b22, -b12 * b12);
    det = det == 0.0 ? 1e-300 : det;
    cnt += det < 0.0 ? 1 : ((b11 < 0.0) != (sc < 0.0) ? 2 : 0);
    const double e1 = fma(-sig, t.go1, t.lo1), e2 = fma(-sig, t.go2, t.lo2);
    const double m1 = fma(-sig, t.gd1, t.ld1), m2 = fma(-sig, t.gd2, t.ld2);
    const double x = fma(-sig, t.xg, t.xl);
    const double s1 = sc * e1, s2 = sc * e2;
    const double n11 = fma(det, m1, -(s1 * e1) * b22);
    const double n22 = fma(det, m2, -(s2 * e2) * b11);
    const double n12 = fma(det, x, (s1 * e2) * b12);
    if (rescale) {
        const double f = inv_pow2_of(fmax(fmax(fabs(n11), fabs(n22)), fmax(fabs(n12), 1e-300)));
        b11 = n11 * f;
        b22 = n22 * f;
        b12 = n12 * f;
        sc = det * f;
    } else {
        b11 = n11;
        b22 = n22;
        b12 = n12;
        sc = det;
    }
}

// The same inertia count with the block elimination run from both ends at once
// (Sylvester's law holds for any elimination order): blocks 0 .. M-1 top-down and
// K-1 .. M+1 bottom-up (the middle node of an odd n first), two independent
// chains per lane of half the length, then the meeting block
// A_M + C_M - D_M (the Schur complements of both sides). sb: bottom table.
__device__ int pencil_count_2e(const Pencil& P, const SturmStep* __restrict__ st, const SturmStep* __restrict__ sb,
                               double sig, SturmStep* __restrict__ shT, SturmStep* __restrict__ shB) {
    const int n = P.n;
    const int K = n / 2;
    const bool odd = (n & 1) != 0;
    const int M = (K - 1) / 2;
    const int LT = M, LB = K - 1 - M;   // LB = LT or LT + 1
    double b11 = pm(P, 0, sig), b22 = pm(P, n - 1, sig), b12 = pf(P, n - 1, sig), sc = 1.0;
    double c11, c22, c12, tc;
    int cnt = 0;
    if (odd) {
        // the middle node K, coupled to nodes K-1 and K+1 of block K-1 by f(K-1), f(K)
        double cm = pm(P, K, sig);
        cm = cm == 0.0 ? 1e-300 : cm;
        cnt += cm < 0.0 ? 1 : 0;
        const double u1 = pf(P, K - 1, sig), u2 = pf(P, K, sig);
        c11 = fma(cm, pm(P, K - 1, sig), -u1 * u1);
        c22 = fma(cm, pm(P, K + 1, sig), -u2 * u2);
        c12 = -u1 * u2;
        tc = cm;
    } else {
        c11 = pm(P, K - 1, sig);
        c22 = pm(P, K, sig);
        c12 = pf(P, K - 1, sig);
        tc = 1.0;
    }
    for (int j0 = 0; j0 < LB; j0 += BS_CHUNK) {
        const int jend = min(LB, j0 + BS_CHUNK);
        __syncthreads();
        const int t = (int)threadIdx.x;
        if (j0 + t < LT) shT[t] = st[j0 + t];
        if (j0 + t < LB) shB[t] = sb[K - 2 - (j0 + t)];
        __syncthreads();
        // two steps of each chain per iteration with two coefficient sets, so that the
        // LDS reads of the next steps overlap the arithmetic (no register copies)
        SturmStep ta = shT[0], ba = shB[0];
        for (int j = j0; j < jend; j += 2) {
            const int l1 = min(j + 1, jend - 1) - j0;
            const SturmStep tb = shT[l1], bb = shB[l1];
            if (j < LT) sturm_step(ta, sig, (j & 3) == 3, b11, b22, b12, sc, cnt);
            sturm_step(ba, sig, (j & 3) == 3, c11, c22, c12, tc, cnt);
            const int l2 = min(j + 2, jend - 1) - j0;
            ta = shT[l2];
            ba = shB[l2];
            if (j + 1 < jend) {
                if (j + 1 < LT) sturm_step(tb, sig, ((j + 1) & 3) == 3, b11, b22, b12, sc, cnt);
                sturm_step(bb, sig, ((j + 1) & 3) == 3, c11, c22, c12, tc, cnt);
            }
        }
    }
    // meeting block: A_M = B / s, C_M = C / t, both holding D_M once
    const SturmStep d = sb[M];
    const double is = 1.0 / sc, it = 1.0 / tc;
    const double m1 = fma(-sig, d.gd1, d.ld1), m2 = fma(-sig, d.gd2, d.ld2), x = fma(-sig, d.xg, d.xl);
    const double a11 = fma(b11, is, fma(c11, it, -m1));
    const double a22 = fma(b22, is, fma(c22, it, -m2));
    const double a12 = fma(b12, is, fma(c12, it, -x));
    double det = fma(a11, a22, -a12 * a12);
    det = det == 0.0 ? 1e-300 : det;
    cnt += det < 0.0 ? 1 : (a11 < 0.0 ? 2 : 0);
    return cnt;
}

// the two-ended count from this many node pairs on
constexpr int BS_TWO_ENDED_K = 64;

// One workgroup per eigenvalue index first + i. Each round evaluates 256 shifts
// spread over [lo, hi] (endpoints included) and keeps the sub-interval that
// holds the eigenvalue. The first round tries the caller's tight bracket
// (lo0[i], hi0[i]) and falls back to the global bracket when its endpoint counts
// do not enclose the index.
__global__ __launch_bounds__(64 * BS_WAVES) void bisect_scaled_kernel(Pencil P, const SturmStep* __restrict__ st,
                                                                      const SturmStep* __restrict__ sb,
                                                                      double l1c, double hfac, double glo,
                                                                      double ghi, double rtol, double atol,
                                                                      int first, int nw, double* __restrict__ lam) {
    __shared__ unsigned long long mk[BS_WAVES];
    __shared__ int flags[2];
    __shared__ SturmStep stsh[BS_CHUNK];
    __shared__ SturmStep stsb[BS_CHUNK];
    const bool two_ended = P.n / 2 >= BS_TWO_ENDED_K;
    const int i = blockIdx.x;
    if (i >= nw) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int idx = first + i;
    const int NS = 64 * BS_WAVES;
    // tight bracket: eigenvalue idx of the P1 pencil lies above lc = l1c ceil(idx/2)^2 (the
    // polygon's Laplace-Beltrami eigenvalue, of which the P1 value is a Rayleigh-Ritz
    // upper bound) by about the interpolation excess lc^2 <h^2>/12 (hfac = <h^2>/12 with
    // <h^2> = sum h^3 / sum h); measured on star, ellipse, random and perturbed curves
    // the deviation from lc (1 + hfac lc) stays within 0.32 of that excess, so the
    // bracket [lc (1 + 0.2 hfac lc), lc (1 + 1.6 hfac lc)] with small safety margins
    double lo, hi;
    if (idx == 0) {
        lo = -1e-6 * l1c;
        hi = 0.5 * l1c;
    } else {
        const double kk = (double)((idx + 1) / 2);
        const double lc = l1c * kk * kk;
        lo = lc * (1.0 + 0.2 * hfac * lc) * (1.0 - 1e-9);
        hi = lc * (1.0 + 1.6 * hfac * lc) * (1.0 + 1e-9) + 1e-9 * l1c;
    }
    if (!(hi > lo)) {
        lo = glo;
        hi = ghi;
    }
    bool checked = false;
    for (int it = 0; it < 48; ++it) {
        const double w = hi - lo;
        if (w <= fmax(rtol * fmax(fabs(lo), fabs(hi)), atol)) break;
        const double s = tid == NS - 1 ? hi : lo + w * (double)tid / (double)(NS - 1);
        const int cnt = two_ended ? pencil_count_2e(P, st, sb, s, stsh, stsb) : pencil_count_scaled(P, st, s, stsh);
        const unsigned long long m = __ballot(cnt > idx);
        if (lane == 0) mk[wv] = m;
        if (tid == 0) flags[0] = cnt > idx;                 // eigenvalue below lo
        if (tid == NS - 1) flags[1] = cnt <= idx;           // eigenvalue above hi
        __syncthreads();
        int j = NS;
        for (int q = 0; q < BS_WAVES; ++q)
            if (mk[q]) {
                j = q * 64 + __ffsll(mk[q]) - 1;
                break;
            }
        const bool bad = flags[0] || flags[1];
        __syncthreads();
        if (bad) {
            if (checked) break;   // cannot happen for a valid global bracket; keep the last interval
            lo = glo;
            hi = ghi;
            checked = true;
            continue;
        }
        checked = true;
        // j >= 1: count(s_{j-1}) <= idx < count(s_j)
        const double nlo = lo + w * (double)(j - 1) / (double)(NS - 1);
        const double nhi = j == NS - 1 ? hi : lo + w * (double)j / (double)(NS - 1);
        if (!(nhi - nlo < w)) break;
        lo = nlo;
        hi = nhi;
    }
    if (tid == 0) lam[i] = 0.5 * (lo + hi);
}

// ---------------------------------------------------------------- folded ordering
__device__ __forceinline__ int node_of(int r, int n) {
    if ((n & 1) && r == n - 1) return (n - 1) / 2;
    return (r & 1) ? n - 1 - (r >> 1) : (r >> 1);
}

// Folded band of L and of G: entries [t][r] = X[node(r)][node(r + t - 2)], t = 0..4
// (zero outside the matrix), so that L - sigma G = Lb - sigma Gb in band form.
__global__ void fold_bands_kernel(Pencil P, double* __restrict__ Lb, double* __restrict__ Gb) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = P.n;
    if (r >= n) return;
    const int a = node_of(r, n);
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        const int cpos = r + t - 2;
        double vl = 0.0, vg = 0.0;
        if (cpos >= 0 && cpos < n) {
            const int b = node_of(cpos, n);
            if (b == a) { vl = P.ld[a]; vg = P.gd[a]; }
            else if (b == (a + 1 == n ? 0 : a + 1)) { vl = P.lo[a]; vg = P.go[a]; }
            else if (a == (b + 1 == n ? 0 : b + 1)) { vl = P.lo[b]; vg = P.go[b]; }
        }
        Lb[(int64_t)t * n + r] = vl;
        Gb[(int64_t)t * n + r] = vg;
    }
}

// ---------------------------------------------------------------- two-ended inverse iteration
// The folded band A = L - sigma G (bandwidth 2) is eliminated from both ends at
// once: the top half eliminates columns 0 .. mt-1 downward (rows j, j+1, j+2 as
// pivot candidates, partial pivoting), the bottom half eliminates columns
// n-1 .. n-mb upward, i.e. the same downward elimination of the reversed matrix
// A' = J A J (A'[j][j + t - 2] is band entry 4 - t of row n-1-j), with
// mt + mb = n - 4. The rows each half touches are disjoint (top: rows <= mt+1,
// bottom: rows >= mt+2), so both are the partial-pivoting LU steps of the
// one-ended elimination, and they leave four rows coupling the four unknowns
// x_{mt} .. x_{mt+3}: the two reduced rows of each half. That 4 x 4 system is
// solved with partial pivoting, then each half back-substitutes outward.
// One thread per (eigenvalue, half); the chains are n/2 long instead of n.
//
// Factor records, per half, as separate arrays indexed [step j][eigenvalue i]
// (each wave's load of one field is one contiguous 512 or 1024-byte run):
// multipliers (l1, l2), (u_{j,j+1}, u_{j,j+2}), (u_{j,j+3}, u_{j,j+4}), (1/u_jj, z_j)
// with z the forward-eliminated right-hand side of the current solve, and the
// pivot choice (0, 1, 2). M = steps x eigenvalues entries per array.
struct FacView {
    double2* L;
    double2* U12;
    double2* U34;
    double2* IZ;
    int* P;
};

__host__ __device__ inline size_t fac_half_bytes(int64_t M) { return (size_t)M * (4 * 16 + 4); }

__device__ __forceinline__ FacView fac_view(char* base, int64_t M, int h) {
    char* b = base + (size_t)h * fac_half_bytes(M);
    FacView f;
    f.L = reinterpret_cast<double2*>(b);
    f.U12 = reinterpret_cast<double2*>(b + (size_t)M * 16);
    f.U34 = reinterpret_cast<double2*>(b + (size_t)M * 32);
    f.IZ = reinterpret_cast<double2*>(b + (size_t)M * 48);
    f.P = reinterpret_cast<int*>(b + (size_t)M * 64);
    return f;
}

__device__ __forceinline__ int trow(int h, int j, int n) { return h == 0 ? j : n - 1 - j; }

// Entry (row, i) of a [rows][nw] array by a 32-bit byte offset from its uniform base
// (the host keeps these arrays below 4 GiB): one offset per lane instead of a
// 64-bit address per array.
template <typename T>
__device__ __forceinline__ T* at32(T* base, int row, int nw, int i) {
    const uint32_t off = ((uint32_t)row * (uint32_t)nw + (uint32_t)i) * (uint32_t)sizeof(T);
    return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off);
}
template <typename T>
__device__ __forceinline__ const T* at32(const T* base, int row, int nw, int i) {
    const uint32_t off = ((uint32_t)row * (uint32_t)nw + (uint32_t)i) * (uint32_t)sizeof(T);
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}

// 1/d: hardware reciprocal estimate refined by two Newton steps r <- r + r (1 - d r)
__device__ __forceinline__ double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

// Pseudo-random start vector entries in [-1/2, 1/2): Marsaglia's xorshift32
// (J. Stat. Softw. 8(14), 2003; shifts 13, 17, 5) run along the rows each half
// eliminates, from a seed mixed from (eigenvalue index, half). Every row enters
// exactly one half's window once, so this defines one start vector per
// eigenvalue; six shift/xor operations per row beside the elimination.
struct StartSeq {
    uint32_t z;
    __device__ StartSeq(int i, int h) {
        z = (uint32_t)i * 0x9E3779B1u ^ (uint32_t)(h + 1) * 0x85EBCA77u;
        z ^= z >> 15;
        z *= 0x2C1B3C6Du;
        z ^= z >> 12;
        z |= 1u;   // xorshift32 has no zero state
    }
    __device__ __forceinline__ double next() {
        z ^= z << 13;
        z ^= z >> 17;
        z ^= z << 5;
        return (double)z * (1.0 / 4294967296.0) - 0.5;
    }
};

// Factorisation of both halves (blockIdx.y = half) with the forward elimination
// of the pseudo-random right-hand side (the first inverse-iteration step): z into
// the factor records, the reduced interface rows and their right-hand sides into IF
// ([half][10][nw]: row mt (or mt+3) coefficients, row mt+1 (or mt+2)
// coefficients, two right-hand sides).
__global__ __launch_bounds__(64) void invit_factor_kernel(int n, int mt, int mb, const double* __restrict__ Lb,
                                                          const double* __restrict__ Gb,
                                                          const double* __restrict__ sig, int nw, double pivmin,
                                                          char* __restrict__ fac, int64_t M,
                                                          double* __restrict__ IF) {
    const int h = blockIdx.y;
    const int m = h == 0 ? mt : mb;
    const int lane = threadIdx.x & 63;
    const int i0 = blockIdx.x * 64 + lane;
    const int i = min(i0, nw - 1);          // idle lanes repeat the last eigenvalue, store nothing
    const bool act = i0 < nw;
    const double s = sig[i];
    const FacView F = fac_view(fac, M, h);
    auto band = [&](const double* B, int t, int j) {   // entry t of row j of A (h = 0) or A' (h = 1)
        return h == 0 ? B[(int64_t)t * n + j] : B[(int64_t)(4 - t) * n + (n - 1 - j)];
    };
    // window rows A, B, C (the rows j, j+1, j+2 of the partly eliminated band,
    // shifted to the columns j .. j+4) and their right-hand-side entries
    double A[5], Bw[5], Cw[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        A[t] = t + 2 < 5 ? band(Lb, t + 2, 0) - s * band(Gb, t + 2, 0) : 0.0;
        Bw[t] = t + 1 < 5 ? band(Lb, t + 1, 1) - s * band(Gb, t + 1, 1) : 0.0;
        Cw[t] = band(Lb, t, 2) - s * band(Gb, t, 2);
    }
    StartSeq sq(i, h);
    double yA = sq.next();   // rows 0, 1, 2 of this half's elimination order
    double yB = sq.next();
    double yC = sq.next();
    __shared__ double rows[64][10];
    for (int j0 = 0; j0 < m; j0 += 64) {
        // stage band rows j0+3 .. j0+66 in LDS (one per lane); every lane reads them all
        const int rr = min(j0 + 3 + lane, n - 1);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 5; ++t) {
            rows[lane][t] = band(Lb, t, rr);
            rows[lane][5 + t] = band(Gb, t, rr);
        }
        __syncthreads();
        const int jend = min(m, j0 + 64);
        for (int j = j0; j < jend; ++j) {
            // band row j + 3 (entering the window at the end of this step), read from
            // LDS first so that its latency overlaps the elimination
            double nl[5], ng[5];
#pragma unroll
            for (int t = 0; t < 5; ++t) {
                nl[t] = rows[j - j0][t];
                ng[t] = rows[j - j0][5 + t];
            }
            const double ynext = sq.next();   // row j + 3 (j + 3 <= n - 2)
            // partial pivoting among the rows j, j+1, j+2 (rows j+1, j+2 exist: j + 2 <= m + 1
            // <= n - 3), as selects: pivot row U, remaining rows R1, R2 in their order
            const double fa = fabs(A[0]), fb = fabs(Bw[0]), fc = fabs(Cw[0]);
            const bool sB = fb > fa;
            const bool sC = fc > (sB ? fb : fa);
            const bool sBo = sB && !sC;
            const int p = sC ? 2 : (sB ? 1 : 0);
            double U[5], R1[5], R2[5];
#pragma unroll
            for (int t = 0; t < 5; ++t) {
                U[t] = sC ? Cw[t] : (sB ? Bw[t] : A[t]);
                R1[t] = sBo ? A[t] : Bw[t];
                R2[t] = sC ? A[t] : Cw[t];
            }
            const double yU = sC ? yC : (sB ? yB : yA);
            const double yR1 = sBo ? yA : yB;
            const double yR2 = sC ? yA : yC;
            const double u0 = fabs(U[0]) < pivmin ? (U[0] < 0.0 ? -pivmin : pivmin) : U[0];
            const double inv = recip(u0);
            const double l1 = R1[0] * inv, l2 = R2[0] * inv;
            if (act) {
                *at32(F.L, j, nw, i) = make_double2(l1, l2);
                *at32(F.P, j, nw, i) = p;
                *at32(F.IZ, j, nw, i) = make_double2(inv, yU);
                *at32(F.U12, j, nw, i) = make_double2(U[1], U[2]);
                *at32(F.U34, j, nw, i) = make_double2(U[3], U[4]);
            }
            // eliminate and shift the window by one column
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                A[t] = fma(-l1, U[t + 1], R1[t + 1]);
                Bw[t] = fma(-l2, U[t + 1], R2[t + 1]);
            }
            A[4] = 0.0;
            Bw[4] = 0.0;
#pragma unroll
            for (int t = 0; t < 5; ++t) Cw[t] = fma(-s, ng[t], nl[t]);
            yA = fma(-l1, yU, yR1);
            yB = fma(-l2, yU, yR2);
            yC = ynext;
        }
    }
    // the two reduced rows and their right-hand sides
    double w0[5], w1[5];
    const double y0 = yA, y1 = yB;
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        w0[t] = A[t];
        w1[t] = Bw[t];
    }
    if (act) {
        double* q = IF + (int64_t)h * 10 * nw + i;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            q[(int64_t)t * nw] = w0[t];
            q[(int64_t)(4 + t) * nw] = w1[t];
        }
        q[(int64_t)8 * nw] = y0;
        q[(int64_t)9 * nw] = y1;
    }
}

// The interface unknowns x_{mt} .. x_{mt+3} from the four reduced rows (Gaussian
// elimination with partial pivoting, pivots kept above pivmin in magnitude).
__device__ __forceinline__ void interface_solve(const double* __restrict__ IF, int nw, int i, double pivmin,
                                                double (&x)[4]) {
    double a[4][4], b[4];
    const double* T = IF + i;
    const double* B = IF + (int64_t)10 * nw + i;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        a[0][q] = T[(int64_t)q * nw];
        a[1][q] = T[(int64_t)(4 + q) * nw];
        a[2][q] = B[(int64_t)(3 - q) * nw];          // bottom rows: reversed column order
        a[3][q] = B[(int64_t)(7 - q) * nw];
    }
    b[0] = T[(int64_t)8 * nw];
    b[1] = T[(int64_t)9 * nw];
    b[2] = B[(int64_t)8 * nw];
    b[3] = B[(int64_t)9 * nw];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int p = k;
        double best = fabs(a[k][k]);
#pragma unroll
        for (int r = k + 1; r < 4; ++r)
            if (fabs(a[r][k]) > best) {
                best = fabs(a[r][k]);
                p = r;
            }
#pragma unroll
        for (int r = k + 1; r < 4; ++r)
            if (p == r) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double t = a[k][c];
                    a[k][c] = a[r][c];
                    a[r][c] = t;
                }
                const double t = b[k];
                b[k] = b[r];
                b[r] = t;
            }
        if (fabs(a[k][k]) < pivmin) a[k][k] = a[k][k] < 0.0 ? -pivmin : pivmin;
        const double inv = 1.0 / a[k][k];
#pragma unroll
        for (int r = k + 1; r < 4; ++r) {
            const double f = a[r][k] * inv;
#pragma unroll
            for (int c = k + 1; c < 4; ++c) a[r][c] -= f * a[k][c];
            b[r] -= f * b[k];
        }
    }
#pragma unroll
    for (int k = 3; k >= 0; --k) {
        double v = b[k];
#pragma unroll
        for (int c = k + 1; c < 4; ++c) v -= a[k][c] * x[c];
        x[k] = v / a[k][k];
    }
}

// steps whose operands are in flight ahead of use (load chunks of the back
// substitution, register ring of the forward elimination)
constexpr int IV_DB = 16;
constexpr int IV_DF = 15;

// Interface solve, then back substitution U x = z of each half outward from the
// interface (x node-major [n][nw]). Each wave runs one dependent chain per lane,
// so only loads issued well ahead hide the memory latency: the operands of
// IV_DB steps ((1/u_jj, z_j) and the four superdiagonal entries, three loads per
// step, within the 63 outstanding memory operations a wave can track) are all
// issued before the first of those steps runs.
__global__ __launch_bounds__(64) void invit_back_kernel(int n, int mt, int mb, int nw,
                                                        char* __restrict__ fac, int64_t M,
                                                        const double* __restrict__ IF, double pivmin,
                                                        double* __restrict__ X) {
    const int h = blockIdx.y;
    const int m = h == 0 ? mt : mb;
    const int lane = threadIdx.x & 63;
    const int i0 = blockIdx.x * 64 + lane;
    const bool act = i0 < nw;
    const int i = min(i0, nw - 1);
    const FacView F = fac_view(fac, M, h);
    double xi[4];
    interface_solve(IF, nw, i, pivmin, xi);
    double x1, x2, x3, x4;   // x_{j+1} .. x_{j+4} in the half's own row order
    if (h == 0) {
        x1 = xi[0]; x2 = xi[1]; x3 = xi[2]; x4 = xi[3];
        if (act) {
            X[(int64_t)node_of(mt, n) * nw + i] = xi[0];
            X[(int64_t)node_of(mt + 1, n) * nw + i] = xi[1];
        }
    } else {
        x1 = xi[3]; x2 = xi[2]; x3 = xi[1]; x4 = xi[0];
        if (act) {
            X[(int64_t)node_of(mt + 2, n) * nw + i] = xi[2];
            X[(int64_t)node_of(mt + 3, n) * nw + i] = xi[3];
        }
    }
    // the terms of older unknowns are summed first so that the chain between
    // steps is one FMA and one product
    auto step = [&](int j, double inv, double2 u12, double2 u34, double z) {
        const double part = fma(-u34.y, x4, fma(-u34.x, x3, fma(-u12.y, x2, z)));
        const double v = fma(-u12.x, x1, part) * inv;
        if (act) *at32(X, node_of(trow(h, j, n), n), nw, i) = v;
        x4 = x3;
        x3 = x2;
        x2 = x1;
        x1 = v;
    };
    // chunks of IV_DB steps: all their loads are issued before the first step of
    // the chunk runs
    int j0 = m - 1;     // next step to run (descending)
    for (; j0 - (IV_DB - 1) >= 0; j0 -= IV_DB) {
        double2 riz[IV_DB], ru12[IV_DB], ru34[IV_DB];
#pragma unroll
        for (int q = 0; q < IV_DB; ++q) {
            riz[q] = *at32(F.IZ, j0 - q, nw, i);
            ru12[q] = *at32(F.U12, j0 - q, nw, i);
            ru34[q] = *at32(F.U34, j0 - q, nw, i);
        }
#pragma unroll
        for (int q = 0; q < IV_DB; ++q) step(j0 - q, riz[q].x, ru12[q], ru34[q], riz[q].y);
    }
    for (; j0 >= 0; --j0) {
        const double2 iz = *at32(F.IZ, j0, nw, i);
        step(j0, iz.x, *at32(F.U12, j0, nw, i), *at32(F.U34, j0, nw, i), iz.y);
    }
}

// W = G X for node-major X [n][nw] (the right-hand side of the second solve).
__global__ void gx_nodemajor_kernel(Pencil P, int nw, const double* __restrict__ X, double* __restrict__ W) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = P.n;
    if (t >= (int64_t)n * nw) return;
    const int k = (int)(t / nw), i = (int)(t % nw);
    const int km = k == 0 ? n - 1 : k - 1, kp = k + 1 == n ? 0 : k + 1;
    W[t] = P.gd[k] * X[(int64_t)k * nw + i] + P.go[km] * X[(int64_t)km * nw + i] +
           P.go[k] * X[(int64_t)kp * nw + i];
}

// Forward elimination of W (node-major, G X) for both halves, z into the factor
// records, the interface right-hand sides into IF. Step j works on the window
// rows (y0, y1) and the entering row j + 2 of W; the multipliers, pivot choices and entering rows run IV_DF - 1
// steps ahead in a register ring, as in the back substitution. Slot q holds the
// operands of the next step j = q (mod IV_DF), and the entering row of step j - 1
// stays in its slot until step j has used it, so no ring register is copied
// while its load is in flight.
__global__ __launch_bounds__(64) void invit_fwd_kernel(int n, int mt, int mb, int nw,
                                                       char* __restrict__ fac, int64_t M,
                                                       const double* __restrict__ WZ, double* __restrict__ IF) {
    const int h = blockIdx.y;
    const int m = h == 0 ? mt : mb;
    const int lane = threadIdx.x & 63;
    const int i0 = blockIdx.x * 64 + lane;
    const bool act = i0 < nw;
    const int i = min(i0, nw - 1);
    const FacView F = fac_view(fac, M, h);
    auto rnode = [&](int j) { return node_of(trow(h, j, n), n); };
    double y0 = WZ[(int64_t)rnode(0) * nw + i], y1 = WZ[(int64_t)rnode(1) * nw + i];
    // one elimination step on the rows (y0, y1, a2): returns nothing, leaves the
    // two reduced rows in (y0, y1)
    auto step = [&](int j, int p, double2 l, double a2) {
        // row interchange as selects (an indexed form would go through scratch memory)
        const double a0 = y0, a1 = y1;
        const double u = p == 1 ? a1 : (p == 2 ? a2 : a0);
        const double b1 = p == 1 ? a0 : a1;
        const double b2 = p == 2 ? a0 : a2;
        if (act) at32(F.IZ, j, nw, i)->y = u;
        y0 = fma(-l.x, u, b1);
        y1 = fma(-l.y, u, b2);
    };
    int rp[IV_DF];
    double2 rl[IV_DF];
    double rr[IV_DF];
    // row j + 3 <= m + 2 <= n - 2 always exists
    auto load = [&](int j, int q) {
        rl[q] = *at32(F.L, j, nw, i);
        rp[q] = *at32(F.P, j, nw, i);
        rr[q] = *at32(WZ, rnode(j + 3), nw, i);
    };
    int j0 = 0;
    if (m >= 2 * IV_DF - 1) {
        rr[IV_DF - 1] = WZ[(int64_t)rnode(2) * nw + i];
#pragma unroll
        for (int q = 0; q < IV_DF - 1; ++q) load(q, q);
        for (; j0 + 2 * IV_DF - 1 <= m; j0 += IV_DF) {
            step(j0, rp[0], rl[0], rr[IV_DF - 1]);
            load(j0 - 1 + IV_DF, IV_DF - 1);
#pragma unroll
            for (int q = 1; q < IV_DF; ++q) {
                step(j0 + q, rp[q], rl[q], rr[q - 1]);
                load(j0 + q - 1 + IV_DF, q - 1);
            }
        }
        // slots 0 .. IV_DF - 2 hold steps j0 .. j0 + IV_DF - 2 (all < m), slot IV_DF - 1
        // the entering row of step j0 - 1
        step(j0, rp[0], rl[0], rr[IV_DF - 1]);
#pragma unroll
        for (int q = 1; q < IV_DF - 1; ++q) step(j0 + q, rp[q], rl[q], rr[q - 1]);
        j0 += IV_DF - 1;
    }
    // W is read-only here: the entering row of step j0 is row j0 + 2
    double y2 = WZ[(int64_t)rnode(j0 + 2) * nw + i];
    for (; j0 < m; ++j0) {
        const double r = *at32(WZ, rnode(j0 + 3), nw, i);
        const double2 l = *at32(F.L, j0, nw, i);
        step(j0, *at32(F.P, j0, nw, i), make_double2(l.x, l.y), y2);
        y2 = r;
    }
    if (act) {
        IF[(int64_t)(h * 10 + 8) * nw + i] = y0;
        IF[(int64_t)(h * 10 + 9) * nw + i] = y1;
    }
}

__device__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Gram-Schmidt in the G inner product inside each cluster [cb[c], cb[c+1]) of
// vector-major X (vector j at X + j n, contiguous; one workgroup per cluster):
// every pass over a vector is one coalesced sweep.
__global__ __launch_bounds__(256) void cluster_gs_vm_kernel(Pencil P, const int* __restrict__ cb,
                                                            double* __restrict__ X) {
    __shared__ double sh[256];
    const int n = P.n;
    const int c0 = cb[blockIdx.x], c1 = cb[blockIdx.x + 1];
    for (int j = c0; j < c1; ++j) {
        double* xj = X + (int64_t)j * n;
        for (int i = c0; i <= j; ++i) {
            const double* xi = X + (int64_t)i * n;
            double part = 0.0;
            for (int k = threadIdx.x; k < n; k += blockDim.x) {
                const int km = k == 0 ? n - 1 : k - 1, kp = k + 1 == n ? 0 : k + 1;
                part += xi[k] * (P.gd[k] * xj[k] + P.go[km] * xj[km] + P.go[k] * xj[kp]);
            }
            const double dot = block_sum(part, sh);
            if (i < j) {
                for (int k = threadIdx.x; k < n; k += blockDim.x) xj[k] -= dot * xi[k];
            } else {
                const double sc = 1.0 / sqrt(dot);
                for (int k = threadIdx.x; k < n; k += blockDim.x) xj[k] *= sc;
            }
            __syncthreads();
        }
    }
}

// out[c][r] = in[r][c] for a rows x cols row-major input (32 x 32 LDS tiles)
__global__ void transpose_kernel(const double* __restrict__ in, int rows, int cols, double* __restrict__ out) {
    __shared__ double t[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    for (int k = threadIdx.y; k < 32; k += blockDim.y) {
        const int r = by + k, c = bx + threadIdx.x;
        if (r < rows && c < cols) t[k][threadIdx.x] = in[(int64_t)r * cols + c];
    }
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += blockDim.y) {
        const int c = bx + k, r = by + threadIdx.x;
        if (r < rows && c < cols) out[(int64_t)c * rows + r] = t[threadIdx.x][k];
    }
}


// Reported eigenvalues: Rayleigh-Ritz inside each cluster [cb[c], cb[c+1]) of the
// final G-orthonormal vectors X (vector-major, n x nw): H_ab = x_a^T L x_b with
// x^T L y = sum_k (x_{k+1} - x_k)(y_{k+1} - y_k) / h_k (periodic; for a = b a sum of
// non-negative terms), and the eigenvalues of the small symmetric H by cyclic
// Jacobi rotations (clusters of more than RR_MAX vectors keep their diagonal).
// Vectors within a cluster are arbitrary combinations after the Gram-Schmidt
// step, so a per-vector quotient would average the cluster's eigenvalues.
constexpr int RR_MAX = 8;
__global__ void cluster_ritz_kernel(const double* __restrict__ h, int n, const double* __restrict__ X,
                                    const int* __restrict__ cb, double* __restrict__ out) {
    __shared__ double sh[256];
    __shared__ double H[RR_MAX][RR_MAX];
    const int c0 = cb[blockIdx.x], c1 = cb[blockIdx.x + 1];
    const int m = c1 - c0;
    const bool full = m <= RR_MAX;
    for (int a = 0; a < m; ++a) {
        for (int b = full ? a : a; b < (full ? m : a + 1); ++b) {
            const double* x = X + (int64_t)(c0 + a) * n;
            const double* y = X + (int64_t)(c0 + b) * n;
            double acc = 0.0;
            for (int k = threadIdx.x; k < n; k += blockDim.x) {
                const int kp = k + 1 == n ? 0 : k + 1;
                acc += (x[kp] - x[k]) * (y[kp] - y[k]) / h[k];
            }
            sh[threadIdx.x] = acc;
            __syncthreads();
            for (int s = blockDim.x / 2; s > 0; s >>= 1) {
                if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
                __syncthreads();
            }
            if (threadIdx.x == 0) {
                if (full) {
                    H[a][b] = sh[0];
                    H[b][a] = sh[0];
                } else {
                    out[c0 + a] = sh[0];
                }
            }
            __syncthreads();
        }
    }
    if (threadIdx.x != 0 || !full) return;
    auto& A = H;   // rotated in place (LDS)
    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                tot += A[i][j] * A[i][j];
                if (i != j) off += A[i][j] * A[i][j];
            }
        if (off <= 1e-32 * tot) break;
        for (int p = 0; p < m - 1; ++p)
            for (int q = p + 1; q < m; ++q) {
                if (A[p][q] == 0.0) continue;
                const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < m; ++k) {   // A <- J^T A J
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = cs * akp - sn * akq;
                    A[k][q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < m; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = cs * apk - sn * aqk;
                    A[q][k] = sn * apk + cs * aqk;
                }
            }
    }
    // eigenvalues ascending (static-index sorting network in registers)
    double d[RR_MAX];
#pragma unroll
    for (int i = 0; i < RR_MAX; ++i) d[i] = i < m ? A[i][i] : 1e308;
#pragma unroll
    for (int i = 0; i < RR_MAX; ++i)
#pragma unroll
        for (int j = 0; j + 1 < RR_MAX - i; ++j) {   // bubble sort with static indices
            const double lo = fmin(d[j], d[j + 1]), hi = fmax(d[j], d[j + 1]);
            d[j] = lo;
            d[j + 1] = hi;
        }
#pragma unroll
    for (int i = 0; i < RR_MAX; ++i)
        if (i < m) out[c0 + i] = d[i];
}

// ---------------------------------------------------------------- host driver
// ---------------------------------------------------------------- homogeneous meshes
// Paper, Laplacian Filters, Two-Dimensional Case: with all panels of length h, G
// and L are circulant (G = (h/6) circ(4, 1, .., 1), L = (1/h) circ(2, -1, .., -1)),
// the DFT diagonalises both, and the pencil eigenpairs are
//   mu_m = lambda_L / lambda_G = 12 sin^2(pi m/n) / (h^2 (2 + cos(2 pi m/n))),
//   vectors cos(2 pi m j/n), sin(2 pi m j/n),
// mu increasing in min(m, n - m): the filter keeps the lowest frequencies and needs
// no eigensolver. Column c of the basis holds mode code[c] = 2 m + (1 for the sine),
// scaled to G-norm one: 1/sqrt(n lambda_G) for m = 0 and m = n/2, sqrt(2/(n lambda_G))
// otherwise.
__global__ void dft_basis_kernel(int n, double h, const int* __restrict__ code, double* __restrict__ X) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int col = blockIdx.y;
    const int m = code[col] >> 1;
    const bool sine = code[col] & 1;
    double sm, cm, sv, cv;
    sincospi(2.0 * (double)m / (double)n, &sm, &cm);
    const double lamg = (h / 3.0) * (2.0 + cm);
    const double w = (m == 0 || 2 * m == n) ? 1.0 : 2.0;
    sincospi(2.0 * (double)(((int64_t)m * j) % n) / (double)n, &sv, &cv);
    X[(int64_t)col * n + j] = (sine ? sv : cv) * sqrt(w / ((double)n * lamg));
}

static void dft_filter_basis(Op& op, int n_modes, bool keep_null, double cluster_rtol) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    const double h = op.h_mean;
    const int start = keep_null ? 0 : 1;
    int want = keep_null ? n_modes : n_modes - 1;
    FDS_REQUIRE(want >= 1 && start + want <= n, FDS_ERR_ARG, "n_modes out of range");
    // modes in increasing order of mu: m = 0, then (cos, sin) for m = 1 .. (n-1)/2, then
    // the single m = n/2 for even n
    std::vector<int> code;
    std::vector<double> mu;
    auto mu_of = [&](int m) {
        const double s = std::sin(kPiHost * m / n);
        return 12.0 * s * s / (h * h * (2.0 + std::cos(2.0 * kPiHost * m / n)));
    };
    code.push_back(0);
    mu.push_back(0.0);
    for (int m = 1; 2 * m < n; ++m) {
        code.push_back(2 * m);
        code.push_back(2 * m + 1);
        mu.push_back(mu_of(m));
        mu.push_back(mu_of(m));
    }
    if (n % 2 == 0) {
        code.push_back(n);
        mu.push_back(mu_of(n / 2));
    }
    code.erase(code.begin(), code.begin() + start);
    mu.erase(mu.begin(), mu.begin() + start);
    // the cut guard of the general path: never split a (near-)degenerate group
    int ne = want;
    while (ne < (int)mu.size() && mu[ne] - mu[ne - 1] <= cluster_rtol * std::max(std::fabs(mu[ne - 1]), std::fabs(mu[ne])))
        ++ne;
    code.resize(ne);
    FDS_REQUIRE(ne <= 65535, FDS_ERR_NOTIMPL, "more than 65535 filter modes");
    op.filt_lam.assign(mu.begin(), mu.begin() + std::min((int)mu.size(), ne + 2));
    int* dcode = static_cast<int*>(c.dmalloc(sizeof(int) * ne));
    FDS_HIP_TRY(hipMemcpyAsync(dcode, code.data(), sizeof(int) * ne, hipMemcpyHostToDevice, c.stream));
    double* X = static_cast<double*>(c.dmalloc(sizeof(double) * (size_t)n * ne));
    {
        KScope _ks(c, "filter_dft");
        hipLaunchKernelGGL(dft_basis_kernel, dim3((n + 255) / 256, ne), dim3(256), 0, c.stream, n, h, dcode, X);
    }
    FDS_HIP_TRY(hipGetLastError());
    // the kept eigenvalues stay readable through lam_dev like the general path's Ritz values
    double* dlam = static_cast<double*>(c.dmalloc(sizeof(double) * ne));
    FDS_HIP_TRY(hipMemcpyAsync(dlam, mu.data(), sizeof(double) * ne, hipMemcpyHostToDevice, c.stream));
    // the host vectors above must outlive the copies from pageable memory
    FDS_HIP_TRY(hipStreamSynchronize(c.stream));
    c.dfree(dcode);
    c.dfree(op.lam_dev);
    op.lam_dev = dlam;
    op.lam_dev_n = ne;
    c.dfree(op.Vg);
    c.dfree(op.Vn);
    op.Vn = nullptr;
    op.Vg = X;
    op.n_eff = ne;
}

// Host quantities of the eigensolver for one mesh and filtering point: the
// pencil's spectrum bounds (Gershgorin on the host panel lengths,
// 0 <= lambda <= max_i (|l_ii| + |l_i,i-1| + |l_i,i+1|) / lambda_min(G)), the
// index range of the wanted eigenvalues and the tight-bracket coefficients.
struct EigSetup {
    double gmin, gmax, lam_hi, mnorm, l1c, hfac;
    int start, want, extra;
};

static EigSetup eig_setup(Op& op, int n_modes, bool keep_null) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    const std::vector<double>& hh = op.h_host;
    EigSetup e{};
    double lmax = 0.0;
    gram_gershgorin(hh, e.gmin, e.gmax);
    for (int i = 0; i < n; ++i) {
        const double hm = hh[i == 0 ? n - 1 : i - 1], hp = hh[i];
        lmax = std::max(lmax, 2.0 / hm + 2.0 / hp);
    }
    e.lam_hi = 1.01 * lmax / e.gmin;
    e.mnorm = lmax + e.lam_hi * e.gmax;
    e.start = keep_null ? 0 : 1;
    e.want = keep_null ? n_modes : n_modes - 1;
    FDS_REQUIRE(e.want >= 1 && e.start + e.want <= n, FDS_ERR_ARG, "n_modes out of range");
    // One workgroup per eigenvalue, each alone on a compute unit for the whole
    // latency-bound recurrence: two eigenvalues past the cut guard it against a
    // split cluster, one when the second would put a workgroup past a multiple
    // of the CU count (a wider cluster at the cut is found and bisected again).
    int ncu = 0;
    FDS_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c.device));
    e.extra = (ncu > 0 && (e.want + 2) % ncu == 1) ? 1 : 2;
    // Tight brackets: the P1 pencil is the Rayleigh-Ritz discretisation of -d^2/ds^2
    // on the polygon of perimeter Ph, whose eigenvalues are (2 pi k/Ph)^2 (k = 0, 1, 1,
    // 2, 2, ...), so eigenvalue index idx lies above lam_c = (2 pi ceil(idx/2)/Ph)^2, and
    // its relative excess is about lam_c <h^2>/12 with <h^2> = sum h^3 / sum h (exactly
    // to leading order on uniform meshes); the kernel brackets the eigenvalue by 0.2 and
    // 1.6 times that excess (see bisect_scaled_kernel), checks each bracket with the
    // inertia counts and falls back to the global one. The eigenvalues are wanted to
    // 2e-8 relative only (below), and the reported eigenvalues are the Rayleigh
    // quotients of the final vectors (Rayleigh-Ritz inside each cluster).
    double Ph = 0.0, h3 = 0.0;
    for (double v : hh) {
        Ph += v;
        h3 += v * v * v;
    }
    e.l1c = (2.0 * kPiHost / Ph) * (2.0 * kPiHost / Ph);
    e.hfac = h3 / (12.0 * Ph);
    return e;
}

// The folded bands and the Sturm-step table of the pencil (device buffers).
static void eig_tables(Op& op, double*& Lb, double*& Gb, SturmStep*& dst) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    Pencil P{op.l_diag, op.l_off, op.g_diag, op.g_off, n};
    Lb = static_cast<double*>(c.dmalloc(sizeof(double) * 5 * (size_t)n));
    Gb = static_cast<double*>(c.dmalloc(sizeof(double) * 5 * (size_t)n));
    {
        KScope _ks(c, "filter_fold");
        hipLaunchKernelGGL(fold_bands_kernel, dim3((n + 255) / 256), dim3(256), 0, c.stream, P, Lb, Gb);
    }
    FDS_HIP_TRY(hipGetLastError());
    const int K = n / 2;
    // top-down steps [K - 1], then the bottom-up table [K]
    dst = static_cast<SturmStep*>(c.dmalloc(sizeof(SturmStep) * (size_t)(std::max(K - 1, 1) + std::max(K, 1))));
    {
        KScope _ks(c, "filter_bisect");
        hipLaunchKernelGGL(sturm_steps_kernel, dim3((K + 255) / 256), dim3(256), 0, c.stream, P, dst,
                           dst + std::max(K - 1, 1));
    }
    FDS_HIP_TRY(hipGetLastError());
}

static void launch_bisect(Op& op, const EigSetup& e, const SturmStep* dst, int nw, double rtol, double* dlam) {
    Ctx& c = *op.ctx;
    Pencil P{op.l_diag, op.l_off, op.g_diag, op.g_off, (int)op.n};
    {
        KScope _ks(c, "filter_bisect");
        const int K = (int)op.n / 2;
        hipLaunchKernelGGL(bisect_scaled_kernel, dim3(nw), dim3(64 * BS_WAVES), 0, c.stream, P, dst,
                           dst + std::max(K - 1, 1), e.l1c, e.hfac,
                           -1e-3 * e.lam_hi, e.lam_hi, rtol, 4e-16 * e.lam_hi, e.start, nw, dlam);
    }
    FDS_HIP_TRY(hipGetLastError());
}

// Starts the eigensolver of filtering point n_modes (null mode kept) on the
// current stream: tables and the first bisection, results left on the device
// for compute_filter_basis.
void prefetch_filter_eigs(Op& op, int n_modes) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    const EigSetup e = eig_setup(op, n_modes, true);
    double *Lb = nullptr, *Gb = nullptr;
    SturmStep* dst = nullptr;
    eig_tables(op, Lb, Gb, dst);
    const int nw = std::min(n - e.start, e.want + e.extra);
    double* dlam = static_cast<double*>(c.dmalloc(sizeof(double) * nw));
    launch_bisect(op, e, dst, nw, 2e-8, dlam);
    op.pre_active = true;
    op.pre_modes = n_modes;
    op.pre_nw = nw;
    op.pre_extra = e.extra;
    op.pre_Lb = Lb;
    op.pre_Gb = Gb;
    op.pre_steps = dst;
    op.pre_lam = dlam;
}

void compute_filter_basis(Op& op, int n_modes, bool keep_null, double cluster_rtol) {
    Ctx& c = *op.ctx;
    // a started eigensolver is used when it matches, otherwise released
    const bool pre = op.pre_active && op.pre_modes == n_modes && keep_null;
    double* pLam = nullptr;
    if (op.pre_active) {
        op.pre_active = false;
        if (!pre) {
            c.dfree(op.pre_Lb);
            c.dfree(op.pre_Gb);
            c.dfree(op.pre_steps);
            c.dfree(op.pre_lam);
            op.pre_Lb = op.pre_Gb = nullptr;
            op.pre_steps = nullptr;
            op.pre_lam = nullptr;
        }
    }
    if (op.homog) {
        gram_gershgorin(op.h_host, op.cheb_lo, op.cheb_hi);
        dft_filter_basis(op, n_modes, keep_null, cluster_rtol);
        return;
    }
    const int n = (int)op.n;
    const EigSetup e = eig_setup(op, n_modes, keep_null);
    op.cheb_lo = e.gmin;
    op.cheb_hi = e.gmax;
    const double mnorm = e.mnorm;
    Pencil P{op.l_diag, op.l_off, op.g_diag, op.g_off, n};
    double *Lb = nullptr, *Gb = nullptr;
    SturmStep* dst = nullptr;
    if (pre) {
        Lb = op.pre_Lb;
        Gb = op.pre_Gb;
        dst = static_cast<SturmStep*>(op.pre_steps);
        pLam = op.pre_lam;
        op.pre_Lb = op.pre_Gb = nullptr;
        op.pre_steps = nullptr;
        op.pre_lam = nullptr;
    } else {
        eig_tables(op, Lb, Gb, dst);
    }
    const int start = e.start;
    int want = e.want;
    int extra = e.extra;
    // eigenvalues start .. start+nw-1 (a few beyond the cut for the cluster guard)
    std::vector<double> lam;
    int nw = 0;
    // Precision of the shifts: inverse iteration needs them accurate against the gap
    // between the kept and the excluded modes only (components of other kept modes
    // stay inside the kept subspace). 2e-8 relative (two rounds of 256 shifts from the
    // brackets) damps the excluded modes by 2e-8 / (relative gap at the cut) per
    // solve, ~1e-6 for the usual gap between Fourier pairs; when the cut gap is below
    // 2e-3 (a damping above 1e-5 per solve) the eigenvalues are bisected again to 6e-10.
    double rtol = 2e-8;
    double* dlam = nullptr;   // the device eigenvalues of the last bisection (kept as the shifts)
    for (;;) {
        nw = std::min(n - start, want + extra);
        c.dfree(dlam);
        if (pLam) {   // the first launch was made by prefetch_filter_eigs with these parameters
            dlam = pLam;
            pLam = nullptr;
        } else {
            dlam = static_cast<double*>(c.dmalloc(sizeof(double) * nw));
            launch_bisect(op, e, dst, nw, rtol, dlam);
        }
        lam.assign(nw, 0.0);
        // read through a pinned buffer (no staging copy) and wait at once
        double* hl = static_cast<double*>(c.pinned_host(sizeof(double) * nw));
        FDS_HIP_TRY(hipMemcpyAsync(hl ? hl : lam.data(), dlam, sizeof(double) * nw, hipMemcpyDeviceToHost,
                                   c.stream));
        FDS_HIP_TRY(hipStreamSynchronize(c.stream));
        if (hl) std::copy(hl, hl + nw, lam.begin());
        int ne = want;
        while (ne < nw) {
            const double a = lam[ne - 1], b = lam[ne];
            if (b - a > cluster_rtol * std::max(std::fabs(a), std::fabs(b))) break;
            ++ne;
        }
        if (ne < nw || start + nw == n) {
            if (ne < nw && rtol > 6e-10 &&
                lam[ne] - lam[ne - 1] < 2e-3 * std::max(std::fabs(lam[ne]), std::fabs(lam[ne - 1]))) {
                rtol = 6e-10;
                continue;
            }
            want = std::min(ne, nw);
            break;
        }
        extra *= 4;
    }
    const int ne = want;
    op.filt_lam = lam;
    lam.resize(ne);
    // clusters for the inverse iteration: relative gaps below 1e-5 of the scale
    const double scale = std::max(lam[ne - 1], 1e-300);
    std::vector<int> cb{0};
    for (int i = 1; i < ne; ++i)
        if (lam[i] - lam[i - 1] > 1e-5 * scale) cb.push_back(i);
    cb.push_back(ne);
    const int ncl = (int)cb.size() - 1;

    // the shifts: the first ne device eigenvalues, as read (nw >= ne entries)
    double* dsig = dlam;
    int* dcb = static_cast<int*>(c.dmalloc(sizeof(int) * (ncl + 1)));
    FDS_HIP_TRY(hipMemcpyAsync(dcb, cb.data(), sizeof(int) * (ncl + 1), hipMemcpyHostToDevice, c.stream));
    // two-ended elimination: mt steps from the top, mb from the bottom, 4 interface rows
    const int mt = (n - 4) / 2, mb = n - 4 - mt;
    const int64_t facM = (int64_t)mb * ne;     // entries per record array (mb >= mt)
    FDS_REQUIRE(facM * 16 < ((int64_t)1 << 32) && (int64_t)n * ne * 8 < ((int64_t)1 << 32), FDS_ERR_NOTIMPL,
                "inverse-iteration arrays above 4 GiB");
    char* fac = static_cast<char*>(c.dmalloc(2 * fac_half_bytes(facM)));
    double* IF = static_cast<double*>(c.dmalloc(sizeof(double) * 20 * (size_t)ne));
    double* Xn = static_cast<double*>(c.dmalloc(sizeof(double) * (size_t)n * ne));   // node-major
    double* Wk = static_cast<double*>(c.dmalloc(sizeof(double) * (size_t)n * ne));
    const dim3 egrid((unsigned)((ne + 63) / 64), 2);
    const double pivmin = 1e-15 * mnorm;
    {
        KScope _ks(c, "filter_invit_factor");
        hipLaunchKernelGGL(invit_factor_kernel, egrid, dim3(64), 0, c.stream, n, mt, mb, Lb, Gb, dsig, ne, pivmin,
                           fac, facM, IF);
    }
    FDS_HIP_TRY(hipGetLastError());
    // inverse iteration from a pseudo-random right-hand side: two solves, each
    // damping the excluded modes by (shift error) / (gap at the cut); Gram-Schmidt
    // inside clusters once the solves are done
    for (int it = 0; it < 2; ++it) {
        if (it > 0) {
            KScope _ks(c, "filter_invit_fwd");
            const int64_t tot = (int64_t)n * ne;
            hipLaunchKernelGGL(gx_nodemajor_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c.stream, P,
                               ne, Xn, Wk);
            hipLaunchKernelGGL(invit_fwd_kernel, egrid, dim3(64), 0, c.stream, n, mt, mb, ne, fac, facM, Wk, IF);
        }
        FDS_HIP_TRY(hipGetLastError());
        {
            KScope _ks(c, "filter_invit_back");
            hipLaunchKernelGGL(invit_back_kernel, egrid, dim3(64), 0, c.stream, n, mt, mb, ne, fac, facM, IF,
                               pivmin, Xn);
        }
        FDS_HIP_TRY(hipGetLastError());
    }
    // to vector-major (each eigenvector contiguous)
    double* X = static_cast<double*>(c.dmalloc(sizeof(double) * (size_t)n * ne));
    {
        KScope _ks(c, "transpose");
        hipLaunchKernelGGL(transpose_kernel, dim3((ne + 31) / 32, (n + 31) / 32), dim3(32, 8), 0, c.stream, Xn, n,
                           ne, X);
    }
    FDS_HIP_TRY(hipGetLastError());
    // Gram-Schmidt in the G inner product inside each cluster (a degenerate pair's two
    // vectors are independent combinations of its eigenvectors after the solves; the
    // other components are already damped to rounding), with G-normalisation
    {
        KScope _ks(c, "filter_cluster_gs");
        hipLaunchKernelGGL(cluster_gs_vm_kernel, dim3(ncl), dim3(256), 0, c.stream, P, dcb, X);
    }
    FDS_HIP_TRY(hipGetLastError());
    // Newton-Schulz in the G inner product: with M = V^T G V = I + E (|E| ~ 1e-12 after
    // the inverse iteration), V <- V (3I - M)/2 leaves V^T G V = I + O(E^2): one pass.
    double* M = static_cast<double*>(c.dmalloc(sizeof(double) * (size_t)ne * ne));
    for (int pass = 0; pass < 1; ++pass) {
        gram_mul<double>(c, op.g_diag, op.g_off, n, X, ne, n, 1.0, 0.0, Wk, n);
        dgemm(c, OP_T, OP_N, ne, ne, n, 1.0, X, n, Wk, n, 0.0, M, ne);
        dgemm(c, OP_N, OP_N, n, ne, ne, -0.5, X, n, M, ne, 0.0, Xn, n);
        daxpby(c, 1.0, Xn, 1.5, X, (int64_t)n * ne);
    }
    c.dfree(M);
    // reported eigenvalues: Rayleigh-Ritz values of the final vectors per cluster
    {
        KScope _ks(c, "filter_rayleigh");
        hipLaunchKernelGGL(cluster_ritz_kernel, dim3(ncl), dim3(256), 0, c.stream, op.h, n, X, dcb, dsig);
    }
    FDS_HIP_TRY(hipGetLastError());
    // the Ritz values stay on the device until they are read (no host wait here)
    c.dfree(op.lam_dev);
    op.lam_dev = dsig;
    op.lam_dev_n = ne;
    c.dfree(Wk);
    c.dfree(Xn);
    c.dfree(fac);
    c.dfree(IF);
    c.dfree(dcb);
    c.dfree(Lb);
    c.dfree(Gb);
    c.dfree(dst);
    c.dfree(op.Vg);
    c.dfree(op.Vn);
    op.Vn = nullptr;
    op.Vg = X;
    op.n_eff = ne;
}

}  // namespace fds
