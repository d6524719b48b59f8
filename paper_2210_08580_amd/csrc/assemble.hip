// Dense Galerkin assembly of S, N (Maue form) and D (paper, Notation and
// Background: [S]_ij = <phi_i, S phi_j>, [N]_ij = <phi_i, N phi_j>,
// [D]_ij = <phi_i, D phi_j>, g2 = (i/4) H0^(1)(kR)).
//
// For a panel pair (p, q) with x on p and y on q the 2x2 local blocks are
//   S_ab  = int_p int_q psi_a(x) psi_b(y) g,      I0 = sum_ab S_ab,
//   N_ab  = s_a s_b I0/(h_p h_q) - k^2 (n_p.n_q) S_ab,   s_0 = -1, s_1 = +1,
//   D_ab  = int_p int_q psi_a psi_b dg/dn_y,
// and entry (i, j) sums the blocks of the four pairs (p, q) in
// {i-1, i} x {j-1, j} (panel p carries psi_0 of node p, psi_1 of node p+1).
//
// Far pairs (|p - q| >= 2 mod n): tensor Gauss rules of 8 down to 2 points per
//   panel, the order chosen per wavefront and row panel (the largest any lane
//   needs) from the gap d between the panels, h = max(h_p, h_q) and kh. The
//   n-point error has an oscillation part ~ C_n (kh)^{2n} (phase kR moves by at
//   most kh along a panel; C_2 ~ 1.4e-2, C_3 ~ 1.9e-4, C_4 ~ 5e-8 for these
//   kernels) and a part from the kernel's singularity at distance d that decays
//   like (d/h)^{-2n} (Bernstein ellipse). Against a 20-point rule the thresholds
//   below keep both at the rounding level of the arithmetic used (the onsets
//   measured over random panel orientations, with margins of 1.5 to 2.5):
//     FP64 (<= ~1e-15 relative): 6 points for d >= 6 h and 5 for d >= 12 h
//       (kh <= 0.2), 4 for d >= 32 h (kh <= 0.1), 3 for d >= 200 h (kh <= 0.016);
//     FP32 (<= ~1e-8, below its rounding): 4 points for d >= 6 h (kh <= 0.5),
//       3 for d >= 16 h (kh <= 0.15), 2 for d >= 200 h (kh <= 0.025).
//   One wavefront owns a 63 x 63 output tile: its 64 lanes hold the 64
//   column panels j0-1 .. j0+62 (Gauss points in registers); the wave walks
//   the row panels (wave-uniform, scalar loads), and for each row forms the
//   column entries from its own psi_1 part plus the psi_0 part of the next
//   lane (one cross-lane shuffle). S and N are symmetric and D(j,i) uses the
//   same Hankel values, so a tile above the diagonal also writes its mirror
//   tile: every Hankel evaluation serves S, N, D and D^T.
// Near pairs (self, adjacent): logarithmic parts integrated exactly (closed
//   form on a self pair, Duffy's corner split on adjacent pairs), smooth
//   remainders with the same 8 x 8 rule; the S and N bands |i - j| <= 2 are
//   then symmetrised.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "fds_internal.h"
#include "hankel.h"
#include "near.h"

namespace fds {

constexpr int TB = 63;          // output columns (= rows) per tile
constexpr int WAVES = 4;        // wavefronts per workgroup

// reduced far-field rules: [order 4: xi, w psi_0, w psi_1][order 3: same]
// Reduced Gauss rules on [0, 1] for n = 2 .. 6 points, rule n at offset
// low_rule_offset(n): xi[n], w psi_0(xi)[n], w psi_1(xi)[n].
constexpr int WLOW_DOUBLES = 60;
struct WLow {
    double r[WLOW_DOUBLES];
};
__host__ __device__ constexpr int low_rule_offset(int n) { return 3 * ((n - 1) * n / 2 - 1); }
static_assert(low_rule_offset(7) == WLOW_DOUBLES, "reduced-rule table size");

struct FarParams {
    const double* __restrict__ gx;
    const double* __restrict__ gy;
    const double* __restrict__ h;
    const double* __restrict__ nx;
    const double* __restrict__ ny;
    const void* __restrict__ tab;     // HK_TAB (FP64) or HK32_TAB (FP32)
    const double* __restrict__ nodes;
    void* __restrict__ S;             // complex128 or complex64, row-major n x n
    void* __restrict__ Nm;
    void* __restrict__ D;
    int bw;                           // FP32 operators: N on the cyclic band |d| <= bw is written as
                                      // zero here (asm_nband_kernel computes it in FP64); -1: no band
    double k;
    int n;
    int nsub;
    int tr;
    int64_t nwork;
};

__device__ __forceinline__ float2 fma_cr(float s, float2 a, float2 acc) {
    return make_float2(fmaf(s, a.x, acc.x), fmaf(s, a.y, acc.y));
}

__device__ __forceinline__ double2 shfl_down1(double2 v) {
    return make_double2(__shfl_down(v.x, 1, 64), __shfl_down(v.y, 1, 64));
}
__device__ __forceinline__ float2 shfl_down1(float2 v) {
    return make_float2(__shfl_down(v.x, 1, 64), __shfl_down(v.y, 1, 64));
}

__device__ __forceinline__ void to_out(double2 v, double2& o) { o = v; }
__device__ __forceinline__ void to_out(double2 v, float2& o) { o = make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ void to_out(float2 v, float2& o) { o = v; }

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// LDS copies shared by the workgroup: the Bessel table and the quadrature rules.
template <int TAB_BYTES>
struct FarShared {
    __attribute__((aligned(16))) char tab[TAB_BYTES];
    double wsh[16];            // w_b psi_0(xi_b), w_b psi_1(xi_b)
    double rl[WLOW_DOUBLES];   // reduced rules (n = 2 .. 6): xi, w psi_0, w psi_1
};
typedef FarShared<8 * HF_TAB_DOUBLES> FarShared64;
typedef FarShared<4 * HF32_TAB_FLOATS> FarShared32;

template <int TAB_BYTES>
__device__ __forceinline__ void far_shared_setup(FarShared<TAB_BYTES>& sh, const void* tabg, const W8& wt,
                                                 const WLow& wl) {
    const int4* src = static_cast<const int4*>(tabg);
    int4* dst = reinterpret_cast<int4*>(sh.tab);
    for (int t = threadIdx.x; t < TAB_BYTES / 16; t += blockDim.x) dst[t] = src[t];
    if (threadIdx.x < 8) {
        sh.wsh[threadIdx.x] = wt.wp0[threadIdx.x];
        sh.wsh[8 + threadIdx.x] = wt.wp1[threadIdx.x];
    }
    if (threadIdx.x < WLOW_DOUBLES) sh.rl[threadIdx.x] = wl.r[threadIdx.x];
    __syncthreads();
}

// MG consecutive output entries (MG * sizeof(T) = 32 bytes, 32-byte aligned) as
// 16-byte stores issued together.
template <typename T, int MG>
__device__ __forceinline__ void store_group(T* __restrict__ p, const T (&v)[MG]) {
    if constexpr (sizeof(T) == 8) {
        float4* q = reinterpret_cast<float4*>(p);
#pragma unroll
        for (int u = 0; u < MG / 2; ++u) {
            const float2 a = *reinterpret_cast<const float2*>(&v[2 * u]);
            const float2 b = *reinterpret_cast<const float2*>(&v[2 * u + 1]);
            q[u] = make_float4(a.x, a.y, b.x, b.y);
        }
    } else {
#pragma unroll
        for (int u = 0; u < MG; ++u) p[u] = v[u];
    }
}

// Tile of a work item: row range [i0, i1), column block j0, whether it mirrors.
struct FarTile {
    int i0, i1, j0;
    bool mirror;
};
__device__ __forceinline__ FarTile far_tile(const FarParams& P, int64_t work) {
    const int64_t tile = work / P.nsub;
    const int sub = (int)(work - tile * P.nsub);
    int J = (int)((sqrt(8.0 * (double)tile + 1.0) - 1.0) * 0.5);
    while ((int64_t)J * (J + 1) / 2 > tile) --J;
    while ((int64_t)(J + 1) * (J + 2) / 2 <= tile) ++J;
    const int I = (int)(tile - (int64_t)J * (J + 1) / 2);
    FarTile t;
    t.i0 = I * TB + sub * P.tr;
    t.i1 = min(min(I * TB + (sub + 1) * P.tr, I * TB + TB), P.n);
    t.j0 = J * TB;
    t.mirror = I != J;
    return t;
}

// Writes the entries (i, col) of S, N, D and, above the diagonal, the mirror entries
// (col, i) of S, N (symmetric) and D (from the transposed double layer T). The mirror
// entries of MG consecutive rows are kept and written together: MG * sizeof(OT) = 32
// bytes per lane, one whole memory sector, instead of MG partial writes to it spread
// over the row loop (single 8- or 16-byte column-strided stores cost 2.7x and 1.8x the
// stored bytes in write traffic). Groups that straddle the work item's rows are
// written entry by entry.
template <typename OT, int MG>
struct MirrorRows {
    OT mS[MG], mN[MG], mT[MG];
};
template <typename OT, int MG>
__device__ __forceinline__ void far_store(OT* __restrict__ oS, OT* __restrict__ oN, OT* __restrict__ oD, int n,
                                          const FarTile& T, bool mgroup, int i, int col, OT wS, OT wN, OT wD, OT wT,
                                          MirrorRows<OT, MG>& M) {
    const int64_t rc = (int64_t)i * n + col;
    oS[rc] = wS;
    oN[rc] = wN;
    oD[rc] = wD;
    if (!T.mirror) return;
    const int g = i - i % MG;   // i >= 0: the group's first row
    if (mgroup && g >= T.i0 && g + MG <= T.i1) {
        const int r = i - g;   // uniform over the wave: registers by constant index
#pragma unroll
        for (int u = 0; u < MG; ++u)
            if (u == r) {
                M.mS[u] = wS;
                M.mN[u] = wN;
                M.mT[u] = wT;
            }
        if (r == MG - 1) {
            const int64_t cr = (int64_t)col * n + g;
            store_group<OT, MG>(oS + cr, M.mS);
            store_group<OT, MG>(oN + cr, M.mN);
            store_group<OT, MG>(oD + cr, M.mT);
        }
    } else {
        const int64_t cr = (int64_t)col * n + i;
        oS[cr] = wS;
        oN[cr] = wN;
        oD[cr] = wT;
    }
}

// FP64 far pass: b-sums of one row point, (S, D, T) x (psi_0, psi_1) of the column panel.
struct Far64Sum {
    double2 s0, s1, d0, d1, t0, t1;
};
struct Far64Blk {   // 2 x 2 blocks [alpha][beta] of S, D, T of a panel pair (without hp hq)
    double2 S[2][2], D[2][2], T[2][2];
};
struct Far64Geo {
    double k, k4;   // k, k/4
    double nxp, nyp, nxq, nyq;
};

// One point pair: 1/R by the FP64 reciprocal square root refined by one Newton
// step (a few ulp; R2 is a normal number for distinct points), so neither a square
// root nor a division is needed: g = (i/4) H0(kR), c = (ik/4) H1(kR)/R.
__device__ __forceinline__ void far64_point(double xa, double ya, double yb, double zb, double w0, double w1,
                                            const Far64Geo& G, const double* tab, Far64Sum& A) {
    const double dx = xa - yb, dy = ya - zb;
    const double R2 = fma(dx, dx, dy * dy);
    const double r0 = __builtin_amdgcn_rsq(R2);
    const double ri = r0 * fma(-0.5 * R2, r0 * r0, 1.5);
    const Bessel01 bs = hf_eval(G.k * (R2 * ri), tab);
    const double2 g = make_double2(-0.25 * bs.y0, 0.25 * bs.j0);
    const double kr = G.k4 * ri;
    const double2 c = make_double2(-kr * bs.y1, kr * bs.j1);
    const double dq = fma(dx, G.nxq, dy * G.nyq);
    const double dp = -fma(dx, G.nxp, dy * G.nyp);
    const double2 cd = make_double2(c.x * dq, c.y * dq), ct = make_double2(c.x * dp, c.y * dp);
    A.s0 = fma_cr(w0, g, A.s0);
    A.s1 = fma_cr(w1, g, A.s1);
    A.d0 = fma_cr(w0, cd, A.d0);
    A.d1 = fma_cr(w1, cd, A.d1);
    A.t0 = fma_cr(w0, ct, A.t0);
    A.t1 = fma_cr(w1, ct, A.t1);
}

__device__ __forceinline__ void far64_fold(double wa0, double wa1, const Far64Sum& A, Far64Blk& B) {
    B.S[0][0] = fma_cr(wa0, A.s0, B.S[0][0]); B.S[0][1] = fma_cr(wa0, A.s1, B.S[0][1]);
    B.S[1][0] = fma_cr(wa1, A.s0, B.S[1][0]); B.S[1][1] = fma_cr(wa1, A.s1, B.S[1][1]);
    B.D[0][0] = fma_cr(wa0, A.d0, B.D[0][0]); B.D[0][1] = fma_cr(wa0, A.d1, B.D[0][1]);
    B.D[1][0] = fma_cr(wa1, A.d0, B.D[1][0]); B.D[1][1] = fma_cr(wa1, A.d1, B.D[1][1]);
    B.T[0][0] = fma_cr(wa0, A.t0, B.T[0][0]); B.T[0][1] = fma_cr(wa0, A.t1, B.T[0][1]);
    B.T[1][0] = fma_cr(wa1, A.t0, B.T[1][0]); B.T[1][1] = fma_cr(wa1, A.t1, B.T[1][1]);
}

// The 3-point rule on [0, 1]: xi = 1/2 -+ sqrt(3/20), 1/2; w = 5/18, 4/9, 5/18.
constexpr double G3_X0 = 0.11270166537925831148;
constexpr double G3_X2 = 0.88729833462074168852;
constexpr double G3_W0 = 0.27777777777777777778;
constexpr double G3_W1 = 0.44444444444444444444;

// Adds the blocks of one far panel pair with the NO-point rule to B: NO = 3
// (constants, fully unrolled; the column points in yq), 4, 5, 6 (points and
// weights from the LDS rule table rl), 8 (the panels' stored Gauss points).
template <int NO>
__device__ __forceinline__ void far64_blocks(const FarParams& P, int p, int q, double px0, double py0, double pex,
                                             double pey, double qx0, double qy0, double qex, double qey,
                                             const double (&yq)[6], const Far64Geo& G, const double* tab,
                                             const double* rl, const double* wsh, Far64Blk& B) {
    const double2 z = make_double2(0.0, 0.0);
    if constexpr (NO == 3) {
        const double xs[3] = {G3_X0, 0.5, G3_X2};
        const double w0s[3] = {G3_W0 * (1.0 - G3_X0), G3_W1 * 0.5, G3_W0 * (1.0 - G3_X2)};
        const double w1s[3] = {G3_W0 * G3_X0, G3_W1 * 0.5, G3_W0 * G3_X2};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double xa = fma(xs[a], pex, px0), ya = fma(xs[a], pey, py0);
            Far64Sum A = {z, z, z, z, z, z};
#pragma unroll
            for (int b = 0; b < 3; ++b) far64_point(xa, ya, yq[2 * b], yq[2 * b + 1], w0s[b], w1s[b], G, tab, A);
            far64_fold(w0s[a], w1s[a], A, B);
        }
    } else {
        const double* rx = rl + low_rule_offset(NO < 8 ? NO : 2);
#pragma unroll 1
        for (int a = 0; a < NO; ++a) {
            double xa, ya, wa0, wa1;
            if constexpr (NO == 8) {
                xa = P.gx[8 * p + a];
                ya = P.gy[8 * p + a];
                wa0 = wsh[a];
                wa1 = wsh[8 + a];
            } else {
                xa = fma(rx[a], pex, px0);
                ya = fma(rx[a], pey, py0);
                wa0 = rx[NO + a];
                wa1 = rx[2 * NO + a];
            }
            Far64Sum A = {z, z, z, z, z, z};
#pragma unroll 1
            for (int b = 0; b < NO; ++b) {
                double yb, zb, w0, w1;
                if constexpr (NO == 8) {
                    yb = P.gx[8 * q + b];
                    zb = P.gy[8 * q + b];
                    w0 = wsh[b];
                    w1 = wsh[8 + b];
                } else {
                    yb = fma(rx[b], qex, qx0);
                    zb = fma(rx[b], qey, qy0);
                    w0 = rx[NO + b];
                    w1 = rx[2 * NO + b];
                }
                far64_point(xa, ya, yb, zb, w0, w1, G, tab, A);
            }
            far64_fold(wa0, wa1, A, B);
        }
    }
}

// One work item (nsub-th of a 63 x 63 tile) of an FP64 operator, executed by one
// wavefront.
__device__ __forceinline__ void far_work_item64(const FarParams& P, int64_t work, FarShared64& sh) {
    typedef double2 CT;
    const double* tab = reinterpret_cast<const double*>(sh.tab);
    const int lane = threadIdx.x & 63;
    const FarTile T = far_tile(P, work);
    const int i0 = T.i0, i1 = T.i1, j0 = T.j0;
    if (i0 >= i1) return;
    const int n = P.n;
    double2* __restrict__ oS = static_cast<double2*>(P.S);
    double2* __restrict__ oN = static_cast<double2*>(P.Nm);
    double2* __restrict__ oD = static_cast<double2*>(P.D);

    const int qraw = j0 - 1 + lane;
    const bool qvalid = qraw < n;
    const int q = qraw < 0 ? n - 1 : (qvalid ? qraw : 0);
    const int col = j0 + lane;
    const bool writes = (lane < TB) && (col < n);

    const double hq = P.h[q], nxq = P.nx[q], nyq = P.ny[q];
    const double k = P.k;
    // panel q as node + t * edge (for the reduced rules) and its midpoint
    const int q1 = q + 1 == n ? 0 : q + 1;
    const double qx0 = P.nodes[2 * q], qy0 = P.nodes[2 * q + 1];
    const double qex = P.nodes[2 * q1] - qx0, qey = P.nodes[2 * q1 + 1] - qy0;
    const double qcx = qx0 + 0.5 * qex, qcy = qy0 + 0.5 * qey;
    const double yq[6] = {fma(G3_X0, qex, qx0), fma(G3_X0, qey, qy0), qcx, qcy, fma(G3_X2, qex, qx0),
                          fma(G3_X2, qey, qy0)};

    const CT z = CT{0, 0};
    CT pS0 = z, pS1 = z, pN0 = z, pN1 = z, pD0 = z, pD1 = z, pT0 = z, pT1 = z;
    MirrorRows<double2, 2> M;
    const bool mgroup = T.mirror && (n % 2) == 0;

    for (int pr = i0 - 1; pr < i1; ++pr) {
        const int p = pr < 0 ? pr + n : pr;
        int dd = p - q;
        dd = dd < 0 ? -dd : dd;
        const int cd = dd < n - dd ? dd : n - dd;
        const bool active = qvalid && cd > 1;
        const double hp = P.h[p], nxp = P.nx[p], nyp = P.ny[p];
        const int p1 = p + 1 == n ? 0 : p + 1;
        const double px0 = P.nodes[2 * p], py0 = P.nodes[2 * p + 1];
        const double pex = P.nodes[2 * p1] - px0, pey = P.nodes[2 * p1 + 1] - py0;
        // quadrature order for this row panel, uniform over the wavefront (the largest
        // any lane needs); gap = |midpoint distance| - (hp + hq)/2 against multiples of
        // hm = max(hp, hq), compared squared
        const float mx = (float)(px0 + 0.5 * pex - qcx), my = (float)(py0 + 0.5 * pey - qcy);
        const float m2 = fmaf(mx, mx, my * my);
        const float hmf = (float)fmax(hp, hq), hsf = (float)(0.5 * (hp + hq)), kh = (float)k * hmf;
        const float e3 = fmaf(200.0f, hmf, hsf), e4 = fmaf(32.0f, hmf, hsf);
        const float e5 = fmaf(12.0f, hmf, hsf), e6 = fmaf(6.0f, hmf, hsf);
        const bool over3 = active && !(kh <= 0.016f && m2 >= e3 * e3);
        const bool over4 = active && !(kh <= 0.1f && m2 >= e4 * e4);
        const bool over5 = active && !(kh <= 0.2f && m2 >= e5 * e5);
        const bool over6 = active && !(kh <= 0.2f && m2 >= e6 * e6);
        const int ord = __ballot(over6) ? 8 : (__ballot(over5) ? 6 : (__ballot(over4) ? 5 : (__ballot(over3) ? 4 : 3)));
        Far64Blk B;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) B.S[a][b] = B.D[a][b] = B.T[a][b] = z;
        CT I0h = z;   // sum of the four S blocks divided by hp hq (the Maue term)
        if (active) {
            const Far64Geo G{k, 0.25 * k, nxp, nyp, nxq, nyq};
            if (ord == 3)
                far64_blocks<3>(P, p, q, px0, py0, pex, pey, qx0, qy0, qex, qey, yq, G, tab, sh.rl, sh.wsh, B);
            else if (ord == 4)
                far64_blocks<4>(P, p, q, px0, py0, pex, pey, qx0, qy0, qex, qey, yq, G, tab, sh.rl, sh.wsh, B);
            else if (ord == 5)
                far64_blocks<5>(P, p, q, px0, py0, pex, pey, qx0, qy0, qex, qey, yq, G, tab, sh.rl, sh.wsh, B);
            else if (ord == 6)
                far64_blocks<6>(P, p, q, px0, py0, pex, pey, qx0, qy0, qex, qey, yq, G, tab, sh.rl, sh.wsh, B);
            else
                far64_blocks<8>(P, p, q, px0, py0, pex, pey, qx0, qy0, qex, qey, yq, G, tab, sh.rl, sh.wsh, B);
            I0h = cadd(cadd(B.S[0][0], B.S[0][1]), cadd(B.S[1][0], B.S[1][1]));
            const double hh = hp * hq;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    B.S[a][b] = cscale(B.S[a][b], hh);
                    B.D[a][b] = cscale(B.D[a][b], hh);
                    B.T[a][b] = cscale(B.T[a][b], hh);
                }
        }
        const CT S00 = B.S[0][0], S01 = B.S[0][1], S10 = B.S[1][0], S11 = B.S[1][1];
        const CT D00 = B.D[0][0], D01 = B.D[0][1], D10 = B.D[1][0], D11 = B.D[1][1];
        const CT T00 = B.T[0][0], T01 = B.T[0][1], T10 = B.T[1][0], T11 = B.T[1][1];
        // Maue form of N from S: N_ab = s_a s_b I0/(hp hq) - k^2 (np.nq) S_ab
        const double kk = -k * k * fma(nxp, nxq, nyp * nyq);
        const CT N00 = cadd(I0h, cscale(S00, kk));
        const CT N01 = csub(cscale(S01, kk), I0h);
        const CT N10 = csub(cscale(S10, kk), I0h);
        const CT N11 = cadd(I0h, cscale(S11, kk));

        if (pr >= i0) {
            const int i = pr;
            // row i receives psi_0 of the current row panel and psi_1 of the previous one
            const CT rS0 = cadd(S00, pS0), rS1 = cadd(S01, pS1);
            const CT rN0 = cadd(N00, pN0), rN1 = cadd(N01, pN1);
            const CT rD0 = cadd(D00, pD0), rD1 = cadd(D01, pD1);
            const CT rT0 = cadd(T00, pT0), rT1 = cadd(T01, pT1);
            const CT nS = shfl_down1(rS0), nN = shfl_down1(rN0);
            const CT nD = shfl_down1(rD0), nT = shfl_down1(rT0);
            if (writes)
                far_store<double2, 2>(oS, oN, oD, n, T, mgroup, i, col, cadd(rS1, nS), cadd(rN1, nN),
                                      cadd(rD1, nD), cadd(rT1, nT), M);
        }
        pS0 = S10; pS1 = S11; pN0 = N10; pN1 = N11;
        pD0 = D10; pD1 = D11; pT0 = T10; pT1 = T11;
    }
}

// ------------------------------------------------ FP32 far pass (complex64 operators)
// Kernel values and sums in FP32; point coordinates, distances and the Bessel
// argument in FP64 (the table variable is an FP32 offset from an FP64 interval
// centre, so the rounding of x never enters). N only off the FP64 band, where
// the four panel pairs of every entry are >= 3 panels apart, so the Maue sum
// (which cancels like (h/R)^2 there) is replaced by the integrated-back kernel
//   d_sx d_sy g - k^2 (n_p.n_q) g = k^2 g (u v - nn) + c (nn - 2 u v),
//   u = tau_p.d/R, v = tau_q.d/R, nn = n_p.n_q = tau_p.tau_q.
// Weights carry the panel lengths (row: h_p w_a psi_alpha, column: h_q w_b psi_beta),
// so the pair blocks need no final scaling.
struct Far32Col {   // per lane: the column panel q
    double qx0, qy0, qex, qey;
    float nxq, nyq, hq;
};
struct Far32Row {   // wave-uniform: the row panel p
    double px0, py0, pex, pey;
    float nxp, nyp, hp, nn;
};
struct Far32Sum {   // b-sums of one row point: (S, D, T, H) x (psi_0, psi_1) of the column panel
    float2 s0, s1, d0, d1, t0, t1, h0, h1;
};
struct Far32Blk {   // 2 x 2 blocks of the pair: [alpha][beta] of S, D, T, H
    float2 S[2][2], D[2][2], T[2][2], H[2][2];
};

__device__ __forceinline__ void far32_point(double xa, double ya, double yb, double zb, float w0, float w1,
                                            double k, float kq, float kk2q, const Far32Row& r, const Far32Col& cq,
                                            const float* tab, Far32Sum& A) {
    const double dx = xa - yb, dy = ya - zb;
    const double R2 = fma(dx, dx, dy * dy);
    // FP32 reciprocal square root refined by one Newton step in FP64 (relative
    // error ~1e-14: the Bessel argument needs FP64 accuracy, nothing else does)
    const double r0 = (double)__builtin_amdgcn_rsqf((float)R2);
    const double ri = r0 * fma(-0.5 * R2, r0 * r0, 1.5);
    const Bessel01f bs = hf32_eval(k * (R2 * ri), tab);
    const float ir = (float)ri;
    const float dxf = (float)dx, dyf = (float)dy;
    // g = (i/4) H0 and c = (ik/4) H1 / R
    const float2 g = make_float2(-0.25f * bs.y0, 0.25f * bs.j0);
    const float kr = kq * ir;
    const float2 c = make_float2(-kr * bs.y1, kr * bs.j1);
    const float dq = fmaf(dxf, cq.nxq, dyf * cq.nyq);
    const float dp = -fmaf(dxf, r.nxp, dyf * r.nyp);
    const float u = fmaf(dyf, r.nxp, -dxf * r.nyp) * ir;
    const float v = fmaf(dyf, cq.nxq, -dxf * cq.nyq) * ir;
    const float uv = u * v;
    const float a1 = kk2q * (uv - r.nn), a2 = fmaf(-2.0f, uv, r.nn);
    const float2 hk = make_float2(fmaf(a1, g.x, a2 * c.x), fmaf(a1, g.y, a2 * c.y));
    const float2 cd = make_float2(c.x * dq, c.y * dq), ct = make_float2(c.x * dp, c.y * dp);
    A.s0 = fma_cr(w0, g, A.s0);
    A.s1 = fma_cr(w1, g, A.s1);
    A.d0 = fma_cr(w0, cd, A.d0);
    A.d1 = fma_cr(w1, cd, A.d1);
    A.t0 = fma_cr(w0, ct, A.t0);
    A.t1 = fma_cr(w1, ct, A.t1);
    A.h0 = fma_cr(w0, hk, A.h0);
    A.h1 = fma_cr(w1, hk, A.h1);
}

__device__ __forceinline__ void far32_fold(float wa0, float wa1, const Far32Sum& A, Far32Blk& B) {
    B.S[0][0] = fma_cr(wa0, A.s0, B.S[0][0]); B.S[0][1] = fma_cr(wa0, A.s1, B.S[0][1]);
    B.S[1][0] = fma_cr(wa1, A.s0, B.S[1][0]); B.S[1][1] = fma_cr(wa1, A.s1, B.S[1][1]);
    B.D[0][0] = fma_cr(wa0, A.d0, B.D[0][0]); B.D[0][1] = fma_cr(wa0, A.d1, B.D[0][1]);
    B.D[1][0] = fma_cr(wa1, A.d0, B.D[1][0]); B.D[1][1] = fma_cr(wa1, A.d1, B.D[1][1]);
    B.T[0][0] = fma_cr(wa0, A.t0, B.T[0][0]); B.T[0][1] = fma_cr(wa0, A.t1, B.T[0][1]);
    B.T[1][0] = fma_cr(wa1, A.t0, B.T[1][0]); B.T[1][1] = fma_cr(wa1, A.t1, B.T[1][1]);
    B.H[0][0] = fma_cr(wa0, A.h0, B.H[0][0]); B.H[0][1] = fma_cr(wa0, A.h1, B.H[0][1]);
    B.H[1][0] = fma_cr(wa1, A.h0, B.H[1][0]); B.H[1][1] = fma_cr(wa1, A.h1, B.H[1][1]);
}

// The 2-point rule (xi = 1/2 -+ 1/(2 sqrt 3), w = 1/2), fully unrolled: w psi_0 and
// w psi_1 at the two points are (c_hi, c_lo) and (c_lo, c_hi).
constexpr double G2_LO = 0.21132486540518711775;
constexpr double G2_HI = 0.78867513459481288225;
constexpr float G2_CHI = 0.39433756729740644113f;
constexpr float G2_CLO = 0.10566243270259355887f;

// Adds the blocks of one far panel pair with the NO-point rule to B: NO = 2 (constants), 3 or 4
// (points and weights from the LDS rule table rl), 8 (the panels' stored Gauss
// points and the weights wsh).
template <int NO>
__device__ __forceinline__ void far32_blocks(const FarParams& P, int p, int q, const Far32Row& r,
                                             const Far32Col& cq, const double (&yq)[4], float kq, float kk2q,
                                             const float* tab, const double* rl, const double* wsh, Far32Blk& B) {
    const double k = P.k;
    const float2 z = make_float2(0.f, 0.f);
    if constexpr (NO == 2) {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const double xi = a == 0 ? G2_LO : G2_HI;
            const double xa = fma(xi, r.pex, r.px0), ya = fma(xi, r.pey, r.py0);
            Far32Sum A = {z, z, z, z, z, z, z, z};
            far32_point(xa, ya, yq[0], yq[1], cq.hq * G2_CHI, cq.hq * G2_CLO, k, kq, kk2q, r, cq, tab, A);
            far32_point(xa, ya, yq[2], yq[3], cq.hq * G2_CLO, cq.hq * G2_CHI, k, kq, kk2q, r, cq, tab, A);
            const float wa0 = r.hp * (a == 0 ? G2_CHI : G2_CLO), wa1 = r.hp * (a == 0 ? G2_CLO : G2_CHI);
            far32_fold(wa0, wa1, A, B);
        }
    } else {
        const double* rx = rl + low_rule_offset(NO < 8 ? NO : 2);
#pragma unroll 1
        for (int a = 0; a < NO; ++a) {
            double xa, ya;
            float wa0, wa1;
            if constexpr (NO == 8) {
                xa = P.gx[8 * p + a];
                ya = P.gy[8 * p + a];
                wa0 = (float)(r.hp * wsh[a]);
                wa1 = (float)(r.hp * wsh[8 + a]);
            } else {
                xa = fma(rx[a], r.pex, r.px0);
                ya = fma(rx[a], r.pey, r.py0);
                wa0 = (float)(r.hp * rx[NO + a]);
                wa1 = (float)(r.hp * rx[2 * NO + a]);
            }
            Far32Sum A = {z, z, z, z, z, z, z, z};
            constexpr int UB = NO == 8 ? 1 : NO;
#pragma unroll UB
            for (int b = 0; b < NO; ++b) {
                double yb, zb;
                float w0, w1;
                if constexpr (NO == 8) {
                    yb = P.gx[8 * q + b];
                    zb = P.gy[8 * q + b];
                    w0 = (float)(cq.hq * wsh[b]);
                    w1 = (float)(cq.hq * wsh[8 + b]);
                } else {
                    yb = fma(rx[b], cq.qex, cq.qx0);
                    zb = fma(rx[b], cq.qey, cq.qy0);
                    w0 = (float)(cq.hq * rx[NO + b]);
                    w1 = (float)(cq.hq * rx[2 * NO + b]);
                }
                far32_point(xa, ya, yb, zb, w0, w1, k, kq, kk2q, r, cq, tab, A);
            }
            far32_fold(wa0, wa1, A, B);
        }
    }
}

// One work item of a complex64 operator. The Gauss order (8 down to 2 points per
// panel) is taken per row panel as the largest any lane of the wavefront needs
// (thresholds in the comment at the top of this file); the squared midpoint
// distance is compared, which needs no square root.
__device__ __forceinline__ void far_work_item32(const FarParams& P, int64_t work, FarShared32& sh) {
    const float* tab = reinterpret_cast<const float*>(sh.tab);
    const int lane = threadIdx.x & 63;
    const FarTile T = far_tile(P, work);
    const int i0 = T.i0, i1 = T.i1, j0 = T.j0;
    if (i0 >= i1) return;
    const int n = P.n;
    float2* __restrict__ oS = static_cast<float2*>(P.S);
    float2* __restrict__ oN = static_cast<float2*>(P.Nm);
    float2* __restrict__ oD = static_cast<float2*>(P.D);

    const int qraw = j0 - 1 + lane;
    const bool qvalid = qraw < n;
    const int q = qraw < 0 ? n - 1 : (qvalid ? qraw : 0);
    const int col = j0 + lane;
    const bool writes = (lane < TB) && (col < n);
    const double k = P.k;
    const float kq = (float)(0.25 * k), kk2q = (float)(k * k);
    const float kf = (float)k;

    Far32Col cq;
    {
        const int q1 = q + 1 == n ? 0 : q + 1;
        cq.qx0 = P.nodes[2 * q];
        cq.qy0 = P.nodes[2 * q + 1];
        cq.qex = P.nodes[2 * q1] - cq.qx0;
        cq.qey = P.nodes[2 * q1 + 1] - cq.qy0;
        cq.nxq = (float)P.nx[q];
        cq.nyq = (float)P.ny[q];
        cq.hq = (float)P.h[q];
    }
    const double yq[4] = {fma(G2_LO, cq.qex, cq.qx0), fma(G2_LO, cq.qey, cq.qy0), fma(G2_HI, cq.qex, cq.qx0),
                          fma(G2_HI, cq.qey, cq.qy0)};
    const double qcx = fma(0.5, cq.qex, cq.qx0), qcy = fma(0.5, cq.qey, cq.qy0);

    const float2 z = make_float2(0.f, 0.f);
    float2 pS0 = z, pS1 = z, pH0 = z, pH1 = z, pD0 = z, pD1 = z, pT0 = z, pT1 = z;
    MirrorRows<float2, 4> M;
    const bool mgroup = T.mirror && (n % 4) == 0;

    for (int pr = i0 - 1; pr < i1; ++pr) {
        const int p = pr < 0 ? pr + n : pr;
        int dd = p - q;
        dd = dd < 0 ? -dd : dd;
        // far pairs whose four entries (offsets o - 1 .. o + 1, o = q - p) do not all
        // lie in the FP64 band (those are left to the band kernel)
        const int cd = dd < n - dd ? dd : n - dd;
        const bool active = qvalid && cd > 1 && cd >= P.bw;
        Far32Row r;
        const int p1 = p + 1 == n ? 0 : p + 1;
        r.px0 = P.nodes[2 * p];
        r.py0 = P.nodes[2 * p + 1];
        r.pex = P.nodes[2 * p1] - r.px0;
        r.pey = P.nodes[2 * p1 + 1] - r.py0;
        const double nxp = P.nx[p], nyp = P.ny[p];
        r.nxp = (float)nxp;
        r.nyp = (float)nyp;
        r.hp = (float)P.h[p];
        r.nn = fmaf(r.nxp, cq.nxq, r.nyp * cq.nyq);
        // orders: 4 for gap >= 6 hm (kh <= 0.5), 3 for >= 16 hm (kh <= 0.15), 2 for
        // >= 200 hm (kh <= 0.025), else 8; gap = |midpoint distance| - (hp + hq)/2
        const float mx = (float)(fma(0.5, r.pex, r.px0) - qcx), my = (float)(fma(0.5, r.pey, r.py0) - qcy);
        const float m2 = fmaf(mx, mx, my * my);
        const float hm = fmaxf(r.hp, cq.hq), hs = 0.5f * (r.hp + cq.hq), kh = kf * hm;
        const float e2 = fmaf(200.0f, hm, hs), e3 = fmaf(16.0f, hm, hs), e4 = fmaf(6.0f, hm, hs);
        const bool over2 = active && !(kh <= 0.025f && m2 >= e2 * e2);
        const bool over3 = active && !(kh <= 0.15f && m2 >= e3 * e3);
        const bool over4 = active && !(kh <= 0.5f && m2 >= e4 * e4);
        const int ord = __ballot(over4) ? 8 : (__ballot(over3) ? 4 : (__ballot(over2) ? 3 : 2));
        Far32Blk B;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) B.S[a][b] = B.D[a][b] = B.T[a][b] = B.H[a][b] = z;
        if (active) {
            if (ord == 2) far32_blocks<2>(P, p, q, r, cq, yq, kq, kk2q, tab, sh.rl, sh.wsh, B);
            else if (ord == 3) far32_blocks<3>(P, p, q, r, cq, yq, kq, kk2q, tab, sh.rl, sh.wsh, B);
            else if (ord == 4) far32_blocks<4>(P, p, q, r, cq, yq, kq, kk2q, tab, sh.rl, sh.wsh, B);
            else far32_blocks<8>(P, p, q, r, cq, yq, kq, kk2q, tab, sh.rl, sh.wsh, B);
        }
        if (pr >= i0) {
            const int i = pr;
            // row i receives psi_0 of the current row panel and psi_1 of the previous one
            const float2 rS0 = cadd(B.S[0][0], pS0), rS1 = cadd(B.S[0][1], pS1);
            const float2 rH0 = cadd(B.H[0][0], pH0), rH1 = cadd(B.H[0][1], pH1);
            const float2 rD0 = cadd(B.D[0][0], pD0), rD1 = cadd(B.D[0][1], pD1);
            const float2 rT0 = cadd(B.T[0][0], pT0), rT1 = cadd(B.T[0][1], pT1);
            const float2 nS = shfl_down1(rS0), nH = shfl_down1(rH0);
            const float2 nD = shfl_down1(rD0), nT = shfl_down1(rT0);
            // cyclic offset col - i in (-n/2, n/2]; N on the band is kept in complex128
            // (asm_nband_kernel), the complex64 matrix holds zeros there
            int dcy = col - i;
            dcy = dcy < 0 ? dcy + n : dcy;
            dcy = 2 * dcy > n ? dcy - n : dcy;
            const bool inband = (dcy < 0 ? -dcy : dcy) <= P.bw;
            const float2 vN = inband ? z : cadd(rH1, nH);
            if (writes)
                far_store<float2, 4>(oS, oN, oD, n, T, mgroup, i, col, cadd(rS1, nS), vN, cadd(rD1, nD),
                                     cadd(rT1, nT), M);
        }
        pS0 = B.S[1][0]; pS1 = B.S[1][1]; pH0 = B.H[1][0]; pH1 = B.H[1][1];
        pD0 = B.D[1][0]; pD1 = B.D[1][1]; pT0 = B.T[1][0]; pT1 = B.T[1][1];
    }
}

__global__ __launch_bounds__(64 * WAVES, 2) void asm_far_kernel64(FarParams P, W8 wt, WLow wl) {
    __shared__ FarShared64 sh;
    far_shared_setup(sh, P.tab, wt, wl);
    const int64_t work = (int64_t)blockIdx.x * WAVES + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (work >= P.nwork) return;
    far_work_item64(P, work, sh);
}

__global__ __launch_bounds__(64 * WAVES, 2) void asm_far_kernel32(FarParams P, W8 wt, WLow wl) {
    __shared__ FarShared32 sh;
    far_shared_setup(sh, P.tab, wt, wl);
    const int64_t work = (int64_t)blockIdx.x * WAVES + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (work >= P.nwork) return;
    far_work_item32(P, work, sh);
}

// Many operators in one launch: a persistent grid whose wavefronts take work
// items from a global counter until the queue (all tiles of all operators,
// prefix[j] = first item of operator j) is exhausted; every wavefront exits
// once the counter passes the total.
template <bool F32>
__global__ __launch_bounds__(64 * WAVES, 2) void asm_far_batch_kernel(const FarParams* __restrict__ jobs,
                                                                      const int64_t* __restrict__ prefix, int njobs,
                                                                      unsigned long long* __restrict__ counter,
                                                                      const void* __restrict__ tabg, W8 wt,
                                                                      WLow wl) {
    typedef typename std::conditional<F32, FarShared32, FarShared64>::type SH;
    __shared__ SH sh;
    far_shared_setup(sh, tabg, wt, wl);
    const int64_t total = prefix[njobs];
    for (;;) {
        unsigned long long w = 0;
        if ((threadIdx.x & 63) == 0) w = atomicAdd(counter, 1ull);
        w = __shfl(w, 0, 64);
        if ((int64_t)w >= total) break;
        int lo = 0, hi = njobs - 1;   // last j with prefix[j] <= w
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= (int64_t)w) lo = mid;
            else hi = mid - 1;
        }
        const int j = __builtin_amdgcn_readfirstlane(lo);
        if constexpr (F32) far_work_item32(jobs[j], (int64_t)w - prefix[j], sh);
        else far_work_item64(jobs[j], (int64_t)w - prefix[j], sh);
    }
}

__global__ void zero_u64_kernel(unsigned long long* p) { *p = 0ull; }

// ------------------------------------------------ the band of complex64 operators
// The hypersingular N of the mixed-precision operators on the cyclic band
// |j - i| <= w, in FP64 and stored in complex128 (its O(1) entries near the
// diagonal meet eigenvalues O(h) on smooth vectors, so FP32 errors there would
// be amplified ~1/h), and S and D there in FP64 (complex64 output). The FP32 far
// pass leaves out the panel pairs whose four entries all lie in the band.
// Far panel pairs only: the self and adjacent pairs follow in asm_near /
// asm_band.
// Pass 1 (asm_nband_blocks_kernel): one wavefront per 64 consecutive row panels p
// and one panel offset o = q - p in [2, w + 1], uniform over the wavefront and
// with it the quadrature order. It stores the 2 x 2 blocks of S, N, D and of the
// transposed double layer T (D(j, i) from the same kernel values) of the pair
// (p, p + o) as blk[o - 2][m][p], m = 4 kind + 2 a + b.
// Pass 2 (asm_nband_combine_kernel): one thread per entry (i, d), d in [0, w],
// j = i + d: X(i, j) = B(i, d)[0][0] + B(i, d - 1)[0][1] + B(i - 1, d)[1][1]
// + B(i - 1, d + 1)[1][0] with B(p, o) = 0 for |o| <= 1; N and S are symmetric
// and D(j, i) is the same sum over T, so (j, i) is written from the same thread.
struct NBandParams {
    const double* __restrict__ gx;
    const double* __restrict__ gy;
    const double* __restrict__ h;
    const double* __restrict__ nx;
    const double* __restrict__ ny;
    const double* __restrict__ nodes;
    const double* __restrict__ tab;   // HF_TAB (FP64 far-field set)
    double2* __restrict__ blk;        // [w][16][n] pair blocks
    double2* __restrict__ nband;      // [n][2 w + 1]
    float2* __restrict__ S;           // complex64 S, N (zero on the band) and D, row-major n x n
    float2* __restrict__ D;
    double k;
    int n, w;
    int nrb;                          // row blocks of 64
};

__global__ __launch_bounds__(64 * WAVES) void asm_nband_blocks_kernel(NBandParams P, W8 wt, WLow wl) {
    __shared__ double tab[HF_TAB_DOUBLES];
    __shared__ double wsh[16];
    __shared__ double rl[WLOW_DOUBLES];
    for (int t = threadIdx.x; t < HF_TAB_DOUBLES; t += blockDim.x) tab[t] = P.tab[t];
    if (threadIdx.x < 8) {
        wsh[threadIdx.x] = wt.wp0[threadIdx.x];
        wsh[8 + threadIdx.x] = wt.wp1[threadIdx.x];
    }
    if (threadIdx.x < WLOW_DOUBLES) rl[threadIdx.x] = wl.r[threadIdx.x];
    __syncthreads();
    const int wave = blockIdx.x * WAVES + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (wave >= P.nrb * P.w) return;
    const int oi = wave / P.nrb, rb = wave - oi * P.nrb;
    const int o = oi + 2;
    const int n = P.n;
    const int lane = threadIdx.x & 63;
    const int pr = rb * 64 + lane;
    const bool valid = pr < n;
    const int p = valid ? pr : n - 1;
    int q = p + o;
    q = q >= n ? q - n : q;
    const double k = P.k;
    const double hp = P.h[p], nxp = P.nx[p], nyp = P.ny[p];
    const double hq = P.h[q], nxq = P.nx[q], nyq = P.ny[q];
    const int p1 = p + 1 == n ? 0 : p + 1, q1 = q + 1 == n ? 0 : q + 1;
    const double px0 = P.nodes[2 * p], py0 = P.nodes[2 * p + 1];
    const double pex = P.nodes[2 * p1] - px0, pey = P.nodes[2 * p1 + 1] - py0;
    const double qx0 = P.nodes[2 * q], qy0 = P.nodes[2 * q + 1];
    const double qex = P.nodes[2 * q1] - qx0, qey = P.nodes[2 * q1 + 1] - qy0;
    int ord = 0;
    if (valid) {
        const double hm = fmax(hp, hq);
        const double dist = hypot(px0 + 0.5 * pex - qx0 - 0.5 * qex, py0 + 0.5 * pey - qy0 - 0.5 * qey) - 0.5 * (hp + hq);
        const double kh = k * hm;
        ord = 8;
        if (kh <= 0.2 && dist >= 12.0 * hm) ord = 6;
        if (kh <= 0.2 && dist >= 24.0 * hm) ord = 5;
        if (kh <= 0.1 && dist >= 64.0 * hm) ord = 4;
        if (kh <= 0.016 && dist >= 512.0 * hm) ord = 3;
    }
    const int no = __builtin_amdgcn_readfirstlane(wave_max_int(ord));
    const double2 z = make_double2(0.0, 0.0);
    double2 S[2][2] = {{z, z}, {z, z}}, D[2][2] = {{z, z}, {z, z}}, T[2][2] = {{z, z}, {z, z}};
    const double* rx = rl + low_rule_offset(no < 8 ? no : 2);
#pragma unroll 1
    for (int a = 0; a < no; ++a) {
        double xa, ya, wa0, wa1;
        if (no == 8) {
            xa = P.gx[8 * p + a];
            ya = P.gy[8 * p + a];
            wa0 = wsh[a];
            wa1 = wsh[8 + a];
        } else {
            xa = px0 + rx[a] * pex;
            ya = py0 + rx[a] * pey;
            wa0 = rx[no + a];
            wa1 = rx[2 * no + a];
        }
        double2 g0 = z, g1 = z, d0 = z, d1 = z, t0 = z, t1 = z;
#pragma unroll 1
        for (int b = 0; b < no; ++b) {
            double yb, zb, w0, w1;
            if (no == 8) {
                yb = P.gx[8 * q + b];
                zb = P.gy[8 * q + b];
                w0 = wsh[b];
                w1 = wsh[8 + b];
            } else {
                yb = qx0 + rx[b] * qex;
                zb = qy0 + rx[b] * qey;
                w0 = rx[no + b];
                w1 = rx[2 * no + b];
            }
            const double dx = xa - yb, dy = ya - zb;
            const double R2 = fma(dx, dx, dy * dy);
            const double r0 = __builtin_amdgcn_rsq(R2);
            const double ri = r0 * fma(-0.5 * R2, r0 * r0, 1.5);
            const Bessel01 bs = hf_eval(k * (R2 * ri), tab);
            const double2 g = make_double2(-0.25 * bs.y0, 0.25 * bs.j0);
            const double kr = 0.25 * k * ri;
            const double2 c = make_double2(-kr * bs.y1, kr * bs.j1);
            const double dq = fma(dx, nxq, dy * nyq), dp = -fma(dx, nxp, dy * nyp);
            const double2 cd = cscale(c, dq), ct = cscale(c, dp);
            g0 = fma_cr(w0, g, g0);
            g1 = fma_cr(w1, g, g1);
            d0 = fma_cr(w0, cd, d0);
            d1 = fma_cr(w1, cd, d1);
            t0 = fma_cr(w0, ct, t0);
            t1 = fma_cr(w1, ct, t1);
        }
        S[0][0] = fma_cr(wa0, g0, S[0][0]); S[0][1] = fma_cr(wa0, g1, S[0][1]);
        S[1][0] = fma_cr(wa1, g0, S[1][0]); S[1][1] = fma_cr(wa1, g1, S[1][1]);
        D[0][0] = fma_cr(wa0, d0, D[0][0]); D[0][1] = fma_cr(wa0, d1, D[0][1]);
        D[1][0] = fma_cr(wa1, d0, D[1][0]); D[1][1] = fma_cr(wa1, d1, D[1][1]);
        T[0][0] = fma_cr(wa0, t0, T[0][0]); T[0][1] = fma_cr(wa0, t1, T[0][1]);
        T[1][0] = fma_cr(wa1, t0, T[1][0]); T[1][1] = fma_cr(wa1, t1, T[1][1]);
    }
    if (!valid) return;
    const double hh = hp * hq;
    // Maue form N_ab = s_a s_b I0/(hp hq) - k^2 (n_p.n_q) S_ab; the sums above lack the
    // factor hp hq of S_ab and I0, which cancels in the first term
    const double2 I0h = cadd(cadd(S[0][0], S[0][1]), cadd(S[1][0], S[1][1]));
    const double kk = -k * k * fma(nxp, nxq, nyp * nyq) * hh;
    double2* out = P.blk + (size_t)oi * 16 * n + p;
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
        for (int b2 = 0; b2 < 2; ++b2) {
            const int m = 2 * a2 + b2;
            const double2 nab = a2 == b2 ? cadd(I0h, cscale(S[a2][b2], kk)) : csub(cscale(S[a2][b2], kk), I0h);
            out[(size_t)(0 + m) * n] = cscale(S[a2][b2], hh);
            out[(size_t)(4 + m) * n] = nab;
            out[(size_t)(8 + m) * n] = cscale(D[a2][b2], hh);
            out[(size_t)(12 + m) * n] = cscale(T[a2][b2], hh);
        }
}

__global__ __launch_bounds__(256) void asm_nband_combine_kernel(NBandParams P) {
    const int n = P.n, w = P.w;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * (w + 1)) return;
    const int d = (int)(t / n), i = (int)(t - (int64_t)d * n);
    const int im = i == 0 ? n - 1 : i - 1;
    double2 x[4];   // S, N, D, T
#pragma unroll
    for (int kd = 0; kd < 4; ++kd) x[kd] = make_double2(0.0, 0.0);
    // (p, o, a, b): (i, d, 0, 0), (i, d - 1, 0, 1), (i - 1, d, 1, 1), (i - 1, d + 1, 1, 0)
    const int ps[4] = {i, i, im, im}, os[4] = {d, d - 1, d, d + 1}, ms[4] = {0, 1, 3, 2};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (os[u] < 2) continue;
        const double2* b = P.blk + (size_t)(os[u] - 2) * 16 * n + ps[u];
#pragma unroll
        for (int kd = 0; kd < 4; ++kd) x[kd] = cadd(x[kd], b[(size_t)(4 * kd + ms[u]) * n]);
    }
    int j = i + d;
    j = j >= n ? j - n : j;
    const int bs = 2 * w + 1;
    const float2 sf = make_float2((float)x[0].x, (float)x[0].y);
    P.nband[(int64_t)i * bs + w + d] = x[1];
    P.S[(int64_t)i * n + j] = sf;
    P.D[(int64_t)i * n + j] = make_float2((float)x[2].x, (float)x[2].y);
    if (d > 0) {
        P.nband[(int64_t)j * bs + w - d] = x[1];
        P.S[(int64_t)j * n + i] = sf;
        P.D[(int64_t)j * n + i] = make_float2((float)x[3].x, (float)x[3].y);
    }
}

// ----------------------------------------------------------------- near pairs
struct NearParams {
    const double* __restrict__ gx;
    const double* __restrict__ gy;
    const double* __restrict__ h;
    const double* __restrict__ nx;
    const double* __restrict__ ny;
    const double* __restrict__ tab;
    const double* __restrict__ gl32;   // x[32], w[32] on [0,1]
    double2* __restrict__ nb;          // [n][3][8]: S00 S01 S10 S11 D00 D01 D10 D11
    double k;
    int n;
};

__global__ __launch_bounds__(128) void asm_near_block_kernel(NearParams P, W8 wt) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = P.n;
    if (t >= 3 * n) return;
    const int p = t / 3, s = t - 3 * (t / 3);
    const int q = s == 0 ? (p == 0 ? n - 1 : p - 1) : (s == 1 ? p : (p + 1 == n ? 0 : p + 1));
    double2 So[2][2], Do[2][2];
    near_pair_blocks<true>(P.gx + 8 * p, P.gy + 8 * p, P.gx + 8 * q, P.gy + 8 * q, P.h[p], P.h[q], P.nx[p],
                           P.ny[p], P.nx[q], P.ny[q], s, P.k, P.tab, P.gl32, wt, So, Do);
    double2* out = P.nb + (int64_t)t * 8;
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
        for (int b2 = 0; b2 < 2; ++b2) {
            out[2 * a2 + b2] = So[a2][b2];
            out[4 + 2 * a2 + b2] = Do[a2][b2];
        }
}

struct BandParams {
    const double* __restrict__ h;
    const double* __restrict__ nx;
    const double* __restrict__ ny;
    const double2* __restrict__ nb;
    void* __restrict__ S;
    void* __restrict__ Nm;
    void* __restrict__ D;
    double2* __restrict__ nband;     // FP32 operators: N on the cyclic band |d| <= bw (complex128)
    int bw;
    double k;
    int n;
};

// Near-pair contribution to entry (r, c): pairs (p, q) = (r - a, c - b).
__device__ void near_entry(const BandParams& P, int r, int c, double2& s, double2& nn, double2& d) {
    const int n = P.n;
    s = nn = d = make_double2(0.0, 0.0);
    for (int a = 0; a < 2; ++a) {
        const int p = (r - a + n) % n;
        for (int b = 0; b < 2; ++b) {
            const int q = (c - b + n) % n;
            int slot = -1;
            if (q == p) slot = 1;
            else if (q == (p + 1) % n) slot = 2;
            else if (q == (p + n - 1) % n) slot = 0;
            if (slot < 0) continue;
            const double2* blk = P.nb + ((int64_t)p * 3 + slot) * 8;
            const double2 I0 = cadd(cadd(blk[0], blk[1]), cadd(blk[2], blk[3]));
            const double hh = P.h[p] * P.h[q];
            const double kk = -P.k * P.k * (P.nx[p] * P.nx[q] + P.ny[p] * P.ny[q]);
            const double sg = (a == b) ? 1.0 : -1.0;
            const double2 sab = blk[2 * a + b];
            s = cadd(s, sab);
            nn = cadd(nn, cadd(cscale(I0, sg / hh), cscale(sab, kk)));
            d = cadd(d, blk[4 + 2 * a + b]);
        }
    }
}

__device__ __forceinline__ double2 ld_c(const double2* p, int64_t i) { return p[i]; }
__device__ __forceinline__ double2 ld_c(const float2* p, int64_t i) {
    const float2 v = p[i];
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st_c(double2* p, int64_t i, double2 v) { p[i] = v; }
__device__ __forceinline__ void st_c(float2* p, int64_t i, double2 v) { p[i] = make_float2((float)v.x, (float)v.y); }

// Adds the near-pair blocks to the band |i - j| <= 2 (in FP64) and symmetrises S, N there.
template <typename CT>
__global__ void asm_band_kernel(BandParams P) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = P.n;
    if (t >= 3 * n) return;
    CT* S = static_cast<CT*>(P.S);
    CT* Nm = static_cast<CT*>(P.Nm);
    CT* D = static_cast<CT*>(P.D);
    const int i = t / 3, dlt = t - 3 * (t / 3);
    const int j = (i + dlt) % n;
    double2 s1, n1, d1;
    near_entry(P, i, j, s1, n1, d1);
    const int64_t ij = (int64_t)i * n + j, ji = (int64_t)j * n + i;
    // N: FP32 operators keep N near the diagonal in the complex128 band array
    // (filled by the FP64 band pass of the far kernel); the near pairs add there.
    constexpr bool split = std::is_same<CT, float2>::value;
    const int bs = 2 * P.bw + 1;
    if (dlt == 0) {
        st_c(S, ij, cadd(ld_c(S, ij), s1));
        if constexpr (split) {
            double2* e = P.nband + (int64_t)i * bs + P.bw;
            *e = cadd(*e, n1);
        } else {
            st_c(Nm, ij, cadd(ld_c(Nm, ij), n1));
        }
        st_c(D, ij, cadd(ld_c(D, ij), d1));
        return;
    }
    double2 s2, n2, d2;
    near_entry(P, j, i, s2, n2, d2);
    const double2 sa = cscale(cadd(cadd(ld_c(S, ij), s1), cadd(ld_c(S, ji), s2)), 0.5);
    st_c(S, ij, sa);
    st_c(S, ji, sa);
    if constexpr (split) {
        double2* eij = P.nband + (int64_t)i * bs + P.bw + dlt;
        double2* eji = P.nband + (int64_t)j * bs + P.bw - dlt;
        const double2 na = cscale(cadd(cadd(*eij, n1), cadd(*eji, n2)), 0.5);
        *eij = na;
        *eji = na;
    } else {
        const double2 na = cscale(cadd(cadd(ld_c(Nm, ij), n1), cadd(ld_c(Nm, ji), n2)), 0.5);
        st_c(Nm, ij, na);
        st_c(Nm, ji, na);
    }
    st_c(D, ij, cadd(ld_c(D, ij), d1));
    st_c(D, ji, cadd(ld_c(D, ji), d2));
}

static void far_rules(const Op& op, W8& wt, WLow& wlow) {
    for (int a = 0; a < 8; ++a) {
        wt.wp0[a] = op.rule.w[a] * (1.0 - op.rule.xi[a]);
        wt.wp1[a] = op.rule.w[a] * op.rule.xi[a];
    }
    for (int nq = 2; nq <= 6; ++nq) {
        double x[6], w[6];
        gauss_legendre_01(nq, x, w);
        double* r = wlow.r + low_rule_offset(nq);
        for (int a = 0; a < nq; ++a) {
            r[a] = x[a];
            r[nq + a] = w[a] * (1.0 - x[a]);
            r[2 * nq + a] = w[a] * x[a];
        }
    }
}

static FarParams far_params(Op& op) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    FarParams fp;
    fp.gx = op.gx; fp.gy = op.gy; fp.h = op.h; fp.nx = op.nx; fp.ny = op.ny;
    const bool f32 = op.prec == FDS_FP32;
    fp.tab = f32 ? (const void*)c.hf_tab32 : (const void*)c.hf_tab;
    fp.nodes = op.nodes;
    fp.S = f32 ? (void*)op.S32 : (void*)op.S;
    fp.Nm = f32 ? (void*)op.N32 : (void*)op.Nm;
    fp.D = f32 ? (void*)op.D32 : (void*)op.D;
    fp.k = op.k;
    fp.n = n;
    fp.bw = f32 ? op.nbw : -1;
    const int64_t T = (n + TB - 1) / TB;
    // work items per tile: a quarter tile in FP64 (better balance of the higher orders
    // near the diagonal over the wavefronts), half a tile in FP32
    fp.nsub = f32 ? 2 : 4;
    fp.tr = (TB + fp.nsub - 1) / fp.nsub;
    fp.nwork = T * (T + 1) / 2 * fp.nsub;
    return fp;
}

// self / adjacent pairs and the band correction of one operator
static void launch_near_band(Op& op, const FarParams& fp, const W8& wt) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    const bool f32 = op.prec == FDS_FP32;
    double2* nb = static_cast<double2*>(c.dmalloc(sizeof(double2) * 24 * (size_t)n));
    NearParams np;
    np.gx = op.gx; np.gy = op.gy; np.h = op.h; np.nx = op.nx; np.ny = op.ny;
    np.tab = c.hk_tab; np.gl32 = c.gl32; np.nb = nb; np.k = op.k; np.n = n;
    {
        KScope _ks(c, "asm_near");
        hipLaunchKernelGGL(asm_near_block_kernel, dim3((3 * n + 127) / 128), dim3(128), 0, c.stream,
                       np, wt);
    }
    FDS_HIP_TRY(hipGetLastError());
    BandParams bp;
    bp.h = op.h; bp.nx = op.nx; bp.ny = op.ny; bp.nb = nb;
    bp.S = fp.S; bp.Nm = fp.Nm; bp.D = fp.D; bp.k = op.k; bp.n = n;
    bp.nband = op.Nband;
    bp.bw = op.nbw;
    {
        KScope _ks(c, "asm_band");
        if (f32)
            hipLaunchKernelGGL(asm_band_kernel<float2>, dim3((3 * n + 127) / 128), dim3(128), 0, c.stream, bp);
        else
            hipLaunchKernelGGL(asm_band_kernel<double2>, dim3((3 * n + 127) / 128), dim3(128), 0, c.stream, bp);
    }
    FDS_HIP_TRY(hipGetLastError());
    c.dfree(nb);   // stream-ordered release (see Ctx::dfree)
}

// S, N, D on the cyclic band |d| <= nbw of complex64 operators, in FP64.
static void launch_nband(Op& op, const W8& wt, const WLow& wlow) {
    Ctx& c = *op.ctx;
    NBandParams P;
    P.gx = op.gx; P.gy = op.gy; P.h = op.h; P.nx = op.nx; P.ny = op.ny; P.nodes = op.nodes;
    P.tab = c.hf_tab;
    P.nband = op.Nband;
    P.S = op.S32;
    P.D = op.D32;
    P.k = op.k;
    P.n = (int)op.n;
    P.w = op.nbw;
    P.nrb = (P.n + 63) / 64;
    P.blk = static_cast<double2*>(c.dmalloc(sizeof(double2) * 16 * (size_t)P.n * std::max(P.w, 1)));
    {
        KScope _ks(c, "asm_nband");
        const unsigned nb1 = (unsigned)(((int64_t)P.nrb * P.w + WAVES - 1) / WAVES);
        if (nb1 > 0)
            hipLaunchKernelGGL(asm_nband_blocks_kernel, dim3(nb1), dim3(64 * WAVES), 0, c.stream, P, wt, wlow);
        const int64_t tot = (int64_t)P.n * (P.w + 1);
        hipLaunchKernelGGL(asm_nband_combine_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c.stream, P);
    }
    FDS_HIP_TRY(hipGetLastError());
    c.dfree(P.blk);   // stream-ordered release (see Ctx::dfree)
}

void launch_assemble(Op& op) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    W8 wt;
    WLow wlow;
    far_rules(op, wt, wlow);
    const FarParams fp = far_params(op);
    const bool f32 = op.prec == FDS_FP32;
    const unsigned nblk = (unsigned)((fp.nwork + WAVES - 1) / WAVES);
    {
        KScope _ks(c, "asm_far");
        if (f32)
            hipLaunchKernelGGL(asm_far_kernel32, dim3(nblk), dim3(64 * WAVES), 0, c.stream, fp, wt, wlow);
        else
            hipLaunchKernelGGL(asm_far_kernel64, dim3(nblk), dim3(64 * WAVES), 0, c.stream, fp, wt,
                               wlow);
    }
    FDS_HIP_TRY(hipGetLastError());
    if (f32) launch_nband(op, wt, wlow);
    launch_near_band(op, fp, wt);
}

// All far tiles of several operators of one precision in one persistent launch
// (with complex64 operators: the FP32 pass), then the per-operator FP64 band of
// N (complex64 operators) and the near-pair and band kernels. Geometry must
// already be built.
void launch_assemble_batch(Ctx& c, Op* const* ops, int nops) {
    if (nops <= 0) return;
    std::vector<FarParams> jobs(nops);
    std::vector<int64_t> prefix(nops + 1, 0);
    W8 wt;
    WLow wlow;
    far_rules(*ops[0], wt, wlow);
    const bool f32 = ops[0]->prec == FDS_FP32;
    for (int j = 0; j < nops; ++j) {
        FDS_REQUIRE(ops[j]->prec == ops[0]->prec, FDS_ERR_ARG, "a batch holds operators of one precision");
        jobs[j] = far_params(*ops[j]);
        prefix[j + 1] = prefix[j] + jobs[j].nwork;
    }
    const size_t jb = sizeof(FarParams) * nops, pb = sizeof(int64_t) * (nops + 1);
    char* dbuf = static_cast<char*>(c.dmalloc(jb + pb + 256));
    FarParams* djobs = reinterpret_cast<FarParams*>(dbuf);
    int64_t* dprefix = reinterpret_cast<int64_t*>(dbuf + jb);
    unsigned long long* counter = reinterpret_cast<unsigned long long*>(dbuf + jb + pb + 128 - ((jb + pb) % 128));
    FDS_HIP_TRY(hipMemcpyAsync(djobs, jobs.data(), jb, hipMemcpyHostToDevice, c.stream));
    FDS_HIP_TRY(hipMemcpyAsync(dprefix, prefix.data(), pb, hipMemcpyHostToDevice, c.stream));
    FDS_HIP_TRY(hipStreamSynchronize(c.stream));   // the host tables go out of scope below
    int ncu = 0;
    FDS_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c.device));
    const int64_t want = (prefix[nops] + WAVES - 1) / WAVES;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, 2 * (int64_t)std::max(ncu, 1)));
    {
        KScope _ks(c, "asm_far_batch");
        hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, c.stream, counter);
        if (f32)
            hipLaunchKernelGGL(asm_far_batch_kernel<true>, dim3(grid), dim3(64 * WAVES), 0, c.stream, djobs,
                               dprefix, nops, counter, jobs[0].tab, wt, wlow);
        else
            hipLaunchKernelGGL(asm_far_batch_kernel<false>, dim3(grid), dim3(64 * WAVES), 0, c.stream, djobs,
                               dprefix, nops, counter, jobs[0].tab, wt, wlow);
    }
    FDS_HIP_TRY(hipGetLastError());
    for (int j = 0; j < nops; ++j) {
        if (f32) launch_nband(*ops[j], wt, wlow);
        launch_near_band(*ops[j], jobs[j], wt);
    }
    c.dfree(dbuf);
}

// ---------------------------------------------------------------- Yukawa single layer
// S_y with the kernel (1/2pi) K0(kappa |x - y|) (the single layer at the
// imaginary wavenumber i kappa), the preconditioner of the Yukawa-Calderon
// TE-CFIE (paper, Filters Based Fast Direct Solver, 2D case: the localised
// Calderon preconditioner). FP64, stored row-major as complex128 with zero
// imaginary parts so that the complex products take it unchanged.
// A workgroup forms the 2 x 2 pair blocks of panels [i0 - 1, i0 + YT) x
// [j0 - 1, j0 + YT) in LDS (one per thread: far pairs by the 8 x 8 rule, self
// and adjacent pairs with their logarithmic parts exact) and adds the four that
// meet each entry of its YT x YT tile: entry (i, j) takes block (i - a, j - b)[a][b].
struct YukParams {
    const double* __restrict__ gx;
    const double* __restrict__ gy;
    const double* __restrict__ nodes;
    const double* __restrict__ h;
    const double* __restrict__ nx;
    const double* __restrict__ ny;
    const double* __restrict__ ytab;
    const float* __restrict__ ytab32;   // float32 interval table (FP32 operators)
    const double* __restrict__ gl32;
    double2* __restrict__ Sy;
    double kappa;
    int n;
};

constexpr int YT = 15;   // entries per tile side: (YT + 1)^2 = 256 pair blocks, one per thread

// Gauss order of a far pair from its gap g (midpoint distance minus the two
// half-lengths) in units of the longer panel. The orders keep the quadrature
// error of every block below 1e-13 of the near-diagonal block size against the
// 8 x 8 rule (measured on the star, ellipse and random curves for k R from 0.1 to
// 20: orders 6, 5, 4, 3 first meet it at gaps 2, 5, 14, 58; the thresholds below
// leave a margin of 1.5 to 2).
__device__ __forceinline__ int yukawa_order(double gap) {
    return gap < 3.0 ? 8 : (gap < 8.0 ? 6 : (gap < 24.0 ? 5 : (gap < 100.0 ? 4 : 3)));
}

// Entries of tile row b (rows b*YT .. min(b*YT + YT, n) - 1) use the panel pairs of
// the cyclic run of panels that starts at b*YT - 1; this is its length.
__host__ __device__ inline int yuk_run_len(int b, int n) {
    const int e = b * YT + YT < n ? b * YT + YT : n;
    return e - b * YT + 1;
}

// True when tile (bi, bj) uses the block of a self or adjacent panel pair (cyclic
// panel distance <= 1): the run of row bi widened by one panel on each side meets
// the run of column bj (two cyclic intervals meet iff one holds the other's start).
__host__ __device__ inline bool yuk_tile_near(int bi, int bj, int n) {
    const int li = yuk_run_len(bi, n) + 2, lj = yuk_run_len(bj, n);
    if (li >= n || lj >= n) return true;
    const int si = ((bi * YT - 2) % n + n) % n, sj = ((bj * YT - 1) % n + n) % n;
    return ((sj - si) % n + n) % n < li || ((si - sj) % n + n) % n < lj;
}

// K0 by the unit-interval table with the interval clamped to the table: exact for
// YK_XS <= x < YK_XA (other arguments are redone by yk_k0).
__device__ __forceinline__ double yk_k0_tab(double x, const double* __restrict__ ytab) {
    int c = (int)x;
    c = c < YK_XS ? YK_XS : (c > YK_XA - 1 ? YK_XA - 1 : c);
    const double t = x - ((double)c + 0.5);
    const double* cf = ytab + (c - YK_XS) * (HK_DEG + 1);
    double acc = cf[HK_DEG];
#pragma unroll
    for (int m = HK_DEG - 1; m >= 0; --m) acc = fma(acc, t, cf[m]);
    return acc;
}

// Panel endpoints of a far pair: node and edge vector of p and q.
struct PairGeom {
    double px0, py0, pex, pey, qx0, qy0, qex, qey;
};

// sqrt of a normal positive argument: the hardware reciprocal square root refined
// by two coupled Newton steps for sqrt(s) and 1/(2 sqrt(s)) (Goldschmidt's
// iteration), without the range scaling a general sqrt needs for denormals.
__device__ __forceinline__ double sqrt_normal(double s) {
    const double y = __builtin_amdgcn_rsq(s);
    double g = s * y, hh = 0.5 * y;
    const double r = fma(-hh, g, 0.5);
    g = fma(g, r, g);
    hh = fma(hh, r, hh);
    double d = fma(-g, g, s);
    g = fma(d, hh, g);
    d = fma(-g, g, s);
    return fma(d, hh, g);
}

typedef __attribute__((address_space(4))) const double const_double;

// Point NO-rule node v of a panel: the stored 8-point node or node + xi * edge.
template <int NO>
__device__ __forceinline__ void yuk_node(const YukParams& P, const WLow& wl, int panel, double x0, double y0,
                                         double ex, double ey, int v, double& x, double& y) {
    if (NO == 8) {
        x = P.gx[8 * panel + v];
        y = P.gy[8 * panel + v];
    } else {
        constexpr int off = low_rule_offset(NO < 8 ? NO : 2);
        x = fma(wl.r[off + v], ex, x0);
        y = fma(wl.r[off + v], ey, y0);
    }
}

// Weights w psi_0, w psi_1 of node v of the NO-point rule.
template <int NO>
__device__ __forceinline__ void yuk_wts(const W8& wt, const WLow& wl, int v, double& w0, double& w1) {
    constexpr int off = low_rule_offset(NO < 8 ? NO : 2);
    w0 = NO == 8 ? wt.wp0[v] : wl.r[off + NO + v];
    w1 = NO == 8 ? wt.wp1[v] : wl.r[off + 2 * NO + v];
}

// The NO x NO Gauss product rule of a far pair block (without the factor
// h_p h_q / 2pi), one row of NO kernel values at a time. When every argument of
// the row, over the whole wave, lies in one unit interval of the K0 table (the
// common case: neighbouring pairs see nearly the same distances), the interval's
// coefficients are wave-uniform scalar loads; otherwise each lane reads its own
// from the LDS copy. Returns true when some argument lies outside the table; the
// caller then redoes the block through yk_k0.
typedef __attribute__((address_space(4))) const float const_float;

// K0 at x (float) from the float32 interval table, the interval clamped like yk_k0_tab
__device__ __forceinline__ double yk_k0_tab32(float x, const float* __restrict__ tab) {
    int c = (int)x;
    c = c < YK_XS ? YK_XS : (c > YK_XA - 1 ? YK_XA - 1 : c);
    const float t = x - ((float)c + 0.5f);
    const float* cf = tab + (c - YK_XS) * (YK32_DEG + 1);
    float acc = cf[YK32_DEG];
#pragma unroll
    for (int m = YK32_DEG - 1; m >= 0; --m) acc = fmaf(acc, t, cf[m]);
    return (double)acc;
}

// F32: the kernel values of the table range in single precision (distance squared
// rounded to float, float sqrt, float32 table): relative error ~2e-7, like the FP32
// far field of S, N and D; the accumulation stays in FP64.
template <int NO, bool F32>
__device__ __forceinline__ bool yuk_far_rule(const YukParams& P, const double* __restrict__ ytab, const W8& wt,
                                             const WLow& wl, int p, int q, const PairGeom& g, double acc[2][2]) {
    double yb[NO], zb[NO];
#pragma unroll
    for (int v = 0; v < NO; ++v) yuk_node<NO>(P, wl, q, g.qx0, g.qy0, g.qex, g.qey, v, yb[v], zb[v]);
    bool rare = false;
#pragma unroll 1
    for (int u = 0; u < NO; ++u) {
        double xa, ya, wa0, wa1;
        yuk_node<NO>(P, wl, p, g.px0, g.py0, g.pex, g.pey, u, xa, ya);
        yuk_wts<NO>(wt, wl, u, wa0, wa1);
        typedef typename std::conditional<F32, float, double>::type real;
        real xv[NO];
        real lo = (real)1e30, hi = (real)0;
#pragma unroll
        for (int v = 0; v < NO; ++v) {
            const double dx = xa - yb[v], dy = ya - zb[v];
            const double s2 = fmax(fma(dx, dx, dy * dy), 1e-280);
            if constexpr (F32)
                xv[v] = (float)P.kappa * __builtin_sqrtf((float)s2);
            else
                xv[v] = P.kappa * sqrt_normal(s2);
            lo = fmin(lo, xv[v]);
            hi = fmax(hi, xv[v]);
        }
        rare |= lo < (real)YK_XS || hi >= (real)YK_XA;
        const int c0 = __builtin_amdgcn_readfirstlane((int)xv[0]);
        const bool one = c0 >= YK_XS && c0 < YK_XA && (int)lo == c0 && (int)hi == c0;
        double r0 = 0.0, r1 = 0.0;
        if (__all(one)) {
            if constexpr (F32) {
                const const_float* cf = (const const_float*)(P.ytab32 + (c0 - YK_XS) * (YK32_DEG + 1));
                const float cm = (float)c0 + 0.5f;
#pragma unroll
                for (int v = 0; v < NO; ++v) {
                    const float t = xv[v] - cm;
                    float kf = cf[YK32_DEG];
#pragma unroll
                    for (int m = YK32_DEG - 1; m >= 0; --m) kf = fmaf(kf, t, cf[m]);
                    const double k = (double)kf;
                    double w0, w1;
                    yuk_wts<NO>(wt, wl, v, w0, w1);
                    r0 = fma(w0, k, r0);
                    r1 = fma(w1, k, r1);
                }
            } else {
                const const_double* cf = (const const_double*)(P.ytab + (c0 - YK_XS) * (HK_DEG + 1));
                const double cm = (double)c0 + 0.5;
#pragma unroll
                for (int v = 0; v < NO; ++v) {
                    const double t = xv[v] - cm;
                    double k = cf[HK_DEG];
#pragma unroll
                    for (int m = HK_DEG - 1; m >= 0; --m) k = fma(k, t, cf[m]);
                    double w0, w1;
                    yuk_wts<NO>(wt, wl, v, w0, w1);
                    r0 = fma(w0, k, r0);
                    r1 = fma(w1, k, r1);
                }
            }
        } else {
#pragma unroll
            for (int v = 0; v < NO; ++v) {
                double k;
                if constexpr (F32)
                    k = yk_k0_tab32(xv[v], P.ytab32);
                else
                    k = yk_k0_tab(xv[v], ytab);
                double w0, w1;
                yuk_wts<NO>(wt, wl, v, w0, w1);
                r0 = fma(w0, k, r0);
                r1 = fma(w1, k, r1);
            }
        }
        acc[0][0] = fma(wa0, r0, acc[0][0]);
        acc[0][1] = fma(wa0, r1, acc[0][1]);
        acc[1][0] = fma(wa1, r0, acc[1][0]);
        acc[1][1] = fma(wa1, r1, acc[1][1]);
    }
    return rare;
}

// The same rule with every kernel value through yk_k0 (series and asymptotic
// ranges included).
template <int NO>
__device__ __forceinline__ void yuk_far_rule_any(const YukParams& P, const double* __restrict__ ytab, const W8& wt,
                                              const WLow& wl, int p, int q, const PairGeom& g, double acc[2][2]) {
#pragma unroll 1
    for (int u = 0; u < NO; ++u) {
        double xa, ya, wa0, wa1;
        yuk_node<NO>(P, wl, p, g.px0, g.py0, g.pex, g.pey, u, xa, ya);
        yuk_wts<NO>(wt, wl, u, wa0, wa1);
        double r0 = 0.0, r1 = 0.0;
#pragma unroll 1
        for (int v = 0; v < NO; ++v) {
            double yb, zb, w0, w1;
            yuk_node<NO>(P, wl, q, g.qx0, g.qy0, g.qex, g.qey, v, yb, zb);
            yuk_wts<NO>(wt, wl, v, w0, w1);
            const double dx = xa - yb, dy = ya - zb;
            const double k = yk_k0(P.kappa * sqrt(fma(dx, dx, dy * dy)), ytab);
            r0 = fma(w0, k, r0);
            r1 = fma(w1, k, r1);
        }
        acc[0][0] = fma(wa0, r0, acc[0][0]);
        acc[0][1] = fma(wa0, r1, acc[0][1]);
        acc[1][0] = fma(wa1, r0, acc[1][0]);
        acc[1][1] = fma(wa1, r1, acc[1][1]);
    }
}

template <int NO, bool F32>
__device__ __forceinline__ void yuk_far_order(const YukParams& P, const double* __restrict__ ytab, const W8& wt,
                                              const WLow& wl, int p, int q, const PairGeom& g, double acc[2][2]) {
    if (yuk_far_rule<NO, F32>(P, ytab, wt, wl, p, q, g, acc)) {
        acc[0][0] = acc[0][1] = acc[1][0] = acc[1][1] = 0.0;
        yuk_far_rule_any<NO>(P, ytab, wt, wl, p, q, g, acc);
    }
}

// Block of a far pair (cyclic distance >= 2), the Gauss order chosen by its gap.
template <bool F32>
__device__ __forceinline__ void yuk_far_block(const YukParams& P, const double* __restrict__ ytab, const W8& wt,
                                              const WLow& wl, int p, int q, double B[2][2]) {
    const int n = P.n;
    const int p1 = p + 1 == n ? 0 : p + 1, q1 = q + 1 == n ? 0 : q + 1;
    PairGeom g;
    g.px0 = P.nodes[2 * p];
    g.py0 = P.nodes[2 * p + 1];
    g.qx0 = P.nodes[2 * q];
    g.qy0 = P.nodes[2 * q + 1];
    g.pex = P.nodes[2 * p1] - g.px0;
    g.pey = P.nodes[2 * p1 + 1] - g.py0;
    g.qex = P.nodes[2 * q1] - g.qx0;
    g.qey = P.nodes[2 * q1 + 1] - g.qy0;
    const double hp = P.h[p], hq = P.h[q];
    const double mdx = g.px0 + 0.5 * g.pex - g.qx0 - 0.5 * g.qex, mdy = g.py0 + 0.5 * g.pey - g.qy0 - 0.5 * g.qey;
    const double gap = (sqrt(fma(mdx, mdx, mdy * mdy)) - 0.5 * (hp + hq)) / fmax(hp, hq);
    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    switch (yukawa_order(gap)) {
        case 8: yuk_far_order<8, F32>(P, ytab, wt, wl, p, q, g, acc); break;
        case 6: yuk_far_order<6, F32>(P, ytab, wt, wl, p, q, g, acc); break;
        case 5: yuk_far_order<5, F32>(P, ytab, wt, wl, p, q, g, acc); break;
        case 4: yuk_far_order<4, F32>(P, ytab, wt, wl, p, q, g, acc); break;
        default: yuk_far_order<3, F32>(P, ytab, wt, wl, p, q, g, acc); break;
    }
    const double sc = kInv2Pi * hp * hq;
#pragma unroll
    for (int al = 0; al < 2; ++al)
#pragma unroll
        for (int be = 0; be < 2; ++be) B[al][be] = sc * acc[al][be];
}

__device__ __forceinline__ void yuk_load_table(const YukParams& P, double* ytab) {
    for (int t = threadIdx.x; t < YK_ALL_DOUBLES; t += blockDim.x) ytab[t] = P.ytab[t];
}

// Entry (i, j) of the tile is the sum of the four pair blocks that hold its hat
// functions: blk[a][b] is the block of the panels (i0 - 1 + a, j0 - 1 + b).
__device__ __forceinline__ void yuk_tile_store(const YukParams& P, const double (*blk)[4], int i0, int j0) {
    if (threadIdx.x < YT * YT) {
        const int ti = threadIdx.x / YT, tj = threadIdx.x % YT;
        const int i = i0 + ti, j = j0 + tj;
        if (i < P.n && j < P.n) {
            const int a = ti + 1, b = tj + 1;
            const double v = blk[a * (YT + 1) + b][0] + blk[a * (YT + 1) + b - 1][1] +
                             blk[(a - 1) * (YT + 1) + b][2] + blk[(a - 1) * (YT + 1) + b - 1][3];
            P.Sy[(int64_t)i * P.n + j] = make_double2(v, 0.0);
        }
    }
}

// Tiles that hold no self or adjacent pair: far blocks only. Tiles with such a pair
// return at once (the near kernel owns them).
template <bool F32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void asm_yukawa_far_kernel(YukParams P, W8 wt,
                                                                                                   WLow wl) {
    if (yuk_tile_near(blockIdx.y, blockIdx.x, P.n)) return;
    __shared__ double blk[(YT + 1) * (YT + 1)][4];
    __shared__ double ytab[YK_ALL_DOUBLES];
    yuk_load_table(P, ytab);
    __syncthreads();
    const int n = P.n;
    const int i0 = blockIdx.y * YT, j0 = blockIdx.x * YT;
    const int t = threadIdx.x;
    const int p = (i0 - 1 + t / (YT + 1) + n) % n, q = (j0 - 1 + t % (YT + 1) + n) % n;
    const int d = (q - p + n) % n;
    double B[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    // a self or adjacent pair can sit only in a slot no entry of this tile uses
    if (!(d <= 1 || d == n - 1)) yuk_far_block<F32>(P, ytab, wt, wl, p, q, B);
    blk[t][0] = B[0][0];
    blk[t][1] = B[0][1];
    blk[t][2] = B[1][0];
    blk[t][3] = B[1][1];
    __syncthreads();
    yuk_tile_store(P, blk, i0, j0);
}

// The tiles listed in `tiles` (those with a self or adjacent pair): near pairs by
// the singular quadrature, the rest like the far kernel.
__global__ __launch_bounds__(256) void asm_yukawa_near_kernel(YukParams P, W8 wt, WLow wl,
                                                              const int2* __restrict__ tiles) {
    __shared__ double blk[(YT + 1) * (YT + 1)][4];
    __shared__ double ytab[YK_ALL_DOUBLES];
    yuk_load_table(P, ytab);
    __syncthreads();
    const int n = P.n;
    const int2 tb = tiles[blockIdx.x];
    const int i0 = tb.x * YT, j0 = tb.y * YT;
    const int t = threadIdx.x;
    const int p = (i0 - 1 + t / (YT + 1) + n) % n, q = (j0 - 1 + t % (YT + 1) + n) % n;
    const int d = (q - p + n) % n;
    double B[2][2];
    if (d <= 1 || d == n - 1) {
        const int s = d == 0 ? 1 : (d == 1 ? 2 : 0);
        double2 So[2][2], Do[2][2];
        near_pair_blocks<false, true>(P.gx + 8 * p, P.gy + 8 * p, P.gx + 8 * q, P.gy + 8 * q, P.h[p], P.h[q],
                                      P.nx[p], P.ny[p], P.nx[q], P.ny[q], s, P.kappa, ytab, P.gl32, wt, So, Do);
#pragma unroll
        for (int al = 0; al < 2; ++al)
#pragma unroll
            for (int be = 0; be < 2; ++be) B[al][be] = So[al][be].x;
    } else {
        yuk_far_block<false>(P, ytab, wt, wl, p, q, B);
    }
    blk[t][0] = B[0][0];
    blk[t][1] = B[0][1];
    blk[t][2] = B[1][0];
    blk[t][3] = B[1][1];
    __syncthreads();
    yuk_tile_store(P, blk, i0, j0);
}

// Averages the entries (i, j) and (j, i) on the band |i - j| <= 2 (cyclic), like S.
__global__ void sym_band_kernel(double2* __restrict__ M, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * n) return;
    const int i = t / 3, d = t - 3 * (t / 3);
    if (d == 0) return;
    const int j = (i + d) % n;
    const int64_t ij = (int64_t)i * n + j, ji = (int64_t)j * n + i;
    const double2 a = M[ij], b = M[ji];
    const double2 m = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y + b.y));
    M[ij] = m;
    M[ji] = m;
}

void launch_assemble_yukawa(Op& op, double kappa, double2* Sy) {
    Ctx& c = *op.ctx;
    const int n = (int)op.n;
    W8 wt;
    WLow wlow;
    far_rules(op, wt, wlow);
    YukParams yp;
    yp.gx = op.gx; yp.gy = op.gy; yp.nodes = op.nodes; yp.h = op.h; yp.nx = op.nx; yp.ny = op.ny;
    yp.ytab = c.yk_tab; yp.ytab32 = c.yk_tab32; yp.gl32 = c.gl32; yp.Sy = Sy; yp.kappa = kappa; yp.n = n;
    const int nt = (n + YT - 1) / YT;
    FDS_REQUIRE(nt <= 65535, FDS_ERR_NOTIMPL, "Yukawa operator limited to n <= 983025");
    // Tiles with a self or adjacent pair lie within two tile rows of the diagonal or
    // in the wrap-around corners; the predicate decides among these candidates.
    std::vector<int2> near;
    for (int bi = 0; bi < nt; ++bi) {
        int cand[9] = {bi - 2, bi - 1, bi, bi + 1, bi + 2, 0, 1, nt - 2, nt - 1};
        for (int& v : cand) v = ((v % nt) + nt) % nt;
        std::sort(cand, cand + 9);
        const int nc = (int)(std::unique(cand, cand + 9) - cand);
        for (int k = 0; k < nc; ++k)
            if (yuk_tile_near(bi, cand[k], n)) near.push_back(make_int2(bi, cand[k]));
    }
    int2* dnear = static_cast<int2*>(c.dmalloc(sizeof(int2) * near.size()));
    FDS_HIP_TRY(hipMemcpyAsync(dnear, near.data(), sizeof(int2) * near.size(), hipMemcpyHostToDevice, c.stream));
    {
        KScope _ks(c, "asm_yukawa");
        if (op.prec == FDS_FP32)
            hipLaunchKernelGGL(asm_yukawa_far_kernel<true>, dim3(nt, nt), dim3(256), 0, c.stream, yp, wt, wlow);
        else
            hipLaunchKernelGGL(asm_yukawa_far_kernel<false>, dim3(nt, nt), dim3(256), 0, c.stream, yp, wt, wlow);
        hipLaunchKernelGGL(asm_yukawa_near_kernel, dim3((unsigned)near.size()), dim3(256), 0, c.stream, yp, wt,
                           wlow, dnear);
        hipLaunchKernelGGL(sym_band_kernel, dim3((3 * n + 255) / 256), dim3(256), 0, c.stream, Sy, n);
    }
    FDS_HIP_TRY(hipGetLastError());
    c.dfree(dnear);
}

}  // namespace fds
