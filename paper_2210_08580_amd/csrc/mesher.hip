// Equal-chord (homogeneous) meshes of closed curves, on the host.
//
// Paper, Laplacian Filters, Two-Dimensional Case: the filter is defined through
// the SVD of the orthonormalised Laplacian G^{-1/2} L G^{-1/2}; on a
// homogeneously discretised curve (all panels of one length) G and L are
// circulant, the DFT diagonalises both, and the filter needs no eigensolver.
// This file produces such meshes: n points of the curve whose n chords (cyclic)
// are equal, the points in parameter order starting at t = 0.
//
// The curve is a trigonometric polynomial in Cartesian form,
//   x(t) = sum_{m=0}^{d} ax[m] cos(m t) + bx[m] sin(m t),  y(t) likewise,
// evaluated with the rotation recurrence e^{i(m+1)t} = e^{imt} e^{it}.
//
// Walk: each next parameter is the first one after the current at chord distance
// c (bracketed by steps of c/(4 max|r'|), then Newton's method on
// |r(t) - r(t_i)|^2 - c^2 kept inside the bracket). Closure: c is the root of
// F(c) = |r(t_0) - r(t_{n-1}(c))| - c, which decreases with c (a walk that passes
// t = 2 pi before its last point counts as F = -c); F changes sign between
// L/(2n) and about L/n with L the curve length, and the Illinois variant of
// regula falsi finds the root. The closing chord absorbs the rounding of the
// n - 1 others, so the chords agree to about n times the rounding of c.
#include <cmath>
#include <vector>

#include "fds_internal.h"

namespace fds {

namespace {

struct TrigCurve {
    const double *ax, *bx, *ay, *by;
    int d;
    // position (x, y) and derivative (dx, dy) at t = th + delta, given ch = cos th,
    // sh = sin th: the rotation e^{it} = e^{i th} e^{i delta} keeps the angle exact
    // to the rounding of its sine and cosine even where t itself is a rounded sum
    void eval(double ch, double sh, double delta, double& x, double& y, double& dx, double& dy) const {
        const double cd = std::cos(delta), sd = std::sin(delta);
        const double c1 = ch * cd - sh * sd, s1 = sh * cd + ch * sd;
        double c = 1.0, s = 0.0;
        x = ax[0];
        y = ay[0];
        dx = 0.0;
        dy = 0.0;
        for (int m = 1; m <= d; ++m) {
            const double cn = c * c1 - s * s1, sn = s * c1 + c * s1;
            c = cn;
            s = sn;
            x += ax[m] * c + bx[m] * s;
            y += ay[m] * c + by[m] * s;
            dx += m * (bx[m] * c - ax[m] * s);
            dy += m * (by[m] * c - ay[m] * s);
        }
    }
    void point(double th, double tl, double& x, double& y) const {
        double dx, dy;
        eval(std::cos(th), std::sin(th), tl, x, y, dx, dy);
    }
};

constexpr double kTwoPi = 6.283185307179586476925;

// Parameters are kept as unevaluated sums th + tl (|tl| <= ulp(th)/2), so that the
// n points sit on the curve at their exact parameters, not at rounded ones.
struct Param {
    double th, tl;
};

Param add(Param p, double s) {   // p + s, renormalised (Knuth's two-sum)
    const double a = p.th, b = p.tl + s;
    const double sum = a + b, bb = sum - a;
    return Param{sum, (a - (sum - bb)) + (b - bb)};
}

// Smallest offset s in (0, smax] with |r(t0 + s) - p0| = c; false if there is none.
bool next_offset(const TrigCurve& cv, Param t0, double px, double py, double c, double ds, double smax,
                 double& s1) {
    const double ch = std::cos(t0.th), sh = std::sin(t0.th);
    auto g = [&](double s, double* dg) {
        double x, y, dx, dy;
        cv.eval(ch, sh, t0.tl + s, x, y, dx, dy);
        const double ex = x - px, ey = y - py;
        if (dg) *dg = 2.0 * (ex * dx + ey * dy);
        return ex * ex + ey * ey - c * c;
    };
    double a = 0.0, b = ds, gb = g(b, nullptr);
    while (gb < 0.0) {
        a = b;
        b += ds;
        if (a > smax) return false;
        gb = g(b, nullptr);
    }
    // Newton inside [a, b] (g(a) < 0 <= g(b)), bisection when a step leaves it
    double s = 0.5 * (a + b);
    for (int it = 0; it < 100; ++it) {
        double dg;
        const double gv = g(s, &dg);
        if (gv < 0.0) a = s; else b = s;
        double sn = dg > 0.0 ? s - gv / dg : 0.5 * (a + b);
        if (!(sn > a && sn < b)) sn = 0.5 * (a + b);
        if (sn == s || b - a <= 2.0 * std::ldexp(1.0, std::ilogb(b) - 52)) {
            s = sn;
            break;
        }
        s = sn;
    }
    s1 = s;
    return true;
}

}  // namespace

void equal_chord_mesh(int d, const double* ax, const double* bx, const double* ay, const double* by, int64_t n,
                      double* nodes, double* chord) {
    FDS_REQUIRE(d >= 1 && d <= 4096, FDS_ERR_ARG, "degree must be in 1..4096");
    FDS_REQUIRE(ax && bx && ay && by && nodes, FDS_ERR_ARG, "NULL argument");
    FDS_REQUIRE(n >= 4 && n <= (int64_t)1 << 24, FDS_ERR_ARG, "n must be in 4..2^24");
    for (int m = 0; m <= d; ++m)
        FDS_REQUIRE(std::isfinite(ax[m]) && std::isfinite(bx[m]) && std::isfinite(ay[m]) && std::isfinite(by[m]),
                    FDS_ERR_ARG, "non-finite curve coefficient");
    const TrigCurve cv{ax, bx, ay, by, d};
    // length and speed bound from a fine polyline
    const int K = std::max(4096, 64 * d);
    double len = 0.0, vmax = 0.0, px, py;
    cv.point(0.0, 0.0, px, py);
    for (int k = 1; k <= K; ++k) {
        double x, y, dx, dy;
        cv.eval(std::cos(kTwoPi * k / K), std::sin(kTwoPi * k / K), 0.0, x, y, dx, dy);
        len += std::hypot(x - px, y - py);
        vmax = std::max(vmax, std::hypot(dx, dy));
        px = x;
        py = y;
    }
    FDS_REQUIRE(len > 0.0 && vmax > 0.0, FDS_ERR_ARG, "degenerate curve");
    vmax *= 1.25;   // the sampled maximum of |r'| can miss the peak slightly
    double x0, y0;
    cv.point(0.0, 0.0, x0, y0);
    std::vector<Param> t(n);
    // F(c) and, on success, the parameters of the walk
    auto defect = [&](double c) {
        t[0] = Param{0.0, 0.0};
        const double ds = 0.25 * c / vmax;
        double x = x0, y = y0;
        for (int64_t i = 1; i < n; ++i) {
            double s;
            if (!next_offset(cv, t[i - 1], x, y, c, ds, kTwoPi - t[i - 1].th, s)) return -c;
            t[i] = add(t[i - 1], s);
            if (t[i].th >= kTwoPi) return -c;
            cv.point(t[i].th, t[i].tl, x, y);
        }
        return std::hypot(x0 - x, y0 - y) - c;
    };
    // the sampled length is a polyline's, slightly below the curve's: widen the
    // upper end until the walk closes short of it
    double lo = 0.5 * len / n, hi = len / n;
    double flo = defect(lo), fhi = defect(hi);
    for (int k = 0; k < 64 && fhi > 0.0; ++k) {
        lo = hi;
        flo = fhi;
        hi *= 1.0 + 1.0 / 1024;
        fhi = defect(hi);
    }
    FDS_REQUIRE(flo > 0.0 && fhi <= 0.0, FDS_ERR_ARG, "no equal-chord mesh found (is the curve simple?)");
    double c = hi, fc = fhi;
    int side = 0;
    for (int it = 0; it < 200; ++it) {
        c = (lo * fhi - hi * flo) / (fhi - flo);
        if (!(c > lo && c < hi)) c = 0.5 * (lo + hi);
        fc = defect(c);
        if (fc == 0.0 || hi - lo <= 4.0 * std::ldexp(1.0, std::ilogb(hi) - 52) || std::fabs(fc) <= 1e-16 * c) break;
        if (fc > 0.0) {
            lo = c;
            flo = fc;
            if (side == 1) fhi *= 0.5;   // Illinois: halve the stale end's value
            side = 1;
        } else {
            hi = c;
            fhi = fc;
            if (side == -1) flo *= 0.5;
            side = -1;
        }
    }
    fc = defect(c);
    FDS_REQUIRE(fc > -c, FDS_ERR_ARG, "equal-chord walk did not close");
    for (int64_t i = 0; i < n; ++i) cv.point(t[i].th, t[i].tl, nodes[2 * i], nodes[2 * i + 1]);
    if (chord) *chord = c;
}

}  // namespace fds
