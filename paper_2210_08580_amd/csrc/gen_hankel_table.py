"""Generate hankel_table.inc: coefficients of the device Bessel evaluator.

Three regions of the real argument x > 0 (J0, Y0, J1, Y1):
  x < XS   ascending series (Abramowitz & Stegun 9.1.10, 9.1.11, 9.1.13):
             J0 = sum (-1)^m q^m/(m!)^2,                   q = x^2/4
             Y0 = (2/pi)(log(x/2) + gamma) J0 + (2/pi) sum_{m>=1} (-1)^{m+1} H_m q^m/(m!)^2
             J1 = (x/2) sum (-1)^m q^m/(m!(m+1)!)
             Y1 = -2/(pi x) + (2/pi) log(x/2) J1
                  - (x/(2 pi)) sum (-1)^m (psi(m+1) + psi(m+2)) q^m/(m!(m+1)!)
  XS <= x < XA  piecewise polynomials on unit intervals [c, c+1): each function is
           interpolated at Chebyshev points (50-digit mpmath values) and stored in
           the monomial basis of t = x - (c + 1/2); evaluated by Horner.
  x >= XA  Hankel's asymptotic expansion (A&S 9.2.5-9.2.10):
             H_nu^(1)(x) = sqrt(2/(pi x)) (P + i Q) exp(i (x - (nu/2 + 1/4) pi)),
             P = sum_k (-1)^k a_2k(nu) x^-2k,  Q = sum_k (-1)^k a_{2k+1}(nu) x^-(2k+1),
             a_k(nu) = prod_{j=1..k} (4 nu^2 - (2j-1)^2) / (k! 8^k).
The script checks a float64 emulation of the device formulas against mpmath and
refuses to write the table unless every region is within 4e-16 max(|f|, 1).

The single-precision asymptotic expansion (HK32_ASY_*, shorter than the FP64 one)
serves the far-field FP32 set below beyond its table, checked in a float32
emulation (argument x formed in float64, the phase reduced in float64, everything
after in float32) against 4e-7 max(|f|, 1).

A third set (YK_*) evaluates K0, the modified Bessel function of the second kind
of the Yukawa kernel (1/2pi) K0(kappa R) (Helmholtz at the imaginary wavenumber
i kappa), in FP64:
  x < YK_XS   ascending series (A&S 9.6.12, 9.6.13):
                I0 = sum q^m/(m!)^2,  K0 = -(log(x/2) + gamma) I0 + sum_{m>=1} H_m q^m/(m!)^2
  YK_XS <= x < YK_XA  K0(x) itself (no exponential scaling, so the device needs no exp
                      there) interpolated on unit intervals like the tables above
  x >= YK_XA  K0 = sqrt(pi/(2x)) exp(-x) sum_k a_k(0) x^-k  (A&S 9.7.2)
checked against mpmath in relative error (4e-16 max(|f|, 1) in the series range,
where the log term dominates, 6e-16 relative elsewhere).

Two further sets (HF_*, HF32_*) serve the far-field assembly kernels, one table
lookup for every argument below HF_XF (FP64) or HF32_XF (FP32): quarter-unit
intervals [c/4, (c+1)/4), interpolated like the tables above in t = x - (c + 1/2)/4
(degree HF_DEG or HF32_DEG). On the first eight intervals (x < 2) the table holds
the parts of Y0 and Y1 that stay regular at x = 0,
  Y0r = Y0 - (2/pi) J0 log x,   Y1r = Y1 - (2/pi) J1 log x + 2/(pi x)
(A&S 9.1.11 and 9.1.13 with log(x/2) = log x - log 2: both are power series), and
the evaluator adds the logarithmic and 1/x terms back; above it holds Y0, Y1
themselves. Beyond HF_XF the asymptotic expansions above apply. Checked like the
other sets (FP64: 4e-16 max(|f|, 1); FP32 emulation: 4e-7 max(|f|, 1)).

Run:  python gen_hankel_table.py   (writes hankel_table.inc next to this file)
"""
from __future__ import annotations

import os
import sys

import mpmath as mp
import numpy as np

mp.mp.dps = 50
XS, XA = 2, 25
DEG = 15
NSER = 16
HERE = os.path.dirname(os.path.abspath(__file__))


def series_coeffs():
    cj0, cy0, cj1, cy1 = [], [], [], []
    H = mp.mpf(0)
    for m in range(NSER):
        f2 = mp.factorial(m) ** 2
        f11 = mp.factorial(m) * mp.factorial(m + 1)
        if m >= 1:
            H += mp.mpf(1) / m
        cj0.append((-1) ** m / f2)
        cy0.append(((-1) ** (m + 1)) * H / f2 if m >= 1 else mp.mpf(0))
        cj1.append((-1) ** m / f11)
        cy1.append((-1) ** m * (mp.digamma(m + 1) + mp.digamma(m + 2)) / f11)
    return cj0, cy0, cj1, cy1


def asym_coeffs(nu, nterms):
    a = [mp.mpf(1)]
    for k in range(1, 2 * nterms + 2):
        a.append(a[-1] * (4 * nu * nu - (2 * k - 1) ** 2) / (k * 8))
    P = [(-1) ** k * a[2 * k] for k in range(nterms)]
    Q = [(-1) ** k * a[2 * k + 1] for k in range(nterms)]
    return P, Q, a


def asym_terms_needed(x0, tol=2e-18):
    _, _, a = asym_coeffs(1, 40)
    _, _, a0 = asym_coeffs(0, 40)
    for n in range(2, 40):
        # first neglected terms of P and Q bound the remainders
        nxt = max(abs(a[2 * n]), abs(a[2 * n + 1]) / x0, abs(a0[2 * n]), abs(a0[2 * n + 1]) / x0)
        if nxt / mp.mpf(x0) ** (2 * n) < tol:
            return n
    raise RuntimeError("asymptotic region starts too low")


def fns():
    return [lambda x: mp.besselj(0, x), lambda x: mp.bessely(0, x),
            lambda x: mp.besselj(1, x), lambda x: mp.bessely(1, x)]


def cheb_monomial(f, c, deg=DEG):
    """Monomial coefficients in t = x - (c + 1/2) of the degree-`deg` Chebyshev
    interpolant of f on [c, c+1]."""
    n = deg + 1
    u = [mp.cos(mp.pi * (j + mp.mpf(1) / 2) / n) for j in range(n)]
    vals = [f(c + mp.mpf(1) / 2 + uj / 2) for uj in u]
    # Chebyshev coefficients in u
    ch = []
    for k in range(n):
        s = mp.fsum(vals[j] * mp.cos(k * mp.pi * (j + mp.mpf(1) / 2) / n) for j in range(n))
        ch.append(s * (1 if k == 0 else 2) / n)
    # T_k(u) in monomials of u, then u = 2 t
    mono = [mp.mpf(0)] * n
    Tkm1, Tk = [mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]
    polys = [Tkm1, Tk]
    for k in range(2, n):
        nxt = [mp.mpf(0)] * (k + 1)
        for i, cc in enumerate(polys[-1]):
            nxt[i + 1] += 2 * cc
        for i, cc in enumerate(polys[-2]):
            nxt[i] -= cc
        polys.append(nxt)
    for k in range(n):
        for i, cc in enumerate(polys[k]):
            mono[i] += ch[k] * cc
    return [mono[i] * 2 ** i for i in range(n)]


# ---------------------------------------------------------------- float64 emulation
def horner(c, t):
    acc = np.float64(c[-1])
    for v in c[-2::-1]:
        acc = acc * t + np.float64(v)
    return acc


def emulate(x, tabs, ser, asy):
    x = np.float64(x)
    if x < XS:
        q = x * x / 4
        cj0, cy0, cj1, cy1 = ser
        j0 = horner(cj0, q)
        j1 = 0.5 * x * horner(cj1, q)
        l = np.log(0.5 * x)
        y0 = (2 / np.pi) * ((l + np.euler_gamma) * j0 + q * horner(cy0[1:], q))
        y1 = -2 / (np.pi * x) + (2 / np.pi) * l * j1 - (x / (2 * np.pi)) * horner(cy1, q)
        return j0, y0, j1, y1
    if x < XA:
        c = int(np.floor(x))
        t = x - (c + 0.5)
        return tuple(horner(tabs[f][c - XS], t) for f in range(4))
    P0, Q0, P1, Q1 = asy
    w = 1.0 / (x * x)
    p0, q0 = horner(P0, w), horner(Q0, w) / x
    p1, q1 = horner(P1, w), horner(Q1, w) / x
    amp = np.sqrt(2.0 / (np.pi * x))
    s, co = np.sin(x), np.cos(x)
    r = np.sqrt(0.5)
    c0, s0 = r * (co + s), r * (s - co)          # cos, sin of x - pi/4
    c1, s1 = r * (s - co), -r * (s + co)         # cos, sin of x - 3 pi/4
    return (amp * (p0 * c0 - q0 * s0), amp * (p0 * s0 + q0 * c0),
            amp * (p1 * c1 - q1 * s1), amp * (p1 * s1 + q1 * c1))


def emulate32(x, tabs, ser, asy):
    f4 = np.float32
    x = np.float64(x)

    def h32(c, t):
        acc = f4(c[-1])
        for v in c[-2::-1]:
            acc = f4(acc * t + f4(v))
        return acc
    if x < XS:
        q = f4(x * x / 4)
        xf = f4(x)
        cj0, cy0, cj1, cy1 = ser
        j0 = h32(cj0, q)
        j1 = f4(f4(0.5) * xf * h32(cj1, q))
        l = f4(np.log(f4(0.5) * xf))
        tp = f4(2 / np.pi)
        y0 = f4(tp * f4(f4(l + f4(np.euler_gamma)) * j0 + q * h32(cy0[1:], q)))
        y1 = f4(f4(-tp / xf) + tp * l * j1 - f4(xf * f4(0.5 / np.pi)) * h32(cy1, q))
        return j0, y0, j1, y1
    if x < XA:
        c = int(np.floor(x))
        t = f4(x - (c + 0.5))
        return tuple(h32(tabs[f][c - XS], t) for f in range(4))
    P0, Q0, P1, Q1 = asy
    xf = f4(x)
    w = f4(f4(1) / (xf * xf))
    rx = f4(f4(1) / xf)
    p0, q0 = h32(P0, w), f4(h32(Q0, w) * rx)
    p1, q1 = h32(P1, w), f4(h32(Q1, w) * rx)
    amp = f4(np.sqrt(f4(2 / np.pi) * rx))
    xr = f4(x - 2 * np.pi * np.rint(x / (2 * np.pi)))     # phase reduced in float64
    sn, co = np.sin(xr, dtype=np.float32), np.cos(xr, dtype=np.float32)
    r = f4(np.sqrt(0.5))
    c0, s0 = r * (co + sn), r * (sn - co)
    c1, s1 = r * (sn - co), -r * (sn + co)
    return (amp * (p0 * c0 - q0 * s0), amp * (p0 * s0 + q0 * c0),
            amp * (p1 * c1 - q1 * s1), amp * (p1 * s1 + q1 * c1))


def asym32():
    """Coefficients of the single-precision asymptotic expansion (x >= HF32_XF)."""
    nas = asym_terms_needed(XA, tol=2e-9)
    asy = [[float(v) for v in s] for s in (*asym_coeffs(0, nas)[:2], *asym_coeffs(1, nas)[:2])]
    return asy, nas


YK_XS = 2
YK_XA = 40
YK_NSER = 16


def yk_sets():
    """Series, table and asymptotic coefficients of K0 (FP64)."""
    ci0, ck0 = [], []
    H = mp.mpf(0)
    for m in range(YK_NSER):
        f2 = mp.factorial(m) ** 2
        if m >= 1:
            H += mp.mpf(1) / m
        ci0.append(1 / f2)
        ck0.append(H / f2)
    f = lambda x: mp.besselk(0, x)
    tab = [cheb_monomial(f, c) for c in range(YK_XS, YK_XA)]
    # asymptotic: first neglected term below 1e-18 at x = YK_XA
    a = [mp.mpf(1)]
    for k in range(1, 60):
        a.append(a[-1] * (0 - (2 * k - 1) ** 2) / (k * 8))
    nas = next(k for k in range(2, 60) if abs(a[k]) / mp.mpf(YK_XA) ** k < 1e-18)
    return [float(v) for v in ci0], [float(v) for v in ck0], [[float(v) for v in cc] for cc in tab], \
        [float(v) for v in a[:nas]]


def yk_emulate(x, ci0, ck0, tab, asy):
    x = np.float64(x)
    if x < YK_XS:
        q = x * x / 4
        i0 = horner(ci0, q)
        return -(np.log(0.5 * x) + np.euler_gamma) * i0 + q * horner(ck0[1:], q)
    if x < YK_XA:
        c = int(np.floor(x))
        return horner(tab[c - YK_XS], x - (c + 0.5))
    return np.sqrt(np.pi / (2.0 * x)) * np.exp(-x) * horner(asy, 1.0 / x)


def yk_check(sets):
    xs = np.concatenate([np.geomspace(1e-6, YK_XS, 300, endpoint=False),
                         np.linspace(YK_XS, YK_XA, 3800, endpoint=False),
                         np.linspace(YK_XA, 200, 600)])
    worst = 0.0
    for x in xs:
        ref = float(mp.besselk(0, mp.mpf(float(x))))
        got = float(yk_emulate(x, *sets))
        err = abs(got - ref) / (max(abs(ref), 1.0) if x < YK_XS else abs(ref))
        worst = max(worst, err / (4e-16 if x < YK_XS else 6e-16))
    print(f"K0 set: asymptotic terms {len(sets[3])}; worst error / tolerance {worst:.3f}")
    if worst > 1.0:
        sys.exit("K0 table accuracy check failed")


YK32_DEG = 8


def yk32_table():
    """K0 on the unit intervals of [YK_XS, YK_XA) for single-precision evaluation
    (t = x - c - 1/2 and the Horner sums in float32), checked against mpmath."""
    f = lambda x: mp.besselk(0, x)
    tab = [[float(v) for v in cheb_monomial(f, c, YK32_DEG)] for c in range(YK_XS, YK_XA)]
    f4 = np.float32
    worst = 0.0
    for x in np.linspace(YK_XS, YK_XA, 3800, endpoint=False):
        c = int(np.floor(x))
        t = f4(f4(x) - f4(c + 0.5))
        acc = f4(tab[c - YK_XS][-1])
        for v in tab[c - YK_XS][-2::-1]:
            acc = f4(acc * t + f4(v))
        ref = float(mp.besselk(0, mp.mpf(float(f4(x)))))
        worst = max(worst, abs(float(acc) - ref) / ref)
    print(f"K0 float32 table: worst relative error {worst:.3e}")
    if worst > 6e-7:
        sys.exit("float32 K0 table accuracy check failed")
    return tab


HF_XF = 32
HF_DEG = 9
HF32_XF = 64
HF32_DEG = 5
HF_SMALL = 8      # quarter intervals below x = 2 hold the regular parts


def hf_fns():
    """J0, Y0 (or its regular part), J1, Y1 (or its regular part) on the quarter
    intervals; `small` selects the regular parts."""
    tp = 2 / mp.pi

    def y0r(x):
        return mp.bessely(0, x) - tp * mp.besselj(0, x) * mp.log(x)

    def y1r(x):
        return mp.bessely(1, x) - tp * mp.besselj(1, x) * mp.log(x) + tp / x
    return ([lambda x: mp.besselj(0, x), y0r, lambda x: mp.besselj(1, x), y1r],
            [lambda x: mp.besselj(0, x), lambda x: mp.bessely(0, x), lambda x: mp.besselj(1, x),
             lambda x: mp.bessely(1, x)])


def cheb_monomial_q(f, c, deg):
    """Degree-`deg` Chebyshev interpolant of f on the quarter interval [c/4, (c+1)/4]
    in monomials of t = x - (c + 1/2)/4 (cheb_monomial on the unit interval of the
    scaled function, rescaled)."""
    g = lambda u: f(u / 4)
    mono = cheb_monomial(g, c, deg)          # in s = 4x - (c + 1/2) = 4 t
    return [m * 4 ** i for i, m in enumerate(mono)]


def hf_table(xf, deg):
    small, plain = hf_fns()
    return [[[float(v) for v in cheb_monomial_q((small if c < HF_SMALL else plain)[f], c, deg)]
             for c in range(4 * xf)] for f in range(4)]


def hf_emulate(x, tab, asy, xf):
    x = np.float64(x)
    if x >= xf:
        return emulate(x, None, None, asy)
    c = int(np.floor(4 * x))
    t = x - (c + 0.5) / 4
    j0, y0, j1, y1 = (horner(tab[f][c], t) for f in range(4))
    if c < HF_SMALL:
        l = np.log(x)
        tp = 2 / np.pi
        y0 = y0 + tp * j0 * l
        y1 = y1 + tp * j1 * l - tp / x
    return j0, y0, j1, y1


def hf32_emulate(x, tab, asy32, xf):
    f4 = np.float32
    x = np.float64(x)
    if x >= xf:
        return emulate32(x, None, None, asy32)
    c = int(np.floor(4 * x))
    t = f4(x - (c + 0.5) / 4)

    def h32(cc):
        acc = f4(cc[-1])
        for v in cc[-2::-1]:
            acc = f4(acc * t + f4(v))
        return acc
    j0, y0, j1, y1 = (h32(tab[f][c]) for f in range(4))
    if c < HF_SMALL:
        xf4 = f4(x)
        l = f4(np.log(xf4))
        tp = f4(2 / np.pi)
        y0 = f4(y0 + f4(tp * j0) * l)
        y1 = f4(f4(y1 + f4(tp * j1) * l) - f4(tp * f4(f4(1) / xf4)))
    return j0, y0, j1, y1


def hf_check(tab, asy, xf, emu, tol, label):
    F = fns()
    xs = np.concatenate([np.geomspace(1e-6, 2.0, 400, endpoint=False),
                         np.linspace(2.0, xf, 40 * xf, endpoint=False),
                         np.linspace(xf, 3 * xf, 200)])
    worst = 0.0
    for x in xs:
        got = emu(x, tab, asy, xf)
        for f in range(4):
            ref = float(F[f](mp.mpf(float(x))))
            worst = max(worst, abs(float(got[f]) - ref) / max(1.0, abs(ref)))
    print(f"{label}: worst scaled error {worst:.3e}")
    if worst > tol:
        sys.exit(f"{label} accuracy check failed")


def main():
    ser = series_coeffs()
    nas = asym_terms_needed(XA)
    P0, Q0, _ = asym_coeffs(0, nas)
    P1, Q1, _ = asym_coeffs(1, nas)
    F = fns()
    tabs = [[cheb_monomial(F[f], c) for c in range(XS, XA)] for f in range(4)]
    serd = [[float(v) for v in s] for s in ser]
    asyd = [[float(v) for v in s] for s in (P0, Q0, P1, Q1)]
    tabd = [[[float(v) for v in cc] for cc in tf] for tf in tabs]
    # self-check
    xs = np.concatenate([np.geomspace(1e-6, XS, 300, endpoint=False),
                         np.linspace(XS, XA, 2300, endpoint=False),
                         np.linspace(XA, 120, 400)])
    worst = 0.0
    for x in xs:
        got = emulate(x, tabd, serd, asyd)
        for f in range(4):
            ref = F[f](mp.mpf(float(x)))
            err = abs(float(got[f]) - float(ref)) / max(1.0, abs(float(ref)))
            worst = max(worst, err)
    print(f"asymptotic terms: {nas}; worst scaled error {worst:.3e}")
    if worst > 4e-16:
        sys.exit("table accuracy check failed")
    asy32, nas32 = asym32()
    yk = yk_sets()
    yk_check(yk)
    yk32 = yk32_table()
    hf = hf_table(HF_XF, HF_DEG)
    hf_check(hf, asyd, HF_XF, hf_emulate, 4e-16, f"far FP64 set (quarter intervals to {HF_XF}, degree {HF_DEG})")
    hf32 = hf_table(HF32_XF, HF32_DEG)
    hf_check(hf32, asy32, HF32_XF, hf32_emulate, 4e-7,
             f"far FP32 set (quarter intervals to {HF32_XF}, degree {HF32_DEG})")
    out = os.path.join(HERE, "hankel_table.inc")
    with open(out, "w") as fh:
        fh.write("// Generated by gen_hankel_table.py; do not edit.\n")
        fh.write(f"#define HK_XS {XS}\n#define HK_XA {XA}\n#define HK_DEG {DEG}\n")
        fh.write(f"#define HK_NSER {NSER}\n#define HK_NASY {nas}\n")
        names = ("HK_SER_J0", "HK_SER_Y0", "HK_SER_J1", "HK_SER_Y1")
        for nm, s in zip(names, serd):
            fh.write(f"static constexpr double {nm}[{len(s)}] = {{" +
                     ", ".join(repr(v) for v in s) + "};\n")
        for nm, s in zip(("HK_ASY_P0", "HK_ASY_Q0", "HK_ASY_P1", "HK_ASY_Q1"), asyd):
            fh.write(f"static constexpr double {nm}[{len(s)}] = {{" +
                     ", ".join(repr(v) for v in s) + "};\n")
        nint = XA - XS
        fh.write(f"// [interval c-{XS}][coefficient of t^m][function J0,Y0,J1,Y1]\n")
        fh.write(f"static constexpr double HK_TAB[{nint}][{DEG + 1}][4] = {{\n")
        for c in range(nint):
            fh.write(" {\n")
            for m in range(DEG + 1):
                fh.write("  {" + ", ".join(repr(tabd[f][c][m]) for f in range(4)) + "},\n")
            fh.write(" },\n")
        fh.write("};\n")
        fh.write(f"#define HK32_NASY {nas32}\n")
        for nm, v in zip(("HK32_ASY_P0", "HK32_ASY_Q0", "HK32_ASY_P1", "HK32_ASY_Q1"), asy32):
            fh.write(f"static constexpr float {nm}[{len(v)}] = {{" + ", ".join(repr(x) + "f" for x in
                                                                            np.float32(v).tolist()) + "};\n")
        ci0, ck0, ytab, yasy = yk
        fh.write(f"#define YK_XS {YK_XS}\n#define YK_XA {YK_XA}\n#define YK_NSER {YK_NSER}\n#define YK_NASY {len(yasy)}\n")
        fh.write("static constexpr double YK_SER_I0[%d] = {" % len(ci0) + ", ".join(repr(v) for v in ci0) + "};\n")
        fh.write("static constexpr double YK_SER_K0[%d] = {" % len(ck0) + ", ".join(repr(v) for v in ck0) + "};\n")
        fh.write("static constexpr double YK_ASY[%d] = {" % len(yasy) + ", ".join(repr(v) for v in yasy) + "};\n")
        fh.write(f"// [interval c-{YK_XS}][coefficient of t^m] of K0(x)\n")
        fh.write(f"static constexpr double YK_TAB[{YK_XA - YK_XS}][{DEG + 1}] = {{\n")
        for cc in ytab:
            fh.write("  {" + ", ".join(repr(v) for v in cc) + "},\n")
        fh.write("};\n")
        fh.write(f"#define HF_XF {HF_XF}\n#define HF_DEG {HF_DEG}\n#define HF32_XF {HF32_XF}\n"
                 f"#define HF32_DEG {HF32_DEG}\n#define HF_SMALL {HF_SMALL}\n")
        fh.write("// [quarter interval c][coefficient of t^m][J0, Y0 (regular part for c < HF_SMALL), J1, Y1 (same)]\n")
        fh.write(f"static constexpr double HF_TAB[{4 * HF_XF}][{HF_DEG + 1}][4] = {{\n")
        for c in range(4 * HF_XF):
            fh.write(" {" + ", ".join("{" + ", ".join(repr(hf[f][c][m]) for f in range(4)) + "}"
                                      for m in range(HF_DEG + 1)) + "},\n")
        fh.write("};\n")
        fh.write(f"static constexpr float HF32_TAB[{4 * HF32_XF}][{HF32_DEG + 1}][4] = {{\n")
        for c in range(4 * HF32_XF):
            fh.write(" {" + ", ".join("{" + ", ".join(repr(float(np.float32(hf32[f][c][m]))) + "f" for f in range(4))
                                      + "}" for m in range(HF32_DEG + 1)) + "},\n")
        fh.write("};\n")
        fh.write(f"#define YK32_DEG {YK32_DEG}\n")
        fh.write(f"// the same intervals for float32 evaluation (t and the sums in float32)\n")
        fh.write(f"static constexpr float YK32_TAB[{YK_XA - YK_XS}][{YK32_DEG + 1}] = {{\n")
        for cc in yk32:
            fh.write("  {" + ", ".join(repr(float(np.float32(v))) + "f" for v in cc) + "},\n")
        fh.write("};\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
