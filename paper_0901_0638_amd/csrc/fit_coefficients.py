#!/usr/bin/env python3
"""Generate qm_coeffs.h: the rational approximations the GPU kernels evaluate.

Run from the repository root:  python paper_0901_0638_amd/csrc/fit_coefficients.py

These approximations are fitted here, the rest are the paper's constants:

  * Deep-tail piece of the exponential-coordinate normal quantile.  The
    paper's branchless FP64 rational Q(v) = v p13(v)/q13(v) (Section 7.2,
    Appendix B) is certified only for v <= 42 (u >= 2.875e-19); Section 4.3
    asks only for "reasonable" growth outside.  FP64 inputs reach v = 743.7
    (u = 4.9e-324), so the kernels switch, by a wave-wide vote, to
    Q(v) = s * P7(s)/Q7(s), s = sqrt(v), on 42 < v <= 750.
  * FP32 seed of the FP32+refine form: Q(v) = v * P4(v)/Q5(v) over the whole
    FP32 range v in [0, 103.3] (the paper's (5,6) of Section 6.1 stops at
    v = 25), accurate to ~1e-5 -- only a seed for the FP64 correction step.
  * Mills ratio M(x) = (1 - Phi(x))/phi(x) on [0, 14.5] as P6(x)/Q7(x), the
    only non-trivial part of the FP64 erfc used by the exponential -> normal
    correction step (erfc(x/sqrt2) = 2 phi(x) M(x)), whose x starts at 0;
    and on [1.6, 14.5] as P3(x)/Q4(x) (8.5e-9) for the quantile's outer
    correction, where |z| > 1.6449 and an error e in M moves the result by
    about e/z^2 relative.
  * Central piece of the FP64 quantile (the hybrid of Section 7.3 /
    Appendix C, with a log-free central variable): for |q| <= 0.45,
    q = u - 1/2, Phi^{-1}(u) = q P8(r)/Q8(r), r = 0.2025 - q^2.  All
    coefficients come out positive in r, so their FP64 rounding costs about
    an ulp.  Outside, the exponential-coordinate path above.
  * Central piece of the FP32+refine form, |q| <= 0.45: an FP32 seed
    q S2(r)/S3(r) (2.6e-6), then one FP64 Newton step against
    Phi(z) - u = erf(z/sqrt2)/2 - q with erf(z/sqrt2)/(2z) = E6(z^2) and
    1/phi(z) = G3(z^2), polynomials good to 9.3e-9 and 1.1e-3 on
    |z| <= 1.646.  The result then carries at most 2.7 x 9.3e-9 from E
    (the residual's error divided by phi(z), relative to z) and
    1.1e-3 x 2.6e-6 from G, before its rounding to FP32 (half an ulp,
    6e-8): within the form's 2e-7.
  * The FP64 logarithm of the change of variable v = -log(2 min(u,1-u)):
    log m = 2 atanh f = 2f + f s R6(s), f = (m-1)/(m+1), s = f^2, for the
    reduced argument m in [sqrt(1/2), sqrt(2)] (so s <= 0.0294).

Method: relative-error rational fits by linearised least squares (Loeb
iteration) followed by Lawson reweighting towards minimax, in mpmath at 40
digits on Chebyshev nodes; reference values come from mpmath's erfc/erfinv.
The coefficients are then rounded to FP64 and the error of the rounded
rational is measured exactly on a dense grid and written into the header.
"""
import os
import struct
import sys

import mpmath as mp

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "qm_coeffs.h")


def q_exp(v):
    """Q(v) = Phi^{-1}(1 - e^{-v}/2) (Section 6 formal solution), v >= 0."""
    v = mp.mpf(v)
    if v < mp.log(2):
        return mp.sqrt(2) * mp.erfinv(-mp.expm1(-v))
    f = lambda z: mp.log(mp.erfc(z / mp.sqrt(2)) / 2) + v + mp.log(2)
    return mp.findroot(f, mp.sqrt(2 * v), tol=mp.mpf(10) ** (-mp.mp.dps + 6))


def mills(x):
    x = mp.mpf(x)
    return mp.erfc(x / mp.sqrt(2)) / 2 * mp.sqrt(2 * mp.pi) * mp.exp(x * x / 2)


def cheb_nodes(a, b, n):
    a, b = mp.mpf(a), mp.mpf(b)
    return [a + (b - a) * (mp.cos(mp.pi * (k + mp.mpf(1) / 2) / n) + 1) / 2 for k in range(n)]


def fit_rational(xs, fs, m, n, loeb=15, lawson=40):
    """min max |P/Q / f - 1| over the nodes; P degree m, Q degree n, Q(0) = 1."""
    N = len(xs)
    w = [mp.mpf(1)] * N
    qv = [mp.mpf(1)] * N
    best = None
    for it in range(loeb + lawson):
        rows, rhs = [], []
        for i, (x, f) in enumerate(zip(xs, fs)):
            sc = mp.sqrt(w[i]) / (abs(f) * abs(qv[i]))
            rows.append([sc * x ** j for j in range(m + 1)] + [-sc * f * x ** j for j in range(1, n + 1)])
            rhs.append(sc * f)
        sol = mp.qr_solve(mp.matrix(rows), mp.matrix(rhs))[0]
        p = [sol[j] for j in range(m + 1)]
        q = [mp.mpf(1)] + [sol[m + j] for j in range(1, n + 1)]
        errs = []
        for i, (x, f) in enumerate(zip(xs, fs)):
            qx = mp.polyval(q[::-1], x)
            errs.append(mp.polyval(p[::-1], x) / qx / f - 1)
            if it < loeb:
                qv[i] = qx
        mx = max(abs(e) for e in errs)
        if best is None or mx < best[0]:
            best = (mx, p, q)
        if it >= loeb:
            w = [w[i] * abs(errs[i]) for i in range(N)]
            s = sum(w)
            w = [wi / s * N for wi in w]
    return best


def rounded_error(p, q, xs, fs):
    """Max relative error of the rational with FP64-rounded coefficients."""
    pr = [mp.mpf(float(c)) for c in p]
    qr = [mp.mpf(float(c)) for c in q]
    return max(abs(mp.polyval(pr[::-1], x) / mp.polyval(qr[::-1], x) / f - 1) for x, f in zip(xs, fs))


def fit_log_poly(deg):
    """R(s) with log m = 2f + f s R(s); minimax in the relative error of log m."""
    smax = ((mp.sqrt(2) - 1) / (mp.sqrt(2) + 1)) ** 2
    N = 80
    xs = [smax * (mp.cos(mp.pi * (k + mp.mpf(1) / 2) / N) + 1) / 2 for k in range(N)]
    fs = [(2 * mp.atanh(mp.sqrt(x)) - 2 * mp.sqrt(x)) / (mp.sqrt(x) * x) for x in xs]
    w = [mp.mpf(1)] * N
    best = None
    for _ in range(40):
        rows = [[mp.sqrt(w[i]) * x / 2 * x ** j for j in range(deg + 1)] for i, x in enumerate(xs)]
        rhs = [mp.sqrt(w[i]) * x / 2 * f for i, (x, f) in enumerate(zip(xs, fs))]
        c = mp.qr_solve(mp.matrix(rows), mp.matrix(rhs))[0]
        coef = [c[j] for j in range(deg + 1)]
        errs = [(mp.polyval(coef[::-1], x) - f) * x / 2 for x, f in zip(xs, fs)]
        mx = max(abs(e) for e in errs)
        if best is None or mx < best[0]:
            best = (mx, coef)
        w = [w[i] * abs(errs[i]) for i in range(N)]
        sw = sum(w)
        w = [wi / sw * N for wi in w]
    coef = best[1]
    cr = [mp.mpf(float(x)) for x in coef]
    worst = 0
    lo, hi = mp.sqrt(mp.mpf(1) / 2), mp.sqrt(2)
    for k in range(2001):
        m = lo + (hi - lo) * k / 2000
        f = (m - 1) / (m + 1)
        if f == 0:
            continue
        worst = max(worst, abs((2 * f + f * f * f * mp.polyval(cr[::-1], f * f)) / mp.log(m) - 1))
    return coef, worst


def fit_poly(fun, a, b, deg, nodes=200, rounds=30):
    """Polynomial minimising max |p/f - 1| (Lawson-reweighted least squares)."""
    xs = cheb_nodes(a, b, nodes)
    fv = [fun(x) for x in xs]
    w = [mp.mpf(1)] * nodes
    best = None
    for _ in range(rounds):
        rows = [[mp.sqrt(w[i]) / fv[i] * x ** j for j in range(deg + 1)] for i, x in enumerate(xs)]
        rhs = [mp.sqrt(w[i]) for i in range(nodes)]
        c = mp.qr_solve(mp.matrix(rows), mp.matrix(rhs))[0]
        coef = [c[j] for j in range(deg + 1)]
        errs = [mp.polyval(coef[::-1], x) / f - 1 for x, f in zip(xs, fv)]
        mx = max(abs(e) for e in errs)
        if best is None or mx < best[0]:
            best = (mx, coef)
        w = [w[i] * abs(errs[i]) for i in range(nodes)]
        sw = sum(w)
        w = [wi / sw * nodes for wi in w]
    coef = best[1]
    cr = [mp.mpf(float(x)) for x in coef]
    dense = [a + (b - a) * k / 1500 for k in range(1501)]
    return coef, max(abs(mp.polyval(cr[::-1], x) / fun(x) - 1) for x in dense)


def carr(name, coeffs, comment):
    """C array, highest power first (Horner order)."""
    body = ",\n".join("    %s" % repr(float(c)) for c in coeffs[::-1])
    return "/* %s */\nstatic constexpr double %s[%d] = {\n%s\n};\n" % (comment, name, len(coeffs), body)


def main():
    mp.mp.dps = 40
    out = []

    # --- deep tail piece, s = sqrt(v) on [sqrt(42), sqrt(750)] -------------
    # Fitted in s itself (not a centred variable): Q(v)/s is nearly constant
    # here, so numerator and denominator are nearly proportional, and only
    # with s >= 6.5 and same-sign coefficients does FP64 rounding of the
    # coefficients stay at the 1e-17 level.
    s_lo, s_hi = mp.sqrt(42) - mp.mpf("0.01"), mp.sqrt(750)
    xs = cheb_nodes(s_lo, s_hi, 200)
    fs = [q_exp(x ** 2) / x for x in xs]
    _, p, q = fit_rational(xs, fs, 7, 7)
    dense = [s_lo + (s_hi - s_lo) * k / 1500 for k in range(1501)]
    dfs = [q_exp(x ** 2) / x for x in dense]
    e_tail = rounded_error(p, q, dense, dfs)
    print("tail (7,7): max rel %.3e" % e_tail, file=sys.stderr)
    out.append("static constexpr double QM_TAIL_VMIN = 42.0;\n")
    out.append("static constexpr double QM_TAIL_VMAX = 750.0;\n")
    out.append(carr("QM_TAIL_P", p, "Q(v)/s numerator in s = sqrt(v); rel err %.2e on 42 < v <= 750" % e_tail))
    out.append(carr("QM_TAIL_Q", q, "Q(v)/s denominator in s (constant term 1)"))

    # --- FP32 seed, z/v = P4(v)/Q5(v) on [0, 103.3] --------------------------
    xs = cheb_nodes(mp.mpf("1e-6"), mp.mpf("103.3"), 160)
    fs = [q_exp(x) / x for x in xs]
    _, p, q = fit_rational(xs, fs, 4, 5)
    dense = [mp.mpf("1e-6") + mp.mpf("103.3") * k / 1500 for k in range(1501)]
    dfs = [q_exp(x) / x for x in dense]
    e_seed = rounded_error(p, q, dense, dfs)
    print("seed (4,5): max rel %.3e" % e_seed, file=sys.stderr)
    out.append(carr("QM_SEED_P", p, "FP32 seed numerator in v; rel err %.2e over v in [0,103.3]" % e_seed))
    out.append(carr("QM_SEED_Q", q, "FP32 seed denominator in v (constant term 1)"))

    # --- Mills ratio P6/Q7 on [0, 14.5] -------------------------------------
    xs = cheb_nodes(0, mp.mpf("14.5"), 160)
    fs = [mills(x) for x in xs]
    _, p, q = fit_rational(xs, fs, 6, 7)
    dense = [mp.mpf("14.5") * k / 1500 for k in range(1501)]
    dfs = [mills(x) for x in dense]
    e_m = rounded_error(p, q, dense, dfs)
    print("mills (6,7): max rel %.3e" % e_m, file=sys.stderr)
    out.append(carr("QM_MILLS_P", p, "Mills ratio numerator in x; rel err %.2e on [0,14.5]" % e_m))
    out.append(carr("QM_MILLS_Q", q, "Mills ratio denominator in x (constant term 1)"))

    # --- Mills ratio P3/Q4 on [1.6, 14.5] (the quantile's outer step) --------
    a, b = mp.mpf("1.6"), mp.mpf("14.5")
    xs = cheb_nodes(a, b, 120)
    fs = [mills(x) for x in xs]
    _, p, q = fit_rational(xs, fs, 3, 4)
    dense = [a + (b - a) * k / 1500 for k in range(1501)]
    dfs = [mills(x) for x in dense]
    e_m32 = rounded_error(p, q, dense, dfs)
    print("mills (3,4) on [1.6, 14.5]: max rel %.3e" % e_m32, file=sys.stderr)
    out.append(carr("QM_MILLS32_P", p, "Mills ratio numerator in x; rel err %.2e on [1.6,14.5]" % e_m32))
    out.append(carr("QM_MILLS32_Q", q, "Mills ratio denominator in x (constant term 1)"))

    # --- central piece, Phi^{-1}(1/2 + q)/q = P8(r)/Q8(r), r = X - q^2 ---------
    QC, X = mp.mpf(float(0.45)), mp.mpf(float(0.2025))
    r_lo = X - QC * QC - mp.mpf("1e-12")          # |q| <= 0.45 as FP64 values, with margin
    g = lambda r: mp.sqrt(2 * mp.pi) if r == X else mp.sqrt(2) * mp.erfinv(2 * mp.sqrt(X - r)) / mp.sqrt(X - r)
    xs = cheb_nodes(r_lo, X, 160)
    fs = [g(x) for x in xs]
    _, p, q = fit_rational(xs, fs, 8, 8)
    dense = [r_lo + (X - r_lo) * k / 1500 for k in range(1501)]
    dfs = [g(x) for x in dense]
    e_c = rounded_error(p, q, dense, dfs)
    print("central (8,8): max rel %.3e" % e_c, file=sys.stderr)
    assert all(c > 0 for c in p) and all(c > 0 for c in q)
    out.append("static constexpr double QM_CENTRAL_QMAX = 0.45;\n")
    out.append("static constexpr double QM_CENTRAL_X = 0.2025;\n")
    out.append(carr("QM_CENTRAL_P", p, "Phi^{-1}(1/2 + q)/q numerator in r = 0.2025 - q^2; rel err %.2e for |q| <= 0.45" % e_c))
    out.append(carr("QM_CENTRAL_Q", q, "central denominator in r (constant term 1)"))

    # --- FP32+refine central piece ----------------------------------------
    xs = cheb_nodes(r_lo, X, 120)
    fs = [g(x) for x in xs]
    _, p, q = fit_rational(xs, fs, 2, 3)
    # the seed is evaluated in FP32: measure it with FP32-rounded coefficients
    f32 = lambda c: mp.mpf(struct.unpack("f", struct.pack("f", float(c)))[0])
    e_s = max(abs(mp.polyval([f32(c) for c in p][::-1], x) / mp.polyval([f32(c) for c in q][::-1], x) / f - 1)
              for x, f in zip(dense, dfs))
    print("central FP32 seed (2,3): max rel %.3e" % e_s, file=sys.stderr)
    out.append(carr("QM_C32_SP", p, "FP32 central seed numerator in r = 0.2025 - q^2; rel err %.2e (FP32 coefficients)" % e_s))
    out.append(carr("QM_C32_SQ", q, "FP32 central seed denominator in r (constant term 1)"))
    zmax = mp.sqrt(2) * mp.erfinv(2 * QC) * (1 + mp.mpf("1e-3"))
    Y = zmax * zmax
    erfh = lambda y: mp.erf(mp.sqrt(y / 2)) / (2 * mp.sqrt(y)) if y > 0 else 1 / mp.sqrt(2 * mp.pi)
    coef, e_e = fit_poly(erfh, mp.mpf(0), Y, 6)
    print("central erf E6: max rel %.3e" % e_e, file=sys.stderr)
    out.append(carr("QM_C32_E", coef, "erf(z/sqrt2)/(2z) in y = z^2 <= %.4f; rel err %.2e" % (float(Y), e_e)))
    coef, e_g = fit_poly(lambda y: mp.sqrt(2 * mp.pi) * mp.exp(y / 2), mp.mpf(0), Y, 3)
    print("central 1/phi G3: max rel %.3e" % e_g, file=sys.stderr)
    out.append(carr("QM_C32_G", coef, "1/phi(z) = sqrt(2 pi) e^{y/2} in y = z^2 <= %.4f; rel err %.2e" % (float(Y), e_g)))

    # --- FP64 log kernel: R6(s) ----------------------------------------------
    coef, e_log = fit_log_poly(6)
    print("log R6: max rel %.3e" % e_log, file=sys.stderr)
    out.append(carr("QM_LOG_R", coef, "log m = 2f + f s R(s), s = f^2 <= 0.0294; rel err %.2e" % e_log))

    hdr = [
        "/* qm_coeffs.h -- generated by fit_coefficients.py; do not edit. */\n",
        "#pragma once\n\n",
        "/* Fitted pieces (see fit_coefficients.py for method and domains). */\n",
    ] + out
    with open(OUT, "w") as f:
        f.write("".join(hdr))
    print("wrote", OUT, file=sys.stderr)


if __name__ == "__main__":
    main()
