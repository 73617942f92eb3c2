"""Pins of the real-lambda variance-gamma oracle (oracle/vg_real.c) against
what the paper and the mathematics fix, none of which shares its method
(the Bessel integral K_nu(z) = int e^{-z cosh s} cosh(nu s) ds turned into
a trapezoid over incomplete gamma functions):

  * integer lambda: the finite-sum oracle (vg.c, K_{n+1/2} elementary), to
    the last bit -- a different method altogether;
  * lambda = 1: the target is the base itself, Q(v) = v (Section 8.2);
  * the masses p+, p- against the paper's 2F1 closed form (A&S 6.621.3,
    Section 8.2) at real lambda, and p+ = p- = 1/2 for beta = 0;
  * tail and central masses against mpmath quadrature of the Bessel-function
    density;
  * the map against its defining equation, the tail by mpmath quadrature;
  * the slope at 0, Q'(0) = f0(0+)/f(0) with f(0) = A Gamma(nu) 2^(nu-1)
    alpha^(-nu) from K_nu's leading term (lambda > 1/2);
  * mirror symmetry Q(-v; beta) = -Q(v; -beta); specials; the incomplete
    gamma functions against mpmath.
"""
import math

import numpy as np
import pytest

import oracle

mp = pytest.importorskip("mpmath")


def density(lam, al, be):
    """mpmath Bessel-function density of Section 8.2 (mu = 0) on x > 0."""
    lam, al, be = mp.mpf(lam), mp.mpf(al), mp.mpf(be)
    A = (al ** 2 - be ** 2) ** lam / ((2 * al) ** (lam - 0.5) * mp.sqrt(mp.pi) * mp.gamma(lam))
    return lambda t: A * mp.exp(be * t) * t ** (lam - 0.5) * mp.besselk(lam - 0.5, al * t)


def p_plus_2f1(lam, al, be):
    """Section 8.2: p+ from identity 6.621.3 of Abramowitz & Stegun."""
    lam, al, be = mp.mpf(lam), mp.mpf(al), mp.mpf(be)
    return (2 ** (2 * lam - 1) * ((al + be) / (al - be)) ** lam * mp.gamma(lam + 0.5)
            * mp.hyp2f1(2 * lam, lam, lam + 1, (al + be) / (be - al)) / (mp.sqrt(mp.pi) * mp.gamma(lam + 1)))


def ulps(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    ia, ib = a.view(np.int64), b.view(np.int64)
    return np.abs(ia - ib)


V = np.array([1e-300, 1e-12, 1e-4, 0.01, 0.3, 1.0, 2.5, 7.0, 30.0, 150.0, 700.0])


@pytest.mark.parametrize("lam,al,be", [(2, 1.0, 0.0), (3, 2.0, -1.0), (5, 1.5, 0.6), (8, 1.0, 0.25)])
def test_integer_lambda_equals_finite_sums(lam, al, be):
    v = np.concatenate([V, -V])
    a = oracle.vgr_map(v, lam, al, be)
    b = oracle.vg_map(v, lam, al, be)
    assert ulps(a, b).max() <= 1, (a, b)
    np.testing.assert_allclose(oracle.vgr_masses(lam, al, be), oracle.vg_masses(lam, al, be), rtol=0, atol=4e-16)


@pytest.mark.parametrize("al,be", [(1.0, 0.0), (2.0, -1.0), (1.0, 0.5)])
def test_lambda_one_is_the_base(al, be):
    v = np.concatenate([V[:-1], -V[:-1]])
    assert ulps(oracle.vgr_map(v, 1.0, al, be), v).max() <= 1


@pytest.mark.parametrize("lam,al,be", [(1.5, 1.0, 0.5), (2.5, 2.0, -1.0), (4.25, 1.0, 0.3), (1.1, 1.3, 0.2),
                                       (6.75, 0.7, -0.35)])
def test_masses_match_2f1(lam, al, be):
    mp.mp.dps = 40
    lp, lm = oracle.vgr_masses(lam, al, be)
    ref_p = p_plus_2f1(lam, al, be)
    ref_m = p_plus_2f1(lam, al, -be)           # p- is p+ with beta mirrored
    assert abs(math.exp(lp) / float(ref_p) - 1) < 3e-16
    assert abs(math.exp(lm) / float(ref_m) - 1) < 3e-16
    assert abs(float(ref_p + ref_m) - 1) < 1e-30


@pytest.mark.parametrize("lam", [1.5, 2.5, 3.7])
def test_symmetric_masses_are_half(lam):
    lp, lm = oracle.vgr_masses(lam, 1.3, 0.0)
    assert abs(lp - math.log(0.5)) < 3e-16 and abs(lm - math.log(0.5)) < 3e-16


@pytest.mark.parametrize("lam,al,be,xs", [(1.5, 1.0, 0.5, (0.7, 12.0)), (4.25, 1.0, 0.3, (0.05, 3.0)),
                                          (2.5, 2.0, -1.0, (3.0,))])
def test_tail_and_central_mass_match_quadrature(lam, al, be, xs):
    mp.mp.dps = 20
    f = density(lam, al, be)
    fl = density(lam, al, -be)
    for x in xs:
        ref = mp.quad(f, [x, x + 2, x + 12, x + 60, mp.inf])
        assert abs(oracle.vgr_log_tail(x, lam, al, be) - float(mp.log(ref))) < 2e-15, x
        refl = mp.quad(fl, [x, x + 2, x + 12, x + 60, mp.inf])
        assert abs(oracle.vgr_log_tail(-x, lam, al, be) - float(mp.log(refl))) < 2e-15, x
    for x in (1e-6, 0.3):
        ref = mp.quad(f, [0, x])
        assert abs(oracle.vgr_central_mass(x, lam, al, be) / float(ref) - 1) < 2e-15, x


@pytest.mark.parametrize("lam,al,be,v", [(1.5, 1.0, 0.5, 4.0), (4.25, 1.0, 0.3, 0.9), (4.25, 1.0, 0.3, 15.0),
                                         (1.05, 1.0, 0.3, 0.002), (1.2, 2.0, -1.0, -0.001)])
def test_map_solves_its_equation(lam, al, be, v):
    """1 - F(Q) = p+ e^{-(alpha - beta) v} (v >= 0; v < 0 on the mirrored
    side) at the oracle's Q, with the tail by mpmath quadrature of the
    Bessel-function density (near the origin its central form, the integral
    from 0 to Q): the residual, divided by its derivative, moves Q by at
    most a few parts in 1e16."""
    mp.mp.dps = 20
    if v < 0:                       # v < 0 is the mirrored side: beta -> -beta
        lam, al, be, sgn = lam, al, -be, -1
    else:
        sgn = 1
    f = density(lam, al, be)
    lp, _ = oracle.vgr_masses(lam, al, be)
    x0 = sgn * oracle.vgr_map(np.array([v]), lam, al, -be if sgn < 0 else be)[0]
    va = abs(v)
    if (al - be) * va < 0.5:
        # near the origin the central form, int_0^Q f = p+ (1 - e^{-(alpha - beta) v}), is the well-conditioned one
        mp.mp.dps = 30
        cen = mp.quad(f, [0, x0])
        dx = (mp.exp(lp) * -mp.expm1(-(al - be) * mp.mpf(va)) - cen) / f(mp.mpf(x0))
    else:
        tail = mp.quad(f, [x0, x0 + 2, x0 + 12, x0 + 60, mp.inf])
        resid = mp.log(tail) - (mp.mpf(lp) - (al - be) * mp.mpf(va))
        dx = resid * tail / f(mp.mpf(x0))
    assert abs(float(dx) / x0) < 4e-16, (v, x0, float(dx))


@pytest.mark.parametrize("lam,al,be", [(1.5, 1.0, 0.5), (2.5, 2.0, -1.0), (4.25, 1.0, 0.3), (1.05, 1.0, 0.3),
                                       (1.2, 2.0, -1.0)])
def test_slope_at_zero(lam, al, be):
    """Q(v) ~ Q'(0) v, Q'(0) = p+ (alpha - beta) / f(0), f(0) = A Gamma(nu) 2^(nu-1) alpha^(-nu)."""
    mp.mp.dps = 30
    nu = mp.mpf(lam) - 0.5
    A = (mp.mpf(al) ** 2 - be ** 2) ** lam / ((2 * mp.mpf(al)) ** nu * mp.sqrt(mp.pi) * mp.gamma(lam))
    f0 = A * mp.gamma(nu) * 2 ** (nu - 1) * mp.mpf(al) ** (-nu)
    lp, _ = oracle.vgr_masses(lam, al, be)
    slope = math.exp(lp) * (al - be) / float(f0)
    v = 1e-9
    q = oracle.vgr_map(np.array([v]), lam, al, be)[0]
    assert abs(q / (slope * v) - 1) < 1e-8


def test_mirror_symmetry_and_specials():
    v = np.concatenate([V[:-2], -V[:-2]])
    a = oracle.vgr_map(v, 2.75, 1.0, 0.4)
    b = oracle.vgr_map(-v, 2.75, 1.0, -0.4)
    assert np.array_equal(a, -b)
    s = oracle.vgr_map(np.array([np.nan, np.inf, -np.inf, 0.0, -0.0]), 2.75, 1.0, 0.4)
    assert np.isnan(s[0]) and s[1] == np.inf and s[2] == -np.inf and s[3] == 0 and s[4] == 0
    for bad in ((0.5, 1.0, 0.0), (2.0, 1.0, 1.0), (2.0, 1.0, -1.5), (float("nan"), 1.0, 0.0), (65.0, 1.0, 0.0)):
        assert np.isnan(oracle.vgr_map(np.array([1.0]), *bad)[0]), bad
        with pytest.raises(ValueError):
            oracle.vgr_masses(*bad)


@pytest.mark.parametrize("a", [1.5, 2.0, 3.0, 4.75, 20.5])
def test_incomplete_gamma(a):
    mp.mp.dps = 30
    for y in (1e-8, 0.3, a - 0.5, a + 0.9, a + 2, 3 * a + 10, 400.0):
        up = float(mp.log(mp.gammainc(a, y, mp.inf)))
        lo = float(mp.log(mp.gammainc(a, 0, y)))
        assert abs(oracle.vgr_log_upper_gamma(a, y) - up) <= 4e-16 * max(1.0, abs(up)), (a, y)
        assert abs(oracle.vgr_log_lower_gamma(a, y) - lo) <= 4e-16 * max(1.0, abs(lo)), (a, y)
