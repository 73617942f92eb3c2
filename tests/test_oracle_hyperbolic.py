"""Pins of the hyperbolic oracle (exponential -> hyperbolic recycling,
Section 8.1) against what the mathematics fixes: the closed-form
normalisation, mpmath quadrature and root finding, the paper's initial
slopes, symmetry, and the tail asymptotics."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle

PARAMS = [(1.0, 0.0, 1.0), (2.0, 0.5, 1.0), (1.0, -0.7, 0.3), (5.0, 2.0, 3.0), (1.0, 0.9, 0.01)]


def closed_form_log_c(a, b, d):
    """C = gamma / (2 alpha delta K_1(delta gamma)) (Section 8.1)."""
    a, b, d = mp.mpf(a), mp.mpf(b), mp.mpf(d)
    g = mp.sqrt(a ** 2 - b ** 2)
    return mp.log(g / (2 * a * d * mp.besselk(1, d * g)))


def log_upper_tail(a, b, d, x):
    """log(1 - F(x)), x >= 0, by mpmath quadrature of the integrand scaled to
    O(1) at x: 1 - F(x) = C e^{-alpha r(x) + beta x} int_0^inf
    e^{-alpha (r(x+t) - r(x)) + beta t} dt, r(y) = sqrt(delta^2 + y^2).  (Left
    unscaled, a tail below e^-100 fools mpmath's error estimate.)"""
    a, b, d, x = mp.mpf(a), mp.mpf(b), mp.mpf(d), mp.mpf(x)
    r = lambda y: mp.sqrt(d * d + y * y)
    rx = r(x)
    g = lambda t: mp.exp(-a * (r(x + t) - rx) + b * t)
    w = 1 / max(a * x / rx - b, mp.mpf(1) / 16)            # initial decay length
    t_end = 300 / (a - b) + 10 * d + 10
    pts = sorted(set([mp.mpf(0)] + [w * 2 ** k for k in range(40) if w * 2 ** k < t_end] + [t_end]))
    return closed_form_log_c(a, b, d) - a * rx + b * x + mp.log(mp.quad(g, pts))


def upper_tail(a, b, d, x):
    return mp.exp(log_upper_tail(a, b, d, x))


@pytest.mark.parametrize("a,b,d", PARAMS)
def test_normalisation_and_masses(a, b, d):
    lp, lm, lc = oracle.hyperbolic_masses(a, b, d)
    with mp.workdps(40):
        assert abs(lc - closed_form_log_c(a, b, d)) <= 4e-17
        pp = upper_tail(a, b, d, 0)
        # log p+- to half an ulp of the logarithm
        assert abs(lp - mp.log(pp)) <= 1.2e-16 * abs(mp.log(pp)) + 1e-18
        assert abs(lm - mp.log(1 - pp)) <= 1.2e-16 * abs(mp.log(1 - pp)) + 1e-18
    if b == 0:
        assert lp == lm


@pytest.mark.parametrize("a,b,d", PARAMS)
def test_map_is_the_root_of_the_defining_equation(a, b, d):
    """v >= 0: 1 - F(Q) = p+ e^{-(alpha-beta) v}; v < 0: F(Q) = p- e^{(alpha+beta) v}
    (the latter as the upper tail of the mirrored target); mpmath roots at
    40 digits, both tails, near 0 and far out: within one ulp (the
    residuals of two neighbouring doubles can be closer than the extended-
    precision quadrature resolves)."""
    v = np.array([1e-12, 1e-3, 0.3, 1.0, 3.0, 20.0, 100.0, 600.0])
    v = np.concatenate([v, -v])
    x = oracle.hyperbolic_map(v, a, b, d)
    with mp.workdps(40):
        pp = upper_tail(a, b, d, 0)
        pm = 1 - pp
        for vi, xi in zip(v, x):
            if vi > 0:
                tgt, aa, bb, X = pp * mp.exp(-(a - b) * mp.mpf(vi)), a, b, xi
            else:
                tgt, aa, bb, X = pm * mp.exp((a + b) * mp.mpf(vi)), a, -b, -xi
            if tgt > mp.mpf("0.25"):    # near the centre: the mass of [0, X] (no cancellation)
                side = pp if vi > 0 else pm
                F = lambda t: (side - upper_tail(aa, bb, d, t)) - (side - tgt)
            else:
                F = lambda t: log_upper_tail(aa, bb, d, t) - mp.log(tgt)
            r = mp.findroot(F, (mp.mpf(X) * (1 - mp.mpf("1e-9")), mp.mpf(X) * (1 + mp.mpf("1e-9"))), solver="anderson")
            assert abs(mp.mpf(X) / r - 1) <= 2.3e-16, (a, b, d, vi, xi)


@pytest.mark.parametrize("a,b,d", PARAMS)
def test_initial_slopes(a, b, d):
    """Q'(0+) = p+ (alpha - beta) / f(0) and Q'(0-) = p- (alpha + beta) / f(0),
    f(0) = C e^{-alpha delta} (the paper's initial conditions of the right
    and left problems); one-sided difference quotients at |v| = 1e-10."""
    lp, lm, lc = oracle.hyperbolic_masses(a, b, d)
    f0 = math.exp(lc - a * d)
    h = 1e-10
    q = oracle.hyperbolic_map(np.array([h, -h]), a, b, d)
    assert abs(q[0] / h / (math.exp(lp) * (a - b) / f0) - 1) < 1e-8
    assert abs(-q[1] / h / (math.exp(lm) * (a + b) / f0) - 1) < 1e-8


def test_mirror_symmetry():
    """x -> -x with beta -> -beta exchanges the sides: Q(-v; -beta) = -Q(v; beta)."""
    v = np.array([0.01, 0.7, 2.5, 40.0])
    assert np.array_equal(oracle.hyperbolic_map(-v, 2.0, -0.5, 1.5), -oracle.hyperbolic_map(v, 2.0, 0.5, 1.5))
    w = oracle.hyperbolic_map(np.concatenate([v, -v]), 1.3, 0.0, 0.7)
    assert np.array_equal(w[:4], -w[4:])


@pytest.mark.parametrize("a,b,d", [(1.0, 0.0, 1.0), (2.0, 0.5, 1.0)])
def test_tail_asymptotics(a, b, d):
    """For large v, 1 - F(x) ~ C/(alpha-beta) e^{-(alpha-beta) x - alpha delta^2/(2x)},
    so Q(v) = v + log(C/((alpha-beta) p+))/(alpha-beta) - alpha delta^2/(2 (alpha-beta) v) + O(v^-2)."""
    lp, lm, lc = oracle.hyperbolic_masses(a, b, d)
    r = a - b
    for v in (200.0, 700.0):
        q = oracle.hyperbolic_map(np.array([v]), a, b, d)[0]
        pred = v + (lc - math.log(r) - lp) / r - a * d * d / (2 * r * v)
        assert abs(q - pred) < 20.0 / (r * v * v) + 1e-12 * v, (v, q, pred)


def test_specials_and_invalid():
    x = oracle.hyperbolic_map(np.array([0.0, -0.0, np.inf, -np.inf, np.nan]), 1.0, 0.2, 1.0)
    assert x[0] == 0 and x[2] == np.inf and x[3] == -np.inf and np.isnan(x[4])
    for a, b, d in ((1.0, 1.0, 1.0), (1.0, 0.0, 0.0), (-1.0, 0.0, 1.0), (1.0, 0.0, np.nan)):
        assert np.all(np.isnan(oracle.hyperbolic_map(np.array([0.5]), a, b, d)))
