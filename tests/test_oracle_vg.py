"""Pins of the variance-gamma oracle (exponential -> variance-gamma
recycling with integer lambda, Section 8.2) against what the mathematics
fixes: the paper's closed form of the masses (a 2F1), its remark that
lambda = 1 is the base itself, mpmath quadrature of the density with
K_{lambda-1/2}, mpmath root finding on the defining equation, and the
mirror symmetry."""
import numpy as np
import pytest

import oracle

mp = pytest.importorskip("mpmath")

PARAMS = [(1, 1.0, 0.0), (2, 1.0, 0.0), (2, 1.0, 0.5), (3, 2.0, -1.0), (5, 1.0, 0.3), (16, 2.0, 1.5)]


def paper_p_plus(lam, a, b):
    """p+ as Section 8.2 prints it (A&S 6.621.3 of the integral)."""
    L, A, B = mp.mpf(lam), mp.mpf(a), mp.mpf(b)
    return (2 ** (2 * L - 1) * ((A + B) / (A - B)) ** L * mp.gamma(L + mp.mpf(1) / 2)
            * mp.hyp2f1(2 * L, L, L + 1, (A + B) / (B - A)) / (mp.sqrt(mp.pi) * mp.gamma(L + 1)))


def density(lam, a, b, x):
    L, A, B = mp.mpf(lam), mp.mpf(a), mp.mpf(b)
    x = mp.mpf(x)
    return ((A * A - B * B) ** L * mp.exp(B * x) * abs(x) ** (L - mp.mpf(1) / 2) * mp.besselk(L - mp.mpf(1) / 2, A * abs(x))
            / ((2 * A) ** (L - mp.mpf(1) / 2) * mp.sqrt(mp.pi) * mp.gamma(L)))


def mp_tail(lam, a, b, x):
    """1 - F(x), x > 0, by quadrature of the Bessel-function density, scaled
    by e^{(alpha-beta) x} so that the integrand is O(1) at the lower limit
    (left unscaled, a tail far below 1 fools mpmath's error estimate)."""
    with mp.workdps(30):
        r = mp.mpf(a) - mp.mpf(b)
        x = mp.mpf(x)
        body = mp.quad(lambda t: density(lam, a, b, x + t) * mp.exp(r * x), [0, 1, 5, 20, 60, mp.inf])
        return body * mp.exp(-r * x)


@pytest.mark.parametrize("p", PARAMS, ids=lambda p: "l%d_a%g_b%g" % p)
def test_masses_match_the_papers_closed_form(p):
    lp, lm = oracle.vg_masses(*p)
    with mp.workdps(30):
        want_p = paper_p_plus(*p)
        want_m = paper_p_plus(p[0], p[1], -p[2])      # p- is p+ of the mirrored target
    assert abs(np.exp(lp) / float(want_p) - 1) < 4e-16
    assert abs(np.exp(lm) / float(want_m) - 1) < 4e-16
    assert abs(np.exp(lp) + np.exp(lm) - 1) < 4e-16


def test_lambda_one_is_the_base():
    """Section 8.2: for lambda = 1 the target is the base, Q(v) = v."""
    v = np.concatenate([np.geomspace(1e-300, 1e300, 60), -np.geomspace(1e-300, 1e300, 60)])
    for a, b in ((1.0, 0.0), (2.0, 0.7), (1.0, -0.9)):
        x = oracle.vg_map(v, 1, a, b)
        assert np.max(np.abs(x / v - 1)) <= 2.3e-16


@pytest.mark.parametrize("p", [(2, 1.0, 0.5), (3, 2.0, -1.0), (5, 1.0, 0.3)], ids=lambda p: "l%d_a%g_b%g" % p)
def test_tail_matches_bessel_quadrature(p):
    for x in (0.05, 1.0, 7.0, 30.0):
        got = oracle.vg_log_tail(x, *p)
        want = float(mp.log(mp_tail(*p, x)))
        assert abs(got - want) <= 1e-14 * max(1.0, abs(want)), (p, x, got, want)


@pytest.mark.parametrize("p", [(2, 1.0, 0.5), (4, 1.5, -0.5)], ids=lambda p: "l%d_a%g_b%g" % p)
def test_map_is_the_root_of_the_defining_equation(p):
    """x = Q(v) solves 1 - F(x) = p+ e^{-(alpha-beta) v}, with 1 - F by
    quadrature of the Bessel-function density and p+ from the paper."""
    lam, a, b = p
    with mp.workdps(30):
        pp = paper_p_plus(*p)
        for v in (0.01, 0.4, 3.0, 20.0):
            x = oracle.vg_map(np.array([v]), *p)[0]
            target = pp * mp.exp(-(mp.mpf(a) - mp.mpf(b)) * mp.mpf(v))
            root = mp.findroot(lambda t: mp.log(mp_tail(lam, a, b, t)) - mp.log(target), mp.mpf(x))
            assert abs(x / float(root) - 1) <= 3e-16, (p, v, x, root)


def test_mirror_symmetry():
    v = np.concatenate([np.geomspace(1e-6, 1e3, 40)])
    x1 = oracle.vg_map(-v, 3, 1.5, 0.6)
    x2 = oracle.vg_map(v, 3, 1.5, -0.6)
    assert np.array_equal(x1, -x2)


def test_specials_and_invalid():
    x = oracle.vg_map(np.array([0.0, np.inf, -np.inf, np.nan]), 2, 1.0, 0.0)
    assert x[0] == 0 and x[1] == np.inf and x[2] == -np.inf and np.isnan(x[3])
    for bad in [(1.5, 1.0, 0.0), (0, 1.0, 0.0), (2, 1.0, 1.0), (2, 1.0, -2.0), (2, float("nan"), 0.0)]:
        assert np.isnan(oracle.vg_map(np.array([1.0]), *bad)[0])
