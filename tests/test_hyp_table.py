"""CPU checks of the exponential -> hyperbolic table builder (Section 8.1).

The builder's solution of the left/right recycling ODEs, and its tables
evaluated on the host exactly as the kernel does (cell from the exponent
and leading mantissa bits of t = 1 + |v|/v0, Horner in d = |v| - centre,
the large-v form from v_top on), are compared with the oracle, which solves the
defining equation F(x) = F0(v) by quadrature and bisection.  Closed forms
pin the centre slope (Section 8.1, with K_1 from scipy) and the masses."""
import ctypes
import math

import numpy as np
import pytest

import oracle
import paper_0901_0638_amd as qm

PARAMS = [(1.0, 0.0, 1.0), (1.0, 0.5, 1.0), (2.0, -1.5, 0.3), (1.0, 0.9, 5.0), (1.0, 0.0, 0.001),
          (50.0, 10.0, 0.1)]


def origin_eval(row, a, which):
    """A side's first octave in the origin form (row 0: rho, then the
    coefficients of P3..P0 or P2..P0, highest power first): R = P0(a) +
    w (P1(a) + w (P2(a) + w P3(a))), w = a^rho, as the kernel evaluates it."""
    degs = (0, 1, 2, 4) if which == "f64" else (0, 1, 3)
    w = a ** row[0]
    R, k = 0.0, 1
    for dg in degs:
        p = 0.0
        for _ in range(dg + 1):
            p = p * a + row[k]
            k += 1
        R = R * w + p
    return R


def table_eval(h, rr, rl, v, which="f64"):
    """The kernel's evaluation of a table, in numpy FP64: t = 1 + |v|/v0 by
    one fused multiply-add, the cell from the exponent and top three
    mantissa bits of t, its centre from t with the lower bits replaced; a
    side with an origin form takes it below v0."""
    v = np.asarray(v, np.float64)
    out = np.empty_like(v)
    right, left = (h.right, h.left) if which == "f64" else (h.right32, h.left32)
    for i, x in enumerate(v):
        S, rows = (left, rl) if x < 0 else (right, rr)
        a = abs(x)
        if S.origin and a < S.v0:
            Q = a * origin_eval(rows[0], a, which)
        elif not a < S.v_top:
            if not np.isfinite(a):
                Q = a
            elif S.far_clog == 0:
                Q = a + (S.far_c0 + (S.far_c1 + S.far_c2 / a) / a)
            else:
                Q = a + S.far_c0 + S.far_clog * math.log(a)
                for _ in range(3):
                    Q = a + S.far_c0 + S.far_clog * math.log(Q) + (S.far_c1 + S.far_c2 / Q) / Q
        else:
            t = fma(a, S.inv_v0, 1.0)
            bits = np.float64(t).view(np.uint64)
            hi = int(bits >> np.uint64(32))
            j = min((hi >> 17) - (1023 << 3), len(rows) - 1)   # the kernel's clamp (t may round up to 2^noct)
            tc = np.uint64(((hi & ~((1 << 17) - 1)) | (1 << 16)) << 32).view(np.float64)
            d = fma(-S.v0, float(tc) - 1.0, a)
            R = rows[j][0]
            for c in rows[j][1:]:
                R = R * d + c
            Q = a * R
        out[i] = math.copysign(Q, x)
    return out


def fma(x, y, z):
    """x y + z rounded once (exact rational arithmetic)."""
    from fractions import Fraction
    return float(Fraction(x) * Fraction(y) + Fraction(z))


def probe_points(h, p, seed):
    alpha, beta, _ = p
    rng = np.random.default_rng(seed)
    pts = [rng.exponential(1 / (alpha - beta), 200), -rng.exponential(1 / (alpha + beta), 200),
           np.geomspace(1e-9, 1e7, 40), -np.geomspace(1e-9, 1e7, 40)]
    for S, sgn in ((h.right, 1), (h.left, -1)):
        # every cell boundary of the first octaves of t = 1 + v/v0, v_top
        edges = [S.v0 * (2.0 ** k * (1 + i / qm.HYP_SUB) - 1) for k in range(0, 7) for i in range(qm.HYP_SUB)]
        edges += [S.v_top * (1 - 1e-16), S.v_top, S.v_top * 1.5, S.v_top * 1e3]
        edges = np.array(edges)
        edges = edges[edges > 0]
        pts.append(sgn * edges)
        pts.append(sgn * np.nextafter(edges, 0))
    return np.concatenate(pts)


@pytest.fixture(scope="module", params=PARAMS, ids=lambda p: "a%g_b%g_d%g" % p)
def built(request):
    p = request.param
    h, rr, rl = qm.debug_hyperbolic_table(*p)
    v = probe_points(h, p, 7)
    return p, h, rr, rl, v, oracle.hyperbolic_map(v, *p)


def test_dense_solution_matches_oracle(built):
    """The ODE solution (and the direct tail solve beyond the anchor) is the
    correctly rounded map: within one ulp of the oracle's."""
    p, h, rr, rl, v, ref = built
    q = qm.debug_hyperbolic_dense(*p, v)
    rel = np.abs(q - ref) / np.abs(ref)
    assert rel.max() <= 2.3e-16, (p, rel.max(), v[rel.argmax()])


def test_table_matches_oracle(built):
    p, h, rr, rl, v, ref = built
    got = table_eval(h, rr, rl, v)
    rel = np.abs(got - ref) / np.abs(ref)
    assert rel.max() <= 6e-16, (p, rel.max(), v[rel.argmax()])


def test_fp32_cells_match_oracle(built):
    """The cells for FP32 outputs (degree 7, truncation 1e-10) evaluated in FP64."""
    p, h, _, _, v, ref = built
    _, r32, l32 = qm.debug_hyperbolic_table(*p, which="f32")
    got = table_eval(h, r32, l32, v, "f32")
    rel = np.abs(got - ref) / np.abs(ref)
    assert rel.max() <= 1.2e-10, (p, rel.max(), v[rel.argmax()])


def test_header_layout(built):
    p, h, rr, rl, v, ref = built
    assert ctypes.sizeof(qm.HypTableHeader) == 392
    _, r32, l32 = qm.debug_hyperbolic_table(*p, which="f32")
    for S, rows, rate, deg, bound, S0 in ((h.right, rr, p[0] - p[1], qm.HYP_DEGREE, 1.2e-16, h.right),
                                         (h.left, rl, p[0] + p[1], qm.HYP_DEGREE, 1.2e-16, h.right),
                                         (h.right32, r32, p[0] - p[1], qm.HYP_DEGREE_F32, 1e-10, h.right32),
                                         (h.left32, l32, p[0] + p[1], qm.HYP_DEGREE_F32, 1e-10, h.right32)):
        assert S.degree == deg
        assert S.ncell == qm.HYP_SUB * S.noct and rows.shape == (S.ncell, deg + 1)
        assert 0 < S.noct <= 40
        assert S.v0 == 2.0 ** round(math.log2(S.v0)) and S.inv_v0 * S.v0 == 1.0
        assert S.v0 == S0.v0                      # one v0 for both sides of a cell set
        assert S.v_top == S.v0 * (2.0 ** S.noct - 1)
        assert S.max_rel_err < bound              # FP64: the rounding of R itself, about half an ulp
        # the cells cover the bulk of the base (the FP32 set's large-v form can
        # take over earlier: it needs only 2.5e-11)
        assert S.v_top >= (32 if deg == qm.HYP_DEGREE else 16) / rate


def test_masses_match_oracle(built):
    p, h, *_ = built
    lp, lm, _ = oracle.hyperbolic_masses(*p)
    assert abs(h.log_p_plus - lp) <= 2e-16 * max(1.0, abs(lp)) + 1e-16
    assert abs(h.log_p_minus - lm) <= 2e-16 * max(1.0, abs(lm)) + 1e-16
    assert abs(np.logaddexp(h.log_p_plus, h.log_p_minus)) < 4e-16


def test_centre_slope_closed_form(built):
    """Q'(0+) = 2 p+ (alpha - beta) (alpha delta / gamma) K_1(delta gamma) e^{alpha delta}
    and Q'(0-) likewise with p- and alpha + beta (Section 8.1)."""
    special = pytest.importorskip("scipy.special")
    p, h, rr, rl, *_ = built
    a, b, d = p
    g = math.sqrt(a * a - b * b)
    for S, rows, lpm, rate in ((h.right, rr, h.log_p_plus, a - b), (h.left, rl, h.log_p_minus, a + b)):
        x = -S.v0 / (2 * qm.HYP_SUB)            # d at v = 0 in the first cell (centre v0/16)
        R0 = rows[0][0]
        for c in rows[0][1:]:
            R0 = R0 * x + c
        want = 2 * math.exp(lpm) * rate * (a * d / g) * special.k1e(d * g) * math.exp(a * d - d * g)
        assert abs(R0 / want - 1) < 2e-14, (p, R0, want)


def test_large_v_constant(built):
    """Far out Q - v -> c0 = log(C / ((alpha - beta) p+)) / (alpha - beta), with the
    normalising constant C = gamma / (2 alpha delta K_1(delta gamma))."""
    special = pytest.importorskip("scipy.special")
    p, h, *_ = built
    a, b, d = p
    g = math.sqrt(a * a - b * b)
    log_c = math.log(g / (2 * a * d)) - math.log(special.k1e(d * g)) + d * g
    for S, lpm, rate in ((h.right, h.log_p_plus, a - b), (h.left, h.log_p_minus, a + b)):
        c0 = (log_c - math.log(rate) - lpm) / rate
        assert abs(S.far_c0 - c0) <= 1e-13 * max(1.0, abs(c0)), (p, S.far_c0, c0)


def test_mirror_and_symmetry():
    """beta -> -beta swaps the sides (x -> -x of the target); beta = 0 makes them equal."""
    h1, r1, l1 = qm.debug_hyperbolic_table(1.0, 0.5, 1.0)
    h2, r2, l2 = qm.debug_hyperbolic_table(1.0, -0.5, 1.0)
    assert np.array_equal(r1, l2) and np.array_equal(l1, r2)
    assert h1.log_p_plus == h2.log_p_minus and h1.log_p_minus == h2.log_p_plus
    h0, r0, l0 = qm.debug_hyperbolic_table(1.0, 0.0, 1.0)
    assert np.array_equal(r0, l0) and h0.log_p_plus == h0.log_p_minus
    assert abs(h0.log_p_plus - math.log(0.5)) < 1e-16


def test_invalid_parameters_rejected():
    for p in [(1.0, 1.0, 1.0), (1.0, -1.5, 1.0), (1.0, 0.0, 0.0), (1.0, 0.0, -1.0), (float("nan"), 0.0, 1.0),
              (float("inf"), 0.0, 1.0), (0.0, 0.0, 1.0)]:
        with pytest.raises(ValueError):
            qm.debug_hyperbolic_table(*p)


@pytest.mark.parametrize("p", [(1.0, 0.999999, 1.0), (1.0, -0.999999, 1.0), (1.0, 0.0, 1e-6), (1e-6, 0.0, 1.0),
                               (1000.0, 0.0, 0.001)], ids=lambda p: "a%g_b%g_d%g" % p)
def test_extreme_parameters(p):
    """Near-degenerate skew (|beta| -> alpha), a near-Laplace and a near-flat
    target: the builder finishes (the peak's exponent is formed without
    cancellation) and its table matches the oracle."""
    h, rr, rl = qm.debug_hyperbolic_table(*p)
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.exponential(1 / (p[0] - p[1]), 30), -rng.exponential(1 / (p[0] + p[1]), 30)])
    ref = oracle.hyperbolic_map(v, *p)
    rel = np.abs(table_eval(h, rr, rl, v) - ref) / np.abs(ref)
    assert rel.max() <= 6e-16, (p, rel.max())
