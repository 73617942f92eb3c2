"""CPU checks of the exponential -> variance-gamma tables for real lambda
(Section 8.2): the recycling-ODE builder's cells, evaluated on the host
exactly as the kernel evaluates them, against the real-lambda oracle (the
Bessel-integral masses solved by bisection, which shares no method with
the builder's ODE), and the header's closed forms."""
import numpy as np
import pytest

import oracle
import paper_0901_0638_amd as qm
from tests.test_hyp_table import table_eval

PARAMS = [(1.5, 1.0, 0.5), (2.5, 2.0, -1.0), (4.25, 1.0, 0.3), (1.05, 1.0, 0.3), (1.2, 2.0, -1.0)]


@pytest.fixture(scope="module", params=PARAMS, ids=lambda p: "l%g_a%g_b%g" % p)
def built(request):
    p = request.param
    lam, a, b = p
    h, rr, rl = qm.debug_vg_table(*p)
    rng = np.random.default_rng(12)
    v = [rng.exponential(1 / (a - b), 120), -rng.exponential(1 / (a + b), 120),
         np.geomspace(1e-20, 1e6, 40), -np.geomspace(1e-20, 1e6, 40), [1e300, -1e300]]
    for S, sgn in ((h.right, 1), (h.left, -1)):
        # the first octaves' cell edges (where the x^(2 lambda - 1) term of
        # the density at 0 bends Q most) and the switch to the large-v form
        edges = np.array([S.v0 * (2.0 ** k * (1 + i / qm.HYP_SUB) - 1) for k in range(5) for i in range(qm.HYP_SUB)])
        edges = edges[edges > 0]
        v += [sgn * edges, sgn * edges * (1 + 1e-9), sgn * np.array([S.v_top, np.nextafter(S.v_top, 0), 3 * S.v_top])]
    v = np.concatenate(v)
    return p, h, rr, rl, v, oracle.vgr_map(v, *p)


def test_table_matches_oracle(built):
    p, h, rr, rl, v, ref = built
    rel = np.abs(table_eval(h, rr, rl, v) - ref) / np.abs(ref)
    assert rel.max() <= 6e-16, (p, rel.max(), v[rel.argmax()])


def test_fp32_cells_match_oracle(built):
    p, h, _, _, v, ref = built
    _, r32, l32 = qm.debug_vg_table(*p, which="f32")
    rel = np.abs(table_eval(h, r32, l32, v, "f32") - ref) / np.abs(ref)
    assert rel.max() <= 1.2e-10, (p, rel.max(), v[rel.argmax()])


def test_header(built):
    p, h, rr, rl, v, ref = built
    lam, a, b = p
    lp, lm = oracle.vgr_masses(*p)
    assert abs(h.log_p_plus - lp) <= 2e-16 and abs(h.log_p_minus - lm) <= 2e-16
    assert h.delta == lam
    for S, rate in ((h.right, a - b), (h.left, a + b)):
        assert S.v0 == h.right.v0 and S.degree == qm.HYP_DEGREE and S.ncell == qm.HYP_SUB * S.noct
        assert abs(S.far_clog - (lam - 1) / rate) <= 1e-15 * max(1.0, (lam - 1) / rate)
        assert S.max_rel_err < 1.2e-16


def test_origin_series_where_the_density_is_not_analytic():
    """2 lambda not an integer: the density's |x|^(2 lambda - 1) at 0 puts
    terms v^(m + n rho) in R near the origin, so both sides' first octave
    holds the series in v and v^rho (row 0 starts with rho); 2 lambda an
    integer (lambda = 1.5, 2.5): plain cells throughout."""
    for p, want in (((1.05, 1.0, 0.3), 1), ((1.2, 2.0, -1.0), 1), ((4.25, 1.0, 0.3), 1), ((1.5, 1.0, 0.5), 0),
                    ((2.5, 2.0, -1.0), 0)):
        for which in ("f64", "f32"):
            h, rr, rl = qm.debug_vg_table(*p, which=which)
            sides = (h.right, h.left) if which == "f64" else (h.right32, h.left32)
            for S, rows in zip(sides, (rr, rl)):
                assert S.origin == want, (p, which)
                if want:
                    assert rows[0][0] == 2 * p[0] - 1


def test_origin_series_near_zero_and_at_v0():
    """lambda = 1.05 and 1.2 (rho = 1.1 and 1.4, far from analytic), 1.25
    (rho = 3/2: v^3 and w^2, v^4 and v w^2 coincide, so only the lower
    family's terms are fitted) and 1.1666... (rho = 4/3: v^4 and w^3): the
    origin series against the oracle from v = 1e-300 up to v0 and across
    the switch to the cells at v0, on both sides."""
    for p in ((1.05, 1.0, 0.3), (1.2, 2.0, -1.0), (1.25, 1.0, 0.3), (7.0 / 6.0, 1.0, -0.2)):
        h, rr, rl = qm.debug_vg_table(*p)
        v0 = h.right.v0
        v = np.concatenate([np.geomspace(1e-300, v0, 300), v0 * np.array([0.999999, 1.0, 1.000001, 1.3, 2.0])])
        v = np.concatenate([v, -v])
        ref = oracle.vgr_map(v, *p)
        rel = np.abs(table_eval(h, rr, rl, v) - ref) / np.abs(ref)
        assert rel.max() <= 6e-16, (p, rel.max(), v[rel.argmax()])
