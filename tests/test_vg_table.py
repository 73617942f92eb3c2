"""CPU checks of the exponential -> variance-gamma tables (Section 8.2,
integer lambda): the host evaluation of the tables, exactly as the kernel
evaluates them (the hyperbolic table format, with the log form of the
large-v expansion), against the oracle, and the header's closed forms."""
import math

import numpy as np
import pytest

import oracle
import paper_0901_0638_amd as qm
from tests.test_hyp_table import table_eval

PARAMS = [(1, 1.0, 0.0), (2, 1.0, 0.0), (2, 1.0, 0.5), (3, 2.0, -1.0), (5, 1.0, 0.3), (8, 1.0, 0.0)]


@pytest.fixture(scope="module", params=PARAMS, ids=lambda p: "l%d_a%g_b%g" % p)
def built(request):
    p = request.param
    lam, a, b = p
    h, rr, rl = qm.debug_vg_table(*p)
    rng = np.random.default_rng(11)
    v = [rng.exponential(1 / (a - b), 150), -rng.exponential(1 / (a + b), 150),
         np.geomspace(1e-12, 1e9, 40), -np.geomspace(1e-12, 1e9, 40), [1e300, -1e300]]
    for S, sgn in ((h.right, 1), (h.left, -1)):
        edges = np.array([S.v0 * (2.0 ** k * (1 + i / qm.HYP_SUB) - 1) for k in range(7) for i in range(qm.HYP_SUB)])
        edges = edges[edges > 0]
        v += [sgn * edges, sgn * np.array([S.v_top, np.nextafter(S.v_top, 0), 3 * S.v_top])]
    v = np.concatenate(v)
    return p, h, rr, rl, v, oracle.vg_map(v, *p)


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
    lp, lm = oracle.vg_masses(*p)
    assert abs(h.log_p_plus - lp) <= 2e-16 and abs(h.log_p_minus - lm) <= 2e-16
    assert h.delta == lam
    for S, rate in ((h.right, a - b), (h.left, a + b)):
        assert S.v0 == h.right.v0 and S.degree == qm.HYP_DEGREE and S.ncell == qm.HYP_SUB * S.noct
        # the power of x in the tail, x^(lambda-1), gives the log term (lambda-1)/rate log Q
        assert abs(S.far_clog - (lam - 1) / rate) <= 1e-15 * max(1.0, (lam - 1) / rate)
        assert S.max_rel_err < 1.2e-16


def test_lambda_one_table_is_the_identity():
    h, rr, rl = qm.debug_vg_table(1, 1.3, 0.4)
    v = np.concatenate([np.geomspace(1e-300, 1e300, 200), -np.geomspace(1e-300, 1e300, 200)])
    assert np.max(np.abs(table_eval(h, rr, rl, v) / v - 1)) <= 2.3e-16


def test_invalid_lambda_rejected():
    for p in [(0.5, 1.0, 0.0), (0, 1.0, 0.0), (9, 1.0, 0.0), (8.5, 1.0, 0.0), (2, 1.0, 1.0), (2, float("inf"), 0.0)]:
        with pytest.raises(ValueError):
            qm.debug_vg_table(*p)
