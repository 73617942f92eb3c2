"""GPU parity: the exponential -> hyperbolic recycling map (Section 8.1)
against the oracle."""
import math

import numpy as np
import pytest

import oracle
import qm_inputs as qi
from tests._tol import RTOL_F32, RTOL_F64, as_f32_output, assert_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_0901_0638_amd as qm  # noqa: E402

PARAMS = [(1.0, 0.0, 1.0), (1.0, 0.5, 1.0), (2.0, -1.5, 0.3), (1.0, 0.9, 5.0), (1.0, 0.0, 0.001),
          (50.0, 10.0, 0.1)]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = qm.Context(0)
    yield c
    c.close()


def run_h(ctx, v, p, mu=0.0, dtype=torch.float64):
    d = torch.from_numpy(np.ascontiguousarray(v)).to(dtype).cuda()
    x = torch.empty_like(d)
    qm.qm_recycle_exp_to_hyperbolic(ctx, d, x, *p, mu=mu)
    torch.cuda.synchronize()
    return x.cpu().numpy()


def base_samples(p, n, seed=0):
    lp, lm, _ = oracle.hyperbolic_masses(*p)
    v = qi.recycle_two_sided(n + seed, p[0], p[1], math.exp(lm))
    return v[seed:]


@pytest.mark.parametrize("p", PARAMS, ids=lambda p: "a%g_b%g_d%g" % p)
def test_hyperbolic_f64_base_samples(ctx, p):
    """Samples of the base (rates alpha -+ beta, the target's masses): several
    tiles of 256 x 2 elements and a ragged tail."""
    v = base_samples(p, 20001)
    rep = assert_close(run_h(ctx, v, p), oracle.hyperbolic_map(v, *p), RTOL_F64, "p=%r" % (p,))
    print(p, rep)


@pytest.mark.parametrize("p", PARAMS, ids=lambda p: "a%g_b%g_d%g" % p)
def test_hyperbolic_f64_far_range(ctx, p):
    """Global-memory cells (64/rate < |v| < v_top), the large-v form beyond,
    and magnitudes from the smallest subnormal to 1e300."""
    h, _, _ = qm.debug_hyperbolic_table(*p)
    pts = [np.geomspace(5e-324, 1e300, 700)]
    for S, sgn, rate in ((h.right, 1.0, p[0] - p[1]), (h.left, -1.0, p[0] + p[1])):
        pts.append(sgn * np.geomspace(32 / rate, 4 * S.v_top, 300))
        pts.append(sgn * np.array([S.v_top, np.nextafter(S.v_top, 0), S.v0, np.nextafter(S.v0, 0)]))
    v = np.concatenate(pts + [-pts[0]])
    assert_close(run_h(ctx, v, p), oracle.hyperbolic_map(v, *p), RTOL_F64, "far p=%r" % (p,))


def test_hyperbolic_specials(ctx):
    p = PARAMS[1]
    v = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 1e-300, -1e-300, 5e-324])
    got = run_h(ctx, v, p)
    assert got[0] == 0.0 and got[1] == 0.0
    assert got[2] == np.inf and got[3] == -np.inf and np.isnan(got[4])
    assert_close(got[5:], oracle.hyperbolic_map(v[5:], *p), RTOL_F64, "tiny")


def test_hyperbolic_location(ctx):
    """x = mu + Q(v): for v >= 0 (no cancellation) within the same tolerance."""
    p = PARAMS[1]
    v = np.abs(base_samples(p, 4097, 3))
    ref = 2.5 + oracle.hyperbolic_map(v, *p)
    assert_close(run_h(ctx, v, p, mu=2.5), ref, RTOL_F64, "mu")


@pytest.mark.parametrize("p", PARAMS[:4], ids=lambda p: "a%g_b%g_d%g" % p)
def test_hyperbolic_f32(ctx, p):
    v = base_samples(p, 20003, 5).astype(np.float32)
    v = np.concatenate([v, np.float32([0.0, 1e-30, -1e-30, 3e38, -3e38, np.inf])])
    ref = as_f32_output(oracle.hyperbolic_map(v.astype(np.float64), *p))
    got = run_h(ctx, v, p, dtype=torch.float32)
    assert got.dtype == np.float32
    assert_close(got, ref, RTOL_F32, "f32 p=%r" % (p,))


def test_hyperbolic_ragged_misaligned_inplace(ctx):
    p = PARAMS[2]
    for n in (1, 2, 3, 7, 255, 257, 1025):
        v = base_samples(p, n, 11)
        assert_close(run_h(ctx, v, p), oracle.hyperbolic_map(v, *p), RTOL_F64, "n=%d" % n)
    v = base_samples(p, 3001, 13)
    ref = oracle.hyperbolic_map(v, *p)
    base = torch.from_numpy(np.concatenate([[0.0], v])).cuda()
    out = torch.empty(3001, dtype=torch.float64, device="cuda")
    qm.qm_recycle_exp_to_hyperbolic(ctx, base[1:], out, *p)
    d = torch.from_numpy(v).cuda()
    qm.qm_recycle_exp_to_hyperbolic(ctx, d, d, *p)
    torch.cuda.synchronize()
    assert_close(out.cpu().numpy(), ref, RTOL_F64, "misaligned")
    assert_close(d.cpu().numpy(), ref, RTOL_F64, "in place")
    z = torch.empty(0, dtype=torch.float64, device="cuda")
    qm.qm_recycle_exp_to_hyperbolic(ctx, z, z, *p)


def test_hyperbolic_full_size_sampled(ctx):
    """2^26 base samples of the Section 8.1 illustration (alpha = delta = 1,
    beta = 0) in one launch; 3000 sampled outputs and the extremes against
    the oracle, and the map's monotonicity over the whole output."""
    p = qi.HYPERBOLIC_PARAMS
    n = 1 << 26
    v = qi.recycle_two_sided(n, p[0], p[1], 0.5)
    d = torch.from_numpy(v).cuda()
    x = torch.empty_like(d)
    qm.qm_recycle_exp_to_hyperbolic(ctx, d, x, *p)
    torch.cuda.synchronize()
    got = x.cpu().numpy()
    rng = np.random.default_rng(17)
    idx = np.concatenate([rng.integers(0, n, 3000), [np.argmax(v), np.argmin(v), n - 1]])
    assert_close(got[idx], oracle.hyperbolic_map(v[idx], *p), RTOL_F64, "sampled")
    order = np.argsort(v, kind="stable")
    assert np.all(np.diff(got[order]) >= 0)
    assert np.array_equal(np.sign(got), np.sign(v))


def test_hyperbolic_masses_api(ctx):
    for p in PARAMS:
        lp, lm = qm.qm_hyperbolic_masses(ctx, *p)
        olp, olm, _ = oracle.hyperbolic_masses(*p)
        assert abs(lp - olp) <= 1e-15 and abs(lm - olm) <= 1e-15, p


def test_hyperbolic_errors(ctx):
    d = torch.zeros(16, dtype=torch.float64, device="cuda")
    for bad in [(1.0, 1.0, 1.0), (1.0, 0.0, 0.0), (float("nan"), 0.0, 1.0)]:
        with pytest.raises(qm.QMError):
            qm.qm_recycle_exp_to_hyperbolic(ctx, d, d, *bad)
        with pytest.raises(qm.QMError):
            qm.qm_hyperbolic_masses(ctx, *bad)
    with pytest.raises(qm.QMError):
        qm.qm_recycle_exp_to_hyperbolic(ctx, d, d, 1.0, 0.0, 1.0, mu=float("inf"))
    with pytest.raises(qm.QMError):
        qm.qm_recycle_exp_to_hyperbolic(ctx, d, d, 1.0, 0.0, 1.0, mode=qm.QM_PAPER)
    with pytest.raises(qm.QMError):
        qm.qm_recycle_exp_to_hyperbolic(ctx, d, d, 1.0, 0.0, 1.0, mode=qm.QM_F32_REFINE)
    f = torch.zeros(16, dtype=torch.float32, device="cuda")
    with pytest.raises(qm.QMError):
        qm.qm_recycle_exp_to_hyperbolic(ctx, f, f, 1.0, 0.0, 1.0, mode=qm.QM_PLAIN)
    buf = torch.zeros(17, dtype=torch.float64, device="cuda")
    with pytest.raises(qm.QMError):   # input and output partially overlap
        qm.qm_recycle_exp_to_hyperbolic(ctx, buf[:16], buf[1:], 1.0, 0.0, 1.0)
    torch.cuda.synchronize()
