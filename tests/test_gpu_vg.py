"""GPU parity: the exponential -> variance-gamma map (Section 8.2) against
the oracle: integer lambda (closed-form sides; vg.c) and real lambda (the
recycling-ODE sides; the Bessel-integral oracle vg_real.c)."""
import math

import numpy as np
import pytest

import oracle
import qm_inputs as qi
from tests._tol import RTOL_F32, RTOL_F64, as_f32_output, assert_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_0901_0638_amd as qm  # noqa: E402

PARAMS = [(1, 1.0, 0.0), (2, 1.0, 0.0), (2, 1.0, 0.5), (3, 2.0, -1.0), (5, 1.0, 0.3), (8, 1.0, 0.0)]
REAL = [(1.5, 1.0, 0.5), (2.5, 2.0, -1.0), (4.25, 1.0, 0.3), (1.05, 1.0, 0.3), (1.2, 2.0, -1.0)]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = qm.Context(0)
    yield c
    c.close()


def run(ctx, v, p, mu=0.0, dtype=torch.float64):
    d = torch.from_numpy(np.ascontiguousarray(v)).to(dtype).cuda()
    x = torch.empty_like(d)
    qm.qm_recycle_exp_to_vg(ctx, d, x, *p, mu=mu)
    torch.cuda.synchronize()
    return x.cpu().numpy()


@pytest.mark.parametrize("p", PARAMS, ids=lambda p: "l%d_a%g_b%g" % p)
def test_vg_f64_base_samples_and_far_range(ctx, p):
    lam, a, b = p
    lp, lm = oracle.vg_masses(*p)
    v = qi.two_sided_exponentials(3, 4, 20001, a - b, a + b, math.exp(lm))
    far = np.concatenate([np.geomspace(1e-300, 1e300, 300), -np.geomspace(1e-300, 1e300, 300),
                          np.geomspace(30 / (a - b), 1e7, 100), -np.geomspace(30 / (a + b), 1e7, 100)])
    v = np.concatenate([v, far])
    assert_close(run(ctx, v, p), oracle.vg_map(v, *p), RTOL_F64, "vg %r" % (p,))


@pytest.mark.parametrize("p", PARAMS[1:4], ids=lambda p: "l%d_a%g_b%g" % p)
def test_vg_f32(ctx, p):
    lam, a, b = p
    lp, lm = oracle.vg_masses(*p)
    v = qi.two_sided_exponentials(5, 4, 20003, a - b, a + b, math.exp(lm)).astype(np.float32)
    ref = as_f32_output(oracle.vg_map(v.astype(np.float64), *p))
    got = run(ctx, v, p, dtype=torch.float32)
    assert_close(got, ref, RTOL_F32, "vg f32 %r" % (p,))


def test_vg_specials_location_and_api(ctx):
    p = (3, 1.0, 0.25)
    got = run(ctx, np.array([0.0, np.inf, -np.inf, np.nan]), p)
    assert got[0] == 0 and got[1] == np.inf and got[2] == -np.inf and np.isnan(got[3])
    v = np.abs(qi.two_sided_exponentials(6, 4, 3001, 0.75, 1.25, 0.3))
    # mu > 0 with v >= 0: no cancellation in mu + Q
    assert_close(run(ctx, v, p, mu=1.5), 1.5 + oracle.vg_map(v, *p), RTOL_F64, "mu")
    lp, lm = qm.qm_vg_masses(ctx, *p)
    olp, olm = oracle.vg_masses(*p)
    assert abs(lp - olp) <= 1e-15 and abs(lm - olm) <= 1e-15
    d = torch.zeros(8, dtype=torch.float64, device="cuda")
    for bad in [(0.5, 1.0, 0.0), (0.99, 1.0, 0.0), (9, 1.0, 0.0), (8.5, 1.0, 0.0), (2, 1.0, 1.5)]:
        with pytest.raises(qm.QMError):
            qm.qm_recycle_exp_to_vg(ctx, d, d, *bad)


def test_vg_full_size_sampled(ctx):
    """2^26 base samples of (lambda, alpha, beta) = (2, 1, 0.5) in one launch
    (the benchmark's size); 3000 sampled outputs and the extremes against the
    oracle, and the map's monotonicity over the whole output."""
    p = (2, 1.0, 0.5)
    lp, lm = oracle.vg_masses(*p)
    n = 1 << 26
    v = qi.two_sided_exponentials(2, 3, n, p[1] - p[2], p[1] + p[2], math.exp(lm))
    d = torch.from_numpy(v).cuda()
    x = torch.empty_like(d)
    qm.qm_recycle_exp_to_vg(ctx, d, x, *p)
    torch.cuda.synchronize()
    got = x.cpu().numpy()
    rng = np.random.default_rng(19)
    idx = np.concatenate([rng.integers(0, n, 3000), [np.argmax(v), np.argmin(v), n - 1]])
    assert_close(got[idx], oracle.vg_map(v[idx], *p), RTOL_F64, "sampled")
    order = np.argsort(v, kind="stable")
    assert np.all(np.diff(got[order]) >= 0)


def test_vg_ragged_misaligned_inplace_and_request_checks(ctx):
    """Sizes around the vector width and a workgroup's tile, an input one
    element off 16-byte alignment, in-place use, n = 0; and the request
    checks the entry point shares with batches (dtype/mode pairs, mu, partial
    overlap)."""
    p = (3, 2.0, -1.0)
    lp, lm = oracle.vg_masses(*p)
    for n in (1, 2, 3, 7, 255, 257, 1025):
        v = qi.two_sided_exponentials(8, n, n, 3.0, 1.0, math.exp(lm))
        assert_close(run(ctx, v, p), oracle.vg_map(v, *p), RTOL_F64, "n=%d" % n)
    v = qi.two_sided_exponentials(9, 1, 3001, 3.0, 1.0, math.exp(lm))
    ref = oracle.vg_map(v, *p)
    base = torch.from_numpy(np.concatenate([[0.0], v])).cuda()
    out = torch.empty(3001, dtype=torch.float64, device="cuda")
    qm.qm_recycle_exp_to_vg(ctx, base[1:], out, *p)
    d = torch.from_numpy(v).cuda()
    qm.qm_recycle_exp_to_vg(ctx, d, d, *p)
    torch.cuda.synchronize()
    assert_close(out.cpu().numpy(), ref, RTOL_F64, "misaligned")
    assert_close(d.cpu().numpy(), ref, RTOL_F64, "in place")
    z = torch.empty(0, dtype=torch.float64, device="cuda")
    qm.qm_recycle_exp_to_vg(ctx, z, z, *p)
    f = torch.zeros(16, dtype=torch.float32, device="cuda")
    buf = torch.zeros(17, dtype=torch.float64, device="cuda")
    for call in (lambda: qm.qm_recycle_exp_to_vg(ctx, d, d, *p, mode=qm.QM_F32_REFINE),
                 lambda: qm.qm_recycle_exp_to_vg(ctx, d, d, *p, mode=qm.QM_PAPER),
                 lambda: qm.qm_recycle_exp_to_vg(ctx, f, f, *p, mode=qm.QM_PLAIN),
                 lambda: qm.qm_recycle_exp_to_vg(ctx, d, d, *p, mu=float("inf")),
                 lambda: qm.qm_recycle_exp_to_vg(ctx, buf[:16], buf[1:], *p)):
        with pytest.raises(qm.QMError):
            call()
    torch.cuda.synchronize()


@pytest.mark.parametrize("p", REAL, ids=lambda p: "l%g_a%g_b%g" % p)
def test_vg_real_lambda_f64(ctx, p):
    """Real lambda: base samples with the target's masses, the first octave
    (where the density's x^(2 lambda - 1) term at 0 bends Q; for 2 lambda
    not an integer the origin series on the far path), across v0, and the
    far range out to 1e300."""
    lam, a, b = p
    lp, lm = oracle.vgr_masses(*p)
    v = qi.two_sided_exponentials(7, 4, 3001, a - b, a + b, math.exp(lm))
    far = np.concatenate([np.geomspace(1e-300, 1e300, 120), -np.geomspace(1e-300, 1e300, 120),
                          np.geomspace(1e-7, 1e-2, 60), -np.geomspace(1e-7, 1e-2, 60),
                          np.geomspace(1e-3, 0.03, 64), -np.geomspace(1e-3, 0.03, 64),
                          np.geomspace(30 / (a - b), 1e7, 40), -np.geomspace(30 / (a + b), 1e7, 40)])
    v = np.concatenate([v, far])
    print("case: vg real lambda f64 %r, %d elements" % (p, v.size), flush=True)
    assert_close(run(ctx, v, p), oracle.vgr_map(v, *p), RTOL_F64, "vg real %r" % (p,))


@pytest.mark.parametrize("p", REAL, ids=lambda p: "l%g_a%g_b%g" % p)
def test_vg_real_lambda_f32(ctx, p):
    lam, a, b = p
    lp, lm = oracle.vgr_masses(*p)
    v = qi.two_sided_exponentials(8, 4, 3003, a - b, a + b, math.exp(lm)).astype(np.float32)
    ref = as_f32_output(oracle.vgr_map(v.astype(np.float64), *p))
    got = run(ctx, v, p, dtype=torch.float32)
    assert_close(got, ref, RTOL_F32, "vg real f32 %r" % (p,))


def test_vg_real_lambda_batch_equals_single(ctx):
    """A real-lambda request in a batch beside an integer-lambda one: bitwise
    the single call."""
    reqs, cases = [], []
    for p in ((2.5, 2.0, -1.0), (2, 1.0, 0.5)):
        x = qi.two_sided_exponentials(9, 5, 4097, p[1] - p[2], p[1] + p[2], 0.4)
        d = torch.from_numpy(x).cuda()
        o = torch.full_like(d, float("nan"))
        reqs.append(qm.make_request(qm.QM_EXP_TO_VG, d, o, nu=p[0], hyperbolic=(p[1], p[2], 0.0)))
        cases.append((p, d, o))
    qm.qm_run_batch(ctx, reqs, device_tensor=cases[0][1])
    torch.cuda.synchronize()
    for p, d, o in cases:
        ref = torch.empty_like(d)
        qm.qm_recycle_exp_to_vg(ctx, d, ref, *p)
        torch.cuda.synchronize()
        assert torch.equal(o, ref), p
