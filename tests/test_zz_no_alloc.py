"""GPU: the allocation-free batch entry point (qm_run_batch_noalloc).

Its outputs must be bitwise those of qm_run_batch on the same requests, on
two calls in a row on one stream (the second with fewer and smaller
requests, so that it reuses the device descriptor array the first left
behind), and within tolerance of the oracle.  Requests beyond the limit,
and requests whose table the context does not hold, are rejected before
anything is launched."""
import numpy as np
import pytest

import oracle
import qm_inputs as qi
from tests._tol import RTOL_F32, RTOL_F64, assert_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_0901_0638_amd as qm  # noqa: E402

KIND = {"nq_f32_refine": (qm.QM_NORMAL_QUANTILE, qm.QM_F32_REFINE),
        "nq_f64": (qm.QM_NORMAL_QUANTILE, qm.QM_PLAIN),
        "student_f64": (qm.QM_STUDENT_T, qm.QM_PLAIN),
        "exp_f64": (qm.QM_EXP_TO_NORMAL, qm.QM_PLAIN)}
HYP = (1.0, 0.5, 1.0)
VG = (2.0, 1.0, -0.5)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = qm.Context(0)
    yield c
    c.close()


def requests(seed, count, lo, hi):
    """A request mix plus one hyperbolic and one variance-gamma request;
    inputs on the device, two NaN-filled outputs per request (one for each
    entry point)."""
    mix = qi.request_mix(seed, count, lo, hi)
    ins, xs, refs = [], [], []
    for r in mix:
        x = qi.request_input(seed, r)
        xs.append((r, x))
        ins.append(torch.from_numpy(x).cuda())
    lp, lm, _ = oracle.hyperbolic_masses(*HYP)
    xh = qi.two_sided_exponentials(seed, 7, 30001, HYP[0] - HYP[1], HYP[0] + HYP[1], np.exp(lm))
    xv = qi.two_sided_exponentials(seed, 8, 20003, VG[1] - VG[2], VG[1] + VG[2], 0.4)
    xs += [({"kind": "hyp"}, xh), ({"kind": "vg"}, xv)]
    ins += [torch.from_numpy(xh).cuda(), torch.from_numpy(xv).cuda()]
    outs_a = [torch.full_like(d, float("nan")) for d in ins]
    outs_b = [torch.full_like(d, float("nan")) for d in ins]

    def reqs(outs):
        q = []
        for (r, x), d, o in zip(xs, ins, outs):
            if r["kind"] == "hyp":
                q.append(qm.make_request(qm.QM_EXP_TO_HYPERBOLIC, d, o, hyperbolic=HYP))
            elif r["kind"] == "vg":
                q.append(qm.make_request(qm.QM_EXP_TO_VG, d, o, nu=VG[0], hyperbolic=(VG[1], VG[2], 0.0)))
            else:
                kind, mode = KIND[r["kind"]]
                q.append(qm.make_request(kind, d, o, mode=mode, nu=r["nu"]))
        return q

    return xs, ins, outs_a, outs_b, reqs(outs_a), reqs(outs_b)


def oracle_of(r, x):
    k = r["kind"]
    if k == "hyp":
        return oracle.hyperbolic_map(x, *HYP)
    if k == "vg":
        return oracle.vg_map(x, *VG)
    if k in ("nq_f32_refine", "nq_f64"):
        return oracle.norm_quantile(x.astype(np.float64))
    if k == "student_f64":
        return oracle.student_t_map(x, r["nu"])
    return oracle.exp_to_normal(x)


def check(xs, outs_a, outs_b, rng):
    for (r, x), a, b in zip(xs, outs_a, outs_b):
        ha, hb = a.cpu().numpy(), b.cpu().numpy()
        assert np.array_equal(ha.view(np.uint8), hb.view(np.uint8)), ("not bitwise qm_run_batch's", r)
        if ha.size:
            idx = np.unique(np.concatenate([rng.integers(0, ha.size, 48), [ha.size - 1]]))
            rtol = RTOL_F32 if ha.dtype == np.float32 else RTOL_F64
            assert_close(ha[idx], oracle_of(r, x[idx]), rtol, str(r))


def test_noalloc_equals_run_batch_twice(ctx):
    stream = torch.cuda.current_stream()
    first = requests(11, 300, 10, 17)
    second = requests(12, 40, 8, 12)
    for xs, ins, outs_a, outs_b, reqs_a, reqs_b in (first, second):
        print("case: qm_run_batch reference, %d requests" % len(reqs_a), flush=True)
        qm.qm_run_batch(ctx, reqs_a, stream=stream.cuda_stream)   # builds every table the mix needs
    torch.cuda.synchronize()
    # two allocation-free calls back to back on one stream, no sync between
    for xs, ins, outs_a, outs_b, reqs_a, reqs_b in (first, second):
        print("case: qm_run_batch_noalloc, %d requests" % len(reqs_b), flush=True)
        qm.qm_run_batch_noalloc(ctx, reqs_b, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    for xs, ins, outs_a, outs_b, reqs_a, reqs_b in (first, second):
        check(xs, outs_a, outs_b, rng)


def test_noalloc_rejects_before_launch(ctx):
    n = qm.QM_BATCH_NOALLOC_MAX_REQUESTS + 1
    d = torch.full((n,), 0.5, dtype=torch.float64, device="cuda")
    o = torch.full_like(d, float("nan"))
    reqs = [qm.qm_request(qm.QM_NORMAL_QUANTILE, qm.QM_F64, qm.QM_PLAIN, 0, 0.0, d.data_ptr() + 8 * i,
                          o.data_ptr() + 8 * i, 1, 0) for i in range(n)]
    with pytest.raises(qm.QMError) as e:
        qm.qm_run_batch_noalloc(ctx, reqs, device_tensor=d)
    assert e.value.status == qm.QM_E_INVAL
    # a Student t request whose table was never built in this context
    z = torch.zeros(16, dtype=torch.float64, device="cuda")
    t = torch.full_like(z, float("nan"))
    with pytest.raises(qm.QMError) as e:
        qm.qm_run_batch_noalloc(ctx, [qm.make_request(qm.QM_STUDENT_T, z, t, nu=37.25)], device_tensor=z)
    assert e.value.status == qm.QM_E_INVAL
    torch.cuda.synchronize()
    assert torch.isnan(o).all() and torch.isnan(t).all()      # nothing ran
    # at the limit exactly, it runs
    reqs = reqs[:-1]
    qm.qm_run_batch_noalloc(ctx, reqs, device_tensor=d)
    torch.cuda.synchronize()
    got = o[:-1].cpu().numpy()
    assert np.all(got == 0.0) and np.isnan(o[-1].item())     # w(1/2) = 0; the last was not a request
