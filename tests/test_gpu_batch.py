"""GPU: the persistent batch launch and the serving loop.  Every request's
output must be bitwise identical to the single-request call with the same
kind, dtype and mode, and within tolerance of the oracle."""
import time

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


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = qm.Context(0, hbm_budget_bytes=256 << 20)
    yield c
    c.close()


def single(ctx, kind, mode, nu, inp):
    out = torch.empty_like(inp)
    if kind == qm.QM_NORMAL_QUANTILE:
        qm.qm_normal_quantile(ctx, inp, out, mode)
    elif kind == qm.QM_STUDENT_T:
        qm.qm_recycle_student_t(ctx, inp, out, nu, mode)
    else:
        qm.qm_recycle_exp_to_normal(ctx, inp, out, mode)
    return out


def oracle_of(req, x):
    k = req["kind"]
    if k in ("nq_f32_refine", "nq_f64"):
        return oracle.norm_quantile(x.astype(np.float64))
    if k == "student_f64":
        return oracle.student_t_map(x, req["nu"])
    return oracle.exp_to_normal(x)


def build(seed, count, lo, hi, extra_sizes=()):
    reqs = qi.request_mix(seed, count, lo, hi)
    for i, n in enumerate(extra_sizes):
        reqs[i % len(reqs)]["n"] = n
    ins, outs, qreqs = [], [], []
    for r in reqs:
        x = qi.request_input(seed, r)
        d = torch.from_numpy(x).cuda()
        o = torch.full_like(d, float("nan"))
        kind, mode = KIND[r["kind"]]
        qreqs.append(qm.qm_request(kind, qm.QM_F32 if x.dtype == np.float32 else qm.QM_F64, mode, 0,
                                   r["nu"], d.data_ptr(), o.data_ptr(), x.size, 0))
        ins.append(d)
        outs.append(o)
    return reqs, ins, outs, qreqs


def check_against_single_and_oracle(ctx, reqs, ins, outs, rng):
    for r, d, o, in zip(reqs, ins, outs):
        kind, mode = KIND[r["kind"]]
        ref_single = single(ctx, kind, mode, r["nu"], d)
        torch.cuda.synchronize()
        a, b = o.cpu().numpy(), ref_single.cpu().numpy()
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), ("not bitwise equal", r)
        if a.size:
            idx = np.unique(rng.integers(0, a.size, 64))
            x = d.cpu().numpy()[idx]
            rtol = RTOL_F32 if a.dtype == np.float32 else RTOL_F64
            assert_close(a[idx], oracle_of(r, x), rtol, str(r))


def test_batch_mixed_bitwise_equal_to_single(ctx):
    edge = (0, 1, 3, 32767, 32768, 32769, 65537)
    reqs, ins, outs, qreqs = build(3, 160, 10, 16, edge)
    qm.qm_run_batch(ctx, qreqs, device_tensor=ins[0])
    torch.cuda.synchronize()
    check_against_single_and_oracle(ctx, reqs, ins, outs, np.random.default_rng(0))


def test_batch_misaligned_and_repeat(ctx):
    x = qi.uniform53(3, 7, 100001)
    base = torch.from_numpy(np.concatenate([[0.5], x])).cuda()
    out = torch.empty(100001, dtype=torch.float64, device="cuda")
    r = qm.qm_request(qm.QM_NORMAL_QUANTILE, qm.QM_F64, qm.QM_PLAIN, 0, 0.0, base.data_ptr() + 8,
                      out.data_ptr(), 100001, 0)
    for _ in range(3):
        qm.qm_run_batch(ctx, [r, r], device_tensor=base)
    torch.cuda.synchronize()
    assert_close(out.cpu().numpy(), oracle.norm_quantile(x), RTOL_F64, "misaligned batch")


def test_batch_validation_rejects_whole_batch(ctx):
    reqs, ins, outs, qreqs = build(4, 8, 10, 12)
    bad = qm.qm_request(qm.QM_STUDENT_T, qm.QM_F64, qm.QM_PLAIN, 0, 0.1, ins[0].data_ptr(), outs[0].data_ptr(), 10, 0)
    with pytest.raises(qm.QMError) as e:
        qm.qm_run_batch(ctx, qreqs + [bad], device_tensor=ins[0])
    assert e.value.status == qm.QM_E_INVAL
    torch.cuda.synchronize()
    for o in outs:
        assert torch.isnan(o).all(), "nothing may run when validation fails"


def test_serving_results_equal_single_calls(ctx):
    reqs, ins, outs, qreqs = build(5, 120, 10, 18)
    torch.cuda.synchronize()        # inputs and NaN fills complete before submit
    tickets = [qm.qm_submit(ctx, q) for q in qreqs]
    deadline = time.time() + 60
    pending = set(tickets)
    while pending and time.time() < deadline:
        pending = {t for t in pending if qm.qm_poll(ctx, t) == qm.QM_PENDING}
        time.sleep(0.001)
    assert not pending, "requests did not complete"
    for t in tickets:
        assert qm.qm_poll(ctx, t) == qm.QM_OK
    lat = qm.qm_serving_latencies(ctx)
    assert len(lat) >= len(tickets)
    check_against_single_and_oracle(ctx, reqs, ins, outs, np.random.default_rng(1))


def test_serving_errors(ctx):
    with pytest.raises(qm.QMError) as e:
        qm.qm_poll(ctx, 10 ** 12)
    assert e.value.status == qm.QM_E_TICKET
    d = torch.zeros(64 << 20, dtype=torch.float64, device="cuda")   # 512 MiB in + out > 256 MiB budget
    big = qm.make_request(qm.QM_NORMAL_QUANTILE, d, d)
    with pytest.raises(qm.QMError) as e:
        qm.qm_submit(ctx, big)
    assert e.value.status == qm.QM_E_INVAL


def test_serving_shutdown_with_work_in_flight():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = qm.Context(0, hbm_budget_bytes=64 << 20)
    xs = [torch.from_numpy(qi.uniform53(6, i, 1 << 20)).cuda() for i in range(16)]
    ys = [torch.empty_like(x) for x in xs]
    torch.cuda.synchronize()
    for x, y in zip(xs, ys):
        qm.qm_submit(c, qm.make_request(qm.QM_NORMAL_QUANTILE, x, y))
    t0 = time.time()
    c.close()                       # drains admitted work, fails the rest
    assert time.time() - t0 < 30
    torch.cuda.synchronize()


ALL_COMBOS = [
    (qm.QM_NORMAL_QUANTILE, np.float64, qm.QM_PLAIN), (qm.QM_NORMAL_QUANTILE, np.float64, qm.QM_PAPER),
    (qm.QM_NORMAL_QUANTILE, np.float32, qm.QM_F32_REFINE), (qm.QM_NORMAL_QUANTILE, np.float32, qm.QM_PAPER),
    (qm.QM_NORMAL_QUANTILE, np.float32, qm.QM_PLAIN), (qm.QM_EXP_TO_NORMAL, np.float64, qm.QM_PLAIN),
    (qm.QM_EXP_TO_NORMAL, np.float64, qm.QM_PAPER), (qm.QM_EXP_TO_NORMAL, np.float32, qm.QM_F32_REFINE),
    (qm.QM_EXP_TO_NORMAL, np.float32, qm.QM_PLAIN),
    (qm.QM_STUDENT_T, np.float64, qm.QM_PLAIN), (qm.QM_STUDENT_T, np.float32, qm.QM_F32_REFINE),
]


def combo_input(kind, dtype, n, seed):
    if kind == qm.QM_NORMAL_QUANTILE:
        x = qi.mixture(seed, 0, n, dtype, 0.1, 1e-300 if dtype == np.float64 else 1e-37)
    elif kind == qm.QM_EXP_TO_NORMAL:
        x = qi.exponentials(seed, 1, n).astype(dtype)
        x[::7] *= -1
    else:
        x = qi.normals(seed, 2, n).astype(dtype)
    return np.ascontiguousarray(x)


def test_batch_every_kind_dtype_mode_bitwise(ctx):
    """One batch holding every supported (kind, dtype, mode), several nu and
    ragged sizes: each output equals its single call bit for bit."""
    rng = np.random.default_rng(17)
    qreqs, cases = [], []
    for c, (kind, dtype, mode) in enumerate(ALL_COMBOS):
        for j, n in enumerate((1, 777, 32768 + 5, 70001)):
            x = combo_input(kind, dtype, n, 40 + 4 * c + j)
            d = torch.from_numpy(x).cuda()
            o = torch.full_like(d, float("nan"))
            nu = float(rng.choice([1.0, 2.5, 4.0, 17.0, float("inf")])) if kind == qm.QM_STUDENT_T else 0.0
            qreqs.append(qm.qm_request(kind, qm.QM_F32 if dtype == np.float32 else qm.QM_F64, mode, 0, nu,
                                       d.data_ptr(), o.data_ptr(), n, 0))
            cases.append((kind, mode, nu, d, o))
    qm.qm_run_batch(ctx, qreqs, device_tensor=cases[0][3])
    torch.cuda.synchronize()
    for kind, mode, nu, d, o in cases:
        ref = single(ctx, kind, mode, nu, d)
        torch.cuda.synchronize()
        a, b = o.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (kind, mode, nu, a.size)


def test_batch_full_size_mix_sampled(ctx):
    """The 4096-request mix at its full size (sizes 2^10..2^22, about 2.1e9
    elements, 27 GB), one persistent launch as the benchmark times it;
    sampled outputs of every request against the oracle."""
    reqs = qi.request_mix(3, 4096, 10, 22)
    kinds = {"nq_f32_refine": (qm.QM_NORMAL_QUANTILE, qm.QM_F32, qm.QM_F32_REFINE),
             "nq_f64": (qm.QM_NORMAL_QUANTILE, qm.QM_F64, qm.QM_PLAIN),
             "student_f64": (qm.QM_STUDENT_T, qm.QM_F64, qm.QM_PLAIN),
             "exp_f64": (qm.QM_EXP_TO_NORMAL, qm.QM_F64, qm.QM_PLAIN)}
    ins, outs, qreqs = [], [], []
    for r in reqs:
        x = qi.request_input(3, r)
        d = torch.from_numpy(x).cuda()
        o = torch.empty_like(d)
        kind, dt, mode = kinds[r["kind"]]
        qreqs.append(qm.qm_request(kind, dt, mode, 0, r["nu"], d.data_ptr(), o.data_ptr(), x.size, 0))
        ins.append(d)
        outs.append(o)
    qm.qm_run_batch(ctx, qreqs, device_tensor=ins[0])
    torch.cuda.synchronize()
    rng = np.random.default_rng(23)
    for r, d, o in zip(reqs, ins, outs):
        idx = np.unique(rng.integers(0, d.numel(), 8))
        ti = torch.from_numpy(idx).cuda()
        x = d[ti].cpu().numpy()
        got = o[ti].cpu().numpy()
        rtol = RTOL_F32 if got.dtype == np.float32 else RTOL_F64
        assert_close(got, oracle_of(r, x), rtol, str(r))
    del ins, outs
    torch.cuda.empty_cache()


HYP_PARAMS = [(1.0, 0.0, 1.0), (1.0, 0.5, 1.0), (2.0, -1.5, 0.3)]


def hyperbolic_requests(seed):
    """Exponential -> hyperbolic requests of both dtypes, three parameter
    sets (two locations) and ragged sizes, with a quantile and a Student t
    request between them."""
    reqs, cases = [], []
    for i, p in enumerate(HYP_PARAMS):
        for dtype in (np.float64, np.float32):
            for n in (1, 3001 + 17 * i, 40000 + 3 * i):
                lp, lm, _ = oracle.hyperbolic_masses(*p)
                x = qi.two_sided_exponentials(seed + i, 3, n, p[0] - p[1], p[0] + p[1], np.exp(lm)).astype(dtype)
                d = torch.from_numpy(x).cuda()
                o = torch.full_like(d, float("nan"))
                mu = 0.0 if n != 1 else 0.75
                reqs.append(qm.make_request(qm.QM_EXP_TO_HYPERBOLIC, d, o, hyperbolic=p, mu=mu))
                cases.append((p, mu, d, o))
    u = torch.from_numpy(qi.uniform53(seed, 9, 20000)).cuda()
    w = torch.full_like(u, float("nan"))
    z = torch.from_numpy(qi.normals(seed, 8, 20000)).cuda()
    t = torch.full_like(z, float("nan"))
    reqs.insert(2, qm.make_request(qm.QM_NORMAL_QUANTILE, u, w))
    reqs.insert(5, qm.make_request(qm.QM_STUDENT_T, z, t, nu=4.0))
    return reqs, cases, (u, w, z, t)


def check_hyperbolic_cases(ctx, cases, others):
    rng = np.random.default_rng(5)
    for p, mu, d, o in cases:
        ref = torch.empty_like(d)
        qm.qm_recycle_exp_to_hyperbolic(ctx, d, ref, *p, mu=mu)
        torch.cuda.synchronize()
        a, b = o.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), ("not bitwise equal", p, mu, a.size, a.dtype)
        if mu == 0.0:
            idx = np.unique(rng.integers(0, a.size, 64))
            x = d.cpu().numpy()[idx].astype(np.float64)
            rtol = RTOL_F32 if a.dtype == np.float32 else RTOL_F64
            assert_close(a[idx], oracle.hyperbolic_map(x, *p), rtol, str(p))
    u, w, z, t = others
    assert torch.equal(w, single(ctx, qm.QM_NORMAL_QUANTILE, qm.QM_PLAIN, 0.0, u))
    assert torch.equal(t, single(ctx, qm.QM_STUDENT_T, qm.QM_PLAIN, 4.0, z))


def test_batch_hyperbolic_bitwise_equal_to_single(ctx):
    reqs, cases, others = hyperbolic_requests(60)
    qm.qm_run_batch(ctx, reqs, device_tensor=others[0])
    torch.cuda.synchronize()
    check_hyperbolic_cases(ctx, cases, others)


def test_serving_hyperbolic(ctx):
    reqs, cases, others = hyperbolic_requests(70)
    torch.cuda.synchronize()
    tickets = [qm.qm_submit(ctx, r) for r in reqs]
    deadline = time.time() + 60
    pending = set(tickets)
    while pending and time.time() < deadline:
        pending = {t for t in pending if qm.qm_poll(ctx, t) == qm.QM_PENDING}
        time.sleep(0.001)
    assert not pending, "requests did not complete"
    check_hyperbolic_cases(ctx, cases, others)


def test_batch_hyperbolic_validation(ctx):
    d = torch.zeros(16, dtype=torch.float64, device="cuda")
    good = qm.make_request(qm.QM_EXP_TO_HYPERBOLIC, d, d, hyperbolic=(1.0, 0.0, 1.0))
    for bad in [qm.make_request(qm.QM_EXP_TO_HYPERBOLIC, d, d, hyperbolic=(1.0, 1.0, 1.0)),
                qm.make_request(qm.QM_EXP_TO_HYPERBOLIC, d, d, hyperbolic=(1.0, 0.0, 1.0), mu=float("nan")),
                qm.make_request(qm.QM_EXP_TO_HYPERBOLIC, d, d, mode=qm.QM_PAPER, hyperbolic=(1.0, 0.0, 1.0))]:
        with pytest.raises(qm.QMError):
            qm.qm_run_batch(ctx, [good, bad], device_tensor=d)
        with pytest.raises(qm.QMError):
            qm.qm_submit(ctx, bad)


def test_batch_and_serving_vg(ctx):
    """Variance-gamma requests (lambda in nu) of both dtypes beside a
    hyperbolic one: batch and serving outputs equal the single calls bit
    for bit."""
    params = [(2, 1.0, 0.5), (3, 2.0, -1.0)]
    cases, reqs = [], []
    for i, (lam, a, b) in enumerate(params):
        for dtype in (np.float64, np.float32):
            x = qi.two_sided_exponentials(80 + i, 5, 5000 + 37 * i, a - b, a + b, 0.4).astype(dtype)
            d = torch.from_numpy(x).cuda()
            o = torch.full_like(d, float("nan"))
            reqs.append(qm.make_request(qm.QM_EXP_TO_VG, d, o, nu=lam, hyperbolic=(a, b, 0.0), mu=0.5))
            cases.append(((lam, a, b), d, o))
    h = torch.from_numpy(qi.two_sided_exponentials(90, 5, 3000, 1.0, 1.0, 0.5)).cuda()
    ho = torch.full_like(h, float("nan"))
    reqs.append(qm.make_request(qm.QM_EXP_TO_HYPERBOLIC, h, ho, hyperbolic=(1.0, 0.0, 1.0)))
    qm.qm_run_batch(ctx, reqs, device_tensor=h)
    torch.cuda.synchronize()

    def check():
        for p, d, o in cases:
            ref = torch.empty_like(d)
            qm.qm_recycle_exp_to_vg(ctx, d, ref, *p, mu=0.5)
            torch.cuda.synchronize()
            assert torch.equal(o, ref), p
        ref = torch.empty_like(h)
        qm.qm_recycle_exp_to_hyperbolic(ctx, h, ref, 1.0, 0.0, 1.0)
        torch.cuda.synchronize()
        assert torch.equal(ho, ref)

    check()
    for _, _, o in cases:
        o.fill_(float("nan"))
    ho.fill_(float("nan"))
    torch.cuda.synchronize()
    tickets = [qm.qm_submit(ctx, r) for r in reqs]
    deadline = time.time() + 60
    pending = set(tickets)
    while pending and time.time() < deadline:
        pending = {t for t in pending if qm.qm_poll(ctx, t) == qm.QM_PENDING}
        time.sleep(0.001)
    assert not pending
    check()
    d = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(qm.QMError):
        qm.qm_run_batch(ctx, [qm.make_request(qm.QM_EXP_TO_VG, d, d, nu=8.5, hyperbolic=(1.0, 0.0, 0.0))],
                        device_tensor=d)


def wait_all(ctx, tickets, limit_s=120):
    deadline = time.time() + limit_s
    pending = set(tickets)
    while pending and time.time() < deadline:
        pending = {t for t in pending if qm.qm_poll(ctx, t) == qm.QM_PENDING}
        time.sleep(0.001)
    assert not pending, "%d requests did not complete" % len(pending)


def test_serving_full_size_alone_vs_mix():
    """The serving workload's shape: 200 requests, sizes log-uniform in
    2^12..2^24, the 40/20/30/10 mix (nu uniform in 1..50), each with its own
    inputs, arriving as a Poisson stream at 5000 requests/s so that they are
    admitted while earlier ones run, HBM budget 64 GB.  Every output is
    bitwise the same request run alone, 16 sampled outputs per request are
    within tolerance of the oracle, and the bytes in flight never exceeded
    the budget."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    budget = 64 << 30
    c = qm.Context(0, hbm_budget_bytes=budget)
    try:
        reqs, ins, outs, qreqs = build(5, 200, 12, 24)
        print("serving full size: %d requests, %d elements" % (len(reqs), sum(r["n"] for r in reqs)), flush=True)
        for r in reqs:                      # tables first, as a server warms up
            if r["kind"] == "student_f64":
                qm.qm_recycle_student_t(c, ins[0][:0].double(), outs[0][:0].double(), r["nu"])
        torch.cuda.synchronize()
        rng = np.random.default_rng(55)
        gaps = rng.exponential(1.0 / 5000, len(qreqs))
        t0 = time.perf_counter()
        due = 0.0
        tickets = []
        for q, g in zip(qreqs, gaps):
            due += g
            while time.perf_counter() - t0 < due:
                pass
            tickets.append(qm.qm_submit(c, q))
        wait_all(c, tickets)
        st = qm.qm_serving_stats_of(c)
        print("serving stats", st, flush=True)
        assert st["completed"] == len(tickets) and st["failed"] == 0 and st["queued"] == 0
        assert 0 < st["in_flight_bytes_high_water"] <= budget
        for r, d, o in zip(reqs, ins, outs):
            kind, mode = KIND[r["kind"]]
            alone = single(c, kind, mode, r["nu"], d)
            bits = torch.int32 if o.dtype == torch.float32 else torch.int64
            assert torch.equal(o.view(bits), alone.view(bits)), ("alone vs mix", r)
            del alone
        torch.cuda.synchronize()
        for r, d, o in zip(reqs, ins, outs):
            idx = torch.from_numpy(np.unique(rng.integers(0, d.numel(), 16))).cuda()
            x = d[idx].cpu().numpy()
            got = o[idx].cpu().numpy()
            assert_close(got, oracle_of(r, x), RTOL_F32 if got.dtype == np.float32 else RTOL_F64, str(r))
        del ins, outs
    finally:
        c.close()
        torch.cuda.empty_cache()


def test_serving_budget_high_water_under_burst():
    """A burst of 96 requests of 1 MiB in + 1 MiB out against a 16 MiB
    budget: the server admits at most 8 at a time, so the bytes in flight
    never exceed the budget, and every request completes."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    budget = 16 << 20
    c = qm.Context(0, hbm_budget_bytes=budget)
    try:
        xs = [torch.from_numpy(qi.uniform53(8, i, 1 << 17)).cuda() for i in range(96)]
        ys = [torch.empty_like(x) for x in xs]
        torch.cuda.synchronize()
        tickets = [qm.qm_submit(c, qm.make_request(qm.QM_NORMAL_QUANTILE, x, y)) for x, y in zip(xs, ys)]
        wait_all(c, tickets)
        st = qm.qm_serving_stats_of(c)
        assert st["completed"] == 96 and st["in_flight_bytes"] == 0 and st["in_flight_requests"] == 0
        assert (2 << 20) <= st["in_flight_bytes_high_water"] <= budget, st
        assert st["budget_bytes"] == budget
        for t in tickets:
            status, sub, done = qm.qm_poll_times(c, t)
            assert status == qm.QM_OK and done >= sub > 0
        ref = torch.empty_like(xs[0])
        qm.qm_normal_quantile(c, xs[-1], ref)
        torch.cuda.synchronize()
        assert torch.equal(ref, ys[-1])
    finally:
        c.close()


def test_serving_request_completes_before_its_batch():
    """Per-request completion inside one batch.  A 2^28-element request
    fills the whole 4 GiB budget, so the next group waits and is admitted
    as one batch after it: eight 2^12-element requests (first in the batch,
    so their chunks are claimed first) and one large request that fills the
    budget again.  Each small request is reported complete before the large
    one (its flag, raised by the workgroup that writes its last chunk, not
    the batch's end), and its output is already complete when read at that
    moment, while the large request is still running: bitwise the single
    call."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    budget = 4 << 30
    c = qm.Context(0, hbm_budget_bytes=budget)
    try:
        n_block, n_small = 1 << 28, 1 << 12
        n_big = n_block - 8 * n_small
        block_in = torch.from_numpy(qi.uniform53(11, 0, n_block)).cuda()
        block_out = torch.empty_like(block_in)
        big_in = torch.from_numpy(qi.uniform53(11, 1, n_big)).cuda()
        big_out = torch.full_like(big_in, float("nan"))
        smalls = [torch.from_numpy(qi.uniform53(11, 2 + i, n_small)).cuda() for i in range(8)]
        small_out = [torch.full_like(x, float("nan")) for x in smalls]
        refs = []
        for x in smalls:
            r = torch.empty_like(x)
            qm.qm_normal_quantile(c, x, r)
            refs.append(r)
        torch.cuda.synchronize()
        print("per-request completion: blocker 2^28, 8 x 2^12 + %d in one batch" % n_big, flush=True)
        t_block = qm.qm_submit(c, qm.make_request(qm.QM_NORMAL_QUANTILE, block_in, block_out))
        ts = [qm.qm_submit(c, qm.make_request(qm.QM_NORMAL_QUANTILE, x, y)) for x, y in zip(smalls, small_out)]
        t_big = qm.qm_submit(c, qm.make_request(qm.QM_NORMAL_QUANTILE, big_in, big_out))
        seen = {}
        deadline = time.time() + 60
        while len(seen) < len(ts) and time.time() < deadline:
            for i, t in enumerate(ts):
                if i not in seen and qm.qm_poll(c, t) == qm.QM_OK:
                    # read at once, on the caller's stream, while the batch may still run
                    seen[i] = (small_out[i].cpu(), qm.qm_poll(c, t_big))
        assert len(seen) == len(ts), "small requests did not complete"
        wait_all(c, [t_block, t_big])
        _, _, big_done = qm.qm_poll_times(c, t_big)
        for i, t in enumerate(ts):
            got, big_state = seen[i]
            assert torch.equal(got.view(torch.int64), refs[i].cpu().view(torch.int64)), i
            _, _, done = qm.qm_poll_times(c, t)
            assert done < big_done, (i, done, big_done)
        print("large request still pending when the small ones were read: %d of 8"
              % sum(1 for g, s in seen.values() if s == qm.QM_PENDING), flush=True)
        st = qm.qm_serving_stats_of(c)
        assert st["completed"] == 10 and st["in_flight_bytes"] == 0 and st["in_flight_requests"] == 0
        assert st["in_flight_bytes_high_water"] <= budget
        idx = np.unique(np.random.default_rng(3).integers(0, n_big, 2000))
        got = big_out[torch.from_numpy(idx).cuda()].cpu().numpy()
        assert_close(got, oracle.norm_quantile(big_in[torch.from_numpy(idx).cuda()].cpu().numpy()), RTOL_F64, "big")
        del block_in, block_out, big_in, big_out
    finally:
        c.close()
        torch.cuda.empty_cache()
