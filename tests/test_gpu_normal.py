"""GPU parity: normal quantile and exponential -> normal against the oracle.

Inputs come from the shared seeded generator; the oracle computes every
element (or, at the full 2^28 size, a sample of elements regenerated on the
host by index).  Tolerance: tests/_tol.py.
"""
import numpy as np
import pytest

import oracle
import qm_inputs as qi
from tests._tol import RTOL_F32, RTOL_F64, as_f32_output, assert_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_0901_0638_amd as qm  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = qm.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_nq(ctx, u, mode=qm.QM_PLAIN):
    d = dev(u)
    w = torch.empty_like(d)
    qm.qm_normal_quantile(ctx, d, w, mode)
    torch.cuda.synchronize()
    return w.cpu().numpy()


def run_e(ctx, x, mode=None):
    d = dev(x)
    z = torch.empty_like(d)
    qm.qm_recycle_exp_to_normal(ctx, d, z, mode)
    torch.cuda.synchronize()
    return z.cpu().numpy()


SPECIAL_U = np.array([0.0, 1.0, 0.5, np.nan, -0.25, 1.5, -0.0, np.inf, -np.inf, 5e-324, 2.2250738585072014e-308,
                      1e-300, 2.875e-19, 1 - 2.0 ** -53, 0.5 - 2.0 ** -54, 0.5 + 2.0 ** -53, 0.25, 0.75,
                      1e-10, 1 - 1e-10, 0.9999999, 1e-16])


def test_quantile_f64_uniforms_2e20(ctx):
    """2^20 open uniforms, seed 0 (every element checked)."""
    u = qi.uniforms_2e20()
    rep = assert_close(run_nq(ctx, u), oracle.norm_quantile(u), RTOL_F64, "uniforms 2^20")
    print("uniforms 2^20", rep)


def test_quantile_f64_mixture_2e20(ctx):
    """The 10% deep-tail mixture (u down to 1e-300) at 2^20, every element."""
    u = qi.mixture(1, 0, 1 << 20, np.float64, 0.1, 1e-300)
    rep = assert_close(run_nq(ctx, u), oracle.norm_quantile(u), RTOL_F64, "mixture 2^20")
    print("mixture 2^20", rep)


def test_quantile_f64_specials_and_ragged(ctx):
    got = run_nq(ctx, SPECIAL_U)
    assert_close(got, oracle.norm_quantile(SPECIAL_U), RTOL_F64, "specials")
    for n in (1, 2, 3, 5, 17, 255, 256, 257, 1023):
        u = qi.uniform53(9, n, n)
        assert_close(run_nq(ctx, u), oracle.norm_quantile(u), RTOL_F64, "n=%d" % n)


def test_quantile_f64_deep_tail_sweep(ctx):
    """log-uniform u over the whole double range, including denormals, both sides."""
    rng = np.random.default_rng(3)
    t = 10.0 ** -rng.uniform(0.3, 323.3, 200000)
    t = t[t > 0]
    u = np.concatenate([t, 1.0 - t[t > 1e-16]])
    assert_close(run_nq(ctx, u), oracle.norm_quantile(u), RTOL_F64, "deep tail")


def test_quantile_f64_central_outer_boundary(ctx):
    """Plain mode switches between the central piece (|u - 1/2| <= 0.45) and
    the exponential-coordinate path; both sides of the switch, the switch
    points themselves, and u near 1/4 (where u - 1/2 stops being exact), in
    waves that mix both pieces and waves that hold only one."""
    edges = []
    for c in (0.05, 0.95, 0.25, 0.75):
        x = np.float64(c)
        for _ in range(40):
            edges += [x]
            x = np.nextafter(x, 2.0)
        x = np.float64(c)
        for _ in range(40):
            x = np.nextafter(x, -1.0)
            edges += [x]
    rng = np.random.default_rng(17)
    near = np.concatenate([rng.uniform(0.04, 0.06, 5000), rng.uniform(0.94, 0.96, 5000),
                           rng.uniform(0.2, 0.3, 2000)])
    central_only = rng.uniform(0.06, 0.94, 4096)
    outer_only = np.concatenate([rng.uniform(1e-9, 0.049, 2048), rng.uniform(0.951, 1 - 1e-9, 2048)])
    for name, u in (("edges", np.array(edges)), ("near", near), ("central", central_only), ("outer", outer_only)):
        assert_close(run_nq(ctx, u), oracle.norm_quantile(u), RTOL_F64, name)


def test_quantile_f64_misaligned_and_inplace(ctx):
    u = qi.uniform53(4, 0, 5000)
    ref = oracle.norm_quantile(u)
    base = dev(np.concatenate([[0.3], u, [0.7]]))
    # input at offset 1 (8-byte aligned, not 16), output at offset 0: not co-aligned
    out = torch.empty(5000, dtype=torch.float64, device="cuda")
    qm.qm_normal_quantile(ctx, base[1:5001], out)
    torch.cuda.synchronize()
    assert_close(out.cpu().numpy(), ref, RTOL_F64, "misaligned")
    # both at offset 1: co-aligned with a one-element head
    out2 = torch.zeros(5002, dtype=torch.float64, device="cuda")
    qm.qm_normal_quantile(ctx, base[1:5001], out2[1:5001])
    torch.cuda.synchronize()
    o2 = out2.cpu().numpy()
    assert_close(o2[1:5001], ref, RTOL_F64, "co-aligned head")
    assert o2[0] == 0 and o2[5001] == 0, "wrote outside the output range"
    # in place
    d = dev(u)
    qm.qm_normal_quantile(ctx, d, d)
    torch.cuda.synchronize()
    assert_close(d.cpu().numpy(), ref, RTOL_F64, "in place")


def test_quantile_f64_zero_length_and_errors(ctx):
    d = torch.zeros(4, dtype=torch.float64, device="cuda")
    qm.qm_normal_quantile(ctx, d[:0], d[:0])
    with pytest.raises(qm.QMError) as e:
        qm.qm_normal_quantile(ctx, d, d, mode=qm.QM_F32_REFINE)
    assert e.value.status == qm.QM_E_DTYPE
    lib = qm.load()
    import ctypes
    p = ctypes.c_void_p(d.data_ptr())
    assert lib.qm_normal_quantile(ctx.handle, p, ctypes.c_void_p(d.data_ptr() + 8), 4, qm.QM_F64, 0, None) == qm.QM_E_INVAL
    assert lib.qm_normal_quantile(ctx.handle, p, p, 4, 7, 0, None) == qm.QM_E_INVAL
    assert lib.qm_normal_quantile(ctx.handle, None, p, 4, qm.QM_F64, 0, None) == qm.QM_E_INVAL


def test_quantile_f64_paper_mode_on_its_domain(ctx):
    """Paper constants verbatim (Appendix B): within tolerance for v <= 42."""
    u = qi.uniforms_2e20()
    assert_close(run_nq(ctx, u, qm.QM_PAPER), oracle.norm_quantile(u), RTOL_F64, "paper 13,13")


PAPER_U_MIN = 2.875e-19          # v = 42, the end of the (13,13) rational's domain


def test_quantile_f64_paper_t2_hybrid(ctx):
    """The paper's hybrid as printed (Section 7.3, Appendix C): the T2
    rational behind a whole-wave vote, the (13,13) path otherwise.  2^20
    open uniforms (about 87% of waves all-central, the rest on the branchless
    path), a mixture whose tail stays in the paper's domain (every wave on
    the branchless path), arrays that hold only central values, and the
    values either side of the switch at v = 15.5: all against the oracle."""
    u = qi.uniforms_2e20()
    rep = assert_close(run_nq(ctx, u, qm.QM_PAPER_T2), oracle.norm_quantile(u), RTOL_F64, "t2 uniforms")
    print("t2 uniforms", rep)
    m = qi.mixture(3, 0, 1 << 18, np.float64, 0.1, PAPER_U_MIN)
    assert_close(run_nq(ctx, m, qm.QM_PAPER_T2), oracle.norm_quantile(m), RTOL_F64, "t2 mixture")
    c = np.linspace(0.0011, 0.9989, 100003)
    assert_close(run_nq(ctx, c, qm.QM_PAPER_T2), oracle.norm_quantile(c), RTOL_F64, "t2 central")
    # u where v = |u - 1/2|/sqrt(u(1-u)) crosses 15.5: 1/2 +- (1/2) 15.5/sqrt(1 + 15.5^2)
    edge = 0.5 * 15.5 / np.sqrt(1 + 15.5 ** 2)
    e = np.concatenate([0.5 + edge + np.linspace(-1e-6, 1e-6, 4097), 0.5 - edge + np.linspace(-1e-6, 1e-6, 4097)])
    assert_close(run_nq(ctx, e, qm.QM_PAPER_T2), oracle.norm_quantile(e), RTOL_F64, "t2 switch")


def test_quantile_f64_paper_t2_specials_and_checks(ctx):
    """Specials as in the other forms (the vote sends their waves to the
    branchless path); the mode is FP64 qm_normal_quantile only."""
    sp = np.array([0.0, 1.0, 0.5, np.nan, -0.25, 1.5, -0.0, np.inf, -np.inf, 0.25, 0.75, 1 - 2.0 ** -53,
                   0.5 - 2.0 ** -54, 0.5 + 2.0 ** -53, PAPER_U_MIN, 1e-10, 1 - 1e-10])
    got = run_nq(ctx, sp, qm.QM_PAPER_T2)
    ref = oracle.norm_quantile(sp)
    assert_close(got, ref, RTOL_F64, "t2 specials")
    assert got[0] == -np.inf and got[1] == np.inf and got[6] == -np.inf
    assert got[2] == 0 and not np.signbit(got[2]) and np.all(np.isnan(got[[3, 4, 5, 7, 8]]))
    # an all-central array with u = 1/2 in it: +0 from the T2 branch
    c = np.full(256, 0.5)
    c[1::2] = 0.3
    got = run_nq(ctx, c, qm.QM_PAPER_T2)
    assert np.all(got[::2] == 0) and not np.any(np.signbit(got[::2]))
    f = torch.zeros(64, dtype=torch.float32, device="cuda")
    d = torch.full((64,), 0.25, dtype=torch.float64, device="cuda")
    with pytest.raises(qm.QMError) as e:
        qm.qm_normal_quantile(ctx, f, f, qm.QM_PAPER_T2)
    assert e.value.status == qm.QM_E_DTYPE
    with pytest.raises(qm.QMError) as e:
        qm.qm_recycle_exp_to_normal(ctx, d, d, qm.QM_PAPER_T2)
    assert e.value.status == qm.QM_E_DTYPE
    with pytest.raises(qm.QMError) as e:
        qm.qm_run_batch(ctx, [qm.make_request(qm.QM_NORMAL_QUANTILE, d, d, mode=qm.QM_PAPER_T2)], device_tensor=d)
    assert e.value.status == qm.QM_E_INVAL
    with pytest.raises(qm.QMError) as e:
        qm.qm_generate(ctx, 0, 0, 0, d, qm.QM_NORMAL_QUANTILE, qm.QM_PAPER_T2)
    assert e.value.status == qm.QM_E_INVAL
    torch.cuda.synchronize()


def test_map_kernel_ragged_sizes(ctx):
    """The per-element map kernel (the paper's forms, exp -> normal) streams
    tiles of 256 vectors per wave: sizes below, at and past a tile, with a
    partial last tile, and an input one element off 16-byte alignment."""
    for n in (1, 3, 255, 513, 1025, 5001):
        u = qi.uniform53(9, n, n)
        ref = oracle.norm_quantile(u)
        assert_close(run_nq(ctx, u, qm.QM_PAPER), ref, RTOL_F64, "paper n=%d" % n)
        assert_close(run_nq(ctx, u, qm.QM_PAPER_T2), ref, RTOL_F64, "t2 n=%d" % n)
        x = qi.exponentials(9, n, n)
        x[::3] *= -1
        assert_close(run_e(ctx, x), oracle.exp_to_normal(x), RTOL_F64, "exp n=%d" % n)
        x32 = x.astype(np.float32)
        ref32 = oracle.exp_to_normal(x32.astype(np.float64))
        assert_close(run_e(ctx, x32), ref32, RTOL_F32, "exp f32 n=%d" % n)
    x = qi.exponentials(10, 1, 5001)
    base = torch.from_numpy(np.concatenate([[0.0], x])).cuda()
    out = torch.empty(5001, dtype=torch.float64, device="cuda")
    out2 = torch.empty(5002, dtype=torch.float64, device="cuda")
    qm.qm_recycle_exp_to_normal(ctx, base[1:], out)        # not co-aligned: element-wise
    qm.qm_recycle_exp_to_normal(ctx, base[1:], out2[1:])   # co-aligned: a head element, tiles, a tail
    torch.cuda.synchronize()
    ref = oracle.exp_to_normal(x)
    assert_close(out.cpu().numpy(), ref, RTOL_F64, "exp misaligned")
    assert_close(out2[1:].cpu().numpy(), ref, RTOL_F64, "exp head and tail")


def test_quantile_f64_paper_t2_full_size_sampled(ctx):
    """2^28 open uniforms (the paper's timing input) in the launch the
    benchmark times for this form, sampled as the other full-size tests."""
    u = qi.uniform53(2, 0, 1 << 28)
    check_full_size(ctx, u, lambda c, d, w: qm.qm_normal_quantile(c, d, w, qm.QM_PAPER_T2), RTOL_F64,
                    "t2 2^28", 15, oracle.norm_quantile)


def test_quantile_f32_refine_mixture(ctx):
    """FP32 + FP64-refine on the FP32 mixture (tail down to 1e-37), 2^20."""
    u = qi.mixture(1, 0, 1 << 20, np.float32, 0.1, 1e-37)
    ref = oracle.norm_quantile(u.astype(np.float64))
    rep = assert_close(run_nq(ctx, u, qm.QM_F32_REFINE), ref, RTOL_F32, "f32 refine")
    print("f32 refine", rep)


def test_quantile_f32_refine_edges(ctx):
    rng = np.random.default_rng(8)
    t = (10.0 ** -rng.uniform(0.3, 44.8, 100000)).astype(np.float32)
    t = t[t > 0]
    u = np.concatenate([t, (1.0 - t).astype(np.float32), SPECIAL_U.astype(np.float32),
                        np.array([1.4e-45, 1.2e-38, 0.5 - 2 ** -25, 0.5 + 2 ** -24, 1 - 2 ** -24], np.float32)])
    u = u.astype(np.float32)
    ref = oracle.norm_quantile(u.astype(np.float64))
    assert_close(run_nq(ctx, u, qm.QM_F32_REFINE), ref, RTOL_F32, "f32 refine edges")
    assert_close(run_nq(ctx, u, qm.QM_PLAIN), ref, RTOL_F32, "f32 plain edges")


def test_quantile_f32_refine_central_outer_boundary(ctx):
    """FP32+refine switches between its central piece (FP32 seed + FP64
    Newton against erf) and the exponential-coordinate seed + FP64 Newton
    against erfc at |u - 1/2| = 0.45; both sides and the switch points, every float
    in a window around them, in mixed and single-piece waves.  Before its
    rounding to float the result is within 2.5e-8 of the oracle (central
    piece: E6 and G3 of the Newton step; outer: the Mills ratio and the
    exponential of that step), so it is the oracle value rounded to
    float except within 4e-8 of a midpoint, where it may be the neighbour."""
    edges = []
    for c in (0.05, 0.95, 0.25, 0.75, 0.5):
        x = np.float32(c)
        for _ in range(300):
            edges.append(x)
            x = np.nextafter(x, np.float32(2))
        x = np.float32(c)
        for _ in range(300):
            x = np.nextafter(x, np.float32(-1))
            edges.append(x)
    rng = np.random.default_rng(23)
    u = np.concatenate([np.array(edges, np.float32), rng.uniform(0.04, 0.96, 20000).astype(np.float32),
                        qi.uniform23(6, 0, 1 << 16)])
    ref = oracle.norm_quantile(u.astype(np.float64))
    got = run_nq(ctx, u, qm.QM_F32_REFINE)
    assert_close(got, ref, RTOL_F32, "f32 refine centre/outer")
    r32 = ref.astype(np.float32)
    other = np.nextafter(r32, np.where(ref > r32, np.float32(np.inf), np.float32(-np.inf)))
    mid = (r32.astype(np.float64) + other.astype(np.float64)) / 2
    near = np.abs(ref - mid) <= 4e-8 * np.abs(ref)
    bad = (got != r32) & ~near & (ref != 0)
    assert not bad.any(), (int(bad.sum()), u[bad][:5], got[bad][:5], r32[bad][:5])
    assert np.all((got == r32) | (got == other) | (ref == 0))


def test_quantile_f32_paper_mode(ctx):
    """Paper (5,6) in FP32 (Appendix A): realized error of order 3e-7 down to
    u ~ 1e-11 (Section 6.3); checked at 5e-7 on its domain v <= 25."""
    u = qi.uniform23(5, 0, 1 << 18)
    u = u[np.minimum(u, 1 - u) > 1e-11]
    ref = oracle.norm_quantile(u.astype(np.float64))
    assert_close(run_nq(ctx, u, qm.QM_PAPER), ref, 5e-7, "f32 paper")


def test_exp_to_normal_f64(ctx):
    """Exp(1) samples (seed 2 stream 1), signed copies, and a far-tail sweep."""
    x = qi.exponentials(2, 1, 1 << 20)
    xs = np.concatenate([x, -x[:1000]])
    rep = assert_close(run_e(ctx, xs), oracle.exp_to_normal(xs), RTOL_F64, "exp->normal")
    print("exp->normal", rep)
    rng = np.random.default_rng(4)
    far = np.concatenate([rng.uniform(30, 800, 20000), 10 ** rng.uniform(2.5, 4, 2000),
                          [42.0, 42.0000001, 749.9, 750.0, 750.1, 0.0, -0.0, np.inf, -np.inf, np.nan, 1e-300]])
    assert_close(run_e(ctx, far), oracle.exp_to_normal(far), RTOL_F64, "exp->normal far")


def test_exp_to_normal_f64_paper(ctx):
    x = qi.exponentials(2, 1, 1 << 18)
    assert_close(run_e(ctx, x, qm.QM_PAPER), oracle.exp_to_normal(x), RTOL_F64, "exp->normal paper")


def test_exp_to_normal_f32_plain(ctx):
    """FP32 in/out, QM_PLAIN: the FP64 map of the widened input rounded once,
    so the oracle value rounded to float (a midpoint within 2e-15 aside);
    QM_PAPER is not an FP32 form of this map."""
    x = qi.exponentials(3, 1, 1 << 18).astype(np.float32)
    x = np.concatenate([x, -x[:100], np.array([0, -0.0, 102.9, 103.1, 500, 1e4, np.inf, -np.inf, np.nan], np.float32)])
    ref = oracle.exp_to_normal(x.astype(np.float64))
    got = run_e(ctx, x, qm.QM_PLAIN)
    assert_close(got, as_f32_output(ref), RTOL_F32, "exp->normal f32 plain")
    r32 = ref.astype(np.float32)
    fin = np.isfinite(ref)
    assert np.mean(got[fin] == r32[fin]) > 0.999
    with pytest.raises(qm.QMError) as e:
        run_e(ctx, x[:16], qm.QM_PAPER)
    assert e.value.status == qm.QM_E_DTYPE


def test_exp_to_normal_f32_refine(ctx):
    x = qi.exponentials(2, 1, 1 << 18).astype(np.float32)
    x = np.concatenate([x, -x[:100], np.array([0, 102.9, 103.1, 500, 1e4, np.inf, -np.inf, np.nan], np.float32)])
    x = x.astype(np.float32)
    ref = oracle.exp_to_normal(x.astype(np.float64))
    assert_close(run_e(ctx, x), ref, RTOL_F32, "exp->normal f32 refine")


def full_size_indices(n, seed, tail_of=None):
    """Output indices checked at a full benchmark size: 2^16 random ones,
    whole contiguous runs of 4096 (every element of the waves that wrote
    them) at the start, in the middle of the grid-stride passes and in the
    last pass, the last 300, and, given the inputs, every outer element
    (|u - 1/2| > 0.45) among the first 2^20."""
    rng = np.random.default_rng(seed)
    runs = [np.arange(s, s + 4096) for s in (0, n // 2 + 12288, n - (n >> 4) + 4096, n - 8192)]
    parts = [rng.integers(0, n, 1 << 16), np.arange(n - 300, n)] + runs
    if tail_of is not None:
        head = tail_of[: 1 << 20].astype(np.float64)
        parts.append(np.flatnonzero(np.abs(head - 0.5) > 0.45))
    return np.unique(np.concatenate(parts))


def check_full_size(ctx, u, fn, rtol, what, seed, ref_fn):
    d = torch.from_numpy(u).cuda()
    w = torch.empty_like(d)
    fn(ctx, d, w)
    torch.cuda.synchronize()
    idx = full_size_indices(u.size, seed, u if ref_fn is oracle.norm_quantile else None)
    got = w[torch.from_numpy(idx).cuda()].cpu().numpy()
    ref = ref_fn(u[idx].astype(np.float64))
    if got.dtype == np.float32:
        ref = as_f32_output(ref)
    rep = assert_close(got, ref, rtol, what)
    print(what, len(idx), rep, flush=True)
    del d, w
    torch.cuda.empty_cache()


def test_quantile_f64_full_size_sampled(ctx):
    """The FP64 mixture at its full size 2^28 in the launch configuration the
    benchmark times; 2^16 random outputs, whole runs of 4096 in the first,
    a middle and the last grid-stride passes, the last 300 and every outer
    element among the first 2^20, against the oracle."""
    check_full_size(ctx, qi.mixture_f64(1 << 28), lambda c, d, w: qm.qm_normal_quantile(c, d, w), RTOL_F64,
                    "f64 2^28", 12, oracle.norm_quantile)


def test_quantile_f32_refine_full_size_sampled(ctx):
    """FP32 + FP64 refine on the FP32 mixture at its full size 2^28 (16
    grid-stride passes of the benchmark's launch), sampled as the FP64 test.
    About 4.2% of its elements are fl(1 - t) = 1.0 (t < 2^-25) and compare as
    +inf on both sides; the upper tail is otherwise covered by the exact
    symmetry of the formulas and the edge tests."""
    check_full_size(ctx, qi.mixture_f32(1 << 28),
                    lambda c, d, w: qm.qm_normal_quantile(c, d, w, qm.QM_F32_REFINE), RTOL_F32,
                    "f32 refine 2^28", 13, oracle.norm_quantile)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_exp_to_normal_full_size_sampled(ctx, dtype):
    """Exponential -> normal on the 2^26 Exp(1) recycling workload in the
    benchmark's launch (several grid-stride passes), FP64 and FP32+refine,
    sampled like the quantile."""
    x = qi.recycle_exponentials(1 << 26).astype(dtype)
    check_full_size(ctx, x, lambda c, d, w: qm.qm_recycle_exp_to_normal(c, d, w),
                    RTOL_F64 if dtype == np.float64 else RTOL_F32, "exp->normal 2^26 %s" % np.dtype(dtype).name, 14,
                    oracle.exp_to_normal)
