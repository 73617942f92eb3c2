"""GPU parity: the normal -> Student t recycling map against the oracle."""
import numpy as np
import pytest

import oracle
import qm_inputs as qi
from tests._tol import RTOL_F32, RTOL_F64, as_f32_output, assert_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_0901_0638_amd as qm  # noqa: E402

NUS = [1, 2, 3, 4, 5, 10, 30]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = qm.Context(0)
    yield c
    c.close()


def run_t(ctx, z, nu, mode=None):
    d = torch.from_numpy(np.ascontiguousarray(z)).cuda()
    t = torch.empty_like(d)
    qm.qm_recycle_student_t(ctx, d, t, nu, mode)
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def normals():
    """First 2^16 Box-Muller normals of the recycling workload (seed 2), plus
    every element with |z| > 4 among the first 2^22."""
    z = qi.recycle_normals(1 << 22)
    return np.concatenate([z[: 1 << 16], z[np.abs(z) > 4.0]])


@pytest.mark.parametrize("nu", NUS)
def test_student_f64_workload_normals(ctx, normals, nu):
    rep = assert_close(run_t(ctx, normals, nu), oracle.student_t_map(normals, nu), RTOL_F64, "nu=%s" % nu)
    print("nu", nu, rep)


@pytest.mark.parametrize("nu", [0.3, 0.4, 0.5, 2.5, 7.5, 50])
def test_student_f64_other_nu(ctx, nu):
    rng = np.random.default_rng(int(nu * 10))
    z = np.concatenate([rng.normal(size=20000), rng.uniform(-10, 10, 20000)])
    assert_close(run_t(ctx, z, nu), oracle.student_t_map(z, nu), RTOL_F64, "nu=%s" % nu)


def test_student_f64_edges(ctx):
    z = np.array([0.0, -0.0, 1e-300, -1e-300, 5e-324, 1e-8, np.nan, np.inf, -np.inf, 9.999999, -10.0,
                  8.652, 0.5, 2.0, 7.999999999, 8.0, 8.0000000001])
    for nu in (1, 4, 30):
        got = run_t(ctx, z, nu)
        assert_close(got, oracle.student_t_map(z, nu), RTOL_F64, "edges nu=%s" % nu)
    # ragged sizes (below, at and past a wave's tile of 256 vectors, with a
    # partial last tile), misaligned and in place
    for n in (1, 2, 3, 7, 255, 257, 513, 1025, 5001):
        zz = qi.normals(5, n, n)
        assert_close(run_t(ctx, zz, 3), oracle.student_t_map(zz, 3), RTOL_F64, "n=%d" % n)
    zz = qi.normals(6, 0, 3001)
    base = torch.from_numpy(np.concatenate([[0.0], zz])).cuda()
    out = torch.empty(3001, dtype=torch.float64, device="cuda")
    qm.qm_recycle_student_t(ctx, base[1:], out, 4.0)
    d = torch.from_numpy(zz).cuda()
    qm.qm_recycle_student_t(ctx, d, d, 4.0)
    torch.cuda.synchronize()
    ref = oracle.student_t_map(zz, 4.0)
    assert_close(out.cpu().numpy(), ref, RTOL_F64, "misaligned")
    assert_close(d.cpu().numpy(), ref, RTOL_F64, "in place")


def test_student_identity_and_large_nu(ctx):
    z = qi.normals(7, 0, 4096)
    assert np.array_equal(run_t(ctx, z, float("inf")), z)
    # nu > 1e5: Cornish-Fisher polynomial (Section 3.4)
    t = run_t(ctx, z, 2e5)
    assert_close(t, oracle.student_t_map(z, 2e5), RTOL_F64, "nu=2e5")


def test_student_huge_z_overflows_to_inf(ctx):
    """|z| from 1e150 to the largest double: log t is about z^2/(2 nu), far
    beyond the FP64 range for every nu below 1e300, so t is +-inf (z^2 itself
    overflows from 1.3e154 on).  The oracle saturates where its upper-tail
    probability underflows (|z| about 150), so the exact value is the check."""
    z = np.array([1e150, -1e150, 1.4e154, 1e155, -1e200, 1e300, -1.7976931348623157e308])
    for nu in (0.5, 1, 4, 30, 1000, 1e5, 2e5):
        got = run_t(ctx, z, nu)
        assert np.array_equal(got, np.copysign(np.inf, z)), (nu, got)
    z32 = np.array([1e20, -3e38, 3.4028235e38], np.float32)
    for nu in (1.0, 4.0, 30.0):
        got = run_t(ctx, z32, nu)
        assert np.array_equal(got, np.copysign(np.float32(np.inf), z32)), (nu, got)


def test_student_invalid_nu(ctx):
    d = torch.zeros(8, dtype=torch.float64, device="cuda")
    for nu in (0.29, 0.25, 0.1, 1e-300, 0.0, -1.0, float("nan"), float("-inf")):
        with pytest.raises(qm.QMError) as e:
            qm.qm_recycle_student_t(ctx, d, d, nu)
        assert e.value.status == qm.QM_E_INVAL


@pytest.mark.parametrize("nu", [0.3, 0.5, 1, 2, 4, 8, 10, 20, 30, 50, 80, 100, 1000, 1e5])
def test_student_far_tail(ctx, nu):
    """|z| > 10: the table's further cells (read from global memory) and,
    beyond them, the two-term tail of Section 3.5, which the builder only
    uses where it is as accurate as the cells; up to |z| = 38.5 (the normal
    quantile of the smallest double) that holds for every nu.  Both output
    precisions, and a wave mixing far and table elements."""
    rng = np.random.default_rng(int(nu) + 5)
    far = np.concatenate([np.linspace(10.0, 38.5, 229), -rng.uniform(10.0, 38.5, 64),
                          [10.000000001, 10.198039027185569, 10.198039027185571, 12.0, 12.000000001]])
    mixed = np.concatenate([rng.normal(size=192), far[:64]])     # one far lane per four
    for z in (far, mixed):
        ref = oracle.student_t_map(z, nu)
        assert_close(run_t(ctx, z, nu), ref, RTOL_F64, "far f64 nu=%s" % nu)
        z32 = z.astype(np.float32)
        ref32 = as_f32_output(oracle.student_t_map(z32.astype(np.float64), nu))
        assert_close(run_t(ctx, z32, nu), ref32, RTOL_F32, "far f32 nu=%s" % nu)


def test_student_beyond_cells_formula_bound(ctx):
    """|z| > 40 (no normal quantile of a double lies there): the two-term
    formula alone, within its own O(w^{4/nu}) error, w = K q(|z|)."""
    import math
    z = np.array([40.5, 45.0, 60.0, -50.0, 100.0])
    for nu in (4, 30, 100):
        got = run_t(ctx, z, nu)
        ref = oracle.student_t_map(z, nu)
        lK = math.log(nu) + 0.5 * math.log(math.pi) + math.lgamma(nu / 2) - math.lgamma((nu + 1) / 2)
        for zi, g, r in zip(z, got, ref):
            if np.isinf(r):
                assert g == r, (nu, zi, g)
                continue
            lw = lK + math.log(0.5) + math.log(math.erfc(abs(zi) / math.sqrt(2))) if abs(zi) < 26 else \
                lK - zi * zi / 2 - math.log(abs(zi) * math.sqrt(2 * math.pi))
            assert abs(g / r - 1) <= 10 * math.exp(4 * lw / nu) + 1e-14, (nu, zi, g, r)


@pytest.mark.parametrize("nu", [1, 4, 30])
def test_student_f32_refine(ctx, normals, nu):
    z = normals.astype(np.float32)
    got = run_t(ctx, z, nu)
    ref = as_f32_output(oracle.student_t_map(z.astype(np.float64), nu))
    assert_close(got, ref, RTOL_F32, "f32 nu=%s" % nu)


@pytest.mark.parametrize("nu", [0.3, 0.5, 0.75, 1.5, 2.5, 7.5, 50, 1000, 2e5, float("inf")])
def test_student_f32_refine_other_nu(ctx, nu):
    """FP32 outputs from the degree-7 cells: bulk, the whole table range, and
    the far tail (|z| > 10) including the largest finite floats."""
    rng = np.random.default_rng(7 + int(min(nu, 1e6) * 4))
    z = np.concatenate([rng.normal(size=20000), rng.uniform(-10.5, 10.5, 20000),
                        rng.uniform(10, 38, 2000) * rng.choice([-1, 1], 2000)]).astype(np.float32)
    ref = as_f32_output(oracle.student_t_map(z.astype(np.float64), nu))
    assert_close(run_t(ctx, z, nu), ref, RTOL_F32, "f32 nu=%s" % nu)


def test_student_f32_edges(ctx):
    z = np.array([0.0, -0.0, 1e-45, -1e-45, 1e-38, 1e-8, np.nan, np.inf, -np.inf, 9.999999, -10.0, 10.000001,
                  0.5, 2.0, 7.999999, 8.0, 8.000001, 3.4e38, -3.4e38], dtype=np.float32)
    for nu in (0.5, 1, 4, 30):
        got = run_t(ctx, z, nu)
        ref = as_f32_output(oracle.student_t_map(z.astype(np.float64), nu))
        assert_close(got, ref, RTOL_F32, "f32 edges nu=%s" % nu)
        assert np.signbit(got[1]) and np.signbit(got[3])
    for n in (1, 5, 1023, 1025, 2049, 9001):      # tiles of 1024 floats per wave
        zz = qi.normals(7, n, n).astype(np.float32)
        ref = as_f32_output(oracle.student_t_map(zz.astype(np.float64), 4.0))
        assert_close(run_t(ctx, zz, 4.0), ref, RTOL_F32, "f32 n=%d" % n)


@pytest.mark.parametrize("nu", [1, 4, 30])
def test_student_f32_correctly_rounded(ctx, normals, nu):
    """R is accurate to 1e-10, so the FP32 output is the oracle value rounded
    to nearest except where that value lies within 1e-9 (relative) of a
    midpoint between two floats."""
    z = normals.astype(np.float32)
    got = run_t(ctx, z, nu)
    ref = oracle.student_t_map(z.astype(np.float64), nu)
    r32 = ref.astype(np.float32)
    other = np.nextafter(r32, np.where(ref > r32, np.float32(np.inf), np.float32(-np.inf)))
    mid = (r32.astype(np.float64) + other.astype(np.float64)) / 2
    near_mid = np.abs(ref - mid) <= 1e-9 * np.abs(ref)
    bad = (got != r32) & ~near_mid & np.isfinite(ref)
    assert not bad.any(), (nu, int(bad.sum()), z[bad][:5], got[bad][:5], r32[bad][:5])


def test_student_full_size_sampled(ctx):
    """2^26 normals (the recycling workload) at nu = 4 in the benchmark's
    launch configuration; 2^14 sampled outputs plus the 64 largest |z|."""
    n = 1 << 26
    z = qi.recycle_normals(n)
    d = torch.from_numpy(z).cuda()
    t = torch.empty_like(d)
    qm.qm_recycle_student_t(ctx, d, t, 4.0)
    torch.cuda.synchronize()
    rng = np.random.default_rng(13)
    idx = np.unique(np.concatenate([rng.integers(0, n, 1 << 14), np.argsort(np.abs(z))[-64:]]))
    got = t[torch.from_numpy(idx).cuda()].cpu().numpy()
    assert_close(got, oracle.student_t_map(z[idx], 4.0), RTOL_F64, "2^26 sampled")


@pytest.mark.parametrize("nu", [1.0, 4.0, 30.0])
def test_student_f32_full_size_sampled(ctx, nu):
    """T-R (FP32 in/out) on the 2^26 recycling normals at the benchmark's
    launch shape (several grid-stride passes): 2^13 random outputs, whole
    runs of 1024 in the first, a middle and the last passes, the last 300,
    and every element with |z| > 4, against the oracle."""
    n = 1 << 26
    z = qi.recycle_normals(n).astype(np.float32)
    d = torch.from_numpy(z).cuda()
    t = torch.empty_like(d)
    qm.qm_recycle_student_t(ctx, d, t, nu)
    torch.cuda.synchronize()
    rng = np.random.default_rng(int(nu) + 40)
    runs = [np.arange(s, s + 1024) for s in (0, n // 2 + 3072, n - (n >> 4) + 1024, n - 2048)]
    idx = np.unique(np.concatenate([rng.integers(0, n, 1 << 13), np.arange(n - 300, n),
                                    np.flatnonzero(np.abs(z) > 4.0)] + runs))
    got = t[torch.from_numpy(idx).cuda()].cpu().numpy()
    ref = as_f32_output(oracle.student_t_map(z[idx].astype(np.float64), nu))
    rep = assert_close(got, ref, RTOL_F32, "T-R 2^26 nu=%s" % nu)
    print("T-R 2^26 nu", nu, len(idx), rep, flush=True)
    del d, t
    torch.cuda.empty_cache()
