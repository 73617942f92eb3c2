"""CPU checks of the Student t table builder (no GPU): its recycling-ODE
solution and the per-cell polynomials against the oracle and the paper."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
import paper_0901_0638_amd as qm
from tests import _golden

NUS = [0.3, 0.4, 0.5, 1, 2, 3, 4, 7.5, 10, 30, 50]


def grid():
    rng = np.random.default_rng(21)
    return np.concatenate([np.linspace(-10.4, 10.4, 401), rng.normal(size=200), [1e-300, 1e-9, 3.99999999, 4.0, 4.00000001, 8.652]])


@pytest.mark.parametrize("nu", NUS)
def test_dense_rode_solution_matches_oracle(nu):
    """The two-leg Taylor-series solution of the recycling ODE (forward from
    the centre conditions, backward from the tail condition) agrees with the
    oracle's incomplete-beta inversion to a rounding."""
    z = grid()
    q = qm.debug_student_dense(nu, z)
    ref = oracle.student_t_map(z, nu)
    nz = ref != 0
    assert np.all(q[~nz] == 0)
    rel = np.abs(q[nz] / ref[nz] - 1)
    assert rel.max() <= 2.3e-16, (nu, rel.max(), z[nz][np.argmax(rel)])


def test_dense_large_nu_against_mpmath():
    """nu = 1000: the oracle's log-gamma cancellation grows with nu, so the
    reference here is an mpmath betainc root at 50 digits."""
    nu = 1000.0
    z = np.array([0.3, -1.7, 2.5, 4.2, 6.0, 8.5, 10.0])
    q = qm.debug_student_dense(nu, z)
    with mp.workdps(50):
        a = mp.mpf(nu) / 2
        for zi, qi in zip(z, q):
            s = abs(mp.mpf(zi))
            target = mp.erfc(s / mp.sqrt(2)) / 2
            f = lambda t: mp.log(mp.betainc(a, mp.mpf(1) / 2, 0, nu / (nu + t ** 2), regularized=True) / 2) - mp.log(target)
            T = abs(mp.mpf(qi))
            r = mp.findroot(f, (T * (1 - mp.mpf("1e-10")), T * (1 + mp.mpf("1e-10"))), solver="illinois")
            assert abs(T / r - 1) <= 2.3e-16, (zi, qi)


def test_dense_reproduces_paper_t4_series():
    """Section 3.5 central series (c_0..c_10 for n = 4) near the centre."""
    with mp.workdps(30):
        c = [mp.mpf(x[0]) for x in _golden.keyed("paper_t4_series.txt")["c"]]
        z = np.linspace(-0.5, 0.5, 51)
        q = qm.debug_student_dense(4.0, z)
        for zi, qi in zip(z, q):
            if zi == 0:
                continue
            y = mp.mpf(zi) ** 2
            ref = mp.mpf(zi) * mp.polyval(c[::-1], y)
            assert abs(mp.mpf(qi) / ref - 1) <= 2.5e-16


def eval_table_exact(c, coef, z):
    """Evaluate the stored polynomial exactly (mpmath) at the exact y = z^2:
    isolates the table's content from the device's rounding."""
    out = []
    with mp.workdps(40):
        for zi in z:
            y = mp.mpf(zi) ** 2
            if y > c.y_max:
                out.append(float("nan"))
                continue
            j = min(int(float(y) * c.inv_h), c.ncell - 1)
            d = y - (j * mp.mpf(c.h) + mp.mpf(c.centre_offset))
            r = mp.mpf(0)
            for ck in coef[j]:
                r = r * d + mp.mpf(float(ck))
            out.append(float(mp.mpf(zi) * r))
    return np.array(out)


def check_cells(c, degree):
    assert c.degree == degree and c.stride == degree + 1
    assert 1 <= c.nlds <= c.ncell <= 200 * 8 / c.h
    assert c.y_lds == c.nlds * c.h and c.y_lds >= 100.0 and c.y_lds - c.h < 100.0
    assert c.y_max == c.ncell * c.h and c.y_max - c.h < 40.0 ** 2
    assert math.log2(c.h) == int(math.log2(c.h)) and c.centre_offset == c.h / 2 and c.inv_h == 1 / c.h


def table_grid(c):
    """The table's whole range: dense in y <= 100, then up to y_max."""
    z = grid()
    zt = np.linspace(10.0, math.sqrt(c.y_max) * (1 - 1e-12), 97)
    z = np.concatenate([z[np.abs(z) <= 10], zt, -zt[::7]])
    return z[z != 0]


@pytest.mark.parametrize("nu", NUS + [100, 1e3, 1e5])
def test_table_polynomials_match_oracle(nu):
    """FP64 cells (degree 7 where at most 200 of them cover y <= 100, which
    holds from nu = 3 on, else degree 15): within a few FP64 rounding errors
    of the oracle's incomplete-beta inversion everywhere in the table's
    range."""
    h, c, coef = qm.debug_student_table(nu)
    assert h.identity == 0
    check_cells(c, 7 if nu >= 3 else 15)
    assert c.nlds <= (200 if c.degree == 7 else 480)
    assert c.nlds * (c.degree + 2) * 8 <= 57088        # the LDS the batch kernel leaves a table
    assert c.max_rel_err < 3e-16
    z = table_grid(c)
    t = eval_table_exact(c, coef, z)
    ref = oracle.student_t_map(z, nu)
    # below nu = 1/2 the cells run on to where t overflows, as the map does
    fin = np.isfinite(ref)
    assert np.array_equal(np.isinf(t), ~fin), (nu, z[np.isinf(t) != ~fin][:3])
    rel = np.abs(t[fin] / ref[fin] - 1)
    assert rel.max() <= 4e-16, (nu, rel.max(), z[fin][np.argmax(rel)])
    if nu < 0.5:
        assert not fin.all() and c.y_max > 400


@pytest.mark.parametrize("nu", NUS + [0.75, 1.5])
def test_fp32_cells_match_oracle(nu):
    """FP32-output cells (degree 7, fitted to 1e-10): R within 1e-10 of the
    oracle, far below FP32's half-ulp of 6e-8, so the one rounding to FP32
    decides the result."""
    h, c, coef = qm.debug_student_table(nu, "f32")
    _, c64, _ = qm.debug_student_table(nu)
    check_cells(c, 7)
    if c64.degree == 7:          # same degree, looser tolerance: cells at least as wide
        assert c.h >= c64.h
    assert c.max_rel_err < 1e-10
    z = table_grid(c)
    t = eval_table_exact(c, coef, z)
    ref = oracle.student_t_map(z, nu)
    rel = np.abs(t / ref - 1)
    assert rel.max() <= 1.2e-10, (nu, rel.max(), z[np.argmax(rel)])


def tail_formula(z, nu):
    """Two-term tail of Section 3.5 with exact constants (mpmath):
    t = sqrt(nu) w^{-1/nu} (1 - (nu+1)/(2(nu+2)) w^{2/nu}), w = K q(|z|)."""
    with mp.workdps(40):
        nu = mp.mpf(nu)
        lk = mp.log(nu) + mp.log(mp.pi) / 2 + mp.loggamma(nu / 2) - mp.loggamma((nu + 1) / 2)
        lw = lk + mp.log(mp.erfc(abs(mp.mpf(z)) / mp.sqrt(2)) / 2)
        a = -(nu + 1) / (2 * (nu + 2))
        return float(mp.sqrt(nu) * mp.exp(-lw / nu) * (1 + a * mp.exp(2 * lw / nu)))


@pytest.mark.parametrize("nu", [1, 4, 8, 10, 20, 30, 50, 80])
def test_tail_formula_accurate_beyond_cells(nu):
    """Beyond each cell set's y_max the device uses the two-term tail
    formula; the builder extends the cells until that formula meets the
    cells' tolerance, checked here against the oracle from the cells' edge to
    the largest normal quantile of a double."""
    _, c64, _ = qm.debug_student_table(nu)
    _, c32, _ = qm.debug_student_table(nu, "f32")
    for c, tol in ((c64, 3e-16), (c32, 1e-10)):
        z0 = math.sqrt(c.y_max)
        if z0 >= 38.5:
            continue
        z = np.linspace(z0, 38.5, 9)
        ref = oracle.student_t_map(z, nu)
        for zi, r in zip(z, ref):
            f = tail_formula(zi, nu)
            if np.isinf(r):          # beyond DBL_MAX (small nu): both overflow
                assert f == r, (nu, zi, f)
            else:
                assert abs(f / r - 1) <= tol, (nu, c.degree, zi)
    # and just inside the edge the formula alone would not do: the extension is needed
    if c64.ncell > c64.nlds:
        z = math.sqrt(c64.y_max) - 2.0
        r = oracle.student_t_map(np.array([z]), nu)[0]
        assert abs(tail_formula(z, nu) / r - 1) > 2e-17


def test_dense_far_tail_matches_oracle():
    """The backward leg anchored past |z| = 38: the dense solution agrees
    with the oracle out there too."""
    z = np.array([10.5, 15.0, 22.0, 30.0, 38.4, -35.0])
    for nu in (3, 30, 100):
        q = qm.debug_student_dense(nu, z)
        ref = oracle.student_t_map(z, nu)
        rel = np.abs(q / ref - 1)
        assert rel.max() <= 2.3e-16, (nu, rel)
    with pytest.raises(ValueError):
        qm.debug_student_dense(4.0, np.array([40.5]))


def test_tables_share_tail_constants_and_block():
    """Both cell sets live in one coefficient block, without overlap, and
    the header's tail constants are the Section 3.5 ones."""
    nu = 3.0
    h, c64, _ = qm.debug_student_table(nu)
    _, c32, _ = qm.debug_student_table(nu, "f32")
    assert c64.coef_offset == 0 and c32.coef_offset == c64.ncell * c64.stride
    assert h.tail_a[0] == -(nu + 1) / (2 * (nu + 2))
    with mp.workdps(30):
        lk = mp.log(nu) + mp.log(mp.pi) / 2 + mp.loggamma(nu / 2) - mp.loggamma((nu + 1) / 2)
        assert abs(h.log_K - float(lk)) <= 2e-16 * abs(float(lk))


def test_table_identity_and_cornish_fisher():
    h, c, coef = qm.debug_student_table(float("inf"))
    assert h.identity == 1 and c.ncell == 0 and coef.size == 0
    nu = 2e5
    for which, degree in (("f64", 7), ("f32", 7)):
        h, c, coef = qm.debug_student_table(nu, which)
        assert c.ncell == 1 and c.inv_h == 0 and c.degree == degree
        # the cell polynomial is A&S 26.7.5 (Section 3.4) in y = z^2
        for z in (0.5, 2.0, 6.0):
            y = z * z
            r = np.polyval(coef[0], y)
            cf = (1 + (y + 1) / (4 * nu) + (5 * y * y + 16 * y + 3) / (96 * nu ** 2)
                  + (3 * y ** 3 + 19 * y * y + 17 * y - 15) / (384 * nu ** 3)
                  + (79 * y ** 4 + 776 * y ** 3 + 1482 * y * y - 1920 * y - 945) / (92160 * nu ** 4))
            assert abs(r / cf - 1) < 1e-15


def test_table_rejects_small_nu():
    with pytest.raises(ValueError):
        qm.debug_student_table(0.25)
