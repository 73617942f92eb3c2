"""CPU checks of the Student t table builder (no GPU): its recycling-ODE
solution and the per-cell polynomials against the oracle and the paper."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
import paper_0901_0638_amd as qm
from tests import _golden

NUS = [0.5, 1, 2, 3, 4, 7.5, 10, 30, 50]


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


def eval_table_exact(h, coef, z):
    """Evaluate the stored polynomial exactly (mpmath) at the exact y = z^2:
    isolates the table's content from the device's rounding."""
    out = []
    with mp.workdps(40):
        for zi in z:
            y = mp.mpf(zi) ** 2
            if y > h.y_max:
                out.append(float("nan"))
                continue
            j = min(int(float(y) * h.inv_h), h.ncell - 1)
            d = y - (j * mp.mpf(h.h) + mp.mpf(h.centre_offset))
            r = mp.mpf(0)
            for ck in coef[j]:
                r = r * d + mp.mpf(float(ck))
            out.append(float(mp.mpf(zi) * r))
    return np.array(out)


@pytest.mark.parametrize("nu", NUS)
def test_table_polynomials_match_oracle(nu):
    h, coef, err = qm.debug_student_table(nu)
    assert h.identity == 0 and h.degree == 15 and h.stride == 16
    assert 1 <= h.ncell <= 512 and h.y_max >= 100.0
    assert math.log2(h.h) == int(math.log2(h.h))
    assert err < 3e-16
    z = grid()
    z = z[np.abs(z) <= 10]
    z = z[z != 0]
    t = eval_table_exact(h, coef, z)
    ref = oracle.student_t_map(z, nu)
    rel = np.abs(t / ref - 1)
    assert rel.max() <= 4e-16, (nu, rel.max(), z[np.argmax(rel)])


def test_table_identity_and_cornish_fisher():
    h, coef, _ = qm.debug_student_table(float("inf"))
    assert h.identity == 1 and h.ncell == 0
    nu = 2e5
    h, coef, _ = qm.debug_student_table(nu)
    assert h.ncell == 1 and h.inv_h == 0
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
