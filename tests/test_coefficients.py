"""CPU checks of the fitted rationals the kernels evaluate (qm_coeffs.h),
each against the oracle: the coefficients as stored (FP64), evaluated
exactly in mpmath, so only the fit and the rounding of its coefficients are
under test, not the device's arithmetic."""
import math
import os
import re

import mpmath as mp
import numpy as np

import oracle

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_0901_0638_amd", "csrc", "qm_coeffs.h")


def arrays():
    s = open(HDR).read()
    out = {}
    for m in re.finditer(r"static constexpr double (\w+)\[\d+\] = \{([^}]*)\};", s):
        out[m.group(1)] = [float(x) for x in m.group(2).replace("\n", " ").split(",") if x.strip()]
    for m in re.finditer(r"static constexpr double (\w+) = ([0-9.eE+-]+);", s):
        out[m.group(1)] = float(m.group(2))
    return out


def horner(c, x):
    r = mp.mpf(0)
    for ck in c:
        r = r * x + mp.mpf(ck)
    return r


def test_central_piece_against_oracle():
    """w = q P8(r)/Q8(r), r = 0.2025 - q^2, for |q| <= 0.45: within 1e-16
    of the oracle (plus the oracle's own half-ulp) across the whole piece."""
    c = arrays()
    assert c["QM_CENTRAL_QMAX"] == 0.45 and c["QM_CENTRAL_X"] == 0.2025
    u = np.concatenate([np.linspace(0.05, 0.95, 2001), [0.05, 0.95, 0.5 + 1e-12, 0.5 - 1e-300]])
    ref = oracle.norm_quantile(u)
    with mp.workdps(40):
        for ui, wi in zip(u, ref):
            q = mp.mpf(ui) - mp.mpf("0.5")          # exact in mpmath
            if q == 0:
                continue
            r = mp.mpf(c["QM_CENTRAL_X"]) - q * q
            w = q * horner(c["QM_CENTRAL_P"], r) / horner(c["QM_CENTRAL_Q"], r)
            assert abs(w / mp.mpf(wi) - 1) <= 1e-16 + 2 ** -53, (ui, float(w), wi)


def test_deep_tail_piece_against_oracle():
    """Q(v) = s P7(s)/Q7(s), s = sqrt(v), on 42 < v <= 745 (u down to the
    smallest double)."""
    c = arrays()
    v = np.linspace(42.0, 744.0, 400)
    u = np.exp(-v) / 2
    ref = -oracle.norm_quantile(u)
    with mp.workdps(40):
        for vi, ui, wi in zip(v, u, ref):
            if ui == 0:
                continue
            vv = -mp.log(2 * mp.mpf(ui))            # the v of the stored u, exactly
            s = mp.sqrt(vv)
            w = s * horner(c["QM_TAIL_P"], s) / horner(c["QM_TAIL_Q"], s)
            assert abs(w / mp.mpf(wi) - 1) <= 5e-17 + 2 ** -53, (vi, float(w), wi)


def test_fp32_seed_and_mills_ratio():
    """The FP32 seed is a seed (1.2e-5); the Mills ratio M(x) = (1 - Phi(x))/phi(x)
    behind the exp -> normal correction step's erfc is good to 1.1e-12 on
    [0, 14.5], and the quantile's outer one to 8.6e-9 on [1.6, 14.5]."""
    c = arrays()
    with mp.workdps(30):
        for v in np.linspace(0.01, 103.0, 300):
            u = math.exp(-v) / 2
            ref = -oracle.norm_quantile(np.array([u]))[0]
            vv = -mp.log(2 * mp.mpf(u))
            z = vv * horner(c["QM_SEED_P"], vv) / horner(c["QM_SEED_Q"], vv)
            assert abs(z / ref - 1) <= 1.2e-5
        for x in np.linspace(0.0, 14.5, 300):
            m = horner(c["QM_MILLS_P"], x) / horner(c["QM_MILLS_Q"], x)
            ref = mp.erfc(mp.mpf(x) / mp.sqrt(2)) / 2 * mp.sqrt(2 * mp.pi) * mp.exp(mp.mpf(x) ** 2 / 2)
            assert abs(m / ref - 1) <= 1.1e-12
        for x in np.linspace(1.6, 14.5, 300):
            m = horner(c["QM_MILLS32_P"], x) / horner(c["QM_MILLS32_Q"], x)
            ref = mp.erfc(mp.mpf(x) / mp.sqrt(2)) / 2 * mp.sqrt(2 * mp.pi) * mp.exp(mp.mpf(x) ** 2 / 2)
            assert abs(m / ref - 1) <= 8.6e-9


def test_log_kernel_polynomial():
    """log m = 2f + f s R6(s), f = (m-1)/(m+1), s = f^2, on [sqrt(1/2), sqrt(2)]."""
    c = arrays()
    with mp.workdps(40):
        for m in np.linspace(math.sqrt(0.5), math.sqrt(2.0), 500):
            mm = mp.mpf(m)
            if mm == 1:
                continue
            f = (mm - 1) / (mm + 1)
            s = f * f
            lm = 2 * f + f * s * horner(c["QM_LOG_R"], s)
            assert abs(lm / mp.log(mm) - 1) <= 2e-18


def f32(x):
    return float(np.float32(x))


def test_fp32_central_pieces():
    """FP32+refine central piece: the seed (with FP32 coefficients) within
    2.7e-6, erf(z/sqrt2)/(2z) = E6(z^2) within 9.3e-9 and
    1/phi(z) = G3(z^2) within 1.1e-3, over |q| <= 0.45 (|z| <= 1.646)."""
    c = arrays()
    u = np.linspace(0.05, 0.95, 901)
    ref = oracle.norm_quantile(u)
    with mp.workdps(30):
        for ui, wi in zip(u, ref):
            q = mp.mpf(ui) - mp.mpf("0.5")
            if q == 0:
                continue
            r = mp.mpf(0.2025) - q * q
            z0 = q * horner([f32(x) for x in c["QM_C32_SP"]], r) / horner([f32(x) for x in c["QM_C32_SQ"]], r)
            assert abs(z0 / mp.mpf(wi) - 1) <= 2.7e-6, (ui, float(z0), wi)
            y = mp.mpf(wi) ** 2
            e = horner(c["QM_C32_E"], y) * 2 * mp.mpf(wi)
            assert abs(e / mp.erf(mp.mpf(wi) / mp.sqrt(2)) - 1) <= 9.3e-9
            g = horner(c["QM_C32_G"], y)
            assert abs(g / (mp.sqrt(2 * mp.pi) * mp.exp(y / 2)) - 1) <= 1.1e-3


def test_fp32_central_newton_step_emulated():
    """The whole central FP32+refine evaluation emulated in float32/float64
    (plain numpy, no FMA): within 4e-8 of the oracle before the final
    rounding (the error budget: 2.7 x 9.2e-9 from E, 2.9e-9 from G), so with
    the rounding's half ulp (6e-8) the FP32 result stays within 1e-7 of the
    oracle, inside the form's 2e-7."""
    c = arrays()
    u = np.linspace(0.05, 0.95, 20001).astype(np.float32).astype(np.float64)
    qd = u - 0.5
    qf = u.astype(np.float32) - np.float32(0.5)
    rf = np.float32(0.2025) - qf * qf
    sp = np.zeros_like(rf)
    for x in c["QM_C32_SP"]:
        sp = sp * rf + np.float32(x)
    sq = np.zeros_like(rf)
    for x in c["QM_C32_SQ"]:
        sq = sq * rf + np.float32(x)
    z0 = (qf * sp / sq).astype(np.float64)
    y = z0 * z0
    e = np.zeros_like(y)
    for x in c["QM_C32_E"]:
        e = e * y + x
    g = np.zeros_like(y)
    for x in c["QM_C32_G"]:
        g = g * y + x
    z1 = z0 - (z0 * e - qd) * g
    ref = oracle.norm_quantile(u)
    nz = ref != 0
    assert np.max(np.abs(z1[nz] / ref[nz] - 1)) <= 4e-8
    rounded = z1.astype(np.float32).astype(np.float64)
    assert np.max(np.abs(rounded[nz] / ref[nz] - 1)) <= 1e-7


def exp_refine7(a):
    """The correction step's e^a emulated in float64: a = k ln2 + r, the
    degree-7 Taylor polynomial in r, scaled by 2^k."""
    k = np.rint(a * 1.4426950408889634074)
    r = (a - k * 0.69314718055994528623) - k * 2.3190468138462996154e-17
    p = np.full_like(r, 1.0 / math.factorial(7))
    for i in range(6, -1, -1):
        p = p * r + 1.0 / math.factorial(i)
    return np.ldexp(p, k.astype(np.int64))


def test_fp32_outer_newton_step_emulated():
    """The outer FP32+refine evaluation emulated in float32/float64 (plain
    numpy, no FMA): v = -log(2p) and the seed v S4(v)/S5(v) in float32, then
    one FP64 Newton step x1 = x0 + M(x0) - p sqrt(2 pi) e^{x0^2/2} with the
    [1.6, 14.5] Mills ratio and the degree-7 exponential.  Over p from the
    smallest FP32 denormal to 0.05 the step lands within 3e-8 of the oracle
    before the final rounding (Newton's own error is x0^2 eps^2 / 2 for the
    seed's eps = 1.2e-5: 1.4e-8 at z = 14), and within 1e-7 after it."""
    c = arrays()
    p = np.unique(np.geomspace(1.4e-45, 0.05, 40001).astype(np.float32))
    p = p[p > 0]
    x = (p + p).astype(np.float32)
    sub = x < np.float32(2.0 ** -126)
    xs = np.where(sub, x.astype(np.float64) * 2.0 ** 32, x.astype(np.float64)).astype(np.float32)
    l2 = np.log2(xs.astype(np.float64)).astype(np.float32)
    ln2f = np.float32(0.693147180559945309)
    v = (-l2.astype(np.float64) * float(ln2f) + np.where(sub, 32.0 * float(ln2f), 0.0)).astype(np.float32)
    num = np.zeros_like(v)
    for k in c["QM_SEED_P"]:
        num = (num * v + np.float32(k)).astype(np.float32)
    num = (v * num).astype(np.float32)
    den = np.zeros_like(v)
    for k in c["QM_SEED_Q"]:
        den = (den * v + np.float32(k)).astype(np.float32)
    z0 = (num * (np.float32(1) / den)).astype(np.float32)
    x0 = z0.astype(np.float64)
    p_over_phi = p.astype(np.float64) * 2.5066282746310005024 * exp_refine7(0.5 * (x0 * x0))
    mp_ = np.zeros_like(x0)
    for k in c["QM_MILLS32_P"]:
        mp_ = mp_ * x0 + k
    mq = np.zeros_like(x0)
    for k in c["QM_MILLS32_Q"]:
        mq = mq * x0 + k
    x1 = x0 + (mp_ / mq - p_over_phi)
    ref = -oracle.norm_quantile(p.astype(np.float64))
    assert np.max(np.abs(x1 / ref - 1)) <= 3e-8
    rounded = x1.astype(np.float32).astype(np.float64)
    assert np.max(np.abs(rounded / ref - 1)) <= 1e-7


PAPER_HDR = os.path.join(os.path.dirname(__file__), "..", "paper_0901_0638_amd", "csrc", "qm_paper_coeffs.h")


def paper_arrays():
    """The paper's constants as the header spells them (decimal strings)."""
    s = open(PAPER_HDR).read()
    return {m.group(1): [x.strip().rstrip("f") for x in m.group(2).split(",") if x.strip()]
            for m in re.finditer(r"static constexpr (?:double|float) (\w+)\[\d+\] = \{([^}]*)\};", s)}


def psi_t2(v):
    """Psi(v) = Phi^{-1}((1 + v/sqrt(1 + v^2))/2) (Section 7.3), by mpmath."""
    return mp.sqrt(2) * mp.erfinv(v / mp.sqrt(1 + v * v))


def test_paper_branchless_meets_its_bound():
    """Section 7.2 / Appendix B: Q(v) = v p13(v)/q13(v) within the paper's
    5.4e-17 of Phi^{-1}(1 - e^{-v}/2) on 0 < v <= 42, with the printed
    decimals (a mistyped digit fails) and with the stored doubles (plus the
    coefficients' own rounding)."""
    c = paper_arrays()
    with mp.workdps(60):
        P = [mp.mpf(x) for x in c["QM_PAPER_P13"]]
        Q = [mp.mpf(x) for x in c["QM_PAPER_Q13"]]
        Pd = [mp.mpf(float(x)) for x in c["QM_PAPER_P13"]]
        Qd = [mp.mpf(float(x)) for x in c["QM_PAPER_Q13"]]
        for v in np.concatenate([np.linspace(0.001, 42.0, 700), [1e-12, 42.0]]):
            vv = mp.mpf(v)
            ref = mp.sqrt(2) * mp.erfinv(1 - mp.exp(-vv))
            assert abs(vv * horner(P, vv) / horner(Q, vv) / ref - 1) <= 5.4e-17, v
            assert abs(vv * horner(Pd, vv) / horner(Qd, vv) / ref - 1) <= 5.4e-17 + 2 ** -52, v


def test_paper_t2_rational_meets_its_bound():
    """Section 7.3 / Appendix C: Psi(v) = v P14(v)/Q15(v) within the paper's
    bound 5.55e-17 on 0 < v <= 15.5 (printed decimals and stored doubles);
    Psi(15.5) = 3.07933; and the rational leaves the bound just beyond
    v = 15.5, which is why the hybrid switches there."""
    c = paper_arrays()
    with mp.workdps(40):
        P = [mp.mpf(x) for x in c["QM_PAPER_T2_P14"]]
        Q = [mp.mpf(x) for x in c["QM_PAPER_T2_Q15"]]
        Pd = [mp.mpf(float(x)) for x in c["QM_PAPER_T2_P14"]]
        Qd = [mp.mpf(float(x)) for x in c["QM_PAPER_T2_Q15"]]
        for v in np.concatenate([np.linspace(0.001, 15.5, 700), [1e-9, 15.5]]):
            vv = mp.mpf(v)
            ref = psi_t2(vv)
            assert abs(vv * horner(P, vv) / horner(Q, vv) / ref - 1) <= 5.55e-17, v
            assert abs(vv * horner(Pd, vv) / horner(Qd, vv) / ref - 1) <= 5.55e-17 + 2 ** -52, v
        assert abs(psi_t2(mp.mpf(15.5)) - mp.mpf("3.07933")) < 5e-6
        v = mp.mpf(17)
        assert abs(v * horner(P, v) / horner(Q, v) / psi_t2(v) - 1) > 1e-14
    cst = re.search(r"QM_PAPER_T2_VMAX = ([0-9.]+);", open(PAPER_HDR).read())
    assert float(cst.group(1)) == 15.5


def test_t2_coordinate_emulated():
    """The T2 coordinate as the kernel forms it, v = |u - 1/2| / sqrt(u (1 - u))
    (plain numpy, correctly rounded sqrt), against its exact value: the
    product form stays within 5 ulps where the printed u - u*u loses up to
    5e-14 relative near u = 0.999."""
    u = np.concatenate([np.linspace(1e-3, 1 - 1e-3, 20001), 1 - np.geomspace(1.04e-3, 0.5, 2000),
                        np.geomspace(1e-3, 0.5, 2000)])
    v_prod = np.abs(u - 0.5) / np.sqrt(u * (1.0 - u))
    v_print = np.abs(u - 0.5) / np.sqrt(u - u * u)
    with mp.workdps(40):
        ex = np.array([float(abs(mp.mpf(x) - mp.mpf("0.5")) / mp.sqrt(mp.mpf(x) * (1 - mp.mpf(x)))) for x in u])
    nz = ex != 0
    assert np.all(v_prod[~nz] == 0)
    rel_prod = np.abs(v_prod[nz] / ex[nz] - 1)
    rel_print = np.abs(v_print[nz] / ex[nz] - 1)
    assert rel_prod.max() <= 5 * 2.0 ** -53
    assert rel_print.max() > 1e-14
