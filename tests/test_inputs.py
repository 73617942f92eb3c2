"""The shared seeded input generator: determinism, independence of sub-ranges
and the distributional shape the workloads are defined by."""
import math

import numpy as np

import qm_inputs as qi


def test_philox_block_deterministic_and_key_sensitive():
    a = qi.philox4x32_10([0, 0, 0, 0], [0, 0])
    assert np.array_equal(a, qi.philox4x32_10([0, 0, 0, 0], [0, 0]))
    assert not np.array_equal(a, qi.philox4x32_10([1, 0, 0, 0], [0, 0]))
    assert not np.array_equal(a, qi.philox4x32_10([0, 0, 0, 0], [1, 0]))


def test_uniform53_open_interval_and_moments():
    u = qi.uniform53(0, 0, 1 << 20)
    assert u.min() > 0 and u.max() < 1
    assert abs(u.mean() - 0.5) < 2e-3 and abs(u.var() - 1 / 12) < 2e-3
    # every value is (k + 1/2) 2^-53 for an integer k
    k = u * 2.0 ** 53 - 0.5
    assert np.all(k == np.floor(k))


def test_counter_based_subrange():
    full = qi.normals(2, 0, 1 << 17)
    part = qi.normals(2, 0, 1 << 18)[: 1 << 17]
    assert np.array_equal(full, part)


def test_mixture_shape_f64():
    n = 1 << 21
    u = qi.mixture(1, 0, n, np.float64, 0.1, 1e-300)
    assert u.min() >= 1e-300 * 0.999 and u.max() <= 1.0
    # mirrored tail points below 2^-54 collapse to 1.0 (about 4.7% of all)
    frac_one = (u == 1.0).mean()
    assert 0.043 < frac_one < 0.051
    p = np.minimum(u, 1 - u)
    assert 0.105 < (p < 1e-2).mean() < 0.125


def test_mixture_shape_f32():
    u = qi.mixture(1, 0, 1 << 20, np.float32, 0.1, 1e-37)
    assert u.dtype == np.float32 and u.min() >= np.float32(1e-37) * 0.999


def test_normals_and_exponentials():
    z = qi.normals(2, 0, 1 << 20)
    assert abs(z.mean()) < 5e-3 and abs(z.std() - 1) < 5e-3
    assert np.abs(z).max() <= math.sqrt(-2 * math.log(2.0 ** -54))
    x = qi.exponentials(2, 1, 1 << 20)
    assert x.min() > 0 and abs(x.mean() - 1) < 5e-3
    assert x.max() <= -math.log(2.0 ** -54)
