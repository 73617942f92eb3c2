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


def test_philox_known_answers():
    """Philox4x32-10 against the known-answer vectors published with the
    generator (Salmon, Moraes, Dror & Shaw, SC'11, Random123 distribution):
    counter and key all zeros, all ones, and the digits of pi."""
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for ctr, key, want in kat:
        got = qi.philox4x32_10(ctr, key)
        assert [int(x) for x in got] == want, (ctr, key, [hex(int(x)) for x in got])


def test_u23_formula_every_value_exact_and_open():
    """Every 23-bit k (with arbitrary low bits in the word) gives exactly
    (2k + 1) / 2^24 in FP32, so the largest value, from word 0xFFFFFFFF, is
    1 - 2^-24 < 1 and the smallest 2^-24 > 0."""
    k = np.arange(1 << 23, dtype=np.uint64)
    low = (k * 2654435761) & 0x1FF
    words = ((k << 9) | low).astype(np.uint32)
    u = qi.u23_of_words(words)
    assert np.array_equal(u.astype(np.float64) * 2.0 ** 24, (2 * k + 1).astype(np.float64))
    top = qi.u23_of_words([0xFFFFFFFF, 0])
    assert top[0] == np.float32(1 - 2.0 ** -24) and top[0] < 1 and top[1] == np.float32(2.0 ** -24)


def test_u53_formula_rounding():
    """(k + 1/2) 2^-53 rounded to nearest: exact below k = 2^52, the
    even neighbour of the tie above, and 1.0 for the largest k."""
    from fractions import Fraction
    rng = np.random.default_rng(5)
    k = np.concatenate([rng.integers(0, 1 << 53, 4096, dtype=np.uint64),
                        np.array([0, 1, (1 << 52) - 1, 1 << 52, (1 << 52) + 1, (1 << 53) - 2, (1 << 53) - 1],
                                 dtype=np.uint64)])
    bits = (k << np.uint64(11)) | np.uint64(0x5A5)
    u = qi.u53_of_bits(bits)
    want = np.array([float(Fraction(2 * int(x) + 1, 1 << 54)) for x in k])
    assert np.array_equal(u, want)
    assert u[-1] == 1.0 and u[-2] < 1.0
    assert np.all(u[k < (1 << 52)] * 2.0 ** 54 == (2 * k[k < (1 << 52)] + 1).astype(np.float64))


def test_stream_uses_the_formulas():
    """The stream's uniforms are the formulas applied to its Philox words:
    FP64 element e from words (0,1) or (2,3) of block e/2, FP32 element e
    from word e mod 4 of block e/4."""
    seed, stream, n = 11, 3, 64
    u64 = qi.uniform53(seed, stream, n)
    u32 = qi.uniform23(seed, stream, n)
    for e in range(n):
        b = qi.philox4x32_10([e >> 1, 0, 0, 0], [seed, stream])
        lo, hi = (int(b[0]), int(b[1])) if e % 2 == 0 else (int(b[2]), int(b[3]))
        assert u64[e] == qi.u53_of_bits([(hi << 32) | lo])[0]
        b4 = qi.philox4x32_10([e >> 2, 0, 0, 0], [seed, stream])
        assert u32[e] == qi.u23_of_words([int(b4[e & 3])])[0]
