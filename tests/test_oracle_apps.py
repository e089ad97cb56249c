"""Pins for the oracle's application functions (Discussion and Introduction):
the carry-free 1-D convolution and the distribution of a difference X - Y.

Each is pinned to something computed another way:
  - the Discussion's worked example (7 and 5 give digits (2, 1, 2));
  - carrying the output digits (value sum_a d_a 2^a) must give numpy's
    ordinary 1-D convolution, for every length n, power of two or not;
  - for the difference, the carried value sum_a (d_a - 1) 2^a is i - j, so
    the same collapse must give numpy's 1-D correlation;
  - the D = 1 case written out, deltas, symmetry, total mass.
"""
import numpy as np
import pytest

import oracle
from tests import pins


def carried_values(D, offset=0):
    """Value sum_a (digit_a(k) - offset) * 2^a of every ternary index k."""
    vals = np.zeros(3 ** D, dtype=np.int64)
    for k in range(3 ** D):
        v, kk, w = 0, k, 1
        for _ in range(D):
            v += (kk % 3 - offset) * w
            kk //= 3
            w *= 2
        vals[k] = v
    return vals


def test_carryfree_worked_example():
    g = pins.golden("carry_free_example.json")
    n = 1 << g["D"]
    x = np.zeros(n, dtype=np.int64)
    y = np.zeros(n, dtype=np.int64)
    x[g["i"]] = 1
    y[g["j"]] = 1
    z = oracle.carryfree_naive(x, y)
    assert np.flatnonzero(z).tolist() == [g["k_flat"]]
    assert pins.ternary_digits(g["k_flat"], g["D"]) == g["k_digits_msb_first"]


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13, 16, 100, 256])
def test_carryfree_collapses_to_ordinary_convolution(n):
    g = np.random.default_rng([61, n])
    x = g.integers(-20, 20, n, dtype=np.int64)
    y = g.integers(-20, 20, n, dtype=np.int64)
    z = oracle.carryfree_naive(x, y)
    D = max(0, (n - 1).bit_length())
    ordinary = np.zeros(2 * (1 << D) - 1, dtype=np.int64)
    np.add.at(ordinary, carried_values(D), z)
    ref = np.convolve(x, y)
    assert np.array_equal(ordinary[:ref.size], ref)
    assert not ordinary[ref.size:].any()


@pytest.mark.parametrize("D", [0, 1, 3, 6])
def test_carryfree_equals_hypercube_definition_for_powers_of_two(D):
    g = np.random.default_rng([62, D])
    x = g.integers(0, 16, 1 << D, dtype=np.int64)
    y = g.integers(0, 16, 1 << D, dtype=np.int64)
    pins.assert_bitwise(oracle.carryfree_naive(x, y), pins.scipy_definition(x, y), "carry-free vs scipy")


def test_carryfree_pads_with_zeros():
    g = np.random.default_rng(63)
    x = g.random(11)
    y = g.random(11)
    xp = np.concatenate([x, np.zeros(5)])
    yp = np.concatenate([y, np.zeros(5)])
    assert np.array_equal(oracle.carryfree_naive(x, y), oracle.carryfree_naive(xp, yp))


def test_difference_d1_written_out():
    x = np.array([2, 3], dtype=np.int64)
    y = np.array([5, 7], dtype=np.int64)
    # digit 0: X - Y = -1 (x0 y1); digit 1: 0 (x0 y0 + x1 y1); digit 2: +1 (x1 y0)
    assert oracle.difference_naive(x, y).tolist() == [2 * 7, 2 * 5 + 3 * 7, 3 * 5]


@pytest.mark.parametrize("D", [1, 2, 4, 7])
def test_difference_collapses_to_correlation(D):
    g = np.random.default_rng([64, D])
    x = g.integers(-9, 10, 1 << D, dtype=np.int64)
    y = g.integers(-9, 10, 1 << D, dtype=np.int64)
    z = oracle.difference_naive(x, y)
    n = 1 << D
    diff = np.zeros(2 * n - 1, dtype=np.int64)        # index m + n - 1 for m = i - j
    np.add.at(diff, carried_values(D, offset=1) + n - 1, z)
    assert np.array_equal(diff, np.convolve(x, y[::-1]))


@pytest.mark.parametrize("D", [2, 5])
def test_difference_deltas_symmetry_and_mass(D):
    n = 1 << D
    for i, j in [(0, n - 1), (n - 1, 0), (1, 2), (n // 2, n // 2)]:
        x = np.zeros(n, dtype=np.int64)
        y = np.zeros(n, dtype=np.int64)
        x[i] = 1
        y[j] = 1
        z = oracle.difference_naive(x, y)
        digits = [((i >> (D - 1 - a)) & 1) - ((j >> (D - 1 - a)) & 1) + 1 for a in range(D)]
        k = 0
        for d in digits:
            k = 3 * k + d
        assert np.flatnonzero(z).tolist() == [k]
    g = np.random.default_rng([65, D])
    x = g.integers(0, 50, n, dtype=np.int64)
    y = g.integers(0, 50, n, dtype=np.int64)
    z = oracle.difference_naive(x, y)
    # X - Y and Y - X are mirror images: digit d <-> 2 - d, i.e. k <-> 3^D - 1 - k
    assert np.array_equal(z, oracle.difference_naive(y, x)[::-1])
    assert z.sum() == x.sum() * y.sum()


# ------------------------------------------ max-convolution and its p-norm

def brute_maxconv(x, y, D):
    """max over (i, j) of x[i] y[j] with output digits bit(i) + bit(j), by
    enumerating every pair (independent of the oracle's index logic)."""
    z = np.full(3 ** D, -np.inf)
    for i in range(1 << D):
        for j in range(1 << D):
            k = 0
            for a in range(D - 1, -1, -1):
                k = 3 * k + ((i >> a) & 1) + ((j >> a) & 1)
            z[k] = max(z[k], x[i] * y[j])
    return z


def ones_count(D):
    return np.array([sum(d == 1 for d in pins.ternary_digits(k, D)) for k in range(3 ** D)])


@pytest.mark.parametrize("D", [0, 1, 2, 4, 6])
def test_maxconv_matches_brute_force(D):
    g = np.random.default_rng([66, D])
    x = g.random(1 << D)
    y = g.random(1 << D)
    ks = np.arange(3 ** D, dtype=np.uint64)
    assert np.array_equal(oracle.maxconv_at(x, y, ks), brute_maxconv(x, y, D))


@pytest.mark.parametrize("D", [1, 4, 7])
def test_pnorm_brackets_the_maximum_and_converges(D):
    g = np.random.default_rng([67, D])
    x = g.random(1 << D)
    y = g.random(1 << D)
    ks = np.arange(3 ** D, dtype=np.uint64)
    zmax = oracle.maxconv_at(x, y, ks)
    s = ones_count(D)
    # p = 1 is the ordinary convolution (definition sum)
    assert np.allclose(oracle.pnorm_at(x, y, 1.0, ks), oracle.direct_at(x, y, ks), rtol=1e-15, atol=0)
    for p in (2.0, 7.5, 64.0, 4096.0):
        zp = oracle.pnorm_at(x, y, p, ks)
        assert np.all(zp >= zmax * (1 - 1e-15))
        assert np.all(zp <= zmax * 2.0 ** (s / p) * (1 + 1e-15))
    # scaling an input scales the estimate
    assert np.allclose(oracle.pnorm_at(3 * x, y, 9.0, ks), 3 * oracle.pnorm_at(x, y, 9.0, ks), rtol=1e-14)


def test_pnorm_single_term_is_exact():
    """With one nonzero pair per output the p-norm is that product for any p."""
    x = np.array([0.0, 0.0, 0.0, 0.75])
    y = np.array([0.0, 0.5, 0.0, 0.0])
    ks = np.arange(9, dtype=np.uint64)
    for p in (1.0, 3.0, 100.0):
        z = oracle.pnorm_at(x, y, p, ks)
        assert np.flatnonzero(z).tolist() == [oracle.tern(3) + oracle.tern(1)]
        assert z.max() == 0.375
