"""Pins of the oracle for the distribution of X1 + X2 + X3 (three
independent vectors whose axes are all Bernoulli; Introduction: sums of
multiple probability mass functions), CPU only.

sum3_naive is the definition; sum3_canonical is the per-axis method for three
operands (values at 0, 1, -1 and infinity).  Both are pinned to scipy's
direct N-D convolution, closed forms, the paper's worked-example style deltas,
invariants, exact rational arithmetic within the derived bound, and the
two-operand oracle; planted mistakes in a numpy transcription fail the pins.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.signal

import oracle
from tests import pins
from tests._numpy_method import sum3_per_axis

DTYPES = [np.float64, np.float32, np.int64]


def quad(i: int) -> int:
    """Bits of i read as base-4 digits (bit d -> digit of weight 4^d)."""
    q, p = 0, 1
    while i:
        q += (i & 1) * p
        p *= 4
        i >>= 1
    return q


def digits4(k: int, D: int):
    out = []
    for _ in range(D):
        out.append(k % 4)
        k //= 4
    return out[::-1]


def scipy_sum3(a, b, c):
    D = int(a.size).bit_length() - 1
    if D == 0:
        return a * b * c
    sh = (2,) * D
    return scipy.signal.convolve(scipy.signal.convolve(a.reshape(sh), b.reshape(sh), method="direct"),
                                 c.reshape(sh), method="direct").reshape(-1)


def ints(D, seed, lo=-16, hi=16):
    g = np.random.default_rng([83, D, seed])
    return [g.integers(lo, hi, 1 << D, dtype=np.int64) for _ in range(3)]


def masses(D, seed, dtype=np.float64):
    g = np.random.default_rng([89, D, seed])
    out = []
    for _ in range(3):
        u = g.random(1 << D)
        out.append((u / u.sum()).astype(dtype))
    return out


# ------------------------------------------------------------------ pins
def pin_scipy(impl, D):
    a, b, c = ints(D, 0)
    pins.assert_bitwise(impl(a, b, c), scipy_sum3(a, b, c), f"sum3 vs scipy D={D}")


def pin_all_ones(impl, dtype, D):
    """(1 + t)^3 = 1 + 3t + 3t^2 + t^3 on every axis: z[k] = 3^(digits of k
    equal to 1 or 2); every intermediate is an integer below 2^24 for D <= 7."""
    x = np.ones(1 << D, dtype=dtype)
    n = np.array([sum(d in (1, 2) for d in digits4(k, D)) for k in range(4 ** D)])
    pins.assert_bitwise(impl(x, x.copy(), x.copy()), (3 ** n).astype(dtype), f"sum3 all-ones D={D}")


def pin_deltas(impl, dtype, D):
    g = np.random.default_rng([97, D])
    for _ in range(4):
        i, j, l = (int(v) for v in g.integers(0, 1 << D, 3))
        xs = [np.zeros(1 << D, dtype=dtype) for _ in range(3)]
        xs[0][i], xs[1][j], xs[2][l] = 3, 5, 7
        expect = np.zeros(4 ** D, dtype=dtype)
        expect[quad(i) + quad(j) + quad(l)] = 105
        pins.assert_bitwise(impl(*xs), expect, f"sum3 deltas D={D}")


def pin_sum_int(impl, D):
    a, b, c = ints(D, 1, 0, 16)
    assert int(impl(a, b, c).sum()) == int(a.sum()) * int(b.sum()) * int(c.sum())


def pin_via_pair_convolution(impl, D):
    """int64: X1 + X2 by the two-operand oracle (Algorithm 1), then + X3 by
    the definition of convolution over {0,1,2}^D x {0,1}^D (scipy)."""
    a, b, c = ints(D, 2)
    z12 = oracle.naive(a, b)
    expect = scipy.signal.convolve(z12.reshape((3,) * D), c.reshape((2,) * D), method="direct").reshape(-1) \
        if D else z12 * c
    pins.assert_bitwise(impl(a, b, c), expect, f"sum3 via the pair convolution D={D}")


def exact_sum3(a, b, c):
    D = int(a.size).bit_length() - 1
    z = [Fraction(0)] * (4 ** D)
    fa, fb, fc = ([Fraction(float(v)) for v in t] for t in (a, b, c))
    q = [quad(i) for i in range(1 << D)]
    for i in range(1 << D):
        for j in range(1 << D):
            ab = fa[i] * fb[j]
            for l in range(1 << D):
                z[q[i] + q[j] + q[l]] += ab * fc[l]
    return z


def pin_exact_bound(impl, dtype, D, kind):
    if kind == "mass":
        a, b, c = masses(D, 3, dtype)
    else:
        g = np.random.default_rng([101, D])
        a, b, c = (g.uniform(-1, 1, 1 << D).astype(dtype) for _ in range(3))
    z = impl(a, b, c)
    ex = exact_sum3(a, b, c)
    B = oracle.sum3_bound(a.astype(np.float64), b.astype(np.float64), c.astype(np.float64))
    u = oracle.unit_roundoff(dtype)
    tol = Fraction((5 * D + 2) * u)
    worst = 0.0
    for k in range(4 ** D):
        err = abs(Fraction(float(z[k])) - ex[k])
        assert err <= tol * Fraction(float(B[k])), f"bound violated at k={k}"
        if B[k] > 0:
            worst = max(worst, float(err / Fraction(float(B[k]))) / u)
    return worst


IMPLS = {"naive": oracle.sum3_naive, "canonical": oracle.sum3_canonical}


@pytest.mark.parametrize("impl", sorted(IMPLS))
@pytest.mark.parametrize("D", [0, 1, 2, 4, 6])
def test_sum3_scipy_definition(impl, D):
    pin_scipy(IMPLS[impl], D)


@pytest.mark.parametrize("impl", sorted(IMPLS))
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("D", [0, 1, 3, 6])
def test_sum3_all_ones(impl, dtype, D):
    pin_all_ones(IMPLS[impl], dtype, D)


@pytest.mark.parametrize("impl", sorted(IMPLS))
@pytest.mark.parametrize("dtype", DTYPES)
def test_sum3_deltas(impl, dtype):
    pin_deltas(IMPLS[impl], dtype, 5)


@pytest.mark.parametrize("impl", sorted(IMPLS))
def test_sum3_sum_invariant(impl):
    pin_sum_int(IMPLS[impl], 6)


@pytest.mark.parametrize("D", [0, 1, 3, 7])
def test_sum3_via_pair_convolution(D):
    pin_via_pair_convolution(oracle.sum3_canonical, D)


@pytest.mark.parametrize("D", [7, 9])
def test_sum3_canonical_equals_definition_int64(D):
    a, b, c = ints(D, 4)
    pins.assert_bitwise(oracle.sum3_canonical(a, b, c), oracle.sum3_naive(a, b, c), f"D={D}")


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("D,kind", [(1, "signed"), (2, "signed"), (3, "mass"), (3, "signed")])
def test_sum3_exact_within_bound(dtype, D, kind):
    pin_exact_bound(oracle.sum3_canonical, dtype, D, kind)


def test_sum3_float_order_is_the_transcription():
    """The oracle's float arithmetic is the per-axis method in the stated
    order (forward ascending, (x1^ x2^) x3^, inverse descending): an
    independent numpy transcription gives the same bits."""
    for D in (1, 4, 7):
        for dt in (np.float64, np.float32):
            a, b, c = masses(D, 5, dt)
            pins.assert_bitwise(oracle.sum3_canonical(a, b, c), sum3_per_axis(a, b, c), f"D={D} {dt}")


def test_sum3_direct_at_matches_definition():
    D = 6
    a, b, c = ints(D, 6, 0, 16)
    ks = np.arange(4 ** D, dtype=np.uint64)
    ref = oracle.sum3_naive(a, b, c).astype(np.float64)
    got = oracle.sum3_direct_at(a.astype(np.float64), b.astype(np.float64), c.astype(np.float64), ks)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("D", [8, 10])
def test_sum3_mass_error_within_bound_vs_direct(D):
    a, b, c = masses(D, 7)
    z = oracle.sum3_canonical(a, b, c)
    ks = np.random.default_rng([103, D]).integers(0, 4 ** D, 2048, dtype=np.uint64)
    ref = oracle.sum3_direct_at(a, b, c, ks)
    B = oracle.sum3_bound(a, b, c)[ks.astype(np.int64)]
    err = np.abs(z[ks.astype(np.int64)] - ref)
    assert np.all(err <= (5 * D + 2) * 2.0 ** -53 * B + 2.0 ** -60 * np.abs(ref))
    r = float(np.max(err / B) / 2.0 ** -53)
    pins.error_ratio_band(r, D, lo=0.02)


# ----------------------------------------------- the bound, pinned by closed forms
def test_sum3_bound_all_ones():
    """x1 = x2 = x3 = 1: per axis F4a gives (1, 2, 2, 1), the product
    (1, 8, 8, 1) and |G4| (1, 9, 9, 1): B = 9^(digits equal to 1 or 2)."""
    for D in (0, 1, 3, 6):
        x = np.ones(1 << D)
        n = np.array([sum(d in (1, 2) for d in digits4(k, D)) for k in range(4 ** D)])
        pins.assert_bitwise(oracle.sum3_bound(x, x.copy(), x.copy()), 9.0 ** n, f"D={D}")


def test_sum3_bound_rank1():
    """Outer-product inputs: per axis (P0, P1 + Pi, P1 + P0, Pi) with P0 the
    product of |a|, Pi of |b| and P1 of (|a| + |b|) over the three operands."""
    for D in (1, 3, 5):
        fs = [pins.rank1_factors(D, s) for s in (0, 1000, 2000)]
        per_axis = []
        for d in range(D):
            a = [abs(f[d][0]) for f in fs]
            b = [abs(f[d][1]) for f in fs]
            P0, Pi = a[0] * a[1] * a[2], b[0] * b[1] * b[2]
            P1 = (a[0] + b[0]) * (a[1] + b[1]) * (a[2] + b[2])
            per_axis.append((P0, P1 + Pi, P1 + P0, Pi))
        expect = pins.rank1(per_axis)
        got = oracle.sum3_bound(*(pins.rank1(f) for f in fs))
        pins.assert_bitwise(got, expect, f"rank-1 D={D}")


# --------------------------------------------------------------- pin power
def sum3_pins(impl):
    failed = []
    checks = {
        "scipy": lambda: [pin_scipy(impl, D) for D in (2, 4)],
        "all_ones": lambda: pin_all_ones(impl, np.float64, 4),
        "deltas": lambda: pin_deltas(impl, np.int64, 4),
        "sum": lambda: pin_sum_int(impl, 4),
        "bound": lambda: [pin_exact_bound(impl, np.float64, 3, k) for k in ("mass", "signed")],
        "order": lambda: pins.assert_bitwise(impl(*masses(5, 9)), oracle.sum3_canonical(*masses(5, 9)), "order"),
    }
    for name, fn in checks.items():
        try:
            fn()
        except AssertionError:
            failed.append(name)
    return failed


MUTANTS = {
    "plus_one_instead_of_minus_one": dict(minus_point=False),
    "no_halving": dict(halve=False),
    "inverse_ascending": dict(inverse_order="asc"),
    "forward_descending": dict(forward_order="desc"),
    "top_term_kept": dict(keep_pi=True),
    "product_right_assoc": dict(assoc="right"),
}


def test_sum3_unmodified_transcription_passes():
    assert sum3_pins(lambda a, b, c: sum3_per_axis(a, b, c)) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_sum3_mutant_is_caught(name):
    assert sum3_pins(lambda a, b, c: sum3_per_axis(a, b, c, **MUTANTS[name])), name


def test_sum3_swapped_operand_is_caught():
    assert sum3_pins(lambda a, b, c: sum3_per_axis(a, b, a))
