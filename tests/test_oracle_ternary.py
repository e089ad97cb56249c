"""Pins of the oracle for the convolution of two ternary cubes {0,1,2}^D
(the next link of a chain of sums: the distribution of X1 + X2 + X3 + X4 is
the convolution of the pair sums X1 + X2 and X3 + X4), CPU only.

ternary_naive is the definition; ternary_canonical is the six-product
per-axis method.  Both are pinned to scipy's direct N-D convolution, closed
forms, deltas, invariants, the brute-force four-fold definition through the
two-operand oracle, and exact rational arithmetic within the derived bound;
the bound is pinned by closed forms, and planted mistakes in a numpy
transcription fail the pins.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.signal

import oracle
from tests import pins
from tests._numpy_method import ternary_per_axis

DTYPES = [np.float64, np.float32, np.int64]
WAYS = (1, 2, 3, 2, 1)        # pairs (i, j) in {0,1,2}^2 with i + j = digit
BOUND_ALL_ONES = (1, 6, 7, 6, 1)


def five(i: int, D: int) -> int:
    """Ternary digits of i read as base-5 digits."""
    f, w = 0, 1
    for _ in range(D):
        f += (i % 3) * w
        i //= 3
        w *= 5
    return f


def quint(i: int, D: int) -> int:
    """Bits of i read as base-5 digits (a hypercube index in the 5^D layout)."""
    f, w = 0, 1
    for _ in range(D):
        f += (i & 1) * w
        i >>= 1
        w *= 5
    return f


def digits5(k: int, D: int):
    out = []
    for _ in range(D):
        out.append(k % 5)
        k //= 5
    return out


def ints(D, seed, lo=-16, hi=16):
    g = np.random.default_rng([107, D, seed])
    return [g.integers(lo, hi, 3 ** D, dtype=np.int64) for _ in range(2)]


def masses(D, seed, dtype=np.float64):
    g = np.random.default_rng([109, D, seed])
    out = []
    for _ in range(2):
        u = g.random(3 ** D)
        out.append((u / u.sum()).astype(dtype))
    return out


def scipy_ternary(a, b):
    n = int(a.size)
    D = round(np.log(n) / np.log(3)) if n > 1 else 0
    if D == 0:
        return a * b
    return scipy.signal.convolve(a.reshape((3,) * D), b.reshape((3,) * D), method="direct").reshape(-1)


# ------------------------------------------------------------------ pins
def pin_scipy(impl, D):
    a, b = ints(D, 0)
    pins.assert_bitwise(impl(a, b), scipy_ternary(a, b), f"ternary vs scipy D={D}")


def pin_all_ones(impl, dtype, D):
    """(1 + t + t^2)^2 = 1 + 2t + 3t^2 + 2t^3 + t^4 on every axis."""
    x = np.ones(3 ** D, dtype=dtype)
    expect = np.array([np.prod([WAYS[d] for d in digits5(k, D)]) for k in range(5 ** D)]).astype(dtype)
    pins.assert_bitwise(impl(x, x.copy()), expect, f"ternary all-ones D={D}")


def pin_deltas(impl, dtype, D):
    g = np.random.default_rng([113, D])
    for _ in range(4):
        i, j = (int(v) for v in g.integers(0, 3 ** D, 2))
        a = np.zeros(3 ** D, dtype=dtype)
        b = np.zeros(3 ** D, dtype=dtype)
        a[i], b[j] = 3, 7
        expect = np.zeros(5 ** D, dtype=dtype)
        expect[five(i, D) + five(j, D)] = 21
        pins.assert_bitwise(impl(a, b), expect, f"ternary deltas D={D}")


def pin_sum_int(impl, D):
    a, b = ints(D, 1, 0, 16)
    assert int(impl(a, b).sum()) == int(a.sum()) * int(b.sum())


def pin_sum_of_four(impl, D):
    """int64: the pair sums X1 + X2 and X3 + X4 by the two-operand oracle
    (Algorithm 1), then their convolution, against the four-fold definition
    (every quadruple of hypercube entries)."""
    g = np.random.default_rng([127, D])
    xs = [g.integers(-8, 8, 1 << D, dtype=np.int64) for _ in range(4)]
    got = impl(oracle.naive(xs[0], xs[1]), oracle.naive(xs[2], xs[3]))
    expect = np.zeros(5 ** D, dtype=np.int64)
    q = [quint(i, D) for i in range(1 << D)]
    for i in range(1 << D):
        for j in range(1 << D):
            for k in range(1 << D):
                for m in range(1 << D):
                    expect[q[i] + q[j] + q[k] + q[m]] += xs[0][i] * xs[1][j] * xs[2][k] * xs[3][m]
    pins.assert_bitwise(got, expect, f"sum of four D={D}")


def exact_ternary(a, b):
    n = int(a.size)
    D = round(np.log(n) / np.log(3)) if n > 1 else 0
    z = [Fraction(0)] * (5 ** D)
    fa = [Fraction(float(v)) for v in a]
    fb = [Fraction(float(v)) for v in b]
    f = [five(i, D) for i in range(3 ** D)]
    for i in range(3 ** D):
        for j in range(3 ** D):
            z[f[i] + f[j]] += fa[i] * fb[j]
    return z


def pin_exact_bound(impl, dtype, D, kind):
    if kind == "mass":
        a, b = masses(D, 3, dtype)
    else:
        g = np.random.default_rng([131, D])
        a, b = (g.uniform(-1, 1, 3 ** D).astype(dtype) for _ in range(2))
    z = impl(a, b)
    ex = exact_ternary(a, b)
    B = oracle.ternary_bound(a.astype(np.float64), b.astype(np.float64))
    u = oracle.unit_roundoff(dtype)
    tol = Fraction((5 * D + 1) * u)
    for k in range(5 ** D):
        err = abs(Fraction(float(z[k])) - ex[k])
        assert err <= tol * Fraction(float(B[k])), f"bound violated at k={k}"


IMPLS = {"naive": oracle.ternary_naive, "canonical": oracle.ternary_canonical}


@pytest.mark.parametrize("impl", sorted(IMPLS))
@pytest.mark.parametrize("D", [0, 1, 2, 4, 6])
def test_ternary_scipy_definition(impl, D):
    pin_scipy(IMPLS[impl], D)


@pytest.mark.parametrize("impl", sorted(IMPLS))
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("D", [0, 1, 3, 6])
def test_ternary_all_ones(impl, dtype, D):
    pin_all_ones(IMPLS[impl], dtype, D)


@pytest.mark.parametrize("impl", sorted(IMPLS))
@pytest.mark.parametrize("dtype", DTYPES)
def test_ternary_deltas(impl, dtype):
    pin_deltas(IMPLS[impl], dtype, 4)


@pytest.mark.parametrize("impl", sorted(IMPLS))
def test_ternary_sum_invariant(impl):
    pin_sum_int(IMPLS[impl], 6)


@pytest.mark.parametrize("impl", sorted(IMPLS))
@pytest.mark.parametrize("D", [0, 1, 3])
def test_ternary_sum_of_four(impl, D):
    pin_sum_of_four(IMPLS[impl], D)


@pytest.mark.parametrize("D", [7, 8])
def test_ternary_canonical_equals_definition_int64(D):
    a, b = ints(D, 4)
    pins.assert_bitwise(oracle.ternary_canonical(a, b), oracle.ternary_naive(a, b), f"D={D}")


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("D,kind", [(1, "signed"), (2, "signed"), (3, "mass"), (3, "signed")])
def test_ternary_exact_within_bound(dtype, D, kind):
    pin_exact_bound(oracle.ternary_canonical, dtype, D, kind)


def test_ternary_float_order_is_the_transcription():
    """The oracle's float arithmetic is the per-axis method in the stated
    order (forward ascending, inverse descending, the inverse's terms as
    written): an independent numpy transcription gives the same bits."""
    for D in (1, 4, 7):
        for dt in (np.float64, np.float32):
            a, b = masses(D, 5, dt)
            pins.assert_bitwise(oracle.ternary_canonical(a, b), ternary_per_axis(a, b), f"D={D} {dt}")


def test_ternary_direct_at_matches_definition():
    D = 5
    a, b = ints(D, 6, 0, 16)
    ks = np.arange(5 ** D, dtype=np.uint64)
    ref = oracle.ternary_naive(a, b).astype(np.float64)
    got = oracle.ternary_direct_at(a.astype(np.float64), b.astype(np.float64), ks)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("D", [7, 9])
def test_ternary_mass_error_within_bound_vs_direct(D):
    a, b = masses(D, 7)
    z = oracle.ternary_canonical(a, b)
    ks = np.random.default_rng([137, D]).integers(0, 5 ** D, 2048, dtype=np.uint64)
    ref = oracle.ternary_direct_at(a, b, ks)
    B = oracle.ternary_bound(a, b)[ks.astype(np.int64)]
    err = np.abs(z[ks.astype(np.int64)] - ref)
    assert np.all(err <= (5 * D + 1) * 2.0 ** -53 * B + 2.0 ** -60 * np.abs(ref))
    r = float(np.max(err / B) / 2.0 ** -53)
    assert 0.02 <= r <= 5 * D + 1, f"max |err|/(u B) = {r:.3g}"


# ----------------------------------------------- the bound, pinned by closed forms
def test_ternary_bound_all_ones():
    """a = b = 1: per axis T gives (1, 1, 1, 2, 2, 2), the product
    (1, 1, 1, 4, 4, 4) and |U| (1, 6, 7, 6, 1)."""
    for D in (0, 1, 3, 5):
        x = np.ones(3 ** D)
        expect = np.array([np.prod([BOUND_ALL_ONES[d] for d in digits5(k, D)]) for k in range(5 ** D)],
                          dtype=np.float64)
        pins.assert_bitwise(oracle.ternary_bound(x, x.copy()), expect, f"D={D}")


def test_ternary_bound_rank1():
    """Outer-product inputs: per axis |U|(T|a| . T|b|) of the axis factors."""
    for D in (1, 3, 4):
        fa = pins.rank1_factors(D, 0, width=3)
        fb = pins.rank1_factors(D, 1000, width=3)
        per_axis = []
        for d in range(D):
            a0, a1, a2 = (abs(v) for v in fa[d])
            b0, b1, b2 = (abs(v) for v in fb[d])
            p0, p1, p2 = a0 * b0, a1 * b1, a2 * b2
            q01, q12, q02 = (a0 + a1) * (b0 + b1), (a1 + a2) * (b1 + b2), (a0 + a2) * (b0 + b2)
            per_axis.append((p0, q01 + p0 + p1, q02 + p0 + p2 + p1, q12 + p1 + p2, p2))
        pins.assert_bitwise(oracle.ternary_bound(pins.rank1(fa), pins.rank1(fb)), pins.rank1(per_axis),
                            f"rank-1 D={D}")


# --------------------------------------------------------------- pin power
def ternary_pins(impl):
    failed = []
    checks = {
        "scipy": lambda: [pin_scipy(impl, D) for D in (2, 4)],
        "all_ones": lambda: pin_all_ones(impl, np.float64, 4),
        "deltas": lambda: pin_deltas(impl, np.int64, 3),
        "sum": lambda: pin_sum_int(impl, 4),
        "four": lambda: pin_sum_of_four(impl, 2),
        "bound": lambda: [pin_exact_bound(impl, np.float64, 2, k) for k in ("mass", "signed")],
        "order": lambda: pins.assert_bitwise(impl(*masses(5, 9)), oracle.ternary_canonical(*masses(5, 9)), "order"),
    }
    for name, fn in checks.items():
        try:
            fn()
        except AssertionError:
            failed.append(name)
    return failed


MUTANTS = {
    "q02_sign": dict(q02_sign=-1),
    "c2_drops_p1": dict(keep_p1=False),
    "c1_drops_p1": dict(c1_drop_p1=True),
    "forward_slots_swapped": dict(slot_swap=True),
    "inverse_ascending": dict(inverse_order="asc"),
    "forward_descending": dict(forward_order="desc"),
}


def test_ternary_unmodified_transcription_passes():
    assert ternary_pins(lambda a, b: ternary_per_axis(a, b)) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_ternary_mutant_is_caught(name):
    assert ternary_pins(lambda a, b: ternary_per_axis(a, b, **MUTANTS[name])), name


def test_ternary_swapped_operand_is_caught():
    assert ternary_pins(lambda a, b: ternary_per_axis(a, a))
