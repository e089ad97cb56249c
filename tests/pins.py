"""Pins for a hypercube-convolution implementation ``impl(x, y) -> z``.

Each pin checks the implementation against something fixed outside it: the
paper's worked example and base cases, a library routine for the definition
(scipy's direct N-D convolution), closed forms, invariants, and exact
rational arithmetic within a derived rounding bound.  The same checks run on
the oracle (tests/test_oracle_pins.py) and on deliberately broken variants of
the method (tests/test_oracle_mutants.py), which must each fail at least one.
"""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np
import scipy.signal

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name: str):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def tern_py(i: int) -> int:
    """Bits of i read as ternary digits (bit d -> digit of weight 3^d)."""
    t, p = 0, 1
    while i:
        t += (i & 1) * p
        p *= 3
        i >>= 1
    return t


def ternary_digits(k: int, D: int):
    """Digits of k, most significant (axis 0) first."""
    out = []
    for _ in range(D):
        out.append(k % 3)
        k //= 3
    return out[::-1]


def ones_count_ternary(n3: int) -> np.ndarray:
    k = np.arange(n3)
    c = np.zeros(n3, dtype=np.int64)
    while np.any(k):
        c += (k % 3 == 1)
        k //= 3
    return c


def bits(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a)
    return a.view({8: np.int64, 4: np.int32}[a.dtype.itemsize])


def assert_bitwise(a, b, what=""):
    a, b = np.asarray(a), np.asarray(b)
    assert a.dtype == b.dtype and a.shape == b.shape, what
    if not np.array_equal(bits(a), bits(b)):
        bad = np.nonzero(bits(a) != bits(b))[0]
        raise AssertionError(f"{what}: {bad.size} elements differ, first at {bad[:5]} "
                             f"({a[bad[:3]]} vs {b[bad[:3]]})")


def scipy_definition(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """The definition of convolution via scipy's direct N-D routine on the
    (2,)*D views; the (3,)*D result read in row-major order."""
    D = int(x.size).bit_length() - 1
    if D == 0:
        return x * y
    return scipy.signal.convolve(x.reshape((2,) * D), y.reshape((2,) * D),
                                 method="direct").reshape(-1)


def exact_fraction(x: np.ndarray, y: np.ndarray) -> list:
    """Exact rational convolution of float inputs (every float is a dyadic
    rational), by the definition."""
    D = int(x.size).bit_length() - 1
    n3 = 3 ** D
    z = [Fraction(0)] * n3
    fx = [Fraction(float(v)) for v in x]
    fy = [Fraction(float(v)) for v in y]
    t = [tern_py(i) for i in range(1 << D)]
    for i in range(1 << D):
        for j in range(1 << D):
            z[t[i] + t[j]] += fx[i] * fy[j]
    return z


# --------------------------------------------------------------------------- pins

def pin_worked_example(impl, dtype):
    g = golden("carry_free_example.json")
    D = g["D"]
    x = np.zeros(1 << D, dtype=dtype)
    y = np.zeros(1 << D, dtype=dtype)
    x[g["i"]] = 1
    y[g["j"]] = 1
    z = impl(x, y)
    expect = np.zeros(3 ** D, dtype=dtype)
    expect[g["k_flat"]] = 1
    assert_bitwise(z, expect, "carry-free worked example")


def pin_deltas(impl, dtype, D, seed=0):
    """x = e_i, y = e_j gives z = e_(tern(i)+tern(j)) exactly."""
    g = np.random.default_rng([7, D, seed])
    for _ in range(4):
        i, j = (int(v) for v in g.integers(0, 1 << D, 2))
        x = np.zeros(1 << D, dtype=dtype)
        y = np.zeros(1 << D, dtype=dtype)
        x[i] = 3
        y[j] = 5
        expect = np.zeros(3 ** D, dtype=dtype)
        expect[tern_py(i) + tern_py(j)] = 15
        assert_bitwise(impl(x, y), expect, f"delta D={D} i={i} j={j}")


def pin_d0(impl, dtype):
    x = np.array([3], dtype=dtype)
    y = np.array([-7], dtype=dtype)
    assert_bitwise(impl(x, y), x * y, "D=0 scalar product")


def pin_d1_int(impl):
    g = golden("base_cases.json")
    for case in g["d1_int_cases"]:
        z = impl(np.array(case["x"], dtype=np.int64), np.array(case["y"], dtype=np.int64))
        assert_bitwise(z, np.array(case["z"], dtype=np.int64), "Algorithm 2 base case D=1")


def pin_scipy_int(impl, D, seed=0):
    g = np.random.default_rng([11, D, seed])
    x = g.integers(-16, 16, 1 << D, dtype=np.int64)
    y = g.integers(-16, 16, 1 << D, dtype=np.int64)
    assert_bitwise(impl(x, y), scipy_definition(x, y), f"scipy direct D={D}")


def pin_all_ones(impl, dtype, D):
    """x = y = 1 gives z[k] = 2^(number of ternary digits of k equal to 1);
    every intermediate is 2^a or 3*2^a, so this is exact in every dtype."""
    x = np.ones(1 << D, dtype=dtype)
    expect = (2 ** ones_count_ternary(3 ** D)).astype(dtype)
    assert_bitwise(impl(x, x.copy()), expect, f"all-ones D={D}")


def pin_sum_int(impl, D, seed=0):
    g = np.random.default_rng([13, D, seed])
    x = g.integers(0, 16, 1 << D, dtype=np.int64)
    y = g.integers(0, 16, 1 << D, dtype=np.int64)
    z = impl(x, y)
    assert int(z.sum()) == int(x.sum()) * int(y.sum()), "sum(z) = sum(x) sum(y)"


def pin_marginals_int(impl, D, seed=0):
    """Summing z over the digit of axis a equals the (D-1)-dim convolution of
    the axis-a marginals x[..,0,..] + x[..,1,..] (by scipy's definition)."""
    g = np.random.default_rng([17, D, seed])
    x = g.integers(0, 16, 1 << D, dtype=np.int64)
    y = g.integers(0, 16, 1 << D, dtype=np.int64)
    z = impl(x, y).reshape((3,) * D)
    for a in range(D):
        mx = x.reshape((2,) * D).sum(axis=a).reshape(-1)
        my = y.reshape((2,) * D).sum(axis=a).reshape(-1)
        assert_bitwise(z.sum(axis=a).reshape(-1), scipy_definition(mx, my),
                       f"marginal on axis {a}")


def pin_commutative(impl, dtype, D, seed=0):
    g = np.random.default_rng([19, D, seed])
    x = g.random(1 << D).astype(dtype)
    y = g.random(1 << D).astype(dtype)
    assert_bitwise(impl(x, y), impl(y, x), "commutativity")


def pin_linear_int(impl, D, seed=0):
    g = np.random.default_rng([23, D, seed])
    x1 = g.integers(-8, 8, 1 << D, dtype=np.int64)
    x2 = g.integers(-8, 8, 1 << D, dtype=np.int64)
    y = g.integers(-8, 8, 1 << D, dtype=np.int64)
    assert_bitwise(impl(3 * x1 - 2 * x2, y), 3 * impl(x1, y) - 2 * impl(x2, y), "linearity")


def pin_axis_flip_int(impl, D, seed=0):
    """Reversing every axis of x and y reverses z (flat order reversal)."""
    g = np.random.default_rng([29, D, seed])
    x = g.integers(0, 16, 1 << D, dtype=np.int64)
    y = g.integers(0, 16, 1 << D, dtype=np.int64)
    assert_bitwise(impl(x[::-1].copy(), y[::-1].copy()), impl(x, y)[::-1].copy(), "axis flip")


def pin_paper_accuracy(impl, D, exact_fn=None):
    """Table 1's accuracy inputs: z[0...0] = 1 with zero error, and for these
    structured inputs every float64 output equals the exact integer result
    (by default scipy's direct definition in int64; for large D the caller
    may pass Algorithm 1 in int64, itself pinned to scipy)."""
    x = np.arange(1, (1 << D) + 1, dtype=np.float64)
    z = impl(x, x.copy())
    assert z[0] == 1.0, "smallest result value is 1"
    xi = np.arange(1, (1 << D) + 1, dtype=np.int64)
    exact = (exact_fn or scipy_definition)(xi, xi.copy())
    assert np.array_equal(z, exact.astype(np.float64)), "structured inputs are exact"


def pin_exact_bound(impl, dtype, D, bound_fn, seed=0, kind="signed"):
    """|impl - exact| <= (4D + 2) u B against exact rational arithmetic, with
    B = |G|(F|x| . F|y|) from bound_fn."""
    g = np.random.default_rng([31, D, seed])
    if kind == "signed":
        x = g.uniform(-1, 1, 1 << D).astype(dtype)
        y = g.uniform(-1, 1, 1 << D).astype(dtype)
    else:
        x = g.random(1 << D)
        y = g.random(1 << D)
        x, y = (x / x.sum()).astype(dtype), (y / y.sum()).astype(dtype)
    z = impl(x, y)
    exact = exact_fraction(x, y)
    u = {np.dtype(np.float64): 2.0 ** -53, np.dtype(np.float32): 2.0 ** -24}[np.dtype(dtype)]
    B = bound_fn(x.astype(np.float64), y.astype(np.float64))
    tol = (4 * D + 2) * u
    for k in range(3 ** D):
        err = abs(Fraction(float(z[k])) - exact[k])
        assert err <= Fraction(tol) * Fraction(float(B[k])), \
            f"bound violated at k={k}: err={float(err)} bound={tol * B[k]}"


def pin_d1_rounding(impl):
    """D = 1, x = (1, 2^-53), y = (1, 1).  The method forms the marginal
    fl(1 + 2^-53) = 1 (ties to even), t = 2, and z1 = (t - z0) - z2 =
    (2 - 1) - 2^-53 = 1 - 2^-53 exactly; the exact value is 1 + 2^-53.  An
    implementation that evaluates x1*y0 + x0*y1 directly (Algorithm 2's D = 1
    specialisation) gives 1, and one that subtracts (z0 + z2) gives 1."""
    x = np.array([1.0, 2.0 ** -53])
    y = np.array([1.0, 1.0])
    z = impl(x, y)
    assert_bitwise(z, np.array([1.0, 1.0 - 2.0 ** -53, 2.0 ** -53]), "D=1 rounding order")


def pin_matches_recursion(impl, dtype, D, recursion, seed=0):
    """Bitwise agreement with the three-subproblem recursion of the Methods
    section (z[1] = t - z[0] - z[2], t the convolution of the marginals).  In
    floating point the recursion fixes the order: marginals on axis 0 first,
    and the subtraction on axis 0 last."""
    g = np.random.default_rng([37, D, seed])
    x = g.random(1 << D)
    y = g.random(1 << D)
    x, y = (x / x.sum()).astype(dtype), (y / y.sum()).astype(dtype)
    assert_bitwise(impl(x, y), recursion(x, y), f"matches recursion D={D}")


# ------------------------------------------------------------- rounding bounds
# The bound B = |G|(F|x| . F|y|) and the adjoint bounds are tensor products of
# per-axis factors whenever the inputs are: for x = (x) over axes of
# (a_d, b_d) and y of (c_d, e_d), the forward map gives (|a|, |a|+|b|, |b|),
# the product multiplies per axis, and |G| sends (p0, p1, p2) to
# (p0, p0 + p1 + p2, p2).  These closed forms fix B from both sides: a
# dropped term, a wrong index or a scaled result changes them.

def rank1(factors) -> np.ndarray:
    """Outer product over the axes, axis 0 (first factor) most significant."""
    out = np.ones(1)
    for f in factors:
        out = np.kron(out, np.asarray(f, dtype=np.float64))
    return out


def rank1_factors(D: int, seed: int, width: int = 2, lo: int = 1, hi: int = 4):
    """Per-axis factors of small signed integers (|v| in [lo, hi))."""
    g = np.random.default_rng([61, D, seed, width])
    mag = g.integers(lo, hi, (D, width)).astype(np.float64)
    sign = np.where(g.random((D, width)) < 0.5, -1.0, 1.0)
    return list(mag * sign)


def bound_closed_form(fx, fy) -> np.ndarray:
    per_axis = []
    for (a, b), (c, e) in zip(fx, fy):
        a, b, c, e = abs(a), abs(b), abs(c), abs(e)
        p0, p1, p2 = a * c, (a + b) * (c + e), b * e
        per_axis.append((p0, p0 + p1 + p2, p2))
    return rank1(per_axis)


def bound_closed_form_at(fx, fy, ks) -> np.ndarray:
    """The same closed form at single output indices (digits of k, axis 0
    most significant), as exact products in Python integers or floats."""
    D = len(fx)
    out = []
    for k in ks:
        digits = ternary_digits(int(k), D)
        v = 1.0
        for d, dig in enumerate(digits):
            a, b = (abs(t) for t in fx[d])
            c, e = (abs(t) for t in fy[d])
            p0, p1, p2 = a * c, (a + b) * (c + e), b * e
            v *= (p0, p0 + p1 + p2, p2)[dig]
        out.append(v)
    return np.array(out)


def adjoint_bound_closed_form(fw, fo):
    """Bx for w = (x) of (w0, w1, w2)_d and the other operand (x) of (c, e)_d:
    |G^T| gives (|w0|+|w1|, |w1|, |w2|+|w1|), F|.| gives (|c|, |c|+|e|, |e|),
    the product multiplies per axis, |F^T| gives (g0 + g1, g1 + g2)."""
    per_axis = []
    for (w0, w1, w2), (c, e) in zip(fw, fo):
        w0, w1, w2, c, e = abs(w0), abs(w1), abs(w2), abs(c), abs(e)
        g0, g1, g2 = (w0 + w1) * c, w1 * (c + e), (w2 + w1) * e
        per_axis.append((g0 + g1, g1 + g2))
    return rank1(per_axis)


def pin_bound_all_ones(bound_fn, D):
    """x = y = 1: B[k] = 6^(number of digits of k equal to 1), exactly."""
    x = np.ones(1 << D)
    expect = 6.0 ** ones_count_ternary(3 ** D)
    assert_bitwise(bound_fn(x, x.copy()), expect, f"bound all-ones D={D}")


def pin_bound_rank1(bound_fn, D, seed=0):
    """Outer-product inputs with distinct small integers per axis: every
    intermediate is an integer below 2^53 for D <= 8, so B equals its closed
    form exactly."""
    fx, fy = rank1_factors(D, seed), rank1_factors(D, seed + 1000)
    expect = bound_closed_form(fx, fy)
    assert expect.max() < 2.0 ** 53
    assert_bitwise(bound_fn(rank1(fx), rank1(fy)), expect, f"bound rank-1 D={D}")


def pin_bound_at_closed_forms(bound_at_fn, D, n=64, seed=0):
    """The per-index bound at large D: all-ones inputs give 6^s exactly (s
    digits equal to 1); outer-product inputs give the per-axis product within
    the rounding of D multiplications."""
    g = np.random.default_rng([67, D, seed])
    ks = g.integers(0, 3 ** D, 4 * n, dtype=np.uint64)
    ks = np.array([k for k in ks if sum(d == 1 for d in ternary_digits(int(k), D)) <= 14][:n]
                  + [0, 3 ** D - 1, (3 ** min(D, 14) - 1) // 2], dtype=np.uint64)
    ones = np.ones(1 << D)
    s = np.array([sum(d == 1 for d in ternary_digits(int(k), D)) for k in ks])
    assert_bitwise(bound_at_fn(ones, ones.copy(), ks), 6.0 ** s, f"bound_at all-ones D={D}")
    fx, fy = rank1_factors(D, seed), rank1_factors(D, seed + 1000)
    got = bound_at_fn(rank1(fx), rank1(fy), ks)
    expect = bound_closed_form_at(fx, fy, ks)
    assert np.all(np.abs(got - expect) <= 4 * D * 2.0 ** -53 * expect), \
        f"bound_at rank-1 D={D}: max rel {np.max(np.abs(got - expect) / expect):.3g}"


def pin_adjoint_bound_closed_forms(adjoint_bound_fn, D, seed=0):
    """x = y = w = 1 gives Bx = By = 4^D exactly; outer-product x, y, w give
    the per-axis products (x's factors enter By, y's enter Bx)."""
    ones2, ones3 = np.ones(1 << D), np.ones(3 ** D)
    bx, by = adjoint_bound_fn(ones2, ones2.copy(), ones3)
    assert np.all(bx == 4.0 ** D) and np.all(by == 4.0 ** D), f"adjoint bound all-ones D={D}"
    fx, fy = rank1_factors(D, seed), rank1_factors(D, seed + 1000)
    fw = rank1_factors(D, seed + 2000, width=3)
    bx, by = adjoint_bound_fn(rank1(fx), rank1(fy), rank1(fw))
    ex, ey = adjoint_bound_closed_form(fw, fy), adjoint_bound_closed_form(fw, fx)
    tol = 6 * D * 2.0 ** -53
    assert np.all(np.abs(bx - ex) <= tol * ex), f"adjoint bound x rank-1 D={D}"
    assert np.all(np.abs(by - ey) <= tol * ey), f"adjoint bound y rank-1 D={D}"


def error_ratio_band(ratio: float, D: int, lo: float = 0.05) -> None:
    """The largest measured |err| / (u B) lies between lo and 4D + 2: above
    the certified factor the bound is violated; far below any measured value
    (0.5 to 1.5 on the workloads' masses) the bound would be inflated."""
    assert lo <= ratio <= 4 * D + 2, f"max |err|/(u B) = {ratio:.3g} outside [{lo}, {4 * D + 2}]"
