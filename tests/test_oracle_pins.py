"""Pins of the CPU oracle against facts fixed outside it (CPU only).

The oracle (oracle/) is test infrastructure; these tests are what make it
trustworthy before any GPU result is compared with it.
"""
import numpy as np
import pytest

import hc_inputs
import oracle
from tests import pins

DTYPES = [np.float64, np.float32, np.int64]
IMPLS = {
    "naive": oracle.naive,
    "canonical": oracle.canonical,
    "recursive": oracle.recursive,
    "recursive_mt": lambda x, y: oracle.recursive(x, y, threads=4),
}
EXACT_IMPLS = ["naive", "canonical", "recursive", "recursive_mt"]
METHOD_IMPLS = ["canonical", "recursive", "recursive_mt"]


@pytest.mark.parametrize("impl", EXACT_IMPLS)
@pytest.mark.parametrize("dtype", DTYPES)
def test_worked_example(impl, dtype):
    pins.pin_worked_example(IMPLS[impl], dtype)


@pytest.mark.parametrize("impl", EXACT_IMPLS)
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("D", [1, 2, 5, 8, 10])
def test_deltas(impl, dtype, D):
    pins.pin_deltas(IMPLS[impl], dtype, D)


@pytest.mark.parametrize("impl", EXACT_IMPLS)
@pytest.mark.parametrize("dtype", DTYPES)
def test_d0(impl, dtype):
    pins.pin_d0(IMPLS[impl], dtype)


@pytest.mark.parametrize("impl", EXACT_IMPLS)
def test_d1_base_case_int(impl):
    pins.pin_d1_int(IMPLS[impl])


@pytest.mark.parametrize("impl", METHOD_IMPLS)
def test_d1_rounding_order(impl):
    pins.pin_d1_rounding(IMPLS[impl])


@pytest.mark.parametrize("impl", EXACT_IMPLS)
@pytest.mark.parametrize("D", list(range(0, 11)))
def test_scipy_definition_int(impl, D):
    pins.pin_scipy_int(IMPLS[impl], D)


@pytest.mark.parametrize("impl", EXACT_IMPLS)
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("D", [0, 1, 3, 7, 10])
def test_all_ones(impl, dtype, D):
    pins.pin_all_ones(IMPLS[impl], dtype, D)


@pytest.mark.parametrize("impl", METHOD_IMPLS)
@pytest.mark.parametrize("D", [1, 4, 9, 12])
def test_sum_int(impl, D):
    pins.pin_sum_int(IMPLS[impl], D)


@pytest.mark.parametrize("impl", METHOD_IMPLS)
@pytest.mark.parametrize("D", [1, 3, 6, 9])
def test_marginals_int(impl, D):
    pins.pin_marginals_int(IMPLS[impl], D)


@pytest.mark.parametrize("impl", METHOD_IMPLS)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("D", [1, 5, 11])
def test_commutative(impl, dtype, D):
    pins.pin_commutative(IMPLS[impl], dtype, D)


@pytest.mark.parametrize("impl", METHOD_IMPLS)
@pytest.mark.parametrize("D", [2, 7, 10])
def test_linear_int(impl, D):
    pins.pin_linear_int(IMPLS[impl], D)


@pytest.mark.parametrize("impl", METHOD_IMPLS)
@pytest.mark.parametrize("D", [1, 4, 9])
def test_axis_flip_int(impl, D):
    pins.pin_axis_flip_int(IMPLS[impl], D)


@pytest.mark.parametrize("impl", METHOD_IMPLS)
@pytest.mark.parametrize("D", [1, 4, 8, 12])
def test_paper_accuracy_workload(impl, D):
    pins.pin_paper_accuracy(IMPLS[impl], D, exact_fn=oracle.naive if D > 10 else None)


def test_table1_smallest_value_zero_error():
    """Table 1 reports zero relative error of the method at z[(0,...,0)] = 1
    for D = 11..18; the oracle reproduces that value exactly."""
    g = pins.golden("table1_accuracy.json")
    for D, err in zip(g["D"], g["dc_relative_error_at_smallest"]):
        if D > 16:
            continue  # the recursion at D = 17, 18 takes tens of seconds; the property is structural
        x = np.arange(1, (1 << D) + 1, dtype=np.float64)
        z = oracle.recursive(x, x.copy(), threads=8)
        assert z[0] == g["smallest_value"]
        assert abs(z[0] - 1.0) / 1.0 == err


@pytest.mark.parametrize("impl", METHOD_IMPLS)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("D,kind", [(2, "signed"), (4, "signed"), (5, "mass"), (6, "signed")])
def test_exact_within_bound(impl, dtype, D, kind):
    pins.pin_exact_bound(IMPLS[impl], dtype, D, oracle.bound, kind=kind)


@pytest.mark.parametrize("impl", ["canonical", "recursive_mt"])
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("D", [0, 1, 2, 3, 6, 9, 12])
def test_matches_recursion(impl, dtype, D):
    pins.pin_matches_recursion(IMPLS[impl], dtype, D, oracle.recursive)


@pytest.mark.parametrize("D", [7, 10])
def test_direct_at_matches_definition(D):
    """The per-index definition sum equals scipy's direct convolution (int64)
    and is within a few long-double ulps of it for float64."""
    g = np.random.default_rng([41, D])
    x = g.integers(0, 16, 1 << D, dtype=np.int64)
    y = g.integers(0, 16, 1 << D, dtype=np.int64)
    ks = np.arange(3 ** D, dtype=np.uint64)
    pins.assert_bitwise(oracle.direct_at(x, y, ks), pins.scipy_definition(x, y), "direct_at int64")
    xf, yf = x.astype(np.float64), y.astype(np.float64)
    assert np.array_equal(oracle.direct_at(xf, yf, ks), pins.scipy_definition(x, y).astype(np.float64))


@pytest.mark.parametrize("D", [8, 10])
def test_mass_inputs_within_bound_vs_direct(D):
    """For the workloads' normalised masses the method stays within the
    derived bound of the (compensated) definition at every output."""
    g = np.random.default_rng([43, D])
    x = g.random(1 << D); x /= x.sum()
    y = g.random(1 << D); y /= y.sum()
    z = oracle.canonical(x, y)
    ref = oracle.direct_at(x, y, np.arange(3 ** D, dtype=np.uint64))
    B = oracle.bound(x, y)
    tol = (4 * D + 2) * 2.0 ** -53 * B + 2.0 ** -60 * np.abs(ref)  # + error of the compensated sum
    assert np.all(np.abs(z - ref) <= tol)


@pytest.mark.parametrize("D", [0, 1, 5, 8])
def test_bound_at_matches_full_bound(D):
    """The per-index bound (sub-cube of the digit-1 axes) equals the full
    bound array everywhere; indices with too many 1 digits are refused."""
    g = np.random.default_rng([53, D])
    x = g.uniform(-1, 1, 1 << D)
    y = g.uniform(-1, 1, 1 << D)
    ks = np.arange(3 ** D, dtype=np.uint64)
    assert np.array_equal(oracle.bound_at(x, y, ks), oracle.bound(x, y))
    if D >= 1:
        with pytest.raises(ValueError):
            oracle.bound_at(np.ones(1 << 15), np.ones(1 << 15), [(3 ** 15 - 1) // 2])


def test_tern_map():
    g = pins.golden("carry_free_example.json")
    assert oracle.tern(g["i"]) + oracle.tern(g["j"]) == g["k_flat"]
    assert pins.ternary_digits(g["k_flat"], g["D"]) == g["k_digits_msb_first"]
    t = oracle.tern_map(12)
    assert all(int(t[i]) == pins.tern_py(i) for i in range(0, 4096, 7))


# ----------------------------------------------------------------- adjoint pins

def _loss(x, y, w):
    return float(np.dot(w, oracle.canonical(x, y)))


@pytest.mark.parametrize("D", [1, 3, 6, 9])
def test_adjoint_vs_correlation(D):
    """Transposed-map gradient vs the direct correlation (definition of the
    gradient of sum(w * z)), within the derived adjoint bound."""
    g = np.random.default_rng([47, D])
    x = g.random(1 << D); x /= x.sum()
    y = g.random(1 << D); y /= y.sum()
    w = g.standard_normal(3 ** D)
    gx, gy = oracle.adjoint(x, y, w)
    idx = np.arange(1 << D, dtype=np.uint64)
    cx, cy = oracle.correlation_at(x, y, w, idx)
    bx, by = oracle.adjoint_bound(x, y, w)
    tol = (4 * D + 2) * 2.0 ** -53
    assert np.all(np.abs(gx - cx) <= tol * bx + 1e-300)
    assert np.all(np.abs(gy - cy) <= tol * by + 1e-300)


@pytest.mark.parametrize("D", [2, 5, 8])
def test_adjoint_int_exact(D):
    """int64: the adjoint equals the correlation written with the index map,
    and L = <w, z(x, y)> = <gx, x> = <gy, y> exactly (bilinearity)."""
    g = np.random.default_rng([53, D])
    x = g.integers(-8, 8, 1 << D, dtype=np.int64)
    y = g.integers(-8, 8, 1 << D, dtype=np.int64)
    w = g.integers(-8, 8, 3 ** D, dtype=np.int64)
    gx, gy = oracle.adjoint(x, y, w)
    t = np.array([pins.tern_py(i) for i in range(1 << D)], dtype=np.int64)
    W = w[t[:, None] + t[None, :]]          # W[i, j] = w[tern(i) + tern(j)]
    pins.assert_bitwise(gx, W @ y, "gx correlation")
    pins.assert_bitwise(gy, W.T @ x, "gy correlation")
    L = int(np.dot(w, oracle.canonical(x, y)))
    assert L == int(np.dot(gx, x)) == int(np.dot(gy, y))


@pytest.mark.parametrize("D", [3, 7])
def test_adjoint_finite_differences(D):
    """Central differences with h = 1e-6 on L(x, y) = sum(w * z); L is
    bilinear, so the difference has no truncation error, only rounding."""
    g = np.random.default_rng([59, D])
    x = g.random(1 << D); x /= x.sum()
    y = g.random(1 << D); y /= y.sum()
    w = g.standard_normal(3 ** D)
    gx, gy = oracle.adjoint(x, y, w)
    h = 1e-6
    scale = max(np.abs(gx).max(), np.abs(gy).max())
    for i in g.integers(0, 1 << D, 8):
        e = np.zeros(1 << D); e[i] = h
        fdx = (_loss(x + e, y, w) - _loss(x - e, y, w)) / (2 * h)
        fdy = (_loss(x, y + e, w) - _loss(x, y - e, w)) / (2 * h)
        assert abs(fdx - gx[i]) <= 1e-6 * scale
        assert abs(fdy - gy[i]) <= 1e-6 * scale


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_adjoint_all_ones(dtype):
    """x = y = w = 1: L = sum(z) = sum(x) sum(y), so every partial derivative
    with respect to x[i] is sum(y) = 2^D, exactly in both precisions."""
    D = 6
    x = np.ones(1 << D, dtype=dtype)
    w = np.ones(3 ** D, dtype=dtype)
    gx, gy = oracle.adjoint(x, x.copy(), w)
    assert np.all(gx == 2 ** D) and np.all(gy == 2 ** D)


def _wrap64(v: int) -> int:
    v &= (1 << 64) - 1
    return v - (1 << 64) if v >> 63 else v


@pytest.mark.parametrize("impl", EXACT_IMPLS)
@pytest.mark.parametrize("D", [1, 3, 6])
def test_int64_full_range_wraps_like_the_ring(impl, D):
    """Entries spread over all of int64, so that sums, products and the
    outputs themselves overflow: every implementation agrees with the
    definition summed in unbounded Python integers and reduced modulo 2^64
    (the method's identities hold in the ring of integers modulo 2^64)."""
    g = np.random.default_rng([hc_inputs.SEED, 95, D])
    x = g.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, 1 << D, dtype=np.int64, endpoint=True)
    y = g.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, 1 << D, dtype=np.int64, endpoint=True)
    ref = [0] * 3 ** D
    for i in range(1 << D):
        for j in range(1 << D):
            k = 0
            for a in range(D - 1, -1, -1):
                k = 3 * k + ((i >> a) & 1) + ((j >> a) & 1)
            ref[k] += int(x[i]) * int(y[j])
    expect = np.array([_wrap64(v) for v in ref], dtype=np.int64)
    pins.assert_bitwise(IMPLS[impl](x, y), expect, f"{impl} D={D} full-range int64")


def test_int64_wrapping_intermediate_written_out():
    """D = 1 with x = (2^62, 2^62), y = (1, 0): the forward sum 2^63 wraps,
    yet z = (2^62, 2^62, 0) exactly."""
    x = np.array([1 << 62, 1 << 62], dtype=np.int64)
    y = np.array([1, 0], dtype=np.int64)
    for name in EXACT_IMPLS:
        assert IMPLS[name](x, y).tolist() == [1 << 62, 1 << 62, 0], name


# ------------------------------------------------- the rounding bounds, pinned
# Closed forms fix B from above as well as below (a bound inflated by any
# factor fails them); tests/test_oracle_bound_mutants.py shows that planted
# mistakes in the bound code are caught.

@pytest.mark.parametrize("D", [0, 1, 3, 6, 10, 12])
def test_bound_all_ones_closed_form(D):
    pins.pin_bound_all_ones(oracle.bound, D)


@pytest.mark.parametrize("D", [1, 2, 5, 8])
def test_bound_rank1_closed_form(D):
    pins.pin_bound_rank1(oracle.bound, D)


@pytest.mark.parametrize("D", [12, 16, 20, 21])
def test_bound_at_closed_forms_large_d(D):
    pins.pin_bound_at_closed_forms(oracle.bound_at, D)


@pytest.mark.parametrize("D", [0, 1, 4, 7, 10])
def test_adjoint_bound_closed_forms(D):
    pins.pin_adjoint_bound_closed_forms(oracle.adjoint_bound, D)


@pytest.mark.parametrize("D", [8, 10, 12])
def test_mass_error_ratio_in_band(D):
    """On the workloads' normalised masses the largest |err|/(u B) against
    the compensated definition sum lies in the band the full-size GPU checks
    assert (it measures 0.5 to 1.5 there)."""
    x, y = hc_inputs.pair_masses(D, hc_inputs.W_D16)
    z = oracle.canonical(x, y)
    ks = np.arange(3 ** D, dtype=np.uint64) if D <= 10 else \
        np.random.default_rng([71, D]).integers(0, 3 ** D, 4096, dtype=np.uint64)
    ref = oracle.direct_at(x, y, ks)
    B = oracle.bound_at(x, y, ks) if D > 10 else oracle.bound(x, y)
    r = float(np.max(np.abs(z[ks.astype(np.int64)] - ref) / B) / 2.0 ** -53)
    pins.error_ratio_band(r, D)
