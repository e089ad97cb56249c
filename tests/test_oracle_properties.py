"""Property tests of the oracle with generated shapes and values (hypothesis),
CPU only: for random D and random integer inputs, Algorithm 1, the per-axis
method and the recursion agree with scipy's direct N-D convolution; the sum,
commutativity and linearity hold; float results stay within the derived bound
of the exact (integer-valued) result; the three-operand sum agrees with two
nested scipy convolutions."""
import numpy as np
import scipy.signal
from hypothesis import given, settings, strategies as st

import oracle
from tests import pins

SETTINGS = settings(max_examples=40, deadline=None, derandomize=True)


def vec(draw, D, lo, hi):
    return np.array(draw(st.lists(st.integers(lo, hi), min_size=1 << D, max_size=1 << D)), dtype=np.int64)


@st.composite
def int_pairs(draw, max_d=6, lo=-50, hi=50):
    D = draw(st.integers(0, max_d))
    return D, vec(draw, D, lo, hi), vec(draw, D, lo, hi)


@SETTINGS
@given(int_pairs())
def test_every_int_oracle_is_the_definition(case):
    D, x, y = case
    ref = pins.scipy_definition(x, y)
    for fn in (oracle.naive, oracle.canonical, oracle.recursive):
        pins.assert_bitwise(fn(x, y), ref, f"{fn.__name__} D={D}")


@SETTINGS
@given(int_pairs())
def test_sum_commutativity_linearity(case):
    D, x, y = case
    z = oracle.canonical(x, y)
    assert int(z.sum()) == int(x.sum()) * int(y.sum())
    pins.assert_bitwise(oracle.canonical(y, x), z, "commutativity")
    pins.assert_bitwise(oracle.canonical(2 * x - y, y), 2 * z - oracle.canonical(y, y), "linearity")


@SETTINGS
@given(int_pairs(max_d=7, lo=-1000, hi=1000), st.integers(-40, 40))
def test_float_within_bound_of_exact(case, scale_exp):
    """Integer data scaled by a power of two, computed in float64: the error
    against the exact (integer) result stays within (4D+2) u B."""
    D, x, y = case
    s = 2.0 ** scale_exp
    xf, yf = x.astype(np.float64) * s, y.astype(np.float64) * s
    z = oracle.canonical(xf, yf)
    exact = pins.scipy_definition(x, y).astype(object)
    B = oracle.bound(xf, yf)
    for k in range(3 ** D):
        err = abs(float(z[k]) / (s * s) - int(exact[k]))
        assert err <= (4 * D + 2) * 2.0 ** -53 * B[k] / (s * s) * (1 + 1e-12)


@SETTINGS
@given(st.integers(0, 5), st.data())
def test_sum3_is_two_nested_convolutions(D, data):
    x1, x2, x3 = (vec(data.draw, D, -20, 20) for _ in range(3))
    if D:
        sh = (2,) * D
        ref = scipy.signal.convolve(scipy.signal.convolve(x1.reshape(sh), x2.reshape(sh), method="direct"),
                                    x3.reshape(sh), method="direct").reshape(-1)
    else:
        ref = x1 * x2 * x3
    pins.assert_bitwise(oracle.sum3_canonical(x1, x2, x3), ref, f"sum3 D={D}")
    pins.assert_bitwise(oracle.sum3_naive(x1, x2, x3), ref, f"sum3 naive D={D}")
