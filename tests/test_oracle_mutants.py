"""The pins have power: every plausible mistake planted in a (numpy) copy of
the per-axis method fails at least one pin, while the unmodified copy passes
all of them.  Mistakes are planted on the CPU, never in the GPU path."""
import numpy as np
import pytest

import oracle
from tests import pins
from tests._numpy_method import per_axis


def run_all_pins(impl):
    """Returns the names of the pins the implementation fails."""
    failed = []
    checks = {
        "worked_example": lambda: pins.pin_worked_example(impl, np.float64),
        "deltas": lambda: [pins.pin_deltas(impl, np.int64, D) for D in (3, 6)],
        "d1_int": lambda: pins.pin_d1_int(impl),
        "d1_rounding": lambda: pins.pin_d1_rounding(impl),
        "scipy": lambda: [pins.pin_scipy_int(impl, D) for D in (2, 5)],
        "all_ones": lambda: pins.pin_all_ones(impl, np.float64, 5),
        "sum": lambda: pins.pin_sum_int(impl, 5),
        "marginals": lambda: pins.pin_marginals_int(impl, 4),
        "exact_bound": lambda: pins.pin_exact_bound(impl, np.float64, 4, oracle.bound),
        "recursion": lambda: [pins.pin_matches_recursion(impl, np.float64, D, oracle.recursive)
                              for D in (3, 6)],
    }
    for name, fn in checks.items():
        try:
            fn()
        except AssertionError:
            failed.append(name)
    return failed


def test_unmodified_copy_passes_every_pin():
    assert run_all_pins(lambda x, y: per_axis(x, y)) == []


MUTANTS = {
    "inverse_ascending": dict(inverse_order="asc"),
    "forward_descending": dict(forward_order="desc"),
    "subtract_sum_of_ends": dict(assoc="right"),
    "wrong_sign": dict(sign=+1),
    "dropped_term": dict(drop_p2=True),
    "forward_copies_end": dict(forward_mid="copy"),
    "axis0_is_lsb": dict(lsb_first=True),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    failed = run_all_pins(lambda x, y: per_axis(x, y, **MUTANTS[name]))
    assert failed, f"mutant {name} passed every pin"


def test_transposed_operand_is_caught():
    # x * x instead of x * y
    failed = run_all_pins(lambda x, y: per_axis(x, x))
    assert failed
