"""The bound pins have power: plausible mistakes planted in a copy of the
oracle's C source (built with gcc into a temporary library) each fail at
least one closed-form pin of the rounding bounds, while the unmodified copy
passes all of them.  Mistakes are planted on the CPU only."""
import ctypes
import os

import numpy as np
import pytest

import oracle
from tests import pins

SRC = os.path.join(os.path.dirname(os.path.abspath(oracle.__file__)), "hc_oracle.c")

# (name, exact text in the source, planted replacement)
MUTANTS = [
    ("bound_scaled_by_2", "b[0] = fabs(x[0]) * fabs(y[0]);", "b[0] = 2.0 * fabs(x[0]) * fabs(y[0]);"),
    ("bound_drops_end_term", "b[t + k] = (b[t + k] + b[k]) + b[2 * t + k];", "b[t + k] = b[t + k] + b[k];"),
    ("bound_wrong_half", "s[i] = fabs(x[i]) + fabs(x[h + i]);", "s[i] = fabs(x[i]) + fabs(x[i]);"),
    ("bound_at_digit_swap", "if (digit == 2) base |= (uint64_t)1 << d;", "if (digit == 0) base |= (uint64_t)1 << d;"),
    ("adjoint_bound_drops_w1", "W[(hi * 3 + 0) * n_lo + lo] = w0 + w1;", "W[(hi * 3 + 0) * n_lo + lo] = w0;"),
    ("adjoint_bound_other_operand", "hco_forward_all_f64(which == 0 ? ya : xa, F, T, D);",
     "hco_forward_all_f64(which == 0 ? xa : ya, F, T, D);"),
]


def bound_pins():
    """Names of the closed-form bound pins the current oracle library fails."""
    checks = {
        "all_ones": lambda: [pins.pin_bound_all_ones(oracle.bound, D) for D in (1, 4)],
        "rank1": lambda: [pins.pin_bound_rank1(oracle.bound, D) for D in (2, 5)],
        "at": lambda: pins.pin_bound_at_closed_forms(oracle.bound_at, 13, n=24),
        "adjoint": lambda: [pins.pin_adjoint_bound_closed_forms(oracle.adjoint_bound, D) for D in (1, 4)],
    }
    failed = []
    for name, fn in checks.items():
        try:
            fn()
        except AssertionError:
            failed.append(name)
    return failed


def build_copy(tmp_path, name, old=None, new=None):
    text = open(SRC).read()
    if old is not None:
        assert text.count(old) == 1, f"planting site of {name} not found exactly once"
        text = text.replace(old, new)
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    lib = oracle.build(str(src), str(tmp_path / f"lib{name}.so"),
                       extra_flags=["-I", os.path.dirname(SRC)])
    return oracle.configure(ctypes.CDLL(lib))


def test_unmodified_copy_passes_bound_pins(tmp_path, monkeypatch):
    monkeypatch.setattr(oracle, "_lib", build_copy(tmp_path, "unmodified"))
    assert bound_pins() == []


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_bound_mutant_is_caught(tmp_path, monkeypatch, name, old, new):
    monkeypatch.setattr(oracle, "_lib", build_copy(tmp_path, name, old, new))
    failed = bound_pins()
    assert failed, f"mutant {name} passed every bound pin"
