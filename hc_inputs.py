"""Seeded synthetic inputs for hypercube convolution workloads.

Shared by the tests, the benchmark and the smoke check; holds none of the
method's arithmetic (only random draws and their normalisation), so both the
GPU path's callers and the oracle's callers can use it without sharing code.

Every stream is ``numpy.random.default_rng([SEED, workload_id, pair, role])``
(PCG64), so each pair and operand is reproducible on its own.

Workloads (ids are stable; sizes from the method's hypercube setting, where x
and y hold 2^D values and z holds 3^D):

* 0 -- one pair, D=10, float64 masses
* 1 -- one pair, D=16, int64 values in [0, 15] and float64 masses
* 2 -- one pair, D=20, float64 masses (2^20 inputs, 3^20 outputs)
* 3 -- 4096 pairs with D drawn uniformly from {6, ..., 14}, masses, float64
        and float32
* 4 -- 64 pairs at D=16, float64 masses, loss weights w ~ N(0, 1) per pair
"""
from __future__ import annotations

import numpy as np

SEED = 160800206

W_D10_F64 = 0
W_D16 = 1
W_D20_F64 = 2
W_BATCHED = 3
W_BACKWARD = 4

ROLE_X = 0
ROLE_Y = 1
ROLE_W = 2
ROLE_DIMS = 3


def rng(workload: int, pair: int = 0, role: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED, int(workload), int(pair), int(role)])


def masses(D: int, workload: int, pair: int = 0, role: int = ROLE_X,
           dtype=np.float64) -> np.ndarray:
    """2^D iid Uniform[0,1) values normalised to sum 1 (a probability mass
    function over the hypercube), drawn in float64 and then cast."""
    u = rng(workload, pair, role).random(1 << D)
    x = u / u.sum()
    return x.astype(dtype)


def small_ints(D: int, workload: int, pair: int = 0, role: int = ROLE_X,
               high: int = 16) -> np.ndarray:
    """2^D iid integers in [0, high) as int64."""
    return rng(workload, pair, role).integers(0, high, 1 << D, dtype=np.int64)


def pair_masses(D: int, workload: int, pair: int = 0, dtype=np.float64):
    return (masses(D, workload, pair, ROLE_X, dtype),
            masses(D, workload, pair, ROLE_Y, dtype))


def pair_ints(D: int, workload: int, pair: int = 0, high: int = 16):
    return (small_ints(D, workload, pair, ROLE_X, high),
            small_ints(D, workload, pair, ROLE_Y, high))


def batched_dims(n_pairs: int = 4096, lo: int = 6, hi: int = 14) -> np.ndarray:
    """Per-pair dimensions drawn uniformly from {lo, ..., hi}."""
    return rng(W_BATCHED, 0, ROLE_DIMS).integers(lo, hi + 1, n_pairs).astype(np.int32)


def loss_weights(D: int, workload: int = W_BACKWARD, pair: int = 0,
                 dtype=np.float64) -> np.ndarray:
    """3^D iid N(0, 1) weights w of the loss L = sum(w * z)."""
    return rng(workload, pair, ROLE_W).standard_normal(3 ** D).astype(dtype)


def paper_accuracy_input(D: int, dtype=np.float64) -> np.ndarray:
    """The accuracy workload of the paper's Table 1: x.flat = y.flat =
    [1, 2, ..., 2^D]; the smallest result value z[(0, ..., 0)] is 1."""
    return np.arange(1, (1 << D) + 1).astype(dtype)


def random_pair(D: int, dtype, seed: int, kind: str = "mass"):
    """Generic seeded pair for tests: 'mass' (normalised uniform), 'signed'
    (uniform [-1, 1)), or 'int' (int64 in [0, 16))."""
    g = np.random.default_rng([SEED, 99, int(seed), int(D)])
    n = 1 << D
    if np.dtype(dtype) == np.int64 or kind == "int":
        return (g.integers(0, 16, n, dtype=np.int64), g.integers(0, 16, n, dtype=np.int64))
    if kind == "signed":
        x, y = g.uniform(-1.0, 1.0, n), g.uniform(-1.0, 1.0, n)
    else:
        x, y = g.random(n), g.random(n)
        x, y = x / x.sum(), y / y.sum()
    return x.astype(dtype), y.astype(dtype)
