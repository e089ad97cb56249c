"""CPU oracle for exact hypercube convolution -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product package never imports it
and shares no code with it.

Wraps ``oracle/hc_oracle.c`` (plain C, built with ``-ffp-contract=off``) with
numpy arrays:

* ``naive``      -- Algorithm 1 (naive Cartesian product) on hypercubes.
* ``canonical``  -- the method in per-axis form: forward map on axes
  0..D-1, elementwise product, inverse map on axes D-1..0 (Methods section,
  three-subproblem recursion, unrolled over all axes).
* ``recursive``  -- the three-subproblem recursion itself (memory-light).
* ``adjoint``    -- gradient of ``sum(w * z)`` by transposed maps.
* ``direct_at`` / ``correlation_at`` -- the definitions evaluated at chosen
  indices with compensated long double sums.
* ``bound`` / ``adjoint_bound`` -- magnitudes B with
  ``|computed - exact| <= (4D + 2) u B``.

dtype is taken from the inputs: float64, float32 or int64 (int64 arithmetic
wraps modulo 2^64, which is exact whenever the true result fits in int64).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = [os.path.join(_HERE, "hc_oracle.c"), os.path.join(_HERE, "hc_oracle_impl.h"),
           os.path.join(_HERE, "hc_oracle_sum3.h"), os.path.join(_HERE, "hc_oracle_ternary.h")]

CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-fPIC", "-shared"]

_lib = None


def build(source: str = SOURCES[0], target: str = LIB_PATH, extra_flags=()) -> str:
    """Compile the oracle shared library with gcc (always recompiles)."""
    tmp = target + ".tmp"
    cmd = ["gcc", *CFLAGS, *extra_flags, "-o", tmp, source, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, target)
    return target


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    _lib = configure(ctypes.CDLL(LIB_PATH))
    return _lib


def configure(lib):
    """Declare the argument and result types of the oracle's exports on a
    loaded library (the oracle itself, or a copy built from edited sources
    by the tests that plant mistakes in it)."""
    P = ctypes.c_void_p
    I = ctypes.c_int
    I64 = ctypes.c_int64
    for sfx in ("f64", "f32", "i64"):
        for name, args in (("hco_naive_", [P, P, P, I]),
                           ("hco_canonical_", [P, P, P, I]),
                           ("hco_recursive_", [P, P, P, I, I]),
                           ("hco_adjoint_", [P, P, P, P, P, I]),
                           ("hco_carryfree_naive_", [P, P, ctypes.c_uint64, P]),
                           ("hco_difference_naive_", [P, P, P, I]),
                           ("hco_sum3_naive_", [P, P, P, P, I]),
                           ("hco_sum3_canonical_", [P, P, P, P, I]),
                           ("hco_ternary_naive_", [P, P, P, I]),
                           ("hco_ternary_canonical_", [P, P, P, I])):
            fn = getattr(lib, name + sfx)
            fn.argtypes = args
            fn.restype = I
    lib.hco_pow3.argtypes = [I]
    lib.hco_pow3.restype = ctypes.c_uint64
    lib.hco_tern.argtypes = [ctypes.c_uint64]
    lib.hco_tern.restype = ctypes.c_uint64
    lib.hco_tern_map.argtypes = [I, P]
    lib.hco_tern_map.restype = None
    lib.hco_direct_at_f64.argtypes = [P, P, I, P, I64, P]
    lib.hco_direct_at_f64.restype = None
    lib.hco_direct_at_i64.argtypes = [P, P, I, P, I64, P]
    lib.hco_direct_at_i64.restype = None
    lib.hco_correlation_at_f64.argtypes = [P, P, P, I, P, I64, P, P]
    lib.hco_correlation_at_f64.restype = None
    lib.hco_bound_f64.argtypes = [P, P, P, I]
    lib.hco_bound_f64.restype = I
    lib.hco_maxconv_at_f64.argtypes = [P, P, I, P, I64, P]
    lib.hco_maxconv_at_f64.restype = None
    lib.hco_pnorm_at_f64.argtypes = [P, P, I, ctypes.c_double, P, I64, P]
    lib.hco_pnorm_at_f64.restype = None
    lib.hco_bound_at_f64.argtypes = [P, P, I, P, I64, P]
    lib.hco_bound_at_f64.restype = I
    lib.hco_adjoint_bound_f64.argtypes = [P, P, P, P, P, I]
    lib.hco_adjoint_bound_f64.restype = I
    lib.hco_sum3_direct_at_f64.argtypes = [P, P, P, I, P, I64, P]
    lib.hco_sum3_direct_at_f64.restype = None
    lib.hco_sum3_bound_f64.argtypes = [P, P, P, P, I]
    lib.hco_sum3_bound_f64.restype = I
    lib.hco_ternary_direct_at_f64.argtypes = [P, P, I, P, I64, P]
    lib.hco_ternary_direct_at_f64.restype = None
    lib.hco_ternary_bound_f64.argtypes = [P, P, P, I]
    lib.hco_ternary_bound_f64.restype = I
    return lib


_SFX = {np.dtype(np.float64): "f64", np.dtype(np.float32): "f32", np.dtype(np.int64): "i64"}


def pow3(n: int) -> int:
    return 3 ** n


def dim_of(x: np.ndarray) -> int:
    n = int(x.size)
    D = n.bit_length() - 1
    if n <= 0 or (1 << D) != n:
        raise ValueError(f"hypercube input must have 2^D elements, got {n}")
    return D


def _vec(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a).reshape(-1)
    if a.dtype not in _SFX:
        raise TypeError(f"unsupported dtype {a.dtype}")
    return a


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _pair(x, y):
    x, y = _vec(x), _vec(y)
    if x.dtype != y.dtype or x.size != y.size:
        raise ValueError("x and y must have the same dtype and size")
    return x, y, dim_of(x), _SFX[x.dtype]


def tern(i: int) -> int:
    return int(_load().hco_tern(int(i)))


def tern_map(D: int) -> np.ndarray:
    out = np.empty(1 << D, dtype=np.uint64)
    _load().hco_tern_map(D, _ptr(out))
    return out


def naive(x, y) -> np.ndarray:
    x, y, D, sfx = _pair(x, y)
    z = np.empty(3 ** D, dtype=x.dtype)
    rc = getattr(_load(), "hco_naive_" + sfx)(_ptr(x), _ptr(y), _ptr(z), D)
    if rc:
        raise RuntimeError(f"hco_naive_{sfx} failed ({rc})")
    return z


def canonical(x, y) -> np.ndarray:
    x, y, D, sfx = _pair(x, y)
    z = np.empty(3 ** D, dtype=x.dtype)
    rc = getattr(_load(), "hco_canonical_" + sfx)(_ptr(x), _ptr(y), _ptr(z), D)
    if rc:
        raise RuntimeError(f"hco_canonical_{sfx} failed ({rc})")
    return z


def recursive(x, y, threads: int = 1, out: np.ndarray | None = None) -> np.ndarray:
    x, y, D, sfx = _pair(x, y)
    if out is None:
        out = np.empty(3 ** D, dtype=x.dtype)
    if out.dtype != x.dtype or out.size != 3 ** D or not out.flags.c_contiguous:
        raise ValueError("bad output buffer")
    rc = getattr(_load(), "hco_recursive_" + sfx)(_ptr(x), _ptr(y), _ptr(out), D, int(threads))
    if rc:
        raise RuntimeError(f"hco_recursive_{sfx} failed ({rc})")
    return out


def carryfree_naive(x, y) -> np.ndarray:
    """Carry-free convolution of two length-n vectors (any n >= 1) by its
    definition; 3^D outputs, D = bits of n - 1."""
    x = _vec(x)
    y = _vec(y)
    if x.dtype != y.dtype or x.size != y.size or x.size == 0:
        raise ValueError("x and y must be non-empty vectors of one length and dtype")
    n = x.size
    D = max(0, (n - 1).bit_length())
    z = np.empty(3 ** D, dtype=x.dtype)
    rc = getattr(_load(), "hco_carryfree_naive_" + _SFX[x.dtype])(_ptr(x), _ptr(y), n, _ptr(z))
    if rc:
        raise RuntimeError(f"hco_carryfree_naive failed ({rc})")
    return z


def difference_naive(x, y) -> np.ndarray:
    """Distribution of X - Y by its definition: output digit a is
    bit_a(i) - bit_a(j) + 1."""
    x, y, D, sfx = _pair(x, y)
    z = np.empty(3 ** D, dtype=x.dtype)
    rc = getattr(_load(), "hco_difference_naive_" + sfx)(_ptr(x), _ptr(y), _ptr(z), D)
    if rc:
        raise RuntimeError(f"hco_difference_naive_{sfx} failed ({rc})")
    return z


def adjoint(x, y, w):
    x, y, D, sfx = _pair(x, y)
    w = _vec(w)
    if w.dtype != x.dtype or w.size != 3 ** D:
        raise ValueError("w must have 3^D elements of the input dtype")
    gx = np.empty(1 << D, dtype=x.dtype)
    gy = np.empty(1 << D, dtype=x.dtype)
    rc = getattr(_load(), "hco_adjoint_" + sfx)(_ptr(x), _ptr(y), _ptr(w), _ptr(gx), _ptr(gy), D)
    if rc:
        raise RuntimeError(f"hco_adjoint_{sfx} failed ({rc})")
    return gx, gy


def direct_at(x, y, ks) -> np.ndarray:
    x, y, D, sfx = _pair(x, y)
    ks = np.ascontiguousarray(ks, dtype=np.uint64).reshape(-1)
    if ks.size and int(ks.max()) >= 3 ** D:
        raise ValueError("output index out of range")
    if sfx == "f32":
        raise TypeError("direct_at supports float64 and int64")
    out = np.empty(ks.size, dtype=x.dtype)
    getattr(_load(), "hco_direct_at_" + sfx)(_ptr(x), _ptr(y), D, _ptr(ks), ks.size, _ptr(out))
    return out


def correlation_at(x, y, w, idx):
    x, y, D, sfx = _pair(x, y)
    if sfx != "f64":
        raise TypeError("correlation_at supports float64")
    w = _vec(w)
    idx = np.ascontiguousarray(idx, dtype=np.uint64).reshape(-1)
    if idx.size and int(idx.max()) >= (1 << D):
        raise ValueError("input index out of range")
    gx = np.empty(idx.size, dtype=np.float64)
    gy = np.empty(idx.size, dtype=np.float64)
    _load().hco_correlation_at_f64(_ptr(x), _ptr(y), _ptr(w), D, _ptr(idx), idx.size,
                                   _ptr(gx), _ptr(gy))
    return gx, gy


def _at_f64(fn, x, y, ks, *extra):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    x, y, D, _ = _pair(x, y)
    ks = np.ascontiguousarray(ks, dtype=np.uint64).reshape(-1)
    if ks.size and int(ks.max()) >= 3 ** D:
        raise ValueError("output index out of range")
    out = np.empty(ks.size, dtype=np.float64)
    if extra:
        fn(_ptr(x), _ptr(y), D, *extra, _ptr(ks), ks.size, _ptr(out))
    else:
        fn(_ptr(x), _ptr(y), D, _ptr(ks), ks.size, _ptr(out))
    return out


def maxconv_at(x, y, ks) -> np.ndarray:
    """Max-convolution max x[i]*y[j] over the pairs of each output index."""
    return _at_f64(_load().hco_maxconv_at_f64, x, y, ks)


def pnorm_at(x, y, p, ks) -> np.ndarray:
    """p-norm estimate (sum (x[i] y[j])^p)^(1/p) of the max-convolution at
    the given output indices (nonnegative inputs)."""
    return _at_f64(_load().hco_pnorm_at_f64, x, y, ks, ctypes.c_double(float(p)))


def bound(x, y) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    x, y, D, _ = _pair(x, y)
    b = np.empty(3 ** D, dtype=np.float64)
    _load().hco_bound_f64(_ptr(x), _ptr(y), _ptr(b), D)
    return b


def bound_at(x, y, ks) -> np.ndarray:
    """bound() at selected output indices (each with at most 14 digits equal
    to 1), without forming the whole 3^D array."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    x, y, D, _ = _pair(x, y)
    ks = np.ascontiguousarray(ks, dtype=np.uint64).reshape(-1)
    if ks.size and int(ks.max()) >= 3 ** D:
        raise ValueError("output index out of range")
    out = np.empty(ks.size, dtype=np.float64)
    if _load().hco_bound_at_f64(_ptr(x), _ptr(y), D, _ptr(ks), ks.size, _ptr(out)):
        raise ValueError("bound_at: an index has more than 14 digits equal to 1")
    return out


def adjoint_bound(x, y, w):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    x, y, D, _ = _pair(x, y)
    w = _vec(np.asarray(w, dtype=np.float64))
    bx = np.empty(1 << D, dtype=np.float64)
    by = np.empty(1 << D, dtype=np.float64)
    _load().hco_adjoint_bound_f64(_ptr(x), _ptr(y), _ptr(w), _ptr(bx), _ptr(by), D)
    return bx, by


def _triple(x1, x2, x3):
    x1, x2, x3 = _vec(x1), _vec(x2), _vec(x3)
    if not (x1.dtype == x2.dtype == x3.dtype and x1.size == x2.size == x3.size):
        raise ValueError("x1, x2 and x3 must have the same dtype and size")
    return x1, x2, x3, dim_of(x1), _SFX[x1.dtype]


def sum3_naive(x1, x2, x3) -> np.ndarray:
    """Distribution of X1 + X2 + X3 (three hypercubes, 4^D outputs, base-4
    digit = sum of the three bits) by its definition, every triple of
    entries (D <= 12)."""
    x1, x2, x3, D, sfx = _triple(x1, x2, x3)
    z = np.empty(4 ** D, dtype=x1.dtype)
    rc = getattr(_load(), "hco_sum3_naive_" + sfx)(_ptr(x1), _ptr(x2), _ptr(x3), _ptr(z), D)
    if rc:
        raise RuntimeError(f"hco_sum3_naive_{sfx} failed ({rc})")
    return z


def sum3_canonical(x1, x2, x3) -> np.ndarray:
    """The same distribution by the per-axis method for three operands:
    forward (a0, a0 + a1, a0 - a1, a1) on axes 0..D-1, the product
    (x1^ x2^) x3^, inverse from the values at 0, 1, -1 and infinity on axes
    D-1..0 (D <= 14)."""
    x1, x2, x3, D, sfx = _triple(x1, x2, x3)
    z = np.empty(4 ** D, dtype=x1.dtype)
    rc = getattr(_load(), "hco_sum3_canonical_" + sfx)(_ptr(x1), _ptr(x2), _ptr(x3), _ptr(z), D)
    if rc:
        raise RuntimeError(f"hco_sum3_canonical_{sfx} failed ({rc})")
    return z


def sum3_direct_at(x1, x2, x3, ks) -> np.ndarray:
    """Definition of the three-operand distribution at chosen indices,
    compensated long double sums (float64 data)."""
    x1, x2, x3, D, _ = _triple(*(np.asarray(v, dtype=np.float64) for v in (x1, x2, x3)))
    ks = np.ascontiguousarray(ks, dtype=np.uint64).reshape(-1)
    if ks.size and int(ks.max()) >= 4 ** D:
        raise ValueError("output index out of range")
    out = np.empty(ks.size, dtype=np.float64)
    _load().hco_sum3_direct_at_f64(_ptr(x1), _ptr(x2), _ptr(x3), D, _ptr(ks), ks.size, _ptr(out))
    return out


def sum3_bound(x1, x2, x3) -> np.ndarray:
    """B with |sum3_canonical - exact| <= (5D + 2) u B."""
    x1, x2, x3, D, _ = _triple(*(np.asarray(v, dtype=np.float64) for v in (x1, x2, x3)))
    b = np.empty(4 ** D, dtype=np.float64)
    if _load().hco_sum3_bound_f64(_ptr(x1), _ptr(x2), _ptr(x3), _ptr(b), D):
        raise ValueError("sum3_bound: D out of range")
    return b


def _ternary_pair(a, b):
    a, b = _vec(a), _vec(b)
    if a.dtype != b.dtype or a.size != b.size:
        raise ValueError("a and b must have the same dtype and size")
    n = a.size
    D = 0
    while 3 ** D < n:
        D += 1
    if 3 ** D != n:
        raise ValueError("length must be a power of 3")
    return a, b, D, _SFX[a.dtype]


def ternary_naive(a, b) -> np.ndarray:
    """Convolution of two ternary cubes {0,1,2}^D (3^D values each, the
    layout of the hypercube convolution's output) into 5^D values (base-5
    digit = sum of the two ternary digits) by its definition, every pair of
    entries (D <= 8)."""
    a, b, D, sfx = _ternary_pair(a, b)
    z = np.empty(5 ** D, dtype=a.dtype)
    rc = getattr(_load(), "hco_ternary_naive_" + sfx)(_ptr(a), _ptr(b), _ptr(z), D)
    if rc:
        raise RuntimeError(f"hco_ternary_naive_{sfx} failed ({rc})")
    return z


def ternary_canonical(a, b) -> np.ndarray:
    """The same convolution by the six-product per-axis method: forward
    (a0, a1, a2) -> (a0, a1, a2, a0 + a1, a1 + a2, a0 + a2) on axes 0..D-1,
    the product, inverse (p0, p1, p2, q01, q12, q02) -> (p0, (q01 - p0) - p1,
    ((q02 - p0) - p2) + p1, (q12 - p1) - p2, p2) on axes D-1..0 (D <= 10)."""
    a, b, D, sfx = _ternary_pair(a, b)
    z = np.empty(5 ** D, dtype=a.dtype)
    rc = getattr(_load(), "hco_ternary_canonical_" + sfx)(_ptr(a), _ptr(b), _ptr(z), D)
    if rc:
        raise RuntimeError(f"hco_ternary_canonical_{sfx} failed ({rc})")
    return z


def ternary_direct_at(a, b, ks) -> np.ndarray:
    """Definition of the ternary convolution at chosen output indices,
    compensated long double sums (float64 data)."""
    a, b, D, _ = _ternary_pair(np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64))
    ks = np.ascontiguousarray(ks, dtype=np.uint64).reshape(-1)
    if ks.size and int(ks.max()) >= 5 ** D:
        raise ValueError("output index out of range")
    out = np.empty(ks.size, dtype=np.float64)
    _load().hco_ternary_direct_at_f64(_ptr(a), _ptr(b), D, _ptr(ks), ks.size, _ptr(out))
    return out


def ternary_bound(a, b) -> np.ndarray:
    """B with |ternary_canonical - exact| <= (5D + 1) u B (D <= 10)."""
    a, b, D, _ = _ternary_pair(np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64))
    out = np.empty(5 ** D, dtype=np.float64)
    if _load().hco_ternary_bound_f64(_ptr(a), _ptr(b), _ptr(out), D):
        raise ValueError("ternary_bound: D out of range")
    return out


def unit_roundoff(dtype) -> float:
    """u for the dtype's arithmetic (0 for int64, which is exact modulo 2^64)."""
    dt = np.dtype(dtype)
    if dt == np.float64:
        return 2.0 ** -53
    if dt == np.float32:
        return 2.0 ** -24
    return 0.0
