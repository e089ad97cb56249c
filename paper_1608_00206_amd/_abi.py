"""ctypes binding of libhc (include/hc.h).  Argument marshalling only.

Every function here has the name of the C entry point it calls and takes
plain integers for pointers and streams.  The library must have been built
(``python -m paper_1608_00206_amd.build`` or ``__graft_entry__.build()``);
there is no fallback of any kind when it is missing.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hc.h")

HC_F64, HC_F32, HC_I64 = 0, 1, 2
HC_PLAN_TUNE, HC_PLAN_PERSISTENT, HC_PLAN_PERSISTENT_PAIRS = 1, 2, 4
HC_OK = 0
STATUS_NAMES = {
    0: "HC_OK", 1: "HC_ERR_INVALID_ARG", 2: "HC_ERR_D_RANGE", 3: "HC_ERR_UNSUPPORTED",
    4: "HC_ERR_ALIAS", 5: "HC_ERR_MISALIGNED", 6: "HC_ERR_WORKSPACE", 7: "HC_ERR_NO_DEVICE",
    8: "HC_ERR_HIP",
}
SIZE_MAX = (1 << 64) - 1


class HCError(RuntimeError):
    def __init__(self, code: int, message: str):
        self.code = code
        self.status = STATUS_NAMES.get(code, str(code))
        super().__init__(f"{self.status}: {message}")


_lib = None

class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("alg_bytes", ctypes.c_double)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_U64 = ctypes.c_uint64

SIGNATURES = {
    "hc_abi_version": ([], _I),
    "hc_status_string": ([_I], ctypes.c_char_p),
    "hc_last_error": ([], ctypes.c_char_p),
    "hc_dtype_size": ([_I], _SZ),
    "hc_output_count": ([_I], _U64),
    "hc_workspace_bytes": ([_I, _I, _I], _SZ),
    "hc_convolve": ([_P, _P, _P, _I, _I, _P, _SZ, _P], _I),
    "hc_convolve_batch": ([_P, _P, _P, _I, _I, _I, _P, _SZ, _P], _I),
    "hc_convolve_batch_noalloc": ([_P, _P, _P, _I, _I, _I, _P], _I),
    "hc_backward_workspace_bytes": ([_I, _I, _I], _SZ),
    "hc_convolve_backward_batch": ([_P, _P, _P, _I64, _P, _P, _I, _I, _I, _P, _SZ, _P], _I),
    "hc_convolve_backward": ([_P, _P, _P, _P, _P, _I, _I, _P, _SZ, _P], _I),
    "hc_plan_create_batched": ([ctypes.POINTER(_I), _I, _I, ctypes.c_uint, ctypes.POINTER(_P)], _I),
    "hc_plan_destroy": ([_P], _I),
    "hc_plan_workspace_bytes": ([_P], _SZ),
    "hc_plan_layout": ([_P, ctypes.POINTER(_U64), ctypes.POINTER(_U64)], _I),
    "hc_plan_execute": ([_P, _P, _P, _P, _P, _SZ, _P], _I),
    "hc_plan_check": ([_P], _I),
    "hc_plan_describe": ([_P, ctypes.c_char_p, _SZ], _I),
    "hc_plan_inspect": ([ctypes.POINTER(_I), _I, _I, ctypes.c_uint, ctypes.POINTER(_I64), _I64,
                         ctypes.POINTER(_I64)], _I),
    "hc_carryfree_dim": ([_U64], _I),
    "hc_carryfree_index": ([_U64, _U64], _U64),
    "hc_carryfree_workspace_bytes": ([_U64, _I], _SZ),
    "hc_carryfree_convolve": ([_P, _P, _U64, _P, _I, _P, _SZ, _P], _I),
    "hc_difference_workspace_bytes": ([_I, _I, _I], _SZ),
    "hc_difference_batch": ([_P, _P, _P, _I, _I, _I, _P, _SZ, _P], _I),
    "hc_maxconv_workspace_bytes": ([_I, _I, _I], _SZ),
    "hc_maxconv_pnorm_batch": ([_P, _P, _P, _I, _I, _I, ctypes.c_double, ctypes.c_uint, _P, _SZ, _P], _I),
    "hc_sum3_workspace_bytes": ([_I, _I, _I], _SZ),
    "hc_sum3_batch": ([_P, _P, _P, _P, _I, _I, _I, _P, _SZ, _P], _I),
    "hc_ternary_workspace_bytes": ([_I, _I, _I], _SZ),
    "hc_ternary_convolve_batch": ([_P, _P, _P, _I, _I, _I, _P, _SZ, _P], _I),
    "hc_profile_enable": ([_I], _I),
    "hc_profile_collect": ([ctypes.POINTER(KernelStat), _I, ctypes.POINTER(_I)], _I),
}


def lib():
    """Load libhc.so once; raise loudly if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_1608_00206_amd.build)")
    h = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(h, name)
        fn.argtypes = args
        fn.restype = res
    _lib = h
    return h


def last_error() -> str:
    return lib().hc_last_error().decode()


def check(code: int) -> None:
    if code != HC_OK:
        raise HCError(code, last_error())


def hc_abi_version() -> int:
    return lib().hc_abi_version()


def hc_status_string(code: int) -> str:
    return lib().hc_status_string(code).decode()


def hc_dtype_size(dtype: int) -> int:
    return lib().hc_dtype_size(dtype)


def hc_output_count(D: int) -> int:
    return lib().hc_output_count(D)


def hc_workspace_bytes(D: int, dtype: int, batch: int = 1) -> int:
    return lib().hc_workspace_bytes(D, dtype, batch)


def hc_backward_workspace_bytes(D: int, dtype: int, batch: int = 1) -> int:
    return lib().hc_backward_workspace_bytes(D, dtype, batch)


def hc_convolve(x: int, y: int, z: int, D: int, dtype: int, ws: int, ws_bytes: int, stream: int) -> int:
    return lib().hc_convolve(x, y, z, D, dtype, ws, ws_bytes, stream)


def hc_convolve_batch(x: int, y: int, z: int, D: int, dtype: int, batch: int, ws: int, ws_bytes: int,
                      stream: int) -> int:
    return lib().hc_convolve_batch(x, y, z, D, dtype, batch, ws, ws_bytes, stream)


def hc_convolve_batch_noalloc(x: int, y: int, z: int, D: int, dtype: int, batch: int, stream: int) -> int:
    return lib().hc_convolve_batch_noalloc(x, y, z, D, dtype, batch, stream)


def hc_convolve_backward_batch(x: int, y: int, gz: int, gz_stride: int, gx: int, gy: int, D: int, dtype: int,
                               batch: int, ws: int, ws_bytes: int, stream: int) -> int:
    return lib().hc_convolve_backward_batch(x, y, gz, gz_stride, gx, gy, D, dtype, batch, ws, ws_bytes, stream)


def hc_convolve_backward(x: int, y: int, gz: int, gx: int, gy: int, D: int, dtype: int, ws: int, ws_bytes: int,
                         stream: int) -> int:
    return lib().hc_convolve_backward(x, y, gz, gx, gy, D, dtype, ws, ws_bytes, stream)


def hc_carryfree_dim(n: int) -> int:
    return lib().hc_carryfree_dim(n)


def hc_carryfree_index(i: int, j: int) -> int:
    return lib().hc_carryfree_index(i, j)


def hc_carryfree_workspace_bytes(n: int, dtype: int) -> int:
    return lib().hc_carryfree_workspace_bytes(n, dtype)


def hc_carryfree_convolve(x: int, y: int, n: int, z: int, dtype: int, ws: int, ws_bytes: int, stream: int) -> int:
    return lib().hc_carryfree_convolve(x, y, n, z, dtype, ws, ws_bytes, stream)


def hc_difference_workspace_bytes(D: int, dtype: int, batch: int = 1) -> int:
    return lib().hc_difference_workspace_bytes(D, dtype, batch)


def hc_difference_batch(x: int, y: int, z: int, D: int, dtype: int, batch: int, ws: int, ws_bytes: int,
                        stream: int) -> int:
    return lib().hc_difference_batch(x, y, z, D, dtype, batch, ws, ws_bytes, stream)


def hc_sum3_workspace_bytes(D: int, dtype: int, batch: int = 1) -> int:
    return lib().hc_sum3_workspace_bytes(D, dtype, batch)


def hc_sum3_batch(x1: int, x2: int, x3: int, z: int, D: int, dtype: int, batch: int, ws: int, ws_bytes: int,
                  stream: int) -> int:
    return lib().hc_sum3_batch(x1, x2, x3, z, D, dtype, batch, ws, ws_bytes, stream)


def hc_ternary_workspace_bytes(D: int, dtype: int, batch: int = 1) -> int:
    return lib().hc_ternary_workspace_bytes(D, dtype, batch)


def hc_ternary_convolve_batch(a: int, b: int, z: int, D: int, dtype: int, batch: int, ws: int, ws_bytes: int,
                              stream: int) -> int:
    return lib().hc_ternary_convolve_batch(a, b, z, D, dtype, batch, ws, ws_bytes, stream)


HC_MAXCONV_ROUND = 1
HC_MAXCONV_SEPARATE_ROOT = 2


def hc_maxconv_workspace_bytes(D: int, dtype: int, batch: int = 1) -> int:
    return lib().hc_maxconv_workspace_bytes(D, dtype, batch)


def hc_maxconv_pnorm_batch(x: int, y: int, z: int, D: int, dtype: int, batch: int, p: float, flags: int, ws: int,
                           ws_bytes: int, stream: int) -> int:
    return lib().hc_maxconv_pnorm_batch(x, y, z, D, dtype, batch, p, flags, ws, ws_bytes, stream)


def hc_profile_enable(on: bool) -> int:
    return lib().hc_profile_enable(1 if on else 0)


def hc_profile_collect(capacity: int = 64):
    """Returns [(name, launches, total_ms, alg_bytes)] for the recorded launches."""
    arr = (KernelStat * capacity)()
    n = _I(0)
    check(lib().hc_profile_collect(arr, capacity, ctypes.byref(n)))
    return [(arr[i].name.decode(), int(arr[i].launches), float(arr[i].total_ms), float(arr[i].alg_bytes))
            for i in range(n.value)]


def hc_plan_create_batched(Ds, dtype: int, flags: int = 0) -> int:
    """Returns the plan handle (an integer); raises HCError on failure."""
    arr = (_I * len(Ds))(*[int(d) for d in Ds])
    out = _P(0)
    check(lib().hc_plan_create_batched(arr, len(Ds), dtype, flags, ctypes.byref(out)))
    return out.value


def hc_plan_destroy(plan: int) -> int:
    return lib().hc_plan_destroy(plan)


def hc_plan_workspace_bytes(plan: int) -> int:
    return lib().hc_plan_workspace_bytes(plan)


def hc_plan_layout(plan: int, n_pairs: int):
    xo = (_U64 * (n_pairs + 1))()
    zo = (_U64 * (n_pairs + 1))()
    check(lib().hc_plan_layout(plan, xo, zo))
    return list(xo), list(zo)


def hc_plan_execute(plan: int, x: int, y: int, z: int, ws: int, ws_bytes: int, stream: int) -> int:
    return lib().hc_plan_execute(plan, x, y, z, ws, ws_bytes, stream)


def hc_plan_check(plan: int) -> int:
    return lib().hc_plan_check(plan)


def hc_plan_describe(plan: int) -> str:
    buf = ctypes.create_string_buffer(1 << 16)
    check(lib().hc_plan_describe(plan, buf, len(buf)))
    return buf.value.decode()


def hc_plan_inspect(Ds, dtype: int, flags: int = 0):
    """Groups of the default schedule, host only: list of dicts."""
    arr = (_I * len(Ds))(*[int(d) for d in Ds])
    n = _I64(0)
    check(lib().hc_plan_inspect(arr, len(Ds), dtype, flags, None, 0, ctypes.byref(n)))
    info = (_I64 * (6 * n.value))()
    check(lib().hc_plan_inspect(arr, len(Ds), dtype, flags, info, n.value, ctypes.byref(n)))
    keys = ("D", "pairs", "first_pair", "K", "fwd_passes", "inv_passes")
    return [dict(zip(keys, info[6 * i:6 * i + 6])) for i in range(n.value)]
