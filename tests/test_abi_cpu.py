"""The C ABI on the CPU: the library loads, exports every function that
include/hc.h declares, sizes workspaces, and rejects bad arguments with the
documented status codes before touching the GPU (no compute calls here)."""
import os
import re

import pytest

from paper_1608_00206_amd import _abi

HEADER = _abi.HEADER
FAKE = 0x10000000  # never dereferenced: validation fails before any HIP call


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hc_[a-z_0-9]+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = _abi.lib()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), f"{n} declared in hc.h but not exported"
    assert set(names) == set(_abi.SIGNATURES), "binding and header disagree"


def test_abi_version_and_status_strings():
    assert _abi.hc_abi_version() == 1
    for code, name in _abi.STATUS_NAMES.items():
        assert _abi.hc_status_string(code)
    assert _abi.hc_status_string(999) == "unknown status"


def test_sizes():
    assert _abi.hc_dtype_size(_abi.HC_F64) == 8
    assert _abi.hc_dtype_size(_abi.HC_F32) == 4
    assert _abi.hc_dtype_size(_abi.HC_I64) == 8
    assert _abi.hc_dtype_size(7) == 0
    assert _abi.hc_output_count(0) == 1
    assert _abi.hc_output_count(20) == 3 ** 20
    assert _abi.hc_output_count(22) == 0
    assert _abi.hc_output_count(-1) == 0


def test_workspace_sizes():
    # one fused tile needs no workspace
    for D in range(0, 9):
        assert _abi.hc_workspace_bytes(D, _abi.HC_F64, 1) == 0
    # D = 20 float64: x~ and y~ are 3^12 x 2^8 each, plus staging
    ws = _abi.hc_workspace_bytes(20, _abi.HC_F64, 1)
    assert 2 * 3 ** 12 * 2 ** 8 * 8 <= ws <= 3 * 2 * 3 ** 12 * 2 ** 8 * 8
    assert _abi.hc_workspace_bytes(12, _abi.HC_F64, 4) == 4 * _abi.hc_workspace_bytes(12, _abi.HC_F64, 1)
    assert _abi.hc_workspace_bytes(22, _abi.HC_F64, 1) == _abi.SIZE_MAX
    assert _abi.hc_workspace_bytes(10, 9, 1) == _abi.SIZE_MAX
    assert _abi.hc_workspace_bytes(10, 0, 0) == _abi.SIZE_MAX
    # backward: w_hat (3^D) dominates
    assert _abi.hc_backward_workspace_bytes(16, _abi.HC_F64, 1) >= 3 ** 16 * 8


def _conv(x=FAKE, y=FAKE + (1 << 20), z=FAKE + (1 << 24), D=10, dtype=0, ws=0, wsb=0, batch=1):
    return _abi.hc_convolve_batch(x, y, z, D, dtype, batch, ws, wsb, 0)


@pytest.mark.parametrize("kw,code", [
    (dict(x=0), 1), (dict(y=0), 1), (dict(z=0), 1),
    (dict(D=-1), 2), (dict(D=22), 2),
    (dict(dtype=3), 3), (dict(dtype=-1), 3),
    (dict(batch=0), 1), (dict(batch=70000), 1),
    (dict(x=FAKE + 4), 5), (dict(z=FAKE + (1 << 24) + 4), 5), (dict(dtype=1, y=FAKE + (1 << 20) + 2), 5),
    (dict(D=12, ws=FAKE + (1 << 30) + 8, wsb=1 << 30), 5),
    (dict(z=FAKE + 64), 4),                      # z overlaps x
    (dict(D=12), 6),                              # workspace required but missing
    (dict(D=12, ws=FAKE + (1 << 30), wsb=16), 6),  # too small
])
def test_validation_errors(kw, code):
    rc = _conv(**kw)
    assert rc == code, (rc, _abi.last_error())
    assert _abi.last_error()


def test_workspace_alias_rejected():
    need = _abi.hc_workspace_bytes(12, 0, 1)
    z = FAKE + (1 << 26)
    rc = _conv(D=12, z=z, ws=z + 8 * 100, wsb=need)
    assert rc == 4


def test_backward_validation():
    f = _abi.hc_convolve_backward_batch
    T = 1 << 40  # far apart: no range overlaps unless a test asks for one
    ok = dict(x=T, y=2 * T, gz=3 * T, st=0, gx=4 * T, gy=5 * T, D=8, dt=0, b=1, ws=0, wsb=0)

    def call(**kw):
        a = {**ok, **kw}
        return f(a["x"], a["y"], a["gz"], a["st"], a["gx"], a["gy"], a["D"], a["dt"], a["b"],
                 a["ws"], a["wsb"], 0)

    assert call(dt=2) == 3                   # int64 backward unsupported
    assert call(gx=0, gy=0) == 1             # nothing requested
    assert call(gz=0) == 1
    assert call(st=5) == 1                   # stride neither 0 nor >= 3^D
    assert call(gx=T + 16) == 4              # grad_x overlaps x
    assert call(D=23) == 2
    assert call(D=16) == 6                   # workspace needed


def test_valid_call_reaches_device_check_without_gpu():
    """With valid arguments the only remaining failure on a CPU-only host is
    the missing device (no fallback path computes anything)."""
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except Exception:
        pass
    rc = _conv(D=4)
    assert rc == 7, _abi.last_error()


def test_product_package_does_not_import_oracle():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = os.path.join(root, "paper_1608_00206_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "hc_oracle" not in text and "liboracle" not in text, f


def test_plan_validation():
    f = _abi.lib().hc_plan_create_batched
    import ctypes
    Ds = (ctypes.c_int * 3)(4, 9, 12)
    out = ctypes.c_void_p(0)
    assert f(None, 3, 0, 0, ctypes.byref(out)) == 1
    assert f(Ds, 0, 0, 0, ctypes.byref(out)) == 1
    assert f(Ds, 3, 0, 0, None) == 1
    assert f(Ds, 3, 0, 8, ctypes.byref(out)) == 1          # unknown flag
    assert f(Ds, 3, 0, 2, ctypes.byref(out)) == 3          # persistent kernel disabled
    assert f(Ds, 3, 0, 2 | 4, ctypes.byref(out)) == 1      # the two persistent modes exclude each other
    assert f(Ds, 3, 7, 0, ctypes.byref(out)) == 3          # unknown dtype
    bad = (ctypes.c_int * 2)(4, 17)
    assert f(bad, 2, 0, 0, ctypes.byref(out)) == 2
    assert _abi.lib().hc_plan_workspace_bytes(None) == _abi.SIZE_MAX
    assert _abi.lib().hc_plan_destroy(None) == 0
    assert _abi.lib().hc_plan_execute(None, 0, 0, 0, 0, 0, None) == 1


# ------------------------------------------------ applications (host side)

def test_carryfree_dim_and_index():
    assert [_abi.hc_carryfree_dim(n) for n in (1, 2, 3, 4, 5, 1000, 1 << 21)] == [0, 1, 2, 2, 3, 10, 21]
    assert _abi.hc_carryfree_dim(0) == -1
    assert _abi.hc_carryfree_dim((1 << 21) + 1) == -1
    # the Discussion's example: bits (1,1,1) + (1,0,1) = digits (2,1,2)
    assert _abi.hc_carryfree_index(7, 5) == 2 * 9 + 1 * 3 + 2
    for i, j in [(0, 0), (1, 0), (3, 6), (1000, 77)]:
        k, w, a, b = 0, 1, i, j
        while a or b:
            k += ((a & 1) + (b & 1)) * w
            a, b, w = a >> 1, b >> 1, w * 3
        assert _abi.hc_carryfree_index(i, j) == k


def test_application_workspace_sizes():
    f64 = _abi.HC_F64
    # a power-of-two length needs only the convolution's workspace
    assert _abi.hc_carryfree_workspace_bytes(1 << 12, f64) == _abi.hc_workspace_bytes(12, f64)
    # otherwise two zero-padded copies come first
    assert _abi.hc_carryfree_workspace_bytes(3000, f64) >= 2 * 4096 * 8 + _abi.hc_workspace_bytes(12, f64)
    assert _abi.hc_carryfree_workspace_bytes(0, f64) == _abi.SIZE_MAX
    assert _abi.hc_carryfree_workspace_bytes(5, 9) == _abi.SIZE_MAX
    assert _abi.hc_difference_workspace_bytes(10, f64, 3) >= 3 * 1024 * 8 + _abi.hc_workspace_bytes(10, f64, 3)
    assert _abi.hc_difference_workspace_bytes(-1, f64, 1) == _abi.SIZE_MAX


def test_application_validation():
    x, y, z = FAKE, FAKE + (1 << 22), FAKE + (1 << 26)
    cf = _abi.hc_carryfree_convolve
    assert cf(0, y, 100, z, 0, 0, 0, 0) == 1                   # null x
    assert cf(x, y, 0, z, 0, 0, 0, 0) == 2                      # n = 0
    assert cf(x, y, 100, z, 7, 0, 0, 0) == 3                    # dtype
    assert cf(x + 4, y, 100, z, 0, FAKE + (1 << 30), 1 << 20, 0) == 5   # misaligned
    assert cf(x, y, 100, z, 0, 0, 0, 0) == 6                    # padding needs a workspace
    assert cf(x, y, 100, x + 64, 0, FAKE + (1 << 30), 1 << 20, 0) == 4  # z overlaps x
    df = _abi.hc_difference_batch
    assert df(x, y, z, 22, 0, 1, 0, 0, 0) == 2
    assert df(x, y, z, 10, 0, 0, 0, 0, 0) == 1                   # batch 0
    assert df(x, y, z, 10, 0, 1, 0, 0, 0) == 6                   # no workspace
    assert df(x, y, y + 8, 10, 0, 1, FAKE + (1 << 30), 1 << 20, 0) == 4  # z overlaps y


def test_maxconv_validation():
    x, y, z, ws = FAKE, FAKE + (1 << 22), FAKE + (1 << 26), FAKE + (1 << 30)
    f = _abi.hc_maxconv_pnorm_batch
    big = 1 << 24
    assert _abi.hc_maxconv_workspace_bytes(10, _abi.HC_I64, 1) == _abi.SIZE_MAX
    need = _abi.hc_maxconv_workspace_bytes(10, _abi.HC_F64, 2)
    assert need >= 2 * 2 * 1024 * 8 + _abi.hc_workspace_bytes(10, _abi.HC_F64, 2)
    assert f(x, y, z, 10, _abi.HC_I64, 1, 2.0, 0, ws, big, 0) == 3      # int64 unsupported
    assert f(x, y, z, 10, 0, 1, 0.5, 0, ws, big, 0) == 1                 # p < 1
    assert f(x, y, z, 10, 0, 1, float("nan"), 0, ws, big, 0) == 1
    assert f(x, y, z, 10, 0, 1, float("inf"), 0, ws, big, 0) == 1
    assert f(x, y, z, 10, 0, 1, 2.0, 4, ws, big, 0) == 1                 # unknown flag
    assert f(x, y, z, 10, 0, 1, 2.0, 0, 0, 0, 0) == 6                    # workspace
    assert f(x, y, x + 8, 10, 0, 1, 2.0, 0, ws, big, 0) == 4             # z overlaps x


def test_sum3_validation():
    x1, x2, x3, z, ws = FAKE, FAKE + (1 << 22), FAKE + (1 << 23), FAKE + (1 << 26), FAKE + (1 << 34)
    f = _abi.hc_sum3_batch
    big = 1 << 30
    # workspace: six staging copies of 4^p 2^K entries per item (K = 6 inner
    # axes, p = D - K), none when everything fits one tile
    assert _abi.hc_sum3_workspace_bytes(6, _abi.HC_F64, 1) == 0
    assert _abi.hc_sum3_workspace_bytes(10, _abi.HC_F64, 2) == 2 * 6 * (1 << 14) * 8
    assert _abi.hc_sum3_workspace_bytes(10, _abi.HC_F32, 1) == 6 * (1 << 14) * 4
    assert _abi.hc_sum3_workspace_bytes(17, _abi.HC_F64, 1) == _abi.SIZE_MAX
    assert _abi.hc_sum3_workspace_bytes(8, 9, 1) == _abi.SIZE_MAX
    assert f(0, x2, x3, z, 8, 0, 1, ws, big, 0) == 1              # null input
    assert f(x1, x2, x3, z, 17, 0, 1, ws, big, 0) == 2            # D above 16
    assert f(x1, x2, x3, z, 8, 7, 1, ws, big, 0) == 3             # dtype
    assert f(x1, x2, x3, z, 8, 0, 0, ws, big, 0) == 1             # batch 0
    assert f(x1 + 4, x2, x3, z, 8, 0, 1, ws, big, 0) == 5         # misaligned
    assert f(x1, x2, x3, z, 8, 0, 1, 0, 0, 0) == 6                # workspace missing
    assert f(x1, x2, x3, x3 + 8, 8, 0, 1, ws, big, 0) == 4        # z overlaps x3
    assert f(x1, x2, x3, z, 8, 0, 1, z + 64, big, 0) == 4         # workspace overlaps z


def test_ternary_validation():
    a, b, z, ws = FAKE, FAKE + (1 << 22), FAKE + (1 << 26), FAKE + (1 << 34)
    f = _abi.hc_ternary_convolve_batch
    big = 1 << 30
    # workspace: four forward staging copies of 6^p 3^K entries and two
    # inverse ones of 6^p 5^K per item (K = 4 inner axes, p = D - K)
    assert _abi.hc_ternary_workspace_bytes(4, _abi.HC_F64, 1) == 0
    assert _abi.hc_ternary_workspace_bytes(6, _abi.HC_F64, 2) == 2 * (4 * 36 * 81 + 2 * 36 * 625) * 8
    assert _abi.hc_ternary_workspace_bytes(5, _abi.HC_F32, 1) == (4 * 6 * 81 + 2 * 6 * 625) * 4
    assert _abi.hc_ternary_workspace_bytes(13, _abi.HC_F64, 1) == _abi.SIZE_MAX
    assert _abi.hc_ternary_workspace_bytes(8, 9, 1) == _abi.SIZE_MAX
    assert f(0, b, z, 6, 0, 1, ws, big, 0) == 1                   # null input
    assert f(a, b, z, 13, 0, 1, ws, big, 0) == 2                  # D above 12
    assert f(a, b, z, 6, 7, 1, ws, big, 0) == 3                   # dtype
    assert f(a, b, z, 6, 0, 0, ws, big, 0) == 1                   # batch 0
    assert f(a + 4, b, z, 6, 0, 1, ws, big, 0) == 5               # misaligned
    assert f(a, b, z, 6, 0, 1, 0, 0, 0) == 6                      # workspace missing
    assert f(a, b, b + 8, 6, 0, 1, ws, big, 0) == 4               # z overlaps b
    assert f(a, b, z, 6, 0, 1, z + 64, big, 0) == 4               # workspace overlaps z


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without libhc.so the binding raises instead of computing anything
    another way (there is no CPU fallback)."""
    monkeypatch.setattr(_abi, "_lib", None)
    monkeypatch.setattr(_abi, "LIB_PATH", str(tmp_path / "libhc.so"))
    with pytest.raises(ImportError, match="missing"):
        _abi.hc_abi_version()
    import paper_1608_00206_amd as hc
    with pytest.raises(ImportError):
        hc.workspace_bytes(10, __import__("torch").float64)


def test_binding_rejects_bad_workspace_and_host_tensors():
    """Host-side checks of the binding: a workspace must be one contiguous
    block of enough bytes on the data's device, and host tensors never reach
    the library."""
    import torch

    import paper_1608_00206_amd as hc
    dev = torch.device("cpu")
    good = torch.empty(64, dtype=torch.uint8)
    assert hc._workspace(64, dev, good) is good
    assert hc._workspace(0, dev, good) is None
    with pytest.raises(ValueError):
        hc._workspace(65, dev, good)
    with pytest.raises(ValueError):
        hc._workspace(16, dev, torch.empty(64, dtype=torch.uint8)[::2])
    x = torch.ones(4, dtype=torch.float64)
    with pytest.raises(ValueError, match="HIP device"):
        hc.convolve(x, x)


def _no_gpu():
    try:
        import torch
        return not torch.cuda.is_available()
    except Exception:
        return True


@pytest.mark.skipif(not _no_gpu(), reason="fake pointers must never reach a GPU")
def test_validation_never_crashes_on_random_arguments():
    """Random argument combinations (including out-of-range D, dtype and
    batch, null, misaligned and overlapping pointers, short workspaces) return
    a documented status code; on a host without a GPU even valid ones stop at
    HC_ERR_NO_DEVICE, so nothing is ever launched."""
    from hypothesis import given, settings, strategies as st

    ptrs = st.sampled_from([0, FAKE, FAKE + 4, FAKE + 8, FAKE + (1 << 20), FAKE + (1 << 34), FAKE + (1 << 36) + 2])

    @settings(max_examples=400, deadline=None)
    @given(x=ptrs, y=ptrs, z=ptrs, D=st.integers(-3, 25), dtype=st.integers(-2, 4),
           batch=st.integers(-2, 70000), ws=ptrs, wsb=st.sampled_from([0, 1, 16, 1 << 20, 1 << 40]))
    def run(x, y, z, D, dtype, batch, ws, wsb):
        rc = _abi.hc_convolve_batch(x, y, z, D, dtype, batch, ws, wsb, 0)
        assert rc in (1, 2, 3, 4, 5, 6, 7), rc
        rc = _abi.hc_maxconv_pnorm_batch(x, y, z, D, dtype, max(batch, 0) % 4, 2.0, 0, ws, wsb, 0)
        assert rc in (1, 2, 3, 4, 5, 6, 7), rc
        rc = _abi.hc_difference_batch(x, y, z, D, dtype, batch, ws, wsb, 0)
        assert rc in (1, 2, 3, 4, 5, 6, 7), rc

    run()
