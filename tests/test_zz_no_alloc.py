"""The allocation-free entry point (hc_convolve_batch_noalloc), called
through the C ABI: bitwise equal to hc_convolve_batch with a caller
workspace, on two calls in a row (the second smaller), for every dtype, and
a clear error beyond the scratch limit."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import hc_inputs
from paper_1608_00206_amd import _abi

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
CODES = {torch.float64: _abi.HC_F64, torch.float32: _abi.HC_F32, torch.int64: _abi.HC_I64}
LIMIT = 64 << 20  # HC_NOALLOC_SCRATCH_BYTES


def say(msg):
    print(f"[noalloc] {msg}", file=sys.stderr, flush=True)


def inputs(D, batch, dtype, seed):
    xs, ys = [], []
    for b in range(batch):
        if dtype == torch.int64:
            x, y = hc_inputs.pair_ints(D, 90 + seed, b)
        else:
            x, y = hc_inputs.pair_masses(D, 90 + seed, b)
        xs.append(x)
        ys.append(y)
    x = torch.from_numpy(np.stack(xs)).to(DEV).to(dtype)
    y = torch.from_numpy(np.stack(ys)).to(DEV).to(dtype)
    return x, y


def with_workspace(x, y, D, code, batch, stream):
    z = torch.empty((batch, 3 ** D), dtype=x.dtype, device=DEV)
    nb = _abi.hc_workspace_bytes(D, code, batch)
    ws = torch.empty(max(nb, 16), dtype=torch.uint8, device=DEV)
    _abi.check(_abi.hc_convolve_batch(x.data_ptr(), y.data_ptr(), z.data_ptr(), D, code, batch,
                                      ws.data_ptr(), nb, stream))
    return z


def noalloc(x, y, D, code, batch, stream):
    z = torch.empty((batch, 3 ** D), dtype=x.dtype, device=DEV)
    _abi.check(_abi.hc_convolve_batch_noalloc(x.data_ptr(), y.data_ptr(), z.data_ptr(), D, code, batch, stream))
    return z


def bits(t):
    return t.view(torch.int32) if t.element_size() == 4 else t.view(torch.int64)


# (D, batch) of the first call, then of the second, smaller call
CASES = [
    (torch.float64, (16, 2), (12, 3)),
    (torch.float32, (17, 1), (13, 2)),
    (torch.int64, (15, 3), (9, 1)),
    (torch.float64, (10, 4), (5, 2)),
]


@pytest.mark.parametrize("dtype,first,second", CASES, ids=["f64", "f32", "i64", "f64-small"])
def test_noalloc_matches_workspace_entry_point(dtype, first, second):
    code = CODES[dtype]
    stream = torch.cuda.current_stream(DEV).cuda_stream
    for call, (D, batch) in enumerate((first, second)):
        need = _abi.hc_workspace_bytes(D, code, batch)
        assert 0 <= need <= LIMIT
        say(f"{dtype} call {call}: D={D} batch={batch} workspace {need} bytes")
        x, y = inputs(D, batch, dtype, call)
        z_ref = with_workspace(x, y, D, code, batch, stream)
        z = noalloc(x, y, D, code, batch, stream)
        torch.cuda.synchronize(DEV)
        assert torch.equal(bits(z), bits(z_ref)), f"{dtype} D={D} batch={batch}"


def test_noalloc_back_to_back_on_one_stream():
    """Two calls ordered on one stream without a synchronisation between
    them share the scratch safely; both outputs are right."""
    code = _abi.HC_F64
    stream = torch.cuda.current_stream(DEV).cuda_stream
    xa, ya = inputs(14, 2, torch.float64, 5)
    xb, yb = inputs(13, 1, torch.float64, 6)
    za = noalloc(xa, ya, 14, code, 2, stream)
    zb = noalloc(xb, yb, 13, code, 1, stream)
    ra = with_workspace(xa, ya, 14, code, 2, stream)
    rb = with_workspace(xb, yb, 13, code, 1, stream)
    torch.cuda.synchronize(DEV)
    assert torch.equal(bits(za), bits(ra)) and torch.equal(bits(zb), bits(rb))


@pytest.mark.parametrize("D,dtype,batch", [(17, torch.float64, 1), (16, torch.float64, 3), (18, torch.float32, 1)])
def test_noalloc_rejects_beyond_limit(D, dtype, batch):
    code = CODES[dtype]
    assert _abi.hc_workspace_bytes(D, code, batch) > LIMIT
    x = torch.zeros((batch, 1 << D), dtype=dtype, device=DEV)
    z = torch.empty((batch, 3 ** D), dtype=dtype, device=DEV)
    rc = _abi.hc_convolve_batch_noalloc(x.data_ptr(), x.data_ptr(), z.data_ptr(), D, code, batch,
                                        torch.cuda.current_stream(DEV).cuda_stream)
    assert rc == 6, (rc, _abi.last_error())  # HC_ERR_WORKSPACE
    assert "holds" in _abi.last_error()
