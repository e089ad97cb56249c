"""The C ABI under HIP graph capture and concurrent streams.

Every entry point only enqueues kernels on the caller's stream (no
allocation, no memset, no synchronisation), so a caller can capture a call
into a graph and replay it.  Each replay is checked against the eager result,
with eager work and synchronisation between replays.  Calls on different
streams with their own workspaces run concurrently and stay bitwise correct.
"""
import numpy as np
import pytest
import torch

import hc_inputs
import oracle
import paper_1608_00206_amd as hc
from tests import pins

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def on_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("D", [6, 13])
def test_forward_and_backward_captured_in_a_graph(D):
    x, y = hc_inputs.random_pair(D, np.float64, 21)
    w = np.random.default_rng([hc_inputs.SEED, 90, D]).standard_normal(3 ** D)
    X, Y, W = on_gpu(x)[None], on_gpu(y)[None], on_gpu(w)[None]
    Z = torch.empty((1, 3 ** D), dtype=torch.float64, device=DEV)
    GX = torch.empty_like(X)
    GY = torch.empty_like(Y)
    wsf = torch.empty(max(hc.workspace_bytes(D, torch.float64), 16), dtype=torch.uint8, device=DEV)
    wsb = torch.empty(max(hc.backward_workspace_bytes(D, torch.float64), 16), dtype=torch.uint8, device=DEV)
    ref_z = oracle.canonical(x, y)
    ref_gx, ref_gy = oracle.adjoint(x, y, w)

    def work():
        hc.convolve_batch(X, Y, out=Z, workspace=wsf)
        gx, gy = hc.convolve_backward(X, Y, W, workspace=wsb)
        GX.copy_(gx)
        GY.copy_(gy)

    s = torch.cuda.Stream(device=DEV)
    s.wait_stream(torch.cuda.current_stream(DEV))
    with torch.cuda.stream(s):
        work()                                  # warm-up outside the capture
    torch.cuda.current_stream(DEV).wait_stream(s)
    torch.cuda.synchronize(DEV)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        work()
    for rep in range(4):
        Z.zero_()
        GX.zero_()
        GY.zero_()
        torch.cuda.synchronize(DEV)
        g.replay()
        torch.cuda.synchronize(DEV)
        pins.assert_bitwise(Z[0].cpu().numpy(), ref_z, f"replay {rep}: z")
        pins.assert_bitwise(GX[0].cpu().numpy(), ref_gx, f"replay {rep}: grad_x")
        pins.assert_bitwise(GY[0].cpu().numpy(), ref_gy, f"replay {rep}: grad_y")
        # eager work between replays, on the same buffers
        hc.convolve_batch(Y, X, out=Z, workspace=wsf)
        torch.cuda.synchronize(DEV)


def test_concurrent_streams():
    jobs = []
    for k, D in enumerate([9, 12, 14, 15]):
        x, y = hc_inputs.random_pair(D, np.float64, 30 + k)
        X, Y = on_gpu(x), on_gpu(y)
        Z = torch.empty(3 ** D, dtype=torch.float64, device=DEV)
        ws = torch.empty(max(hc.workspace_bytes(D, torch.float64), 16), dtype=torch.uint8, device=DEV)
        jobs.append((D, x, y, X, Y, Z, ws, torch.cuda.Stream(device=DEV)))
    torch.cuda.synchronize(DEV)
    for rep in range(3):
        for D, x, y, X, Y, Z, ws, s in jobs:
            with torch.cuda.stream(s):
                hc.convolve(X, Y, out=Z, workspace=ws)
        torch.cuda.synchronize(DEV)
        for D, x, y, X, Y, Z, ws, s in jobs:
            pins.assert_bitwise(Z.cpu().numpy(), oracle.canonical(x, y), f"D={D} rep {rep}")
