"""GPU parity of the backward path (gradient of sum(w * z)) against the CPU
oracle's transposed maps (bitwise), the direct correlation (within the
derived bound), central finite differences, and torch.autograd.gradcheck."""
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


def gpu_grad(x, y, w):
    gx, gy = hc.convolve_backward(on_gpu(x)[None], on_gpu(y)[None], on_gpu(w)[None])
    torch.cuda.synchronize(DEV)
    return gx[0].cpu().numpy(), gy[0].cpu().numpy()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("D", list(range(0, 14)))
def test_backward_matches_oracle(dtype, D):
    x, y = hc_inputs.random_pair(D, dtype, seed=300 + D, kind="mass")
    w = np.random.default_rng([5, D]).standard_normal(3 ** D).astype(dtype)
    gx, gy = gpu_grad(x, y, w)
    rx, ry = oracle.adjoint(x, y, w)
    pins.assert_bitwise(gx, rx, f"grad_x D={D}")
    pins.assert_bitwise(gy, ry, f"grad_y D={D}")


@pytest.mark.parametrize("plan", [dict(HC_FUSED_K="2"), dict(HC_FUSED_K="5"), dict(HC_INV_MAXM="2"),
                                  dict(HC_INV_MAXM="4"), dict(HC_INV_MAXM="5"), dict(HC_INV_REG="1"),
                                  dict(HC_INV_REG="2"), dict(HC_INV_REG="3"), dict(HC_GRID_PER_CU="2")])
def test_backward_every_plan_identical(plan, monkeypatch):
    for k, v in plan.items():
        monkeypatch.setenv(k, v)
    D = 12
    x, y = hc_inputs.random_pair(D, np.float64, seed=31, kind="signed")
    w = np.random.default_rng([6, D]).standard_normal(3 ** D)
    gx, gy = gpu_grad(x, y, w)
    rx, ry = oracle.adjoint(x, y, w)
    pins.assert_bitwise(gx, rx, f"grad_x {plan}")
    pins.assert_bitwise(gy, ry, f"grad_y {plan}")


def test_backward_vs_correlation_within_bound():
    D = 11
    x, y = hc_inputs.random_pair(D, np.float64, seed=33, kind="mass")
    w = np.random.default_rng([7, D]).standard_normal(3 ** D)
    gx, gy = gpu_grad(x, y, w)
    idx = np.arange(1 << D, dtype=np.uint64)
    cx, cy = oracle.correlation_at(x, y, w, idx)
    bx, by = oracle.adjoint_bound(x, y, w)
    tol = (4 * D + 2) * 2.0 ** -53
    assert np.all(np.abs(gx - cx) <= tol * bx)
    assert np.all(np.abs(gy - cy) <= tol * by)


@pytest.mark.parametrize("broadcast", [False, True])
def test_backward_batch(broadcast):
    D, B = 10, 4
    pairs = [hc_inputs.random_pair(D, np.float64, seed=40 + b) for b in range(B)]
    W = np.random.default_rng([8, D]).standard_normal((1 if broadcast else B, 3 ** D))
    X = on_gpu(np.stack([p[0] for p in pairs]))
    Y = on_gpu(np.stack([p[1] for p in pairs]))
    gz = on_gpu(W[0]).expand(B, 3 ** D) if broadcast else on_gpu(W)
    gx, gy = hc.convolve_backward(X, Y, gz)
    torch.cuda.synchronize(DEV)
    for b, (x, y) in enumerate(pairs):
        rx, ry = oracle.adjoint(x, y, W[0 if broadcast else b])
        pins.assert_bitwise(gx[b].cpu().numpy(), rx, f"grad_x item {b}")
        pins.assert_bitwise(gy[b].cpu().numpy(), ry, f"grad_y item {b}")


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_shared_weights_match_materialised_copies(dtype):
    """With grad_z of batch stride 0 the library computes the adjoint of w
    once for all items; the gradients equal those of B materialised copies of
    w, bit for bit (D = 14: outer passes and the fused adjoint tile)."""
    D, B = 14, 6
    pairs = [hc_inputs.random_pair(D, dtype, seed=60 + b) for b in range(B)]
    X = on_gpu(np.stack([p[0] for p in pairs]))
    Y = on_gpu(np.stack([p[1] for p in pairs]))
    w = on_gpu(np.random.default_rng([10, D]).standard_normal(3 ** D).astype(dtype))
    gx1, gy1 = hc.convolve_backward(X, Y, w.expand(B, 3 ** D))
    gx2, gy2 = hc.convolve_backward(X, Y, w.expand(B, 3 ** D).contiguous())
    torch.cuda.synchronize(DEV)
    iv = torch.int64 if np.dtype(dtype) == np.float64 else torch.int32
    assert torch.equal(gx1.view(iv), gx2.view(iv))
    assert torch.equal(gy1.view(iv), gy2.view(iv))
    rx, ry = oracle.adjoint(pairs[3][0], pairs[3][1], w.cpu().numpy())
    pins.assert_bitwise(gx1[3].cpu().numpy(), rx, "grad_x item 3, shared w")
    pins.assert_bitwise(gy1[3].cpu().numpy(), ry, "grad_y item 3, shared w")


def test_only_one_gradient_requested():
    D = 12
    x, y = hc_inputs.random_pair(D, np.float64, seed=50)
    w = np.random.default_rng([9, D]).standard_normal(3 ** D)
    rx, ry = oracle.adjoint(x, y, w)
    gx, gy = hc.convolve_backward(on_gpu(x)[None], on_gpu(y)[None], on_gpu(w)[None], need_y=False)
    assert gy is None
    pins.assert_bitwise(gx[0].cpu().numpy(), rx, "grad_x alone")
    gx, gy = hc.convolve_backward(on_gpu(x)[None], on_gpu(y)[None], on_gpu(w)[None], need_x=False)
    assert gx is None
    pins.assert_bitwise(gy[0].cpu().numpy(), ry, "grad_y alone")


def test_autograd_function_and_finite_differences():
    D = 9
    x, y = hc_inputs.random_pair(D, np.float64, seed=60)
    w = np.random.default_rng([10, D]).standard_normal(3 ** D)
    tx = on_gpu(x).requires_grad_(True)
    ty = on_gpu(y).requires_grad_(True)
    tw = on_gpu(w)
    z = hc.HypercubeConv.apply(tx, ty)
    (z * tw).sum().backward()
    rx, ry = oracle.adjoint(x, y, w)
    pins.assert_bitwise(tx.grad.cpu().numpy(), rx, "autograd grad_x")
    pins.assert_bitwise(ty.grad.cpu().numpy(), ry, "autograd grad_y")
    # central differences with h = 1e-6; the loss is bilinear, so only rounding remains
    h = 1e-6
    scale = max(np.abs(rx).max(), np.abs(ry).max())

    def loss(a, b):
        return float((hc.convolve(on_gpu(a), on_gpu(b)) * tw).sum().item())

    for i in np.random.default_rng(11).integers(0, 1 << D, 16):
        e = np.zeros(1 << D)
        e[i] = h
        assert abs((loss(x + e, y) - loss(x - e, y)) / (2 * h) - rx[i]) <= 1e-6 * scale
        assert abs((loss(x, y + e) - loss(x, y - e)) / (2 * h) - ry[i]) <= 1e-6 * scale


@pytest.mark.parametrize("D", [0, 2, 4])
def test_gradcheck(D):
    x, y = hc_inputs.random_pair(D, np.float64, seed=70 + D, kind="signed")
    tx = on_gpu(x).requires_grad_(True)
    ty = on_gpu(y).requires_grad_(True)
    assert torch.autograd.gradcheck(hc.HypercubeConv.apply, (tx, ty), eps=1e-6, atol=1e-9, rtol=1e-7)


def test_int64_backward_unsupported():
    x = torch.zeros(1, 8, dtype=torch.int64, device=DEV)
    with pytest.raises(hc.HCError) as e:
        hc.convolve_backward(x, x.clone(), torch.zeros(1, 27, dtype=torch.int64, device=DEV))
    assert e.value.status == "HC_ERR_UNSUPPORTED"
