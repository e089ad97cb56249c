"""GPU parity of the forward path against the CPU oracle (MI355X only).

Floating point: the GPU applies the method's maps in the same order as the
oracle's per-axis form (forward axes ascending, inverse descending, no FMA
contraction), so the bar is bitwise equality, which is stricter than the
1e-12 (float64) / 1e-5 (float32) relative-to-max|z| tolerance also asserted.
int64: bitwise equality with the oracle and with Algorithm 1 (exact).
"""
import os

import numpy as np
import pytest
import torch

import hc_inputs
import oracle
import paper_1608_00206_amd as hc
from tests import pins

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
TORCH = {np.dtype(np.float64): torch.float64, np.dtype(np.float32): torch.float32,
         np.dtype(np.int64): torch.int64}
TOL = {np.dtype(np.float64): 1e-12, np.dtype(np.float32): 1e-5, np.dtype(np.int64): 0.0}


def on_gpu(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def gpu_conv(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    z = hc.convolve(on_gpu(x), on_gpu(y))
    torch.cuda.synchronize(DEV)
    return z.cpu().numpy()


def check(z_gpu: np.ndarray, z_ref: np.ndarray, what: str):
    tol = TOL[z_ref.dtype]
    if tol:
        scale = float(np.abs(z_ref).max()) or 1.0
        rel = float(np.abs(z_gpu.astype(np.float64) - z_ref.astype(np.float64)).max()) / scale
        assert rel <= tol, f"{what}: relative error {rel} above {tol}"
    pins.assert_bitwise(z_gpu, z_ref, what)


def _pair(D, dtype, seed, kind="mass"):
    return hc_inputs.random_pair(D, dtype, seed, kind)


@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.int64])
@pytest.mark.parametrize("D", list(range(0, 15)))
def test_forward_matches_oracle(dtype, D):
    """Every D from 0 (one scalar product) to 14 (six outer axes, full
    inverse groups and ragged column tiles)."""
    kind = "int" if dtype == np.int64 else ("signed" if D % 2 else "mass")
    x, y = _pair(D, dtype, seed=D, kind=kind)
    check(gpu_conv(x, y), oracle.canonical(x, y), f"D={D} {np.dtype(dtype)}")


@pytest.mark.parametrize("D", [3, 7, 10])
def test_int64_matches_algorithm1(D):
    x, y = _pair(D, np.int64, seed=100 + D, kind="int")
    pins.assert_bitwise(gpu_conv(x, y), oracle.naive(x, y), "Algorithm 1")


@pytest.mark.parametrize("plan", [
    dict(HC_FUSED_K="1"), dict(HC_FUSED_K="3"), dict(HC_FUSED_K="5"), dict(HC_FUSED_K="7"),
    dict(HC_INV_MAXM="1"), dict(HC_INV_MAXM="2"), dict(HC_INV_MAXM="3"), dict(HC_INV_MAXM="4"),
    dict(HC_INV_MAXM="5"), dict(HC_INV_REG="1"), dict(HC_INV_REG="2"), dict(HC_INV_REG="3"),
    dict(HC_FUSED_K="4", HC_INV_MAXM="5", HC_INV_REG="3"), dict(HC_GRID_PER_CU="2"),
    dict(HC_FUSED_K="2", HC_GRID_PER_CU="1", HC_INV_REG="2"),
])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_every_plan_gives_identical_bits(plan, dtype, monkeypatch):
    """Fusion depth, inverse grouping and tile width change only the schedule:
    the result is bitwise the oracle's for every choice (also a race detector)."""
    for k, v in plan.items():
        monkeypatch.setenv(k, v)
    D = 13
    x, y = _pair(D, dtype, seed=7, kind="signed")
    check(gpu_conv(x, y), oracle.canonical(x, y), f"plan {plan}")


@pytest.mark.parametrize("dtype", [np.float64, np.int64])
def test_uniform_batch(dtype):
    D, B = 11, 5
    pairs = [_pair(D, dtype, seed=200 + b, kind="int" if dtype == np.int64 else "mass") for b in range(B)]
    X = on_gpu(np.stack([p[0] for p in pairs]))
    Y = on_gpu(np.stack([p[1] for p in pairs]))
    Z = hc.convolve_batch(X, Y)
    torch.cuda.synchronize(DEV)
    Z = Z.cpu().numpy()
    for b, (x, y) in enumerate(pairs):
        check(Z[b], oracle.canonical(x, y), f"batch item {b}")


@pytest.mark.parametrize("D", [1, 5, 9, 12])
def test_int64_full_range_matches_algorithm1(D):
    """Entries over all of int64: sums, products and outputs overflow, and
    the GPU's wrapping arithmetic must still equal Algorithm 1 modulo 2^64."""
    g = np.random.default_rng([hc_inputs.SEED, 96, D])
    lo, hi = np.iinfo(np.int64).min, np.iinfo(np.int64).max
    x = g.integers(lo, hi, 1 << D, dtype=np.int64, endpoint=True)
    y = g.integers(lo, hi, 1 << D, dtype=np.int64, endpoint=True)
    pins.assert_bitwise(gpu_conv(x, y), oracle.naive(x, y), f"D={D} full-range int64")


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_signed_zeros_and_exact_cancellation(dtype):
    """Inputs drawn from {-1, -0, +0, 1}: most outputs cancel exactly, and
    the sign of every zero must match the oracle's order of operations."""
    D = 10
    g = np.random.default_rng([hc_inputs.SEED, 97])
    vals = np.array([-1.0, -0.0, 0.0, 1.0], dtype=dtype)
    x = vals[g.integers(0, 4, 1 << D)]
    y = vals[g.integers(0, 4, 1 << D)]
    ref = oracle.canonical(x, y)
    assert np.count_nonzero(np.signbit(ref) & (ref == 0)) > 0
    pins.assert_bitwise(gpu_conv(x, y), ref, "signed zeros")


@pytest.mark.parametrize("D", [3, 9])
def test_maximum_batch(D):
    """65535 items, the largest batch (grid y): D = 3 runs as one fused tile
    per item, D = 9 adds an outer forward and an inverse pass; the first, the
    last and 62 sampled items are checked bitwise against the oracle."""
    B = 65535
    g = np.random.default_rng([hc_inputs.SEED, 91, D])
    X = g.random((B, 1 << D))
    Y = g.random((B, 1 << D))
    Z = hc.convolve_batch(on_gpu(X), on_gpu(Y))
    torch.cuda.synchronize(DEV)
    items = np.unique(np.concatenate([[0, B - 1], g.choice(B, 62, replace=False)]))
    Zs = Z[torch.from_numpy(items).to(DEV)].cpu().numpy()
    for row, b in enumerate(items):
        check(Zs[row], oracle.canonical(X[b], Y[b]), f"item {b} of {B}")
    del Z
    torch.cuda.empty_cache()


def test_worked_example_and_deltas():
    pins.pin_worked_example(gpu_conv, np.float64)
    for D in (2, 9, 12):
        pins.pin_deltas(gpu_conv, np.int64, D)


@pytest.mark.parametrize("D", [5, 11, 13])
def test_all_ones_closed_form(D):
    for dtype in (np.float64, np.float32, np.int64):
        pins.pin_all_ones(gpu_conv, dtype, D)


def test_paper_accuracy_workload():
    """Table 1's inputs x = y = [1..2^D]: z[0...0] = 1 and every float64
    output equals the exact integer result."""
    pins.pin_paper_accuracy(gpu_conv, 12, exact_fn=oracle.naive)


def test_config_d10_float64():
    """Workload: one pair at D = 10, normalised masses; against Algorithm 1
    within 1e-12 of max|z| and bitwise against the per-axis oracle."""
    D = 10
    x, y = hc_inputs.pair_masses(D, hc_inputs.W_D10_F64)
    z = gpu_conv(x, y)
    z1 = oracle.naive(x, y)
    assert np.abs(z - z1).max() <= 1e-12 * np.abs(z1).max()
    check(z, oracle.canonical(x, y), "D=10 masses")


def test_output_written_completely():
    """The output is written at every index (a pre-filled NaN canary survives
    nowhere)."""
    D = 13
    x, y = _pair(D, np.float64, seed=3)
    z = torch.full((3 ** D,), float("nan"), dtype=torch.float64, device=DEV)
    hc.convolve(on_gpu(x), on_gpu(y), out=z)
    torch.cuda.synchronize(DEV)
    assert not torch.isnan(z).any().item()


def test_inputs_unchanged():
    D = 13
    x, y = _pair(D, np.float64, seed=4)
    tx, ty = on_gpu(x), on_gpu(y)
    hc.convolve(tx, ty)
    torch.cuda.synchronize(DEV)
    pins.assert_bitwise(tx.cpu().numpy(), x, "x unchanged")
    pins.assert_bitwise(ty.cpu().numpy(), y, "y unchanged")


def test_errors_raise():
    x = torch.zeros(8, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        hc.convolve(x, torch.zeros(16, dtype=torch.float64, device=DEV))
    with pytest.raises(TypeError):
        hc.convolve(x.to(torch.int32), x.to(torch.int32))
    # z overlapping x is rejected on the host, before any launch
    with pytest.raises(hc.HCError) as e:
        hc._abi.check(hc._abi.hc_convolve(x.data_ptr(), x.data_ptr(), x.data_ptr() + 16, 3, 0, 0, 0, 0))
    assert e.value.status == "HC_ERR_ALIAS"


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_element_aligned_slices(dtype):
    """Inputs and output at odd element offsets (as inside packed batches)."""
    D = 11
    x, y = _pair(D, dtype, seed=9)
    X = on_gpu(np.concatenate([np.zeros(1, dtype), x]))
    Y = on_gpu(np.concatenate([np.zeros(3, dtype), y]))
    Z = torch.zeros(3 ** D + 5, dtype=TORCH[np.dtype(dtype)], device=DEV)
    hc.convolve(X[1:], Y[3:], out=Z[5:])
    torch.cuda.synchronize(DEV)
    check(Z[5:].cpu().numpy(), oracle.canonical(x, y), "odd offsets")
    assert not Z[:5].any().item()
