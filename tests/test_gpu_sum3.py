"""GPU parity of the distribution of X1 + X2 + X3 (hc_sum3_batch) through the
C ABI: integers bitwise against the oracle's definition (every triple of
entries); every dtype bitwise against the oracle's per-axis method for three
operands; batches; the all-ones closed form at D = 15; sampled outputs of a
D = 16 integer case against the definition at single indices."""
import sys

import numpy as np
import pytest
import torch

import hc_inputs
import oracle
import paper_1608_00206_amd as hc
from tests import pins

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
DTYPES = [np.float64, np.float32, np.int64]


def say(msg):
    print(f"[sum3] {msg}", file=sys.stderr, flush=True)


def on_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def triple(D, dtype, seed, batch=None):
    g = np.random.default_rng([hc_inputs.SEED, 91, seed, D])
    shape = (1 << D,) if batch is None else (batch, 1 << D)
    if np.dtype(dtype) == np.int64:
        return [g.integers(0, 16, shape, dtype=np.int64) for _ in range(3)]
    out = []
    for _ in range(3):
        u = g.random(shape)
        out.append((u / u.sum(axis=-1, keepdims=True)).astype(dtype))
    return out


def run(xs):
    return hc.sum3(*(on_gpu(x) for x in xs))


# D < 6: one tile of D axes; D >= 6: six-axis tiles, then p = D - 6 outer axes
# as p mod 4 axes in registers and groups of four (D = 10: one group of four
# alone; D = 13: 3 + 4)
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("D", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13])
def test_sum3_matches_oracle_method(dtype, D):
    xs = triple(D, dtype, 1)
    say(f"D={D} {np.dtype(dtype).name}")
    z = run(xs)
    torch.cuda.synchronize(DEV)
    pins.assert_bitwise(z.cpu().numpy(), oracle.sum3_canonical(*xs), f"sum3 D={D}")


@pytest.mark.parametrize("D", [0, 3, 6, 8])
def test_sum3_int64_matches_definition(D):
    xs = triple(D, np.int64, 2)
    z = run(xs)
    torch.cuda.synchronize(DEV)
    pins.assert_bitwise(z.cpu().numpy(), oracle.sum3_naive(*xs), f"sum3 int64 definition D={D}")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("D,B", [(9, 5), (11, 3)])
def test_sum3_batch_and_inputs_unchanged(dtype, D, B):
    xs = triple(D, dtype, 3, batch=B)
    t = [on_gpu(x) for x in xs]
    copies = [a.clone() for a in t]
    z = hc.sum3_batch(*t)
    torch.cuda.synchronize(DEV)
    for a, c in zip(t, copies):
        assert torch.equal(a, c)
    z = z.cpu().numpy()
    for b in range(B):
        pins.assert_bitwise(z[b], oracle.sum3_canonical(xs[0][b], xs[1][b], xs[2][b]), f"item {b}")


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_sum3_d14_every_output(dtype):
    D = 14
    xs = triple(D, dtype, 4)
    z = run(xs)
    torch.cuda.synchronize(DEV)
    pins.assert_bitwise(z.cpu().numpy(), oracle.sum3_canonical(*xs), f"sum3 D=14 {np.dtype(dtype).name}")


def test_sum3_d15_all_ones_closed_form():
    """x1 = x2 = x3 = 1 (int64): z[k] = 3^(digits of k equal to 1 or 2),
    checked for every one of the 4^15 outputs against the closed form
    computed with torch integer ops."""
    D = 15
    one = torch.ones(1 << D, dtype=torch.int64, device=DEV)
    z = hc.sum3(one, one.clone(), one.clone())
    k = torch.arange(4 ** D, dtype=torch.int64, device=DEV)
    n = torch.zeros_like(k)
    for _ in range(D):
        d = k & 3
        n += ((d == 1) | (d == 2)).to(torch.int64)
        k >>= 2
    del k
    expect = torch.pow(torch.full_like(n, 3), n)
    assert torch.equal(z, expect)


def test_sum3_d16_int64_sampled_definition():
    """D = 16 (4^16 outputs, 34 GB): sampled outputs against the definition at
    single indices (exact for these small integers), the corners, and the
    total mass."""
    D = 16
    xs = triple(D, np.int64, 5)
    say("D=16 int64: GPU")
    z = run(xs)
    torch.cuda.synchronize(DEV)
    g = np.random.default_rng([hc_inputs.SEED, 92])
    ks = np.unique(np.concatenate([g.integers(0, 4 ** D, 512, dtype=np.uint64),
                                   np.array([0, 4 ** D - 1], dtype=np.uint64)]))
    got = z[torch.from_numpy(ks.astype(np.int64)).to(DEV)].cpu().numpy()
    ref = oracle.sum3_direct_at(*(x.astype(np.float64) for x in xs), ks)
    assert np.array_equal(got.astype(np.float64), ref)
    total = int(z.sum().item())
    assert total == int(xs[0].sum()) * int(xs[1].sum()) * int(xs[2].sum())
    del z
    torch.cuda.empty_cache()


def test_sum3_d16_float64_exact_on_binary_inputs():
    """D = 16 float64 with inputs in {0, 1}: every forward value is an integer
    below 2^17, every product below 2^51, and the inverse's halvings divide
    even integers, so the method is exact in float64 and every one of the
    4^16 outputs must equal the int64 result of the same inputs (itself
    checked against the definition at sampled indices)."""
    D = 16
    g = np.random.default_rng([hc_inputs.SEED, 93])
    xs = [g.integers(0, 2, 1 << D, dtype=np.int64) for _ in range(3)]
    say("D=16 float64 on binary inputs: GPU")
    zf = hc.sum3(*(on_gpu(x.astype(np.float64)) for x in xs))
    zi = hc.sum3(*(on_gpu(x) for x in xs))
    torch.cuda.synchronize(DEV)
    n = zf.numel()
    step = 1 << 28
    for a in range(0, n, step):
        b = min(n, a + step)
        assert torch.equal(zf[a:b], zi[a:b].to(torch.float64)), f"chunk {a}"
    ks = np.unique(np.random.default_rng([hc_inputs.SEED, 94]).integers(0, 4 ** D, 256, dtype=np.uint64))
    got = zf[torch.from_numpy(ks.astype(np.int64)).to(DEV)].cpu().numpy()
    ref = oracle.sum3_direct_at(*(x.astype(np.float64) for x in xs), ks)
    assert np.array_equal(got, ref)
    del zf, zi
    torch.cuda.empty_cache()
